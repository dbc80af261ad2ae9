"""Planted mistakes in the oracle (on the CPU, via monkeypatch) must each be
caught by at least one of the pins in test_oracle_pins: a dropped term, a
wrong sign, a wrong index or a missing normalisation."""
import numpy as np
import pytest

import oracle.apf as oapf
import oracle.fdfd as ofd
import tests.test_oracle_pins as pins


def _mut_eps_sign(monkeypatch):
    orig = ofd.row_blocks

    def bad(prob, eps):
        return orig(prob, -eps)           # +h^2 eps instead of -h^2 eps
    monkeypatch.setattr(ofd, "row_blocks", bad)


def _mut_half_row_index(monkeypatch):
    orig = ofd.row_blocks

    def bad(prob, eps):
        D, u = orig(prob, eps)
        _, s_half = ofd.stretch_profile(prob)
        u = np.array([-1.0 / s_half[j] for j in range(prob.ny - 1)])   # j-1/2 for j+1/2
        return D, u
    monkeypatch.setattr(ofd, "row_blocks", bad)


def _mut_source_norm(monkeypatch):
    orig = ofd.source_block

    def bad(prob, row, orders):
        q = ofd.propagation_constant(prob, orders, ofd.medium_eps(prob, row))
        return orig(prob, row, orders) / np.sqrt(np.sin(q))[None, :]
    monkeypatch.setattr(ofd, "source_block", bad)


def _mut_grad_sign(monkeypatch):
    orig = oapf.gradient_from_fields
    monkeypatch.setattr(oapf, "gradient_from_fields", lambda p, Y, L: -orig(p, Y, L))


def _mut_adjoint_conj(monkeypatch):
    orig = oapf.adjoint_fields
    monkeypatch.setattr(oapf, "adjoint_fields", lambda p, s, G: orig(p, s, np.conj(G)))


def _mut_pml_alpha(monkeypatch):
    monkeypatch.setattr(ofd, "pml_alpha", lambda h, e, L, m, R0: 0.0)


MUTATIONS = {
    "eps_sign": (_mut_eps_sign, [pins.test_uniform_slab_converges_to_airy_at_second_order]),
    "half_row_index": (_mut_half_row_index, [pins.test_uniform_slab_converges_to_airy_at_second_order,
                                             pins.test_flux_conservation_lossless]),
    "source_norm": (_mut_source_norm, [pins.test_uniform_slab_converges_to_airy_at_second_order]),
    "grad_sign": (_mut_grad_sign, [pins.test_gradient_central_differences]),
    "adjoint_conj": (_mut_adjoint_conj, [pins.test_gradient_central_differences]),
    "no_pml": (_mut_pml_alpha, [pins.test_flux_conservation_lossless,
                                pins.test_uniform_slab_converges_to_airy_at_second_order]),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    plant, checks = MUTATIONS[name]
    plant(monkeypatch)
    caught = 0
    for check in checks:
        try:
            check()
        except (AssertionError, ValueError, np.linalg.LinAlgError):
            caught += 1
    assert caught >= 1, name
