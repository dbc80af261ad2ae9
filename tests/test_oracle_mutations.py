"""Planted mistakes in the oracle (on the CPU, via monkeypatch) must each be
caught by at least one of the pins in test_oracle_pins, test_oracle_splitter
or test_oracle_objectives: a dropped term, a wrong sign, a wrong index, a
missing normalisation or conjugation, a missing periodic image."""
import numpy as np
import pytest

import oracle.apf as oapf
import oracle.fdfd as ofd
import oracle.objectives as oobj
import oracle.splitter as osp
import tests.test_oracle_objectives as opins
import tests.test_oracle_pins as pins
import tests.test_oracle_splitter as spins


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


def _mut_mirror_sign(monkeypatch):
    def bad(edges, nx, mirror, eps_ridge, eps_gap):
        e = np.asarray(edges, dtype=np.float64)
        full = osp.full_edges(e, nx, mirror)
        J = np.zeros((e.size, nx))
        de = eps_ridge - eps_gap
        for k in range(e.size):
            J[k, osp.cell_of(full[k], nx)] += (-1.0 if k % 2 == 0 else 1.0) * de
            if mirror:
                q = full.size - 1 - k
                J[k, osp.cell_of(full[q], nx)] += (-1.0 if q % 2 == 0 else 1.0) * de   # image moves with +1
        return J
    monkeypatch.setattr(osp, "jacobian", bad)


def _mut_coverage_no_wrap(monkeypatch):
    def bad(edges, nx, mirror):
        e = osp.full_edges(edges, nx, mirror)
        lo = np.arange(nx, dtype=np.float64) - 0.5
        frac = np.zeros(nx)
        for r in range(e.size // 2):
            frac += np.clip(np.minimum(lo + 1.0, e[2 * r + 1]) - np.maximum(lo, e[2 * r]), 0.0, None)
        return frac
    monkeypatch.setattr(osp, "coverage", bad)


def _mut_fom_orders(monkeypatch):
    def bad(in_orders, out_orders, t1=0.5):
        d = np.asarray(out_orders)[:, None] - np.asarray(in_orders)[None, :]
        return np.where(np.abs(d) == 2, t1, 0.0)       # the +-2 orders
    monkeypatch.setattr(osp, "targets", bad)


def _mut_fom_no_conj(monkeypatch):
    orig = osp.fom

    def bad(S, i, o, t1=0.5):
        f, G = orig(S, i, o, t1)
        return f, np.conj(G)
    monkeypatch.setattr(osp, "fom", bad)


def _mut_group_no_deviation(monkeypatch):
    orig = oobj.group_fom

    def bad(S, i, o, delta, gmax=2):
        f, G = orig(S, i, o, delta, gmax)
        T = oobj.targets(i, o, delta, gmax)
        return f, np.where(T, -np.conj(S), 0.0)        # the penalty's derivative dropped
    monkeypatch.setattr(oobj, "group_fom", bad)


def _mut_sampled_adjoint_columns(monkeypatch):
    def bad(prob, eps, G, solver=None):
        if solver is None:
            solver = oapf.make_solver(prob, eps)
        cols = np.nonzero(np.any(G != 0, axis=0))[0]
        Y = oapf.forward_fields(prob, solver, cols)
        src = ofd.projection_row(prob).T @ G[:, :cols.size]         # adjoint from the wrong input columns
        Lam = solver.solve(oapf._rhs_on_row(prob, prob.prj_row, src))
        return oapf.gradient_from_fields(prob, Y, Lam), cols, Y
    monkeypatch.setattr(oapf, "grad_sampled_inputs", bad)


def _mut_augmented_blocks(monkeypatch):
    orig = oapf.grad_augmented_params

    def bad(prob, eps, G, col_pixel, col_sigma, param_begin, n_sub):
        d, S = orig(prob, eps, np.conj(G), col_pixel, col_sigma, param_begin, n_sub)   # dF/dS conjugated
        return d, S
    monkeypatch.setattr(oapf, "grad_augmented_params", bad)


def _mut_compress_phase(monkeypatch):
    import oracle.compress as oc
    orig = oc.decompression

    def bad(prob, pad):
        DC, DB = orig(prob, pad)
        return DC, np.conj(DB)                        # wrong sign of the inverse transform's phase
    monkeypatch.setattr(oc, "decompression", bad)


def _mut_compress_grad_conj(monkeypatch):
    import oracle.compress as oc
    orig = oc.decompression

    def grad_bad(prob, eps, G, pad, half_px, solver=None):
        DC, DB = orig(prob, pad)
        if solver is None:
            solver = oapf.make_solver(prob, eps)
        Bt = oc.source_basis(prob, pad, half_px)
        Ct = oc.projection_basis(prob, pad, half_px)
        Y = solver.solve(oapf._rhs_on_row(prob, prob.src_row, Bt))
        S = DC @ (Ct @ Y[prob.prj_row]) @ DB
        Gp = DC.conj().T @ G @ DB.conj().T                 # adjoint instead of transpose
        Lam = solver.solve(oapf._rhs_on_row(prob, prob.prj_row, Ct.T @ Gp))
        return S, oapf.gradient_from_fields(prob, Y, Lam)
    monkeypatch.setattr(oc, "grad_compressed", grad_bad)


def _compress_grad_pin():
    import tests.test_oracle_compress as cpins
    cpins.test_truncated_compressed_gradient_matches_central_differences()


def _compress_pin():
    import tests.test_oracle_compress as cpins
    cpins.test_untruncated_compression_reproduces_S(6)


def _sampled_pin():
    pins.test_sampled_input_gradient_equals_the_full_gradient(16, 60, 0.15, "row")


MUTATIONS = {
    "compress_phase": (_mut_compress_phase, [_compress_pin]),
    "compress_grad_conj": (_mut_compress_grad_conj, [_compress_grad_pin]),
    "augmented_conj": (_mut_augmented_blocks, [pins.test_augmented_parameter_gradient_pins]),
    "sampled_adjoint_columns": (_mut_sampled_adjoint_columns, [_sampled_pin]),
    "mirror_sign": (_mut_mirror_sign, [spins.test_jacobian_matches_finite_differences,
                                       spins.test_edge_gradient_matches_central_differences]),
    "coverage_no_wrap": (_mut_coverage_no_wrap,
                         [spins.test_coverage_conserves_width_is_binary_on_cell_edges_and_mirror_symmetric]),
    "fom_orders": (_mut_fom_orders, [spins.test_table_s2_design_splits_into_the_pm1_orders]),
    "fom_no_conj": (_mut_fom_no_conj, [spins.test_fom_wirtinger_derivative_matches_central_differences]),
    "group_no_deviation": (_mut_group_no_deviation, [opins.test_group_fom_derivative_matches_central_differences]),
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
