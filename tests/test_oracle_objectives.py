"""Pins of the grouped multi-angle objective (oracle/objectives.py) against
the mathematics: its Wirtinger derivative against central differences of f
in the real and imaginary directions, the closed form when every target of
an input carries the same power (no penalty: f = -sum p), the target count
of interior and edge inputs, and the workload's channel count and group
spacing (4,559 orders with |a| < 0.95 W/lambda at W = 2,400 lambda; a
24-wavelength supercell's orders, 100 apart)."""
import numpy as np
import pytest

from paper_2306_09257_amd import inputs
import oracle.objectives as oobj


def test_group_fom_derivative_matches_central_differences():
    rng = np.random.default_rng(5)
    ins, outs = np.arange(-3, 4), np.arange(-6, 7)
    S = 0.4 * (rng.standard_normal((13, 7)) + 1j * rng.standard_normal((13, 7)))
    _, G = oobj.group_fom(S, ins, outs, 2)
    T = oobj.targets(ins, outs, 2)
    h = 1e-6
    for n, m in zip(*np.nonzero(T | (rng.random(T.shape) < 0.1))):
        for d in (1.0, 1j):
            Sp, Sm = S.copy(), S.copy()
            Sp[n, m] += h * d
            Sm[n, m] -= h * d
            fd = (oobj.group_fom(Sp, ins, outs, 2)[0] - oobj.group_fom(Sm, ins, outs, 2)[0]) / (2 * h)
            assert abs(fd - 2.0 * np.real(G[n, m] * d)) < 1e-7, (n, m, d)


def test_equal_target_powers_have_no_penalty():
    ins, outs = np.arange(-2, 3), np.arange(-8, 9)
    T = oobj.targets(ins, outs, 3)
    rng = np.random.default_rng(6)
    amp = rng.uniform(0.1, 0.5, ins.size)
    S = np.where(T, amp[None, :] * np.exp(1j * rng.uniform(0, 6.3, T.shape)), 0.0)
    f, G = oobj.group_fom(S, ins, outs, 3)
    assert f == pytest.approx(-np.sum(T.sum(0) * amp ** 2), rel=1e-13)
    assert np.allclose(G[T], -np.conj(S[T]), atol=1e-15) and not np.any(G[~T])


def test_target_counts_interior_and_edge():
    outs = np.arange(-20, 21)
    T = oobj.targets(np.array([0, 15, -20]), outs, 5, gmax=2)
    assert list(T.sum(0)) == [5, 4, 3]


def test_multiangle_workload_recipe():
    orders = inputs.channel_orders(48000, 0.05, sin_max=0.95)
    assert orders.size == 4559 and orders[0] == -2279
    assert int(round(48000 * 0.05 / 24.0)) == 100
