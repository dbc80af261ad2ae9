"""Pins of the oracle's B/C compression (Supplement Sec. 1 as this library
reads it): the transforms are exact when nothing is truncated, the
decompression undoes a known compressed block, the compressed columns are
localized, and the truncation error falls as the window widens."""
import numpy as np
import pytest

from paper_2306_09257_amd import inputs
import oracle.apf as oapf
import oracle.compress as oc


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("pad", [0, 6, 11])
def test_untruncated_compression_reproduces_S(pad):
    prob, eps, w = inputs.tiny_problem(nx=64, ny=60, seed=3, in_orders=np.arange(-3, 4, dtype=np.int32),
                                       out_orders=np.arange(-2, 2, dtype=np.int32))
    S = oapf.scattering_matrix(prob, eps)
    Sc = oc.scattering_matrix_compressed(prob, eps, pad, half_px=prob.nx)
    assert _rel(Sc, S) < 1e-12


def test_decompression_undoes_a_known_compressed_block():
    """S' = F^c W T W F for an arbitrary T over the extended orders: the
    decompression returns gamma T beta on the original orders."""
    prob, eps, w = inputs.tiny_problem(nx=64, ny=60, seed=3)
    pad = 8
    ext_b, w_b, t_b = oc.extended(prob.out_orders, pad)
    ext_a, w_a, t_a = oc.extended(prob.in_orders, pad)
    Mc, Mb = ext_b.size, ext_a.size
    rng = np.random.default_rng(4)
    T = rng.standard_normal((Mc, Mb)) + 1j * rng.standard_normal((Mc, Mb))
    Fc = np.exp(2j * np.pi * np.outer(np.arange(Mc), np.arange(Mc)) / Mc)
    F = np.exp(-2j * np.pi * np.outer(np.arange(Mb), np.arange(Mb)) / Mb)
    Sp = (Fc * w_b[None, :]) @ T @ (w_a[:, None] * F)
    DC, DB = oc.decompression(prob, pad)
    import oracle.fdfd as ofd
    q_in = ofd.propagation_constant(prob, prob.in_orders, ofd.medium_eps(prob, prob.src_row))
    q_out = ofd.propagation_constant(prob, prob.out_orders, ofd.medium_eps(prob, prob.prj_row))
    want = np.sqrt(np.sin(q_out))[:, None] * T[np.ix_(t_b, t_a)] * (-2j * np.sqrt(np.sin(q_in)))[None, :]
    assert _rel(DC @ Sp @ DB, want) < 1e-12


def test_compressed_columns_are_localized_and_truncation_error_falls_with_the_window():
    prob = inputs.make_problem(480, 92)
    rng = np.random.default_rng(3)
    eps = inputs.eps_binary_smoothed(prob, rng)
    pad = 20
    full = oc.source_basis(prob, pad, half_px=prob.nx)
    Mx = full.shape[1]
    i = np.arange(prob.nx)
    for j in (0, Mx // 3):
        xj = j * prob.nx / Mx
        d = np.minimum(np.abs(i - xj), prob.nx - np.abs(i - xj))
        col = np.abs(full[:, j]) ** 2
        assert col[d <= 60].sum() > 0.999 * col.sum()          # 99.9% of the energy within +-3 wavelengths
    solver = oapf.make_solver(prob, eps)
    S = oapf.scattering_matrix(prob, eps, solver=solver)
    errs = [_rel(oc.scattering_matrix_compressed(prob, eps, pad, half_px=hw, solver=solver), S) for hw in (30, 60, 90)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 3e-4, errs


def _small_case():
    return inputs.tiny_problem(nx=64, ny=60, seed=3, in_orders=np.arange(-3, 4, dtype=np.int32),
                               out_orders=np.arange(-2, 2, dtype=np.int32))


@pytest.mark.parametrize("pad", [0, 6])
def test_untruncated_compressed_gradient_is_the_plain_gradient(pad):
    prob, eps, w = _small_case()
    S, g, _ = oapf.solve_S_and_grad(prob, eps, w=w)
    _, G = oapf.weighted_power(S, w)
    Sc, gc = oc.grad_compressed(prob, eps, G, pad, half_px=prob.nx)
    assert _rel(Sc, S) < 1e-12 and _rel(gc, g) < 1e-11


def test_truncated_compressed_gradient_matches_central_differences():
    """The gradient of the compressed route is the exact derivative of the
    decompressed S it returns (truncated to a narrow window, so that S differs
    from the plain one), whatever G' = D_C^T G D_B^T makes of dF/dS."""
    prob, eps, w = _small_case()
    pad, hw = 6, 9.0
    Sc, _ = oc.grad_compressed(prob, eps, np.zeros((prob.n_out, prob.n_in), complex), pad, hw)
    assert _rel(Sc, oapf.scattering_matrix(prob, eps)) > 1e-4      # the truncation matters here
    _, G = oapf.weighted_power(Sc, w)
    _, g = oc.grad_compressed(prob, eps, G, pad, hw)
    step = 1e-4
    for (r, i) in [(0, 0), (5, 17), (13, 40), (19, 63)]:
        fs = []
        for sgn in (1.0, -1.0):
            e = eps.copy()
            e[prob.design_row0 + r, i] += sgn * step
            fs.append(oapf.weighted_power(oc.scattering_matrix_compressed(prob, e, pad, hw), w)[0])
        fd = (fs[0] - fs[1]) / (2 * step)
        assert abs(fd - g[r, i]) < 1e-7 * np.abs(g).max(), (r, i, fd, g[r, i])
