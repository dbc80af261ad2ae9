"""Oracle of the B/C compression of Supplement Sec. 1 (reading of this
library; the supplement gives the recipe in one sentence: pad the channels,
weight them by a Hann window, Fourier transform to space, truncate to a
window of a few wavelengths, and undo the transforms after the partial
factorization).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Reading.  The input orders a_lo..a_hi (consecutive) are extended by pad_lo
below and pad_hi above (pad_lo = pad // 2), M' = M + pad orders
a'_t = a_lo - pad_lo + t, t = 0..M'-1, with window weights
w_t = sin^2(pi (t + 1/2) / M').  Compressed source column j = 0..M'-1 on the
source row:
    b_j(i) = sum_t w_t phi_{a'_t}(i) exp(-2 pi i t j / M'),   phi_a(i) = exp(2 pi i a i / nx)/sqrt(nx),
localized around x_j = j nx / M' and set to zero where the periodic distance
|i - x_j| exceeds half the window (truncation).  Compressed projection row j
on the projection row:
    c_j(i) = sum_t w_t conj(phi_{b'_t}(i)) exp(+2 pi i t j / M').
Without truncation S' = C~ A^-1 B~ = F^c W T W F with T = Q A^-1 P over the
extended orders, so the scattering matrix of the original channels is
    S = D_C S' D_B,  D_C[b, j] = gamma_b exp(-2 pi i t_b j / M'_C) / (M'_C w_{t_b}),
                     D_B[j, a] = exp(+2 pi i t_a j / M'_B) beta_a / (M'_B w_{t_a}),
with beta_a = -2i sqrt(sin q_a) and gamma_b = sqrt(sin q_b) the channel
normalisations of B and C; with truncation it is an approximation.
"""
from __future__ import annotations

import numpy as np

from . import apf, fdfd


def extended(orders, pad):
    """(extended orders, window weights, index t of each original order)."""
    o = np.asarray(orders)
    if o.size > 1 and not np.all(np.diff(o) == 1):
        raise ValueError("channel orders must be consecutive")
    lo = pad // 2
    ext = np.arange(o[0] - lo, o[0] - lo + o.size + pad)
    Mx = ext.size
    w = np.sin(np.pi * (np.arange(Mx) + 0.5) / Mx) ** 2
    return ext, w, np.arange(o.size) + lo


def _window_mask(nx, Mx, half_px):
    i = np.arange(nx)[:, None]
    xj = np.arange(Mx)[None, :] * nx / Mx
    d = np.abs(i - xj)
    d = np.minimum(d, nx - d)
    return d <= half_px


def source_basis(prob, pad, half_px):
    """nx x M'_B compressed (truncated) source columns on the source row."""
    ext, w, _ = extended(prob.in_orders, pad)
    Mx = ext.size
    i = np.arange(prob.nx)
    P = np.exp(2j * np.pi * np.outer(i, ext) / prob.nx) / np.sqrt(prob.nx)
    F = np.exp(-2j * np.pi * np.outer(np.arange(Mx), np.arange(Mx)) / Mx)
    Bh = P @ (w[:, None] * F)
    return np.where(_window_mask(prob.nx, Mx, half_px), Bh, 0.0)


def projection_basis(prob, pad, half_px):
    """M'_C x nx compressed (truncated) projection rows on the projection row."""
    ext, w, _ = extended(prob.out_orders, pad)
    Mx = ext.size
    i = np.arange(prob.nx)
    Q = np.exp(-2j * np.pi * np.outer(ext, i) / prob.nx) / np.sqrt(prob.nx)
    Fc = np.exp(2j * np.pi * np.outer(np.arange(Mx), np.arange(Mx)) / Mx)
    Ch = (Fc * w[None, :]) @ Q
    return np.where(_window_mask(prob.nx, Mx, half_px).T, Ch, 0.0)


def decompression(prob, pad):
    """(D_C, D_B) of the module docstring."""
    ext_b, w_b, t_b = extended(prob.out_orders, pad)
    ext_a, w_a, t_a = extended(prob.in_orders, pad)
    Mc, Mb = ext_b.size, ext_a.size
    q_in = fdfd.propagation_constant(prob, prob.in_orders, fdfd.medium_eps(prob, prob.src_row))
    q_out = fdfd.propagation_constant(prob, prob.out_orders, fdfd.medium_eps(prob, prob.prj_row))
    beta = -2j * np.sqrt(np.sin(q_in))
    gamma = np.sqrt(np.sin(q_out))
    DC = gamma[:, None] * np.exp(-2j * np.pi * np.outer(t_b, np.arange(Mc)) / Mc) / (Mc * w_b[t_b][:, None])
    DB = np.exp(2j * np.pi * np.outer(np.arange(Mb), t_a) / Mb) * (beta / (Mb * w_a[t_a]))[None, :]
    return DC, DB


def compressed_schur(prob, eps, pad, half_px, solver=None):
    """S' = C~ A^-1 B~ with the truncated compressed channels."""
    if solver is None:
        solver = apf.make_solver(prob, eps)
    Bt = source_basis(prob, pad, half_px)
    Y = solver.solve(apf._rhs_on_row(prob, prob.src_row, Bt))
    return projection_basis(prob, pad, half_px) @ Y[prob.prj_row]


def scattering_matrix_compressed(prob, eps, pad, half_px, solver=None):
    """S of the original channels from the compressed factorization."""
    Sp = compressed_schur(prob, eps, pad, half_px, solver)
    DC, DB = decompression(prob, pad)
    return DC @ Sp @ DB


def grad_compressed(prob, eps, G, pad, half_px, solver=None):
    """Eq. (3) over the compressed channels: the exact gradient of f(S) with
    S = D_C S' D_B and S' = C~ A^-1 B~.  Since dS/dp = D_C (dS'/dp) D_B, the
    derivative with respect to S' is G' = D_C^T G D_B^T, and the gradient is
    the one of the plain route with (B~, C~, G') in place of (B, C, G):
    forward fields A^-1 B~, weighted adjoint fields A^-1 C~^T G'.
    Returns (S, grad)."""
    if solver is None:
        solver = apf.make_solver(prob, eps)
    Bt = source_basis(prob, pad, half_px)
    Ct = projection_basis(prob, pad, half_px)
    DC, DB = decompression(prob, pad)
    Y = solver.solve(apf._rhs_on_row(prob, prob.src_row, Bt))
    S = DC @ (Ct @ Y[prob.prj_row]) @ DB
    Gp = DC.T @ G @ DB.T
    Lam = solver.solve(apf._rhs_on_row(prob, prob.prj_row, Ct.T @ Gp))
    return S, apf.gradient_from_fields(prob, Y, Lam)
