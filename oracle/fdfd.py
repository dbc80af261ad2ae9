"""Oracle discretisation of the 2D TM operator, sources and projections.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper (Sec. 2) takes A as the discretised -laplacian - (omega/c)^2 eps_r
for TM waves, with a perfectly matched layer, and states that A is symmetric
(reciprocity) while d A / d p_k is diagonal on the affected pixels.  It leaves
the stencil, PML form and channel normalisation to its solver package, so the
oracle fixes them as follows (the same reading the library documents):

* Ez on nodes (i, j), i = 0..nx-1 periodic in x, j = 0..ny-1 rows top to
  bottom, spacing dx in both directions, eps real per node, E = 0 beyond the
  first and last rows.
* Time convention exp(-i omega t).  Uniaxial PML stretching y only:
  s(d) = 1 + i alpha (d/L)^m for d > 0 pixels past the PML's inner face (the
  half-row between the PML and the first physical row), with m = pml_power,
  alpha = (m+1) ln(1/R0) / (2 h sqrt(eps_pml) L) and h = k0 dx.
* The dx^2-scaled operator, symmetric by construction:
    (A E)_ij = s_j (2E_ij - E_i+1,j - E_i-1,j)
             + (1/s_j+1/2 + 1/s_j-1/2) E_ij - E_i,j+1 / s_j+1/2 - E_i,j-1 / s_j-1/2
             - h^2 eps_ji s_j E_ij
* Channel a: phi_a(i) = exp(2 pi i a i / nx)/sqrt(nx), propagation constant q_a
  in (0, pi) from sin^2(q/2) = h^2 eps/4 - sin^2(pi a / nx).
  B[(i, j_s), a] = -2i sqrt(sin q_a) phi_a(i)  (a unit-flux outgoing wave),
  C[b, (i, j_p)] = sqrt(sin q_b) conj(phi_b(i)),  D = 0 (transmission).
"""
from __future__ import annotations

import math

import numpy as np


def pml_alpha(h: float, eps_pml: float, L: int, m: int, R0: float) -> float:
    return (m + 1) * math.log(1.0 / R0) / (2.0 * h * math.sqrt(eps_pml) * L)


def stretch_profile(prob):
    """Return (s_row[ny], s_half[ny+1]); s_half[j] is s at y = j - 1/2."""
    h = prob.h
    m = prob.pml_power
    ny = prob.ny
    Lt, Lb = prob.npml_top, prob.npml_bot
    at = pml_alpha(h, prob.eps_top, Lt, m, prob.pml_R0) if Lt > 0 else 0.0
    ab = pml_alpha(h, prob.eps_bot, Lb, m, prob.pml_R0) if Lb > 0 else 0.0
    yt = Lt - 0.5
    yb = ny - Lb - 0.5

    def s_at(y):
        if Lt > 0 and y < yt:
            d = yt - y
            return 1.0 + 1j * at * (d / Lt) ** m
        if Lb > 0 and y > yb:
            d = y - yb
            return 1.0 + 1j * ab * (d / Lb) ** m
        return 1.0 + 0.0j

    s_row = np.array([s_at(float(j)) for j in range(ny)], dtype=np.complex128)
    s_half = np.array([s_at(j - 0.5) for j in range(ny + 1)], dtype=np.complex128)
    return s_row, s_half


def row_blocks(prob, eps):
    """Block-tridiagonal form in y-row blocks.

    Returns (D, u): D[j] is the nx x nx diagonal block of row j (x-periodic
    second difference plus the y diagonal terms) and u[j] (j = 0..ny-2) the
    scalar that multiplies the identity in both off-diagonal blocks between
    rows j and j+1 (A is symmetric)."""
    nx, ny = prob.nx, prob.ny
    h2 = prob.h ** 2
    s_row, s_half = stretch_profile(prob)
    D = np.zeros((ny, nx, nx), dtype=np.complex128)
    idx = np.arange(nx)
    for j in range(ny):
        sj = s_row[j]
        diag = 2.0 * sj + 1.0 / s_half[j + 1] + 1.0 / s_half[j] - h2 * eps[j, :] * sj
        D[j, idx, idx] = diag
        D[j, idx, (idx + 1) % nx] += -sj
        D[j, idx, (idx - 1) % nx] += -sj
    u = np.array([-1.0 / s_half[j + 1] for j in range(ny - 1)], dtype=np.complex128)
    return D, u


def node(prob, i, j):
    """Row-major node index used by the oracle's dense forms."""
    return j * prob.nx + i


def assemble_dense(prob, eps):
    """Dense N x N operator (tiny grids only)."""
    nx, ny = prob.nx, prob.ny
    N = nx * ny
    D, u = row_blocks(prob, eps)
    A = np.zeros((N, N), dtype=np.complex128)
    for j in range(ny):
        A[j * nx:(j + 1) * nx, j * nx:(j + 1) * nx] = D[j]
    for j in range(ny - 1):
        r = np.arange(nx)
        A[j * nx + r, (j + 1) * nx + r] = u[j]
        A[(j + 1) * nx + r, j * nx + r] = u[j]
    return A


def propagation_constant(prob, a, eps_medium):
    """q in (0, pi) of channel order a in a homogeneous layer; raises for
    evanescent orders."""
    a = np.asarray(a, dtype=np.float64)
    rhs = prob.h ** 2 * eps_medium / 4.0 - np.sin(np.pi * a / prob.nx) ** 2
    if np.any(rhs <= 0.0) or np.any(rhs >= 1.0):
        raise ValueError("channel order does not propagate on this grid")
    return 2.0 * np.arcsin(np.sqrt(rhs))


def fourier_modes(prob, orders):
    """phi[i, a] = exp(2 pi i a i / nx) / sqrt(nx)."""
    i = np.arange(prob.nx)[:, None]
    a = np.asarray(orders, dtype=np.float64)[None, :]
    return np.exp(2j * np.pi * a * i / prob.nx) / math.sqrt(prob.nx)


def medium_eps(prob, row):
    """Permittivity of the homogeneous layer a source or projection row sits
    in: the top medium above the design slab, the bottom medium below it."""
    if row < prob.design_row0:
        return prob.eps_top
    if row >= prob.design_row1:
        return prob.eps_bot
    raise ValueError("source/projection rows must lie outside the design slab")


def source_block(prob, row, orders):
    """Row-local source block nx x M: column a is -2i sqrt(sin q_a) phi_a."""
    q = propagation_constant(prob, orders, medium_eps(prob, row))
    return -2j * np.sqrt(np.sin(q))[None, :] * fourier_modes(prob, orders)


def projection_block(prob, row, orders):
    """Row-local projection block M x nx: row b is sqrt(sin q_b) conj(phi_b)."""
    q = propagation_constant(prob, orders, medium_eps(prob, row))
    return np.sqrt(np.sin(q))[:, None] * np.conj(fourier_modes(prob, orders)).T


def source_row(prob):
    """B restricted to row src_row, nx x M_in."""
    return source_block(prob, prob.src_row, prob.in_orders)


def projection_row(prob):
    """C restricted to row prj_row, M_out x nx."""
    return projection_block(prob, prob.prj_row, prob.out_orders)


def source_dense(prob):
    B = np.zeros((prob.nx * prob.ny, prob.n_in), dtype=np.complex128)
    B[prob.src_row * prob.nx:(prob.src_row + 1) * prob.nx, :] = source_row(prob)
    return B


def projection_dense(prob):
    C = np.zeros((prob.n_out, prob.nx * prob.ny), dtype=np.complex128)
    C[:, prob.prj_row * prob.nx:(prob.prj_row + 1) * prob.nx] = projection_row(prob)
    return C


def sigma_design(prob):
    """d A_kk / d eps_k for every node, [ny][nx]: -h^2 s_j (Eq. 2 with a
    single-pixel U_k, so Sigma_k is this scalar)."""
    s_row, _ = stretch_profile(prob)
    return np.repeat((-(prob.h ** 2) * s_row)[:, None], prob.nx, axis=1)
