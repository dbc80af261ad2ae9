"""Oracle for the beam-splitter workload: ridge permittivity from edge
positions, its Jacobian, the figure of merit of Eq. (5) and the chain rule to
the edge positions.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Geometry (Sec. 3 and Supplement Table S2).  A period of nx grid cells holds
ridges between consecutive edge pairs (x_1, x_2), (x_3, x_4), ... measured in
units of the grid spacing along the periodic axis; node j stands for the cell
[j - 1/2, j + 1/2).  With mirror symmetry (Sec. 3, Fig. 2b) the parameters
are the edges of the first half period and the full edge list is
x_1 .. x_N, nx - x_N, .., nx - x_1 (the reflection y -> -y about the central
plane, which sits at x = nx / 2).

Sub-pixel smoothing (the paper gives only that d A / d p_k touches the
diagonal entries of the pixels whose permittivity p_k modifies, Sec. 2): a
cell's permittivity is the gap value plus (ridge - gap) times the fraction of
the cell covered by ridges, on every row of the ridge band.  Moving a left
edge by dx changes the covered length of the cell holding it by -dx, a right
edge by +dx, so d eps_j / d x_k = -/+ (eps_ridge - eps_gap) for the cell j
holding x_k (the cell with j - 1/2 <= x_k < j + 1/2, periodic) and zero
elsewhere.

Figure of merit, Eq. (5): f = sum_nm (|T_nm|^2 - t_nm)^2 with t_nm = 1/2 at
the +-1 diffraction orders (output order = input order +- 1) and 0 else; its
Wirtinger derivative is dF/dT = 2 (|T|^2 - t) conj(T) (the paper's
df/dT_nm).
"""
from __future__ import annotations

import numpy as np


def full_edges(edges, nx, mirror):
    """Edge list of the whole period (mirror: append nx - x in reverse)."""
    e = np.asarray(edges, dtype=np.float64)
    if mirror:
        e = np.concatenate([e, nx - e[::-1]])
    if e.size % 2:
        raise ValueError("ridges need an even number of edges")
    return e


def coverage(edges, nx, mirror):
    """Fraction of each cell [j - 1/2, j + 1/2) covered by the ridges
    [x_{2r-1}, x_{2r}] (periodic images included), summed over ridges."""
    e = full_edges(edges, nx, mirror)
    lo = np.arange(nx, dtype=np.float64) - 0.5
    hi = lo + 1.0
    frac = np.zeros(nx)
    for r in range(e.size // 2):
        a, b = e[2 * r], e[2 * r + 1]
        for shift in (-nx, 0, nx):
            frac += np.clip(np.minimum(hi, b + shift) - np.maximum(lo, a + shift), 0.0, None)
    return frac


def ridges_eps(eps, prob, edges, mirror, eps_ridge, eps_gap):
    """Copy of eps ([ny][nx]) with the design rows set from the edges."""
    out = np.array(eps, dtype=np.float64, copy=True)
    frac = coverage(edges, prob.nx, mirror)
    out[prob.design_row0:prob.design_row1, :] = eps_gap + (eps_ridge - eps_gap) * frac[None, :]
    return out


def cell_of(x, nx):
    """Index of the cell holding x (periodic)."""
    return int(np.floor(x + 0.5)) % nx


def jacobian(edges, nx, mirror, eps_ridge, eps_gap):
    """d eps_j / d p_k as a dense (n_params x nx) array: each free edge moves
    its own cell and, with mirror symmetry, its image's cell (d x' / d x = -1)."""
    e = np.asarray(edges, dtype=np.float64)
    n = e.size
    full = full_edges(e, nx, mirror)
    J = np.zeros((n, nx))
    de = eps_ridge - eps_gap
    for k in range(n):
        sign = -1.0 if k % 2 == 0 else 1.0          # left edges even (0-based)
        J[k, cell_of(full[k], nx)] += sign * de
        if mirror:
            q = full.size - 1 - k                   # the image's place in the list
            sq = -1.0 if q % 2 == 0 else 1.0
            J[k, cell_of(full[q], nx)] += -sq * de
    return J


def edge_gradient(grad_eps_design, edges, nx, mirror, eps_ridge, eps_gap):
    """df/dp_k = sum over design rows and cells of df/deps times d eps / d p_k."""
    g = np.asarray(grad_eps_design).sum(axis=0)
    return jacobian(edges, nx, mirror, eps_ridge, eps_gap) @ g


def targets(in_orders, out_orders, t1=0.5):
    """t_nm: t1 where out order - in order = +-1, 0 elsewhere."""
    d = np.asarray(out_orders)[:, None] - np.asarray(in_orders)[None, :]
    return np.where(np.abs(d) == 1, t1, 0.0)


def fom(S, in_orders, out_orders, t1=0.5):
    """Eq. (5) and its Wirtinger derivative dF/dS."""
    t = targets(in_orders, out_orders, t1)
    p = np.abs(S) ** 2
    f = float(np.sum((p - t) ** 2))
    return f, 2.0 * (p - t) * np.conj(S)
