"""Oracle linear solvers: textbook block LU of the banded FDFD operator.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Two orderings of the same block LU with partial pivoting inside each diagonal
block (numpy.linalg.solve is LAPACK's gesv):

* RowBlockLU: y-row blocks of size nx; A is block tridiagonal (the x
  periodicity lives inside each block).  Cost ~ ny nx^3; for small nx.
* CyclicColumnLU: x-column blocks of size ny; A is block tridiagonal with a
  periodic wrap (block-cyclic), eliminated with a border column.  Cost
  ~ nx ny^3; for wide strips.

Both solve A X = R for X with R given on the full grid as [ny][nx][k].
"""
from __future__ import annotations

import numpy as np

from . import fdfd


class RowBlockLU:
    """Block Thomas algorithm in y-row blocks.

    Delta_0 = D_0, Delta_j = D_j - u_{j-1}^2 Delta_{j-1}^{-1}; forward sweep
    y_j = r_j - u_{j-1} Delta_{j-1}^{-1} y_{j-1}; back sweep
    x_j = Delta_j^{-1} (y_j - u_j x_{j+1})."""

    def __init__(self, prob, eps):
        self.prob = prob
        D, u = fdfd.row_blocks(prob, eps)
        self.u = u
        ny, nx = prob.ny, prob.nx
        self.delta = np.empty_like(D)
        self.delta[0] = D[0]
        eye = np.eye(nx, dtype=np.complex128)
        for j in range(1, ny):
            inv_prev = np.linalg.solve(self.delta[j - 1], eye)
            self.delta[j] = D[j] - (u[j - 1] ** 2) * inv_prev

    def solve(self, R):
        R = np.asarray(R, dtype=np.complex128)
        ny = self.prob.ny
        y = np.empty_like(R)
        y[0] = R[0]
        for j in range(1, ny):
            y[j] = R[j] - self.u[j - 1] * np.linalg.solve(self.delta[j - 1], y[j - 1])
        x = np.empty_like(R)
        x[ny - 1] = np.linalg.solve(self.delta[ny - 1], y[ny - 1])
        for j in range(ny - 2, -1, -1):
            x[j] = np.linalg.solve(self.delta[j], y[j] - self.u[j] * x[j + 1])
        return x


def column_blocks(prob, eps):
    """x-column form: T[i] (ny x ny, tridiagonal in y) and the diagonal
    coupling e (length ny) between neighbouring columns, E = diag(e)."""
    nx, ny = prob.nx, prob.ny
    h2 = prob.h ** 2
    s_row, s_half = fdfd.stretch_profile(prob)
    base = 2.0 * s_row + 1.0 / s_half[1:] + 1.0 / s_half[:-1]
    T = np.zeros((nx, ny, ny), dtype=np.complex128)
    jj = np.arange(ny)
    for i in range(nx):
        T[i, jj, jj] = base - h2 * eps[:, i] * s_row
    off = -1.0 / s_half[1:ny]
    T[:, jj[:-1], jj[1:]] = off
    T[:, jj[1:], jj[:-1]] = off
    return T, -s_row


class CyclicColumnLU:
    """Block LU of the block-cyclic tridiagonal system in x-column blocks.

    Columns 0..nx-2 are eliminated in order; column nx-1 is the border that
    the periodic wrap couples to column 0.  For pivot column i the row holds
    Delta_i (diagonal), E towards column i+1 and F_i towards the border; the
    border row holds R_i towards column i and the accumulated block Z."""

    def __init__(self, prob, eps, store=True):
        self.prob = prob
        nx, ny = prob.nx, prob.ny
        if nx < 3:
            raise ValueError("need nx >= 3")
        self.T, e = column_blocks(prob, eps)
        self.e = e
        self.E = np.diag(e)

    def solve(self, R):
        """R: [ny][nx][k] -> X: [ny][nx][k]."""
        prob = self.prob
        nx, ny = prob.nx, prob.ny
        R = np.asarray(R, dtype=np.complex128)
        k = R.shape[2]
        b = [R[:, i, :] for i in range(nx)]
        E = self.E
        zero = np.zeros((ny, ny), dtype=np.complex128)
        last = nx - 1
        delta = self.T[0].copy()
        F = E.copy()                      # row 0 -> border (periodic wrap)
        Rb = E.copy()                     # border row -> column 0
        Z = self.T[last].copy()
        y_last = b[last].copy()
        y = b[0].copy()
        XU, XF, XY = [], [], []
        for i in range(0, nx - 1):
            if i + 1 <= nx - 2:
                rhs = np.concatenate([E, F, y], axis=1)
            else:
                # the upper neighbour of column nx-2 is the border itself; its
                # coupling E was folded into F (and into Rb) one step earlier
                rhs = np.concatenate([zero, F, y], axis=1)
            sol = np.linalg.solve(delta, rhs)
            xu, xf, xy = sol[:, :ny], sol[:, ny:2 * ny], sol[:, 2 * ny:]
            XU.append(xu)
            XF.append(xf)
            XY.append(xy)
            Z = Z - Rb @ xf
            y_last = y_last - Rb @ xy
            if i + 1 <= nx - 2:
                # row i+1 couples to column i through E
                delta = self.T[i + 1] - self.e[:, None] * xu
                F_orig = E if i + 1 == nx - 2 else zero
                F = F_orig - self.e[:, None] * xf
                y = b[i + 1] - self.e[:, None] * xy
                R_orig = E if i + 1 == nx - 2 else zero
                Rb = R_orig - Rb @ xu
        x = [None] * nx
        x[last] = np.linalg.solve(Z, y_last)
        for i in range(nx - 2, -1, -1):
            xi = XY[i] - XF[i] @ x[last]
            if i + 1 <= nx - 2:
                xi = xi - XU[i] @ x[i + 1]
            x[i] = xi
        return np.stack(x, axis=1)
