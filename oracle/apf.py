"""Oracle scattering matrix, objective and permittivity gradient.

TEST INFRASTRUCTURE ONLY (see the package docstring).

APF computes, by partial factorisation of the augmented matrix
K = [A, B; C, D], the Schur complement D - C A^-1 B = -S (Sec. 2).  That is
exact linear algebra, so the oracle does not imitate the factorisation: it
solves with A and forms the definitions directly.

Main route (any size the block solvers handle):
    Y = A^-1 B,   S = C Y - D,
    G = dF/dS (Wirtinger, supplied by the caller or from `weighted_power`),
    Lam = A^-T (C^T G)     (the M_in weighted adjoint problems of Sec. 2,
                            one per input, summed over outputs),
    df/deps_k = -2 Re( sigma_k sum_m Lam_km Y_km )   (Eqs. 1-3, u_k = e_k).

Cross-check routes for tiny grids (dense matrices):
    * `grad_conventional`: the loop over inputs of Supplement Eq. (S1),
    * `grad_augmented`: the augmented S~ = [C; U^T] A^-1 [B, U] of Eq. (4)
      with U = the design-pixel selection, then Eq. (3) per pixel,
    * `schur_of_K`: partial Gaussian elimination of the dense K with
      partial pivoting among the A rows (the APF mechanics themselves).
"""
from __future__ import annotations

import numpy as np

from . import blocksolve, fdfd


def make_solver(prob, eps, kind="auto"):
    if kind == "auto":
        kind = "row" if prob.nx <= 4 * prob.ny else "column"
    if kind == "row":
        return blocksolve.RowBlockLU(prob, eps)
    if kind == "column":
        return blocksolve.CyclicColumnLU(prob, eps)
    raise ValueError(kind)


def _rhs_on_row(prob, row, block):
    """Full-grid right-hand side [ny][nx][k] that is `block` (nx x k) on one row."""
    R = np.zeros((prob.ny, prob.nx, block.shape[1]), dtype=np.complex128)
    R[row] = block
    return R


def forward_fields(prob, solver, cols=None):
    """Y = A^-1 B on the full grid, [ny][nx][M_in] (or the chosen inputs)."""
    Bs = fdfd.source_row(prob)
    if cols is not None:
        Bs = Bs[:, cols]
    return solver.solve(_rhs_on_row(prob, prob.src_row, Bs))


def scattering_matrix(prob, eps, solver=None, D=None):
    """S = C A^-1 B - D (D = 0 unless given)."""
    if solver is None:
        solver = make_solver(prob, eps)
    Y = forward_fields(prob, solver)
    S = fdfd.projection_row(prob) @ Y[prob.prj_row]
    if D is not None:
        S = S - D
    return S


def scattering_block(prob, eps, src_row, in_orders, prj_row, out_orders,
                     solver=None, subtract_incident=False):
    """One block of the generalised scattering matrix between arbitrary
    source and projection rows: C_p A^-1 B_s - D, with D = I when the
    projection sits on the source row (the incident wave is removed, Sec. 2:
    D subtracts the baseline)."""
    if solver is None:
        solver = make_solver(prob, eps)
    Bs = fdfd.source_block(prob, src_row, in_orders)
    Y = solver.solve(_rhs_on_row(prob, src_row, Bs))
    S = fdfd.projection_block(prob, prj_row, out_orders) @ Y[prj_row]
    if subtract_incident:
        S = S - (np.asarray(out_orders)[:, None] == np.asarray(in_orders)[None, :])
    return S


def weighted_power(S, w):
    """f = sum_nm w_nm |S_nm|^2 and its Wirtinger derivative dF/dS = w conj(S)."""
    f = float(np.sum(w * np.abs(S) ** 2))
    G = w * np.conj(S)
    return f, G


def adjoint_fields(prob, solver, G):
    """Lam = A^-T (C^T G): the weighted adjoint fields, [ny][nx][M_in].

    A is symmetric, so the same solver applies; `grad_conventional` checks
    this against an explicit transpose solve."""
    Cs = fdfd.projection_row(prob)           # M_out x nx
    src = Cs.T @ G                            # nx x M_in
    return solver.solve(_rhs_on_row(prob, prob.prj_row, src))


def gradient_from_fields(prob, Y, Lam):
    """df/deps_k over the design rows: -2 Re(sigma_k sum_m Lam_km Y_km)."""
    sig = fdfd.sigma_design(prob)
    r0, r1 = prob.design_row0, prob.design_row1
    acc = np.sum(Lam[r0:r1] * Y[r0:r1], axis=2)
    return -2.0 * np.real(sig[r0:r1] * acc)


def solve_S_and_grad(prob, eps, G=None, w=None, solver=None):
    """S and df/deps on the design rows.  Give either G (dF/dS) or weights w
    for f = sum w |S|^2.  Returns (S, grad, f or None)."""
    if solver is None:
        solver = make_solver(prob, eps)
    Y = forward_fields(prob, solver)
    S = fdfd.projection_row(prob) @ Y[prob.prj_row]
    f = None
    if G is None:
        f, G = weighted_power(S, w)
    Lam = adjoint_fields(prob, solver, G)
    return S, gradient_from_fields(prob, Y, Lam), f


def grad_sampled_inputs(prob, eps, G, solver=None):
    """Gradient for a G whose nonzero entries sit in a few input columns: only
    those inputs' forward and adjoint fields are needed (any grid size)."""
    if solver is None:
        solver = make_solver(prob, eps)
    cols = np.nonzero(np.any(G != 0, axis=0))[0]
    Y = forward_fields(prob, solver, cols)
    Cs = fdfd.projection_row(prob)
    src = Cs.T @ G[:, cols]
    Lam = solver.solve(_rhs_on_row(prob, prob.prj_row, src))
    return gradient_from_fields(prob, Y, Lam), cols, Y


# ----------------------------------------------------------------------------
# dense cross-check routes (tiny grids)
# ----------------------------------------------------------------------------

def design_nodes(prob):
    r = np.arange(prob.design_row0, prob.design_row1)
    i = np.arange(prob.nx)
    return (r[:, None] * prob.nx + i[None, :]).ravel()


def grad_conventional(prob, eps, G):
    """Supplement Eq. (S1): for each input m, C_adj = sum_n G_nm C_n, an
    adjoint solve with A^T and a forward solve with A."""
    A = fdfd.assemble_dense(prob, eps)
    B = fdfd.source_dense(prob)
    C = fdfd.projection_dense(prob)
    sig = fdfd.sigma_design(prob).ravel()
    k = design_nodes(prob)
    g = np.zeros(k.size)
    for m in range(prob.n_in):
        c_adj = G[:, m] @ C                          # row vector
        z = np.linalg.solve(A.T, c_adj)              # z = c_adj A^-1
        y = np.linalg.solve(A, B[:, m])
        g -= 2.0 * np.real(z[k] * sig[k] * y[k])
    return g.reshape(prob.n_design_rows, prob.nx)


def grad_augmented(prob, eps, G):
    """Eq. (4) with U = design-pixel selection, then Eq. (3) and Eq. (1)."""
    A = fdfd.assemble_dense(prob, eps)
    B = fdfd.source_dense(prob)
    C = fdfd.projection_dense(prob)
    k = design_nodes(prob)
    N = A.shape[0]
    U = np.zeros((N, k.size))
    U[k, np.arange(k.size)] = 1.0
    Bt = np.concatenate([B, U], axis=1)
    Ct = np.concatenate([C, U.T], axis=0)
    St = Ct @ np.linalg.solve(A, Bt)
    mo, mi = prob.n_out, prob.n_in
    CAU = St[:mo, mi:]                               # C A^-1 U
    UAB = St[mo:, :mi]                               # U^T A^-1 B
    sig = fdfd.sigma_design(prob).ravel()[k]
    g = np.empty(k.size)
    for t in range(k.size):
        dS = -np.outer(CAU[:, t], UAB[t, :]) * sig[t]
        g[t] = np.sum(2.0 * np.real(G * dS))
    return g.reshape(prob.n_design_rows, prob.nx), St[:mo, :mi]


def schur_of_K(A, B, C, D):
    """Partial factorisation of K = [A, B; C, D]: eliminate the first N
    unknowns with row pivoting among the A rows; the trailing block is the
    Schur complement D - C A^-1 B."""
    N = A.shape[0]
    K = np.block([[A, B], [C, D]]).astype(np.complex128)
    for k in range(N):
        p = k + int(np.argmax(np.abs(K[k:N, k])))
        if p != k:
            K[[k, p], :] = K[[p, k], :]
        piv = K[k, k]
        l = K[k + 1:, k] / piv
        K[k + 1:, k + 1:] -= np.outer(l, K[k, k + 1:])
        K[k + 1:, k] = 0.0
    return K[N:, N:]


def objective_fd(prob, eps, w, pixels, step):
    """Central finite differences of f = sum w |S|^2 on chosen design pixels
    (row-in-slab, column) pairs."""
    out = []
    for (r, i) in pixels:
        ep = eps.copy()
        em = eps.copy()
        ep[prob.design_row0 + r, i] += step
        em[prob.design_row0 + r, i] -= step
        fp, _ = weighted_power(scattering_matrix(prob, ep), w)
        fm, _ = weighted_power(scattering_matrix(prob, em), w)
        out.append((fp - fm) / (2.0 * step))
    return np.array(out)


def grad_augmented_params(prob, eps, G, col_pixel, col_sigma, param_begin, n_sub):
    """Gradient with respect to general parameters p_k by the augmented matrix
    of Eq. (4) with the matrix division of Sec. 2 (Fig. 1d), dense (tiny grids).

    dA/dp_k = U_k Sigma_k U_k^T (Eq. (2)): the columns of U_k are the unit
    vectors of the design pixels col_pixel[c] (row-major over the design
    rows) for c in [param_begin[k], param_begin[k+1]), Sigma_k holds
    col_sigma[c].  The parameters are split into n_sub consecutive groups;
    group n gives S~(n) = [C; U(n)^T] A^-1 [B, U(n)] and Eq. (3) is applied to
    its blocks C A^-1 U(n) and U(n)^T A^-1 B without merging:
        df/dp_k = sum_nm 2 Re(G_nm dS_nm/dp_k),
        dS/dp_k = -(C A^-1 U_k) Sigma_k (U_k^T A^-1 B).
    Returns (dfdp, S) with S = C A^-1 B from the first group."""
    A = fdfd.assemble_dense(prob, eps)
    B = fdfd.source_dense(prob)
    C = fdfd.projection_dense(prob)
    N = A.shape[0]
    mo, mi = prob.n_out, prob.n_in
    pb = np.asarray(param_begin)
    n_params = pb.size - 1
    nodes = design_nodes(prob)[np.asarray(col_pixel)]
    dfdp = np.zeros(n_params)
    S_first = None
    for group in np.array_split(np.arange(n_params), n_sub):
        if group.size == 0:
            continue
        c0, c1 = pb[group[0]], pb[group[-1] + 1]
        r = c1 - c0
        U = np.zeros((N, r))
        U[nodes[c0:c1], np.arange(r)] = 1.0
        St = np.concatenate([C, U.T], axis=0) @ np.linalg.solve(A, np.concatenate([B, U], axis=1))
        if S_first is None:
            S_first = St[:mo, :mi]
        CAU = St[:mo, mi:]
        UAB = St[mo:, :mi]
        for k in group:
            for c in range(pb[k], pb[k + 1]):
                j = c - c0
                dS = -np.outer(CAU[:, j], UAB[j, :]) * col_sigma[c]
                dfdp[k] += np.sum(2.0 * np.real(G * dS))
    return dfdp, S_first
