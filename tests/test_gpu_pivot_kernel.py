"""Kernel unit tests of the pivot-block kernel through the test hook
apf_test_pivot_block: for block sizes across all six register-blocked
shapes (and their boundaries), the pivot order equals partial pivoting by
largest modulus in numpy, the stored inverses satisfy U^-1 L^-1 F[perm] = I,
the pivot spread equals min |u_kk| / max |u_kk|; a block with a zero column,
a block with a zero row and a block with a NaN report APF_ESINGULAR (the
kernel itself runs to its end), and a block that needs pivoting at every
step (zero diagonal) is factored."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SIZES = [1, 2, 7, 16, 17, 31, 32, 33, 47, 48, 49, 63, 64, 65, 80, 95, 96, 97, 127, 128]


def _lu_partial(F):
    """numpy LU with partial pivoting (largest modulus, lowest row on ties):
    (perm, |u_kk|)."""
    A = F.astype(complex).copy()
    p = A.shape[0]
    unused = np.ones(p, bool)
    perm, u = [], []
    for k in range(p):
        m = np.where(unused, np.abs(A[:, k]) ** 2, -1.0)
        r = int(np.argmax(m))
        perm.append(r)
        u.append(abs(A[r, k]))
        unused[r] = False
        rows = np.nonzero(unused)[0]
        A[rows, k:] -= np.outer(A[rows, k] / A[r, k], A[r, k:])
    return np.array(perm), np.array(u)


def _run(F):
    from paper_2306_09257_amd import binding
    p = F.shape[0]
    Fd = torch.as_tensor(F, dtype=torch.complex128, device="cuda").contiguous()
    tri = torch.zeros((p, p), dtype=torch.complex128, device="cuda")
    perm = torch.zeros(p, dtype=torch.int32, device="cuda")
    q = binding.pivot_block_hook(Fd, tri, perm)
    return tri.cpu().numpy(), perm.cpu().numpy(), q


@pytest.mark.parametrize("p", SIZES)
def test_pivot_block_kernel_matches_partial_pivoting(p):
    rng = np.random.default_rng(p)
    F = rng.standard_normal((p, p)) + 1j * rng.standard_normal((p, p))
    tri, perm, q = _run(F)
    perm_o, u_o = _lu_partial(F)
    Linv = np.tril(tri, -1) + np.eye(p)
    Uinv = np.triu(tri)
    err = np.linalg.norm(Uinv @ Linv @ F[perm] - np.eye(p)) / np.sqrt(p)
    print(f"[gpu] pivot block p={p}: |U^-1 L^-1 F[perm] - I| {err:.2e}, spread {q:.4e}", flush=True)
    assert np.array_equal(perm, perm_o)
    assert err < 1e-11
    assert abs(q - u_o.min() / u_o.max()) < 1e-10 * (u_o.min() / u_o.max())


def test_pivot_block_needing_a_swap_at_every_step():
    p = 40
    rng = np.random.default_rng(1)
    F = np.zeros((p, p), complex)
    F[np.arange(p), (np.arange(p) + 1) % p] = rng.standard_normal(p) + 2.0   # zero diagonal
    tri, perm, q = _run(F)
    assert np.array_equal(perm, _lu_partial(F)[0])
    assert np.linalg.norm(np.triu(tri) @ (np.tril(tri, -1) + np.eye(p)) @ F[perm] - np.eye(p)) < 1e-12


@pytest.mark.parametrize("kind", ["zero_column", "zero_row", "nan"])
@pytest.mark.parametrize("p", [12, 40, 70, 110])
def test_singular_or_non_finite_block_reports_esingular(kind, p):
    from paper_2306_09257_amd import binding
    rng = np.random.default_rng(p + 1)
    F = rng.standard_normal((p, p)) + 1j * rng.standard_normal((p, p))
    if kind == "zero_column":
        F[:, p // 2] = 0.0
    elif kind == "zero_row":
        F[p // 3, :] = 0.0
    else:
        F[p // 2, p // 3] = np.nan
    print(f"[gpu] singular pivot block {kind} p={p}", flush=True)
    with pytest.raises(binding.APFError) as ei:
        _run(F)
    assert ei.value.status == binding.APF_ESINGULAR
    # the kernel ran to its end: a regular block afterwards is factored
    G = rng.standard_normal((p, p)) + 1j * rng.standard_normal((p, p))
    tri, perm, q = _run(G)
    assert np.array_equal(perm, _lu_partial(G)[0])


@pytest.mark.parametrize("p", SIZES)
def test_symmetric_mode_reads_the_lower_triangle_and_keeps_the_order(p):
    """Symmetric mode on a complex symmetric block whose strict upper triangle
    holds NaNs (never read): no row exchanges (perm is the identity), the
    inverses satisfy U^-1 L^-1 F = I, U = D L^T (the L D L^T factorization)
    and the pivot spread is that of the unpivoted elimination."""
    from paper_2306_09257_amd import binding
    rng = np.random.default_rng(100 + p)
    X = rng.standard_normal((p, p)) + 1j * rng.standard_normal((p, p))
    F = X + X.T + 4.0 * np.sqrt(p) * np.eye(p)
    Fin = F.copy()
    Fin[np.triu_indices(p, 1)] = np.nan
    Fd = torch.as_tensor(Fin, dtype=torch.complex128, device="cuda").contiguous()
    tri = torch.zeros((p, p), dtype=torch.complex128, device="cuda")
    perm = torch.zeros(p, dtype=torch.int32, device="cuda")
    q = binding.pivot_block_hook(Fd, tri, perm, sym=True)
    tri, perm = tri.cpu().numpy(), perm.cpu().numpy()
    Linv = np.tril(tri, -1) + np.eye(p)
    Uinv = np.triu(tri)
    err = np.linalg.norm(Uinv @ Linv @ F - np.eye(p)) / np.sqrt(p)
    L, U = np.linalg.inv(Linv), np.linalg.inv(Uinv)
    esym = np.linalg.norm(U - np.diag(np.diag(U)) @ L.T) / np.linalg.norm(U)
    # unpivoted elimination: |u_kk| in numpy
    A = F.copy()
    u = []
    for k in range(p):
        u.append(abs(A[k, k]))
        A[k + 1:, k:] -= np.outer(A[k + 1:, k] / A[k, k], A[k, k:])
    u = np.array(u)
    print(f"[gpu] symmetric pivot block p={p}: |U^-1 L^-1 F - I| {err:.2e}, |U - D L^T| {esym:.2e}", flush=True)
    assert np.array_equal(perm, np.arange(p))
    assert np.isfinite(tri[np.tril_indices(p)]).all() and np.isfinite(Uinv).all()
    assert err < 1e-12 and esym < 1e-12
    assert abs(q - u.min() / u.max()) < 1e-10 * (u.min() / u.max())


def test_symmetric_mode_reports_a_zero_leading_pivot():
    """Without row exchanges a zero diagonal entry is a zero pivot:
    APF_ESINGULAR (partial pivoting factors the same block)."""
    from paper_2306_09257_amd import binding
    p = 24
    rng = np.random.default_rng(5)
    X = rng.standard_normal((p, p)) + 1j * rng.standard_normal((p, p))
    F = X + X.T
    F[0, 0] = 0.0
    Fd = torch.as_tensor(F, dtype=torch.complex128, device="cuda").contiguous()
    tri = torch.zeros((p, p), dtype=torch.complex128, device="cuda")
    perm = torch.zeros(p, dtype=torch.int32, device="cuda")
    with pytest.raises(binding.APFError) as ei:
        binding.pivot_block_hook(Fd, tri, perm, sym=True)
    assert ei.value.status == binding.APF_ESINGULAR
    binding.pivot_block_hook(Fd, tri, perm)
    assert np.array_equal(perm.cpu().numpy(), _lu_partial(F)[0])
