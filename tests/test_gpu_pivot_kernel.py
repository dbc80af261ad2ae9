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
