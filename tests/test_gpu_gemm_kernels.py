"""Kernel unit tests of the batched complex GEMM (the factorization's task
format) through the test hook apf_test_gemm, against a plain numpy
reference of the same task semantics: operand layouts (transposed A, row
maps of B), triangular masks (stored-index rules of the packed pivot-block
factors), Cin forms (mapped rows, own indexing, column offset, column
range), accumulation into C (per-row EXT_ADD, G_C_ACC, G_ACC_CHUNK), the
launch's column offset and N or K limit, edge tiles and k tails of the
LDS-direct stages, the XCD tile order, and the six kernel forms (FP64
four-product, three-product, four-product on the deep-K kernel, FP32, and
FP64 four-product and FP32 with the tiles of at most 32 valid rows on the
thin kernels, as the factorization and sweep lists run them)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F = dict(TRANS_A=1, NEG=2, CIN=4, B_COFF=8, CIN_COFF=16, B_EXT=32, A_TRI_L=128, A_TRI_U=256,
         B_TRI_L=512, B_TRI_U=1024, CIN_OWN=8192, C_ACC=16384, K_LIM=65536, ACC_CHUNK=131072,
         C_COFF=524288, CIN_RANGE=1048576, CONTRACT=2048, NO_STORE=4096)
EXT_ADD = 1 << 30
MASK = EXT_ADD - 1


def _c(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def reference(flags, M, N, K, A, lda, B, ldb, C0, ldc, Cin=None, ldcin=0, b_offset=0, browmap=None,
              crowmap=None, ccolmap=None, cin_c0=0, cin_w=0, coff=0, nlim=1 << 30, aux=None, auxmap=None,
              part0=None, pstride=0):
    """C after the task, and (G_CONTRACT) the gradient partials: per output
    row and 32-column group, the sum of Re(C(i, j) aux(oi, j))."""
    has = lambda f: bool(flags & F[f])
    Ke = min(K, nlim) if has("K_LIM") else K
    Ne = N if (has("K_LIM") or N < nlim) else nlim
    Aop = np.zeros((M, Ke), complex)
    for i in range(M):
        for k in range(Ke):
            r, c = (k, i) if has("TRANS_A") else (i, k)
            v = A[r * lda + c]
            if has("A_TRI_L"):
                v = v if r > c else (1.0 if r == c else 0.0)
            if has("A_TRI_U"):
                v = v if r <= c else 0.0
            Aop[i, k] = v
    base = (b_offset if has("B_EXT") else 0) + (coff if has("B_COFF") else 0)
    Bop = np.zeros((Ke, Ne), complex)
    for k in range(Ke):
        row = browmap[k] if browmap is not None else k
        for j in range(Ne):
            v = B[base + row * ldb + j]
            if has("B_TRI_L"):
                v = v if k > j else (1.0 if k == j else 0.0)
            if has("B_TRI_U"):
                v = v if k <= j else 0.0
            Bop[k, j] = v
    P = Aop @ Bop
    if has("NEG"):
        P = -P
    out = C0.copy()
    cbase = coff if has("C_COFF") else 0
    cacc = has("C_ACC") or (has("ACC_CHUNK") and coff > 0)
    part = None if part0 is None else part0.copy()
    for i in range(M):
        m = int(crowmap[i]) if crowmap is not None else i
        oi, addold = m & MASK, bool(m & EXT_ADD)
        for j in range(Ne):
            oj = int(ccolmap[j]) if ccolmap is not None else j
            v = P[i, j]
            if has("CIN"):
                ib = coff if has("CIN_COFF") else 0
                ci = i if has("CIN_OWN") else oi
                if has("CIN_RANGE"):
                    cj = coff + j - cin_c0
                    if 0 <= cj < cin_w:
                        v += Cin[ib + ci * ldcin + cj]
                else:
                    v += Cin[ib + ci * ldcin + (j if has("CIN_OWN") else oj)]
            if addold or cacc:
                v += C0[cbase + oi * ldc + oj]
            if has("CONTRACT"):
                P[i, j] = v          # the contraction takes the final value
            if not has("NO_STORE"):
                out[cbase + oi * ldc + oj] = v
        if has("CONTRACT") and auxmap[oi] >= 0:
            for g in range((Ne + 31) // 32):
                js = np.arange(32 * g, min(32 * g + 32, Ne))
                part[((coff + 32 * g) // 32) * pstride + auxmap[oi]] = np.sum(
                    (P[i, js] * aux[oi * ldc + js]).real)
    return out if part is None else (out, part)


def _dev(a, dtype=torch.complex128):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


CASES = {
    "plain_ragged": dict(M=100, N=130, K=37),
    "interior_k_tail": dict(M=128, N=192, K=203),
    "trans_a_interior": dict(M=128, N=128, K=64, flags=["TRANS_A"]),
    "trans_a_edges_tail": dict(M=77, N=150, K=45, flags=["TRANS_A"]),
    "b_rows_mapped": dict(M=128, N=128, K=77, browmap=True, flags=["TRANS_A"]),
    "mapped_out_cin_ext_add": dict(M=96, N=100, K=40, crowmap=True, ccolmap=True, flags=["NEG", "CIN"]),
    "own_cin_accumulate": dict(M=70, N=64, K=33, flags=["CIN", "CIN_OWN", "C_ACC"]),
    "ext_b_offset_coff_nlim": dict(M=64, N=192, K=50, nlim=100, coff=64, b_offset=7,
                                   flags=["B_EXT", "B_COFF", "C_COFF"]),
    "k_limited_chunk_acc": dict(M=64, N=64, K=300, nlim=150, coff=64, flags=["K_LIM", "ACC_CHUNK"]),
    "cin_column_range": dict(M=80, N=128, K=24, coff=64, cin_c0=100, cin_w=50, flags=["CIN", "CIN_RANGE"]),
    "tri_a_lower_perm": dict(M=96, N=120, K=96, browmap=True, flags=["A_TRI_L"]),
    "tri_a_upper_trans": dict(M=100, N=70, K=100, flags=["A_TRI_U", "TRANS_A"]),
    "tri_b_upper": dict(M=90, N=90, K=90, flags=["B_TRI_U"]),
    "tri_b_lower": dict(M=50, N=70, K=70, flags=["B_TRI_L"]),
    "xcd_order": dict(M=300, N=520, K=64, xcd=True),
    "degenerate_1x1x1": dict(M=1, N=1, K=1),
    "no_k_cin_only": dict(M=20, N=30, K=0, flags=["CIN"]),
    # tiles with at most 16 or 32 valid rows (per-wave column strips, operands
    # loaded straight into registers)
    "thin16_b_rows_mapped_k_tail": dict(M=11, N=200, K=39, browmap=True, flags=["NEG", "CIN"]),
    "thin32_b_rows_mapped_trans": dict(M=27, N=150, K=62, browmap=True, flags=["TRANS_A", "NEG"]),
    "thin32_long_k_mapped_out": dict(M=22, N=90, K=449, crowmap=True, ccolmap=True, flags=["CIN"]),
    "thin_ext_coff_nlim": dict(M=10, N=192, K=50, nlim=100, coff=64, b_offset=7,
                               flags=["B_EXT", "B_COFF", "C_COFF"]),
    "thin_k_limited_chunk_acc": dict(M=16, N=64, K=300, nlim=150, coff=64, flags=["K_LIM", "ACC_CHUNK"]),
    "thin_cin_range_coff": dict(M=30, N=70, K=5, coff=64, cin_c0=90, cin_w=30,
                                flags=["CIN", "CIN_RANGE", "CIN_COFF"]),
    # thin tiles with a triangular operand (the leaves' L21 = F21 U^-1 and
    # Z = L21 L^-1, the small fronts' L^-1 P^T F12, X12 = U^-1 U12, LC1T)
    "thin_tri_a_lower_perm": dict(M=20, N=130, K=20, browmap=True, flags=["A_TRI_L"]),
    "thin_tri_a_upper": dict(M=9, N=36, K=9, flags=["A_TRI_U"]),
    "thin_tri_a_upper_trans": dict(M=30, N=70, K=30, flags=["A_TRI_U", "TRANS_A"]),
    "thin_tri_b_upper": dict(M=26, N=38, K=38, flags=["B_TRI_U"]),
    "thin_tri_b_lower_neg_cin": dict(M=26, N=70, K=70, flags=["B_TRI_L", "NEG", "CIN"]),
    # the sweeps' contraction (gradient partials per 32-column group)
    "contract_thin16_no_store": dict(M=11, N=150, K=39, browmap=True, crowmap=True, coff=64,
                                     flags=["TRANS_A", "NEG", "CIN", "CONTRACT", "NO_STORE"]),
    "contract_thin32": dict(M=27, N=100, K=62, browmap=True, flags=["NEG", "CIN", "CONTRACT"]),
    "contract_ragged": dict(M=100, N=130, K=37, crowmap=True, flags=["TRANS_A", "CONTRACT"]),
    "contract_interior": dict(M=128, N=128, K=40, browmap=True, flags=["TRANS_A", "NEG", "CONTRACT"]),
}


@pytest.mark.parametrize("form", [0, 1, 2, 3, 4, 5], ids=["four", "three", "four_deep", "fp32", "four_thin",
                                                      "fp32_thin"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_gemm_kernel_matches_the_task_semantics(name, form):
    from paper_2306_09257_amd import binding
    c = CASES[name]
    M, N, K = c["M"], c["N"], c["K"]
    flags = sum(F[f] for f in c.get("flags", []))
    rng = np.random.default_rng(abs(hash(name)) % 2 ** 32)
    trans = bool(flags & F["TRANS_A"])
    lda = (M if trans else K) + 3
    A = _c(rng, (K if trans else M) * lda + 1)
    nb_rows = K + 23 if c.get("browmap") else K
    ldb = N + 5 + c.get("coff", 0)
    b_offset = c.get("b_offset", 0)
    B = _c(rng, b_offset + max(nb_rows, 1) * ldb + 1)
    browmap = rng.permutation(nb_rows)[:K].astype(np.int32) if c.get("browmap") else None
    crow = None
    out_rows = M
    if c.get("crowmap"):
        out_rows = M + 17
        crow = rng.permutation(out_rows)[:M].astype(np.int64)
        crow = np.where(rng.random(M) < 0.5, crow | EXT_ADD, crow).astype(np.int32)
    ccol = rng.permutation(N + 9)[:N].astype(np.int32) if c.get("ccolmap") else None
    ldc = (N + 9 if ccol is not None else N) + 2 + c.get("coff", 0)
    C0 = _c(rng, out_rows * ldc + c.get("coff", 0) + 1)
    ldcin = N + 11 + c.get("coff", 0)
    Cin = _c(rng, (out_rows + 1) * ldcin + c.get("coff", 0) + 64) if flags & F["CIN"] else None
    kw = dict(b_offset=b_offset, cin_c0=c.get("cin_c0", 0), cin_w=c.get("cin_w", 0), coff=c.get("coff", 0),
              nlim=c.get("nlim", 1 << 30))
    contract = bool(flags & F["CONTRACT"])
    ckw = {}
    if contract:
        # auxmap: a permutation of the slots with a quarter of the rows unmapped
        aux = _c(rng, out_rows * ldc + 1)
        slots = out_rows + 5
        auxmap = rng.permutation(slots)[:out_rows].astype(np.int32)
        auxmap[rng.random(out_rows) < 0.25] = -1
        ngrp = (c.get("coff", 0) + ((N + 63) // 64) * 64) // 32
        part0 = np.full(ngrp * slots, np.nan)
        ckw = dict(aux=aux, auxmap=auxmap, part0=part0, pstride=slots)
    want = reference(flags, M, N, K, A, lda, B, ldb, C0, ldc, Cin=Cin, ldcin=ldcin, browmap=browmap,
                     crowmap=crow, ccolmap=ccol, **kw, **ckw)
    if contract:
        want, want_part = want
        partd = _dev(part0, torch.float64)
        hk = dict(aux=_dev(aux), auxmap=_dev(auxmap, torch.int32), part=partd, pstride=slots)
    else:
        hk = {}
    Cd = _dev(C0)
    binding.gemm_hook(form, flags, M, N, K, _dev(A), lda, _dev(B), ldb, Cd, ldc,
                      Cin=None if Cin is None else _dev(Cin), ldcin=ldcin,
                      browmap=None if browmap is None else _dev(browmap, torch.int32),
                      crowmap=None if crow is None else _dev(crow, torch.int32),
                      ccolmap=None if ccol is None else _dev(ccol, torch.int32), xcd=c.get("xcd", False), **kw,
                      **hk)
    got = Cd.cpu().numpy()
    scale = max(np.linalg.norm(want), 1e-300)
    err = np.linalg.norm(got - want) / scale
    tol = 1e-6 if form in (3, 5) else 1e-13
    print(f"[gpu] gemm {name} form {form}: rel err {err:.2e}", flush=True)
    assert err < tol, (name, form, err)
    if contract:
        gotp = partd.cpu().numpy()
        sel = ~np.isnan(want_part)
        perr = np.linalg.norm(gotp[sel] - want_part[sel]) / max(np.linalg.norm(want_part[sel]), 1e-300)
        # slots the reference leaves unset: untouched, or zero for column
        # groups past N inside the last tile
        other = gotp[~sel]
        print(f"[gpu] gemm {name} form {form}: partials rel err {perr:.2e}", flush=True)
        assert perr < (1e-5 if form in (3, 5) else 1e-12), (name, form, perr)
        assert np.all(np.isnan(other) | (other == 0.0)), (name, form)
