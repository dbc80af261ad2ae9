"""ctypes binding of the APF C ABI (include/apf.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Tensors passed in are torch device tensors; the HIP stream is
torch's current stream.  If the library is not built, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libapf.so")

APF_OK = 0
APF_EINVAL = -1
APF_ENOMEM = -2
APF_EHIP = -3
APF_ESINGULAR = -4
APF_ENOTCONV = -5
APF_ESTATE = -6
APF_AUG_SKIP_UU = 1
APF_FP64 = 0
APF_MIXED = 1
APF_MIXED_REFINED = 2

ENTRY_POINTS = ("apf_create", "apf_analyze", "apf_assemble", "apf_factor_schur", "apf_factor_schur_batched",
                "apf_weighted_power", "apf_splitter_fom", "apf_group_fom", "apf_ridges_eps", "apf_ridges_grad",
                "apf_grad", "apf_set_rhs_chunk", "apf_set_lowrank", "apf_set_profiling", "apf_destroy",
                "apf_last_error", "apf_query", "apf_front", "apf_weighted_power_noalloc", "apf_set_refinement",
                "apf_grad_augmented", "apf_ridges_grad_augmented", "apf_autotune", "apf_tuning_apply",
                "apf_set_compression", "apf_set_gradient", "apf_set_symmetric", "apf_test_gemm",
                "apf_test_pivot_block")
PROFILE_CLASSES = ("stencil", "zero", "assemble", "inverse", "gemm_factor", "gemm_schur", "gemm_sweep",
                   "contract", "wpow", "refine", "adjoint_source")


class APFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"APF status {status}: {msg}")
        self.status = status


class _Desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("dx_over_lambda", ctypes.c_double),
                ("npml_top", ctypes.c_int32), ("npml_bot", ctypes.c_int32),
                ("pml_R0", ctypes.c_double), ("pml_power", ctypes.c_int32),
                ("eps_top", ctypes.c_double), ("eps_bot", ctypes.c_double),
                ("src_row", ctypes.c_int32), ("prj_row", ctypes.c_int32),
                ("design_row0", ctypes.c_int32), ("design_row1", ctypes.c_int32),
                ("n_in", ctypes.c_int32), ("n_out", ctypes.c_int32),
                ("in_orders", ctypes.POINTER(ctypes.c_int32)),
                ("out_orders", ctypes.POINTER(ctypes.c_int32)),
                ("leaf_size", ctypes.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libapf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2306_09257_amd/build.py")
    lib = ctypes.CDLL(path)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    lib.apf_create.argtypes = [ctypes.POINTER(_Desc), ctypes.POINTER(vp)]
    lib.apf_analyze.argtypes = [vp]
    lib.apf_assemble.argtypes = [vp, vp, vp]
    lib.apf_factor_schur.argtypes = [vp, i32, vp, vp]
    lib.apf_factor_schur_batched.argtypes = [ctypes.POINTER(vp), i32, i32, ctypes.POINTER(vp), vp]
    lib.apf_weighted_power.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.apf_weighted_power_noalloc.argtypes = [vp, vp, ctypes.c_int64, vp, vp, vp]
    lib.apf_splitter_fom.argtypes = [vp, vp, dbl, vp, vp, vp]
    lib.apf_group_fom.argtypes = [vp, vp, i32, i32, vp, vp, vp]
    lib.apf_ridges_eps.argtypes = [vp, vp, i32, i32, dbl, dbl, vp, vp]
    lib.apf_ridges_grad.argtypes = [vp, vp, i32, i32, dbl, dbl, vp, vp, vp]
    lib.apf_grad.argtypes = [vp, vp, vp, vp]
    lib.apf_set_profiling.argtypes = [vp, i32]
    lib.apf_set_rhs_chunk.argtypes = [vp, i32]
    lib.apf_set_lowrank.argtypes = [vp, i32]
    lib.apf_set_refinement.argtypes = [vp, i32, dbl]
    lib.apf_set_compression.argtypes = [vp, i32, dbl]
    lib.apf_set_gradient.argtypes = [vp, i32]
    lib.apf_set_symmetric.argtypes = [vp, i32]
    lib.apf_test_pivot_block.argtypes = [i32, vp, vp, vp, ctypes.POINTER(dbl), i32, vp]
    lib.apf_test_gemm.argtypes = [i32, i32, i32, i32, i32, vp, i32, vp, i32, ctypes.c_int64, vp, i32, vp, i32,
                                  vp, vp, vp, i32, i32, i32, i32, i32, vp, vp, vp, i32, vp]
    lib.apf_autotune.argtypes = [ctypes.POINTER(vp), i32, i32, ctypes.c_char_p, vp]
    lib.apf_tuning_apply.argtypes = [ctypes.POINTER(vp), i32, ctypes.c_char_p, vp]
    lib.apf_grad_augmented.argtypes = [vp, i32, vp, vp, i32, vp, i32, i32, vp, vp, vp, ctypes.POINTER(i32), vp]
    lib.apf_ridges_grad_augmented.argtypes = [vp, vp, i32, i32, dbl, dbl, i32, i32, vp, vp, vp,
                                              ctypes.POINTER(i32), vp]
    lib.apf_destroy.argtypes = [vp]
    lib.apf_last_error.argtypes = []
    lib.apf_last_error.restype = ctypes.c_char_p
    lib.apf_query.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(dbl)]
    lib.apf_front.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    for name in ENTRY_POINTS:
        if name != "apf_last_error":
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status):
    if status != APF_OK:
        raise APFError(status, _lib.apf_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class APF:
    """One APF problem: the handle of include/apf.h.

    `prob` is a problem description with the fields of apf_problem_desc
    (paper_2306_09257_amd.inputs.Problem)."""

    def __init__(self, prob, leaf_size: int = 0):
        lib = load_library()
        self.prob = prob
        self._in = np.ascontiguousarray(prob.in_orders, dtype=np.int32)
        self._out = np.ascontiguousarray(prob.out_orders, dtype=np.int32)
        d = _Desc(prob.nx, prob.ny, prob.dx_over_lambda, prob.npml_top, prob.npml_bot,
                  prob.pml_R0, prob.pml_power, prob.eps_top, prob.eps_bot,
                  prob.src_row, prob.prj_row, prob.design_row0, prob.design_row1,
                  self._in.size, self._out.size,
                  self._in.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                  self._out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                  leaf_size)
        h = ctypes.c_void_p()
        _check(lib.apf_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self._lib = lib

    # -- host-side -----------------------------------------------------------
    def analyze(self):
        _check(self._lib.apf_analyze(self._h))
        return self

    def query(self, key: str) -> float:
        v = ctypes.c_double()
        _check(self._lib.apf_query(self._h, key.encode(), ctypes.byref(v)))
        return v.value

    def set_rhs_chunk(self, max_chunk: int):
        """Cap the sweeps' right-hand-side chunk (before the first assemble)."""
        _check(self._lib.apf_set_rhs_chunk(self._h, int(max_chunk)))
        return self

    def set_symmetric(self, on=True):
        """The symmetric route (L D L^T pivot blocks, the products' symmetry),
        before the first assemble."""
        _check(self._lib.apf_set_symmetric(self._h, 1 if on else 0))
        return self

    def set_lowrank(self, levels):
        """Depth of the low-rank sweep subtrees (0 forbids them; False/True
        mean 0 and 2), before the first assemble."""
        lv = (2 if levels else 0) if isinstance(levels, bool) else int(levels)
        _check(self._lib.apf_set_lowrank(self._h, lv))
        return self

    def set_compression(self, pad: int, window_wavelengths: float = 3.0):
        """B/C compression (after analyze, before the first assemble): pad the
        channel sets by `pad` orders, Hann-weight, transform to localized
        columns truncated to the window; pad = -1 switches it off."""
        _check(self._lib.apf_set_compression(self._h, int(pad), float(window_wavelengths)))
        return self

    def set_gradient(self, on: bool):
        """Prepare the gradient sweeps (default) or only S (after analyze,
        before the first assemble)."""
        _check(self._lib.apf_set_gradient(self._h, 1 if on else 0))
        return self

    def set_refinement(self, max_iter: int, tol: float = 1e-10):
        """Enable APF_MIXED_REFINED (before the first assemble): max_iter
        corrections after the first solve, APF_ENOTCONV above tol."""
        _check(self._lib.apf_set_refinement(self._h, int(max_iter), float(tol)))
        return self

    def set_profiling(self, on, gemm_only: bool = False):
        """Event timing of every launch (on), of the GEMM launches only
        (on and gemm_only), or none."""
        _check(self._lib.apf_set_profiling(self._h, (2 if gemm_only else 1) if on else 0))

    def profile(self):
        """{class: (ms, launches)} summed since profiling was enabled."""
        return {c: (self.query("ms_" + c), int(self.query("launches_" + c))) for c in PROFILE_CLASSES}

    def front(self, f: int):
        info = (ctypes.c_int32 * 8)()
        _check(self._lib.apf_front(self._h, f, info, None, None))
        p, b = info[2], info[3]
        piv = (ctypes.c_int32 * max(p, 1))()
        bnd = (ctypes.c_int32 * max(b, 1))()
        _check(self._lib.apf_front(self._h, f, info, piv, bnd))
        return list(info), np.array(piv[:p], dtype=np.int64), np.array(bnd[:b], dtype=np.int64)

    # -- device-side ---------------------------------------------------------
    def assemble(self, eps):
        """eps: float64 [ny][nx] device tensor."""
        assert eps.dtype.is_floating_point and eps.is_contiguous() and eps.is_cuda
        assert tuple(eps.shape) == (self.prob.ny, self.prob.nx)
        self._eps = eps
        _check(self._lib.apf_assemble(self._h, _ptr(eps), _stream()))

    def factor_schur(self, S=None, precision: int = APF_FP64):
        import torch
        if S is None:
            S = torch.empty((self.prob.n_out, self.prob.n_in), dtype=torch.complex128, device="cuda")
        assert S.dtype == torch.complex128 and S.is_contiguous()
        _check(self._lib.apf_factor_schur(self._h, precision, _ptr(S), _stream()))
        return S

    def weighted_power(self, S, w):
        import torch
        f = torch.empty((), dtype=torch.float64, device=S.device)
        G = torch.empty_like(S)
        assert w.dtype == torch.float64 and w.is_contiguous() and S.is_contiguous()
        _check(self._lib.apf_weighted_power(self._h, _ptr(S), _ptr(w), _ptr(f), _ptr(G), _stream()))
        return f, G

    def splitter_fom(self, S, t1: float = 0.5):
        """Eq. (5) figure of merit and dF/dS (device tensors)."""
        import torch
        assert S.dtype == torch.complex128 and S.is_contiguous()
        f = torch.empty((), dtype=torch.float64, device=S.device)
        G = torch.empty_like(S)
        _check(self._lib.apf_splitter_fom(self._h, _ptr(S), float(t1), _ptr(f), _ptr(G), _stream()))
        return f, G

    def group_fom(self, S, delta: int, gmax: int = 2):
        """Grouped multi-angle objective and dF/dS (device tensors)."""
        import torch
        assert S.dtype == torch.complex128 and S.is_contiguous()
        f = torch.empty((), dtype=torch.float64, device=S.device)
        G = torch.empty_like(S)
        _check(self._lib.apf_group_fom(self._h, _ptr(S), int(delta), int(gmax), _ptr(f), _ptr(G), _stream()))
        return f, G

    def ridges_eps(self, edges, eps, mirror: bool, eps_ridge: float, eps_gap: float):
        """Writes the design rows of eps ([ny][nx] float64, device) from the
        edge positions (float64 device tensor, grid units)."""
        import torch
        assert edges.dtype == torch.float64 and edges.is_contiguous() and edges.is_cuda
        assert eps.dtype == torch.float64 and eps.is_contiguous() and tuple(eps.shape) == (self.prob.ny, self.prob.nx)
        _check(self._lib.apf_ridges_eps(self._h, _ptr(edges), edges.numel(), int(mirror), float(eps_ridge),
                                        float(eps_gap), _ptr(eps), _stream()))
        return eps

    def ridges_grad(self, edges, grad_eps, mirror: bool, eps_ridge: float, eps_gap: float):
        """df/d(edges) from df/deps of the design rows."""
        import torch
        assert edges.dtype == torch.float64 and edges.is_contiguous() and edges.is_cuda
        assert grad_eps.dtype == torch.float64 and grad_eps.is_contiguous()
        assert tuple(grad_eps.shape) == (self.prob.n_design_rows, self.prob.nx)
        out = torch.empty_like(edges)
        _check(self._lib.apf_ridges_grad(self._h, _ptr(edges), edges.numel(), int(mirror), float(eps_ridge),
                                         float(eps_gap), _ptr(grad_eps), _ptr(out), _stream()))
        return out

    def grad(self, dfdS, out=None):
        import torch
        assert dfdS.dtype == torch.complex128 and dfdS.is_contiguous()
        if out is None:
            out = torch.empty((self.prob.n_design_rows, self.prob.nx), dtype=torch.float64, device=dfdS.device)
        _check(self._lib.apf_grad(self._h, _ptr(dfdS), _ptr(out), _stream()))
        return out

    def grad_augmented(self, dfdS, col_pixel, col_sigma, param_begin, n_sub: int = 0, skip_uu: bool = False,
                       want_S: bool = False):
        """df/dp for dA/dp_k = U_k Sigma_k U_k^T by the parameter-augmented
        factorization with n_sub sub-factorizations (0: chosen from the sizes).
        col_pixel / col_sigma / param_begin: host arrays (see apf.h).
        Returns (dfdp, S or None, n_sub used)."""
        import torch
        assert dfdS.dtype == torch.complex128 and dfdS.is_contiguous()
        pix = np.ascontiguousarray(col_pixel, dtype=np.int32)
        sig = np.ascontiguousarray(col_sigma, dtype=np.float64)
        pb = np.ascontiguousarray(param_begin, dtype=np.int32)
        assert pix.size == sig.size and pb.size >= 2
        out = torch.empty(pb.size - 1, dtype=torch.float64, device=dfdS.device)
        S = torch.empty_like(dfdS) if want_S else None
        used = ctypes.c_int32()
        _check(self._lib.apf_grad_augmented(
            self._h, pix.size, pix.ctypes.data_as(ctypes.c_void_p), sig.ctypes.data_as(ctypes.c_void_p),
            pb.size - 1, pb.ctypes.data_as(ctypes.c_void_p), int(n_sub), APF_AUG_SKIP_UU if skip_uu else 0,
            _ptr(dfdS), _ptr(S) if S is not None else None, _ptr(out), ctypes.byref(used), _stream()))
        return out, S, used.value

    def ridges_grad_augmented(self, edges, dfdS, mirror: bool, eps_ridge: float, eps_gap: float, n_sub: int = 0,
                              skip_uu: bool = False):
        """df/d(edges) by the parameter-augmented factorization (U_k: the
        cells of edge k and of its mirror image on every design row).
        Returns (dfdp, n_sub used)."""
        import torch
        assert edges.dtype == torch.float64 and edges.is_contiguous() and edges.is_cuda
        assert dfdS.dtype == torch.complex128 and dfdS.is_contiguous()
        out = torch.empty_like(edges)
        used = ctypes.c_int32()
        _check(self._lib.apf_ridges_grad_augmented(
            self._h, _ptr(edges), edges.numel(), int(mirror), float(eps_ridge), float(eps_gap), int(n_sub),
            APF_AUG_SKIP_UU if skip_uu else 0, _ptr(dfdS), None, _ptr(out), ctypes.byref(used), _stream()))
        return out, used.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.apf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def weighted_power_noalloc(S, w, f=None, G=None):
    """f = sum w |S|^2 and dF/dS = w conj(S) through the allocation-free entry
    point (no handle; the outputs are the caller's: pass f and G to keep the
    call free of allocations)."""
    import torch
    lib = load_library()
    assert S.dtype == torch.complex128 and S.is_contiguous() and w.dtype == torch.float64 and w.is_contiguous()
    assert S.numel() == w.numel()
    if f is None:
        f = torch.empty((), dtype=torch.float64, device=S.device)
    if G is None:
        G = torch.empty_like(S)
    _check(lib.apf_weighted_power_noalloc(_ptr(S), _ptr(w), S.numel(), _ptr(f), _ptr(G), _stream()))
    return f, G


def autotune(apfs, reps: int = 3, save_path: Optional[str] = None):
    """Time the GEMM lists of the plan these handles run (one handle: its
    factorization and gradient; several: their batched factorization) in each
    kernel form, apply the fastest per bucket and optionally save the table."""
    lib = load_library()
    hs = (ctypes.c_void_p * len(apfs))(*[a._h.value for a in apfs])
    _check(lib.apf_autotune(hs, len(apfs), int(reps), save_path.encode() if save_path else None, _stream()))


# internal GEMM task flags the kernel test hook accepts (values of the
# library's task format)
GEMM_FLAGS = dict(TRANS_A=1, NEG=2, CIN=4, B_COFF=8, CIN_COFF=16, B_EXT=32, A_TRI_L=128, A_TRI_U=256,
                  B_TRI_L=512, B_TRI_U=1024, CIN_OWN=8192, C_ACC=16384, K_LIM=65536, ACC_CHUNK=131072,
                  C_COFF=524288, CIN_RANGE=1048576, CONTRACT=2048, NO_STORE=4096)
EXT_ADD = 1 << 30


def gemm_hook(form, flags, M, N, K, A, lda, B, ldb, C, ldc, Cin=None, ldcin=0, b_offset=0, browmap=None,
              crowmap=None, ccolmap=None, cin_c0=0, cin_w=0, coff=0, nlim=1 << 30, xcd=False, aux=None,
              auxmap=None, part=None, pstride=0):
    """Kernel test hook: one GEMM of the internal task format on kernel form
    `form` (see apf_test_gemm in include/apf.h); tensors on the GPU (complex128
    operands, int32 maps, float64 partials)."""
    lib = load_library()
    p = lambda t: None if t is None else _ptr(t)
    _check(lib.apf_test_gemm(int(form), int(flags), int(M), int(N), int(K), _ptr(A), int(lda), _ptr(B), int(ldb),
                             int(b_offset), p(Cin), int(ldcin), _ptr(C), int(ldc), p(browmap), p(crowmap), p(ccolmap),
                             int(cin_c0), int(cin_w), int(coff), int(nlim), 1 if xcd else 0, p(aux), p(auxmap),
                             p(part), int(pstride), _stream()))


def pivot_block_hook(F, tri, perm, sym=False):
    """Kernel test hook: the pivot-block kernel on one p x p block (device
    tensors: F, tri complex128 [p][p], perm int32 [p]; sym: the symmetric
    mode, lower triangle of F read, no row exchanges); returns the pivot
    spread (raises APFError with APF_ESINGULAR for a singular block)."""
    lib = load_library()
    q = ctypes.c_double(0.0)
    _check(lib.apf_test_pivot_block(int(F.shape[0]), _ptr(F), _ptr(tri), _ptr(perm), ctypes.byref(q),
                                    1 if sym else 0, _stream()))
    return q.value


def tuning_apply(apfs, path: str):
    """Apply a saved autotune table to the plan these handles run."""
    lib = load_library()
    hs = (ctypes.c_void_p * len(apfs))(*[a._h.value for a in apfs])
    _check(lib.apf_tuning_apply(hs, len(apfs), path.encode(), _stream()))


def factor_schur_batched(apfs, S_list=None, precision: int = APF_FP64):
    """One batched partial factorization of several assembled problems.
    Returns the list of S tensors (complex128 [n_out][n_in] each)."""
    import torch
    lib = load_library()
    if S_list is None:
        S_list = [torch.empty((a.prob.n_out, a.prob.n_in), dtype=torch.complex128, device="cuda") for a in apfs]
    hs = (ctypes.c_void_p * len(apfs))(*[a._h.value for a in apfs])
    ss = (ctypes.c_void_p * len(apfs))(*[S.data_ptr() for S in S_list])
    _check(lib.apf_factor_schur_batched(hs, len(apfs), precision, ss, _stream()))
    return S_list


def solve(apf: APF, eps, precision: int = APF_FP64):
    """S = C A^-1 B for the permittivity map eps ([ny][nx] float64, device)."""
    apf.assemble(eps)
    return apf.factor_schur(precision=precision)


class StaleFactorsError(RuntimeError):
    """The handle was factorized again between an autograd forward and its
    backward, so its factors belong to another permittivity."""


def check_factor_epoch(apf, saved: int) -> None:
    """Raise StaleFactorsError unless `apf` has run exactly the factorizations
    counted in `saved` (its "n_factorizations" statistic at forward time)."""
    now = int(apf.query("n_factorizations"))
    if now != saved:
        raise StaleFactorsError(
            f"the APF handle was factorized {now - saved} more time(s) after this forward pass; its factors "
            f"no longer belong to the forward permittivity (use one handle per pending backward)")


def make_autograd_function():
    """torch.autograd.Function around the library: forward S(eps), backward
    grad_eps from the weighted adjoint of apf_grad.  torch hands backward
    grad_S = 2 conj(dF/dS) for a real loss (its convention for complex
    inputs), so the Wirtinger derivative passed to the library is
    conj(grad_S)/2.  apf_grad uses the factors the handle holds, so backward
    checks that no other factorization ran on the handle since this forward
    (StaleFactorsError otherwise)."""
    import torch

    class APFFunction(torch.autograd.Function):
        @staticmethod
        def forward(ctx, eps_design, apf: APF, eps_background, precision=APF_FP64):
            prob = apf.prob
            eps = eps_background.clone()
            eps[prob.design_row0:prob.design_row1] = eps_design
            apf.assemble(eps.contiguous())
            S = apf.factor_schur(precision=precision)
            ctx.apf = apf
            ctx.epoch = int(apf.query("n_factorizations"))
            return S

        @staticmethod
        def backward(ctx, grad_S):
            check_factor_epoch(ctx.apf, ctx.epoch)
            dfdS = (grad_S.conj() * 0.5).contiguous()
            g = ctx.apf.grad(dfdS)
            return g, None, None, None

    return APFFunction
