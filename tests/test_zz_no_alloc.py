"""The allocation-free objective entry point (apf_weighted_power_noalloc)
against apf_weighted_power through the C ABI: two calls in a row, the second
on a smaller S, each bitwise equal to the handle-based entry point (same
reduction order), and the host-side argument checks."""
import ctypes

import numpy as np
import pytest

from paper_2306_09257_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _handle_result(prob, eps, w_d):
    from paper_2306_09257_amd import binding
    apf = binding.APF(prob).analyze()
    apf.assemble(torch.as_tensor(eps, dtype=torch.float64, device="cuda"))
    S = apf.factor_schur()
    f, G = apf.weighted_power(S, w_d)
    return apf, S, f, G


def test_noalloc_objective_equals_the_handle_entry_point_twice_second_smaller():
    from paper_2306_09257_amd import binding
    lib = binding.load_library()
    big = inputs.tiny_problem(nx=130, ny=60, seed=31)        # 41 x 41 channels
    small = inputs.tiny_problem(nx=40, ny=60, seed=32)       # 11 x 11 channels
    results = []
    for prob, eps, w in (big, small):
        print(f"[gpu] noalloc objective on {prob.n_out}x{prob.n_in}", flush=True)
        w_d = torch.as_tensor(w, dtype=torch.float64, device="cuda")
        apf, S, f_ref, G_ref = _handle_result(prob, eps, w_d)
        f = torch.full((), float("nan"), dtype=torch.float64, device="cuda")
        G = torch.full_like(S, complex(float("nan"), float("nan")))
        st = lib.apf_weighted_power_noalloc(ctypes.c_void_p(S.data_ptr()), ctypes.c_void_p(w_d.data_ptr()),
                                            S.numel(), ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(G.data_ptr()),
                                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == binding.APF_OK, lib.apf_last_error()
        torch.cuda.synchronize()
        assert torch.equal(G, G_ref)
        assert float(f) == float(f_ref)
        # and against the plain definition on the host
        Sh, wh = S.cpu().numpy(), w
        assert abs(float(f) - float(np.sum(wh * np.abs(Sh) ** 2))) < 1e-13 * float(f)
        results.append(float(f))
    assert results[0] != results[1]


def test_noalloc_objective_rejects_bad_arguments_on_the_host():
    from paper_2306_09257_amd import binding
    lib = binding.load_library()
    buf = torch.zeros(4, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    for n in (0, -5, (1 << 40) + 1):
        assert lib.apf_weighted_power_noalloc(p, p, n, p, p, None) == binding.APF_EINVAL
    assert lib.apf_weighted_power_noalloc(None, p, 1, p, p, None) == binding.APF_EINVAL
    assert b"null" in lib.apf_last_error()
