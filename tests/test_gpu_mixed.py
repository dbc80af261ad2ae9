"""The APF_MIXED precision option (front GEMMs and sweeps on FP32 MFMA, FP64
storage, pivot blocks and reductions, no refinement): it must run through
the single and the batched entry points with identical results, and stay
within the accuracy measured for it.  Measured relative errors against the
FP64 oracle: ~1e-3 (S) and ~1e-2 (gradient) on the 240 x 92 random-eps
problem, where nearly singular pivot blocks amplify FP32 rounding; ~1e-4
against the FP64 path at 24000 x 160."""
import numpy as np
import pytest

from paper_2306_09257_amd import inputs
import oracle.apf as oapf

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_mixed_single_and_batched_agree_and_are_near_the_oracle():
    from paper_2306_09257_amd import binding
    items = [inputs.tiny_problem(nx=48, ny=60, seed=21), inputs.metasurface_small(seed=0)]
    apfs = []
    for prob, eps, w in items:
        a = binding.APF(prob).analyze()
        a.assemble(torch.as_tensor(eps, dtype=torch.float64, device="cuda"))
        apfs.append(a)
    Sb = [S.cpu().numpy() for S in binding.factor_schur_batched(apfs, precision=binding.APF_MIXED)]
    for a, (prob, eps, w), S_b in zip(apfs, items, Sb):
        a.assemble(torch.as_tensor(eps, dtype=torch.float64, device="cuda"))
        S = a.factor_schur(precision=binding.APF_MIXED)
        f, G = a.weighted_power(S, torch.as_tensor(w, dtype=torch.float64, device="cuda"))
        g = a.grad(G).cpu().numpy()
        S = S.cpu().numpy()
        assert np.array_equal(S, S_b)
        S_o, g_o, _ = oapf.solve_S_and_grad(prob, eps, w=w)
        eS, eg = _rel(S, S_o), _rel(g, g_o)
        print(f"[gpu] mixed {prob.nx}x{prob.ny}: rel err S {eS:.2e} grad {eg:.2e}", flush=True)
        assert np.isfinite(S).all() and np.isfinite(g).all()
        assert eS < 5e-3 and eg < 5e-2
