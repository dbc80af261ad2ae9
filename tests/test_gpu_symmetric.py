"""The symmetric route (apf_set_symmetric: L D L^T pivot blocks, U12 and Z
as transposes, contribution blocks on their lower tiles) against the CPU
FP64 oracle on every small grid of the LU route's parity cases, at 240 x 92
and at 1200 x 92 with the low-rank sweep subtrees (1e-10 normwise and in
every column block); against the LU route at full size (24000 x 160, S and
the gradient over all 960,000 pixels); and the precisions and entry points
it does not combine with."""
import numpy as np
import pytest

from paper_2306_09257_amd import inputs
import oracle.apf as oapf
from tests.parity import worst_block
from tests.test_gpu_parity import CASES, _PROBLEM_KEYS, _check, _dev, _rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


def _run_sym(prob, eps, w, leaf=0, sym=True):
    from paper_2306_09257_amd import binding
    print(f"[gpu] symmetric={sym} nx={prob.nx} ny={prob.ny} n_in={prob.n_in} leaf={leaf}", flush=True)
    apf = binding.APF(prob, leaf_size=leaf).analyze().set_symmetric(sym)
    apf.assemble(_dev(eps, torch.float64))
    S = apf.factor_schur()
    f, G = apf.weighted_power(S, _dev(w, torch.float64))
    g = apf.grad(G)
    torch.cuda.synchronize()
    return apf, S.cpu().numpy(), g.cpu().numpy()


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c['nx']}x{c['ny']}-leaf{c['leaf']}")
def test_symmetric_route_matches_oracle_small(case):
    kw = {k: (np.asarray(v, np.int32) if isinstance(v, list) else v)
          for k, v in case.items() if k in _PROBLEM_KEYS}
    prob, eps, w = inputs.tiny_problem(nx=case["nx"], ny=case["ny"], seed=case["seed"], **kw)
    apf, S, g = _run_sym(prob, eps, w, case["leaf"])
    S_o, g_o, f_o = oapf.solve_S_and_grad(prob, eps, w=w)
    _check(S, g, S_o, g_o, f"symmetric {prob.nx}x{prob.ny}")
    assert apf.query("pivot_spread_min") > 0


def test_symmetric_route_240x92_and_its_work_count():
    """240 x 92 against the oracle; the executed factorization MACs of the
    symmetric plan are below the LU plan's (U12, Z and the upper
    contribution tiles are not formed)."""
    prob, eps, w = inputs.metasurface_small(seed=0)
    apf, S, g = _run_sym(prob, eps, w)
    S_o, g_o, _ = oapf.solve_S_and_grad(prob, eps, w=w)
    _check(S, g, S_o, g_o, "symmetric 240x92")
    lu, _, _ = _run_sym(prob, eps, w, sym=False)
    c_sym, c_lu = apf.query("gemm_cmacs_factor"), lu.query("gemm_cmacs_factor")
    print(f"[gpu] factorization complex MACs: symmetric {c_sym:.3e}, LU {c_lu:.3e}", flush=True)
    assert 0 < c_sym < c_lu


def test_symmetric_route_with_low_rank_subtrees_1200x92():
    prob = inputs.make_problem(1200, 92)
    rng = np.random.default_rng(11)
    eps = inputs.eps_binary_smoothed(prob, rng)
    w = inputs.weights_uniform(prob, rng)
    apf, S, g = _run_sym(prob, eps, w)
    assert apf.query("lowrank_roots") > 0
    S_o, g_o, _ = oapf.solve_S_and_grad(prob, eps, w=w)
    _check(S, g, S_o, g_o, "symmetric 1200x92 low-rank subtrees")


def test_symmetric_route_runs_in_fp64_only():
    """APF_MIXED on a symmetric handle is refused: measured before the
    refusal, its unpivoted blocks amplified the FP32 rounding to S 3.8e-5 and
    gradient 1.5e-4 against the oracle at 240 x 92 (LU route: 1.2e-6 and
    8.4e-6).  The handle still factors in FP64 afterwards."""
    from paper_2306_09257_amd import binding
    prob, eps, w = inputs.metasurface_small(seed=0)
    apf = binding.APF(prob).analyze().set_symmetric(True)
    apf.assemble(_dev(eps, torch.float64))
    with pytest.raises(binding.APFError) as ei:
        apf.factor_schur(precision=binding.APF_MIXED)
    assert ei.value.status == binding.APF_EINVAL
    S = apf.factor_schur().cpu().numpy()
    S_o = oapf.scattering_matrix(prob, eps)
    assert _rel(S, S_o) < TOL


def test_symmetric_route_refuses_batches_the_augmented_route_and_refinement():
    from paper_2306_09257_amd import binding
    prob, eps, w = inputs.tiny_problem(nx=24, ny=60, seed=0)
    apf = binding.APF(prob).analyze().set_symmetric(True)
    apf.assemble(_dev(eps, torch.float64))
    with pytest.raises(binding.APFError) as ei:
        binding.factor_schur_batched([apf])
    assert ei.value.status == binding.APF_EINVAL
    other = binding.APF(prob).analyze()
    other.assemble(_dev(eps, torch.float64))
    with pytest.raises(binding.APFError) as ei:
        binding.autotune([apf, other], reps=1)
    assert ei.value.status == binding.APF_EINVAL
    dfdS = torch.zeros((prob.n_out, prob.n_in), dtype=torch.complex128, device="cuda")
    with pytest.raises(binding.APFError) as ei:
        apf.grad_augmented(dfdS, [0, 1], [-1.0, -1.0], [0, 2])
    assert ei.value.status == binding.APF_EINVAL
    with pytest.raises(binding.APFError) as ei:
        apf.factor_schur(precision=binding.APF_MIXED_REFINED)
    assert ei.value.status in (binding.APF_EINVAL, binding.APF_ESTATE)


def test_symmetric_and_lu_routes_agree_at_full_size():
    """24000 x 160 (3.84M unknowns, 2,399 x 2,399 channels): S and the
    gradient over all 960,000 pixels of the symmetric route against the LU
    route's, normwise and in every column block, within 1e-10."""
    prob, eps, w = inputs.metasurface_wide(seed=1)
    res = {}
    for sym in (True, False):
        apf, S, g = _run_sym(prob, eps, w, sym=sym)
        res[sym] = (S, g, apf.query("gemm_cmacs_factor"))
        apf.close()
        torch.cuda.empty_cache()
    (S1, g1, c1), (S0, g0, c0) = res[True], res[False]
    eS, eS_blk = _rel(S1, S0), worst_block(S1, S0, axis=1)
    eg, eg_blk = _rel(g1, g0), worst_block(g1, g0, axis=1)
    print(f"[gpu] full size symmetric vs LU: S {eS:.2e} (worst block {eS_blk:.2e}), grad {eg:.2e} "
          f"(worst block {eg_blk:.2e}); factorization complex MACs {c1:.3e} vs {c0:.3e}", flush=True)
    assert eS < TOL and eS_blk < TOL and eg < TOL and eg_blk < TOL
    assert c1 < c0


def test_symmetric_route_without_sweep_data_and_with_plain_sweeps():
    """The symmetric route with the plan for S only (no sweep data: no X12,
    no Z transposes) and with the low-rank subtrees forbidden (every sweep
    front reads its Z, the transpose of X12) against the oracle at 1200 x 92."""
    from paper_2306_09257_amd import binding
    prob = inputs.make_problem(1200, 92)
    rng = np.random.default_rng(11)
    eps = inputs.eps_binary_smoothed(prob, rng)
    w = inputs.weights_uniform(prob, rng)
    S_o, g_o, _ = oapf.solve_S_and_grad(prob, eps, w=w)
    a = binding.APF(prob).analyze().set_symmetric(True).set_gradient(False)
    a.assemble(_dev(eps, torch.float64))
    S = a.factor_schur().cpu().numpy()
    eS = _rel(S, S_o)
    print(f"[gpu] symmetric 1200x92, S only: S {eS:.2e}", flush=True)
    assert eS < TOL and worst_block(S, S_o, axis=1) < TOL
    a.close()
    b = binding.APF(prob).analyze().set_symmetric(True).set_lowrank(0)
    b.assemble(_dev(eps, torch.float64))
    S = b.factor_schur()
    f, G = b.weighted_power(S, _dev(w, torch.float64))
    g = b.grad(G)
    torch.cuda.synchronize()
    assert b.query("lowrank_roots") == 0
    _check(S.cpu().numpy(), g.cpu().numpy(), S_o, g_o, "symmetric 1200x92 plain sweeps")
