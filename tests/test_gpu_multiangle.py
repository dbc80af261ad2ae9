"""Paper-scale multi-angle workload through the C ABI: 48000 x 160 grid
(7.68M unknowns), 4,559 x 4,559 channels, 1.92M design pixels; the right-hand
sides do not fit the sweep arrays at once, so the gradient runs in chunks.
Against values the CPU FP64 oracle wrote once
(tests/golden/make_multiangle_golden.py):

* two full columns of S;
* the grouped objective's derivative on those columns, formed on the GPU
  (apf_group_fom) from the GPU's S, against the oracle's from the oracle's S;
* the gradient for that derivative, at 2,000 seeded pixels and in 2-norm;
* the objective and its derivative over all of S, GPU kernel against the
  oracle formula applied to the same S; passivity of every column;

on the LU route and on the symmetric route.
"""
import os
import time

import numpy as np
import pytest

from paper_2306_09257_amd import inputs
import oracle.objectives as oobj
from tests.parity import worst_block, worst_block_sampled

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "multiangle_48000x160_seed2.npz")
TOL = 1e-10


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.mark.parametrize("route", ["lu", "symmetric"])
def test_multiangle_48000x160_against_oracle_samples(route):
    """On the default LU route (the 1e-10 bar; measured S 3.0e-13, gradient
    1.5e-12, worst blocks 9.5e-13 and 4.1e-12) and on the symmetric route
    (L D L^T pivot blocks without row exchanges), against the same
    oracle-written values.  The symmetric route loses about three digits on
    this workload (measured S 1.0e-10, gradient 1.1e-10, worst blocks
    4.0e-10 and 4.2e-10: some pivot blocks need the row exchanges it does
    without) and is held to 1e-9 only."""
    from paper_2306_09257_amd import binding
    gold = np.load(GOLDEN, allow_pickle=False)
    prob, eps, delta = inputs.metasurface_multiangle(seed=2)
    print(f"[gpu] multi-angle {prob.nx}x{prob.ny}, {prob.n_in} x {prob.n_out} channels, delta {delta}, "
          f"{route} route", flush=True)
    apf = binding.APF(prob).analyze().set_symmetric(route == "symmetric")
    dev = torch.device("cuda:0")
    apf.assemble(torch.as_tensor(eps, dtype=torch.float64, device=dev))
    S = apf.factor_schur()
    f, G_full = apf.group_fom(S, delta)
    torch.cuda.synchronize()
    cols = gold["cols"]
    G = torch.zeros_like(S)
    G[:, torch.as_tensor(cols, device=dev)] = G_full[:, torch.as_tensor(cols, device=dev)]
    t0 = time.perf_counter()
    g = apf.grad(G)
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    S_h, G_h, g_h = S.cpu().numpy(), G_full.cpu().numpy(), g.cpu().numpy()
    eS = _rel(S_h[:, cols], gold["S_cols"])
    eG = _rel(G_h[:, cols], gold["G_cols"])
    eg = _rel(g_h.ravel()[gold["pixels"]], gold["grad"])
    en = abs(np.linalg.norm(g_h) - float(gold["grad_norm"])) / float(gold["grad_norm"])
    eS_blk = worst_block(S_h[:, cols], gold["S_cols"], axis=0)
    eg_blk = worst_block_sampled(g_h.ravel()[gold["pixels"]], gold["grad"], gold["pixels"] % prob.nx, prob.nx)
    f_o, G_o = oobj.group_fom(S_h, prob.in_orders, prob.out_orders, delta)
    print(f"[gpu] rhs chunk {apf.query('rhs_chunk'):.0f}; rel err S columns {eS:.2e}, dF/dS columns {eG:.2e}, "
          f"sampled grad {eg:.2e}, grad norm {en:.2e}; objective kernel f {abs(float(f) - f_o) / abs(f_o):.2e}, "
          f"dF/dS {_rel(G_h, G_o):.2e}; worst blocks S {eS_blk:.2e}, grad {eg_blk:.2e}; gradient call "
          f"{t_grad:.2f} s", flush=True)
    print(f"[gpu] {route} route: smallest pivot spread {apf.query('pivot_spread_min'):.3e} "
          f"(front {apf.query('pivot_spread_front'):.0f})", flush=True)
    assert apf.query("rhs_chunk") < prob.n_in      # the chunked sweeps take part
    # the pivot spread tells a caller whether the factorization stayed safe:
    # measured 5.3e-4 with partial pivoting, 5.0e-10 without row exchanges
    spread = apf.query("pivot_spread_min")
    assert (spread > 1e-5) if route == "lu" else (0 < spread < 1e-6)
    tol = TOL if route == "lu" else 1e-9
    assert eS < tol and eG < tol and eg < tol and en < tol
    assert eS_blk < tol and eg_blk < tol
    assert abs(float(f) - f_o) < 1e-12 * abs(f_o) and _rel(G_h, G_o) < 1e-12
    flux = np.sum(np.abs(S_h) ** 2, axis=0)
    assert np.all(np.isfinite(S_h)) and flux.max() <= 1.0 + 1e-9
