"""The parameter-augmented route of Sec. 2 (Eq. (4) with U divided into N_sub
sub-factorizations, Eq. (3) applied to each sub's blocks) through the C ABI:

* random parameterizations eps(p) = eps0 + sum_k p_k J_k on small grids,
  against the oracle's dense Eq. (4) route at 1e-10 for several N_sub, with
  and without the U^T A^-1 U block, and its S block against the oracle's S;
* the beam splitter (Sec. 3, Table S2 design, r_k = 48 pixels per mirrored
  edge, M_p = 3,840): the edge gradient equals the chain rule through the
  per-pixel gradient (apf_ridges_grad) and the oracle's edge gradient at
  1e-10, for N_sub = 1, 3 (the paper's choice) and the size-chosen one.
"""
import json
import os
import time

import numpy as np
import pytest

from paper_2306_09257_amd import inputs
import oracle.apf as oapf
import oracle.splitter as osp
from tests.parity import rel
from tests.test_oracle_pins import _param_spec

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


@pytest.mark.parametrize("nx,ny,dx,n_params", [(16, 60, 0.15, 7), (48, 92, 0.05, 12)])
def test_augmented_parameter_gradient_matches_the_oracle(nx, ny, dx, n_params):
    from paper_2306_09257_amd import binding
    prob, eps, w = inputs.tiny_problem(nx=nx, ny=ny, seed=41, dx_over_lambda=dx)
    rng = np.random.default_rng(9)
    pix, jac, pb = _param_spec(prob, rng, n_params=n_params)
    sigma = -prob.h ** 2 * jac
    print(f"[gpu] augmented {nx}x{ny}: {n_params} parameters, {pix.size} columns", flush=True)
    apf = binding.APF(prob).analyze()
    apf.assemble(_dev(eps))
    S = apf.factor_schur()
    f, G = apf.weighted_power(S, _dev(w))
    d_o, S_o = oapf.grad_augmented_params(prob, eps, G.cpu().numpy(), pix, sigma, pb, 1)
    for n_sub in (1, 3, 0):
        for skip in (False, True):
            d, S_aug, used = apf.grad_augmented(G, pix, sigma, pb, n_sub=n_sub, skip_uu=skip, want_S=True)
            d, S_aug = d.cpu().numpy(), S_aug.cpu().numpy()
            print(f"[gpu]   n_sub {n_sub} -> {used}, skip_uu {skip}: dfdp {rel(d, d_o):.2e}, S {rel(S_aug, S_o):.2e}",
                  flush=True)
            assert used == (n_sub if n_sub else used) and 1 <= used <= n_params
            assert rel(d, d_o) < TOL and rel(S_aug, S_o) < TOL
    # the handle's factors are valid afterwards: the plain gradient follows
    g = apf.grad(G).cpu().numpy()
    _, g_o, _ = oapf.solve_S_and_grad(prob, eps, w=w)
    assert rel(g, g_o) < TOL


def test_splitter_edge_gradient_by_the_augmented_route():
    from paper_2306_09257_amd import binding
    with open(os.path.join(GOLDEN, "splitter_table_s2.json")) as fh:
        gold = json.load(fh)
    prob = inputs.splitter_problem(1024)
    edges = inputs.splitter_edges_to_grid(gold["edges_um"], prob.nx)
    ER, EG = inputs.SPLITTER_EPS_RIDGE, inputs.SPLITTER_EPS_AIR
    print(f"[gpu] splitter {prob.nx}x{prob.ny}, {edges.size} free edges, augmented route", flush=True)
    apf = binding.APF(prob).analyze()
    e_d = _dev(edges)
    eps = _dev(prob.background_eps())
    apf.ridges_eps(e_d, eps, True, ER, EG)
    apf.assemble(eps)
    S = apf.factor_schur()
    f, G = apf.splitter_fom(S)
    g_eps = apf.grad(G)
    chain = apf.ridges_grad(e_d, g_eps, True, ER, EG).cpu().numpy()
    eps_o = osp.ridges_eps(prob.background_eps(), prob, edges, True, ER, EG)
    S_o = oapf.scattering_matrix(prob, eps_o)
    _, G_o = osp.fom(S_o, prob.in_orders, prob.out_orders)
    _, g_eps_o, _ = oapf.solve_S_and_grad(prob, eps_o, G=G_o)
    g_e_o = osp.edge_gradient(g_eps_o, edges, prob.nx, True, ER, EG)
    timings = {}
    for n_sub in (1, 3, 0):
        for skip in (False, True):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            d, used = apf.ridges_grad_augmented(e_d, G, True, ER, EG, n_sub=n_sub, skip_uu=skip)
            torch.cuda.synchronize()
            timings[(used, skip)] = time.perf_counter() - t0
            d = d.cpu().numpy()
            print(f"[gpu]   n_sub {n_sub} -> {used}, skip_uu {skip}: vs chain rule {rel(d, chain):.2e}, "
                  f"vs oracle {rel(d, g_e_o):.2e}, {1e3 * timings[(used, skip)]:.1f} ms", flush=True)
            assert rel(d, chain) < TOL and rel(d, g_e_o) < TOL
