"""Differentiation in the loop on the 12,000 x 140 workload (1.68M unknowns,
1,199 x 1,199 channels, 480,000 design pixels), through the autograd
Function over the C ABI:

* the initial design against values the CPU FP64 oracle wrote once
  (tests/golden/make_design_loop_golden.py): two columns of S and the
  gradient for dF/dS supported on those two inputs, at 2,000 seeded pixels
  and in 2-norm over all pixels;
* 200 Adam steps (learning rate 0.02, eps clipped to [1, 4] after each step)
  that raise f = sum w |S|^2; every 20 steps the adjoint gradient at 32
  seeded pixels is compared with finite differences of f evaluated on the
  GPU FP64 path.

Finite differences.  The fourth-order central difference
  (8 [f(x+h) - f(x-h)] - [f(x+2h) - f(x-2h)]) / (12 h),  h = 1e-2,
has a truncation error of order h^4 |f^(5)| / 30 and a rounding error of
about 3 e_f / (2 h), e_f being the absolute rounding error of one evaluation
of f (measured here: e_f ~ 5e-12, i.e. 1e-14 |f|, from the FD error at
h = 1e-3).  That floor, ~5e-10 per pixel, is absolute, while the gradient
shrinks as the optimisation converges (|dF/deps| per pixel falls from ~3e-3
to ~4e-5 over the 200 steps).  The check therefore bounds the error of the
32 sampled entries by 1e-6 of max(|g_32|, |g_32 at step 0|): strictly
relative at the start, relative to the initial gradient scale later.  The
plain central difference at h = 1e-6 is rounding-limited (e_f / h ~ 5e-6 per
pixel, ~1e-5 of the initial gradient) and is checked at the start at 1e-4.
"""
import os

import numpy as np
import pytest

from paper_2306_09257_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "design_loop_12000x140_seed4.npz")
TOL_ORACLE = 1e-10
TOL_FD = {"4th-order h=1e-2": 1e-6, "central h=1e-6": 1e-4}


def _f_of(apf, eps_full, w_d):
    apf.assemble(eps_full)
    S = apf.factor_schur()
    f, _ = apf.weighted_power(S, w_d)
    return float(f)


def test_design_loop_12000x140_initial_design_against_oracle():
    from paper_2306_09257_amd import binding
    gold = np.load(GOLDEN, allow_pickle=False)
    prob, eps, w = inputs.design_loop(seed=4)
    print(f"[gpu] design loop {prob.nx}x{prob.ny}, {prob.n_in} channels: oracle samples", flush=True)
    apf = binding.APF(prob).analyze()
    dev = torch.device("cuda:0")
    apf.assemble(torch.as_tensor(eps, dtype=torch.float64, device=dev))
    S = apf.factor_schur()
    cols = gold["cols"]
    G = torch.zeros((prob.n_out, prob.n_in), dtype=torch.complex128, device=dev)
    G[:, torch.as_tensor(cols, device=dev)] = torch.as_tensor(gold["G_cols"], device=dev)
    g = apf.grad(G).cpu().numpy()
    S_h = S.cpu().numpy()
    eS = np.linalg.norm(S_h[:, cols] - gold["S_cols"]) / np.linalg.norm(gold["S_cols"])
    eg = np.linalg.norm(g.ravel()[gold["pixels"]] - gold["grad"]) / np.linalg.norm(gold["grad"])
    en = abs(np.linalg.norm(g) - float(gold["grad_norm"])) / float(gold["grad_norm"])
    print(f"[gpu] rel err S columns {eS:.2e}, sampled grad {eg:.2e}, grad norm {en:.2e}", flush=True)
    assert eS < TOL_ORACLE and eg < TOL_ORACLE and en < TOL_ORACLE


def test_design_loop_12000x140_adam_with_finite_difference_checks():
    from paper_2306_09257_amd import binding
    prob, eps, w = inputs.design_loop(seed=4)
    dev = torch.device("cuda:0")
    apf = binding.APF(prob).analyze()
    Fn = binding.make_autograd_function()
    r0, r1 = prob.design_row0, prob.design_row1
    eps_bg = torch.as_tensor(eps, dtype=torch.float64, device=dev)
    w_d = torch.as_tensor(w, dtype=torch.float64, device=dev)
    x = torch.as_tensor(eps[r0:r1], dtype=torch.float64, device=dev).clone().requires_grad_(True)
    opt = torch.optim.Adam([x], lr=0.02)
    pix = np.random.default_rng(7).choice(x.numel(), size=32, replace=False)
    f_hist, fd_err, g_ref = [], [], None
    for step in range(200):
        opt.zero_grad()
        S = Fn.apply(x, apf, eps_bg)
        f = (w_d * S.abs() ** 2).sum()
        (-f).backward()
        f_hist.append(float(f.detach()))
        if step % 20 == 0:
            g_adj = (-x.grad).flatten()[torch.as_tensor(pix, device=dev)].cpu().numpy()
            base = eps_bg.clone()
            base[r0:r1] = x.detach()
            kinds = ["4th-order h=1e-2"] + (["central h=1e-6"] if step == 0 else [])
            for kind in kinds:
                g_fd = np.empty(pix.size)
                for n, p in enumerate(pix):
                    i, j = divmod(int(p), prob.nx)

                    def f_at(d):
                        e = base.clone()
                        e[r0 + i, j] += d
                        return _f_of(apf, e, w_d)

                    if kind.startswith("4th"):
                        h = 1e-2
                        g_fd[n] = (8 * (f_at(h) - f_at(-h)) - (f_at(2 * h) - f_at(-2 * h))) / (12 * h)
                    else:
                        h = 1e-6
                        g_fd[n] = (f_at(h) - f_at(-h)) / (2 * h)
                if g_ref is None:
                    g_ref = float(np.linalg.norm(g_adj))
                err = float(np.linalg.norm(g_fd - g_adj) / max(np.linalg.norm(g_adj), g_ref))
                fd_err.append((step, kind, err))
                print(f"[gpu] step {step} f {f_hist[-1]:.6f} FD {kind}: err {err:.2e} "
                      f"(|g_32| {np.linalg.norm(g_adj):.3e}, max abs err {np.abs(g_fd - g_adj).max():.3e})",
                      flush=True)
        opt.step()
        with torch.no_grad():
            x.clamp_(1.0, 4.0)
    print(f"[gpu] f: {f_hist[0]:.6f} -> {f_hist[-1]:.6f}", flush=True)
    for step, kind, err in fd_err:
        assert err < TOL_FD[kind], (step, kind, err)
    assert f_hist[-1] > f_hist[0]
