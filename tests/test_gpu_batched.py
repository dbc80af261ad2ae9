"""Batched factorization of uneven problems (different grids, wavelengths
and channel counts) through apf_factor_schur_batched: every S must equal the
single-problem factorization bit for bit (the same kernels on the same data),
match the CPU FP64 oracle, and stay equal over repeated graph replays with
eager work in between."""
import numpy as np
import pytest

from paper_2306_09257_amd import inputs
import oracle.apf as oapf

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _assembled(items):
    from paper_2306_09257_amd import binding
    apfs = []
    for prob, eps, w in items:
        a = binding.APF(prob).analyze()
        a.assemble(torch.as_tensor(eps, dtype=torch.float64, device="cuda"))
        apfs.append(a)
    return apfs


def test_batched_equals_single_and_oracle():
    from paper_2306_09257_amd import binding
    items = inputs.batch_uneven(seed=3, count=6, nx_max=480, nx_step=120)
    print("[gpu] batch of", [(p.nx, p.ny, p.n_in) for p, _, _ in items], flush=True)
    apfs = _assembled(items)
    S_b = [S.cpu().numpy() for S in binding.factor_schur_batched(apfs)]
    for a, (prob, eps, w), Sb in zip(apfs, items, S_b):
        a.assemble(torch.as_tensor(eps, dtype=torch.float64, device="cuda"))
        S1 = a.factor_schur().cpu().numpy()
        assert np.array_equal(S1, Sb)
        So = oapf.scattering_matrix(prob, eps)
        assert np.linalg.norm(Sb - So) / np.linalg.norm(So) < 1e-10


def test_batched_graph_replays_match_eager_and_grad_follows():
    from paper_2306_09257_amd import binding
    items = inputs.batch_uneven(seed=5, count=4, nx_max=360, nx_step=120)
    apfs = _assembled(items)
    outs = [torch.empty((p.n_out, p.n_in), dtype=torch.complex128, device="cuda") for p, _, _ in items]
    # eager reference (profiling on disables capture)
    apfs[0].set_profiling(True)
    binding.factor_schur_batched(apfs, outs)
    apfs[0].set_profiling(False)
    ref = [S.cpu().numpy().copy() for S in outs]
    for rep in range(4):
        for S in outs:
            S.zero_()
        torch.cuda.synchronize()
        junk = torch.randn(1000, 1000, device="cuda") @ torch.randn(1000, 1000, device="cuda")
        binding.factor_schur_batched(apfs, outs)      # captured on the first pass, replayed after
        torch.cuda.synchronize()
        del junk
        for S, R in zip(outs, ref):
            assert np.array_equal(S.cpu().numpy(), R), f"replay {rep}"
    # the factors of each handle serve apf_grad afterwards
    for a, (prob, eps, w), S in zip(apfs, items, outs):
        f, G = a.weighted_power(S, torch.as_tensor(w, dtype=torch.float64, device="cuda"))
        g = a.grad(G).cpu().numpy()
        _, g_o, _ = oapf.solve_S_and_grad(prob, eps, w=w)
        assert np.linalg.norm(g - g_o) / np.linalg.norm(g_o) < 1e-10
