"""B/C compression through the C ABI (Supplement Sec. 1, this library's
reading): the compressed factorization's S against the oracle's compressed
route (same padding, window and truncation) at 1e-10, and, with nothing
truncated, against the plain oracle S at 1e-10; its distance from the
uncompressed S at the paper's window; the state and argument checks."""
import numpy as np
import pytest

from paper_2306_09257_amd import inputs
import oracle.apf as oapf
import oracle.compress as oc
from tests.parity import rel, worst_block

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _gpu_S(prob, eps, pad, window, leaf=0):
    from paper_2306_09257_amd import binding
    apf = binding.APF(prob, leaf_size=leaf).analyze().set_compression(pad, window)
    apf.assemble(_dev(eps))
    S = apf.factor_schur().cpu().numpy()
    return apf, S


@pytest.mark.parametrize("nx,ny,pad,window,leaf", [(64, 60, 6, 3.0, 0), (240, 92, 10, 3.0, 0), (480, 92, 20, 6.0, 16),
                                                   (130, 60, 7, 2.0, 128)])
def test_compressed_S_matches_the_oracle_route(nx, ny, pad, window, leaf):
    prob = inputs.make_problem(nx, ny)
    rng = np.random.default_rng(nx)
    eps = inputs.eps_binary_smoothed(prob, rng)
    print(f"[gpu] compressed {nx}x{ny}, {prob.n_in} channels, pad {pad}, window {window}", flush=True)
    _, S = _gpu_S(prob, eps, pad, window, leaf)
    half_px = 0.5 * window / prob.dx_over_lambda
    S_oc = oc.scattering_matrix_compressed(prob, eps, pad, half_px)
    S_o = oapf.scattering_matrix(prob, eps)
    print(f"[gpu]   vs oracle compressed {rel(S, S_oc):.2e} (worst column block {worst_block(S, S_oc, axis=1):.2e}); "
          f"compression error {rel(S_oc, S_o):.2e}", flush=True)
    assert rel(S, S_oc) < TOL and worst_block(S, S_oc, axis=1) < TOL


def test_untruncated_compression_gives_the_plain_S():
    prob = inputs.make_problem(240, 92)
    rng = np.random.default_rng(5)
    eps = inputs.eps_binary_smoothed(prob, rng)
    _, S = _gpu_S(prob, eps, 8, 2.0 * prob.nx * prob.dx_over_lambda)     # window wider than the period
    S_o = oapf.scattering_matrix(prob, eps)
    print(f"[gpu] untruncated compression vs plain oracle {rel(S, S_o):.2e}", flush=True)
    assert rel(S, S_o) < TOL


def test_compression_state_and_argument_checks():
    from paper_2306_09257_amd import binding
    prob, eps, w = inputs.tiny_problem(nx=64, ny=60, seed=3)
    fresh = binding.APF(prob)
    with pytest.raises(binding.APFError) as ei:
        fresh.set_compression(4, 3.0)                  # before the analysis
    assert ei.value.status == binding.APF_ESTATE
    apf = binding.APF(prob).analyze()
    for bad in ((-2, 3.0), (4, 0.0), (4, float("nan")), (4, 0.01)):
        with pytest.raises(binding.APFError) as ei:
            apf.set_compression(*bad)
        assert ei.value.status == binding.APF_EINVAL
    gap = binding.APF(inputs.make_problem(64, 60, in_orders=np.array([-2, 0, 1], np.int32))).analyze()
    with pytest.raises(binding.APFError) as ei:
        gap.set_compression(4, 3.0)                    # non-consecutive orders
    assert ei.value.status == binding.APF_EINVAL
    apf.set_compression(4, 3.0)
    apf.assemble(_dev(eps))
    with pytest.raises(binding.APFError) as ei:
        apf.set_compression(-1, 0.0)                   # after the first assembly
    assert ei.value.status == binding.APF_ESTATE
    S = apf.factor_schur()
    f, G = apf.weighted_power(S, _dev(w))
    with pytest.raises(binding.APFError) as ei:
        apf.grad(G)
    assert ei.value.status == binding.APF_EINVAL
    # switched off again before the plan: the plain path, gradient included
    plain = binding.APF(prob).analyze().set_compression(4, 3.0).set_compression(-1, 0.0)
    plain.assemble(_dev(eps))
    S2 = plain.factor_schur()
    f2, G2 = plain.weighted_power(S2, _dev(w))
    S_o, g_o, _ = oapf.solve_S_and_grad(prob, eps, w=w)
    assert rel(S2.cpu().numpy(), S_o) < TOL and rel(plain.grad(G2).cpu().numpy(), g_o) < TOL
