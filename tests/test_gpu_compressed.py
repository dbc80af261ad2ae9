"""B/C compression through the C ABI (Supplement Sec. 1, this library's
reading): the compressed factorization's S against the oracle's compressed
route (same padding, window and truncation) at 1e-10, and, with nothing
truncated, against the plain oracle S at 1e-10; its distance from the
uncompressed S at the paper's window; the gradient over the compressed
channels (Eq. (3) with dF/dS~ = D_C^T dF/dS D_B^T) against the oracle's
compressed route at 1e-10, with chunked sweeps and both low-rank depths; the
state and argument checks."""
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
    # without the gradient sweeps: the same S, and apf_grad is refused
    nog = binding.APF(prob).analyze().set_compression(4, 3.0).set_gradient(False)
    nog.assemble(_dev(eps))
    S_n = nog.factor_schur()
    assert nog.query("n_sweep_rows") == 0 and nog.query("n_sweep_rows") < apf.query("n_sweep_rows")
    assert torch.equal(S_n, S)
    f, G = nog.weighted_power(S_n, _dev(w))
    with pytest.raises(binding.APFError) as ei:
        nog.grad(G)
    assert ei.value.status == binding.APF_ESTATE
    # switched off again before the plan: the plain path, gradient included
    plain = binding.APF(prob).analyze().set_compression(4, 3.0).set_compression(-1, 0.0)
    plain.assemble(_dev(eps))
    S2 = plain.factor_schur()
    f2, G2 = plain.weighted_power(S2, _dev(w))
    S_o, g_o, _ = oapf.solve_S_and_grad(prob, eps, w=w)
    assert rel(S2.cpu().numpy(), S_o) < TOL and rel(plain.grad(G2).cpu().numpy(), g_o) < TOL


@pytest.mark.parametrize("nx,ny,pad,window,chunk,lowrank", [(64, 60, 6, 3.0, 0, 1), (240, 92, 24, 3.0, 0, 1),
                                                           (130, 60, 7, 2.0, 0, 0), (480, 92, 20, 8.0, 64, 2),
                                                           (960, 92, 40, 3.0, 64, 1)])
def test_compressed_gradient_matches_the_oracle_route(nx, ny, pad, window, chunk, lowrank):
    from paper_2306_09257_amd import binding
    prob = inputs.make_problem(nx, ny)
    rng = np.random.default_rng(nx + 1)
    eps = inputs.eps_binary_smoothed(prob, rng)
    w = rng.uniform(0.0, 1.0, size=(prob.n_out, prob.n_in))
    half_px = 0.5 * window / prob.dx_over_lambda
    S_oc = oc.scattering_matrix_compressed(prob, eps, pad, half_px)
    G = w * np.conj(S_oc)
    print(f"[gpu] compressed gradient {nx}x{ny}, {prob.n_in} channels, pad {pad}, window {window}, chunk {chunk}, "
          f"low-rank {lowrank}", flush=True)
    apf = binding.APF(prob).analyze().set_compression(pad, window).set_rhs_chunk(chunk).set_lowrank(lowrank)
    apf.assemble(_dev(eps))
    S = apf.factor_schur()
    g = apf.grad(torch.as_tensor(G, dtype=torch.complex128, device="cuda")).cpu().numpy()
    S_o2, g_oc = oc.grad_compressed(prob, eps, G, pad, half_px)
    _, g_plain, _ = oapf.solve_S_and_grad(prob, eps, G=G)
    print(f"[gpu]   S {rel(S.cpu().numpy(), S_oc):.2e}; gradient vs oracle compressed {rel(g, g_oc):.2e} "
          f"(worst column block {worst_block(g, g_oc, axis=1):.2e}), compressed vs plain oracle gradient "
          f"{rel(g_oc, g_plain):.2e}; rhs chunk {apf.query('rhs_chunk'):.0f}", flush=True)
    assert rel(S_o2, S_oc) < 1e-13
    if chunk:
        assert apf.query("rhs_chunk") < pad + prob.n_in
    assert rel(g, g_oc) < TOL and worst_block(g, g_oc, axis=1) < TOL


def test_mixed_precision_with_compression_stays_near_the_fp64_compressed_route():
    """APF_MIXED on a compressed handle: the S~ blocks run on FP32 MFMA like
    every front GEMM, the decompression stays FP64; S and the gradient stay
    within the mixed path's accuracy of the FP64 compressed result (the
    bound is that of the uncompressed mixed path at 24000 x 160, 3.4e-5 for S
    and 1.7e-4 for the gradient against FP64, with a margin; measured here
    9.5e-6 and 1.4e-4)."""
    from paper_2306_09257_amd import binding
    prob = inputs.make_problem(480, 92)
    rng = np.random.default_rng(7)
    eps = inputs.eps_binary_smoothed(prob, rng)
    w = rng.uniform(0.0, 1.0, size=(prob.n_out, prob.n_in))
    apf = binding.APF(prob).analyze().set_compression(20, 6.0)
    apf.assemble(_dev(eps))
    S64 = apf.factor_schur(precision=binding.APF_FP64)
    f64, G64 = apf.weighted_power(S64, _dev(w))
    g64 = apf.grad(G64).cpu().numpy()
    apf.assemble(_dev(eps))
    S32 = apf.factor_schur(precision=binding.APF_MIXED)
    f32, G32 = apf.weighted_power(S32, _dev(w))
    g32 = apf.grad(G32).cpu().numpy()
    eS, eg = rel(S32.cpu().numpy(), S64.cpu().numpy()), rel(g32, g64)
    print(f"[gpu] compressed 480x92, mixed against FP64: S {eS:.2e}, gradient {eg:.2e}", flush=True)
    assert eS < 5e-5 and eg < 5e-4
