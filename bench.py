#!/usr/bin/env python3
"""APF solves per second (S and the full permittivity gradient) on one MI355X.

One step = assemble A from eps + multifrontal partial factorization of
K = [A, B; C, 0] giving S + objective f = sum w|S|^2 and its Wirtinger
derivative + the gradient over every design pixel (weighted-adjoint sweeps
and contraction).  The symbolic analysis depends only on the grid and is done
once, outside the timed region.  Inputs (eps, w) are resident in HBM.

Workload (default, the largest single-GPU configuration): 2,400-wavelength
multi-angle metasurface, 48,000 x 160 grid (7.68M unknowns, dx = lambda/20),
4,559 input x 4,559 output channels (all orders within sin(theta) < 0.95),
1.92M design pixels of binary {1, 4} permittivity smoothed by a 3-px-FWHM
Gaussian, grouped objective (five target orders per input, 100 orders apart,
with a uniformity penalty).  --workload metasurface_24000x160 runs the
1,200-wavelength metasurface (2,399 x 2,399 channels, f = sum w |S|^2).
Synthetic, seeded.

Prints one JSON line.  The roofline block is for the batched complex FP64
MFMA GEMM kernels (k_gemm, its three-product variant k_gemm_k3 and the
low-rank k_lowrank_w): their algorithmic flops (8 per complex MAC of the
M x N x K products the tasks specify, a triangular factor counting only its
stored triangle) over their HIP-event time in the timed region; traffic is
their HBM bytes per launch from the committed counter summary under
profiles/, or null when that summary was taken on other sources.  The same
block reports the flops the MFMA units execute (6 per complex MAC where the
three-product form runs) over the same time.  The cpu_baseline block times
the CPU FP64 oracle on three narrow strips of the same layout and
permittivity recipe, fits the two coefficients of the oracle's cost model
(grid term, channel term) on two of them, checks the fit on the third and
scales it to the full workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFLOPS = 78.6
FP32_MFMA_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "metasurface_24000x160": dict(kind="wide", nx=24000, seed=1),
    "metasurface_240x92": dict(kind="small", seed=0),
    "batch64_uneven": dict(kind="batch", seed=3, count=64),
    "multiangle_48000x160": dict(kind="multiangle", nx=48000, seed=2),
}


def make_workload(name):
    from paper_2306_09257_amd import inputs
    spec = WORKLOADS[name]
    if spec["kind"] == "wide":
        return inputs.metasurface_wide(seed=spec["seed"], nx=spec["nx"])
    if spec["kind"] == "multiangle":
        # the grouped objective takes the place of the weights
        return inputs.metasurface_multiangle(seed=spec["seed"], nx=spec["nx"])
    return inputs.metasurface_small(seed=spec["seed"])


SOURCE_DIRS = ("paper_2306_09257_amd/csrc", "include")


def sources_digest():
    """sha256 over the library sources (kernels, plan building, headers): the
    identity of the code whose hardware counters a profile summary records."""
    h = hashlib.sha256()
    for d in SOURCE_DIRS:
        for name in sorted(os.listdir(os.path.join(ROOT, d))):
            if name.endswith((".hip", ".cpp", ".h")):
                with open(os.path.join(ROOT, d, name), "rb") as f:
                    h.update(name.encode())
                    h.update(f.read())
    return h.hexdigest()


def profiled_traffic(workload, precision):
    """HBM bytes per k_gemm launch recorded by the committed counter summary
    profiles/k_gemm_<workload>_<precision>.md (FETCH_SIZE and WRITE_SIZE
    passes, scaled by a plain copy's counts), if it was taken on the current
    sources.  Returns (bytes or None, note)."""
    path = os.path.join(ROOT, "profiles", f"k_gemm_{workload}_{precision}.md")
    if not os.path.exists(path):
        return None, f"no counter summary {os.path.relpath(path, ROOT)}"
    fields = {}
    with open(path) as f:
        for line in f:
            for key in ("traffic_bytes_per_launch", "sources_sha256"):
                if line.startswith(key + ":"):
                    fields[key] = line.split(":", 1)[1].strip()
    if "traffic_bytes_per_launch" not in fields or "sources_sha256" not in fields:
        return None, f"{os.path.relpath(path, ROOT)} records no traffic"
    if fields["sources_sha256"] != sources_digest():
        return None, f"{os.path.relpath(path, ROOT)} was taken on other sources"
    return float(fields["traffic_bytes_per_launch"]), os.path.relpath(path, ROOT)


def oracle_cost_terms(nx, ny, m):
    """The two terms of the oracle's cyclic column-block solve for S and the
    gradient, in complex MACs: two solves (forward, weighted adjoint), each
    eliminating nx column blocks of size ny (a grid term ~ nx ny^3: the block
    LU and the border updates) against m right-hand sides (a channel term
    ~ nx ny^2 m: triangular solves and back substitution)."""
    return 2.0 * nx * ny ** 3, 2.0 * nx * ny ** 2 * m


def cpu_model_name():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_strip_seconds(workload, nx, dx_over_lambda):
    """Oracle S + gradient (forward solve, objective, weighted adjoint solve,
    contraction) on an nx-wide strip of the workload's layout and eps recipe;
    the channel set follows the workload (all orders, or sin < 0.95) at the
    given grid step, which sets the channel count."""
    import numpy as np
    from paper_2306_09257_amd import inputs
    import oracle.apf as oapf
    import oracle.fdfd as ofd
    import oracle.objectives as oobj
    multi = WORKLOADS[workload]["kind"] == "multiangle"
    orders = inputs.channel_orders(nx, dx_over_lambda, sin_max=0.95 if multi else 1.0)
    prob = inputs.make_problem(nx, 160, dx_over_lambda=dx_over_lambda, in_orders=orders)
    rng = np.random.default_rng(WORKLOADS[workload]["seed"])
    eps = inputs.eps_binary_smoothed(prob, rng)
    w = inputs.weights_uniform(prob, rng)
    t0 = time.perf_counter()
    solver = oapf.make_solver(prob, eps, "column")
    Y = oapf.forward_fields(prob, solver)
    S = ofd.projection_row(prob) @ Y[prob.prj_row]
    if multi:
        _, G = oobj.group_fom(S, prob.in_orders, prob.out_orders, max(1, round(nx * dx_over_lambda / 24)))
    else:
        _, G = oapf.weighted_power(S, w)
    Lam = oapf.adjoint_fields(prob, solver, G)
    oapf.gradient_from_fields(prob, Y, Lam)
    return time.perf_counter() - t0, prob


def _oracle_full_rate(workload, budget_s=10.0):
    """Oracle S + gradient on the workload itself, repeated for about
    budget_s seconds (workloads the oracle finishes in well under a second).
    Returns (solves per second, repetitions, seconds)."""
    import oracle.apf as oapf
    prob, eps, w = make_workload(workload)
    reps, t0 = 0, time.perf_counter()
    while True:
        oapf.solve_S_and_grad(prob, eps, w=w)
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= budget_s:
            return reps / dt, reps, dt


def cpu_baseline(prob_full, workload):
    """The oracle timed on three strips of the workload (same layout, eps
    recipe and objective): a 480-wide strip at the workload's grid step, the
    same strip at dx = lambda/5 (four times the channels, so that the channel
    term dominates) -- these two fix the coefficients of the grid and the
    channel term -- and a 960-wide strip at the workload's step, on which the
    fitted model is checked.  The fitted model then gives the full
    workload's time."""
    import numpy as np
    try:
        from threadpoolctl import threadpool_info
        cores = max(i["num_threads"] for i in threadpool_info()) if threadpool_info() else os.cpu_count()
    except Exception:
        cores = os.cpu_count()
    if WORKLOADS[workload]["kind"] == "small":
        rate, reps, dt = _oracle_full_rate(workload)
        return {"value": rate, "unit": "solves/s", "cores": int(cores), "kind": "oracle",
                "cpu_model": cpu_model_name(),
                "sample": f"oracle S+grad on the workload itself, {reps} solves in {dt:.1f} s",
                "sample_seconds": dt}
    dx = 0.05
    pts = []
    for nx, d in ((480, dx), (480, 0.2), (960, dx)):
        t, p = _oracle_strip_seconds(workload, nx, d)
        pts.append((nx, p.n_in, t, oracle_cost_terms(nx, p.ny, p.n_in)))
    M = np.array([pts[0][3], pts[1][3]])
    a, b = np.linalg.solve(M, np.array([pts[0][2], pts[1][2]]))
    pred = a * pts[2][3][0] + b * pts[2][3][1]
    check_err = (pred - pts[2][2]) / pts[2][2]
    ga, gb = oracle_cost_terms(prob_full.nx, prob_full.ny, prob_full.n_in)
    t_full = a * ga + b * gb
    return {
        "value": 1.0 / t_full, "unit": "solves/s", "cores": int(cores), "kind": "oracle",
        "cpu_model": cpu_model_name(),
        "sample": "oracle S+grad on strips of the same layout, eps recipe and objective: "
                  + "; ".join(f"{nx}x160 with {m} channels {t:.2f} s" for nx, m, t, _ in pts)
                  + f"; model t = a*2*nx*ny^3 + b*2*nx*ny^2*M fitted on the first two "
                  f"(a = {a:.3e} s, b = {b:.3e} s per complex MAC), off by {100 * check_err:+.1f}% on the "
                  f"third; full workload {t_full:.0f} s ({ga:.2e} + {gb:.2e} MAC)",
        "sample_seconds": sum(t for _, _, t, _ in pts),
        "model_check_rel_err": check_err,
    }


def batch_cpu_baseline(items):
    """The oracle's S (one forward solve with all inputs, then the projection)
    timed on six problems of the batch spread over its cost range; the two
    coefficients of the column-block solver's cost (grid term nx ny^3,
    channel term nx ny^2 M) are fitted to them by least squares and give the
    whole batch's time."""
    import numpy as np
    import oracle.apf as oapf
    try:
        from threadpoolctl import threadpool_info
        cores = max(i["num_threads"] for i in threadpool_info()) if threadpool_info() else os.cpu_count()
    except Exception:
        cores = os.cpu_count()
    terms = [(p.nx * p.ny ** 3, p.nx * p.ny ** 2 * p.n_in) for p, _, _ in items]
    order = np.argsort([t[0] + t[1] for t in terms])
    pick = [int(order[int(round(q * (len(order) - 1) * 0.5))]) for q in np.linspace(0.0, 1.0, 6)]
    rows, ts = [], []
    for i in pick:
        prob, eps, _ = items[i]
        t0 = time.perf_counter()
        oapf.scattering_matrix(prob, eps, solver=oapf.make_solver(prob, eps, "column"))
        ts.append(time.perf_counter() - t0)
        rows.append(terms[i])
    coef, *_ = np.linalg.lstsq(np.array(rows, dtype=float), np.array(ts), rcond=None)
    pred = np.array(rows, dtype=float) @ coef
    total = float(np.array(terms, dtype=float).sum(axis=0) @ coef)
    return {
        "value": len(items) / total, "unit": "factorizations/s", "cores": int(cores), "kind": "oracle",
        "cpu_model": cpu_model_name(),
        "sample": "oracle S on problems " + ", ".join(f"{items[i][0].nx}x{items[i][0].ny} ({items[i][0].n_in} ch) "
                                                      f"{t:.2f} s" for i, t in zip(pick, ts))
                  + f"; least-squares fit of t = a nx ny^3 + b nx ny^2 M (a = {coef[0]:.3e}, b = {coef[1]:.3e}), "
                  f"worst fit error {100 * float(np.max(np.abs(pred - ts) / ts)):.0f}%; whole batch {total:.0f} s",
        "sample_seconds": float(sum(ts)),
    }


def bench_batch(args):
    """64 independent problems of uneven size (nx 120..4800, ny 60/92/140,
    lambda/lambda0 in [0.9, 1.1]) factorized by one batched call per step;
    value = problems factorized per second (S of every problem), after the
    autotuner picked the GEMM kernel forms of the merged plan (outside the
    timed region).  The same steps with the fixed rule, and the problems
    factorized one call each, are timed beside it."""
    import torch
    from paper_2306_09257_amd import binding, inputs
    spec = WORKLOADS[args.workload]
    items = inputs.batch_uneven(seed=spec["seed"], count=spec["count"])
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    apfs, epss, outs = [], [], []
    for prob, eps, w in items:
        a = binding.APF(prob, leaf_size=args.leaf).analyze()
        e = torch.as_tensor(eps, dtype=torch.float64, device=dev).contiguous()
        a.assemble(e)
        apfs.append(a)
        epss.append(e)
        outs.append(torch.empty((prob.n_out, prob.n_in), dtype=torch.complex128, device=dev))
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0

    def step():
        for a, e in zip(apfs, epss):
            a.assemble(e)
        binding.factor_schur_batched(apfs, outs)

    def timed():
        binding.factor_schur_batched(apfs, outs)      # merged plan + graph capture
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def gemm_profile():
        # one eager step with the GEMM launches timed (profiling disables the graph)
        apfs[0].set_profiling(True, gemm_only=True)
        step()
        torch.cuda.synchronize()
        p = apfs[0].profile()
        apfs[0].set_profiling(False)
        return p["gemm_factor"][0] + p["gemm_schur"][0], p["gemm_factor"][1] + p["gemm_schur"][1]

    dt_fixed = timed()
    gemm_ms_fixed, _ = gemm_profile()
    t0 = time.perf_counter()
    binding.autotune(apfs, reps=2)
    t_tune = time.perf_counter() - t0
    dt = timed()
    gemm_ms, gemm_launches = gemm_profile()
    # the same problems, one factorization call each
    t1 = time.perf_counter()
    for _ in range(args.steps):
        for a, e, S in zip(apfs, epss, outs):
            a.assemble(e)
            a.factor_schur(S)
    torch.cuda.synchronize()
    dt_seq = time.perf_counter() - t1
    n = len(items)
    cm = sum(a.query("gemm_cmacs_factor") + a.query("gemm_cmacs_schur") for a in apfs)
    achieved = 8.0 * cm / (gemm_ms * 1e-3) / 1e12
    out = {
        "metric": "APF factorizations/sec (S), batch of uneven problems",
        "value": n * args.steps / dt, "unit": "factorizations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c128 (f64)", "data": "synthetic",
        "config": {"workload": args.workload, "problems": n,
                   "unknowns_total": int(sum(p.nx * p.ny for p, _, _ in items)),
                   "nx_range": [min(p.nx for p, _, _ in items), max(p.nx for p, _, _ in items)],
                   "channels_range": [min(p.n_in for p, _, _ in items), max(p.n_in for p, _, _ in items)],
                   "precision": "fp64"},
        "roofline": {"kernel": "k_gemm / k_gemm_thin / k_gemm_thin_tri / k_gemm_k3 (merged batched complex FP64 MFMA GEMMs of a step)",
                     "bound": "mfma", "achieved": achieved, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_MFMA_PEAK_TFLOPS, "traffic": None,
                     "flop_per_step": 8.0 * cm, "launches_per_step": gemm_launches,
                     "avg_launch_ms": gemm_ms / max(gemm_launches, 1),
                     "gemm_ms_per_step": gemm_ms, "gemm_ms_per_step_fixed_rule": gemm_ms_fixed},
        "fixed_rule_ms_per_step": 1e3 * dt_fixed / args.steps,
        "autotune_s": t_tune,
        "sequential_ms_per_step": 1e3 * dt_seq / args.steps,
        "batched_speedup": dt_seq / dt,
        "setup_s": t_plan,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = batch_cpu_baseline(items)
    print(json.dumps(out), flush=True)


def compression_error(args, prob, eps_d, w, w_d, grouped, S, grad, prec):
    """Relative distance of the compressed step's S, f and gradient from an
    uncompressed handle's (outside the timed region)."""
    import torch
    from paper_2306_09257_amd import binding
    ref = binding.APF(prob, leaf_size=args.leaf).analyze()
    if args.lowrank >= 0:
        ref.set_lowrank(args.lowrank)
    if args.factor_only:
        ref.set_gradient(False)
    ref.assemble(eps_d)
    S0 = ref.factor_schur(precision=prec)
    out = {"S": float(torch.linalg.norm(S - S0) / torch.linalg.norm(S0))}
    f0, G0 = ref.group_fom(S0, w) if grouped else ref.weighted_power(S0, w_d)
    if not args.factor_only:
        f1 = (ref.group_fom(S, w) if grouped else ref.weighted_power(S, w_d))[0]
        g0 = ref.grad(G0)
        torch.cuda.synchronize()
        out["f"] = float(abs(f1 - f0) / abs(f0))
        out["grad"] = float(torch.linalg.norm(grad - g0) / torch.linalg.norm(g0))
    del ref
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="multiangle_48000x160", choices=sorted(WORKLOADS))
    ap.add_argument("--leaf", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB (a known-size "
                         "reference for hardware byte counters)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed", "refined"],
                    help="mixed: front GEMMs and sweeps on FP32 MFMA (FP64 storage, pivots, reductions); "
                         "refined: the mixed factorization plus FP64 iterative refinement of the forward and "
                         "adjoint fields")
    ap.add_argument("--refine-iters", type=int, default=2)
    ap.add_argument("--factor-only", action="store_true",
                    help="time assemble + factorization (S) per step on a handle without the gradient sweeps "
                         "(metric: factorizations/s)")
    ap.add_argument("--compress", default="",
                    help="PAD,WINDOW: B/C compression with PAD extra orders and a WINDOW-wavelength truncation; "
                         "after the timed steps, S, f and the gradient are compared with an uncompressed handle")
    ap.add_argument("--lowrank", type=int, default=-1,
                    help="levels of the low-rank sweep subtrees (0-2; default: the library's)")
    ap.add_argument("--symmetric", action="store_true",
                    help="the symmetric route: L D L^T pivot blocks and the symmetric products (FP64)")
    args = ap.parse_args()
    if args.symmetric and (args.compress or args.precision != "fp64"):
        print("--symmetric runs in FP64 only and does not combine with --compress", file=sys.stderr)
        sys.exit(2)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the APF path here is a "
              f"single-GPU build", file=sys.stderr)
        sys.exit(2)

    if WORKLOADS[args.workload]["kind"] == "batch":
        bench_batch(args)
        return

    import numpy as np
    import torch
    from paper_2306_09257_amd import binding

    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    prob, eps, w = make_workload(args.workload)
    print(f"[bench] workload {args.workload}: {prob.nx}x{prob.ny}, {prob.n_in}x{prob.n_out} channels",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    apf = binding.APF(prob, leaf_size=args.leaf).analyze()
    if args.precision == "refined":
        apf.set_refinement(args.refine_iters, 1e-10)
    if args.lowrank >= 0:
        apf.set_lowrank(args.lowrank)
    if args.symmetric:
        apf.set_symmetric(True)
    if args.compress:
        pad, window = args.compress.split(",")
        apf.set_compression(int(pad), float(window))
    if args.factor_only:
        apf.set_gradient(False)
    t_an = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    eps_d = torch.as_tensor(eps, dtype=torch.float64, device=dev).contiguous()
    grouped = WORKLOADS[args.workload]["kind"] == "multiangle"
    w_d = None if grouped else torch.as_tensor(w, dtype=torch.float64, device=dev).contiguous()
    S = torch.empty((prob.n_out, prob.n_in), dtype=torch.complex128, device=dev)
    grad = torch.empty((prob.n_design_rows, prob.nx), dtype=torch.float64, device=dev)

    prec = {"fp64": binding.APF_FP64, "mixed": binding.APF_MIXED, "refined": binding.APF_MIXED_REFINED}[args.precision]

    def step():
        apf.assemble(eps_d)
        apf.factor_schur(S, precision=prec)
        if args.factor_only:
            return None
        f, G = apf.group_fom(S, w) if grouped else apf.weighted_power(S, w_d)
        apf.grad(G, out=grad)
        return f

    t0 = time.perf_counter()
    step()                      # first call builds the device plan
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    print(f"[bench] analysis {t_an:.2f} s, first step (plan + run) {t_plan:.2f} s", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # the timed steps carry HIP events around the GEMM-family launches only
    # (the roofline figures); the per-phase times come from one more step
    # with every launch timed, outside the timed region
    apf.set_profiling(True, gemm_only=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = apf.profile()
    apf.set_profiling(True)
    step()
    torch.cuda.synchronize()
    prof_all = apf.profile()
    apf.set_profiling(False)
    ms_step = 1e3 * dt / args.steps
    value = args.steps / dt

    cm = {k: apf.query("gemm_cmacs_" + k) for k in ("factor", "schur", "sweep", "k3", "lowrank_w")}
    # the refined path runs neither the Schur product nor the sweeps of the
    # plain paths (its S and gradient come from the refined fields): its
    # roofline covers the factorization GEMMs only
    classes = ("gemm_factor",) if args.precision == "refined" else ("gemm_factor", "gemm_schur", "gemm_sweep")
    if args.precision == "refined" or args.compress:
        cm["schur"] = 0.0                         # (compressed: S~ blocks and decompression not counted)
    if args.precision == "refined" or args.factor_only:
        cm["sweep"] = cm["lowrank_w"] = 0.0
    if args.compress:
        cm["k3"] = cm["sweep"] if args.precision == "fp64" else 0.0   # the deep lists: sweeps' adjoint source only
    sparse_k = apf.query("adjoint_source_sparse_k")
    if sparse_k > 0:
        # the weighted adjoint source ran as the sparse kernel (not a GEMM):
        # its dense product is neither run nor counted
        v = apf.query("gemm_cmacs_vinit")
        cm["sweep"] -= v
        cm["k3"] -= v
    gemm_ms = sum(prof[c][0] for c in classes) / args.steps
    gemm_launches = sum(prof[c][1] for c in classes) / args.steps
    gemm_cm = cm["factor"] + cm["schur"] + cm["sweep"]
    gemm_flop = 8.0 * gemm_cm
    achieved = gemm_flop / (gemm_ms * 1e-3) / 1e12
    # flops the MFMA units execute: 6 per complex MAC of the three-product
    # form (FP64 deep lists and the low-rank W kernel), 8 elsewhere
    k3 = cm["k3"] if args.precision == "fp64" else cm["lowrank_w"]
    executed = (8.0 * (gemm_cm - k3) + 6.0 * k3) / (gemm_ms * 1e-3) / 1e12
    peak = FP64_MFMA_PEAK_TFLOPS if args.precision == "fp64" else FP32_MFMA_PEAK_TFLOPS
    if args.compress or args.factor_only or args.lowrank >= 0 or args.leaf or args.symmetric:
        traffic, traffic_note = None, "the counter summaries cover the default plan options only"
    else:
        traffic, traffic_note = profiled_traffic(args.workload, args.precision)
    roofline = {
        "kernel": "k_gemm / k_gemm_thin / k_gemm_thin_tri / k_gemm_k3 / k_lowrank_w (batched complex %s MFMA GEMMs, all launches of a step)"
                  % ("FP64" if args.precision == "fp64" else "FP32"),
        "bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
        "frac": achieved / peak, "traffic": traffic, "traffic_unit": "HBM bytes per launch",
        "traffic_source": traffic_note,
        "flop_per_step": gemm_flop, "launches_per_step": gemm_launches,
        "avg_launch_ms": gemm_ms / max(gemm_launches, 1),
        "executed": executed, "executed_frac": executed / peak,
        "executed_note": "MFMA flops issued: 6 per complex MAC in the three-product form, 8 otherwise",
    }
    phases = {c: round(prof_all[c][0], 3) for c in prof_all}

    out = {
        "metric": ("APF factorizations/sec (S) at N unknowns, M channels" if args.factor_only
                   else "APF solves/sec (S+grad f) at N unknowns, M channels"),
        "value": value, "unit": "factorizations/s" if args.factor_only else "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "c128 (f64)", "mixed": "c64 (f32) front GEMMs, f64 storage",
                  "refined": "c64 (f32) front GEMMs + f64 refinement"}[args.precision], "data": "synthetic",
        "config": {"workload": args.workload, "nx": prob.nx, "ny": prob.ny, "unknowns": prob.nx * prob.ny,
                   "n_in": prob.n_in, "n_out": prob.n_out, "design_pixels": prob.n_design_rows * prob.nx,
                   "precision": args.precision, "leaf_size": args.leaf or 48,
                   "compression": args.compress or None,
                   "route": "symmetric (L D L^T)" if args.symmetric else "LU"},
        "roofline": roofline,
        "phase_ms_per_step": phases,
        "analysis_s": t_an,
        "adjoint_source": ({"kind": "sparse", "nonzeros_per_input_max": int(sparse_k),
                            "ms_per_step": prof_all["adjoint_source"][0]} if sparse_k > 0 else {"kind": "dense GEMM"}),
        "factor_cmacs_algorithmic": apf.query("algo_factor_cmacs"),
    }
    if args.precision == "refined":
        out["refine"] = {"chunk": apf.query("refine_chunk"), "residual_first": apf.query("refine_residual_first"),
                         "residual_final": apf.query("refine_residual"),
                         "retained_factor_bytes": apf.query("retained_factor_bytes"),
                         "ms_refine_per_step": prof_all["refine"][0]}
    if args.precision in ("mixed", "refined") and not args.compress:
        # accuracy of the mixed result against the FP64 path
        S_m, g_m = S.clone(), grad.clone()
        apf.assemble(eps_d)
        S64 = apf.factor_schur(precision=binding.APF_FP64)
        f64, G64 = apf.group_fom(S64, w) if grouped else apf.weighted_power(S64, w_d)
        g64 = apf.grad(G64)
        torch.cuda.synchronize()
        out["mixed_rel_err_vs_fp64"] = {
            "S": float(torch.linalg.norm(S_m - S64) / torch.linalg.norm(S64)),
            "grad": float(torch.linalg.norm(g_m - g64) / torch.linalg.norm(g64))}
    if args.compress:
        out["compression_vs_uncompressed"] = compression_error(args, prob, eps_d, w, w_d, grouped, S, grad, prec)
    if not args.no_cpu_baseline and not args.factor_only:
        out["cpu_baseline"] = cpu_baseline(prob, args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
