"""Writes tests/golden/design_loop_12000x140_seed4.npz with the CPU FP64
oracle only: for the initial design of the 12000 x 140 differentiation-in-the-
loop workload (seed 4), the S columns of two inputs, the Wirtinger derivative
G = w conj(S) restricted to those two inputs (zero elsewhere), and the
gradient for that G at 2,000 seeded design pixels.  Run from the repository
root: python tests/golden/make_design_loop_golden.py (a few minutes on eight
cores)."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from paper_2306_09257_amd import inputs  # noqa: E402
import oracle.apf as oapf  # noqa: E402
import oracle.fdfd as ofd  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "design_loop_12000x140_seed4.npz")


def main():
    prob, eps, w = inputs.design_loop(seed=4)
    cols = np.array([3, prob.n_in // 3], dtype=np.int64)
    t0 = time.time()
    solver = oapf.make_solver(prob, eps, "column")
    Y = oapf.forward_fields(prob, solver, cols)
    S_cols = ofd.projection_row(prob) @ Y[prob.prj_row]
    G = np.zeros((prob.n_out, prob.n_in), dtype=np.complex128)
    G[:, cols] = w[:, cols] * np.conj(S_cols)
    g, _, _ = oapf.grad_sampled_inputs(prob, eps, G, solver)
    rng = np.random.default_rng(2025)
    flat = rng.choice(g.size, size=2000, replace=False)
    np.savez(OUT, cols=cols, S_cols=S_cols, G_cols=G[:, cols], pixels=flat,
             grad=g.ravel()[flat], grad_norm=np.linalg.norm(g), seconds=time.time() - t0)
    print(f"wrote {OUT} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
