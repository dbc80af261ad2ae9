"""Writes tests/golden/batch64_uneven_seed3.npz with the CPU FP64 oracle only:
for every problem of the 64-problem uneven batch (seed 3: nx 120..4,800,
ny in {60, 92, 140}, lambda/lambda0 in [0.9, 1.1]), the S columns of the
first, the middle and the last input.  Run from the repository root:
python tests/golden/make_batch_golden.py (about 15 minutes on eight cores)."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from paper_2306_09257_amd import inputs  # noqa: E402
import oracle.apf as oapf  # noqa: E402
import oracle.fdfd as ofd  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch64_uneven_seed3.npz")


def main():
    items = inputs.batch_uneven(seed=3, count=64)
    t0 = time.time()
    cols_all, S_all, offs = [], [], [0]
    for i, (prob, eps, w) in enumerate(items):
        cols = np.unique(np.array([0, prob.n_in // 2, prob.n_in - 1], dtype=np.int64))
        solver = oapf.make_solver(prob, eps)
        Y = oapf.forward_fields(prob, solver, cols)
        S_cols = ofd.projection_row(prob) @ Y[prob.prj_row]           # n_out x len(cols)
        cols_all.append(cols)
        S_all.append(S_cols.T.ravel())                                 # column-major by input
        offs.append(offs[-1] + S_cols.size)
        print(f"{i}: {prob.nx}x{prob.ny}, {prob.n_in} channels, {time.time() - t0:.0f} s", flush=True)
    np.savez(OUT, ncols=np.array([c.size for c in cols_all]), cols=np.concatenate(cols_all),
             S=np.concatenate(S_all), offsets=np.array(offs), seconds=time.time() - t0)
    print(f"wrote {OUT} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
