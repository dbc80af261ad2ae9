"""Error measures of the GPU parity tests (host-side numpy only).

Normwise errors over a whole array can hide a few wrong blocks, so every
oracle comparison also reports the worst relative error over column blocks:
input columns of S, grid columns (x) of the gradient."""
import numpy as np

NBLK = 16


def rel(a, b):
    """||a - b|| / ||b|| (Frobenius / 2-norm)."""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def worst_block(a, b, axis=-1, nblk=NBLK):
    """Largest rel() over up to nblk contiguous blocks of indices along
    `axis` (fewer when the axis is shorter)."""
    a, b = np.asarray(a), np.asarray(b)
    n = a.shape[axis]
    worst = 0.0
    for idx in np.array_split(np.arange(n), min(nblk, n)):
        worst = max(worst, rel(np.take(a, idx, axis=axis), np.take(b, idx, axis=axis)))
    return worst


def worst_block_sampled(vals, ref, xs, nx, nblk=NBLK):
    """Largest rel() over the samples grouped by the x block (of nblk equal
    blocks of the nx grid columns) their pixel lies in."""
    vals, ref, xs = np.asarray(vals), np.asarray(ref), np.asarray(xs)
    blk = (xs * nblk) // nx
    worst = 0.0
    for b in np.unique(blk):
        m = blk == b
        worst = max(worst, rel(vals[m], ref[m]))
    return worst
