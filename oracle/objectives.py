"""Oracle objective for the multi-angle splitter workload.

TEST INFRASTRUCTURE ONLY (see the package docstring).

For each input a the targets are the outputs whose order differs from a's by
g * delta, |g| <= gmax (those that exist).  With p = |S|^2,
    f = - sum_a sum_{t in T(a)} p_ta + sum_a sum_{t in T(a)} (p_ta - mu_a)^2,
mu_a the mean of p over T(a): transmit into the target orders, evenly.  Its
Wirtinger derivative: df/dp_ta = -1 + 2 (p_ta - mu_a) (the mean's own
derivative cancels, since the deviations sum to zero), dF/dS = df/dp conj(S)
on the targets and 0 elsewhere.
"""
from __future__ import annotations

import numpy as np


def targets(in_orders, out_orders, delta, gmax=2):
    """Boolean [n_out][n_in] mask of the target entries."""
    d = np.asarray(out_orders)[:, None] - np.asarray(in_orders)[None, :]
    return (d % delta == 0) & (np.abs(d) <= gmax * delta)


def group_fom(S, in_orders, out_orders, delta, gmax=2):
    """f and dF/dS of the grouped objective (loops over inputs, plainly)."""
    T = targets(in_orders, out_orders, delta, gmax)
    p = np.abs(S) ** 2
    f = 0.0
    G = np.zeros_like(S)
    for a in range(S.shape[1]):
        t = np.nonzero(T[:, a])[0]
        if t.size == 0:
            continue
        mu = p[t, a].mean()
        f += -p[t, a].sum() + ((p[t, a] - mu) ** 2).sum()
        G[t, a] = (-1.0 + 2.0 * (p[t, a] - mu)) * np.conj(S[t, a])
    return float(f), G
