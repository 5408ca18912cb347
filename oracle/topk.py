"""FP64/FP32 oracle of the sparse semantic state (Sec. 3.1, "Sparse
Semantic Representation").

TEST INFRASTRUCTURE ONLY: the tests use this module; the product package
never does.  Plain numpy.

* Selection: a Gaussian keeps the k classes with the highest probability
  of the distribution it is initialised from (a row of `dist`, chosen by
  `pixel`), in decreasing order; equal probabilities keep the smaller class
  index first; NaN counts as -inf.  The kept values are the probabilities
  themselves (-inf stored as 0), or, with `renormalize`, those values
  divided by their sum (float32, summed in kept order).
* Fixed-index update: with the indices held fixed, each kept value moves
  toward a new observation, v <- (1 - rate) v + rate * dist[pixel][index]
  (float32, in this order of operations).

Parity status: selection is pinned (a hand example with ties and NaN, brute
force over all k-subsets).  The update rule is PARITY UNPINNED: the paper
says the kept values are updated with their indices fixed but gives no
rule (in mapping they are refined through the semantic loss's gradient), so
the convex step above is a reading of this project's own; its test checks
the stated rule, not anything the paper fixes.
"""
from __future__ import annotations

import numpy as np


def select(dist, pixel, k, renormalize=False):
    dist = np.asarray(dist, np.float32)
    rows = dist if pixel is None else dist[np.asarray(pixel, np.int64)]
    n, C = rows.shape
    key = np.where(np.isnan(rows), -np.inf, rows.astype(np.float64))
    cls = np.broadcast_to(np.arange(C), (n, C))
    order = np.lexsort((cls, -key), axis=-1)[:, :k]  # primary: value descending; then index ascending
    val = np.take_along_axis(np.where(np.isnan(rows), -np.inf, rows), order, axis=1).astype(np.float32)
    val = np.where(np.isneginf(val), np.float32(0.0), val).astype(np.float32)
    if renormalize:
        s = np.zeros(n, np.float32)
        for m in range(k):
            s = (s + val[:, m]).astype(np.float32)
        val = np.where(s[:, None] > 0, val / np.where(s > 0, s, 1)[:, None], val).astype(np.float32)
    return order.astype(np.uint8), val


def update(dist, pixel, sem_idx, sem_val, rate):
    dist = np.asarray(dist, np.float32)
    rows = dist if pixel is None else dist[np.asarray(pixel, np.int64)]
    obs = np.take_along_axis(rows, np.asarray(sem_idx, np.int64), axis=1)
    r = np.float32(rate)
    return ((np.float32(1.0) - r) * np.asarray(sem_val, np.float32) + r * obs).astype(np.float32)
