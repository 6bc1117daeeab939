"""Comparison helpers for parity tests: gap masks, agreement and graph recall.

* A sample's assignment is *decided* when, over its candidate set, the second
  smallest float64 distance exceeds the smallest by more than ``rel`` of the
  smallest, and the current cluster is either the closest or beyond that gap.
  Integer outputs must match exactly on decided samples; on the rest the GPU's
  choice must still be within ``rel`` of the best.
* Graph recall (Sec. 5.1 evaluation protocol: top-1 recall): a row counts as
  a hit when its first entry lies at the exact nearest-neighbour distance
  (ties count).  recall@kappa is |G[i] cap KNN(i)| / kappa.
"""
import numpy as np

from .gkmeans import candidates


def assign_gap_mask(X, C, labels_in, G_ids, rel=1e-5):
    X64 = np.asarray(X, np.float32).astype(np.float64)
    C64 = np.asarray(C, np.float32).astype(np.float64)
    labels_in = np.asarray(labels_in, np.int64)
    G_ids = np.asarray(G_ids, np.int64)
    n, k = X64.shape[0], C64.shape[0]
    decided = np.empty(n, bool)
    best = np.empty(n, np.float64)
    for s in range(0, n, 4096):
        e = min(n, s + 4096)
        if G_ids.shape[1] >= k:
            cand = np.broadcast_to(np.arange(k), (e - s, k))
        else:
            cand = candidates(labels_in[s:e], labels_in, G_ids[s:e])
        diff = X64[s:e, None, :] - C64[cand]
        d = np.einsum("ijk,ijk->ij", diff, diff)
        # distinct clusters only: duplicates of the minimum are not a second value
        d_sorted = np.sort(d, axis=1)
        m = d_sorted[:, 0]
        big = np.where(np.equal(cand, cand[np.arange(e - s), d.argmin(1)][:, None]), np.inf, d)
        second = big.min(axis=1)
        decided[s:e] = (second - m) > rel * m
        best[s:e] = m
    return decided, best


def agreement(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float((a == b).mean()) if a.size else 1.0


def recall_top1(G_d2, exact_d2_1nn):
    """Fraction of rows whose first entry is at the exact 1-NN distance."""
    return float((np.asarray(G_d2)[:, 0] <= np.asarray(exact_d2_1nn)).mean())


def recall_at_kappa(G_ids, exact_ids):
    G_ids = np.asarray(G_ids)
    exact_ids = np.asarray(exact_ids)
    hits = [len(np.intersect1d(G_ids[r], exact_ids[r])) for r in range(G_ids.shape[0])]
    return float(np.mean(hits) / G_ids.shape[1])
