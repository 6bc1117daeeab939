"""Alg. 3 (KNN graph construction with fast k-means) in float64.

* Graph entries hold squared L2 distances (Eqn. 1 / Eqn. 4 use squared norms).
  The stored value of a pair is its float64 squared distance rounded to float32
  (the storage format); lists are ordered by (stored value, id) ascending.
* Random initial lists (Alg. 3, initialisation): row i takes min(kappa, n-1)
  distinct ids other than i, drawn by Floyd's algorithm on stream
  (GRAPH_INIT, 0, i) over [0, n-1) and shifted past i.
* k0 = max(1, floor(n / xi)) clusters per round (Sec. 4.3; max(1, .) covers
  n < xi).
* Each round (Alg. 3 loop): a fresh TwoMeans(k0) with round tag t, its means,
  then one GK-means^- sweep with the current graph ("t is fixed to 1", Sec. 4.5).
* Exhaustive comparison inside each cluster; the pair <i, j> updates G[i] and
  G[j].  A pair is "visited" for row i when j is already in G[i]; the row keeps
  the kappa smallest (value, id) entries of its old list and the new pairs.

Pins (tests/test_oracle_pins.py): one round with k0 = 1 is an exact brute-force
KNN graph (checked against scipy's cKDTree); rows sorted, self-free and
duplicate-free with stored values equal to the recomputed distances; the
kappa-th value of every row never increases from one round to the next; tau = 0
returns the initial graph.
"""
import numpy as np

from . import rng
from .twomeans import twomeans
from .gkmeans import centroid_update, gk_assign


def pair_key(X64, i, J):
    """Stored value of the pairs (i, J): float64 squared distance rounded to float32."""
    diff = X64[J] - X64[i][None, :]
    return np.einsum("ij,ij->i", diff, diff).astype(np.float32)


def sort_rows(ids, d2):
    """Order every row by (d2, id) ascending."""
    out_i = np.empty_like(ids)
    out_d = np.empty_like(d2)
    for r in range(ids.shape[0]):
        o = np.lexsort((ids[r], d2[r]))
        out_i[r] = ids[r][o]
        out_d[r] = d2[r][o]
    return out_i, out_d


def graph_init(X, kappa, seed):
    X64 = np.asarray(X, np.float32).astype(np.float64)
    n = X64.shape[0]
    assert 1 <= kappa <= n - 1
    keys = np.array(
        [rng.stream_key(seed, rng.stream_id(rng.PURPOSE_GRAPH_INIT, 0, i)) for i in range(n)],
        dtype=np.uint64,
    )
    v = rng.floyd_sample_rows(keys, n - 1, kappa)
    ids = v + (v >= np.arange(n)[:, None])
    d2 = np.empty((n, kappa), np.float32)
    for i in range(n):
        d2[i] = pair_key(X64, i, ids[i])
    ids, d2 = sort_rows(ids, d2)
    return ids.astype(np.int32), d2


def merge_row(ids, d2, new_ids, new_d2, kappa):
    """Keep the kappa smallest (value, id) of the old row and the new pairs; a new
    id already present in the row is a visited pair and is skipped."""
    fresh = ~np.isin(new_ids, ids)
    all_i = np.concatenate([ids, new_ids[fresh]])
    all_d = np.concatenate([d2, new_d2[fresh]])
    o = np.lexsort((all_i, all_d))[:kappa]
    return all_i[o], all_d[o]


def refine_cluster(A64, mem, G_rows, D_rows):
    """Alg. 3 inner loops for one cluster S_m: every pair <i, j> of its members
    (global ids ``mem``, rows A64 in float64 in the same order) updates G[i]
    and G[j].  G_rows / D_rows are the members' current lists; returns the
    updated lists (the other rows of the graph are not touched)."""
    kappa = G_rows.shape[1]
    out_i = np.array(G_rows, dtype=np.int64, copy=True)
    out_d = np.array(D_rows, dtype=np.float32, copy=True)
    if len(mem) < 2:
        return out_i, out_d
    diff = A64[:, None, :] - A64[None, :, :]
    D = np.einsum("ijk,ijk->ij", diff, diff).astype(np.float32)
    for a in range(len(mem)):
        others = np.concatenate([np.arange(a), np.arange(a + 1, len(mem))])
        out_i[a], out_d[a] = merge_row(out_i[a], out_d[a], np.asarray(mem)[others], D[a, others], kappa)
    return out_i, out_d


def refine(X, G_ids, G_d2, labels):
    """Exhaustive comparison inside every cluster of ``labels`` and list update."""
    X64 = np.asarray(X, np.float32).astype(np.float64)
    G_ids = np.array(G_ids, dtype=np.int64, copy=True)
    G_d2 = np.array(G_d2, dtype=np.float32, copy=True)
    order = np.argsort(labels, kind="stable")
    bounds = np.flatnonzero(np.diff(np.asarray(labels)[order])) + 1
    for mem in np.split(order, bounds):
        G_ids[mem], G_d2[mem] = refine_cluster(X64[mem], mem, G_ids[mem], G_d2[mem])
    return G_ids.astype(np.int32), G_d2


def build_round(X, G_ids, G_d2, k0, seed, t, bisect_iters=2):
    """One pass of the Alg. 3 loop; returns the new graph and the cluster labels."""
    labels = twomeans(X, k0, seed, t, bisect_iters)
    C, _, _ = centroid_update(X, labels, k0, np.zeros((k0, X.shape[1]), np.float32))
    labels, _, _ = gk_assign(X, C, labels, G_ids)
    G_ids, G_d2 = refine(X, G_ids, G_d2, labels)
    return G_ids, G_d2, labels


def knn_build(X, kappa, xi=50, tau=10, seed=0, bisect_iters=2, history=False):
    X = np.asarray(X, np.float32)
    n = X.shape[0]
    k0 = max(1, n // xi)
    G_ids, G_d2 = graph_init(X, kappa, seed)
    hist = [(G_ids, G_d2)]
    for t in range(tau):
        G_ids, G_d2, _ = build_round(X, G_ids, G_d2, k0, seed, t, bisect_iters)
        hist.append((G_ids, G_d2))
    if history:
        return G_ids, G_d2, hist
    return G_ids, G_d2
