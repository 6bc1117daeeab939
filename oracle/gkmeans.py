"""Alg. 2 in its Lloyd form ("GK-means^-", Sec. 4.2 and the configuration test
of Sec. 5.2), the centroid update, the distortion (Eqn. 4) and the fit loop,
in float64.

Candidate collection (Alg. 2, the loop over the kappa neighbours): for sample
i, Q_i holds the cluster labels of its kappa graph neighbours.  The Lloyd form
replaces the Delta-I move of Eqn. 3 by "seek the closest centroid among the
collected clusters" (Sec. 4.2).  Readings (design notes):

* Q_i also holds the current label of i, so staying put is always possible.
* Jacobi sweep: every read uses labels_in and the fixed centroids C; the result
  goes to labels_out, so it is independent of the visiting order.
* Tie rule: i leaves its cluster only if some candidate is strictly closer;
  among several closest candidates the smallest cluster id wins.
* When kappa >= k the candidate list is every cluster 0..k-1, so the sweep is
  exactly a Lloyd assignment.
* Update (Eqn. 1 / Sec. 1): C_r is the float64 mean of the members of cluster r
  rounded to float32 (the storage format of C); a cluster with no members keeps
  its previous centroid.  Composite vectors D_r (Eqn. 2) are the float64 sums.

Pins (tests/test_oracle_pins.py): kappa >= k equals scipy's cdist argmin; the
complete graph (kappa = n-1) equals an exhaustive argmin over non-empty
clusters; hand-worked 1-D fixtures in tests/golden/; the update equals a pandas
group-by mean (and, for integer data, group-by sums bit for bit); the direct
distortion equals scipy.cluster.vq distances and the Eqn. 2 identity; the fit's
distortion never increases.
"""
import numpy as np

from . import rng
from .twomeans import twomeans

CHUNK = 4096


def _dist_to(X64, C64, cand):
    """Squared L2 distance of each row i to the centroids cand[i, :] (float64)."""
    diff = X64[:, None, :] - C64[cand]
    return np.einsum("ijk,ijk->ij", diff, diff)


def candidates(cur, labels_all, G_rows):
    """Q_i as a padded array for a block of rows: column 0 is the row's current
    label ``cur``, then the labels (looked up in the full label array) of its
    kappa neighbours; duplicates are kept, they do not change the argmin."""
    return np.concatenate([cur[:, None], labels_all[G_rows]], axis=1)


def _decide(Xb, C64, cur, cand):
    """The decision of a block of rows Xb (float64) with current labels cur and
    candidate lists cand: stay unless a candidate is strictly closer; among
    the closest candidates the smallest id.  Returns (labels, best_d2)."""
    d = _dist_to(Xb, C64, cand)
    dcur = np.einsum("ij,ij->i", Xb - C64[cur], Xb - C64[cur])
    m = d.min(axis=1)
    big = np.iinfo(np.int64).max
    newlab = np.where(d == m[:, None], cand, big).min(axis=1)
    stay = dcur <= m
    return np.where(stay, cur, newlab), np.where(stay, dcur, m)


def gk_assign(X, C, labels_in, G_ids):
    """One Jacobi sweep of the graph-restricted assignment.

    Returns (labels_out int32, best_d2 float64, n_moved)."""
    n = np.asarray(X).shape[0]
    out, best = gk_assign_rows(X, C, labels_in, G_ids, np.arange(n))
    moved = int((out != np.asarray(labels_in)).sum())
    return out, best, moved


def gk_assign_rows(X, C, labels_in, G_ids, rows):
    """The same sweep for the given rows only (every row's label still enters
    the candidate lists): (labels_out int32, best_d2 float64) of those rows.
    Used to check sampled outputs of problems too large to sweep in full: X
    and G_ids need only support shape and row indexing by the rows asked for."""
    rows = np.asarray(rows, np.int64)
    C64 = np.asarray(C, np.float32).astype(np.float64)
    labels_in = np.asarray(labels_in, np.int64)
    k = C64.shape[0]
    kappa = G_ids.shape[1]
    out = np.empty(rows.size, np.int32)
    best = np.empty(rows.size, np.float64)
    for s in range(0, rows.size, CHUNK):
        e = min(rows.size, s + CHUNK)
        r = rows[s:e]
        Xb = np.asarray(X[r], np.float32).astype(np.float64)
        cur = labels_in[r]
        if kappa >= k:
            cand = np.broadcast_to(np.arange(k), (e - s, k))
        else:
            cand = candidates(cur, labels_in, np.asarray(G_ids[r], np.int64))
        out[s:e], best[s:e] = _decide(Xb, C64, cur, cand)
    return out, best


def dense_assign(X, C):
    """Exhaustive nearest centroid, ties to the smallest id (used by the random
    initialisation)."""
    X64 = np.asarray(X, np.float32).astype(np.float64)
    C64 = np.asarray(C, np.float32).astype(np.float64)
    n, k = X64.shape[0], C64.shape[0]
    out = np.empty(n, np.int32)
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        cand = np.broadcast_to(np.arange(k), (e - s, k))
        d = _dist_to(X64[s:e], C64, cand)
        out[s:e] = d.argmin(axis=1)  # argmin returns the first (smallest id) minimum
    return out


def centroid_update(X, labels, k, C_prev):
    """Means of the members of each cluster (float64 sums, float32 result)."""
    X64 = np.asarray(X, np.float32).astype(np.float64)
    labels = np.asarray(labels, np.int64)
    d = X64.shape[1]
    counts = np.bincount(labels, minlength=k).astype(np.int64)
    order = np.argsort(labels, kind="stable")
    sums = np.zeros((k, d), np.float64)
    nz = np.nonzero(counts)[0]
    if len(nz):
        starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
        sums[nz] = np.add.reduceat(X64[order], starts[nz], axis=0)
    C = np.array(C_prev, dtype=np.float32, copy=True)
    C[nz] = (sums[nz] / counts[nz, None]).astype(np.float32)
    return C, counts.astype(np.int32), sums


def distortion(X, C, labels):
    """Eqn. 4: mean over samples of ||x_i - C_{label(i)}||^2 (float64)."""
    X64 = np.asarray(X, np.float32).astype(np.float64)
    C64 = np.asarray(C, dtype=np.float64)
    diff = X64 - C64[np.asarray(labels, np.int64)]
    return float(np.einsum("ij,ij->", diff, diff) / X64.shape[0])


def distortion_identity(X, sums, counts):
    """Eqn. 2 route: with C_r the exact mean D_r / n_r,
    n*E = sum_i ||x_i||^2 - I, where I = sum_r D_r'D_r / n_r."""
    X64 = np.asarray(X, np.float32).astype(np.float64)
    counts = np.asarray(counts, np.float64)
    nz = counts > 0
    I = float((np.einsum("ij,ij->i", sums[nz], sums[nz]) / counts[nz]).sum())
    return (float(np.einsum("ij,ij->", X64, X64)) - I) / X64.shape[0]


INIT_TWOMEANS = 0
INIT_RANDOM = 1


def random_init_ids(n, k, seed):
    """k distinct sample ids (Floyd, stream RANDOM_INIT), in draw order."""
    key = rng.stream_key(seed, rng.stream_id(rng.PURPOSE_RANDOM_INIT, 0, 0))
    return np.array(rng.floyd_sample(key, n, k), dtype=np.int64)


def init_labels(X, k, seed, init, iters=2):
    X = np.asarray(X, np.float32)
    if init == INIT_RANDOM:
        ids = random_init_ids(X.shape[0], k, seed)
        C0 = X[ids].copy()
        return dense_assign(X, C0), C0
    labels = twomeans(X, k, seed, rng.ROUND_FIT, iters)
    return labels, np.zeros((k, X.shape[1]), np.float32)


def fit(X, k, G_ids, T, seed, init=INIT_TWOMEANS, bisect_iters=2, early_stop=False, labels0=None, C0=None):
    """GK-means^- fit.  labels_0 from the initialisation (Alg. 2 starts from
    Alg. 1; the random form picks k distinct rows as seeds), or given
    (labels0, with C0 holding the centroids of the clusters it leaves empty:
    the iterations of Alg. 2 continued from a partition); C_0 = means of
    labels_0.  For t = 1..T: assign with the graph, update, distortion.
    Returns (labels, C, counts, trace[E_0..E_T'], iters_run, moved list)."""
    X = np.asarray(X, np.float32)
    if labels0 is not None:
        labels = np.asarray(labels0, np.int64).copy()
        Cseed = np.asarray(C0, np.float32).copy() if C0 is not None else np.zeros((k, X.shape[1]), np.float32)
    else:
        labels, Cseed = init_labels(X, k, seed, init, bisect_iters)
    C, counts, _ = centroid_update(X, labels, k, Cseed)
    trace = [distortion(X, C, labels)]
    moved_hist = []
    it = 0
    for t in range(1, T + 1):
        labels, _, moved = gk_assign(X, C, labels, G_ids)
        C, counts, _ = centroid_update(X, labels, k, C)
        trace.append(distortion(X, C, labels))
        moved_hist.append(moved)
        it = t
        if early_stop and moved == 0:
            break
    return labels, C, counts, np.array(trace), it, moved_hist
