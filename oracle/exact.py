"""Textbook references the pins reduce to (float64).

* ``brute_knn``: the exact kappa-NN list of every row, ordered by the same stored
  key as the graph (float64 squared distance rounded to float32, then id).
* ``lloyd_assign``: exhaustive nearest centroid (Eqn. 1's q(x)), restricted to a
  subset of clusters when given, ties to the smallest id.

These are plain definitions; the tests pin them in turn against scipy
(cKDTree, cdist), which shares no code with them.
"""
import numpy as np


def sqdist_matrix(A, B):
    """float64 squared distances, direct difference form."""
    A = np.asarray(A, np.float32).astype(np.float64)
    B = np.asarray(B, np.float32).astype(np.float64)
    out = np.empty((A.shape[0], B.shape[0]), np.float64)
    step = max(1, 2_000_000 // max(1, B.shape[0] * A.shape[1]))
    for s in range(0, A.shape[0], step):
        diff = A[s : s + step, None, :] - B[None, :, :]
        out[s : s + step] = np.einsum("ijk,ijk->ij", diff, diff)
    return out


def brute_knn(X, kappa, rows=None):
    """Exact kappa-NN (self excluded) of the given rows (default: all)."""
    X = np.asarray(X, np.float32)
    n = X.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    ids = np.empty((len(rows), kappa), np.int32)
    d2 = np.empty((len(rows), kappa), np.float32)
    for s in range(0, len(rows), 256):
        r = rows[s : s + 256]
        D = sqdist_matrix(X[r], X).astype(np.float32)
        for a, i in enumerate(r):
            key_d = D[a].copy()
            idx = np.arange(n)
            mask = idx != i
            o = np.lexsort((idx[mask], key_d[mask]))[:kappa]
            ids[s + a] = idx[mask][o]
            d2[s + a] = key_d[mask][o]
    return ids, d2


def lloyd_assign(X, C, allowed=None):
    """Exhaustive argmin over centroids (or over the ``allowed`` cluster ids)."""
    D = sqdist_matrix(X, C)
    if allowed is not None:
        mask = np.full(C.shape[0], np.inf)
        mask[np.asarray(allowed)] = 0.0
        D = D + mask[None, :]
    return D.argmin(axis=1).astype(np.int32)
