"""The boost form of GK-means (Alg. 2 as printed; Sec. 3.1, Eqn. 3).

Test infrastructure only: nothing in the package imports this module.

Alg. 2 moves one sample at a time: x_i goes from its cluster u to the cluster
v of its neighbours' clusters that maximises the gain of the objective
I = sum_r D_r'D_r / n_r (Eqn. 2), as soon as that gain (Eqn. 3) is positive.
Two forms are written out here:

* ``boost_sequential`` -- the printed algorithm: samples in index order,
  every positive move applied at once (D, n updated before the next sample).
* ``boost_rounds`` -- the data-parallel reading the library implements.  In a
  round every sample computes its best move against the same state; each
  cluster then keeps, among the positive moves touching it (as source or as
  target), the one with the largest priority key, and exactly the moves that
  keep both of their clusters are applied.  No two applied moves share a
  cluster, so each one's gain is unchanged by the others and I rises by
  exactly their sum: the round equals the same moves made one after the other
  by Alg. 2, in any order.

Arithmetic (shared reading with the library, so that decisions agree bit for
bit): D_r is the exact sum of the float32 rows of cluster r rounded once to
float64 (math.fsum), the mean c_r = D_r / n_r in float64; the gain of Eqn. 3
is evaluated in the equivalent form

    dI(x, u -> v) = n_u/(n_u-1) ||x - c_u||^2 - n_v/(n_v+1) ||x - c_v||^2

(the first term 0 when n_u = 1: the move empties u), with every squared
distance summed over the dimensions in order, one rounding per operation
(no fused multiply-add), and the coefficients as float64 quotients.  The best
target is the smallest weighted distance n_v/(n_v+1)||x - c_v||^2 over the
clusters of the neighbours other than u (smallest id among equal ones); the
move is proposed when the own weighted distance is strictly larger.

Priority of a proposal in round t: (h << 32) | i, where h is the top 32 bits
of the first SplitMix64 draw of stream (PURPOSE_BOOST, t, i) under the fit's
seed (rng.py); larger wins.

Pins (tests/test_oracle_pins.py): Eqn. 3 written out literally equals the
weighted form and the brute-force change of I for random moves; a hand-worked
1-D case where the boost rule moves a sample that the Lloyd rule keeps;
two proposals on one cluster apply only the larger key; a round's change of I
equals the sum of its applied gains and equals the same moves applied one by
one with Eqn. 3; I never decreases; a state with no proposal is a fixed point
of both forms.
"""
import math

import numpy as np

from . import rng

PURPOSE_BOOST = 4


def composite(X, labels, k):
    """D_r (exact sums rounded once to float64) and n_r."""
    X = np.asarray(X, np.float32)
    labels = np.asarray(labels, np.int64)
    d = X.shape[1]
    n_r = np.bincount(labels, minlength=k).astype(np.int64)
    D = np.zeros((k, d), np.float64)
    order = np.argsort(labels, kind="stable")
    starts = np.concatenate([[0], np.cumsum(n_r)])
    for r in np.nonzero(n_r)[0]:
        rows = X[order[starts[r]:starts[r + 1]]].astype(np.float64)
        for j in range(d):
            D[r, j] = math.fsum(rows[:, j])
    return D, n_r


def objective(D, n_r):
    """I = sum_r D_r'D_r / n_r over non-empty clusters (Eqn. 2)."""
    nz = n_r > 0
    return float(sum(math.fsum(D[r] * D[r]) / n_r[r] for r in np.nonzero(nz)[0]))


def delta_I(x, D_u, n_u, D_v, n_v):
    """Eqn. 3 written out: the change of I when x moves from u to v (an empty
    cluster, before or after the move, contributes nothing)."""
    x = np.asarray(x, np.float64)
    a = D_v + x
    b = D_u - x
    t1 = float(a @ a) / (n_v + 1)
    t2 = float(b @ b) / (n_u - 1) if n_u > 1 else 0.0
    t3 = float(D_v @ D_v) / n_v if n_v > 0 else 0.0
    t4 = float(D_u @ D_u) / n_u
    return t1 + t2 - t3 - t4


def sq_dist_seq(x, c):
    """||x - c||^2 summed over the dimensions in order, rows of c at once
    (one rounding per subtraction, square and addition)."""
    x = np.asarray(x, np.float64)
    c = np.atleast_2d(np.asarray(c, np.float64))
    acc = np.zeros(c.shape[0], np.float64)
    for j in range(x.shape[0]):
        df = x[j] - c[:, j]
        acc = acc + df * df
    return acc


def weights(n_r, own):
    """Coefficient of a cluster of n_r members: n/(n-1) for the own cluster
    (0 when n = 1), n/(n+1) for a target."""
    n = np.asarray(n_r, np.float64)
    if own:
        return np.where(n > 1, n / np.maximum(n - 1.0, 1.0), 0.0)
    return n / (n + 1.0)


def best_move(x, u, cand, D, n_r):
    """(v, dI) of the best move of x out of u among the clusters `cand`
    (other than u), or (-1, 0) when none is positive."""
    cand = np.array(sorted(set(int(c) for c in cand) - {int(u)}), np.int64)
    if len(cand) == 0:
        return -1, 0.0
    means = D[np.concatenate([[u], cand])] / n_r[np.concatenate([[u], cand])][:, None]
    dist = sq_dist_seq(x, means)
    w_u = weights(n_r[u], True) * dist[0]
    w = weights(n_r[cand], False) * dist[1:]
    j = int(np.argmin(w))  # first minimum: the smallest id (cand is sorted)
    if w_u > w[j]:
        return int(cand[j]), float(w_u - w[j])
    return -1, 0.0


def priority(seed, rnd, i):
    key = rng.stream_key(seed, rng.stream_id(PURPOSE_BOOST, rnd, i))
    return ((rng.draw(key, 0) >> 32) << 32) | (i & 0xFFFFFFFF)


def boost_round(X, labels, G, D, n_r, seed, rnd):
    """One data-parallel round.  Returns (new labels, applied moves as a list
    of (i, u, v, gain), number of proposals)."""
    X = np.asarray(X, np.float32)
    labels = np.asarray(labels, np.int64)
    props = []
    for i in range(X.shape[0]):
        u = labels[i]
        v, g = best_move(X[i], u, labels[G[i]], D, n_r)
        if v >= 0:
            props.append((i, u, v, g, priority(seed, rnd, i)))
    win = {}
    for i, u, v, g, key in props:
        for r in (u, v):
            if key > win.get(r, -1):
                win[r] = key
    applied = [(i, u, v, g) for i, u, v, g, key in props if win[u] == key and win[v] == key]
    out = labels.copy()
    for i, u, v, g in applied:
        out[i] = v
    return out, applied, len(props)


def boost_rounds(X, k, G, labels0, T, seed, C0=None):
    """Up to T rounds from labels0 (stops after a round with no proposal).
    Returns (labels, C float32 means (C0 kept for empty clusters), counts,
    trace E_0..E_t (Eqn. 4 through Eqn. 2), rounds run, moves per round)."""
    X = np.asarray(X, np.float32)
    n = X.shape[0]
    sxx = math.fsum(np.einsum("ij,ij->i", X.astype(np.float64), X.astype(np.float64)))
    labels = np.asarray(labels0, np.int64).copy()
    D, n_r = composite(X, labels, k)
    trace = [(sxx - objective(D, n_r)) / n]
    moves = []
    t = 0
    for t in range(1, T + 1):
        labels, applied, nprop = boost_round(X, labels, G, D, n_r, seed, t)
        D, n_r = composite(X, labels, k)
        trace.append((sxx - objective(D, n_r)) / n)
        moves.append(len(applied))
        if nprop == 0:
            break
    C = np.zeros((k, X.shape[1]), np.float32) if C0 is None else np.array(C0, np.float32, copy=True)
    nz = n_r > 0
    C[nz] = (D[nz] / n_r[nz, None]).astype(np.float32)
    return labels, C, n_r.astype(np.int32), np.array(trace), t, moves


def boost_sequential(X, k, G, labels0, iters):
    """Alg. 2 as printed: each iteration visits the samples in index order and
    moves a sample as soon as its best gain (Eqn. 3, over the clusters of its
    neighbours) is positive.  Returns (labels, I after each iteration, moves
    per iteration)."""
    X = np.asarray(X, np.float32)
    labels = np.asarray(labels0, np.int64).copy()
    D, n_r = composite(X, labels, k)
    Is, mv = [], []
    for _ in range(iters):
        m = 0
        for i in range(X.shape[0]):
            u = labels[i]
            v, g = best_move(X[i], u, labels[G[i]], D, n_r)
            if v >= 0:
                x = X[i].astype(np.float64)
                D[u] -= x
                D[v] += x
                n_r[u] -= 1
                n_r[v] += 1
                labels[i] = v
                m += 1
        Is.append(objective(D, n_r))
        mv.append(m)
        if m == 0:
            break
    return labels, Is, mv
