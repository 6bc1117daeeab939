"""Approximate nearest-neighbour search over the built KNN graph.

Test infrastructure only: nothing in the package imports this module.

Sec. 4.3 notes that the graph of Alg. 3 also serves nearest-neighbour search
but gives no search algorithm.  The search written out here is the usual
best-first (beam) search over a KNN graph:

* a result set W of at most ef points and a candidate set C, both seeded with
  the entry points; every point is looked at once (a visited set);
* repeatedly take the closest candidate c out of C; stop when it is farther
  than the farthest of W while W is full; otherwise look at every graph
  neighbour of c not seen yet, and put it in W and C when W is not full or it
  is closer than the farthest of W (W then drops its farthest point);
* stop as well once max_visits points have been looked at;
* the answer is the top_k closest of W.

Order: points are compared by (d2, id), d2 the squared distance summed over
the dimensions in order in float64 with one rounding per operation and
rounded once to float32 (the keys of the graph, reading 16).  Entry points:
``n_entry`` distinct ids per query by Floyd's sampling keyed by
(seed, PURPOSE_SEARCH, query index) (rng.py).

``search_list`` is the same search with W and C in one sorted list of ef
entries carrying an expanded flag: the next point to expand is the first
unexpanded entry; the search ends when every entry is expanded.  It makes the
same expansions in the same order (every candidate outside W is farther than
the farthest of W, so the classic loop stops or skips at it), which the pins
check; the library implements this form.

Pins (tests/test_oracle_pins.py): with ef and max_visits at least n on a
connected graph both forms return the exact neighbours (brute force); the two
forms agree on random graphs and queries, including cut-off searches; recall
does not decrease with ef on average.
"""
import heapq

import numpy as np

from . import rng

PURPOSE_SEARCH = 5


def sq_key(q, x):
    """float32 of the float64 squared distance summed in dimension order."""
    q = np.asarray(q, np.float64)
    x = np.asarray(x, np.float64)
    acc = 0.0
    for j in range(q.shape[0]):
        df = q[j] - x[j]
        acc = acc + df * df
    return float(np.float32(acc))


def sq_keys(q, X):
    """sq_key of q against every row of X (vectorised over rows, same order
    and roundings)."""
    q = np.asarray(q, np.float64)
    X = np.atleast_2d(np.asarray(X, np.float64))
    acc = np.zeros(X.shape[0], np.float64)
    for j in range(q.shape[0]):
        df = q[j] - X[:, j]
        acc = acc + df * df
    return acc.astype(np.float32).astype(np.float64)


def entry_points(n, n_entry, seed, qi):
    key = rng.stream_key(seed, rng.stream_id(PURPOSE_SEARCH, 0, qi))
    return [int(v) for v in rng.floyd_sample(key, n, min(n_entry, n))]


def search_classic(X, G, q, entries, ef, top_k, max_visits):
    X = np.asarray(X, np.float32)
    visited = set()
    W = []  # max-heap of (-d, -id)
    C = []  # min-heap of (d, id)
    for e in entries:
        if e in visited:
            continue
        visited.add(e)
        d = sq_key(q, X[e])
        heapq.heappush(C, (d, e))
        heapq.heappush(W, (-d, -e))
        if len(W) > ef:
            heapq.heappop(W)
    while C:
        d, c = heapq.heappop(C)
        worst = (-W[0][0], -W[0][1])
        if len(W) >= ef and (d, c) > worst:
            break
        if len(visited) >= max_visits:
            break
        for b in G[c]:
            b = int(b)
            if b in visited:
                continue
            visited.add(b)
            db = sq_key(q, X[b])
            worst = (-W[0][0], -W[0][1])
            if len(W) < ef or (db, b) < worst:
                heapq.heappush(C, (db, b))
                heapq.heappush(W, (-db, -b))
                if len(W) > ef:
                    heapq.heappop(W)
    res = sorted((-a, -b) for a, b in W)
    return [i for _, i in res[:top_k]], [d for d, _ in res[:top_k]]


def search_list(X, G, q, entries, ef, top_k, max_visits):
    X = np.asarray(X, np.float32)
    visited = set()
    L = []  # sorted list of [d, id, expanded]
    for e in entries:
        if e in visited:
            continue
        visited.add(e)
        L.append([sq_key(q, X[e]), e, False])
    L.sort()
    L = L[:ef]
    while True:
        nxt = next((t for t in range(len(L)) if not L[t][2]), -1)
        if nxt < 0 or len(visited) >= max_visits:
            break
        L[nxt][2] = True
        c = L[nxt][1]
        fresh = []
        for b in G[c]:
            b = int(b)
            if b not in visited:
                visited.add(b)
                fresh.append(b)
        if fresh:
            keys = sq_keys(q, X[fresh])
            L = sorted(L + [[float(k), b, False] for k, b in zip(keys, fresh)])[:ef]
    return [e[1] for e in L[:top_k]], [e[0] for e in L[:top_k]]


def search_all(X, G, Q, ef, top_k, max_visits, n_entry, seed, form="list"):
    """Every query of Q; returns (ids, d2) arrays of shape (m, top_k) (-1 /
    inf past the end of a short answer)."""
    f = search_list if form == "list" else search_classic
    m = Q.shape[0]
    ids = np.full((m, top_k), -1, np.int64)
    d2 = np.full((m, top_k), np.inf)
    for i in range(m):
        a, b = f(X, G, Q[i], entry_points(X.shape[0], n_entry, seed, i), ef, top_k, max_visits)
        ids[i, :len(a)] = a
        d2[i, :len(b)] = b
    return ids, d2
