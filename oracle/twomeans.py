"""Alg. 1 (TwoMeans, the two-means tree) in float64.

The paper's loop pops the largest cluster, bisects it, adjusts the two halves
to equal size and pushes both back until k clusters exist (Alg. 1; Sec. 3.2).
Readings where the listing is silent (listed in the design notes):

* Schedule.  With exactly balanced splits every node of depth j holds
  floor(n/2^j) or ceil(n/2^j) samples, so "pop the largest" finishes a depth
  before the next one starts.  Full depths are split while 2*nodes <= k; at the
  last depth the (k - nodes) largest nodes are split, ties to the lower node
  index.
* Bisection of a node S (members in ascending id order): two distinct members
  drawn from stream (TWOMEANS, round, 2^depth + node) seed the two centroids;
  ``iters`` Lloyd 2-means steps follow (assign to u when ||x-c_u||^2 <=
  ||x-c_v||^2; each centroid becomes the float64 mean of its side, stored in
  float32; an empty side keeps its centroid).
* "Adjust to equal size": members are ordered by
  (delta = ||x-c_u||^2 - ||x-c_v||^2, id) with the final centroids; the first
  ceil(s/2) form the left child, the rest the right child.
* Leaves are numbered left to right.

The paper also folds boost k-means into the bisection (Sec. 3.2); this
implementation uses Lloyd 2-means steps instead (a stated reading).

Pins (tests/test_oracle_pins.py): hand-worked 2-D bisections
(tests/golden/bisect_2d.json: the two Lloyd steps spelled out, a distance tie
that goes to u, an empty side that keeps its centroid, a delta tie that only
float32-rounded centroids produce); the bisection's centroids equal scipy's
kmeans2 run for the same two steps from the same seeds; the level-synchronous
schedule gives the leaves, in order, of a literal priority-queue run of Alg. 1;
balanced sizes and the delta-order invariant at every split; d = 1 with k = 2^L
gives the equal-frequency quantile bins of the sorted data (an independent
np.argsort route); k = 1 gives all zeros and k = n gives singletons.
"""
import numpy as np

from . import rng


def tree_shape(n, k):
    """Sizes of the nodes at each depth, and which nodes split, for n samples into
    k leaves.  Returns a list of (sizes, split_flags) per depth that is split."""
    assert 1 <= k <= n
    sizes = [n]
    out = []
    while len(sizes) < k:
        m = len(sizes)
        if 2 * m <= k:
            flags = [True] * m
        else:
            need = k - m
            order = sorted(range(m), key=lambda i: (-sizes[i], i))
            chosen = set(order[:need])
            flags = [i in chosen for i in range(m)]
        out.append((list(sizes), flags))
        nxt = []
        for s, f in zip(sizes, flags):
            if f:
                nxt += [(s + 1) // 2, s // 2]
            else:
                nxt.append(s)
        sizes = nxt
    return out


def _sqdist(A, c):
    diff = A - c[None, :]
    return np.einsum("ij,ij->i", diff, diff)


def seed_pair(seed, rnd, depth, node, s):
    """Positions (r0, r1), 0 <= r0 != r1 < s, of the two members whose rows seed
    the bisection of node ``node`` at depth ``depth`` (Alg. 1 starts each split
    from two samples): counter draws 0 and 1 of stream (TWOMEANS, rnd,
    2^depth + node); r1 is drawn over the s - 1 other positions."""
    key = rng.stream_key(seed, rng.stream_id(rng.PURPOSE_TWOMEANS, rnd, (1 << depth) + node))
    r0 = rng.below(rng.draw(key, 0), s)
    r1 = rng.below(rng.draw(key, 1), s - 1)
    if r1 >= r0:
        r1 += 1
    return r0, r1


def lloyd_steps(A, cu, cv, iters):
    """``iters`` Lloyd 2-means steps from the centroids (cu, cv) over the rows A
    (float64): a row joins u when ||x-c_u||^2 <= ||x-c_v||^2, then each centroid
    becomes the float64 mean of its side stored in float32; a side with no rows
    keeps its centroid.  Returns the final (c_u, c_v) as float64 arrays holding
    float32 values."""
    cu = np.asarray(cu, np.float32).astype(np.float64)
    cv = np.asarray(cv, np.float32).astype(np.float64)
    for _ in range(iters):
        to_u = _sqdist(A, cu) <= _sqdist(A, cv)
        if to_u.any():
            cu = A[to_u].mean(axis=0).astype(np.float32).astype(np.float64)
        if (~to_u).any():
            cv = A[~to_u].mean(axis=0).astype(np.float32).astype(np.float64)
    return cu, cv


def split_node(A, members, r0, r1, iters=2):
    """Bisect the node whose rows are A (float64, in the order of ``members``,
    ascending ids) from the seed rows at positions r0 and r1: Lloyd steps, then
    "adjust to equal size" (Alg. 1): members ordered by (delta, id) with
    delta = ||x-c_u||^2 - ||x-c_v||^2 at the final centroids; the first
    ceil(s/2) form the left child.  Returns (left, right, c_u, c_v) with the
    children in ascending id order and the centroids as float32."""
    members = np.asarray(members)
    s = len(members)
    cu, cv = lloyd_steps(A, A[r0], A[r1], iters)
    delta = _sqdist(A, cu) - _sqdist(A, cv)
    order = np.lexsort((members, delta))
    h = (s + 1) // 2
    left = np.sort(members[order[:h]])
    right = np.sort(members[order[h:]])
    return left, right, cu.astype(np.float32), cv.astype(np.float32)


def bisect(X64, members, seed, rnd, depth, node, iters=2):
    """Split one node; returns (left, right) member arrays in ascending id order
    and the final (c_u, c_v) as float32."""
    s = len(members)
    assert s >= 2
    r0, r1 = seed_pair(seed, rnd, depth, node, s)
    return split_node(X64[members], members, r0, r1, iters)


def twomeans(X, k, seed, rnd=rng.ROUND_FIT, iters=2, return_nodes=False):
    """Alg. 1: labels in [0, k) for the rows of X (float32 n x d)."""
    X64 = np.asarray(X, dtype=np.float32).astype(np.float64)
    n = X64.shape[0]
    assert 1 <= k <= n
    nodes = [np.arange(n, dtype=np.int64)]
    depth = 0
    while len(nodes) < k:
        m = len(nodes)
        if 2 * m <= k:
            split = [True] * m
        else:
            order = sorted(range(m), key=lambda i: (-len(nodes[i]), i))
            chosen = set(order[: k - m])
            split = [i in chosen for i in range(m)]
        nxt = []
        for idx, (S, f) in enumerate(zip(nodes, split)):
            if f:
                L, R, _, _ = bisect(X64, S, seed, rnd, depth, idx, iters)
                nxt += [L, R]
            else:
                nxt.append(S)
        nodes = nxt
        depth += 1
    labels = np.empty(n, dtype=np.int32)
    for r, S in enumerate(nodes):
        labels[S] = r
    if return_nodes:
        return labels, nodes
    return labels
