"""Pins of the FP64 oracle against things other than itself: published values,
library routines (scipy, pandas), closed forms, invariants and hand-worked
fixtures.  CPU only."""
import json
import os

import numpy as np
import pytest
from scipy.cluster.vq import vq
from scipy.spatial import cKDTree
from scipy.spatial.distance import cdist

from oracle import exact, gkmeans, knng, metrics, rng, twomeans
from paper_1705_01813_amd import datagen

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- RNG ----

def test_splitmix64_published_sequence():
    vals = [int(l, 16) for l in open(os.path.join(GOLD, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    got = [rng.draw(0, c) for c in range(len(vals))]
    assert got == vals
    got_np = [int(rng.draw_np(np.zeros(1, np.uint64), c)[0]) for c in range(len(vals))]
    assert got_np == vals


def test_below_and_floyd_are_uniform_and_distinct():
    key = rng.stream_key(7, rng.stream_id(rng.PURPOSE_GRAPH_INIT, 0, 3))
    s = rng.floyd_sample(key, 1000, 1000)
    assert sorted(s) == list(range(1000))
    # chi-square on below(): 64 bins, 64k draws
    r = rng.draw_np(np.full(65536, rng.stream_key(1, 2), np.uint64), 0)
    keys = rng.mix64_np(np.arange(65536, dtype=np.uint64))
    v = rng.below_np(rng.draw_np(keys, 0), 64).astype(np.int64)
    h = np.bincount(v, minlength=64)
    chi2 = ((h - 1024.0) ** 2 / 1024.0).sum()
    assert chi2 < 120  # 63 dof: p ~ 1e-5 threshold
    # Floyd: every value equally likely to be chosen (m=20, cnt=5, 20000 rows)
    keys = rng.mix64_np(np.arange(20000, dtype=np.uint64) + np.uint64(99))
    rows = rng.floyd_sample_rows(keys, 20, 5)
    assert all(len(set(r)) == 5 for r in rows[:200])
    cnt = np.bincount(rows.ravel(), minlength=20)
    exp = 20000 * 5 / 20
    assert (((cnt - exp) ** 2) / exp).sum() < 50
    # vectorised rows equal the scalar algorithm
    for r in range(5):
        assert list(rows[r]) == rng.floyd_sample(int(keys[r]), 20, 5)


# ------------------------------------------------------- assignment ----

@pytest.mark.parametrize("case", [0, 1])
def test_assign_hand_worked(case):
    c = _gold("assign_1d.json")["cases"][case]
    lab, best, moved = gkmeans.gk_assign(np.array(c["X"], np.float32), np.array(c["C"], np.float32),
                                         np.array(c["labels_in"]), np.array(c["G"]))
    assert lab.tolist() == c["labels_out"]
    assert np.allclose(best, c["best_d2"])
    assert moved == c["moved"]


def test_assign_kappa_ge_k_is_lloyd():
    X = datagen.mixture(600, 8, 12, seed=3, sigma=1.5)
    rs = np.random.default_rng(0)
    C = X[rs.choice(600, 10, replace=False)] + 0.1
    labels_in = rs.integers(0, 10, 600)
    G = np.stack([rs.choice(np.delete(np.arange(600), i), 10, replace=False) for i in range(600)])
    lab, _, _ = gkmeans.gk_assign(X, C, labels_in, G)
    ref = cdist(X.astype(np.float64), C.astype(np.float64), "sqeuclidean").argmin(1)
    assert (lab == ref).all()


def test_assign_complete_graph_is_lloyd_over_nonempty():
    X = datagen.mixture(120, 5, 6, seed=5, sigma=2.0)
    k = 40
    rs = np.random.default_rng(1)
    C = rs.normal(size=(k, 5)).astype(np.float32) * 8
    labels_in = rs.integers(0, 25, 120)  # clusters 25..39 hold no sample
    G = np.stack([np.delete(np.arange(120), i) for i in range(120)])  # kappa = n-1 = 119 >= k
    G = G[:, :119]
    # kappa >= k: candidates are all clusters -> plain Lloyd
    lab_all, _, _ = gkmeans.gk_assign(X, C, labels_in, G)
    assert (lab_all == cdist(X.astype(np.float64), C.astype(np.float64), "sqeuclidean").argmin(1)).all()
    # kappa < k with the complete graph (k raised above n-1): candidates are the
    # non-empty clusters, so the sweep is Lloyd restricted to them
    k2 = 200
    C2 = np.concatenate([C, rs.normal(size=(k2 - k, 5)).astype(np.float32)])
    lab, _, _ = gkmeans.gk_assign(X, C2, labels_in, G)
    D = cdist(X.astype(np.float64), C2.astype(np.float64), "sqeuclidean")
    allowed = np.unique(labels_in)
    ref = allowed[D[:, allowed].argmin(1)]
    assert (lab == ref).all()


def test_assign_tiny_enumeration():
    """n <= 12: Q_i written out element by element with Python sets."""
    rs = np.random.default_rng(2)
    for trial in range(20):
        n, d, k, kappa = 12, 3, 5, 3
        X = rs.normal(size=(n, d)).astype(np.float32)
        C = rs.normal(size=(k, d)).astype(np.float32)
        lab_in = rs.integers(0, k, n)
        G = np.stack([rs.choice(np.delete(np.arange(n), i), kappa, replace=False) for i in range(n)])
        lab, _, _ = gkmeans.gk_assign(X, C, lab_in, G)
        for i in range(n):
            Q = {int(lab_in[i])} | {int(lab_in[j]) for j in G[i]}
            dist = {q: float(sum((float(X[i, t]) - float(C[q, t])) ** 2 for t in range(d))) for q in Q}
            m = min(dist.values())
            want = int(lab_in[i]) if dist[int(lab_in[i])] == m else min(q for q in Q if dist[q] == m)
            assert lab[i] == want


def test_assign_enumeration_beyond_one_block():
    """n spans several of the oracle's row blocks: sampled rows enumerated by
    hand must agree (neighbour labels come from the whole label array)."""
    rs = np.random.default_rng(12)
    n, d, k, kappa = 9000, 4, 300, 6
    X = rs.normal(size=(n, d)).astype(np.float32)
    C = rs.normal(size=(k, d)).astype(np.float32)
    lab_in = rs.integers(0, k, n)
    G = rs.integers(0, n, size=(n, kappa))
    lab, _, moved = gkmeans.gk_assign(X, C, lab_in, G)
    for i in list(rs.choice(n, 200, replace=False)) + [0, 4095, 4096, 8191, 8192, n - 1]:
        Q = {int(lab_in[i])} | {int(lab_in[j]) for j in G[i]}
        dist = {q: float(sum((float(X[i, t]) - float(C[q, t])) ** 2 for t in range(d))) for q in Q}
        m = min(dist.values())
        want = int(lab_in[i]) if dist[int(lab_in[i])] == m else min(q for q in Q if dist[q] == m)
        assert lab[i] == want
    assert moved == int((lab != lab_in).sum())


def test_assign_rows_restricted():
    """gk_assign_rows on sampled rows (any order, a row repeated) returns each
    row's label and best distance as written out by hand from the whole label
    array, and the same rows of the full sweep; kappa >= k included."""
    rs = np.random.default_rng(21)
    for n, d, k, kappa in [(9000, 4, 300, 6), (500, 3, 4, 6)]:
        X = rs.normal(size=(n, d)).astype(np.float32)
        C = rs.normal(size=(k, d)).astype(np.float32)
        lab_in = rs.integers(0, k, n)
        G = rs.integers(0, n, size=(n, kappa))
        rows = np.concatenate([rs.choice(n, 300, replace=False), [0, n - 1, 0]])
        lab, best = gkmeans.gk_assign_rows(X, C, lab_in, G, rows)
        full, full_best, _ = gkmeans.gk_assign(X, C, lab_in, G)
        assert np.array_equal(lab, full[rows]) and np.array_equal(best, full_best[rows])
        for t, i in enumerate(rows):
            Q = set(range(k)) if kappa >= k else {int(lab_in[i])} | {int(lab_in[j]) for j in G[i]}
            dist = {q: float(sum((float(X[i, u]) - float(C[q, u])) ** 2 for u in range(d))) for q in Q}
            m = min(dist.values())
            want = int(lab_in[i]) if dist[int(lab_in[i])] == m else min(q for q in Q if dist[q] == m)
            assert lab[t] == want
            assert abs(best[t] - dist[want]) <= 1e-12 * max(1.0, dist[want])


# ----------------------------------------------------------- update ----

def test_update_hand_worked_and_identity():
    u = _gold("assign_1d.json")["update"]
    X = np.array(u["X"], np.float32)
    C, counts, sums = gkmeans.centroid_update(X, np.array(u["labels"]), 4, np.array(u["C_prev"], np.float32))
    assert np.allclose(C, np.array(u["C"], np.float32))
    assert counts.tolist() == u["counts"]
    E_exact_means = gkmeans.distortion(X, np.where(counts[:, None] > 0, sums / np.maximum(counts, 1)[:, None], 0),
                                       np.array(u["labels"]))
    assert abs(E_exact_means - u["E"]) < 1e-12
    assert abs(gkmeans.distortion_identity(X, sums, counts) - u["E"]) < 1e-12


def test_update_matches_pandas_groupby():
    import pandas as pd

    X = datagen.mixture(3000, 7, 20, seed=8)
    labels = np.random.default_rng(3).integers(0, 50, 3000)
    labels[labels == 17] = 18  # make cluster 17 empty
    Cprev = np.full((50, 7), -1.0, np.float32)
    C, counts, sums = gkmeans.centroid_update(X, labels, 50, Cprev)
    df = pd.DataFrame(X.astype(np.float64))
    df["l"] = labels
    g = df.groupby("l")
    mean = g.mean()
    assert (counts[mean.index] == g.size().values).all()
    assert counts.sum() == 3000 and counts[17] == 0
    assert np.array_equal(C[mean.index], mean.values.astype(np.float32))
    assert (C[17] == -1).all()
    assert np.allclose(counts[:, None] * C.astype(np.float64), sums, rtol=1e-6)


def test_update_integer_data_sums_exact():
    import pandas as pd

    X = datagen.integer_grid(5000, 16, seed=4)
    labels = np.random.default_rng(5).integers(0, 64, 5000)
    _, counts, sums = gkmeans.centroid_update(X, labels, 64, np.zeros((64, 16), np.float32))
    df = pd.DataFrame(X.astype(np.int64))
    df["l"] = labels
    ref = df.groupby("l").sum().values.astype(np.float64)
    assert np.array_equal(sums, ref)  # integer sums far below 2^53 are exact


# -------------------------------------------------------- distortion ----

def test_distortion_matches_vq_and_identity():
    X = datagen.mixture(4000, 12, 30, seed=9)
    labels = np.random.default_rng(6).integers(0, 30, 4000)
    C, counts, sums = gkmeans.centroid_update(X, labels, 30, np.zeros((30, 12), np.float32))
    E = gkmeans.distortion(X, C, labels)
    # scipy.cluster.vq: distance of each sample to its own code (a code book of one row each)
    dist = np.array([vq(X[i:i + 1].astype(np.float64), C[labels[i]:labels[i] + 1].astype(np.float64))[1][0]
                     for i in range(0, 4000, 1)])
    assert abs(E - (dist ** 2).mean()) <= 1e-10 * E
    means = sums / counts[:, None]
    assert abs(gkmeans.distortion(X, means, labels) - gkmeans.distortion_identity(X, sums, counts)) <= 1e-12 * E


def test_fit_distortion_never_increases():
    X = datagen.mixture(2000, 6, 25, seed=10)
    G, _ = exact.brute_knn(X, 8)
    for init in (gkmeans.INIT_RANDOM, gkmeans.INIT_TWOMEANS):
        lab, C, counts, trace, it, moved = gkmeans.fit(X, 25, G, 10, seed=3, init=init)
        assert (np.diff(trace) <= 1e-12 * trace[0]).all(), trace
        assert counts.sum() == 2000
        # every centroid equals the mean of its members
        C2, _, _ = gkmeans.centroid_update(X, lab, 25, C)
        assert np.array_equal(C, C2)
        # a further sweep from a fixed point moves nothing
        if moved[-1] == 0:
            l2, _, m2 = gkmeans.gk_assign(X, C, lab, G)
            assert m2 == 0 and (l2 == lab).all()


def test_fit_resumed_from_its_labels_continues_it():
    """Alg. 2's iterations continued from a partition: T1 sweeps, then T2
    sweeps from the labels and centroids they end with, are the T1 + T2
    sweeps of one fit (an empty cluster keeps the centroid it had)."""
    X = datagen.mixture(1500, 5, 30, seed=12)
    G, _ = exact.brute_knn(X, 6)
    k = 40  # more clusters than components: some empty out along the way
    for init in (gkmeans.INIT_RANDOM, gkmeans.INIT_TWOMEANS):
        lab, C, cnt, tr, _, mv = gkmeans.fit(X, k, G, 7, seed=5, init=init)
        l1, C1, _, t1, _, _ = gkmeans.fit(X, k, G, 3, seed=5, init=init)
        l2, C2, c2, t2, _, mv2 = gkmeans.fit(X, k, G, 4, seed=0, labels0=l1, C0=C1)
        assert np.array_equal(l2, lab) and np.array_equal(C2, C) and np.array_equal(c2, cnt)
        assert mv2 == mv[3:]
        assert t2[0] == t1[-1] and np.array_equal(t2[1:], tr[4:])


def test_random_init_labels_are_exhaustive_argmin():
    X = datagen.mixture(500, 4, 10, seed=11)
    lab0, C0 = gkmeans.init_labels(X, 10, 5, gkmeans.INIT_RANDOM)
    ids = gkmeans.random_init_ids(500, 10, 5)
    assert len(set(ids.tolist())) == 10
    assert np.array_equal(C0, X[ids])
    assert (lab0 == cdist(X.astype(np.float64), C0.astype(np.float64), "sqeuclidean").argmin(1)).all()


# ---------------------------------------------------------- TwoMeans ----

def _check_tree(X, k, seed):
    lab, nodes = twomeans.twomeans(X, k, seed, 0, return_nodes=True)
    n = X.shape[0]
    assert len(nodes) == k
    assert np.array_equal(np.sort(np.concatenate(nodes)), np.arange(n))
    sizes = sorted({len(S) for S in nodes})
    assert len(sizes) <= 4
    # shape predicted from (n, k) alone
    shape = twomeans.tree_shape(n, k)
    return lab, nodes, shape


def _sides(A, cu, cv):
    """Rows joining u and v, written out with Python floats (u on a tie)."""
    u, v = [], []
    for r, x in enumerate(A.tolist()):
        du = sum((a - b) ** 2 for a, b in zip(x, cu))
        dv = sum((a - b) ** 2 for a, b in zip(x, cv))
        (u if du <= dv else v).append(r)
    return u, v


@pytest.mark.parametrize("case", [0, 1, 2])
def test_bisect_hand_worked(case):
    """Hand-worked two-step bisections (tests/golden/bisect_2d.json): the
    centroids after each Lloyd step, and the children.  The cases hold a
    distance tie that must go to u, an empty side that keeps its centroid, and
    a delta tie that exists only for the float32-rounded mean."""
    c = _gold("bisect_2d.json")["cases"][case]
    A = np.array(c["A"], np.float32).astype(np.float64)
    members = np.array(c["members"])
    prev = (c["A"][c["r0"]], c["A"][c["r1"]])
    for it, st in enumerate(c["after_step"], 1):
        # the fixture's sides follow from the previous centroids
        assert _sides(A, *prev) == (st["u"], st["v"])
        cu, cv = twomeans.lloyd_steps(A, A[c["r0"]], A[c["r1"]], it)
        assert cu.tolist() == st["c_u"] and cv.tolist() == st["c_v"]
        prev = (st["c_u"], st["c_v"])
    L, R, cu, cv = twomeans.split_node(A, members, c["r0"], c["r1"], 2)
    assert L.tolist() == c["left"] and R.tolist() == c["right"]
    assert cu.tolist() == c["after_step"][-1]["c_u"] and cv.tolist() == c["after_step"][-1]["c_v"]


def test_bisect_matches_scipy_kmeans2():
    """The bisection's final centroids equal scipy's kmeans2 run for the same
    two Lloyd steps from the same seed rows (tie-free data; kmeans2 keeps
    float64 means, so they agree within float32 rounding).  One or three steps
    of kmeans2 land far away on this data, so the step count is pinned."""
    from scipy.cluster.vq import kmeans2

    for s in range(6):
        X = datagen.mixture(400, 4, 3, seed=100 + s, sigma=4.0)
        A = X.astype(np.float64)
        r0, r1 = twomeans.seed_pair(7, 0, 3, s, 400)
        _, _, cu, cv = twomeans.bisect(A, np.arange(400), 7, 0, 3, s, 2)
        got = np.stack([cu, cv]).astype(np.float64)
        scale = np.abs(A).max()
        for it in (1, 2, 3):
            cb, _ = kmeans2(A, A[[r0, r1]].copy(), iter=it, minit="matrix", missing="warn")
            err = np.abs(cb - got).max()
            if it == 2:
                assert err <= 4 * np.finfo(np.float32).eps * scale, err
            elif s != 5:  # seed pair 5 has converged by the second step
                assert err > 1e-3 * scale


def test_seed_pair_distinct_and_uniform():
    """Seed positions are two distinct members; over many nodes every ordered
    pair of positions is about equally likely (chi-square, s = 6)."""
    cnt = np.zeros((6, 6))
    for node in range(30000):
        r0, r1 = twomeans.seed_pair(3, 1, 15, node, 6)
        assert 0 <= r0 < 6 and 0 <= r1 < 6 and r0 != r1
        cnt[r0, r1] += 1
    exp = 30000 / 30.0
    off = ~np.eye(6, dtype=bool)
    assert (((cnt[off] - exp) ** 2) / exp).sum() < 70  # 29 dof, p ~ 1e-4


def _pq_leaves(n, k):
    """Alg. 1 as a literal priority queue: pop the largest cluster, split it
    into ceil(s/2) and floor(s/2), push both, until k clusters exist.  Ties in
    size go to the shallower cluster, then the leftmost (the paper leaves ties
    open).  Returns the leaf sizes from left to right."""
    import heapq

    heap = [(-n, 0, ())]  # (-size, depth, path from the root: 0 left, 1 right)
    while len(heap) < k:
        neg, depth, path = heapq.heappop(heap)
        s = -neg
        heapq.heappush(heap, (-((s + 1) // 2), depth + 1, path + (0,)))
        heapq.heappush(heap, (-(s // 2), depth + 1, path + (1,)))
    return [-neg for neg, _, _ in sorted(heap, key=lambda t: t[2])]


def _shape_leaves(n, k):
    shape = twomeans.tree_shape(n, k)
    if not shape:
        return [n]
    sizes, flags = shape[-1]
    return [c for s, f in zip(sizes, flags) for c in (((s + 1) // 2, s // 2) if f else (s,))]


@pytest.mark.parametrize("n", [1000, 2047, 10007])
def test_level_synchronous_schedule_is_pop_the_largest(n):
    """Splitting depth by depth (the last depth: the largest nodes, leftmost
    first) gives the same leaves, in order, as the literal pop-the-largest
    queue of Alg. 1, and the oracle's tree puts exactly those sizes in its
    leaves 0..k-1."""
    for k in (1, 2, 7, 100, 299, 777, n // 3, n - 1, n):
        want = _pq_leaves(n, k)
        assert _shape_leaves(n, k) == want, (n, k)
        if n == 1000 and k in (7, 100, 299, 777):
            X = datagen.mixture(n, 3, 9, seed=k)
            lab = twomeans.twomeans(X, k, seed=2, rnd=0)
            assert np.bincount(lab, minlength=k).tolist() == want


@pytest.mark.parametrize("n,k", [(1000, 7), (1000, 16), (777, 100), (64, 64), (50, 1), (300, 299)])
def test_twomeans_balanced(n, k):
    X = datagen.mixture(n, 5, 9, seed=n + k)
    lab, nodes, shape = _check_tree(X, k, seed=1)
    sizes = [len(S) for S in nodes]
    if k == n:
        assert sizes == [1] * n
    if k == 1:
        assert (lab == 0).all()
    assert np.bincount(lab, minlength=k).tolist() == sizes


def test_twomeans_split_invariant():
    X = datagen.mixture(500, 6, 5, seed=3).astype(np.float32)
    X64 = X.astype(np.float64)
    S = np.arange(500)
    L, R, cu, cv = twomeans.bisect(X64, S, seed=4, rnd=0, depth=0, node=0)
    assert len(L) == 250 and len(R) == 250
    du = ((X64 - cu.astype(np.float64)) ** 2).sum(1)
    dv = ((X64 - cv.astype(np.float64)) ** 2).sum(1)
    delta = du - dv
    assert delta[L].max() <= delta[R].min()


@pytest.mark.parametrize("L", [1, 2, 3, 5])
def test_twomeans_1d_quantile_bins(L):
    """d=1, k=2^L: delta is monotone in x, so every leaf is a run of consecutive
    values of the sorted data with the balanced sizes."""
    rs = np.random.default_rng(L)
    n = 1000 + 37 * L
    X = rs.normal(size=(n, 1)).astype(np.float32)
    lab = twomeans.twomeans(X, 2 ** L, seed=9, rnd=0)
    order = np.argsort(X[:, 0], kind="stable")
    runs = lab[order]
    changes = np.count_nonzero(np.diff(runs))
    assert changes == 2 ** L - 1  # each leaf is one contiguous run
    sizes = np.bincount(lab)
    expected = [n]
    for _ in range(L):
        expected = [s for e in expected for s in ((e + 1) // 2, e // 2)]
    assert sorted(sizes.tolist()) == sorted(expected)


# ------------------------------------------------------------- graph ----

def test_graph_hand_worked():
    g = _gold("assign_1d.json")["graph"]
    X = np.array(g["X"], np.float32)
    ids, d2 = knng.knn_build(X, g["kappa"], xi=50, tau=1, seed=3)
    assert ids.tolist() == g["ids"]
    assert d2.tolist() == g["d2"]


def _check_rows(X, ids, d2):
    X64 = X.astype(np.float64)
    n, kappa = ids.shape
    for i in range(n):
        assert i not in ids[i]
        assert len(set(ids[i].tolist())) == kappa
        key = list(zip(d2[i].tolist(), ids[i].tolist()))
        assert key == sorted(key)
        rec = ((X64[ids[i]] - X64[i]) ** 2).sum(1).astype(np.float32)
        assert np.array_equal(rec, d2[i])


def test_graph_init_rows_valid():
    X = datagen.mixture(300, 4, 5, seed=12)
    ids, d2 = knng.graph_init(X, 10, seed=2)
    _check_rows(X, ids, d2)
    ids2, _ = knng.graph_init(X[:11], 10, seed=2)  # kappa = n-1: everybody else
    for i in range(11):
        assert sorted(ids2[i].tolist()) == [j for j in range(11) if j != i]


def test_one_round_with_one_cluster_is_exact_knn():
    X = datagen.mixture(90, 6, 4, seed=13)  # n < 2*xi -> k0 = 1
    ids, d2 = knng.knn_build(X, 7, xi=50, tau=1, seed=4)
    _check_rows(X, ids, d2)
    tree = cKDTree(X.astype(np.float64))
    dd, ii = tree.query(X.astype(np.float64), k=8)
    assert np.array_equal(ids, ii[:, 1:].astype(np.int32))  # continuous data: no ties
    assert np.allclose(d2, (dd[:, 1:] ** 2), rtol=1e-6)
    e_ids, e_d2 = exact.brute_knn(X, 7)
    assert np.array_equal(ids, e_ids) and np.array_equal(d2, e_d2)


def test_build_rounds_monotone_and_tau0():
    X = datagen.mixture(1500, 8, 30, seed=14)
    G0 = knng.graph_init(X, 10, seed=6)
    ids0, d20 = knng.knn_build(X, 10, xi=50, tau=0, seed=6)
    assert np.array_equal(ids0, G0[0]) and np.array_equal(d20, G0[1])
    _, _, hist = knng.knn_build(X, 10, xi=50, tau=4, seed=6, history=True)
    for (a_i, a_d), (b_i, b_d) in zip(hist, hist[1:]):
        assert (b_d[:, -1] <= a_d[:, -1]).all()
        assert (b_d[:, 0] <= a_d[:, 0]).all()
    _check_rows(X, *hist[-1])
    e_ids, e_d2 = exact.brute_knn(X, 10)
    rec = metrics.recall_top1(hist[-1][1], e_d2[:, 0])
    assert rec > 0.6  # Sec. 4.3: recall rises above 0.6 within a few rounds
    assert metrics.recall_top1(hist[0][1], e_d2[:, 0]) < 0.05


def test_exact_refs_match_scipy():
    X = datagen.mixture(400, 5, 6, seed=15)
    ids, d2 = exact.brute_knn(X, 5)
    tree = cKDTree(X.astype(np.float64))
    dd, ii = tree.query(X.astype(np.float64), k=6)
    assert np.array_equal(ids, ii[:, 1:])
    C = X[:9] + 0.5
    assert (exact.lloyd_assign(X, C) == cdist(X.astype(np.float64), C.astype(np.float64), "sqeuclidean").argmin(1)).all()


def test_metrics_hand_worked():
    """recall@kappa, top-1 recall and label agreement on lists written out by
    hand."""
    G = np.array([[1, 2, 3], [0, 2, 4], [5, 6, 7]])
    exact_ids = np.array([[3, 1, 9], [4, 2, 0], [1, 2, 3]])
    # row 0 finds {1, 3} of {3, 1, 9}, row 1 all three, row 2 none: 5 of 9
    assert metrics.recall_at_kappa(G, exact_ids) == 5 / 9
    # first entries 1.0, 2.5, 0.5 against exact 1-NN distances 1.0, 2.0, 0.5:
    # rows 0 and 2 sit at the exact distance (a tie counts), row 1 does not
    G_d2 = np.array([[1.0, 2.0], [2.5, 3.0], [0.5, 0.5]], np.float32)
    assert metrics.recall_top1(G_d2, np.array([1.0, 2.0, 0.5], np.float32)) == 2 / 3
    assert metrics.agreement([1, 2, 3, 4], [1, 0, 3, 4]) == 0.75
    assert metrics.agreement([], []) == 1.0


def test_gap_mask_flags_near_ties():
    X = np.array([[0.0], [1.0]], np.float32)
    C = np.array([[-1.0], [1.0], [3.0]], np.float32)
    dec, best = metrics.assign_gap_mask(X, C, np.array([2, 2]), np.array([[1], [0]]))
    # Q = {2} only (both neighbours are in cluster 2): a single candidate is decided
    assert dec.tolist() == [True, True]
    dec, _ = metrics.assign_gap_mask(X, C, np.array([0, 1]), np.array([[1], [0]]))
    assert dec.tolist() == [False, True]  # x=0 is equidistant from -1 and 1


# ---------------------------------------------------------------- boost form --
from oracle import boost  # noqa: E402


def _objective_direct(X, labels, k):
    """I = sum_r ||sum of members||^2 / n_r computed from the partition alone."""
    X64 = np.asarray(X, np.float64)
    tot = 0.0
    for r in range(k):
        m = X64[np.asarray(labels) == r]
        if len(m):
            s = m.sum(0)
            tot += float(s @ s) / len(m)
    return tot


def test_boost_eqn3_equals_weighted_form_and_objective_change():
    rs = np.random.default_rng(5)
    X = datagen.mixture(300, 7, 6, seed=13)
    k = 9
    labels = rs.integers(0, k, 300)
    D, n_r = boost.composite(X, labels, k)
    I0 = boost.objective(D, n_r)
    assert abs(I0 - _objective_direct(X, labels, k)) <= 1e-10 * I0
    for _ in range(200):
        i = int(rs.integers(0, 300))
        u = int(labels[i])
        v = int(rs.integers(0, k))
        if v == u:
            continue
        x = X[i].astype(np.float64)
        lit = boost.delta_I(x, D[u], n_r[u], D[v], n_r[v])
        cu, cv = D[u] / n_r[u], (D[v] / n_r[v] if n_r[v] else np.zeros(7))
        wu = boost.weights(n_r[u], True) * float(((x - cu) ** 2).sum())
        wv = boost.weights(n_r[v], False) * float(((x - cv) ** 2).sum())
        assert abs(lit - (wu - wv)) <= 1e-9 * I0
        moved = labels.copy()
        moved[i] = v
        assert abs(lit - (_objective_direct(X, moved, k) - I0)) <= 1e-9 * I0


def test_boost_hand_worked_move_the_lloyd_rule_keeps():
    g = json.load(open(os.path.join(GOLD, "boost_1d.json")))
    X = np.array(g["X"], np.float32)[:, None]
    G = np.array(g["graph"])
    lab0 = np.array(g["labels0"])
    D, n_r = boost.composite(X, lab0, 2)
    assert boost.objective(D, n_r) == g["I0"]
    assert boost.delta_I(X[1].astype(np.float64), D[0], n_r[0], D[1], n_r[1]) == g["gain_sample1"]
    assert boost.best_move(X[1], 0, [1], D, n_r) == (1, g["gain_sample1"])
    # the Lloyd rule keeps sample 1 where it is
    lloyd, _, _ = gkmeans.gk_assign(X, (D / n_r[:, None]).astype(np.float32), lab0, G)
    assert lloyd[1] == 0
    lab1, applied, nprop = boost.boost_round(X, lab0, G, D, n_r, seed=1, rnd=1)
    assert list(lab1) == g["labels1"] and nprop == 1 and applied[0][:3] == (1, 0, 1)
    D1, n1 = boost.composite(X, lab1, 2)
    assert boost.objective(D1, n1) == g["I1"]


def test_boost_conflicting_proposals_apply_the_larger_key():
    # samples 1 and 2 both propose into cluster 1 (and leave cluster 0): one
    # move per cluster, the larger priority key wins
    X = np.array([[0.0], [2.0], [2.1], [0.1], [3.5]], np.float32)
    lab0 = np.array([0, 0, 0, 0, 1])
    G = np.array([[3], [4], [4], [0], [1]])
    D, n_r = boost.composite(X, lab0, 2)
    assert boost.best_move(X[1], 0, [1], D, n_r)[0] == 1
    assert boost.best_move(X[2], 0, [1], D, n_r)[0] == 1
    for rnd in range(1, 6):
        lab1, applied, nprop = boost.boost_round(X, lab0, G, D, n_r, seed=3, rnd=rnd)
        assert nprop == 2 and len(applied) == 1
        win = max((1, 2), key=lambda i: boost.priority(3, rnd, i))
        assert applied[0][0] == win and lab1[win] == 1 and lab1[3 - win] == 0


def test_boost_round_gain_is_the_sum_of_independent_moves():
    X = datagen.mixture(400, 5, 8, seed=21)
    k = 12
    G, _ = exact.brute_knn(X, 6)
    labels = np.random.default_rng(2).integers(0, k, 400)
    D, n_r = boost.composite(X, labels, k)
    I0 = boost.objective(D, n_r)
    lab1, applied, nprop = boost.boost_round(X, labels, G, D, n_r, seed=7, rnd=1)
    assert 1 <= len(applied) <= nprop
    used = [r for _, u, v, _ in applied for r in (u, v)]
    assert len(used) == len(set(used))  # no cluster in two applied moves
    D1, n1 = boost.composite(X, lab1, k)
    gain = sum(g for *_, g in applied)
    assert abs(boost.objective(D1, n1) - I0 - gain) <= 1e-9 * I0
    # the same moves one after the other (Eqn. 3 on the running state), in
    # reverse order: each gain is the one the round computed
    Dq, nq = D.copy(), n_r.copy()
    for i, u, v, g in reversed(applied):
        x = X[i].astype(np.float64)
        assert abs(boost.delta_I(x, Dq[u], nq[u], Dq[v], nq[v]) - g) <= 1e-9 * I0
        Dq[u] -= x
        Dq[v] += x
        nq[u] -= 1
        nq[v] += 1


def test_boost_rounds_monotone_and_stop_at_a_fixed_point():
    X = datagen.mixture(600, 4, 10, seed=22)
    k = 15
    G, _ = exact.brute_knn(X, 8)
    lab0 = gkmeans.init_labels(X, k, 9, gkmeans.INIT_TWOMEANS)[0]
    lab, C, cnt, tr, t, moves = boost.boost_rounds(X, k, G, lab0, 200, seed=9)
    assert (np.diff(tr) <= 1e-12 * tr[0]).all()
    assert moves[-1] == 0 and t < 200  # converged: the last round proposed nothing
    assert cnt.sum() == 600 and np.array_equal(cnt, np.bincount(lab, minlength=k))
    # no positive move is left for the printed sequential form either
    lab2, Is, mv = boost.boost_sequential(X, k, G, lab, 1)
    assert mv == [0] and np.array_equal(lab2, lab)


def test_boost_sequential_never_decreases_the_objective():
    X = datagen.mixture(500, 3, 7, seed=23)
    k = 10
    G, _ = exact.brute_knn(X, 5)
    lab0 = np.random.default_rng(4).integers(0, k, 500)
    D, n_r = boost.composite(X, lab0, k)
    lab, Is, mv = boost.boost_sequential(X, k, G, lab0, 6)
    assert Is[0] >= boost.objective(D, n_r) and all(b >= a - 1e-9 * a for a, b in zip(Is, Is[1:]))
    assert mv[0] > 0


# ----------------------------------------------------------- graph search --
from oracle import anns  # noqa: E402


def _connected_graph(X, kappa, seed):
    """Exact (kappa-1)-NN lists plus the next row id (a ring), checked connected."""
    G, _ = exact.brute_knn(X, kappa - 1)
    r = ((np.arange(X.shape[0]) + 1) % X.shape[0])[:, None]
    G = np.concatenate([G, r], 1)
    seen, stack = {0}, [0]
    while stack:
        for b in G[stack.pop()]:
            if int(b) not in seen:
                seen.add(int(b))
                stack.append(int(b))
    assert len(seen) == X.shape[0]
    return G


def test_search_with_full_budget_is_exact():
    A = datagen.mixture(640, 6, 12, seed=31)
    X, Q = A[:600], A[600:]
    G = _connected_graph(X, 8, 1)
    ids, d2 = anns.search_all(X, G, Q, ef=600, top_k=10, max_visits=10**6, n_entry=1, seed=3, form="classic")
    for i in range(Q.shape[0]):
        dd = ((X.astype(np.float64) - Q[i].astype(np.float64)) ** 2).sum(1)
        order = np.lexsort((np.arange(600), dd.astype(np.float32)))
        assert list(ids[i]) == list(order[:10])
        np.testing.assert_array_equal(d2[i], dd.astype(np.float32)[order[:10]].astype(np.float64))


def test_search_list_form_equals_classic_form():
    rs = np.random.default_rng(9)
    A = datagen.mixture(1560, 5, 30, seed=33)
    X, Q = A[:1500], A[1500:]
    for kappa, ef, visits, n_entry in [(6, 8, 10**6, 1), (10, 32, 10**6, 3), (10, 64, 60, 1), (4, 16, 200, 2)]:
        G = rs.integers(0, 1500, (1500, kappa)) if kappa == 4 else exact.brute_knn(X, kappa)[0]
        a = anns.search_all(X, G, Q, ef, 5, visits, n_entry, seed=kappa, form="list")
        b = anns.search_all(X, G, Q, ef, 5, visits, n_entry, seed=kappa, form="classic")
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), (kappa, ef, visits)


def test_search_keys_and_recall_trend():
    A = datagen.mixture(3080, 8, 40, seed=35)
    X, Q = A[:3000], A[3000:]
    G = _connected_graph(X, 10, 2)
    # the keys are the float32 of the float64 squared distance
    k = anns.sq_keys(Q[0], X[:50])
    np.testing.assert_array_equal(k, np.array([anns.sq_key(Q[0], x) for x in X[:50]]))
    assert np.abs(k - ((X[:50].astype(np.float64) - Q[0]) ** 2).sum(1)).max() <= 1e-6 * k.max()
    truth = np.array([np.argsort(((X.astype(np.float64) - q) ** 2).sum(1), kind="stable")[:10] for q in Q])
    rec = []
    for ef in (10, 20, 40, 80):
        ids, _ = anns.search_all(X, G, Q, ef, 10, 10**6, 1, seed=5)
        rec.append(np.mean([len(set(a) & set(b)) / 10.0 for a, b in zip(ids, truth)]))
    assert all(b >= a - 0.02 for a, b in zip(rec, rec[1:])) and rec[-1] > rec[0] + 0.4 and rec[-1] > 0.8
