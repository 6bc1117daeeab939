"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Every case is seeded and synthetic (mixtures shaped like the paper's
workloads).  Integer outputs are compared exactly: the library decides every
comparison on float64 values (float32 screens with rigorous margins, float64
re-evaluation inside them), like the oracle, so labels, graph ids and sizes
must agree bit for bit.  Float outputs: centroids within one float32 ulp
(bit-exact on integer data), sums to 1e-12 relative, distortion to 1e-12
relative, graph distances bit-exact (both sides round the float64 squared
distance to float32)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import anns, boost, exact, gkmeans, knng, rng, twomeans  # noqa: E402
from paper_1705_01813_amd import datagen, knnkm  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = knnkm.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rand_graph(n, kappa, seed):
    rs = np.random.default_rng(seed)
    G = np.empty((n, kappa), np.int32)
    for i in range(n):
        c = rs.choice(n - 1, kappa, replace=False)
        G[i] = c + (c >= i)
    return G


# --------------------------------------------------------------------- RNG --
def test_rng_matches_oracle(ctx):
    say("rng")
    for seed, stream, ctr0 in [(0, 0, 0), (123, rng.stream_id(2, 7, 99), 5), (2**63 + 11, 2**60, 1000)]:
        out = torch.zeros(64, dtype=torch.uint64, device=DEV)
        knnkm.knnkm_rng_draw(ctx, seed, stream, ctr0, out)
        got = [int(v) & (2**64 - 1) for v in host(out.view(torch.int64)).tolist()]
        key = rng.stream_key(seed, stream)
        want = [rng.draw(key, ctr0 + c) for c in range(64)]
        assert got == want


# -------------------------------------------------------------- assignment --
ASSIGN_CASES = [
    # n, d, k, kappa
    (1000, 1, 20, 5),
    (2048, 7, 40, 10),
    (5003, 32, 100, 10),
    (3001, 64, 300, 20),
    (4097, 100, 50, 1),
    (3000, 128, 200, 20),
    (2000, 200, 100, 50),
    (1500, 512, 120, 50),
    (1200, 33, 600, 128),
]


@pytest.mark.parametrize("n,d,k,kappa", ASSIGN_CASES)
def test_assign_parity(ctx, n, d, k, kappa):
    say("assign", n, d, k, kappa)
    X = datagen.mixture(n, d, max(2, k // 2), seed=n + d)
    rs = np.random.default_rng(k + kappa)
    C = (X[rs.choice(n, k, replace=False)] + rs.normal(0, 0.3, size=(k, d))).astype(np.float32)
    lab_in = rs.integers(0, k, n).astype(np.int32)
    G = rand_graph(n, kappa, seed=d)
    want, best, moved = gkmeans.gk_assign(X, C, lab_in, G)
    out = torch.empty(n, dtype=torch.int32, device=DEV)
    bd = torch.empty(n, dtype=torch.float32, device=DEV)
    mv = torch.zeros(1, dtype=torch.int64, device=DEV)
    knnkm.knn_assign(ctx, dev(X), dev(C), dev(G), dev(lab_in), out, bd, mv)
    got = host(out)
    assert np.array_equal(got, want)
    assert int(host(mv)[0]) == moved
    np.testing.assert_allclose(host(bd), best, rtol=2e-6, atol=1e-6)


def test_assign_ties_and_duplicates(ctx):
    say("assign ties")
    rs = np.random.default_rng(5)
    n, d, k, kappa = 700, 16, 30, 8
    X = rs.integers(0, 4, size=(n, d)).astype(np.float32)  # many exact ties
    C = rs.integers(0, 4, size=(k, d)).astype(np.float32)
    C[10] = C[3]  # identical centroids: smallest id must win
    C[20] = C[3]
    lab_in = rs.integers(0, k, n).astype(np.int32)
    G = rand_graph(n, kappa, seed=1)
    want, _, moved = gkmeans.gk_assign(X, C, lab_in, G)
    out = torch.empty(n, dtype=torch.int32, device=DEV)
    mv = torch.zeros(1, dtype=torch.int64, device=DEV)
    knnkm.knn_assign(ctx, dev(X), dev(C), dev(G), dev(lab_in), out, None, mv)
    assert np.array_equal(host(out), want)
    assert int(host(mv)[0]) == moved


def test_assign_full_size_sampled(ctx):
    """knn_assign at the full 1M x 128 workload size (the integer mixture,
    k = 10,000, kappa = 20; random input labels, so rows have many
    candidates): 4,000 sampled rows plus the first and the last against the
    oracle row by row, and the moved count against the whole output."""
    n, d, k, kappa = 1_000_000, 128, 10_000, 20
    say("assign full size", n, d, k, kappa)
    X = datagen.config_data("c2", seed=77)
    rs = np.random.default_rng(5)
    C = (X[rs.choice(n, k, replace=False)] + rs.normal(0, 4.0, size=(k, d))).astype(np.float32)
    lab_in = rs.integers(0, k, n).astype(np.int32)
    c = rs.integers(0, n - 1, size=(n, kappa))
    G = (c + (c >= np.arange(n)[:, None])).astype(np.int32)
    out = torch.empty(n, dtype=torch.int32, device=DEV)
    bd = torch.empty(n, dtype=torch.float32, device=DEV)
    mv = torch.zeros(1, dtype=torch.int64, device=DEV)
    knnkm.knn_assign(ctx, dev(X), dev(C), dev(G), dev(lab_in), out, bd, mv)
    got, got_bd = host(out), host(bd)
    assert int(host(mv)[0]) == int((got != lab_in).sum())
    rows = np.concatenate([rs.choice(n, 4000, replace=False), [0, n - 1]])
    want, want_bd = gkmeans.gk_assign_rows(X, C, lab_in, G, rows)
    assert np.array_equal(got[rows], want)
    np.testing.assert_allclose(got_bd[rows], want_bd, rtol=2e-6, atol=1e-6)


class _HostRows:
    """The rows of a device matrix at the given ids, copied to the host and
    indexable by those ids (the oracle's row-restricted sweep reads no other)."""

    def __init__(self, mat, ids):
        ids = np.asarray(ids, np.int64)
        self.shape = tuple(int(v) for v in mat.shape)
        self.data = mat[torch.from_numpy(ids).to(mat.device)].cpu().numpy()
        self.pos = {int(v): t for t, v in enumerate(ids)}

    def __getitem__(self, r):
        return self.data[[self.pos[int(v)] for v in np.atleast_1d(r)]]


def test_assign_full_size_c3_sampled(ctx):
    """knn_assign at the full 10M x 512 size of the precision-form workload
    (its mixture recipe, k = 1,000,000, kappa = 50; row offsets beyond 2^31
    elements): 2,000 sampled rows plus the first and the last against the
    oracle, and the moved count against the whole output."""
    c = datagen.CONFIGS["c3"]
    n, d, k, kappa = 10_000_000, 512, 1_000_000, 50
    say("assign full size c3", n, d, k, kappa)
    Xd = datagen.mixture_device(n, d, c["comps"], 31, c["centre"], c["lo"], c["hi"], c["sigma"], c["clip"],
                                c["integer"], device=DEV)
    g = torch.Generator(device=DEV)
    g.manual_seed(3)
    Cd = (Xd[torch.randint(0, n, (k,), generator=g, device=DEV)]
          + 0.1 * torch.randn((k, d), generator=g, device=DEV)).contiguous()
    labd = torch.randint(0, k, (n,), generator=g, device=DEV).to(torch.int32)
    nb = torch.randint(0, n - 1, (n, kappa), generator=g, device=DEV)
    Gd = (nb + (nb >= torch.arange(n, device=DEV)[:, None])).to(torch.int32)
    del nb
    out = torch.empty(n, dtype=torch.int32, device=DEV)
    bd = torch.empty(n, dtype=torch.float32, device=DEV)
    mv = torch.zeros(1, dtype=torch.int64, device=DEV)
    knnkm.knn_assign(ctx, Xd, Cd, Gd, labd, out, bd, mv)
    got, got_bd, lab = host(out), host(bd), host(labd)
    assert int(host(mv)[0]) == int((got != lab).sum())
    rs = np.random.default_rng(6)
    rows = np.concatenate([rs.choice(n, 2000, replace=False), [0, n - 1]])
    want, want_bd = gkmeans.gk_assign_rows(_HostRows(Xd, rows), host(Cd), lab, _HostRows(Gd, rows), rows)
    assert np.array_equal(got[rows], want)
    np.testing.assert_allclose(got_bd[rows], want_bd, rtol=2e-6, atol=1e-6)


def test_assign_kappa_ge_k_is_exact_lloyd(ctx):
    say("assign dense")
    from scipy.spatial.distance import cdist

    X = datagen.mixture(3000, 24, 15, seed=4)
    rs = np.random.default_rng(9)
    C = X[rs.choice(3000, 12, replace=False)] + 0.25
    lab_in = rs.integers(0, 12, 3000).astype(np.int32)
    G = rand_graph(3000, 12, seed=2)
    out = torch.empty(3000, dtype=torch.int32, device=DEV)
    knnkm.knn_assign(ctx, dev(X), dev(C.astype(np.float32)), dev(G), dev(lab_in), out)
    ref = cdist(X.astype(np.float64), C.astype(np.float32).astype(np.float64), "sqeuclidean").argmin(1)
    assert np.array_equal(host(out), ref)


# ------------------------------------------------------- update, distortion --
@pytest.mark.parametrize("n,d,k", [(1000, 3, 17), (10000, 32, 100), (20011, 128, 700), (3000, 512, 40),
                                   (5000, 64, 1), (700, 9, 650)])
def test_update_parity(ctx, n, d, k):
    say("update", n, d, k)
    X = datagen.mixture(n, d, 20, seed=n)
    rs = np.random.default_rng(d)
    lab = rs.integers(0, k, n).astype(np.int32)
    if k > 5:
        lab[lab == 4] = 5  # an empty cluster keeps its previous centroid
    Cprev = rs.normal(size=(k, d)).astype(np.float32)
    C_want, cnt_want, sums_want = gkmeans.centroid_update(X, lab, k, Cprev)
    C = dev(Cprev)
    cnt = torch.empty(k, dtype=torch.int32, device=DEV)
    sums = torch.empty((k, d), dtype=torch.float64, device=DEV)
    knnkm.centroid_update(ctx, dev(X), dev(lab), C, cnt, sums)
    assert np.array_equal(host(cnt), cnt_want)
    np.testing.assert_allclose(host(sums), sums_want, rtol=1e-12, atol=1e-9)
    Cg = host(C)
    ulps = np.abs(Cg.view(np.int32).astype(np.int64) - C_want.view(np.int32).astype(np.int64))
    assert ulps.max() <= 1
    E = torch.zeros(1, dtype=torch.float64, device=DEV)
    knnkm.distortion(ctx, dev(X), C, dev(lab), E)
    e_want = gkmeans.distortion(X, Cg, lab)
    assert abs(float(host(E)[0]) - e_want) <= 1e-12 * e_want


def test_update_and_distortion_full_size(ctx):
    """centroid_update and distortion at the full 1M x 128 size (the integer
    mixture, k = 10,000, random labels with one empty cluster): counts,
    float64 sums and float32 centroids bit for bit against the oracle on every
    cluster (integer data: exact sums), the distortion within 1e-12."""
    n, d, k = 1_000_000, 128, 10_000
    say("update full size", n, d, k)
    X = datagen.config_data("c2", seed=55)
    rs = np.random.default_rng(55)
    lab = rs.integers(0, k, n).astype(np.int32)
    lab[lab == 7] = 8  # cluster 7 is empty: keeps its previous centroid
    Cprev = rs.normal(size=(k, d)).astype(np.float32)
    C_want, cnt_want, sums_want = gkmeans.centroid_update(X, lab, k, Cprev)
    Xd, labd = dev(X), dev(lab)
    C = dev(Cprev)
    cnt = torch.empty(k, dtype=torch.int32, device=DEV)
    sums = torch.empty((k, d), dtype=torch.float64, device=DEV)
    knnkm.centroid_update(ctx, Xd, labd, C, cnt, sums)
    assert np.array_equal(host(cnt), cnt_want)
    assert np.array_equal(host(sums), sums_want)
    assert np.array_equal(host(C), C_want)
    E = torch.zeros(1, dtype=torch.float64, device=DEV)
    knnkm.distortion(ctx, Xd, C, labd, E)
    e_want = 0.0
    for s0 in range(0, n, 100_000):
        diff = X[s0:s0 + 100_000].astype(np.float64) - C_want[lab[s0:s0 + 100_000]].astype(np.float64)
        e_want += float(np.einsum("ij,ij->", diff, diff))
    e_want /= n
    assert abs(float(host(E)[0]) - e_want) <= 1e-12 * e_want


def test_update_integer_data_bit_exact(ctx):
    say("update integer")
    X = datagen.integer_grid(30000, 128, seed=3)
    lab = np.random.default_rng(1).integers(0, 300, 30000).astype(np.int32)
    C_want, cnt_want, sums_want = gkmeans.centroid_update(X, lab, 300, np.zeros((300, 128), np.float32))
    C = torch.zeros((300, 128), dtype=torch.float32, device=DEV)
    cnt = torch.empty(300, dtype=torch.int32, device=DEV)
    sums = torch.empty((300, 128), dtype=torch.float64, device=DEV)
    knnkm.centroid_update(ctx, dev(X), dev(lab), C, cnt, sums)
    assert np.array_equal(host(sums), sums_want)
    assert np.array_equal(host(C), C_want)


# --------------------------------------------------------------- TwoMeans --
@pytest.mark.parametrize("n,d,k", [(1000, 1, 8), (1000, 5, 7), (5000, 32, 200), (9000, 128, 100),
                                   (20000, 16, 3), (3000, 64, 3000), (4500, 8, 1), (2100, 300, 33)])
def test_twomeans_parity(ctx, n, d, k):
    say("twomeans", n, d, k)
    X = datagen.mixture(n, d, 30, seed=n + k)
    want = twomeans.twomeans(X, k, seed=7, rnd=3)
    lab = torch.empty(n, dtype=torch.int32, device=DEV)
    knnkm.knnkm_twomeans(ctx, dev(X), k, 7, 3, 2, lab)
    got = host(lab)
    assert np.array_equal(got, want), f"agreement {np.mean(got == want):.6f}"


@pytest.mark.parametrize("n,d,k,distinct", [(12000, 8, 37, 40), (9000, 16, 100, 3), (30000, 4, 9, 7)])
def test_twomeans_parity_duplicate_rows(ctx, n, d, k, distinct):
    """Rows drawn from a few distinct rows: many members share a delta (and
    both seeds can be the same row, making every delta zero), so inside nodes
    larger than one tile the ids decide which members go left."""
    say("twomeans duplicate rows", n, d, k, distinct)
    base = datagen.mixture(distinct, d, 3, seed=n + distinct)
    X = np.ascontiguousarray(base[np.random.default_rng(n).integers(0, distinct, n)])
    want = twomeans.twomeans(X, k, seed=7, rnd=3)
    lab = torch.empty(n, dtype=torch.int32, device=DEV)
    knnkm.knnkm_twomeans(ctx, dev(X), k, 7, 3, 2, lab)
    got = host(lab)
    assert np.array_equal(got, want), f"agreement {np.mean(got == want):.6f}"


@pytest.mark.parametrize("n,d,k,iters", [(200_003, 128, 2000, 2), (50_000, 3, 20_000, 2), (30_000, 512, 300, 1),
                                         (4097, 64, 4097, 2), (100_000, 24, 97, 3), (1024, 7, 1000, 0)])
def test_twomeans_subtree_finish_same_bits(ctx, n, d, k, iters):
    """Subtrees of at most 1,024 (or 300) members finished by one block each
    give the labels of the per-depth kernels, bit for bit (leaves of one
    member, a partial last depth, no Lloyd step, d = 512)."""
    say("twomeans subtree finish", n, d, k, iters)
    X = dev(datagen.mixture(n, d, 50, seed=n + 5))

    def run(on):
        knnkm.knnkm_enable_subtree_finish(ctx, on)
        lab = torch.empty(n, dtype=torch.int32, device=DEV)
        knnkm.knnkm_twomeans(ctx, X, k, 7, 3, iters, lab)
        return host(lab)

    try:
        ref = run(0)
        for lim in (1, 300):  # roots up to 1,024 members, up to 300
            got = run(lim)
            assert np.array_equal(ref, got), (lim, f"agreement {np.mean(ref == got):.6f}")
    finally:
        knnkm.knnkm_enable_subtree_finish(ctx, True)


def _leaf_sizes(n, k):
    """Leaf sizes, left to right, of the oracle's tree shape."""
    shape = twomeans.tree_shape(n, k)
    if not shape:
        return [n]
    sizes, flags = shape[-1]
    out = []
    for sz, f in zip(sizes, flags):
        out += [(sz + 1) // 2, sz // 2] if f else [sz]
    return out


def test_twomeans_full_size_shape(ctx):
    """TwoMeans at the full sizes of the fits it initialises: the 1M x 128
    workload (k = 10,000), whose leaves hold exactly the oracle's tree-shape
    sizes in leaf order and equal the per-depth kernels' leaves bit for bit,
    and the 10M x 512 workload (k = 1,000,000), whose leaves hold the tree-shape
    sizes."""
    say("twomeans full size")
    n, k = 1_000_000, 10_000
    X = dev(datagen.config_data("c2", seed=1234))
    labs = []
    try:
        for on in (True, False):
            knnkm.knnkm_enable_subtree_finish(ctx, on)
            lab = torch.empty(n, dtype=torch.int32, device=DEV)
            knnkm.knnkm_twomeans(ctx, X, k, 1234, knnkm.ROUND_FIT, 2, lab)
            labs.append(host(lab))
    finally:
        knnkm.knnkm_enable_subtree_finish(ctx, True)
    assert np.array_equal(labs[0], labs[1])
    assert np.array_equal(np.bincount(labs[0], minlength=k), _leaf_sizes(n, k))
    del X
    c = datagen.CONFIGS["c3"]
    n, k = 10_000_000, 1_000_000
    X = datagen.mixture_device(n, 512, c["comps"], 31, c["centre"], c["lo"], c["hi"], c["sigma"], c["clip"],
                               c["integer"], device=DEV)
    lab = torch.empty(n, dtype=torch.int32, device=DEV)
    knnkm.knnkm_twomeans(ctx, X, k, 5, knnkm.ROUND_FIT, 2, lab)
    assert np.array_equal(np.bincount(host(lab), minlength=k), _leaf_sizes(n, k))


def test_batch_subtree_finish_same_bits(ctx):
    """Many jobs in one tree launch (graph rounds and the fit's initial
    clusters): jobs whose nodes reach 1,024 members at different depths, one
    job small enough to be finished from the root."""
    sizes = [3000, 701, 1500, 64, 9000, 2201]
    Xs, n_off, ks, seeds = _batch(sizes, 40, seed=77)
    X = dev(np.concatenate(Xs))
    n, kappa, K = int(n_off[-1]), 8, sum(ks)
    p = knnkm.default_params(kappa=kappa, max_iters=6, seed=5)
    say("batch subtree finish", sizes, ks)

    def run(on):
        knnkm.knnkm_enable_subtree_finish(ctx, on)
        gi = torch.empty((n, kappa), dtype=torch.int32, device=DEV)
        gd = torch.empty((n, kappa), dtype=torch.float32, device=DEV)
        lab = torch.empty(n, dtype=torch.int32, device=DEV)
        C = torch.empty((K, 40), dtype=torch.float32, device=DEV)
        cnt = torch.empty(K, dtype=torch.int32, device=DEV)
        tr = knnkm.knnkm_fit_batched(ctx, X, n_off, ks, seeds, p, gi, gd, lab, C, cnt)
        return host(gi), host(gd), host(lab), host(C), host(cnt), np.asarray(tr)

    try:
        ref = run(False)
        got = run(True)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b)
    finally:
        knnkm.knnkm_enable_subtree_finish(ctx, True)


# ------------------------------------------------------------------- graph --
@pytest.mark.parametrize("n,d,kappa", [(50, 4, 49), (1000, 32, 10), (3001, 128, 50), (500, 512, 20),
                                       (300, 16, 128)])
def test_graph_init_parity(ctx, n, d, kappa):
    say("graph_init", n, d, kappa)
    X = datagen.mixture(n, d, 10, seed=n)
    want_i, want_d = knng.graph_init(X, kappa, seed=11)
    gi = torch.empty((n, kappa), dtype=torch.int32, device=DEV)
    gd = torch.empty((n, kappa), dtype=torch.float32, device=DEV)
    knnkm.knnkm_graph_init(ctx, dev(X), kappa, 11, gi, gd)
    assert np.array_equal(host(gi), want_i)
    assert np.array_equal(host(gd), want_d)


def _graph_diff(got_i, got_d, want_i, want_d, lab=None):
    bad = np.flatnonzero((got_i != want_i).any(1) | (got_d != want_d).any(1))
    if len(bad) == 0:
        return ""
    r = bad[0]
    msg = f"{len(bad)} rows differ; first row {r}"
    if lab is not None:
        msg += f" (cluster {lab[r]} of size {(lab == lab[r]).sum()})"
    return msg + f"\n got ids {got_i[r].tolist()}\n want    {want_i[r].tolist()}\n got d2 {got_d[r].tolist()}\n want   {want_d[r].tolist()}"


@pytest.mark.parametrize("precision", [knnkm.FP32, knnkm.BF16_RERANK])
@pytest.mark.parametrize("n,d,kappa,k", [(2000, 32, 10, 40), (3000, 128, 20, 60), (600, 512, 20, 10),
                                         (600, 512, 50, 10), (1000, 256, 50, 12), (1500, 20, 8, 3),
                                         (400, 64, 30, 1), (3000, 512, 50, 10), (2500, 16, 10, 2),
                                         (1200, 32, 10, 100), (1000, 512, 20, 80)])
def test_refine_parity(ctx, precision, n, d, kappa, k):
    say("refine", precision, n, d, kappa, k)
    X = datagen.mixture(n, d, 12, seed=d + k)
    gi0, gd0 = knng.graph_init(X, kappa, seed=5)
    lab = np.random.default_rng(3).integers(0, k, n).astype(np.int32)
    want_i, want_d = knng.refine(X, gi0, gd0, lab)
    gi, gd = dev(gi0), dev(gd0)
    knnkm.knnkm_graph_refine(ctx, dev(X), dev(lab), k, precision, gi, gd)
    got_i, got_d = host(gi), host(gd)
    msg = _graph_diff(got_i, got_d, want_i, want_d, lab)
    assert not msg, msg
    # the same clusters once more: every pair is now visited or too far, so
    # no row changes (the visited test of the list update, Alg. 3)
    knnkm.knnkm_graph_refine(ctx, dev(X), dev(lab), k, precision, gi, gd)
    msg = _graph_diff(host(gi), host(gd), want_i, want_d, lab)
    assert not msg, "second pass changed rows: " + msg


@pytest.mark.parametrize("n,k", [(1000, 80), (1500, 30), (1200, 12), (1500, 5)])
def test_refine_parity_odd_d(ctx, n, k):
    """d = 13 (rows read element by element, not in 16-byte pieces) for
    clusters of about 12, 50, 100 and 300 members: every refinement path."""
    d, kappa = 13, 10
    say("refine odd d", n, d, kappa, k)
    X = datagen.mixture(n, d, 7, seed=k + 1)
    gi0, gd0 = knng.graph_init(X, kappa, seed=13)
    lab = np.random.default_rng(k + 1).integers(0, k, n).astype(np.int32)
    want_i, want_d = knng.refine(X, gi0, gd0, lab)
    for precision in (knnkm.FP32, knnkm.BF16_RERANK):
        gi, gd = dev(gi0), dev(gd0)
        knnkm.knnkm_graph_refine(ctx, dev(X), dev(lab), k, precision, gi, gd)
        msg = _graph_diff(host(gi), host(gd), want_i, want_d, lab)
        assert not msg, msg


@pytest.mark.parametrize("n,k", [(1500, 100), (2000, 40), (4000, 50), (3000, 6)])
def test_refine_parity_long_lists(ctx, n, k):
    """kappa = 100 (every lane of a merging wavefront holds two list entries)
    for clusters of about 15, 50, 80 and 500 members: the one-tile kernel
    (at most 16 members) and the 17-64-member one, the 65-128-member kernels
    and the tiled one."""
    d, kappa = 24, 100
    say("refine long lists", n, d, kappa, k)
    X = datagen.mixture(n, d, 9, seed=k)
    gi0, gd0 = knng.graph_init(X, kappa, seed=11)
    lab = np.random.default_rng(k).integers(0, k, n).astype(np.int32)
    want_i, want_d = knng.refine(X, gi0, gd0, lab)
    for precision in (knnkm.FP32, knnkm.BF16_RERANK):
        gi, gd = dev(gi0), dev(gd0)
        knnkm.knnkm_graph_refine(ctx, dev(X), dev(lab), k, precision, gi, gd)
        msg = _graph_diff(host(gi), host(gd), want_i, want_d, lab)
        assert not msg, msg


@pytest.mark.parametrize("n,d,k", [(1000, 64, 10), (1200, 128, 12), (1500, 512, 30), (900, 512, 30),
                                   (1200, 64, 4)])
def test_refine_duplicate_rows(ctx, n, d, k):
    """Clusters full of exact and near duplicates (integer rows, a few
    coordinates moved by one): zero and tiny distances against large norms,
    whose Gram keys cannot be certified, so the exact kernels recompute them
    from the rows: clusters of about 100 (the 65-128-member kernels) hold more
    such pairs than the list takes and recompute every pair, clusters of
    about 50 and 30 at d = 512 (the 17-64-member kernel) fewer; clusters of
    about 300 take the tiled kernels for 129-1024 members."""
    say("refine duplicate rows", n, d, k)
    rng = np.random.default_rng(d + k)
    base = rng.integers(100, 256, size=(6, d)).astype(np.float32)
    X = base[rng.integers(0, 6, n)]
    bump = (rng.random((n, d)) < 2.0 / d).astype(np.float32)
    X = np.ascontiguousarray(X + bump * (rng.random(n) < 0.5)[:, None])
    kappa = 20
    gi0, gd0 = knng.graph_init(X, kappa, seed=7)
    lab = rng.integers(0, k, n).astype(np.int32)
    want_i, want_d = knng.refine(X, gi0, gd0, lab)
    for precision in (knnkm.FP32, knnkm.BF16_RERANK):
        gi, gd = dev(gi0), dev(gd0)
        knnkm.knnkm_graph_refine(ctx, dev(X), dev(lab), k, precision, gi, gd)
        msg = _graph_diff(host(gi), host(gd), want_i, want_d, lab)
        assert not msg, msg


@pytest.mark.parametrize("precision", [knnkm.FP32, knnkm.BF16_RERANK])
def test_knn_build_parity(ctx, precision):
    n, d, kappa = 3000, 32, 10
    say("knn_build", precision, n, d, kappa)
    X = datagen.mixture(n, d, 30, seed=21)
    want_i, want_d = knng.knn_build(X, kappa, xi=50, tau=3, seed=8)
    p = knnkm.default_params(kappa=kappa, xi=50, tau=3, seed=8, precision=precision)
    gi = torch.empty((n, kappa), dtype=torch.int32, device=DEV)
    gd = torch.empty((n, kappa), dtype=torch.float32, device=DEV)
    knnkm.knn_build(ctx, dev(X), p, gi, gd)
    assert np.array_equal(host(gi), want_i)
    assert np.array_equal(host(gd), want_d)


def test_knn_build_one_cluster_is_exact(ctx):
    say("knn_build k0=1")
    X = datagen.mixture(90, 12, 5, seed=2)
    p = knnkm.default_params(kappa=9, xi=50, tau=1, seed=3)
    gi = torch.empty((90, 9), dtype=torch.int32, device=DEV)
    gd = torch.empty((90, 9), dtype=torch.float32, device=DEV)
    knnkm.knn_build(ctx, dev(X), p, gi, gd)
    e_i, e_d = exact.brute_knn(X, 9)
    assert np.array_equal(host(gi), e_i)
    assert np.array_equal(host(gd), e_d)


# --------------------------------------------------------------------- fit --
@pytest.mark.parametrize("init", [knnkm.INIT_RANDOM, knnkm.INIT_TWOMEANS])
def test_fit_parity(ctx, init):
    n, d, k, kappa, T = 6000, 32, 60, 10, 8
    say("fit", init, n, d, k, kappa, T)
    X = datagen.mixture(n, d, 60, seed=31)
    G, _ = knng.knn_build(X, kappa, xi=50, tau=2, seed=4)
    lab_w, C_w, cnt_w, tr_w, it_w, _ = gkmeans.fit(X, k, G, T, seed=6, init=init)
    p = knnkm.default_params(kappa=kappa, max_iters=T, seed=6, init=init)
    lab = torch.empty(n, dtype=torch.int32, device=DEV)
    C = torch.empty((k, d), dtype=torch.float32, device=DEV)
    cnt = torch.empty(k, dtype=torch.int32, device=DEV)
    tr, it = knnkm.knn_kmeans_fit(ctx, dev(X), k, dev(G), p, lab, C, cnt)
    assert it == it_w
    assert np.array_equal(host(lab), lab_w)
    assert np.array_equal(host(cnt), cnt_w)
    np.testing.assert_allclose(tr, tr_w, rtol=1e-9)
    assert (np.diff(tr) <= 1e-12 * tr[0]).all()


def test_fit_resume_continues_the_fit(ctx):
    """Resume (init from labels): T1 sweeps, then T2 sweeps from the labels
    and centroids they end with, equal one fit of T1 + T2 sweeps (integer
    data: every sum is exact, so the rebuilt float64 sums equal the
    fixed-point ones) and the oracle's fit resumed the same way; labels
    outside [0, k) are rejected."""
    n, d, k, kappa, T1, T2 = 6000, 32, 80, 10, 4, 5
    say("fit resume", n, d, k, kappa, T1, T2)
    X = datagen.mixture(n, d, 60, seed=41, lo=0.0, hi=255.0, sigma=20.0, clip=(0.0, 255.0), integer=True)
    G, _ = knng.knn_build(X, kappa, xi=50, tau=2, seed=4)
    Xd, Gd = dev(X), dev(G)

    def run(T, init, lab=None, C=None):
        p = knnkm.default_params(kappa=kappa, max_iters=T, seed=6, init=init)
        lab = torch.empty(n, dtype=torch.int32, device=DEV) if lab is None else lab
        C = torch.empty((k, d), dtype=torch.float32, device=DEV) if C is None else C
        cnt = torch.empty(k, dtype=torch.int32, device=DEV)
        tr, it = knnkm.knn_kmeans_fit(ctx, Xd, k, Gd, p, lab, C, cnt)
        return lab, C, cnt, tr

    lab, C, cnt, tr = run(T1 + T2, knnkm.INIT_TWOMEANS)
    l1, C1, _, t1 = run(T1, knnkm.INIT_TWOMEANS)
    l1h, C1h = host(l1), host(C1)
    l2, C2, c2, t2 = run(T2, knnkm.INIT_LABELS, l1, C1)
    assert np.array_equal(host(l2), host(lab))
    assert np.array_equal(host(C2), host(C))
    assert np.array_equal(host(c2), host(cnt))
    np.testing.assert_allclose(t2[0], t1[-1], rtol=1e-12)
    np.testing.assert_allclose(t2[1:], tr[T1 + 1:], rtol=1e-12)
    w_lab, w_C, w_cnt, w_tr, _, _ = gkmeans.fit(X, k, G, T2, seed=0, labels0=l1h, C0=C1h)
    assert np.array_equal(host(l2), w_lab)
    assert np.array_equal(host(c2), w_cnt)
    assert np.array_equal(host(C2), w_C)
    np.testing.assert_allclose(t2, w_tr, rtol=1e-9)
    bad = torch.from_numpy(l1h.copy()).to(DEV)
    bad[17] = k
    with pytest.raises(knnkm.KnnkmError) as e:
        run(2, knnkm.INIT_LABELS, bad, C1)
    assert e.value.status == knnkm.EINVAL and "outside" in str(e.value)


@pytest.mark.parametrize("n,d,k,kappa", [(6000, 32, 60, 10), (3000, 512, 100, 50), (2500, 300, 40, 20)])
def test_workspace_estimate_bounds_a_build_and_fit(n, d, k, kappa):
    """The planning estimate bounds the workspace a fresh context grows to in
    knn_build + knn_kmeans_fit (narrow and wide rows)."""
    say("workspace estimate", n, d, k, kappa)
    X = dev(datagen.mixture(n, d, 40, seed=n + d, sigma=0.5, centre="normal"))
    p = knnkm.default_params(kappa=kappa, xi=50, tau=2, max_iters=5, seed=3)
    c = knnkm.Context(0)
    try:
        gi = torch.empty((n, kappa), dtype=torch.int32, device=DEV)
        gd = torch.empty((n, kappa), dtype=torch.float32, device=DEV)
        knnkm.knn_build(c, X, p, gi, gd)
        lab = torch.empty(n, dtype=torch.int32, device=DEV)
        C = torch.empty((k, d), dtype=torch.float32, device=DEV)
        cnt = torch.empty(k, dtype=torch.int32, device=DEV)
        knnkm.knn_kmeans_fit(c, X, k, gi, p, lab, C, cnt)
        held = c.workspace_bytes()
    finally:
        c.close()
    est = knnkm.knnkm_workspace_estimate(n, d, k, p)
    say("held", held, "estimate", est)
    assert 0 < held <= est


@pytest.mark.parametrize("init,n,d,k,kappa,T", [(knnkm.INIT_TWOMEANS, 1500, 8, 30, 8, 40),
                                                 (knnkm.INIT_RANDOM, 1200, 5, 20, 10, 60),
                                                 (knnkm.INIT_TWOMEANS, 700, 33, 12, 70, 30)])
def test_boost_fit_parity(ctx, init, n, d, k, kappa, T):
    """The boost form (Alg. 2 as printed, Eqn. 3) in data-parallel rounds:
    labels, counts, centroids and the rounds run equal the oracle's rounds
    bit for bit, the trace within 1e-9, and I never decreases (the applied
    moves of a round share no cluster)."""
    say("boost fit", init, n, d, k, kappa, T)
    X = datagen.mixture(n, d, max(2, k // 2), seed=d + k)
    G, _ = knng.knn_build(X, kappa, xi=50, tau=2, seed=4)
    lab0, C0 = gkmeans.init_labels(X, k, 6, init)
    w_lab, w_C, w_cnt, w_tr, w_t, w_mv = boost.boost_rounds(X, k, G, lab0, T, seed=6, C0=C0)
    p = knnkm.default_params(kappa=kappa, max_iters=T, seed=6, init=init)
    lab = torch.empty(n, dtype=torch.int32, device=DEV)
    C = torch.empty((k, d), dtype=torch.float32, device=DEV)
    cnt = torch.empty(k, dtype=torch.int32, device=DEV)
    tr, t = knnkm.knn_boost_fit(ctx, dev(X), k, dev(G), p, lab, C, cnt)
    say("rounds", t, "moves", w_mv[:8])
    assert t == w_t
    assert np.array_equal(host(lab), w_lab)
    assert np.array_equal(host(cnt), w_cnt)
    assert np.array_equal(host(C), w_C)
    np.testing.assert_allclose(tr, w_tr, rtol=1e-9)
    assert (np.diff(tr) <= 1e-12 * tr[0]).all()


def test_boost_fit_converges_to_a_fixed_point_of_alg2(ctx):
    """Rounds until no sample proposes: the printed sequential Alg. 2 makes no
    move from the returned state, and the labels equal the oracle's."""
    n, d, k, kappa = 900, 4, 15, 8
    say("boost fixed point", n, d, k, kappa)
    X = datagen.mixture(n, d, 10, seed=22)
    G, _ = exact.brute_knn(X, kappa)
    p = knnkm.default_params(kappa=kappa, max_iters=500, seed=9)
    lab = torch.empty(n, dtype=torch.int32, device=DEV)
    C = torch.empty((k, d), dtype=torch.float32, device=DEV)
    cnt = torch.empty(k, dtype=torch.int32, device=DEV)
    tr, t = knnkm.knn_boost_fit(ctx, dev(X), k, dev(G), p, lab, C, cnt)
    assert t < 500
    got = host(lab)
    lab2, _, mv = boost.boost_sequential(X, k, G, got, 1)
    assert mv == [0]
    lab0 = gkmeans.init_labels(X, k, 9, gkmeans.INIT_TWOMEANS)[0]
    w_lab = boost.boost_rounds(X, k, G, lab0, 500, seed=9)[0]
    assert np.array_equal(got, w_lab)


@pytest.mark.parametrize("n,d,kappa,ef,top_k,visits,n_entry,comps", [(3000, 8, 10, 16, 10, 1920, 1, 25),
                                                                      (2500, 33, 20, 64, 20, 1920, 4, 25),
                                                                      (4000, 5, 70, 128, 128, 1920, 16, 25),
                                                                      (3000, 12, 10, 32, 8, 60, 2, 25),
                                                                      (8000, 24, 100, 128, 128, 5000, 8, 1)])
def test_graph_search_parity(ctx, n, d, kappa, ef, top_k, visits, n_entry, comps):
    """Best-first search over a built graph: ids and keys of every query
    equal the oracle's search bit for bit (full and cut-off searches, several
    entry points, kappa above one wavefront, a visit limit above 1,920 that
    takes the larger table of visited points and binds on some queries)."""
    say("graph search", n, d, kappa, ef, top_k, visits, n_entry, comps)
    A = datagen.mixture(n + 200, d, comps, seed=d + kappa)
    X, Q = A[:n], A[n:]
    p = knnkm.default_params(kappa=kappa, xi=50, tau=3, seed=5)
    gi = torch.empty((n, kappa), dtype=torch.int32, device=DEV)
    gd = torch.empty((n, kappa), dtype=torch.float32, device=DEV)
    Xd = dev(X)
    knnkm.knn_build(ctx, Xd, p, gi, gd)
    G = host(gi)
    ids = torch.empty((Q.shape[0], top_k), dtype=torch.int32, device=DEV)
    d2 = torch.empty((Q.shape[0], top_k), dtype=torch.float32, device=DEV)
    knnkm.knn_graph_search(ctx, Xd, gi, dev(Q), ef, top_k, ids, d2, max_visits=visits, n_entry=n_entry, seed=11)
    w_i, w_d = anns.search_all(X, G, Q, ef, top_k, visits, n_entry, seed=11)
    assert np.array_equal(host(ids), w_i)
    assert np.array_equal(host(d2).astype(np.float64), w_d)


def test_assign_autotune_same_result(ctx):
    """The autotuner times every launch shape on the call's own data; the
    results do not depend on the shape it keeps."""
    n, d, k, kappa = 70000, 40, 700, 12
    say("assign autotune", n, d, k, kappa)
    X = dev(datagen.mixture(n, d, 700, seed=44))
    G = dev(np.random.default_rng(9).integers(0, n, (n, kappa)).astype(np.int32))
    C = dev(datagen.mixture(k, d, 700, seed=45))
    lab0 = dev(np.random.default_rng(3).integers(0, k, n).astype(np.int32))

    def run(tune):
        knnkm.knnkm_autotune(ctx, tune)
        out = torch.empty(n, dtype=torch.int32, device=DEV)
        best = torch.empty(n, dtype=torch.float32, device=DEV)
        mv = torch.zeros(1, dtype=torch.int64, device=DEV)
        knnkm.knn_assign(ctx, X, C, G, lab0, out, best, mv)
        return host(out), host(best), host(mv)

    try:
        a = run(False)
        b = run(True)
        c = run(True)
        for u, v, w in zip(a, b, c):
            assert np.array_equal(u, v) and np.array_equal(u, w)
        table = knnkm.knnkm_autotune_table()
        say("tuned", table.strip())
        assert "knn_assign" in table and "n_bin=2^16" in table
    finally:
        knnkm.knnkm_autotune(ctx, True)


SHAPES = [(1, 64, 0), (2, 64, 0), (4, 64, 0), (1, 128, 0), (2, 128, 0), (4, 128, 0), (1, 64, 1), (2, 128, 1)]


@pytest.mark.parametrize("n,d,k,kappa", [(3001, 3, 60, 5), (5000, 32, 150, 20), (4099, 128, 90, 20),
                                         (2500, 512, 40, 50), (3000, 24, 50, 40), (2000, 16, 30, 30)])
def test_assign_shapes_same_bits(ctx, n, d, k, kappa):
    """Every launch shape (samples per row group and pass, samples per block,
    rows loaded first or lazily) gives the same labels, best distances and
    moved count, with and without best distances requested (without them,
    single-candidate samples skip their distances)."""
    say("assign shapes", n, d, k, kappa)
    X = dev(datagen.mixture(n, d, k, seed=n + d))
    C = dev(datagen.mixture(k, d, k, seed=7 * k))
    G = dev(rand_graph(n, kappa, 3)) if kappa < k else None
    # every other sample hands its label to its neighbours, so that many
    # samples have their own cluster as the only candidate
    lab_np = np.random.default_rng(1).integers(0, k, n).astype(np.int32)
    if G is not None:
        Gh = host(G)
        for i in range(0, n, 2):
            lab_np[Gh[i]] = lab_np[i]
    lab = dev(lab_np)
    ref = None
    try:
        for gs, pb, lazy in SHAPES:
            knnkm.knnkm_set_assign_shape(ctx, gs, pb, lazy)
            for want_best in (True, False):
                out = torch.empty(n, dtype=torch.int32, device=DEV)
                best = torch.empty(n, dtype=torch.float32, device=DEV) if want_best else None
                mv = torch.zeros(1, dtype=torch.int64, device=DEV)
                knnkm.knn_assign(ctx, X, C, G, lab, out, best_d2=best, n_moved=mv, kappa=kappa)
                got = (host(out), host(best).view(np.uint32) if want_best else None, int(host(mv)[0]))
                if ref is None:
                    ref = got
                else:
                    assert np.array_equal(got[0], ref[0]), (gs, pb, lazy, want_best)
                    if want_best:
                        assert np.array_equal(got[1], ref[1]), (gs, pb, lazy)
                    assert got[2] == ref[2], (gs, pb, lazy, want_best)
    finally:
        knnkm.knnkm_set_assign_shape(ctx, 0)


def test_fit_graph_equals_eager(ctx):
    """Sweeps 3..T replay a captured graph; every replay matches the eager
    launches (odd T leaves one eager sweep after the pairs), with eager work
    and synchronisations between the runs."""
    n, d, k, kappa, T = 5000, 24, 70, 10, 9
    say("fit graph vs eager", n, d, k, kappa, T)
    X = dev(datagen.mixture(n, d, 70, seed=12))
    G = dev(rand_graph(n, kappa, 5))
    p = knnkm.default_params(kappa=kappa, max_iters=T, seed=3)

    def run(graphs):
        knnkm.knnkm_enable_graphs(ctx, graphs)
        lab = torch.empty(n, dtype=torch.int32, device=DEV)
        C = torch.empty((k, d), dtype=torch.float32, device=DEV)
        cnt = torch.empty(k, dtype=torch.int32, device=DEV)
        tr, it = knnkm.knn_kmeans_fit(ctx, X, k, G, p, lab, C, cnt)
        return host(lab), host(C), host(cnt), tr, it

    try:
        ref = run(False)
        for rep in range(3):
            got = run(True)
            for a, b in zip(ref[:4], got[:4]):
                assert np.array_equal(a, b), rep
            assert got[4] == ref[4] == T
            # unrelated eager work on the same stream between replays (one
            # more sweep from the final state, twice: deterministic)
            Cd, Ld = torch.from_numpy(ref[1]).to(DEV), torch.from_numpy(ref[0]).to(DEV)
            t1 = torch.empty(n, dtype=torch.int32, device=DEV)
            t2 = torch.empty(n, dtype=torch.int32, device=DEV)
            knnkm.knn_assign(ctx, X, Cd, G, Ld, t1)
            knnkm.knn_assign(ctx, X, Cd, G, Ld, t2)
            assert np.array_equal(host(t1), host(t2))
    finally:
        knnkm.knnkm_enable_graphs(ctx, True)


def test_fit_full_size_fixed_point(ctx):
    """The 1M x 128 workload as the benchmark runs it (knn_build, then
    knn_kmeans_fit with T = 30, captured-graph sweeps and active sets).  It
    converges within the 30 sweeps, so its labels are a fixed point of the
    assignment with the returned centroids: no sample moves on the GPU, and
    sampled rows get the oracle's own decision.  The centroids of sampled
    clusters are the float32 means of their members (integer data: the
    float64 sums are exact), the counts are the label histogram and the traced
    distortion is Eqn. 4 of the returned partition."""
    n, d, k, kappa, T = 1_000_000, 128, 10_000, 20, 30
    say("fit full size", n, d, k, kappa, T)
    X = datagen.config_data("c2", seed=1234)
    Xd = dev(X)
    p = knnkm.default_params(kappa=kappa, xi=50, tau=10, max_iters=T, seed=1234)
    gi = torch.empty((n, kappa), dtype=torch.int32, device=DEV)
    gd = torch.empty((n, kappa), dtype=torch.float32, device=DEV)
    knnkm.knn_build(ctx, Xd, p, gi, gd)
    lab = torch.empty(n, dtype=torch.int32, device=DEV)
    C = torch.empty((k, d), dtype=torch.float32, device=DEV)
    cnt = torch.empty(k, dtype=torch.int32, device=DEV)
    tr, it = knnkm.knn_kmeans_fit(ctx, Xd, k, gi, p, lab, C, cnt)
    assert it == T
    out = torch.empty(n, dtype=torch.int32, device=DEV)
    mv = torch.zeros(1, dtype=torch.int64, device=DEV)
    knnkm.knn_assign(ctx, Xd, C, gi, lab, out, None, mv)
    labs, Ch, cnth, G = host(lab), host(C), host(cnt), host(gi)
    assert int(host(mv)[0]) == 0 and np.array_equal(host(out), labs)
    rs = np.random.default_rng(9)
    rows = np.concatenate([rs.choice(n, 4000, replace=False), [0, n - 1]])
    want, _ = gkmeans.gk_assign_rows(X, Ch, labs, G, rows)
    assert np.array_equal(want, labs[rows])
    counts = np.bincount(labs, minlength=k)
    assert np.array_equal(cnth, counts)
    order = np.argsort(labs, kind="stable")
    start = np.concatenate([[0], np.cumsum(counts)])
    for r in rs.choice(np.nonzero(counts)[0], 200, replace=False):
        m = X[order[start[r]:start[r + 1]]].astype(np.float64)
        assert np.array_equal(Ch[r], (m.sum(0) / len(m)).astype(np.float32)), r
    E = 0.0
    for s0 in range(0, n, 100_000):
        diff = X[s0:s0 + 100_000].astype(np.float64) - Ch[labs[s0:s0 + 100_000]].astype(np.float64)
        E += float(np.einsum("ij,ij->", diff, diff))
    E /= n
    assert abs(tr[-1] - E) <= 1e-9 * E, (tr[-1], E)


def test_knn_build_full_size_properties(ctx):
    """knn_build at the full 1M x 128 size as the benchmark runs it: every row
    holds kappa distinct ids other than its own, sorted by (d2, id), and on
    4,000 sampled rows every d2 is the float32 of the exact squared distance
    (integer data: the float64 sum is exact)."""
    n, d, kappa = 1_000_000, 128, 20
    say("knn_build full size", n, d, kappa)
    X = datagen.config_data("c2", seed=1234)
    p = knnkm.default_params(kappa=kappa, xi=50, tau=10, max_iters=30, seed=1234)
    gi = torch.empty((n, kappa), dtype=torch.int32, device=DEV)
    gd = torch.empty((n, kappa), dtype=torch.float32, device=DEV)
    knnkm.knn_build(ctx, dev(X), p, gi, gd)
    G, D = host(gi), host(gd)
    assert G.min() >= 0 and G.max() < n
    assert not (G == np.arange(n)[:, None]).any()
    Gs = np.sort(G, axis=1)
    assert (np.diff(Gs, axis=1) != 0).all()
    ok = (D[:, 1:] > D[:, :-1]) | ((D[:, 1:] == D[:, :-1]) & (G[:, 1:] > G[:, :-1]))
    assert ok.all()
    rows = np.random.default_rng(4).choice(n, 4000, replace=False)
    diff = X[rows][:, None, :].astype(np.float64) - X[G[rows]].astype(np.float64)
    exact = np.einsum("ijk,ijk->ij", diff, diff).astype(np.float32)
    assert np.array_equal(D[rows], exact)


def test_fit_update_exact_at_scale(ctx):
    """The incremental update at a size whose composite vectors (Eqn. 2,
    k x d x 16 bytes of fixed point) far exceed the caches: every centroid is
    the float32 rounding of its members' mean, every traced distortion is the
    Eqn. 2 value of its partition, and two fits give the same bits."""
    n, d, k, kappa, T = 2_000_000, 128, 200_000, 50, 4
    say("fit update at scale", n, d, k, kappa, T)
    X = datagen.mixture_device(n, d, k, 1234, centre="normal", sigma=0.5, device=DEV)
    gi = torch.empty((n, kappa), dtype=torch.int32, device=DEV)
    gd = torch.empty((n, kappa), dtype=torch.float32, device=DEV)
    p = knnkm.default_params(kappa=kappa, tau=2, max_iters=T, seed=1234, precision=knnkm.BF16_RERANK)
    knnkm.knn_build(ctx, X, p, gi, gd)
    sxx = sum(float((X[i:i + 250_000].double() ** 2).sum()) for i in range(0, n, 250_000))
    runs = []
    for rep in range(2):
        lab = torch.empty(n, dtype=torch.int32, device=DEV)
        C = torch.empty((k, d), dtype=torch.float32, device=DEV)
        cnt = torch.empty(k, dtype=torch.int32, device=DEV)
        tr, it = knnkm.knn_kmeans_fit(ctx, X, k, gi, p, lab, C, cnt)
        assert it == T
        s = torch.zeros((k, d), dtype=torch.float64, device=DEV)
        s.index_add_(0, lab.long(), X.double())
        c = torch.bincount(lab.long(), minlength=k)
        assert torch.equal(c.int(), cnt)
        nz = c > 0
        mean = s[nz] / c[nz, None].double()
        # float32 rounding of the mean: within half an ulp (the float64 sum
        # here may itself be rounded, so a hair of slack)
        ulp = torch.abs(mean.float()).double() * 2.0**-23 + 2.0**-149
        err = torch.abs(C[nz].double() - mean)
        assert bool((err <= 0.5 * ulp * (1 + 1e-6)).all()), float((err / ulp).max())
        e_last = (sxx - float(((s[nz] ** 2).sum(1) / c[nz].double()).sum())) / n
        assert abs(tr[-1] - e_last) <= 1e-12 * e_last, (tr[-1], e_last)
        runs.append((host(lab), host(C), tr))
        del s, mean, err, ulp
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1], runs[1][1])
    assert np.array_equal(runs[0][2], runs[1][2])


def test_fit_wide_paths_agree_at_scale(ctx):
    """A wide-row fit at a size where the second sweep moves more than n/8
    samples (its sums are rebuilt: the fit resumes from random labels), late
    sweeps are driven by the changed-
    centroid bits, the graph-entry labels and the drift bounds, and the
    centroid shadow is refreshed by every update: the same labels, centroids,
    counts and trace with the partial distances over the 8-bit shadow, the
    bfloat16 shadow and the float32 rows, and with them switched off (the
    full-distance kernels, none of those paths); every centroid is the float32
    rounding of its members' mean and the last traced distortion the Eqn. 2
    value of the returned partition."""
    n, d, k, kappa, T = 400_000, 512, 40_000, 50, 12
    say("wide fit paths at scale", n, d, k, kappa, T)
    X = datagen.mixture_device(n, d, k, 77, centre="normal", sigma=0.5, device=DEV)
    gi = torch.empty((n, kappa), dtype=torch.int32, device=DEV)
    gd = torch.empty((n, kappa), dtype=torch.float32, device=DEV)
    p = knnkm.default_params(kappa=kappa, tau=2, max_iters=T, seed=77, precision=knnkm.BF16_RERANK)
    knnkm.knn_build(ctx, X, p, gi, gd)
    p.init = knnkm.INIT_LABELS
    lab0 = dev(np.random.default_rng(5).integers(0, k, n).astype(np.int32))
    res = {}
    try:
        for pd in (1, 3, 2, 0):
            knnkm.knnkm_enable_partial_distances(ctx, pd)
            lab = lab0.clone()
            C = torch.zeros((k, d), dtype=torch.float32, device=DEV)  # kept for clusters the labels leave empty
            cnt = torch.empty(k, dtype=torch.int32, device=DEV)
            if pd == 1:
                knnkm.knnkm_enable_timing(ctx, 2)  # per-sweep counts
            tr, it = knnkm.knn_kmeans_fit(ctx, X, k, gi, p, lab, C, cnt)
            assert it == T
            res[pd] = (lab, C, cnt, tr)
            if pd == 1:
                moved = knnkm.knnkm_sweep_stats(ctx)["moved"]
                knnkm.knnkm_enable_timing(ctx, False)
    finally:
        knnkm.knnkm_enable_partial_distances(ctx, True)
        knnkm.knnkm_enable_timing(ctx, False)
    say("moved per sweep", moved)
    assert moved[1] > n // 8 and moved[-1] < n // 100  # the rebuilt second update and sparse late ones
    lab, C, cnt, tr = res[1]
    for pd in (3, 2, 0):
        assert torch.equal(lab, res[pd][0]), pd
        assert torch.equal(C, res[pd][1]), pd
        assert torch.equal(cnt, res[pd][2]), pd
        assert np.array_equal(tr, res[pd][3]), pd
    s = torch.zeros((k, d), dtype=torch.float64, device=DEV)
    s.index_add_(0, lab.long(), X.double())
    c = torch.bincount(lab.long(), minlength=k)
    assert torch.equal(c.int(), cnt)
    nz = c > 0
    mean = s[nz] / c[nz, None].double()
    ulp = torch.abs(mean.float()).double() * 2.0**-23 + 2.0**-149
    assert bool((torch.abs(C[nz].double() - mean) <= 0.5 * ulp * (1 + 1e-6)).all())
    sxx = float((X.double() ** 2).sum())
    e_last = (sxx - float(((s[nz] ** 2).sum(1) / c[nz].double()).sum())) / n
    assert abs(tr[-1] - e_last) <= 1e-12 * e_last, (tr[-1], e_last)
    assert all(tr[t + 1] <= tr[t] * (1 + 1e-12) for t in range(T))


@pytest.mark.parametrize("n,d,k,kappa,T,early", [(20000, 32, 200, 10, 12, False), (200_003, 128, 2000, 20, 9, False),
                                                 (30002, 16, 300, 8, 15, True), (5001, 512, 60, 20, 7, False),
                                                 (777, 3, 25, 6, 10, False)])
def test_fit_active_sets_same_bits(ctx, n, d, k, kappa, T, early):
    """From the second sweep on the fit looks only at samples that had several
    candidates, moved, or have a neighbour that moved; with active sets off
    every sample is looked at.  Labels, centroids, counts, trace and the
    number of sweeps are the same bits, with graph replay and with early
    stopping."""
    say("fit active sets", n, d, k, kappa, T, early)
    X = dev(datagen.mixture(n, d, k, seed=n + 3))
    p = knnkm.default_params(kappa=kappa, max_iters=T, seed=9, early_stop=early)
    gi = torch.empty((n, kappa), dtype=torch.int32, device=DEV)
    gd = torch.empty((n, kappa), dtype=torch.float32, device=DEV)
    knnkm.knn_build(ctx, X, p, gi, gd)

    def run(active):
        knnkm.knnkm_enable_active_sets(ctx, active)
        lab = torch.empty(n, dtype=torch.int32, device=DEV)
        C = torch.empty((k, d), dtype=torch.float32, device=DEV)
        cnt = torch.empty(k, dtype=torch.int32, device=DEV)
        tr, it = knnkm.knn_kmeans_fit(ctx, X, k, gi, p, lab, C, cnt)
        return host(lab), host(C), host(cnt), np.asarray(tr), it

    try:
        ref = run(False)
        for rep in range(2):
            got = run(True)
            for a, b in zip(ref[:4], got[:4]):
                assert np.array_equal(a, b), rep
            assert got[4] == ref[4]
    finally:
        knnkm.knnkm_enable_active_sets(ctx, True)


@pytest.mark.parametrize("n,d,k,kappa,sigma,few", [(32768, 16, 64, 12, 0.1, True), (16384, 8, 16, 8, 0.02, True),
                                                   (20000, 32, 200, 10, 1.0, False)])
def test_fit_first_sweep_marks_same_bits(ctx, n, d, k, kappa, sigma, few):
    """After the first sweep the fit marks the moved samples and the rows
    listing them, or every row once the moved samples number at least
    n/(kappa+1).  The first sweep is replayed through the public calls
    (TwoMeans init with the fit's seed and round tag, its means, one
    knn_assign) to check which rule these data take; either way the fit with
    active sets equals the fit without, bit for bit."""
    say("fit first-sweep marks", n, d, k, kappa, sigma, few)
    X = dev(datagen.mixture(n, d, k, seed=n + 3, sigma=sigma))
    p = knnkm.default_params(kappa=kappa, max_iters=8, seed=9)
    gi = torch.empty((n, kappa), dtype=torch.int32, device=DEV)
    gd = torch.empty((n, kappa), dtype=torch.float32, device=DEV)
    knnkm.knn_build(ctx, X, p, gi, gd)
    init = torch.empty(n, dtype=torch.int32, device=DEV)
    knnkm.knnkm_twomeans(ctx, X, k, 9, knnkm.ROUND_FIT, p.bisect_iters, init)
    C0 = torch.zeros((k, d), dtype=torch.float32, device=DEV)
    c0 = torch.empty(k, dtype=torch.int32, device=DEV)
    knnkm.centroid_update(ctx, X, init, C0, c0)
    lab1 = torch.empty(n, dtype=torch.int32, device=DEV)
    knnkm.knn_assign(ctx, X, C0, gi, init, lab1)
    moved = int((lab1 != init).sum())
    assert (moved < (n + kappa) // (kappa + 1)) == few, moved

    def run(active):
        knnkm.knnkm_enable_active_sets(ctx, active)
        lab = torch.empty(n, dtype=torch.int32, device=DEV)
        C = torch.empty((k, d), dtype=torch.float32, device=DEV)
        cnt = torch.empty(k, dtype=torch.int32, device=DEV)
        tr, it = knnkm.knn_kmeans_fit(ctx, X, k, gi, p, lab, C, cnt)
        return host(lab), host(C), host(cnt), np.asarray(tr), it

    try:
        ref = run(False)
        got = run(True)
        for a, b in zip(ref[:4], got[:4]):
            assert np.array_equal(a, b)
        assert got[4] == ref[4]
    finally:
        knnkm.knnkm_enable_active_sets(ctx, True)


def test_batch_active_sets_same_bits(ctx):
    """The same for a batched fit (jobs of different sizes, one of them with
    kappa >= k, evaluated in full every sweep)."""
    sizes = [3000, 701, 1500, 64, 2201]  # 7466 rows: the last flag word is partly padding
    Xs, n_off, ks, seeds = _batch(sizes, 24, seed=41)
    ks[3] = 2  # kappa >= k: that job is exhaustive
    X = dev(np.concatenate(Xs))
    n, kappa, K = int(n_off[-1]), 10, sum(ks)
    p = knnkm.default_params(kappa=kappa, max_iters=9, seed=4)
    say("batch active sets", sizes, ks)

    def run(active):
        knnkm.knnkm_enable_active_sets(ctx, active)
        gi = torch.empty((n, kappa), dtype=torch.int32, device=DEV)
        gd = torch.empty((n, kappa), dtype=torch.float32, device=DEV)
        lab = torch.empty(n, dtype=torch.int32, device=DEV)
        C = torch.empty((K, 24), dtype=torch.float32, device=DEV)
        cnt = torch.empty(K, dtype=torch.int32, device=DEV)
        tr = knnkm.knnkm_fit_batched(ctx, X, n_off, ks, seeds, p, gi, gd, lab, C, cnt)
        return host(gi), host(lab), host(C), host(cnt), np.asarray(tr)

    try:
        ref = run(False)
        got = run(True)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b)
    finally:
        knnkm.knnkm_enable_active_sets(ctx, True)


# ----------------------------------------------------------------- batching --
def _batch(sizes, d, seed):
    Xs = [datagen.mixture(nq, d, max(2, nq // 32), seed=seed + q) for q, nq in enumerate(sizes)]
    n_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    ks = [max(1, -(-nq // 32)) for nq in sizes]
    seeds = [1000 + 17 * q for q in range(len(sizes))]
    return Xs, n_off, ks, seeds


def _run_alone(ctx, Xq, k, p):
    nq, d = Xq.shape
    gi = torch.empty((nq, p.kappa), dtype=torch.int32, device=DEV)
    gd = torch.empty((nq, p.kappa), dtype=torch.float32, device=DEV)
    Xd = dev(Xq)
    knnkm.knn_build(ctx, Xd, p, gi, gd)
    lab = torch.empty(nq, dtype=torch.int32, device=DEV)
    C = torch.empty((k, d), dtype=torch.float32, device=DEV)
    cnt = torch.empty(k, dtype=torch.int32, device=DEV)
    tr, _ = knnkm.knn_kmeans_fit(ctx, Xd, k, gi, p, lab, C, cnt)
    return host(gi), host(gd), host(lab), host(C), host(cnt), tr


@pytest.mark.parametrize("init", [knnkm.INIT_TWOMEANS, knnkm.INIT_RANDOM])
def test_batch_equals_alone(ctx, init):
    sizes = [64, 97, 300, 1000, 2500, 130, 64, 777]
    d, kappa, T = 24, 8, 6
    say("batch vs alone", init, sizes)
    Xs, n_off, ks, seeds = _batch(sizes, d, seed=40)
    X = np.concatenate(Xs)
    n, K = X.shape[0], sum(ks)
    p = knnkm.default_params(kappa=kappa, xi=50, tau=3, max_iters=T, init=init)
    gi = torch.empty((n, kappa), dtype=torch.int32, device=DEV)
    gd = torch.empty((n, kappa), dtype=torch.float32, device=DEV)
    lab = torch.empty(n, dtype=torch.int32, device=DEV)
    C = torch.empty((K, d), dtype=torch.float32, device=DEV)
    cnt = torch.empty(K, dtype=torch.int32, device=DEV)
    tr = knnkm.knnkm_fit_batched(ctx, dev(X), n_off, ks, seeds, p, gi, gd, lab, C, cnt)
    gi, gd, lab, C, cnt = host(gi), host(gd), host(lab), host(C), host(cnt)
    k_off = np.concatenate([[0], np.cumsum(ks)])
    for q, Xq in enumerate(Xs):
        r0, r1, c0, c1 = n_off[q], n_off[q + 1], k_off[q], k_off[q + 1]
        p.seed = seeds[q]
        a_gi, a_gd, a_lab, a_C, a_cnt, a_tr = _run_alone(ctx, Xq, ks[q], p)
        assert np.array_equal(gi[r0:r1] - r0, a_gi), q
        assert np.array_equal(gd[r0:r1], a_gd), q
        assert np.array_equal(lab[r0:r1], a_lab), q
        assert np.array_equal(C[c0:c1], a_C), q
        assert np.array_equal(cnt[c0:c1], a_cnt), q
        assert np.array_equal(tr[q], a_tr), q


def test_batch_full_size_equals_alone(ctx):
    """The batching form at its full size (4,096 jobs, n ~ U[64, 4096],
    d = 128, k = ceil(n/32), kappa = 8, T = 20, per-job seeds): eight jobs
    spread over the batch, the last one included, give the same graph, labels,
    centroids, counts and trace bits alone as inside the batch."""
    m, d, kappa, T = 4096, 128, 8, 20
    say("batch full size", m)
    sizes = datagen.instance_sizes(m, 2024).astype(np.int64)
    ks = [int(-(-n // 32)) for n in sizes]
    n_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    k_off = np.concatenate([[0], np.cumsum(ks)]).astype(np.int64)
    seeds = [2024 * 7919 + q for q in range(m)]
    X = datagen.batch_mixture_device(sizes, d, ks, 2024, device=DEV)
    p = knnkm.default_params(kappa=kappa, xi=50, tau=10, max_iters=T)

    def outs(n, k):
        return (torch.empty((n, kappa), dtype=torch.int32, device=DEV),
                torch.empty((n, kappa), dtype=torch.float32, device=DEV),
                torch.empty(n, dtype=torch.int32, device=DEV),
                torch.empty((k, d), dtype=torch.float32, device=DEV),
                torch.empty(k, dtype=torch.int32, device=DEV))

    gi, gd, lab, C, cnt = outs(int(n_off[-1]), int(k_off[-1]))
    tr = knnkm.knnkm_fit_batched(ctx, X, n_off, ks, seeds, p, gi, gd, lab, C, cnt)
    jobs = sorted(np.random.default_rng(8).choice(m - 1, 7, replace=False).tolist()) + [m - 1]
    for j in jobs:
        r0, r1, c0, c1 = int(n_off[j]), int(n_off[j + 1]), int(k_off[j]), int(k_off[j + 1])
        o = outs(r1 - r0, c1 - c0)
        t1 = knnkm.knnkm_fit_batched(ctx, X[r0:r1], [0, r1 - r0], [ks[j]], [seeds[j]], p, *o)
        assert torch.equal(o[0] + r0, gi[r0:r1]) and torch.equal(o[1], gd[r0:r1]), j
        assert torch.equal(o[2], lab[r0:r1]) and torch.equal(o[3], C[c0:c1]) and torch.equal(o[4], cnt[c0:c1]), j
        assert np.array_equal(t1[0], tr[j]), j


def test_batch_graph_equals_eager(ctx):
    sizes = [80, 400, 1200, 90]
    d, kappa, T = 16, 8, 8
    say("batch graph vs eager", sizes)
    Xs, n_off, ks, seeds = _batch(sizes, d, seed=21)
    X = dev(np.concatenate(Xs))
    n, K = int(n_off[-1]), sum(ks)
    p = knnkm.default_params(kappa=kappa, xi=50, tau=2, max_iters=T)

    def run(graphs):
        knnkm.knnkm_enable_graphs(ctx, graphs)
        out = [torch.empty((n, kappa), dtype=torch.int32, device=DEV),
               torch.empty((n, kappa), dtype=torch.float32, device=DEV),
               torch.empty(n, dtype=torch.int32, device=DEV),
               torch.empty((K, d), dtype=torch.float32, device=DEV),
               torch.empty(K, dtype=torch.int32, device=DEV)]
        tr = knnkm.knnkm_fit_batched(ctx, X, n_off, ks, seeds, p, *out)
        return [host(t) for t in out] + [tr]

    try:
        a, b = run(False), run(True)
        for u, v in zip(a, b):
            assert np.array_equal(u, v)
    finally:
        knnkm.knnkm_enable_graphs(ctx, True)


def test_batch_matches_oracle(ctx):
    sizes = [70, 200, 450]
    d, kappa, T = 16, 8, 4
    say("batch vs oracle", sizes)
    Xs, n_off, ks, seeds = _batch(sizes, d, seed=77)
    X = np.concatenate(Xs)
    n, K = X.shape[0], sum(ks)
    p = knnkm.default_params(kappa=kappa, xi=50, tau=2, max_iters=T)
    gi = torch.empty((n, kappa), dtype=torch.int32, device=DEV)
    gd = torch.empty((n, kappa), dtype=torch.float32, device=DEV)
    lab = torch.empty(n, dtype=torch.int32, device=DEV)
    C = torch.empty((K, d), dtype=torch.float32, device=DEV)
    cnt = torch.empty(K, dtype=torch.int32, device=DEV)
    tr = knnkm.knnkm_fit_batched(ctx, dev(X), n_off, ks, seeds, p, gi, gd, lab, C, cnt)
    gi, lab = host(gi), host(lab)
    for q, Xq in enumerate(Xs):
        r0, r1 = n_off[q], n_off[q + 1]
        w_i, w_d = knng.knn_build(Xq, kappa, xi=50, tau=2, seed=seeds[q])
        assert np.array_equal(gi[r0:r1] - r0, w_i), q
        w_lab, _, _, w_tr, _, _ = gkmeans.fit(Xq, ks[q], w_i, T, seed=seeds[q])
        assert np.array_equal(lab[r0:r1], w_lab), q
        np.testing.assert_allclose(tr[q], w_tr, rtol=1e-9)


def test_batch_random_init_many_small_jobs(ctx):
    """Random initialisation in a batch of many small jobs whose row ranges
    share 32-bit words of the seed bitmap, with k_q at or near n_q (nearly
    every row is a seed, so a lost bitmap bit would duplicate a seed): each
    job's labels and trace equal the oracle's fit of that job alone."""
    rs = np.random.default_rng(606)
    m, d, kappa, T = 192, 4, 8, 2
    sizes = rs.integers(9, 41, m).astype(np.int64)
    ks = [int(nq - (q % 3)) for q, nq in enumerate(sizes)]
    seeds = [31 * q + 5 for q in range(m)]
    say("batch random init, many small jobs", m)
    Xs = [rs.normal(size=(int(nq), d)).astype(np.float32) for nq in sizes]
    X = np.concatenate(Xs)
    n_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n, K = X.shape[0], sum(ks)
    p = knnkm.default_params(kappa=kappa, xi=50, tau=1, max_iters=T, init=knnkm.INIT_RANDOM)
    gi = torch.empty((n, kappa), dtype=torch.int32, device=DEV)
    gd = torch.empty((n, kappa), dtype=torch.float32, device=DEV)
    lab = torch.empty(n, dtype=torch.int32, device=DEV)
    C = torch.empty((K, d), dtype=torch.float32, device=DEV)
    cnt = torch.empty(K, dtype=torch.int32, device=DEV)
    tr = knnkm.knnkm_fit_batched(ctx, dev(X), n_off, ks, seeds, p, gi, gd, lab, C, cnt)
    gi, lab = host(gi), host(lab)
    for q, Xq in enumerate(Xs):
        r0, r1 = n_off[q], n_off[q + 1]
        w_i, _ = knng.knn_build(Xq, kappa, xi=50, tau=1, seed=seeds[q])
        assert np.array_equal(gi[r0:r1] - r0, w_i), q
        w_lab, _, _, w_tr, _, _ = gkmeans.fit(Xq, ks[q], w_i, T, seed=seeds[q], init=gkmeans.INIT_RANDOM)
        assert np.array_equal(lab[r0:r1], w_lab), q
        # with k_q = n_q the distortion is 0; the GPU evaluates it through the
        # Eqn. 2 identity, whose float64 cancellation error scales with the
        # mean squared norm of the rows
        scale = float((Xq.astype(np.float64) ** 2).sum(1).mean())
        np.testing.assert_allclose(tr[q], w_tr, rtol=1e-9, atol=1e-12 * scale)


def test_c1_end_to_end(ctx):
    """The plain-method workload at its full size (10,000 x 32 from a
    100-component mixture; knn_build with kappa = 10, xi = 50, tau = 10; fit
    with k = 100, T = 20 from the seed-fixed random initialisation) through
    the C ABI against the oracle's knn_build + fit: graph ids and distances,
    labels and counts bit for bit, the distortion trace within 1e-9, and a
    trace that never increases."""
    from oracle import metrics

    c = datagen.CONFIGS["c1"]
    n, d, k, kappa, T, seed = c["n"], c["d"], 100, 10, 20, 1234
    say("c1 end to end", n, d, k, kappa, T)
    X = datagen.config_data("c1", seed=seed)
    Xd = dev(X)
    p = knnkm.default_params(kappa=kappa, xi=50, tau=10, max_iters=T, seed=seed, init=knnkm.INIT_RANDOM)
    gi = torch.empty((n, kappa), dtype=torch.int32, device=DEV)
    gd = torch.empty((n, kappa), dtype=torch.float32, device=DEV)
    knnkm.knn_build(ctx, Xd, p, gi, gd)
    lab = torch.empty(n, dtype=torch.int32, device=DEV)
    C = torch.empty((k, d), dtype=torch.float32, device=DEV)
    cnt = torch.empty(k, dtype=torch.int32, device=DEV)
    tr, it = knnkm.knn_kmeans_fit(ctx, Xd, k, gi, p, lab, C, cnt)
    w_i, w_d = knng.knn_build(X, kappa, xi=50, tau=10, seed=seed)
    assert np.array_equal(host(gi), w_i)
    assert np.array_equal(host(gd), w_d)
    w_lab, w_C, w_cnt, w_tr, w_it, _ = gkmeans.fit(X, k, w_i, T, seed=seed, init=gkmeans.INIT_RANDOM)
    got = host(lab)
    assert metrics.agreement(got, w_lab) >= 0.999
    assert it == w_it and np.array_equal(got, w_lab)
    assert np.array_equal(host(cnt), w_cnt)
    np.testing.assert_allclose(host(C), w_C, rtol=2 ** -23, atol=0)
    np.testing.assert_allclose(tr, w_tr, rtol=1e-9)
    assert (np.diff(tr) <= 1e-12 * tr[0]).all()


def _refine_round_sampled(ctx, Xd, G0i, G0d, k0, seed, t, precision, clusters, rs):
    """One round of graph construction replayed through the public calls
    (two-means tree with round tag t, its means, one graph-restricted sweep,
    the intra-cluster refinement), then the refined rows of `clusters` sampled
    clusters against the oracle's refinement of exactly those clusters (their
    members' rows and old lists copied to the host)."""
    n, d = Xd.shape
    lab = torch.empty(n, dtype=torch.int32, device=DEV)
    knnkm.knnkm_twomeans(ctx, Xd, k0, seed, t, 2, lab)
    C = torch.zeros((k0, d), dtype=torch.float32, device=DEV)
    cnt = torch.empty(k0, dtype=torch.int32, device=DEV)
    knnkm.centroid_update(ctx, Xd, lab, C, cnt)
    lab2 = torch.empty_like(lab)
    knnkm.knn_assign(ctx, Xd, C, G0i, lab, lab2)
    gi, gd = G0i.clone(), G0d.clone()
    knnkm.knnkm_graph_refine(ctx, Xd, lab2, k0, precision, gi, gd)
    torch.cuda.synchronize()
    labels = lab2.long()
    sizes = torch.bincount(labels, minlength=k0)
    nonempty = torch.nonzero(sizes >= 2).flatten().cpu().numpy()
    pick = rs.choice(nonempty, clusters, replace=False)
    order = torch.argsort(labels, stable=True)
    starts = torch.cumsum(sizes, 0) - sizes
    checked = 0
    for c in pick:
        mem_d = order[int(starts[c]):int(starts[c]) + int(sizes[c])]
        mem = mem_d.cpu().numpy()
        A64 = Xd[mem_d].cpu().numpy().astype(np.float64)
        w_i, w_d = knng.refine_cluster(A64, mem, G0i[mem_d].cpu().numpy(), G0d[mem_d].cpu().numpy())
        assert np.array_equal(gi[mem_d].cpu().numpy(), w_i), int(c)
        assert np.array_equal(gd[mem_d].cpu().numpy(), w_d), int(c)
        checked += len(mem)
    return checked


def test_refine_full_size_c2_sampled_clusters(ctx):
    """A graph-construction round at the 1M x 128 workload size (k0 = 20,000
    clusters, kappa = 20, float32 screen), replayed step by step through the
    public calls from the random initial lists: every member row of 200
    sampled clusters equals the oracle's refinement of those clusters."""
    n, d, kappa, seed = 1_000_000, 128, 20, 11
    say("refine full size c2", n, d, kappa)
    X = datagen.config_data("c2", seed=seed)
    Xd = dev(X)
    gi = torch.empty((n, kappa), dtype=torch.int32, device=DEV)
    gd = torch.empty((n, kappa), dtype=torch.float32, device=DEV)
    knnkm.knnkm_graph_init(ctx, Xd, kappa, seed, gi, gd)
    rows = _refine_round_sampled(ctx, Xd, gi, gd, n // 50, seed, 0, knnkm.FP32, 200, np.random.default_rng(1))
    say("rows checked", rows)
    assert rows >= 200 * 2


def test_refine_full_size_c3_sampled_clusters_bf16(ctx):
    """The same at the 10M x 512 size of the precision form (k0 = 200,000,
    kappa = 50, bfloat16 screen with float32/float64 re-rank), from the
    graph after one earlier round: 200 sampled clusters bit for bit."""
    c = datagen.CONFIGS["c3"]
    n, d, kappa, seed = 10_000_000, 512, 50, 12
    say("refine full size c3 bf16", n, d, kappa)
    Xd = datagen.mixture_device(n, d, c["comps"], seed, c["centre"], c["lo"], c["hi"], c["sigma"], c["clip"],
                                c["integer"], device=DEV)
    gi = torch.empty((n, kappa), dtype=torch.int32, device=DEV)
    gd = torch.empty((n, kappa), dtype=torch.float32, device=DEV)
    p = knnkm.default_params(kappa=kappa, xi=50, tau=1, seed=seed, precision=knnkm.BF16_RERANK)
    knnkm.knn_build(ctx, Xd, p, gi, gd)
    rows = _refine_round_sampled(ctx, Xd, gi, gd, n // 50, seed, 1, knnkm.BF16_RERANK, 200,
                                 np.random.default_rng(2))
    say("rows checked", rows)
    assert rows >= 200 * 2


@pytest.mark.parametrize("n,d,k,kappa", [(6000, 512, 300, 50), (5000, 300, 200, 63), (4099, 264, 500, 10),
                                         (3000, 384, 40, 20)])
def test_assign_wide_partial_distances(ctx, n, d, k, kappa):
    """Wide rows: the early-abandoned partial distances (over the 8-bit
    shadow, the bfloat16 shadow or the float32 rows) give the oracle's labels
    and moved count, and the same labels as the full-distance kernel, from
    random input labels (many candidates per sample and many moves) and from
    the labels one sweep later (fewer moves)."""
    say("assign wide", n, d, k, kappa)
    X = datagen.mixture(n, d, max(2, k // 2), seed=d + k, sigma=0.5, centre="normal")
    rs = np.random.default_rng(d)
    C = (X[rs.choice(n, k, replace=False)] + rs.normal(0, 0.1, size=(k, d))).astype(np.float32)
    G = rand_graph(n, kappa, seed=k)
    lab_rand = rs.integers(0, k, n).astype(np.int32)
    lab_near, _, _ = gkmeans.gk_assign(X, C, lab_rand, G)
    Xd, Cd, Gd = dev(X), dev(C), dev(G)
    for lab_in in (lab_rand, lab_near.astype(np.int32)):
        want, _, want_mv = gkmeans.gk_assign(X, C, lab_in, G)
        got = {}
        try:
            for pd in (1, 3, 2, 0):
                knnkm.knnkm_enable_partial_distances(ctx, pd)
                out = torch.empty(n, dtype=torch.int32, device=DEV)
                mv = torch.zeros(1, dtype=torch.int64, device=DEV)
                knnkm.knn_assign(ctx, Xd, Cd, Gd, dev(lab_in), out, None, mv)
                got[pd] = (host(out), int(host(mv)[0]))
        finally:
            knnkm.knnkm_enable_partial_distances(ctx, True)
        for pd in (1, 3, 2, 0):
            assert np.array_equal(got[pd][0], want), pd
            assert got[pd][1] == want_mv, pd


def test_assign_wide_near_ties(ctx):
    """Wide rows whose candidates sit at equal or nearly equal distances
    (duplicated centroids, a centroid copied with one coordinate nudged by one
    ulp): the float64 pass and the tie rule decide as in the oracle, with the
    partial distances over each shadow and over the float32 rows."""
    n, d, k, kappa = 2000, 512, 64, 30
    say("assign wide ties")
    X = datagen.mixture(n, d, 16, seed=5, sigma=0.5, centre="normal")
    rs = np.random.default_rng(3)
    base = X[rs.choice(n, k // 2, replace=False)].copy()
    C = np.concatenate([base, base]).astype(np.float32)  # every centroid twice
    C[k // 2 + 1, 7] = np.nextafter(C[k // 2 + 1, 7], np.float32(np.inf))
    G = rand_graph(n, kappa, seed=8)
    lab_in = rs.integers(0, k, n).astype(np.int32)
    want, _, want_mv = gkmeans.gk_assign(X, C, lab_in, G)
    try:
        for pd in (1, 3, 2):
            knnkm.knnkm_enable_partial_distances(ctx, pd)
            out = torch.empty(n, dtype=torch.int32, device=DEV)
            mv = torch.zeros(1, dtype=torch.int64, device=DEV)
            knnkm.knn_assign(ctx, dev(X), dev(C), dev(G), dev(lab_in), out, None, mv)
            assert np.array_equal(host(out), want), pd
            assert int(host(mv)[0]) == want_mv, pd
    finally:
        knnkm.knnkm_enable_partial_distances(ctx, True)


@pytest.mark.parametrize("d", [512, 320])
def test_fit_wide_partial_distances_same_bits(ctx, d):
    """A fit on wide rows (the library's graph, active sets on) gives the same
    labels, centroids, counts and trace with the partial-distance kernels on
    (reading the 8-bit or the bfloat16 centroid shadow, or float32 centroids
    only) and off, and the oracle's labels and trace."""
    n, k, kappa, T = 6000, 300, 50, 8
    say("fit wide", d)
    X = datagen.mixture(n, d, 500, seed=d, sigma=0.5, centre="normal")
    Xd = dev(X)
    p = knnkm.default_params(kappa=kappa, xi=50, tau=2, max_iters=T, seed=4)
    gi = torch.empty((n, kappa), dtype=torch.int32, device=DEV)
    gd = torch.empty((n, kappa), dtype=torch.float32, device=DEV)
    knnkm.knn_build(ctx, Xd, p, gi, gd)
    res = {}
    try:
        for pd in (1, 3, 2, 0):
            knnkm.knnkm_enable_partial_distances(ctx, pd)
            lab = torch.empty(n, dtype=torch.int32, device=DEV)
            C = torch.empty((k, d), dtype=torch.float32, device=DEV)
            cnt = torch.empty(k, dtype=torch.int32, device=DEV)
            tr, it = knnkm.knn_kmeans_fit(ctx, Xd, k, gi, p, lab, C, cnt)
            res[pd] = (host(lab), host(C), host(cnt), tr)
    finally:
        knnkm.knnkm_enable_partial_distances(ctx, True)
    for mode in (3, 2, 0):
        for a, b in zip(res[1], res[mode]):
            assert np.array_equal(a, b), mode
    w_lab, _, _, w_tr, _, _ = gkmeans.fit(X, k, host(gi), T, seed=4)
    assert np.array_equal(res[1][0], w_lab)
    np.testing.assert_allclose(res[1][3], w_tr, rtol=1e-9)


def test_batch_wide_rows_with_small_jobs(ctx):
    """A batch of wide-row jobs, some with fewer clusters than kappa (every
    cluster of the job is a candidate): graph and fit equal those with the
    partial-distance kernels reading the 8-bit shadow (d = 300: partial
    16-byte units and a partial last chunk), the bfloat16 one or float32
    centroids only, or switched off, and the oracle's."""
    sizes = [120, 900, 64, 1500]
    d, kappa, T = 300, 16, 5
    say("batch wide rows", sizes)
    Xs = [datagen.mixture(nq, d, max(2, nq // 40), seed=90 + q, sigma=0.5, centre="normal")
          for q, nq in enumerate(sizes)]
    n_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    ks = [3, 60, 12, 200]  # jobs 0 and 2: k_q <= kappa
    seeds = [70 + q for q in range(len(sizes))]
    X = dev(np.concatenate(Xs))
    n, K = int(n_off[-1]), sum(ks)
    p = knnkm.default_params(kappa=kappa, xi=50, tau=2, max_iters=T)

    def run(pd):
        knnkm.knnkm_enable_partial_distances(ctx, pd)
        out = [torch.empty((n, kappa), dtype=torch.int32, device=DEV),
               torch.empty((n, kappa), dtype=torch.float32, device=DEV),
               torch.empty(n, dtype=torch.int32, device=DEV),
               torch.empty((K, d), dtype=torch.float32, device=DEV),
               torch.empty(K, dtype=torch.int32, device=DEV)]
        tr = knnkm.knnkm_fit_batched(ctx, X, n_off, ks, seeds, p, *out)
        return [host(t) for t in out] + [tr]

    try:
        a, b, c, e = run(1), run(0), run(2), run(3)
    finally:
        knnkm.knnkm_enable_partial_distances(ctx, True)
    for u, v, w, z in zip(a, b, c, e):
        assert np.array_equal(u, v) and np.array_equal(u, w) and np.array_equal(u, z)
    k_off = np.concatenate([[0], np.cumsum(ks)])
    for q, Xq in enumerate(Xs):
        w_i, _ = knng.knn_build(Xq, kappa, xi=50, tau=2, seed=seeds[q])
        assert np.array_equal(a[0][n_off[q]:n_off[q + 1]] - n_off[q], w_i), q
        w_lab, _, _, w_tr, _, _ = gkmeans.fit(Xq, ks[q], w_i, T, seed=seeds[q])
        assert np.array_equal(a[2][n_off[q]:n_off[q + 1]], w_lab), q
        np.testing.assert_allclose(a[5][q], w_tr, rtol=1e-9)
