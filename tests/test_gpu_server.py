"""Serving form on the GPU: jobs submitted to the request loop while others run
return exactly what the same job returns alone (graph, labels, centroids,
counts, distortion trace), served jobs of both dimensionalities equal the
FP64 oracle's build and fit of that job, and the HBM budget bounds what is
admitted."""
import threading
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import gkmeans, knng  # noqa: E402
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


def _alone(ctx, X, k, p):
    """The job alone through knn_build + knn_kmeans_fit."""
    n, d = X.shape
    Xd = torch.from_numpy(np.ascontiguousarray(X)).to(DEV)
    gi = torch.empty((n, p.kappa), dtype=torch.int32, device=DEV)
    gd = torch.empty((n, p.kappa), dtype=torch.float32, device=DEV)
    knnkm.knn_build(ctx, Xd, p, gi, gd)
    lab = torch.empty(n, dtype=torch.int32, device=DEV)
    C = torch.empty((k, d), dtype=torch.float32, device=DEV)
    cnt = torch.empty(k, dtype=torch.int32, device=DEV)
    tr, _ = knnkm.knn_kmeans_fit(ctx, Xd, k, gi, p, lab, C, cnt)
    torch.cuda.synchronize()
    return gi.cpu().numpy(), lab.cpu().numpy(), C.cpu().numpy(), cnt.cpu().numpy(), tr


def _jobs(count, seed):
    r = np.random.default_rng(seed)
    out = []
    for j in range(count):
        n = int(r.integers(64, 3000))
        d = int(r.choice([16, 32]))
        X = datagen.mixture(n, d, max(2, n // 32), seed=seed * 1000 + j)
        if j % 3 == 0:  # a strided view: rows of a wider host array
            W = np.zeros((n, d + 5), np.float32)
            W[:, :d] = X
            X = W[:, :d]
        p = knnkm.default_params(kappa=8, xi=50, tau=3, max_iters=6, seed=500 + j)
        out.append((X, max(1, -(-n // 32)), p))
    return out


def _check_same(ctx, jobs, results):
    for j, ((X, k, p), res) in enumerate(zip(jobs, results)):
        gi, lab, C, cnt, tr = _alone(ctx, X, k, p)
        assert res["info"]["status"] == knnkm.OK
        assert np.array_equal(res["G_ids"], gi), j
        assert np.array_equal(res["labels"], lab), j
        assert np.array_equal(res["C"], C), j
        assert np.array_equal(res["counts"], cnt), j
        assert np.array_equal(res["trace"], tr), j


def _check_oracle(jobs, results, picks):
    """Served jobs against the oracle's knn_build + fit of the same job: graph
    ids, labels and counts bit for bit, centroids within one float32 ulp, the
    trace within 1e-9."""
    for j in picks:
        (X, k, p), res = jobs[j], results[j]
        X = np.ascontiguousarray(X)
        w_i, _ = knng.knn_build(X, p.kappa, xi=p.xi, tau=p.tau, seed=p.seed)
        assert np.array_equal(res["G_ids"], w_i), j
        w_lab, w_C, w_cnt, w_tr, _, _ = gkmeans.fit(X, k, w_i, p.max_iters, seed=p.seed, init=p.init)
        assert np.array_equal(res["labels"], w_lab), j
        assert np.array_equal(res["counts"], w_cnt), j
        np.testing.assert_allclose(res["C"], w_C, rtol=2 ** -23, atol=0)
        np.testing.assert_allclose(res["trace"], w_tr, rtol=1e-9)


def test_server_alone_equals_mix(ctx):
    jobs = _jobs(24, seed=3)
    say("server mix", [(X.shape, k) for X, k, _ in jobs])
    tickets = [None] * len(jobs)
    with knnkm.Server(device=0, slots=3, max_batch_jobs=8, hbm_budget_bytes=8 * 10**9) as S:
        def client():
            r = np.random.default_rng(9)
            for j, (X, k, p) in enumerate(jobs):
                tickets[j] = S.submit(X, k, p, want_graph=True)
                if j >= 12:  # the first half arrives at once, the rest spread out
                    time.sleep(float(r.uniform(0, 0.004)))

        th = threading.Thread(target=client)
        th.start()
        th.join()
        results = [S.wait(t) for t in tickets]
        st = S.stats()
    say("stats", st)
    assert st["completed"] == len(jobs) and st["failed"] == 0
    assert st["max_batch_jobs_seen"] > 1
    assert st["ws_overruns"] == 0
    assert len({r["info"]["batch"] for r in results}) < len(jobs)
    _check_same(ctx, jobs, results)
    # two served jobs of each dimensionality against the oracle
    picks = [j for j, (X, _, _) in enumerate(jobs) if X.shape[1] == 16][:2] + \
            [j for j, (X, _, _) in enumerate(jobs) if X.shape[1] == 32][:2]
    say("oracle check of served jobs", picks)
    assert len(picks) == 4
    _check_oracle(jobs, results, picks)


def test_server_tight_budget(ctx):
    jobs = _jobs(8, seed=5)
    say("server tight budget")
    # room for about one job at a time
    with knnkm.Server(device=-1) as dry:
        need = max(dry.wait(dry.submit(X, k, p))["info"]["footprint_bytes"] for X, k, p in jobs)
    budget = int(need * 1.3)
    with knnkm.Server(device=0, slots=4, hbm_budget_bytes=budget) as S:
        tickets = [S.submit(X, k, p, want_graph=True) for X, k, p in jobs]
        results = [S.wait(t) for t in tickets]
        st = S.stats()
    say("stats", st, "budget", budget)
    assert st["completed"] == len(jobs) and st["bytes_peak"] <= budget and st["ws_overruns"] == 0
    _check_same(ctx, jobs, results)
