"""Request loop of the serving form, driven on a dry server (device = -1): the
same admission, batching and bookkeeping code runs, every batch goes through
the batched driver's argument checks, and nothing touches a GPU."""
import threading

import numpy as np
import pytest

from paper_1705_01813_amd import knnkm

GB = 10**9


def _job(rng, n, d, k, seed=0, **kw):
    X = rng.standard_normal((n, d)).astype(np.float32)
    kw = {"kappa": 8, "tau": 2, "max_iters": 4, **kw}
    p = knnkm.default_params(seed=seed, **kw)
    return X, k, p


def test_server_config_validation():
    for kw in (dict(slots=0), dict(slots=17), dict(max_batch_jobs=0), dict(max_batch_rows=0),
               dict(hbm_budget_bytes=0)):
        with pytest.raises(knnkm.KnnkmError) as e:
            knnkm.Server(device=-1, **kw)
        assert e.value.status == knnkm.EINVAL


def test_server_rejects_invalid_and_oversized_jobs():
    rng = np.random.default_rng(0)
    with knnkm.Server(device=-1, slots=1, hbm_budget_bytes=64 << 20) as S:
        X, k, p = _job(rng, 100, 8, 4)
        with pytest.raises(knnkm.KnnkmError) as e:
            S.submit(X, 101, p)                       # k > n
        assert e.value.status == knnkm.EINVAL
        with pytest.raises(knnkm.KnnkmError):
            S.submit(X[:8], 2, p)                     # fewer than kappa + 1 rows
        bad = knnkm.default_params(kappa=8, xi=1)
        with pytest.raises(knnkm.KnnkmError) as e:
            S.submit(X, k, bad)
        assert "xi" in str(e.value)
        big = np.zeros((400_000, 64), np.float32)     # ~100 MB of rows alone
        with pytest.raises(knnkm.KnnkmError) as e:
            S.submit(big, 100, p)
        assert e.value.status == knnkm.ENOMEM and "budget" in str(e.value)
        t = S.submit(X, k, p)
        assert S.wait(t)["info"]["status"] == knnkm.OK
        st = S.stats()
        assert st["rejected"] == 4 and st["completed"] == 1 and st["submitted"] == 1
        with pytest.raises(knnkm.KnnkmError):
            S.wait(t)                                 # a ticket is waited for once


def test_server_batches_are_homogeneous_fifo_and_within_budget():
    rng = np.random.default_rng(1)
    budget = 2 * GB
    jobs, tickets = [], []
    with knnkm.Server(device=-1, slots=3, max_batch_jobs=5, max_batch_rows=3000, hbm_budget_bytes=budget) as S:
        lock = threading.Lock()

        def client(c):
            r = np.random.default_rng(100 + c)
            for i in range(40):
                n = int(r.integers(20, 2000))
                d = int(r.choice([4, 8]))
                X, k, p = _job(r, n, d, max(1, n // 32), seed=1000 * c + i, tau=int(r.choice([1, 2])))
                t = S.submit(X, k, p)
                with lock:
                    jobs.append((t, n, d, p.tau))
                    tickets.append(t)

        errors = []

        def guarded(c):
            try:
                client(c)
            except Exception as e:  # surfaced below
                errors.append(e)

        th = [threading.Thread(target=guarded, args=(c,)) for c in range(4)]
        for x in th:
            x.start()
        for x in th:
            x.join()
        assert not errors, errors
        res = {t: S.wait(t)["info"] for t in tickets}
        st = S.stats()
    assert st["completed"] == 160 and st["failed"] == 0 and st["queued"] == 0 and st["running"] == 0
    assert st["bytes_peak"] <= budget
    by_batch = {}
    for t, n, d, tau in jobs:
        info = res[t]
        assert info["status"] == knnkm.OK
        assert info["t_submit"] <= info["t_admit"] <= info["t_done"]
        by_batch.setdefault(info["batch"], []).append((t, n, d, tau))
    for b, members in by_batch.items():
        assert len({(d, tau) for _, _, d, tau in members}) == 1      # one class per batch
        assert len(members) == res[members[0][0]]["batch_jobs"] <= 5
        if len(members) > 1:
            assert sum(n for _, n, _, _ in members) <= 3000
    # within a class, jobs are admitted in submission order
    for cls in {(d, tau) for _, _, d, tau in jobs}:
        seq = sorted((t, res[t]["batch"]) for t, _, d, tau in jobs if (d, tau) == cls)
        assert all(a[1] <= b[1] for a, b in zip(seq, seq[1:]))


def test_server_wait_timeout_and_drain_on_close():
    rng = np.random.default_rng(2)
    S = knnkm.Server(device=-1, slots=2)
    ts = [S.submit(*_job(rng, 300, 8, 9, seed=i)) for i in range(10)]
    out = [S.wait(t, timeout_ms=10_000) for t in ts]
    assert all(o is not None and o["info"]["status"] == knnkm.OK for o in out)
    S.close()
