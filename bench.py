#!/usr/bin/env python3
"""Benchmark of the KNN-graph-supported k-means hot path on one MI355X.

One step = the whole path over one input already resident in HBM:
knn_build (Alg. 3: random lists, tau rounds of TwoMeans + one graph-restricted
sweep + intra-cluster comparison) followed by knn_kmeans_fit (Alg. 2 in its
Lloyd form: TwoMeans initialisation, then T sweeps of assignment, centroid
update and distortion).

The default workload is the precision form at 10M x 512 into k = 1M clusters
(the synthetic stand-in for the paper's Table 2 task).  Printed value: samples
assigned per second per iteration, n / (time of one fit iteration), from HIP
events the library records on its stream inside the timed steps.  The
end-to-end fit time (build + fit) is ms_per_step.  The roofline entries are
the assignment kernel (knn_assign): averaged over the fit's sweeps, and for the
first sweep alone (every sample looked at); each names the bytes it counts.

Beside it the line carries the per-sweep record of one fit, the precision
report (graph recall and distortion error against float64 references), the two
added forms measured in the same run ("batching": many independent small jobs
in one batched call against the same jobs one at a time; "serving": a Poisson
stream through the request loop with continuous batching against the same
stream served one job at a time), and the FP64 oracle timed on the host on
slices of the same state.  --config c4 / c5 run those forms at full size and
print their own line; --candidate-sharing measures how many candidate clusters
consecutive samples share.

Usage: python bench.py [--config c3] [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CONFIGS = {
    # name: data recipe + method parameters
    "c1": dict(data="c1", n=10_000, d=32, k=100, kappa=10, T=20, init=1, precision=0, xi=50, tau=10,
               desc="n=10,000 d=32 k=100 kappa=10 T=20 random init; 100-component Gaussian mixture"),
    "c2": dict(data="c2", n=1_000_000, d=128, k=10_000, kappa=20, T=30, init=0, precision=0, xi=50, tau=10,
               desc="n=1,000,000 d=128 k=10,000 kappa=20 T=30 xi=50 tau=10 TwoMeans init; "
                    "SIFT1M-shaped integer mixture (10,000 components, sigma 20, clipped to [0,255])"),
    "c3": dict(data="c3", n=10_000_000, d=512, k=1_000_000, kappa=50, T=30, init=0, precision=1, xi=50,
               tau=10, desc="n=10,000,000 d=512 k=1,000,000 kappa=50 T=30 BF16-screened graph build; "
                            "VLAD10M-shaped mixture (1,000,000 components, sigma 0.5)"),
}

HBM_PEAK_GBS = 8000.0

# many independent small jobs: n ~ U[64, 4096], d = 128, k = ceil(n/32),
# ceil(n/32) mixture components (centres U[-10,10], sigma 1), kappa = 8, T = 20
C4 = dict(m=4096, d=128, kappa=8, T=20, xi=50, tau=10)
# serving stream: Poisson arrivals at 200 jobs/s, n log-uniform in [1e3, 1e6],
# d in {64, 128, 256}, k = n/100, kappa = 16, T = 20, budget 200 GB
C5 = dict(rate=200.0, seconds=60.0, dims=(64, 128, 256), kappa=16, T=20, xi=50, tau=10, budget=200 * 10**9,
          pool_rows=1_000_000)


def exact_neighbours(X, rows, kappa):
    """Ids of the kappa nearest other rows of X[rows] (plain PyTorch float64
    on the GPU, blockwise over X)."""
    import torch

    n = X.shape[0]
    q = X[rows].double()
    qn = (q * q).sum(1, keepdim=True)
    best_d, best_i = None, None
    step = 1 << 20
    for s0 in range(0, n, step):
        xb = X[s0:s0 + step].double()
        dd = qn + (xb * xb).sum(1)[None, :] - 2.0 * (q @ xb.T)
        ids = torch.arange(s0, s0 + xb.shape[0], device=X.device)
        dd[ids[None, :] == rows[:, None]] = float("inf")
        if best_d is None:
            cd, ci = dd, ids[None, :].expand_as(dd)
        else:
            cd, ci = torch.cat([best_d, dd], 1), torch.cat([best_i, ids[None, :].expand_as(dd)], 1)
        best_d, pos = torch.topk(cd, kappa, dim=1, largest=False)
        best_i = torch.gather(ci, 1, pos)
    return best_i


def tau_study(n, seed, log, taus=(0, 1, 2, 3, 4, 5, 6, 8, 10, 14), kappa=20, samples=1000, T=30):
    """Graph quality and clustering distortion as functions of the number of
    construction rounds tau (Sec. 4.3): on n rows of the 1M x 128 recipe,
    knn_build with tau rounds, the top-1 recall and recall@kappa of the graph
    on sampled rows (exact float64 neighbours), and the distortion of a
    30-iteration GK-means fit (Lloyd form) into n/100 clusters with that graph."""
    import torch

    from paper_1705_01813_amd import datagen, knnkm

    dev = "cuda:0"
    X = torch.from_numpy(datagen.config_data("c2", seed=seed, n=n)).to(dev)
    d = X.shape[1]
    k = max(1, n // 100)
    g = torch.Generator(device="cpu").manual_seed(seed)
    rows = torch.randint(0, n, (samples,), generator=g).to(dev)
    ex = exact_neighbours(X, rows, kappa)
    ctx = knnkm.Context(0)
    gi = torch.empty((n, kappa), dtype=torch.int32, device=dev)
    gd = torch.empty((n, kappa), dtype=torch.float32, device=dev)
    lab = torch.empty(n, dtype=torch.int32, device=dev)
    C = torch.empty((k, d), dtype=torch.float32, device=dev)
    cnt = torch.empty(k, dtype=torch.int32, device=dev)
    out = []
    for kappa, tau in graphs:
        gi = torch.empty((n, kappa), dtype=torch.int32, device=dev)
        gd = torch.empty((n, kappa), dtype=torch.float32, device=dev)
        p = knnkm.default_params(kappa=kappa, xi=50, tau=tau, max_iters=T, seed=seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        knnkm.knn_build(ctx, X, p, gi, gd)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        got = gi[rows].long()
        top1 = float((got[:, 0] == ex[:, 0]).double().mean())
        hits = sum(len(set(a.tolist()) & set(b.tolist())) for a, b in zip(got, ex))
        tr, _ = knnkm.knn_kmeans_fit(ctx, X, k, gi, p, lab, C, cnt)
        out.append({"tau": tau, "build_s": tb, "recall_top1": top1, "recall_at_kappa": hits / float(samples * kappa),
                    "fit_E_T": float(tr[-1])})
        log(f"tau {tau}: build {tb:.3f} s, top-1 recall {top1:.3f}, E_T {tr[-1]:.6g}")
    ctx.close()
    return {"workload": f"n={n} rows of the 1M x 128 recipe, d={d}, kappa={kappa}, xi=50; fit k={k}, T={T}; "
                        f"recall on {samples} sampled rows against exact float64 neighbours", "sweep": out}


SEARCH = dict(n=1_000_000, d=128, xi=50, r=16)


def search_bench(nq, seed, log, recipe="lowrank", efs=(10, 16, 32, 64, 128), entries=(1, 16), visits=(1920, 7680),
                 graphs=((20, 10), (50, 10), (50, 32)), top_k=10, samples=1000):
    """Nearest-neighbour search over the built graph (knn_graph_search).
    n + nq rows of one recipe (the low-intrinsic-dimension ``lowrank`` recipe,
    or the clustering mixture of the 1M x 128 workload), the last nq held out
    as queries; the graph of knn_build over the rest for each (kappa, tau); the top-1
    recall of the graph on sampled rows; recall@top_k of the search against
    exact float64 neighbours and queries per second for several list sizes ef
    and entry counts."""
    import torch

    from paper_1705_01813_amd import datagen, knnkm

    dev = "cuda:0"
    n, d = SEARCH["n"], SEARCH["d"]
    if recipe == "lowrank":
        A = torch.from_numpy(datagen.lowrank(n + nq, d, seed, r=SEARCH["r"])).to(dev)
    else:
        A = torch.from_numpy(datagen.config_data("c2", seed=seed, n=n + nq)).to(dev)
    X, Q = A[:n], A[n:].contiguous()
    # exact neighbours of the queries (plain PyTorch float64), blockwise
    truth = []
    for q0 in range(0, nq, 1024):
        q = Q[q0:q0 + 1024].double()
        best_d, best_i = None, None
        for s0 in range(0, n, 1 << 18):
            xb = X[s0:s0 + (1 << 18)].double()
            dd = (q * q).sum(1, keepdim=True) + (xb * xb).sum(1)[None, :] - 2.0 * (q @ xb.T)
            ids = torch.arange(s0, s0 + xb.shape[0], device=dev)[None, :].expand_as(dd)
            if best_d is not None:
                dd, ids = torch.cat([best_d, dd], 1), torch.cat([best_i, ids], 1)
            best_d, pos = torch.topk(dd, top_k, dim=1, largest=False)
            best_i = torch.gather(ids, 1, pos)
        truth.append(best_i)
    truth = torch.cat(truth).cpu().numpy()
    rows_s = np.random.Generator(np.random.PCG64(seed + 7)).choice(n, samples, replace=False)
    nn1 = exact_neighbours(X, torch.from_numpy(rows_s).to(dev), 1)[:, 0].cpu().numpy()
    ctx = knnkm.Context(0)
    out_i = torch.empty((nq, top_k), dtype=torch.int32, device=dev)
    out_d = torch.empty((nq, top_k), dtype=torch.float32, device=dev)
    rows = []
    for kappa, tau in graphs:
        gi = torch.empty((n, kappa), dtype=torch.int32, device=dev)
        gd = torch.empty((n, kappa), dtype=torch.float32, device=dev)
        p = knnkm.default_params(kappa=kappa, xi=SEARCH["xi"], tau=tau, seed=seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        knnkm.knn_build(ctx, X, p, gi, gd)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        g = gi.cpu().numpy()
        r1 = float(np.mean(g[rows_s, 0] == nn1))
        log(f"search graph kappa={kappa} tau={tau}: built in {tb:.2f} s, top-1 recall {r1:.4f}")
        for mv, ne, ef in [(mv, ne, ef) for mv in visits for ne in entries for ef in efs]:
            args = dict(max_visits=mv, n_entry=ne, seed=seed)
            knnkm.knn_graph_search(ctx, X, gi, Q, ef, top_k, out_i, out_d, **args)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            knnkm.knn_graph_search(ctx, X, gi, Q, ef, top_k, out_i, out_d, **args)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            got = out_i.cpu().numpy().astype(np.int64)
            rec = float(np.mean([len(set(a.tolist()) & set(b.tolist())) / float(top_k) for a, b in zip(got, truth)]))
            rows.append({"kappa": kappa, "tau": tau, "graph_top1_recall": r1, "build_s": tb, "max_visits": mv,
                         "entries": ne, "ef": ef, f"recall_at_{top_k}": rec, "queries_per_s": nq / dt,
                         "ms": dt * 1e3})
            log(f"search kappa={kappa} tau={tau} visits<={mv} entries={ne} ef={ef}: recall@{top_k} {rec:.4f}, "
                f"{nq / dt:.0f} queries/s")
    ctx.close()
    what = (f"lowrank recipe (intrinsic dimension {SEARCH['r']}, SIFT-like integers)" if recipe == "lowrank"
            else "the 1M x 128 clustering mixture")
    return {"workload": f"n={n:,} d={d} {what}; {nq} held-out rows of the same draw as queries; graph of "
                        f"knn_build (xi={SEARCH['xi']}); recall@{top_k} against exact float64 "
                        "neighbours; one launch over all queries", "sweep": rows}


def scaling_sweeps(seed, log, ns=(10_000, 100_000, 1_000_000, 10_000_000), ks=(1024, 2048, 4096, 8192), T=30):
    """Sec. 5.4's scalability tests on the 10M x 512 recipe (d = 512, ten rows
    per mixture component): n varied at k = 1,024, and k varied at n = 10^6;
    each point is knn_build (tau = 10, xi = 50, bfloat16 screen) plus a
    30-iteration fit."""
    import torch

    from paper_1705_01813_amd import datagen, knnkm

    dev = "cuda:0"
    c = datagen.CONFIGS["c3"]
    kappa = 50
    ctx = knnkm.Context(0)

    def point(X, k):
        n, d = X.shape
        p = knnkm.default_params(kappa=kappa, xi=50, tau=10, max_iters=T, seed=seed, precision=knnkm.BF16_RERANK)
        gi = torch.empty((n, kappa), dtype=torch.int32, device=dev)
        gd = torch.empty((n, kappa), dtype=torch.float32, device=dev)
        lab = torch.empty(n, dtype=torch.int32, device=dev)
        C = torch.empty((k, d), dtype=torch.float32, device=dev)
        cnt = torch.empty(k, dtype=torch.int32, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        knnkm.knn_build(ctx, X, p, gi, gd)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tr, _ = knnkm.knn_kmeans_fit(ctx, X, k, gi, p, lab, C, cnt)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return {"n": n, "k": k, "build_s": t1 - t0, "fit_s": t2 - t1, "total_s": t2 - t0, "E_T": float(tr[-1])}

    def data(n):
        return datagen.mixture_device(n, c["d"], max(1, n // 10), seed, c["centre"], c["lo"], c["hi"], c["sigma"],
                                      c["clip"], c["integer"], device=dev)

    by_n, by_k = [], []
    for n in ns:
        X = data(n)
        by_n.append(point(X, 1024))
        log(f"scaling n={n}, k=1024: {by_n[-1]}")
        del X
    X = data(1_000_000)
    for k in ks:
        by_k.append(point(X, k))
        log(f"scaling n=1M, k={k}: {by_k[-1]}")
    del X
    ctx.close()
    return {"workload": "10M x 512 recipe (d=512, ten rows per component, sigma 0.5), kappa=50, tau=10, xi=50, "
                        "bfloat16 screen, T=30", "k1024_varying_n": by_n, "n1M_varying_k": by_k}


def precision_report(ctx, X, p, G_ids, G_d2, labels, C, trace, samples, seed, log):
    """Quality of a precision-form result, against references computed with
    plain PyTorch in float64 on the GPU (independent of the library's kernels):
    recall@kappa of the graph on sampled rows against exact neighbours, the
    relative error of the reported final distortion against the float64
    distortion of the returned labels, and whether the FP32-screened build gives
    the same graph as the BF16-screened one."""
    import torch

    from paper_1705_01813_amd import knnkm

    n, d = X.shape
    kappa = G_ids.shape[1]
    g = torch.Generator(device="cpu").manual_seed(seed)
    rows = torch.randint(0, n, (samples,), generator=g).to(X.device)
    best_i = exact_neighbours(X, rows, kappa)
    step = 1 << 20
    got = G_ids[rows].long()
    hits = sum(len(set(a.tolist()) & set(b.tolist())) for a, b in zip(got, best_i))
    recall = hits / float(samples * kappa)
    # distortion of the returned labels in float64 (means recomputed)
    lab = labels.long()
    k = C.shape[0]
    sums = torch.zeros((k, d), dtype=torch.float64, device=X.device)
    cnt = torch.bincount(lab, minlength=k).double()
    for s0 in range(0, n, step):
        sums.index_add_(0, lab[s0:s0 + step], X[s0:s0 + step].double())
    means = sums / cnt.clamp(min=1)[:, None]
    e = 0.0
    for s0 in range(0, n, step):
        diff = X[s0:s0 + step].double() - means[lab[s0:s0 + step]]
        e += float((diff * diff).sum())
    e /= n
    log(f"precision report: recall@{kappa} {recall:.4f} on {samples} rows, E {trace[-1]:.9g} vs {e:.9g}")
    # the same build with the FP32 screen
    pf = knnkm.Params.from_buffer_copy(p)
    pf.precision = knnkm.FP32
    gi2 = torch.empty_like(G_ids)
    gd2 = torch.empty_like(G_d2)
    knnkm.knn_build(ctx, X, pf, gi2, gd2)
    same = bool(torch.equal(gi2, G_ids) and torch.equal(gd2, G_d2))
    del gi2, gd2
    return {"recall_at_kappa_sampled": recall, "recall_rows": samples,
            "distortion_reported": float(trace[-1]), "distortion_fp64_of_labels": e,
            "distortion_rel_error": abs(float(trace[-1]) - e) / e,
            "bf16_graph_equals_fp32_graph": same,
            "reference": "plain PyTorch float64 on the GPU (exact neighbours of sampled rows; means and "
                         "distortion of the returned labels)"}


ASSIGN_SOURCES = ("assign.hip", "assign_pd.hip")  # the fit assignment kernels


def assign_source_sha256():
    """Key of the assignment kernels' code: the sources with // comments and
    blank lines left out (a comment edit keeps a measured traffic valid)."""
    import hashlib
    import re

    h = hashlib.sha256()
    for f in ASSIGN_SOURCES:
        for line in open(os.path.join(ROOT, "paper_1705_01813_amd", "csrc", f), encoding="utf-8"):
            code = re.sub(r"//.*$", "", line).strip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()


def measured_traffic(config, key="traffic_bytes_per_launch"):
    """HBM bytes per fit assignment launch from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter on a plain copy
    of known size), or None when that summary is missing, is for another
    workload, or predates the current source of the assignment kernels."""
    path = os.path.join(ROOT, "profiles", f"knn_assign_{config}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            a, b = line.split("=", 1)
            kv[a.strip()] = b.strip()
    if kv.get("assign_source_sha256") != assign_source_sha256() or key not in kv:
        return None
    return float(kv[key])


def traffic_summary(config, fetch_csv, write_csv, bench_json):
    """Writes profiles/knn_assign_<config>_traffic.txt from two rocprofv3
    counter runs of `bench.py --config <config> --steps 1 --warmup 0
    --counters` (FETCH_SIZE, then WRITE_SIZE) and that run's JSON line: the
    fit assignment launches of the kernel pass (the last fit of the run) with
    their list compactions, each counter scaled by its value on the 1 GiB copy
    at the end of the run.  Host only."""
    import csv

    def per_dispatch(path, counter):
        rows = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            key = int(r["Dispatch_Id"])
            nm = r["Kernel_Name"]
            v = float(r["Counter_Value"])
            if key in rows:
                rows[key] = (nm, rows[key][1] + v, int(r["Grid_Size"]))
            else:
                rows[key] = (nm, v, int(r["Grid_Size"]))
        return [(k,) + rows[k] for k in sorted(rows)]

    line = [ln for ln in open(bench_json) if ln.startswith("{")][-1]
    b = json.loads(line)
    sw = b["sweeps"]
    launches = len(sw["assign_ms"])
    out = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        ds = per_dispatch(path, counter)
        # the copy: the last elementwise dispatch of the run (torch.mul over
        # 2^28 floats; the fill before it writes and reads next to nothing)
        copy = [x for x in ds if "elementwise" in x[1]][-1]
        scale = float(1 << 20) / copy[2]  # KiB of the 1 GiB stream
        assign = [i for i, x in enumerate(ds) if "k_assign" in x[1]]
        last = assign[-launches:]
        total = sum(ds[i][2] for i in last)
        compact = sum(x[2] for x in ds[last[0]:last[-1] + 1] if "k_act_compact" in x[1])
        out[counter] = {"scale": scale, "copy_kib": copy[2], "raw_kib_per_launch": (total + compact) / launches,
                        "first_kib": ds[last[0]][2],
                        "first_kernel": ds[last[0]][1].replace("(anonymous namespace)::", "").replace("void ", "",
                                                                                                      1).split("(")[0]}
    f, w = out["FETCH_SIZE"], out["WRITE_SIZE"]
    fetch_b = f["raw_kib_per_launch"] * 1024 * f["scale"]
    write_b = w["raw_kib_per_launch"] * 1024 * w["scale"]
    first_b = (f["first_kib"] * f["scale"] + w["first_kib"] * w["scale"]) * 1024
    cfg = CONFIGS[config]
    n, d, k, kappa = cfg["n"], cfg["d"], cfg["k"], cfg["kappa"]
    ev = sum(sw["evaluated"][1:]) + n
    ls = sum(sw["listed"][1:]) + n
    alg = (sum(assign_bytes(n, d, k, kappa, e, l) for e, l in zip(sw["evaluated"][1:], sw["listed"][1:]))
           + assign_bytes(n, d, k, kappa)) / launches
    path = os.path.join(ROOT, "profiles", f"knn_assign_{config}_traffic.txt")
    with open(path, "w") as fh:
        fh.write(f"# knn_assign on the {cfg['desc']} workload: HBM traffic per fit assignment launch\n")
        fh.write("# Commands (one MI355X; R = the repository root; one counter per run):\n")
        for c, o in (("FETCH_SIZE", "out_fetch"), ("WRITE_SIZE", "out_write")):
            fh.write(f"#   cd /tmp && timeout -s KILL 600 rocprofv3 --pmc {c} --kernel-include-regex "
                     f"\"k_assign|k_act_compact|elementwise\" -d {o} -o run --output-format csv -- python3 "
                     f"$R/bench.py --config {config} --steps 1 --warmup 0 --counters > {o}.json\n")
        fh.write(f"#   python3 $R/bench.py --config {config} --traffic-summary out_fetch/run_counter_collection.csv "
                 f"out_write/run_counter_collection.csv out_fetch.json\n")
        fh.write("# bench.py --counters runs the workload with every sweep as its own dispatch, then a 1 GiB "
                 "elementwise copy.\n")
        fh.write(f"# FETCH_SIZE of the 1 GiB copy read {f['copy_kib']:.0f} KiB (scale {f['scale']:.4f}); "
                 f"WRITE_SIZE {w['copy_kib']:.0f} KiB (scale {w['scale']:.4f}).\n")
        fh.write(f"# The last fit's {launches} assignment launches (the kernel pass of the run) and the list "
                 "compactions between them; totals per launch:\n")
        fh.write(f"fetch_kib_per_launch_raw = {f['raw_kib_per_launch']:.1f}\n")
        fh.write(f"write_kib_per_launch_raw = {w['raw_kib_per_launch']:.1f}\n")
        fh.write(f"fetch_bytes_per_launch = {fetch_b:.0f}\n")
        fh.write(f"write_bytes_per_launch = {write_b:.0f}\n")
        fh.write(f"traffic_bytes_per_launch = {fetch_b + write_b:.0f}\n")
        fh.write(f"algorithmic_bytes_per_launch = {alg:.0f}\n")
        fh.write(f"# (per launch: graph rows, neighbour, own and output labels of the {ls / launches:.0f} samples "
                 f"listed on average; rows of the {ev / launches:.0f} samples evaluated; centroids once; a flag "
                 "byte per sample; listed and evaluated counts from the same run's JSON line)\n")
        fh.write(f"traffic_over_algorithmic = {(fetch_b + write_b) / alg:.3f}\n")
        fh.write(f"# first launch ({f['first_kernel']}: every sample looked at and evaluated)\n")
        fh.write(f"first_traffic_bytes = {first_b:.0f}\n")
        fh.write(f"first_algorithmic_bytes = {assign_bytes(n, d, k, kappa):.0f}\n")
        fh.write(f"assign_source_sha256 = {assign_source_sha256()}\n")
    return path


def _pct(v, q):
    return float(np.percentile(np.asarray(v, np.float64), q)) if len(v) else None


def bench_batching(m, sample, seed, log):
    """Batched call over m jobs against the same jobs one at a time."""
    import torch

    from paper_1705_01813_amd import datagen, knnkm

    dev = "cuda:0"
    sizes = datagen.instance_sizes(m, seed).astype(np.int64)
    ks = [int(-(-n // 32)) for n in sizes]
    n_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    k_off = np.concatenate([[0], np.cumsum(ks)]).astype(np.int64)
    seeds = [seed * 7919 + q for q in range(m)]
    d, kappa = C4["d"], C4["kappa"]
    N, K = int(n_off[-1]), int(k_off[-1])
    X = datagen.batch_mixture_device(sizes, d, ks, seed, device=dev)
    p = knnkm.default_params(kappa=kappa, xi=C4["xi"], tau=C4["tau"], max_iters=C4["T"])

    def outs(n, k):
        return (torch.empty((n, kappa), dtype=torch.int32, device=dev),
                torch.empty((n, kappa), dtype=torch.float32, device=dev),
                torch.empty(n, dtype=torch.int32, device=dev),
                torch.empty((k, d), dtype=torch.float32, device=dev),
                torch.empty(k, dtype=torch.int32, device=dev))

    ctx = knnkm.Context(0)
    gi, gd, lab, C, cnt = outs(N, K)
    knnkm.knnkm_fit_batched(ctx, X, n_off, ks, seeds, p, gi, gd, lab, C, cnt)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    knnkm.knnkm_fit_batched(ctx, X, n_off, ks, seeds, p, gi, gd, lab, C, cnt)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    log(f"batched: {m} jobs, {N} rows in {t_batch:.3f} s")
    # the same jobs one at a time (a sample of them), same entry point, m = 1
    one = []
    same = True
    for q in range(-2, sample):
        j = max(q, 0)
        r0, r1, c0, c1 = int(n_off[j]), int(n_off[j + 1]), int(k_off[j]), int(k_off[j + 1])
        o = outs(r1 - r0, c1 - c0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        knnkm.knnkm_fit_batched(ctx, X[r0:r1], [0, r1 - r0], [ks[j]], [seeds[j]], p, *o)
        torch.cuda.synchronize()
        if q >= 0:  # the first two calls warm up
            one.append(time.perf_counter() - t0)
            same = same and bool(torch.equal(o[2], lab[r0:r1]) and torch.equal(o[3], C[c0:c1])
                                 and torch.equal(o[4], cnt[c0:c1]) and torch.equal(o[0] + r0, gi[r0:r1]))
    ctx.close()
    rows_sample = int(n_off[sample])
    # one-at-a-time time of all m jobs, extrapolated from the sample by rows
    t_one_all = sum(one) * N / rows_sample
    return {
        "workload": f"{m} independent jobs, n ~ U[64,4096] (sum {N} rows), d={d}, k=ceil(n/32) (sum {K}), "
                    f"kappa={kappa}, T={C4['T']}, tau={C4['tau']}, xi={C4['xi']}, per-job seeds",
        "batched_s": t_batch,
        "batched_jobs_per_s": m / t_batch,
        "one_at_a_time_jobs_per_s": len(one) / sum(one),
        "one_at_a_time_s_extrapolated": t_one_all,
        "speedup": t_one_all / t_batch,
        "one_at_a_time_latency_ms": {"p50": 1e3 * _pct(one, 50), "p99": 1e3 * _pct(one, 99)},
        "one_at_a_time_sample": f"first {sample} jobs ({rows_sample} rows), extrapolated to all jobs by rows",
        "identical_on_sample": same,
    }


def bench_serving(seconds, seed, log, rate=None, single_seconds=10.0):
    """The serving stream through the request loop (continuous batching, 4
    slots) and through the same loop restricted to one job at a time."""
    import threading

    import torch

    from paper_1705_01813_amd import datagen, knnkm

    rate = rate or C5["rate"]
    stream = datagen.serving_stream(rate, seconds, seed, dims=C5["dims"])
    P = C5["pool_rows"]
    pools = {}
    for i, d in enumerate(C5["dims"]):
        # per-d pool of mixture rows (P/100 components, centres U[-10,10],
        # sigma 1) in pinned host memory; a job is a random slice of it
        Xd = datagen.mixture_device(P, d, P // 100, seed + i, device="cuda:0")
        pools[d] = torch.empty((P, d), dtype=torch.float32, pin_memory=True)
        pools[d].copy_(Xd)
        del Xd
    torch.cuda.synchronize()
    rs = np.random.default_rng(seed)
    jobs = []
    for j, (t, n, d) in enumerate(stream):
        off = int(rs.integers(0, P - n + 1))
        jobs.append((t, pools[d][off:off + n], max(1, n // 100), j))

    def run(slots, max_jobs):
        S = knnkm.Server(device=0, slots=slots, max_batch_jobs=max_jobs, hbm_budget_bytes=C5["budget"])
        tickets = [None] * len(jobs)
        t_start = time.perf_counter()

        def client():
            for j, (t, X, k, sd) in enumerate(jobs):
                delay = t_start + t - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                p = knnkm.default_params(kappa=C5["kappa"], xi=C5["xi"], tau=C5["tau"], max_iters=C5["T"],
                                         seed=sd)
                tickets[j] = S.submit(X, k, p)

        th = threading.Thread(target=client)
        th.start()
        infos = []
        done = 0
        for j in range(len(jobs)):
            while tickets[j] is None:
                time.sleep(0.0005)
            r = S.wait(tickets[j])
            infos.append(r["info"])
            done += 1
            if done % 100 == 0:
                log(f"serving (slots={slots}, batch<={max_jobs}): {done}/{len(jobs)} done")
        th.join()
        st = S.stats()
        S.close()
        lat = [i["t_done"] - i["t_submit"] for i in infos]
        span = max(i["t_done"] for i in infos) - min(i["t_submit"] for i in infos)
        return {
            "jobs": len(infos),
            "jobs_per_s": len(infos) / span,
            "makespan_s": span,
            "latency_ms": {"p50": 1e3 * _pct(lat, 50), "p99": 1e3 * _pct(lat, 99), "max": 1e3 * max(lat)},
            "queue_wait_ms_p50": 1e3 * _pct([i["t_admit"] - i["t_submit"] for i in infos], 50),
            "batches": st["batches"],
            "mean_batch_jobs": len(infos) / max(1, st["batches"]),
            "max_queued": st["max_queued"],
            "hbm_peak_charged_gb": st["bytes_peak"] / 1e9,
            "ws_overruns": st["ws_overruns"],
            "keeps_up": span <= window[0] * 1.05,
        }

    rows = sum(int(X.shape[0]) for _, X, _, _ in jobs)
    log(f"serving: {len(jobs)} jobs ({rows} rows) over {seconds} s")
    window = [seconds]  # arrival window of the jobs run() serves
    cont = run(4, 4096)
    # one job at a time: the whole stream for short windows; for longer ones
    # the jobs arriving in the first single_seconds (its throughput does not
    # depend on the window; its queueing latency grows with it)
    all_jobs = jobs
    if single_seconds and single_seconds < seconds:
        jobs = [j for j in all_jobs if j[0] < single_seconds]
        window[0] = single_seconds
    single = run(1, 1)
    single["sampled"] = (f"jobs arriving in the first {single_seconds:g} s ({len(jobs)} of {len(all_jobs)})"
                         if len(jobs) < len(all_jobs) else "every job")
    return {
        "workload": f"Poisson arrivals at {rate:g} jobs/s for {seconds:g} s ({len(all_jobs)} jobs, {rows} rows): "
                    f"n = round(10^U[3,6]), d in {{64,128,256}}, k = n/100, kappa={C5['kappa']}, "
                    f"T={C5['T']}, tau={C5['tau']}, xi={C5['xi']}; rows are random slices of a per-d "
                    f"mixture pool in pinned host memory; HBM budget {C5['budget'] / 1e9:g} GB",
        "continuous_batching": cont,
        "one_at_a_time": single,
        "speedup_jobs_per_s": cont["jobs_per_s"] / single["jobs_per_s"],
    }


def assign_bytes(n, d, k, kappa, evaluated=None, listed=None):
    # per sample looked at: graph row, neighbour labels, own and output label,
    # visiting order; per sample whose distances are evaluated: its row (a
    # sample whose neighbours all share its cluster needs none); centroids
    # once; with active sets, one flag byte per sample for the list
    ev = n if evaluated is None else evaluated
    ls = n if listed is None else listed
    return ls * (8 * kappa + 12) + ev * 4 * d + 4 * k * d + (n if listed is not None else 0)


def make_data(cfg, seed, device):
    import torch

    from paper_1705_01813_amd import datagen

    c = datagen.CONFIGS[cfg["data"]]
    if cfg["n"] >= 5_000_000:
        return datagen.mixture_device(cfg["n"], c["d"], c["comps"], seed, c["centre"], c["lo"], c["hi"],
                                      c["sigma"], c["clip"], c["integer"], device=device)
    X = datagen.config_data(cfg["data"], seed=seed, n=cfg["n"])
    return torch.from_numpy(X).to(device)


class _Rows:
    """Rows of a device matrix at given ids, copied to the host and indexable
    by those ids (the oracle's row-restricted sweep reads no other rows)."""

    def __init__(self, mat, ids):
        import torch

        ids = np.asarray(ids, np.int64)
        self.shape = tuple(int(v) for v in mat.shape)
        self.data = mat[torch.from_numpy(ids).to(mat.device)].cpu().numpy()
        self.pos = np.full(int(ids.max()) + 1, -1, np.int64)
        self.pos[ids] = np.arange(ids.size)

    def __getitem__(self, r):
        return self.data[self.pos[np.asarray(r, np.int64)]]


def _host_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    env = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS",
                                          "BLIS_NUM_THREADS") if os.environ.get(k) is not None}
    return model, len(os.sched_getaffinity(0)), env


def cpu_baseline(ctx, X, G_ids, cfg, seed, budget_s, log):
    """The FP64 oracle's iteration (graph-restricted assignment, centroid
    update, distortion) on slices of the GPU's own state -- the fit's initial
    partition (TwoMeans labels and their means) and the graph the GPU built --
    timed on the host.  Slices of growing size (up to 100k rows) run until the
    time budget is spent; the per-iteration time for all n rows is extrapolated
    linearly in the slice size (least squares over the slices)."""
    import torch

    from oracle import gkmeans
    from paper_1705_01813_amd import knnkm

    n, d = X.shape
    k = cfg["k"]
    lab0 = torch.empty(n, dtype=torch.int32, device=X.device)
    knnkm.knnkm_twomeans(ctx, X, k, seed, 0xFFFF, 2, lab0)
    C0 = torch.zeros((k, d), dtype=torch.float32, device=X.device)
    cnt = torch.empty(k, dtype=torch.int32, device=X.device)
    knnkm.centroid_update(ctx, X, lab0, C0, cnt)
    torch.cuda.synchronize()
    labels = lab0.cpu().numpy()
    C = C0.cpu().numpy()
    del C0, cnt, lab0
    rs = np.random.default_rng(seed)
    sizes, times = [], []
    m, spent, cpu_spent = 12_500, 0.0, 0.0
    while m <= min(n, 100_000) and (len(sizes) < 2 or spent < budget_s):
        start = int(rs.integers(0, n - m + 1))
        rows = np.arange(start, start + m)
        Xr, Gr = _Rows(X, rows), _Rows(G_ids, rows)
        w0, c0 = time.perf_counter(), time.process_time()
        out, _ = gkmeans.gk_assign_rows(Xr, C, labels, Gr, rows)
        Cn, _, _ = gkmeans.centroid_update(Xr.data, out, k, C)
        gkmeans.distortion(Xr.data, Cn, out)
        dt = time.perf_counter() - w0
        cpu_spent += time.process_time() - c0
        spent += dt
        sizes.append(m)
        times.append(dt)
        log(f"oracle iteration on a {m}-row slice: {dt:.2f} s")
        m *= 2
    b, a = np.polyfit(np.asarray(sizes, np.float64), np.asarray(times, np.float64), 1) if len(sizes) > 1 \
        else (times[0] / sizes[0], 0.0)
    t_full = a + b * n
    model, affinity, env = _host_info()
    used = cpu_spent / spent if spent > 0 else 1.0
    return {
        "value": n / t_full,
        "unit": "samples assigned/s per iteration",
        "cores": max(1, int(round(used))),
        "kind": "oracle",
        "sample": f"one oracle iteration (assign + update + distortion, numpy float64) on row slices of "
                  f"{sizes} of the GPU's state for this workload (TwoMeans partition with its means, the GPU's "
                  f"graph, all k={k} centroids); per-iteration time for n={n} extrapolated linearly in the "
                  f"slice size: {t_full:.1f} s = {a:.2f} s + {b * 1e3:.4f} ms/row",
        "extrapolated": True,
        "slice_seconds": dict(zip([str(v) for v in sizes], times)),
        "cpu_over_wall": used,
        "host": {"cpu_model": model, "affinity_cores": affinity, "blas_env": env},
    }


def xi_sweep(n, seed, log, xis=(50, 100, 256, 512), kappa=50):
    """One graph-refinement round (Alg. 3 inner loops) at d = 512 on n rows of
    the 10M x 512 recipe, for cluster sizes xi: the clusters are a TwoMeans
    partition into n / xi leaves, the graph the random initial lists.  Per xi
    and screen precision: the round's time, the dense Gram flops of the
    clusters (2 xi d per member), the rate against the MFMA peaks -- also the
    float64 one: clusters of 33 to 1024 members form their Gram in float64 on
    MFMA whatever the screen precision -- and the ceiling the round's bytes put
    on it (member rows and graph rows read once: 4d + 8 kappa per member)."""
    import torch

    from paper_1705_01813_amd import datagen, knnkm

    dev = "cuda:0"
    c = datagen.CONFIGS["c3"]
    d = c["d"]
    X = datagen.mixture_device(n, d, max(1, n // 10), seed, c["centre"], c["lo"], c["hi"], c["sigma"], c["clip"],
                               c["integer"], device=dev)
    ctx = knnkm.Context(0)
    gi0 = torch.empty((n, kappa), dtype=torch.int32, device=dev)
    gd0 = torch.empty((n, kappa), dtype=torch.float32, device=dev)
    knnkm.knnkm_graph_init(ctx, X, kappa, seed, gi0, gd0)
    lab = torch.empty(n, dtype=torch.int32, device=dev)
    out = []
    peaks = {"fp32": 157.3, "bf16": 2500.0, "fp64": 78.6}
    for xi in xis:
        k0 = max(1, n // xi)
        knnkm.knnkm_twomeans(ctx, X, k0, seed, 0, 2, lab)
        flops = 2.0 * d * float((torch.bincount(lab.long(), minlength=k0).double() ** 2).sum())
        bytes_ = n * (4 * d + 8 * kappa)
        row = {"xi": xi, "k0": k0, "gram_flops": flops, "bytes": bytes_, "flop_per_byte": flops / bytes_}
        for name, prec in (("fp32", knnkm.FP32), ("bf16", knnkm.BF16_RERANK)):
            gi, gd = gi0.clone(), gd0.clone()
            knnkm.knnkm_graph_refine(ctx, X, lab, k0, prec, gi, gd)  # warm-up (same inputs)
            gi.copy_(gi0)
            gd.copy_(gd0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            knnkm.knnkm_graph_refine(ctx, X, lab, k0, prec, gi, gd)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            tf = flops / (ms * 1e-3) / 1e12
            cap = min(1.0, (flops / bytes_) * HBM_PEAK_GBS / 1e3 / peaks[name])
            row[name] = {"refine_ms": ms, "gram_tflops": tf, "frac_of_mfma_peak": tf / peaks[name],
                         "frac_of_fp64_mfma_peak": tf / peaks["fp64"], "hbm_ceiling_frac_of_mfma_peak": cap}
            log(f"xi {xi}: k0 {k0}, {name} screen: {ms:.2f} ms, {tf:.2f} TFLOP/s")
        out.append(row)
    ctx.close()
    return {"workload": f"one refinement round, n={n} rows of the 10M x 512 recipe, d={d}, kappa={kappa}, "
                        "TwoMeans clusters of xi members, random initial lists",
            "peaks_tflops": peaks, "sweep": out}


def candidate_sharing(ctx, X, G_ids, k, seed, log):
    """How many distinct candidate clusters T consecutive samples of the fit's
    working order (the cluster order of the initial partition) have together,
    against the sum of their own counts: the reuse a tile of T samples could
    get from staging candidate centroid rows once."""
    import torch

    from paper_1705_01813_amd import knnkm

    n = X.shape[0]
    lab = torch.empty(n, dtype=torch.int32, device=X.device)
    knnkm.knnkm_twomeans(ctx, X, k, seed, 0xFFFF, 2, lab)
    order = torch.argsort(lab.long(), stable=True)
    cand = torch.cat([lab[:, None], lab[G_ids.long()]], 1)[order]
    srt = torch.sort(cand, 1)[0]
    per = (1 + (srt[:, 1:] != srt[:, :-1]).sum(1)).double()
    total = float(per.sum())
    out = {"candidates_per_sample": total / n}
    w = cand.shape[1]
    for T in (4, 16, 64, 256, 1024, 8192):
        m = n // T
        union = 0
        rows_per = max(1, (1 << 27) // (T * w))
        for r0 in range(0, m, rows_per):
            blk = cand[r0 * T:min(m, r0 + rows_per) * T].reshape(-1, T * w)
            sb = torch.sort(blk, 1)[0]
            union += int((1 + (sb[:, 1:] != sb[:, :-1]).sum(1)).sum())
        own = float(per[:m * T].sum())
        out[f"tile_{T}"] = {"distinct_per_tile": union / m, "sum_per_tile": own / m, "reuse": own / union}
        log(f"tile {T}: {out[f'tile_{T}']}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3", choices=sorted(CONFIGS) + ["c4", "c5"])
    ap.add_argument("--no-forms", action="store_true", help="skip the batching and serving measurements")
    ap.add_argument("--no-precision", action="store_true", help="skip the precision report")
    ap.add_argument("--counters", action="store_true",
                    help="for counter runs: sweeps as separate dispatches (no graph), no forms or oracle, "
                         "then a 1 GiB elementwise copy that calibrates the memory counters")
    ap.add_argument("--traffic-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "BENCH_JSON"),
                    help="host only: write the committed traffic summary of --config from two counter runs")
    ap.add_argument("--boost", type=int, default=0, metavar="R",
                    help="after the timed steps, run the boost form (knn_boost_fit) for up to R rounds from the same "
                         "graph and initialisation and report its rounds, time and distortion beside the Lloyd form's")
    ap.add_argument("--tau-study", type=int, default=0, metavar="N",
                    help="graph recall and fit distortion against the number of construction rounds on N rows")
    ap.add_argument("--search", type=int, default=0, metavar="Q",
                    help="graph search: Q held-out queries against a 1M x 128 graph, recall@10 and queries/s")
    ap.add_argument("--search-recipe", default="lowrank", choices=["lowrank", "mixture"],
                    help="input recipe of --search")
    ap.add_argument("--scaling", action="store_true",
                    help="the scalability sweeps at d=512: n from 10k to 10M at k=1024, k from 1024 to 8192 at n=1M")
    ap.add_argument("--xi-sweep", type=int, default=0, metavar="N",
                    help="time one refinement round at d=512 on N rows for xi in 50, 100, 256, 512")
    ap.add_argument("--candidate-sharing", action="store_true",
                    help="after one build, measure the candidate clusters shared by consecutive samples")
    ap.add_argument("--forms-jobs", type=int, default=4096, help="jobs of the batching measurement")
    ap.add_argument("--forms-sample", type=int, default=64, help="jobs timed one at a time")
    ap.add_argument("--serve-seconds", type=float, default=None,
                    help="arrival window of the serving run (default 2 s beside the main line, 60 s for c5)")
    ap.add_argument("--seed", type=int, default=1234)
    ap.add_argument("--pd-mode", type=int, default=None, choices=[0, 1, 2, 3],
                    help="wide-row partial distances: 0 off, 1 8-bit shadow (the library's default), 2 float32 "
                         "only, 3 bfloat16 shadow")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    args = ap.parse_args()
    if args.traffic_summary:
        print(traffic_summary(args.config, *args.traffic_summary))
        return 0
    if args.gpus != 1:
        print("bench.py runs on one GPU only: --gpus N with N > 1 is not supported "
              "(there is no multi-GPU path)", file=sys.stderr)
        return 2

    import torch

    from paper_1705_01813_amd import knnkm

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if args.tau_study:
        print(json.dumps({"tau_study": tau_study(args.tau_study, args.seed, log)}), flush=True)
        return 0
    if args.search:
        print(json.dumps({"search": search_bench(args.search, args.seed, log, recipe=args.search_recipe)}),
              flush=True)
        return 0
    if args.scaling:
        print(json.dumps({"scaling": scaling_sweeps(args.seed, log)}), flush=True)
        return 0
    if args.xi_sweep:
        print(json.dumps({"xi_sweep": xi_sweep(args.xi_sweep, args.seed, log)}), flush=True)
        return 0
    if args.config == "c4":
        b = bench_batching(C4["m"], args.forms_sample, args.seed, log)
        print(json.dumps({"metric": "jobs/s", "value": b["batched_jobs_per_s"], "unit": "jobs/s", "n_gpus": 1,
                          "higher_is_better": True, "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                          "config": {"workload": b["workload"]}, "batching": b}), flush=True)
        return 0
    if args.config == "c5":
        sv = bench_serving(args.serve_seconds or C5["seconds"], args.seed, log)
        c = sv["continuous_batching"]
        print(json.dumps({"metric": "jobs/s; p50/p99 job latency", "value": c["jobs_per_s"], "unit": "jobs/s",
                          "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "f32",
                          "data": "synthetic", "config": {"workload": sv["workload"]}, "serving": sv}),
              flush=True)
        return 0

    cfg = CONFIGS[args.config]
    dev = "cuda:0"
    torch.cuda.set_device(0)
    n, d, k, kappa, T = cfg["n"], cfg["d"], cfg["k"], cfg["kappa"], cfg["T"]
    log(f"config {args.config}: {cfg['desc']}")
    X = make_data(cfg, args.seed, dev)
    G_ids = torch.empty((n, kappa), dtype=torch.int32, device=dev)
    G_d2 = torch.empty((n, kappa), dtype=torch.float32, device=dev)
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    C = torch.empty((k, d), dtype=torch.float32, device=dev)
    counts = torch.empty(k, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()

    ctx = knnkm.Context(0)
    knnkm.knnkm_enable_timing(ctx, True)
    if args.pd_mode is not None:
        knnkm.knnkm_enable_partial_distances(ctx, args.pd_mode)
    if args.counters:
        knnkm.knnkm_enable_graphs(ctx, False)
        args.no_forms = args.no_cpu_baseline = args.no_precision = True
    p = knnkm.default_params(kappa=kappa, xi=cfg["xi"], tau=cfg["tau"], max_iters=T, seed=args.seed,
                             init=cfg["init"], precision=cfg["precision"])

    if args.candidate_sharing:
        knnkm.knn_build(ctx, X, p, G_ids, G_d2)
        res = candidate_sharing(ctx, X, G_ids, k, args.seed, log)
        print(json.dumps({"candidate_sharing": res, "config": {"workload": f"{args.config}: {cfg['desc']}"}}),
              flush=True)
        ctx.close()
        return 0

    def step():
        knnkm.knn_build(ctx, X, p, G_ids, G_d2)
        return knnkm.knn_kmeans_fit(ctx, X, k, G_ids, p, labels, C, counts)

    for w in range(args.warmup):
        step()
        log(f"warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    phases = []
    t0 = time.perf_counter()
    for s in range(args.steps):
        trace, iters = step()
        phases.append(knnkm.knnkm_phase_times(ctx))
        log(f"step {s + 1}/{args.steps}: E_0={trace[0]:.6g} E_T={trace[-1]:.6g} phases={phases[-1]}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / args.steps

    mean = {key: float(np.mean([ph[key] for ph in phases])) for key in phases[0]}
    iter_ms = mean["fit_iters_ms"] / max(1.0, mean["iters"])
    value = n / (iter_ms / 1000.0)
    # kernel pass (after the timed steps): the fit again, with HIP events around
    # every assignment launch, which then runs its sweeps eagerly
    knnkm.knnkm_enable_timing(ctx, 2)
    knnkm.knn_kmeans_fit(ctx, X, k, G_ids, p, labels, C, counts)
    kp = knnkm.knnkm_phase_times(ctx)
    sw = knnkm.knnkm_sweep_stats(ctx)
    knnkm.knnkm_enable_timing(ctx, 1)
    log(f"sweeps: {sw}")
    launches = max(1.0, kp["assign_launches"])
    assign_ms = kp["assign_ms"] / launches
    evaluated = kp["assign_evaluated"] / launches if kp["assign_evaluated"] >= 0 else None
    listed = kp["assign_listed"] / launches if kp["assign_listed"] >= 0 else None
    bytes_assign = assign_bytes(n, d, k, kappa, evaluated, listed)
    achieved = bytes_assign / (assign_ms / 1000.0) / 1e9
    first_ms = sw["assign_ms"][0]
    bytes_first = assign_bytes(n, d, k, kappa)
    achieved_first = bytes_first / (first_ms / 1000.0) / 1e9
    counted = ("per launch: for every sample looked at its graph row and neighbour labels (8 kappa B) and "
               "its own label, output label and visiting order (12 B); for every sample whose distances are "
               "evaluated its row (4d B); the centroids once (4kd B); with active sets one flag byte per "
               "sample")
    out = {
        "metric": "samples assigned/s per iteration",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {cfg['desc']}", "n": n, "d": d, "k": k, "kappa": kappa,
                   "iterations": T, "xi": cfg["xi"], "tau": cfg["tau"],
                   "graph_screen": "bf16" if cfg["precision"] else "fp32"},
        "end_to_end_fit_s": ms_per_step / 1000.0,
        "phases_ms": {"knn_build": mean["build_ms"], "fit_init": mean["fit_init_ms"],
                      "fit_iterations": mean["fit_iters_ms"], "per_iteration": iter_ms,
                      "knn_assign_per_launch": assign_ms, "knn_assign_first_sweep": first_ms},
        "final_distortion": float(trace[-1]),
        "roofline": {"kernel": "knn_assign (fit sweeps, average per launch)", "bound": "hbm",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.config),
                     "algorithmic_bytes_per_launch": bytes_assign, "bytes_counted": counted,
                     "evaluated_samples_per_launch": evaluated, "listed_samples_per_launch": listed,
                     "launches_timed": kp["assign_launches"], "avg_launch_ms": assign_ms},
        "roofline_first_sweep": {"kernel": "knn_assign (first fit sweep: every sample looked at and evaluated)",
                                 "bound": "hbm", "achieved": achieved_first, "peak": HBM_PEAK_GBS,
                                 "unit": "GB/s", "frac": achieved_first / HBM_PEAK_GBS,
                                 "traffic": measured_traffic(args.config, "first_traffic_bytes"),
                                 "algorithmic_bytes_per_launch": bytes_first,
                                 "bytes_counted": "n (8 kappa + 12) + n 4d + 4kd: every graph row, neighbour "
                                                  "label, own and output label and sample row, and the "
                                                  "centroids once",
                                 "launch_ms": first_ms},
        "sweeps": sw,
    }
    out["autotuned_shapes"] = [ln for ln in knnkm.knnkm_autotune_table().splitlines() if ln]
    out["workspace_gb"] = {"held": ctx.workspace_bytes() / 1e9,
                           "planning_estimate": knnkm.knnkm_workspace_estimate(n, d, k, p) / 1e9}
    if args.boost:
        pb = knnkm.Params.from_buffer_copy(p)
        pb.max_iters = args.boost
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lab_b, C_b, cnt_b = torch.empty_like(labels), torch.empty_like(C), torch.empty_like(counts)
        tb, rb = knnkm.knn_boost_fit(ctx, X, k, G_ids, pb, lab_b, C_b, cnt_b)
        torch.cuda.synchronize()
        tbs = time.perf_counter() - t0
        out["boost_form"] = {"rounds": rb, "converged": rb < args.boost, "seconds": tbs,
                             "ms_per_round": 1e3 * tbs / max(1, rb), "E_0": float(tb[0]), "E_final": float(tb[-1]),
                             "lloyd_E_T": float(trace[-1]),
                             "E_final_over_lloyd": float(tb[-1]) / float(trace[-1]),
                             "note": "Alg. 2 as printed (Eqn. 3 moves) in conflict-free data-parallel rounds, from "
                                     "the same graph and initial partition as the Lloyd form's fit"}
        log(f"boost form: {rb} rounds in {tbs:.2f} s, E {tb[-1]:.6g} (Lloyd form {trace[-1]:.6g})")
        del lab_b, C_b, cnt_b
    if cfg["precision"] and not args.no_precision:
        out["precision"] = precision_report(ctx, X, p, G_ids, G_d2, labels, C, trace, 64, args.seed, log)
    del labels, C, counts
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("timing the oracle on the host")
        out["cpu_baseline"] = cpu_baseline(ctx, X, G_ids, cfg, args.seed, args.cpu_seconds, log)
    ctx.close()
    del X, G_ids, G_d2
    torch.cuda.empty_cache()
    if args.counters:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB read, 1 GiB written
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
    if not args.no_forms:
        out["batching"] = bench_batching(args.forms_jobs, args.forms_sample, args.seed, log)
        out["serving"] = bench_serving(args.serve_seconds or 2.0, args.seed, log)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
