#!/usr/bin/env python3
"""Benchmark of the KNN-graph-supported k-means hot path on one MI355X.

One step = the whole path over one input already resident in HBM:
knn_build (Alg. 3: random lists, tau rounds of TwoMeans + one graph-restricted
sweep + intra-cluster comparison) followed by knn_kmeans_fit (Alg. 2 in its
Lloyd form: TwoMeans initialisation, then T sweeps of assignment, centroid
update and distortion).

Printed value: samples assigned per second per iteration, n / (time of one fit
iteration), from HIP events the library records on its stream inside the timed
steps.  The end-to-end fit time (build + fit) is ms_per_step.  The roofline
entry is the assignment kernel (knn_assign), whose algorithmic bytes per launch
are n*(4d + 8*kappa + 12) + 4*k*d.

Usage: python bench.py [--config c2] [--steps K] [--warmup W] [--gpus 1]
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


def assign_bytes(n, d, k, kappa):
    # X rows, graph rows, neighbour labels, own label, output label, visiting
    # order, centroids (each read once)
    return n * (4 * d + 8 * kappa + 12) + 4 * k * d


def make_data(cfg, seed, device):
    import torch

    from paper_1705_01813_amd import datagen

    c = datagen.CONFIGS[cfg["data"]]
    if cfg["n"] >= 5_000_000:
        return datagen.mixture_device(cfg["n"], c["d"], c["comps"], seed, c["centre"], c["lo"], c["hi"],
                                      c["sigma"], c["clip"], c["integer"], device=device)
    X = datagen.config_data(cfg["data"], seed=seed, n=cfg["n"])
    return torch.from_numpy(X).to(device)


def cpu_baseline(cfg, seed, budget_s):
    """The FP64 oracle's fit iterations on a bounded slice of the same recipe."""
    from oracle import gkmeans, knng
    from paper_1705_01813_amd import datagen

    m = min(cfg["n"], 20_000 if cfg["d"] <= 128 else 5_000)
    k = max(2, (cfg["k"] * m) // cfg["n"])
    X = datagen.config_data(cfg["data"], seed=seed, n=m)
    G, _ = knng.knn_build(X, cfg["kappa"], xi=cfg["xi"], tau=2, seed=seed)
    labels = np.random.default_rng(seed).integers(0, k, m).astype(np.int32)
    C, _, _ = gkmeans.centroid_update(X, labels, k, np.zeros((k, X.shape[1]), np.float32))
    iters, t_total = 0, 0.0
    while t_total < budget_s or iters == 0:
        t0 = time.perf_counter()
        labels, _, _ = gkmeans.gk_assign(X, C, labels, G)
        C, _, _ = gkmeans.centroid_update(X, labels, k, C)
        gkmeans.distortion(X, C, labels)
        t_total += time.perf_counter() - t0
        iters += 1
    return {
        "value": m * iters / t_total,
        "unit": "samples assigned/s per iteration",
        "cores": 1,
        "kind": "oracle",
        "sample": f"first {m} rows of the same recipe, k={k}, kappa={cfg['kappa']}, graph from the oracle's "
                  f"own knn_build (tau=2); {iters} oracle iterations (assign + update + distortion) "
                  f"in {t_total:.1f} s; numpy float64, single thread",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2", choices=sorted(CONFIGS))
    ap.add_argument("--seed", type=int, default=1234)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: --gpus N with N > 1 is not supported "
              "(there is no multi-GPU path)", file=sys.stderr)
        return 2

    import torch

    from paper_1705_01813_amd import knnkm

    cfg = CONFIGS[args.config]
    dev = "cuda:0"
    torch.cuda.set_device(0)
    n, d, k, kappa, T = cfg["n"], cfg["d"], cfg["k"], cfg["kappa"], cfg["T"]
    print(f"[bench] config {args.config}: {cfg['desc']}", file=sys.stderr, flush=True)
    X = make_data(cfg, args.seed, dev)
    G_ids = torch.empty((n, kappa), dtype=torch.int32, device=dev)
    G_d2 = torch.empty((n, kappa), dtype=torch.float32, device=dev)
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    C = torch.empty((k, d), dtype=torch.float32, device=dev)
    counts = torch.empty(k, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()

    ctx = knnkm.Context(0)
    knnkm.knnkm_enable_timing(ctx, True)
    p = knnkm.default_params(kappa=kappa, xi=cfg["xi"], tau=cfg["tau"], max_iters=T, seed=args.seed,
                             init=cfg["init"], precision=cfg["precision"])

    def step():
        knnkm.knn_build(ctx, X, p, G_ids, G_d2)
        return knnkm.knn_kmeans_fit(ctx, X, k, G_ids, p, labels, C, counts)

    for w in range(args.warmup):
        step()
        print(f"[bench] warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    phases = []
    t0 = time.perf_counter()
    for s in range(args.steps):
        trace, iters = step()
        phases.append(knnkm.knnkm_phase_times(ctx))
        print(f"[bench] step {s + 1}/{args.steps}: E_0={trace[0]:.6g} E_T={trace[-1]:.6g} "
              f"phases={phases[-1]}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / args.steps

    mean = {key: float(np.mean([ph[key] for ph in phases])) for key in phases[0]}
    iter_ms = mean["fit_iters_ms"] / max(1.0, mean["iters"])
    value = n / (iter_ms / 1000.0)
    assign_ms = mean["assign_ms"] / max(1.0, mean["assign_launches"])
    bytes_assign = assign_bytes(n, d, k, kappa)
    achieved = bytes_assign / (assign_ms / 1000.0) / 1e9
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
                      "knn_assign_per_launch": assign_ms},
        "final_distortion": float(trace[-1]),
        "roofline": {"kernel": "knn_assign", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": bytes_assign},
    }
    ctx.close()
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg, args.seed, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
