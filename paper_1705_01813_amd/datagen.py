"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no arithmetic of the clustering method; it only draws input
matrices.  Both the HIP path and the oracle consume the same float32 arrays it
returns.  Recipes (stand-ins for the paper's datasets, Table 1):

* ``mixture``: an isotropic Gaussian mixture.  Component of each sample uniform,
  centres uniform in a box or standard normal, per-dimension noise sigma,
  optional clipping and rounding to integers (half to even) before storage as
  float32.  With centres U[0,255]^128, sigma 20, clipped and rounded it has the
  shape of SIFT1M (1M x 128 non-negative integer features); with centres
  N(0,1)^512 and sigma 0.5 it has the shape of VLAD10M (10M x 512).
* ``integer_grid``: integers in [0, 255] (exact in float32 and bfloat16).
* ``lowrank``: features of low intrinsic dimension, for nearest-neighbour
  search.  A latent z in R^r is an overlapping Gaussian mixture (component
  means N(0, spread^2 I), unit covariance); the feature is an offset plus a
  random linear map of z (entries N(0, 1/r), scaled) plus isotropic noise,
  clipped and rounded like SIFT.  Unlike the well-separated mixtures above,
  whose KNN graphs fall apart into one piece per component, it has the
  continuous local structure that a search over a KNN graph walks through.

Host generation uses numpy's PCG64; ``mixture_device`` draws the same recipe
with torch on a GPU (different bits, same distribution) for sizes where host
generation would dominate the run.
"""
import numpy as np

CONFIGS = {
    # name: (n, d, components, centre kind, centre lo, centre hi, sigma, clip, round)
    "c1": dict(n=10_000, d=32, comps=100, centre="uniform", lo=-10.0, hi=10.0, sigma=1.0,
               clip=None, integer=False),
    "c2": dict(n=1_000_000, d=128, comps=10_000, centre="uniform", lo=0.0, hi=255.0, sigma=20.0,
               clip=(0.0, 255.0), integer=True),
    "c3": dict(n=10_000_000, d=512, comps=1_000_000, centre="normal", lo=0.0, hi=1.0, sigma=0.5,
               clip=None, integer=False),
}


def mixture(n, d, comps, seed, centre="uniform", lo=-10.0, hi=10.0, sigma=1.0, clip=None,
            integer=False, return_components=False):
    rs = np.random.Generator(np.random.PCG64(seed))
    if centre == "uniform":
        centres = rs.uniform(lo, hi, size=(comps, d))
    else:
        centres = rs.standard_normal(size=(comps, d))
    comp = rs.integers(0, comps, size=n)
    X = np.empty((n, d), np.float32)
    step = 1 << 16
    for s in range(0, n, step):
        e = min(n, s + step)
        blk = centres[comp[s:e]] + sigma * rs.standard_normal(size=(e - s, d))
        if clip is not None:
            np.clip(blk, clip[0], clip[1], out=blk)
        if integer:
            blk = np.rint(blk)
        X[s:e] = blk.astype(np.float32)
    if return_components:
        return X, comp
    return X


def config_data(name, seed=1234, n=None):
    c = dict(CONFIGS[name])
    if n is not None:
        c["n"] = n
    return mixture(c["n"], c["d"], c["comps"], seed, c["centre"], c["lo"], c["hi"], c["sigma"],
                   c["clip"], c["integer"])


def mixture_device(n, d, comps, seed, centre="uniform", lo=-10.0, hi=10.0, sigma=1.0, clip=None,
                   integer=False, device="cuda"):
    """Same recipe drawn with torch on ``device`` (for 10^7-row inputs)."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    if centre == "uniform":
        centres = torch.rand((comps, d), generator=g, device=device) * (hi - lo) + lo
    else:
        centres = torch.randn((comps, d), generator=g, device=device)
    comp = torch.randint(0, comps, (n,), generator=g, device=device)
    X = torch.empty((n, d), dtype=torch.float32, device=device)
    step = 1 << 20
    for s in range(0, n, step):
        e = min(n, s + step)
        blk = centres[comp[s:e]] + sigma * torch.randn((e - s, d), generator=g, device=device)
        if clip is not None:
            blk.clamp_(clip[0], clip[1])
        if integer:
            blk = torch.round(blk)
        X[s:e] = blk
    return X


def lowrank(n, d, seed, r=16, comps=100, spread=2.0, scale=20.0, offset=100.0, noise=4.0,
            clip=(0.0, 255.0), integer=True):
    rs = np.random.Generator(np.random.PCG64(seed))
    W = rs.standard_normal(size=(r, d)) * (scale / np.sqrt(r))
    means = spread * rs.standard_normal(size=(comps, r))
    comp = rs.integers(0, comps, size=n)
    X = np.empty((n, d), np.float32)
    step = 1 << 16
    for s in range(0, n, step):
        e = min(n, s + step)
        z = means[comp[s:e]] + rs.standard_normal(size=(e - s, r))
        blk = offset + z @ W + noise * rs.standard_normal(size=(e - s, d))
        if clip is not None:
            np.clip(blk, clip[0], clip[1], out=blk)
        if integer:
            blk = np.rint(blk)
        X[s:e] = blk.astype(np.float32)
    return X


def integer_grid(n, d, seed, hi=255):
    rs = np.random.Generator(np.random.PCG64(seed))
    return rs.integers(0, hi + 1, size=(n, d)).astype(np.float32)


def instance_sizes(m, seed, lo=64, hi=4096):
    """Sizes of m independent small clustering jobs, n ~ U[lo, hi]."""
    rs = np.random.Generator(np.random.PCG64(seed))
    return rs.integers(lo, hi + 1, size=m)


def batch_mixture_device(sizes, d, comps, seed, lo=-10.0, hi=10.0, sigma=1.0, device="cuda"):
    """Independent mixtures, one per job, concatenated: job q has sizes[q] rows
    from comps[q] equal-weight components with centres U[lo, hi]^d and noise
    sigma (drawn with torch on ``device`` in one pass)."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    sizes_t = torch.as_tensor(np.asarray(sizes, np.int64), device=device)
    comps_t = torch.as_tensor(np.asarray(comps, np.int64), device=device)
    c_off = torch.cumsum(comps_t, 0) - comps_t
    centres = torch.rand((int(comps_t.sum()), d), generator=g, device=device) * (hi - lo) + lo
    job = torch.repeat_interleave(torch.arange(len(sizes), device=device), sizes_t)
    u = torch.rand(job.shape[0], generator=g, device=device, dtype=torch.float64)
    comp = c_off[job] + (u * comps_t[job]).long().minimum(comps_t[job] - 1)
    X = torch.empty((job.shape[0], d), dtype=torch.float32, device=device)
    step = 1 << 20
    for s in range(0, X.shape[0], step):
        e = min(X.shape[0], s + step)
        X[s:e] = centres[comp[s:e]] + sigma * torch.randn((e - s, d), generator=g, device=device)
    return X


def serving_stream(rate, seconds, seed, n_lo=1e3, n_hi=1e6, dims=(64, 128, 256)):
    """Poisson arrivals: (arrival time s, n, d) with n = round(10^U[log10 n_lo,
    log10 n_hi]) and d uniform over ``dims``."""
    rs = np.random.Generator(np.random.PCG64(seed))
    t, out = 0.0, []
    while True:
        t += rs.exponential(1.0 / rate)
        if t >= seconds:
            return out
        n = int(round(10 ** rs.uniform(np.log10(n_lo), np.log10(n_hi))))
        out.append((t, n, int(rs.choice(dims))))
