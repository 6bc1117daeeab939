"""ctypes binding of libknnkm.so (the C ABI in include/knnkm.h).

Argument marshalling only: tensors are checked for device, dtype and layout and
their device pointers are passed through; every computation runs in the HIP
library.  Loading fails loudly when the library has not been built.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libknnkm.so")

OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, EAGAIN = 0, 1, 2, 3, 4, 5
FP32, BF16_RERANK = 0, 1
INIT_TWOMEANS, INIT_RANDOM, INIT_LABELS = 0, 1, 2
ROUND_FIT = 0xFFFF
MAX_D, MAX_KAPPA = 512, 128

# Entry points declared in include/knnkm.h (checked against the header by the tests).
EXPORTS = [
    "knnkm_create", "knnkm_destroy", "knnkm_set_stream", "knnkm_last_error",
    "knnkm_default_params", "knnkm_workspace_bytes", "knnkm_workspace_estimate", "knn_assign", "centroid_update",
    "distortion", "knnkm_twomeans", "knnkm_graph_init", "knnkm_graph_refine", "knn_build",
    "knn_kmeans_fit", "knn_boost_fit", "knn_graph_search", "distortion_noalloc", "knnkm_rng_draw", "knnkm_enable_timing", "knnkm_phase_times", "knnkm_sweep_stats",
    "knnkm_fit_batched", "knnkm_enable_graphs", "knnkm_enable_active_sets", "knnkm_enable_subtree_finish",
    "knnkm_autotune", "knnkm_autotune_table", "knnkm_set_assign_shape", "knnkm_enable_partial_distances",
    "knnkm_server_create", "knnkm_server_submit", "knnkm_server_wait",
    "knnkm_server_stats_get", "knnkm_server_last_error", "knnkm_server_destroy",
]


class Params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("kappa", ctypes.c_int32),
        ("xi", ctypes.c_int32),
        ("tau", ctypes.c_int32),
        ("bisect_iters", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("init", ctypes.c_int32),
        ("max_iters", ctypes.c_int32),
        ("early_stop", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
    ]


class ServerConfig(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("device", ctypes.c_int32),
        ("slots", ctypes.c_int32),
        ("max_batch_jobs", ctypes.c_int32),
        ("max_batch_rows", ctypes.c_int64),
        ("hbm_budget_bytes", ctypes.c_int64),
    ]


class Job(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("d", ctypes.c_int32),
        ("n", ctypes.c_int64),
        ("ldx", ctypes.c_int64),
        ("X_host", ctypes.c_void_p),
        ("k", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("params", Params),
        ("labels_host", ctypes.c_void_p),
        ("C_host", ctypes.c_void_p),
        ("counts_host", ctypes.c_void_p),
        ("G_ids_host", ctypes.c_void_p),
        ("trace_host", ctypes.c_void_p),
    ]


class JobInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("slot", ctypes.c_int32),
        ("batch", ctypes.c_int64),
        ("batch_jobs", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("footprint_bytes", ctypes.c_int64),
        ("t_submit", ctypes.c_double),
        ("t_admit", ctypes.c_double),
        ("t_done", ctypes.c_double),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in (
        "submitted", "completed", "failed", "rejected", "batches", "queued", "running", "max_queued",
        "max_batch_jobs_seen", "bytes_in_use", "bytes_peak", "ws_overruns")]


class KnnkmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"knnkm status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime under the same soname; load it first so
        # the library binds to the runtime that owns the caller's streams/memory.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1705_01813_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        sig = {
            "knnkm_create": [ctypes.c_int, P, ctypes.POINTER(P)],
            "knnkm_destroy": [P],
            "knnkm_set_stream": [P, P],
            "knnkm_default_params": [ctypes.POINTER(Params)],
            "knnkm_workspace_bytes": [P, ctypes.POINTER(i64)],
            "knnkm_workspace_estimate": [i64, i32, i32, ctypes.POINTER(Params), ctypes.POINTER(i64)],
            "knn_assign": [P, P, i64, i32, i64, P, i32, P, i32, P, P, P, P],
            "centroid_update": [P, P, i64, i32, i64, P, i32, P, P, P],
            "distortion": [P, P, i64, i32, i64, P, i32, P, P],
            "distortion_noalloc": [P, P, i64, i32, i64, P, i32, P, P],
            "knnkm_twomeans": [P, P, i64, i32, i64, i32, u64, i32, i32, P],
            "knnkm_graph_init": [P, P, i64, i32, i64, i32, u64, P, P],
            "knnkm_graph_refine": [P, P, i64, i32, i64, P, i32, i32, P, P, i32],
            "knn_build": [P, P, i64, i32, i64, ctypes.POINTER(Params), P, P],
            "knn_kmeans_fit": [P, P, i64, i32, i64, i32, P, ctypes.POINTER(Params), P, P, P, P, P],
            "knn_boost_fit": [P, P, i64, i32, i64, i32, P, ctypes.POINTER(Params), P, P, P, P, P],
            "knn_graph_search": [P, P, i64, i32, i64, P, i32, P, i64, i64, i32, i32, i32, i32, u64, P, P],
            "knnkm_rng_draw": [P, u64, u64, u64, i64, P],
            "knnkm_fit_batched": [P, P, i32, i64, i32, P, P, P, ctypes.POINTER(Params), P, P, P, P, P, P],
            "knnkm_enable_timing": [P, i32],
            "knnkm_enable_graphs": [P, i32],
            "knnkm_enable_active_sets": [P, i32],
            "knnkm_enable_subtree_finish": [P, i32],
            "knnkm_autotune": [P, i32],
            "knnkm_enable_partial_distances": [P, i32],
            "knnkm_set_assign_shape": [P, i32, i32, i32],
            "knnkm_autotune_table": [P, i64, ctypes.POINTER(i64)],
            "knnkm_phase_times": [P, P, i32],
            "knnkm_sweep_stats": [P, P, P, P, P, i32, P],
            "knnkm_server_create": [ctypes.POINTER(ServerConfig), ctypes.POINTER(P)],
            "knnkm_server_submit": [P, ctypes.POINTER(Job), ctypes.POINTER(u64)],
            "knnkm_server_wait": [P, u64, i64, ctypes.POINTER(JobInfo)],
            "knnkm_server_stats_get": [P, ctypes.POINTER(ServerStats)],
            "knnkm_server_destroy": [P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.knnkm_last_error.argtypes = [P]
        L.knnkm_last_error.restype = ctypes.c_char_p
        L.knnkm_server_last_error.argtypes = []
        L.knnkm_server_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def default_params(**kw):
    p = Params()
    _chk(None, lib().knnkm_default_params(ctypes.byref(p)))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


def _chk(ctx, st):
    if st != OK:
        raise KnnkmError(st, lib().knnkm_last_error(ctx).decode())


def _ptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    import torch

    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def _rows(X):
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be a 2-D row-major tensor")
    return X.shape[0], X.shape[1], X.stride(0)


class Context:
    """A library context on one device, launching on a torch stream."""

    def __init__(self, device=0, stream=None, dry=False):
        self._h = ctypes.c_void_p()
        if dry:
            _chk(None, lib().knnkm_create(-1, None, ctypes.byref(self._h)))
            self.device = -1
            return
        import torch

        self.device = device
        s = stream if stream is not None else torch.cuda.current_stream(device)
        _chk(None, lib().knnkm_create(device, ctypes.c_void_p(s.cuda_stream), ctypes.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def set_stream(self, stream):
        _chk(self._h, lib().knnkm_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)))

    def workspace_bytes(self):
        v = ctypes.c_int64()
        _chk(self._h, lib().knnkm_workspace_bytes(self._h, ctypes.byref(v)))
        return v.value

    def close(self):
        if self._h:
            lib().knnkm_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def knn_assign(ctx, X, C, G_ids, labels_in, labels_out, best_d2=None, n_moved=None, kappa=None):
    import torch

    n, d, ldx = _rows(X)
    k = C.shape[0]
    kap = kappa if kappa is not None else G_ids.shape[1]
    st = lib().knn_assign(ctx.handle, _ptr(X, torch.float32, "X"), n, d, ldx, _ptr(C, torch.float32, "C"), k,
                          _ptr(G_ids, torch.int32, "G_ids"), kap, _ptr(labels_in, torch.int32, "labels_in"),
                          _ptr(labels_out, torch.int32, "labels_out"), _ptr(best_d2, torch.float32, "best_d2"),
                          _ptr(n_moved, torch.int64, "n_moved"))
    _chk(ctx.handle, st)


def centroid_update(ctx, X, labels, C, counts, sums=None):
    import torch

    n, d, ldx = _rows(X)
    st = lib().centroid_update(ctx.handle, _ptr(X, torch.float32, "X"), n, d, ldx,
                               _ptr(labels, torch.int32, "labels"), C.shape[0], _ptr(C, torch.float32, "C"),
                               _ptr(counts, torch.int32, "counts"), _ptr(sums, torch.float64, "sums"))
    _chk(ctx.handle, st)


def distortion(ctx, X, C, labels, E):
    import torch

    n, d, ldx = _rows(X)
    st = lib().distortion(ctx.handle, _ptr(X, torch.float32, "X"), n, d, ldx, _ptr(C, torch.float32, "C"),
                          C.shape[0], _ptr(labels, torch.int32, "labels"), _ptr(E, torch.float64, "E"))
    _chk(ctx.handle, st)


def distortion_noalloc(ctx, X, C, labels, E):
    """Allocation-free variant of distortion (fixed library scratch)."""
    import torch

    n, d, ldx = _rows(X)
    st = lib().distortion_noalloc(ctx.handle, _ptr(X, torch.float32, "X"), n, d, ldx, _ptr(C, torch.float32, "C"),
                                  C.shape[0], _ptr(labels, torch.int32, "labels"), _ptr(E, torch.float64, "E"))
    _chk(ctx.handle, st)


def knnkm_twomeans(ctx, X, k, seed, round_tag, bisect_iters, labels):
    import torch

    n, d, ldx = _rows(X)
    st = lib().knnkm_twomeans(ctx.handle, _ptr(X, torch.float32, "X"), n, d, ldx, k, seed, round_tag,
                              bisect_iters, _ptr(labels, torch.int32, "labels"))
    _chk(ctx.handle, st)


def knnkm_graph_init(ctx, X, kappa, seed, G_ids, G_d2):
    import torch

    n, d, ldx = _rows(X)
    st = lib().knnkm_graph_init(ctx.handle, _ptr(X, torch.float32, "X"), n, d, ldx, kappa, seed,
                                _ptr(G_ids, torch.int32, "G_ids"), _ptr(G_d2, torch.float32, "G_d2"))
    _chk(ctx.handle, st)


def knnkm_graph_refine(ctx, X, labels, k, precision, G_ids, G_d2):
    import torch

    n, d, ldx = _rows(X)
    st = lib().knnkm_graph_refine(ctx.handle, _ptr(X, torch.float32, "X"), n, d, ldx,
                                  _ptr(labels, torch.int32, "labels"), k, precision,
                                  _ptr(G_ids, torch.int32, "G_ids"), _ptr(G_d2, torch.float32, "G_d2"),
                                  G_ids.shape[1])
    _chk(ctx.handle, st)


def knn_build(ctx, X, params, G_ids, G_d2):
    import torch

    n, d, ldx = _rows(X)
    st = lib().knn_build(ctx.handle, _ptr(X, torch.float32, "X"), n, d, ldx, ctypes.byref(params),
                         _ptr(G_ids, torch.int32, "G_ids"), _ptr(G_d2, torch.float32, "G_d2"))
    _chk(ctx.handle, st)


def knnkm_workspace_estimate(n, d, k, params):
    """Planning estimate of the workspace of knn_build + knn_kmeans_fit (bytes)."""
    v = ctypes.c_int64()
    st = lib().knnkm_workspace_estimate(n, d, k, ctypes.byref(params), ctypes.byref(v))
    if st != OK:
        raise KnnkmError(st, "knnkm_workspace_estimate: invalid arguments")
    return v.value


def knn_kmeans_fit(ctx, X, k, G_ids, params, labels, C, counts):
    """Returns (trace of E_0..E_T as numpy, iterations run)."""
    import torch

    n, d, ldx = _rows(X)
    trace = np.zeros(params.max_iters + 1, np.float64)
    it = ctypes.c_int32()
    st = lib().knn_kmeans_fit(ctx.handle, _ptr(X, torch.float32, "X"), n, d, ldx, k,
                              _ptr(G_ids, torch.int32, "G_ids"), ctypes.byref(params),
                              _ptr(labels, torch.int32, "labels"), _ptr(C, torch.float32, "C"),
                              _ptr(counts, torch.int32, "counts"),
                              trace.ctypes.data_as(ctypes.c_void_p), ctypes.byref(it))
    _chk(ctx.handle, st)
    return trace[: it.value + 1], it.value


def knn_boost_fit(ctx, X, k, G_ids, params, labels, C, counts):
    """Boost form.  Returns (trace of E_0..E_t as numpy, rounds run)."""
    import torch

    n, d, ldx = _rows(X)
    trace = np.zeros(params.max_iters + 1, np.float64)
    it = ctypes.c_int32()
    st = lib().knn_boost_fit(ctx.handle, _ptr(X, torch.float32, "X"), n, d, ldx, k,
                             _ptr(G_ids, torch.int32, "G_ids"), ctypes.byref(params),
                             _ptr(labels, torch.int32, "labels"), _ptr(C, torch.float32, "C"),
                             _ptr(counts, torch.int32, "counts"),
                             trace.ctypes.data_as(ctypes.c_void_p), ctypes.byref(it))
    _chk(ctx.handle, st)
    return trace[: it.value + 1], it.value


def knn_graph_search(ctx, X, G_ids, Q, ef, top_k, out_ids, out_d2, max_visits=1920, n_entry=1, seed=0):
    """Best-first search over the graph for the rows of Q (device tensors)."""
    import torch

    n, d, ldx = _rows(X)
    m, dq, ldq = _rows(Q)
    if dq != d:
        raise ValueError("knn_graph_search: Q and X differ in d")
    st = lib().knn_graph_search(ctx.handle, _ptr(X, torch.float32, "X"), n, d, ldx, _ptr(G_ids, torch.int32, "G_ids"),
                                int(G_ids.shape[1]), _ptr(Q, torch.float32, "Q"), m, ldq, ef, top_k, max_visits,
                                n_entry, ctypes.c_uint64(seed), _ptr(out_ids, torch.int32, "out_ids"),
                                _ptr(out_d2, torch.float32, "out_d2"))
    _chk(ctx.handle, st)


def knnkm_fit_batched(ctx, X, n_off, ks, seeds, params, G_ids, G_d2, labels, C, counts):
    """Batching form.  n_off: m+1 row offsets, ks: m cluster counts, seeds: m
    seeds (host sequences).  Returns the traces as an m x (max_iters+1) array."""
    import torch

    n, d, ldx = _rows(X)
    m = len(ks)
    noff = np.ascontiguousarray(n_off, dtype=np.int64)
    karr = np.ascontiguousarray(ks, dtype=np.int32)
    sarr = np.ascontiguousarray(seeds, dtype=np.uint64)
    if noff.shape != (m + 1,) or sarr.shape != (m,) or int(noff[-1]) != n:
        raise ValueError("job tables do not match X")
    trace = np.zeros((m, params.max_iters + 1), np.float64)
    st = lib().knnkm_fit_batched(ctx.handle, _ptr(X, torch.float32, "X"), d, ldx, m,
                                 noff.ctypes.data_as(ctypes.c_void_p), karr.ctypes.data_as(ctypes.c_void_p),
                                 sarr.ctypes.data_as(ctypes.c_void_p), ctypes.byref(params),
                                 _ptr(G_ids, torch.int32, "G_ids"), _ptr(G_d2, torch.float32, "G_d2"),
                                 _ptr(labels, torch.int32, "labels"), _ptr(C, torch.float32, "C"),
                                 _ptr(counts, torch.int32, "counts"), trace.ctypes.data_as(ctypes.c_void_p))
    _chk(ctx.handle, st)
    return trace


def knnkm_enable_graphs(ctx, on=True):
    _chk(ctx.handle, lib().knnkm_enable_graphs(ctx.handle, 1 if on else 0))


def knnkm_enable_active_sets(ctx, on=True):
    _chk(ctx.handle, lib().knnkm_enable_active_sets(ctx.handle, 1 if on else 0))


def knnkm_enable_subtree_finish(ctx, on=True):
    """on: False/0 off, True/1 on (subtree roots up to 1,024 members), or the root size limit."""
    _chk(ctx.handle, lib().knnkm_enable_subtree_finish(ctx.handle, int(on)))


def knnkm_enable_partial_distances(ctx, on=True):
    """on: False/0 off, True/1 on (bfloat16 centroid shadow in the build and
    fit sweeps), 2 on with float32 centroids only."""
    _chk(ctx.handle, lib().knnkm_enable_partial_distances(ctx.handle, int(on)))


def knnkm_autotune(ctx, on=True):
    _chk(ctx.handle, lib().knnkm_autotune(ctx.handle, 1 if on else 0))


def knnkm_set_assign_shape(ctx, gs=0, pb=64, lazy=0):
    """Fix the assignment's launch shape (gs = 0: automatic)."""
    _chk(ctx.handle, lib().knnkm_set_assign_shape(ctx.handle, int(gs), int(pb), int(lazy)))


def knnkm_autotune_table():
    """The tuned launch shapes of this process, one line per entry."""
    need = ctypes.c_int64()
    _chk(None, lib().knnkm_autotune_table(None, 0, ctypes.byref(need)))
    buf = ctypes.create_string_buffer(max(1, need.value))
    _chk(None, lib().knnkm_autotune_table(buf, need.value, ctypes.byref(need)))
    return buf.value.decode()


def knnkm_enable_timing(ctx, on=True):
    """on: False/0 off, True/1 phases, 2 phases and every fit assignment."""
    _chk(ctx.handle, lib().knnkm_enable_timing(ctx.handle, int(on)))


PHASES = ("build_ms", "fit_init_ms", "fit_iters_ms", "assign_ms", "iters", "assign_launches", "assign_evaluated",
          "assign_listed")


def knnkm_phase_times(ctx):
    out = np.zeros(len(PHASES), np.float64)
    _chk(ctx.handle, lib().knnkm_phase_times(ctx.handle, out.ctypes.data_as(ctypes.c_void_p), len(PHASES)))
    return dict(zip(PHASES, out.tolist()))


def knnkm_sweep_stats(ctx, max_sweeps=1024):
    """Per-sweep record of the last fit: assignment ms, listed, evaluated and
    moved samples (lists; -1 where not recorded)."""
    ms = np.zeros(max_sweeps, np.float64)
    cnt = [np.zeros(max_sweeps, np.int64) for _ in range(3)]
    n_out = ctypes.c_int32(0)
    st = lib().knnkm_sweep_stats(ctx.handle, ms.ctypes.data_as(ctypes.c_void_p),
                                 *[c.ctypes.data_as(ctypes.c_void_p) for c in cnt], max_sweeps,
                                 ctypes.byref(n_out))
    _chk(ctx.handle, st)
    k = n_out.value
    return {"assign_ms": ms[:k].tolist(), "listed": cnt[0][:k].tolist(), "evaluated": cnt[1][:k].tolist(),
            "moved": cnt[2][:k].tolist()}


def knnkm_rng_draw(ctx, seed, stream, ctr0, out):
    import torch

    st = lib().knnkm_rng_draw(ctx.handle, seed, stream, ctr0, out.numel(), _ptr(out, torch.uint64, "out"))
    _chk(ctx.handle, st)


# ------------------------------------------------------------- serving form --
def _server_chk(st):
    if st != OK:
        raise KnnkmError(st, lib().knnkm_server_last_error().decode())


def _host_rows(X):
    """(pointer, n, d, ldx) of a host float32 matrix with unit column stride."""
    try:
        import torch
    except ImportError:  # pragma: no cover
        torch = None
    if torch is not None and isinstance(X, torch.Tensor):
        if X.is_cuda or X.dtype != torch.float32 or X.dim() != 2 or X.stride(1) != 1:
            raise ValueError("X must be a 2-D float32 host tensor with unit column stride")
        return X.data_ptr(), X.shape[0], X.shape[1], X.stride(0)
    X = np.asarray(X)
    if X.dtype != np.float32 or X.ndim != 2 or X.strides[1] != 4 or X.strides[0] % 4:
        raise ValueError("X must be a 2-D float32 array with unit column stride")
    return X.ctypes.data, X.shape[0], X.shape[1], X.strides[0] // 4


class Server:
    """Request loop of the library (knnkm_server_*).  submit() queues a job and
    returns its ticket; wait() returns its result.  The host rows and the
    result arrays of a job are kept alive here until it has been waited for."""

    def __init__(self, device=0, slots=4, max_batch_jobs=4096, max_batch_rows=1 << 24,
                 hbm_budget_bytes=200 * 10**9):
        cfg = ServerConfig(ctypes.sizeof(ServerConfig), device, slots, max_batch_jobs, max_batch_rows,
                           int(hbm_budget_bytes))
        self._h = ctypes.c_void_p()
        _server_chk(lib().knnkm_server_create(ctypes.byref(cfg), ctypes.byref(self._h)))
        self._live = {}

    def submit(self, X, k, params, want_graph=False):
        ptr, n, d, ldx = _host_rows(X)
        out = {
            "labels": np.empty(n, np.int32),
            "C": np.empty((k, d), np.float32),
            "counts": np.empty(k, np.int32),
            "trace": np.empty(params.max_iters + 1, np.float64),
            "G_ids": np.empty((n, params.kappa), np.int32) if want_graph else None,
        }

        def p(a):
            return None if a is None else a.ctypes.data

        job = Job(ctypes.sizeof(Job), d, n, ldx, ptr, k, 0, params, p(out["labels"]), p(out["C"]),
                  p(out["counts"]), p(out["G_ids"]), p(out["trace"]))
        t = ctypes.c_uint64()
        _server_chk(lib().knnkm_server_submit(self._h, ctypes.byref(job), ctypes.byref(t)))
        self._live[t.value] = (X, out)
        return t.value

    def wait(self, ticket, timeout_ms=-1):
        """The job's outputs and timing, or None if it has not finished within
        timeout_ms.  Raises KnnkmError if the job failed."""
        info = JobInfo()
        st = lib().knnkm_server_wait(self._h, ticket, timeout_ms, ctypes.byref(info))
        if st == EAGAIN:
            return None
        held = self._live.pop(ticket, None)
        _server_chk(st)
        out = held[1]
        out["info"] = {f: getattr(info, f) for f, _ in JobInfo._fields_ if f != "pad_"}
        return out

    def stats(self):
        s = ServerStats()
        _server_chk(lib().knnkm_server_stats_get(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self._h:
            lib().knnkm_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
