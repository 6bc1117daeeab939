"""C ABI checks that need no GPU: the library loads, exports every function the
header declares, and rejects invalid arguments before any launch (dry
context, device = -1)."""
import ctypes
import os
import re

import pytest

from paper_1705_01813_amd import knnkm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "knnkm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:knnkm_status|const char\*)\s+(\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_header_function():
    names = _header_functions()
    assert len(names) >= 15
    L = knnkm.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(knnkm.EXPORTS) == names


def test_default_params_match_paper_defaults():
    p = knnkm.default_params()
    assert p.struct_size == ctypes.sizeof(knnkm.Params)
    assert (p.kappa, p.xi, p.tau) == (50, 50, 10)  # Sec. 4.4
    assert p.max_iters == 30  # Sec. 5.4


@pytest.fixture
def dry():
    c = knnkm.Context(dry=True)
    yield c
    c.close()


def _call(fn, *args):
    return getattr(knnkm.lib(), fn)(*args)


def test_dry_context_validation(dry):
    h = dry.handle
    X = ctypes.c_void_p(0x1000)
    P = ctypes.c_void_p(0x2000)
    # knn_assign: k > n, bad kappa, null pointers, aliasing, d too large
    assert _call("knn_assign", h, X, 10, 4, 4, P, 11, P, 3, P, ctypes.c_void_p(0x3000), None, None) == knnkm.EINVAL
    assert _call("knn_assign", h, X, 10, 4, 4, P, 5, P, 0, P, ctypes.c_void_p(0x3000), None, None) == knnkm.EINVAL
    assert _call("knn_assign", h, X, 1000, 4, 4, P, 500, P, 129, P, ctypes.c_void_p(0x3000), None, None) == knnkm.EUNSUPPORTED
    assert _call("knn_assign", h, X, 10, 4, 3, P, 5, P, 3, P, ctypes.c_void_p(0x3000), None, None) == knnkm.EINVAL
    assert "ldx" in knnkm.lib().knnkm_last_error(h).decode()
    assert _call("knn_assign", h, None, 10, 4, 4, P, 5, P, 3, P, ctypes.c_void_p(0x3000), None, None) == knnkm.EINVAL
    assert _call("knn_assign", h, X, 10, 4, 4, P, 5, P, 3, P, P, None, None) == knnkm.EINVAL
    assert _call("knn_assign", h, X, 10, 600, 600, P, 5, P, 3, P, ctypes.c_void_p(0x3000), None, None) == knnkm.EUNSUPPORTED
    assert _call("knn_assign", h, X, 10, 4, 4, P, 5, P, 3, P, ctypes.c_void_p(0x3000), None, None) == knnkm.OK
    # kappa >= k: the graph may be null (exhaustive candidates)
    assert _call("knn_assign", h, X, 10, 4, 4, P, 3, None, 3, P, ctypes.c_void_p(0x3000), None, None) == knnkm.OK
    # centroid_update / distortion
    assert _call("centroid_update", h, X, 10, 4, 4, P, 0, P, P, None) == knnkm.EINVAL
    assert _call("centroid_update", h, X, 10, 4, 4, None, 3, P, P, None) == knnkm.EINVAL
    assert _call("distortion", h, X, 10, 4, 4, P, 3, P, None) == knnkm.EINVAL
    # twomeans
    assert _call("knnkm_twomeans", h, X, 10, 4, 4, 11, 0, 0, 2, P) == knnkm.EINVAL
    assert _call("knnkm_twomeans", h, X, 10, 4, 4, 3, 0, 0x10000, 2, P) == knnkm.EINVAL
    # graph
    assert _call("knnkm_graph_init", h, X, 10, 4, 4, 10, 0, P, P) == knnkm.EINVAL
    assert _call("knnkm_graph_init", h, X, 1000, 4, 4, 200, 0, P, P) == knnkm.EUNSUPPORTED
    assert _call("knnkm_graph_refine", h, X, 10, 4, 4, P, 3, 7, P, P, 3) == knnkm.EINVAL
    p = knnkm.default_params(kappa=5)
    assert _call("knn_build", h, X, 10, 4, 4, ctypes.byref(p), P, P) == knnkm.OK
    p.xi = 1
    assert _call("knn_build", h, X, 10, 4, 4, ctypes.byref(p), P, P) == knnkm.EINVAL
    p = knnkm.default_params(kappa=5)
    p.struct_size = 4
    assert _call("knn_build", h, X, 10, 4, 4, ctypes.byref(p), P, P) == knnkm.EINVAL
    p = knnkm.default_params(kappa=5, max_iters=3)
    assert _call("knn_kmeans_fit", h, X, 10, 4, 4, 3, P, ctypes.byref(p), P, P, P, None, None) == knnkm.OK
    assert _call("knn_kmeans_fit", h, X, 10, 4, 4, 3, None, ctypes.byref(p), P, P, P, None, None) == knnkm.OK
    p.kappa = 2
    assert _call("knn_kmeans_fit", h, X, 10, 4, 4, 3, None, ctypes.byref(p), P, P, P, None, None) == knnkm.EINVAL
    p.init = 9
    assert _call("knn_kmeans_fit", h, X, 10, 4, 4, 3, P, ctypes.byref(p), P, P, P, None, None) == knnkm.EINVAL
    assert "init" in knnkm.lib().knnkm_last_error(h).decode()
    # null context
    assert _call("knn_assign", None, X, 10, 4, 4, P, 5, P, 3, P, ctypes.c_void_p(0x3000), None, None) == knnkm.EINVAL


def test_batched_validation(dry):
    h = dry.handle
    X = ctypes.c_void_p(0x1000)
    P = ctypes.c_void_p(0x2000)
    p = knnkm.default_params(kappa=8)

    def call(noff, ks, seeds, m=None):
        m = len(ks) if m is None else m
        a = (ctypes.c_int64 * len(noff))(*noff)
        b = (ctypes.c_int32 * len(ks))(*ks)
        c = (ctypes.c_uint64 * len(seeds))(*seeds)
        return knnkm.lib().knnkm_fit_batched(h, X, 16, 16, m, a, b, c, ctypes.byref(p), P, P, P, P, P, None)

    assert call([0, 64, 200], [2, 5], [1, 2]) == knnkm.OK
    assert call([0, 64, 200], [2, 5], [1, 2], m=0) == knnkm.EINVAL
    assert call([1, 64, 200], [2, 5], [1, 2]) == knnkm.EINVAL      # n_off[0] != 0
    assert call([0, 5, 200], [2, 5], [1, 2]) == knnkm.EINVAL       # job with fewer than kappa+1 rows
    assert call([0, 64, 200], [65, 5], [1, 2]) == knnkm.EINVAL     # k > n
    assert call([0, 64, 200], [0, 5], [1, 2]) == knnkm.EINVAL      # k < 1
    p.init = knnkm.INIT_LABELS                                      # resume is knn_kmeans_fit only
    assert call([0, 64, 200], [2, 5], [1, 2]) == knnkm.EINVAL
    assert "knn_kmeans_fit only" in knnkm.lib().knnkm_last_error(h).decode()
    p.init = 3
    assert call([0, 64, 200], [2, 5], [1, 2]) == knnkm.EINVAL


def test_assign_shape_validation(dry):
    h = dry.handle
    for gs, pb, lazy in [(1, 64, 0), (2, 128, 0), (4, 64, 0), (4, 128, 0), (1, 64, 1), (2, 128, 1), (0, 0, 0)]:
        assert _call("knnkm_set_assign_shape", h, gs, pb, lazy) == knnkm.OK, (gs, pb, lazy)
    for gs, pb, lazy in [(8, 64, 0), (3, 64, 0), (2, 96, 0), (-1, 64, 0), (4, 64, 1), (1, 64, 2)]:
        assert _call("knnkm_set_assign_shape", h, gs, pb, lazy) == knnkm.EINVAL, (gs, pb, lazy)


def test_subtree_finish_validation(dry):
    h = dry.handle
    for on in (0, 1, 2, 256, 1024):
        assert _call("knnkm_enable_subtree_finish", h, on) == knnkm.OK, on
    for on in (-1, 1025, 4096):
        assert _call("knnkm_enable_subtree_finish", h, on) == knnkm.EINVAL, on
    assert _call("knnkm_enable_subtree_finish", h, 1) == knnkm.OK


def test_workspace_estimate_validation():
    p = knnkm.default_params(kappa=10)
    a = knnkm.knnkm_workspace_estimate(10_000, 32, 100, p)
    b = knnkm.knnkm_workspace_estimate(1_000_000, 32, 100, p)
    c = knnkm.knnkm_workspace_estimate(1_000_000, 512, 100, p)
    assert 0 < a < b < c
    for n, d, k in [(0, 32, 1), (100, 0, 1), (100, 32, 0), (100, 32, 101)]:
        with pytest.raises(knnkm.KnnkmError) as e:
            knnkm.knnkm_workspace_estimate(n, d, k, p)
        assert e.value.status == knnkm.EINVAL


def test_graph_search_validation(dry):
    h = dry.handle
    X = ctypes.c_void_p(0x1000)
    P = ctypes.c_void_p(0x2000)
    O = ctypes.c_void_p(0x3000)

    def call(n=100, d=8, kappa=10, m=5, ef=16, top_k=10, visits=1920, n_entry=1, ldx=None):
        return knnkm.lib().knn_graph_search(h, X, n, d, d if ldx is None else ldx, P, kappa, X, m, d, ef, top_k,
                                            visits, n_entry, ctypes.c_uint64(0), O, O)

    assert call() == knnkm.OK
    assert call(m=0) == knnkm.OK
    assert call(visits=7680, ef=128, top_k=128, n_entry=16) == knnkm.OK
    for kw in [dict(visits=7681), dict(visits=0), dict(ef=129), dict(top_k=17), dict(top_k=0), dict(n_entry=17),
               dict(n_entry=0), dict(kappa=0), dict(ldx=7), dict(n=0), dict(m=-1)]:
        assert call(**kw) == knnkm.EINVAL, kw
    assert call(d=513) == knnkm.EUNSUPPORTED


def test_partial_distances_modes(dry):
    for on in (0, 1, 2, 3):
        assert _call("knnkm_enable_partial_distances", dry.handle, on) == knnkm.OK, on
    for on in (-1, 4):
        assert _call("knnkm_enable_partial_distances", dry.handle, on) == knnkm.EINVAL, on
    assert _call("knnkm_enable_partial_distances", dry.handle, 1) == knnkm.OK
