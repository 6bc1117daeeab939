"""The allocation-free distortion entry point (fixed library scratch) against
the existing distortion entry point, through the C ABI: the same bits on two
calls in a row (the second on a smaller input, so stale scratch contents
from the first would show), the oracle's Eqn. 4 value within 1e-12, and a
size beyond the fixed scratch rejected before any launch."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import gkmeans  # noqa: E402
from paper_1705_01813_amd import datagen, knnkm  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = knnkm.Context(0)
    yield c
    c.close()


def _case(n, d, k, seed):
    X = datagen.mixture(n, d, k, seed=seed)
    rs = np.random.default_rng(seed)
    labels = rs.integers(0, k, n).astype(np.int32)
    C = (X[rs.choice(n, k, replace=False)] + 0.5).astype(np.float32)
    return X, C, labels


def test_distortion_noalloc_equals_distortion(ctx):
    # 17,000,000 rows need more than 65,536 partial blocks (the tile path);
    # the second call is far smaller
    for n, d, k, seed in [(17_000_000, 8, 300, 1), (300_001, 130, 900, 2), (5_000, 40, 70, 3)]:
        print("[case] distortion_noalloc", n, d, k, flush=True)
        X, C, labels = _case(n, d, k, seed)
        Xd = torch.from_numpy(X).to(DEV)
        Cd = torch.from_numpy(C).to(DEV)
        ld = torch.from_numpy(labels).to(DEV)
        e_ref = torch.zeros(1, dtype=torch.float64, device=DEV)
        e_na = torch.full((1,), -1.0, dtype=torch.float64, device=DEV)
        knnkm.distortion(ctx, Xd, Cd, ld, e_ref)
        knnkm.distortion_noalloc(ctx, Xd, Cd, ld, e_na)
        torch.cuda.synchronize()
        got, ref = float(e_na.cpu()[0]), float(e_ref.cpu()[0])
        assert got == ref, (n, got, ref)
        if n <= 400_000:
            want = gkmeans.distortion(X, C, labels)
            assert abs(got - want) <= 1e-12 * want


def test_distortion_noalloc_rejects_beyond_scratch(ctx):
    X = torch.zeros((4, 4), dtype=torch.float32, device=DEV)
    C = torch.zeros((2, 4), dtype=torch.float32, device=DEV)
    lab = torch.zeros(4, dtype=torch.int32, device=DEV)
    E = torch.zeros(1, dtype=torch.float64, device=DEV)
    P = ctypes.c_void_p
    st = knnkm.lib().distortion_noalloc(ctx.handle, P(X.data_ptr()), 200_000_000, 4, 4, P(C.data_ptr()), 2,
                                        P(lab.data_ptr()), P(E.data_ptr()))
    assert st == knnkm.EUNSUPPORTED
    assert "scratch" in knnkm.lib().knnkm_last_error(ctx.handle).decode()
