"""GPU test of pba_solve_dense_noalloc, the Cholesky solve that allocates
nothing (callers that cannot allocate): through the C ABI, on device buffers
the test allocates with the HIP runtime the library itself links, its result
must equal that of pba_solve_reduced's Cholesky path on the same reduced
system, on two calls in a row (the second with a smaller system), and a size
above the documented maximum is rejected before any device work."""
import ctypes as C

import numpy as np
import pytest

import scenes

pytestmark = pytest.mark.gpu

pba = pytest.importorskip("paper_1704_06967_amd.pba")

_hip = C.CDLL("libamdhip64.so.7")
_hip.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
_hip.hipFree.argtypes = [C.c_void_p]
_hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
_hip.hipDeviceSynchronize.argtypes = []
H2D, D2H = 1, 2


def _ok(e):
    assert e == 0, f"HIP error {e}"


class Dev:
    """A device copy of a numpy array (freed by close)."""

    def __init__(self, a):
        self.a = np.ascontiguousarray(a)
        self.p = C.c_void_p()
        _ok(_hip.hipMalloc(C.byref(self.p), max(self.a.nbytes, 8)))
        _ok(_hip.hipMemcpy(self.p, self.a.ctypes.data, self.a.nbytes, H2D))

    def get(self):
        out = np.empty_like(self.a)
        _ok(_hip.hipMemcpy(out.ctypes.data, self.p, out.nbytes, D2H))
        return out

    def close(self):
        _ok(_hip.hipFree(self.p))


def reduced_system(scene, precision=pba.PBA_FP64):
    """S, b of the first FC iteration at level 0 and pba_solve_reduced's Cholesky solution."""
    s = pba.Solver(mode=pba.PBA_FC, precision=precision, n_levels=1, pattern=scene.pattern, huber_k=scene.huber_k)
    s.set_scene(scene)
    s.iterate(0, 1)
    S, b = s.fetch(pba.PBA_DBG_S), s.fetch(pba.PBA_DBG_B)
    rep, x = s.solve_reduced(pba.PBA_SOLVER_CHOL)
    s.close()
    n = b.size
    return S.reshape(n, n), b, x


def solve_noalloc(S, b):
    n = b.size
    dS, db, dx = Dev(S), Dev(b), Dev(np.full(n, np.nan))
    dinfo = Dev(np.full(1, -7, np.int32))
    try:
        pba.check(pba.pba_solve_dense_noalloc(n, dS.p, db.p, dx.p, dinfo.p, None))
        _ok(_hip.hipDeviceSynchronize())
        return dx.get(), int(dinfo.get()[0])
    finally:
        for d in (dS, db, dx, dinfo):
            d.close()


def test_noalloc_solve_matches_reduced_solve():
    mid = scenes.mid(n_per_host=400, n_frames=30)       # 6F = 180
    tiny = scenes.tiny()                                  # 6F = 24
    S1, b1, x1 = reduced_system(mid)
    S2, b2, x2 = reduced_system(tiny)
    assert b1.size == 180 and b2.size == 24
    # two calls in a row, the second smaller: the scratch keeps the first call's
    # factor, which must not leak into the second
    y1, info1 = solve_noalloc(S1, b1)
    y2, info2 = solve_noalloc(S2, b2)
    assert info1 == 0 and info2 == 0
    # the same kernels on the same system: FP64 agreement to rounding
    for y, x, S, b in ((y1, x1, S1, b1), (y2, x2, S2, b2)):
        assert np.all(np.isfinite(y))
        np.testing.assert_allclose(y, x, rtol=0, atol=1e-12 * np.abs(x).max())
        res = np.linalg.norm(S @ y + b) / np.linalg.norm(b)
        assert res <= 1e-10, res


def test_noalloc_solve_after_larger_tiled_system():
    """A system above the short-chain size (n = 384: 12 tiles, separate panel
    and trailing-update launches), then the small one again."""
    rng = np.random.default_rng(5)
    n = 384
    A = rng.normal(size=(n, n))
    S = A @ A.T + n * np.eye(n)
    b = rng.normal(size=n)
    y, info = solve_noalloc(S, b)
    assert info == 0
    ref = -np.linalg.solve(S, b)
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-10 * np.abs(ref).max())
    tiny = scenes.tiny()
    S2, b2, x2 = reduced_system(tiny)
    y2, info2 = solve_noalloc(S2, b2)
    assert info2 == 0
    np.testing.assert_allclose(y2, x2, rtol=0, atol=1e-12 * np.abs(x2).max())


def test_noalloc_reports_indefinite_system():
    n = 64
    S = np.eye(n)
    S[10, 10] = -1.0
    y, info = solve_noalloc(S, np.ones(n))
    assert info == 1


def test_noalloc_rejects_sizes_beyond_the_maximum():
    st = pba.pba_solve_dense_noalloc(pba.PBA_NOALLOC_MAX_N + 1, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), None,
                                     None)
    assert st == pba.PBA_E_INVALID
    assert "768" in pba.last_error()
