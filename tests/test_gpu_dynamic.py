"""GPU parity of the keyframe drop (pba_drop_frame; sliding window, dynamic
Hessian) against the oracle's GaussNewton.drop_frame: the dropped frame's
observations leave the window and, within an IC level, the reduced system is
formed again from the records kept at p(0) without a new linearization."""
import numpy as np
import pytest

import scenes
from oracle.gn import GaussNewton, Problem
from tests.oracle_refs import depth_errors_ok, rot_err, trans_rel_err

pytestmark = pytest.mark.gpu

pba = pytest.importorskip("paper_1704_06967_amd.pba")


@pytest.fixture(scope="module")
def mid_small():
    return scenes.mid(n_per_host=300)


def make(sc, mode, precision, **kw):
    s = pba.Solver(mode=pba.PBA_IC_PROXY if mode == "ic" else pba.PBA_FC, precision=precision,
                   n_levels=sc.n_levels, pattern=sc.pattern, huber_k=sc.huber_k, **kw)
    s.set_scene(sc)
    return s


@pytest.mark.parametrize("mode,f", [("ic", 6), ("ic", 13), ("fc", 12)])
def test_drop_mid_level_fp64_matches_oracle(mid_small, mode, f):
    """Two iterations of level 1, the drop, three more: every iteration's
    statistics, the reduced system after the drop (IC) and the iterates."""
    sc = mid_small
    s = make(sc, mode, pba.PBA_FP64)
    gn = GaussNewton(Problem.from_scene(sc), mode)
    s.iterate(2, 2)
    gn.iterate(2, 2)
    s.iterate(1, 2)
    gn.iterate(1, 2)
    s.drop_frame(f)
    gn.drop_frame(f)
    if mode == "ic":
        S = s.fetch(pba.PBA_DBG_S)
        np.testing.assert_allclose(S, gn.red.S, rtol=0, atol=1e-10 * np.abs(gn.red.S).max())
    st = s.iterate(1, 3)
    ost = gn.iterate(1, 3)
    # dropping host 6 leaves frames 4, 5, 7 and 8 without any observation and
    # frames 3 and 9 seen from one host only: the reduced system's conditioning
    # amplifies FP64 rounding more than on the full problem
    e_en = max(abs(a["energy"] / o["energy"] - 1) for a, o in zip(st, ost))
    e_disp = max(abs(a["max_disp_px"] - o["max_disp_px"]) for a, o in zip(st, ost))
    poses, d = s.get_params()
    e_rot, e_tr = rot_err(poses, gn.poses).max(), trans_rel_err(poses, gn.poses).max()
    e_d = np.abs(d / gn.d - 1).max()
    print(f"drop {mode} frame {f}: energy {e_en:.2e}, disp {e_disp:.2e}, rot {e_rot:.2e}, trans {e_tr:.2e}, "
          f"inv depth {e_d:.2e}")
    assert all(a["n_active"] == o["n_active"] for a, o in zip(st, ost))
    assert e_en <= 1e-8 and e_disp <= 1e-7
    assert e_rot <= 1e-8 and e_tr <= 1e-8 and e_d <= 1e-7
    ev, oev = s.evaluate(1), gn.evaluate(1)
    assert ev["n_active"] == oev["n_active"]
    assert abs(ev["energy"] / oev["energy"] - 1) <= 1e-8


@pytest.mark.parametrize("precision", [pba.PBA_FP32, pba.PBA_MIXED_BF16])
def test_drop_single_precision_within_bars(mid_small, precision):
    sc = mid_small
    s = make(sc, "ic", precision)
    gn = GaussNewton(Problem.from_scene(sc), "ic")
    s.iterate(2, 3)
    gn.iterate(2, 3)
    s.iterate(1, 1)
    gn.iterate(1, 1)
    s.drop_frame(18)
    gn.drop_frame(18)
    s.iterate(1, 3)
    gn.iterate(1, 3)
    s.iterate(0, 3)
    gn.iterate(0, 3)
    poses, d = s.get_params()
    assert rot_err(poses, gn.poses).max() <= 1e-5
    assert trans_rel_err(poses, gn.poses).max() <= 1e-5
    ok, q99, worst = depth_errors_ok(d, gn.d)
    assert ok, (q99, worst)


def test_drop_before_the_solve_then_solve(mid_small):
    """A drop before any level: every later level set-up leaves the dropped
    observations out; the whole coarse-to-fine solve (graph) matches."""
    sc = mid_small
    s = make(sc, "ic", pba.PBA_FP64, flags=pba.PBA_FLAG_GRAPH)
    s.drop_frame(12)
    res, _ = s.solve(4, 5e-3)
    gn = GaussNewton(Problem.from_scene(sc), "ic")
    gn.drop_frame(12)
    it = gn.solve(4, 5e-3)
    assert list(res.iters)[:3] == list(reversed(it))
    poses, d = s.get_params()
    assert rot_err(poses, gn.poses).max() <= 1e-8
    assert np.abs(d / gn.d - 1).max() <= 1e-8


def test_drop_in_one_window_leaves_the_other(mid_small):
    """Two windows in one context: dropping a frame of window 1 changes only
    window 1, which then matches the oracle's drop."""
    w0 = scenes.window(1, n_kf=5, pts_per_host=150, width=640, height=360)
    w1 = scenes.window(2, n_kf=6, pts_per_host=150, width=640, height=360)
    b = pba.Solver(mode=pba.PBA_IC_PROXY, precision=pba.PBA_FP64, n_levels=1, n_windows=2)
    b.set_scene(w0, window=0)
    b.set_scene(w1, window=1)
    b.iterate(0, 1)
    b.drop_frame(3, window=1)
    b.iterate(0, 3)
    for w, sc, drop in ((0, w0, None), (1, w1, 3)):
        gn = GaussNewton(Problem.from_scene(sc), "ic")
        gn.iterate(0, 1)
        if drop is not None:
            gn.drop_frame(drop)
        gn.iterate(0, 3)
        pb, db = b.get_params(w)
        assert rot_err(pb, gn.poses).max() <= 1e-8
        assert np.abs(db / gn.d - 1).max() <= 1e-8


def test_drop_invalid_arguments(mid_small):
    sc = mid_small
    s = make(sc, "ic", pba.PBA_FP64)
    for f, w in ((0, 0), (-1, 0), (sc.n_frames, 0), (3, 1)):
        with pytest.raises(pba.PbaError) as e:
            s.drop_frame(f, window=w)
        assert e.value.status == pba.PBA_E_INVALID
    e2 = pba.Solver(mode=pba.PBA_IC_PROXY, precision=pba.PBA_FP64, n_levels=sc.n_levels)
    with pytest.raises(pba.PbaError) as e:
        e2.drop_frame(3)
    assert e.value.status == pba.PBA_E_STATE
