"""GPU parity of the batched form: independent windows held by one context
(n_windows > 1) run through the same kernels in one launch per step, with a
block-diagonal reduced system (one gauge pin and one damping per window), and
the whole solve captured as one HIP graph (PBA_FLAG_GRAPH).

Every window of the batch must equal the same window solved alone by the
library (FP64: to rounding) and by the FP64 oracle; the captured graph must
reproduce the uncaptured launches, replay after replay."""
import numpy as np
import pytest

import scenes
from oracle.gn import GaussNewton, Problem
from tests.oracle_refs import depth_errors_ok, rot_err, trans_rel_err

pytestmark = pytest.mark.gpu

pba = pytest.importorskip("paper_1704_06967_amd.pba")


@pytest.fixture(scope="module")
def wins():
    # uneven windows: 5, 7 and 6 keyframes, 150-250 points per keyframe, 640x360
    return [scenes.window(s, n_kf=k, pts_per_host=p, width=640, height=360)
            for s, k, p in ((1, 5, 150), (2, 7, 250), (3, 6, 200))]


def make(n_windows, mode, precision, flags=0, **kw):
    return pba.Solver(mode=pba.PBA_IC_PROXY if mode == "ic" else pba.PBA_FC, precision=precision,
                      n_levels=1, n_windows=n_windows, flags=flags, **kw)


def load(s, wins):
    for w, sc in enumerate(wins):
        s.set_scene(sc, window=w)


@pytest.mark.parametrize("mode", ["ic", "fc"])
def test_batched_equals_single_fp64(wins, mode):
    b = make(len(wins), mode, pba.PBA_FP64)
    load(b, wins)
    st = b.iterate(0, 5)
    assert len(st) == 5
    for w, sc in enumerate(wins):
        s = make(1, mode, pba.PBA_FP64)
        s.set_scene(sc)
        s.iterate(0, 5)
        p1, d1 = s.get_params()
        pb, db = b.get_params(w)
        assert rot_err(pb, p1).max() <= 1e-12
        assert trans_rel_err(pb, p1).max() <= 1e-12
        np.testing.assert_allclose(db, d1, rtol=1e-12)
        gn = GaussNewton(Problem.from_scene(sc), mode)
        gn.iterate(0, 5)
        assert rot_err(pb, gn.poses).max() <= 1e-8
        assert trans_rel_err(pb, gn.poses).max() <= 1e-8
        assert np.abs(db / gn.d - 1).max() <= 1e-8
    # statistics are sums over the windows
    tot = sum(GaussNewton(Problem.from_scene(sc), mode).iterate(0, 1)[0]["n_active"] for sc in wins)
    assert st[0]["n_active"] == tot


@pytest.mark.parametrize("mode", ["ic", "fc"])
def test_batched_fp32_vs_oracle(wins, mode):
    b = make(len(wins), mode, pba.PBA_FP32)
    load(b, wins)
    b.iterate(0, 5)
    for w, sc in enumerate(wins):
        gn = GaussNewton(Problem.from_scene(sc), mode)
        gn.iterate(0, 5)
        pb, db = b.get_params(w)
        assert rot_err(pb, gn.poses).max() <= 1e-5
        assert trans_rel_err(pb, gn.poses).max() <= 1e-5
        ok, q99, worst = depth_errors_ok(db, gn.d)
        assert ok, (w, q99, worst)


@pytest.mark.parametrize("precision", [pba.PBA_FP64, pba.PBA_FP32])
def test_graph_replays_match_launches(wins, precision):
    """The solve captured once and replayed three times (with eager calls in
    between) gives the uncaptured solve's result every time."""
    ref = make(len(wins), "ic", precision)
    load(ref, wins)
    r_ref, _ = ref.solve(5, 0.0)
    p_ref = [ref.get_params(w) for w in range(len(wins))]
    g = make(len(wins), "ic", precision, flags=pba.PBA_FLAG_GRAPH)
    load(g, wins)
    for rep in range(3):
        for w, sc in enumerate(wins):
            g.set_params(sc.poses_init, sc.inv_depth_init, window=w)
        r, _ = g.solve(5, 0.0)
        assert list(r.iters) == list(r_ref.iters)
        assert r.final_rmse == r_ref.final_rmse
        for w in range(len(wins)):
            pg, dg = g.get_params(w)
            np.testing.assert_array_equal(pg, p_ref[w][0])
            np.testing.assert_array_equal(dg, p_ref[w][1])
        g.evaluate(0)  # eager work between replays


def test_graph_single_problem_pyramid():
    """One problem, 3 levels with the convergence gate: the captured solve equals
    the launched one (iteration counts and parameters)."""
    sc = scenes.mid(n_per_host=300)
    kw = dict(mode=pba.PBA_IC_PROXY, precision=pba.PBA_FP32, n_levels=3, pattern=sc.pattern, huber_k=sc.huber_k)
    a = pba.Solver(**kw)
    a.set_scene(sc)
    ra, _ = a.solve(10, 5e-3)
    g = pba.Solver(flags=pba.PBA_FLAG_GRAPH, **kw)
    g.set_scene(sc)
    for _ in range(2):
        g.set_params(sc.poses_init, sc.inv_depth_init)
        rg, _ = g.solve(10, 5e-3)
        assert list(rg.iters) == list(ra.iters)
        np.testing.assert_array_equal(g.get_params()[0], a.get_params()[0])
        np.testing.assert_array_equal(g.get_params()[1], a.get_params()[1])


def test_batched_invalid_usage(wins):
    b = make(2, "ic", pba.PBA_FP32)
    b.set_scene(wins[0], window=0)
    with pytest.raises(pba.PbaError) as e:
        b.iterate(0, 1)  # window 1 not set
    assert e.value.status == pba.PBA_E_STATE
    with pytest.raises(pba.PbaError):
        b.set_frames(wins[1].images[:, :100, :100], wins[1].intrinsics, wins[1].poses_init, window=1)
    with pytest.raises(pba.PbaError):
        b.set_scene(wins[1], window=2)


@pytest.mark.parametrize("mode", ["ic", "fc"])
def test_autotune_keeps_results(wins, mode):
    """The autotuner changes launch shapes and, for the IC residual pass, the
    lane mapping (a thread per observation or a lane per patch pixel): the
    iterates after tuning equal the untuned ones bit for bit when the mapping
    is the default one, and to the rounding of the per-observation FP64 sums
    otherwise."""
    a = make(len(wins), mode, pba.PBA_FP32)
    load(a, wins)
    a.iterate(0, 3)
    b = make(len(wins), mode, pba.PBA_FP32)
    load(b, wins)
    rep = b.autotune(0, 3)
    assert len(rep["candidates"]) >= 9 and rep["chosen"] in rep["candidates"]
    assert all(c["us"] > 0 for c in rep["candidates"])
    if mode == "ic":
        assert {c["lanes"] for c in rep["candidates"]} == {1, 8}
    b.iterate(0, 3)
    same = mode == "fc" or rep["chosen"]["lanes"] == 1
    for w in range(len(wins)):
        pa, da = a.get_params(w)
        pb, db = b.get_params(w)
        if same:
            np.testing.assert_array_equal(pa, pb)
            np.testing.assert_array_equal(da, db)
        else:
            # FP32 residuals: a sum that differs in its last FP64 bits can round
            # a later iteration's r or J to the neighbouring float
            np.testing.assert_allclose(pb, pa, rtol=0, atol=1e-6)
            np.testing.assert_allclose(db, da, rtol=1e-6)


def test_residual_lane_mappings_fp64_agree(wins):
    """The IC residual pass with a lane per patch pixel against a thread per
    observation, in FP64: the per-pixel arithmetic is shared and only the
    order of the additions of an observation's 8 products differs, so the
    per-iteration energies and active counts, the reduced right-hand side and
    the iterates agree to the rounding of FP64 sums."""
    runs = []
    for flags in (0, pba.PBA_FLAG_LANE_PER_PIXEL):
        s = make(len(wins), "ic", pba.PBA_FP64, flags=flags)
        load(s, wins)
        st = s.iterate(0, 4)
        runs.append((st, s.fetch(pba.PBA_DBG_B), [s.get_params(w) for w in range(len(wins))]))
        s.close()
    (st1, b1, p1), (st8, b8, p8) = runs
    for a1, a8 in zip(st1, st8):
        assert a1["n_active"] == a8["n_active"]
        assert abs(a8["energy"] / a1["energy"] - 1) <= 1e-12
    # b = g_p - sum h g_d / H_dd cancels: its rounding is relative to its largest entries
    np.testing.assert_allclose(b8, b1, rtol=0, atol=1e-10 * np.abs(b1).max())
    for (q1, d1), (q8, d8) in zip(p1, p8):
        np.testing.assert_allclose(q8, q1, rtol=0, atol=1e-10)
        np.testing.assert_allclose(d8, d1, rtol=1e-9)


def test_residual_lane_per_pixel_fp32_vs_oracle(wins):
    """The lane-per-pixel mapping in FP32 against the FP64 oracle, 5 IC
    iterations per window: every pose and inverse depth within the bars."""
    b = make(len(wins), "ic", pba.PBA_FP32, flags=pba.PBA_FLAG_LANE_PER_PIXEL)
    load(b, wins)
    b.iterate(0, 5)
    for w, sc in enumerate(wins):
        gn = GaussNewton(Problem.from_scene(sc), "ic")
        gn.iterate(0, 5)
        pb, db = b.get_params(w)
        assert rot_err(pb, gn.poses).max() <= 1e-5
        assert trans_rel_err(pb, gn.poses).max() <= 1e-5
        ok, q99, worst = depth_errors_ok(db, gn.d)
        assert ok, (w, q99, worst)


@pytest.fixture(scope="module")
def full_windows():
    # the first three windows of the benchmark's batch, at the batched
    # workload's size: 1280x720, 5-9 keyframes, 1000-3000 points per keyframe
    return [scenes.window(i) for i in range(3)]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("mode", ["ic", "fc"])
def test_batched_mixed_full_size_vs_oracle(full_windows, mode):
    """The batched workload's launch configuration (mixed form, one context
    for all windows, autotuned residual launch shape, the solve captured as one
    HIP graph, 5 iterations without the convergence test) against the FP64
    oracle's 5 iterations of each window: every pose and every inverse depth
    within the contract's bars, and the batch's photometric RMSE (over all
    windows' usable residuals) within 1e-4."""
    nw = len(full_windows)
    b = make(nw, mode, pba.PBA_MIXED_BF16, flags=pba.PBA_FLAG_GRAPH)
    load(b, full_windows)
    b.autotune(0, 3)
    for w, sc in enumerate(full_windows):
        b.set_params(sc.poses_init, sc.inv_depth_init, window=w)
    b.solve(5, 0.0)
    ev = b.evaluate(0)
    sq, cnt = 0.0, 0
    for w, sc in enumerate(full_windows):
        gn = GaussNewton(Problem.from_scene(sc), mode)
        gn.iterate(0, 5)
        pb, db = b.get_params(w)
        rot = rot_err(pb, gn.poses).max()
        trans = trans_rel_err(pb, gn.poses).max()
        ok, q99, worst = depth_errors_ok(db, gn.d)
        print(f"batched mixed {mode} window {w} ({sc.n_frames} keyframes, {sc.n_points} points, {sc.n_obs} "
              f"observations): rot {rot:.2e} rad, trans {trans:.2e}, inv depth p99 {q99:.2e} max {worst:.2e}")
        assert rot <= 1e-5 and trans <= 1e-5, w
        assert ok, (w, q99, worst)
        oev = gn.evaluate(0)
        sq += oev["sq"]
        cnt += oev["n_active"]
    assert ev["n_active"] == cnt
    assert abs(ev["rmse"] / np.sqrt(sq / cnt) - 1) <= 1e-4
