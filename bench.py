#!/usr/bin/env python3
"""Throughput of proxy-template inverse-compositional photometric bundle
adjustment on one MI355X, against forward-compositional Gauss-Newton on the
same GPU and the FP64 CPU oracle.

Workload: the mid problem - 30 frames 640x480 (float32) on a 360-degree orbit
around a seeded value-noise ellipsoid (axes 1.0/0.8/0.6), 3-level pyramid,
5 host frames x 4000 points, 8-pixel patches, Huber k = 9/255, image noise
sigma 2/255; residuals and Jacobians in FP32, reductions, Schur complement and
Cholesky in FP64.

One step = one coarse-to-fine solve (3 levels, at most --max-iters Gauss-Newton
iterations per level, convergence at 5e-3 px) from the same perturbed start,
inputs resident on the GPU. The library's calls are synchronous on its own
stream, so wall-clock time around them brackets the device work.

Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
# L2-miss bytes per level-0 launch from two rocprofv3 counter runs: FETCH_SIZE
# (bytes the L2 fetched from HBM or the memory-attached last-level cache) x 2.000
# + WRITE_SIZE x 1.000, both scales from a 256 MiB device copy
# (profiles/ic_iteration_kernels_traffic_mid_precision.md); valid only for the kernel
# sources whose combined hash is given
MEASURED_TRAFFIC = {"k_ic_residual": {"mid": 17164595, "precision": 128371917},
                    "k_ic_step": {"mid": 11062170},
                    "sources_sha256_16": "5241330df0b5690d"}
KERNEL_SOURCES = ("pba_kernels.hip", "pba_solver.hip", "pba_depth.hpp", "pba_device.hpp", "pba_internal.hpp")
# the same for the joint pose-brightness linearization (mid workload rendered
# with per-frame brightness; profiles/aff_linearize_traffic_mid.md)
MEASURED_TRAFFIC_AFFINE = {"k_aff_linearize": {"mid": 93969920}, "sources_sha256_16": "99c380c06b139b79"}
AFFINE_SOURCES = ("pba_affine.hip", "pba_affine.hpp", "pba_device.hpp", "pba_internal.hpp")


def kernel_sources_sha(files=KERNEL_SOURCES):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1704_06967_amd", "csrc", f),
                  "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    table, files = MEASURED_TRAFFIC, KERNEL_SOURCES
    if kernel in MEASURED_TRAFFIC_AFFINE:
        table, files = MEASURED_TRAFFIC_AFFINE, AFFINE_SOURCES
    if kernel_sources_sha(files) != table["sources_sha256_16"]:
        return None
    return table[kernel].get(workload)


METRIC = "GN iters/s & residuals/s, IC-proxy vs FC on same GPU at equal final photo-RMSE"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def level_pixels(scene, level):
    """Level-`level` target pixels of every residual at the scene's starting
    parameters (host patch pixel -> warp -> projection), for byte counting."""
    P = scene.pattern.shape[0]
    N = scene.n_points
    obs_point = np.repeat(np.arange(N), np.diff(scene.obs_ptr))
    host = scene.host_frame[obs_point]
    tgt = scene.obs_frame
    s = 2.0 ** level
    K = scene.intrinsics
    uv = (scene.host_uv[obs_point].astype(float) + 0.5) / s - 0.5
    pu = uv[:, None, 0] + scene.pattern[None, :, 0]
    pv = uv[:, None, 1] + scene.pattern[None, :, 1]
    Kh, Kt = K[host] / np.array([s, s, 1, 1]), K[tgt] / np.array([s, s, 1, 1])
    Kh[:, 2:] = (K[host, 2:] + 0.5) / s - 0.5
    Kt[:, 2:] = (K[tgt, 2:] + 0.5) / s - 0.5
    x = (pu - Kh[:, None, 2]) / Kh[:, None, 0]
    y = (pv - Kh[:, None, 3]) / Kh[:, None, 1]
    Rp = scene.poses_init[:, :9].reshape(-1, 3, 3)
    tp = scene.poses_init[:, 9:]
    R = Rp[tgt] @ np.swapaxes(Rp[host], 1, 2)
    t = tp[tgt] - np.einsum("oij,oj->oi", R, tp[host])
    d = scene.inv_depth_init[obs_point]
    v = (R[:, None, :, 0] * x[..., None] + R[:, None, :, 1] * y[..., None] + R[:, None, :, 2]
         + d[:, None, None] * t[:, None, :])
    qu = Kt[:, None, 0] * v[..., 0] / v[..., 2] + Kt[:, None, 2]
    qv = Kt[:, None, 1] * v[..., 1] / v[..., 2] + Kt[:, None, 3]
    return tgt, qu, qv


def _pairs(scene):
    """(host, target) pair of every observation and the number of distinct pairs."""
    host = scene.host_frame[np.repeat(np.arange(scene.n_points), np.diff(scene.obs_ptr))]
    key = host.astype(np.int64) * scene.n_frames + scene.obs_frame
    uniq, counts = np.unique(key, return_counts=True)
    return uniq.size, counts


def _unique_texels(scene, level, halo):
    """Distinct target texels of the bilinear footprints at the starting
    parameters: 2 x 2 (halo 0) or the 4 x 4 of the interpolated central
    differences (halo 1)."""
    F, H, W = scene.images.shape
    Wl, Hl = W >> level, H >> level
    tgt, qu, qv = level_pixels(scene, level)
    ok = (qu >= 1) & (qu <= Wl - 3) & (qv >= 1) & (qv <= Hl - 3)
    j0 = np.floor(qu[ok]).astype(np.int64)
    i0 = np.floor(qv[ok]).astype(np.int64)
    f = np.broadcast_to(tgt[:, None], qu.shape)[ok].astype(np.int64)
    base = (f * Hl + i0) * Wl + j0
    offs = [di * Wl + dj for di in range(-halo, 2 + halo) for dj in range(-halo, 2 + halo)]
    return int(np.unique(np.concatenate([base + o for o in offs])).size)


def ic_residual_bytes(scene, level=0, real=4):
    """Algorithmic bytes of one launch of the IC residual kernel at `level`:
    per observation its point and pair index, mask byte and the 10-value FP64
    record it writes and its g_d once more (contiguous, for the depth
    readers); per observed point its pixel, two depths and the 8 template
    records (I0, gradient, usable); per pair the FP64 level intrinsics of host
    and target (8 values), the FP64 current relative pose (12) and the
    relative pose at p(0) in the element type (12); the target texels touched
    by the bilinear 2x2 footprints, each counted once."""
    O = scene.n_obs
    P = scene.pattern.shape[0]
    n_obs_pts = int(np.count_nonzero(np.diff(scene.obs_ptr)))
    n_pairs, _ = _pairs(scene)
    texels = _unique_texels(scene, level, 0)
    reads = (O * (4 + 4 + 1) + n_obs_pts * (8 + 8 + 8 + P * 4 * real) + n_pairs * (8 * 8 + 12 * 8 + 12 * real)
             + texels * real)
    writes = O * 11 * 8   # FP64 sums for every element type
    return {"bytes": int(reads + writes), "reads": int(reads), "writes": int(writes), "unique_texels": int(texels),
            "observations": O, "residual_slots": O * 8}


def fc_linearize_bytes(scene, level=0, real=4):
    """Algorithmic bytes of one launch of the FC linearization (every
    iteration): as the IC residual kernel, without the p(0) pose, plus the
    4 x 4 texel footprints of the interpolated gradients and the 38-value
    FP64 record of every observation (written by lanes in 8-value strides)."""
    O = scene.n_obs
    P = scene.pattern.shape[0]
    n_obs_pts = int(np.count_nonzero(np.diff(scene.obs_ptr)))
    n_pairs, _ = _pairs(scene)
    texels = _unique_texels(scene, level, 1)
    reads = O * (4 + 4 + 1) + n_obs_pts * (8 + 8 + P * 4 * real) + n_pairs * (8 * 8 + 12 * 8) + texels * real
    writes = O * 38 * 8
    return {"bytes": int(reads + writes), "reads": int(reads), "writes": int(writes), "unique_texels": int(texels),
            "observations": O}


def ic_step_bytes(scene, real=4, pair_chunk=512):
    """Algorithmic bytes of one launch of the fused IC step (solve and depth
    update of one iteration): S^-1 of the reduced system once (8 (6F)^2),
    the pair-chunk partials (9 doubles each), per pair the geometry at p(0)
    and at the current iterate (16 doubles each) read and the next one
    written (16 doubles + 12 values), the poses and the p(0) poses read and
    the poses written (12 doubles per frame each); per point its observation
    range, pixel, depth diagonal, depth and p(0) depth read and its depth
    written; per observation its pair index, h (6 values) and g_d."""
    F, N, O = scene.n_frames, scene.n_points, scene.n_obs
    n_pairs, counts = _pairs(scene)
    nch = int(np.sum((counts + pair_chunk - 1) // pair_chunk))
    n6 = 6 * F
    reads = (8 * n6 * n6 + nch * 9 * 8 + n_pairs * 2 * 16 * 8 + 2 * 12 * F * 8 + N * (4 + 8 + 8 + 8 + 8)
             + O * (4 + 7 * 8))
    writes = n_pairs * (16 * 8 + 12 * real) + 12 * F * 8 + N * 8
    return {"bytes": int(reads + writes), "reads": int(reads), "writes": int(writes), "sinv_bytes": 8 * n6 * n6,
            "pair_chunks": nch}


def roofline_obj(kernel, nbytes, avg_ms, launches, traffic=None, note=None):
    gbs = nbytes["bytes"] / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    r = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel,
         "avg_launch_us": round(avg_ms * 1e3, 3), "launches": int(launches),
         "algorithmic_bytes_per_launch": nbytes["bytes"], "bytes_detail": nbytes}
    if note:
        r["note"] = note
    return r


def run_steps(solver, poses0, d0, steps, max_iters, conv_px):
    times, iters, active, results = [], 0, 0, []
    for _ in range(steps):
        t0 = time.perf_counter()
        solver.set_params(poses0, d0)
        res, _ = solver.solve(max_iters, conv_px)
        times.append(time.perf_counter() - t0)
        iters += res.total_iters
        active += res.active_residuals
        results.append(res.as_dict())
    return times, iters, active, results


CAPS = (1, 2, 3, 4, 6, 8, 10, 14, 20, 30, 40)


def rmse_vs_time(pba, scene, mode, precision, conv_px, caps=CAPS, reps=3, recentre=0):
    """Final level-0 photometric RMSE and solve time of whole coarse-to-fine
    solves with at most k iterations per level, for every cap k (each solve
    one graph launch, timed to its end; median of `reps` replays after a
    capturing run), until a solve converges at every level."""
    s = pba.Solver(mode=mode, precision=precision, flags=pba.PBA_FLAG_GRAPH, n_levels=scene.n_levels,
                   pattern=scene.pattern, huber_k=scene.huber_k, recentre_every=recentre)
    s.set_scene(scene)
    p0, d0 = scene.poses_init, scene.inv_depth_init
    pts = []
    for k in caps:
        s.set_params(p0, d0)
        try:
            s.solve(k, conv_px)  # capture
        except pba.PbaError as e:
            # the iteration diverged: the solver stops on an indefinite reduced system
            pts.append({"cap": k, "error": str(e)})
            log(f"  {'IC' if mode == pba.PBA_IC_PROXY else 'FC'} recentre={recentre} cap {k}: {e}")
            break
        ts, res = [], None
        for _ in range(reps):
            s.set_params(p0, d0)
            t0 = time.perf_counter()
            res, _ = s.solve(k, conv_px)
            ts.append(time.perf_counter() - t0)
        r = res.as_dict()
        if not (np.isfinite(r["final_rmse"]) and r["final_rmse"] > 0):
            # every residual left the images: the iteration diverged
            pts.append({"cap": k, "error": f"final RMSE {r['final_rmse']} (no active residual)"})
            break
        pts.append({"cap": k, "ms": round(float(np.median(ts)) * 1e3, 4), "rmse": r["final_rmse"],
                    "iters": r["iters"][:scene.n_levels], "converged": bool(r["converged"])})
        if all(i < k for i in r["iters"][:scene.n_levels]):
            break   # every level stopped on the convergence test
    s.close()
    return pts


def equal_rmse_section(pba, scene, precision, conv_px, final_cap, caps=CAPS, recentre=3):
    """Time to equal final photometric RMSE (IC vs FC on the same GPU). The
    final RMSE of a method is that of its solve with final_cap iterations per
    level (the headline solve), r* the larger of IC's and FC's, and each
    method's time that of its cheapest solve in the sweep whose RMSE is within
    r* (1 + 1e-3). Beside them: IC with proxy re-centring every `recentre`
    iterations, and every method's best RMSE over the sweep."""
    curves = {"ic": rmse_vs_time(pba, scene, pba.PBA_IC_PROXY, precision, conv_px, caps),
              f"ic_recentre{recentre}": rmse_vs_time(pba, scene, pba.PBA_IC_PROXY, precision, conv_px, caps,
                                                     recentre=recentre),
              "fc": rmse_vs_time(pba, scene, pba.PBA_FC, precision, conv_px, caps)}

    def at_cap(pts):
        sel = [p for p in pts if p["cap"] <= final_cap and "rmse" in p]
        return sel[-1]["rmse"] if sel else None

    r_star = max(at_cap(curves["ic"]), at_cap(curves["fc"]))

    def first(pts):
        ok = [p for p in pts if "rmse" in p and p["rmse"] <= r_star * (1 + 1e-3)]
        return min(ok, key=lambda p: p["ms"]) if ok else None

    out = {"r_star": r_star, "final_cap": final_cap}
    for name, pts in curves.items():
        f = first(pts)
        good = [p for p in pts if "rmse" in p]
        best = min(good, key=lambda p: p["rmse"])
        out[name] = {"ms_to_r_star": f["ms"] if f else None, "cap_to_r_star": f["cap"] if f else None,
                     "final_rmse": at_cap(pts), "best_rmse": best["rmse"], "best_cap": best["cap"],
                     "converged": good[-1]["converged"], "diverged_at_cap": pts[-1]["cap"] if "error" in pts[-1]
                     else None, "curve": pts}
    a, b = out["ic"]["ms_to_r_star"], out["fc"]["ms_to_r_star"]
    out["ic_speedup"] = round(b / a, 3) if a and b else None
    out["note"] = ("whole solves (graph launches) with at most `cap` iterations per level, timed to completion; "
                   "IC's level-0 RMSE rises after its first few iterations on this workload (its fixed point is "
                   "not FC's), so r* is set by IC's final solve; with re-centring the iteration diverges at larger "
                   "caps (diverged_at_cap: the solver reported an indefinite reduced system or lost every "
                   "residual)")
    return out


def converged_section(pba, precision, max_iters=40, conv_px=5e-3, reps=10):
    """IC and FC run to convergence (the Sec. 4.1 test at every level) on a
    variant of the mid workload on which IC's fixed point is FC's: targets
    within +-2 frames (24 degrees) and no image noise (on mid itself the wider
    baselines and the noise move IC's fixed point away from FC's). Each solve
    is one graph launch, timed to its end (median of `reps`)."""
    import scenes

    sc = scenes.mid(reach=2, noise_sigma=0.0)
    out = {"workload": "mid geometry, targets within +-2 frames (24 deg), no image noise: 5 hosts x 4000 points, "
                       f"{sc.n_obs} observations; at most {max_iters} iterations per level, convergence at "
                       f"{conv_px} px", "points": sc.n_points, "observations": sc.n_obs}
    for name, mode in (("ic", pba.PBA_IC_PROXY), ("fc", pba.PBA_FC)):
        s = pba.Solver(mode=mode, precision=precision, flags=pba.PBA_FLAG_GRAPH, n_levels=sc.n_levels,
                       pattern=sc.pattern, huber_k=sc.huber_k)
        s.set_scene(sc)
        s.solve(max_iters, conv_px)  # capture
        ts, res = [], None
        for _ in range(reps):
            s.set_params(sc.poses_init, sc.inv_depth_init)
            t0 = time.perf_counter()
            res, _ = s.solve(max_iters, conv_px)
            ts.append(time.perf_counter() - t0)
        r = res.as_dict()
        s.close()
        out[name] = {"ms_per_solve": round(float(np.median(ts)) * 1e3, 4), "iters": r["iters"][:sc.n_levels],
                     "converged": bool(r["converged"]), "final_rmse": r["final_rmse"]}
    ic, fc = out["ic"], out["fc"]
    out["rmse_ic_over_fc"] = ic["final_rmse"] / fc["final_rmse"]
    out["ic_speedup_to_convergence"] = round(fc["ms_per_solve"] / ic["ms_per_solve"], 3)
    return out


def dynamic_section(pba, scene, reps=10, frame=13):
    """Sliding-window keyframe drop on the mid workload (FP32, IC at level 0):
    the time of pba_drop_frame, which forms the reduced system again from the
    records kept at p(0), against the time of a level start, which
    linearizes every residual first (both synchronous calls, median of
    `reps`)."""
    kw = dict(mode=pba.PBA_IC_PROXY, precision=pba.PBA_FP32, n_levels=scene.n_levels, pattern=scene.pattern,
              huber_k=scene.huber_k)
    drop_ms, start_ms = [], []
    for _ in range(reps):
        s = pba.Solver(**kw)
        s.set_scene(scene)
        s.iterate(0, 2)
        t0 = time.perf_counter()
        s.drop_frame(frame)
        drop_ms.append((time.perf_counter() - t0) * 1e3)
        s.set_params(scene.poses_init, scene.inv_depth_init)
        t0 = time.perf_counter()
        s.iterate(0, 0)   # the level start alone (linearization, Schur complement, factor, inverse)
        start_ms.append((time.perf_counter() - t0) * 1e3)
        s.close()
    d, st = float(np.median(drop_ms)), float(np.median(start_ms))
    return {"workload": f"mid, IC FP32 at level 0: drop frame {frame} after 2 iterations", "drop_ms": round(d, 4),
            "level_start_ms": round(st, 4), "drop_over_level_start": round(d / st, 3),
            "note": "host wall time of the synchronous calls (median); the drop sums the pair blocks, h and H_dd "
                    "again from the records at p(0) instead of linearizing every residual"}


def aff_linearize_bytes(scene, level=0, real=4):
    """Algorithmic bytes of one launch of the joint (brightness) linearization:
    per observation its point and pair indices, window flag and frozen-set
    mask, its FC record (38 values) and brightness record (42 values, FP64)
    written; per observed point its pixel, depth and template (P x 4 values);
    per pair its geometry (12 doubles), level intrinsics (8 doubles) and the
    brightness of its two frames (4 doubles); the 4 x 4 texel footprints of
    the interpolated gradients once."""
    O = scene.n_obs
    P = scene.pattern.shape[0]
    n_obs_pts = int(np.count_nonzero(np.diff(scene.obs_ptr)))
    n_pairs, _ = _pairs(scene)
    texels = _unique_texels(scene, level, 1)
    reads = O * (4 + 4 + 1 + 1) + n_obs_pts * (8 + 8 + P * 4 * real) + n_pairs * (12 + 8 + 4) * 8 + texels * real
    writes = O * (38 + 42) * 8
    return {"bytes": int(reads + writes), "reads": int(reads), "writes": int(writes), "unique_texels": int(texels),
            "observations": O}


def affine_section(pba, scene, iters=10, reps=3):
    """Per-frame affine brightness in the FC iteration on the mid workload
    rendered with seeded brightness (FP32 images, FP64 system), from the true
    geometry with the brightness unknown: host wall time per joint iteration
    at level 0 (median over `reps` runs of `iters`), the plain
    FC iteration on the same images beside it, and the joint linearization's
    launch time (HIP events) against its algorithmic bytes."""
    import dataclasses
    from scenes.brightness import brighten, seeded_ab
    ab = seeded_ab(scene.n_frames, 11)
    sc = dataclasses.replace(scene, images=brighten(scene.images, ab), poses_init=scene.poses_gt,
                             inv_depth_init=scene.inv_depth_gt)
    kw = dict(mode=pba.PBA_FC, precision=pba.PBA_FP32, n_levels=sc.n_levels, pattern=sc.pattern,
              huber_k=sc.huber_k, flags=pba.PBA_FLAG_TIMING)
    aff_ms, fc_ms, lin_ms, lin_n, rmse = [], [], 0.0, 0, None
    for _ in range(reps):
        s = pba.Solver(**kw)
        s.set_scene(sc)
        s.set_affine(np.zeros((sc.n_frames, 2)))
        s.iterate(0, 1)                      # level start, frozen set
        t0 = time.perf_counter()
        st = s.iterate(0, iters)
        aff_ms.append((time.perf_counter() - t0) * 1e3 / iters)
        tm = s.timing()
        lin_ms, lin_n = tm["residual_ms"][0], tm["residual_launches"][0]
        ab_err = float(np.abs(s.get_affine() - ab).max())
        rmse = st[-1]["rmse"]
        s.close()
        p = pba.Solver(**kw)
        p.set_scene(sc)
        p.iterate(0, 1)
        t0 = time.perf_counter()
        sp = p.iterate(0, iters)
        fc_ms.append((time.perf_counter() - t0) * 1e3 / iters)
        plain_rmse = sp[-1]["rmse"]
        p.close()
    avg = lin_ms / max(1, lin_n)
    return {"workload": f"mid rendered with per-frame brightness (|a| <= 0.15, |b| <= 0.05), FC FP32 at level 0, "
                        f"{iters} iterations from the true geometry",
            "ms_per_joint_iteration": round(float(np.median(aff_ms)), 4),
            "ms_per_plain_fc_iteration": round(float(np.median(fc_ms)), 4),
            "rmse_after": rmse, "plain_fc_rmse_after": plain_rmse, "brightness_max_err": ab_err,
            "roofline": roofline_obj("k_aff_linearize", aff_linearize_bytes(sc), avg, lin_n,
                                     traffic=measured_traffic("k_aff_linearize", "mid")),
            "note": "both enqueue the iterations of a call as one batch (one host synchronization)"}


def _predicted_positions(scene, poses, inv_depth):
    """Level-0 pixel of every observation's point centre in its target frame
    under the given parameters (the tracker's prediction)."""
    obs_point = np.repeat(np.arange(scene.n_points), np.diff(scene.obs_ptr))
    hf = scene.host_frame[obs_point]
    tf = scene.obs_frame
    K = scene.intrinsics
    c = scene.host_uv[obs_point].astype(float)
    x = np.stack([(c[:, 0] - K[hf, 2]) / K[hf, 0], (c[:, 1] - K[hf, 3]) / K[hf, 1], np.ones(len(c))], 1)
    Rh, th = poses[hf, :9].reshape(-1, 3, 3), poses[hf, 9:]
    Rf, tf_ = poses[tf, :9].reshape(-1, 3, 3), poses[tf, 9:]
    R = Rf @ np.swapaxes(Rh, 1, 2)
    t = tf_ - np.einsum("nij,nj->ni", R, th)
    v = np.einsum("nij,nj->ni", R, x) + inv_depth[obs_point][:, None] * t
    return np.stack([K[tf, 0] * v[:, 0] / v[:, 2] + K[tf, 2], K[tf, 1] * v[:, 1] / v[:, 2] + K[tf, 3]], 1)


def _pose_errors(poses, ref):
    e = param_errors(poses, np.ones(1), ref, np.ones(1))
    return {"rot_max_rad": e["rot_max_rad"], "trans_rel_max": e["trans_rel_max"]}


def frontend_section(pba, scene, reps=5, corners_per_frame=2000):
    """The base solution of Sec. 4.1 on the mid workload, stage by stage: Harris
    corners of every host frame; robust tracks of the workload's points from
    their host into each target, predicted from the starting parameters;
    geometric BA of the tracked observations (FP64, FC iteration, one outlier
    removal); then the FC photometric solve from its result (the fourth step).
    Host wall time of the synchronous calls (median of `reps` for the first
    three)."""
    kw = dict(n_levels=scene.n_levels, pattern=scene.pattern, huber_k=scene.huber_k)
    s = pba.Solver(mode=pba.PBA_FC, precision=pba.PBA_FP64, **kw)
    s.set_frames(scene.images, scene.intrinsics, scene.poses_init)
    hosts = sorted(set(int(h) for h in scene.host_frame))
    t_c, n_c = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        for h in hosts:
            uv, _ = s.corners(h, cell=8, margin=8, max_corners=corners_per_frame)
            n_c.append(uv.shape[0])
        t_c.append((time.perf_counter() - t0) * 1e3 / len(hosts))
    obs_point = np.repeat(np.arange(scene.n_points), np.diff(scene.obs_ptr))
    obs_host = scene.host_frame[obs_point].astype(np.int32)
    obs_target = scene.obs_frame.astype(np.int32)
    guess = _predicted_positions(scene, scene.poses_init, scene.inv_depth_init)
    xs = scene.host_uv[obs_point].astype(float)
    t_t = []
    for _ in range(reps):
        t0 = time.perf_counter()
        pos, st, fb = s.track(obs_host, xs, obs_target, guess, radius=4, n_iters=10, min_eig=1e-6, fb_px=0.5)
        t_t.append((time.perf_counter() - t0) * 1e3)
    ok = st == pba.PBA_TRACK_OK
    # points and observations of the tracks that held
    keep_pt = np.zeros(scene.n_points, bool)
    keep_pt[obs_point[ok]] = True
    cnt = np.bincount(obs_point[ok], minlength=scene.n_points)[keep_pt]
    optr = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int32)
    hf, huv = scene.host_frame[keep_pt], scene.host_uv[keep_pt]
    d0 = scene.inv_depth_init[keep_pt]
    s.set_points(hf, huv, d0, optr, obs_target[ok])
    t_g, res = [], None
    for _ in range(reps):
        s.set_params(scene.poses_init, d0)
        s.set_tracks(pos[ok])
        t0 = time.perf_counter()
        res, status, inl = s.geo_solve(30, conv_px=5e-3, huber_px=2.0, outlier_px=3.0)
        t_g.append((time.perf_counter() - t0) * 1e3)
    poses_g, d_g = s.get_params()
    s.close()
    out = {
        "workload": f"mid: {len(hosts)} host frames 640x480; {obs_point.size} tracks (each workload observation, "
                    "predicted from the starting parameters); FP64",
        "corners": {"ms_per_frame": round(float(np.median(t_c)), 4), "per_frame": int(np.median(n_c)),
                    "cell": 8, "max_corners": corners_per_frame},
        "tracks": {"ms": round(float(np.median(t_t)), 4), "n": int(obs_point.size), "ok": int(ok.sum()),
                   "status_counts": np.bincount(st, minlength=4).tolist(), "radius": 4, "iters_per_level": 10,
                   "levels": scene.n_levels},
        "geometric_ba": {"ms": round(float(np.median(t_g)), 4), "points": int(keep_pt.sum()),
                         "observations": int(ok.sum()), "iters": [res.iters[0], res.iters[1]],
                         "converged": bool(res.converged), "rmse_px": res.final_rmse,
                         "inliers": int(res.final_active)},
        "pose_error_vs_truth": {"start": _pose_errors(scene.poses_init, scene.poses_gt),
                                "geometric": _pose_errors(poses_g, scene.poses_gt)},
        "note": "host wall time of the synchronous calls, allocation and host copies included",
    }
    # step 4: the FC photometric solve from the geometric result
    f = pba.Solver(mode=pba.PBA_FC, precision=pba.PBA_FP32, **kw)
    f.set_frames(scene.images, scene.intrinsics, poses_g)
    f.set_points(hf, huv, d_g, optr, obs_target[ok])
    t0 = time.perf_counter()
    r, _ = f.solve(10, 5e-3)
    poses_p, _ = f.get_params()
    out["photometric_fc"] = {"ms": round((time.perf_counter() - t0) * 1e3, 4), "iters": list(r.iters[:scene.n_levels]),
                             "final_rmse": r.final_rmse, **_pose_errors(poses_p, scene.poses_gt)}
    f.close()
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(scene, n_iters=10):
    """The FP64 oracle on a bounded sample of the same workload: level 0 of the
    mid problem, IC setup plus n_iters iterations, once on every core the
    process may use (BLAS threads = affinity cores) and once on one thread."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle.gn import GaussNewton, Problem

    cores = len(os.sched_getaffinity(0))
    runs = {}
    for threads in (cores, 1):
        with threadpool_limits(threads):
            P = Problem.from_scene(scene)
            P.layout(0)
            t0 = time.perf_counter()
            gn = GaussNewton(P, "ic")
            gn.iterate(0, n_iters)
            runs[threads] = time.perf_counter() - t0
    dt = runs[cores]
    blas = [{"api": i.get("internal_api"), "threads": i.get("num_threads")} for i in threadpool_info()]
    return {"value": round(n_iters / dt, 3), "unit": "GN iters/s", "cores": cores, "kind": "oracle",
            "sample": f"mid workload, level 0 only: IC setup + {n_iters} iterations (960k residuals each), "
                      f"{dt:.1f} s with {cores} BLAS threads, {runs[1]:.1f} s on 1 thread",
            "seconds": round(dt, 3), "one_thread": {"value": round(n_iters / runs[1], 3), "seconds": round(runs[1], 3)},
            "cpu_model": cpu_model(), "blas": blas}


def param_errors(poses, d, ref_poses, ref_d):
    """Per-result error of (poses, inverse depths) against a reference."""
    R = poses[:, :9].reshape(-1, 3, 3)
    Rr = ref_poses[:, :9].reshape(-1, 3, 3)
    rot = 2.0 * np.arcsin(np.clip(np.linalg.norm((R - Rr).reshape(len(R), -1), axis=1) / (2.0 * np.sqrt(2.0)), 0, 1))
    tn = np.linalg.norm(ref_poses[:, 9:], axis=1).max()
    tr = np.linalg.norm(poses[:, 9:] - ref_poses[:, 9:], axis=1) / max(tn, 1e-12)
    rel = np.abs(d / ref_d - 1.0)
    return {"rot_max_rad": float(rot.max()), "trans_rel_max": float(tr.max()),
            "inv_depth_rel_p50": float(np.median(rel)), "inv_depth_rel_p99": float(np.quantile(rel, 0.99)),
            "inv_depth_rel_max": float(rel.max())}


ORACLE_LEVEL_ITERS = 3   # IC iterations per level of the capped oracle comparison (precision workload)


def oracle_ic_capped(scene, iters=ORACLE_LEVEL_ITERS):
    """The FP64 oracle's IC solve of `scene`, `iters` iterations per level (run
    in a worker process, overlapped with the GPU sections)."""
    from threadpoolctl import threadpool_limits

    from oracle.gn import GaussNewton, Problem

    with threadpool_limits(4):
        t0 = time.perf_counter()
        gn = GaussNewton(Problem.from_scene(scene), "ic")
        for level in reversed(range(scene.n_levels)):
            gn.iterate(level, iters)
        return gn.poses, gn.d, gn.evaluate(0)["rmse"], time.perf_counter() - t0


def errors_vs_oracle(pba, sc, precision, oracle, iters=ORACLE_LEVEL_ITERS):
    """Per-result error of the library's IC solve (`iters` iterations per
    level, no convergence stop) against the oracle's, with the contract's bars."""
    s = pba.Solver(mode=pba.PBA_IC_PROXY, precision=precision, n_levels=sc.n_levels, pattern=sc.pattern,
                   huber_k=sc.huber_k)
    s.set_scene(sc)
    for level in reversed(range(sc.n_levels)):
        s.iterate(level, iters)
    poses, d = s.get_params()
    rmse = s.evaluate(0)["rmse"]
    s.close()
    op, od, ormse, osec = oracle
    e = param_errors(poses, d, op, od)
    e["rmse_rel"] = abs(rmse / ormse - 1.0)
    e["within_bars"] = bool(e["rot_max_rad"] <= 1e-5 and e["trans_rel_max"] <= 1e-5 and e["inv_depth_rel_max"] <= 1e-5
                            and e["rmse_rel"] <= 1e-4)
    e["inv_depth_points_above_bar"] = int(np.count_nonzero(np.abs(d / od - 1.0) > 1e-5))
    e["oracle_seconds"] = round(osec, 1)
    return e


def precision_section(pba, steps, max_iters, conv_px, sc=None, event_timing=True):
    """The precision workload (120 frames 640x480 around a value-noise torus,
    10 hosts x 20000 points, 6.4M residuals per level-0 iteration, 6F = 720):
    IC in the mixed form (BF16 MFMA pose blocks) timed per solve, and its result
    against the FP64 path's (which matches the FP64 oracle to rounding in the
    parity tests); FC in the mixed form for comparison."""
    import scenes

    if sc is None:
        t0 = time.perf_counter()
        sc = scenes.precision()
        log(f"scene precision: {sc.n_points} points, {sc.n_obs} observations ({time.perf_counter() - t0:.1f} s)")
    kw = dict(n_levels=sc.n_levels, pattern=sc.pattern, huber_k=sc.huber_k)
    out = {"workload": "precision: 120 frames 640x480 f32, value-noise torus, 3-level pyramid, 10 hosts x 20000 "
                       "points (4 targets each), 8-px patches; 6F = 720",
           "points": sc.n_points, "observations": sc.n_obs, "residuals_per_iter": sc.n_residuals(),
           "reduced_system": 6 * sc.n_frames}
    p0, d0 = sc.poses_init, sc.inv_depth_init
    nb = ic_residual_bytes(sc, 0, 4)
    results = {}
    for name, mode, prec, n in (("ic_mixed", pba.PBA_IC_PROXY, pba.PBA_MIXED_BF16, steps),
                                ("ic_fp64", pba.PBA_IC_PROXY, pba.PBA_FP64, 1),
                                ("fc_mixed", pba.PBA_FC, pba.PBA_MIXED_BF16, max(1, steps // 2))):
        # solves replayed as captured graphs; the residual kernel timed with
        # events in a second context (events are not captured)
        s = pba.Solver(mode=mode, precision=prec, flags=pba.PBA_FLAG_GRAPH, **kw)
        s.set_scene(sc)
        s.set_params(p0, d0)
        s.solve(max_iters, conv_px)  # warm-up (captures the graph)
        t, iters, active, res = run_steps(s, p0, d0, n, max_iters, conv_px)
        poses, d = s.get_params()
        results[name] = (poses, d)
        s.close()
        tm = {"residual_ms": [0.0] * 4, "residual_launches": [0] * 4}
        if event_timing:
            e = pba.Solver(mode=mode, precision=prec, flags=pba.PBA_FLAG_TIMING, **kw)
            e.set_scene(sc)
            e.set_params(p0, d0)
            e.solve(max_iters, conv_px)
            e.timing()
            e.set_params(p0, d0)
            e.solve(max_iters, conv_px)
            tm = e.timing()
            e.close()
        avg_us = tm["residual_ms"][0] / max(1, tm["residual_launches"][0]) * 1e3
        out[name] = {"ms_per_solve": round(float(np.mean(t)) * 1e3, 3), "iters_per_solve": res[-1]["iters"],
                     "gn_iters_per_s": round(iters / float(np.sum(t)), 2),
                     "residuals_per_s": round(active / float(np.sum(t)), 1), "final_rmse": res[-1]["final_rmse"],
                     "residual_kernel_avg_us_level0": round(avg_us, 3)}
        if mode == pba.PBA_IC_PROXY and prec == pba.PBA_MIXED_BF16 and avg_us > 0:
            gbs = nb["bytes"] / (avg_us * 1e-6) / 1e9
            out["residual_roofline"] = {"kernel": "k_ic_residual<float> (level 0)", "bound": "hbm",
                                        "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                        "frac": round(gbs / HBM_PEAK_GBS, 4),
                                        "traffic": measured_traffic("k_ic_residual", "precision"), "avg_launch_us": round(avg_us, 3),
                                        "algorithmic_bytes_per_launch": nb["bytes"], "bytes_detail": nb}
        log(f"precision {name}: {out[name]['ms_per_solve']} ms per solve, residual kernel {avg_us:.1f} us")
    out["ic_mixed_vs_fp64"] = param_errors(*results["ic_mixed"], *results["ic_fp64"])
    out["ic_mixed_rmse_rel_vs_fp64"] = abs(out["ic_mixed"]["final_rmse"] / out["ic_fp64"]["final_rmse"] - 1)
    out["note"] = ("ic_mixed_vs_fp64: the timed mixed-form IC solve against the FP64 IC solve of the same problem "
                   "(same iteration counts); vs_oracle: IC solves with 3 iterations per level against the FP64 "
                   "oracle's, bars rotation 1e-5 rad, translation 1e-5 relative, every inverse depth 1e-5 "
                   "relative, RMSE 1e-4 relative")
    return out, sc


def _one_thread():
    from threadpoolctl import threadpool_limits

    threadpool_limits(1)


def make_windows(n, workers):
    """The batched workload's windows (seeds 0..n-1), built in worker processes
    (one BLAS thread each) before this process touches the GPU."""
    import concurrent.futures as cf
    import multiprocessing as mp

    import scenes

    if workers <= 1:
        return [scenes.window(i) for i in range(n)]
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork"),
                                initializer=_one_thread) as ex:
        return list(ex.map(scenes.window, range(n)))


def batched_section(pba, wins, steps, iters):
    """The batched workload: len(wins) independent windows (5-9 keyframes,
    1000-3000 points per keyframe, 1280x720) in one context, IC in the mixed
    form, `iters` Gauss-Newton iterations each; the whole solve is one HIP graph
    launch, the residual kernel's launch shape autotuned on the batch. Every
    window of a batch completes with the batch, so the batch's launch-to-end
    time is every window's latency in the batched form; the per-window
    latencies of windows solved alone (one context each) are reported beside
    it."""
    nw = len(wins)
    out = {"workload": f"batched: {nw} windows, 5-9 keyframes 1280x720 f32 (textured planes + spheres), 1000-3000 "
                       f"points per keyframe, 8-px patches, {iters} IC iterations each, one graph launch",
           "windows": nw, "keyframes": [w.n_frames for w in wins], "points": int(sum(w.n_points for w in wins)),
           "observations": int(sum(w.n_obs for w in wins)),
           "residuals_per_iter": int(sum(w.n_residuals() for w in wins))}
    kw = dict(mode=pba.PBA_IC_PROXY, precision=pba.PBA_MIXED_BF16, n_levels=1)
    b = pba.Solver(n_windows=nw, flags=pba.PBA_FLAG_GRAPH, **kw)
    for i, w in enumerate(wins):
        b.set_scene(w, window=i)
    t0 = time.perf_counter()
    out["autotune"] = b.autotune(0, 20)
    out["autotune_s"] = round(time.perf_counter() - t0, 3)

    def reset():
        for i, w in enumerate(wins):
            b.set_params(w.poses_init, w.inv_depth_init, window=i)

    reset()
    b.solve(iters, 0.0)  # capture + first replay
    lat = []
    for _ in range(steps):
        reset()
        t1 = time.perf_counter()
        res, _ = b.solve(iters, 0.0)
        lat.append(time.perf_counter() - t1)
    lat = np.array(lat)
    out.update({"ms_per_batch": round(float(lat.mean()) * 1e3, 3), "windows_per_s": round(nw / float(lat.mean()), 1),
                "batch_latency_ms_p50": round(float(np.percentile(lat, 50)) * 1e3, 3),
                "batch_latency_ms_p99": round(float(np.percentile(lat, 99)) * 1e3, 3),
                "gn_iters_per_s": round(nw * iters / float(lat.mean()), 1),
                "residuals_per_s": round(res.active_residuals / float(lat.mean()), 1)})
    pb = [b.get_params(i) for i in range(nw)]
    b.close()
    # the same windows one context at a time (each its own graph), for the batching gain
    one = []
    err = 0.0
    for i, w in enumerate(wins):
        s = pba.Solver(flags=pba.PBA_FLAG_GRAPH, **kw)
        s.set_scene(w)
        s.solve(iters, 0.0)
        s.set_params(w.poses_init, w.inv_depth_init)
        t1 = time.perf_counter()
        s.solve(iters, 0.0)
        one.append(time.perf_counter() - t1)
        p1, d1 = s.get_params()
        err = max(err, float(np.abs(p1 - pb[i][0]).max()), float(np.abs(d1 / pb[i][1] - 1).max()))
        s.close()
    out["one_window_per_context"] = {"windows": len(one), "ms_per_window": round(float(np.mean(one)) * 1e3, 3),
                                     "window_latency_ms_p50": round(float(np.percentile(one, 50)) * 1e3, 3),
                                     "window_latency_ms_p99": round(float(np.percentile(one, 99)) * 1e3, 3),
                                     "windows_per_s": round(1.0 / float(np.mean(one)), 1)}
    out["batched_vs_single_max_abs_diff"] = err
    return out


def learned_section(pba, train_scenes, sc, n_systems, steps):
    """The learned form: the network is trained on the GPU on block couplings
    of n_systems reduced systems produced by FC iterations of the method on
    the tiny, mid and precision workloads (restarted from seeded perturbations
    of their starts), then PCG with the learned blocks, PCG with block Jacobi
    and the tiled Cholesky solve the 1800 x 1800 reduced system of the learned
    workload (300 frames, 30 hosts x 30000 points) to a relative residual of
    1e-8. The three solutions agree to that residual, so a Gauss-Newton step
    taken with any of them (and the photometric RMSE it reaches) is the same."""
    out = {"workload": "learned: 300 frames 640x480 f32, 3 spheres + box, 30 hosts x 30000 points, 3-level "
                       "pyramid; reduced system 1800 x 1800 FP64 at the start of level 0 (FC linearization)",
           "points": sc.n_points, "observations": sc.n_obs, "reduced_system": 6 * sc.n_frames}
    rng = np.random.default_rng(5)
    Gs, sizes, failed = [], [], []
    t0 = time.perf_counter()
    per = [max(1, n_systems // 10), (n_systems * 7) // 10, n_systems - max(1, n_systems // 10) - (n_systems * 7) // 10]
    for tsc, count in zip(train_scenes, per):
        s = pba.Solver(mode=pba.PBA_FC, precision=pba.PBA_FP32, n_levels=tsc.n_levels, pattern=tsc.pattern,
                       huber_k=tsc.huber_k)
        s.set_scene(tsc)
        got, bad = 0, 0
        while got < count:
            P = tsc.poses_init.copy()
            P[1:, 9:] += 2e-3 * np.abs(tsc.poses_init[1:, 9:]).mean() * rng.normal(size=P[1:, 9:].shape)
            s.set_params(P, tsc.inv_depth_init * (1.0 + 1e-3 * rng.normal(size=tsc.n_points)))
            try:
                for level in reversed(range(tsc.n_levels)):
                    for _ in range(4):
                        if got >= count:
                            break
                        s.iterate(level, 1)
                        Gs.append(s.pc_harvest())
                        got += 1
            except pba.PbaError:  # a start whose reduced system lost definiteness: counted, next start
                bad += 1
                if bad > 100:
                    raise
                continue
        sizes.append(got)
        failed.append(bad)
        s.close()
    G = np.concatenate(Gs)
    out["training"] = {"systems": int(sum(sizes)), "systems_per_workload": {"tiny": sizes[0], "mid": sizes[1],
                                                                               "precision": sizes[2]},
                       "blocks": int(G.shape[0]), "harvest_s": round(time.perf_counter() - t0, 2),
                       "failed_starts": {"tiny": failed[0], "mid": failed[1], "precision": failed[2]}}
    kw = dict(mode=pba.PBA_FC, precision=pba.PBA_FP64, n_levels=sc.n_levels, pattern=sc.pattern, huber_k=sc.huber_k)
    s = pba.Solver(**kw)
    s.set_scene(sc)
    s.pc_init(1)
    rep = s.pc_train(G, steps=steps, batch=1024, lr=1e-3, seed=2)
    out["training"].update({k: rep[k] for k in ("steps", "samples", "first_loss", "final_loss", "jacobi_loss",
                                                 "trained_loss", "ms")})
    s.iterate(0, 1)  # assembles S and b at level 0 (FC linearization at the start)
    res = {}
    xs = {}
    for name, solver in (("cholesky", pba.PBA_SOLVER_CHOL), ("pcg_block_jacobi", pba.PBA_SOLVER_PCG_JACOBI),
                         ("pcg_learned", pba.PBA_SOLVER_PCG_LEARNED),
                         ("pcg_loss_minimizer", pba.PBA_SOLVER_PCG_BLOCKOPT)):
        s.solve_reduced(solver, 1e-8, 20000, want_x=False)  # warm-up
        reps = [s.solve_reduced(solver, 1e-8, 20000, want_x=True) for _ in range(3)]
        r, x = reps[-1]
        res[name] = {"iters": r["iters"], "rel_residual": r["rel_residual"], "fallback": r["fallback"],
                     "ms": round(float(np.median([q[0]["ms"] for q in reps])), 4),
                     "ms_setup": round(float(np.median([q[0]["ms_setup"] for q in reps])), 4)}
        xs[name] = x
    xc = xs["cholesky"]
    for name in ("pcg_block_jacobi", "pcg_learned", "pcg_loss_minimizer"):
        res[name]["rel_error_vs_cholesky"] = float(np.linalg.norm(xs[name] - xc) / np.linalg.norm(xc))
    out["solvers"] = res
    # learned / block Jacobi: below 1 the trained blocks save PCG iterations
    out["learned_over_jacobi_iters"] = round(res["pcg_learned"]["iters"] / max(1, res["pcg_block_jacobi"]["iters"]), 3)
    out["loss_minimizer_over_jacobi_iters"] = round(res["pcg_loss_minimizer"]["iters"]
                                                    / max(1, res["pcg_block_jacobi"]["iters"]), 3)
    out["learned_pcg_vs_cholesky_time"] = round(res["cholesky"]["ms"] / res["pcg_learned"]["ms"], 3)
    s.close()
    return out


def calibrate_copy(nbytes):
    """A device-to-device copy of nbytes (the runtime's copy kernel), so that the
    HBM counters of a profiling run can be scaled by a transfer of known size."""
    import ctypes as C

    hip = C.CDLL("libamdhip64.so")
    a, b = C.c_void_p(), C.c_void_p()
    assert hip.hipMalloc(C.byref(a), C.c_size_t(nbytes)) == 0
    assert hip.hipMalloc(C.byref(b), C.c_size_t(nbytes)) == 0
    assert hip.hipMemset(a, 1, C.c_size_t(nbytes)) == 0
    for _ in range(3):
        assert hip.hipMemcpy(b, a, C.c_size_t(nbytes), 3) == 0  # hipMemcpyDeviceToDevice
    assert hip.hipDeviceSynchronize() == 0
    hip.hipFree(a)
    hip.hipFree(b)
    log(f"copy calibration: 3 device copies of {nbytes} bytes")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--max-iters", type=int, default=10)
    ap.add_argument("--conv-px", type=float, default=5e-3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-trace", action="store_true", help="skip the equal-RMSE sweeps")
    ap.add_argument("--no-event-timing", action="store_true",
                    help="skip the contexts that time kernels with HIP events (the rooflines then read 0)")
    ap.add_argument("--fc-steps", type=int, default=None, help="FC solves to time (default: --steps)")
    ap.add_argument("--no-precision", action="store_true", help="skip the precision-workload section")
    ap.add_argument("--no-oracle-check", action="store_true",
                    help="skip the precision workload's comparison with the FP64 oracle")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-windows section")
    ap.add_argument("--no-frontend", action="store_true", help="skip the front-end (base solution) section")
    ap.add_argument("--no-affine", action="store_true", help="skip the affine-brightness section")
    ap.add_argument("--windows", type=int, default=64, help="windows of the batched section")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner section")
    ap.add_argument("--train-systems", type=int, default=2000, help="reduced systems harvested for training")
    ap.add_argument("--train-steps", type=int, default=2000, help="optimizer steps of the network")
    ap.add_argument("--workers", type=int, default=min(16, len(os.sched_getaffinity(0))),
                    help="processes that build the batched windows")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="also run device copies of BYTES (scale for profiler byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the solver has no multi-GPU path "
              "(points would shard over GPUs with an all-reduce of the FP64 reduced pose system; not built).",
              file=sys.stderr)
        sys.exit(2)

    import scenes

    wins = None
    if not args.no_batched:
        t0 = time.perf_counter()
        wins = make_windows(args.windows, args.workers)
        log(f"{len(wins)} windows built ({time.perf_counter() - t0:.1f} s)")
    precision_scene, oracle_job, oracle_pool = None, None, None
    if not args.no_precision:
        import concurrent.futures as cf
        import multiprocessing as mp

        t0 = time.perf_counter()
        precision_scene = scenes.precision()
        log(f"scene precision: {precision_scene.n_points} points ({time.perf_counter() - t0:.1f} s)")
        if not args.no_oracle_check:
            # the oracle's capped solve runs in a worker (forked before this process
            # touches the GPU) while the GPU sections run
            oracle_pool = cf.ProcessPoolExecutor(max_workers=1, mp_context=mp.get_context("fork"))
            oracle_job = oracle_pool.submit(oracle_ic_capped, precision_scene)
    learned_scene = None
    if not args.no_learned:
        t0 = time.perf_counter()
        learned_scene = scenes.learned()
        log(f"scene learned: {learned_scene.n_points} points ({time.perf_counter() - t0:.1f} s)")
    from paper_1704_06967_amd import pba

    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
    t0 = time.perf_counter()
    scene = scenes.mid()
    log(f"scene mid: {scene.n_points} points, {scene.n_obs} observations, {scene.n_residuals()} residuals "
        f"({time.perf_counter() - t0:.1f} s)")
    kw = dict(precision=pba.PBA_FP32, n_levels=scene.n_levels, pattern=scene.pattern, huber_k=scene.huber_k)
    # the timed solves run as captured graphs (one launch per solve); twin
    # contexts without graphs time the residual kernels with HIP events
    ic = pba.Solver(mode=pba.PBA_IC_PROXY, flags=pba.PBA_FLAG_GRAPH, **kw)
    fc = pba.Solver(mode=pba.PBA_FC, flags=pba.PBA_FLAG_GRAPH, **kw)
    twins = not args.no_event_timing
    ic_ev = pba.Solver(mode=pba.PBA_IC_PROXY, flags=pba.PBA_FLAG_TIMING, **kw) if twins else None
    fc_ev = pba.Solver(mode=pba.PBA_FC, flags=pba.PBA_FLAG_TIMING, **kw) if twins else None
    ctxs = [s for s in (ic, fc, ic_ev, fc_ev) if s is not None]
    for s in ctxs:
        s.set_scene(scene)
    p0, d0 = scene.poses_init, scene.inv_depth_init

    for _ in range(args.warmup):
        for s in ctxs:
            s.set_params(p0, d0)
            s.solve(args.max_iters, args.conv_px)
    zero = {k: [0.0] * 4 for k in ("residual_launches", "residual_ms", "step_launches", "step_ms")}
    if twins:
        ic_ev.timing()
        fc_ev.timing()
    log("warmup done")

    ic_t, ic_iters, ic_active, ic_res = run_steps(ic, p0, d0, args.steps, args.max_iters, args.conv_px)
    log(f"IC: {args.steps} solves, {np.mean(ic_t) * 1e3:.3f} ms each")
    fc_steps = args.fc_steps or args.steps
    fc_t, fc_iters, fc_active, fc_res = run_steps(fc, p0, d0, fc_steps, args.max_iters, args.conv_px)
    log(f"FC: {fc_steps} solves, {np.mean(fc_t) * 1e3:.3f} ms each")
    ic_tm, fc_tm = zero, zero
    if twins:
        run_steps(ic_ev, p0, d0, args.steps, args.max_iters, args.conv_px)
        ic_tm = ic_ev.timing()
        run_steps(fc_ev, p0, d0, fc_steps, args.max_iters, args.conv_px)
        fc_tm = fc_ev.timing()

    total = float(np.sum(ic_t))
    value = ic_iters / total
    ic_res_s = ic_active / total
    fc_total = float(np.sum(fc_t))

    # rooflines of the per-iteration kernels at level 0 (HIP events recorded by
    # each kernel's own dispatch in the event-timed twins); the headline object
    # is the one of the IC kernel with the larger total time over the solves
    nb_res = ic_residual_bytes(scene, 0, 4)
    res_l0 = ic_tm["residual_launches"][0]
    res_ms = ic_tm["residual_ms"][0] / max(1, res_l0)
    rl_res = roofline_obj("k_ic_residual<float> (level 0)", nb_res, res_ms, res_l0, measured_traffic("k_ic_residual", "mid"))
    step_l0 = ic_tm["step_launches"][0]
    step_ms = ic_tm["step_ms"][0] / max(1, step_l0)
    rl_step = roofline_obj("k_ic_step<float> (level 0)", ic_step_bytes(scene, 4), step_ms, step_l0,
                           measured_traffic("k_ic_step", "mid"),
                           note="one launch per iteration: the reduced solve (S^-1 b) and the pose update in "
                                "every workgroup, then each depth workgroup's depth step; bound by dependent "
                                "load latency and the per-CU return rate, not HBM bandwidth")
    fc_l0 = fc_tm["residual_launches"][0]
    fc_ms = fc_tm["residual_ms"][0] / max(1, fc_l0)
    rl_fc = roofline_obj("k_linearize<float, FC> (level 0)", fc_linearize_bytes(scene, 0, 4), fc_ms, fc_l0)
    res_total = sum(ic_tm["residual_ms"])
    step_total = sum(ic_tm["step_ms"])
    roofline = dict(rl_step if step_total > res_total else rl_res)
    roofline["dominant_by"] = (f"total time over the timed IC solves: k_ic_step {step_total:.2f} ms, "
                               f"k_ic_residual {res_total:.2f} ms (all levels)")
    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GN iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "mid: 30 frames 640x480 f32, 360-deg orbit of a value-noise ellipsoid, 3-level "
                               "pyramid, 5 hosts x 4000 points, 8-px patches, Huber 9/255, noise 2/255; "
                               "FP32 residuals/Jacobians, FP64 reductions/Schur/Cholesky",
                   "points": scene.n_points, "observations": scene.n_obs, "residuals_per_iter": scene.n_residuals(),
                   "frames": scene.n_frames, "reduced_system": 6 * scene.n_frames, "max_iters_per_level":
                       args.max_iters, "conv_px": args.conv_px, "mode": "IC-proxy (value), FC (comparison)"},
        "residuals_per_s": round(ic_res_s, 1),
        "ic": {"ms_per_solve": round(np.mean(ic_t) * 1e3, 4), "ms_per_solve_p50": round(np.median(ic_t) * 1e3, 4),
               "iters_per_solve": ic_res[-1]["iters"], "gn_iters_per_s": round(value, 2),
               "residuals_per_s": round(ic_res_s, 1), "final_rmse": ic_res[-1]["final_rmse"]},
        "fc": {"ms_per_solve": round(np.mean(fc_t) * 1e3, 4), "iters_per_solve": fc_res[-1]["iters"],
               "gn_iters_per_s": round(fc_iters / fc_total, 2), "residuals_per_s": round(fc_active / fc_total, 1),
               "final_rmse": fc_res[-1]["final_rmse"],
               "linearize_avg_us_level0": round(fc_tm["residual_ms"][0] / max(1, fc_tm["residual_launches"][0])
                                                * 1e3, 3)},
        "ic_speedup_per_solve": round(np.mean(fc_t) / np.mean(ic_t), 3),
        "roofline": roofline,
        "kernel_rooflines": {"ic_residual": rl_res, "ic_step": rl_step, "fc_linearize": rl_fc},
    }
    if not args.no_trace:
        t0 = time.perf_counter()
        line["equal_rmse"] = equal_rmse_section(pba, scene, pba.PBA_FP32, args.conv_px, args.max_iters)
        log(f"equal RMSE (mid): {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    line["dynamic_hessian"] = dynamic_section(pba, scene)
    log(f"keyframe drop: {line['dynamic_hessian']} ({time.perf_counter() - t0:.1f} s)")
    if not args.no_affine:
        t0 = time.perf_counter()
        line["affine_brightness"] = affine_section(pba, scene)
        log(f"affine brightness: {time.perf_counter() - t0:.1f} s: {line['affine_brightness']}")
    if not args.no_frontend:
        t0 = time.perf_counter()
        line["frontend"] = frontend_section(pba, scene)
        log(f"front end: {time.perf_counter() - t0:.1f} s: {line['frontend']}")
    if not args.no_trace:
        t0 = time.perf_counter()
        line["equal_rmse_converged"] = converged_section(pba, pba.PBA_FP32)
        log(f"converged solves: {time.perf_counter() - t0:.1f} s: {line['equal_rmse_converged']}")
    if not args.no_precision:
        line["precision_form"], precision_scene = precision_section(pba, max(1, min(args.steps, 5)), args.max_iters,
                                                                    args.conv_px, precision_scene,
                                                                    not args.no_event_timing)
        if not args.no_trace:
            t0 = time.perf_counter()
            line["precision_form"]["equal_rmse_fp32"] = equal_rmse_section(pba, precision_scene, pba.PBA_FP32,
                                                                           args.conv_px, args.max_iters,
                                                                           caps=(1, 2, 3, 5, 8, 10, 14, 20))
            log(f"equal RMSE (precision): {time.perf_counter() - t0:.1f} s")
    if learned_scene is not None:
        t0 = time.perf_counter()
        train = [scenes.tiny(), scene, scenes.precision() if args.no_precision else precision_scene]
        line["learned_form"] = learned_section(pba, train, learned_scene, args.train_systems, args.train_steps)
        log(f"learned: {time.perf_counter() - t0:.1f} s")
    if wins is not None:
        line["batched_form"] = batched_section(pba, wins, max(3, min(args.steps, 20)), 5)
        log(f"batched: {line['batched_form']['ms_per_batch']} ms per batch of {len(wins)} windows")
    if oracle_job is not None:
        log("waiting for the oracle's capped solve of the precision workload ...")
        oracle = oracle_job.result()
        oracle_pool.shutdown()
        pf = line["precision_form"]
        pf["vs_oracle"] = {name: errors_vs_oracle(pba, precision_scene, prec, oracle)
                           for name, prec in (("ic_mixed", pba.PBA_MIXED_BF16), ("ic_fp32", pba.PBA_FP32))}
        log(f"precision vs oracle: {pf['vs_oracle']}")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(scene)
    for s in ctxs:
        s.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
