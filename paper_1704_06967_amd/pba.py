"""ctypes binding of libpba (include/pba.h).

Argument marshalling only: every step of the Gauss-Newton path runs in the HIP
library. Importing this module fails loudly when libpba.so has not been built;
there is no fallback implementation.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpba.so")

PBA_OK, PBA_E_INVALID, PBA_E_STATE, PBA_E_OOM, PBA_E_DEVICE, PBA_E_NUMERIC, PBA_E_NOT_CONVERGED = 0, -1, -2, -3, -4, -5, -6
PBA_FC, PBA_IC_PROXY = 0, 1
PBA_FP64, PBA_FP32, PBA_MIXED_BF16 = 0, 1, 2
PBA_SOLVER_CHOL, PBA_SOLVER_PCG_JACOBI, PBA_SOLVER_PCG_LEARNED, PBA_SOLVER_PCG_BLOCKOPT = 0, 1, 2, 3
PBA_PC_N_PARAMS = 77077
PBA_HOST, PBA_DEVICE = 0, 1
PBA_NOALLOC_MAX_N = 768
PBA_FLAG_TIMING, PBA_FLAG_GRAPH, PBA_FLAG_LANE_PER_PIXEL = 1, 2, 4
PBA_MAX_PATTERN = 8
PBA_MAX_LEVELS = 4
PBA_MAX_WINDOWS = 4096
PBA_FE_MAX_CELLS, PBA_FE_MAX_RADIUS = 8192, 5
PBA_TRACK_OK, PBA_TRACK_LOW_TEXTURE, PBA_TRACK_LEFT_IMAGE, PBA_TRACK_FB = 0, 1, 2, 3
PBA_DBG_S, PBA_DBG_B, PBA_DBG_OBS_REC, PBA_DBG_TEMPLATE, PBA_DBG_HDD, PBA_DBG_MASK, PBA_DBG_DTHETA = 1, 2, 3, 4, 5, 6, 7
PBA_DBG_PAIR_H, PBA_DBG_PAIRS = 8, 9
REC_STRIDE = 40


class pba_config(C.Structure):
    _fields_ = [
        ("mode", C.c_int32), ("precision", C.c_int32), ("n_levels", C.c_int32), ("pattern_n", C.c_int32),
        ("pattern_uv", C.c_int32 * (2 * PBA_MAX_PATTERN)), ("huber_k", C.c_double), ("damping_rel", C.c_double),
        ("pinned_frame", C.c_int32), ("solver", C.c_int32), ("n_windows", C.c_int32), ("flags", C.c_int32),
        ("stream", C.c_void_p), ("recentre_every", C.c_int32),
    ]


class pba_iter_stats(C.Structure):
    _fields_ = [
        ("level", C.c_int32), ("iter", C.c_int32), ("n_active", C.c_int64), ("energy", C.c_double),
        ("sq", C.c_double), ("rmse", C.c_double), ("max_disp_px", C.c_double), ("max_step_pose", C.c_double),
        ("max_step_depth", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class pba_result(C.Structure):
    _fields_ = [
        ("iters", C.c_int32 * PBA_MAX_LEVELS), ("total_iters", C.c_int32), ("converged", C.c_int32),
        ("final_energy", C.c_double), ("final_rmse", C.c_double), ("final_active", C.c_int64),
        ("active_residuals", C.c_int64),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["iters"] = list(self.iters)
        return d


class pba_timing(C.Structure):
    _fields_ = [("residual_launches", C.c_int64 * PBA_MAX_LEVELS), ("residual_ms", C.c_double * PBA_MAX_LEVELS),
                ("residuals_processed", C.c_int64 * PBA_MAX_LEVELS), ("step_launches", C.c_int64 * PBA_MAX_LEVELS),
                ("step_ms", C.c_double * PBA_MAX_LEVELS)]


PBA_TUNE_MAX = 16


class pba_tune_report(C.Structure):
    _fields_ = [("n_candidates", C.c_int32), ("block", C.c_int32 * PBA_TUNE_MAX),
                ("grid_mult", C.c_int32 * PBA_TUNE_MAX), ("us", C.c_double * PBA_TUNE_MAX), ("chosen", C.c_int32),
                ("lanes", C.c_int32 * PBA_TUNE_MAX)]

    def as_dict(self):
        n = self.n_candidates

        def shape(i):
            return {"block": self.block[i], "grid_mult": self.grid_mult[i], "lanes": self.lanes[i], "us": self.us[i]}

        return {"candidates": [shape(i) for i in range(n)], "chosen": shape(self.chosen) if n else None}


class pba_train_config(C.Structure):
    _fields_ = [("steps", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("seed", C.c_uint64)]


class pba_train_report(C.Structure):
    _fields_ = [("steps", C.c_int32), ("samples", C.c_int64), ("first_loss", C.c_double), ("final_loss", C.c_double),
                ("jacobi_loss", C.c_double), ("trained_loss", C.c_double), ("ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class pba_reduced_report(C.Structure):
    _fields_ = [("solver", C.c_int32), ("iters", C.c_int32), ("converged", C.c_int32), ("fallback", C.c_int32),
                ("rel_residual", C.c_double), ("ms", C.c_double), ("ms_setup", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PbaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status_string(status)}: {msg}")
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
_lib = C.CDLL(LIB_PATH)

_P = C.c_void_p
_sig = {
    "pba_config_default": (C.c_int, [C.POINTER(pba_config)]),
    "pba_create": (C.c_int, [C.POINTER(pba_config), C.POINTER(_P)]),
    "pba_set_frames": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _P, _P, _P, C.c_int32]),
    "pba_set_points": (C.c_int, [_P, C.c_int32, C.c_int32, _P, _P, _P, _P, _P, C.c_int32]),
    "pba_iterate": (C.c_int, [_P, C.c_int32, C.c_int32, C.POINTER(pba_iter_stats)]),
    "pba_solve": (C.c_int, [_P, C.c_int32, C.c_double, C.POINTER(pba_result)]),
    "pba_evaluate": (C.c_int, [_P, C.c_int32, C.POINTER(pba_iter_stats)]),
    "pba_get_params": (C.c_int, [_P, C.c_int32, _P, _P]),
    "pba_set_params": (C.c_int, [_P, C.c_int32, _P, _P]),
    "pba_drop_frame": (C.c_int, [_P, C.c_int32, C.c_int32]),
    "pba_set_affine": (C.c_int, [_P, _P]),
    "pba_get_affine": (C.c_int, [_P, _P]),
    "pba_fe_corners": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int64, C.c_int32, _P, _P,
                                 C.POINTER(C.c_int32)]),
    "pba_fe_track": (C.c_int, [_P, C.c_int32, C.c_int32, _P, _P, _P, _P, C.c_int32, C.c_int32, C.c_double,
                               C.c_double, _P, _P, _P]),
    "pba_set_tracks": (C.c_int, [_P, C.c_int32, C.c_int32, _P]),
    "pba_geo_solve": (C.c_int, [_P, C.c_int32, C.c_double, C.c_double, C.c_double, _P, C.POINTER(pba_result)]),
    "pba_debug_fetch": (C.c_int, [_P, C.c_int32, _P, C.c_size_t]),
    "pba_get_timing": (C.c_int, [_P, C.POINTER(pba_timing)]),
    "pba_autotune": (C.c_int, [_P, C.c_int32, C.c_int32, C.POINTER(pba_tune_report)]),
    "pba_pc_init": (C.c_int, [_P, C.c_uint64]),
    "pba_pc_set_weights": (C.c_int, [_P, _P, C.c_size_t]),
    "pba_pc_get_weights": (C.c_int, [_P, _P, C.c_size_t]),
    "pba_pc_harvest": (C.c_int, [_P, _P, C.c_size_t, C.POINTER(C.c_int32)]),
    "pba_pc_train": (C.c_int, [_P, C.c_int64, _P, C.POINTER(pba_train_config), C.POINTER(pba_train_report)]),
    "pba_pc_gradient": (C.c_int, [_P, C.c_int32, _P, C.POINTER(C.c_double), _P]),
    "pba_pc_infer": (C.c_int, [_P, C.c_int32, _P, _P]),
    "pba_solve_reduced": (C.c_int, [_P, C.c_int32, C.c_double, C.c_int32, _P, C.POINTER(pba_reduced_report)]),
    "pba_solve_dense_noalloc": (C.c_int, [C.c_int32, _P, _P, _P, _P, _P]),
    "pba_destroy": (None, [_P]),
    "pba_last_error": (C.c_char_p, [_P]),
    "pba_status_string": (C.c_char_p, [C.c_int]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f

EXPORTED = tuple(_sig)


def status_string(s):
    return pba_status_string(s).decode()


def last_error(ctx=None):
    return pba_last_error(ctx).decode()


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def check(status, ctx=None):
    if status != PBA_OK:
        raise PbaError(status, last_error(ctx))
    return status


def default_config(**kw):
    cfg = pba_config()
    check(pba_config_default(C.byref(cfg)))
    for k, v in kw.items():
        if k == "pattern":
            pat = np.asarray(v, np.int32).reshape(-1, 2)
            cfg.pattern_n = pat.shape[0]
            for i, x in enumerate(pat.reshape(-1)):
                cfg.pattern_uv[i] = int(x)
        else:
            setattr(cfg, k, v)
    return cfg


class Solver:
    """One context of the library (marshalling only)."""

    def __init__(self, **cfg_kw):
        self.cfg = default_config(**cfg_kw)
        h = C.c_void_p()
        check(pba_create(C.byref(self.cfg), C.byref(h)))
        self.ctx = h
        self.real = np.float64 if self.cfg.precision == PBA_FP64 else np.float32
        nw = self.cfg.n_windows
        self.Fw, self.Nw, self.Ow = [0] * nw, [0] * nw, [0] * nw
        self._win = [dict() for _ in range(nw)]

    def close(self):
        if self.ctx:
            pba_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, s):
        return check(s, self.ctx)

    @property
    def F(self):
        return sum(self.Fw)

    @property
    def N(self):
        return sum(self.Nw)

    @property
    def O(self):
        return sum(self.Ow)

    def set_frames(self, images, intrinsics, poses, window=0):
        images = np.ascontiguousarray(images, np.float32)
        F, H, W = images.shape
        self._chk(pba_set_frames(self.ctx, window, F, W, H, _ptr(images),
                                 _ptr(np.ascontiguousarray(intrinsics, np.float64)),
                                 _ptr(np.ascontiguousarray(poses, np.float64)), PBA_HOST))
        self.H, self.W = H, W
        self.Fw[window] = F
        self.Nw[window] = self.Ow[window] = 0

    def set_points(self, host_frame, host_uv, inv_depth, obs_ptr, obs_frame, window=0):
        hf = np.ascontiguousarray(host_frame, np.int32)
        optr = np.ascontiguousarray(obs_ptr, np.int32)
        ofr = np.ascontiguousarray(obs_frame, np.int32)
        self._chk(pba_set_points(self.ctx, window, hf.shape[0], _ptr(hf),
                                 _ptr(np.ascontiguousarray(host_uv, np.float32)),
                                 _ptr(np.ascontiguousarray(inv_depth, np.float64)), _ptr(optr), _ptr(ofr), PBA_HOST))
        self.Nw[window], self.Ow[window] = hf.shape[0], int(optr[-1])
        self._win[window] = dict(host_frame=hf, obs_ptr=optr, obs_frame=ofr)

    def set_scene(self, scene, poses=None, inv_depth=None, window=0):
        self.set_frames(scene.images, scene.intrinsics, scene.poses_init if poses is None else poses, window)
        self.set_points(scene.host_frame, scene.host_uv, scene.inv_depth_init if inv_depth is None else inv_depth,
                        scene.obs_ptr, scene.obs_frame, window)

    def iterate(self, level, n_iters):
        st = (pba_iter_stats * max(1, n_iters))()
        self._chk(pba_iterate(self.ctx, level, n_iters, st))
        return [st[i].as_dict() for i in range(n_iters)]

    def solve(self, max_iters_per_level, conv_px=5e-3):
        res = pba_result()
        s = pba_solve(self.ctx, max_iters_per_level, conv_px, C.byref(res))
        if s not in (PBA_OK, PBA_E_NOT_CONVERGED):
            self._chk(s)
        return res, s

    def evaluate(self, level=0):
        st = pba_iter_stats()
        self._chk(pba_evaluate(self.ctx, level, C.byref(st)))
        return st.as_dict()

    def get_params(self, window=0):
        poses = np.zeros((self.Fw[window], 12))
        d = np.zeros(self.Nw[window])
        self._chk(pba_get_params(self.ctx, window, _ptr(poses), _ptr(d)))
        return poses, d

    def set_params(self, poses, inv_depth, window=0):
        self._chk(pba_set_params(self.ctx, window, _ptr(np.ascontiguousarray(poses, np.float64)),
                                 _ptr(np.ascontiguousarray(inv_depth, np.float64))))

    def drop_frame(self, frame, window=0):
        self._chk(pba_drop_frame(self.ctx, window, frame))

    def set_affine(self, ab):
        """Per-frame brightness (a_f, b_f) [F, 2]; turns the brightness model
        on for iterate / solve / evaluate. None turns it off."""
        if ab is None:
            self._chk(pba_set_affine(self.ctx, None))
            return
        ab = np.ascontiguousarray(ab, np.float64).reshape(-1, 2)
        self._chk(pba_set_affine(self.ctx, _ptr(ab)))

    def get_affine(self):
        ab = np.zeros((self.Fw[0], 2))
        self._chk(pba_get_affine(self.ctx, _ptr(ab)))
        return ab

    # ---- front end (corners, tracks, geometric bundle adjustment)

    def corners(self, frame, cell=8, margin=8, min_response=0, max_corners=2000, window=0):
        """(uv [K, 2] int32 as (column, row), response [K] int64), best first."""
        uv = np.zeros((max(1, max_corners), 2), np.int32)
        resp = np.zeros(max(1, max_corners), np.int64)
        n = C.c_int32()
        self._chk(pba_fe_corners(self.ctx, window, frame, cell, margin, int(min_response), max_corners, _ptr(uv),
                                 _ptr(resp), C.byref(n)))
        return uv[: n.value].copy(), resp[: n.value].copy()

    def track(self, host_frame, host_uv, target_frame, guess_uv, radius=4, n_iters=10, min_eig=1e-6, fb_px=0.5,
              window=0):
        """(positions [T, 2], status [T], forward-backward distance [T])."""
        hf = np.ascontiguousarray(host_frame, np.int32).reshape(-1)
        tf = np.ascontiguousarray(target_frame, np.int32).reshape(-1)
        xu = np.ascontiguousarray(host_uv, np.float64).reshape(-1, 2)
        gu = np.ascontiguousarray(guess_uv, np.float64).reshape(-1, 2)
        n = hf.shape[0]
        out = np.zeros((n, 2))
        st = np.zeros(n, np.int32)
        fb = np.zeros(n)
        self._chk(pba_fe_track(self.ctx, window, n, _ptr(hf), _ptr(xu), _ptr(tf), _ptr(gu), radius, n_iters,
                               min_eig, fb_px, _ptr(out), _ptr(st), _ptr(fb)))
        return out, st, fb

    def set_tracks(self, obs_uv, window=0):
        z = np.ascontiguousarray(obs_uv, np.float64).reshape(-1, 2)
        self._chk(pba_set_tracks(self.ctx, window, z.shape[0], _ptr(z)))

    def geo_solve(self, max_iters, conv_px=5e-3, huber_px=2.0, outlier_px=0.0):
        """(pba_result, status, inliers [O] uint8); PBA_E_NOT_CONVERGED is returned, not raised."""
        res = pba_result()
        inl = np.zeros(max(1, self.O), np.uint8)
        s = pba_geo_solve(self.ctx, max_iters, conv_px, huber_px, outlier_px, _ptr(inl), C.byref(res))
        if s not in (PBA_OK, PBA_E_NOT_CONVERGED):
            self._chk(s)
        return res, s, inl[: self.O].copy()

    def fetch(self, what):
        n6 = 6 * self.F
        s_shape = (n6, n6) if len(self.Fw) == 1 else (sum(36 * f * f for f in self.Fw),)
        shapes = {
            PBA_DBG_S: (s_shape, np.float64), PBA_DBG_B: ((n6,), np.float64),
            PBA_DBG_OBS_REC: ((self.O, REC_STRIDE), np.float64),
            PBA_DBG_TEMPLATE: ((self.N, self.cfg.pattern_n, 4), self.real),
            PBA_DBG_HDD: ((self.N,), np.float64), PBA_DBG_MASK: ((self.O,), np.uint8),
            PBA_DBG_DTHETA: ((n6,), np.float64),
            PBA_DBG_PAIR_H: lambda: ((self.n_pairs(), 21), np.float64),
            PBA_DBG_PAIRS: lambda: ((self.n_pairs(), 2), np.int32),
        }
        shape, dt = shapes[what]() if callable(shapes[what]) else shapes[what]
        out = np.zeros(shape, dt)
        self._chk(pba_debug_fetch(self.ctx, what, _ptr(out), out.nbytes))
        return out

    def n_pairs(self):
        total = 0
        for w in self._win:
            if not w:
                continue
            host = np.repeat(w["host_frame"].astype(np.int64), np.diff(w["obs_ptr"]))
            total += int(np.unique(host * (1 << 31) + w["obs_frame"]).size)
        return total

    def autotune(self, level=0, reps=20):
        rep = pba_tune_report()
        self._chk(pba_autotune(self.ctx, level, reps, C.byref(rep)))
        return rep.as_dict()

    # ---- learned preconditioner and reduced-system solvers
    def pc_init(self, seed=0):
        self._chk(pba_pc_init(self.ctx, seed))

    def pc_set_weights(self, w):
        w = np.ascontiguousarray(w, np.float32)
        self._chk(pba_pc_set_weights(self.ctx, _ptr(w), w.size))

    def pc_get_weights(self):
        w = np.zeros(PBA_PC_N_PARAMS, np.float32)
        self._chk(pba_pc_get_weights(self.ctx, _ptr(w), w.size))
        return w

    def pc_harvest(self):
        G = np.zeros((self.F, 21), np.float32)
        nb = C.c_int32()
        self._chk(pba_pc_harvest(self.ctx, _ptr(G), G.size, C.byref(nb)))
        return G[:nb.value]

    def pc_train(self, G, steps=2000, batch=1024, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, seed=0):
        G = np.ascontiguousarray(G, np.float32).reshape(-1, 21)
        cfg = pba_train_config(steps, batch, lr, beta1, beta2, eps, seed)
        rep = pba_train_report()
        self._chk(pba_pc_train(self.ctx, G.shape[0], _ptr(G), C.byref(cfg), C.byref(rep)))
        return rep.as_dict()

    def pc_gradient(self, G):
        G = np.ascontiguousarray(G, np.float32).reshape(-1, 21)
        loss = C.c_double()
        grad = np.zeros(PBA_PC_N_PARAMS, np.float32)
        self._chk(pba_pc_gradient(self.ctx, G.shape[0], _ptr(G), C.byref(loss), _ptr(grad)))
        return loss.value, grad

    def pc_infer(self, G):
        G = np.ascontiguousarray(G, np.float32).reshape(-1, 21)
        Y = np.zeros((G.shape[0], 21), np.float32)
        self._chk(pba_pc_infer(self.ctx, G.shape[0], _ptr(G), _ptr(Y)))
        return Y

    def solve_reduced(self, solver, tol=1e-8, max_iters=5000, want_x=True):
        x = np.zeros(6 * self.F) if want_x else None
        rep = pba_reduced_report()
        self._chk(pba_solve_reduced(self.ctx, solver, tol, max_iters, _ptr(x), C.byref(rep)))
        return rep.as_dict(), x

    def timing(self):
        t = pba_timing()
        self._chk(pba_get_timing(self.ctx, C.byref(t)))
        return {k: list(getattr(t, k)) for k, _ in t._fields_}
