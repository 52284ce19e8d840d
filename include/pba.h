/*
 * pba.h - C ABI of libpba, photometric bundle adjustment on one MI355X (gfx950).
 *
 * The library runs the Gauss-Newton iteration of photometric bundle adjustment
 * over 6-DoF frame poses and per-point inverse depths (Ham, Lucey & Singh,
 * "Proxy Templates for Inverse Compositional Photometric Bundle Adjustment",
 * arXiv 1704.06967), in two forms:
 *   - forward compositional (FC): the Jacobian and the Hessian are rebuilt and
 *     factorized at every iteration (the paper's baseline, Sec. 1-2);
 *   - inverse compositional with proxy templates (IC): the Jacobian (Sec. 3.4,
 *     3.5) and H = J^T W0 J are built once per pyramid level; each iteration
 *     recomputes the Huber weights, forms g = J^T W r, solves dp = -H^{-1} g and
 *     composes the warps (Sec. 3.5 steps 1-4, Sec. 3.6 update equations).
 *
 * Problem (eq:energy, eq:warp): frames f with images I_f and world->camera
 * poses (R_f, t_f); points n with a host frame h(n), a host pixel, one inverse
 * depth d_n shared by the points' patch pixels, and the list of frames that
 * observe them. One residual per (point, observing frame, patch pixel):
 *   r = I_h(x) - I_f(W(x; p)),  W(x; p) = <R x~ + d t>,
 * with (R, t) the pose of f relative to h. Images are bilinear functions
 * (Notation); the energy is the Huber norm of the residuals (eq:energy).
 *
 * Conventions (the paper states none):
 *   - pixel centres at integer coordinates, u = column, v = row;
 *   - intrinsics per frame (fx, fy, cx, cy) at level 0; level l uses f / 2^l
 *     and (c + 0.5) / 2^l - 0.5; level l+1 is the 2x2 box average of level l;
 *   - a pose is 12 doubles: R row-major, then t (X_cam = R X_world + t);
 *   - pose increments are decoupled left increments R <- exp(w) R, t <- t + dt,
 *     ordered (w_x, w_y, w_z, t_x, t_y, t_z);
 *   - a residual is usable when its host pattern pixel and its target pixel lie
 *     in [1, W_l - 3] x [1, H_l - 3], the point is in front of the target
 *     camera and d > 0. The usable set is frozen at the start of a level; a
 *     frozen residual that leaves the image later gets weight 0;
 *   - the reduced pose system pins one frame (identity rows, zero rhs) and
 *     damps pose and depth diagonals by damping_rel times their mean.
 *
 * Ownership: pba_set_* deep-copy their inputs (host or device memory, per the
 * `mem` argument); the caller may free them on return. Output buffers are owned
 * by the caller. The context owns every device buffer it allocates.
 *
 * Errors: every entry point returns a pba_status; nothing aborts or throws
 * across the ABI. Arguments are validated before any device work; on error the
 * context state is unchanged and pba_last_error() describes the cause.
 *
 * Calls on one context are synchronous with respect to the host (they return
 * after the device work they enqueue has finished). One context must not be
 * used from two threads at once; distinct contexts are independent.
 */
#ifndef PBA_H
#define PBA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pba_ctx pba_ctx;

typedef enum {
    PBA_OK = 0,
    PBA_E_INVALID = -1,      /* an argument is out of range or inconsistent */
    PBA_E_STATE = -2,        /* call out of order (e.g. iterate before set_points) */
    PBA_E_OOM = -3,          /* device allocation failed */
    PBA_E_DEVICE = -4,       /* no usable gfx950 device, or a HIP call failed */
    PBA_E_NUMERIC = -5,      /* reduced system not positive definite; parameters unchanged */
    PBA_E_NOT_CONVERGED = -6 /* pba_solve hit its iteration cap on the finest level */
} pba_status;

enum { PBA_FC = 0, PBA_IC_PROXY = 1 };                        /* pba_config.mode */
enum { PBA_FP64 = 0, PBA_FP32 = 1, PBA_MIXED_BF16 = 2 };      /* pba_config.precision */
/* reduced solvers; PBA_SOLVER_PCG_BLOCKOPT: PCG with the blocks that minimize the learned
 * preconditioner's training loss exactly, P^_i = (I + G_i)^{-1} (the bound of any network) */
enum { PBA_SOLVER_CHOL = 0, PBA_SOLVER_PCG_JACOBI = 1, PBA_SOLVER_PCG_LEARNED = 2, PBA_SOLVER_PCG_BLOCKOPT = 3 };
enum { PBA_HOST = 0, PBA_DEVICE = 1 };                        /* memory of input pointers */
enum { PBA_FLAG_TIMING = 1, PBA_FLAG_GRAPH = 2, PBA_FLAG_LANE_PER_PIXEL = 4 };   /* pba_config.flags */

#define PBA_MAX_PATTERN 8
#define PBA_MAX_LEVELS 4
#define PBA_MAX_WINDOWS 4096

typedef struct {
    int32_t mode;        /* PBA_FC or PBA_IC_PROXY */
    int32_t precision;   /* PBA_FP64: all arithmetic in double. PBA_FP32: images,
                            template, residuals r, Huber weights and Jacobians in
                            float; the warp and projection of every patch pixel, the
                            bilinear interpolants of intensity and gradient (r and
                            the forward-compositional Jacobian row are rounded to
                            float once), the per-observation sums of products
                            (stored as double), reductions, Schur complement and
                            Cholesky in double. PBA_MIXED_BF16: as PBA_FP32, except
                            that every pair's pose-pose block sum w J^T J is
                            contracted on BF16 MFMA: sqrt(w) J on a fixed-point grid
                            per 64 residuals (four exact bfloat16 terms), FP32
                            accumulation that is exact on that grid, double sums
                            across groups; h and H_dd are double sums over the same
                            rows */
    int32_t n_levels;    /* image pyramid levels, 1..PBA_MAX_LEVELS */
    int32_t pattern_n;   /* patch pixels per point, 1..PBA_MAX_PATTERN */
    int32_t pattern_uv[2 * PBA_MAX_PATTERN]; /* (du, dv) offsets in level pixels, |du|,|dv| <= 4 */
    double huber_k;      /* Huber threshold in intensity units (> 0; +inf = least squares) */
    double damping_rel;  /* diagonal damping relative to the mean diagonal (>= 0) */
    int32_t pinned_frame;/* frame whose pose is held fixed (gauge), or -1 */
    int32_t solver;      /* PBA_SOLVER_CHOL (the Gauss-Newton iterations factor or invert S) */
    int32_t n_windows;   /* independent problems (windows) held by the context,
                            1..PBA_MAX_WINDOWS. With n_windows > 1 (batched form) every
                            window has its own frames, points, pinned frame (the index
                            pinned_frame within the window) and damping, all windows
                            have the same image size and at most 30 frames each, and
                            they are solved together: one launch per step over all
                            windows, a block-diagonal reduced system */
    int32_t flags;       /* PBA_FLAG_TIMING: time the per-iteration residual kernel
                            (with pba_set_affine: the joint linearization)
                            with HIP events (read with pba_get_timing; not recorded
                            while PBA_FLAG_GRAPH replays a graph).
                            PBA_FLAG_GRAPH: pba_solve captures its whole coarse-to-fine
                            solve (every level start and max_iters gated iterations)
                            as one HIP graph on the context's stream at its first
                            call and replays it on later calls with the same
                            max_iters and conv_px; the graph is dropped (and captured
                            again when needed) when points are set, when max_iters
                            or conv_px change, when pba_autotune picks a launch
                            shape, and when pba_set_affine turns the brightness
                            model on or off. pba_iterate never uses the graph.
                            PBA_FLAG_LANE_PER_PIXEL: the IC residual pass starts with
                            one lane per patch pixel (8 per observation) instead of one
                            thread per observation (pba_autotune may pick either); the
                            two add an observation's pixel products in different
                            orders, so results agree to the rounding of those FP64
                            sums */
    void *stream;        /* hipStream_t to run on, or NULL for a library-owned stream */
    int32_t recentre_every; /* proxy re-centring (Sec. 3.6: the proxy update holds near
                            p(0)): with m > 0, IC re-linearizes after every m
                            iterations of a level, with p(0) the current parameters (J,
                            W0, H, S and S^-1 formed again, as at a level start); within
                            pba_solve's device schedule, captured graphs included, and
                            across pba_iterate calls. 0 (default): the paper's IC.
                            0..1000; ignored by FC */
} pba_config;

typedef struct {
    int32_t level;          /* pyramid level of this iteration */
    int32_t iter;           /* iteration index within the level */
    int64_t n_active;       /* residuals that contributed (weight > 0) */
    double energy;          /* sum of Huber norms at the parameters the iteration started from */
    double sq;              /* sum of squared residuals over the same set */
    double rmse;            /* sqrt(sq / n_active) */
    double max_disp_px;     /* largest level-0 displacement of any observation's point
                               centre caused by this iteration's update (Sec. 4.1 test) */
    double max_step_pose;   /* max |dtheta| over all frames and components */
    double max_step_depth;  /* max |dd| over all points */
} pba_iter_stats;

typedef struct {
    int32_t iters[PBA_MAX_LEVELS]; /* iterations run per level (index = level) */
    int32_t total_iters;
    int32_t converged;             /* 1 if the finest level met conv_px */
    double final_energy;           /* at the returned parameters, level 0, fresh usable set */
    double final_rmse;
    int64_t final_active;
    int64_t active_residuals;      /* sum over the iterations that ran of their n_active */
} pba_result;

typedef struct {
    /* per pyramid level, launches of the per-iteration residual kernel (IC: the
       residual / J^T W r kernel; FC: the linearization kernel) that did work */
    int64_t residual_launches[PBA_MAX_LEVELS];
    double residual_ms[PBA_MAX_LEVELS];         /* their summed duration (HIP events on the
                                                   context's stream; needs PBA_FLAG_TIMING) */
    int64_t residuals_processed[PBA_MAX_LEVELS];/* residual slots those launches covered */
    /* IC on one window with the fused step (solve and depth update in one launch per
       iteration): launches of that step kernel that did work and their summed duration;
       0 on the other paths */
    int64_t step_launches[PBA_MAX_LEVELS];
    double step_ms[PBA_MAX_LEVELS];
} pba_timing;

/* Debug / verification buffers for pba_debug_fetch (element type in brackets;
 * "real" is double for PBA_FP64, float otherwise). */
enum {
    PBA_DBG_S = 1,          /* [double 6F x 6F] damped, pinned Schur complement of the last
                               system assembled (row-major); for 6F > 192 the buffer holds
                               its Cholesky factor (lower triangle) once it has been factored */
    PBA_DBG_B = 2,          /* [double 6F] reduced right-hand side of the last iteration */
    PBA_DBG_OBS_REC = 3,    /* [double O x 40] per-observation blocks: 0-20 upper triangle of
                               sum w J_th^T J_th (row-major), 21-26 sum w J_th J_d, 27 sum w J_d^2,
                               28-33 sum w J_th r, 34 sum w J_d r, 35 energy, 36 sum r^2,
                               37 active count (relative-pose coordinates). IC: the linearization
                               at p(0) (the iterations keep g, g_d and the statistics in a
                               compact buffer of their own) */
    PBA_DBG_TEMPLATE = 4,   /* [real N x P x 4] (I0, dI0/du, dI0/dv, usable) at the current level */
    PBA_DBG_HDD = 5,        /* [double N] damped depth diagonal of the last system */
    PBA_DBG_MASK = 6,       /* [uint8 O] bit j set if patch pixel j is in the frozen usable set */
    PBA_DBG_DTHETA = 7,     /* [double 6F] pose step of the last iteration */
    PBA_DBG_PAIR_H = 8,     /* [double Pn x 21] per (host, target) pair: upper triangle of the
                               pose-pose block sum w J_th^T J_th in relative coordinates, as
                               last assembled */
    PBA_DBG_PAIRS = 9       /* [int32 Pn x 2] (host frame, target frame) of every pair */
};

/* Fill *cfg with defaults: IC, FP32, 1 level, the 8-pixel diamond pattern
 * {(0,0),(0,-2),(-1,-1),(1,-1),(-2,0),(2,0),(-1,1),(1,1)}, Huber 9/255,
 * damping 1e-6, frame 0 pinned, Cholesky, one window, no flags, own stream. */
pba_status pba_config_default(pba_config *cfg);

/* Create a context on the current HIP device (must be gfx950). Validates *cfg. */
pba_status pba_create(const pba_config *cfg, pba_ctx **out);

/* Define the frames of window `window` (0..n_windows-1): n_frames images of
 * width x height pixels (images [F][H][W] float32, row-major), intrinsics [F][4]
 * (fx, fy, cx, cy, level-0 pixels), poses [F][12] world->camera (Sec. 1: the
 * SE(3) pose of each frame; frame indices are local to the window). Resets any
 * points previously set on that window. Width and height must be
 * >= 8 * 2^(n_levels-1); in a batched context every window has the same size and
 * at most 30 frames. A batched context assembles its windows on the first call
 * that needs them. */
pba_status pba_set_frames(pba_ctx *ctx, int32_t window, int32_t n_frames, int32_t width, int32_t height,
                          const float *images, const double *intrinsics, const double *poses, int32_t mem);

/* Define the points of window `window` (0..n_windows-1), Sec. 3 eq:energy: host_frame
 * [N], host_uv [N][2] (level-0 pixel of the point centre), inv_depth [N] (> 0, one
 * per point, shared by its patch pixels), and the observing frames in CSR form
 * (obs_ptr [N+1], obs_frame [O]; per point strictly increasing, never the host).
 * A host frame may have at most 20 distinct target frames. These parameters
 * become the starting point of the next level. */
pba_status pba_set_points(pba_ctx *ctx, int32_t window, int32_t n_points, const int32_t *host_frame,
                          const float *host_uv, const double *inv_depth, const int32_t *obs_ptr,
                          const int32_t *obs_frame, int32_t mem);

/* Run exactly n_iters Gauss-Newton iterations on pyramid `level` (all windows).
 * If the context's current level differs (or parameters were set since), the
 * level starts over: p(0) := current parameters, usable set frozen, and in IC
 * mode the constant system of Sec. 3.4-3.5 (proxy Jacobian, W0, H = J^T W0 J, the
 * depth Schur complement and its factorization) is built once. Each IC iteration
 * is Sec. 3.5 steps 1-4 (Huber weights at the current residuals, g = J^T W r,
 * dp = -H^{-1} g) followed by the update equations of Sec. 3.6; each FC iteration
 * rebuilds J and H at the current parameters and applies R <- exp(dw) R,
 * t <- t + dt, d <- d + dd (Sec. 1-2). stats: n_iters entries or NULL (statistics
 * summed over the windows). PBA_E_NUMERIC: the reduced system lost definiteness;
 * the parameters stay at the last good iterate. */
pba_status pba_iterate(pba_ctx *ctx, int32_t level, int32_t n_iters, pba_iter_stats *stats);

/* Coarse-to-fine solve: for each level from n_levels-1 down to 0, start the
 * level and iterate (as pba_iterate) until max_disp_px < conv_px or
 * max_iters_per_level iterations. The test is the convergence criterion of
 * Sec. 4.1 (largest level-0 pixel displacement of the reprojected point centres
 * caused by one update; the paper uses 5e-3 px); conv_px < 0 runs every
 * iteration. In a batched context the test applies to all windows together.
 * Returns PBA_E_NOT_CONVERGED (with *out filled and parameters updated) if level
 * 0 did not converge. */
pba_status pba_solve(pba_ctx *ctx, int32_t max_iters_per_level, double conv_px, pba_result *out);

/* Energy / RMSE at the current parameters on `level` over the residuals usable
 * at those parameters (not the frozen set). Fills level, n_active, energy, sq, rmse. */
pba_status pba_evaluate(pba_ctx *ctx, int32_t level, pba_iter_stats *out);

/* Copy the current parameters of window `window` out (host memory): poses [F][12],
 * inv_depth [N]. */
pba_status pba_get_params(pba_ctx *ctx, int32_t window, double *poses, double *inv_depth);

/* Overwrite the current parameters of window `window` (host memory); the next
 * iterate restarts the level. */
pba_status pba_set_params(pba_ctx *ctx, int32_t window, const double *poses, const double *inv_depth);

/* Sliding window, keyframe drop (Sec. 4.2: in the DSO integration every
 * change of the keyframe set still cost a new Hessian; a dynamic Hessian is
 * named as the next speed-up). Takes frame `frame` (0..frames of the window - 1, not the
 * pinned frame) of window `window` out of the window: every observation of a
 * point that the frame hosts and every observation whose target it is. The
 * frame keeps its pose and the points keep their depths, no longer
 * constrained (their steps are zero); iteration statistics, the convergence
 * test and pba_evaluate skip the dropped observations from now on. Within an
 * IC level the reduced system is formed again without a new linearization:
 * the pair blocks, h and H_dd are summed from the per-observation records kept
 * at the level's p(0), then the depth Schur complement, its Cholesky factor
 * and inverse (PBA_MIXED_BF16, whose pose blocks come from its MFMA
 * contraction, linearizes again at p(0)); the result equals the level's set-up
 * at p(0) of the problem without those observations. FC takes the drop at its
 * next iteration. A dropped frame cannot come back (set the points again).
 * Synchronous. Errors: PBA_E_INVALID (window, frame or pinned frame),
 * PBA_E_STATE (frames or points not set), PBA_E_NUMERIC (the new reduced
 * system is not positive definite). */
pba_status pba_drop_frame(pba_ctx *ctx, int32_t window, int32_t frame);

/* Per-frame affine brightness in the FC iteration. The method assumes
 * brightness constancy (Sec. 3, eq:energy); its prior-art discussion (Sec. 2)
 * notes that direct methods elsewhere model the photometric response
 * explicitly. Model (a reading; the paper gives none): frame f has a log-gain
 * a_f and an offset b_f, and the residual of a patch pixel of a point hosted
 * by h and observed by f is
 *     r = I_h(x) - b_h - e^{a_h - a_f} (I_f(W(x; p)) - b_f),
 * the paper's residual at a = b = 0. pba_set_affine(ctx, ab) with ab = host
 * double [F][2] (a_f, b_f per frame, level-independent) turns the model on:
 * from then on pba_iterate, pba_solve and pba_evaluate of this context run
 * the joint Gauss-Newton iteration over 6 pose and 2 brightness parameters
 * per frame and the inverse depths (the depths eliminated by their Schur
 * complement, the 8F x 8F system solved by Cholesky, all in FP64; the pinned
 * frame keeps its pose and brightness; the brightness block is damped by
 * damping_rel times the mean of its diagonal; the brightness update is
 * additive), the iterations of a call enqueued with one host synchronization
 * at the end (pba_solve: its whole coarse-to-fine schedule, a device gate
 * stopping each level at conv_px, captured as one HIP graph with
 * PBA_FLAG_GRAPH). The frozen residual
 * set, Huber weights, pose and depth damping and the convergence test are the
 * FC iteration's. ab = NULL turns the model off (the parameters are kept for
 * pba_get_affine). Needs mode PBA_FC, precision PBA_FP64 or PBA_FP32 and one
 * window; pba_set_frames with another frame count resets the brightness to
 * zero. Errors: PBA_E_INVALID (mode, precision, windows, non-finite values),
 * PBA_E_STATE (frames or points not set); pba_iterate and pba_solve return
 * PBA_E_NUMERIC when the joint system is not positive definite (the
 * failing iteration leaves the parameters as the previous one left them, and
 * the level stops there). */
pba_status pba_set_affine(pba_ctx *ctx, const double *ab);
/* The current brightness parameters, host double [F][2] (zeros before
 * pba_set_affine). Errors: PBA_E_INVALID (ab NULL), PBA_E_STATE (no frames). */
pba_status pba_get_affine(pba_ctx *ctx, double *ab);

/* ---- Front end for p(0): the first three steps of the base solution of
 * Sec. 4.1 (Harris corners, robust KLT tracking, geometric bundle adjustment
 * with outlier removal). Its fourth step, the forward-compositional
 * photometric bundle adjustment, is pba_solve on a PBA_FC context. The paper
 * names the methods and gives no parameters; the readings are stated per
 * call. All arrays of these calls are host memory, owned by the caller. */

#define PBA_FE_MAX_CELLS 8192   /* corner cells per image that one call takes */
#define PBA_FE_MAX_RADIUS 5     /* tracking window of at most 11 x 11 pixels */

/* Harris corners of level 0 of frame `frame` of window `window` (after
 * pba_set_frames). The image is quantized to 8 bits (rint(I * 255) in single
 * precision, clamped to 0..255); gx, gy are the central differences times
 * two; Sxx, Syy, Sxy their products summed over a 5 x 5 box; the response
 * R = 16 (Sxx Syy - Sxy^2) - (Sxx + Syy)^2 (kappa = 1/16, scaled by 16) is an
 * exact integer. A candidate lies at least max(margin, 4) pixels inside the
 * image, has R > min_response and is a 3 x 3 maximum (strictly above the
 * neighbours before it in raster order, not below those after it). Each cell
 * of cell x cell pixels (2..16) keeps its best candidate (largest R, then
 * first in raster order), and the max_corners best cells come back, best
 * first: uv [max_corners][2] (column, row), response [max_corners] (may be
 * NULL), *n_out their number. The image may hold at most PBA_FE_MAX_CELLS
 * cells. Synchronous. Errors: PBA_E_INVALID (ranges, NULL outputs),
 * PBA_E_STATE (no frames), PBA_E_DEVICE / PBA_E_OOM. */
pba_status pba_fe_corners(pba_ctx *ctx, int32_t window, int32_t frame, int32_t cell, int32_t margin,
                          int64_t min_response, int32_t max_corners, int32_t *uv, int64_t *response,
                          int32_t *n_out);

/* Track status codes of pba_fe_track. */
#define PBA_TRACK_OK 0
#define PBA_TRACK_LOW_TEXTURE 1   /* smaller eigenvalue of H / window pixels below min_eig */
#define PBA_TRACK_LEFT_IMAGE 2    /* a window left the usable area u in [1, W-3], v in [1, H-3] */
#define PBA_TRACK_FB 3            /* tracked back, it missed the start by more than fb_px */

/* Robust tracks of n points: the window of (2 radius + 1)^2 pixels around
 * host_uv[i] (level-0 pixels) in frame host_frame[i] into frame
 * target_frame[i] of window `window`, from the predicted level-0 position
 * guess_uv[i]. Translational Lucas-Kanade in inverse-compositional form over
 * the context's pyramid, coarsest level first (the displacement doubles from
 * one level to the next): per level the window's bilinear intensities T and
 * gradients G in the host (central differences, bilinearly interpolated),
 * H = sum G G^T, then n_iters updates d <- d - H^{-1} sum G (I_target(x + d) - T).
 * The position found is tracked back into the host the same way; the track is
 * kept if that returns within fb_px. FP64 arithmetic on the context's images.
 * Outputs: uv_out [n][2] (level-0 position in the target), status_out [n]
 * (PBA_TRACK_*), fb_out [n] (forward-backward distance; may be NULL).
 * radius 1..PBA_FE_MAX_RADIUS, n_iters 1..100. Synchronous. Errors:
 * PBA_E_INVALID (ranges, non-finite positions, NULL arrays), PBA_E_STATE,
 * PBA_E_DEVICE / PBA_E_OOM. */
pba_status pba_fe_track(pba_ctx *ctx, int32_t window, int32_t n, const int32_t *host_frame, const double *host_uv,
                        const int32_t *target_frame, const double *guess_uv, int32_t radius, int32_t n_iters,
                        double min_eig, double fb_px, double *uv_out, int32_t *status_out, double *fb_out);

/* The tracked level-0 position of every observation of pba_set_points
 * (obs_uv [n_obs][2], the CSR order of that call), for pba_geo_solve.
 * One-window contexts only (window 0). Errors: PBA_E_INVALID (window, n_obs
 * not the observation count, non-finite), PBA_E_STATE (no points). */
pba_status pba_set_tracks(pba_ctx *ctx, int32_t window, int32_t n_obs, const double *obs_uv);

/* Geometric bundle adjustment of the poses and inverse depths from the
 * current parameters: one 2-D residual e = pi_f(R x~ + d t) - z per
 * observation (level-0 pixels; the relative pose and inverse depth of
 * eq:warp; z its pba_set_tracks position), the Huber weight of |e| with
 * threshold huber_px on both rows, and otherwise the FC iteration: its
 * normal equations, gauge pin, damping, depth Schur complement, Cholesky,
 * update and convergence test (largest point-centre displacement below
 * conv_px, at most max_iters iterations). With outlier_px > 0 the
 * observations whose |e| exceeds it (or whose point lies behind the camera)
 * are then removed and the solve runs again. The context keeps the result
 * as its parameters. out->iters[0] / [1]: iterations of the two passes;
 * final_energy / final_rmse / final_active: Huber energy, RMS reprojection
 * error (pixels) and count of the inliers at the end; inliers [n_obs] (may
 * be NULL): 1 for the observations kept. Synchronous. Errors: PBA_E_STATE
 * (no tracks), PBA_E_INVALID, PBA_E_NUMERIC (reduced system not positive
 * definite), PBA_E_NOT_CONVERGED (the last pass hit max_iters; parameters
 * and outputs are still written). */
pba_status pba_geo_solve(pba_ctx *ctx, int32_t max_iters, double conv_px, double huber_px, double outlier_px,
                         uint8_t *inliers, pba_result *out);

/* Result of pba_autotune: the launch shapes tried for the per-iteration
 * residual kernel (IC: the residual / J^T W r kernel; FC: the linearization
 * kernel) and their measured mean launch time. */
#define PBA_TUNE_MAX 16
typedef struct {
    int32_t n_candidates;
    int32_t block[PBA_TUNE_MAX];     /* threads per workgroup (tiles of block / lanes observations) */
    int32_t grid_mult[PBA_TUNE_MAX]; /* 0: one tile per workgroup; m > 0: persistent grid of m
                                        workgroups per compute unit striding over the tiles */
    double us[PBA_TUNE_MAX];         /* mean time per launch (microseconds, HIP events) */
    int32_t chosen;                  /* index of the fastest, now used by the context */
    int32_t lanes[PBA_TUNE_MAX];     /* threads per observation: IC 1 (one thread runs the
                                        observation's patch pixels) or 8 (one per pixel; the
                                        sums agree to the rounding of FP64 sums of 8 terms);
                                        FC 8 */
} pba_tune_report;

/* Project autotuner: (re)starts `level` at the current parameters, times every
 * candidate launch shape of the per-iteration residual kernel over `reps`
 * launches on the context's own data, and keeps the fastest for all later
 * iterations (a captured solve graph is rebuilt). The timed launches only
 * rewrite per-observation sums that the next iteration recomputes. `out` may
 * be NULL. PBA_MIXED_BF16 in FC mode has a fixed shape (n_candidates = 0). */
pba_status pba_autotune(pba_ctx *ctx, int32_t level, int32_t reps, pba_tune_report *out);

/* ---- Learned block preconditioner for PCG on the reduced pose system (project-defined: the
 * paper inverts or factorizes the reduced system). Block whitening: S_ii = C_i C_i^T,
 * S^_ij = C_i^{-1} S_ij C_j^{-T}, coupling G_i = sum_{j != i} S^_ij S^_ij^T (6x6, stored as its
 * upper triangle, row-major, 21 floats). Features of block i: upper(G_i) / (1 + tr G_i) and
 * log(1 + tr G_i). Network 22 -> 256 -> 256 -> 21 (ReLU), weights packed as W1 [256][22], b1,
 * W2 [256][256], b2, W3 [21][256], b3 (PBA_PC_N_PARAMS floats). Output y: lower factor L of
 * a 6x6 (row-major lower triangle, exp on the diagonal); block of M^{-1}:
 * C_i^{-T} L L^T C_i^{-1} (y = 0: block Jacobi). Training loss of a block:
 * tr(P A P) - 2 tr(P) + 6 with P = L L^T, A = I + G_i (mean over a batch). Inference runs in
 * FP16 on MFMA, training in FP32 with Adam, PCG in FP64. One window only (n_windows = 1). */
#define PBA_PC_N_PARAMS 77077

typedef struct {
    int32_t steps;                /* optimizer steps */
    int32_t batch;                /* blocks per step, 1..65536 */
    float lr, beta1, beta2, eps;  /* Adam */
    uint64_t seed;                /* order of the samples (reshuffled every pass) */
} pba_train_config;

typedef struct {
    int32_t steps;
    int64_t samples;
    double first_loss, final_loss; /* mean block loss of the first and the last batch */
    double jacobi_loss;            /* mean loss of block Jacobi (y = 0) over all samples: mean tr G */
    double trained_loss;           /* mean loss of the trained network (FP32) over all samples */
    double ms;                     /* GPU time of the optimizer steps */
} pba_train_report;

typedef struct {
    int32_t solver;        /* PBA_SOLVER_* used */
    int32_t iters;         /* PCG iterations (0 for Cholesky) */
    int32_t converged;     /* PCG reached tol */
    int32_t fallback;      /* PCG did not reach tol in max_iters: x is the Cholesky solution */
    double rel_residual;   /* ||S x + b|| / ||b|| of the returned x */
    double ms;             /* GPU time of the whole solve */
    double ms_setup;       /* of which preconditioner set-up (whitening, network, blocks) or
                              factorization (Cholesky) */
} pba_reduced_report;

/* Weights: He-initialized hidden layers and a zero output layer (block Jacobi) from `seed`. */
pba_status pba_pc_init(pba_ctx *ctx, uint64_t seed);
/* Copy n == PBA_PC_N_PARAMS weights in / out (host memory). */
pba_status pba_pc_set_weights(pba_ctx *ctx, const float *w, size_t n);
pba_status pba_pc_get_weights(pba_ctx *ctx, float *w, size_t n);
/* Couplings G_i of the context's current reduced system (the last one assembled: IC at the
 * level start, FC in the last iteration) into G_out [6F / 6][21] (n_floats must be >= 21 F);
 * *n_blocks receives F. Training samples are gathered this way from any contexts. */
pba_status pba_pc_harvest(pba_ctx *ctx, float *G_out, size_t n_floats, int32_t *n_blocks);
/* Train the network on the GPU on n_samples couplings G [n_samples][21] (host memory). */
pba_status pba_pc_train(pba_ctx *ctx, int64_t n_samples, const float *G, const pba_train_config *cfg,
                        pba_train_report *rep);
/* One FP32 forward and backward pass on n_samples couplings: mean loss and its gradient
 * (PBA_PC_N_PARAMS floats, packed like the weights). */
pba_status pba_pc_gradient(pba_ctx *ctx, int32_t n_samples, const float *G, double *loss, float *grad);
/* FP16 network outputs y [n_samples][21] for the given couplings. */
pba_status pba_pc_infer(pba_ctx *ctx, int32_t n_samples, const float *G, float *Y);
/* Solve S x = -b for the context's current reduced system and right-hand side (those of the
 * last iteration) with PBA_SOLVER_CHOL (tiled Cholesky), PBA_SOLVER_PCG_JACOBI,
 * PBA_SOLVER_PCG_LEARNED or PBA_SOLVER_PCG_BLOCKOPT (relative residual tol, at most max_iters iterations, Cholesky as
 * the fallback). x_out: host [6F] or NULL. */
pba_status pba_solve_reduced(pba_ctx *ctx, int32_t solver, double tol, int32_t max_iters, double *x_out,
                             pba_reduced_report *rep);

/* ---- Cholesky solve without allocation
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the PBA_SOLVER_CHOL path of
 * pba_solve_reduced (the tiled FP64-MFMA Cholesky and the tile-blocked triangular
 * solves) applied to a caller's system, with no context and no allocation. The
 * factor, the inverses of its diagonal tiles and a failure flag live in a static
 * scratch array of the library (4.9 MB, one copy per GPU, held until the process ends).
 *   n     unknowns, 1 .. PBA_NOALLOC_MAX_N; larger systems are rejected (PBA_E_INVALID)
 *   S     device, double [n][n] row-major, symmetric positive definite (read only)
 *   b     device, double [n];  x: device, double [n], receives x = -S^{-1} b
 *   info  device int32 or NULL: 0 after a successful factorization, 1 if a pivot was
 *         not positive (x is then not written)
 *   stream  hipStream_t (NULL: the null stream)
 * Asynchronous on `stream`: returns after enqueueing (PBA_OK), or before any device work
 * on an invalid argument. Every call on one GPU shares its scratch array, which keeps the
 * last call's contents (the call clears the flag itself): calls that overlap on one GPU
 * (other streams, other host threads) race and must be serialized by the caller.
 * The first call on a device looks up the array's device address (no allocation). */
#define PBA_NOALLOC_MAX_N 768
pba_status pba_solve_dense_noalloc(int32_t n, const double *S, const double *b, double *x, int32_t *info,
                                   void *stream);

/* Copy an internal buffer (PBA_DBG_*) to host memory; bytes must match its size exactly. */
pba_status pba_debug_fetch(pba_ctx *ctx, int32_t what, void *out, size_t bytes);

/* Kernel timing accumulated since the last call (then reset). */
pba_status pba_get_timing(pba_ctx *ctx, pba_timing *out);

/* Release the context and all its device memory. NULL is allowed. */
void pba_destroy(pba_ctx *ctx);

/* Message of the last error on this context (never NULL; "" if none). */
const char *pba_last_error(const pba_ctx *ctx);

/* Static name of a status code. */
const char *pba_status_string(pba_status s);

#ifdef __cplusplus
}
#endif
#endif /* PBA_H */
