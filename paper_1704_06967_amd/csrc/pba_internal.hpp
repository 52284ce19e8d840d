// Internal declarations of libpba: context state, device buffer layout and the
// kernel launch interface shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pba.h"

namespace pba {

// Per-observation record (T = float or double), one per (point, observing
// frame): blocks of the Gauss-Newton system in relative-pose coordinates.
enum RecField : int {
    REC_H = 0,        // 21: upper triangle (row-major) of sum w J_th^T J_th
    REC_h = 21,       // 6: sum w J_th J_d
    REC_HDD = 27,     // 1: sum w J_d^2
    REC_G = 28,       // 6: sum w J_th r
    REC_GD = 34,      // 1: sum w J_d r
    REC_E = 35,       // 1: sum of Huber norms
    REC_SQ = 36,      // 1: sum r^2
    REC_CNT = 37,     // 1: number of contributing residuals
    REC_STRIDE = 40
};
// Gradient record: g (6), g_d, energy, sum r^2, count. In the full record these
// are the fields REC_G .. REC_CNT; the IC iterations keep them in a compact
// record of IC_REC values per observation.
enum {
    GR_G = 0,
    GR_GD = 6,
    GR_E = 7,
    GR_SQ = 8,
    GR_CNT = 9,
    IC_REC = 10
};

// Per-pair geometry in double: R_fh (9), t_fh (3), t_h (3), pad.
constexpr int GEO_STRIDE = 16;
// Per-pair relative pose for the residual kernels: R (9), t (3).
constexpr int REL_STRIDE = 12;
// Per-iteration statistics slot layout (double).
enum StatField : int {
    ST_E = 0, ST_SQ = 1, ST_CNT = 2, ST_DISP = 3, ST_STEP_P = 4, ST_STEP_D = 5, ST_STRIDE = 8
};

constexpr int WAVE = 64;
constexpr int LANES_PER_OBS = 8;   // one lane per patch pixel
constexpr int BLOCK = 256;         // threads per block for residual kernels
constexpr int MAX_HOST_TARGETS = 20;  // target frames per host frame (Schur Gram size)
constexpr int PAIR_CHUNK = 512;       // observations per pair-reduction workgroup
constexpr int LDS_CHOL_MAX_N = 180;   // largest reduced system factored in one workgroup's LDS
constexpr int TILED_MIN_N = 96;
constexpr int IC_STEP_PTS = 128;      // points per depth workgroup of the fused IC step (1024 threads / 8)
constexpr int STEP_SEL_STRIDE = 64;   // ints per workgroup in the fused step's frame lists       // one-window systems from this size on use the tiled multi-workgroup path
constexpr int TCHOL_TILE = 32;        // tile edge of the tiled Cholesky for larger systems

// Independent problems (windows) held by one context: frames, points and pairs
// of window w are the contiguous ranges [off[w], off[w + 1]) of the global
// arrays; the reduced system is block diagonal, window w's block (6 F_w square)
// starting at S_off[w] doubles (its packed factor at L_off[w]). One window is
// the single-problem case.
struct WinArgs {
    int nwin;
    const int *frame_off, *pair_off, *point_off, *S_off, *L_off;  // [nwin + 1]
    const int *frame_win, *point_win;                             // [F], [N]
};

// Launch shape of a residual kernel: threads per workgroup (tiles of block / 8
// observations) and, when grid_mult > 0, a persistent grid of grid_mult
// workgroups per compute unit striding over the tiles.
struct LaunchShape {
    int block = 256;
    int grid_mult = 0;
    int lanes = 1;   // IC residual pass: threads per observation (1 or 8)
};

// Learned block preconditioner (network 22 -> 256 -> 256 -> 21) and PCG state.
constexpr int PC_IN = 22, PC_HID = 256, PC_OUT = 21;
constexpr int PC_OFF_B1 = PC_HID * PC_IN, PC_OFF_W2 = PC_OFF_B1 + PC_HID, PC_OFF_B2 = PC_OFF_W2 + PC_HID * PC_HID,
              PC_OFF_W3 = PC_OFF_B2 + PC_HID, PC_OFF_B3 = PC_OFF_W3 + PC_OUT * PC_HID,
              PC_N_PARAMS = PC_OFF_B3 + PC_OUT;
struct PcState {
    float *w = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;  // FP32 weights, Adam moments, gradient
    _Float16 *wh = nullptr;                                           // padded FP16 copy for inference
    bool have_w = false;
    int adam_step = 0;
    int nb_cap = 0;                                                   // blocks of the current system
    double *Ci = nullptr, *G = nullptr, *P = nullptr;
    float *X = nullptr, *Y = nullptr;
    int *flag = nullptr;
    int n_cap = 0;                                                    // PCG vectors
    double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *part = nullptr, *sc = nullptr;
    int *st = nullptr;
    int b_cap = 0;                                                    // training batch scratch
    float *Z1 = nullptr, *H1 = nullptr, *Z2 = nullptr, *H2 = nullptr, *Yt = nullptr, *dY = nullptr, *D1 = nullptr,
          *D2 = nullptr, *lossv = nullptr, *Xb = nullptr, *Gb = nullptr;
    int *idx = nullptr;
    double *lsum = nullptr;
    int64_t ns = 0, ns_cap = 0;                                       // training samples
    float *Gs = nullptr, *Xs = nullptr;
};

struct LevelDev {
    int W = 0, H = 0;
    void *img = nullptr;      // T [F][H][W]
    void *K = nullptr;        // T [F][4] level intrinsics
    void *tmpl = nullptr;     // T [N][P][4] (I0, gu, gv, usable) at the host patch pixels
    void *pcam = nullptr;     // double [Pn][8] host and target level intrinsics of every pair
    bool tmpl_valid = false;
};

// Static structure derived from the observation lists (built on the host at set_points).
struct Structure {
    int n_pairs = 0;
    std::vector<int> obs_point, obs_pair;             // [O]
    std::vector<int> pair_host, pair_target;          // [Pn]
    std::vector<int> pair_obs_ptr, pair_obs_idx;      // CSR pair -> obs
    std::vector<int> pchunk_begin, pchunk_end;        // chunks of pair_obs_idx (one pair each)
    std::vector<int> pair_chunk_ptr;                  // CSR pair -> chunks
    std::vector<int> frame_pair_ptr, frame_pair_item; // CSR frame -> (pair*2 + is_host)
    // hosts and their extended frame sets for the depth Schur Gram
    std::vector<int> hosts;                           // distinct host frames
    std::vector<int> host_m;                          // targets per host
    std::vector<int> pair_local;                      // [Pn] index of the pair within its host
    std::vector<int> pair_hidx;                       // [Pn] host index
    std::vector<int> host_pts;                        // points grouped by host
    std::vector<int> chunk_host, chunk_begin, chunk_end, chunk_off; // Gram chunks (into host_pts)
    std::vector<int> host_chunk_ptr;                  // CSR host -> chunks
    // nonzero 6x6 blocks of the reduced system and their contributions
    std::vector<int> blk_fa, blk_fb;                  // [nblk]
    std::vector<int> blk_pp_ptr, blk_pp_item;         // (pair*4 + kind) kind 0 AtHA 1 BtHB 2 AtHB 3 BtHA
    std::vector<int> blk_g_ptr, blk_g_item;           // (host index, a, b) packed: hidx*4096 + a*64 + b
    size_t gram_floats = 0;                           // total doubles of all chunk partials
};

struct Ctx {
    pba_config cfg{};
    std::string err;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    size_t real_size = 4;  // sizeof(T)

    // state machine
    bool have_frames = false, have_points = false;
    int cur_level = -1;            // level whose linearization / frozen set is current
    int iters_in_level = 0;
    int since_lin = 0;   // iterations since the level's (re-)linearization

    // frames
    int F = 0, W = 0, H = 0;
    std::vector<double> K0;        // [F][4]
    LevelDev lv[PBA_MAX_LEVELS];

    // points
    int N = 0, O = 0, P = 0;
    Structure st;

    // windows (host copies of the offsets; see WinArgs)
    int nwin = 1;
    std::vector<int> win_frame_off, win_point_off, win_pair_off, win_S_off, win_L_off;
    // internal order of points and observations (see load_points): internal
    // point i is the caller's point pt_caller[i] (global, windows after one
    // another), internal observation o the caller's observation obs_caller[o]
    std::vector<int> pt_caller, obs_caller;
    int *d_win_frame_off = nullptr, *d_win_pair_off = nullptr, *d_win_point_off = nullptr, *d_win_S_off = nullptr,
        *d_win_L_off = nullptr, *d_frame_win = nullptr, *d_point_win = nullptr;
    double *d_wstat = nullptr;                         // [nwin][4] per-window E, SQ, CNT, max pose step
    WinArgs win() const {
        return WinArgs{nwin, d_win_frame_off, d_win_pair_off, d_win_point_off, d_win_S_off, d_win_L_off,
                       d_frame_win, d_point_win};
    }

    // device buffers (generic pointers; element type per precision)
    double *d_poses = nullptr, *d_poses0 = nullptr;   // [F][12]
    double *d_poses_alt = nullptr;                    // [F][12] second pose buffer of the fused IC step
    int batch_k = 0;                                  // index of the iteration being enqueued in its batch
    // per depth workgroup of the fused IC step (IC_STEP_PTS points each): the
    // frames its points observe, [count, frames ..., 64-bit mask] at stride
    // STEP_SEL_STRIDE (empty when a window has more than 60 frames)
    int *d_step_sel = nullptr;
    int step_sel_max = 0;                             // most frames of one workgroup
    double *d_K0 = nullptr;                           // [F][4] level-0 intrinsics
    double *d_depth = nullptr, *d_depth0 = nullptr;   // [N]
    int *d_host_frame = nullptr, *d_obs_ptr = nullptr, *d_obs_frame = nullptr, *d_obs_point = nullptr,
        *d_obs_pair = nullptr, *d_pair_host = nullptr, *d_pair_target = nullptr, *d_pair_obs_ptr = nullptr,
        *d_pair_obs_idx = nullptr, *d_frame_pair_ptr = nullptr, *d_frame_pair_item = nullptr,
        *d_pair_local = nullptr, *d_pair_hidx = nullptr, *d_host_m = nullptr, *d_host_frames = nullptr,
        *d_host_pts = nullptr, *d_chunk_host = nullptr, *d_chunk_begin = nullptr, *d_chunk_end = nullptr,
        *d_chunk_off = nullptr, *d_host_chunk_ptr = nullptr, *d_blk_fa = nullptr, *d_blk_fb = nullptr,
        *d_blk_pp_ptr = nullptr, *d_blk_pp_item = nullptr, *d_blk_g_ptr = nullptr, *d_blk_g_item = nullptr,
        *d_pchunk_begin = nullptr, *d_pchunk_end = nullptr, *d_pair_chunk_ptr = nullptr;
    float *d_host_uv = nullptr;                        // [N][2]
    uint8_t *d_mask = nullptr;                         // [O]
    uint8_t *d_obs_live = nullptr;                     // [O] 1 while the observation is in the window (pba_drop_frame)
    void *d_rec = nullptr;                             // double [O][REC_STRIDE]
    void *d_icr = nullptr;                             // double [O][IC_REC] gradient records of the IC iterations
    double *d_gdo = nullptr;                           // [O] their g_d field again, contiguous
    double *d_geo0 = nullptr, *d_geo_a = nullptr, *d_geo_b = nullptr;   // [Pn][GEO_STRIDE]
    void *d_rel0 = nullptr, *d_rel_a = nullptr, *d_rel_b = nullptr;      // T [Pn][REL_STRIDE]
    double *d_pairH = nullptr;                         // [Pn][21]
    double *d_pairY = nullptr;                         // [Pn][9] (6 + e, sq, cnt)
    double *d_partH = nullptr, *d_partY = nullptr;     // per pair chunk partials [nch][21], [nch][9]
    double *d_obsmap = nullptr;                        // [O][12] observation couplings for the Gram
    double *d_hc = nullptr;                            // [O][6] h_o of the last system (relative coordinates)
    double *d_Hdd = nullptr, *d_gd = nullptr;          // [N] (Hdd damped after assembly)
    double *d_mu = nullptr;                            // [nwin][2] mu_p, mu_d
    double *d_gram = nullptr;                          // chunk partials
    double *d_S = nullptr;                             // [6F][6F] reduced system / factor
    double *d_Sinv = nullptr;                          // IC: S^{-1} at p(0) [6F][6F]
    double *d_Lfac = nullptr;                          // IC: packed Cholesky factor of S, then 1 / L(k, k)
    double *d_Sfac = nullptr;                          // tiled path: factor of S [6F][6F]
    double *d_Linv = nullptr;                          // inverses of its diagonal tiles [nt][32][32]
    double *d_b = nullptr, *d_dtheta = nullptr;        // [6F]
    double *d_dth_rel = nullptr;                       // [Pn][6]
    double *d_stats = nullptr;                         // [cap][ST_STRIDE]
    int stats_cap = 0;
    int *d_flag = nullptr;                             // device error flag (non-SPD)
    int *d_gate = nullptr;                             // 1 while the current solve level runs
    int *d_count = nullptr;                            // iterations run per level [PBA_MAX_LEVELS]
    int *d_count_base = nullptr;                       // of those, before the level's last re-centring
    double *d_du_part = nullptr;                       // depth-update block maxima [blocks][2]
    double *d_pairK0 = nullptr;                        // [Pn][8] level-0 intrinsics of host and target
    int *d_pc_slot = nullptr;  // [pair chunks][PAIR_CHUNK][4] observation (-1: none), point, point's range

    // front end: geometric bundle adjustment on tracked positions
    double *d_obs_z = nullptr;     // [O][2] tracked level-0 position of every observation
    uint8_t *d_geo_in = nullptr;   // [O] 1 while the observation is a geometric inlier
    bool geo_mode = false;         // the FC iteration linearizes the reprojection error
    double geo_huber = 1.0;        // its Huber threshold (level-0 pixels)

    // current double-buffer orientation
    bool flip = false;

    // learned preconditioner and PCG
    PcState pc;
    bool s_valid = false;                              // d_S / d_b hold an assembled system
    bool tiled() const { return nwin == 1 && 6 * F >= TILED_MIN_N; }  // tiled Cholesky path (else one-workgroup LDS)

    // launch shapes of the per-iteration residual kernels (autotuned)
    int n_cu = 256;
    LaunchShape tune_res, tune_lin;

    // a whole coarse-to-fine solve captured as one HIP graph (PBA_FLAG_GRAPH)
    hipGraphExec_t solve_graph = nullptr;
    int graph_iters = -1;
    double graph_conv = -1.0;
    double *d_eval = nullptr;                          // sums of the evaluation kernel and their block partials
    size_t eval_cap = 0;

    // timing
    std::vector<hipEvent_t> ev_pool;
    int64_t t_launches[PBA_MAX_LEVELS] = {0, 0, 0, 0}, t_res[PBA_MAX_LEVELS] = {0, 0, 0, 0};
    double t_ms[PBA_MAX_LEVELS] = {0.0, 0.0, 0.0, 0.0};
    int64_t t_step_launches[PBA_MAX_LEVELS] = {0, 0, 0, 0};
    double t_step_ms[PBA_MAX_LEVELS] = {0.0, 0.0, 0.0, 0.0};
};

// ---- kernel launchers (pba_kernels.hip); T selects float or double.
template <typename T> struct Launch {
    static void convert_images(hipStream_t s, const float *src, T *dst, size_t n);
    static void downsample(hipStream_t s, const T *src, T *dst, int F, int Ws, int Hs, int Wd, int Hd);
    static void level_K(hipStream_t s, const double *K0, T *K, int F, int level);
    static void make_template(hipStream_t s, Ctx &c, int level);
    static void relpose(hipStream_t s, Ctx &c, const double *poses, double *geo, T *rel);
    static void ic_linearize(hipStream_t s, Ctx &c, int level);
    // e0 / e1 (optional): events recorded by the dispatch itself at the kernel's start and end
    // level start: gate / flag / count, p(0) copies, relative poses at p(0) (one launch)
    static void level_begin(hipStream_t s, Ctx &c, int level, bool clear_flag, bool recentre = false);
    static void ic_residual(hipStream_t s, Ctx &c, int level, const double *geo_cur, hipEvent_t e0 = nullptr,
                            hipEvent_t e1 = nullptr);
    static void ic_residual_shape(hipStream_t s, Ctx &c, int level, const double *geo_cur, LaunchShape sh,
                                  hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
    static void fc_linearize_shape(hipStream_t s, Ctx &c, int level, const double *geo_cur, LaunchShape sh);
    static void fc_linearize(hipStream_t s, Ctx &c, int level, const double *geo_cur, bool write_mask,
                             hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
    static void evaluate(hipStream_t s, Ctx &c, int level);
    static void point_reduce(hipStream_t s, Ctx &c, bool with_hdd);
    static void pair_reduce_H(hipStream_t s, Ctx &c);
    // prev_stat (IC): the previous iteration's statistics slot; its end (statistics,
    // count, convergence gate) is taken by this kernel from the depth update's maxima
    static void pair_reduce_y(hipStream_t s, Ctx &c, double *prev_stat = nullptr, double conv_px = -1.0,
                              int level = 0);
    static void depth_update(hipStream_t s, Ctx &c, const double *geo_old, const double *geo_new, double *stat,
                             double conv_px, int level, bool finish = true);
};

// learned preconditioner and PCG (pba_learned.hip)
void pc_whiten(hipStream_t s, Ctx &c, int nb);                      // C_i^{-1}, G_i, features of S
void pc_infer(hipStream_t s, Ctx &c, int m, const float *X, float *Y);
void pc_blocks(hipStream_t s, Ctx &c, int nb, const float *Y);      // Y = nullptr: block Jacobi
void pc_blocks_opt(hipStream_t s, Ctx &c, int nb);                 // P^ = (I + G_i)^{-1}
void pc_to_half(hipStream_t s, Ctx &c);
void pc_features(hipStream_t s, int m, const float *G, float *X);
void pc_gather(hipStream_t s, int m, const int *idx, const float *src, int width, float *dst);
void pc_forward_backward(hipStream_t s, Ctx &c, int m, const float *X, const float *G, float *grad, float *lossv);
void pc_adam(hipStream_t s, Ctx &c, float lr, float b1, float b2, float eps, int step);
void pc_sum(hipStream_t s, int n, const float *v, double *out);
void pcg_init(hipStream_t s, Ctx &c, int n);
void pcg_iterations(hipStream_t s, Ctx &c, int n, int k, double tol);
void pc_resid(hipStream_t s, Ctx &c, int n, const double *x, double *part);   // (S x + b)^2 row-group sums
void launch_tsolve(hipStream_t s, Ctx &c, const double *b, double *x);        // x = -S^{-1} b, tiled factor

// mixed precision linearization (pair order, BF16 MFMA pose blocks into the pair chunk partials)
void launch_linearize_mixed(hipStream_t s, Ctx &c, int level, bool ic, const double *geo_cur, bool write_mask,
                            hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// precision-independent launchers (double only)
void launch_mu(hipStream_t s, Ctx &c, const double *geo);
void launch_gram(hipStream_t s, Ctx &c, const double *geo, const void *rec, bool rec_double);
void launch_assemble_s(hipStream_t s, Ctx &c, const double *geo);
void launch_ic_factor(hipStream_t s, Ctx &c);
void launch_solve(hipStream_t s, Ctx &c, const double *geo_lin, double *geo_next, void *rel_next,
                  bool rel_double, double *stat);
void launch_sum_stats(hipStream_t s, Ctx &c, const void *rec, bool rec_double, double *out3);
size_t sum_stats_doubles(const Ctx &c);  // size of out3 (the sums and the block partials)
// pose_sync (fused IC step, last iteration of a batch): after an odd number of
// iterations the current poses are copied back from the second pose buffer.
void launch_conv(hipStream_t s, Ctx &c, double *stat, double conv_px, int nparts, int level, bool pose_sync = false);
// IC on one window whose step fits the solve's LDS cache: the solve and the
// depth step of an iteration run as one kernel (launch_ic_step).
bool ic_fused(const Ctx &c);
void launch_ic_step(hipStream_t s, Ctx &c, const double *geo_lin, const double *geo_old, double *geo_next,
                    void *rel_next, bool rel_double, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
int du_nparts(const Ctx &c);   // blocks of the depth step (parts of its convergence maxima)
// count[level] = 0, optionally flag = 0, then gate = (flag == 0)
void launch_open(hipStream_t s, Ctx &c, int level, bool clear_flag);
void launch_drop_frame(hipStream_t s, Ctx &c, int frame);
void launch_ic_inverse(hipStream_t s, Ctx &c);
void launch_tchol(hipStream_t s, Ctx &c, bool copy = true);   // (copy S to d_Sfac and) factor d_Sfac in tiles
void launch_tinv(hipStream_t s, Ctx &c);    // S^{-1} from the tiled factor
// Error of a call that has no context: recorded for pba_last_error(NULL).
pba_status fail_global(pba_status s, const std::string &msg);
void launch_copy_d(hipStream_t s, const double *src, double *dst, size_t n);  // device copy as a kernel
void launch_fill(hipStream_t s, double *p, size_t n, double v, const int *gate);

// front end (pba_frontend.hip): corners of one frame (R: [H][W] response scratch,
// cell_R / cell_idx / rank: per-cell scratch), tracks, geometric BA records and outliers
void launch_fe_corners(hipStream_t s, Ctx &c, int frame, int cell, int margin, long long min_resp, int K,
                       long long *R, long long *cell_R, int *cell_idx, int *rank, int *uv, long long *resp,
                       int *count);
void launch_fe_track(hipStream_t s, Ctx &c, int n, const int *host, const double *host_uv, const int *target,
                     const double *guess, int radius, int n_iters, double min_eig, double fb_px, int levels,
                     double *out_uv, int *out_status, double *out_fb);
void launch_geo_linearize(hipStream_t s, Ctx &c, const double *geo_cur, hipEvent_t e0 = nullptr,
                          hipEvent_t e1 = nullptr);
void launch_geo_outliers(hipStream_t s, Ctx &c, const double *geo_cur, double limit);

}  // namespace pba
