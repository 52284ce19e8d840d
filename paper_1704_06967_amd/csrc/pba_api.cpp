// Host runtime of libpba: the C ABI declared in include/pba.h.
//
// Every entry point validates its arguments on the host before touching the
// device, so error paths are testable without a GPU. Device work is enqueued on
// the context's stream; each entry point synchronizes that stream before it
// returns.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
#include <random>
#include <string>
#include <vector>

#include "pba_affine.hpp"
#include "pba_internal.hpp"

using namespace pba;

// Inputs of one window of a batched context, held on the host until every
// window is set (the global arrays are assembled at the first call that needs
// them).
struct WinStage {
    bool have_frames = false, have_points = false;
    int F = 0;
    std::vector<float> img;          // [F][H][W]
    std::vector<double> K, P;        // [F][4], [F][12]
    int N = 0;
    std::vector<int> hf, optr, ofr;  // window-local frame indices
    std::vector<float> uv;
    std::vector<double> d;
};

struct pba_ctx {
    Ctx c;
    std::vector<WinStage> stage;     // n_windows > 1 only
    bool dirty = false;              // staged inputs not yet assembled
    int stage_W = 0, stage_H = 0;
    AffBufs aff;                     // per-frame affine brightness (pba_set_affine)
};

namespace {

thread_local std::string g_create_err;

constexpr int GRAM_CHUNK = 128;  // points per Gram workgroup

pba_status fail(Ctx *c, pba_status s, const std::string &msg) {
    if (c)
        c->err = msg;
    else
        g_create_err = msg;
    return s;
}

#define HIPCHK(expr)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(&c, e_ == hipErrorOutOfMemory ? PBA_E_OOM : PBA_E_DEVICE,                  \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                        \
    } while (0)

template <typename P>
hipError_t dalloc(P *&p, size_t bytes) {
    if (p) {
        (void)hipFree((void *)p);
        p = nullptr;
    }
    if (bytes == 0) bytes = 8;
    return hipMalloc((void **)&p, bytes);
}

template <typename P>
void dfree(P *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

bool finite_all(const double *p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// Copy n elements of caller memory (host or device) into a host vector.
template <typename V>
hipError_t fetch(std::vector<V> &dst, const V *src, size_t n, int mem) {
    dst.resize(n);
    if (n == 0) return hipSuccess;
    if (mem == PBA_DEVICE) return hipMemcpy(dst.data(), src, n * sizeof(V), hipMemcpyDeviceToHost);
    std::memcpy(dst.data(), src, n * sizeof(V));
    return hipSuccess;
}

template <typename V>
hipError_t upload(Ctx &c, V *&dptr, const std::vector<V> &v) {
    hipError_t e = dalloc(dptr, v.size() * sizeof(V));
    if (e != hipSuccess) return e;
    if (v.empty()) return hipSuccess;
    return hipMemcpyAsync(dptr, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice, c.stream);
}

void drop_graph(Ctx &c);

void release_points(Ctx &c) {
    drop_graph(c);
    c.s_valid = false;
    for (int **p : {&c.d_host_frame, &c.d_obs_ptr, &c.d_obs_frame, &c.d_obs_point, &c.d_obs_pair, &c.d_pair_host,
                    &c.d_pair_target, &c.d_pair_obs_ptr, &c.d_pair_obs_idx, &c.d_frame_pair_ptr,
                    &c.d_frame_pair_item, &c.d_pair_local, &c.d_pair_hidx, &c.d_host_m, &c.d_host_frames,
                    &c.d_host_pts, &c.d_chunk_host, &c.d_chunk_begin, &c.d_chunk_end, &c.d_chunk_off,
                    &c.d_host_chunk_ptr, &c.d_blk_fa, &c.d_blk_fb, &c.d_blk_pp_ptr, &c.d_blk_pp_item,
                    &c.d_blk_g_ptr, &c.d_blk_g_item, &c.d_pchunk_begin, &c.d_pchunk_end, &c.d_pair_chunk_ptr})
        dfree(*p);
    for (int **p : {&c.d_win_pair_off, &c.d_win_point_off, &c.d_point_win}) dfree(*p);
    dfree(c.d_host_uv);
    dfree(c.d_mask);
    dfree(c.d_obs_live);
    dfree(c.d_rec);
    dfree(c.d_depth);
    dfree(c.d_depth0);
    for (double **p : {&c.d_geo0, &c.d_geo_a, &c.d_geo_b, &c.d_pairH, &c.d_pairY, &c.d_Hdd, &c.d_gd,
                       &c.d_gram, &c.d_dth_rel, &c.d_partH, &c.d_partY, &c.d_obsmap, &c.d_hc})
        dfree(*p);
    dfree(c.d_rel0);
    dfree(c.d_rel_a);
    dfree(c.d_rel_b);
    dfree(c.d_icr);
    dfree(c.d_gdo);
    dfree(c.d_obs_z);
    dfree(c.d_geo_in);
    for (int l = 0; l < PBA_MAX_LEVELS; ++l) {
        dfree(c.lv[l].tmpl);
        dfree(c.lv[l].pcam);
        c.lv[l].tmpl_valid = false;
    }
    c.have_points = false;
    c.cur_level = -1;
    c.N = c.O = 0;
}

void release_frames(Ctx &c) {
    release_points(c);
    for (int l = 0; l < PBA_MAX_LEVELS; ++l) {
        dfree(c.lv[l].img);
        dfree(c.lv[l].K);
        c.lv[l].W = c.lv[l].H = 0;
    }
    for (double **p : {&c.d_poses, &c.d_poses0, &c.d_poses_alt, &c.d_K0, &c.d_S, &c.d_Sinv, &c.d_Lfac, &c.d_Sfac, &c.d_Linv, &c.d_b,
                       &c.d_dtheta, &c.d_stats, &c.d_mu})
        dfree(*p);
    dfree(c.d_flag);
    dfree(c.d_gate);
    dfree(c.d_count);
    dfree(c.d_count_base);
    dfree(c.d_du_part);
    dfree(c.d_pairK0);
    dfree(c.d_pc_slot);
    dfree(c.d_step_sel);
    for (int **p : {&c.d_win_frame_off, &c.d_win_S_off, &c.d_win_L_off, &c.d_frame_win}) dfree(*p);
    dfree(c.d_wstat);
    c.stats_cap = 0;
    c.have_frames = false;
    c.F = 0;
}

std::string validate_config(const pba_config *cfg) {
    if (!cfg) return "cfg is NULL";
    if (cfg->mode != PBA_FC && cfg->mode != PBA_IC_PROXY) return "mode must be PBA_FC or PBA_IC_PROXY";
    if (cfg->precision != PBA_FP64 && cfg->precision != PBA_FP32 && cfg->precision != PBA_MIXED_BF16)
        return "unknown precision";
    if (cfg->n_levels < 1 || cfg->n_levels > PBA_MAX_LEVELS) return "n_levels must be in 1..4";
    if (cfg->pattern_n < 1 || cfg->pattern_n > PBA_MAX_PATTERN) return "pattern_n must be in 1..8";
    for (int j = 0; j < cfg->pattern_n; ++j)
        if (std::abs(cfg->pattern_uv[2 * j]) > 4 || std::abs(cfg->pattern_uv[2 * j + 1]) > 4)
            return "pattern offsets must satisfy |du|, |dv| <= 4";
    if (!(cfg->huber_k > 0.0)) return "huber_k must be > 0";
    if (!(cfg->damping_rel >= 0.0) || !std::isfinite(cfg->damping_rel)) return "damping_rel must be finite and >= 0";
    if (cfg->pinned_frame < -1) return "pinned_frame must be >= -1";
    if (cfg->solver != PBA_SOLVER_CHOL) return "solver must be PBA_SOLVER_CHOL (PCG: pba_solve_reduced)";
    if (cfg->n_windows < 1 || cfg->n_windows > PBA_MAX_WINDOWS) return "n_windows must be in 1..PBA_MAX_WINDOWS";
    if (cfg->flags & ~(PBA_FLAG_TIMING | PBA_FLAG_GRAPH | PBA_FLAG_LANE_PER_PIXEL)) return "unknown flag bits";
    if (cfg->recentre_every < 0 || cfg->recentre_every > 1000) return "recentre_every must be in 0..1000";
    return "";
}

bool is_fp64(const Ctx &c) { return c.cfg.precision == PBA_FP64; }
bool is_mixed(const Ctx &c) { return c.cfg.precision == PBA_MIXED_BF16; }

// ---- structure of the problem: pairs, host groups, Gram chunks, nonzero blocks
std::string build_structure(Ctx &c, const std::vector<int> &host_frame, const std::vector<int> &obs_ptr,
                            const std::vector<int> &obs_frame) {
    Structure &s = c.st;
    s = Structure();
    const int N = c.N, O = c.O, F = c.F;
    s.obs_point.resize(O);
    for (int n = 0; n < N; ++n)
        for (int o = obs_ptr[n]; o < obs_ptr[n + 1]; ++o) s.obs_point[o] = n;
    std::map<long long, int> pid;
    for (int o = 0; o < O; ++o) pid[(long long)host_frame[s.obs_point[o]] * F + obs_frame[o]] = 0;
    s.n_pairs = 0;
    for (auto &kv : pid) {
        kv.second = s.n_pairs++;
        s.pair_host.push_back((int)(kv.first / F));
        s.pair_target.push_back((int)(kv.first % F));
    }
    const int Pn = s.n_pairs;
    s.obs_pair.resize(O);
    for (int o = 0; o < O; ++o) s.obs_pair[o] = pid[(long long)host_frame[s.obs_point[o]] * F + obs_frame[o]];
    s.pair_obs_ptr.assign(Pn + 1, 0);
    for (int o = 0; o < O; ++o) s.pair_obs_ptr[s.obs_pair[o] + 1]++;
    for (int p = 0; p < Pn; ++p) s.pair_obs_ptr[p + 1] += s.pair_obs_ptr[p];
    s.pair_obs_idx.resize(O);
    {
        std::vector<int> fill(s.pair_obs_ptr.begin(), s.pair_obs_ptr.end() - 1);
        for (int o = 0; o < O; ++o) s.pair_obs_idx[fill[s.obs_pair[o]]++] = o;
    }
    s.pair_chunk_ptr.assign(Pn + 1, 0);
    for (int p = 0; p < Pn; ++p) {
        for (int b = s.pair_obs_ptr[p]; b < s.pair_obs_ptr[p + 1]; b += PAIR_CHUNK) {
            s.pchunk_begin.push_back(b);
            s.pchunk_end.push_back(std::min(s.pair_obs_ptr[p + 1], b + PAIR_CHUNK));
        }
        s.pair_chunk_ptr[p + 1] = (int)s.pchunk_begin.size();
    }
    s.frame_pair_ptr.assign(F + 1, 0);
    for (int p = 0; p < Pn; ++p) {
        s.frame_pair_ptr[s.pair_target[p] + 1]++;
        s.frame_pair_ptr[s.pair_host[p] + 1]++;
    }
    for (int f = 0; f < F; ++f) s.frame_pair_ptr[f + 1] += s.frame_pair_ptr[f];
    s.frame_pair_item.resize(2 * Pn);
    {
        std::vector<int> fill(s.frame_pair_ptr.begin(), s.frame_pair_ptr.end() - 1);
        for (int p = 0; p < Pn; ++p) {  // pair order inside every frame list
            s.frame_pair_item[fill[s.pair_target[p]]++] = p * 2;
            s.frame_pair_item[fill[s.pair_host[p]]++] = p * 2 + 1;
        }
    }
    // host groups (pairs are sorted by host, then target)
    std::vector<int> hidx_of_frame(F, -1);
    s.pair_local.resize(Pn);
    s.pair_hidx.resize(Pn);
    for (int p = 0; p < Pn; ++p) {
        const int h = s.pair_host[p];
        if (hidx_of_frame[h] < 0) {
            hidx_of_frame[h] = (int)s.hosts.size();
            s.hosts.push_back(h);
            s.host_m.push_back(0);
        }
        const int hi = hidx_of_frame[h];
        s.pair_hidx[p] = hi;
        s.pair_local[p] = s.host_m[hi]++;
    }
    for (size_t hi = 0; hi < s.hosts.size(); ++hi)
        if (s.host_m[hi] > MAX_HOST_TARGETS)
            return "host frame " + std::to_string(s.hosts[hi]) + " has " + std::to_string(s.host_m[hi]) +
                   " distinct target frames (limit " + std::to_string(MAX_HOST_TARGETS) + ")";
    const int NH = (int)s.hosts.size();
    // points grouped by host (points without observations are skipped)
    std::vector<std::vector<int>> by_host(NH);
    for (int n = 0; n < N; ++n)
        if (obs_ptr[n + 1] > obs_ptr[n]) by_host[hidx_of_frame[host_frame[n]]].push_back(n);
    s.host_chunk_ptr.assign(NH + 1, 0);
    size_t off = 0;
    for (int hi = 0; hi < NH; ++hi) {
        const int E = 6 * (s.host_m[hi] + 1);
        const int b0 = (int)s.host_pts.size();
        for (int n : by_host[hi]) s.host_pts.push_back(n);
        const int b1 = (int)s.host_pts.size();
        for (int b = b0; b < b1; b += GRAM_CHUNK) {
            s.chunk_host.push_back(hi);
            s.chunk_begin.push_back(b);
            s.chunk_end.push_back(std::min(b1, b + GRAM_CHUNK));
            s.chunk_off.push_back((int)off);
            off += (size_t)E * E;
        }
        s.host_chunk_ptr[hi + 1] = (int)s.chunk_host.size();
    }
    s.gram_floats = off;
    if (off > (size_t)INT32_MAX) return "too many points for the Schur Gram buffers";
    // nonzero blocks of S
    // every 6 x 6 block of each window's S (structurally zero ones written as
    // zeros by the assembly, so that S needs no clearing pass)
    std::map<long long, std::pair<std::vector<int>, std::vector<int>>> blk;
    auto key = [F](int a, int b) { return (long long)a * F + b; };
    for (int w = 0; w + 1 < (int)c.win_frame_off.size(); ++w)
        for (int a = c.win_frame_off[w]; a < c.win_frame_off[w + 1]; ++a)
            for (int b = c.win_frame_off[w]; b < c.win_frame_off[w + 1]; ++b) blk[key(a, b)];
    for (int p = 0; p < Pn; ++p) {
        const int t = s.pair_target[p], h = s.pair_host[p];
        blk[key(t, t)].first.push_back(p * 4 + 0);
        blk[key(h, h)].first.push_back(p * 4 + 1);
        blk[key(t, h)].first.push_back(p * 4 + 2);
        blk[key(h, t)].first.push_back(p * 4 + 3);
    }
    for (int hi = 0; hi < NH; ++hi) {
        std::vector<int> ext;
        for (int p = 0; p < Pn; ++p)
            if (s.pair_hidx[p] == hi) ext.push_back(s.pair_target[p]);
        ext.push_back(s.hosts[hi]);
        for (int a = 0; a < (int)ext.size(); ++a)
            for (int b = 0; b < (int)ext.size(); ++b)
                blk[key(ext[a], ext[b])].second.push_back(hi * 4096 + a * 64 + b);
    }
    s.blk_pp_ptr.push_back(0);
    s.blk_g_ptr.push_back(0);
    for (auto &kv : blk) {
        s.blk_fa.push_back((int)(kv.first / F));
        s.blk_fb.push_back((int)(kv.first % F));
        for (int it : kv.second.first) s.blk_pp_item.push_back(it);
        for (int it : kv.second.second) s.blk_g_item.push_back(it);
        s.blk_pp_ptr.push_back((int)s.blk_pp_item.size());
        s.blk_g_ptr.push_back((int)s.blk_g_item.size());
    }
    return "";
}

// ---- level start and iterations, per element type

// The IC system of the level at p(0): J (Sec. 3.4) and W0, H = J^T W0 J, the
// depth Schur complement, its Cholesky factor and inverse. With linearize
// false (a keyframe dropped mid-level) the pair blocks, h and H_dd are summed
// again from the per-observation records kept at p(0) (those of dropped
// observations are zero) and the residuals are not evaluated again; the
// mixed form, whose pose blocks come from its MFMA contraction rather than
// from the records, linearizes again at p(0).
template <typename T>
void ic_system(Ctx &c, int level, bool linearize) {
    hipStream_t s = c.stream;
    if (is_mixed(c)) {
        launch_linearize_mixed(s, c, level, true, c.d_geo0, true);
    } else {
        if (linearize) Launch<T>::ic_linearize(s, c, level);
        Launch<T>::pair_reduce_H(s, c);
    }
    Launch<T>::point_reduce(s, c, true);
    launch_mu(s, c, c.d_geo0);
    launch_gram(s, c, c.d_geo0, c.d_rec, true);
    launch_assemble_s(s, c, c.d_geo0);
    launch_ic_factor(s, c);
    launch_ic_inverse(s, c);
}
// Opens the level's gate (clear_flag: also clears the failure flag) and sets up
// the level. recentre: proxy re-centring inside the level (IC): the same set-up
// at the current parameters, gated (no effect once the level's gate is closed),
// keeping the level's iteration count.
template <typename T>
pba_status start_level(Ctx &c, int level, bool clear_flag, bool recentre = false) {
    hipStream_t s = c.stream;
    if (!c.lv[level].tmpl_valid) {
        Launch<T>::make_template(s, c, level);
        c.lv[level].tmpl_valid = true;
    }
    Launch<T>::level_begin(s, c, level, clear_flag, recentre);
    c.flip = false;
    if (c.cfg.mode == PBA_IC_PROXY) {
        ic_system<T>(c, level, true);
        c.s_valid = true;
    } else {
        c.s_valid = false;
    }
    HIPCHK(hipGetLastError());
    c.cur_level = level;
    if (!recentre) c.iters_in_level = 0;
    c.since_lin = 0;
    return PBA_OK;
}

// Iterations between proxy re-centrings (0: none; FC: none).
int recentre_every(const Ctx &c) { return c.cfg.mode == PBA_IC_PROXY ? c.cfg.recentre_every : 0; }

pba_status recentre_level(Ctx &c, int level) {
    return is_fp64(c) ? start_level<double>(c, level, false, true) : start_level<float>(c, level, false, true);
}

template <typename T>
// prev_stat (IC, not the first iteration of a batch): the previous iteration's
// statistics slot, finished by this iteration's pair sums; last: the final
// iteration of the batch, whose end runs as a kernel of its own.
pba_status one_iteration(Ctx &c, int level, double *stat, hipEvent_t ev0, hipEvent_t ev1, double conv_px,
                         double *prev_stat, bool last, hipEvent_t ev2 = nullptr, hipEvent_t ev3 = nullptr) {
    hipStream_t s = c.stream;
    double *geo_cur = c.flip ? c.d_geo_b : c.d_geo_a;
    double *geo_next = c.flip ? c.d_geo_a : c.d_geo_b;
    T *rel_cur = (T *)(c.flip ? c.d_rel_b : c.d_rel_a);
    T *rel_next = (T *)(c.flip ? c.d_rel_a : c.d_rel_b);
    const bool fused = ic_fused(c);
    if (c.cfg.mode == PBA_IC_PROXY) {
        Launch<T>::ic_residual(s, c, level, geo_cur, ev0, ev1);
        Launch<T>::pair_reduce_y(s, c, prev_stat, conv_px, level);
        if (fused)
            launch_ic_step(s, c, c.d_geo0, geo_cur, geo_next, rel_next, is_fp64(c), ev2, ev3);
        else
            launch_solve(s, c, c.d_geo0, geo_next, rel_next, is_fp64(c), stat);
    } else {
        if (c.geo_mode)
            launch_geo_linearize(s, c, geo_cur, ev0, ev1);   // reprojection error (front end)
        else if (is_mixed(c))
            launch_linearize_mixed(s, c, level, false, geo_cur, c.iters_in_level == 0, ev0, ev1);
        else
            Launch<T>::fc_linearize(s, c, level, geo_cur, c.iters_in_level == 0, ev0, ev1);
        Launch<T>::point_reduce(s, c, true);
        if (c.geo_mode || !is_mixed(c)) Launch<T>::pair_reduce_H(s, c);
        launch_mu(s, c, geo_cur);
        launch_gram(s, c, geo_cur, c.d_rec, true);
        launch_assemble_s(s, c, geo_cur);
        if (c.tiled()) launch_tchol(s, c, false);   // the assembly wrote S into the factor buffer too
        Launch<T>::pair_reduce_y(s, c);
        launch_solve(s, c, geo_cur, geo_next, rel_next, is_fp64(c), stat);
    }
    // IC: the end of the iteration (statistics, convergence gate) is taken by the
    // next iteration's pair sums, or by a kernel of its own after the last one
    const bool finish = c.cfg.mode != PBA_IC_PROXY || last;
    if (!fused)
        Launch<T>::depth_update(s, c, geo_cur, geo_next, stat, conv_px, level, finish);
    else if (finish)
        launch_conv(s, c, stat, conv_px, du_nparts(c), level, true);
    HIPCHK(hipGetLastError());
    c.s_valid = true;
    c.flip = !c.flip;
    c.iters_in_level++;
    return PBA_OK;
}

pba_status ensure_stats(Ctx &c, int n) {
    if (n <= c.stats_cap) return PBA_OK;
    int cap = std::max(n, 64);
    HIPCHK(dalloc(c.d_stats, (size_t)cap * ST_STRIDE * sizeof(double)));
    c.stats_cap = cap;
    return PBA_OK;
}

pba_status ensure_events(Ctx &c, size_t n) {
    while (c.ev_pool.size() < n) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        c.ev_pool.push_back(e);
    }
    return PBA_OK;
}

void drop_graph(Ctx &c) {
    if (c.solve_graph) (void)hipGraphExecDestroy(c.solve_graph);
    c.solve_graph = nullptr;
    c.graph_iters = -1;
}

void fill_stats(const double *h, int level, int it0, int n, pba_iter_stats *out) {
    for (int k = 0; k < n; ++k) {
        const double *x = h + (size_t)k * ST_STRIDE;
        pba_iter_stats &o = out[k];
        o.level = level;
        o.iter = it0 + k;
        o.n_active = (int64_t)std::llround(x[ST_CNT]);
        o.energy = x[ST_E];
        o.sq = x[ST_SQ];
        o.rmse = o.n_active > 0 ? std::sqrt(x[ST_SQ] / (double)o.n_active) : 0.0;
        o.max_disp_px = x[ST_DISP];
        o.max_step_pose = x[ST_STEP_P];
        o.max_step_depth = x[ST_STEP_D];
    }
}

// Enqueue n_iters iterations without host synchronization. With conv_px >= 0
// the device closes the gate after the first iteration whose largest
// point-centre displacement is below conv_px and the remaining launches return
// at once. Returns the number of iterations that ran in *ran.
pba_status run_iterations(Ctx &c, int level, int n_iters, pba_iter_stats *out, double conv_px = -1.0,
                          int *ran = nullptr) {
    pba_status st;
    if ((st = ensure_stats(c, n_iters)) != PBA_OK) return st;
    const bool timing = (c.cfg.flags & PBA_FLAG_TIMING) != 0;
    if (timing && (st = ensure_events(c, 4 * (size_t)n_iters)) != PBA_OK) return st;
    launch_open(c.stream, c, level, true);
    const int it0 = c.iters_in_level;
    const bool flip0 = c.flip;
    const int since0 = c.since_lin, m = recentre_every(c);
    // segments between proxy re-centrings: each is a batch of its own (the
    // pose buffers alternate within a batch and are synchronized at its end)
    std::vector<int> seg_start{0};
    int kb = 0;   // iteration within the current segment
    for (int k = 0; k < n_iters; ++k) {
        if (m > 0 && c.since_lin == m) {
            if ((st = recentre_level(c, level)) != PBA_OK) return st;
            seg_start.push_back(k);
            kb = 0;
        }
        hipEvent_t e0 = timing ? c.ev_pool[4 * k] : nullptr, e1 = timing ? c.ev_pool[4 * k + 1] : nullptr;
        hipEvent_t e2 = timing ? c.ev_pool[4 * k + 2] : nullptr, e3 = timing ? c.ev_pool[4 * k + 3] : nullptr;
        double *stat = c.d_stats + (size_t)k * ST_STRIDE;
        c.batch_k = kb;
        double *prev = kb > 0 ? stat - ST_STRIDE : nullptr;
        const bool last = k == n_iters - 1 || (m > 0 && c.since_lin + 1 == m);
        ++kb;
        c.since_lin++;
        st = is_fp64(c) ? one_iteration<double>(c, level, stat, e0, e1, conv_px, prev, last, e2, e3)
                        : one_iteration<float>(c, level, stat, e0, e1, conv_px, prev, last, e2, e3);
        if (st != PBA_OK) return st;
    }
    std::vector<double> hs((size_t)n_iters * ST_STRIDE);
    int flag = 0, count = 0;
    if (n_iters > 0)
        HIPCHK(hipMemcpyAsync(hs.data(), c.d_stats, hs.size() * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipMemcpyAsync(&flag, c.d_flag, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipMemcpyAsync(&count, c.d_count + level, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    HIPCHK(hipGetLastError());
    // host view of the double buffers follows the iterations that actually ran:
    // those of the last segment that ran, from its start (flip0 and since0 for
    // the segment that continues the previous call)
    c.iters_in_level = it0 + count;
    {
        size_t si = 0;
        while (si + 1 < seg_start.size() && seg_start[si + 1] < count) ++si;
        const int j = count - seg_start[si];
        c.flip = (si == 0 ? flip0 : false) != (j % 2 == 1);
        c.since_lin = (si == 0 ? since0 : 0) + j;
    }
    n_iters = count;
    if (ran) *ran = count;
    if (timing) {
        for (int k = 0; k < n_iters; ++k) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, c.ev_pool[4 * k], c.ev_pool[4 * k + 1]));
            c.t_ms[level] += ms;
            c.t_launches[level]++;
            c.t_res[level] += (int64_t)c.O * LANES_PER_OBS;
            if (c.cfg.mode == PBA_IC_PROXY && ic_fused(c)) {
                HIPCHK(hipEventElapsedTime(&ms, c.ev_pool[4 * k + 2], c.ev_pool[4 * k + 3]));
                c.t_step_ms[level] += ms;
                c.t_step_launches[level]++;
            }
        }
    }
    if (out) fill_stats(hs.data(), level, it0, n_iters, out);
    if (flag) return fail(&c, PBA_E_NUMERIC, "reduced pose system is not positive definite");
    return PBA_OK;
}

pba_status do_start_level(Ctx &c, int level) {
    pba_status st = is_fp64(c) ? start_level<double>(c, level, true) : start_level<float>(c, level, true);
    if (st != PBA_OK) return st;
    if (c.cfg.mode == PBA_IC_PROXY) {
        int flag = 0;
        HIPCHK(hipMemcpyAsync(&flag, c.d_flag, sizeof(int), hipMemcpyDeviceToHost, c.stream));
        HIPCHK(hipStreamSynchronize(c.stream));
        if (flag) {
            c.cur_level = -1;
            return fail(&c, PBA_E_NUMERIC, "reduced pose system at p(0) is not positive definite");
        }
    }
    return PBA_OK;
}

// The whole coarse-to-fine solve (every level's start and max_iters iterations,
// each with the device convergence gate) enqueued without host synchronization;
// with PBA_FLAG_GRAPH it is captured once as a HIP graph and replayed. Level l's
// statistics go to d_stats[(n_levels - 1 - l) * max_iters + k].
template <typename T>
void aff_enqueue(Ctx &c, AffBufs &a, int level, bool first, double *stat, double conv_px, hipEvent_t e0,
                 hipEvent_t e1);

// aff: the joint pose-brightness iteration (pba_set_affine) instead of the plain one
pba_status enqueue_solve(Ctx &c, int max_iters, double conv_px, bool events, AffBufs *aff = nullptr) {
    for (int level = c.cfg.n_levels - 1; level >= 0; --level) {
        // a failure at a coarser level keeps the gate closed for the rest
        const bool clear = level == c.cfg.n_levels - 1;
        pba_status st = is_fp64(c) ? start_level<double>(c, level, clear) : start_level<float>(c, level, clear);
        if (st != PBA_OK) return st;
        const int slot = c.cfg.n_levels - 1 - level;
        if (aff) {
            // the pair geometry of the current parameters in the first buffer
            if (is_fp64(c))
                Launch<double>::relpose(c.stream, c, c.d_poses, c.d_geo_a, (double *)c.d_rel_a);
            else
                Launch<float>::relpose(c.stream, c, c.d_poses, c.d_geo_a, (float *)c.d_rel_a);
            c.flip = false;
            for (int k = 0; k < max_iters; ++k) {
                const size_t idx = (size_t)slot * max_iters + k;
                hipEvent_t e0 = events ? c.ev_pool[4 * idx] : nullptr, e1 = events ? c.ev_pool[4 * idx + 1] : nullptr;
                if (is_fp64(c))
                    aff_enqueue<double>(c, *aff, level, k == 0, c.d_stats + idx * ST_STRIDE, conv_px, e0, e1);
                else
                    aff_enqueue<float>(c, *aff, level, k == 0, c.d_stats + idx * ST_STRIDE, conv_px, e0, e1);
            }
            continue;
        }
        const int m = recentre_every(c);
        for (int k = 0; k < max_iters; ++k) {
            // proxy re-centring every m iterations (gated: nothing once the level
            // has converged); each segment is a batch of its own
            const int kb = m > 0 ? k % m : k;
            if (m > 0 && k > 0 && kb == 0 && (st = recentre_level(c, level)) != PBA_OK) return st;
            const size_t idx = (size_t)slot * max_iters + k;
            double *stat = c.d_stats + idx * ST_STRIDE;
            hipEvent_t e0 = events ? c.ev_pool[4 * idx] : nullptr, e1 = events ? c.ev_pool[4 * idx + 1] : nullptr;
            hipEvent_t e2 = events ? c.ev_pool[4 * idx + 2] : nullptr, e3 = events ? c.ev_pool[4 * idx + 3] : nullptr;
            double *prev = kb > 0 ? stat - ST_STRIDE : nullptr;
            const bool last = k == max_iters - 1 || (m > 0 && kb == m - 1);
            c.batch_k = kb;
            st = is_fp64(c) ? one_iteration<double>(c, level, stat, e0, e1, conv_px, prev, last, e2, e3)
                            : one_iteration<float>(c, level, stat, e0, e1, conv_px, prev, last, e2, e3);
            if (st != PBA_OK) return st;
        }
    }
    return PBA_OK;
}

pba_status solve_batch(Ctx &c, int max_iters, double conv_px, pba_result &res, AffBufs *aff = nullptr) {
    pba_status st;
    const int L = c.cfg.n_levels;
    if ((st = ensure_stats(c, L * max_iters)) != PBA_OK) return st;
    // residual-kernel timing with HIP events (not inside a captured graph)
    const bool timing = (c.cfg.flags & PBA_FLAG_TIMING) && !(c.cfg.flags & PBA_FLAG_GRAPH);
    if (timing && (st = ensure_events(c, 4 * (size_t)L * max_iters)) != PBA_OK) return st;
    // templates of every level first (they depend on the points only)
    for (int level = 0; level < L; ++level)
        if (!c.lv[level].tmpl_valid) {
            if (is_fp64(c))
                Launch<double>::make_template(c.stream, c, level);
            else
                Launch<float>::make_template(c.stream, c, level);
            c.lv[level].tmpl_valid = true;
        }
    if (c.cfg.flags & PBA_FLAG_GRAPH) {
        if (!c.solve_graph || c.graph_iters != max_iters || c.graph_conv != conv_px) {
            drop_graph(c);
            hipGraph_t g = nullptr;
            HIPCHK(hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal));
            st = enqueue_solve(c, max_iters, conv_px, false, aff);
            hipError_t e = hipStreamEndCapture(c.stream, &g);
            if (st != PBA_OK) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            HIPCHK(e);
            e = hipGraphInstantiate(&c.solve_graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            HIPCHK(e);
            c.graph_iters = max_iters;
            c.graph_conv = conv_px;
        }
        HIPCHK(hipGraphLaunch(c.solve_graph, c.stream));
    } else if ((st = enqueue_solve(c, max_iters, conv_px, timing, aff)) != PBA_OK) {
        return st;
    }
    std::vector<double> hs((size_t)L * max_iters * ST_STRIDE);
    int flag = 0, counts[PBA_MAX_LEVELS] = {0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(hs.data(), c.d_stats, hs.size() * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipMemcpyAsync(&flag, c.d_flag, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipMemcpyAsync(counts, c.d_count, sizeof(counts), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    HIPCHK(hipGetLastError());
    std::vector<pba_iter_stats> its(max_iters);
    if (timing) {
        for (int level = L - 1; level >= 0; --level)
            for (int k = 0; k < counts[level]; ++k) {
                const size_t idx = (size_t)(L - 1 - level) * max_iters + k;
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, c.ev_pool[4 * idx], c.ev_pool[4 * idx + 1]));
                c.t_ms[level] += ms;
                c.t_launches[level]++;
                c.t_res[level] += (int64_t)c.O * LANES_PER_OBS;
                if (!aff && c.cfg.mode == PBA_IC_PROXY && ic_fused(c)) {
                    HIPCHK(hipEventElapsedTime(&ms, c.ev_pool[4 * idx + 2], c.ev_pool[4 * idx + 3]));
                    c.t_step_ms[level] += ms;
                    c.t_step_launches[level]++;
                }
            }
    }
    for (int level = L - 1; level >= 0; --level) {
        const int k = counts[level];
        fill_stats(hs.data() + (size_t)(L - 1 - level) * max_iters * ST_STRIDE, level, 0, k, its.data());
        for (int i = 0; i < k; ++i) res.active_residuals += its[i].n_active;
        res.iters[level] = k;
        res.total_iters += k;
        if (level == 0) res.converged = (k > 0 && its[k - 1].max_disp_px < conv_px) ? 1 : 0;
    }
    // host view of the level-0 double buffers: the iterations of the last
    // segment (since the last re-centring) that ran
    c.cur_level = 0;
    c.iters_in_level = counts[0];
    if (aff) {
        c.flip = false;   // the joint iteration keeps the pair geometry in the first buffer
        c.s_valid = false;
    } else {
        const int m = recentre_every(c), kl = counts[0];
        const int seg = (m > 0 && kl > 0) ? kl - m * ((kl - 1) / m) : kl;
        c.flip = seg % 2 == 1;
        c.since_lin = seg;
    }
    if (flag) {
        c.cur_level = -1;
        return fail(&c, PBA_E_NUMERIC, "reduced pose system is not positive definite");
    }
    return PBA_OK;
}

// ---- device state from host arrays (one window, or the assembled windows)

// Frames: images (host or device float32 [F][H][W]), level-0 intrinsics and
// poses, and the window partition of the frames.
pba_status load_frames(Ctx &c, int n_frames, int width, int height, const float *images, int mem,
                       const std::vector<double> &K, const std::vector<double> &Pz, const std::vector<int> &frame_off) {
    HIPCHK(hipStreamSynchronize(c.stream));
    release_frames(c);
    c.F = n_frames;
    c.W = width;
    c.H = height;
    c.K0 = K;
    c.nwin = (int)frame_off.size() - 1;
    c.win_frame_off = frame_off;
    const size_t npx = (size_t)n_frames * width * height;
    const size_t rs = c.real_size;
    int W = width, H = height;
    for (int l = 0; l < c.cfg.n_levels; ++l) {
        c.lv[l].W = W;
        c.lv[l].H = H;
        HIPCHK(dalloc(c.lv[l].img, (size_t)n_frames * W * H * rs));
        HIPCHK(dalloc(c.lv[l].K, (size_t)n_frames * 4 * rs));
        W /= 2;
        H /= 2;
    }
    float *staging = nullptr;
    const float *src = images;
    if (mem == PBA_HOST) {
        HIPCHK(dalloc(staging, npx * sizeof(float)));
        HIPCHK(hipMemcpyAsync(staging, images, npx * sizeof(float), hipMemcpyHostToDevice, c.stream));
        src = staging;
    }
    HIPCHK(dalloc(c.d_K0, K.size() * sizeof(double)));
    HIPCHK(hipMemcpyAsync(c.d_K0, K.data(), K.size() * sizeof(double), hipMemcpyHostToDevice, c.stream));
    if (is_fp64(c)) {
        Launch<double>::convert_images(c.stream, src, (double *)c.lv[0].img, npx);
        for (int l = 1; l < c.cfg.n_levels; ++l)
            Launch<double>::downsample(c.stream, (double *)c.lv[l - 1].img, (double *)c.lv[l].img, n_frames,
                                       c.lv[l - 1].W, c.lv[l - 1].H, c.lv[l].W, c.lv[l].H);
        for (int l = 0; l < c.cfg.n_levels; ++l) Launch<double>::level_K(c.stream, c.d_K0, (double *)c.lv[l].K, n_frames, l);
    } else {
        Launch<float>::convert_images(c.stream, src, (float *)c.lv[0].img, npx);
        for (int l = 1; l < c.cfg.n_levels; ++l)
            Launch<float>::downsample(c.stream, (float *)c.lv[l - 1].img, (float *)c.lv[l].img, n_frames,
                                      c.lv[l - 1].W, c.lv[l - 1].H, c.lv[l].W, c.lv[l].H);
        for (int l = 0; l < c.cfg.n_levels; ++l) Launch<float>::level_K(c.stream, c.d_K0, (float *)c.lv[l].K, n_frames, l);
    }
    // per-window blocks of the reduced system
    std::vector<int> frame_win(n_frames);
    c.win_S_off.assign(c.nwin + 1, 0);
    c.win_L_off.assign(c.nwin + 1, 0);
    for (int w = 0; w < c.nwin; ++w) {
        const long long nw = 6LL * (frame_off[w + 1] - frame_off[w]);
        for (int f = frame_off[w]; f < frame_off[w + 1]; ++f) frame_win[f] = w;
        if (c.win_S_off[w] + nw * nw > INT32_MAX) return fail(&c, PBA_E_INVALID, "reduced system too large");
        c.win_S_off[w + 1] = (int)(c.win_S_off[w] + nw * nw);
        c.win_L_off[w + 1] = (int)(c.win_L_off[w] + nw * (nw + 1) / 2 + nw);
    }
    HIPCHK(upload(c, c.d_win_frame_off, c.win_frame_off));
    HIPCHK(upload(c, c.d_frame_win, frame_win));
    HIPCHK(upload(c, c.d_win_S_off, c.win_S_off));
    HIPCHK(upload(c, c.d_win_L_off, c.win_L_off));
    const size_t n6 = 6 * (size_t)n_frames;
    const size_t nS = (size_t)c.win_S_off[c.nwin], nL = (size_t)c.win_L_off[c.nwin];
    HIPCHK(dalloc(c.d_poses, Pz.size() * sizeof(double)));
    HIPCHK(dalloc(c.d_poses0, Pz.size() * sizeof(double)));
    HIPCHK(dalloc(c.d_poses_alt, Pz.size() * sizeof(double)));
    HIPCHK(hipMemcpyAsync(c.d_poses, Pz.data(), Pz.size() * sizeof(double), hipMemcpyHostToDevice, c.stream));
    HIPCHK(dalloc(c.d_S, nS * sizeof(double)));
    if (c.cfg.mode == PBA_IC_PROXY) {
        HIPCHK(dalloc(c.d_Sinv, nS * sizeof(double)));
        HIPCHK(dalloc(c.d_Lfac, nL * sizeof(double)));
    }
    if (c.tiled()) {
        const size_t nt = (n6 + TCHOL_TILE - 1) / TCHOL_TILE;
        HIPCHK(dalloc(c.d_Sfac, n6 * n6 * sizeof(double)));
        HIPCHK(dalloc(c.d_Linv, nt * TCHOL_TILE * TCHOL_TILE * sizeof(double)));
    }
    HIPCHK(dalloc(c.d_b, 2 * n6 * sizeof(double)));
    HIPCHK(dalloc(c.d_dtheta, n6 * sizeof(double)));
    HIPCHK(dalloc(c.d_mu, 2 * (size_t)c.nwin * sizeof(double)));
    HIPCHK(dalloc(c.d_wstat, 4 * (size_t)c.nwin * sizeof(double)));
    HIPCHK(dalloc(c.d_flag, sizeof(int)));
    HIPCHK(dalloc(c.d_gate, sizeof(int)));
    HIPCHK(dalloc(c.d_count, PBA_MAX_LEVELS * sizeof(int)));
    HIPCHK(dalloc(c.d_count_base, PBA_MAX_LEVELS * sizeof(int)));
    HIPCHK(hipMemsetAsync(c.d_flag, 0, sizeof(int), c.stream));
    HIPCHK(hipMemsetAsync(c.d_count, 0, PBA_MAX_LEVELS * sizeof(int), c.stream));
    HIPCHK(hipMemsetAsync(c.d_count_base, 0, PBA_MAX_LEVELS * sizeof(int), c.stream));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c.stream));
    dfree(staging);
    c.have_frames = true;
    c.cur_level = -1;
    return PBA_OK;
}

// Bits of x and y interleaved (x in the even bits): the Z-order of a cell.
uint64_t morton2(uint32_t x, uint32_t y) {
    uint64_t m = 0;
    for (int b = 0; b < 16; ++b) m |= ((uint64_t)((x >> b) & 1u) << (2 * b)) | ((uint64_t)((y >> b) & 1u) << (2 * b + 1));
    return m;
}

// Internal order of the points of every window: by host frame, then by the
// Z-order of the host pixel's 4 x 4-pixel cell (ties in the caller's order).
// Neighbouring points of a host warp to neighbouring positions of each target,
// so consecutive observations share texel lines and a contiguous range of
// points (which the residual kernel maps to one XCD) stays in a compact image
// region. Returns the caller's index of every internal point.
std::vector<int> spatial_order(int n_points, const std::vector<int> &hf, const std::vector<float> &uv,
                               const std::vector<int> &point_off) {
    std::vector<int> perm(n_points);
    std::vector<uint64_t> key(n_points);
    for (int n = 0; n < n_points; ++n) {
        perm[n] = n;
        const uint32_t cx = (uint32_t)std::max(0.0f, uv[2 * (size_t)n]) >> 2;
        const uint32_t cy = (uint32_t)std::max(0.0f, uv[2 * (size_t)n + 1]) >> 2;
        key[n] = ((uint64_t)(uint32_t)hf[n] << 32) | morton2(cx & 0xffffu, cy & 0xffffu);
    }
    for (size_t w = 0; w + 1 < point_off.size(); ++w)
        std::stable_sort(perm.begin() + point_off[w], perm.begin() + point_off[w + 1],
                         [&](int a, int b) { return key[a] < key[b]; });
    return perm;
}

pba_status load_points_ordered(Ctx &c, int n_points, const std::vector<int> &hf, const std::vector<float> &uv,
                               const std::vector<double> &d, const std::vector<int> &optr,
                               const std::vector<int> &ofr, const std::vector<int> &point_off);

// Points and observations (global frame indices, the caller's order) and
// their window partition: reordered (spatial_order) and loaded.
pba_status load_points(Ctx &c, int n_points, const std::vector<int> &hf, const std::vector<float> &uv,
                       const std::vector<double> &d, const std::vector<int> &optr, const std::vector<int> &ofr,
                       const std::vector<int> &point_off) {
    const std::vector<int> perm = spatial_order(n_points, hf, uv, point_off);
    std::vector<int> hf2(n_points), optr2(n_points + 1, 0), ofr2(ofr.size()), obs_caller(ofr.size());
    std::vector<float> uv2(2 * (size_t)n_points);
    std::vector<double> d2(n_points);
    for (int i = 0; i < n_points; ++i) {
        const int n = perm[i];
        hf2[i] = hf[n];
        uv2[2 * (size_t)i] = uv[2 * (size_t)n];
        uv2[2 * (size_t)i + 1] = uv[2 * (size_t)n + 1];
        d2[i] = d[n];
        int o2 = optr2[i];
        for (int o = optr[n]; o < optr[n + 1]; ++o, ++o2) {
            ofr2[o2] = ofr[o];
            obs_caller[o2] = o;
        }
        optr2[i + 1] = o2;
    }
    const pba_status st = load_points_ordered(c, n_points, hf2, uv2, d2, optr2, ofr2, point_off);
    if (st == PBA_OK) {
        c.pt_caller = perm;
        c.obs_caller = std::move(obs_caller);
    }
    return st;
}

pba_status load_points_ordered(Ctx &c, int n_points, const std::vector<int> &hf, const std::vector<float> &uv,
                               const std::vector<double> &d, const std::vector<int> &optr,
                               const std::vector<int> &ofr, const std::vector<int> &point_off) {
    const long long O = optr[n_points];
    HIPCHK(hipStreamSynchronize(c.stream));
    release_points(c);
    c.N = n_points;
    c.O = (int)O;
    const std::string e = build_structure(c, hf, optr, ofr);
    if (!e.empty()) {
        c.N = c.O = 0;
        return fail(&c, PBA_E_INVALID, e);
    }
    const Structure &s = c.st;
    // window partition of points and pairs (pairs are sorted by host frame)
    c.win_point_off = point_off;
    std::vector<int> point_win(n_points), frame_win(c.F);
    for (int w = 0; w < c.nwin; ++w) {
        for (int n = point_off[w]; n < point_off[w + 1]; ++n) point_win[n] = w;
        for (int f = c.win_frame_off[w]; f < c.win_frame_off[w + 1]; ++f) frame_win[f] = w;
    }
    c.win_pair_off.assign(c.nwin + 1, 0);
    for (int p = 0; p < s.n_pairs; ++p) c.win_pair_off[frame_win[s.pair_host[p]] + 1]++;
    for (int w = 0; w < c.nwin; ++w) c.win_pair_off[w + 1] += c.win_pair_off[w];
    HIPCHK(upload(c, c.d_win_point_off, c.win_point_off));
    HIPCHK(upload(c, c.d_win_pair_off, c.win_pair_off));
    HIPCHK(upload(c, c.d_point_win, point_win));
    HIPCHK(upload(c, c.d_host_frame, hf));
    HIPCHK(upload(c, c.d_obs_ptr, optr));
    HIPCHK(upload(c, c.d_obs_frame, ofr));
    HIPCHK(upload(c, c.d_host_uv, uv));
    HIPCHK(upload(c, c.d_obs_point, s.obs_point));
    HIPCHK(upload(c, c.d_obs_pair, s.obs_pair));
    HIPCHK(upload(c, c.d_pair_host, s.pair_host));
    HIPCHK(upload(c, c.d_pair_target, s.pair_target));
    HIPCHK(upload(c, c.d_pair_obs_ptr, s.pair_obs_ptr));
    HIPCHK(upload(c, c.d_pair_obs_idx, s.pair_obs_idx));
    HIPCHK(upload(c, c.d_frame_pair_ptr, s.frame_pair_ptr));
    HIPCHK(upload(c, c.d_frame_pair_item, s.frame_pair_item));
    HIPCHK(upload(c, c.d_pair_local, s.pair_local));
    HIPCHK(upload(c, c.d_pair_hidx, s.pair_hidx));
    HIPCHK(upload(c, c.d_host_m, s.host_m));
    HIPCHK(upload(c, c.d_host_frames, s.hosts));
    HIPCHK(upload(c, c.d_host_pts, s.host_pts));
    HIPCHK(upload(c, c.d_chunk_host, s.chunk_host));
    HIPCHK(upload(c, c.d_chunk_begin, s.chunk_begin));
    HIPCHK(upload(c, c.d_chunk_end, s.chunk_end));
    HIPCHK(upload(c, c.d_chunk_off, s.chunk_off));
    HIPCHK(upload(c, c.d_host_chunk_ptr, s.host_chunk_ptr));
    HIPCHK(upload(c, c.d_blk_fa, s.blk_fa));
    HIPCHK(upload(c, c.d_blk_fb, s.blk_fb));
    HIPCHK(upload(c, c.d_blk_pp_ptr, s.blk_pp_ptr));
    HIPCHK(upload(c, c.d_blk_pp_item, s.blk_pp_item));
    HIPCHK(upload(c, c.d_blk_g_ptr, s.blk_g_ptr));
    HIPCHK(upload(c, c.d_blk_g_item, s.blk_g_item));
    HIPCHK(upload(c, c.d_pchunk_begin, s.pchunk_begin));
    HIPCHK(upload(c, c.d_pchunk_end, s.pchunk_end));
    HIPCHK(upload(c, c.d_pair_chunk_ptr, s.pair_chunk_ptr));
    HIPCHK(upload(c, c.d_depth, d));
    HIPCHK(dalloc(c.d_depth0, std::max<size_t>(1, n_points) * sizeof(double)));
    const size_t rs = c.real_size;
    const int Pn = s.n_pairs;
    HIPCHK(dalloc(c.d_mask, std::max<size_t>(1, O)));
    HIPCHK(dalloc(c.d_obs_live, std::max<size_t>(1, O)));
    HIPCHK(hipMemsetAsync(c.d_obs_live, 1, std::max<size_t>(1, O), c.stream));
    HIPCHK(dalloc(c.d_rec, (size_t)O * REC_STRIDE * sizeof(double)));   // records: FP64 for every element type
    HIPCHK(dalloc(c.d_geo0, (size_t)Pn * GEO_STRIDE * sizeof(double)));
    HIPCHK(dalloc(c.d_geo_a, (size_t)Pn * GEO_STRIDE * sizeof(double)));
    HIPCHK(dalloc(c.d_geo_b, (size_t)Pn * GEO_STRIDE * sizeof(double)));
    HIPCHK(dalloc(c.d_rel0, (size_t)Pn * REL_STRIDE * rs));
    HIPCHK(dalloc(c.d_rel_a, (size_t)Pn * REL_STRIDE * rs));
    HIPCHK(dalloc(c.d_rel_b, (size_t)Pn * REL_STRIDE * rs));
    HIPCHK(dalloc(c.d_pairH, (size_t)Pn * 21 * sizeof(double)));
    HIPCHK(dalloc(c.d_pairY, (size_t)Pn * 9 * sizeof(double)));
    HIPCHK(dalloc(c.d_partH, s.pchunk_begin.size() * 21 * sizeof(double)));
    HIPCHK(dalloc(c.d_partY, s.pchunk_begin.size() * 9 * sizeof(double)));
    HIPCHK(dalloc(c.d_obsmap, (size_t)O * 12 * sizeof(double)));
    HIPCHK(dalloc(c.d_hc, (size_t)O * 6 * sizeof(double)));
    HIPCHK(dalloc(c.d_Hdd, (size_t)n_points * sizeof(double)));
    HIPCHK(dalloc(c.d_gd, (size_t)n_points * sizeof(double)));
    HIPCHK(dalloc(c.d_gram, s.gram_floats * sizeof(double)));
    HIPCHK(dalloc(c.d_dth_rel, (size_t)Pn * 6 * sizeof(double)));
    HIPCHK(dalloc(c.d_du_part, 2 * (size_t)std::max(1, (n_points + 31) / 32) * sizeof(double)));
    {
        std::vector<double> pk((size_t)Pn * 8);
        for (int p = 0; p < Pn; ++p)
            for (int k = 0; k < 4; ++k) {
                pk[8 * (size_t)p + k] = c.K0[4 * (size_t)s.pair_host[p] + k];
                pk[8 * (size_t)p + 4 + k] = c.K0[4 * (size_t)s.pair_target[p] + k];
            }
        HIPCHK(upload(c, c.d_pairK0, pk));
        // per slot t of pair chunk k (slot k * PAIR_CHUNK + t): the observation,
        // its point and the point's observation range; observation -1 past the
        // chunk's end
        const size_t nsl = s.pchunk_begin.size() * (size_t)PAIR_CHUNK;
        std::vector<int> sl(4 * std::max<size_t>(nsl, 1), 0);
        for (size_t k = 0; k < s.pchunk_begin.size(); ++k)
            for (int t = 0; t < PAIR_CHUNK; ++t) {
                int *e = &sl[4 * (k * PAIR_CHUNK + t)];
                const int i = s.pchunk_begin[k] + t;
                if (i >= s.pchunk_end[k]) {
                    e[0] = -1;
                    continue;
                }
                const int o = s.pair_obs_idx[i], n = s.obs_point[o];
                e[0] = o;
                e[1] = n;
                e[2] = optr[n];
                e[3] = optr[n + 1];
            }
        HIPCHK(upload(c, c.d_pc_slot, sl));
        // frames each depth workgroup of the fused IC step observes
        dfree(c.d_step_sel);
        c.step_sel_max = 0;
        const int nbk = (n_points + IC_STEP_PTS - 1) / IC_STEP_PTS;
        if (c.F <= STEP_SEL_STRIDE - 4 && nbk > 0) {
            std::vector<unsigned long long> mask((size_t)nbk, 0ull);
            for (int o = 0; o < O; ++o) {
                const int p = s.obs_pair[o];
                mask[(size_t)(s.obs_point[o] / IC_STEP_PTS)] |= (1ull << s.pair_host[p]) | (1ull << s.pair_target[p]);
            }
            std::vector<int> sel((size_t)nbk * STEP_SEL_STRIDE, 0);
            for (int b = 0; b < nbk; ++b) {
                int *e = sel.data() + (size_t)b * STEP_SEL_STRIDE;
                for (int f = 0; f < c.F; ++f)
                    if ((mask[(size_t)b] >> f) & 1ull) e[1 + e[0]++] = f;
                e[STEP_SEL_STRIDE - 2] = (int)(unsigned)(mask[(size_t)b] & 0xffffffffull);
                e[STEP_SEL_STRIDE - 1] = (int)(unsigned)(mask[(size_t)b] >> 32);
                c.step_sel_max = std::max(c.step_sel_max, e[0]);
            }
            HIPCHK(upload(c, c.d_step_sel, sel));
        }
    }
    HIPCHK(dalloc(c.d_icr, (size_t)O * IC_REC * sizeof(double)));
    HIPCHK(dalloc(c.d_gdo, (size_t)O * sizeof(double)));
    for (int l = 0; l < c.cfg.n_levels; ++l) {
        HIPCHK(dalloc(c.lv[l].tmpl, (size_t)n_points * c.P * 4 * rs));
        HIPCHK(dalloc(c.lv[l].pcam, (size_t)std::max(1, Pn) * 8 * sizeof(double)));
        c.lv[l].tmpl_valid = false;
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c.stream));
    c.have_points = true;
    c.cur_level = -1;
    return PBA_OK;
}

// Batched context: assemble the staged windows into the global problem (frames
// and points of window w follow those of windows < w).
pba_status assemble_windows(pba_ctx *ctx) {
    Ctx &c = ctx->c;
    const int nw = c.cfg.n_windows;
    std::vector<int> frame_off(nw + 1, 0), point_off(nw + 1, 0);
    for (int w = 0; w < nw; ++w) {
        const WinStage &st = ctx->stage[w];
        if (!st.have_frames || !st.have_points)
            return fail(&c, PBA_E_STATE, "window " + std::to_string(w) + " has no frames or points");
        frame_off[w + 1] = frame_off[w] + st.F;
        point_off[w + 1] = point_off[w] + st.N;
    }
    const int F = frame_off[nw], N = point_off[nw];
    const int W = ctx->stage_W, H = ctx->stage_H;
    const size_t fpx = (size_t)W * H;
    // images straight into one device buffer, window by window
    HIPCHK(hipStreamSynchronize(c.stream));
    release_frames(c);
    float *dimg = nullptr;
    HIPCHK(dalloc(dimg, (size_t)F * fpx * sizeof(float)));
    std::vector<double> K, Pz;
    for (int w = 0; w < nw; ++w) {
        const WinStage &st = ctx->stage[w];
        HIPCHK(hipMemcpyAsync(dimg + (size_t)frame_off[w] * fpx, st.img.data(), st.img.size() * sizeof(float),
                              hipMemcpyHostToDevice, c.stream));
        K.insert(K.end(), st.K.begin(), st.K.end());
        Pz.insert(Pz.end(), st.P.begin(), st.P.end());
    }
    pba_status r = load_frames(c, F, W, H, dimg, PBA_DEVICE, K, Pz, frame_off);
    dfree(dimg);
    if (r != PBA_OK) return r;
    std::vector<int> hf, optr{0}, ofr;
    std::vector<float> uv;
    std::vector<double> d;
    hf.reserve(N);
    for (int w = 0; w < nw; ++w) {
        const WinStage &st = ctx->stage[w];
        for (int n = 0; n < st.N; ++n) {
            hf.push_back(st.hf[n] + frame_off[w]);
            for (int o = st.optr[n]; o < st.optr[n + 1]; ++o) ofr.push_back(st.ofr[o] + frame_off[w]);
            optr.push_back((int)ofr.size());
        }
        uv.insert(uv.end(), st.uv.begin(), st.uv.end());
        d.insert(d.end(), st.d.begin(), st.d.end());
    }
    r = load_points(c, N, hf, uv, d, optr, ofr, point_off);
    if (r != PBA_OK) return r;
    ctx->dirty = false;
    return PBA_OK;
}

// Device state current (assembles a batched context's staged windows).
pba_status ready(pba_ctx *ctx) {
    Ctx &c = ctx->c;
    if (c.cfg.n_windows > 1 && ctx->dirty) return assemble_windows(ctx);
    if (!c.have_points) return fail(&c, PBA_E_STATE, "pba_set_frames and pba_set_points must be called first");
    return PBA_OK;
}

// ---- learned preconditioner buffers

void release_pc(Ctx &c) {
    PcState &p = c.pc;
    for (float **q : {&p.w, &p.m, &p.v, &p.grad, &p.X, &p.Y, &p.Z1, &p.H1, &p.Z2, &p.H2, &p.Yt, &p.dY, &p.D1, &p.D2,
                      &p.lossv, &p.Xb, &p.Gb, &p.Gs, &p.Xs})
        dfree(*q);
    for (double **q : {&p.Ci, &p.G, &p.P, &p.x, &p.r, &p.z, &p.p, &p.q, &p.part, &p.sc, &p.lsum}) dfree(*q);
    dfree(p.wh);
    dfree(p.flag);
    dfree(p.st);
    dfree(p.idx);
    p = PcState();
}

pba_status pc_ensure_weights(Ctx &c) {
    PcState &p = c.pc;
    if (p.w) return PBA_OK;
    HIPCHK(dalloc(p.w, PC_N_PARAMS * sizeof(float)));
    HIPCHK(dalloc(p.m, PC_N_PARAMS * sizeof(float)));
    HIPCHK(dalloc(p.v, PC_N_PARAMS * sizeof(float)));
    HIPCHK(dalloc(p.grad, PC_N_PARAMS * sizeof(float)));
    HIPCHK(dalloc(p.wh, (size_t)(256 * 32 + 256 * 256 + 32 * 256) * sizeof(_Float16)));
    HIPCHK(dalloc(p.lsum, sizeof(double)));
    HIPCHK(dalloc(p.flag, sizeof(int)));
    HIPCHK(dalloc(p.st, 2 * sizeof(int)));
    return PBA_OK;
}

pba_status pc_ensure_system(Ctx &c, int nb) {
    PcState &p = c.pc;
    if (nb <= p.nb_cap) return PBA_OK;
    const size_t n = 6 * (size_t)nb, parts = (n + 7) / 8 + 1;
    HIPCHK(dalloc(p.Ci, (size_t)nb * 36 * sizeof(double)));
    HIPCHK(dalloc(p.G, (size_t)nb * 21 * sizeof(double)));
    HIPCHK(dalloc(p.P, (size_t)nb * 36 * sizeof(double)));
    HIPCHK(dalloc(p.X, (size_t)nb * PC_IN * sizeof(float)));
    HIPCHK(dalloc(p.Y, (size_t)nb * PC_OUT * sizeof(float)));
    for (double **q : {&p.x, &p.r, &p.z, &p.p, &p.q}) HIPCHK(dalloc(*q, n * sizeof(double)));
    HIPCHK(dalloc(p.part, parts * sizeof(double)));
    HIPCHK(dalloc(p.sc, 4 * sizeof(double)));
    p.nb_cap = nb;
    return PBA_OK;
}

pba_status pc_ensure_batch(Ctx &c, int B) {
    PcState &p = c.pc;
    if (B <= p.b_cap) return PBA_OK;
    for (float **q : {&p.Z1, &p.H1, &p.Z2, &p.H2, &p.D1, &p.D2}) HIPCHK(dalloc(*q, (size_t)B * 256 * sizeof(float)));
    HIPCHK(dalloc(p.Yt, (size_t)B * PC_OUT * sizeof(float)));
    HIPCHK(dalloc(p.dY, (size_t)B * PC_OUT * sizeof(float)));
    HIPCHK(dalloc(p.lossv, (size_t)B * sizeof(float)));
    HIPCHK(dalloc(p.Xb, (size_t)B * PC_IN * sizeof(float)));
    HIPCHK(dalloc(p.Gb, (size_t)B * 21 * sizeof(float)));
    HIPCHK(dalloc(p.idx, (size_t)B * sizeof(int)));
    p.b_cap = B;
    return PBA_OK;
}

// Samples G [m][21] to the device (Gb) and their features (Xb).
pba_status pc_upload_samples(Ctx &c, int m, const float *G) {
    pba_status st;
    if ((st = pc_ensure_batch(c, m)) != PBA_OK) return st;
    for (int i = 0; i < m * 21; ++i)
        if (!std::isfinite(G[i])) return fail(&c, PBA_E_INVALID, "couplings must be finite");
    HIPCHK(hipMemcpyAsync(c.pc.Gb, G, (size_t)m * 21 * sizeof(float), hipMemcpyHostToDevice, c.stream));
    pc_features(c.stream, m, c.pc.Gb, c.pc.Xb);
    return PBA_OK;
}

// ---- per-frame affine brightness in the FC iteration (pba_set_affine)

void aff_release(AffBufs &a) {
    for (double **p : {&a.ab, &a.arec, &a.M, &a.fac, &a.Linv, &a.b, &a.x, &a.dphi, &a.poses_old, &a.stats}) dfree(*p);
    dfree(a.maxb);
    dfree(a.flag);
    a = AffBufs();
}

// Buffers for the context's current frames and observations; the brightness
// parameters are kept while the frame count is unchanged, else set to zero.
pba_status aff_ensure(Ctx &c, AffBufs &a) {
    if (a.ab && a.F == c.F && a.O == c.O) return PBA_OK;
    drop_graph(c);   // a captured solve holds the old buffers
    const bool keep_ab = a.ab && a.F == c.F;
    const size_t n8 = 8 * (size_t)c.F, nt = (n8 + TCHOL_TILE - 1) / TCHOL_TILE, d = sizeof(double);
    if (!keep_ab) {
        HIPCHK(dalloc(a.ab, 2 * (size_t)c.F * d));
        HIPCHK(hipMemsetAsync(a.ab, 0, 2 * (size_t)c.F * d, c.stream));
    }
    HIPCHK(dalloc(a.arec, (size_t)c.O * AFF_STRIDE * d));
    HIPCHK(dalloc(a.M, n8 * n8 * d));
    HIPCHK(dalloc(a.fac, n8 * n8 * d));
    HIPCHK(dalloc(a.Linv, nt * TCHOL_TILE * TCHOL_TILE * d));
    HIPCHK(dalloc(a.b, n8 * d));
    HIPCHK(dalloc(a.x, n8 * d));
    HIPCHK(dalloc(a.dphi, 2 * (size_t)c.F * d));
    HIPCHK(dalloc(a.poses_old, 12 * (size_t)c.F * d));
    HIPCHK(dalloc(a.stats, sum_stats_doubles(c) * d));
    HIPCHK(dalloc(a.maxb, 4 * sizeof(unsigned long long)));
    HIPCHK(dalloc(a.flag, 2 * sizeof(int)));
    HIPCHK(hipMemsetAsync(a.flag, 0, 2 * sizeof(int), c.stream));
    a.F = c.F;
    a.O = c.O;
    return PBA_OK;
}

std::string aff_check(const Ctx &c) {
    if (c.cfg.mode != PBA_FC) return "the brightness model runs in the FC iteration (mode PBA_FC)";
    if (c.cfg.precision == PBA_MIXED_BF16) return "the brightness model needs PBA_FP64 or PBA_FP32";
    if (c.nwin != 1) return "the brightness model takes one window (n_windows = 1)";
    return "";
}

// Residual statistics of the brightness model at the current parameters over
// the residuals usable there (level's template), into out (energy, sq, count).
template <typename T>
pba_status aff_evaluate(Ctx &c, AffBufs &a, int level, double out[3]) {
    hipStream_t s = c.stream;
    if (!c.lv[level].tmpl_valid) {
        Launch<T>::make_template(s, c, level);
        c.lv[level].tmpl_valid = true;
    }
    double *geo = c.flip ? c.d_geo_b : c.d_geo_a;
    Launch<T>::relpose(s, c, c.d_poses, geo, (T *)(c.flip ? c.d_rel_b : c.d_rel_a));
    launch_aff_linearize(s, c, a, level, geo, 2);
    if (c.O > 0)
        launch_sum_stats(s, c, c.d_rec, true, a.stats);
    else
        launch_fill(s, a.stats, 3, 0.0, nullptr);
    HIPCHK(hipMemcpyAsync(out, a.stats, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipGetLastError());
    return PBA_OK;
}

// One joint iteration at `level` (the level started), enqueued: the records,
// the FC assembly of the pose block, the joint system, its solve, the
// updates and the iteration's end (statistics slot `stat`, count, gate). e0 /
// e1 (optional): events around the linearization.
template <typename T>
void aff_enqueue(Ctx &c, AffBufs &a, int level, bool first, double *stat, double conv_px, hipEvent_t e0,
                 hipEvent_t e1) {
    hipStream_t s = c.stream;
    double *geo = c.d_geo_a;
    if (e0) (void)hipEventRecord(e0, s);
    launch_aff_linearize(s, c, a, level, geo, first ? 1 : 0);
    if (e1) (void)hipEventRecord(e1, s);
    Launch<T>::point_reduce(s, c, true);
    Launch<T>::pair_reduce_H(s, c);
    launch_mu(s, c, geo);
    launch_gram(s, c, geo, c.d_rec, true);
    launch_assemble_s(s, c, geo);
    if (c.O > 0)
        launch_sum_stats(s, c, c.d_rec, true, a.stats);
    else
        launch_fill(s, a.stats, 3, 0.0, nullptr);
    launch_aff_system(s, c, a, geo);
    launch_dense_solve(s, 8 * c.F, a.M, a.fac, a.Linv, a.b, a.x, a.flag, c.d_gate);
    launch_aff_update(s, c, a, geo);
    launch_aff_stat(s, c, a, level, stat, conv_px);
    Launch<T>::relpose(s, c, c.d_poses, geo, (T *)c.d_rel_a);   // the pair geometry of the current parameters
}

// Up to n_iters joint iterations at `level` (started) without host
// synchronization in between; with conv_px >= 0 the device stops after the
// first whose displacement is below conv_px. One synchronization at the end;
// *ran = the iterations that ran.
pba_status aff_run(Ctx &c, AffBufs &a, int level, int n_iters, double conv_px, pba_iter_stats *out, int *ran) {
    pba_status st;
    if ((st = aff_ensure(c, a)) != PBA_OK) return st;
    if ((st = ensure_stats(c, n_iters)) != PBA_OK) return st;
    const bool timing = (c.cfg.flags & PBA_FLAG_TIMING) != 0;
    if (timing && (st = ensure_events(c, 2 * (size_t)n_iters)) != PBA_OK) return st;
    launch_open(c.stream, c, level, true);
    // the current pair geometry in the first buffer
    if (is_fp64(c))
        Launch<double>::relpose(c.stream, c, c.d_poses, c.d_geo_a, (double *)c.d_rel_a);
    else
        Launch<float>::relpose(c.stream, c, c.d_poses, c.d_geo_a, (float *)c.d_rel_a);
    c.flip = false;
    const int it0 = c.iters_in_level;
    for (int k = 0; k < n_iters; ++k) {
        hipEvent_t e0 = timing ? c.ev_pool[2 * k] : nullptr, e1 = timing ? c.ev_pool[2 * k + 1] : nullptr;
        double *stat = c.d_stats + (size_t)k * ST_STRIDE;
        if (is_fp64(c))
            aff_enqueue<double>(c, a, level, it0 + k == 0, stat, conv_px, e0, e1);
        else
            aff_enqueue<float>(c, a, level, it0 + k == 0, stat, conv_px, e0, e1);
    }
    HIPCHK(hipGetLastError());
    std::vector<double> hs((size_t)n_iters * ST_STRIDE);
    int flag = 0, count = 0;
    if (n_iters > 0)
        HIPCHK(hipMemcpyAsync(hs.data(), c.d_stats, hs.size() * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipMemcpyAsync(&flag, c.d_flag, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipMemcpyAsync(&count, c.d_count + level, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    HIPCHK(hipGetLastError());
    c.s_valid = false;   // d_S holds the pose block only
    c.iters_in_level = it0 + count;
    if (timing)
        for (int k = 0; k < count; ++k) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, c.ev_pool[2 * k], c.ev_pool[2 * k + 1]));
            c.t_ms[level] += ms;
            c.t_launches[level]++;
            c.t_res[level] += (int64_t)c.O * LANES_PER_OBS;
        }
    if (out) fill_stats(hs.data(), level, it0, count, out);
    if (ran) *ran = count;
    if (flag) return fail(&c, PBA_E_NUMERIC, "joint pose-brightness system is not positive definite");
    return PBA_OK;
}

std::string pc_system_check(Ctx &c) {
    if (c.nwin != 1) return "the reduced-system solvers take one window (n_windows = 1)";
    if (!c.s_valid) return "no reduced system assembled yet (run an iteration first)";
    return "";
}

}  // namespace

// ================================================================ C ABI

namespace pba {
pba_status fail_global(pba_status s, const std::string &msg) { return fail(nullptr, s, msg); }
}  // namespace pba

extern "C" {

const char *pba_status_string(pba_status s) {
    switch (s) {
        case PBA_OK: return "PBA_OK";
        case PBA_E_INVALID: return "PBA_E_INVALID";
        case PBA_E_STATE: return "PBA_E_STATE";
        case PBA_E_OOM: return "PBA_E_OOM";
        case PBA_E_DEVICE: return "PBA_E_DEVICE";
        case PBA_E_NUMERIC: return "PBA_E_NUMERIC";
        case PBA_E_NOT_CONVERGED: return "PBA_E_NOT_CONVERGED";
    }
    return "unknown status";
}

const char *pba_last_error(const pba_ctx *ctx) { return ctx ? ctx->c.err.c_str() : g_create_err.c_str(); }

pba_status pba_config_default(pba_config *cfg) {
    if (!cfg) return fail(nullptr, PBA_E_INVALID, "cfg is NULL");
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->mode = PBA_IC_PROXY;
    cfg->precision = PBA_FP32;
    cfg->n_levels = 1;
    cfg->pattern_n = 8;
    const int pat[16] = {0, 0, 0, -2, -1, -1, 1, -1, -2, 0, 2, 0, -1, 1, 1, 1};
    std::memcpy(cfg->pattern_uv, pat, sizeof(pat));
    cfg->huber_k = 9.0 / 255.0;
    cfg->damping_rel = 1e-6;
    cfg->pinned_frame = 0;
    cfg->solver = PBA_SOLVER_CHOL;
    cfg->n_windows = 1;
    cfg->flags = 0;
    cfg->stream = nullptr;
    return PBA_OK;
}

pba_status pba_create(const pba_config *cfg, pba_ctx **out) {
    if (!out) return fail(nullptr, PBA_E_INVALID, "out is NULL");
    *out = nullptr;
    const std::string v = validate_config(cfg);
    if (!v.empty()) return fail(nullptr, PBA_E_INVALID, v);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(nullptr, PBA_E_DEVICE, "no HIP device");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(nullptr, PBA_E_DEVICE, "hipGetDevice failed");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return fail(nullptr, PBA_E_DEVICE, "hipGetDeviceProperties failed");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, PBA_E_DEVICE, std::string("device is ") + prop.gcnArchName + ", libpba needs gfx950");
    pba_ctx *ctx = new pba_ctx();
    Ctx &c = ctx->c;
    c.cfg = *cfg;
    if (cfg->flags & PBA_FLAG_LANE_PER_PIXEL) c.tune_res.lanes = 8;
    c.device = dev;
    c.P = cfg->pattern_n;
    c.real_size = cfg->precision == PBA_FP64 ? sizeof(double) : sizeof(float);
    {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
            c.n_cu = ncu;
    }
    if (cfg->n_windows > 1) ctx->stage.resize(cfg->n_windows);
    if (cfg->stream) {
        c.stream = (hipStream_t)cfg->stream;
        c.own_stream = false;
    } else {
        if (hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking) != hipSuccess) {
            delete ctx;
            return fail(nullptr, PBA_E_DEVICE, "hipStreamCreate failed");
        }
        c.own_stream = true;
    }
    *out = ctx;
    return PBA_OK;
}

void pba_destroy(pba_ctx *ctx) {
    if (!ctx) return;
    Ctx &c = ctx->c;
    if (c.stream) (void)hipStreamSynchronize(c.stream);
    release_frames(c);
    dfree(c.d_eval);
    release_pc(c);
    aff_release(ctx->aff);
    for (hipEvent_t e : c.ev_pool) (void)hipEventDestroy(e);
    if (c.own_stream && c.stream) (void)hipStreamDestroy(c.stream);
    delete ctx;
}

pba_status pba_set_frames(pba_ctx *ctx, int32_t window, int32_t n_frames, int32_t width, int32_t height,
                          const float *images, const double *intrinsics, const double *poses, int32_t mem) {
    if (!ctx) return fail(nullptr, PBA_E_INVALID, "ctx is NULL");
    Ctx &c = ctx->c;
    if (window < 0 || window >= c.cfg.n_windows)
        return fail(&c, PBA_E_INVALID, "window must be in 0..n_windows-1");
    if (mem != PBA_HOST && mem != PBA_DEVICE) return fail(&c, PBA_E_INVALID, "mem must be PBA_HOST or PBA_DEVICE");
    if (n_frames < 1) return fail(&c, PBA_E_INVALID, "n_frames must be >= 1");
    const int minsz = 8 << (c.cfg.n_levels - 1);
    if (width < minsz || height < minsz)
        return fail(&c, PBA_E_INVALID, "width and height must be >= " + std::to_string(minsz));
    if ((long long)n_frames * width * height > (1LL << 34)) return fail(&c, PBA_E_INVALID, "images too large");
    if (!images || !intrinsics || !poses) return fail(&c, PBA_E_INVALID, "NULL input array");
    if (c.cfg.pinned_frame >= n_frames) return fail(&c, PBA_E_INVALID, "pinned_frame >= n_frames");
    if (c.cfg.n_windows > 1) {
        if (6 * n_frames > LDS_CHOL_MAX_N)
            return fail(&c, PBA_E_INVALID, "a window of a batched context holds at most " +
                                               std::to_string(LDS_CHOL_MAX_N / 6) + " frames");
        for (int w = 0; w < c.cfg.n_windows; ++w)
            if (w != window && ctx->stage[w].have_frames && (width != ctx->stage_W || height != ctx->stage_H))
                return fail(&c, PBA_E_INVALID, "every window of a batched context must have the same image size");
    }
    std::vector<double> K, Pz;
    HIPCHK(fetch(K, intrinsics, (size_t)n_frames * 4, mem));
    HIPCHK(fetch(Pz, poses, (size_t)n_frames * 12, mem));
    if (!finite_all(K.data(), K.size())) return fail(&c, PBA_E_INVALID, "intrinsics not finite");
    for (int f = 0; f < n_frames; ++f)
        if (!(K[4 * f] > 0.0) || !(K[4 * f + 1] > 0.0)) return fail(&c, PBA_E_INVALID, "focal lengths must be > 0");
    if (!finite_all(Pz.data(), Pz.size())) return fail(&c, PBA_E_INVALID, "poses not finite");
    for (int f = 0; f < n_frames; ++f) {
        const double *R = Pz.data() + 12 * f;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double s = 0.0;
                for (int k = 0; k < 3; ++k) s += R[3 * i + k] * R[3 * j + k];
                if (std::fabs(s - (i == j ? 1.0 : 0.0)) > 1e-6)
                    return fail(&c, PBA_E_INVALID, "pose " + std::to_string(f) + " rotation is not orthonormal");
            }
    }
    const size_t npx = (size_t)n_frames * width * height;
    if (mem == PBA_HOST) {
        for (size_t i = 0; i < npx; ++i)
            if (!std::isfinite(images[i])) return fail(&c, PBA_E_INVALID, "images contain non-finite values");
    }
    if (c.cfg.n_windows > 1) {
        WinStage &st = ctx->stage[window];
        HIPCHK(fetch(st.img, images, npx, mem));
        st.F = n_frames;
        st.K = K;
        st.P = Pz;
        st.have_frames = true;
        st.have_points = false;  // as for one window: the points follow the frames
        ctx->stage_W = width;
        ctx->stage_H = height;
        ctx->dirty = true;
        return PBA_OK;
    }
    return load_frames(c, n_frames, width, height, images, mem, K, Pz, {0, n_frames});
}

pba_status pba_set_points(pba_ctx *ctx, int32_t window, int32_t n_points, const int32_t *host_frame,
                          const float *host_uv, const double *inv_depth, const int32_t *obs_ptr,
                          const int32_t *obs_frame, int32_t mem) {
    if (!ctx) return fail(nullptr, PBA_E_INVALID, "ctx is NULL");
    Ctx &c = ctx->c;
    if (window < 0 || window >= c.cfg.n_windows)
        return fail(&c, PBA_E_INVALID, "window must be in 0..n_windows-1");
    const bool batched = c.cfg.n_windows > 1;
    if (batched ? !ctx->stage[window].have_frames : !c.have_frames)
        return fail(&c, PBA_E_STATE, "pba_set_frames must be called first");
    if (mem != PBA_HOST && mem != PBA_DEVICE) return fail(&c, PBA_E_INVALID, "mem must be PBA_HOST or PBA_DEVICE");
    if (n_points < 0) return fail(&c, PBA_E_INVALID, "n_points must be >= 0");
    if (n_points > 0 && (!host_frame || !host_uv || !inv_depth || !obs_ptr))
        return fail(&c, PBA_E_INVALID, "NULL input array");
    if (!obs_ptr) return fail(&c, PBA_E_INVALID, "obs_ptr is NULL");
    const int F = batched ? ctx->stage[window].F : c.F;
    const int W = batched ? ctx->stage_W : c.W, H = batched ? ctx->stage_H : c.H;
    std::vector<int> hf, optr, ofr;
    std::vector<float> uv;
    std::vector<double> d;
    HIPCHK(fetch(optr, obs_ptr, (size_t)n_points + 1, mem));
    if (optr[0] != 0) return fail(&c, PBA_E_INVALID, "obs_ptr[0] must be 0");
    for (int n = 0; n < n_points; ++n)
        if (optr[n + 1] < optr[n]) return fail(&c, PBA_E_INVALID, "obs_ptr must be non-decreasing");
    const long long O = optr[n_points];
    if (O > (1LL << 28)) return fail(&c, PBA_E_INVALID, "too many observations");
    if (O > 0 && !obs_frame) return fail(&c, PBA_E_INVALID, "obs_frame is NULL");
    HIPCHK(fetch(hf, host_frame, (size_t)n_points, mem));
    HIPCHK(fetch(uv, host_uv, 2 * (size_t)n_points, mem));
    HIPCHK(fetch(d, inv_depth, (size_t)n_points, mem));
    HIPCHK(fetch(ofr, obs_frame, (size_t)O, mem));
    for (int n = 0; n < n_points; ++n) {
        if (hf[n] < 0 || hf[n] >= F) return fail(&c, PBA_E_INVALID, "host_frame out of range at point " + std::to_string(n));
        if (!std::isfinite(d[n]) || !(d[n] > 0.0))
            return fail(&c, PBA_E_INVALID, "inv_depth must be finite and > 0 at point " + std::to_string(n));
        if (!std::isfinite(uv[2 * n]) || !std::isfinite(uv[2 * n + 1]) || uv[2 * n] < 0 || uv[2 * n] > W - 1 ||
            uv[2 * n + 1] < 0 || uv[2 * n + 1] > H - 1)
            return fail(&c, PBA_E_INVALID, "host_uv outside the image at point " + std::to_string(n));
        for (int o = optr[n]; o < optr[n + 1]; ++o) {
            if (ofr[o] < 0 || ofr[o] >= F) return fail(&c, PBA_E_INVALID, "obs_frame out of range");
            if (ofr[o] == hf[n]) return fail(&c, PBA_E_INVALID, "a point cannot observe its own host frame");
            if (o > optr[n] && ofr[o] <= ofr[o - 1])
                return fail(&c, PBA_E_INVALID, "obs_frame must be strictly increasing within a point");
        }
    }
    if (batched) {
        WinStage &st = ctx->stage[window];
        st.N = n_points;
        st.hf = std::move(hf);
        st.optr = std::move(optr);
        st.ofr = std::move(ofr);
        st.uv = std::move(uv);
        st.d = std::move(d);
        st.have_points = true;
        ctx->dirty = true;
        return PBA_OK;
    }
    return load_points(c, n_points, hf, uv, d, optr, ofr, {0, n_points});
}

pba_status pba_iterate(pba_ctx *ctx, int32_t level, int32_t n_iters, pba_iter_stats *stats) {
    if (!ctx) return fail(nullptr, PBA_E_INVALID, "ctx is NULL");
    Ctx &c = ctx->c;
    if (level < 0 || level >= c.cfg.n_levels) return fail(&c, PBA_E_INVALID, "level out of range");
    if (n_iters < 0) return fail(&c, PBA_E_INVALID, "n_iters must be >= 0");
    pba_status st;
    if ((st = ready(ctx)) != PBA_OK) return st;
    if (c.cur_level != level && (st = do_start_level(c, level)) != PBA_OK) return st;
    if (ctx->aff.on) return aff_run(c, ctx->aff, level, n_iters, -1.0, stats, nullptr);
    return run_iterations(c, level, n_iters, stats);
}

pba_status pba_evaluate(pba_ctx *ctx, int32_t level, pba_iter_stats *out) {
    if (!ctx) return fail(nullptr, PBA_E_INVALID, "ctx is NULL");
    Ctx &c = ctx->c;
    if (level < 0 || level >= c.cfg.n_levels) return fail(&c, PBA_E_INVALID, "level out of range");
    if (!out) return fail(&c, PBA_E_INVALID, "out is NULL");
    pba_status st;
    if ((st = ready(ctx)) != PBA_OK) return st;
    hipStream_t s = c.stream;
    if (ctx->aff.on) {
        double h[3];
        if ((st = aff_ensure(c, ctx->aff)) != PBA_OK) return st;
        st = is_fp64(c) ? aff_evaluate<double>(c, ctx->aff, level, h) : aff_evaluate<float>(c, ctx->aff, level, h);
        if (st != PBA_OK) return st;
        std::memset(out, 0, sizeof(*out));
        out->level = level;
        out->n_active = (int64_t)std::llround(h[2]);
        out->energy = h[0];
        out->sq = h[1];
        out->rmse = out->n_active > 0 ? std::sqrt(h[1] / (double)out->n_active) : 0.0;
        return PBA_OK;
    }
    // relative poses at the current parameters go to the buffer the next iteration reads
    double *geo = c.flip ? c.d_geo_b : c.d_geo_a;
    if (c.eval_cap < sum_stats_doubles(c)) {
        HIPCHK(dalloc(c.d_eval, sum_stats_doubles(c) * sizeof(double)));
        c.eval_cap = sum_stats_doubles(c);
    }
    if (is_fp64(c)) {
        if (!c.lv[level].tmpl_valid) Launch<double>::make_template(s, c, level);
        Launch<double>::relpose(s, c, c.d_poses, geo, (double *)(c.flip ? c.d_rel_b : c.d_rel_a));
        Launch<double>::evaluate(s, c, level);
    } else {
        if (!c.lv[level].tmpl_valid) Launch<float>::make_template(s, c, level);
        Launch<float>::relpose(s, c, c.d_poses, geo, (float *)(c.flip ? c.d_rel_b : c.d_rel_a));
        Launch<float>::evaluate(s, c, level);
    }
    c.lv[level].tmpl_valid = true;
    if (c.O > 0)
        launch_sum_stats(s, c, c.d_rec, true, c.d_eval);
    else
        launch_fill(s, c.d_eval, 3, 0.0, nullptr);
    double h[3];
    HIPCHK(hipMemcpyAsync(h, c.d_eval, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::memset(out, 0, sizeof(*out));
    out->level = level;
    out->n_active = (int64_t)std::llround(h[2]);
    out->energy = h[0];
    out->sq = h[1];
    out->rmse = out->n_active > 0 ? std::sqrt(h[1] / (double)out->n_active) : 0.0;
    return PBA_OK;
}

pba_status pba_solve(pba_ctx *ctx, int32_t max_iters_per_level, double conv_px, pba_result *out) {
    if (!ctx) return fail(nullptr, PBA_E_INVALID, "ctx is NULL");
    Ctx &c = ctx->c;
    if (max_iters_per_level < 1) return fail(&c, PBA_E_INVALID, "max_iters_per_level must be >= 1");
    if (!(conv_px >= 0.0)) return fail(&c, PBA_E_INVALID, "conv_px must be >= 0");
    pba_status st;
    if ((st = ready(ctx)) != PBA_OK) return st;
    pba_result res;
    std::memset(&res, 0, sizeof(res));
    if (ctx->aff.on && (st = aff_ensure(c, ctx->aff)) != PBA_OK) return st;
    if ((st = solve_batch(c, max_iters_per_level, conv_px, res, ctx->aff.on ? &ctx->aff : nullptr)) != PBA_OK)
        return st;
    pba_iter_stats ev;
    if ((st = pba_evaluate(ctx, 0, &ev)) != PBA_OK) return st;
    res.final_energy = ev.energy;
    res.final_rmse = ev.rmse;
    res.final_active = ev.n_active;
    if (out) *out = res;
    if (!res.converged) return fail(&c, PBA_E_NOT_CONVERGED, "level 0 did not reach conv_px");
    return PBA_OK;
}

pba_status pba_get_params(pba_ctx *ctx, int32_t window, double *poses, double *inv_depth) {
    if (!ctx) return fail(nullptr, PBA_E_INVALID, "ctx is NULL");
    Ctx &c = ctx->c;
    if (window < 0 || window >= c.cfg.n_windows) return fail(&c, PBA_E_INVALID, "window must be in 0..n_windows-1");
    if (c.cfg.n_windows > 1) {
        pba_status st;
        if ((st = ready(ctx)) != PBA_OK) return st;
    }
    if (!c.have_frames) return fail(&c, PBA_E_STATE, "no frames set");
    const int f0 = c.win_frame_off[window], f1 = c.win_frame_off[window + 1];
    if (poses)
        HIPCHK(hipMemcpyAsync(poses, c.d_poses + 12 * (size_t)f0, (size_t)(f1 - f0) * 12 * sizeof(double),
                              hipMemcpyDeviceToHost, c.stream));
    std::vector<double> dn;
    const int n0 = c.have_points ? c.win_point_off[window] : 0, n1 = c.have_points ? c.win_point_off[window + 1] : 0;
    if (inv_depth && n1 > n0) {
        dn.resize((size_t)(n1 - n0));
        HIPCHK(hipMemcpyAsync(dn.data(), c.d_depth + n0, dn.size() * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    }
    HIPCHK(hipStreamSynchronize(c.stream));
    for (int i = n0; i < n1 && inv_depth; ++i) inv_depth[c.pt_caller[i] - n0] = dn[(size_t)(i - n0)];
    return PBA_OK;
}

pba_status pba_set_params(pba_ctx *ctx, int32_t window, const double *poses, const double *inv_depth) {
    if (!ctx) return fail(nullptr, PBA_E_INVALID, "ctx is NULL");
    Ctx &c = ctx->c;
    if (window < 0 || window >= c.cfg.n_windows) return fail(&c, PBA_E_INVALID, "window must be in 0..n_windows-1");
    pba_status st;
    if ((st = ready(ctx)) != PBA_OK) return st;
    const int f0 = c.win_frame_off[window], f1 = c.win_frame_off[window + 1];
    const int n0 = c.win_point_off[window], n1 = c.win_point_off[window + 1];
    if (poses && !finite_all(poses, (size_t)(f1 - f0) * 12)) return fail(&c, PBA_E_INVALID, "poses not finite");
    if (inv_depth) {
        for (int n = 0; n < n1 - n0; ++n)
            if (!std::isfinite(inv_depth[n]) || !(inv_depth[n] > 0.0))
                return fail(&c, PBA_E_INVALID, "inv_depth must be finite and > 0");
    }
    if (poses)
        HIPCHK(hipMemcpyAsync(c.d_poses + 12 * (size_t)f0, poses, (size_t)(f1 - f0) * 12 * sizeof(double),
                              hipMemcpyHostToDevice, c.stream));
    std::vector<double> dn;
    if (inv_depth && n1 > n0) {
        dn.resize((size_t)(n1 - n0));
        for (int i = n0; i < n1; ++i) dn[(size_t)(i - n0)] = inv_depth[c.pt_caller[i] - n0];
        HIPCHK(hipMemcpyAsync(c.d_depth + n0, dn.data(), dn.size() * sizeof(double), hipMemcpyHostToDevice, c.stream));
    }
    HIPCHK(hipStreamSynchronize(c.stream));
    c.cur_level = -1;
    return PBA_OK;
}

pba_status pba_drop_frame(pba_ctx *ctx, int32_t window, int32_t frame) {
    if (!ctx) return fail(nullptr, PBA_E_INVALID, "ctx is NULL");
    Ctx &c = ctx->c;
    if (window < 0 || window >= c.cfg.n_windows) return fail(&c, PBA_E_INVALID, "window must be in 0..n_windows-1");
    pba_status st;
    if ((st = ready(ctx)) != PBA_OK) return st;
    const int f0 = c.win_frame_off[window], nf = c.win_frame_off[window + 1] - f0;
    if (frame < 0 || frame >= nf) return fail(&c, PBA_E_INVALID, "frame out of range for the window");
    if (frame == c.cfg.pinned_frame) return fail(&c, PBA_E_INVALID, "the gauge (pinned) frame cannot be dropped");
    launch_drop_frame(c.stream, c, f0 + frame);
    if (c.cfg.mode == PBA_IC_PROXY && c.cur_level >= 0 && c.s_valid) {
        // mid-level: the system again from the records kept at p(0)
        launch_open(c.stream, c, c.cur_level, true);
        if (is_fp64(c))
            ic_system<double>(c, c.cur_level, false);
        else
            ic_system<float>(c, c.cur_level, false);
    }
    HIPCHK(hipStreamSynchronize(c.stream));
    HIPCHK(hipGetLastError());
    int flag = 0;
    HIPCHK(hipMemcpy(&flag, c.d_flag, sizeof(int), hipMemcpyDeviceToHost));
    if (flag) {
        c.cur_level = -1;
        return fail(&c, PBA_E_NUMERIC, "reduced pose system is not positive definite");
    }
    return PBA_OK;
}

pba_status pba_set_affine(pba_ctx *ctx, const double *ab) {
    if (!ctx) return fail(nullptr, PBA_E_INVALID, "ctx is NULL");
    Ctx &c = ctx->c;
    if (!ab) {
        if (ctx->aff.on) drop_graph(c);
        ctx->aff.on = false;
        return PBA_OK;
    }
    pba_status st;
    if ((st = ready(ctx)) != PBA_OK) return st;
    const std::string why = aff_check(c);
    if (!why.empty()) return fail(&c, PBA_E_INVALID, why);
    if (!finite_all(ab, 2 * (size_t)c.F)) return fail(&c, PBA_E_INVALID, "brightness parameters not finite");
    if ((st = aff_ensure(c, ctx->aff)) != PBA_OK) return st;
    HIPCHK(hipMemcpyAsync(ctx->aff.ab, ab, 2 * (size_t)c.F * sizeof(double), hipMemcpyHostToDevice, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    if (!ctx->aff.on) drop_graph(c);
    ctx->aff.on = true;
    return PBA_OK;
}

pba_status pba_get_affine(pba_ctx *ctx, double *ab) {
    if (!ctx) return fail(nullptr, PBA_E_INVALID, "ctx is NULL");
    Ctx &c = ctx->c;
    if (!ab) return fail(&c, PBA_E_INVALID, "ab is NULL");
    if (!c.have_frames) return fail(&c, PBA_E_STATE, "pba_set_frames must be called first");
    const size_t n = 2 * (size_t)c.F;
    if (!ctx->aff.ab || ctx->aff.F != c.F) {
        std::fill(ab, ab + n, 0.0);
        return PBA_OK;
    }
    HIPCHK(hipMemcpyAsync(ab, ctx->aff.ab, n * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    return PBA_OK;
}

// ---- front end (Sec. 4.1 base solution: corners, tracks, geometric BA)

pba_status pba_fe_corners(pba_ctx *ctx, int32_t window, int32_t frame, int32_t cell, int32_t margin,
                          int64_t min_response, int32_t max_corners, int32_t *uv, int64_t *response,
                          int32_t *n_out) {
    if (!ctx) return fail(nullptr, PBA_E_INVALID, "ctx is NULL");
    Ctx &c = ctx->c;
    if (!uv || !n_out) return fail(&c, PBA_E_INVALID, "uv and n_out must not be NULL");
    if (!c.have_frames) return fail(&c, PBA_E_STATE, "pba_set_frames must be called first");
    if (window < 0 || window >= c.nwin) return fail(&c, PBA_E_INVALID, "window must be in 0..n_windows-1");
    const int f0 = c.win_frame_off[window], nf = c.win_frame_off[window + 1] - f0;
    if (frame < 0 || frame >= nf) return fail(&c, PBA_E_INVALID, "frame out of range for the window");
    if (cell < 2 || cell > 16) return fail(&c, PBA_E_INVALID, "cell must be in 2..16");
    if (margin < 0) return fail(&c, PBA_E_INVALID, "margin must be >= 0");
    if (max_corners < 0) return fail(&c, PBA_E_INVALID, "max_corners must be >= 0");
    const int W = c.lv[0].W, H = c.lv[0].H;
    const long long ncells = (long long)((W + cell - 1) / cell) * ((H + cell - 1) / cell);
    if (ncells > PBA_FE_MAX_CELLS) return fail(&c, PBA_E_INVALID, "more than PBA_FE_MAX_CELLS cells: use larger cells");
    *n_out = 0;
    if (max_corners == 0) return PBA_OK;
    long long *R = nullptr, *cell_R = nullptr, *resp = nullptr;
    int *cell_idx = nullptr, *rank = nullptr, *duv = nullptr, *count = nullptr;
    hipError_t e = hipSuccess;
    if ((e = dalloc(R, (size_t)W * H * sizeof(long long))) == hipSuccess &&
        (e = dalloc(cell_R, (size_t)ncells * sizeof(long long))) == hipSuccess &&
        (e = dalloc(cell_idx, (size_t)ncells * sizeof(int))) == hipSuccess &&
        (e = dalloc(rank, (size_t)ncells * sizeof(int))) == hipSuccess &&
        (e = dalloc(duv, (size_t)max_corners * 2 * sizeof(int))) == hipSuccess &&
        (e = dalloc(resp, (size_t)max_corners * sizeof(long long))) == hipSuccess &&
        (e = dalloc(count, sizeof(int))) == hipSuccess) {
        launch_fe_corners(c.stream, c, f0 + frame, cell, margin, min_response, max_corners, R, cell_R, cell_idx,
                          rank, duv, resp, count);
        int n = 0;
        if ((e = hipMemcpyAsync(&n, count, sizeof(int), hipMemcpyDeviceToHost, c.stream)) == hipSuccess &&
            (e = hipStreamSynchronize(c.stream)) == hipSuccess && n > 0) {
            if ((e = hipMemcpyAsync(uv, duv, (size_t)n * 2 * sizeof(int), hipMemcpyDeviceToHost, c.stream)) ==
                    hipSuccess &&
                response)
                e = hipMemcpyAsync(response, resp, (size_t)n * sizeof(long long), hipMemcpyDeviceToHost, c.stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
        }
        if (e == hipSuccess) e = hipGetLastError();
        if (e == hipSuccess) *n_out = n;
    }
    for (long long **p : {&R, &cell_R, &resp}) dfree(*p);
    for (int **p : {&cell_idx, &rank, &duv, &count}) dfree(*p);
    if (e != hipSuccess) return fail(&c, PBA_E_DEVICE, std::string("HIP error: ") + hipGetErrorString(e));
    return PBA_OK;
}

pba_status pba_fe_track(pba_ctx *ctx, int32_t window, int32_t n, const int32_t *host_frame, const double *host_uv,
                        const int32_t *target_frame, const double *guess_uv, int32_t radius, int32_t n_iters,
                        double min_eig, double fb_px, double *uv_out, int32_t *status_out, double *fb_out) {
    if (!ctx) return fail(nullptr, PBA_E_INVALID, "ctx is NULL");
    Ctx &c = ctx->c;
    if (!c.have_frames) return fail(&c, PBA_E_STATE, "pba_set_frames must be called first");
    if (window < 0 || window >= c.nwin) return fail(&c, PBA_E_INVALID, "window must be in 0..n_windows-1");
    if (n < 0) return fail(&c, PBA_E_INVALID, "n must be >= 0");
    if (n == 0) return PBA_OK;
    if (!host_frame || !host_uv || !target_frame || !guess_uv || !uv_out || !status_out)
        return fail(&c, PBA_E_INVALID, "input and output arrays must not be NULL");
    if (radius < 1 || radius > PBA_FE_MAX_RADIUS) return fail(&c, PBA_E_INVALID, "radius must be in 1..PBA_FE_MAX_RADIUS");
    if (n_iters < 1 || n_iters > 100) return fail(&c, PBA_E_INVALID, "n_iters must be in 1..100");
    if (!(min_eig >= 0.0) || !(fb_px >= 0.0)) return fail(&c, PBA_E_INVALID, "min_eig and fb_px must be >= 0");
    const int f0 = c.win_frame_off[window], nf = c.win_frame_off[window + 1] - f0;
    std::vector<int> hf(n), tf(n);
    for (int i = 0; i < n; ++i) {
        if (host_frame[i] < 0 || host_frame[i] >= nf || target_frame[i] < 0 || target_frame[i] >= nf)
            return fail(&c, PBA_E_INVALID, "frame index out of range for the window");
        hf[i] = f0 + host_frame[i];
        tf[i] = f0 + target_frame[i];
    }
    if (!finite_all(host_uv, 2 * (size_t)n) || !finite_all(guess_uv, 2 * (size_t)n))
        return fail(&c, PBA_E_INVALID, "positions must be finite");
    int *dh = nullptr, *dt = nullptr, *dst = nullptr;
    double *dxu = nullptr, *dg = nullptr, *dout = nullptr, *dfb = nullptr;
    hipError_t e = hipSuccess;
    std::vector<double> fb(n);
    if ((e = dalloc(dh, (size_t)n * sizeof(int))) == hipSuccess && (e = dalloc(dt, (size_t)n * sizeof(int))) == hipSuccess &&
        (e = dalloc(dst, (size_t)n * sizeof(int))) == hipSuccess &&
        (e = dalloc(dxu, (size_t)n * 2 * sizeof(double))) == hipSuccess &&
        (e = dalloc(dg, (size_t)n * 2 * sizeof(double))) == hipSuccess &&
        (e = dalloc(dout, (size_t)n * 2 * sizeof(double))) == hipSuccess &&
        (e = dalloc(dfb, (size_t)n * sizeof(double))) == hipSuccess &&
        (e = hipMemcpyAsync(dh, hf.data(), (size_t)n * sizeof(int), hipMemcpyHostToDevice, c.stream)) == hipSuccess &&
        (e = hipMemcpyAsync(dt, tf.data(), (size_t)n * sizeof(int), hipMemcpyHostToDevice, c.stream)) == hipSuccess &&
        (e = hipMemcpyAsync(dxu, host_uv, (size_t)n * 2 * sizeof(double), hipMemcpyHostToDevice, c.stream)) ==
            hipSuccess &&
        (e = hipMemcpyAsync(dg, guess_uv, (size_t)n * 2 * sizeof(double), hipMemcpyHostToDevice, c.stream)) ==
            hipSuccess) {
        launch_fe_track(c.stream, c, n, dh, dxu, dt, dg, radius, n_iters, min_eig, fb_px, c.cfg.n_levels, dout, dst,
                        dfb);
        if ((e = hipGetLastError()) == hipSuccess &&
            (e = hipMemcpyAsync(uv_out, dout, (size_t)n * 2 * sizeof(double), hipMemcpyDeviceToHost, c.stream)) ==
                hipSuccess &&
            (e = hipMemcpyAsync(status_out, dst, (size_t)n * sizeof(int), hipMemcpyDeviceToHost, c.stream)) ==
                hipSuccess &&
            (e = hipMemcpyAsync(fb.data(), dfb, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, c.stream)) ==
                hipSuccess)
            e = hipStreamSynchronize(c.stream);
    }
    for (int **p : {&dh, &dt, &dst}) dfree(*p);
    for (double **p : {&dxu, &dg, &dout, &dfb}) dfree(*p);
    if (e != hipSuccess) return fail(&c, PBA_E_DEVICE, std::string("HIP error: ") + hipGetErrorString(e));
    if (fb_out) std::memcpy(fb_out, fb.data(), (size_t)n * sizeof(double));
    return PBA_OK;
}

pba_status pba_set_tracks(pba_ctx *ctx, int32_t window, int32_t n_obs, const double *obs_uv) {
    if (!ctx) return fail(nullptr, PBA_E_INVALID, "ctx is NULL");
    Ctx &c = ctx->c;
    pba_status st;
    if ((st = ready(ctx)) != PBA_OK) return st;
    if (c.nwin != 1 || window != 0) return fail(&c, PBA_E_INVALID, "tracks are taken by one-window contexts (window 0)");
    if (n_obs != c.O) return fail(&c, PBA_E_INVALID, "n_obs must equal the observations of pba_set_points");
    if (n_obs > 0 && !obs_uv) return fail(&c, PBA_E_INVALID, "obs_uv is NULL");
    if (!finite_all(obs_uv, 2 * (size_t)n_obs)) return fail(&c, PBA_E_INVALID, "obs_uv must be finite");
    std::vector<double> z(2 * (size_t)c.O);
    for (int o = 0; o < c.O; ++o) {
        const int oc = c.obs_caller[o];
        z[2 * (size_t)o] = obs_uv[2 * (size_t)oc];
        z[2 * (size_t)o + 1] = obs_uv[2 * (size_t)oc + 1];
    }
    HIPCHK(upload(c, c.d_obs_z, z));
    dfree(c.d_geo_in);
    HIPCHK(dalloc(c.d_geo_in, std::max<size_t>(1, c.O)));
    HIPCHK(hipStreamSynchronize(c.stream));
    return PBA_OK;
}

pba_status pba_geo_solve(pba_ctx *ctx, int32_t max_iters, double conv_px, double huber_px, double outlier_px,
                         uint8_t *inliers, pba_result *out) {
    if (!ctx) return fail(nullptr, PBA_E_INVALID, "ctx is NULL");
    Ctx &c = ctx->c;
    pba_status st;
    if ((st = ready(ctx)) != PBA_OK) return st;
    if (!c.d_obs_z && c.O > 0) return fail(&c, PBA_E_STATE, "pba_set_tracks must be called first");
    if (max_iters < 1) return fail(&c, PBA_E_INVALID, "max_iters must be >= 1");
    if (!(conv_px >= 0.0) || !(huber_px > 0.0)) return fail(&c, PBA_E_INVALID, "conv_px >= 0 and huber_px > 0 required");
    if (!(outlier_px > 0.0) && outlier_px != 0.0) return fail(&c, PBA_E_INVALID, "outlier_px must be >= 0");
    pba_result res;
    std::memset(&res, 0, sizeof(res));
    std::vector<pba_iter_stats> stats((size_t)max_iters);
    // the FC iteration on the reprojection error at level 0; the context's own
    // mode comes back on every return, and its next photometric call starts a
    // level afresh
    struct ModeGuard {
        Ctx &c;
        int mode;
        ~ModeGuard() {
            c.cfg.mode = mode;
            c.geo_mode = false;
            c.cur_level = -1;
            c.s_valid = false;
        }
    } guard{c, c.cfg.mode};
    c.cfg.mode = PBA_FC;
    c.geo_mode = true;
    c.geo_huber = huber_px;
    c.cur_level = -1;
    if (c.O > 0) HIPCHK(hipMemsetAsync(c.d_geo_in, 1, (size_t)c.O, c.stream));
    // relative geometry of every pair at the current poses, into the buffer the
    // next iteration reads
    auto current_geo = [&c]() {
        double *geo = c.flip ? c.d_geo_b : c.d_geo_a;
        if (is_fp64(c))
            Launch<double>::relpose(c.stream, c, c.d_poses, geo, (double *)(c.flip ? c.d_rel_b : c.d_rel_a));
        else
            Launch<float>::relpose(c.stream, c, c.d_poses, geo, (float *)(c.flip ? c.d_rel_b : c.d_rel_a));
        return geo;
    };
    const int passes = outlier_px > 0.0 ? 2 : 1;
    for (int pass = 0; pass < passes && st == PBA_OK; ++pass) {
        if (pass == 1) launch_geo_outliers(c.stream, c, current_geo(), outlier_px);
        st = do_start_level(c, 0);
        int ran = 0;
        if (st == PBA_OK) st = run_iterations(c, 0, max_iters, stats.data(), conv_px, &ran);
        if (st == PBA_OK) {
            res.iters[pass] = ran;
            res.total_iters += ran;
            res.converged = ran > 0 && stats[(size_t)ran - 1].max_disp_px < conv_px;
        }
    }
    if (st == PBA_OK) {
        // energy and RMS reprojection error over the inliers at the final parameters
        launch_open(c.stream, c, 0, true);
        launch_geo_linearize(c.stream, c, current_geo());
        if (c.eval_cap < sum_stats_doubles(c)) {
            dfree(c.d_eval);
            HIPCHK(dalloc(c.d_eval, sum_stats_doubles(c) * sizeof(double)));
            c.eval_cap = sum_stats_doubles(c);
        }
        double h[3] = {0.0, 0.0, 0.0};
        if (c.O > 0) {
            launch_sum_stats(c.stream, c, c.d_rec, true, c.d_eval);
            HIPCHK(hipMemcpyAsync(h, c.d_eval, sizeof(h), hipMemcpyDeviceToHost, c.stream));
        }
        std::vector<uint8_t> in((size_t)c.O);
        if (inliers && c.O > 0)
            HIPCHK(hipMemcpyAsync(in.data(), c.d_geo_in, (size_t)c.O, hipMemcpyDeviceToHost, c.stream));
        HIPCHK(hipStreamSynchronize(c.stream));
        HIPCHK(hipGetLastError());
        res.final_energy = h[0];
        res.final_active = (int64_t)std::llround(h[2]);
        res.final_rmse = res.final_active > 0 ? std::sqrt(h[1] / (double)res.final_active) : 0.0;
        if (inliers)
            for (int o = 0; o < c.O; ++o) inliers[c.obs_caller[o]] = in[(size_t)o];
    }
    if (st != PBA_OK) return st;
    if (out) *out = res;
    if (!res.converged) return fail(&c, PBA_E_NOT_CONVERGED, "the geometric solve did not reach conv_px");
    return PBA_OK;
}

pba_status pba_debug_fetch(pba_ctx *ctx, int32_t what, void *out, size_t bytes) {
    if (!ctx) return fail(nullptr, PBA_E_INVALID, "ctx is NULL");
    Ctx &c = ctx->c;
    if (!out) return fail(&c, PBA_E_INVALID, "out is NULL");
    pba_status st0;
    if ((st0 = ready(ctx)) != PBA_OK) return st0;
    const size_t n6 = 6 * (size_t)c.F;
    const void *src = nullptr;
    size_t need = 0;
    switch (what) {
        case PBA_DBG_S: src = c.d_S; need = (size_t)c.win_S_off[c.nwin] * sizeof(double); break;
        case PBA_DBG_B: src = c.d_b; need = n6 * sizeof(double); break;
        case PBA_DBG_OBS_REC: src = c.d_rec; need = (size_t)c.O * REC_STRIDE * sizeof(double); break;
        case PBA_DBG_TEMPLATE: {
            const int l = c.cur_level < 0 ? 0 : c.cur_level;
            src = c.lv[l].tmpl;
            need = (size_t)c.N * c.P * 4 * c.real_size;
            break;
        }
        case PBA_DBG_HDD: src = c.d_Hdd; need = (size_t)c.N * sizeof(double); break;
        case PBA_DBG_MASK: src = c.d_mask; need = (size_t)c.O; break;
        case PBA_DBG_DTHETA: src = c.d_dtheta; need = n6 * sizeof(double); break;
        case PBA_DBG_PAIR_H: src = c.d_pairH; need = (size_t)c.st.n_pairs * 21 * sizeof(double); break;
        case PBA_DBG_PAIRS: {
            need = (size_t)c.st.n_pairs * 2 * sizeof(int32_t);
            if (bytes != need) return fail(&c, PBA_E_INVALID, "bytes must be " + std::to_string(need));
            int32_t *o = static_cast<int32_t *>(out);
            for (int p = 0; p < c.st.n_pairs; ++p) {
                o[2 * p] = c.st.pair_host[p];
                o[2 * p + 1] = c.st.pair_target[p];
            }
            return PBA_OK;
        }
        default: return fail(&c, PBA_E_INVALID, "unknown debug buffer");
    }
    if (bytes != need) return fail(&c, PBA_E_INVALID, "bytes must be " + std::to_string(need));
    // per-point and per-observation buffers go back to the caller's order
    const std::vector<int> *rows = nullptr;
    if (what == PBA_DBG_OBS_REC || what == PBA_DBG_MASK) rows = &c.obs_caller;
    if (what == PBA_DBG_TEMPLATE || what == PBA_DBG_HDD) rows = &c.pt_caller;
    if (!rows || need == 0) {
        if (need) HIPCHK(hipMemcpyAsync(out, src, need, hipMemcpyDeviceToHost, c.stream));
        HIPCHK(hipStreamSynchronize(c.stream));
        return PBA_OK;
    }
    std::vector<char> tmp(need);
    HIPCHK(hipMemcpyAsync(tmp.data(), src, need, hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    const size_t row = need / rows->size();
    char *o = static_cast<char *>(out);
    for (size_t i = 0; i < rows->size(); ++i) std::memcpy(o + (size_t)(*rows)[i] * row, tmp.data() + i * row, row);
    return PBA_OK;
}

pba_status pba_autotune(pba_ctx *ctx, int32_t level, int32_t reps, pba_tune_report *out) {
    if (!ctx) return fail(nullptr, PBA_E_INVALID, "ctx is NULL");
    Ctx &c = ctx->c;
    if (level < 0 || level >= c.cfg.n_levels) return fail(&c, PBA_E_INVALID, "level out of range");
    if (reps < 1 || reps > 10000) return fail(&c, PBA_E_INVALID, "reps must be in 1..10000");
    pba_status st;
    if ((st = ready(ctx)) != PBA_OK) return st;
    if ((st = do_start_level(c, level)) != PBA_OK) return st;
    pba_tune_report rep;
    std::memset(&rep, 0, sizeof(rep));
    const bool ic = c.cfg.mode == PBA_IC_PROXY;
    if (!ic && is_mixed(c)) {
        if (out) *out = rep;
        return PBA_OK;
    }
    std::vector<LaunchShape> cand;
    if (ic)   // a thread per observation, then a lane per patch pixel
        cand = {{64, 0, 1}, {128, 0, 1}, {256, 0, 1}, {512, 0, 1}, {1024, 0, 1}, {256, 2, 1}, {256, 4, 1},
                {128, 0, 8}, {256, 0, 8}, {512, 0, 8}, {256, 2, 8}, {256, 4, 8}};
    else
        cand = {{64, 0}, {128, 0}, {256, 0}, {512, 0}, {256, 2}, {256, 4}, {256, 8}, {512, 2}, {512, 4}};
    if ((st = ensure_events(c, 2)) != PBA_OK) return st;
    hipEvent_t e0 = c.ev_pool[0], e1 = c.ev_pool[1];
    const double *geo = c.flip ? c.d_geo_b : c.d_geo_a;
    auto launch = [&](LaunchShape sh) {
        if (ic) {
            if (is_fp64(c))
                Launch<double>::ic_residual_shape(c.stream, c, level, geo, sh);
            else
                Launch<float>::ic_residual_shape(c.stream, c, level, geo, sh);
        } else {
            if (is_fp64(c))
                Launch<double>::fc_linearize_shape(c.stream, c, level, geo, sh);
            else
                Launch<float>::fc_linearize_shape(c.stream, c, level, geo, sh);
        }
    };
    launch_open(c.stream, c, level, true);
    int best = 0;
    for (size_t k = 0; k < cand.size(); ++k) {
        for (int w = 0; w < 2; ++w) launch(cand[k]);
        HIPCHK(hipEventRecord(e0, c.stream));
        for (int r = 0; r < reps; ++r) launch(cand[k]);
        HIPCHK(hipEventRecord(e1, c.stream));
        HIPCHK(hipEventSynchronize(e1));
        HIPCHK(hipGetLastError());
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        rep.block[k] = cand[k].block;
        rep.grid_mult[k] = cand[k].grid_mult;
        rep.lanes[k] = ic ? cand[k].lanes : 8;
        rep.us[k] = 1e3 * ms / reps;
        if (rep.us[k] < rep.us[best]) best = (int)k;
    }
    rep.n_candidates = (int)cand.size();
    rep.chosen = best;
    if (ic)
        c.tune_res = cand[best];
    else
        c.tune_lin = cand[best];
    drop_graph(c);
    // the level restarts at the next iteration (the FC frozen set is rewritten by it)
    c.cur_level = -1;
    if (out) *out = rep;
    return PBA_OK;
}


pba_status pba_pc_init(pba_ctx *ctx, uint64_t seed) {
    if (!ctx) return fail(nullptr, PBA_E_INVALID, "ctx is NULL");
    Ctx &c = ctx->c;
    pba_status st;
    if ((st = pc_ensure_weights(c)) != PBA_OK) return st;
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    std::vector<float> w(PC_N_PARAMS, 0.0f);
    const double s1 = std::sqrt(2.0 / PC_IN), s2 = std::sqrt(2.0 / PC_HID);
    for (int i = 0; i < PC_HID * PC_IN; ++i) w[i] = (float)(s1 * nd(rng));
    for (int i = 0; i < PC_HID * PC_HID; ++i) w[PC_OFF_W2 + i] = (float)(s2 * nd(rng));
    return pba_pc_set_weights(ctx, w.data(), w.size());
}

pba_status pba_pc_set_weights(pba_ctx *ctx, const float *w, size_t n) {
    if (!ctx) return fail(nullptr, PBA_E_INVALID, "ctx is NULL");
    Ctx &c = ctx->c;
    if (!w || n != (size_t)PC_N_PARAMS) return fail(&c, PBA_E_INVALID, "need PBA_PC_N_PARAMS weights");
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(w[i])) return fail(&c, PBA_E_INVALID, "weights must be finite");
    pba_status st;
    if ((st = pc_ensure_weights(c)) != PBA_OK) return st;
    HIPCHK(hipMemcpyAsync(c.pc.w, w, n * sizeof(float), hipMemcpyHostToDevice, c.stream));
    HIPCHK(hipMemsetAsync(c.pc.m, 0, n * sizeof(float), c.stream));
    HIPCHK(hipMemsetAsync(c.pc.v, 0, n * sizeof(float), c.stream));
    pc_to_half(c.stream, c);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c.stream));
    c.pc.adam_step = 0;
    c.pc.have_w = true;
    return PBA_OK;
}

pba_status pba_pc_get_weights(pba_ctx *ctx, float *w, size_t n) {
    if (!ctx) return fail(nullptr, PBA_E_INVALID, "ctx is NULL");
    Ctx &c = ctx->c;
    if (!w || n != (size_t)PC_N_PARAMS) return fail(&c, PBA_E_INVALID, "need PBA_PC_N_PARAMS weights");
    if (!c.pc.have_w) return fail(&c, PBA_E_STATE, "no weights (pba_pc_init or pba_pc_set_weights)");
    HIPCHK(hipMemcpyAsync(w, c.pc.w, n * sizeof(float), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    return PBA_OK;
}

pba_status pba_pc_harvest(pba_ctx *ctx, float *G_out, size_t n_floats, int32_t *n_blocks) {
    if (!ctx) return fail(nullptr, PBA_E_INVALID, "ctx is NULL");
    Ctx &c = ctx->c;
    pba_status st;
    if ((st = ready(ctx)) != PBA_OK) return st;
    const std::string e = pc_system_check(c);
    if (!e.empty()) return fail(&c, PBA_E_STATE, e);
    const int nb = c.F;
    if (!G_out || n_floats < (size_t)nb * 21) return fail(&c, PBA_E_INVALID, "G_out needs 21 F floats");
    if ((st = pc_ensure_weights(c)) != PBA_OK) return st;
    if ((st = pc_ensure_system(c, nb)) != PBA_OK) return st;
    HIPCHK(hipMemsetAsync(c.pc.flag, 0, sizeof(int), c.stream));
    pc_whiten(c.stream, c, nb);
    std::vector<double> G((size_t)nb * 21);
    int flag = 0;
    HIPCHK(hipMemcpyAsync(G.data(), c.pc.G, G.size() * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipMemcpyAsync(&flag, c.pc.flag, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    if (flag) return fail(&c, PBA_E_NUMERIC, "a diagonal block of S is not positive definite");
    for (size_t i = 0; i < G.size(); ++i) G_out[i] = (float)G[i];
    if (n_blocks) *n_blocks = nb;
    return PBA_OK;
}

pba_status pba_pc_gradient(pba_ctx *ctx, int32_t n_samples, const float *G, double *loss, float *grad) {
    if (!ctx) return fail(nullptr, PBA_E_INVALID, "ctx is NULL");
    Ctx &c = ctx->c;
    if (n_samples < 1 || n_samples > 65536 || !G) return fail(&c, PBA_E_INVALID, "need 1..65536 samples");
    if (!c.pc.have_w) return fail(&c, PBA_E_STATE, "no weights (pba_pc_init or pba_pc_set_weights)");
    pba_status st;
    if ((st = pc_upload_samples(c, n_samples, G)) != PBA_OK) return st;
    pc_forward_backward(c.stream, c, n_samples, c.pc.Xb, c.pc.Gb, c.pc.grad, c.pc.lossv);
    pc_sum(c.stream, n_samples, c.pc.lossv, c.pc.lsum);
    double ls = 0.0;
    HIPCHK(hipMemcpyAsync(&ls, c.pc.lsum, sizeof(double), hipMemcpyDeviceToHost, c.stream));
    if (grad) HIPCHK(hipMemcpyAsync(grad, c.pc.grad, PC_N_PARAMS * sizeof(float), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c.stream));
    if (loss) *loss = ls / n_samples;
    return PBA_OK;
}

pba_status pba_pc_infer(pba_ctx *ctx, int32_t n_samples, const float *G, float *Y) {
    if (!ctx) return fail(nullptr, PBA_E_INVALID, "ctx is NULL");
    Ctx &c = ctx->c;
    if (n_samples < 1 || n_samples > 65536 || !G || !Y) return fail(&c, PBA_E_INVALID, "need 1..65536 samples");
    if (!c.pc.have_w) return fail(&c, PBA_E_STATE, "no weights (pba_pc_init or pba_pc_set_weights)");
    pba_status st;
    if ((st = pc_upload_samples(c, n_samples, G)) != PBA_OK) return st;
    pc_infer(c.stream, c, n_samples, c.pc.Xb, c.pc.Yt);
    HIPCHK(hipMemcpyAsync(Y, c.pc.Yt, (size_t)n_samples * PC_OUT * sizeof(float), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c.stream));
    return PBA_OK;
}

pba_status pba_pc_train(pba_ctx *ctx, int64_t n_samples, const float *G, const pba_train_config *cfg,
                        pba_train_report *rep) {
    if (!ctx) return fail(nullptr, PBA_E_INVALID, "ctx is NULL");
    Ctx &c = ctx->c;
    if (!cfg || !G || n_samples < 1 || n_samples > (1LL << 26)) return fail(&c, PBA_E_INVALID, "bad training input");
    if (cfg->steps < 0 || cfg->batch < 1 || cfg->batch > 65536 || !(cfg->lr > 0.0f) || !(cfg->beta1 >= 0.0f) ||
        !(cfg->beta1 < 1.0f) || !(cfg->beta2 >= 0.0f) || !(cfg->beta2 < 1.0f) || !(cfg->eps > 0.0f))
        return fail(&c, PBA_E_INVALID, "bad training configuration");
    if (!c.pc.have_w) return fail(&c, PBA_E_STATE, "no weights (pba_pc_init or pba_pc_set_weights)");
    for (int64_t i = 0; i < n_samples * 21; ++i)
        if (!std::isfinite(G[i])) return fail(&c, PBA_E_INVALID, "couplings must be finite");
    PcState &p = c.pc;
    pba_status st;
    const int B = (int)std::min<int64_t>(cfg->batch, n_samples);
    if ((st = pc_ensure_batch(c, B)) != PBA_OK) return st;
    // samples and their features on the device
    dfree(p.Gs);
    dfree(p.Xs);
    HIPCHK(dalloc(p.Gs, (size_t)n_samples * 21 * sizeof(float)));
    HIPCHK(dalloc(p.Xs, (size_t)n_samples * PC_IN * sizeof(float)));
    HIPCHK(hipMemcpyAsync(p.Gs, G, (size_t)n_samples * 21 * sizeof(float), hipMemcpyHostToDevice, c.stream));
    pc_features(c.stream, (int)n_samples, p.Gs, p.Xs);
    p.ns = n_samples;
    int *didx = nullptr;
    HIPCHK(dalloc(didx, (size_t)n_samples * sizeof(int)));
    std::mt19937_64 rng(cfg->seed);
    std::vector<int> perm(n_samples);
    std::iota(perm.begin(), perm.end(), 0);
    pba_train_report r;
    std::memset(&r, 0, sizeof(r));
    r.samples = n_samples;
    double jl = 0.0;
    for (int64_t i = 0; i < n_samples; ++i)
        for (int k = 0; k < 6; ++k) jl += (double)G[21 * i + k * 6 - k * (k - 1) / 2];
    r.jacobi_loss = jl / n_samples;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    int64_t pos = n_samples;  // reshuffle at the first step
    HIPCHK(hipEventRecord(e0, c.stream));
    for (int step = 0; step < cfg->steps; ++step) {
        if (pos + B > n_samples) {
            std::shuffle(perm.begin(), perm.end(), rng);
            HIPCHK(hipMemcpyAsync(didx, perm.data(), perm.size() * sizeof(int), hipMemcpyHostToDevice, c.stream));
            HIPCHK(hipStreamSynchronize(c.stream));  // perm is reused by the next reshuffle
            pos = 0;
        }
        pc_gather(c.stream, B, didx + pos, p.Xs, PC_IN, p.Xb);
        pc_gather(c.stream, B, didx + pos, p.Gs, 21, p.Gb);
        pos += B;
        pc_forward_backward(c.stream, c, B, p.Xb, p.Gb, p.grad, p.lossv);
        if (step == 0 || step == cfg->steps - 1) {
            pc_sum(c.stream, B, p.lossv, p.lsum);
            double ls = 0.0;
            HIPCHK(hipMemcpyAsync(&ls, p.lsum, sizeof(double), hipMemcpyDeviceToHost, c.stream));
            HIPCHK(hipStreamSynchronize(c.stream));
            (step == 0 ? r.first_loss : r.final_loss) = ls / B;
        }
        pc_adam(c.stream, c, cfg->lr, cfg->beta1, cfg->beta2, cfg->eps, ++p.adam_step);
    }
    HIPCHK(hipEventRecord(e1, c.stream));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    r.ms = ms;
    r.steps = cfg->steps;
    // mean loss of the trained network over all samples (FP32 forward, chunks of B)
    double tot = 0.0;
    for (int64_t i0 = 0; i0 < n_samples; i0 += B) {
        const int m = (int)std::min<int64_t>(B, n_samples - i0);
        pc_forward_backward(c.stream, c, m, p.Xs + i0 * PC_IN, p.Gs + i0 * 21, p.grad, p.lossv);
        pc_sum(c.stream, m, p.lossv, p.lsum);
        double ls = 0.0;
        HIPCHK(hipMemcpyAsync(&ls, p.lsum, sizeof(double), hipMemcpyDeviceToHost, c.stream));
        HIPCHK(hipStreamSynchronize(c.stream));
        tot += ls;
    }
    r.trained_loss = tot / n_samples;
    pc_to_half(c.stream, c);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c.stream));
    dfree(didx);
    if (rep) *rep = r;
    return PBA_OK;
}

pba_status pba_solve_reduced(pba_ctx *ctx, int32_t solver, double tol, int32_t max_iters, double *x_out,
                             pba_reduced_report *rep) {
    if (!ctx) return fail(nullptr, PBA_E_INVALID, "ctx is NULL");
    Ctx &c = ctx->c;
    if (solver != PBA_SOLVER_CHOL && solver != PBA_SOLVER_PCG_JACOBI && solver != PBA_SOLVER_PCG_LEARNED &&
        solver != PBA_SOLVER_PCG_BLOCKOPT)
        return fail(&c, PBA_E_INVALID, "unknown solver");
    if (!(tol > 0.0) || max_iters < 1) return fail(&c, PBA_E_INVALID, "tol must be > 0 and max_iters >= 1");
    pba_status st;
    if ((st = ready(ctx)) != PBA_OK) return st;
    const std::string e = pc_system_check(c);
    if (!e.empty()) return fail(&c, PBA_E_STATE, e);
    if (solver == PBA_SOLVER_PCG_LEARNED && !c.pc.have_w)
        return fail(&c, PBA_E_STATE, "no weights (pba_pc_init, pba_pc_set_weights or pba_pc_train)");
    const int nb = c.F, n = 6 * c.F;
    if ((st = pc_ensure_weights(c)) != PBA_OK) return st;
    if ((st = pc_ensure_system(c, nb)) != PBA_OK) return st;
    if (!c.d_Sfac) {
        const size_t nt = (n + TCHOL_TILE - 1) / TCHOL_TILE;
        HIPCHK(dalloc(c.d_Sfac, (size_t)n * n * sizeof(double)));
        HIPCHK(dalloc(c.d_Linv, nt * TCHOL_TILE * TCHOL_TILE * sizeof(double)));
    }
    if ((st = ensure_events(c, 3)) != PBA_OK) return st;
    hipEvent_t e0 = c.ev_pool[0], e1 = c.ev_pool[1], e2 = c.ev_pool[2];
    hipStream_t s = c.stream;
    pba_reduced_report r;
    std::memset(&r, 0, sizeof(r));
    r.solver = solver;
    const double *xdev = c.pc.x;
    auto cholesky = [&](bool timed_setup) -> pba_status {
        launch_open(s, c, 0, true);  // gate open, flag clear
        launch_tchol(s, c);
        if (timed_setup) HIPCHK(hipEventRecord(e1, s));
        launch_tsolve(s, c, c.d_b, c.pc.x);
        return PBA_OK;
    };
    HIPCHK(hipEventRecord(e0, s));
    if (solver == PBA_SOLVER_CHOL) {
        if ((st = cholesky(true)) != PBA_OK) return st;
    } else {
        HIPCHK(hipMemsetAsync(c.pc.flag, 0, sizeof(int), s));
        pc_whiten(s, c, nb);
        if (solver == PBA_SOLVER_PCG_LEARNED) {
            pc_infer(s, c, nb, c.pc.X, c.pc.Y);
            pc_blocks(s, c, nb, c.pc.Y);
        } else if (solver == PBA_SOLVER_PCG_BLOCKOPT) {
            pc_blocks_opt(s, c, nb);
        } else {
            pc_blocks(s, c, nb, nullptr);
        }
        HIPCHK(hipEventRecord(e1, s));
        pcg_init(s, c, n);
        int hst[2] = {0, 0};
        const int chunk = 16;
        int done_iters = 0;
        while (done_iters < max_iters) {
            const int k = std::min(chunk, max_iters - done_iters);
            pcg_iterations(s, c, n, k, tol);
            done_iters += k;
            HIPCHK(hipMemcpyAsync(hst, c.pc.st, sizeof(hst), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (hst[0]) break;
        }
        int pflag = 0;
        HIPCHK(hipMemcpyAsync(&pflag, c.pc.flag, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (pflag) return fail(&c, PBA_E_NUMERIC, "a diagonal block of S is not positive definite");
        r.iters = hst[1];
        r.converged = hst[0] && hst[1] <= max_iters ? 1 : 0;
        if (!r.converged) {
            r.fallback = 1;
            if ((st = cholesky(false)) != PBA_OK) return st;
        }
    }
    HIPCHK(hipEventRecord(e2, s));
    // relative residual of the returned x
    const int parts = (n + 7) / 8;
    pc_resid(s, c, n, xdev, c.pc.part);
    std::vector<double> hp(parts), hb(n);
    int cflag = 0;
    HIPCHK(hipMemcpyAsync(hp.data(), c.pc.part, parts * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hb.data(), c.d_b, n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&cflag, c.d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    if (x_out) HIPCHK(hipMemcpyAsync(x_out, xdev, n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    if ((solver == PBA_SOLVER_CHOL || r.fallback) && cflag)
        return fail(&c, PBA_E_NUMERIC, "reduced pose system is not positive definite");
    double rr = 0.0, bb = 0.0;
    for (double v : hp) rr += v;
    for (double v : hb) bb += v * v;
    r.rel_residual = bb > 0.0 ? std::sqrt(rr / bb) : std::sqrt(rr);
    float ms = 0.f, ms1 = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e2));
    HIPCHK(hipEventElapsedTime(&ms1, e0, e1));
    r.ms = ms;
    r.ms_setup = ms1;
    if (rep) *rep = r;
    return PBA_OK;
}

pba_status pba_get_timing(pba_ctx *ctx, pba_timing *out) {
    if (!ctx) return fail(nullptr, PBA_E_INVALID, "ctx is NULL");
    Ctx &c = ctx->c;
    if (!out) return fail(&c, PBA_E_INVALID, "out is NULL");
    for (int l = 0; l < PBA_MAX_LEVELS; ++l) {
        out->residual_launches[l] = c.t_launches[l];
        out->residual_ms[l] = c.t_ms[l];
        out->residuals_processed[l] = c.t_res[l];
        out->step_launches[l] = c.t_step_launches[l];
        out->step_ms[l] = c.t_step_ms[l];
        c.t_launches[l] = 0;
        c.t_ms[l] = 0.0;
        c.t_res[l] = 0;
        c.t_step_launches[l] = 0;
        c.t_step_ms[l] = 0.0;
    }
    return PBA_OK;
}

}  // extern "C"
