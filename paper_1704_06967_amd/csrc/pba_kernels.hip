// HIP kernels of libpba for CDNA4 (gfx950, wave64).
//
// The linearization kernels put one observation (point n seen in frame f) on
// 8 consecutive lanes, one lane per patch pixel, 8 observations per
// wavefront; each observation reduces its lanes with cross-lane DPP moves and
// writes one record of Gauss-Newton blocks in relative-pose coordinates. The
// IC iteration's residual pass runs one observation per thread. Every later
// reduction (per point, per pair, per frame) runs in a fixed order in FP64, so
// results are bitwise reproducible run to run (no floating-point atomics).
#include <hip/hip_ext.h>

#include "pba_depth.hpp"
#include "pba_device.hpp"
#include "pba_internal.hpp"

#include <algorithm>

namespace pba {

#define CHECK_LAUNCH() (void)hipGetLastError()

// ------------------------------------------------------------ images

template <typename T>
__global__ void k_convert(const float *__restrict__ src, T *__restrict__ dst, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (T)src[i];
}

// Level l+1 = 2x2 box average of level l.
template <typename T>
__global__ void k_downsample(const T *__restrict__ src, T *__restrict__ dst, int F, int Ws, int Hs, int Wd,
                             int Hd) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t total = (size_t)F * Wd * Hd;
    if (i >= total) return;
    int x = i % Wd;
    int y = (i / Wd) % Hd;
    int f = i / ((size_t)Wd * Hd);
    const T *s = src + (size_t)f * Ws * Hs + (size_t)(2 * y) * Ws + 2 * x;
    dst[i] = T(0.25) * (((s[0] + s[1]) + s[Ws]) + s[Ws + 1]);
}

template <typename T>
__global__ void k_level_K(const double *__restrict__ K0, T *__restrict__ K, int F, int level) {
    int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const double s = 1.0 / (double)(1 << level);
    K[4 * f + 0] = (T)(K0[4 * f + 0] * s);
    K[4 * f + 1] = (T)(K0[4 * f + 1] * s);
    K[4 * f + 2] = (T)((K0[4 * f + 2] + 0.5) * s - 0.5);
    K[4 * f + 3] = (T)((K0[4 * f + 3] + 0.5) * s - 0.5);
}

// Level intrinsics (FP64, every element type) of every pair's host and target
// frames, side by side, so that a residual reads its camera data with its pair
// index alone: f / 2^l and (c + 0.5) / 2^l - 0.5 from the level-0 values.
__global__ void k_pair_cam(int Pn, const int *__restrict__ pair_host, const int *__restrict__ pair_target,
                           const double *__restrict__ K0, int level, double *__restrict__ pcam) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= Pn * 8) return;
    const int p = e >> 3, k = e & 7;
    const int f = k < 4 ? pair_host[p] : pair_target[p];
    const double s = 1.0 / (double)(1 << level), k0 = K0[4 * f + (k & 3)];
    pcam[e] = (k & 3) < 2 ? k0 * s : (k0 + 0.5) * s - 0.5;
}

// Template data at every host patch pixel: I0, the interpolated central-difference
// gradient, and whether the pixel is usable at this level.
template <typename T>
__global__ void k_template(int N, int P, PatternArg pat, const float *__restrict__ host_uv,
                           const int *__restrict__ host_frame, const T *__restrict__ img, int W, int H, T scale,
                           T *__restrict__ tmpl) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * P) return;
    int n = idx / P, j = idx % P;
    const T u = ((T)host_uv[2 * n] + T(0.5)) * scale - T(0.5) + (T)pat.du[j];
    const T v = ((T)host_uv[2 * n + 1] + T(0.5)) * scale - T(0.5) + (T)pat.dv[j];
    T I = 0, gu = 0, gv = 0, ok = 0;
    if (usable(u, v, W, H)) {
        double Id, gud, gvd;
        bilinear_grad(img + (size_t)host_frame[n] * W * H, W, u, v, Id, gud, gvd);
        I = (T)Id;
        gu = (T)gud;
        gv = (T)gvd;
        ok = 1;
    }
    tmpl[4 * idx + 0] = I;
    tmpl[4 * idx + 1] = gu;
    tmpl[4 * idx + 2] = gv;
    tmpl[4 * idx + 3] = ok;
}

// ------------------------------------------------------------ poses

// Relative pose of every (host, target) pair: R = R_f R_h^T, t = t_f - R t_h.
template <typename T>
__global__ void k_relpose(int Pn, const int *__restrict__ pair_host, const int *__restrict__ pair_target,
                          const double *__restrict__ poses, double *__restrict__ geo, T *__restrict__ rel) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= Pn) return;
    const double *Ph = poses + 12 * pair_host[p];
    const double *Pf = poses + 12 * pair_target[p];
    double R[9];
    mat3_mul_bt(Pf, Ph, R);
    double t[3];
    for (int i = 0; i < 3; ++i) t[i] = Pf[9 + i] - (R[i * 3] * Ph[9] + R[i * 3 + 1] * Ph[10] + R[i * 3 + 2] * Ph[11]);
    double *g = geo + GEO_STRIDE * p;
    for (int i = 0; i < 9; ++i) g[i] = R[i];
    for (int i = 0; i < 3; ++i) g[9 + i] = t[i];
    for (int i = 0; i < 3; ++i) g[12 + i] = Ph[9 + i];
    g[15] = 0.0;
    T *r = rel + REL_STRIDE * p;
    for (int i = 0; i < 9; ++i) r[i] = (T)R[i];
    for (int i = 0; i < 3; ++i) r[9 + i] = (T)t[i];
}

// Start of a level, one launch: the level's gate, failure flag (cleared with
// clear_flag) and iteration count; p(0) copies of the poses and inverse depths;
// the relative poses of every pair at p(0), kept as the IC linearization point
// (geo0, rel0) and as the current iterate (geo_a, rel_a). With recentre set
// (proxy re-centring inside a level) the gate, flag and count are left as they
// are, nothing happens once the gate is closed, and count_base receives the
// iterations run so far (the pose buffers alternate from this point on).
template <typename T>
__global__ void k_level_begin(int F, int N, int Pn, const double *__restrict__ poses, double *__restrict__ poses0,
                              const double *__restrict__ depth, double *__restrict__ depth0,
                              const int *__restrict__ pair_host, const int *__restrict__ pair_target,
                              double *__restrict__ geo0, T *__restrict__ rel0, double *__restrict__ geo_a,
                              T *__restrict__ rel_a, int *__restrict__ gate, int *__restrict__ flag,
                              int *__restrict__ count, int *__restrict__ count_base, int clear_flag, int recentre) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (recentre) {
        if (*gate == 0) return;
        if (i == 0) *count_base = *count;
    } else if (i == 0) {
        if (clear_flag) *flag = 0;
        *gate = *flag == 0 ? 1 : 0;
        *count = 0;
        *count_base = 0;
    }
    if (i < 12 * F) poses0[i] = poses[i];
    if (i < N) depth0[i] = depth[i];
    if (i < Pn) {
        const double *Ph = poses + 12 * pair_host[i];
        const double *Pf = poses + 12 * pair_target[i];
        double R[9];
        mat3_mul_bt(Pf, Ph, R);
        double t[3];
        for (int k = 0; k < 3; ++k) t[k] = Pf[9 + k] - (R[k * 3] * Ph[9] + R[k * 3 + 1] * Ph[10] + R[k * 3 + 2] * Ph[11]);
        double *g0 = geo0 + GEO_STRIDE * i, *ga = geo_a + GEO_STRIDE * i;
        T *r0 = rel0 + REL_STRIDE * i, *ra = rel_a + REL_STRIDE * i;
        for (int k = 0; k < 9; ++k) {
            g0[k] = ga[k] = R[k];
            r0[k] = ra[k] = (T)R[k];
        }
        for (int k = 0; k < 3; ++k) {
            g0[9 + k] = ga[9 + k] = t[k];
            r0[9 + k] = ra[9 + k] = (T)t[k];
            g0[12 + k] = ga[12 + k] = Ph[9 + k];
        }
        g0[15] = ga[15] = 0.0;
    }
}

// ------------------------------------------------------------ residual kernels

template <typename T>
struct ResArgs {
    int O, P, W, H;
    PatternArg pat;
    double scale;        // 1 / 2^level
    T huber_k;
    const int *obs_point, *obs_pair, *pair_host, *pair_target;
    const float *host_uv;
    const T *img;        // level image stack
    const T *tmpl;       // [N][P][4]
    const double *geo;   // current pair geometry [Pn][GEO_STRIDE]: relative R, t; host t
    const T *rel0;       // relative poses at p(0) (IC Jacobian)
    const double *depth, *depth0;
    uint8_t *mask;
    const uint8_t *live; // 1 while the observation is in the window
    double *rec;         // per-observation records (FP64 for every element type)
    const double *pcam;  // per pair: host and target level intrinsics (fx, fy, cx, cy) x 2
    double *icr;         // IC iterations: per observation g (6), g_d, energy, sum r^2, count (FP64)
    double *gdo;         // IC iterations: g_d again, one value per observation (for the depth readers)
    const int *gate;     // device flag: 0 = the solve has converged, skip the work
};

// Normalized template coordinates of patch pixel j of point n (host
// intrinsics). The warp of every element type runs in FP64: single-precision
// pixel coordinates near 600 carry 3e-5 px of rounding, which moves r by the
// image gradient times that (and the inverse depths of weakly constrained
// points by 1e-5 relative and more); only the sampled intensities, J and the
// sums run in the element type.
template <typename T>
__device__ __forceinline__ void template_xy(const ResArgs<T> &a, int n, int j, const double *Kh, double &x,
                                            double &y) {
    const double u = ((double)a.host_uv[2 * n] + 0.5) * a.scale - 0.5 + (double)a.pat.du[j];
    const double v = ((double)a.host_uv[2 * n + 1] + 0.5) * a.scale - 0.5 + (double)a.pat.dv[j];
    x = (u - Kh[2]) * (1.0 / Kh[0]);
    y = (v - Kh[3]) * (1.0 / Kh[1]);
}

// Linearization of one residual (observation o, patch pixel j), shared by the
// FC iteration and the IC setup. IC: J from the proxy warp at p(0) (Sec. 3.4)
// and W0 from the residual at p(0). FC: J at the current parameters from the
// target gradient. Returns whether the residual contributes.
template <typename T, bool IC>
__device__ __forceinline__ bool lin_eval(const ResArgs<T> &a, int o, int j, int write_mask, T (&J)[7], T &r, T &w,
                                         T &rho) {
#pragma unroll
    for (int p = 0; p < 7; ++p) J[p] = 0;
    r = w = rho = 0;
    if (o < 0 || o >= a.O || j >= a.P) return false;
    const int n = a.obs_point[o], pr = a.obs_pair[o];
    const int f = a.pair_target[pr];
    const double *Kh = a.pcam + 8 * pr;   // the pair's host and target intrinsics (one load step fewer than K[frame])
    const double *Kt = Kh + 4;
    const T *tp = a.tmpl + 4 * ((size_t)n * a.P + j);
    const T I0 = tp[0], gu0 = tp[1], gv0 = tp[2];
    const bool host_ok = tp[3] != T(0);
    // the frozen set: written from the usable residuals of the observations
    // still in the window, or read
    const bool frozen = write_mask ? a.live[o] != 0 : ((a.mask[o] >> j) & 1) != 0;
    double x, y;
    template_xy(a, n, j, Kh, x, y);
    const double *R = a.geo + GEO_STRIDE * pr;
    const double *t = R + 9;
    const double d = a.depth[n];
    const double Rx0 = R[0] * x + R[1] * y + R[2];
    const double Rx1 = R[3] * x + R[4] * y + R[5];
    const double Rx2 = R[6] * x + R[7] * y + R[8];
    const double vx = Rx0 + d * t[0], vy = Rx1 + d * t[1], vz = Rx2 + d * t[2];
    if (!(host_ok && frozen && d > 0.0 && vz > 0.0)) return false;
    const double iz = 1.0 / vz;   // one FP64 division for the projection
    const double ux = vx * iz, uy = vy * iz;
    const double qu = Kt[0] * ux + Kt[2], qv = Kt[1] * uy + Kt[3];
    if (!usable(qu, qv, a.W, a.H)) return false;
    const T *imf = a.img + (size_t)f * a.W * a.H;
    double If;
    if (IC) {
        If = bilinear(imf, a.W, qu, qv);
        const T *R0 = a.rel0 + REL_STRIDE * pr;
        const T d0 = (T)a.depth0[n];
        ic_jacobian((T)x, (T)y, R0, R0 + 9, d0, recip(d0), gu0, gv0, (T)Kh[0], (T)Kh[1], J);
    } else {
        // the row in FP64 from the FP64 gradient, rounded to T once
        double gu, gv, Jd[7];
        bilinear_grad(imf, a.W, qu, qv, If, gu, gv);
        fc_jacobian(Rx0, Rx1, Rx2, vz, ux, uy, t, d, gu, gv, Kt[0], Kt[1], Jd);
#pragma unroll
        for (int p = 0; p < 7; ++p) J[p] = (T)Jd[p];
    }
    r = (T)((double)I0 - If);   // rounded once (bilinear)
    huber(r, a.huber_k, w, rho);
    return true;
}

// Tile of the i-th workgroup in an XCD-aware order. Workgroups are dispatched
// to the 8 XCDs in turn (workgroup i to XCD i mod 8), and each XCD has its own
// L2; this bijection of [0, ntiles) gives XCD x one contiguous range of tiles
// (ntiles / 8 of them, one more for the first ntiles mod 8 XCDs), so that
// neighbouring observations (points are stored in a spatial order) meet in
// one L2.
__device__ __forceinline__ int xcd_tile(int i, int ntiles) {
    const int q = ntiles >> 3, r = ntiles & 7, x = i & 7;
    return x * q + min(x, r) + (i >> 3);
}

// Sum over an observation's 8 lanes of a per-residual product, in FP64 for
// every element type, into the field slot that lane j of the observation
// stores (fields p with p % 8 == j, slot p / 8). Single-precision products and
// sums would round the pose block, h and H_dd of an observation independently
// (a few units in the last place of each), which breaks the consistency of the
// depth Schur complement and moves the FP32 iterates by up to 1e-5 relative;
// from FP64 sums the record is rounded to T once. The empty asm keeps the
// compiler from fusing the product into the first addition, so that every
// lane of the group ends with the same sum.
template <int NS>
__device__ __forceinline__ void obs_sum_field(double (&mine)[NS], int j, int p, double v) {
    pin_reg(v);
    v = wave_sum8(v);
    mine[p >> 3] = (j == (p & 7)) ? v : mine[p >> 3];
}

// Linearization in observation order: the 38-value record of every
// observation (lane j stores fields j, j + 8, ...). NB threads per workgroup
// (NB / 8 observations per tile); the grid strides over the tiles, so that it
// can be launched one tile per workgroup or as a persistent grid.
template <typename T, bool IC, int NB>
__global__ __launch_bounds__(NB) void k_linearize(ResArgs<T> a, int write_mask) {
    if (*a.gate == 0) return;
    const int ntiles = (a.O + NB / 8 - 1) / (NB / 8);
    for (int it = blockIdx.x; it < ntiles; it += gridDim.x) {
        const int tile = xcd_tile(it, ntiles);
        const int gid = tile * NB + threadIdx.x;
        const int o = gid >> 3, j = gid & 7;
        T J[7], r, w, rho;
        const bool valid = lin_eval<T, IC>(a, o, j, write_mask, J, r, w, rho);
        if (write_mask) {
            const unsigned long long bal = __ballot(valid);
            if (j == 0 && o < a.O) a.mask[o] = (uint8_t)((bal >> (threadIdx.x & 56)) & 0xFFull);
        }
        double mine[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        const double wd = (double)w;
        int k = 0;
#pragma unroll
        for (int p = 0; p < 6; ++p)
#pragma unroll
            for (int q = p; q < 6; ++q) obs_sum_field(mine, j, k++, wd * J[p] * J[q]);
#pragma unroll
        for (int p = 0; p < 6; ++p) obs_sum_field(mine, j, REC_h + p, wd * J[p] * J[6]);
        obs_sum_field(mine, j, REC_HDD, wd * J[6] * J[6]);
#pragma unroll
        for (int p = 0; p < 7; ++p) obs_sum_field(mine, j, REC_G + p, wd * J[p] * r);
        obs_sum_field(mine, j, REC_E, valid ? (double)rho : 0.0);
        obs_sum_field(mine, j, REC_SQ, valid ? (double)r * r : 0.0);
        obs_sum_field(mine, j, REC_CNT, valid ? 1.0 : 0.0);
        if (o < a.O) {
            double *rec = a.rec + (size_t)o * REC_STRIDE;
#pragma unroll
            for (int i = 0; i < 5; ++i)
                if (8 * i + j <= REC_CNT) rec[8 * i + j] = mine[i];
        }
    }
}

// Mixed precision: residuals and J in FP32, the pose-pose block of every pair
// contracted on BF16 MFMA. The kernel walks one pair chunk per block (pair
// order), so that a wavefront's 64 residuals (8 observations x 8 patch pixels)
// belong to one pair. The rows u = sqrt(w) J_theta of a 64-residual group are
// put on a fixed-point grid per component p: with S_p the power of two at or
// above the group's largest |u_p|, u_p / S_p = t0 + t1 + t2 + t3, term k an
// integer (|i| <= 128) times 2^-(7 + 8k), i.e. exactly a bfloat16 (the
// quantized row differs from u by at most 2^-32 S_p: a residual whose |u_p| is
// 1e-3 of the group's largest keeps 2e-7 relative, where three terms left
// 6e-5, enough to move the FC iterates of weakly constrained points by 2e-5
// in inverse depth after 5 iterations). Every product of two such terms is an
// integer multiple of one unit per term pair (unit k + l), and the at most 4 x
// 64 products of one unit in a group (two 16x16x32 MFMAs per term pair) sum
// to below 2^22 units, so the FP32 accumulation of v_mfma_f32_16x16x32_bf16
// is exact whatever its internal order: the sixteen term products are kept in
// seven accumulators by unit and added, smallest unit first, scaled by
// S_p S_q, in FP64. The pose block is thus the exact Gram of the quantized
// rows, and h and H_dd of the record are FP64 sums over the same quantized
// rows: the per-point blocks of the depth Schur complement stay consistent
// (PSD as a Gram), which a rounded FP32 accumulation (~1e-7 relative, out of
// step with FP64 h and H_dd) does not keep: that moved the iterates along the
// weak directions of S by up to 1e-4 relative in inverse depth. The four
// wavefronts' FP64 sums are added in a fixed order into the chunk partial (21
// values) that the damping kernel sums per pair.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <bool IC>
__global__ __launch_bounds__(BLOCK) void k_linearize_mixed(ResArgs<float> a, int write_mask,
                                                           const int *__restrict__ chunk_begin,
                                                           const int *__restrict__ chunk_end,
                                                           const int *__restrict__ pair_obs_idx,
                                                           double *__restrict__ partH) {
    constexpr int NS = 4;  // fixed-point terms
    constexpr int NU = 7;  // accumulators by unit: term index sum 0..6
    // per wavefront: the terms of u^T as 16 x 64 bfloat16 (rows 6..15 stay zero)
    __shared__ __attribute__((aligned(16))) __bf16 ut[BLOCK / 64][NS][16][64];
    __shared__ double wsum[BLOCK / 64][36];
    if (*a.gate == 0) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int e = lane; e < NS * 16 * 64; e += 64) (&ut[wv][0][0][0])[e] = (__bf16)0.0f;
    const int c = blockIdx.x, cb = chunk_begin[c], ce = chunk_end[c];
    const int j = lane & 7;
    // this lane's elements of the 16 x 16 Gram: rows 4 (lane / 16) + i, column lane % 16
    const int col = lane & 15, row0 = 4 * (lane >> 4);
    double tot[4] = {0.0, 0.0, 0.0, 0.0};
    for (int g = wv; 8 * g < ce - cb; g += BLOCK / 64) {
        const int pos = cb + 8 * g + (lane >> 3);
        const int o = pos < ce ? pair_obs_idx[pos] : -1;
        float J[7], r, w, rho;
        const bool valid = lin_eval<float, IC>(a, o, j, write_mask, J, r, w, rho);
        if (write_mask) {
            const unsigned long long bal = __ballot(valid);
            if (j == 0 && o >= 0) a.mask[o] = (uint8_t)((bal >> (lane & 56)) & 0xFFull);
        }
        // rows u = sqrt(w) J on the group's fixed-point grid
        const double sw = sqrt((double)w);
        const double ud = sw * (double)J[6];
        double uq[6], scale[6];
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            const double u = sw * (double)J[p];
            const double m = wave_max(fabs(u));
            int ex = 0;
            (void)frexp(m, &ex);                     // m < 2^ex (m = 0: ex = 0)
            scale[p] = ldexp(1.0, ex);
            double rem = u / scale[p];               // |rem| < 1, exact (power-of-two scale)
            double q = 0.0;
#pragma unroll
            for (int t = 0; t < NS; ++t) {
                // term t: rem rounded to a multiple of 2^-(7 + 8t); the
                // remainder stays exact, |rem| <= 2^-(8 + 8t)
                const double g = ldexp(1.0, 7 + 8 * t);
                const double term = rint(rem * g) / g;
                rem -= term;
                q += term;                           // exact (fits in 53 bits)
                ut[wv][t][p][lane] = (__bf16)(float)term;   // exactly a bfloat16
            }
            uq[p] = scale[p] * q;                    // exact
        }
        // per-observation fields (all but the pose-pose block: REC_h .. REC_CNT,
        // which are contiguous), FP64 sums as in k_linearize, h and H_dd over
        // the quantized rows; field REC_h + p goes to slot p / 8 of lane p % 8
        double mine[3] = {0.0, 0.0, 0.0};
        const double wd = (double)w;
#pragma unroll
        for (int p = 0; p < 6; ++p) obs_sum_field(mine, j, p, uq[p] * ud);
        obs_sum_field(mine, j, REC_HDD - REC_h, ud * ud);
#pragma unroll
        for (int p = 0; p < 7; ++p) obs_sum_field(mine, j, REC_G - REC_h + p, wd * J[p] * r);
        obs_sum_field(mine, j, REC_E - REC_h, valid ? (double)rho : 0.0);
        obs_sum_field(mine, j, REC_SQ - REC_h, valid ? (double)r * r : 0.0);
        obs_sum_field(mine, j, REC_CNT - REC_h, valid ? 1.0 : 0.0);
        if (o >= 0) {
            double *rec = a.rec + (size_t)o * REC_STRIDE + REC_h;
#pragma unroll
            for (int i = 0; i < 3; ++i)
                if (8 * i + j <= REC_CNT - REC_h) rec[8 * i + j] = mine[i];
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        f32x4 acc[NU];
#pragma unroll
        for (int m = 0; m < NU; ++m) acc[m] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int k0 = 32 * s + 8 * (lane >> 4);
            bf16x8 f[NS];
#pragma unroll
            for (int t = 0; t < NS; ++t) f[t] = *reinterpret_cast<const bf16x8 *>(&ut[wv][t][lane & 15][k0]);
#pragma unroll
            for (int ta = 0; ta < NS; ++ta)
#pragma unroll
                for (int tb = 0; tb < NS; ++tb)
                    acc[ta + tb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f[ta], f[tb], acc[ta + tb], 0, 0, 0);
        }
        __builtin_amdgcn_wave_barrier();
        // the exact FP32 sums (smallest unit first) in FP64, then S_p S_q
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int rw = row0 + i;
            double t = (double)acc[NU - 1][i];
#pragma unroll
            for (int m = NU - 2; m >= 0; --m) t += (double)acc[m][i];
            double sr = 0.0, sc = 0.0;   // S of the element's row and column (selects, no indexed registers)
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                sr = rw == p ? scale[p] : sr;
                sc = col == p ? scale[p] : sc;
            }
            tot[i] += t * sr * sc;
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int rw = row0 + i;
        if (rw < 6 && col < 6) wsum[wv][rw * 6 + col] = tot[i];
    }
    __syncthreads();
    if (threadIdx.x < 21) {
        int p = 0, k = threadIdx.x;
        while (k >= 6 - p) {
            k -= 6 - p;
            ++p;
        }
        const int pq = p * 6 + p + k;
        double sum = 0.0;
        for (int w2 = 0; w2 < BLOCK / 64; ++w2) sum += wsum[w2][pq];
        partH[21 * (size_t)c + threadIdx.x] = sum;
    }
}

// IC iteration: residuals at the current parameters, Huber weights, and
// g = J^T W r with the constant proxy Jacobian (Sec. 3.5 steps 1-2), per
// observation the ten FP64 sums of its patch pixels' products (J_theta w r,
// J_d w r, the Huber norm, r^2, the count). One thread per observation: it
// loads the pair's data (host and target intrinsics, the current relative
// pose, the relative pose at p(0)) and the point's once, runs the patch
// pixels in pairs (every load of a pair issued first) and keeps the ten sums
// in registers, so no cross-lane reduction and no broadcast is needed; the
// threads of a wavefront share the pair loads through the caches. NB threads
// per workgroup, tiles of NB observations, grid-stride over the tiles in the
// XCD-aware order; the ten sums go out as the observation's contiguous record.

// The observation's data: the pair's projection and p(0) pose, the point's
// pixel and inverse depths.
template <typename T>
struct IcObs {
    double Q[12];            // (qu vz, qv vz, vz) = Q (x, y, 1, d)
    double cx, cy, ifx, ify; // host intrinsics: principal point, 1 / focal lengths
    double uc, vc, d;        // level pixel of the point, current inverse depth
    T R0[12];                // relative R (row-major), t at p(0)
    T d0, id0, fx, fy;       // inverse depth at p(0) and its reciprocal, host focal lengths
    const T *img, *tmpl;     // target level image, the point's template records
    unsigned m;              // pixels usable at p(0)
};

// The pair's part of the observation's data from its intrinsics K (host fx
// fy cx cy, target fx fy cx cy) and current relative pose G (R row-major, t).
template <typename T>
__device__ __forceinline__ void ic_obs_pair(const double (&K)[8], const double (&G)[12], IcObs<T> &ob) {
    ob.ifx = 1.0 / K[0];
    ob.ify = 1.0 / K[1];
    ob.cx = K[2];
    ob.cy = K[3];
    ob.fx = (T)K[0];
    ob.fy = (T)K[1];
    // rows of diag(fx_t, fy_t, 1) [R | t] + (cx_t, cy_t, 0) e3^T [R | t]: the
    // warp and projection of lin_eval with the target intrinsics folded in
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        ob.Q[k] = K[4] * G[k] + K[6] * G[6 + k];
        ob.Q[4 + k] = K[5] * G[3 + k] + K[7] * G[6 + k];
        ob.Q[8 + k] = G[6 + k];
    }
    ob.Q[3] = K[4] * G[9] + K[6] * G[11];
    ob.Q[7] = K[5] * G[10] + K[7] * G[11];
    ob.Q[11] = G[11];
}

// The point's pixel at the level and its inverse depths.
template <typename T>
__device__ __forceinline__ void ic_obs_point(const ResArgs<T> &a, float hu, float hv, double d, double d0,
                                             IcObs<T> &ob) {
    ob.uc = ((double)hu + 0.5) * a.scale - 0.5;
    ob.vc = ((double)hv + 0.5) * a.scale - 0.5;
    ob.d = d;
    ob.d0 = (T)d0;
    ob.id0 = recip(ob.d0);
}

template <typename T>
__device__ __forceinline__ void ic_obs_load(const ResArgs<T> &a, int o, IcObs<T> &ob) {
    const int n = a.obs_point[o], pr = a.obs_pair[o];
    const int f = a.pair_target[pr];
    double K[8], G[12];
#pragma unroll
    for (int k = 0; k < 8; ++k) K[k] = a.pcam[8 * pr + k];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        G[k] = a.geo[GEO_STRIDE * pr + k];
        ob.R0[k] = a.rel0[REL_STRIDE * pr + k];
    }
    ic_obs_pair(K, G, ob);
    ic_obs_point(a, a.host_uv[2 * n], a.host_uv[2 * n + 1], a.depth[n], a.depth0[n], ob);
    ob.img = a.img + (size_t)f * a.W * a.H;
    ob.tmpl = a.tmpl + 4 * (size_t)n * a.P;
}

// First step of patch pixel j: the warp (FP64, as template_xy and lin_eval),
// the template and texel loads. A pixel that does not contribute reads the
// in-bounds cell at (1, 1) and is masked.
template <typename T>
struct IcPix {
    bool ok;
    double fa, fb;   // the position's fractions in its cell
    T x, y, tq[3], tx[4];
};

template <typename T>
__device__ __forceinline__ void ic_pixel_template(const IcObs<T> &ob, int j, IcPix<T> &px) {
    const T *tp = ob.tmpl + 4 * j;
    px.tq[0] = tp[0];
    px.tq[1] = tp[1];
    px.tq[2] = tp[2];
}

// (with_template false: px.tq already holds the pixel's template record)
template <typename T>
__device__ __forceinline__ void ic_pixel_load(const ResArgs<T> &a, const IcObs<T> &ob, int j, IcPix<T> &px,
                                              bool with_template = true) {
    if (with_template) ic_pixel_template(ob, j, px);
    const double x = (ob.uc + (double)a.pat.du[j] - ob.cx) * ob.ifx;
    const double y = (ob.vc + (double)a.pat.dv[j] - ob.cy) * ob.ify;
    const double vz = ob.Q[8] * x + ob.Q[9] * y + ob.Q[10] + ob.d * ob.Q[11];
    const double hu = ob.Q[0] * x + ob.Q[1] * y + ob.Q[2] + ob.d * ob.Q[3];
    const double hv = ob.Q[4] * x + ob.Q[5] * y + ob.Q[6] + ob.d * ob.Q[7];
    const double iz = recip_nr(vz);
    const double qu = hu * iz, qv = hv * iz;
    px.ok = ((ob.m >> j) & 1u) && ob.d > 0.0 && vz > 0.0 && usable(qu, qv, a.W, a.H);
    const double su = px.ok ? qu : 1.0, sv = px.ok ? qv : 1.0;
    const double fu = floor(su), fv = floor(sv);
    const int cj = (int)fu, ci = (int)fv;
    px.fa = su - fu;
    px.fb = sv - fv;
    const T *r0 = ob.img + (size_t)ci * a.W + cj;
    px.tx[0] = r0[0];
    px.tx[1] = r0[1];
    px.tx[2] = r0[a.W];
    px.tx[3] = r0[a.W + 1];
    px.x = (T)x;
    px.y = (T)y;
}

// Second step: residual (rounded once), Huber weight, proxy Jacobian and the
// pixel's ten FP64 products, added to c (nothing when it does not contribute).
template <typename T>
__device__ __forceinline__ void ic_pixel_add(const ResArgs<T> &a, const IcObs<T> &ob, const IcPix<T> &px,
                                             double (&c)[IC_REC]) {
    if (px.ok) {
        const double If = bilerp(px.fa, px.fb, px.tx[0], px.tx[1], px.tx[2], px.tx[3]);
        const T r = (T)((double)px.tq[0] - If);
        T w, rho;
        huber(r, a.huber_k, w, rho);
        T J[7];
        ic_jacobian(px.x, px.y, ob.R0, ob.R0 + 9, ob.d0, ob.id0, px.tq[1], px.tq[2], ob.fx, ob.fy, J);
        const double wr = (double)w * r;
#pragma unroll
        for (int k = 0; k < 7; ++k) c[k] += wr * (double)J[k];
        c[7] += (double)rho;
        c[8] += (double)r * r;
        c[9] += 1.0;
    }
}

template <typename T, int NB>
__global__ __launch_bounds__(NB) void k_ic_residual(ResArgs<T> a) {
    if (__builtin_amdgcn_readfirstlane(__hip_atomic_load(a.gate, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == 0)
        return;
    const int ntiles = (a.O + NB - 1) / NB;
    for (int it = blockIdx.x; it < ntiles; it += gridDim.x) {
        const int o = xcd_tile(it, ntiles) * NB + threadIdx.x;
        if (o >= a.O) continue;
        IcObs<T> ob;
        ob.m = a.mask[o];
        double c[IC_REC] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (ob.m != 0u) {
            ic_obs_load(a, o, ob);
#pragma unroll
            for (int j0 = 0; j0 < 8; j0 += 2) {
                IcPix<T> px[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    px[i].ok = false;
                    if (j0 + i < a.P) ic_pixel_load(a, ob, j0 + i, px[i]);
                }
                ic_pixel_add(a, ob, px[0], c);
                ic_pixel_add(a, ob, px[1], c);
            }
        }
        double *rec = a.icr + (size_t)o * IC_REC;
#pragma unroll
        for (int k = 0; k < IC_REC; ++k) rec[k] = c[k];
        a.gdo[o] = c[GR_GD];
    }
}

// The same pass with one lane per patch pixel (8 lanes per observation, 8
// times the wavefronts): the pair's data (intrinsics, current pose, p(0)
// pose: 13 slices of 16 bytes in the FP32 form, 16 in FP64) and the point's
// pixel and inverse depths are loaded once per observation, lane j taking
// slices j and j + 8 (lanes 0-2 the point's), and read across the 8 lanes by
// ds_swizzle; each lane forms its pixel's products with the arithmetic
// above, and a butterfly over the 8 lanes adds them. The sums agree with the
// thread-per-observation pass to the rounding of FP64 sums of 8 terms (the
// order of the additions differs); the autotuner picks between the two.
template <typename T, int NB>
__global__ __launch_bounds__(NB) void k_ic_residual8(ResArgs<T> a) {
    if (__builtin_amdgcn_readfirstlane(__hip_atomic_load(a.gate, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == 0)
        return;
    const int ntiles = (a.O + NB / 8 - 1) / (NB / 8);
    for (int it = blockIdx.x; it < ntiles; it += gridDim.x) {
        const int gid = xcd_tile(it, ntiles) * NB + threadIdx.x;
        const int o = gid >> 3, j = gid & 7;
        const bool in = o < a.O;
        const int n = in ? a.obs_point[o] : 0, pr = in ? a.obs_pair[o] : 0;
        IcObs<T> ob;
        ob.m = in ? (unsigned)a.mask[o] : 0u;
        constexpr int NSL = 10 + (12 * (int)sizeof(T)) / 16;
        typedef int I4 __attribute__((ext_vector_type(4)));
        I4 sl0 = {0, 0, 0, 0}, sl1 = {0, 0, 0, 0};
        double pt = 0.0;
        int f = 0;
        if (ob.m != 0u) {
            auto slice = [&](int k) -> const I4 * {
                if (k < 4) return reinterpret_cast<const I4 *>(a.pcam + 8 * pr + 2 * k);
                if (k < 10) return reinterpret_cast<const I4 *>(a.geo + GEO_STRIDE * pr + 2 * (k - 4));
                return reinterpret_cast<const I4 *>(a.rel0 + REL_STRIDE * pr) + (k - 10);
            };
            sl0 = *slice(j);
            if (j + 8 < NSL) sl1 = *slice(j + 8);
            if (j < 3)
                pt = j == 0 ? *reinterpret_cast<const double *>(a.host_uv + 2 * n) : (j == 1 ? a.depth[n] : a.depth0[n]);
            f = a.pair_target[pr];
        }
        ob.tmpl = a.tmpl + 4 * (size_t)n * a.P;
        IcPix<T> px;
        px.ok = false;
        px.tq[0] = px.tq[1] = px.tq[2] = T(0);
        if (ob.m != 0u && j < a.P) ic_pixel_template(ob, j, px);
        // keep the compiler from sinking these loads into the branches below
        pin_reg(sl0);
        pin_reg(sl1);
        pin_reg(pt);
        pin_reg(f);
#pragma unroll
        for (int k = 0; k < 3; ++k) pin_reg(px.tq[k]);
        // intrinsics and current pose (words 0-39), the point's pixel and depth
        int q[40];
        bcast8_words(sl0, sl1, q, std::make_integer_sequence<int, 40>{});
        double K[8], G[12];
#pragma unroll
        for (int k = 0; k < 8; ++k) K[k] = __hiloint2double(q[2 * k + 1], q[2 * k]);
#pragma unroll
        for (int k = 0; k < 12; ++k) G[k] = __hiloint2double(q[17 + 2 * k], q[16 + 2 * k]);
        const double uv = bcast8<0>(pt), d = bcast8<1>(pt);
        const long long uvb = __double_as_longlong(uv);
        ic_obs_pair(K, G, ob);
        ob.uc = ((double)__int_as_float((int)uvb) + 0.5) * a.scale - 0.5;
        ob.vc = ((double)__int_as_float((int)(uvb >> 32)) + 0.5) * a.scale - 0.5;
        ob.d = d;
        ob.img = a.img + (size_t)f * a.W * a.H;
        if (ob.m != 0u && j < a.P) ic_pixel_load(a, ob, j, px, false);
        // the p(0) pose (slices 10 and up, all in sl1) only now, so that it
        // is not held in registers across the loads
        pin_reg(sl1);
        constexpr int NR0 = 12 * (int)sizeof(T) / 4;
        int q0[NR0];
        bcast8_words_from<40>(sl1, q0, std::make_integer_sequence<int, NR0>{});
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            if constexpr (sizeof(T) == 8)
                ob.R0[k] = (T)__hiloint2double(q0[2 * k + 1], q0[2 * k]);
            else
                ob.R0[k] = (T)__int_as_float(q0[k]);
        }
        ob.d0 = (T)bcast8<2>(pt);
        ob.id0 = recip(ob.d0);
        double p[IC_REC] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        ic_pixel_add(a, ob, px, p);
#pragma unroll
        for (int k = 0; k < IC_REC; ++k) {
            pin_reg(p[k]);   // every lane of the group ends with the same sum
            p[k] = wave_sum8(p[k]);
        }
        double v0 = p[0];
#pragma unroll
        for (int k = 1; k < 8; ++k) v0 = j == k ? p[k] : v0;
        const double v1 = j == 0 ? p[8] : p[9];
        if (in) {
            double *rec = a.icr + (size_t)o * IC_REC;
            rec[j] = v0;
            if (j < 2) rec[8 + j] = v1;
            if (j == GR_GD) a.gdo[o] = v0;
        }
    }
}


// Energy and RMSE at the current parameters over the residuals usable at those
// parameters (fresh set); writes the record's statistics fields only.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_evaluate(ResArgs<T> a) {
    const int gid = blockIdx.x * BLOCK + threadIdx.x;
    const int o = gid >> 3, j = gid & 7;
    T c[3] = {0, 0, 0};
    if (o < a.O && j < a.P) {
        const int n = a.obs_point[o], pr = a.obs_pair[o];
        const int f = a.pair_target[pr];
        const double *Kh = a.pcam + 8 * pr, *Kt = Kh + 4;
        const T *tp = a.tmpl + 4 * ((size_t)n * a.P + j);
        double x, y;
        template_xy(a, n, j, Kh, x, y);
        const double *R = a.geo + GEO_STRIDE * pr;
        const double *t = R + 9;
        const double d = a.depth[n];
        const double vz = R[6] * x + R[7] * y + R[8] + d * t[2];
        if (tp[3] != T(0) && a.live[o] && d > 0.0 && vz > 0.0) {
            const double vx = R[0] * x + R[1] * y + R[2] + d * t[0];
            const double vy = R[3] * x + R[4] * y + R[5] + d * t[1];
            const double iz = 1.0 / vz;
            const double qu = Kt[0] * (vx * iz) + Kt[2], qv = Kt[1] * (vy * iz) + Kt[3];
            if (usable(qu, qv, a.W, a.H)) {
                const T r = (T)((double)tp[0] - bilinear(a.img + (size_t)f * a.W * a.H, a.W, qu, qv));
                T w, rho;
                huber(r, a.huber_k, w, rho);
                c[0] = rho;
                c[1] = r * r;
                c[2] = T(1);
            }
        }
    }
    for (int p = 0; p < 3; ++p) c[p] = wave_sum8(c[p]);
    if (j == 0 && o < a.O) {
        double *rec = a.rec + (size_t)o * REC_STRIDE;
        rec[REC_E] = c[0];
        rec[REC_SQ] = c[1];
        rec[REC_CNT] = c[2];
    }
}

// End-of-iteration statistics and the convergence gate (see k_conv).
struct ConvArgs {
    const double *wstat;
    int nwin;
    double *stat;
    double conv_px;
    int *gate, *count;
    const int *flag;
    const int *count_base;   // iterations before the last re-centring of the level
};

// Statistics of an iteration from the block maxima (largest point-centre
// displacement, largest depth step) and the per-window statistics of the solve,
// added over the windows in order; closes the gate once the displacement is
// below conv_px (conv_px >= 0). One block; md / ms are its thread-0 maxima.
__device__ void conv_finish(const ConvArgs &cv, double md, double ms) {
    if (*cv.flag) {
        *cv.gate = 0;
        return;
    }
    double e = 0.0, sq = 0.0, cnt = 0.0, sp = 0.0;
    for (int w = 0; w < cv.nwin; ++w) {
        e += cv.wstat[4 * w];
        sq += cv.wstat[4 * w + 1];
        cnt += cv.wstat[4 * w + 2];
        sp = fmax(sp, cv.wstat[4 * w + 3]);
    }
    cv.stat[ST_E] = e;
    cv.stat[ST_SQ] = sq;
    cv.stat[ST_CNT] = cnt;
    cv.stat[ST_STEP_P] = sp;
    cv.stat[ST_DISP] = md;
    cv.stat[ST_STEP_D] = ms;
    *cv.count += 1;
    if (cv.conv_px >= 0.0 && md < cv.conv_px) *cv.gate = 0;
}

// Block maxima of the pairs (part[2 i], part[2 i + 1]), i < nparts; valid in thread 0.
__device__ void block_max2(const double *part, int nparts, double &md, double &ms, double (*red)[16]) {
    md = 0.0;
    ms = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
        md = fmax(md, part[2 * i]);
        ms = fmax(ms, part[2 * i + 1]);
    }
    md = wave_max(md);
    ms = wave_max(ms);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = md;
        red[1][threadIdx.x >> 6] = ms;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        // the (non-negative) wavefront maxima over the lanes of row 0
        const int l = threadIdx.x, nw = blockDim.x >> 6;
        md = row_max16(l < nw ? red[0][l] : 0.0);
        ms = row_max16(l < nw ? red[1][l] : 0.0);
    }
}

// ------------------------------------------------------------ reductions

// Block-wide sum of NV doubles per thread (up to 16 wavefronts) in a fixed
// order: a butterfly in every wavefront, then one over the wavefront partials
// in wavefront 0. Result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double v[NV], double *lds /* [NV * 16] */) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int p = 0; p < NV; ++p)
        v[p] = wave_sum(v[p]);
    if (lane == 0)
        for (int p = 0; p < NV; ++p) lds[wv * NV + p] = v[p];
    __syncthreads();
    if (wv == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int p = 0; p < NV; ++p) v[p] = row_sum16(lane < nw ? lds[lane * NV + p] : 0.0);
    }
    __syncthreads();
}

// Per point: sum of the depth blocks over the point's observations.
template <typename T>
__global__ __launch_bounds__(256) void k_point_reduce(int N, const int *__restrict__ obs_ptr,
                                                      const double *__restrict__ rec, double *__restrict__ Hdd,
                                                      double *__restrict__ gd, int with_hdd,
                                                      const int *__restrict__ gate) {
    if (*gate == 0) return;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    double hs = 0.0, gs = 0.0;
    if (n < N) {
        const int o0 = obs_ptr[n], o1 = obs_ptr[n + 1];
#pragma unroll 4
        for (int o = o0; o < o1; ++o) {
            const double *r = rec + (size_t)o * REC_STRIDE;
            hs += r[REC_HDD];
            gs += (double)r[REC_GD];
        }
        gd[n] = gs;
        if (with_hdd) Hdd[n] = hs;
    }
}

// Per chunk of one pair's observations (at most PAIR_CHUNK, one per thread):
// sum of the pose-pose block (21 values). Chunk partials are added per pair in
// chunk order by the consumer. slot: per thread of each chunk (observation,
// point, the point's observation range), observation -1 past the chunk's end.
template <typename T>
__global__ __launch_bounds__(PAIR_CHUNK) void k_pair_chunk_H(const int4 *__restrict__ slot, const double *__restrict__ rec,
                                                      double *__restrict__ partH, const int *__restrict__ gate) {
    __shared__ double lds[21 * 16];
    if (*gate == 0) return;
    const int c = blockIdx.x;
    const int o = slot[(size_t)c * PAIR_CHUNK + threadIdx.x].x;
    double v[21];
    for (int k = 0; k < 21; ++k) v[k] = 0.0;
    if (o >= 0) {
        const double *r = rec + (size_t)o * REC_STRIDE;
        for (int k = 0; k < 21; ++k) v[k] += r[REC_H + k];
    }
    block_sum<21>(v, lds);
    if (threadIdx.x == 0)
        for (int k = 0; k < 21; ++k) partH[21 * c + k] = v[k];
}

// Per chunk of one pair's observations (at most PAIR_CHUNK, one per thread):
// reduced right-hand side contribution sum_o (g_o - h_o g_d,n / H_dd,n) (depth
// elimination of the gradient) and the energy statistics. gr / gs: gradient
// records (GR_* fields) and their stride; gd / gds: g_d of every observation
// and its stride; hc: h_o, 6 values per observation.
template <typename T>
__global__ __launch_bounds__(PAIR_CHUNK) void k_pair_chunk_y(const int4 *__restrict__ slot, const double *__restrict__ hc,
                                                             const double *__restrict__ gr, int gs,
                                                             const double *__restrict__ gd, int gds,
                                                             const double *__restrict__ Hdd,
                                                             double *__restrict__ partY, const int *__restrict__ gate,
                                                             const double *__restrict__ du_part, int du_nparts,
                                                             ConvArgs cv) {
    __shared__ double lds[9 * 16];
    __shared__ double red[2][16];
    const int c = blockIdx.x;
    // the thread's slot and the gate (a vector load) in one memory step; a
    // closed gate leaves every sum zero (the sums are then not used), so that
    // all waves of the block reach its barriers
    const int4 sd = slot[(size_t)c * PAIR_CHUNK + threadIdx.x];
    const bool live = __builtin_amdgcn_readfirstlane(
                          __hip_atomic_load(gate, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0;
    // block 0 also ends the previous iteration (IC): the depth update's block
    // maxima (loaded now, reduced after the pair sums) give its largest
    // displacement and depth step, its statistics and the convergence gate. If
    // that closes the gate, this iteration's sums are simply not used. Only
    // block 0 writes the gate, after all its waves have read it.
    const bool finish_prev = du_part != nullptr && blockIdx.x == 0 && live;
    double pmd = 0.0, pms = 0.0;
    if (finish_prev)
        for (int i = threadIdx.x; i < du_nparts; i += blockDim.x) {
            pmd = fmax(pmd, du_part[2 * i]);
            pms = fmax(pms, du_part[2 * i + 1]);
        }
    double v[9];
    for (int k = 0; k < 9; ++k) v[k] = 0.0;
    if (live && sd.x >= 0) {
        const int o = sd.x, n = sd.y, q0 = sd.z, q1 = sd.w;
        const double2 *h2 = reinterpret_cast<const double2 *>(hc + 6 * (size_t)o);
        const double *g = gr + (size_t)o * gs;
        double gdn = 0.0;  // g_d,n: the point's records in order (bitwise the per-point sum)
#pragma unroll 4
        for (int q = q0; q < q1; ++q) gdn += gd[(size_t)q * gds];
        const double s = gdn / Hdd[n];
        for (int k = 0; k < 3; ++k) {
            const double2 hk = h2[k];
            v[2 * k] += (double)g[GR_G + 2 * k] - hk.x * s;
            v[2 * k + 1] += (double)g[GR_G + 2 * k + 1] - hk.y * s;
        }
        v[6] += (double)g[GR_E];
        v[7] += (double)g[GR_SQ];
        v[8] += (double)g[GR_CNT];
    }
    block_sum<9>(v, lds);
    if (threadIdx.x == 0 && live)
        for (int k = 0; k < 9; ++k) partY[9 * c + k] = v[k];
    if (finish_prev) {
        pmd = wave_max(pmd);
        pms = wave_max(pms);
        if ((threadIdx.x & 63) == 0) {
            red[0][threadIdx.x >> 6] = pmd;
            red[1][threadIdx.x >> 6] = pms;
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            const int l = threadIdx.x, nw = blockDim.x >> 6;
            pmd = row_max16(l < nw ? red[0][l] : 0.0);
            pms = row_max16(l < nw ? red[1][l] : 0.0);
            if (l == 0) conv_finish(cv, pmd, pms);
        }
    }
}

// Sums of the record statistics (energy, squared residuals, count): block
// partials over SUM_OBS observations each, then one block adds them in order.
constexpr int SUM_OBS = 2048;

template <typename T>
__global__ __launch_bounds__(256) void k_sum_stats(int O, const T *__restrict__ rec, double *__restrict__ part) {
    __shared__ double lds[3 * 16];
    double v[3] = {0.0, 0.0, 0.0};
    const int o1 = min(O, (blockIdx.x + 1) * SUM_OBS);
    for (int o = blockIdx.x * SUM_OBS + threadIdx.x; o < o1; o += blockDim.x) {
        const T *r = rec + (size_t)o * REC_STRIDE;
        v[0] += (double)r[REC_E];
        v[1] += (double)r[REC_SQ];
        v[2] += (double)r[REC_CNT];
    }
    block_sum<3>(v, lds);
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) part[3 * blockIdx.x + k] = v[k];
}

__global__ void k_sum_parts3(int np, const double *__restrict__ part, double *__restrict__ out) {
    if (threadIdx.x >= 3) return;
    double s = 0.0;
    for (int b = 0; b < np; ++b) s += part[3 * b + threadIdx.x];
    out[threadIdx.x] = s;
}

// Depth step of every point after the pose step and the block maxima of the
// point-centre displacement and of the depth step (k_conv finishes the
// iteration from them); DU_PTS points per block.
template <typename T>
__global__ __launch_bounds__(256) void k_depth_update(
    int N, int ic, const int *__restrict__ obs_ptr, const int *__restrict__ obs_pair,
    const float *__restrict__ host_uv, const double *__restrict__ pairK0, const double *__restrict__ hc,
    const double *__restrict__ gd, int gds, const double *__restrict__ Hdd, const double *__restrict__ dth_rel,
    const double *__restrict__ geo_old, const double *__restrict__ geo_new, double *__restrict__ depth,
    const double *__restrict__ depth0, double *__restrict__ part, const int *__restrict__ gate,
    const int *__restrict__ flag, const uint8_t *__restrict__ live) {
    __shared__ double lds[depth_lds_doubles(256)];
    double md = 0.0, ms = 0.0;
    const int n0 = blockIdx.x * DU_PTS;
    const DepthPoint pt = depth_point<false>(N, n0, obs_ptr, host_uv, Hdd, depth, depth0);
    if (!depth_points<T, 256>(N, n0, ic, pt, obs_pair, pairK0, hc, gd, gds, dth_rel, geo_old, geo_new, depth, gate,
                              flag, lds, md, ms, live))
        return;
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = md;
        part[2 * blockIdx.x + 1] = ms;
    }
}

// ------------------------------------------------------------ launchers

static inline unsigned nblk(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

template <typename T>
static ResArgs<T> res_args(Ctx &c, int level, const double *geo_cur) {
    ResArgs<T> a{};
    a.O = c.O;
    a.P = c.P;
    a.W = c.lv[level].W;
    a.H = c.lv[level].H;
    a.pat.n = c.cfg.pattern_n;
    for (int j = 0; j < 8; ++j) {
        a.pat.du[j] = j < c.cfg.pattern_n ? c.cfg.pattern_uv[2 * j] : 0;
        a.pat.dv[j] = j < c.cfg.pattern_n ? c.cfg.pattern_uv[2 * j + 1] : 0;
    }
    a.scale = 1.0 / (double)(1 << level);
    a.huber_k = (T)c.cfg.huber_k;
    a.obs_point = c.d_obs_point;
    a.obs_pair = c.d_obs_pair;
    a.pair_host = c.d_pair_host;
    a.pair_target = c.d_pair_target;
    a.host_uv = c.d_host_uv;
    a.img = (const T *)c.lv[level].img;
    a.tmpl = (const T *)c.lv[level].tmpl;
    a.geo = geo_cur;
    a.rel0 = (const T *)c.d_rel0;
    a.depth = c.d_depth;
    a.depth0 = c.d_depth0;
    a.mask = c.d_mask;
    a.live = c.d_obs_live;
    a.rec = (double *)c.d_rec;
    a.pcam = (const double *)c.lv[level].pcam;
    a.icr = (double *)c.d_icr;
    a.gdo = c.d_gdo;
    a.gate = c.d_gate;
    return a;
}

static ConvArgs conv_args(Ctx &c, double *stat, double conv_px, int level) {
    return ConvArgs{c.d_wstat, c.nwin, stat, conv_px, c.d_gate, c.d_count + level, c.d_flag, c.d_count_base + level};
}

// Gradient records of the current iteration: the compact IC records or the
// G .. CNT fields of the full record (FC).
template <typename T>
static void grad_records(const Ctx &c, const double *&gr, int &gs) {
    if (c.cfg.mode == PBA_IC_PROXY) {
        gr = (const double *)c.d_icr;
        gs = IC_REC;
    } else {
        gr = (const double *)c.d_rec + REC_G;
        gs = REC_STRIDE;
    }
}

// g_d of every observation of the current iteration and its stride: the
// contiguous copy the IC residual pass writes, or the full record's field (FC).
static void grad_gd(const Ctx &c, const double *&gd, int &gds) {
    if (c.cfg.mode == PBA_IC_PROXY) {
        gd = c.d_gdo;
        gds = 1;
    } else {
        gd = (const double *)c.d_rec + REC_GD;
        gds = REC_STRIDE;
    }
}

template <typename T>
void Launch<T>::convert_images(hipStream_t s, const float *src, T *dst, size_t n) {
    k_convert<T><<<nblk(n, 256), 256, 0, s>>>(src, dst, n);
    CHECK_LAUNCH();
}

template <typename T>
void Launch<T>::downsample(hipStream_t s, const T *src, T *dst, int F, int Ws, int Hs, int Wd, int Hd) {
    k_downsample<T><<<nblk((size_t)F * Wd * Hd, 256), 256, 0, s>>>(src, dst, F, Ws, Hs, Wd, Hd);
    CHECK_LAUNCH();
}

template <typename T>
void Launch<T>::level_K(hipStream_t s, const double *K0, T *K, int F, int level) {
    k_level_K<T><<<nblk(F, 64), 64, 0, s>>>(K0, K, F, level);
    CHECK_LAUNCH();
}

template <typename T>
void Launch<T>::make_template(hipStream_t s, Ctx &c, int level) {
    ResArgs<T> a = res_args<T>(c, level, nullptr);
    const size_t n = (size_t)c.N * c.P;
    if (n == 0) return;
    k_template<T><<<nblk(n, 256), 256, 0, s>>>(c.N, c.P, a.pat, c.d_host_uv, c.d_host_frame, a.img, a.W, a.H,
                                               (T)a.scale, (T *)c.lv[level].tmpl);
    CHECK_LAUNCH();
    if (c.st.n_pairs > 0) {
        k_pair_cam<<<nblk((size_t)c.st.n_pairs * 8, 256), 256, 0, s>>>(c.st.n_pairs, c.d_pair_host,
                                                                      c.d_pair_target, c.d_K0, level,
                                                                      (double *)c.lv[level].pcam);
        CHECK_LAUNCH();
    }
}

template <typename T>
void Launch<T>::level_begin(hipStream_t s, Ctx &c, int level, bool clear_flag, bool recentre) {
    const int m = std::max(std::max(12 * c.F, c.N), std::max(c.st.n_pairs, 1));
    k_level_begin<T><<<nblk(m, 256), 256, 0, s>>>(c.F, c.N, c.st.n_pairs, c.d_poses, c.d_poses0, c.d_depth,
                                                  c.d_depth0, c.d_pair_host, c.d_pair_target, c.d_geo0,
                                                  (T *)c.d_rel0, c.d_geo_a, (T *)c.d_rel_a, c.d_gate, c.d_flag,
                                                  c.d_count + level, c.d_count_base + level, clear_flag ? 1 : 0,
                                                  recentre ? 1 : 0);
    CHECK_LAUNCH();
}

template <typename T>
void Launch<T>::relpose(hipStream_t s, Ctx &c, const double *poses, double *geo, T *rel) {
    if (c.st.n_pairs == 0) return;
    k_relpose<T><<<nblk(c.st.n_pairs, 64), 64, 0, s>>>(c.st.n_pairs, c.d_pair_host, c.d_pair_target, poses, geo,
                                                       rel);
    CHECK_LAUNCH();
}

// Launch, with the start and end of the kernel recorded into e0 / e1 by the
// dispatch itself when they are given (timing of the kernel alone).
template <typename K, typename... A>
static void launch_ev(K kernel, unsigned g, unsigned b, hipStream_t s, hipEvent_t e0, hipEvent_t e1, A... args) {
    if (e0 || e1)
        hipExtLaunchKernelGGL(kernel, dim3(g), dim3(b), 0, s, e0, e1, 0, args...);
    else
        hipLaunchKernelGGL(kernel, dim3(g), dim3(b), 0, s, args...);
}

// Grid of a launch shape: one tile of nb / 8 observations per workgroup, or a
// persistent grid of grid_mult workgroups per compute unit striding over them.
static unsigned shape_grid(const Ctx &c, LaunchShape sh, int lanes_per_obs = LANES_PER_OBS) {
    const size_t tiles = ((size_t)c.O * lanes_per_obs + sh.block - 1) / sh.block;
    if (sh.grid_mult <= 0) return (unsigned)tiles;
    return (unsigned)std::min<size_t>(tiles, (size_t)sh.grid_mult * c.n_cu);
}

template <typename T, bool IC>
static void launch_linearize_shape(hipStream_t s, const Ctx &c, const ResArgs<T> &a, int write_mask, LaunchShape sh,
                                   hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
    const unsigned g = shape_grid(c, sh);
    switch (sh.block) {
        case 64: launch_ev(k_linearize<T, IC, 64>, g, 64, s, e0, e1, a, write_mask); break;
        case 128: launch_ev(k_linearize<T, IC, 128>, g, 128, s, e0, e1, a, write_mask); break;
        case 512: launch_ev(k_linearize<T, IC, 512>, g, 512, s, e0, e1, a, write_mask); break;
        default: launch_ev(k_linearize<T, IC, 256>, g, 256, s, e0, e1, a, write_mask); break;
    }
}

template <typename T>
void Launch<T>::ic_linearize(hipStream_t s, Ctx &c, int level) {
    if (c.O == 0) return;
    // at p(0): the poses and the inverse depths of the level's linearization
    ResArgs<T> a = res_args<T>(c, level, c.d_geo0);
    a.depth = c.d_depth0;
    launch_linearize_shape<T, true>(s, c, a, 1, LaunchShape{});
    CHECK_LAUNCH();
}

template <typename T>
void Launch<T>::fc_linearize(hipStream_t s, Ctx &c, int level, const double *geo_cur, bool write_mask,
                             hipEvent_t e0, hipEvent_t e1) {
    if (c.O == 0) return;
    ResArgs<T> a = res_args<T>(c, level, geo_cur);
    launch_linearize_shape<T, false>(s, c, a, write_mask ? 1 : 0, c.tune_lin, e0, e1);
    CHECK_LAUNCH();
}

void launch_linearize_mixed(hipStream_t s, Ctx &c, int level, bool ic, const double *geo_cur, bool write_mask,
                            hipEvent_t e0, hipEvent_t e1) {
    const int nch = (int)c.st.pchunk_begin.size();
    if (c.O == 0 || nch == 0) return;
    ResArgs<float> a = res_args<float>(c, level, geo_cur);
    if (ic) a.depth = c.d_depth0;   // IC linearizes at p(0)
    if (ic)
        launch_ev(k_linearize_mixed<true>, nch, BLOCK, s, e0, e1, a, 1, (const int *)c.d_pchunk_begin,
                  (const int *)c.d_pchunk_end, (const int *)c.d_pair_obs_idx, c.d_partH);
    else
        launch_ev(k_linearize_mixed<false>, nch, BLOCK, s, e0, e1, a, write_mask ? 1 : 0,
                  (const int *)c.d_pchunk_begin, (const int *)c.d_pchunk_end, (const int *)c.d_pair_obs_idx,
                  c.d_partH);
    CHECK_LAUNCH();
}

template <typename T>
void Launch<T>::ic_residual(hipStream_t s, Ctx &c, int level, const double *geo_cur, hipEvent_t e0, hipEvent_t e1) {
    ic_residual_shape(s, c, level, geo_cur, c.tune_res, e0, e1);
}

template <typename T>
void Launch<T>::ic_residual_shape(hipStream_t s, Ctx &c, int level, const double *geo_cur, LaunchShape sh,
                                  hipEvent_t e0, hipEvent_t e1) {
    if (c.O == 0) return;
    ResArgs<T> a = res_args<T>(c, level, geo_cur);
    const unsigned g = shape_grid(c, sh, sh.lanes == 8 ? 8 : 1);
    if (sh.lanes == 8) {
        switch (sh.block) {
            case 128: launch_ev(k_ic_residual8<T, 128>, g, 128, s, e0, e1, a); break;
            case 512: launch_ev(k_ic_residual8<T, 512>, g, 512, s, e0, e1, a); break;
            default: launch_ev(k_ic_residual8<T, 256>, g, 256, s, e0, e1, a); break;
        }
    } else {
        switch (sh.block) {
            case 64: launch_ev(k_ic_residual<T, 64>, g, 64, s, e0, e1, a); break;
            case 128: launch_ev(k_ic_residual<T, 128>, g, 128, s, e0, e1, a); break;
            case 512: launch_ev(k_ic_residual<T, 512>, g, 512, s, e0, e1, a); break;
            case 1024: launch_ev(k_ic_residual<T, 1024>, g, 1024, s, e0, e1, a); break;
            default: launch_ev(k_ic_residual<T, 256>, g, 256, s, e0, e1, a); break;
        }
    }
    CHECK_LAUNCH();
}

template <typename T>
void Launch<T>::fc_linearize_shape(hipStream_t s, Ctx &c, int level, const double *geo_cur, LaunchShape sh) {
    if (c.O == 0) return;
    ResArgs<T> a = res_args<T>(c, level, geo_cur);
    launch_linearize_shape<T, false>(s, c, a, 1, sh);
    CHECK_LAUNCH();
}

template <typename T>
void Launch<T>::evaluate(hipStream_t s, Ctx &c, int level) {
    if (c.O == 0) return;
    ResArgs<T> a = res_args<T>(c, level, c.flip ? c.d_geo_b : c.d_geo_a);
    k_evaluate<T><<<nblk((size_t)c.O * LANES_PER_OBS, BLOCK), BLOCK, 0, s>>>(a);
    CHECK_LAUNCH();
}

template <typename T>
void Launch<T>::point_reduce(hipStream_t s, Ctx &c, bool with_hdd) {
    if (c.N == 0) return;
    k_point_reduce<T><<<nblk(c.N, 256), 256, 0, s>>>(c.N, c.d_obs_ptr, (const double *)c.d_rec, c.d_Hdd, c.d_gd,
                                                     with_hdd ? 1 : 0, c.d_gate);
    CHECK_LAUNCH();
}

template <typename T>
void Launch<T>::pair_reduce_H(hipStream_t s, Ctx &c) {
    const int nch = (int)c.st.pchunk_begin.size();
    if (nch == 0) return;
    k_pair_chunk_H<T><<<nch, PAIR_CHUNK, 0, s>>>((const int4 *)c.d_pc_slot, (const double *)c.d_rec, c.d_partH, c.d_gate);
    CHECK_LAUNCH();
}

template <typename T>
void Launch<T>::pair_reduce_y(hipStream_t s, Ctx &c, double *prev_stat, double conv_px, int level) {
    const int nch = (int)c.st.pchunk_begin.size();
    if (nch == 0) {
        // no pair chunks to carry the previous iteration's end: its own kernel
        if (prev_stat) launch_conv(s, c, prev_stat, conv_px, du_nparts(c), level);
        return;
    }
    const double *gr;
    int gs;
    grad_records<T>(c, gr, gs);
    const double *gd;
    int gds;
    grad_gd(c, gd, gds);
    k_pair_chunk_y<T><<<nch, PAIR_CHUNK, 0, s>>>((const int4 *)c.d_pc_slot, c.d_hc, gr, gs, gd, gds, c.d_Hdd,
                                                 c.d_partY, c.d_gate, prev_stat ? c.d_du_part : nullptr,
                                                 du_nparts(c), conv_args(c, prev_stat, conv_px, level));
    CHECK_LAUNCH();
}


template <typename T>
void Launch<T>::depth_update(hipStream_t s, Ctx &c, const double *geo_old, const double *geo_new, double *stat,
                             double conv_px, int level, bool finish) {
    const int nb = (int)nblk(c.N, DU_PTS);
    const double *gd;
    int gds;
    grad_gd(c, gd, gds);
    if (c.N > 0)
        k_depth_update<T><<<nb, 256, 0, s>>>(c.N, c.cfg.mode == PBA_IC_PROXY ? 1 : 0, c.d_obs_ptr, c.d_obs_pair,
                                             c.d_host_uv, c.d_pairK0, c.d_hc, gd, gds, c.d_Hdd,
                                             c.d_dth_rel, geo_old, geo_new, c.d_depth, c.d_depth0, c.d_du_part,
                                             c.d_gate, c.d_flag, c.d_obs_live);
    CHECK_LAUNCH();
    if (finish) launch_conv(s, c, stat, conv_px, du_nparts(c), level);
}

// End of an iteration without points (single block): the iteration
// statistics and the convergence gate from nparts block maxima.
// With np > 0 (the fused IC step, which alternates two pose buffers: iteration
// k of a batch reads buffer k mod 2), the poses are then copied back from
// pose_alt when the batch ran an odd number of iterations; this runs whether or
// not the gate is open.
__global__ __launch_bounds__(256) void k_conv(const double *__restrict__ part, int nparts, ConvArgs cv,
                                              const double *__restrict__ pose_alt, double *__restrict__ pose,
                                              int np) {
    __shared__ double red[2][16];
    __shared__ int ran;
    if (*cv.gate != 0) {
        double md, ms;
        block_max2(part, nparts, md, ms, red);
        if (threadIdx.x == 0) conv_finish(cv, md, ms);
    }
    if (np == 0) return;
    __syncthreads();
    if (threadIdx.x == 0) ran = *cv.count - *cv.count_base;
    __syncthreads();
    if (ran & 1)
        for (int e = threadIdx.x; e < np; e += blockDim.x) pose[e] = pose_alt[e];
}

// Start of a batch of iterations: clear the level's iteration count and
// (clear_flag) the failure flag, and open the gate unless a failure is flagged
// (a kernel, so that it can be captured in a graph).
__global__ void k_open(int *__restrict__ gate, int *__restrict__ flag, int *__restrict__ count,
                       int *__restrict__ count_base, int clear_flag) {
    if (threadIdx.x == 0) {
        if (clear_flag) *flag = 0;
        *gate = *flag == 0 ? 1 : 0;
        *count = 0;
        *count_base = 0;
    }
}

// Keyframe drop (sliding window): every observation of a point hosted by
// frame f or with target f leaves the window: its live flag and frozen
// pixels are cleared and its record zeroed, so that sums over the records
// (pair blocks, h, H_dd, the gradient) no longer see it.
__global__ void k_drop_frame(int O, int f, const int *__restrict__ obs_pair, const int *__restrict__ pair_host,
                             const int *__restrict__ pair_target, uint8_t *__restrict__ live,
                             uint8_t *__restrict__ mask, double *__restrict__ rec) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= O) return;
    const int p = obs_pair[o];
    if (pair_host[p] != f && pair_target[p] != f) return;
    live[o] = 0;
    mask[o] = 0;
    double *r = rec + (size_t)o * REC_STRIDE;
    for (int k = 0; k < REC_STRIDE; ++k) r[k] = 0.0;
}

void launch_drop_frame(hipStream_t s, Ctx &c, int frame) {
    if (c.O == 0) return;
    k_drop_frame<<<nblk(c.O, 256), 256, 0, s>>>(c.O, frame, c.d_obs_pair, c.d_pair_host, c.d_pair_target,
                                                c.d_obs_live, c.d_mask, (double *)c.d_rec);
    CHECK_LAUNCH();
}

void launch_conv(hipStream_t s, Ctx &c, double *stat, double conv_px, int nparts, int level, bool pose_sync) {
    k_conv<<<1, 256, 0, s>>>(c.d_du_part, nparts, conv_args(c, stat, conv_px, level), c.d_poses_alt, c.d_poses,
                             pose_sync ? 12 * c.F : 0);
    CHECK_LAUNCH();
}

void launch_open(hipStream_t s, Ctx &c, int level, bool clear_flag) {
    k_open<<<1, 64, 0, s>>>(c.d_gate, c.d_flag, c.d_count + level, c.d_count_base + level, clear_flag ? 1 : 0);
    CHECK_LAUNCH();
}

void launch_sum_stats(hipStream_t s, Ctx &c, const void *rec, bool rec_double, double *out3) {
    // out3 has room for the block partials after the three sums (see sum_stats_doubles)
    const int np = (c.O + SUM_OBS - 1) / SUM_OBS;
    if (rec_double)
        k_sum_stats<double><<<np, 256, 0, s>>>(c.O, (const double *)rec, out3 + 3);
    else
        k_sum_stats<float><<<np, 256, 0, s>>>(c.O, (const float *)rec, out3 + 3);
    k_sum_parts3<<<1, 64, 0, s>>>(np, out3 + 3, out3);
    CHECK_LAUNCH();
}

size_t sum_stats_doubles(const Ctx &c) { return 3 + 3 * (size_t)((c.O + SUM_OBS - 1) / SUM_OBS); }

template struct Launch<float>;
template struct Launch<double>;

}  // namespace pba
