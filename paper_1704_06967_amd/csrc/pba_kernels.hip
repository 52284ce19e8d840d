// HIP kernels of libpba for CDNA4 (gfx950, wave64).
//
// Residual-level kernels put one observation (point n seen in frame f) on 8
// consecutive lanes, one lane per patch pixel, 8 observations per wavefront.
// Each observation reduces its lanes with cross-lane DPP moves and writes one
// record of Gauss-Newton blocks in relative-pose coordinates. Every later
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

// Level intrinsics of every pair's host and target frames, side by side, so
// that a residual reads its camera data with its pair index alone.
template <typename T>
__global__ void k_pair_cam(int Pn, const int *__restrict__ pair_host, const int *__restrict__ pair_target,
                           const T *__restrict__ K, T *__restrict__ pcam) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= Pn * 8) return;
    const int p = e >> 3, k = e & 7;
    const int f = k < 4 ? pair_host[p] : pair_target[p];
    pcam[e] = K[4 * f + (k & 3)];
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
        bilinear_grad(img + (size_t)host_frame[n] * W * H, W, u, v, I, gu, gv);
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
// (geo0, rel0) and as the current iterate (geo_a, rel_a).
template <typename T>
__global__ void k_level_begin(int F, int N, int Pn, const double *__restrict__ poses, double *__restrict__ poses0,
                              const double *__restrict__ depth, double *__restrict__ depth0,
                              const int *__restrict__ pair_host, const int *__restrict__ pair_target,
                              double *__restrict__ geo0, T *__restrict__ rel0, double *__restrict__ geo_a,
                              T *__restrict__ rel_a, int *__restrict__ gate, int *__restrict__ flag,
                              int *__restrict__ count, int clear_flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        if (clear_flag) *flag = 0;
        *gate = *flag == 0 ? 1 : 0;
        *count = 0;
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
    T scale;             // 1 / 2^level
    T huber_k;
    const int *obs_point, *obs_pair, *pair_host, *pair_target;
    const float *host_uv;
    const T *img;        // level image stack
    const T *K;          // level intrinsics [F][4]
    const T *tmpl;       // [N][P][4]
    const T *rel;        // current relative poses
    const T *rel0;       // relative poses at p(0) (IC)
    const double *depth, *depth0;
    uint8_t *mask;
    T *rec;
    const T *pcam;       // per pair: host and target level intrinsics (fx, fy, cx, cy) x 2
    T *icr;              // IC iterations: per observation g (6), g_d, energy, sum r^2, count
    const int *gate;     // device flag: 0 = the solve has converged, skip the work
};

// Normalized template coordinates of patch pixel j of point n (host intrinsics).
template <typename T>
__device__ __forceinline__ void template_xy(const ResArgs<T> &a, int n, int j, const T *Kh, T &x, T &y) {
    const T u = ((T)a.host_uv[2 * n] + T(0.5)) * a.scale - T(0.5) + (T)a.pat.du[j];
    const T v = ((T)a.host_uv[2 * n + 1] + T(0.5)) * a.scale - T(0.5) + (T)a.pat.dv[j];
    x = (u - Kh[2]) / Kh[0];
    y = (v - Kh[3]) / Kh[1];
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
    const T *Kh = a.pcam + 8 * pr;   // the pair's host and target intrinsics (one load step fewer than K[frame])
    const T *Kt = Kh + 4;
    const T *tp = a.tmpl + 4 * ((size_t)n * a.P + j);
    const T I0 = tp[0], gu0 = tp[1], gv0 = tp[2];
    const bool host_ok = tp[3] != T(0);
    bool frozen = true;
    if (!write_mask) frozen = (a.mask[o] >> j) & 1;
    T x, y;
    template_xy(a, n, j, Kh, x, y);
    const T *R = a.rel + REL_STRIDE * pr;
    const T *t = R + 9;
    const T d = (T)a.depth[n];
    const T Rx0 = R[0] * x + R[1] * y + R[2];
    const T Rx1 = R[3] * x + R[4] * y + R[5];
    const T Rx2 = R[6] * x + R[7] * y + R[8];
    const T vx = Rx0 + d * t[0], vy = Rx1 + d * t[1], vz = Rx2 + d * t[2];
    if (!(host_ok && frozen && d > T(0) && vz > T(0))) return false;
    const T ux = vx / vz, uy = vy / vz;
    const T qu = Kt[0] * ux + Kt[2], qv = Kt[1] * uy + Kt[3];
    if (!usable(qu, qv, a.W, a.H)) return false;
    const T *imf = a.img + (size_t)f * a.W * a.H;
    T If, gu, gv;
    if (IC) {
        If = bilinear(imf, a.W, qu, qv);
        const T *R0 = a.rel0 + REL_STRIDE * pr;
        ic_jacobian(x, y, R0, R0 + 9, (T)a.depth0[n], gu0, gv0, Kh[0], Kh[1], J);
    } else {
        bilinear_grad(imf, a.W, qu, qv, If, gu, gv);
        fc_jacobian(Rx0, Rx1, Rx2, vz, ux, uy, t, d, gu, gv, Kt[0], Kt[1], J);
    }
    r = I0 - If;
    huber(r, a.huber_k, w, rho);
    return true;
}

// Linearization in observation order: the 38-value record of every
// observation (lane j == 0 writes it). NB threads per workgroup (NB / 8
// observations per tile); the grid strides over the tiles, so that it can be
// launched one tile per workgroup or as a persistent grid.
template <typename T, bool IC, int NB>
__global__ __launch_bounds__(NB) void k_linearize(ResArgs<T> a, int write_mask) {
    if (*a.gate == 0) return;
    const int ntiles = (a.O + NB / 8 - 1) / (NB / 8);
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int gid = tile * NB + threadIdx.x;
        const int o = gid >> 3, j = gid & 7;
        T J[7], r, w, rho;
        const bool valid = lin_eval<T, IC>(a, o, j, write_mask, J, r, w, rho);
        if (write_mask) {
            const unsigned long long bal = __ballot(valid);
            if (j == 0 && o < a.O) a.mask[o] = (uint8_t)((bal >> (threadIdx.x & 56)) & 0xFFull);
        }
        T v[38];
        int k = 0;
        for (int p = 0; p < 6; ++p)
            for (int q = p; q < 6; ++q) v[k++] = w * J[p] * J[q];
        for (int p = 0; p < 6; ++p) v[21 + p] = w * J[p] * J[6];
        v[27] = w * J[6] * J[6];
        for (int p = 0; p < 7; ++p) v[28 + p] = w * J[p] * r;
        v[35] = valid ? rho : T(0);
        v[36] = valid ? r * r : T(0);
        v[37] = valid ? T(1) : T(0);
#pragma unroll
        for (int p = 0; p < 38; ++p) v[p] = wave_sum8(v[p]);
        if (j == 0 && o < a.O) {
            T *rec = a.rec + (size_t)o * REC_STRIDE;
#pragma unroll
            for (int p = 0; p < 38; ++p) rec[p] = v[p];
        }
    }
}

// Mixed precision: residuals and J in FP32, the pose-pose block of every pair
// contracted on BF16 MFMA. The kernel walks one pair chunk per block (pair
// order), so that a wavefront's 64 residuals (8 observations x 8 patch pixels)
// belong to one pair. Each u = sqrt(w) J_theta is split into three bfloat16
// terms u = hi + mid + lo (each the rounding of what the previous ones leave),
// and sum u u^T keeps every product of combined order >= 2^-24:
//   A1 + (A2 + A2^T) + (A3 + A3^T) + A4,  A1 = sum hi hi^T, A2 = sum hi mid^T,
//   A3 = sum hi lo^T, A4 = sum mid mid^T
// (the dropped mid lo and lo lo terms are below 2^-25 relative), so the block
// keeps FP32-level agreement with the depth couplings computed from the same
// rows; a two-term split (2^-17) is not enough: its error is of the order of
// the relative damping along the gauge direction of S. Each 64-residual group's
// four products come from v_mfma_f32_16x16x32_bf16 (FP32 accumulation) and are
// added to per-lane FP32 running sums with Kahan compensation; the four
// wavefronts of the block are then added in FP64 in a fixed order into the
// chunk partial (21 values) that the damping kernel sums per pair. The
// per-observation record gets every field except the pose-pose block.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void kahan_add(float &s, float &c, float v) {
    const float y = v - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

template <bool IC>
__global__ __launch_bounds__(BLOCK) void k_linearize_mixed(ResArgs<float> a, int write_mask,
                                                           const int *__restrict__ chunk_begin,
                                                           const int *__restrict__ chunk_end,
                                                           const int *__restrict__ pair_obs_idx,
                                                           double *__restrict__ partH) {
    constexpr int NS = 3;  // split terms hi, mid, lo
    constexpr int NA = 4;  // products A1..A4
    // per wavefront: the split terms of u^T as 16 x 64 bfloat16 (rows 6..15 stay zero)
    __shared__ __attribute__((aligned(16))) __bf16 ut[BLOCK / 64][NS][16][64];
    __shared__ double wsum[BLOCK / 64][NA][36];
    if (*a.gate == 0) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int e = lane; e < NS * 16 * 64; e += 64) (&ut[wv][0][0][0])[e] = (__bf16)0.0f;
    const int c = blockIdx.x, cb = chunk_begin[c], ce = chunk_end[c];
    const int j = lane & 7;
    float sa[NA][4], ca[NA][4];
#pragma unroll
    for (int m = 0; m < NA; ++m)
#pragma unroll
        for (int i = 0; i < 4; ++i) sa[m][i] = ca[m][i] = 0.0f;
    for (int g = wv; 8 * g < ce - cb; g += BLOCK / 64) {
        const int pos = cb + 8 * g + (lane >> 3);
        const int o = pos < ce ? pair_obs_idx[pos] : -1;
        float J[7], r, w, rho;
        const bool valid = lin_eval<float, IC>(a, o, j, write_mask, J, r, w, rho);
        if (write_mask) {
            const unsigned long long bal = __ballot(valid);
            if (j == 0 && o >= 0) a.mask[o] = (uint8_t)((bal >> (lane & 56)) & 0xFFull);
        }
        // per-observation fields (all but the pose-pose block)
        float v[17];
        for (int p = 0; p < 6; ++p) v[p] = w * J[p] * J[6];
        v[6] = w * J[6] * J[6];
        for (int p = 0; p < 7; ++p) v[7 + p] = w * J[p] * r;
        v[14] = valid ? rho : 0.0f;
        v[15] = valid ? r * r : 0.0f;
        v[16] = valid ? 1.0f : 0.0f;
#pragma unroll
        for (int p = 0; p < 17; ++p) v[p] = wave_sum8(v[p]);
        if (j == 0 && o >= 0) {
            float *rec = a.rec + (size_t)o * REC_STRIDE;
#pragma unroll
            for (int p = 0; p < 7; ++p) rec[REC_h + p] = v[p];   // REC_h (6) and REC_HDD
#pragma unroll
            for (int p = 0; p < 7; ++p) rec[REC_G + p] = v[7 + p];  // REC_G (6) and REC_GD
            rec[REC_E] = v[14];
            rec[REC_SQ] = v[15];
            rec[REC_CNT] = v[16];
        }
        // pose block: stage the split terms of u = sqrt(w) J_theta, transposed
        const float sw = sqrtf(w);
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            const float u = sw * J[p];
            const __bf16 hi = (__bf16)u;
            const float r1 = u - (float)hi;
            const __bf16 mid = (__bf16)r1;
            ut[wv][0][p][lane] = hi;
            ut[wv][1][p][lane] = mid;
            ut[wv][2][p][lane] = (__bf16)(r1 - (float)mid);
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        f32x4 acc[NA];
#pragma unroll
        for (int m = 0; m < NA; ++m) acc[m] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int k0 = 32 * s + 8 * (lane >> 4);
            const bf16x8 fh = *reinterpret_cast<const bf16x8 *>(&ut[wv][0][lane & 15][k0]);
            const bf16x8 fm = *reinterpret_cast<const bf16x8 *>(&ut[wv][1][lane & 15][k0]);
            const bf16x8 fl = *reinterpret_cast<const bf16x8 *>(&ut[wv][2][lane & 15][k0]);
            acc[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fh, fh, acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fh, fm, acc[1], 0, 0, 0);
            acc[2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fh, fl, acc[2], 0, 0, 0);
            acc[3] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fm, fm, acc[3], 0, 0, 0);
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int m = 0; m < NA; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i) kahan_add(sa[m][i], ca[m][i], acc[m][i]);
    }
    // lane l holds rows 4 (l / 16) + i, column l % 16 of the 16 x 16 sums
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int row = 4 * (lane >> 4) + i, col = lane & 15;
        if (row < 6 && col < 6)
#pragma unroll
            for (int m = 0; m < NA; ++m) wsum[wv][m][row * 6 + col] = (double)sa[m][i] - (double)ca[m][i];
    }
    __syncthreads();
    if (threadIdx.x < 21) {
        int p = 0, k = threadIdx.x;
        while (k >= 6 - p) {
            k -= 6 - p;
            ++p;
        }
        const int q = p + k, pq = p * 6 + q, qp = q * 6 + p;
        double sum = 0.0;
        for (int w2 = 0; w2 < BLOCK / 64; ++w2) {
            const double *W = &wsum[w2][0][0];
            sum += W[pq] + (W[36 + pq] + W[36 + qp]) + (W[72 + pq] + W[72 + qp]) + W[108 + pq];
        }
        partH[21 * (size_t)c + threadIdx.x] = sum;
    }
}

// IC iteration: residuals at the current parameters, Huber weights, and
// g = J^T W r with the constant proxy Jacobian (Sec. 3.5 steps 1-2). NB threads
// per workgroup, tiles of NB / 8 observations, grid-stride over the tiles.
// Three dependent memory steps per residual: the observation (with the gate),
// then the point, pair pose and pair camera data, then the target texels. The
// ten sums of an observation go out as one contiguous record (two stores per
// wavefront).
template <typename T, int NB>
__global__ __launch_bounds__(NB) void k_ic_residual(ResArgs<T> a) {
    const int ntiles = (a.O + NB / 8 - 1) / (NB / 8);
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int gid = tile * NB + threadIdx.x;
        const int o = gid >> 3, j = gid & 7;
        const bool in = o < a.O;
        const int n = in ? a.obs_point[o] : 0, pr = in ? a.obs_pair[o] : 0;
        const unsigned m = in ? (unsigned)a.mask[o] : 0u;
        // the gate as a vector load, in flight together with the observation's
        const int gv = __hip_atomic_load(a.gate, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__builtin_amdgcn_readfirstlane(gv) == 0) return;
        T c[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        // second step: every load that depends only on (n, pr, j), issued
        // before any branch. The pair's intrinsics and both relative poses (32
        // values) and the point's host pixel and inverse depths are loaded once
        // per observation, a slice per lane (lane j: values 4j..4j+3 of
        // pcam | rel | rel0; lanes 0-2: host_uv, depth, depth0), and read across
        // the observation's 8 lanes: a lane's loads return 11 values instead of
        // 43, and the per-CU return path is what bounds this step.
        typedef T T4 __attribute__((ext_vector_type(4)));
        const bool act = in && j < a.P && ((m >> j) & 1);
        T4 sl = {0, 0, 0, 0};
        double pt = 0.0;
        if (in && m != 0u) {
            const T *src = j < 2 ? a.pcam + 8 * pr + 4 * j
                                 : (j < 5 ? a.rel + REL_STRIDE * pr + 4 * (j - 2)
                                          : a.rel0 + REL_STRIDE * pr + 4 * (j - 5));
            sl = *reinterpret_cast<const T4 *>(src);
            if (j < 3)
                pt = j == 0 ? *reinterpret_cast<const double *>(a.host_uv + 2 * n) : (j == 1 ? a.depth[n] : a.depth0[n]);
        }
        T tp[4] = {0, 0, 0, 0};
        int f = 0;
        if (act) {
#pragma unroll
            for (int k = 0; k < 4; ++k) tp[k] = a.tmpl[4 * ((size_t)n * a.P + j) + k];
            f = a.pair_target[pr];
        }
        // keep the compiler from sinking these loads into the branches below
        // (the pins follow every load, so that all of them are in flight)
        pin_reg(sl);
        pin_reg(pt);
        pin_reg(f);
#pragma unroll
        for (int k = 0; k < 4; ++k) pin_reg(tp[k]);
        // the group's values, read by the whole wavefront
        T q[32];
        bcast8_slices(sl, q, std::make_integer_sequence<int, 32>{});
        const double uv = bcast8<0>(pt), dd = bcast8<1>(pt), dd0 = bcast8<2>(pt);
        if (act) {
            const T *cam = q, *R = q + 8, *R0 = q + 20;   // cam: host, target (fx, fy, cx, cy)
            const long long uvb = __double_as_longlong(uv);
            const T hu = (T)__int_as_float((int)uvb), hv = (T)__int_as_float((int)(uvb >> 32));
            const T d = (T)dd, d0 = (T)dd0;
            // pattern offset of lane j by selects (no lane-indexed argument loads)
            float du = a.pat.du[0], dv = a.pat.dv[0];
#pragma unroll
            for (int k = 1; k < 8; ++k) {
                du = j == k ? a.pat.du[k] : du;
                dv = j == k ? a.pat.dv[k] : dv;
            }
            const T u = (hu + T(0.5)) * a.scale - T(0.5) + (T)du;
            const T v = (hv + T(0.5)) * a.scale - T(0.5) + (T)dv;
            const T x = (u - cam[2]) / cam[0], y = (v - cam[3]) / cam[1];
            const T *t = R + 9;
            const T vz = R[6] * x + R[7] * y + R[8] + d * t[2];
            const T vx = R[0] * x + R[1] * y + R[2] + d * t[0];
            const T vy = R[3] * x + R[4] * y + R[5] + d * t[1];
            if (d > T(0) && vz > T(0)) {
                const T qu = cam[4] * (vx / vz) + cam[6], qv = cam[5] * (vy / vz) + cam[7];
                if (usable(qu, qv, a.W, a.H)) {
                    // third step: the target texels
                    const T If = bilinear(a.img + (size_t)f * a.W * a.H, a.W, qu, qv);
                    const T r = tp[0] - If;
                    T w, rho;
                    huber(r, a.huber_k, w, rho);
                    T J[7];
                    ic_jacobian(x, y, R0, R0 + 9, d0, tp[1], tp[2], cam[0], cam[1], J);
                    const T wr = w * r;
#pragma unroll
                    for (int p = 0; p < 7; ++p) c[p] = wr * J[p];
                    c[7] = rho;
                    c[8] = r * r;
                    c[9] = T(1);
                }
            }
        }
#pragma unroll
        for (int p = 0; p < 10; ++p) c[p] = wave_sum8(c[p]);
        // every lane of the observation holds the sums: lane j stores field j
        // (and lanes 0, 1 fields 8, 9)
        T v0 = c[0];
#pragma unroll
        for (int p = 1; p < 8; ++p) v0 = j == p ? c[p] : v0;
        const T v1 = j == 0 ? c[8] : c[9];
        if (in) {
            T *rec = a.icr + (size_t)o * IC_REC;
            rec[j] = v0;
            if (j < 2) rec[8 + j] = v1;
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
        const int h = a.pair_host[pr], f = a.pair_target[pr];
        const T *Kh = a.K + 4 * h;
        const T *Kt = a.K + 4 * f;
        const T *tp = a.tmpl + 4 * ((size_t)n * a.P + j);
        T x, y;
        template_xy(a, n, j, Kh, x, y);
        const T *R = a.rel + REL_STRIDE * pr;
        const T *t = R + 9;
        const T d = (T)a.depth[n];
        const T vz = R[6] * x + R[7] * y + R[8] + d * t[2];
        if (tp[3] != T(0) && d > T(0) && vz > T(0)) {
            const T vx = R[0] * x + R[1] * y + R[2] + d * t[0];
            const T vy = R[3] * x + R[4] * y + R[5] + d * t[1];
            const T qu = Kt[0] * (vx / vz) + Kt[2], qv = Kt[1] * (vy / vz) + Kt[3];
            if (usable(qu, qv, a.W, a.H)) {
                const T r = tp[0] - bilinear(a.img + (size_t)f * a.W * a.H, a.W, qu, qv);
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
        T *rec = a.rec + (size_t)o * REC_STRIDE;
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
                                                      const T *__restrict__ rec, double *__restrict__ Hdd,
                                                      double *__restrict__ gd, int with_hdd,
                                                      const int *__restrict__ gate) {
    if (*gate == 0) return;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    double hs = 0.0, gs = 0.0;
    if (n < N) {
        const int o0 = obs_ptr[n], o1 = obs_ptr[n + 1];
#pragma unroll 4
        for (int o = o0; o < o1; ++o) {
            const T *r = rec + (size_t)o * REC_STRIDE;
            hs += (double)r[REC_HDD];
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
__global__ __launch_bounds__(PAIR_CHUNK) void k_pair_chunk_H(const int4 *__restrict__ slot, const T *__restrict__ rec,
                                                      double *__restrict__ partH, const int *__restrict__ gate) {
    __shared__ double lds[21 * 16];
    if (*gate == 0) return;
    const int c = blockIdx.x;
    const int o = slot[(size_t)c * PAIR_CHUNK + threadIdx.x].x;
    double v[21];
    for (int k = 0; k < 21; ++k) v[k] = 0.0;
    if (o >= 0) {
        const T *r = rec + (size_t)o * REC_STRIDE;
        for (int k = 0; k < 21; ++k) v[k] += (double)r[REC_H + k];
    }
    block_sum<21>(v, lds);
    if (threadIdx.x == 0)
        for (int k = 0; k < 21; ++k) partH[21 * c + k] = v[k];
}

// Per chunk of one pair's observations (at most PAIR_CHUNK, one per thread):
// reduced right-hand side contribution sum_o (g_o - h_o g_d,n / H_dd,n) (depth
// elimination of the gradient) and the energy statistics. gr / gs: gradient
// records (GR_* fields) and their stride; h_o from the full record; prange: the
// observation range of each observation's point.
template <typename T>
__global__ __launch_bounds__(PAIR_CHUNK) void k_pair_chunk_y(const int4 *__restrict__ slot, const T *__restrict__ rec,
                                                             const T *__restrict__ gr, int gs,
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
        const T *r = rec + (size_t)o * REC_STRIDE;
        const T *g = gr + (size_t)o * gs;
        double gdn = 0.0;  // g_d,n: the point's records in order (bitwise the per-point sum)
#pragma unroll 4
        for (int q = q0; q < q1; ++q) gdn += (double)gr[(size_t)q * gs + GR_GD];
        const double s = gdn / Hdd[n];
        for (int k = 0; k < 6; ++k) v[k] += (double)g[GR_G + k] - (double)r[REC_h + k] * s;
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
    const float *__restrict__ host_uv, const double *__restrict__ pairK0, const T *__restrict__ rec,
    const T *__restrict__ gr, int gs, const double *__restrict__ Hdd, const double *__restrict__ dth_rel,
    const double *__restrict__ geo_old, const double *__restrict__ geo_new, double *__restrict__ depth,
    const double *__restrict__ depth0, double *__restrict__ part, const int *__restrict__ gate,
    const int *__restrict__ flag) {
    __shared__ double lds[depth_lds_doubles(256)];
    double md = 0.0, ms = 0.0;
    const int n0 = blockIdx.x * DU_PTS;
    const DepthPoint pt = depth_point<false>(N, n0, obs_ptr, host_uv, Hdd, depth, depth0);
    if (!depth_points<T, 256>(N, n0, ic, pt, obs_pair, pairK0, rec, gr, gs, dth_rel, geo_old, geo_new, depth, gate,
                              flag, lds, md, ms))
        return;
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = md;
        part[2 * blockIdx.x + 1] = ms;
    }
}

// ------------------------------------------------------------ launchers

static inline unsigned nblk(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

template <typename T>
static ResArgs<T> res_args(Ctx &c, int level, const T *rel_cur) {
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
    a.scale = T(1) / T(1 << level);
    a.huber_k = (T)c.cfg.huber_k;
    a.obs_point = c.d_obs_point;
    a.obs_pair = c.d_obs_pair;
    a.pair_host = c.d_pair_host;
    a.pair_target = c.d_pair_target;
    a.host_uv = c.d_host_uv;
    a.img = (const T *)c.lv[level].img;
    a.K = (const T *)c.lv[level].K;
    a.tmpl = (const T *)c.lv[level].tmpl;
    a.rel = rel_cur;
    a.rel0 = (const T *)c.d_rel0;
    a.depth = c.d_depth;
    a.depth0 = c.d_depth0;
    a.mask = c.d_mask;
    a.rec = (T *)c.d_rec;
    a.pcam = (const T *)c.lv[level].pcam;
    a.icr = (T *)c.d_icr;
    a.gate = c.d_gate;
    return a;
}

static ConvArgs conv_args(Ctx &c, double *stat, double conv_px, int level) {
    return ConvArgs{c.d_wstat, c.nwin, stat, conv_px, c.d_gate, c.d_count + level, c.d_flag};
}

// Gradient records of the current iteration: the compact IC records or the
// G .. CNT fields of the full record (FC).
template <typename T>
static void grad_records(const Ctx &c, const T *&gr, int &gs) {
    if (c.cfg.mode == PBA_IC_PROXY) {
        gr = (const T *)c.d_icr;
        gs = IC_REC;
    } else {
        gr = (const T *)c.d_rec + REC_G;
        gs = REC_STRIDE;
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
                                               a.scale, (T *)c.lv[level].tmpl);
    CHECK_LAUNCH();
    if (c.st.n_pairs > 0) {
        k_pair_cam<T><<<nblk((size_t)c.st.n_pairs * 8, 256), 256, 0, s>>>(
            c.st.n_pairs, c.d_pair_host, c.d_pair_target, a.K, (T *)c.lv[level].pcam);
        CHECK_LAUNCH();
    }
}

template <typename T>
void Launch<T>::level_begin(hipStream_t s, Ctx &c, int level, bool clear_flag) {
    const int m = std::max(std::max(12 * c.F, c.N), std::max(c.st.n_pairs, 1));
    k_level_begin<T><<<nblk(m, 256), 256, 0, s>>>(c.F, c.N, c.st.n_pairs, c.d_poses, c.d_poses0, c.d_depth,
                                                  c.d_depth0, c.d_pair_host, c.d_pair_target, c.d_geo0,
                                                  (T *)c.d_rel0, c.d_geo_a, (T *)c.d_rel_a, c.d_gate, c.d_flag,
                                                  c.d_count + level, clear_flag ? 1 : 0);
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
static unsigned shape_grid(const Ctx &c, LaunchShape sh) {
    const size_t tiles = ((size_t)c.O * LANES_PER_OBS + sh.block - 1) / sh.block;
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
    ResArgs<T> a = res_args<T>(c, level, (const T *)c.d_rel0);
    launch_linearize_shape<T, true>(s, c, a, 1, LaunchShape{});
    CHECK_LAUNCH();
}

template <typename T>
void Launch<T>::fc_linearize(hipStream_t s, Ctx &c, int level, const T *rel_cur, bool write_mask, hipEvent_t e0,
                             hipEvent_t e1) {
    if (c.O == 0) return;
    ResArgs<T> a = res_args<T>(c, level, rel_cur);
    launch_linearize_shape<T, false>(s, c, a, write_mask ? 1 : 0, c.tune_lin, e0, e1);
    CHECK_LAUNCH();
}

void launch_linearize_mixed(hipStream_t s, Ctx &c, int level, bool ic, const float *rel_cur, bool write_mask,
                            hipEvent_t e0, hipEvent_t e1) {
    const int nch = (int)c.st.pchunk_begin.size();
    if (c.O == 0 || nch == 0) return;
    ResArgs<float> a = res_args<float>(c, level, rel_cur);
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
void Launch<T>::ic_residual(hipStream_t s, Ctx &c, int level, const T *rel_cur, hipEvent_t e0, hipEvent_t e1) {
    ic_residual_shape(s, c, level, rel_cur, c.tune_res, e0, e1);
}

template <typename T>
void Launch<T>::ic_residual_shape(hipStream_t s, Ctx &c, int level, const T *rel_cur, LaunchShape sh, hipEvent_t e0,
                                  hipEvent_t e1) {
    if (c.O == 0) return;
    ResArgs<T> a = res_args<T>(c, level, rel_cur);
    const unsigned g = shape_grid(c, sh);
    switch (sh.block) {
        case 64: launch_ev(k_ic_residual<T, 64>, g, 64, s, e0, e1, a); break;
        case 128: launch_ev(k_ic_residual<T, 128>, g, 128, s, e0, e1, a); break;
        case 512: launch_ev(k_ic_residual<T, 512>, g, 512, s, e0, e1, a); break;
        case 1024: launch_ev(k_ic_residual<T, 1024>, g, 1024, s, e0, e1, a); break;
        default: launch_ev(k_ic_residual<T, 256>, g, 256, s, e0, e1, a); break;
    }
    CHECK_LAUNCH();
}

template <typename T>
void Launch<T>::fc_linearize_shape(hipStream_t s, Ctx &c, int level, const T *rel_cur, LaunchShape sh) {
    if (c.O == 0) return;
    ResArgs<T> a = res_args<T>(c, level, rel_cur);
    launch_linearize_shape<T, false>(s, c, a, 1, sh);
    CHECK_LAUNCH();
}

template <typename T>
void Launch<T>::evaluate(hipStream_t s, Ctx &c, int level) {
    if (c.O == 0) return;
    const T *rel = (const T *)(c.flip ? c.d_rel_b : c.d_rel_a);
    ResArgs<T> a = res_args<T>(c, level, rel);
    k_evaluate<T><<<nblk((size_t)c.O * LANES_PER_OBS, BLOCK), BLOCK, 0, s>>>(a);
    CHECK_LAUNCH();
}

template <typename T>
void Launch<T>::point_reduce(hipStream_t s, Ctx &c, bool with_hdd) {
    if (c.N == 0) return;
    k_point_reduce<T><<<nblk(c.N, 256), 256, 0, s>>>(c.N, c.d_obs_ptr, (const T *)c.d_rec, c.d_Hdd, c.d_gd,
                                                     with_hdd ? 1 : 0, c.d_gate);
    CHECK_LAUNCH();
}

template <typename T>
void Launch<T>::pair_reduce_H(hipStream_t s, Ctx &c) {
    const int nch = (int)c.st.pchunk_begin.size();
    if (nch == 0) return;
    k_pair_chunk_H<T><<<nch, PAIR_CHUNK, 0, s>>>((const int4 *)c.d_pc_slot, (const T *)c.d_rec, c.d_partH, c.d_gate);
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
    const T *gr;
    int gs;
    grad_records<T>(c, gr, gs);
    k_pair_chunk_y<T><<<nch, PAIR_CHUNK, 0, s>>>((const int4 *)c.d_pc_slot, (const T *)c.d_rec, gr, gs, c.d_Hdd,
                                                 c.d_partY, c.d_gate, prev_stat ? c.d_du_part : nullptr,
                                                 du_nparts(c), conv_args(c, prev_stat, conv_px, level));
    CHECK_LAUNCH();
}


template <typename T>
void Launch<T>::depth_update(hipStream_t s, Ctx &c, const double *geo_old, const double *geo_new, double *stat,
                             double conv_px, int level, bool finish) {
    const int nb = (int)nblk(c.N, DU_PTS);
    const T *gr;
    int gs;
    grad_records<T>(c, gr, gs);
    if (c.N > 0)
        k_depth_update<T><<<nb, 256, 0, s>>>(c.N, c.cfg.mode == PBA_IC_PROXY ? 1 : 0, c.d_obs_ptr, c.d_obs_pair,
                                             c.d_host_uv, c.d_pairK0, (const T *)c.d_rec, gr, gs, c.d_Hdd,
                                             c.d_dth_rel, geo_old, geo_new, c.d_depth, c.d_depth0, c.d_du_part,
                                             c.d_gate, c.d_flag);
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
    if (threadIdx.x == 0) ran = *cv.count;
    __syncthreads();
    if (ran & 1)
        for (int e = threadIdx.x; e < np; e += blockDim.x) pose[e] = pose_alt[e];
}

// Start of a batch of iterations: clear the level's iteration count and
// (clear_flag) the failure flag, and open the gate unless a failure is flagged
// (a kernel, so that it can be captured in a graph).
__global__ void k_open(int *__restrict__ gate, int *__restrict__ flag, int *__restrict__ count, int clear_flag) {
    if (threadIdx.x == 0) {
        if (clear_flag) *flag = 0;
        *gate = *flag == 0 ? 1 : 0;
        *count = 0;
    }
}

void launch_conv(hipStream_t s, Ctx &c, double *stat, double conv_px, int nparts, int level, bool pose_sync) {
    k_conv<<<1, 256, 0, s>>>(c.d_du_part, nparts, conv_args(c, stat, conv_px, level), c.d_poses_alt, c.d_poses,
                             pose_sync ? 12 * c.F : 0);
    CHECK_LAUNCH();
}

void launch_open(hipStream_t s, Ctx &c, int level, bool clear_flag) {
    k_open<<<1, 64, 0, s>>>(c.d_gate, c.d_flag, c.d_count + level, clear_flag ? 1 : 0);
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
