// Per-frame affine brightness in the forward-compositional iteration.
//
// Reading (the paper names explicit photometric modelling, as in DSO, in its
// prior-art discussion, Sec. 2, and gives no model): frame f has a log-gain
// a_f and an offset b_f; the target intensity is brought into the host's
// photometric units before it is compared with the template,
//     r = I_h(x) - b_h - g (I_f(W(x; p)) - b_f),   g = e^{a_h - a_f},
// the paper's residual at a = b = 0. Its derivatives: the FC Jacobian of the
// plain residual times g for the geometry, and (-g (I_f - b_f), -1,
// g (I_f - b_f), g) for (a_h, b_h, a_f, b_f). The unknowns are 6 pose and 2
// brightness parameters per frame and the inverse depths.
//
// One iteration: each observation's FC record (pose-pose block, h, H_dd,
// gradients; read by the FC kernels, which form the pose part of the depth
// Schur complement as before) and its brightness record (pose-brightness and
// brightness-brightness blocks, the brightness-depth coupling and gradient);
// then the 8F x 8F reduced system: the pose block from the FC assembly, the
// direct terms of the brightness rows and of the right-hand side summed per
// pair chunk, their depth Schur terms summed in LDS per host chunk, each
// chunk's sums added once (FP64 atomic adds, so these sums are not bitwise
// reproducible between runs), the brightness
// damping (damping_rel times the mean of the brightness diagonal) and the pin
// (the pinned frame's 8 rows); the tiled Cholesky solve; the
// pose, brightness and depth updates and the convergence measure. All
// arithmetic in FP64 (the images and templates in the context's type).
#include <algorithm>
#include <climits>

#include "pba_device.hpp"
#include "pba_affine.hpp"
#include "pba_internal.hpp"

namespace pba {

template <typename T>
struct AffArgs {
    int O, P, W, H;
    double scale, huber_k;
    int du[8], dv[8];
    const int *obs_point, *obs_pair, *pair_host, *pair_target;
    const float *host_uv;
    const T *img, *tmpl;
    const double *geo, *pcam, *depth, *ab;
    uint8_t *mask;
    const uint8_t *live;
    double *rec, *arec;
    const int *gate;   // 0: the level has converged or failed, skip the work (modes 0 and 1)
};

// Both records of every observation. mode 0: linearize over the frozen set;
// 1: decide the frozen set at these parameters, then linearize; 2: statistics
// over the set usable at these parameters only (the mask is not touched).
// One thread per observation over its patch pixels. The two records of a
// wavefront's 64 observations are contiguous in memory; they are staged in LDS
// and stored by the wavefront as consecutive doubles (a thread's own stores
// would land 320 and 336 bytes apart between lanes). A lane past the last
// observation repeats the last one and stores nothing.
constexpr int AFF_LIN_THREADS = 128;

template <typename T>
__global__ __launch_bounds__(AFF_LIN_THREADS) void k_aff_linearize(AffArgs<T> a, int mode) {
    __shared__ double stage[AFF_LIN_THREADS / WAVE][WAVE][AFF_STRIDE];
    if (mode != 2 && *a.gate == 0) return;
    const int o_raw = blockIdx.x * blockDim.x + threadIdx.x;
    const bool has = o_raw < a.O;
    const int o = has ? o_raw : a.O - 1;
    const int n = a.obs_point[o], p = a.obs_pair[o];
    const int h = a.pair_host[p], f = a.pair_target[p];
    const double *g = a.geo + GEO_STRIDE * p, *K = a.pcam + 8 * p;
    const double d = a.depth[n];
    const double ah = a.ab[2 * h], bh = a.ab[2 * h + 1], af = a.ab[2 * f], bf = a.ab[2 * f + 1];
    const double gain = exp(ah - af);
    const T *img = a.img + (size_t)f * a.W * a.H;
    double H21[21], hv[6], hdd = 0.0, gv6[6], gd = 0.0, E = 0.0, SQ = 0.0, CNT = 0.0;
    double C[24], Pp[10], hp[4], gp[4];
    for (int k = 0; k < 21; ++k) H21[k] = 0.0;
    for (int k = 0; k < 6; ++k) hv[k] = gv6[k] = 0.0;
    for (int k = 0; k < 24; ++k) C[k] = 0.0;
    for (int k = 0; k < 10; ++k) Pp[k] = 0.0;
    for (int k = 0; k < 4; ++k) hp[k] = gp[k] = 0.0;
    unsigned m = mode == 0 ? (unsigned)a.mask[o] : 0u;
    const bool live = a.live[o] != 0;
    for (int j = 0; j < a.P; ++j) {
        const T *tp = a.tmpl + 4 * ((size_t)n * a.P + j);
        const double u = ((double)a.host_uv[2 * n] + 0.5) * a.scale - 0.5 + (double)a.du[j];
        const double v = ((double)a.host_uv[2 * n + 1] + 0.5) * a.scale - 0.5 + (double)a.dv[j];
        const double x = (u - K[2]) / K[0], y = (v - K[3]) / K[1];
        const double Rx0 = g[0] * x + g[1] * y + g[2], Rx1 = g[3] * x + g[4] * y + g[5];
        const double Rx2 = g[6] * x + g[7] * y + g[8];
        const double v0 = Rx0 + d * g[9], v1 = Rx1 + d * g[10], vz = Rx2 + d * g[11];
        const bool front = vz > 0.0;
        const double vzs = front ? vz : 1.0;
        const double ux = v0 / vzs, uy = v1 / vzs;
        const double qu = K[4] * ux + K[6], qv = K[5] * uy + K[7];
        const bool ok_now = (double)tp[3] != 0.0 && d > 0.0 && front && usable(qu, qv, a.W, a.H);
        if (mode == 1 && ok_now) m |= 1u << j;
        const bool use = live && ok_now && (mode == 2 || ((m >> j) & 1u));
        if (!use) continue;
        double If, gu, gvv;
        bilinear_grad(img, a.W, qu, qv, If, gu, gvv);
        const double r = (double)tp[0] - bh - gain * (If - bf);
        double w, rho;
        huber(r, a.huber_k, w, rho);
        E += rho;
        SQ += r * r;
        CNT += 1.0;
        if (mode == 2) continue;
        double J[7];
        const double t3[3] = {g[9], g[10], g[11]};
        fc_jacobian(Rx0, Rx1, Rx2, vz, ux, uy, t3, d, gu, gvv, K[4], K[5], J);
        for (int k = 0; k < 7; ++k) J[k] *= gain;
        const double e = gain * (If - bf);
        const double Jp[4] = {-e, -1.0, e, gain};
        int t = 0;
        for (int i = 0; i < 6; ++i)
            for (int k = i; k < 6; ++k) H21[t++] += w * J[i] * J[k];
        for (int i = 0; i < 6; ++i) {
            hv[i] += w * J[i] * J[6];
            gv6[i] += w * J[i] * r;
            for (int k = 0; k < 4; ++k) C[4 * i + k] += w * J[i] * Jp[k];
        }
        hdd += w * J[6] * J[6];
        gd += w * J[6] * r;
        t = 0;
        for (int i = 0; i < 4; ++i) {
            for (int k = i; k < 4; ++k) Pp[t++] += w * Jp[i] * Jp[k];
            hp[i] += w * Jp[i] * J[6];
            gp[i] += w * Jp[i] * r;
        }
    }
    if (mode == 1 && has) a.mask[o] = (uint8_t)m;
    if (mode == 2) {
        if (has) {
            double *rc = a.rec + (size_t)o * REC_STRIDE;
            rc[REC_E] = E;
            rc[REC_SQ] = SQ;
            rc[REC_CNT] = CNT;
        }
        return;
    }
    const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int o_first = blockIdx.x * blockDim.x + w * WAVE;
    const int cnt = max(0, min(WAVE, a.O - o_first));
    double *row = stage[w][lane];
    for (int k = 0; k < 21; ++k) row[REC_H + k] = H21[k];
    for (int k = 0; k < 6; ++k) {
        row[REC_h + k] = hv[k];
        row[REC_G + k] = gv6[k];
    }
    row[REC_HDD] = hdd;
    row[REC_GD] = gd;
    row[REC_E] = E;
    row[REC_SQ] = SQ;
    row[REC_CNT] = CNT;
    for (int k = REC_CNT + 1; k < REC_STRIDE; ++k) row[k] = 0.0;
    __syncthreads();
    double *dst = a.rec + (size_t)o_first * REC_STRIDE;
    for (int i = lane; i < cnt * REC_STRIDE; i += WAVE) dst[i] = stage[w][i / REC_STRIDE][i % REC_STRIDE];
    __syncthreads();
    for (int k = 0; k < 24; ++k) row[AFF_C + k] = C[k];
    for (int k = 0; k < 10; ++k) row[AFF_P + k] = Pp[k];
    for (int k = 0; k < 4; ++k) {
        row[AFF_h + k] = hp[k];
        row[AFF_G + k] = gp[k];
    }
    __syncthreads();
    dst = a.arec + (size_t)o_first * AFF_STRIDE;
    for (int i = lane; i < cnt * AFF_STRIDE; i += WAVE) dst[i] = stage[w][i / AFF_STRIDE][i % AFF_STRIDE];
}

constexpr int AFF_EMAX = MAX_HOST_TARGETS + 1;
constexpr int AFF_LDS_MAX = 65536;   // bytes of dynamic LDS per workgroup
constexpr int AFF_GROUP = 32;        // lanes per point in k_aff_schur (two points per wavefront)
constexpr int AFF_DIRECT = 44;       // values summed per pair: C (24), P (10), G_phi (4), g (6)
static_assert(MAX_HOST_TARGETS < AFF_GROUP, "one lane per observation of a point");

__device__ __forceinline__ double group_sum_d(double v) {   // over aligned groups of AFF_GROUP lanes
#pragma unroll
    for (int off = AFF_GROUP / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

// The direct terms of the brightness rows, summed per pair chunk (the
// observations of one pair; one thread each) and added to the reduced system
// once per chunk in absolute coordinates: the pose-brightness blocks (A^T C
// for the target's pose, B^T C for the host's), the brightness-brightness
// block, the brightness gradients and the pose gradients (A^T g, B^T g).
__global__ __launch_bounds__(PAIR_CHUNK) void k_aff_pairs(int F, const int *__restrict__ pchunk_begin,
                                                          const int *__restrict__ pchunk_end,
                                                          const int *__restrict__ pair_obs_idx,
                                                          const int *__restrict__ obs_pair,
                                                          const int *__restrict__ pair_host,
                                                          const int *__restrict__ pair_target,
                                                          const double *__restrict__ geo,
                                                          const double *__restrict__ rec,
                                                          const double *__restrict__ arec, double *__restrict__ M,
                                                          double *__restrict__ b, double *__restrict__ diag_phi,
                                                          const int *__restrict__ gate) {
    __shared__ double part[PAIR_CHUNK / WAVE][AFF_DIRECT];
    if (*gate == 0) return;
    __shared__ double tot[AFF_DIRECT];
    const int k0 = pchunk_begin[blockIdx.x], k1 = pchunk_end[blockIdx.x];
    const int idx = k0 + (int)threadIdx.x;
    double v[AFF_DIRECT];
    if (idx < k1) {
        const int o = pair_obs_idx[idx];
        const double *ar = arec + (size_t)o * AFF_STRIDE, *rc = rec + (size_t)o * REC_STRIDE;
#pragma unroll
        for (int i = 0; i < 34; ++i) v[i] = ar[AFF_C + i];   // C and P are contiguous
#pragma unroll
        for (int i = 0; i < 4; ++i) v[34 + i] = ar[AFF_G + i];
#pragma unroll
        for (int i = 0; i < 6; ++i) v[38 + i] = rc[REC_G + i];
    } else {
#pragma unroll
        for (int i = 0; i < AFF_DIRECT; ++i) v[i] = 0.0;
    }
    const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
#pragma unroll
    for (int i = 0; i < AFF_DIRECT; ++i) {
        double x = v[i];
#pragma unroll
        for (int off = WAVE / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, WAVE);
        if (lane == 0) part[w][i] = x;
    }
    __syncthreads();
    if (threadIdx.x < AFF_DIRECT) {
        double x = 0.0;
        for (int q = 0; q < (int)(blockDim.x / WAVE); ++q) x += part[q][threadIdx.x];
        tot[threadIdx.x] = x;
    }
    __syncthreads();
    if (k1 <= k0) return;
    const int p = obs_pair[pair_obs_idx[k0]], h = pair_host[p], f = pair_target[p];
    const double *gm = geo + GEO_STRIDE * p;
    const int F6 = 6 * F;
    const size_t n8 = 8 * (size_t)F;
    const int col[4] = {F6 + 2 * h, F6 + 2 * h + 1, F6 + 2 * f, F6 + 2 * f + 1};   // (a_h, b_h, a_f, b_f)
    const int t = threadIdx.x;
    if (t < 4) {   // column t of C: pose-brightness blocks
        double cv[6], ta[6], tb[6];
        for (int i = 0; i < 6; ++i) cv[i] = tot[4 * i + t];
        apply_At(gm, cv, ta);
        apply_Bt(gm, cv, tb);
        for (int i = 0; i < 6; ++i) {
            unsafeAtomicAdd(M + (size_t)col[t] * n8 + 6 * f + i, ta[i]);
            unsafeAtomicAdd(M + (size_t)(6 * f + i) * n8 + col[t], ta[i]);
            unsafeAtomicAdd(M + (size_t)col[t] * n8 + 6 * h + i, tb[i]);
            unsafeAtomicAdd(M + (size_t)(6 * h + i) * n8 + col[t], tb[i]);
        }
        unsafeAtomicAdd(b + col[t], tot[34 + t]);
    } else if (t == 4) {   // brightness-brightness block
        int q = 0;
        for (int i = 0; i < 4; ++i)
            for (int k = i; k < 4; ++k, ++q) {
                const double x = tot[24 + q];
                unsafeAtomicAdd(M + (size_t)col[i] * n8 + col[k], x);
                if (i != k)
                    unsafeAtomicAdd(M + (size_t)col[k] * n8 + col[i], x);
                else
                    unsafeAtomicAdd(diag_phi + (col[i] - F6), x);
            }
    } else if (t == 5) {   // pose gradients
        double ta[6], tb[6];
        apply_At(gm, tot + 38, ta);
        apply_Bt(gm, tot + 38, tb);
        for (int i = 0; i < 6; ++i) {
            unsafeAtomicAdd(b + 6 * f + i, ta[i]);
            unsafeAtomicAdd(b + 6 * h + i, tb[i]);
        }
    }
}

// The depth Schur terms of the brightness rows and of the whole right-hand
// side, over the points of one host chunk (points of one host frame; one
// workgroup each): with u_p the point's couplings over the host's frame set
// (host and targets; per frame its pose, A^T h or for the host the sum of
// B^T h, and its brightness, h_phi), the brightness rows get
// -sum_p u_p,phi u_p^T / H_dd and the right-hand side -sum_p u_p g_d / H_dd.
// The couplings of a batch of points go to LDS as the rows of a matrix U
// (points x 8E, zero where a point does not observe a frame; one 32-lane
// group per point, one lane per observation), then the threads form the
// entries of the 2E x 8E block and of the 8E right-hand side as dot products
// over the batch's rows and add them to the global system (once per chunk
// when the chunk fits one batch: up to 128 points for frame sets of 7
// frames, 48 for the largest). The pose-pose terms come from the FC assembly.
constexpr int AFF_SCHUR_THREADS = 1024, AFF_SCHUR_GROUPS = AFF_SCHUR_THREADS / AFF_GROUP;

__global__ __launch_bounds__(AFF_SCHUR_THREADS) void k_aff_schur(
    int F, int Emax, const int *__restrict__ chunk_host, const int *__restrict__ chunk_begin,
    const int *__restrict__ chunk_end, const int *__restrict__ host_m, const int *__restrict__ hosts,
    const int *__restrict__ host_pts, const int *__restrict__ obs_ptr, const int *__restrict__ obs_pair,
    const int *__restrict__ pair_local, const int *__restrict__ pair_target, const double *__restrict__ geo,
    const double *__restrict__ rec, const double *__restrict__ arec, const double *__restrict__ Hdd,
    const double *__restrict__ gdn, double *__restrict__ M, double *__restrict__ b, const int *__restrict__ gate) {
    extern __shared__ double lds[];
    if (*gate == 0) return;
    const int ch = blockIdx.x, hi = chunk_host[ch];
    const int E = min(host_m[hi] + 1, Emax), nb = 2 * E, n8 = 8 * E, n6 = 6 * E;
    int *fr = (int *)lds;                           // frame of each frame-set index [Emax]
    double *wv = lds + (Emax + 1) / 2 + 1;          // per batch row: 1 / H_dd, then g_d / H_dd
    // rows of U per batch: as many as the dynamic LDS holds
    const int Pb = min(128, (int)((AFF_LDS_MAX / sizeof(double) - ((Emax + 1) / 2 + 1)) / (n8 + 2)));
    double *gv = wv + Pb, *U = gv + Pb;             // U [Pb][8E]: pose (6e + k), then brightness (6E + 2e + l)
    for (int i = threadIdx.x; i < Emax; i += blockDim.x) fr[i] = i == 0 ? hosts[hi] : -1;
    const int nent = nb * n8, ntot = nent + n8;     // brightness-row entries, then right-hand side entries
    const int F6 = 6 * F;
    const size_t N8 = 8 * (size_t)F;
    const int g = threadIdx.x / AFF_GROUP, lane = threadIdx.x % AFF_GROUP;
    const int q0 = chunk_begin[ch], q1 = chunk_end[ch];
    for (int sb = q0; sb < q1; sb += Pb) {
        const int rows = min(Pb, q1 - sb);
        __syncthreads();   // the previous batch's rows are no longer read
        for (int i = threadIdx.x; i < rows * n8; i += blockDim.x) U[i] = 0.0;
        __syncthreads();
        for (int row = g; row < rows; row += AFF_SCHUR_GROUPS) {
            const int n = host_pts[sb + row];
            const int o0 = obs_ptr[n], m = min(obs_ptr[n + 1] - o0, E - 1);
            double *u = U + (size_t)row * n8;
            double tb[6] = {0, 0, 0, 0, 0, 0}, ph0 = 0.0, ph1 = 0.0;
            if (lane < m) {
                const int o = o0 + lane, p = obs_pair[o];
                const int e = 1 + pair_local[p];
                const double *gm = geo + GEO_STRIDE * p;
                const double *hv = rec + (size_t)o * REC_STRIDE + REC_h, *ar = arec + (size_t)o * AFF_STRIDE;
                apply_Bt(gm, hv, tb);
                ph0 = ar[AFF_h];
                ph1 = ar[AFF_h + 1];
                if (e < E) {   // (the structure keeps every host within AFF_EMAX frames)
                    fr[e] = pair_target[p];   // the same value from every writer
                    double ta[6];
                    apply_At(gm, hv, ta);
                    for (int k = 0; k < 6; ++k) u[6 * e + k] = ta[k];
                    u[n6 + 2 * e] = ar[AFF_h + 2];
                    u[n6 + 2 * e + 1] = ar[AFF_h + 3];
                }
            }
            for (int k = 0; k < 6; ++k) tb[k] = group_sum_d(tb[k]);
            ph0 = group_sum_d(ph0);
            ph1 = group_sum_d(ph1);
            if (lane == 0) {
                for (int k = 0; k < 6; ++k) u[k] = tb[k];
                u[n6] = ph0;
                u[n6 + 1] = ph1;
                const double iH = 1.0 / Hdd[n];
                wv[row] = iH;
                gv[row] = gdn[n] * iH;
            }
        }
        __syncthreads();
        // the batch's sums, into the global system (hardware FP64 atomics on device memory)
        for (int i = threadIdx.x; i < ntot; i += blockDim.x) {
            const int c = i < nent ? i % n8 : i - nent;
            double sum = 0.0;
            if (i < nent) {
                const int r = i / n8;
                for (int q = 0; q < rows; ++q) sum += U[q * n8 + n6 + r] * U[q * n8 + c] * wv[q];
            } else {
                for (int q = 0; q < rows; ++q) sum += U[q * n8 + c] * gv[q];
            }
            if (sum == 0.0) continue;
            const int fc = c < n6 ? fr[c / 6] : fr[(c - n6) >> 1];
            if (fc < 0) continue;
            const size_t C = c < n6 ? (size_t)(6 * fc + c % 6) : (size_t)(F6 + 2 * fc + ((c - n6) & 1));
            if (i >= nent) {
                unsafeAtomicAdd(b + C, -sum);
                continue;
            }
            const int r = i / n8, fa = fr[r >> 1];
            if (fa < 0) continue;
            const size_t R = F6 + 2 * fa + (r & 1);
            unsafeAtomicAdd(M + R * N8 + C, -sum);
            if (c < n6) unsafeAtomicAdd(M + C * N8 + R, -sum);
        }
    }
}

// M <- 0 and the pose block <- the FC assembly's damped, pinned S; b, the
// brightness diagonal and the maxima <- 0.
__global__ void k_aff_clear(int F, const double *__restrict__ S, double *__restrict__ M, double *__restrict__ b,
                            double *__restrict__ diag_phi, unsigned long long *__restrict__ maxb,
                            const int *__restrict__ gate) {
    if (*gate == 0) return;
    const int n8 = 8 * F, F6 = 6 * F;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < (size_t)n8 * n8) {
        const int r = (int)(e / n8), c = (int)(e % n8);
        M[e] = (r < F6 && c < F6) ? S[(size_t)r * F6 + c] : 0.0;
    }
    if (e < (size_t)n8) b[e] = 0.0;
    if (e < (size_t)2 * F) diag_phi[e] = 0.0;
    if (e < 4) maxb[e] = 0ull;
}

// Brightness damping (damping_rel times the mean of the brightness diagonal
// before the pin; damping_rel when that mean is 0) and the pin of frame
// `pinned`: its 8 rows and columns become the identity, its rhs 0. One block.
__global__ void k_aff_finish(int F, int pinned, double damping_rel, double *__restrict__ M, double *__restrict__ b,
                             const double *__restrict__ diag_phi, const int *__restrict__ gate) {
    if (*gate == 0) return;
    __shared__ double mu;
    const int n8 = 8 * F, F6 = 6 * F;
    if (threadIdx.x == 0) {
        double sdg = 0.0;
        for (int k = 0; k < 2 * F; ++k) sdg += diag_phi[k];
        const double mean = F > 0 ? sdg / (2.0 * F) : 0.0;
        mu = mean > 0.0 ? damping_rel * mean : damping_rel;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 2 * F; k += blockDim.x) M[(size_t)(F6 + k) * n8 + F6 + k] += mu;
    __syncthreads();
    if (pinned < 0 || pinned >= F) return;
    for (int q = 0; q < 8; ++q) {
        const int r = q < 6 ? 6 * pinned + q : F6 + 2 * pinned + (q - 6);
        for (int c = threadIdx.x; c < n8; c += blockDim.x) {
            M[(size_t)r * n8 + c] = 0.0;
            M[(size_t)c * n8 + r] = 0.0;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            M[(size_t)r * n8 + r] = 1.0;
            b[r] = 0.0;
        }
        __syncthreads();
    }
}

// Pose (FC increment) and brightness updates of every frame; the old poses go
// to poses_old. Nothing when the solve failed (flag set).
__global__ void k_aff_frames(int F, const double *__restrict__ x, double *__restrict__ poses,
                             double *__restrict__ poses_old, double *__restrict__ ab, const int *__restrict__ flag) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F || *flag) return;
    double *P = poses + 12 * f;
    for (int k = 0; k < 12; ++k) poses_old[12 * f + k] = P[k];
    const double *dx = x + 6 * f;
    double dR[9], R[9];
    so3_exp(dx, dR);
    mat3_mul(dR, P, R);
    for (int k = 0; k < 9; ++k) P[k] = R[k];
    for (int k = 0; k < 3; ++k) P[9 + k] += dx[3 + k];
    ab[2 * f] += x[6 * F + 2 * f];
    ab[2 * f + 1] += x[6 * F + 2 * f + 1];
}

// Depth back-substitution dd = -(g_d + h^T (A dth_f + B dth_h) + h_phi^T dphi) / H_dd
// per point, then the largest point-centre displacement (old parameters
// against new, level-0 camera) and the largest depth step (maxb[0], maxb[1],
// as the bits of non-negative doubles).
__global__ __launch_bounds__(256) void k_aff_depths(int N, int F, const int *__restrict__ obs_ptr,
                                                    const int *__restrict__ obs_pair,
                                                    const int *__restrict__ pair_host,
                                                    const int *__restrict__ pair_target,
                                                    const double *__restrict__ geo_old,
                                                    const double *__restrict__ poses,
                                                    const double *__restrict__ pairK0,
                                                    const float *__restrict__ host_uv,
                                                    const double *__restrict__ rec, const double *__restrict__ arec,
                                                    const double *__restrict__ Hdd, const double *__restrict__ gdn,
                                                    const double *__restrict__ x, double *__restrict__ depth,
                                                    const uint8_t *__restrict__ live,
                                                    unsigned long long *__restrict__ maxb,
                                                    const int *__restrict__ flag) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N || *flag) return;
    const int o0 = obs_ptr[n], o1 = obs_ptr[n + 1];
    const int F6 = 6 * F;
    double s = gdn[n];
    for (int o = o0; o < o1; ++o) {
        const int p = obs_pair[o], h = pair_host[p], f = pair_target[p];
        const double *gm = geo_old + GEO_STRIDE * p;
        double ra[6], rb[6];
        apply_A(gm, x + 6 * f, ra);
        apply_B(gm, x + 6 * h, rb);
        const double *hv = rec + (size_t)o * REC_STRIDE + REC_h;
        for (int k = 0; k < 6; ++k) s += hv[k] * (ra[k] + rb[k]);
        const double *hp = arec + (size_t)o * AFF_STRIDE + AFF_h;
        s += hp[0] * x[F6 + 2 * h] + hp[1] * x[F6 + 2 * h + 1] + hp[2] * x[F6 + 2 * f] + hp[3] * x[F6 + 2 * f + 1];
    }
    const double d_old = depth[n];
    const double dd = o1 > o0 ? -s / Hdd[n] : 0.0;
    const double d_new = d_old + dd;
    depth[n] = d_new;
    double md = 0.0;
    for (int o = o0; o < o1; ++o) {
        if (!live[o]) continue;
        const int p = obs_pair[o], h = pair_host[p], f = pair_target[p];
        const double *Kp = pairK0 + 8 * p;
        const double xx = ((double)host_uv[2 * n] - Kp[2]) / Kp[0], yy = ((double)host_uv[2 * n + 1] - Kp[3]) / Kp[1];
        // old: the pair geometry of the iteration; new: from the updated poses
        const double *Ph = poses + 12 * h, *Pf = poses + 12 * f;
        double Rn[9], tn[3];
        mat3_mul_bt(Pf, Ph, Rn);
        for (int k = 0; k < 3; ++k) tn[k] = Pf[9 + k] - (Rn[3 * k] * Ph[9] + Rn[3 * k + 1] * Ph[10] + Rn[3 * k + 2] * Ph[11]);
        const double *go = geo_old + GEO_STRIDE * p;
        double q[2][2];
        bool ok = true;
        for (int w = 0; w < 2; ++w) {
            const double *R = w ? Rn : go;
            const double *t = w ? tn : go + 9;
            const double dd2 = w ? d_new : d_old;
            const double vx = R[0] * xx + R[1] * yy + R[2] + dd2 * t[0];
            const double vy = R[3] * xx + R[4] * yy + R[5] + dd2 * t[1];
            const double vz = R[6] * xx + R[7] * yy + R[8] + dd2 * t[2];
            ok = ok && vz > 0.0;
            const double vzs = vz > 0.0 ? vz : 1.0;
            q[w][0] = Kp[4] * vx / vzs + Kp[6];
            q[w][1] = Kp[5] * vy / vzs + Kp[7];
        }
        if (ok) md = fmax(md, hypot(q[1][0] - q[0][0], q[1][1] - q[0][1]));
    }
    atomicMax(maxb, (unsigned long long)__double_as_longlong(md));
    atomicMax(maxb + 1, (unsigned long long)__double_as_longlong(fabs(dd)));
}

// End of a joint iteration: its statistics slot (energy, sum r^2 and count
// at the linearization, the displacement, the largest pose and depth steps),
// the level's iteration count, and the gate: closed after a failed solve
// (flag 1, also raised in the context's failure flag) or, with conv_px >= 0,
// after the first iteration whose displacement is below conv_px. One block.
__global__ void k_aff_stat(int F, const double *__restrict__ x, const double *__restrict__ sums,
                           const unsigned long long *__restrict__ maxb, const int *__restrict__ flag,
                           int *__restrict__ gate, int *__restrict__ count, int *__restrict__ ctx_flag,
                           double *__restrict__ stat, double conv_px) {
    __shared__ double red[1024 / WAVE];
    if (*gate == 0) return;
    if (*flag == 1) {
        if (threadIdx.x == 0) {
            *ctx_flag = 1;
            *gate = 0;
        }
        return;
    }
    double mp = 0.0;
    for (int i = threadIdx.x; i < 6 * F; i += blockDim.x) mp = fmax(mp, fabs(x[i]));
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) mp = fmax(mp, __shfl_xor(mp, off, WAVE));
    if (threadIdx.x % WAVE == 0) red[threadIdx.x / WAVE] = mp;
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int w = 1; w < (int)(blockDim.x / WAVE); ++w) mp = fmax(mp, red[w]);
    const double disp = __longlong_as_double((long long)maxb[0]);
    stat[ST_E] = sums[0];
    stat[ST_SQ] = sums[1];
    stat[ST_CNT] = sums[2];
    stat[ST_DISP] = disp;
    stat[ST_STEP_P] = mp;
    stat[ST_STEP_D] = __longlong_as_double((long long)maxb[1]);
    *count += 1;
    if (conv_px >= 0.0 && disp < conv_px) *gate = 0;
}

// ------------------------------------------------------------ launchers

static inline unsigned nblk(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

template <typename T>
static AffArgs<T> aff_args(Ctx &c, const AffBufs &ab, int level, const double *geo) {
    AffArgs<T> a{};
    a.O = c.O;
    a.P = c.cfg.pattern_n;
    a.W = c.lv[level].W;
    a.H = c.lv[level].H;
    a.scale = 1.0 / (double)(1 << level);
    a.huber_k = c.cfg.huber_k;
    for (int j = 0; j < 8; ++j) {
        a.du[j] = j < a.P ? c.cfg.pattern_uv[2 * j] : 0;
        a.dv[j] = j < a.P ? c.cfg.pattern_uv[2 * j + 1] : 0;
    }
    a.obs_point = c.d_obs_point;
    a.obs_pair = c.d_obs_pair;
    a.pair_host = c.d_pair_host;
    a.pair_target = c.d_pair_target;
    a.host_uv = c.d_host_uv;
    a.img = (const T *)c.lv[level].img;
    a.tmpl = (const T *)c.lv[level].tmpl;
    a.geo = geo;
    a.pcam = (const double *)c.lv[level].pcam;
    a.depth = c.d_depth;
    a.ab = ab.ab;
    a.mask = c.d_mask;
    a.live = c.d_obs_live;
    a.rec = (double *)c.d_rec;
    a.arec = ab.arec;
    a.gate = c.d_gate;
    return a;
}

void launch_aff_linearize(hipStream_t s, Ctx &c, const AffBufs &ab, int level, const double *geo, int mode) {
    if (c.O == 0) return;
    if (c.cfg.precision == PBA_FP64)
        k_aff_linearize<double><<<nblk(c.O, AFF_LIN_THREADS), AFF_LIN_THREADS, 0, s>>>(aff_args<double>(c, ab, level, geo), mode);
    else
        k_aff_linearize<float><<<nblk(c.O, AFF_LIN_THREADS), AFF_LIN_THREADS, 0, s>>>(aff_args<float>(c, ab, level, geo), mode);
}

void launch_aff_system(hipStream_t s, Ctx &c, const AffBufs &a, const double *geo) {
    const int F = c.F, n8 = 8 * F;
    k_aff_clear<<<nblk((size_t)n8 * n8, 256), 256, 0, s>>>(F, c.d_S, a.M, a.b, a.dphi, a.maxb, c.d_gate);
    const int npc = (int)c.st.pchunk_begin.size();
    if (npc > 0)
        k_aff_pairs<<<npc, PAIR_CHUNK, 0, s>>>(F, c.d_pchunk_begin, c.d_pchunk_end, c.d_pair_obs_idx, c.d_obs_pair,
                                               c.d_pair_host, c.d_pair_target, geo, (const double *)c.d_rec, a.arec,
                                               a.M, a.b, a.dphi, c.d_gate);
    const int nch = (int)c.st.chunk_host.size();
    if (nch > 0) {
        int Emax = 1;
        for (int m : c.st.host_m) Emax = std::max(Emax, std::min(m + 1, AFF_EMAX));
        k_aff_schur<<<nch, AFF_SCHUR_THREADS, AFF_LDS_MAX, s>>>(
            F, Emax, c.d_chunk_host, c.d_chunk_begin, c.d_chunk_end, c.d_host_m, c.d_host_frames, c.d_host_pts,
            c.d_obs_ptr, c.d_obs_pair, c.d_pair_local, c.d_pair_target, geo, (const double *)c.d_rec, a.arec,
            c.d_Hdd, c.d_gd, a.M, a.b, c.d_gate);
    }
    k_aff_finish<<<1, 256, 0, s>>>(F, c.cfg.pinned_frame, c.cfg.damping_rel, a.M, a.b, a.dphi, c.d_gate);
}

void launch_aff_update(hipStream_t s, Ctx &c, const AffBufs &a, const double *geo_old) {
    const int F = c.F;
    k_aff_frames<<<nblk(F, 64), 64, 0, s>>>(F, a.x, c.d_poses, a.poses_old, a.ab, a.flag);
    if (c.N > 0)
        k_aff_depths<<<nblk(c.N, 256), 256, 0, s>>>(c.N, F, c.d_obs_ptr, c.d_obs_pair, c.d_pair_host, c.d_pair_target,
                                                    geo_old, c.d_poses, c.d_pairK0, c.d_host_uv,
                                                    (const double *)c.d_rec, a.arec, c.d_Hdd, c.d_gd, a.x, c.d_depth,
                                                    c.d_obs_live, a.maxb, a.flag);
}

void launch_aff_stat(hipStream_t s, Ctx &c, const AffBufs &a, int level, double *stat, double conv_px) {
    k_aff_stat<<<1, 256, 0, s>>>(c.F, a.x, a.stats, a.maxb, a.flag, c.d_gate, c.d_count + level, c.d_flag, stat,
                                 conv_px);
}

}  // namespace pba
