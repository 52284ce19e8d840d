// FP64 kernels of the reduced pose system: depth damping, the per-host Gram of
// the depth Schur complement, assembly of S, Cholesky, the IC inverse, and the
// single-workgroup solve + pose update of every iteration.
#include <hip/hip_ext.h>

#include "pba_depth.hpp"
#include "pba_device.hpp"
#include "pba_internal.hpp"
#include "pba_tile.hpp"

#include <algorithm>

namespace pba {

constexpr int SOLVE_THREADS = 1024;
constexpr int MU_LDS_PAIRS = 512;               // pair sums of the damping kernel kept in LDS up to this many pairs
constexpr int LDS_DOUBLES = 152 * 1024 / 8;   // packed lower triangle of S (+ panel scratch) when it fits
constexpr int LDS_MAX_N = LDS_CHOL_MAX_N;     // n (n + 1) / 2 + 17 n <= LDS_DOUBLES; 3 rows per lane
constexpr int IC_SPLIT_N = 256;               // IC systems above this size: multi-workgroup S^{-1} b
constexpr int WNS = 3;                        // rows per lane in the wavefront solves (n <= 192)
constexpr int GRAM_G = 32;                    // points per Gram step
constexpr int GRAM_SLOTS = 8;                 // observation slots per point per load pass
constexpr int GRAM_EMAX = 6 * (MAX_HOST_TARGETS + 1);

__device__ __forceinline__ double sym21(const double *u, int a, int b) {
    // upper triangle (row-major) of a symmetric 6x6
    if (a > b) {
        int t = a;
        a = b;
        b = t;
    }
    return u[a * 6 - a * (a - 1) / 2 + (b - a)];
}

// X^T H Y entry (r, c) for 6x6 X, Y and H given by its upper triangle.
__device__ __forceinline__ double xthy(const double *X, const double *H21, const double *Y, int r, int c) {
    double s = 0.0;
    for (int a = 0; a < 6; ++a) {
        double t = 0.0;
        for (int b = 0; b < 6; ++b) t += sym21(H21, a, b) * Y[b * 6 + c];
        s += X[a * 6 + r] * t;
    }
    return s;
}

// Fixed-order block sum of NV doubles per thread (up to 16 wavefronts): a
// butterfly in every wavefront, then one over the wavefront partials in
// wavefront 0; result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum_d(double v[NV], double *lds /* [NV * 16] */) {
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

__global__ void k_fill(double *__restrict__ p, size_t n, double v, const int *__restrict__ gate) {
    if (gate && *gate == 0) return;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Per window (one block each): pair sums of the pose-pose blocks (chunk
// partials added in order) and the damping of the pose and depth diagonals:
// mu = damping_rel x mean diagonal of the window's undamped blocks (damping_rel
// when that mean is zero).
__global__ __launch_bounds__(1024) void k_mu(WinArgs wa, double damping, const int *__restrict__ pair_chunk_ptr,
                                             const double *__restrict__ partH, double *__restrict__ pairH,
                                             const double *__restrict__ geo, const double *__restrict__ Hdd,
                                             double *__restrict__ mu, const int *__restrict__ gate) {
    __shared__ double lds[2 * 16];
    __shared__ double hl[MU_LDS_PAIRS * 21];   // the pair sums, when the window's pairs fit
    if (*gate == 0) return;
    const int w = blockIdx.x;
    const int p0 = wa.pair_off[w], p1 = wa.pair_off[w + 1];
    const bool in_lds = p1 - p0 <= MU_LDS_PAIRS;
    for (int e = threadIdx.x; e < (p1 - p0) * 21; e += blockDim.x) {
        const int p = p0 + e / 21, k = e % 21;
        const int c0 = pair_chunk_ptr[p], c1 = pair_chunk_ptr[p + 1];
        double s = 0.0;
#pragma unroll 8
        for (int c = c0; c < c1; ++c) s += partH[21 * c + k];
        pairH[21 * p + k] = s;
        if (in_lds) hl[e] = s;
    }
    // the sums are read back from LDS (no wait for the global stores) unless
    // the window has more pairs than that holds
    if (!in_lds) __threadfence_block();
    __syncthreads();
    double v[2] = {0.0, 0.0};
    for (int e = threadIdx.x; e < (p1 - p0) * 6; e += blockDim.x) {
        const int p = p0 + e / 6, r = e % 6;
        double a[6], bcol[6];
        abs_map_columns(geo + GEO_STRIDE * p, r, a, bcol);
        const double *H = in_lds ? hl + 21 * (p - p0) : pairH + 21 * p;
        v[0] += quad6(a, H, a) + quad6(bcol, H, bcol);
    }
    const int n0 = wa.point_off[w], n1 = wa.point_off[w + 1];
#pragma unroll 8
    for (int n = n0 + threadIdx.x; n < n1; n += blockDim.x) v[1] += Hdd[n];
    block_sum_d<2>(v, lds);
    if (threadIdx.x == 0) {
        const int Fw = wa.frame_off[w + 1] - wa.frame_off[w], Nw = n1 - n0;
        const double mp = Fw > 0 ? v[0] / (6.0 * Fw) : 0.0, md = Nw > 0 ? v[1] / Nw : 0.0;
        mu[2 * w] = mp > 0.0 ? damping * mp : damping;
        mu[2 * w + 1] = md > 0.0 ? damping * md : damping;
    }
}

__global__ void k_damp_hdd(int N, double *__restrict__ Hdd, const double *__restrict__ mu,
                           const int *__restrict__ point_win, const int *__restrict__ gate) {
    if (*gate == 0) return;
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n < N) Hdd[n] += mu[2 * point_win[n] + 1];
}

// Coupling of every observation to its target and host poses in absolute
// coordinates, scaled for the Schur Gram: (A^T h_o, B^T h_o) / sqrt(H_dd,n).
// hc receives h_o itself, 6 contiguous values per observation, for the
// system's readers of h alone (the rhs pair sums and the depth step), which
// would otherwise take it out of the 40-value records.
template <typename T>
__global__ __launch_bounds__(256) void k_obs_map(int O, const int *__restrict__ obs_point,
                                                 const int *__restrict__ obs_pair, const T *__restrict__ rec,
                                                 const double *__restrict__ Hdd, const double *__restrict__ geo,
                                                 double *__restrict__ map, double *__restrict__ hc,
                                                 const int *__restrict__ gate) {
    if (*gate == 0) return;
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= O) return;
    const T *h = rec + (size_t)o * REC_STRIDE + REC_h;
    double hv[6], ua[6], ub[6];
    for (int a = 0; a < 6; ++a) hv[a] = (double)h[a];
    double2 *hco = reinterpret_cast<double2 *>(hc + 6 * (size_t)o);
    for (int a = 0; a < 3; ++a) hco[a] = make_double2(hv[2 * a], hv[2 * a + 1]);
    const double *g = geo + GEO_STRIDE * obs_pair[o];
    apply_At(g, hv, ua);
    apply_Bt(g, hv, ub);
    const double s = 1.0 / sqrt(Hdd[obs_point[o]]);
    double *m = map + 12 * (size_t)o;
    for (int a = 0; a < 6; ++a) {
        m[a] = ua[a] * s;
        m[6 + a] = ub[a] * s;
    }
}

// Depth Schur complement, one chunk of one host frame's points per block:
// T += U^T U with row n of U = [A_1^T h_1, ..., A_m^T h_m, sum_o B_o^T h_o] / sqrt(H_dd,n),
// the coupling of point n to each of the host's target frames and to the host,
// in absolute coordinates. T is E x E, E = 6 (m + 1). Every step stages U^T for
// GRAM_G points in LDS (E padded to a multiple of 16) and adds U^T U on FP64
// MFMA (v_mfma_f64_16x16x4, K = GRAM_G): each wavefront owns a fixed set of
// 16 x 16 output tiles whose accumulators stay in registers across the steps.
typedef double gram_f64x4 __attribute__((ext_vector_type(4)));
constexpr int GRAM_EP = (GRAM_EMAX + 15) / 16 * 16;   // padded E
constexpr int GRAM_TP = GRAM_G + 1;                   // LDS pitch of U^T rows
constexpr int GRAM_TILES = (GRAM_EP / 16) * (GRAM_EP / 16);
constexpr int GRAM_TPW = (GRAM_TILES + 3) / 4;        // output tiles per wavefront (4 wavefronts)

__global__ __launch_bounds__(256) void k_gram(const int *__restrict__ chunk_host, const int *__restrict__ chunk_begin,
                                              const int *__restrict__ chunk_end, const int *__restrict__ chunk_off,
                                              const int *__restrict__ host_m, const int *__restrict__ host_pts,
                                              const int *__restrict__ obs_ptr, const int *__restrict__ obs_pair,
                                              const int *__restrict__ pair_local, const double *__restrict__ map,
                                              double *__restrict__ gram, const int *__restrict__ gate) {
    static_assert(GRAM_G % 4 == 0, "MFMA K steps of 4 points");
    __shared__ double ut[GRAM_EP * GRAM_TP];
    __shared__ double ub[GRAM_G][GRAM_SLOTS][6];
    if (*gate == 0) return;
    const int c = blockIdx.x;
    const int m = host_m[chunk_host[c]];
    const int E = 6 * (m + 1);
    const int nt = (E + 15) / 16;
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
    gram_f64x4 acc[GRAM_TPW];
#pragma unroll
    for (int k = 0; k < GRAM_TPW; ++k) acc[k] = gram_f64x4{0.0, 0.0, 0.0, 0.0};
    for (int base = chunk_begin[c]; base < chunk_end[c]; base += GRAM_G) {
        const int G = min(GRAM_G, chunk_end[c] - base);
        for (int e = threadIdx.x; e < 16 * nt * GRAM_TP; e += blockDim.x) ut[e] = 0.0;
        __syncthreads();
        {
            // one observation slot per thread: its target block goes straight to
            // U^T, its host block is summed over the point's observations below
            const int q = threadIdx.x / GRAM_SLOTS, slot = threadIdx.x % GRAM_SLOTS;
            double hb[6] = {0, 0, 0, 0, 0, 0};
            if (q < G) {
                const int n = host_pts[base + q];
                for (int o = obs_ptr[n] + slot; o < obs_ptr[n + 1]; o += GRAM_SLOTS) {
                    const double *mo = map + 12 * (size_t)o;
                    const int i6 = 6 * pair_local[obs_pair[o]];
                    for (int r = 0; r < 6; ++r) {
                        ut[(i6 + r) * GRAM_TP + q] = mo[r];
                        hb[r] += mo[6 + r];
                    }
                }
            }
            for (int r = 0; r < 6; ++r) ub[q][slot][r] = hb[r];
        }
        __syncthreads();
        if (threadIdx.x < GRAM_G * 6) {
            const int q = threadIdx.x / 6, r = threadIdx.x % 6;
            double s = 0.0;
            for (int k = 0; k < GRAM_SLOTS; ++k) s += ub[q][k][r];
            ut[(6 * m + r) * GRAM_TP + q] = s;
        }
        __syncthreads();
        // tile t = (I, J) of U^T U: rows 16 I .., columns 16 J .. of T
#pragma unroll
        for (int k = 0; k < GRAM_TPW; ++k) {
            const int t = wv + 4 * k;
            if (t < nt * nt) {
                const int I = t / nt, J = t % nt;
                gram_f64x4 a4 = acc[k];
#pragma unroll
                for (int s = 0; s < GRAM_G / 4; ++s) {
                    const double av = ut[(16 * I + (l & 15)) * GRAM_TP + 4 * s + (l >> 4)];
                    const double bv = ut[(16 * J + (l & 15)) * GRAM_TP + 4 * s + (l >> 4)];
                    a4 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, a4, 0, 0, 0);
                }
                acc[k] = a4;
            }
        }
        __syncthreads();
    }
    // element i of lane l: row 16 I + l / 16 + 4 i, column 16 J + l % 16
#pragma unroll
    for (int k = 0; k < GRAM_TPW; ++k) {
        const int t = wv + 4 * k;
        if (t < nt * nt) {
            const int I = t / nt, J = t % nt;
            const int col = 16 * J + (l & 15);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * I + (l >> 4) + 4 * i;
                if (row < E && col < E) gram[(size_t)chunk_off[c] + (size_t)row * E + col] = acc[k][i];
            }
        }
    }
}

// Reduced pose system S = H_pp + mu_p I - sum_n h_n h_n^T / H_dd,n, one nonzero
// 6x6 block per workgroup: mapped pair blocks (A^T H A, B^T H B, A^T H B, B^T H A)
// minus the host Gram blocks, then the gauge pin (identity rows / columns) of
// the window's pinned frame; written into the window's diagonal block of S.
__global__ __launch_bounds__(64) void k_assemble_s(WinArgs wa, int pinned, const int *__restrict__ blk_fa,
                                                   const int *__restrict__ blk_fb, const int *__restrict__ pp_ptr,
                                                   const int *__restrict__ pp_item, const int *__restrict__ g_ptr,
                                                   const int *__restrict__ g_item, const int *__restrict__ host_m,
                                                   const int *__restrict__ host_chunk_ptr,
                                                   const int *__restrict__ chunk_off, const double *__restrict__ pairH,
                                                   const double *__restrict__ geo, const double *__restrict__ gram,
                                                   const double *__restrict__ mu, double *__restrict__ S,
                                                   double *__restrict__ Sfac, const int *__restrict__ gate) {
    if (*gate == 0) return;
    const int b = blockIdx.x;
    if (threadIdx.x >= 36) return;
    const int r = threadIdx.x / 6, c = threadIdx.x % 6;
    const int fa = blk_fa[b], fb = blk_fb[b];
    const int w = wa.frame_win[fa], f0 = wa.frame_off[w], nw = 6 * (wa.frame_off[w + 1] - f0);
    const int la = fa - f0, lb = fb - f0;
    double val = 0.0;
    const int i0 = pp_ptr[b], i1 = pp_ptr[b + 1];
#pragma unroll 2
    for (int i = i0; i < i1; ++i) {
        const int p = pp_item[i] >> 2, kind = pp_item[i] & 3;
        double ar[6], br[6], ac[6], bc[6], x[6], y[6];
        abs_map_columns(geo + GEO_STRIDE * p, r, ar, br);
        abs_map_columns(geo + GEO_STRIDE * p, c, ac, bc);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            x[k] = (kind == 0 || kind == 2) ? ar[k] : br[k];
            y[k] = (kind == 0 || kind == 3) ? ac[k] : bc[k];
        }
        val += quad6(x, pairH + 21 * p, y);
    }
    for (int i = g_ptr[b]; i < g_ptr[b + 1]; ++i) {
        const int it = g_item[i];
        const int hi = it >> 12, a = (it >> 6) & 63, bb = it & 63;
        const int E = 6 * (host_m[hi] + 1);
        const size_t idx = (size_t)(6 * a + r) * E + 6 * bb + c;
        const int ch0 = host_chunk_ptr[hi], ch1 = host_chunk_ptr[hi + 1];
#pragma unroll 8
        for (int ch = ch0; ch < ch1; ++ch) val -= gram[(size_t)chunk_off[ch] + idx];
    }
    if (fa == fb && r == c) val += mu[2 * w];
    if (pinned >= 0 && (la == pinned || lb == pinned)) val = (fa == fb && r == c) ? 1.0 : 0.0;
    const size_t at = (size_t)wa.S_off[w] + (size_t)(6 * la + r) * nw + 6 * lb + c;
    S[at] = val;
    if (Sfac) Sfac[at] = val;   // one tiled window: the factorization's working copy
}

// ---- dense SPD helpers for one workgroup of SOLVE_THREADS threads (packed
// lower triangle in LDS, or the full row-major matrix in global memory when it
// does not fit)

struct PackedLds {
    double *p;
    __device__ double &operator()(int i, int j) const { return p[i * (i + 1) / 2 + j]; }
};
// L L^T x = b on one wavefront without barriers: lane l owns rows l, l+64, l+128
// and keeps them in registers; invd holds 1 / L(k, k). Forward substitution may
// start at row k0 when b is zero above it.
template <class M>
__device__ void wave_chol_solve(M L, const double *invd, int n, double (&x)[WNS], int k0) {
    const int lane = threadIdx.x & 63;
    for (int k = k0; k < n; ++k) {
        const int s = k >> 6, src = k & 63;
        double bk = 0.0;
#pragma unroll
        for (int q = 0; q < WNS; ++q)
            if (q == s) bk = __shfl(x[q], src, 64);
        const double yk = bk * invd[k];
#pragma unroll
        for (int q = 0; q < WNS; ++q) {
            const int i = lane + 64 * q;
            if (i == k)
                x[q] = yk;
            else if (i > k && i < n)
                x[q] -= L(i, k) * yk;
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        const int s = k >> 6, src = k & 63;
        double yk = 0.0;
#pragma unroll
        for (int q = 0; q < WNS; ++q)
            if (q == s) yk = __shfl(x[q], src, 64);
        const double xk = yk * invd[k];
#pragma unroll
        for (int q = 0; q < WNS; ++q) {
            const int i = lane + 64 * q;
            if (i == k)
                x[q] = xk;
            else if (i < k)
                x[q] -= L(k, i) * xk;
        }
    }
}

// ---- blocked Cholesky of a packed lower triangle held in LDS (n <= 192),
// panel width CHOL_NB: a single wavefront factors each diagonal block without
// barriers, one thread per row solves the panel below it, and the trailing
// update runs on a 32 x 32 thread grid that reads a transposed copy of the
// panel (consecutive rows contiguous, so the reads are conflict-free).
constexpr int CHOL_NB = 16;

__device__ __forceinline__ int pidx(int i, int j) { return i * (i + 1) / 2 + j; }

// A: packed lower triangle (LDS), panel: CHOL_NB * n doubles of LDS scratch,
// invd: n doubles (LDS or global) receiving 1 / L(k, k), fail: LDS flag.
// Returns false in every thread if a pivot is not positive.
__device__ __forceinline__ bool chol_blocked(double *A, int n, double *panel, double *invd, int *fail) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int tr = threadIdx.x >> 5, tc = threadIdx.x & 31;
    if (threadIdx.x == 0) *fail = 0;
    __syncthreads();
    for (int k0 = 0; k0 < n; k0 += CHOL_NB) {
        const int kb = min(CHOL_NB, n - k0);
        if (wv == 0) {
            for (int j = 0; j < kb; ++j) {
                const double p = A[pidx(k0 + j, k0 + j)];
                if (!(p > 0.0)) {
                    if (lane == 0) *fail = 1;
                    break;
                }
                const double l = sqrt(p), inv = 1.0 / l;
                double aij = 0.0;
                if (lane > j && lane < kb) {
                    aij = A[pidx(k0 + lane, k0 + j)] * inv;
                    A[pidx(k0 + lane, k0 + j)] = aij;
                }
                if (lane == j) {
                    A[pidx(k0 + j, k0 + j)] = l;
                    invd[k0 + j] = inv;
                }
                __builtin_amdgcn_wave_barrier();
                if (lane > j && lane < kb)
                    for (int c = j + 1; c <= lane; ++c) A[pidx(k0 + lane, k0 + c)] -= aij * A[pidx(k0 + c, k0 + j)];
                __builtin_amdgcn_wave_barrier();
            }
        }
        __syncthreads();
        if (*fail) return false;
        const int k1 = k0 + kb, m = n - k1;
        // rows below the block: x L11^T = a, kept in the transposed panel
        for (int r = threadIdx.x; r < m; r += blockDim.x) {
            const int i = k1 + r;
            double x[CHOL_NB];
#pragma unroll
            for (int c = 0; c < CHOL_NB; ++c) x[c] = c < kb ? A[pidx(i, k0 + c)] : 0.0;
#pragma unroll
            for (int c = 0; c < CHOL_NB; ++c) {
                if (c < kb) {
                    double s = x[c];
#pragma unroll
                    for (int q = 0; q < c; ++q) s -= x[q] * A[pidx(k0 + c, k0 + q)];
                    x[c] = s * invd[k0 + c];
                    A[pidx(i, k0 + c)] = x[c];
                    panel[c * n + r] = x[c];
                }
            }
        }
        __syncthreads();
        // trailing update A22 -= L21 L21^T (lower entries)
        for (int ia = tr; ia < m; ia += 32) {
            double xi[CHOL_NB];
#pragma unroll
            for (int c = 0; c < CHOL_NB; ++c) xi[c] = c < kb ? panel[c * n + ia] : 0.0;
            for (int jb = tc; jb <= ia; jb += 32) {
                double s = 0.0;
#pragma unroll
                for (int c = 0; c < CHOL_NB; ++c)
                    if (c < kb) s += xi[c] * panel[c * n + jb];
                A[pidx(k1 + ia, k1 + jb)] -= s;
            }
        }
        __syncthreads();
    }
    return true;
}

// IC setup: Cholesky factorization of S, once per level (the paper's "H need
// only be inverted once"), one window per workgroup. The factor is stored
// packed (lower, row-major) followed by 1 / L(k, k).
__global__ __launch_bounds__(SOLVE_THREADS) void k_ic_factor(WinArgs wa, double *__restrict__ S_all,
                                                             double *__restrict__ L_all, int *__restrict__ flag,
                                                             const int *__restrict__ gate) {
    __shared__ double lds[LDS_DOUBLES];
    __shared__ int fail;
    if (*gate == 0) return;
    const int w = blockIdx.x;
    const int n = 6 * (wa.frame_off[w + 1] - wa.frame_off[w]);
    const double *S = S_all + wa.S_off[w];
    double *Lout = L_all + wa.L_off[w];
    const int np = n * (n + 1) / 2;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e % n;
        if (j <= i) lds[pidx(i, j)] = S[e];
    }
    __syncthreads();
    if (!chol_blocked(lds, n, lds + np, Lout + np, &fail)) {
        if (threadIdx.x == 0) *flag = 1;
        return;
    }
    for (int e = threadIdx.x; e < np; e += blockDim.x) Lout[e] = lds[e];
}

// IC setup: S^{-1} = L^{-T} L^{-1} from the packed factor, one column per
// wavefront over ceil(n / 16) workgroups per window (each holds the factor in
// LDS). With S^{-1} stored, every iteration's step is one matrix-vector product.
__global__ __launch_bounds__(SOLVE_THREADS) void k_ic_inverse(WinArgs wa, const double *__restrict__ L_all,
                                                              double *__restrict__ Sinv_all,
                                                              const int *__restrict__ flag,
                                                              const int *__restrict__ gate) {
    __shared__ double lds[LDS_DOUBLES];
    if (*gate == 0 || *flag) return;
    const int w = blockIdx.y;
    const int n = 6 * (wa.frame_off[w + 1] - wa.frame_off[w]);
    if ((int)blockIdx.x * (SOLVE_THREADS / 64) >= n) return;
    const double *Lfac = L_all + wa.L_off[w];
    double *Sinv = Sinv_all + wa.S_off[w];
    const int np = n * (n + 1) / 2;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int e = threadIdx.x; e < np + n; e += blockDim.x) lds[e] = Lfac[e];
    __syncthreads();
    const int c = blockIdx.x * (SOLVE_THREADS / 64) + wv;
    if (c >= n) return;
    double x[WNS];
#pragma unroll
    for (int q = 0; q < WNS; ++q) x[q] = (lane + 64 * q == c) ? 1.0 : 0.0;
    wave_chol_solve(PackedLds{lds}, lds + np, n, x, c);
#pragma unroll
    for (int q = 0; q < WNS; ++q) {
        const int i = lane + 64 * q;
        if (i < n) Sinv[(size_t)c * n + i] = x[q];
    }
}

void launch_ic_inverse(hipStream_t s, Ctx &c) {
    if (c.tiled()) {
        launch_tinv(s, c);
        return;
    }
    int nmax = 0;
    for (int w = 0; w < c.nwin; ++w) nmax = std::max(nmax, 6 * (c.win_frame_off[w + 1] - c.win_frame_off[w]));
    const dim3 grid((nmax + SOLVE_THREADS / 64 - 1) / (SOLVE_THREADS / 64), c.nwin);
    k_ic_inverse<<<grid, SOLVE_THREADS, 0, s>>>(c.win(), c.d_Lfac, c.d_Sinv, c.d_flag, c.d_gate);
}

// Paths of the per-iteration solve, one kernel instance each (so that each
// gets a register allocation of its own).
enum SolvePath { SOLVE_IC = 0, SOLVE_FC_PACKED = 1, SOLVE_FC_TILED = 2 };

// IC window cache at the top of the solve's LDS. Doubles: current poses [12 F],
// p(0) poses [12 F], pair geometry at the linearization [GEO_STRIDE P], dtheta
// [n rounded up to even], pair sums [9 P]; then ints: window-local host
// and target frame of every pair [2 P], the frames' item pointers [F + 1], the
// pairs' chunk pointers [P + 1] and the frames' items [2 P] (a window's items
// are its pairs' host and target entries, so they start at 2 p0).
// With pair_out (the fused IC step), every pair's next geometry and relative
// step [P][GEO_STRIDE + 6] sit above the cache, at the very top of LDS.
__host__ __device__ inline int solve_out_doubles(int P, bool pair_out) { return pair_out ? (GEO_STRIDE + 6) * P : 0; }
__host__ __device__ inline int solve_cache_doubles(int F, int P, bool pair_out = false) {
    const int nq = (6 * F + 1) & ~1;
    const int ints = 2 * P + (F + 1) + (P + 1) + 2 * P;
    return 24 * F + GEO_STRIDE * P + nq + 9 * P + (ints + 1) / 2 + solve_out_doubles(P, pair_out);
}

// Batched copy of the concatenation of NS global segments (segment s starts
// at src[s] and ends at the cumulative length end[s]) into LDS, K elements per
// thread per batch: fetch() issues the first batch into registers, store()
// writes it and copies any further batches. Elements past the end are not
// loaded (a load under an inactive mask moves no data); the first nsub
// elements are stored less sub.
template <int NS, int K, typename V>
struct LdsGather {
    const V *src[NS];
    int end[NS];
    const V *dummy;
    V v[K];
    __device__ __forceinline__ void fetch(int b) {
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const int e = b + (int)threadIdx.x + u * SOLVE_THREADS;
            const V *p = dummy;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int beg = s ? end[s - 1] : 0;
                p = (e >= beg && e < end[s]) ? src[s] + (e - beg) : p;
            }
            v[u] = V(0);
            if (e < end[NS - 1]) v[u] = *p;
        }
    }
    __device__ __forceinline__ void put(V *dst, int b, V sub, int nsub) {
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const int e = b + (int)threadIdx.x + u * SOLVE_THREADS;
            if (e < end[NS - 1]) dst[e] = e < nsub ? v[u] - sub : v[u];
        }
    }
    __device__ __forceinline__ void store(V *dst, V sub, int nsub) {
        put(dst, 0, sub, nsub);
        for (int b = K * SOLVE_THREADS; b < end[NS - 1]; b += K * SOLVE_THREADS) {
            fetch(b);
            put(dst, b, sub, nsub);
        }
    }
};

// Keeps a wave-uniform value's load ahead of this point (so that the loads of
// one batch are not split by a later branch).
template <typename V>
__device__ __forceinline__ void pin_sreg(V v) {
    asm volatile("" ::"s"(v));
}

// S^{-1} entries that every thread of the IC product (up to IC_SPLIT_N
// unknowns) prefetches at the start: SV_REG rows in registers, up to SV_LDS
// more in a thread-private LDS area.
constexpr int SV_REG = 21, SV_LDS = 15;

// One solve per iteration and window (one workgroup each):
//  0. pair sums of the reduced gradient from their chunk partials;
//  1. reduced right-hand side b_f = sum over the frame's pairs of A^T y (target) or
//     B^T y (host), zero on the window's pinned frame;
//  2. dtheta = -S^{-1} b (IC: product with the stored inverse; FC: Cholesky of
//     the freshly assembled S and two triangular solves);
//  3. pose update: IC R <- R_k R0^T exp(dw)^T R0, t <- t_k - R_k R0^T dt (Sec. 3.6);
//     FC R <- exp(dw) R, t <- t + dt;
//  4. the next relative poses of every pair and the relative steps A dth_f + B dth_h.
// Window statistics (energy, squared residuals, count, largest pose step) go
// to wstat[w]; the convergence kernel adds them over the windows.
// With CACHE (IC), one batch of loads at the start brings every input that no
// other load feeds (poses, pair geometry, the index lists and, up to
// IC_SPLIT_N unknowns, S^{-1}) into LDS and registers, so that the only
// dependent global loads left are the chunk partials. A single window's ranges
// come as arguments (one_F >= 0: frames and pairs from 0), others' are loaded.
template <typename T, int PATH, bool CACHE>
__device__ __forceinline__ bool solve_window(
    double *lds, double *red, bool writer, bool pair_out, WinArgs wa, int one_F, int one_P, int pinned, int stage, const int *__restrict__ frame_pair_ptr,
    const int *__restrict__ frame_pair_item, const int *__restrict__ pair_host, const int *__restrict__ pair_target,
    const int *__restrict__ pair_chunk_ptr, const double *__restrict__ partY, double *__restrict__ pairY,
    const double *__restrict__ geo_lin, const double *__restrict__ S_all, const double *__restrict__ Sfac,
    const double *__restrict__ Linv, const double *__restrict__ Sinv_all, double *poses,
    const double *__restrict__ poses0, double *__restrict__ b_all, double *__restrict__ dth_all,
    double *__restrict__ dth_rel, double *__restrict__ geo_next, T *__restrict__ rel_next,
    double *__restrict__ wstat, int *__restrict__ flag, int *__restrict__ gate, double *poses_out,
    const int *__restrict__ sel = nullptr, int sel_ncw = 0, int one_nch = -1) {
    constexpr bool ic = PATH == SOLVE_IC, tiled = PATH == SOLVE_FC_TILED, packed = PATH == SOLVE_FC_PACKED;
    static_assert(ic || !CACHE, "the LDS cache serves the IC path");

    // the gate, the failure flag and the window's ranges
    const int w = blockIdx.x;
    const int gv = *gate, fv = *flag;
    int f0 = 0, fe = one_F, p0 = 0, p1 = one_P, soff = 0;
    if (one_F < 0) {
        f0 = wa.frame_off[w];
        fe = wa.frame_off[w + 1];
        p0 = wa.pair_off[w];
        p1 = wa.pair_off[w + 1];
        soff = wa.S_off[w];
        pin_sreg(f0);
        pin_sreg(fe);
        pin_sreg(p0);
        pin_sreg(p1);
        pin_sreg(soff);
    }

    const int F = fe - f0, P = p1 - p0;
    const int n = 6 * F, nq = (n + 1) & ~1;
    const double *S = S_all + soff;
    const double *Sinv = Sinv_all + soff;
    double *b_out = b_all + 6 * f0;
    double *dth_out = dth_all + 6 * f0;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    // rhs / solution in LDS (FC packed: after the packed factor; the panel scratch follows)
    double *bx = lds + (packed ? n * (n + 1) / 2 : 0);
    // IC product layout up to IC_SPLIT_N unknowns: thread (g, j) takes column j
    // and rows g + NG u; group partials after bx
    // and rows g + NG u; group partials after bx. With sel (IC cache path), only
    // the columns of the listed frames: sel = [count, frames ..., mask (2 ints)]
    // at stride STEP_SEL_STRIDE, column slot k of thread (g, k) the (k % 6)-th
    // unknown of frame sel[1 + k / 6], sel_ncw slots per group
    const bool subset = CACHE && sel != nullptr;
    const int ncw = subset ? sel_ncw : (n + 63) & ~63;
    const int NG = ncw ? SOLVE_THREADS / ncw : 1;
    const int mg = threadIdx.x / max(ncw, 1), mk = threadIdx.x % max(ncw, 1);
    int nsel = F, mj = mk;
    unsigned long long fmask = ~0ull;
    if (subset) {
        nsel = sel[0];
        fmask = (unsigned long long)(unsigned)sel[STEP_SEL_STRIDE - 2] |
                ((unsigned long long)(unsigned)sel[STEP_SEL_STRIDE - 1] << 32);
        mj = 6 * sel[1 + min(mk / 6, STEP_SEL_STRIDE - 4)] + mk % 6;   // slots past the list: frame 0, unused
    }
    const int ncols = 6 * nsel;   // product columns (n without sel)
    double *const part = bx + nq;

    // the cache (IC) and its end; scratch of the steps stays below it
    double *const ctop = CACHE ? lds + LDS_DOUBLES - solve_cache_doubles(F, P, pair_out) : lds + LDS_DOUBLES;
    double *const c_out = lds + LDS_DOUBLES - solve_out_doubles(P, pair_out);   // [P][GEO_STRIDE], then [P][6]
    double *const c_pose = ctop, *const c_pose0 = c_pose + 12 * F, *const c_geo = c_pose0 + 12 * F;
    double *const c_dth = c_geo + GEO_STRIDE * P, *const c_y = c_dth + nq;
    int *const c_host = reinterpret_cast<int *>(c_y + 9 * P), *const c_target = c_host + P;
    int *const c_fptr = c_target + P, *const c_cptr = c_fptr + F + 1, *const c_item = c_cptr + P + 1;
    // S^{-1} prefetch (CACHE, up to IC_SPLIT_N unknowns): SV_REG rows per
    // thread in registers, then ul more in LDS after the group partials (the
    // right-hand side's item maps then stay below them); ul is a multiple of 3
    const bool pre = CACHE && n <= IC_SPLIT_N;
    double *const c_sinv = part + SOLVE_THREADS;
    // (with sel every row fits the registers: the LDS rows then hold the staged
    // chunk partials instead)
    const int ul = (pre && !subset) ? min(SV_LDS, (int)((ctop - c_sinv) / SOLVE_THREADS)) / 3 * 3 : 0;
    const double *yl = nullptr;   // staged chunk partials
    double sv[SV_REG];
    if constexpr (CACHE) {
        LdsGather<4, 2, double> gd{{poses + 12 * f0, poses0 + 12 * f0, geo_lin + GEO_STRIDE * p0, dth_out},
                                   {12 * F, 24 * F, 24 * F + GEO_STRIDE * P, 24 * F + GEO_STRIDE * P + (stage == 2 ? n : 0)},
                                   wstat + 4 * w};
        LdsGather<5, 1, int> gi{{pair_host + p0, pair_target + p0, frame_pair_ptr + f0, pair_chunk_ptr + p0,
                                 frame_pair_item + 2 * p0},
                                {P, 2 * P, 2 * P + F + 1, 3 * P + F + 2, 5 * P + F + 2},
                                gate};
        gd.fetch(0);
        gi.fetch(0);
        // (sel, one window with one_nch chunks) the chunk partials of the pair
        // sums too, into the LDS rows that a column subset leaves unused
        const bool stage_y = subset && one_nch >= 0 && 9 * one_nch <= (int)(ctop - c_sinv);
        LdsGather<1, 3, double> gy{{partY}, {stage_y ? 9 * one_nch : 0}, wstat + 4 * w};
        if (stage_y) gy.fetch(0);
        const bool col = mg < NG && mk < ncols;
        double sl[SV_LDS];
#pragma unroll
        for (int u = 0; u < SV_LDS; ++u) sl[u] = 0.0;
#pragma unroll
        for (int u = 0; u < SV_REG; ++u) sv[u] = 0.0;
        if (pre) {
            // entries outside the rows, columns or LDS rows are not loaded (the
            // registers were zeroed first, so no load waits on another)
#pragma unroll
            for (int u = 0; u < SV_LDS; ++u) {
                const int i = mg + NG * (SV_REG + u);
                if (col && u < ul && i < n) sl[u] = Sinv[(size_t)i * n + mj];
            }
#pragma unroll
            for (int u = 0; u < SV_REG; ++u) {
                const int i = mg + NG * u;
                if (col && i < n) sv[u] = Sinv[(size_t)i * n + mj];
            }
        }
        if (gv == 0) return false;
        if (fv) {
            if (writer && threadIdx.x == 0) *gate = 0;
            return false;
        }
        gd.store(c_pose, 0.0, 0);
        gi.store(c_host, f0, 2 * P);
        if (stage_y) {
            gy.store(c_sinv, 0.0, 0);
            yl = c_sinv;
        }
#pragma unroll
        for (int u = 0; u < SV_LDS; ++u)
            if (u < ul) c_sinv[u * SOLVE_THREADS + threadIdx.x] = sl[u];
#pragma unroll
        for (int u = 0; u < SV_REG; ++u) pin_reg(sv[u]);
        __syncthreads();
    } else {
        if (gv == 0) return false;
        if (fv) {
            // a factorization of this iteration failed: stop the batch
            if (threadIdx.x == 0) *gate = 0;
            return false;
        }
    }
    auto fptr = [&](int f) { return CACHE ? c_fptr[f - f0] : frame_pair_ptr[f]; };
    auto geo_of = [&](int p) { return CACHE ? c_geo + GEO_STRIDE * (p - p0) : geo_lin + GEO_STRIDE * p; };

    // stage 0: the whole step; stage 1: up to the right-hand side b; stage 2:
    // from dtheta (formed between the stages by k_ic_matvec) to the pose update
    // with the cache, every global store of the step waits for the end of the
    // kernel (results stay in LDS and registers until then)
    double v3[3] = {0.0, 0.0, 0.0};
    if (stage != 2) {
    {
        // pair sums of the chunk partials (chunks in order; loads unrolled so
        // that a pair's chunks are fetched together), and the window's energy
        // statistics as a fixed-order block sum of the pair sums
        for (int e = threadIdx.x; e < P * 9; e += blockDim.x) {
            const int pl = e / 9, k = e % 9;
            const int c0 = CACHE ? c_cptr[pl] : pair_chunk_ptr[p0 + pl];
            const int c1 = CACHE ? c_cptr[pl + 1] : pair_chunk_ptr[p0 + pl + 1];
            double s = 0.0;
            const double *py = yl ? yl : partY;
#pragma unroll 8
            for (int c = c0; c < c1; ++c) s += py[9 * c + k];
            if (CACHE)
                c_y[9 * pl + k] = s;
            else
                pairY[9 * (p0 + pl) + k] = s;
            if (k >= 6) v3[k - 6] += s;
        }
        // global pair sums are read back below only without the cache
        if constexpr (!CACHE) __threadfence_block();
        // the statistics only where they are stored (the barrier either way)
        if (writer)
            block_sum_d<3>(v3, red);
        else
            __syncthreads();
        if (!CACHE && threadIdx.x == 0) {
            wstat[4 * w + 0] = v3[0];
            wstat[4 * w + 1] = v3[1];
            wstat[4 * w + 2] = v3[2];
        }
    }
    // b = sum over the frame's pair items of A_p^T y_p (target) or B_p^T y_p (host),
    // items added in list order. The item maps are formed in parallel into LDS
    // (in chunks of what fits beside the rhs), then every row adds its frame's
    // items of the chunk; rows of the pinned frame stay zero.
    {
        double *cb = bx + nq;
        const int cap_items = (int)(((pre ? c_sinv : ctop) - cb) / 6);
        const int i0 = fptr(f0), i1 = fptr(f0 + F);
        for (int e = threadIdx.x; e < n; e += blockDim.x) bx[e] = 0.0;
        for (int c0 = i0; c0 < i1; c0 += cap_items) {
            const int c1 = min(i1, c0 + cap_items);
            for (int i = c0 + threadIdx.x; i < c1; i += blockDim.x) {
                const int it = CACHE ? c_item[i - i0] : frame_pair_item[i];
                const int p = it >> 1, is_host = it & 1;
                double yv[6], out[6];
                for (int a = 0; a < 6; ++a) yv[a] = CACHE ? c_y[9 * (p - p0) + a] : pairY[9 * p + a];
                if (is_host)
                    apply_Bt(geo_of(p), yv, out);
                else
                    apply_At(geo_of(p), yv, out);
                double *o = cb + 6 * (i - c0);
                for (int a = 0; a < 6; ++a) o[a] = out[a];
            }
            __syncthreads();
            for (int e = threadIdx.x; e < n; e += blockDim.x) {
                const int lf = e / 6, r = e % 6, f = f0 + lf;
                if (lf == pinned) continue;
                const int a0 = max(c0, fptr(f)), a1 = min(c1, fptr(f + 1));
                double s = bx[e];
                for (int i = a0; i < a1; ++i) s += cb[6 * (i - c0) + r];
                bx[e] = s;
            }
            __syncthreads();
        }
        if (!CACHE)
            for (int e = threadIdx.x; e < n; e += blockDim.x) b_out[e] = bx[e];
    }
    __syncthreads();
    }
    // pair sums, right-hand side and energy statistics to global memory
    auto store_b = [&]() {
        for (int e = threadIdx.x; e < 9 * P; e += blockDim.x) pairY[9 * p0 + e] = c_y[e];
        for (int e = threadIdx.x; e < n; e += blockDim.x) b_out[e] = bx[e];
        if (threadIdx.x == 0) {
            wstat[4 * w + 0] = v3[0];
            wstat[4 * w + 1] = v3[1];
            wstat[4 * w + 2] = v3[2];
        }
    };
    if (stage == 1) {
        if (CACHE) store_b();
        return false;
    }
    if (stage == 2) {
        // dtheta is in global memory (and in the cache)
    } else if constexpr (ic) {
        // dtheta = -S^{-1} b with the inverse formed at p(0) (stored by
        // columns; S^{-1} is symmetric). Up to IC_SPLIT_N unknowns: NG groups
        // of threads, each thread one column j and every NG-th row i, so that
        // a wavefront reads 64 consecutive entries of a row; rows prefetched at
        // the start first (registers, then LDS), the rest loaded in batches of
        // 12; group partials added in group order.
        if (n <= IC_SPLIT_N) {
            const int g = mg, j = mj;
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
            if (g < NG && mk < ncols) {
                int u0 = 0;
                if (pre) {
#pragma unroll
                    for (int u = 0; u < SV_REG; u += 3) {
                        const int i = g + NG * u;
                        s0 += sv[u] * bx[min(i, n - 1)];
                        s1 += sv[u + 1] * bx[min(i + NG, n - 1)];
                        s2 += sv[u + 2] * bx[min(i + 2 * NG, n - 1)];
                    }
                    for (int u = 0; u < ul; u += 3) {
                        const int i = g + NG * (SV_REG + u);
                        const double *q = c_sinv + u * SOLVE_THREADS + threadIdx.x;
                        s0 += q[0] * bx[min(i, n - 1)];
                        s1 += q[SOLVE_THREADS] * bx[min(i + NG, n - 1)];
                        s2 += q[2 * SOLVE_THREADS] * bx[min(i + 2 * NG, n - 1)];
                    }
                    u0 = SV_REG + ul;
                }
                constexpr int U = 12;
                for (int i0 = g + NG * u0; i0 < n; i0 += U * NG) {
                    double v[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int i = i0 + u * NG;
                        v[u] = i < n ? Sinv[(size_t)i * n + j] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < U; u += 3) {
                        const int i = i0 + u * NG;
                        s0 += v[u] * (i < n ? bx[i] : 0.0);
                        s1 += v[u + 1] * (i + NG < n ? bx[i + NG] : 0.0);
                        s2 += v[u + 2] * (i + 2 * NG < n ? bx[i + 2 * NG] : 0.0);
                    }
                }
            }
            if (g < NG) part[g * ncw + mk] = (s0 + s1) + s2;
            __syncthreads();
            if (threadIdx.x < ncols) {
                // thread (0, k): its column j
                double s = 0.0;
                for (int q = 0; q < NG; ++q) s += part[q * ncw + threadIdx.x];
                if (CACHE)
                    c_dth[j] = -s;
                else
                    dth_out[j] = -s;
            }
        } else {
            for (int i = wv; i < n; i += nw) {
                const double *row = Sinv + (size_t)i * n;
                double s = 0.0;
#pragma unroll 8
                for (int j = lane; j < n; j += 64) s += row[j] * bx[j];
                s = wave_sum(s);
                if (lane == 0) {
                    if (CACHE)
                        c_dth[i] = -s;
                    else
                        dth_out[i] = -s;
                }
            }
        }
    } else if constexpr (packed) {
        // FC: factor the S assembled this iteration
        const int np = n * (n + 1) / 2;
        double *invd = red + 64;
        {
            for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
                const int i = e / n, j = e % n;
                if (j <= i) lds[pidx(i, j)] = S[e];
            }
            __syncthreads();
            if (!chol_blocked(lds, n, lds + np + n, invd, reinterpret_cast<int *>(red + 64 + LDS_MAX_N))) {
                if (threadIdx.x == 0) {
                    *flag = 1;
                    *gate = 0;
                }
                return false;
            }
        }
        if (wv == 0) {
            double x[WNS];
#pragma unroll
            for (int q = 0; q < WNS; ++q) {
                const int i = lane + 64 * q;
                x[q] = i < n ? bx[i] : 0.0;
            }
            wave_chol_solve(PackedLds{lds}, invd, n, x, 0);
#pragma unroll
            for (int q = 0; q < WNS; ++q) {
                const int i = lane + 64 * q;
                if (i < n) dth_out[i] = -x[q];
            }
        }
    } else {
        // FC, one window on the tiled path: S was factored in tiles before this kernel
        tile_chol_solve<SOLVE_THREADS>(Sfac, Linv, n, bx, lds + n, 0);
        for (int i = threadIdx.x; i < n; i += blockDim.x) dth_out[i] = -bx[i];
    }
    // with the cache, no thread reads back what this kernel stored globally:
    // a fence here would only wait for those stores
    if constexpr (!CACHE) __threadfence_block();
    __syncthreads();
    const double *dth = CACHE ? c_dth : dth_out;
    // largest pose step (where it is stored)
    if (writer) {
        double mx = 0.0;
        for (int i = threadIdx.x; i < n; i += blockDim.x) mx = fmax(mx, fabs(dth[i]));
        mx = wave_max(mx);
        if (lane == 0) red[wv] = mx;
    }
    // pose update
    for (int lf = threadIdx.x; lf < F; lf += blockDim.x) {
        if (!((fmask >> (lf & 63)) & 1ull)) continue;   // (sel) a frame whose step was not formed
        const double *x = dth + 6 * lf;
        const double *P = CACHE ? c_pose + 12 * lf : poses + 12 * (f0 + lf);
        double dR[9], Rn[9], tn[3];
        so3_exp(x, dR);
        if (ic) {
            const double *P0 = CACHE ? c_pose0 + 12 * lf : poses0 + 12 * (f0 + lf);
            double A[9], Q[9];
            mat3_mul_bt(P, P0, Q);  // R_k R0^T
            mat3_mul_bt(Q, dR, A);  // R_k R0^T dR^T
            mat3_mul(A, P0, Rn);    // ... R0
            for (int i = 0; i < 3; ++i) tn[i] = P[9 + i] - (Q[3 * i] * x[3] + Q[3 * i + 1] * x[4] + Q[3 * i + 2] * x[5]);
        } else {
            mat3_mul(dR, P, Rn);
            for (int i = 0; i < 3; ++i) tn[i] = P[9 + i] + x[3 + i];
        }
        double *Pn = CACHE ? c_pose + 12 * lf : poses + 12 * (f0 + lf);
        for (int i = 0; i < 9; ++i) Pn[i] = Rn[i];
        for (int i = 0; i < 3; ++i) Pn[9 + i] = tn[i];
    }
    if constexpr (!CACHE) __threadfence_block();
    __syncthreads();
    if (writer && wv == 0) {
        const double m2 = row_max16(lane < nw ? red[lane] : 0.0);
        if (lane == 0) wstat[4 * w + 3] = m2;
    }
    // next relative poses and relative steps per pair (frames window-local)
    const double *pose_w = CACHE ? c_pose : poses + 12 * f0;
    for (int p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
        const int h = CACHE ? c_host[p - p0] : pair_host[p] - f0;
        const int t = CACHE ? c_target[p - p0] : pair_target[p] - f0;
        const double *Ph = pose_w + 12 * h;
        const double *Pf = pose_w + 12 * t;
        double R[9];
        mat3_mul_bt(Pf, Ph, R);
        double tr[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) tr[i] = Pf[9 + i] - (R[3 * i] * Ph[9] + R[3 * i + 1] * Ph[10] + R[3 * i + 2] * Ph[11]);
        // geometry [R, t, t_host, 0] of the pair at the new poses
        auto put_geo = [&](double *g) {
#pragma unroll
            for (int i = 0; i < 9; ++i) g[i] = R[i];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                g[9 + i] = tr[i];
                g[12 + i] = Ph[9 + i];
            }
            g[15] = 0.0;
        };
        if (writer) {
            put_geo(geo_next + GEO_STRIDE * p);
            T *rl = rel_next + REL_STRIDE * p;
#pragma unroll
            for (int i = 0; i < 9; ++i) rl[i] = (T)R[i];
#pragma unroll
            for (int i = 0; i < 3; ++i) rl[9 + i] = (T)tr[i];
        }
        if (pair_out) put_geo(c_out + GEO_STRIDE * (p - p0));
        double xf[6], xh[6], af[6], bh[6];
        for (int a = 0; a < 6; ++a) {
            xf[a] = dth[6 * t + a];
            xh[a] = dth[6 * h + a];
        }
        apply_A(geo_of(p), xf, af);
        apply_B(geo_of(p), xh, bh);
        if (writer)
            for (int r = 0; r < 6; ++r) dth_rel[6 * p + r] = af[r] + bh[r];
        if (pair_out)
            for (int r = 0; r < 6; ++r) c_out[GEO_STRIDE * P + 6 * (p - p0) + r] = af[r] + bh[r];
    }
    if constexpr (CACHE) {
        if (writer) {
            if (stage == 0) {
                store_b();
                for (int e = threadIdx.x; e < n; e += blockDim.x) dth_out[e] = c_dth[e];
            }
            for (int e = threadIdx.x; e < 12 * F; e += blockDim.x) poses_out[12 * f0 + e] = c_pose[e];
        }
    }
    return true;
}

template <typename T, int PATH, bool CACHE>
__global__ __launch_bounds__(SOLVE_THREADS) void k_solve(
    WinArgs wa, int one_F, int one_P, int pinned, int stage, const int *__restrict__ frame_pair_ptr,
    const int *__restrict__ frame_pair_item, const int *__restrict__ pair_host, const int *__restrict__ pair_target,
    const int *__restrict__ pair_chunk_ptr, const double *__restrict__ partY, double *__restrict__ pairY,
    const double *__restrict__ geo_lin, const double *__restrict__ S_all, const double *__restrict__ Sfac,
    const double *__restrict__ Linv, const double *__restrict__ Sinv_all, double *__restrict__ poses,
    const double *__restrict__ poses0, double *__restrict__ b_all, double *__restrict__ dth_all,
    double *__restrict__ dth_rel, double *__restrict__ geo_next, T *__restrict__ rel_next,
    double *__restrict__ wstat, int *__restrict__ flag, int *__restrict__ gate) {
    __shared__ double lds[LDS_DOUBLES];
    __shared__ double red[64 + 2 * LDS_MAX_N + 2];
    solve_window<T, PATH, CACHE>(lds, red, true, false, wa, one_F, one_P, pinned, stage, frame_pair_ptr,
                                 frame_pair_item, pair_host, pair_target, pair_chunk_ptr, partY, pairY, geo_lin, S_all,
                                 Sfac, Linv, Sinv_all, poses, poses0, b_all, dth_all, dth_rel, geo_next, rel_next,
                                 wstat, flag, gate, poses);
}

static_assert(IC_STEP_PTS == SOLVE_THREADS / DU_SLOTS, "one depth workgroup of the fused IC step: 8 lanes per point");

// One IC iteration's solve and depth step in one launch (one window on the
// cache path, so that no kernel boundary separates them): every workgroup
// forms the step itself (the pair sums and S^{-1} b repeat cheaply from L2).
// Workgroup 0 stores the solve's results (the updated poses into poses_out, a
// buffer no workgroup of the launch reads) and has no points; workgroup
// b > 0 then updates the depths of points [(b - 1) IC_STEP_PTS, b IC_STEP_PTS)
// from the relative steps and poses of the pairs it holds in LDS, and part[b - 1]
// receives its maxima of the displacement and of the depth step.
template <typename T>
__global__ __launch_bounds__(SOLVE_THREADS) void k_ic_step(
    WinArgs wa, int one_F, int one_P, int pinned, const int *__restrict__ frame_pair_ptr,
    const int *__restrict__ frame_pair_item, const int *__restrict__ pair_host, const int *__restrict__ pair_target,
    const int *__restrict__ pair_chunk_ptr, const double *__restrict__ partY, double *__restrict__ pairY,
    const double *__restrict__ geo_lin, const double *__restrict__ Sinv_all, const double *__restrict__ poses_in,
    double *__restrict__ poses_out, const double *__restrict__ poses0, double *__restrict__ b_all,
    double *__restrict__ dth_all, double *__restrict__ dth_rel, double *__restrict__ geo_next,
    T *__restrict__ rel_next, double *__restrict__ wstat, int *__restrict__ flag, int *__restrict__ gate, int N,
    const int *__restrict__ obs_ptr, const int *__restrict__ obs_pair, const float *__restrict__ host_uv,
    const double *__restrict__ pairK0, const double *__restrict__ hc, const double *__restrict__ gd, int gds,
    const double *__restrict__ Hdd, const double *__restrict__ geo_old, double *__restrict__ depth,
    const double *__restrict__ depth0, double *__restrict__ part, const int *__restrict__ step_sel, int sel_ncw,
    int nch, const uint8_t *__restrict__ live) {
    __shared__ double lds[LDS_DOUBLES];
    __shared__ double red[64 + 2 * LDS_MAX_N + 2];
    const bool writer = blockIdx.x == 0;
    // a depth workgroup's point data, issued before the step (used after it)
    const int b = blockIdx.x - 1;
    DepthPoint pt{0, 0, 0.0, 0.0, 1.0, 0.0, 1.0};
    if (!writer) pt = depth_point<true>(N, b * IC_STEP_PTS, obs_ptr, host_uv, Hdd, depth, depth0);
    // a depth workgroup forms the step of the frames its points observe only
    const int *sel = (writer || sel_ncw == 0) ? nullptr : step_sel + (size_t)(blockIdx.x - 1) * STEP_SEL_STRIDE;
    if (!solve_window<T, SOLVE_IC, true>(lds, red, writer, !writer, wa, one_F, one_P, pinned, 0,
                                         frame_pair_ptr, frame_pair_item, pair_host, pair_target, pair_chunk_ptr,
                                         partY, pairY, geo_lin, nullptr, nullptr, nullptr, Sinv_all,
                                         const_cast<double *>(poses_in), poses0, b_all, dth_all, dth_rel, geo_next,
                                         rel_next, wstat, flag, gate, poses_out, sel, sel_ncw, nch))
        return;
    if (writer) return;
    __syncthreads();
    // the step's scratch is free now; the pairs' results stay at the top of LDS
    const int P = one_P;
    const double *c_out = lds + LDS_DOUBLES - solve_out_doubles(P, true);
    double md = 0.0, ms = 0.0;
    depth_points<T, SOLVE_THREADS>(N, b * IC_STEP_PTS, 1, pt, obs_pair, pairK0, hc, gd, gds, c_out + GEO_STRIDE * P,
                                   geo_old, c_out, depth, nullptr, nullptr, lds, md, ms, live);
    if (threadIdx.x == 0) {
        part[2 * b] = md;
        part[2 * b + 1] = ms;
    }
}

// dtheta = -S^{-1} b of one large window (IC between the two solve stages):
// one wavefront per row, lane loads unrolled so that several are in flight.
__global__ __launch_bounds__(256) void k_ic_matvec(int n, const double *__restrict__ Sinv, const double *__restrict__ b,
                                                   double *__restrict__ dth, const int *__restrict__ flag,
                                                   const int *__restrict__ gate) {
    if (*gate == 0 || *flag) return;
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    const double *row = Sinv + (size_t)i * n;
    double s = 0.0;
#pragma unroll 8
    for (int j = lane; j < n; j += 64) s += row[j] * b[j];
    s = wave_sum(s);
    if (lane == 0) dth[i] = -s;
}

// ------------------------------------------------------------ launchers

static inline unsigned nb(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

void launch_fill(hipStream_t s, double *p, size_t n, double v, const int *gate) {
    if (n == 0) return;
    k_fill<<<nb(n, 256), 256, 0, s>>>(p, n, v, gate);
}

void launch_mu(hipStream_t s, Ctx &c, const double *geo) {
    k_mu<<<c.nwin, 1024, 0, s>>>(c.win(), c.cfg.damping_rel, c.d_pair_chunk_ptr, c.d_partH, c.d_pairH, geo, c.d_Hdd,
                                 c.d_mu, c.d_gate);
    if (c.N) k_damp_hdd<<<nb(c.N, 256), 256, 0, s>>>(c.N, c.d_Hdd, c.d_mu, c.d_point_win, c.d_gate);
}

void launch_gram(hipStream_t s, Ctx &c, const double *geo, const void *rec, bool rec_double) {
    const int nch = (int)c.st.chunk_host.size();
    if (nch == 0 || c.O == 0) return;
    if (rec_double)
        k_obs_map<double><<<nb(c.O, 256), 256, 0, s>>>(c.O, c.d_obs_point, c.d_obs_pair, (const double *)rec,
                                                       c.d_Hdd, geo, c.d_obsmap, c.d_hc, c.d_gate);
    else
        k_obs_map<float><<<nb(c.O, 256), 256, 0, s>>>(c.O, c.d_obs_point, c.d_obs_pair, (const float *)rec,
                                                      c.d_Hdd, geo, c.d_obsmap, c.d_hc, c.d_gate);
    k_gram<<<nch, 256, 0, s>>>(c.d_chunk_host, c.d_chunk_begin, c.d_chunk_end, c.d_chunk_off, c.d_host_m,
                               c.d_host_pts, c.d_obs_ptr, c.d_obs_pair, c.d_pair_local, c.d_obsmap, c.d_gram,
                               c.d_gate);
}

void launch_assemble_s(hipStream_t s, Ctx &c, const double *geo) {
    // every block of every window's S is written (zeros where no pair or Gram
    // item contributes), so S needs no clearing pass
    const int nbk = (int)c.st.blk_fa.size();
    k_assemble_s<<<nbk, 64, 0, s>>>(c.win(), c.cfg.pinned_frame, c.d_blk_fa, c.d_blk_fb, c.d_blk_pp_ptr,
                                    c.d_blk_pp_item, c.d_blk_g_ptr, c.d_blk_g_item, c.d_host_m, c.d_host_chunk_ptr,
                                    c.d_chunk_off, c.d_pairH, geo, c.d_gram, c.d_mu, c.d_S,
                                    c.tiled() ? c.d_Sfac : nullptr, c.d_gate);
}

void launch_ic_factor(hipStream_t s, Ctx &c) {
    if (c.tiled()) {
        launch_tchol(s, c, false);   // the assembly wrote S into the factor buffer too
        return;
    }
    k_ic_factor<<<c.nwin, SOLVE_THREADS, 0, s>>>(c.win(), c.d_S, c.d_Lfac, c.d_flag, c.d_gate);
}

// Whether every window's IC cache fits in LDS beside the step's scratch and
// the windows' items start at twice their first pair.
static bool solve_cache_fits(const Ctx &c, bool pair_out = false) {
    const std::vector<int> &fp = c.st.frame_pair_ptr;
    if (c.win_frame_off.size() != (size_t)c.nwin + 1 || c.win_pair_off.size() != (size_t)c.nwin + 1) return false;
    for (int w = 0; w < c.nwin; ++w) {
        const int f0 = c.win_frame_off[w], f1 = c.win_frame_off[w + 1];
        const int p0 = c.win_pair_off[w], p1 = c.win_pair_off[w + 1];
        if ((size_t)f1 >= fp.size() || fp[f0] != 2 * p0 || fp[f1] != 2 * p1) return false;
        const int nq = (6 * (f1 - f0) + 1) & ~1;
        if (LDS_DOUBLES - solve_cache_doubles(f1 - f0, p1 - p0, pair_out) < nq + std::max(SOLVE_THREADS, 6 * 64))
            return false;
    }
    return true;
}

// One window starting at frame, pair and S offset 0 (its ranges go as arguments).
static bool one_window(const Ctx &c) {
    return c.nwin == 1 && c.win_frame_off.size() == 2 && c.win_pair_off.size() == 2 && c.win_S_off.size() >= 1 &&
           c.win_frame_off[0] == 0 && c.win_pair_off[0] == 0 && c.win_S_off[0] == 0;
}

// Column slots per group of a depth workgroup's product (0: every workgroup
// forms the whole step): the listed frames' unknowns rounded up to 32, when
// every thread's rows then fit its prefetch registers.
static int step_sel_ncw(const Ctx &c) {
    if (!c.d_step_sel || c.step_sel_max <= 0 || 6 * c.step_sel_max >= 6 * c.F) return 0;
    const int ncw = (6 * c.step_sel_max + 31) & ~31;
    const int ng = SOLVE_THREADS / ncw;
    return (6 * c.F + ng - 1) / ng <= SV_REG ? ncw : 0;
}

// Every workgroup of the fused step repeats the solve and holds a compute unit
// (its LDS), so the step is fused only while its grid is one round on the
// device: more points keep the solve and the depth step as separate kernels.
bool ic_fused(const Ctx &c) {
    return c.cfg.mode == PBA_IC_PROXY && one_window(c) && 6 * c.F <= IC_SPLIT_N && c.N > 0 &&
           1 + (int)nb(c.N, IC_STEP_PTS) <= c.n_cu && solve_cache_fits(c, true);
}

int du_nparts(const Ctx &c) {
    if (c.N <= 0) return 0;
    return (int)nb(c.N, ic_fused(c) ? IC_STEP_PTS : DU_PTS);
}

template <typename T>
static void ic_step_kernel(hipStream_t s, Ctx &c, const double *geo_lin, const double *geo_old, double *geo_next,
                           T *rel_next, hipEvent_t e0, hipEvent_t e1) {
    // iteration k of a batch reads pose buffer k mod 2 and writes the other
    // (the convergence kernel at the batch's end copies back after odd counts)
    const bool odd = (c.batch_k & 1) != 0;
    double *p_in = odd ? c.d_poses_alt : c.d_poses, *p_out = odd ? c.d_poses : c.d_poses_alt;
    // with events: recorded by the dispatch itself (the kernel's own duration);
    // without, a plain launch
    const dim3 grid(1 + nb(c.N, IC_STEP_PTS)), block(SOLVE_THREADS);
    auto launch = [&](auto... kargs) {
        if (e0 || e1)
            hipExtLaunchKernelGGL(k_ic_step<T>, grid, block, 0, s, e0, e1, 0, kargs...);
        else
            k_ic_step<T><<<grid, block, 0, s>>>(kargs...);
    };
    launch(c.win(), c.win_frame_off[1], c.win_pair_off[1], c.cfg.pinned_frame, c.d_frame_pair_ptr, c.d_frame_pair_item,
        c.d_pair_host, c.d_pair_target, c.d_pair_chunk_ptr, c.d_partY, c.d_pairY, geo_lin, c.d_Sinv, p_in, p_out,
        c.d_poses0, c.d_b, c.d_dtheta, c.d_dth_rel, geo_next, rel_next, c.d_wstat, c.d_flag, c.d_gate, c.N,
        c.d_obs_ptr, c.d_obs_pair, c.d_host_uv, c.d_pairK0, c.d_hc, c.d_gdo, 1, c.d_Hdd, geo_old, c.d_depth,
        c.d_depth0, c.d_du_part, c.d_step_sel, step_sel_ncw(c), (int)c.st.pchunk_begin.size(), c.d_obs_live);
}

void launch_ic_step(hipStream_t s, Ctx &c, const double *geo_lin, const double *geo_old, double *geo_next,
                    void *rel_next, bool rel_double, hipEvent_t e0, hipEvent_t e1) {
    if (rel_double)
        ic_step_kernel<double>(s, c, geo_lin, geo_old, geo_next, (double *)rel_next, e0, e1);
    else
        ic_step_kernel<float>(s, c, geo_lin, geo_old, geo_next, (float *)rel_next, e0, e1);
}

template <typename T, int PATH, bool CACHE>
static void solve_kernel(hipStream_t s, Ctx &c, int stage, const double *geo_lin, double *geo_next, T *rel_next) {
    const bool one = one_window(c);
    k_solve<T, PATH, CACHE><<<c.nwin, SOLVE_THREADS, 0, s>>>(
        c.win(), one ? c.win_frame_off[1] : -1, one ? c.win_pair_off[1] : -1, c.cfg.pinned_frame, stage, c.d_frame_pair_ptr, c.d_frame_pair_item, c.d_pair_host, c.d_pair_target,
        c.d_pair_chunk_ptr, c.d_partY, c.d_pairY, geo_lin, c.d_S, c.d_Sfac, c.d_Linv, c.d_Sinv, c.d_poses,
        c.d_poses0, c.d_b, c.d_dtheta, c.d_dth_rel, geo_next, rel_next, c.d_wstat, c.d_flag, c.d_gate);
}

template <typename T>
static void solve_path(hipStream_t s, Ctx &c, int stage, bool cache, const double *geo_lin, double *geo_next,
                       T *rel_next) {
    if (c.cfg.mode == PBA_IC_PROXY) {
        if (cache)
            solve_kernel<T, SOLVE_IC, true>(s, c, stage, geo_lin, geo_next, rel_next);
        else
            solve_kernel<T, SOLVE_IC, false>(s, c, stage, geo_lin, geo_next, rel_next);
    } else if (c.tiled()) {
        solve_kernel<T, SOLVE_FC_TILED, false>(s, c, stage, geo_lin, geo_next, rel_next);
    } else {
        solve_kernel<T, SOLVE_FC_PACKED, false>(s, c, stage, geo_lin, geo_next, rel_next);
    }
}

void launch_solve(hipStream_t s, Ctx &c, const double *geo_lin, double *geo_next, void *rel_next, bool rel_double,
                  double *stat) {
    (void)stat;
    const bool ic = c.cfg.mode == PBA_IC_PROXY;
    const int n = 6 * c.F;
    const bool cache = ic && solve_cache_fits(c);
    // IC on one large window: the product with S^{-1} spread over many workgroups
    const bool split = ic && c.nwin == 1 && n > IC_SPLIT_N;
    auto solve = [&](int stage) {
        if (rel_double)
            solve_path<double>(s, c, stage, cache, geo_lin, geo_next, (double *)rel_next);
        else
            solve_path<float>(s, c, stage, cache, geo_lin, geo_next, (float *)rel_next);
    };
    if (!split) {
        solve(0);
        return;
    }
    solve(1);
    k_ic_matvec<<<nb(n, 4), 256, 0, s>>>(n, c.d_Sinv, c.d_b, c.d_dtheta, c.d_flag, c.d_gate);
    solve(2);
}

}  // namespace pba
