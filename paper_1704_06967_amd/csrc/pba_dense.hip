// Dense FP64 kernels for reduced pose systems too large for one workgroup's
// LDS (6F > 180): a tiled right-looking Cholesky over 32 x 32 tiles whose panel
// and trailing products run on FP64 MFMA (v_mfma_f64_16x16x4), the inverse of
// every diagonal factor tile, and tile-blocked triangular solves built on them.
#include "pba_device.hpp"
#include "pba_internal.hpp"
#include "pba_tile.hpp"

namespace pba {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int TP = TB + 1;       // LDS row pitch (doubles)

__device__ __forceinline__ double &tl(double *t, int r, int c) { return t[r * TP + c]; }
__device__ __forceinline__ double tl(const double *t, int r, int c) { return t[r * TP + c]; }

// Tile (I, J) of the row-major n x n matrix into LDS; entries outside the matrix are 0.
__device__ __forceinline__ void load_tile(const double *__restrict__ A, int n, int I, int J, double *t) {
    for (int e = threadIdx.x; e < TB * TB; e += blockDim.x) {
        const int r = e / TB, c = e % TB, gr = TB * I + r, gc = TB * J + c;
        tl(t, r, c) = (gr < n && gc < n) ? A[(size_t)gr * n + gc] : 0.0;
    }
}

__device__ __forceinline__ void store_tile(double *__restrict__ A, int n, int I, int J, const double *t) {
    for (int e = threadIdx.x; e < TB * TB; e += blockDim.x) {
        const int r = e / TB, c = e % TB, gr = TB * I + r, gc = TB * J + c;
        if (gr < n && gc < n) A[(size_t)gr * n + gc] = tl(t, r, c);
    }
}

// One wavefront's 16 x 16 quadrant (qr, qc) of X Y^T for 32 x 32 LDS tiles X, Y
// (FP64 MFMA, K = 32 in 8 steps of 4). Operand lanes: A[row = l % 16][k = l / 16],
// B[k = l / 16][col = l % 16]; result element i of lane l is row l / 16 + 4 i,
// column l % 16 of the quadrant.
__device__ __forceinline__ f64x4 quad_xyT(const double *X, const double *Y, int qr, int qc) {
    const int l = threadIdx.x & 63;
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < TB / 4; ++s) {
        const double a = X[(16 * qr + (l & 15)) * TP + 4 * s + (l >> 4)];
        const double b = Y[(16 * qc + (l & 15)) * TP + 4 * s + (l >> 4)];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    return acc;
}

// Value of v in lane l (uniform l), as a scalar read of the register.
__device__ __forceinline__ double readlane_d(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Factor the LDS tile t = L L^T in place (rows and columns >= nb are made the
// identity first), and write L^{-1} (identity on the padding) to Linv_g.
// Called by a whole 256-thread block; wavefront 0 does the work with the tile
// in registers (lane r holds row r): each column step reads the pivot and the
// column's entries of the other rows with scalar lane reads, so the 32 steps
// need no LDS round trips or barriers. Lane c then forms column c of L^{-1} by
// forward substitution. Returns false in every thread when a pivot is not
// positive.
__device__ __forceinline__ bool tile_potrf_inv(double *t, int nb, double *__restrict__ Linv_g, double *invd, int *fail) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (threadIdx.x == 0) *fail = 0;
    __syncthreads();
    if (wv == 0) {
        double row[TB];
#pragma unroll
        for (int c = 0; c < TB; ++c) {
            double v = 0.0;
            if (lane < TB) v = (lane < nb && c < nb) ? tl(t, lane, c) : (lane == c ? 1.0 : 0.0);
            row[c] = v;
        }
        bool ok = true;
#pragma unroll
        for (int j = 0; j < TB; ++j) {
            const double p = readlane_d(row[j], j);
            ok = ok && p > 0.0;
            const double l = sqrt(p > 0.0 ? p : 1.0), inv = 1.0 / l;
            const double a = lane > j ? row[j] * inv : (lane == j ? l : row[j]);
            row[j] = a;
#pragma unroll
            for (int c = j + 1; c < TB; ++c) {
                const double ac = readlane_d(a, c);
                if (lane >= c && lane < TB) row[c] -= a * ac;
            }
        }
        if (!ok) {
            if (lane == 0) *fail = 1;
        } else {
            if (lane < TB) {
#pragma unroll
                for (int c = 0; c < TB; ++c) tl(t, lane, c) = c <= lane ? row[c] : 0.0;
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (lane < TB) invd[lane] = 1.0 / tl(t, lane, lane);
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // column `lane` of L^{-1}: x[i] = (delta_i,lane - sum_k<i L(i, k) x[k]) / L(i, i)
            // (every lane reads the same L(i, k): LDS broadcasts; four partial
            // sums shorten the dependent chains)
            double x[TB];
#pragma unroll
            for (int i = 0; i < TB; ++i) {
                double s0 = (i == lane) ? 1.0 : 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
                for (int k = 0; k < i; k += 4) {
                    s0 -= tl(t, i, k) * x[k];
                    if (k + 1 < i) s1 -= tl(t, i, k + 1) * x[k + 1];
                    if (k + 2 < i) s2 -= tl(t, i, k + 2) * x[k + 2];
                    if (k + 3 < i) s3 -= tl(t, i, k + 3) * x[k + 3];
                }
                x[i] = (i >= lane) ? ((s0 + s1) + (s2 + s3)) * invd[i] : 0.0;
            }
            if (lane < TB) {
#pragma unroll
                for (int i = 0; i < TB; ++i) Linv_g[i * TB + lane] = x[i];
            }
        }
    }
    __syncthreads();
    return *fail == 0;
}

__device__ __forceinline__ void chol_fail(int *flag, int *gate) {
    if (threadIdx.x == 0) {
        *flag = 1;
        *gate = 0;
    }
}

// Tile (0, 0).
__global__ __launch_bounds__(256) void k_tchol_first(int n, double *__restrict__ A, double *__restrict__ Linv,
                                                     int *__restrict__ flag, int *__restrict__ gate) {
    __shared__ double t[TB * TP];
    __shared__ double invd[TB];
    __shared__ int fail;
    if (*gate == 0 || *flag) return;
    load_tile(A, n, 0, 0, t);
    __syncthreads();
    if (!tile_potrf_inv(t, min(TB, n), Linv, invd, &fail)) {
        chol_fail(flag, gate);
        return;
    }
    store_tile(A, n, 0, 0, t);
}

// Panel of step kt: L_I,kt = A_I,kt L_kt,kt^{-T} for the tile rows I > kt (one per block).
__global__ __launch_bounds__(256) void k_tchol_panel(int n, int kt, double *__restrict__ A,
                                                     const double *__restrict__ Linv, const int *__restrict__ flag,
                                                     const int *__restrict__ gate) {
    __shared__ double ta[TB * TP], tv[TB * TP];
    if (*gate == 0 || *flag) return;
    const int I = kt + 1 + blockIdx.x;
    load_tile(A, n, I, kt, ta);
    const double *Lv = Linv + (size_t)kt * TB * TB;
    for (int e = threadIdx.x; e < TB * TB; e += blockDim.x) tl(tv, e / TB, e % TB) = Lv[e];
    __syncthreads();
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, qr = wv >> 1, qc = wv & 1;
    const f64x4 acc = quad_xyT(ta, tv, qr, qc);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) tl(ta, 16 * qr + (l >> 4) + 4 * i, 16 * qc + (l & 15)) = acc[i];
    __syncthreads();
    store_tile(A, n, I, kt, ta);
}

// Trailing update of step kt: A_IJ -= L_I,kt L_J,kt^T for kt < J <= I (one tile
// per block, lower-triangle order); the block of tile (kt+1, kt+1) then factors
// it and writes its inverse, which the next panel uses.
__global__ __launch_bounds__(256) void k_tchol_update(int n, int kt, double *__restrict__ A,
                                                      double *__restrict__ Linv, int *__restrict__ flag,
                                                      int *__restrict__ gate) {
    __shared__ double ti[TB * TP], tj[TB * TP], tc[TB * TP];
    __shared__ double invd[TB];
    __shared__ int fail;
    if (*gate == 0 || *flag) return;
    // blockIdx.x -> (i, j), j <= i, in row-major lower-triangle order
    const int b = blockIdx.x;
    int i = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= b) ++i;
    while (i * (i + 1) / 2 > b) --i;
    const int j = b - i * (i + 1) / 2;
    const int I = kt + 1 + i, J = kt + 1 + j;
    load_tile(A, n, I, kt, ti);
    if (I != J) load_tile(A, n, J, kt, tj);
    load_tile(A, n, I, J, tc);
    __syncthreads();
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, qr = wv >> 1, qc = wv & 1;
    const f64x4 acc = quad_xyT(ti, I != J ? tj : ti, qr, qc);
#pragma unroll
    for (int q = 0; q < 4; ++q) tl(tc, 16 * qr + (l >> 4) + 4 * q, 16 * qc + (l & 15)) -= acc[q];
    __syncthreads();
    if (I == kt + 1 && J == kt + 1) {
        if (!tile_potrf_inv(tc, min(TB, n - TB * I), Linv + (size_t)I * TB * TB, invd, &fail)) {
            chol_fail(flag, gate);
            return;
        }
    }
    store_tile(A, n, I, J, tc);
}

// S^{-1} column by column from the tiled factor (one column per block; by
// symmetry it is stored as a row).
__global__ __launch_bounds__(256) void k_tinv_columns(int n, const double *__restrict__ L,
                                                      const double *__restrict__ Linv, double *__restrict__ Sinv,
                                                      const int *__restrict__ flag, const int *__restrict__ gate) {
    extern __shared__ double dyn[];
    if (*gate == 0 || *flag) return;
    double *x = dyn;
    double *tmp = dyn + n;
    for (int col = blockIdx.x; col < n; col += gridDim.x) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = (i == col) ? 1.0 : 0.0;
        __syncthreads();
        tile_chol_solve<256>(L, Linv, n, x, tmp, col / TB);
        for (int i = threadIdx.x; i < n; i += blockDim.x) Sinv[(size_t)col * n + i] = x[i];
        __syncthreads();
    }
}

__global__ void k_copy_d(const double *__restrict__ src, double *__restrict__ dst, size_t n,
                         const int *__restrict__ gate) {
    if (gate && *gate == 0) return;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

void launch_copy_d(hipStream_t s, const double *src, double *dst, size_t n) {
    if (n == 0) return;
    k_copy_d<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(src, dst, n, nullptr);
}

// x = -(L L^T)^{-1} b with the tiled factor (one workgroup).
__global__ __launch_bounds__(1024) void k_tsolve(int n, const double *__restrict__ L, const double *__restrict__ Linv,
                                                 const double *__restrict__ b, double *__restrict__ x,
                                                 const int *__restrict__ flag) {
    extern __shared__ double dyn[];
    if (*flag) return;
    double *v = dyn, *tmp = dyn + n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v[i] = -b[i];
    __syncthreads();
    tile_chol_solve<1024>(L, Linv, n, v, tmp, 0);
    for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = v[i];
}

void launch_tsolve(hipStream_t s, Ctx &c, const double *b, double *x) {
    const int n = 6 * c.F;
    const size_t lds = ((size_t)n + tile_solve_tmp(1024)) * sizeof(double);
    k_tsolve<<<1, 1024, lds, s>>>(n, c.d_Sfac, c.d_Linv, b, x, c.d_flag);
}

void launch_tchol(hipStream_t s, Ctx &c) {
    const int n = 6 * c.F, nt = (n + TB - 1) / TB;
    const size_t nn = (size_t)n * n;
    k_copy_d<<<(unsigned)((nn + 255) / 256), 256, 0, s>>>(c.d_S, c.d_Sfac, nn, c.d_gate);
    k_tchol_first<<<1, 256, 0, s>>>(n, c.d_Sfac, c.d_Linv, c.d_flag, c.d_gate);
    for (int kt = 0; kt + 1 < nt; ++kt) {
        const int m = nt - kt - 1;
        k_tchol_panel<<<m, 256, 0, s>>>(n, kt, c.d_Sfac, c.d_Linv, c.d_flag, c.d_gate);
        k_tchol_update<<<m * (m + 1) / 2, 256, 0, s>>>(n, kt, c.d_Sfac, c.d_Linv, c.d_flag, c.d_gate);
    }
}

void launch_tinv(hipStream_t s, Ctx &c) {
    const int n = 6 * c.F;
    const size_t lds = ((size_t)n + tile_solve_tmp(256)) * sizeof(double);
    k_tinv_columns<<<std::min(n, 2048), 256, lds, s>>>(n, c.d_Sfac, c.d_Linv, c.d_Sinv, c.d_flag, c.d_gate);
}

}  // namespace pba
