// Tile-blocked triangular solves with the tiled Cholesky factor of a reduced
// pose system (row-major n x n lower tiles, inverse diagonal tiles), shared by
// the per-iteration solve and the inverse of S.
#pragma once

#include "pba_internal.hpp"

namespace pba {

constexpr int TB = TCHOL_TILE;   // tile edge
static_assert(TB == 32, "the tile solves reduce over halves of a wavefront");

// LDS scratch (doubles) that tile_chol_solve<NT> needs beside x.
constexpr int tile_solve_tmp(int nt_threads) { return TB * (nt_threads / TB) + TB + TB * (TB + 1); }

// L L^T x = b for the tiled factor (x in LDS, overwritten), one block of NT
// threads. Forward substitution starts at tile k0 (b is zero above it). Every
// tile step stages the inverse diagonal tile in LDS (one load per thread,
// overlapped with the step's panel loads) and forms its product with 32-lane
// sums over half wavefronts. tmp: tile_solve_tmp(NT) doubles of LDS.
template <int NT>
__device__ void tile_chol_solve(const double *__restrict__ L, const double *__restrict__ Linv, int n, double *x,
                                double *tmp, int k0) {
    const int nt = (n + TB - 1) / TB;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    constexpr int NW = NT / 64, Q = NT / TB, RP = NT / TB, RPW = TB / NW;
    static_assert(Q <= TB, "partials per column exceed a 32-lane sum");
    double *t = tmp + TB * Q;
    double *lv = t + TB;                                   // [TB][TB + 1]
    const int kk = threadIdx.x & (TB - 1), rr = threadIdx.x / TB;
    for (int K = k0; K < nt; ++K) {
        const int r0 = TB * K;
        // t_r = x_r - sum_{c < r0} L(r0 + r, c) x_c: wavefront wv owns rows
        // wv + NW u, lanes over columns; the rows' loads are interleaved so that
        // all of them are in flight together
        {
            double s[RPW];
#pragma unroll
            for (int u = 0; u < RPW; ++u) s[u] = 0.0;
#pragma unroll 2
            for (int c = TB * k0 + lane; c < r0; c += 64) {
                const double xc = x[c];
#pragma unroll
                for (int u = 0; u < RPW; ++u) {
                    const int r = wv + NW * u;
                    if (r0 + r < n) s[u] += L[(size_t)(r0 + r) * n + c] * xc;
                }
            }
#pragma unroll
            for (int u = 0; u < RPW; ++u) {
                const int r = wv + NW * u;
                const double v = wave_sum(s[u]);
                if (lane == 0) t[r] = (r0 + r < n) ? x[r0 + r] - v : 0.0;
            }
        }
        {
            const double *Lk = Linv + (size_t)K * TB * TB;
            for (int e = threadIdx.x; e < TB * TB; e += NT) lv[(e / TB) * (TB + 1) + e % TB] = Lk[e];
        }
        __syncthreads();
        // x_r = sum_{k <= r} Linv_K(r, k) t_k
        for (int r = rr; r < TB; r += RP) {
            const double v = half_sum32(kk <= r ? lv[r * (TB + 1) + kk] * t[kk] : 0.0);
            if (kk == 0 && r0 + r < n) x[r0 + r] = v;
        }
        __syncthreads();
    }
    for (int K = nt - 1; K >= 0; --K) {
        const int r0 = TB * K;
        // partials of sum_{i >= r0 + TB} L(i, r0 + r) x_i: thread (r, q) over rows i = ... + q (mod Q)
        {
            const int r = threadIdx.x % TB, q = threadIdx.x / TB;
            double s = 0.0;
            if (r0 + r < n) {
#pragma unroll 8
                for (int i = r0 + TB + q; i < n; i += Q) s += L[(size_t)i * n + r0 + r] * x[i];
            }
            tmp[q * TB + r] = s;
        }
        {
            const double *Lk = Linv + (size_t)K * TB * TB;
            for (int e = threadIdx.x; e < TB * TB; e += NT) lv[(e / TB) * (TB + 1) + e % TB] = Lk[e];
        }
        __syncthreads();
        for (int r = rr; r < TB; r += RP) {
            const double v = half_sum32(kk < Q ? tmp[kk * TB + r] : 0.0);
            if (kk == 0) t[r] = (r0 + r < n) ? x[r0 + r] - v : 0.0;
        }
        __syncthreads();
        // x_r = sum_{k >= r} Linv_K(k, r) t_k
        for (int r = rr; r < TB; r += RP) {
            const double v = half_sum32(kk >= r ? lv[kk * (TB + 1) + r] * t[kk] : 0.0);
            if (kk == 0 && r0 + r < n) x[r0 + r] = v;
        }
        __syncthreads();
    }
}

// LDS scratch (doubles) of tile_chol_solve_packed.
constexpr int TILE_PACKED_TMP = TB + TB * (TB + 1);

// Packed lower triangle of the row-major n x n factor into LDS (n (n + 1) / 2
// doubles): thread over packed indices, loads unrolled so that several are in
// flight per thread.
template <int NT>
__device__ __forceinline__ void load_packed_lower(const double *__restrict__ L, int n, double *Lp) {
    const int np = n * (n + 1) / 2;
#pragma unroll 8
    for (int p = threadIdx.x; p < np; p += NT) {
        // row of packed index p: floor((sqrt(8 p + 1) - 1) / 2), exact in double
        // (8 p + 1 is an odd square exactly at row starts; otherwise its root is
        // far from an integer), so no correction branches
        const int i = (int)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
        Lp[p] = L[(size_t)i * n + (p - i * (i + 1) / 2)];
    }
}

// L L^T x = b with the packed factor Lp in LDS (x in LDS, overwritten), one
// block of NT threads, right-looking over the 32-row tiles. Forward: x_K = Linv_K x_K, then
// every later row subtracts L(i, tile K) x_K (one thread per row). Backward:
// x_K = Linv_K^T x_K, then every earlier row subtracts L(tile K, j)^T x_K.
// Each step has two phases of 32 multiply-adds per thread and no cross-lane
// sums; the inverse diagonal tile is staged in LDS from registers loaded one
// step ahead. Forward substitution starts at tile k0 (b is zero above it).
// tmp: TILE_PACKED_TMP doubles of LDS.
template <int NT>
__device__ void tile_chol_solve_packed(const double *Lp, const double *__restrict__ Linv, int n, double *x,
                                      double *tmp, int k0) {
    auto L = [&](int i, int j) { return Lp[i * (i + 1) / 2 + j]; };
    const int nt = (n + TB - 1) / TB;
    constexpr int PE = TB * TB / NT > 0 ? TB * TB / NT : 1;
    const int tid = threadIdx.x;
    double *t = tmp;                                       // [TB]
    double *lv = tmp + TB;                                 // [TB][TB + 1]
    double pre[PE];                                        // the next inverse diagonal tile
    auto fetch = [&](int K) {
        const double *Lk = Linv + (size_t)K * TB * TB;
#pragma unroll
        for (int u = 0; u < PE; ++u) {
            const int e = tid + NT * u;
            pre[u] = e < TB * TB ? Lk[e] : 0.0;
        }
    };
    auto stage = [&]() {
#pragma unroll
        for (int u = 0; u < PE; ++u) {
            const int e = tid + NT * u;
            if (e < TB * TB) lv[(e / TB) * (TB + 1) + e % TB] = pre[u];
        }
    };
    fetch(k0);
    for (int K = k0; K < nt; ++K) {
        const int r0 = TB * K;
        stage();
        fetch(K + 1 < nt ? K + 1 : nt - 1);   // the last forward step fetches the first backward tile
        __syncthreads();
        if (tid < TB) {
            // Linv_K is lower triangular (zeros stored above the diagonal); x
            // past n reads as 0: no branches, so that all loads are in flight
            double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k = 0; k < TB; ++k) {
                const double xv = x[min(r0 + k, n - 1)];
                s[k & 3] += lv[tid * (TB + 1) + k] * (r0 + k < n ? xv : 0.0);
            }
            t[tid] = (s[0] + s[1]) + (s[2] + s[3]);
        }
        __syncthreads();
        if (tid < TB && r0 + tid < n) x[r0 + tid] = t[tid];
        for (int i = r0 + TB + tid; i < n; i += NT) {
            double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k = 0; k < TB; ++k) s[k & 3] += L(i, r0 + k) * t[k];
            x[i] -= (s[0] + s[1]) + (s[2] + s[3]);
        }
        __syncthreads();
    }
    for (int K = nt - 1; K >= 0; --K) {
        const int r0 = TB * K;
        stage();
        if (K > 0) fetch(K - 1);
        __syncthreads();
        if (tid < TB) {
            double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k = 0; k < TB; ++k) {
                const double xv = x[min(r0 + k, n - 1)];
                s[k & 3] += lv[k * (TB + 1) + tid] * (r0 + k < n ? xv : 0.0);
            }
            t[tid] = (s[0] + s[1]) + (s[2] + s[3]);
        }
        __syncthreads();
        if (tid < TB && r0 + tid < n) x[r0 + tid] = t[tid];
        for (int j = tid; j < r0; j += NT) {
            // rows past n: clamped address, t_k = 0 there
            double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k = 0; k < TB; ++k) s[k & 3] += L(min(r0 + k, n - 1), j) * t[k];
            x[j] -= (s[0] + s[1]) + (s[2] + s[3]);
        }
        __syncthreads();
    }
}

}  // namespace pba
