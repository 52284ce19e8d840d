// Tile-blocked triangular solves with the tiled Cholesky factor of a reduced
// pose system (row-major n x n lower tiles, inverse diagonal tiles), shared by
// the per-iteration solve and the inverse of S.
#pragma once

#include "pba_internal.hpp"

namespace pba {

constexpr int TB = TCHOL_TILE;   // tile edge

// LDS scratch (doubles) that tile_chol_solve<NT> needs beside x.
constexpr int tile_solve_tmp(int nt_threads) { return TB * (nt_threads / TB) + TB + TB * (TB + 1); }

// L L^T x = b for the tiled factor (x in LDS, overwritten), one block of NT
// threads. Forward substitution starts at tile k0 (b is zero above it). Every
// tile step stages the inverse diagonal tile in LDS (one load per thread,
// overlapped with the step's panel loads) and forms its product with 32-lane
// shuffle sums. tmp: tile_solve_tmp(NT) doubles of LDS.
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
                double v = s[u];
                for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
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
            double v = kk <= r ? lv[r * (TB + 1) + kk] * t[kk] : 0.0;
            for (int o = TB / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
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
            double v = kk < Q ? tmp[kk * TB + r] : 0.0;
            for (int o = TB / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
            if (kk == 0) t[r] = (r0 + r < n) ? x[r0 + r] - v : 0.0;
        }
        __syncthreads();
        // x_r = sum_{k >= r} Linv_K(k, r) t_k
        for (int r = rr; r < TB; r += RP) {
            double v = kk >= r ? lv[kk * (TB + 1) + r] * t[kk] : 0.0;
            for (int o = TB / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
            if (kk == 0 && r0 + r < n) x[r0 + r] = v;
        }
        __syncthreads();
    }
}

}  // namespace pba
