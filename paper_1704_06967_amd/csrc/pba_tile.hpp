// Tile-blocked triangular solves with the tiled Cholesky factor of a reduced
// pose system (row-major n x n lower tiles, inverse diagonal tiles), shared by
// the per-iteration solve and the inverse of S.
#pragma once

#include "pba_internal.hpp"

namespace pba {

constexpr int TB = TCHOL_TILE;   // tile edge

// L L^T x = b for the tiled factor (x in LDS, overwritten), one block of NT
// threads. Forward substitution starts at tile k0 (b is zero above it).
// tmp: LDS scratch of at least TB * (NT / TB) + TB doubles.
template <int NT>
__device__ void tile_chol_solve(const double *__restrict__ L, const double *__restrict__ Linv, int n, double *x,
                                double *tmp, int k0) {
    const int nt = (n + TB - 1) / TB;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    constexpr int NW = NT / 64, Q = NT / TB;
    double *t = tmp + TB * Q;
    for (int K = k0; K < nt; ++K) {
        const int r0 = TB * K;
        // t_r = x_r - sum_{c < r0} L(r0 + r, c) x_c: one wavefront per row, lanes over columns
        for (int r = wv; r < TB; r += NW) {
            double s = 0.0;
            if (r0 + r < n)
                for (int c = TB * k0 + lane; c < r0; c += 64) s += L[(size_t)(r0 + r) * n + c] * x[c];
            for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
            if (lane == 0) t[r] = (r0 + r < n) ? x[r0 + r] - s : 0.0;
        }
        __syncthreads();
        if (threadIdx.x < TB) {
            const int r = threadIdx.x;
            const double *Lv = Linv + (size_t)K * TB * TB + r * TB;
            double y = 0.0;
            for (int k = 0; k <= r; ++k) y += Lv[k] * t[k];
            if (r0 + r < n) x[r0 + r] = y;
        }
        __syncthreads();
    }
    for (int K = nt - 1; K >= 0; --K) {
        const int r0 = TB * K;
        // t_r = y_r - sum_{i >= r0 + TB} L(i, r0 + r) x_i: thread (r, q) over rows i = ... + q (mod Q)
        {
            const int r = threadIdx.x % TB, q = threadIdx.x / TB;
            double s = 0.0;
            if (r0 + r < n)
                for (int i = r0 + TB + q; i < n; i += Q) s += L[(size_t)i * n + r0 + r] * x[i];
            tmp[q * TB + r] = s;
        }
        __syncthreads();
        if (threadIdx.x < TB) {
            const int r = threadIdx.x;
            double s = 0.0;
            for (int q = 0; q < Q; ++q) s += tmp[q * TB + r];
            t[r] = (r0 + r < n) ? x[r0 + r] - s : 0.0;
        }
        __syncthreads();
        if (threadIdx.x < TB) {
            const int r = threadIdx.x;
            const double *Lv = Linv + (size_t)K * TB * TB;
            double y = 0.0;
            for (int k = r; k < TB; ++k) y += Lv[k * TB + r] * t[k];
            if (r0 + r < n) x[r0 + r] = y;
        }
        __syncthreads();
    }
}

}  // namespace pba
