// Dense FP64 kernels for reduced pose systems too large for one workgroup's
// LDS (6F > 180): a tiled right-looking Cholesky over 32 x 32 tiles whose panel
// and trailing products run on FP64 MFMA (v_mfma_f64_16x16x4), the inverse of
// every diagonal factor tile, and tile-blocked triangular solves built on them.
#include "pba_device.hpp"
#include "pba_affine.hpp"
#include "pba_internal.hpp"
#include "pba_tile.hpp"

#include <mutex>
#include <string>

namespace pba {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int TP = TB + 1;       // LDS row pitch (doubles)

__device__ __forceinline__ double &tl(double *t, int r, int c) { return t[r * TP + c]; }
__device__ __forceinline__ double tl(const double *t, int r, int c) { return t[r * TP + c]; }

// A thread's share of a tile for the 256-thread tile kernels: tile_fetch loads
// it into registers, tile_put stores it into an LDS tile, so that the loads of
// all the tiles a kernel needs are in flight together (entries outside the
// matrix are 0 and are not loaded).
constexpr int TILE_THREADS = 256, TILE_PER = TB * TB / TILE_THREADS;
struct TileRegs {
    double v[TILE_PER];
};

__device__ __forceinline__ void tile_fetch(const double *__restrict__ A, int n, int I, int J, TileRegs &r) {
#pragma unroll
    for (int u = 0; u < TILE_PER; ++u) {
        const int e = threadIdx.x + TILE_THREADS * u, gr = TB * I + e / TB, gc = TB * J + e % TB;
        r.v[u] = 0.0;
        if (gr < n && gc < n) r.v[u] = A[(size_t)gr * n + gc];
    }
}

__device__ __forceinline__ void tile_put(double *t, const TileRegs &r) {
#pragma unroll
    for (int u = 0; u < TILE_PER; ++u) {
        const int e = threadIdx.x + TILE_THREADS * u;
        tl(t, e / TB, e % TB) = r.v[u];
    }
}

// Tile (I, J) of the row-major n x n matrix into LDS (256 threads).
__device__ __forceinline__ void load_tile(const double *__restrict__ A, int n, int I, int J, double *t) {
    TileRegs r;
    tile_fetch(A, n, I, J, r);
    tile_put(t, r);
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

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int SP = 17;   // LDS pitch of the 16 x 16 scratch blocks

// Factors a 16-column register panel in place (lane r holds row r; the
// diagonal of column j sits in lane base + j; rows past the tile hold 0).
// After column j's multipliers are formed, the next column is updated first,
// with the pivot row's multiplier read from its lane, so that the next pivot's
// square root and reciprocal are formed before the rest of column j's
// rank-one update is broadcast through LDS (bc, 16 doubles) and applied; the
// operations and operands are those of the plain column loop. The update runs
// on every lane (entries above the diagonal take values that are never read).
// Returns whether every pivot was positive.
__device__ __forceinline__ bool panel_factor16(double (&row)[16], int base, double *bc) {
    const int l = threadIdx.x & 63;
    double p = readlane_d(row[0], base);
    bool ok = p > 0.0;
    double lj = sqrt(p > 0.0 ? p : 1.0), inv = 1.0 / lj;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const double a = l > base + j ? row[j] * inv : (l == base + j ? lj : row[j]);
        row[j] = a;
        if (j < 15) {
            const double an = readlane_d(a, base + j + 1);
            row[j + 1] -= a * an;
            const double pn = readlane_d(row[j + 1], base + j + 1);
            ok = ok && pn > 0.0;
            const double ljn = sqrt(pn > 0.0 ? pn : 1.0), invn = 1.0 / ljn;
            if (j < 14) {
                if (l > base + j + 1 && l < base + 16) bc[l - base] = a;
                wave_sync();
#pragma unroll
                for (int c = j + 2; c < 16; ++c) row[c] -= a * bc[c];
                wave_sync();
            }
            lj = ljn;
            inv = invn;
        }
    }
    return ok;
}

// Factor the LDS tile t = L L^T in place (rows and columns >= nb are made the
// identity first), and write L^{-1} (identity on the padding) to Linv_g.
// Called by a whole 256-thread block; wavefront 0 does the work, blocked 2 x 2
// in 16-wide panels. Panel 1 (columns 0-15 of all 32 rows) and, after the
// update A22 -= L21 L21^T on FP64 MFMA, panel 2 (A22) are factored with the
// rows in registers (lane r holds row r): each column step reads the pivot
// with a scalar lane read and the column's multipliers with broadcast LDS
// reads (one write and one read round trip per column); the rank-one update
// runs on every lane (entries above the diagonal take values that are never
// read and are zeroed when the panel is stored). The
// inverse is [X11 0; X21 X22] with X11 = L11^{-1} and X22 = L22^{-1} formed
// at once by forward substitution (lane c of each half one column) and
// X21 = -X22 (L21 X11) as two MFMA products. s1, s2: LDS scratch of 16 x SP
// doubles each. Returns false in every thread when a pivot is not positive.
__device__ __forceinline__ bool tile_potrf_inv(double *t, int nb, double *__restrict__ Linv_g, double *invd,
                                               double *s1, double *s2, int *fail) {
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (threadIdx.x == 0) *fail = 0;
    __syncthreads();
    if (wv == 0) {
        if (nb < TB && l < TB) {
#pragma unroll
            for (int c = 0; c < TB; ++c)
                if (l >= nb || c >= nb) tl(t, l, c) = (l == c) ? 1.0 : 0.0;
        }
        wave_sync();
        bool ok = true;
        double row[16];
        // panel 1: columns 0..15 of rows 0..31 (L11 and L21)
#pragma unroll
        for (int c = 0; c < 16; ++c) row[c] = l < TB ? tl(t, l, c) : 0.0;
        ok = panel_factor16(row, 0, s1);
        if (l < TB) {
#pragma unroll
            for (int c = 0; c < 16; ++c) tl(t, l, c) = c <= l ? row[c] : 0.0;
        }
        wave_sync();
        // A22 -= L21 L21^T (element i of lane l: row 16 + l / 16 + 4 i, column 16 + l % 16)
        {
            f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const double av = tl(t, 16 + (l & 15), 4 * s + (l >> 4));
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, av, acc, 0, 0, 0);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) tl(t, 16 + (l >> 4) + 4 * i, 16 + (l & 15)) -= acc[i];
        }
        wave_sync();
        // panel 2: A22 on lanes 16..31
#pragma unroll
        for (int c = 0; c < 16; ++c) row[c] = (l >= 16 && l < TB) ? tl(t, l, 16 + c) : 0.0;
        const bool ok2 = panel_factor16(row, 16, s1);
        ok = ok && ok2;
        if (!ok) {
            if (l == 0) *fail = 1;
        } else {
            if (l >= 16 && l < TB) {
#pragma unroll
                for (int c = 0; c < 16; ++c) tl(t, l, 16 + c) = 16 + c <= l ? row[c] : 0.0;
            }
            if (l < 16) {
#pragma unroll
                for (int c = 0; c < 16; ++c) tl(t, l, 16 + c) = 0.0;
            }
            wave_sync();
            if (l < TB) invd[l] = 1.0 / tl(t, l, l);
            wave_sync();
            // X11 (lanes 0..15, column l) and X22 (lanes 16..31, column l - 16):
            // x[i] = (delta_i,c - sum_k<i L(i, k) x[k]) / L(i, i) within the half,
            // four partial sums to shorten the dependent chains
            const int base = l < 16 ? 0 : 16, cc = l & 15;
            double x[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                double q0 = (i == cc) ? 1.0 : 0.0, q1 = 0.0, q2 = 0.0, q3 = 0.0;
#pragma unroll
                for (int k = 0; k < i; k += 4) {
                    q0 -= tl(t, base + i, base + k) * x[k];
                    if (k + 1 < i) q1 -= tl(t, base + i, base + k + 1) * x[k + 1];
                    if (k + 2 < i) q2 -= tl(t, base + i, base + k + 2) * x[k + 2];
                    if (k + 3 < i) q3 -= tl(t, base + i, base + k + 3) * x[k + 3];
                }
                x[i] = (i >= cc) ? ((q0 + q1) + (q2 + q3)) * invd[base + i] : 0.0;
            }
            // s1 = X11^T, s2 = X22^T (row c holds column c)
            if (l < TB) {
                double *sx = l < 16 ? s1 : s2;
#pragma unroll
                for (int i = 0; i < 16; ++i) sx[cc * SP + i] = x[i];
            }
            wave_sync();
            // P = L21 X11 (rows of L21 against rows of X11^T)
            f64x4 pacc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const double av = tl(t, 16 + (l & 15), 4 * s + (l >> 4));
                const double bv = s1[(l & 15) * SP + 4 * s + (l >> 4)];
                pacc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, pacc, 0, 0, 0);
            }
            wave_sync();
            // P row-major into s1 (X11 stays in the registers of lanes 0..15)
#pragma unroll
            for (int i = 0; i < 4; ++i) s1[((l >> 4) + 4 * i) * SP + (l & 15)] = pacc[i];
            wave_sync();
            // X21 = -X22 P (rows of X22 = columns of s2 against rows of P^T = columns of s1)
            f64x4 xacc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const double av = s2[(4 * s + (l >> 4)) * SP + (l & 15)];
                const double bv = s1[(4 * s + (l >> 4)) * SP + (l & 15)];
                xacc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, xacc, 0, 0, 0);
            }
            if (l < 16) {
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    Linv_g[i * TB + l] = x[i];
                    Linv_g[i * TB + 16 + l] = 0.0;
                }
            } else if (l < TB) {
#pragma unroll
                for (int i = 0; i < 16; ++i) Linv_g[(16 + i) * TB + l] = x[i];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) Linv_g[(16 + (l >> 4) + 4 * i) * TB + (l & 15)] = -xacc[i];
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
    __shared__ double s1[16 * SP], s2[16 * SP];
    __shared__ double invd[TB];
    __shared__ int fail;
    if (*gate == 0 || *flag) return;
    load_tile(A, n, 0, 0, t);
    __syncthreads();
    if (!tile_potrf_inv(t, min(TB, n), Linv, invd, s1, s2, &fail)) {
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
    TileRegs ra, rv;
    tile_fetch(A, n, I, kt, ra);
    tile_fetch(Linv + (size_t)kt * TB * TB, TB, 0, 0, rv);   // the inverse diagonal tile (TB x TB)
    tile_put(ta, ra);
    tile_put(tv, rv);
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
    {
        TileRegs ri, rj, rc;
        tile_fetch(A, n, I, kt, ri);
        if (I != J) tile_fetch(A, n, J, kt, rj);
        tile_fetch(A, n, I, J, rc);
        tile_put(ti, ri);
        if (I != J) tile_put(tj, rj);
        tile_put(tc, rc);
    }
    __syncthreads();
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, qr = wv >> 1, qc = wv & 1;
    const f64x4 acc = quad_xyT(ti, I != J ? tj : ti, qr, qc);
#pragma unroll
    for (int q = 0; q < 4; ++q) tl(tc, 16 * qr + (l >> 4) + 4 * q, 16 * qc + (l & 15)) -= acc[q];
    __syncthreads();
    if (I == kt + 1 && J == kt + 1) {
        // ti and tj are free once the update is in tc: scratch of the factor
        if (!tile_potrf_inv(tc, min(TB, n - TB * I), Linv + (size_t)I * TB * TB, invd, ti, tj, &fail)) {
            chol_fail(flag, gate);
            return;
        }
    }
    store_tile(A, n, I, J, tc);
}

// The chain for a few tiles (n <= TCHOL_FUSE_N): every panel is formed in the
// kernel that factors its diagonal tile, so that one launch per step remains.
// A panel block cannot read that tile from the factor (its own block rewrites
// it in place), so it forms it itself: the tile of the unchanged S minus the
// products of its row's factor tiles, in step order, which gives the same
// values to the bit, and factors it.
constexpr int TCHOL_FUSE_N = 8 * TB;

// Diagonal tile J formed again: td holds S_JJ and tm[m] the factor tiles
// L_Jm (m < J), all loaded by the caller; every wavefront subtracts the
// products from its quadrant in step order, then the tile is factored and its
// inverse left in LDS (tw, pitch TP). tv, ti, tj: scratch tiles. Whole block.
__device__ __forceinline__ bool tile_diag_again(int n, int J, double *td, const double *tm, double *tv, double *ti,
                                                double *tj, double *tw, double *invd, int *fail) {
    const int wv = threadIdx.x >> 6, qr = wv >> 1, qc = wv & 1, l = threadIdx.x & 63;
    for (int m = 0; m < J; ++m) {
        const double *L = tm + (size_t)m * TB * TP;
        const f64x4 acc = quad_xyT(L, L, qr, qc);
#pragma unroll
        for (int q = 0; q < 4; ++q) tl(td, 16 * qr + (l >> 4) + 4 * q, 16 * qc + (l & 15)) -= acc[q];
    }
    __syncthreads();
    // inverse written at pitch TB into tv, then copied at pitch TP into tw
    if (!tile_potrf_inv(td, min(TB, n - TB * J), tv, invd, ti, tj, fail)) return false;
    for (int e = threadIdx.x; e < TB * TB; e += blockDim.x) tl(tw, e / TB, e % TB) = tv[e];
    __syncthreads();
    return true;
}

// Panel tile (I, J): A_IJ (in ta) times the inverse's transpose (tw), written back.
__device__ __forceinline__ void tile_panel(double *A, int n, int I, int J, double *ta, const double *tw) {
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, qr = wv >> 1, qc = wv & 1;
    const f64x4 acc = quad_xyT(ta, tw, qr, qc);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) tl(ta, 16 * qr + (l >> 4) + 4 * i, 16 * qc + (l & 15)) = acc[i];
    __syncthreads();
    store_tile(A, n, I, J, ta);
}

// Step 0 of the short chain: block 0 factors tile (0, 0) (writing it and its
// inverse); block I > 0 forms L_I0 = A_I0 L00^{-T}.
__global__ __launch_bounds__(256) void k_tchol_first_panel(int n, const double *__restrict__ S, double *__restrict__ A,
                                                           double *__restrict__ Linv, int *__restrict__ flag,
                                                           int *__restrict__ gate) {
    __shared__ double ta[TB * TP], td[TB * TP], tv[TB * TP], ti[TB * TP], tj[TB * TP], tw[TB * TP];
    __shared__ double invd[TB];
    __shared__ int fail;
    if (*gate == 0 || *flag) return;
    const int I = blockIdx.x;
    if (I == 0) {
        load_tile(A, n, 0, 0, ta);
        __syncthreads();
        if (!tile_potrf_inv(ta, min(TB, n), Linv, invd, ti, tj, &fail)) {
            chol_fail(flag, gate);
            return;
        }
        store_tile(A, n, 0, 0, ta);
        return;
    }
    {
        TileRegs ra, rd;
        tile_fetch(A, n, I, 0, ra);
        tile_fetch(S, n, 0, 0, rd);
        tile_put(ta, ra);
        tile_put(td, rd);
    }
    __syncthreads();
    if (!tile_diag_again(n, 0, td, nullptr, tv, ti, tj, tw, invd, &fail)) {
        chol_fail(flag, gate);
        return;
    }
    tile_panel(A, n, I, 0, ta, tw);
}

// Step kt of the short chain: the trailing update A_IJ -= L_I,kt L_J,kt^T of
// every tile kt < J <= I (one per block, lower-triangle order); the block of
// tile (kt+1, kt+1) then factors it and writes its inverse, and the blocks of
// column kt + 1 form their panel tiles.
__global__ __launch_bounds__(256) void k_tchol_update_panel(int n, int kt, const double *__restrict__ S,
                                                            double *__restrict__ A, double *__restrict__ Linv,
                                                            int *__restrict__ flag, int *__restrict__ gate) {
    __shared__ double ti[TB * TP], tj[TB * TP], tc[TB * TP], td[TB * TP], tw[TB * TP];
    __shared__ double tm[(TCHOL_FUSE_N / TB - 1) * TB * TP];   // L_Jm, m < J (panel blocks)
    __shared__ double invd[TB];
    __shared__ int fail;
    if (*gate == 0 || *flag) return;
    const int b = blockIdx.x;
    int i = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= b) ++i;
    while (i * (i + 1) / 2 > b) --i;
    const int j = b - i * (i + 1) / 2;
    const int I = kt + 1 + i, J = kt + 1 + j;
    const bool panel = J == kt + 1 && I != J;
    // every load of the block in one batch: the update's tiles and, for a panel
    // block, S_JJ and the factor tiles L_Jm of the diagonal tile's row
    {
        constexpr int MM = TCHOL_FUSE_N / TB - 1;
        TileRegs ri, rj, rc, rd, rm[MM];
        tile_fetch(A, n, I, kt, ri);
        if (I != J) tile_fetch(A, n, J, kt, rj);
        tile_fetch(A, n, I, J, rc);
        if (panel) {
            tile_fetch(S, n, J, J, rd);
#pragma unroll
            for (int m = 0; m < MM; ++m)
                if (m < J) tile_fetch(A, n, J, m, rm[m]);
        }
        tile_put(ti, ri);
        if (I != J) tile_put(tj, rj);
        tile_put(tc, rc);
        if (panel) {
            tile_put(td, rd);
#pragma unroll
            for (int m = 0; m < MM; ++m)
                if (m < J) tile_put(tm + (size_t)m * TB * TP, rm[m]);
        }
    }
    __syncthreads();
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, qr = wv >> 1, qc = wv & 1;
    const f64x4 acc = quad_xyT(ti, I != J ? tj : ti, qr, qc);
#pragma unroll
    for (int q = 0; q < 4; ++q) tl(tc, 16 * qr + (l >> 4) + 4 * q, 16 * qc + (l & 15)) -= acc[q];
    __syncthreads();
    if (I == kt + 1 && J == kt + 1) {
        if (!tile_potrf_inv(tc, min(TB, n - TB * I), Linv + (size_t)I * TB * TB, invd, ti, tj, &fail)) {
            chol_fail(flag, gate);
            return;
        }
    } else if (panel) {
        if (!tile_diag_again(n, J, td, tm, tm, ti, tj, tw, invd, &fail)) {
            chol_fail(flag, gate);
            return;
        }
        tile_panel(A, n, I, J, tc, tw);
        return;
    }
    store_tile(A, n, I, J, tc);
}

// S^{-1} column by column from the tiled factor (one column per block; by
// symmetry it is stored as a row). Up to TINV_LDS_N unknowns every block first
// copies the packed factor into LDS, so that the tile steps read only LDS.
constexpr int TINV_LDS_DOUBLES = 18688;   // packed factor, column and solve scratch (146 KB)
constexpr int TINV_LDS_THREADS = 1024;
constexpr int tinv_lds_need(int n) { return n * (n + 1) / 2 + n + TILE_PACKED_TMP; }

__global__ __launch_bounds__(TINV_LDS_THREADS) void k_tinv_columns_lds(int n, const double *__restrict__ L,
                                                                      const double *__restrict__ Linv,
                                                                      double *__restrict__ Sinv,
                                                                      const int *__restrict__ flag,
                                                                      const int *__restrict__ gate) {
    __shared__ double lds[TINV_LDS_DOUBLES];
    if (*gate == 0 || *flag) return;
    double *Lp = lds, *x = Lp + n * (n + 1) / 2, *tmp = x + n;
    load_packed_lower<TINV_LDS_THREADS>(L, n, Lp);
    for (int col = blockIdx.x; col < n; col += gridDim.x) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = (i == col) ? 1.0 : 0.0;
        __syncthreads();
        tile_chol_solve_packed<TINV_LDS_THREADS>(Lp, Linv, n, x, tmp, col / TB);
        for (int i = threadIdx.x; i < n; i += blockDim.x) Sinv[(size_t)col * n + i] = x[i];
        __syncthreads();
    }
}

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

static void tsolve_ptrs(hipStream_t s, int n, const double *fac, const double *Linv, const double *b, double *x,
                        const int *flag) {
    const size_t lds = ((size_t)n + tile_solve_tmp(1024)) * sizeof(double);
    k_tsolve<<<1, 1024, lds, s>>>(n, fac, Linv, b, x, flag);
}

void launch_tsolve(hipStream_t s, Ctx &c, const double *b, double *x) {
    tsolve_ptrs(s, 6 * c.F, c.d_Sfac, c.d_Linv, b, x, c.d_flag);
}

// Tiled factorization of fac (which holds S on entry) in place; S itself is
// read again for the diagonal tiles of the short chain.
static void tchol_ptrs(hipStream_t s, int n, const double *S, double *fac, double *Linv, int *flag, int *gate) {
    const int nt = (n + TB - 1) / TB;
    if (n <= TCHOL_FUSE_N) {
        // S (unchanged by the factorization) holds the diagonal tiles' values
        k_tchol_first_panel<<<nt, 256, 0, s>>>(n, S, fac, Linv, flag, gate);
        for (int kt = 0; kt + 1 < nt; ++kt) {
            const int m = nt - kt - 1;
            k_tchol_update_panel<<<m * (m + 1) / 2, 256, 0, s>>>(n, kt, S, fac, Linv, flag, gate);
        }
        return;
    }
    k_tchol_first<<<1, 256, 0, s>>>(n, fac, Linv, flag, gate);
    for (int kt = 0; kt + 1 < nt; ++kt) {
        const int m = nt - kt - 1;
        k_tchol_panel<<<m, 256, 0, s>>>(n, kt, fac, Linv, flag, gate);
        k_tchol_update<<<m * (m + 1) / 2, 256, 0, s>>>(n, kt, fac, Linv, flag, gate);
    }
}

void launch_tchol(hipStream_t s, Ctx &c, bool copy) {
    const int n = 6 * c.F;
    const size_t nn = (size_t)n * n;
    if (copy) k_copy_d<<<(unsigned)((nn + 255) / 256), 256, 0, s>>>(c.d_S, c.d_Sfac, nn, c.d_gate);
    tchol_ptrs(s, n, c.d_S, c.d_Sfac, c.d_Linv, c.d_flag, c.d_gate);
}

void launch_tinv(hipStream_t s, Ctx &c) {
    const int n = 6 * c.F;
    if (tinv_lds_need(n) <= TINV_LDS_DOUBLES) {
        k_tinv_columns_lds<<<std::min(n, 2048), TINV_LDS_THREADS, 0, s>>>(n, c.d_Sfac, c.d_Linv, c.d_Sinv, c.d_flag, c.d_gate);
    } else {
        const size_t lds = ((size_t)n + tile_solve_tmp(256)) * sizeof(double);
        k_tinv_columns<<<std::min(n, 2048), 256, lds, s>>>(n, c.d_Sfac, c.d_Linv, c.d_Sinv, c.d_flag, c.d_gate);
    }
}

// ------------------------------------------------------------ solve without allocation
// Scratch of pba_solve_dense_noalloc: the factor (n x n), the inverses of its
// diagonal tiles, a failure flag and a gate, for systems of at most
// PBA_NOALLOC_MAX_N unknowns (4.9 MB). Each GPU the library runs on holds its
// own copy until the process ends; every call on that GPU shares it. In host
// code `scratch` names a host-side stand-in, never the device memory: kernels
// get the address that hipGetSymbolAddress returns for the current device.
constexpr int NOALLOC_NT = PBA_NOALLOC_MAX_N / TB;
static_assert(PBA_NOALLOC_MAX_N % TB == 0, "whole tiles");
constexpr size_t NOALLOC_FAC = (size_t)PBA_NOALLOC_MAX_N * PBA_NOALLOC_MAX_N;
constexpr size_t NOALLOC_LINV = (size_t)NOALLOC_NT * TB * TB;
constexpr size_t NOALLOC_DOUBLES = NOALLOC_FAC + NOALLOC_LINV + 2;   // + flag, gate (one int per double)
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_dev[NOALLOC_MAX_DEVICES];   // device address of `scratch` per device

// Copy S into the factor buffer; clear the failure flag and open the gate.
__global__ void k_noalloc_begin(int n, const double *__restrict__ S, double *__restrict__ fac,
                                int *__restrict__ flag, int *__restrict__ gate) {
    const size_t nn = (size_t)n * n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += (size_t)gridDim.x * blockDim.x)
        fac[i] = S[i];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *flag = 0;
        *gate = 1;
    }
}

__global__ void k_noalloc_info(const int *__restrict__ flag, int *__restrict__ info) {
    if (threadIdx.x == 0) *info = *flag ? 1 : 0;
}

// Copy M into the factor buffer; flag = 0 and the solve's gate open while
// `gate` is open, else flag = 2 (no solve; the kernels that read the flag skip).
__global__ void k_dense_begin(int n, const double *__restrict__ M, double *__restrict__ fac, int *__restrict__ flag,
                              const int *__restrict__ gate) {
    const int open = *gate != 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        flag[0] = open ? 0 : 2;
        flag[1] = open;
    }
    if (!open) return;
    const size_t nn = (size_t)n * n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += (size_t)gridDim.x * blockDim.x)
        fac[i] = M[i];
}

void launch_dense_solve(hipStream_t s, int n, const double *M, double *fac, double *Linv, const double *b, double *x,
                        int *flag, const int *gate) {
    const size_t nn = (size_t)n * n;
    k_dense_begin<<<(unsigned)std::min<size_t>(1024, (nn + 255) / 256), 256, 0, s>>>(n, M, fac, flag, gate);
    tchol_ptrs(s, n, M, fac, Linv, flag, flag + 1);
    tsolve_ptrs(s, n, fac, Linv, b, x, flag);
}

}  // namespace pba

extern "C" pba_status pba_solve_dense_noalloc(int32_t n, const double *S, const double *b, double *x,
                                              int32_t *info, void *stream) {
    using namespace pba;
    if (n < 1 || n > PBA_NOALLOC_MAX_N)
        return fail_global(PBA_E_INVALID, "n must be in 1..PBA_NOALLOC_MAX_N (768)");
    if (!S || !b || !x) return fail_global(PBA_E_INVALID, "S, b and x must be device pointers (not NULL)");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail_global(PBA_E_DEVICE, "no usable current device");
    double *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_dev[dev]) {
            void *p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p)
                return fail_global(PBA_E_DEVICE, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
            g_scratch_dev[dev] = static_cast<double *>(p);
        }
        base = g_scratch_dev[dev];
    }
    double *fac = base, *Linv = base + NOALLOC_FAC;
    int *flag = reinterpret_cast<int *>(base + NOALLOC_FAC + NOALLOC_LINV);
    int *gate = reinterpret_cast<int *>(base + NOALLOC_FAC + NOALLOC_LINV + 1);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t nn = (size_t)n * n;
    k_noalloc_begin<<<(unsigned)std::min<size_t>(1024, (nn + 255) / 256), 256, 0, s>>>(n, S, fac, flag, gate);
    tchol_ptrs(s, n, S, fac, Linv, flag, gate);
    tsolve_ptrs(s, n, fac, Linv, b, x, flag);
    if (info) k_noalloc_info<<<1, 64, 0, s>>>(flag, info);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail_global(PBA_E_DEVICE, std::string("launch: ") + hipGetErrorString(e));
    return PBA_OK;
}
