// Learned block preconditioner for PCG on the reduced pose system S x = -b,
// and the PCG iteration itself.
//
//  * block whitening of S (FP64): Cholesky factor of every 6x6 diagonal block,
//    its inverse, and the coupling G_i = sum_{j != i} S^_ij S^_ij^T of the
//    whitened system S^ = D S D^T, D = blockdiag(C_i^{-1});
//  * network 22 -> 256 -> 256 -> 21 (ReLU) on the features of G_i: inference
//    in FP16 on MFMA (v_mfma_f32_16x16x32_f16, FP32 accumulation), training in
//    FP32 (tiled GEMMs, the block loss and its gradient, Adam);
//  * output y -> lower factor L (exp on the diagonal), P^ = L L^T, block of
//    M^{-1}: P_i = C_i^{-T} P^ C_i^{-1} (y = 0 gives block Jacobi);
//  * PCG in FP64: a many-workgroup matrix-vector kernel and a one-workgroup
//    update kernel per iteration, with a device flag that ends the iteration.
#include "pba_device.hpp"
#include "pba_internal.hpp"

#include <algorithm>

namespace pba {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int upper_idx(int r, int c) {  // r <= c, row-major upper triangle of 6x6
    return r * 6 - r * (r - 1) / 2 + (c - r);
}
__device__ __forceinline__ int tri_idx(int r, int c) {  // c <= r, row-major lower triangle of 6x6
    return r * (r + 1) / 2 + c;
}

// ---------------------------------------------------------------- whitening

// One thread per block: C_i^{-1} (lower, full 6x6 row-major) of the Cholesky
// factor of S_ii. flag = 1 when a block is not positive definite.
__global__ void k_pc_block_inv(int nb, int n, const double *__restrict__ S, double *__restrict__ Ci,
                               int *__restrict__ flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    double L[6][6], X[6][6];
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) L[r][c] = c <= r ? S[(size_t)(6 * i + r) * n + 6 * i + c] : 0.0;
    for (int k = 0; k < 6; ++k) {
        double p = L[k][k];
        for (int q = 0; q < k; ++q) p -= L[k][q] * L[k][q];
        if (!(p > 0.0)) {
            *flag = 1;
            return;
        }
        L[k][k] = sqrt(p);
        for (int r = k + 1; r < 6; ++r) {
            double v = L[r][k];
            for (int q = 0; q < k; ++q) v -= L[r][q] * L[k][q];
            L[r][k] = v / L[k][k];
        }
    }
    for (int c = 0; c < 6; ++c)
        for (int r = 0; r < 6; ++r) {
            if (r < c) {
                X[r][c] = 0.0;
                continue;
            }
            double v = (r == c) ? 1.0 : 0.0;
            for (int q = c; q < r; ++q) v -= L[r][q] * X[q][c];
            X[r][c] = v / L[r][r];
        }
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) Ci[36 * (size_t)i + 6 * r + c] = X[r][c];
}

// One 64-lane workgroup per block row i: G_i (upper triangle, 21 values) and
// the 22 features, from the blocks j != i (lanes over j, fixed-order sums).
__global__ __launch_bounds__(64) void k_pc_coupling(int nb, int n, const double *__restrict__ S,
                                                    const double *__restrict__ Ci, double *__restrict__ G,
                                                    float *__restrict__ X, const int *__restrict__ flag) {
    if (*flag) return;
    const int i = blockIdx.x, lane = threadIdx.x;
    double Ai[6][6];
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) Ai[r][c] = Ci[36 * (size_t)i + 6 * r + c];
    double g[21];
    for (int k = 0; k < 21; ++k) g[k] = 0.0;
    for (int j = lane; j < nb; j += 64) {
        if (j == i) continue;
        double B[6][6];
        bool nz = false;
        for (int r = 0; r < 6; ++r)
            for (int c = 0; c < 6; ++c) {
                B[r][c] = S[(size_t)(6 * i + r) * n + 6 * j + c];
                nz = nz || B[r][c] != 0.0;
            }
        if (!nz) continue;
        const double *Aj = Ci + 36 * (size_t)j;
        double M[6][6], T[6][6];
        for (int r = 0; r < 6; ++r)  // M = C_i^{-1} S_ij
            for (int c = 0; c < 6; ++c) {
                double v = 0.0;
                for (int q = 0; q <= r; ++q) v += Ai[r][q] * B[q][c];
                M[r][c] = v;
            }
        for (int r = 0; r < 6; ++r)  // T = M C_j^{-T}
            for (int c = 0; c < 6; ++c) {
                double v = 0.0;
                for (int q = 0; q <= c; ++q) v += M[r][q] * Aj[6 * c + q];
                T[r][c] = v;
            }
        for (int r = 0; r < 6; ++r)
            for (int c = r; c < 6; ++c) {
                double v = 0.0;
                for (int q = 0; q < 6; ++q) v += T[r][q] * T[c][q];
                g[upper_idx(r, c)] += v;
            }
    }
    for (int k = 0; k < 21; ++k)
        for (int o = 32; o >= 1; o >>= 1) g[k] += __shfl_xor(g[k], o, 64);
    if (lane == 0) {
        const double tr = g[upper_idx(0, 0)] + g[upper_idx(1, 1)] + g[upper_idx(2, 2)] + g[upper_idx(3, 3)] +
                          g[upper_idx(4, 4)] + g[upper_idx(5, 5)];
        for (int k = 0; k < 21; ++k) {
            G[21 * (size_t)i + k] = g[k];
            X[22 * (size_t)i + k] = (float)(g[k] / (1.0 + tr));
        }
        X[22 * (size_t)i + 21] = (float)log1p(tr);
    }
}

// Features of given couplings (training samples): X from G (upper triangles).
__global__ void k_pc_features(int m, const float *__restrict__ G, float *__restrict__ X) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const float *g = G + 21 * (size_t)i;
    double tr = 0.0;
    for (int r = 0; r < 6; ++r) tr += (double)g[upper_idx(r, r)];
    for (int k = 0; k < 21; ++k) X[22 * (size_t)i + k] = (float)((double)g[k] / (1.0 + tr));
    X[22 * (size_t)i + 21] = (float)log1p(tr);
}

// ---------------------------------------------------------------- inference (FP16 MFMA)

// Padded FP16 copies of the weights: W1 [256][32] (inputs 22..31 zero),
// W2 [256][256], W3 [32][256] (outputs 21..31 zero); biases stay FP32.
__global__ void k_pc_to_half(const float *__restrict__ w, _Float16 *__restrict__ h) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const float *W1 = w, *W2 = w + PC_OFF_W2, *W3 = w + PC_OFF_W3;
    _Float16 *H1 = h, *H2 = h + 256 * 32, *H3 = H2 + 256 * 256;
    if (e < 256 * 32) {
        const int o = e / 32, k = e % 32;
        H1[e] = (_Float16)(k < PC_IN ? W1[o * PC_IN + k] : 0.0f);
    }
    if (e < 256 * 256) H2[e] = (_Float16)W2[e];
    if (e < 32 * 256) {
        const int o = e / 256, k = e % 256;
        H3[e] = (_Float16)(o < PC_OUT ? W3[o * 256 + k] : 0.0f);
    }
}

// One layer on a 16-row tile: out[16][NOUT] = act(in[16][K] W^T + b), the input
// tile in LDS (FP16, row pitch K + 8), W [NOUT][K] FP16 in global memory. Each
// wavefront computes 16-column output tiles; lane layout of the 16x16x32 MFMA:
// A[row = l % 16][k = 8 (l / 16) + i], B[k = 8 (l / 16) + i][col = l % 16],
// result row 4 (l / 16) + i, column l % 16.
template <int K, int NOUT, bool RELU, bool OUT_HALF>
__device__ __forceinline__ void mlp_layer(const _Float16 *in, const _Float16 *__restrict__ W,
                                          const float *__restrict__ bias, int nbias, void *out, int out_pitch) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int ct = wv; ct < NOUT / 16; ct += nw) {
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k0 = 0; k0 < K; k0 += 32) {
            const int kk = k0 + 8 * (lane >> 4);
            const f16x8 a = *reinterpret_cast<const f16x8 *>(in + (lane & 15) * (K + 8) + kk);
            const f16x8 b = *reinterpret_cast<const f16x8 *>(W + (size_t)(16 * ct + (lane & 15)) * K + kk);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc, 0, 0, 0);
        }
        const int col = 16 * ct + (lane & 15);
        const float bb = col < nbias ? bias[col] : 0.0f;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = 4 * (lane >> 4) + q;
            float v = acc[q] + bb;
            if (RELU) v = fmaxf(v, 0.0f);
            if (OUT_HALF)
                static_cast<_Float16 *>(out)[row * out_pitch + col] = (_Float16)v;
            else
                static_cast<float *>(out)[row * out_pitch + col] = v;
        }
    }
}

__global__ __launch_bounds__(256) void k_pc_infer(int m, const float *__restrict__ X,
                                                  const _Float16 *__restrict__ Wh, const float *__restrict__ w,
                                                  float *__restrict__ Y) {
    __shared__ __attribute__((aligned(16))) _Float16 x0[16 * (32 + 8)];
    __shared__ __attribute__((aligned(16))) _Float16 h1[16 * (256 + 8)];
    __shared__ __attribute__((aligned(16))) _Float16 h2[16 * (256 + 8)];
    __shared__ float y[16 * 32];
    const int r0 = 16 * blockIdx.x;
    for (int e = threadIdx.x; e < 16 * 32; e += blockDim.x) {
        const int r = e / 32, k = e % 32;
        x0[r * 40 + k] = (_Float16)((r0 + r < m && k < PC_IN) ? X[(size_t)(r0 + r) * PC_IN + k] : 0.0f);
    }
    __syncthreads();
    const _Float16 *W1 = Wh, *W2 = Wh + 256 * 32, *W3 = W2 + 256 * 256;
    mlp_layer<32, 256, true, true>(x0, W1, w + PC_OFF_B1, 256, h1, 264);
    __syncthreads();
    mlp_layer<256, 256, true, true>(h1, W2, w + PC_OFF_B2, 256, h2, 264);
    __syncthreads();
    mlp_layer<256, 32, false, false>(h2, W3, w + PC_OFF_B3, PC_OUT, y, 32);
    __syncthreads();
    for (int e = threadIdx.x; e < 16 * PC_OUT; e += blockDim.x) {
        const int r = e / PC_OUT, k = e % PC_OUT;
        if (r0 + r < m) Y[(size_t)(r0 + r) * PC_OUT + k] = y[r * 32 + k];
    }
}

// Blocks of M^{-1}: P_i = C_i^{-T} L L^T C_i^{-1}, L from the output (Y = NULL:
// L = I, block Jacobi).
__global__ void k_pc_blocks(int nb, const float *__restrict__ Y, const double *__restrict__ Ci,
                            double *__restrict__ P) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    double L[6][6];
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) {
            if (c > r)
                L[r][c] = 0.0;
            else if (!Y)
                L[r][c] = (r == c) ? 1.0 : 0.0;
            else {
                const double y = (double)Y[(size_t)i * PC_OUT + tri_idx(r, c)];
                L[r][c] = (r == c) ? exp(y) : y;
            }
        }
    // U = L^T C_i^{-1}; P = U^T U
    const double *A = Ci + 36 * (size_t)i;
    double U[6][6];
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) {
            double v = 0.0;
            for (int q = r; q < 6; ++q) v += L[q][r] * A[6 * q + c];
            U[r][c] = v;
        }
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) {
            double v = 0.0;
            for (int q = 0; q < 6; ++q) v += U[q][r] * U[q][c];
            P[36 * (size_t)i + 6 * r + c] = v;
        }
}

// Blocks of M^{-1} at the minimizer of the block loss itself: tr(P A P) -
// 2 tr P with A = I + G_i is smallest at P^ = A^{-1}, so P_i = C_i^{-T}
// (I + G_i)^{-1} C_i^{-1} = (X C_i^{-1})^T (X C_i^{-1}) with X = R^{-1} and
// A = R R^T (the bound a trained network approaches).
__global__ void k_pc_blocks_opt(int nb, const double *__restrict__ G, const double *__restrict__ Ci,
                                double *__restrict__ P, int *__restrict__ flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    double A[6][6], R[6][6], X[6][6];
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c)
            A[r][c] = (r == c ? 1.0 : 0.0) + G[21 * (size_t)i + (r <= c ? upper_idx(r, c) : upper_idx(c, r))];
    for (int c = 0; c < 6; ++c) {
        double d = A[c][c];
        for (int q = 0; q < c; ++q) d -= R[c][q] * R[c][q];
        if (!(d > 0.0)) {
            *flag = 1;
            return;
        }
        R[c][c] = sqrt(d);
        for (int r = c + 1; r < 6; ++r) {
            double v = A[r][c];
            for (int q = 0; q < c; ++q) v -= R[r][q] * R[c][q];
            R[r][c] = v / R[c][c];
        }
    }
    for (int c = 0; c < 6; ++c)
        for (int r = 0; r < 6; ++r) {
            if (r < c) {
                X[r][c] = 0.0;
                continue;
            }
            double v = (r == c) ? 1.0 : 0.0;
            for (int q = c; q < r; ++q) v -= R[r][q] * X[q][c];
            X[r][c] = v / R[r][r];
        }
    const double *B = Ci + 36 * (size_t)i;
    double W[6][6];   // X C_i^{-1} (both lower)
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) {
            double v = 0.0;
            for (int q = c; q <= r; ++q) v += X[r][q] * B[6 * q + c];
            W[r][c] = v;
        }
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) {
            double v = 0.0;
            for (int q = 0; q < 6; ++q) v += W[q][r] * W[q][c];
            P[36 * (size_t)i + 6 * r + c] = v;
        }
}

// ---------------------------------------------------------------- training (FP32)

// C[M][N] = op(A) op(B) (+ epilogue), 16 x 16 output tile per 256-thread block,
// one output per thread, K in LDS chunks of 16. op(A)[m][k] = TA ? A[k * lda + m]
// : A[m * lda + k]; op(B)[k][n] = TB ? B[n * ldb + k] : B[k * ldb + n].
// EPI 0: C = AB; 1: C = AB + bias[n]; 2: C = relu(AB + bias[n]) with the
// pre-activation stored in Z; 3: C = AB * (Zmask[m][n] > 0).
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float *__restrict__ A, int lda,
                                              const float *__restrict__ B, int ldb, float *__restrict__ C, int ldc,
                                              const float *__restrict__ bias, float *__restrict__ Z, int ldz) {
    __shared__ float as[16][17], bs[16][17];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int m = 16 * blockIdx.y + ty, n = 16 * blockIdx.x + tx;
    float acc = 0.0f;
    for (int k0 = 0; k0 < K; k0 += 16) {
        {
            const int mm = 16 * blockIdx.y + ty, kk = k0 + tx;
            as[ty][tx] = (mm < M && kk < K) ? (TA ? A[(size_t)kk * lda + mm] : A[(size_t)mm * lda + kk]) : 0.0f;
            const int k2 = k0 + ty, n2 = 16 * blockIdx.x + tx;
            bs[ty][tx] = (k2 < K && n2 < N) ? (TB ? B[(size_t)n2 * ldb + k2] : B[(size_t)k2 * ldb + n2]) : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; ++q) acc += as[ty][q] * bs[q][tx];
        __syncthreads();
    }
    if (m < M && n < N) {
        if (EPI == 1) acc += bias[n];
        if (EPI == 2) {
            acc += bias[n];
            Z[(size_t)m * ldz + n] = acc;
            acc = fmaxf(acc, 0.0f);
        }
        if (EPI == 3) acc = Z[(size_t)m * ldz + n] > 0.0f ? acc : 0.0f;
        C[(size_t)m * ldc + n] = acc;
    }
}

// Column sums (bias gradients): out[n] = sum_m A[m][n], in a fixed order:
// COLSUM_COLS columns per 1024-thread block, 16 row groups (rows g, g + 16, ...,
// loads unrolled) whose partials are added in group order.
constexpr int COLSUM_COLS = 64, COLSUM_GROUPS = 16;

__global__ __launch_bounds__(1024) void k_colsum(int M, int N, const float *__restrict__ A, float *__restrict__ out) {
    __shared__ float part[COLSUM_GROUPS][COLSUM_COLS];
    const int c = threadIdx.x % COLSUM_COLS, g = threadIdx.x / COLSUM_COLS;
    const int n = blockIdx.x * COLSUM_COLS + c;
    float s = 0.0f;
    if (n < N) {
#pragma unroll 8
        for (int m = g; m < M; m += COLSUM_GROUPS) s += A[(size_t)m * N + n];
    }
    part[g][c] = s;
    __syncthreads();
    if (g == 0 && n < N) {
        float t = 0.0f;
        for (int k = 0; k < COLSUM_GROUPS; ++k) t += part[k][c];
        out[n] = t;
    }
}

// Block loss l = tr(P A P) - 2 tr(P) + 6 (A = I + G, P = L L^T) of every
// sample and dl/dy scaled by `scale` (1 / batch); per-block losses to lossv.
__global__ void k_pc_loss(int m, const float *__restrict__ Y, const float *__restrict__ G, float scale,
                          float *__restrict__ dY, float *__restrict__ lossv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    float L[6][6], A[6][6], P[6][6], PA[6][6], D[6][6];
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) {
            if (c > r)
                L[r][c] = 0.0f;
            else {
                const float y = Y[(size_t)i * PC_OUT + tri_idx(r, c)];
                L[r][c] = (r == c) ? expf(y) : y;
            }
            const int a = r < c ? r : c, b = r < c ? c : r;
            A[r][c] = G[(size_t)i * 21 + upper_idx(a, b)] + (r == c ? 1.0f : 0.0f);
        }
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) {
            float v = 0.0f;
            for (int q = 0; q < 6; ++q) v += L[r][q] * L[c][q];
            P[r][c] = v;
        }
    float loss = 6.0f;
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) {
            float v = 0.0f;
            for (int q = 0; q < 6; ++q) v += P[r][q] * A[q][c];
            PA[r][c] = v;
        }
    for (int r = 0; r < 6; ++r) {
        for (int q = 0; q < 6; ++q) loss += PA[r][q] * P[q][r];
        loss -= 2.0f * P[r][r];
    }
    // dP = 2 P A - 2 I; dL = (dP + dP^T) L
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) D[r][c] = 2.0f * (PA[r][c] + PA[c][r]) - (r == c ? 4.0f : 0.0f);
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c <= r; ++c) {
            float v = 0.0f;
            for (int q = 0; q < 6; ++q) v += D[r][q] * L[q][c];
            dY[(size_t)i * PC_OUT + tri_idx(r, c)] = scale * (r == c ? v * L[r][c] : v);
        }
    lossv[i] = loss;
}

__global__ void k_gather_rows(int m, const int *__restrict__ idx, const float *__restrict__ src, int width,
                              float *__restrict__ dst) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m * width) return;
    const int r = e / width, k = e % width;
    dst[e] = src[(size_t)idx[r] * width + k];
}

__global__ void k_adam(int n, float *__restrict__ w, const float *__restrict__ g, float *__restrict__ mo,
                       float *__restrict__ ve, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float m = b1 * mo[i] + (1.0f - b1) * gi;
    const float v = b2 * ve[i] + (1.0f - b2) * gi * gi;
    mo[i] = m;
    ve[i] = v;
    w[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// Sum of n floats by one block (fixed order).
__global__ __launch_bounds__(256) void k_sum_f(int n, const float *__restrict__ v, double *__restrict__ out) {
    __shared__ double red[4];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += (double)v[i];
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *out = red[0] + red[1] + red[2] + red[3];
}

// ---------------------------------------------------------------- PCG (FP64)

constexpr int PCG_ROWS = 8;  // rows of S per workgroup in the product

__device__ __forceinline__ void apply_block(const double *P, const double *r, double *z, int n, int t, int nt) {
    for (int e = t; e < n; e += nt) {
        const int i = e / 6, a = e % 6;
        const double *Pi = P + 36 * (size_t)i + 6 * a;
        const double *ri = r + 6 * i;
        double v = 0.0;
        for (int q = 0; q < 6; ++q) v += Pi[q] * ri[q];
        z[e] = v;
    }
}

template <int NV>
__device__ __forceinline__ void bsum(double (&v)[NV], double *red) {  // 1024 threads, result in all threads
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int p = 0; p < NV; ++p)
        for (int o = 32; o >= 1; o >>= 1) v[p] += __shfl_xor(v[p], o, 64);
    __syncthreads();
    if (lane == 0)
        for (int p = 0; p < NV; ++p) red[wv * NV + p] = v[p];
    __syncthreads();
    for (int p = 0; p < NV; ++p) {
        double s = 0.0;
        for (int k = 0; k < nw; ++k) s += red[k * NV + p];
        v[p] = s;
    }
}

// x = 0, r = -b, z = M^{-1} r, p = z; sc = {r.z, |b|^2, |r|^2}; done = 0, iters = 0.
__global__ __launch_bounds__(1024) void k_pcg_init(int n, const double *__restrict__ b, const double *__restrict__ P,
                                                   double *__restrict__ x, double *__restrict__ r,
                                                   double *__restrict__ z, double *__restrict__ p,
                                                   double *__restrict__ sc, int *__restrict__ st) {
    __shared__ double red[16 * 2];
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        x[e] = 0.0;
        r[e] = -b[e];
    }
    __syncthreads();
    apply_block(P, r, z, n, threadIdx.x, blockDim.x);
    __syncthreads();
    double v[2] = {0.0, 0.0};
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        p[e] = z[e];
        v[0] += r[e] * z[e];
        v[1] += r[e] * r[e];
    }
    bsum<2>(v, red);
    if (threadIdx.x == 0) {
        sc[0] = v[0];
        sc[1] = v[1];
        sc[2] = v[1];
        st[0] = v[1] > 0.0 ? 0 : 1;  // done
        st[1] = 0;                   // iterations
    }
}

// q = S p over PCG_ROWS rows per workgroup (a wavefront per row), and the
// workgroup's part of p.q. A lane reads two columns per step (16-byte loads:
// n = 6 F is even, so every row starts 16-byte aligned), four steps unrolled
// so that their loads are in flight together.
__global__ __launch_bounds__(64 * PCG_ROWS) void k_pcg_matvec(int n, const double *__restrict__ S,
                                                              const double *__restrict__ p, double *__restrict__ q,
                                                              double *__restrict__ part, const int *__restrict__ st) {
    __shared__ double red[PCG_ROWS];
    if (st[0]) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int row = PCG_ROWS * blockIdx.x + wv;
    double s = 0.0;
    if (row < n) {
        const double2 *S2 = reinterpret_cast<const double2 *>(S + (size_t)row * n);
        const double2 *p2 = reinterpret_cast<const double2 *>(p);
        const int n2 = n >> 1;
#pragma unroll 4
        for (int c = lane; c < n2; c += 64) {
            const double2 a = S2[c], b = p2[c];
            s += a.x * b.x + a.y * b.y;
        }
    }
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) {
        if (row < n) q[row] = s;
        red[wv] = row < n ? s * p[row] : 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < PCG_ROWS; ++k) t += red[k];
        part[blockIdx.x] = t;
    }
}

// alpha = r.z / p.q; x += alpha p; r -= alpha q; stop when |r|^2 <= tol^2 |b|^2;
// else z = M^{-1} r, beta = r.z' / r.z, p = z + beta p.
__global__ __launch_bounds__(1024) void k_pcg_update(int n, int nparts, const double *__restrict__ part,
                                                     const double *__restrict__ P, double *__restrict__ x,
                                                     double *__restrict__ r, double *__restrict__ z,
                                                     double *__restrict__ p, const double *__restrict__ q,
                                                     double *__restrict__ sc, int *__restrict__ st, double tol2) {
    __shared__ double red[16 * 2];
    if (st[0]) return;
    double v1[1] = {0.0};
    for (int k = threadIdx.x; k < nparts; k += blockDim.x) v1[0] += part[k];
    bsum<1>(v1, red);
    const double pq = v1[0];
    const double alpha = sc[0] / pq;
    double v[1] = {0.0};
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        x[e] += alpha * p[e];
        const double re = r[e] - alpha * q[e];
        r[e] = re;
        v[0] += re * re;
    }
    bsum<1>(v, red);
    const double rr = v[0];
    const bool done = !(rr > tol2 * sc[1]);
    __syncthreads();
    if (threadIdx.x == 0) {
        sc[2] = rr;
        st[1] += 1;
    }
    if (done) {
        if (threadIdx.x == 0) st[0] = 1;
        return;
    }
    apply_block(P, r, z, n, threadIdx.x, blockDim.x);
    __syncthreads();
    double w[1] = {0.0};
    for (int e = threadIdx.x; e < n; e += blockDim.x) w[0] += r[e] * z[e];
    bsum<1>(w, red);
    const double beta = w[0] / sc[0];
    for (int e = threadIdx.x; e < n; e += blockDim.x) p[e] = z[e] + beta * p[e];
    __syncthreads();
    if (threadIdx.x == 0) sc[0] = w[0];
}

// Partial sums of (S x + b)_i^2 over PCG_ROWS rows per workgroup.
__global__ __launch_bounds__(256) void k_resid(int n, const double *__restrict__ S, const double *__restrict__ x,
                                               const double *__restrict__ b, double *__restrict__ part) {
    __shared__ double red[PCG_ROWS];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int rr = wv; rr < PCG_ROWS; rr += 4) {
        const int row = PCG_ROWS * blockIdx.x + rr;
        double s = 0.0;
        if (row < n) {
            const double *Sr = S + (size_t)row * n;
            for (int c = lane; c < n; c += 64) s += Sr[c] * x[c];
        }
        for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) red[rr] = row < n ? (s + b[row]) * (s + b[row]) : 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < PCG_ROWS; ++k) t += red[k];
        part[blockIdx.x] = t;
    }
}

// ---------------------------------------------------------------- launchers

void pc_resid(hipStream_t s, Ctx &c, int n, const double *x, double *part) {
    k_resid<<<(n + PCG_ROWS - 1) / PCG_ROWS, 256, 0, s>>>(n, c.d_S, x, c.d_b, part);
}

static inline unsigned nbk(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

void pc_whiten(hipStream_t s, Ctx &c, int nb) {
    const int n = 6 * nb;
    k_pc_block_inv<<<nbk(nb, 64), 64, 0, s>>>(nb, n, c.d_S, c.pc.Ci, c.pc.flag);
    k_pc_coupling<<<nb, 64, 0, s>>>(nb, n, c.d_S, c.pc.Ci, c.pc.G, c.pc.X, c.pc.flag);
}

void pc_infer(hipStream_t s, Ctx &c, int m, const float *X, float *Y) {
    k_pc_infer<<<nbk(m, 16), 256, 0, s>>>(m, X, c.pc.wh, c.pc.w, Y);
}

void pc_blocks(hipStream_t s, Ctx &c, int nb, const float *Y) {
    k_pc_blocks<<<nbk(nb, 64), 64, 0, s>>>(nb, Y, c.pc.Ci, c.pc.P);
}

void pc_blocks_opt(hipStream_t s, Ctx &c, int nb) {
    k_pc_blocks_opt<<<nbk(nb, 64), 64, 0, s>>>(nb, c.pc.G, c.pc.Ci, c.pc.P, c.pc.flag);
}

void pc_to_half(hipStream_t s, Ctx &c) { k_pc_to_half<<<nbk(256 * 256, 256), 256, 0, s>>>(c.pc.w, c.pc.wh); }

void pc_features(hipStream_t s, int m, const float *G, float *X) {
    if (m > 0) k_pc_features<<<nbk(m, 256), 256, 0, s>>>(m, G, X);
}

void pc_gather(hipStream_t s, int m, const int *idx, const float *src, int width, float *dst) {
    if (m > 0) k_gather_rows<<<nbk((size_t)m * width, 256), 256, 0, s>>>(m, idx, src, width, dst);
}

// Forward and backward over a batch of m samples (X [m][22], G [m][21]) with the
// FP32 weights: the gradient (PC_N_PARAMS floats, packed like the weights) of
// the mean block loss, and the per-sample losses in lossv.
void pc_forward_backward(hipStream_t s, Ctx &c, int m, const float *X, const float *G, float *grad, float *lossv) {
    PcState &p = c.pc;
    const float *w = p.w;
    const dim3 t(256);
    auto grid = [](int M, int N) { return dim3((unsigned)((N + 15) / 16), (unsigned)((M + 15) / 16)); };
    // forward: Z1 = X W1^T + b1, H1 = relu(Z1); Z2, H2; Y = H2 W3^T + b3
    k_gemm<false, true, 2><<<grid(m, 256), t, 0, s>>>(m, 256, PC_IN, X, PC_IN, w, PC_IN, p.H1, 256, w + PC_OFF_B1,
                                                      p.Z1, 256);
    k_gemm<false, true, 2><<<grid(m, 256), t, 0, s>>>(m, 256, 256, p.H1, 256, w + PC_OFF_W2, 256, p.H2, 256,
                                                      w + PC_OFF_B2, p.Z2, 256);
    k_gemm<false, true, 1><<<grid(m, PC_OUT), t, 0, s>>>(m, PC_OUT, 256, p.H2, 256, w + PC_OFF_W3, 256, p.Yt, PC_OUT,
                                                         w + PC_OFF_B3, nullptr, 0);
    k_pc_loss<<<nbk(m, 256), 256, 0, s>>>(m, p.Yt, G, 1.0f / (float)m, p.dY, lossv);
    // backward
    k_gemm<true, false, 0><<<grid(PC_OUT, 256), t, 0, s>>>(PC_OUT, 256, m, p.dY, PC_OUT, p.H2, 256, grad + PC_OFF_W3,
                                                           256, nullptr, nullptr, 0);
    k_colsum<<<nbk(PC_OUT, COLSUM_COLS), 1024, 0, s>>>(m, PC_OUT, p.dY, grad + PC_OFF_B3);
    k_gemm<false, false, 3><<<grid(m, 256), t, 0, s>>>(m, 256, PC_OUT, p.dY, PC_OUT, w + PC_OFF_W3, 256, p.D2, 256,
                                                       nullptr, p.Z2, 256);
    k_gemm<true, false, 0><<<grid(256, 256), t, 0, s>>>(256, 256, m, p.D2, 256, p.H1, 256, grad + PC_OFF_W2, 256,
                                                        nullptr, nullptr, 0);
    k_colsum<<<nbk(256, COLSUM_COLS), 1024, 0, s>>>(m, 256, p.D2, grad + PC_OFF_B2);
    k_gemm<false, false, 3><<<grid(m, 256), t, 0, s>>>(m, 256, 256, p.D2, 256, w + PC_OFF_W2, 256, p.D1, 256, nullptr,
                                                       p.Z1, 256);
    k_gemm<true, false, 0><<<grid(256, PC_IN), t, 0, s>>>(256, PC_IN, m, p.D1, 256, X, PC_IN, grad, PC_IN, nullptr,
                                                          nullptr, 0);
    k_colsum<<<nbk(256, COLSUM_COLS), 1024, 0, s>>>(m, 256, p.D1, grad + PC_OFF_B1);
}

void pc_adam(hipStream_t s, Ctx &c, float lr, float b1, float b2, float eps, int step) {
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    k_adam<<<nbk(PC_N_PARAMS, 256), 256, 0, s>>>(PC_N_PARAMS, c.pc.w, c.pc.grad, c.pc.m, c.pc.v, lr, b1, b2, eps,
                                                 c1, c2);
}

void pc_sum(hipStream_t s, int n, const float *v, double *out) { k_sum_f<<<1, 256, 0, s>>>(n, v, out); }

void pcg_init(hipStream_t s, Ctx &c, int n) {
    PcState &p = c.pc;
    k_pcg_init<<<1, 1024, 0, s>>>(n, c.d_b, p.P, p.x, p.r, p.z, p.p, p.sc, p.st);
}

void pcg_iterations(hipStream_t s, Ctx &c, int n, int k, double tol) {
    PcState &p = c.pc;
    const int parts = (n + PCG_ROWS - 1) / PCG_ROWS;
    for (int i = 0; i < k; ++i) {
        k_pcg_matvec<<<parts, 64 * PCG_ROWS, 0, s>>>(n, c.d_S, p.p, p.q, p.part, p.st);
        k_pcg_update<<<1, 1024, 0, s>>>(n, parts, p.part, p.P, p.x, p.r, p.z, p.p, p.q, p.sc, p.st, tol * tol);
    }
}

}  // namespace pba
