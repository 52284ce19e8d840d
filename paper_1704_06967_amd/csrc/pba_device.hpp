// Device-side math of libpba: bilinear image functions, warps, the proxy-template
// and forward-compositional Jacobian rows, and small 6x6 helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>


namespace pba {

struct PatternArg {
    int n;
    int du[8];
    int dv[8];
};

template <typename T>
__device__ __forceinline__ bool usable(T u, T v, int W, int H) {
    return u >= T(1) && u <= T(W - 3) && v >= T(1) && v <= T(H - 3);
}

// Bilinear interpolation of a row-major image at (u, v) (Notation: image
// functions are bilinear interpolants of the pixel grid), formed in FP64 from
// the image's texels for every element type. The position comes in T or in
// FP64 (P) and the cell is found in P. In FP64 the interpolant of FP32 texels
// at an FP64 position is exact to rounding, so the single-precision paths
// round the residual r = I0 - I once, at the end (to 1e-9 for |r| ~ 0.01),
// where an FP32 interpolation would carry ~1e-7 of rounding, and an FP32
// pixel coordinate near 600 another ~3e-5 px times the gradient.
// The interpolant from the cell's texels (t00 t01 / t10 t11) and the position's
// fractions (a along the row, b down the column).
template <typename T>
__device__ __forceinline__ double bilerp(double a, double b, T t00, T t01, T t10, T t11) {
    return (1.0 - a) * (1.0 - b) * (double)t00 + a * (1.0 - b) * (double)t01 + (1.0 - a) * b * (double)t10 +
           a * b * (double)t11;
}

template <typename T, typename P>
__device__ __forceinline__ double bilinear(const T *__restrict__ im, int W, P u, P v) {
    const int j0 = (int)floor(u), i0 = (int)floor(v);
    const double a = (double)u - (double)j0, b = (double)v - (double)i0;
    const T *r0 = im + (size_t)i0 * W + j0;
    const T *r1 = r0 + W;
    return bilerp(a, b, r0[0], r0[1], r1[0], r1[1]);
}

// Reciprocals. In single precision the hardware's (within 1 ulp), which is
// what the element type carries anyway; in FP64 the correctly rounded one.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// FP64 reciprocal from the hardware's approximation and two Newton steps
// (each squares the relative error), within an ulp of 1/x for the positive,
// normal x of a projection depth.
__device__ __forceinline__ double recip_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// Intensity and gradient at (u, v): the gradient is the central difference on
// the grid, bilinearly interpolated between the four surrounding pixel centres.
// Both interpolants in FP64 from the texels (the differences of neighbouring
// texels are formed in T, exactly when they are within a factor of two), so
// that a single-precision caller rounds the gradient, or the Jacobian made
// from it, once: an interpolated gradient that is small against its four
// corners (and a Jacobian entry that cancels, such as J_d = q . t for a
// gradient across the epipolar line) would otherwise carry the corners'
// rounding, amplified.
template <typename T, typename P>
__device__ __forceinline__ void bilinear_grad(const T *__restrict__ im, int W, P u, P v, double &I, double &gu,
                                              double &gv) {
    const int j0 = (int)floor(u), i0 = (int)floor(v);
    const double a = (double)u - (double)j0, b = (double)v - (double)i0;
    const T *rm = im + (size_t)(i0 - 1) * W + j0;  // row i0-1
    const T *r0 = rm + W;
    const T *r1 = r0 + W;
    const T *r2 = r1 + W;
    I = bilerp(a, b, r0[0], r0[1], r1[0], r1[1]);
    gu = 0.5 * bilerp(a, b, r0[1] - r0[-1], r0[2] - r0[0], r1[1] - r1[-1], r1[2] - r1[0]);
    gv = 0.5 * bilerp(a, b, r1[0] - rm[0], r1[1] - rm[1], r2[0] - r0[0], r2[1] - r0[1]);
}

// Huber IRLS weight and norm (eq:energy).
template <typename T>
__device__ __forceinline__ void huber(T r, T k, T &w, T &rho) {
    const T a = fabs(r);
    if (a <= k) {
        w = T(1);
        rho = T(0.5) * r * r;
    } else {
        if constexpr (sizeof(T) == 4)
            w = k * recip(a);
        else
            w = k / a;
        rho = k * a - T(0.5) * k * k;
    }
}

// Inverse-compositional Jacobian row with proxy templates (Sec. 3.4, 3.5):
// J = [fx gu, fy gv] d phi / d dp at dp = 0, with
//   d phi / d dp = (1/zb) [[1, 0, -x], [0, 1, -y]] [-M [R0 x~]_x | d0 M | M t0],
//   M = R0^T (zb I - t0 e3^T),  zb = [R0 x~ + d0 t0]_z / d0.
// With q = (1/zb)(a0, a1, -a0 x - a1 y) and m = M^T q = zb R0 q - (t0 . R0 q) e3
// the row is J_w = (R0 x~) x m, J_t = d0 m, J_d = m . t0.
// id0 = 1 / d0 (formed once per point by the caller).
template <typename T>
__device__ __forceinline__ void ic_jacobian(T x, T y, const T *R0, const T *t0, T d0, T id0, T gu, T gv, T fx,
                                            T fy, T J[7]) {
    const T Rx0 = R0[0] * x + R0[1] * y + R0[2];
    const T Rx1 = R0[3] * x + R0[4] * y + R0[5];
    const T Rx2 = R0[6] * x + R0[7] * y + R0[8];
    const T zb = (Rx2 + d0 * t0[2]) * id0;
    const T iz = recip(zb);
    const T a0 = fx * gu, a1 = fy * gv;
    const T q0 = a0 * iz, q1 = a1 * iz, q2 = -(a0 * x + a1 * y) * iz;
    const T Rq0 = R0[0] * q0 + R0[1] * q1 + R0[2] * q2;
    const T Rq1 = R0[3] * q0 + R0[4] * q1 + R0[5] * q2;
    const T Rq2 = R0[6] * q0 + R0[7] * q1 + R0[8] * q2;
    const T m0 = zb * Rq0, m1 = zb * Rq1;
    const T m2 = zb * Rq2 - (Rq0 * t0[0] + Rq1 * t0[1] + Rq2 * t0[2]);
    J[0] = Rx1 * m2 - Rx2 * m1;
    J[1] = Rx2 * m0 - Rx0 * m2;
    J[2] = Rx0 * m1 - Rx1 * m0;
    J[3] = d0 * m0;
    J[4] = d0 * m1;
    J[5] = d0 * m2;
    J[6] = m0 * t0[0] + m1 * t0[1] + m2 * t0[2];
}

// Forward-compositional Jacobian row of r = I0 - I_f(W) at the current
// parameters: J = -[fx gu, fy gv] (1/v_z)[[1,0,-u_x],[0,1,-u_y]] [-[R x~]_x | d I | t],
// i.e. with q = -(1/v_z)(a0, a1, -a0 u_x - a1 u_y): J_w = (R x~) x q, J_t = d q, J_d = q . t.
template <typename T>
__device__ __forceinline__ void fc_jacobian(T Rx0, T Rx1, T Rx2, T vz, T ux, T uy, const T *t, T d, T gu, T gv,
                                            T fx, T fy, T J[7]) {
    const T a0 = fx * gu, a1 = fy * gv;
    const T iz = -T(1) / vz;
    const T q0 = a0 * iz, q1 = a1 * iz, q2 = -(a0 * ux + a1 * uy) * iz;
    J[0] = Rx1 * q2 - Rx2 * q1;
    J[1] = Rx2 * q0 - Rx0 * q2;
    J[2] = Rx0 * q1 - Rx1 * q0;
    J[3] = d * q0;
    J[4] = d * q1;
    J[5] = d * q2;
    J[6] = q0 * t[0] + q1 * t[1] + q2 * t[2];
}

// Constant maps from absolute left increments of target f and host h to the
// left increment of their relative pose R_fh = R_f R_h^T, t_fh = t_f - R_fh t_h:
//   A = [[I, 0], [[R_fh t_h]_x, I]],  B = [[-R_fh, 0], [-R_fh [t_h]_x, -R_fh]].
__device__ __forceinline__ void abs_maps(const double *geo, double A[36], double B[36]) {
    const double *R = geo;
    const double *th = geo + 12;
    const double Rt0 = R[0] * th[0] + R[1] * th[1] + R[2] * th[2];
    const double Rt1 = R[3] * th[0] + R[4] * th[1] + R[5] * th[2];
    const double Rt2 = R[6] * th[0] + R[7] * th[1] + R[8] * th[2];
    for (int i = 0; i < 36; ++i) {
        A[i] = 0.0;
        B[i] = 0.0;
    }
    for (int i = 0; i < 6; ++i) A[i * 6 + i] = 1.0;
    // [R t_h]_x in the lower-left block of A
    A[3 * 6 + 1] = -Rt2;
    A[3 * 6 + 2] = Rt1;
    A[4 * 6 + 0] = Rt2;
    A[4 * 6 + 2] = -Rt0;
    A[5 * 6 + 0] = -Rt1;
    A[5 * 6 + 1] = Rt0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            B[i * 6 + j] = -R[i * 3 + j];
            B[(i + 3) * 6 + (j + 3)] = -R[i * 3 + j];
        }
    // -R [t_h]_x
    const double K[9] = {0.0, -th[2], th[1], th[2], 0.0, -th[0], -th[1], th[0], 0.0};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += R[i * 3 + k] * K[k * 3 + j];
            B[(i + 3) * 6 + j] = -s;
        }
}

// Entry (i, j) of [v]_x for v given by a callable component getter.
__device__ __forceinline__ double cross_entry(double v0, double v1, double v2, int i, int j) {
    if (i == j) return 0.0;
    const int m = 3 - i - j;
    const double vm = m == 0 ? v0 : (m == 1 ? v1 : v2);
    return ((j - i + 3) % 3 == 1) ? -vm : vm;
}

// Column r of A and of B (the maps formed by abs_maps), computed entry by entry
// into registers (no indexed private arrays): a[k] = A(k, r), b[k] = B(k, r).
__device__ __forceinline__ void abs_map_columns(const double *geo, int r, double a[6], double b[6]) {
    const double *R = geo, *th = geo + 12;
    const double Rt0 = R[0] * th[0] + R[1] * th[1] + R[2] * th[2];
    const double Rt1 = R[3] * th[0] + R[4] * th[1] + R[5] * th[2];
    const double Rt2 = R[6] * th[0] + R[7] * th[1] + R[8] * th[2];
    const bool rw = r < 3;           // rotation column
    const int rr = rw ? r : r - 3;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        // rows 0-2: A = [I 0], B = [-R 0]
        a[k] = (k == r) ? 1.0 : 0.0;
        b[k] = rw ? -R[3 * k + rr] : 0.0;
        // rows 3-5: A = [[R t_h]_x I], B = [-R [t_h]_x  -R]
        double rth = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q) rth += R[3 * k + q] * cross_entry(th[0], th[1], th[2], q, rr);
        a[3 + k] = rw ? cross_entry(Rt0, Rt1, Rt2, k, rr) : ((3 + k == r) ? 1.0 : 0.0);
        b[3 + k] = rw ? -rth : -R[3 * k + rr];
    }
}

// x^T H y for 6-vectors and H given by its upper triangle (row-major).
__device__ __forceinline__ double quad6(const double x[6], const double *H21, const double y[6]) {
    double s = 0.0;
    int e = 0;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        s += x[a] * H21[e] * y[a];
        ++e;
#pragma unroll
        for (int b = a + 1; b < 6; ++b, ++e) s += H21[e] * (x[a] * y[b] + x[b] * y[a]);
    }
    return s;
}

// The same maps applied to 6-vectors without forming them (geo = R_fh, t_fh, t_h):
//   A x   = (x_w, (R t_h) x x_w + x_t)            A^T y = (y_w - (R t_h) x y_t, y_t)
//   B x   = (-R x_w, -R (t_h x x_w + x_t))        B^T y = (-R^T y_w + t_h x (R^T y_t), -R^T y_t)
__device__ __forceinline__ void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ __forceinline__ void geo_Rth(const double *geo, double *Rt) {
    const double *R = geo, *th = geo + 12;
    for (int i = 0; i < 3; ++i) Rt[i] = R[3 * i] * th[0] + R[3 * i + 1] * th[1] + R[3 * i + 2] * th[2];
}
__device__ __forceinline__ void apply_A(const double *geo, const double *x, double *out) {
    double Rt[3], c[3];
    geo_Rth(geo, Rt);
    cross3(Rt, x, c);
    for (int i = 0; i < 3; ++i) {
        out[i] = x[i];
        out[3 + i] = c[i] + x[3 + i];
    }
}
__device__ __forceinline__ void apply_At(const double *geo, const double *y, double *out) {
    double Rt[3], c[3];
    geo_Rth(geo, Rt);
    cross3(Rt, y + 3, c);
    for (int i = 0; i < 3; ++i) {
        out[i] = y[i] - c[i];
        out[3 + i] = y[3 + i];
    }
}
__device__ __forceinline__ void apply_B(const double *geo, const double *x, double *out) {
    const double *R = geo, *th = geo + 12;
    double c[3];
    cross3(th, x, c);
    for (int i = 0; i < 3; ++i) c[i] += x[3 + i];
    for (int i = 0; i < 3; ++i) {
        out[i] = -(R[3 * i] * x[0] + R[3 * i + 1] * x[1] + R[3 * i + 2] * x[2]);
        out[3 + i] = -(R[3 * i] * c[0] + R[3 * i + 1] * c[1] + R[3 * i + 2] * c[2]);
    }
}
__device__ __forceinline__ void apply_Bt(const double *geo, const double *y, double *out) {
    const double *R = geo, *th = geo + 12;
    double a[3], b[3], c[3];
    for (int i = 0; i < 3; ++i) {
        a[i] = R[i] * y[0] + R[3 + i] * y[1] + R[6 + i] * y[2];          // R^T y_w
        b[i] = R[i] * y[3] + R[3 + i] * y[4] + R[6 + i] * y[5];          // R^T y_t
    }
    cross3(th, b, c);
    for (int i = 0; i < 3; ++i) {
        out[i] = -a[i] + c[i];
        out[3 + i] = -b[i];
    }
}

// Rodrigues' formula exp([w]_x) (row-major 3x3).
__device__ __forceinline__ void so3_exp(const double w[3], double R[9]) {
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double a, b;
    if (th2 < 1e-16) {
        a = 1.0 - th2 / 6.0;
        b = 0.5 - th2 / 24.0;
    } else {
        const double th = sqrt(th2);
        a = sin(th) / th;
        b = (1.0 - cos(th)) / th2;
    }
    const double K[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double kk = 0.0;
            for (int k = 0; k < 3; ++k) kk += K[i * 3 + k] * K[k * 3 + j];
            R[i * 3 + j] = (i == j ? 1.0 : 0.0) + a * K[i * 3 + j] + b * kk;
        }
}

__device__ __forceinline__ void mat3_mul(const double *A, const double *B, double *C) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[i * 3 + k] * B[k * 3 + j];
            C[i * 3 + j] = s;
        }
}

// C = A B^T
__device__ __forceinline__ void mat3_mul_bt(const double *A, const double *B, double *C) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[i * 3 + k] * B[j * 3 + k];
            C[i * 3 + j] = s;
        }
}

// An empty asm statement that takes v in a vector register and may change it:
// the value must exist at this point, so a load feeding it is not moved past it.
template <typename T>
__device__ __forceinline__ void pin_reg(T &v) {
    asm volatile("" : "+v"(v));
}

// Cross-lane exchanges by DPP inside rows of 16 lanes (a few cycles, where a
// shuffle takes an LDS round trip): lane i reads lane i ^ 1 or i ^ 2 (quad
// permutes) and i ^ 4 or i ^ 8 (a row shift left or right by 4 or 8, chosen by
// the lane's bit). The reductions below add in the order of an xor butterfly
// over 1, 2, 4, 8 (then 16, 32 through lane reads), so they match it to the
// bit. Every lane of the groups they reduce must be active.
enum { DPP_XOR1 = 0xb1, DPP_XOR2 = 0x4e, DPP_ROW_SHL = 0x100, DPP_ROW_SHR = 0x110 };

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Lane i ^ M for M = 4 or 8: lanes with bit M clear read M lanes up, the others
// M lanes down (both inside the row).
template <int M, typename T>
__device__ __forceinline__ T dpp_xor(T v) {
    static_assert(M == 4 || M == 8, "row shifts serve the exchanges over 4 and 8");
    const T up = dpp_mov<DPP_ROW_SHL + M>(v), down = dpp_mov<DPP_ROW_SHR + M>(v);
    return (threadIdx.x & M) ? down : up;
}

__device__ __forceinline__ float lane_value(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

__device__ __forceinline__ double lane_value(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over each group of 8 lanes; every lane gets its group's sum.
template <typename T>
__device__ __forceinline__ T wave_sum8(T v) {
    v += dpp_mov<DPP_XOR1>(v);
    v += dpp_mov<DPP_XOR2>(v);
    v += dpp_xor<4>(v);
    return v;
}

// Sum over each row of 16 lanes; every lane gets its row's sum.
template <typename T>
__device__ __forceinline__ T row_sum16(T v) {
    v = wave_sum8(v);
    return v + dpp_xor<8>(v);
}

// Maximum over each row of 16 lanes; every lane gets its row's maximum.
template <typename T>
__device__ __forceinline__ T row_max16(T v) {
    v = fmax(v, dpp_mov<DPP_XOR1>(v));
    v = fmax(v, dpp_mov<DPP_XOR2>(v));
    v = fmax(v, dpp_xor<4>(v));
    return fmax(v, dpp_xor<8>(v));
}

// Sum over the 64 lanes (lane 0's butterfly result: the row sums added as
// (r0 + r1) + (r2 + r3)); every lane gets it.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    v = row_sum16(v);
    return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// Maximum over the 64 lanes; every lane gets it.
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
    v = row_max16(v);
    return fmax(fmax(lane_value(v, 0), lane_value(v, 16)), fmax(lane_value(v, 32), lane_value(v, 48)));
}

// Sum over each half of 32 lanes (lanes 0 and 32's butterfly results); lanes
// 0-31 get the first half's, 32-63 the second half's.
template <typename T>
__device__ __forceinline__ T half_sum32(T v) {
    v = row_sum16(v);
    const T a = lane_value(v, 0) + lane_value(v, 16), b = lane_value(v, 32) + lane_value(v, 48);
    return (threadIdx.x & 32) ? b : a;
}

// Lane S of each aligned group of 8 lanes, read by every lane of the group:
// ds_swizzle in bit-mask mode (within each 32 lanes the source is
// (lane & 0x18) | S). An inactive source lane reads as 0, so the whole group
// must be active.
template <int S>
__device__ __forceinline__ float bcast8(float v) {
    static_assert(S >= 0 && S < 8, "a lane of the group of 8");
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x18 | (S << 5)));
}
template <int S>
__device__ __forceinline__ double bcast8(double v) {
    static_assert(S >= 0 && S < 8, "a lane of the group of 8");
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_swizzle((int)b, 0x18 | (S << 5));
    const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), 0x18 | (S << 5));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Words of 16-byte slices spread over a group of 8 lanes, read by every lane
// of the group: lane l of the group holds slice l in s0 and slice l + 8 in s1;
// out[k] = word k % 4 of slice k / 4 (ds_swizzle in bit-mask mode, as bcast8).
template <typename V, int... K>
__device__ __forceinline__ void bcast8_words(const V &s0, const V &s1, int *out, std::integer_sequence<int, K...>) {
    ((out[K] = __builtin_amdgcn_ds_swizzle(K < 32 ? s0[K % 4] : s1[K % 4], 0x18 | (((K / 4) % 8) << 5))), ...);
}

// Words B + k of the same layout, into out[B + k].
template <int B, typename V, int... K>
__device__ __forceinline__ void bcast8_words_range(const V &s0, const V &s1, int *out,
                                                   std::integer_sequence<int, K...>) {
    ((out[B + K] = __builtin_amdgcn_ds_swizzle((B + K) < 32 ? s0[(B + K) % 4] : s1[(B + K) % 4],
                                               0x18 | ((((B + K) / 4) % 8) << 5))),
     ...);
}

// Words B + k of the same slice layout, all from s1 (slices 8 and up): out[k]
// = word (B + k) % 4 of slice (B + k) / 4.
template <int B, typename V, int... K>
__device__ __forceinline__ void bcast8_words_from(const V &s1, int *out, std::integer_sequence<int, K...>) {
    static_assert(B >= 32, "words of the second slice register");
    ((out[K] = __builtin_amdgcn_ds_swizzle(s1[(B + K) % 4], 0x18 | ((((B + K) / 4) % 8) << 5))), ...);
}

}  // namespace pba
