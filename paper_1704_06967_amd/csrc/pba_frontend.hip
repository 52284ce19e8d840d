// Front end for the starting parameters p(0): the first three steps of the
// base solution of Sec. 4.1 (Harris corners, robust KLT tracking, geometric
// bundle adjustment with outlier removal); the fourth, the FC photometric
// bundle adjustment, is the library's FC solve.
//
// Readings (the paper names the methods only):
//  * corners: the image quantized to 8 bits, central differences times two,
//    a 5 x 5 box structure tensor and kappa = 1/16 scaled by 16, so the
//    response R = 16 det - tr^2 is an exact 64-bit integer and the corner set
//    does not depend on rounding; 3 x 3 maxima (ties to the first pixel in
//    raster order), one per cell, the strongest cells first;
//  * tracking: translational Lucas-Kanade in inverse-compositional form (the
//    window's gradient and H once per level), coarse to fine from a predicted
//    position, a fixed number of iterations per level, then tracked back into
//    the host: kept if it returns within fb_px;
//  * geometric BA: the 2-D reprojection error of each observation with a
//    Huber weight on its norm, written as the FC records of the photometric
//    path (so the pair sums, depth Schur complement, Cholesky, update and
//    convergence test are the FC iteration's), one outlier removal.
#include <hip/hip_ext.h>

#include <climits>

#include "pba_device.hpp"
#include "pba_internal.hpp"

namespace pba {

// ------------------------------------------------------------ corners

constexpr int HR_TW = 32, HR_TH = 8;   // output tile of the response kernel (256 threads)

// rint(v * 255) in single precision (half to even), clamped to [0, 255].
__device__ __forceinline__ int quant8(float v) {
    const float q = rintf(v * 255.0f);
    return (int)fminf(fmaxf(q, 0.0f), 255.0f);
}

// Harris response of one frame: each workgroup stages its tile's 8-bit values
// (3-pixel halo) and gradient products (2-pixel halo) in LDS, then sums the
// 5 x 5 window per pixel. Pixels outside rows / columns 3 .. size - 4 get 0.
template <typename T>
__global__ __launch_bounds__(256) void k_harris(const T *__restrict__ img, int W, int H, long long *__restrict__ R) {
    __shared__ int q[HR_TH + 6][HR_TW + 6];
    __shared__ int pxx[HR_TH + 4][HR_TW + 4], pyy[HR_TH + 4][HR_TW + 4], pxy[HR_TH + 4][HR_TW + 4];
    const int x0 = blockIdx.x * HR_TW, y0 = blockIdx.y * HR_TH;
    for (int k = threadIdx.x; k < (HR_TH + 6) * (HR_TW + 6); k += blockDim.x) {
        const int ly = k / (HR_TW + 6), lx = k % (HR_TW + 6);
        const int y = y0 - 3 + ly, x = x0 - 3 + lx;
        q[ly][lx] = (y >= 0 && y < H && x >= 0 && x < W) ? quant8((float)img[(size_t)y * W + x]) : 0;
    }
    __syncthreads();
    // product (y0 - 2 + ly, x0 - 2 + lx) from the values around q[ly + 1][lx + 1]
    for (int k = threadIdx.x; k < (HR_TH + 4) * (HR_TW + 4); k += blockDim.x) {
        const int ly = k / (HR_TW + 4), lx = k % (HR_TW + 4);
        const int gx = q[ly + 1][lx + 2] - q[ly + 1][lx];
        const int gy = q[ly + 2][lx + 1] - q[ly][lx + 1];
        pxx[ly][lx] = gx * gx;
        pyy[ly][lx] = gy * gy;
        pxy[ly][lx] = gx * gy;
    }
    __syncthreads();
    const int ly = threadIdx.x / HR_TW, lx = threadIdx.x % HR_TW;
    const int y = y0 + ly, x = x0 + lx;
    if (y >= H || x >= W) return;
    long long r = 0;
    if (y >= 3 && y <= H - 4 && x >= 3 && x <= W - 4) {
        int sxx = 0, syy = 0, sxy = 0;
#pragma unroll
        for (int dy = 0; dy < 5; ++dy)
#pragma unroll
            for (int dx = 0; dx < 5; ++dx) {
                sxx += pxx[ly + dy][lx + dx];
                syy += pyy[ly + dy][lx + dx];
                sxy += pxy[ly + dy][lx + dx];
            }
        const long long tr = (long long)sxx + syy;
        r = 16LL * ((long long)sxx * syy - (long long)sxy * sxy) - tr * tr;
    }
    R[(size_t)y * W + x] = r;
}

// Whether candidate (ra, ia) ranks before (rb, ib): a larger response, then
// the smaller raster index; index -1 (no candidate) ranks last.
__device__ __forceinline__ bool ranks_before(long long ra, int ia, long long rb, int ib) {
    if (ia < 0) return false;
    if (ib < 0) return true;
    return ra > rb || (ra == rb && ia < ib);
}

// The best candidate of each cell (one workgroup per cell of at most 16 x 16
// pixels, one pixel per thread): inside the margin, R > min_resp and a 3 x 3
// maximum with ties to the first pixel in raster order.
__global__ __launch_bounds__(256) void k_cell_best(const long long *__restrict__ R, int W, int H, int cell,
                                                   int margin, long long min_resp, int ncx,
                                                   long long *__restrict__ cell_R, int *__restrict__ cell_idx) {
    __shared__ long long sr[256];
    __shared__ int si[256];
    const int c = blockIdx.x, cy = c / ncx, cx = c % ncx, t = threadIdx.x;
    long long best = LLONG_MIN;
    int bi = -1;
    if (t < cell * cell) {
        const int y = cy * cell + t / cell, x = cx * cell + t % cell;
        if (y >= margin && y <= H - 1 - margin && x >= margin && x <= W - 1 - margin) {
            const long long r = R[(size_t)y * W + x];
            bool ok = r > min_resp;
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    if (dy == 0 && dx == 0) continue;
                    const long long nb = R[(size_t)(y + dy) * W + x + dx];
                    const bool before = dy < 0 || (dy == 0 && dx < 0);
                    ok = ok && (before ? r > nb : r >= nb);
                }
            if (ok) {
                best = r;
                bi = y * W + x;
            }
        }
    }
    sr[t] = best;
    si[t] = bi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s && ranks_before(sr[t + s], si[t + s], sr[t], si[t])) {
            sr[t] = sr[t + s];
            si[t] = si[t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        cell_R[c] = sr[0];
        cell_idx[c] = si[0];
    }
}

// The K best cell winners, best first. A candidate's rank is the number of
// candidates that rank before it: every pair is compared once, the grid
// covering (candidate tile, comparison tile), each block staging its
// comparison tile in LDS and adding its counts to the ranks (integer atomics,
// so the sums do not depend on their order). The ranks of the candidates are
// a permutation, so the candidate of rank r < K alone writes output r, and
// count = min(K, candidates) by an atomic maximum (rank and count start at 0).
constexpr int RANK_TILE = 256;

__global__ __launch_bounds__(RANK_TILE) void k_corner_rank(const long long *__restrict__ cell_R,
                                                           const int *__restrict__ cell_idx, int n,
                                                           int *__restrict__ rank) {
    __shared__ long long tr[RANK_TILE];
    __shared__ int ti[RANK_TILE];
    const int i = blockIdx.x * RANK_TILE + threadIdx.x;
    const int j = blockIdx.y * RANK_TILE + threadIdx.x;
    tr[threadIdx.x] = j < n ? cell_R[j] : LLONG_MIN;
    ti[threadIdx.x] = j < n ? cell_idx[j] : -1;
    __syncthreads();
    if (i >= n) return;
    const long long ri = cell_R[i];
    const int ii = cell_idx[i];
    if (ii < 0) return;
    const int m = min(RANK_TILE, n - (int)blockIdx.y * RANK_TILE);
    int cnt = 0;
    for (int k = 0; k < m; ++k) cnt += ranks_before(tr[k], ti[k], ri, ii) ? 1 : 0;
    if (cnt) atomicAdd(rank + i, cnt);
}

__global__ __launch_bounds__(256) void k_corner_emit(const long long *__restrict__ cell_R,
                                                     const int *__restrict__ cell_idx, const int *__restrict__ rank,
                                                     int n, int W, int K, int *__restrict__ uv,
                                                     long long *__restrict__ resp, int *__restrict__ count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int ii = cell_idx[i], r = rank[i];
    if (ii >= 0 && r < K) {
        uv[2 * r] = ii % W;
        uv[2 * r + 1] = ii / W;
        resp[r] = cell_R[i];
        atomicMax(count, r + 1);
    }
}

// ------------------------------------------------------------ tracking

// The image pyramid of the context, level 0 first.
struct PyrArg {
    const void *img[PBA_MAX_LEVELS];
    int W[PBA_MAX_LEVELS], H[PBA_MAX_LEVELS];
    int L;
};

enum TrackStatus : int { TRK_OK = 0, TRK_LOW_TEXTURE = 1, TRK_LEFT_IMAGE = 2, TRK_FB = 3 };

constexpr int KLT_MAX_RADIUS = 5;   // window of at most 11 x 11 = 121 pixels: 2 per lane

// One-way LK of the window around level-0 position (xu, xv) in frame src into
// frame dst from the level-0 guess (gu0, gv0), run by one wavefront (slots
// lane and lane + 64 of the window, rows outer). FP64 arithmetic; the sums
// are the wavefront's (every lane holds them). Returns the status; (ou, ov)
// is the level-0 position found.
template <typename T>
__device__ int lk_one_way(const PyrArg &py, int src, double xu, double xv, int dst, double gu0, double gv0,
                          int radius, int n_iters, double min_eig, double &ou, double &ov) {
    const int lane = threadIdx.x & 63, w = 2 * radius + 1, npx = w * w;
    const int L = py.L;
    double du = (gu0 - xu) / (double)(1 << (L - 1)), dv = (gv0 - xv) / (double)(1 << (L - 1));
    int status = TRK_OK;
    for (int l = L - 1; l >= 0 && status == TRK_OK; --l) {
        if (l < L - 1) {
            du *= 2.0;
            dv *= 2.0;
        }
        const int W = py.W[l], H = py.H[l];
        const T *ims = (const T *)py.img[l] + (size_t)src * W * H;
        const T *imd = (const T *)py.img[l] + (size_t)dst * W * H;
        const double sc = ldexp(1.0, -l);
        const double xl = (xu + 0.5) * sc - 0.5, yl = (xv + 0.5) * sc - 0.5;
        double t0[2] = {0.0, 0.0}, gx[2] = {0.0, 0.0}, gy[2] = {0.0, 0.0}, ofu[2] = {0.0, 0.0},
               ofv[2] = {0.0, 0.0};
        bool has[2], in = true;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int s = lane + 64 * k;
            has[k] = s < npx;
            if (has[k]) {
                ofu[k] = (double)(s % w - radius);
                ofv[k] = (double)(s / w - radius);
                const double pu = xl + ofu[k], pv = yl + ofv[k];
                if (usable(pu, pv, W, H))
                    bilinear_grad(ims, W, pu, pv, t0[k], gx[k], gy[k]);
                else
                    in = false;
            }
        }
        if (!__all(in)) {
            status = TRK_LEFT_IMAGE;
            break;
        }
        const double a = wave_sum(gx[0] * gx[0] + gx[1] * gx[1]);
        const double b = wave_sum(gx[0] * gy[0] + gx[1] * gy[1]);
        const double c = wave_sum(gy[0] * gy[0] + gy[1] * gy[1]);
        const double lam = 0.5 * (a + c) - sqrt(0.25 * (a - c) * (a - c) + b * b);
        if (lam / (double)npx < min_eig) {
            status = TRK_LOW_TEXTURE;
            break;
        }
        const double det = a * c - b * b;
        for (int it = 0; it < n_iters; ++it) {
            double e[2] = {0.0, 0.0};
            bool ok = true;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                if (!has[k]) continue;
                const double pu = xl + du + ofu[k], pv = yl + dv + ofv[k];
                if (usable(pu, pv, W, H))
                    e[k] = bilinear(imd, W, pu, pv) - t0[k];
                else
                    ok = false;
            }
            if (!__all(ok)) {
                status = TRK_LEFT_IMAGE;
                break;
            }
            const double bx = wave_sum(gx[0] * e[0] + gx[1] * e[1]);
            const double by = wave_sum(gy[0] * e[0] + gy[1] * e[1]);
            du -= (c * bx - b * by) / det;
            dv -= (a * by - b * bx) / det;
        }
    }
    ou = xu + du;
    ov = xv + dv;
    return status;
}

// One wavefront per track: forward into the target, then back into the host.
template <typename T>
__global__ __launch_bounds__(256) void k_klt(PyrArg py, int n, const int *__restrict__ host,
                                             const double *__restrict__ host_uv, const int *__restrict__ target,
                                             const double *__restrict__ guess, int radius, int n_iters,
                                             double min_eig, double fb_px, double *__restrict__ out_uv,
                                             int *__restrict__ out_status, double *__restrict__ out_fb) {
    const int tr = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (tr >= n) return;   // the whole wavefront leaves together
    const int h = host[tr], f = target[tr];
    const double xu = host_uv[2 * tr], xv = host_uv[2 * tr + 1];
    double fu, fv, bu, bv;
    int st = lk_one_way<T>(py, h, xu, xv, f, guess[2 * tr], guess[2 * tr + 1], radius, n_iters, min_eig, fu, fv);
    double fb = 0.0;
    if (st == TRK_OK) {
        st = lk_one_way<T>(py, f, fu, fv, h, xu, xv, radius, n_iters, min_eig, bu, bv);
        fb = hypot(bu - xu, bv - xv);
        if (st == TRK_OK && !(fb <= fb_px)) st = TRK_FB;
    }
    if ((threadIdx.x & 63) == 0) {
        out_uv[2 * tr] = fu;
        out_uv[2 * tr + 1] = fv;
        out_status[tr] = st;
        out_fb[tr] = fb;
    }
}

// ------------------------------------------------------------ geometric BA

// Reprojection of observation o's point centre with the pair geometry geo
// (R_fh, t_fh) and level-0 intrinsics Kp (host then target): the normalized
// host coordinates, R x~, v and the level-0 pixel; false behind the camera.
struct GeoProj {
    double x, y, a[3], v[3], qx, qy;
};
__device__ __forceinline__ bool geo_project(const double *g, const double *Kp, double hu, double hv, double d,
                                            GeoProj &p) {
    p.x = (hu - Kp[2]) / Kp[0];
    p.y = (hv - Kp[3]) / Kp[1];
    for (int r = 0; r < 3; ++r) {
        p.a[r] = g[3 * r] * p.x + g[3 * r + 1] * p.y + g[3 * r + 2];
        p.v[r] = p.a[r] + d * g[9 + r];
    }
    if (!(p.v[2] > 0.0)) return false;
    p.qx = Kp[4] * p.v[0] / p.v[2] + Kp[6];
    p.qy = Kp[5] * p.v[1] / p.v[2] + Kp[7];
    return true;
}

// The FC record of every observation for the reprojection error e = q - z:
// J = diag(fx, fy) (1/v_z) [[1, 0, -u_x], [0, 1, -u_y]] [-[R x~]_x | d I | t],
// the Huber weight of |e| (threshold k) on both rows; zero for an observation
// removed as an outlier, out of the window or behind the camera.
__global__ __launch_bounds__(256) void k_geo_linearize(int O, const int *__restrict__ obs_point,
                                                       const int *__restrict__ obs_pair,
                                                       const float *__restrict__ host_uv,
                                                       const double *__restrict__ depth,
                                                       const double *__restrict__ geo,
                                                       const double *__restrict__ pairK0,
                                                       const double *__restrict__ z,
                                                       const uint8_t *__restrict__ inlier,
                                                       const uint8_t *__restrict__ live, double k,
                                                       double *__restrict__ rec, const int *__restrict__ gate) {
    if (*gate == 0) return;
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= O) return;
    const int n = obs_point[o], pr = obs_pair[o];
    const double *g = geo + GEO_STRIDE * pr, *Kp = pairK0 + 8 * pr;
    const double d = depth[n];
    double out[REC_STRIDE];
    for (int i = 0; i < REC_STRIDE; ++i) out[i] = 0.0;
    GeoProj p;
    if (inlier[o] && live[o] && geo_project(g, Kp, (double)host_uv[2 * n], (double)host_uv[2 * n + 1], d, p)) {
        const double iz = 1.0 / p.v[2], ux = p.v[0] * iz, uy = p.v[1] * iz;
        const double ex = p.qx - z[2 * o], ey = p.qy - z[2 * o + 1];
        // dv/dp rows (w, t, d)
        const double dvx[7] = {0.0, p.a[2], -p.a[1], d, 0.0, 0.0, g[9]};
        const double dvy[7] = {-p.a[2], 0.0, p.a[0], 0.0, d, 0.0, g[10]};
        const double dvz[7] = {p.a[1], -p.a[0], 0.0, 0.0, 0.0, d, g[11]};
        double Jx[7], Jy[7];
        for (int c = 0; c < 7; ++c) {
            Jx[c] = Kp[4] * iz * (dvx[c] - ux * dvz[c]);
            Jy[c] = Kp[5] * iz * (dvy[c] - uy * dvz[c]);
        }
        const double nrm = hypot(ex, ey);
        const double w = nrm <= k ? 1.0 : k / nrm;
        int t = 0;
        for (int i = 0; i < 6; ++i)
            for (int j = i; j < 6; ++j) out[REC_H + t++] = w * (Jx[i] * Jx[j] + Jy[i] * Jy[j]);
        for (int i = 0; i < 6; ++i) {
            out[REC_h + i] = w * (Jx[i] * Jx[6] + Jy[i] * Jy[6]);
            out[REC_G + i] = w * (Jx[i] * ex + Jy[i] * ey);
        }
        out[REC_HDD] = w * (Jx[6] * Jx[6] + Jy[6] * Jy[6]);
        out[REC_GD] = w * (Jx[6] * ex + Jy[6] * ey);
        out[REC_E] = nrm <= k ? 0.5 * nrm * nrm : k * nrm - 0.5 * k * k;
        out[REC_SQ] = nrm * nrm;
        out[REC_CNT] = 1.0;
    }
    double2 *dst = reinterpret_cast<double2 *>(rec + (size_t)o * REC_STRIDE);
    for (int i = 0; i < REC_STRIDE / 2; ++i) dst[i] = make_double2(out[2 * i], out[2 * i + 1]);
}

// Outlier removal: an observation stays an inlier while its point lies in
// front of the target camera and |e| <= limit.
__global__ __launch_bounds__(256) void k_geo_outliers(int O, const int *__restrict__ obs_point,
                                                      const int *__restrict__ obs_pair,
                                                      const float *__restrict__ host_uv,
                                                      const double *__restrict__ depth,
                                                      const double *__restrict__ geo,
                                                      const double *__restrict__ pairK0,
                                                      const double *__restrict__ z, double limit,
                                                      uint8_t *__restrict__ inlier) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= O) return;
    const int n = obs_point[o], pr = obs_pair[o];
    GeoProj p;
    const bool front = geo_project(geo + GEO_STRIDE * pr, pairK0 + 8 * pr, (double)host_uv[2 * n],
                                   (double)host_uv[2 * n + 1], depth[n], p);
    const bool keep = front && hypot(p.qx - z[2 * o], p.qy - z[2 * o + 1]) <= limit;
    if (!keep) inlier[o] = 0;
}

// ------------------------------------------------------------ launchers

static inline unsigned nblocks(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }
static inline bool is_fp64(const Ctx &c) { return c.cfg.precision == PBA_FP64; }

void launch_fe_corners(hipStream_t s, Ctx &c, int frame, int cell, int margin, long long min_resp, int K,
                       long long *R, long long *cell_R, int *cell_idx, int *rank, int *uv, long long *resp,
                       int *count) {
    const int W = c.lv[0].W, H = c.lv[0].H;
    const dim3 grid(nblocks(W, HR_TW), nblocks(H, HR_TH));
    if (is_fp64(c))
        k_harris<double><<<grid, 256, 0, s>>>((const double *)c.lv[0].img + (size_t)frame * W * H, W, H, R);
    else
        k_harris<float><<<grid, 256, 0, s>>>((const float *)c.lv[0].img + (size_t)frame * W * H, W, H, R);
    const int ncx = (W + cell - 1) / cell, ncy = (H + cell - 1) / cell, n = ncx * ncy;
    // a candidate's 3 x 3 neighbours lie in the response's defined region
    k_cell_best<<<n, 256, 0, s>>>(R, W, H, cell, margin < 4 ? 4 : margin, min_resp, ncx, cell_R, cell_idx);
    (void)hipMemsetAsync(count, 0, sizeof(int), s);
    (void)hipMemsetAsync(rank, 0, (size_t)n * sizeof(int), s);
    const unsigned nt = nblocks(n, RANK_TILE);
    k_corner_rank<<<dim3(nt, nt), RANK_TILE, 0, s>>>(cell_R, cell_idx, n, rank);
    k_corner_emit<<<nblocks(n, 256), 256, 0, s>>>(cell_R, cell_idx, rank, n, W, K, uv, resp, count);
}

void launch_fe_track(hipStream_t s, Ctx &c, int n, const int *host, const double *host_uv, const int *target,
                     const double *guess, int radius, int n_iters, double min_eig, double fb_px, int levels,
                     double *out_uv, int *out_status, double *out_fb) {
    if (n == 0) return;
    PyrArg py{};
    py.L = levels;
    for (int l = 0; l < levels; ++l) {
        py.img[l] = c.lv[l].img;
        py.W[l] = c.lv[l].W;
        py.H[l] = c.lv[l].H;
    }
    const unsigned g = nblocks(n, 4);
    if (is_fp64(c))
        k_klt<double><<<g, 256, 0, s>>>(py, n, host, host_uv, target, guess, radius, n_iters, min_eig, fb_px, out_uv,
                                        out_status, out_fb);
    else
        k_klt<float><<<g, 256, 0, s>>>(py, n, host, host_uv, target, guess, radius, n_iters, min_eig, fb_px, out_uv,
                                       out_status, out_fb);
}

void launch_geo_linearize(hipStream_t s, Ctx &c, const double *geo_cur, hipEvent_t e0, hipEvent_t e1) {
    if (c.O == 0) return;
    const unsigned g = nblocks(c.O, 256);
    if (e0 || e1)
        hipExtLaunchKernelGGL(k_geo_linearize, dim3(g), dim3(256), 0, s, e0, e1, 0, c.O, c.d_obs_point,
                              c.d_obs_pair, c.d_host_uv, c.d_depth, geo_cur, c.d_pairK0, c.d_obs_z, c.d_geo_in,
                              c.d_obs_live, c.geo_huber, (double *)c.d_rec, c.d_gate);
    else
        k_geo_linearize<<<g, 256, 0, s>>>(c.O, c.d_obs_point, c.d_obs_pair, c.d_host_uv, c.d_depth, geo_cur,
                                          c.d_pairK0, c.d_obs_z, c.d_geo_in, c.d_obs_live, c.geo_huber,
                                          (double *)c.d_rec, c.d_gate);
}

void launch_geo_outliers(hipStream_t s, Ctx &c, const double *geo_cur, double limit) {
    if (c.O == 0) return;
    k_geo_outliers<<<nblocks(c.O, 256), 256, 0, s>>>(c.O, c.d_obs_point, c.d_obs_pair, c.d_host_uv, c.d_depth,
                                                     geo_cur, c.d_pairK0, c.d_obs_z, limit, c.d_geo_in);
}

}  // namespace pba
