// Depth back-substitution of a group of points and the maxima that the
// convergence test takes from it, shared by the depth-update kernel and the
// fused IC step.
#pragma once

#include "pba_device.hpp"
#include "pba_internal.hpp"

namespace pba {

constexpr int DU_SLOTS = 8;   // threads per point, over the point's observations
constexpr int DU_PTS = 256 / DU_SLOTS;   // points per block of the depth-update kernel

// LDS doubles that depth_points<T, NT> takes.
constexpr int depth_lds_doubles(int nt) { return (nt / DU_SLOTS) * (2 * DU_SLOTS + 2) + 2 * (nt / 64); }

// The data of point n0 + threadIdx.x / DU_SLOTS that its depth step reads first.
struct DepthPoint {
    int o0, o1;
    double hu, hv, Hn, d_old, d0;
};

// Loads that data (neutral values past N). EARLY: as relaxed atomic loads,
// which the compiler keeps where they are, so that a caller can issue them
// long before the depth step (the wait comes at their first use).
template <bool EARLY>
__device__ __forceinline__ DepthPoint depth_point(int N, int n0, const int *__restrict__ obs_ptr,
                                                  const float *__restrict__ host_uv, const double *__restrict__ Hdd,
                                                  const double *__restrict__ depth, const double *__restrict__ depth0) {
    const int n = n0 + (int)threadIdx.x / DU_SLOTS;
    auto ld = [](const auto *p) {
        if constexpr (EARLY)
            return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            return *p;
    };
    DepthPoint pt{0, 0, 0.0, 0.0, 1.0, 0.0, 1.0};
    if (n < N) {
        pt.o0 = ld(obs_ptr + n);
        pt.o1 = ld(obs_ptr + n + 1);
        pt.hu = (double)ld(host_uv + 2 * n);
        pt.hv = (double)ld(host_uv + 2 * n + 1);
        pt.Hn = ld(Hdd + n);
        pt.d_old = ld(depth + n);
        pt.d0 = ld(depth0 + n);
    }
    return pt;
}

// Depth step of the NT / DU_SLOTS points from n0 after the pose step (depth
// back-substitution, Sec. 3.5 step 4 for IC, the Schur back-substitution for
// FC): dd = -(g_d + h^T dtheta_rel) / H_dd per point; then the largest
// point-centre displacement (old pose and depth against new, level-0 camera)
// and depth step of the block, valid in thread 0. pt: the thread's point data
// (depth_point); with gate / flag given, the gate is read right after it and
// false comes back when it is closed (nothing written). dth_rel [pair][6] and
// geo_new [pair][GEO_STRIDE] may live in LDS. hc: h_o, 6 values per
// observation; gd: g_d per observation, stride gds. live: the observations
// still in the window (the displacement skips the others).
template <typename T, int NT>
__device__ __forceinline__ bool depth_points(
    int N, int n0, int ic, const DepthPoint &pt, const int *__restrict__ obs_pair,
    const double *__restrict__ pairK0, const double *__restrict__ hc, const double *__restrict__ gd, int gds,
    const double *dth_rel, const double *__restrict__ geo_old, const double *geo_new, double *__restrict__ depth,
    const int *gate, const int *flag, double *lds, double &mdisp_out, double &mstep_out,
    const uint8_t *__restrict__ live) {
    constexpr int NPTS = NT / DU_SLOTS, NW = NT / 64;
    static_assert(NW <= 16, "the block maxima are taken over one row of 16 lanes");
    double(*sp)[DU_SLOTS][2] = reinterpret_cast<double(*)[DU_SLOTS][2]>(lds);
    double *dnew = lds + NPTS * DU_SLOTS * 2, *dold = dnew + NPTS, *red = dold + NPTS;   // red [2][NW]
    const int q = threadIdx.x / DU_SLOTS, slot = threadIdx.x % DU_SLOTS;
    const int n = n0 + q;
    const bool has = n < N;
    const int o0 = pt.o0, o1 = pt.o1;
    const double hu = pt.hu, hv = pt.hv, Hn = pt.Hn, d_old = pt.d_old, d0 = pt.d0;
    if (gate) {
        const int gv = __hip_atomic_load(gate, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int fv = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__builtin_amdgcn_readfirstlane(gv) == 0 || __builtin_amdgcn_readfirstlane(fv) != 0) return false;
    }
    // g_d,n and h_n^T dtheta, slot-parallel over the point's observations
    double s = 0.0, g = 0.0;
    for (int o = o0 + slot; o < o1; o += DU_SLOTS) {
        const double2 *h2 = reinterpret_cast<const double2 *>(hc + 6 * (size_t)o);
        const double *dr = dth_rel + 6 * obs_pair[o];
        g += gd[(size_t)o * gds];
        for (int k = 0; k < 3; ++k) {
            const double2 hk = h2[k];
            s += hk.x * dr[2 * k];
            s += hk.y * dr[2 * k + 1];
        }
    }
    sp[q][slot][0] = g;
    sp[q][slot][1] = s;
    __syncthreads();
    double mstep = 0.0;
    if (slot == 0 && has) {
        double t = 0.0;
        for (int k = 0; k < DU_SLOTS; ++k) t += sp[q][k][0];
        for (int k = 0; k < DU_SLOTS; ++k) t += sp[q][k][1];
        const double dd = -t / Hn;
        const double d_new = ic ? d_old * (d0 - dd) / d0 : d_old + dd;
        depth[n] = d_new;
        dold[q] = d_old;
        dnew[q] = d_new;
        mstep = fabs(dd);
    }
    __syncthreads();
    double mdisp = 0.0;
    for (int o = o0 + slot; o < o1; o += DU_SLOTS) {
        const int p = obs_pair[o];
        const double *Kp = pairK0 + 8 * p;   // host (fx, fy, cx, cy), target (fx, fy, cx, cy)
        const double x = (hu - Kp[2]) / Kp[0], y = (hv - Kp[3]) / Kp[1];
        double qq[2][2];
        bool ok = true;
        for (int s2 = 0; s2 < 2; ++s2) {
            const double *gm = s2 ? geo_new + GEO_STRIDE * p : geo_old + GEO_STRIDE * p;
            const double d = s2 ? dnew[q] : dold[q];
            const double vx = gm[0] * x + gm[1] * y + gm[2] + d * gm[9];
            const double vy = gm[3] * x + gm[4] * y + gm[5] + d * gm[10];
            const double vz = gm[6] * x + gm[7] * y + gm[8] + d * gm[11];
            ok = ok && vz > 0.0;
            const double vzs = vz > 0.0 ? vz : 1.0;
            qq[s2][0] = Kp[4] * vx / vzs + Kp[6];
            qq[s2][1] = Kp[5] * vy / vzs + Kp[7];
        }
        if (ok && live[o]) mdisp = fmax(mdisp, hypot(qq[1][0] - qq[0][0], qq[1][1] - qq[0][1]));
    }
    mdisp = wave_max(mdisp);
    mstep = wave_max(mstep);
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = mdisp;
        red[NW + (threadIdx.x >> 6)] = mstep;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        // the (non-negative) wavefront maxima over the lanes of row 0
        const int l = threadIdx.x;
        mdisp_out = row_max16(l < NW ? red[l] : 0.0);
        mstep_out = row_max16(l < NW ? red[NW + l] : 0.0);
    }
    return true;
}

}  // namespace pba
