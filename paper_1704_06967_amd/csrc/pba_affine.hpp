// Per-frame affine brightness in the forward-compositional iteration: the
// brightness record, the device buffers of the joint system and the launchers
// (pba_affine.hip; the dense solve in pba_dense.hip).
#pragma once

#include "pba_internal.hpp"

namespace pba {

// brightness record per observation (FP64)
enum AffField : int {
    AFF_C = 0,      // 24: sum w J_th (6, relative) x J_phi (4), row-major [6][4]
    AFF_P = 24,     // 10: upper triangle of sum w J_phi^T J_phi, J_phi over (a_h, b_h, a_f, b_f)
    AFF_h = 34,     // 4: sum w J_phi J_d
    AFF_G = 38,     // 4: sum w J_phi r
    AFF_STRIDE = 42
};

// Buffers of the joint iteration (one window of F frames, O observations).
struct AffBufs {
    bool on = false;
    int F = 0, O = 0;                   // sizes the buffers hold
    double *ab = nullptr;               // [F][2] (a_f, b_f)
    double *arec = nullptr;             // [O][AFF_STRIDE]
    double *M = nullptr, *fac = nullptr;// [8F][8F] reduced system, its factor
    double *Linv = nullptr;             // inverses of the factor's diagonal tiles [ceil(8F / 32)][32][32]
    double *b = nullptr, *x = nullptr;  // [8F] right-hand side, increment (poses, then brightness)
    double *dphi = nullptr;             // [2F] brightness diagonal before damping
    double *poses_old = nullptr;        // [F][12]
    double *stats = nullptr;            // sum_stats_doubles(c): E, SQ, CNT and block partials
    unsigned long long *maxb = nullptr; // [4] displacement, depth step (bits of non-negative doubles)
    int *flag = nullptr;                // [2] solve flag (0 solved, 1 not positive definite, 2 skipped), its gate
};

// mode 0: linearize over the frozen set; 1: decide the frozen set (written to
// the context's mask) at these parameters, then linearize; 2: energy, sum r^2
// and count only, over the residuals usable at these parameters
void launch_aff_linearize(hipStream_t s, Ctx &c, const AffBufs &a, int level, const double *geo, int mode);
// the 8F x 8F reduced system and its right-hand side from the FC assembly's
// pose block (c.d_S), the records and the damped H_dd
void launch_aff_system(hipStream_t s, Ctx &c, const AffBufs &a, const double *geo);
// pose, brightness and depth updates from a.x and the convergence maxima
void launch_aff_update(hipStream_t s, Ctx &c, const AffBufs &a, const double *geo_old);
// x = -M^{-1} b by the tiled Cholesky factorization while `gate` is open
// (flag[0] = 0 on entry, 1 when M is not positive definite; x is then not
// written); with the gate closed nothing is solved and flag[0] = 2
void launch_dense_solve(hipStream_t s, int n, const double *M, double *fac, double *Linv, const double *b, double *x,
                        int *flag, const int *gate);
// end of a joint iteration: statistics slot `stat`, the level's count, gate
// (see k_aff_stat)
void launch_aff_stat(hipStream_t s, Ctx &c, const AffBufs &a, int level, double *stat, double conv_px);

}  // namespace pba
