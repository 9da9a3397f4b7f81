// Device state of one split Bregman solve (all n x n FP64 images, row-major).
#pragma once
#include <hip/hip_runtime.h>

namespace kpsb {

struct SBDev {
  int n;
  double lam;        // lambda (lambda_x = lambda_y)
  double thr;        // shrink threshold 1/gamma, gamma = lambda^2 / beta
  int iso;           // 1: isotropic shrink, 0: anisotropic
  double tau_cgls, tau_sb;
  const double* b;
  const double* AtB; // A_k^T b (constant over the solve)
  double *x, *xprev, *r1, *r2, *r3, *w, *f, *z1, *t1;
  double *dx, *dy, *gx, *gy;
  double* part;      // kRedBlocks x 4 partial sums
  double* scal;      // [0] tau  [2] RC_SB  [3] RC_CGLS  [5] tau of the current iteration
  int* flags;        // [0] SB done  [1] CGLS done  [2] iota_total  [3] l_end
};

// Kronecker apply tiling: output tile (64 or 32), terms accumulated per
// workgroup of the second GEMM, and the resulting number of partial images.
struct KpApplyPlan {
  int tile = 64;
  int group = 1;
  int ngroups = 1;
};
KpApplyPlan kp_apply_plan(int n, int k);

void sb_launch_rhs(const SBDev& d, hipStream_t s);
// f from T = sum of the ng partial images at T (stride n^2)
void sb_launch_f(const SBDev& d, const double* T, int ng, int levels, hipStream_t s);
void sb_launch_w_init(const SBDev& d, hipStream_t s);
// z1 = sum of the ng partial images at P, and ||z||^2 partials
void sb_launch_zn(const SBDev& d, const double* P, int ng, hipStream_t s);
void sb_launch_xr(const SBDev& d, hipStream_t s);
// w update and the CGLS stopping test
void sb_launch_w(const SBDev& d, hipStream_t s);
void sb_launch_shrink(const SBDev& d, hipStream_t s);
void sb_launch_check(const SBDev& d, hipStream_t s);

// A_k X (or A_k^T X) as plan.ngroups partial images in P; Z (k x n x n) is
// workspace. Skipped when any of flags[0..nflags) is nonzero.
void launch_kp_apply_parts(const double* Ax, const double* Ay, int n, int k, int transpose,
                           const double* X, double* Z, double* P, const KpApplyPlan& plan,
                           const int* flags, int nflags, hipStream_t s);
// Y = sum of the ng partial images at P (stride NN), fixed order
void launch_sum_parts(const double* P, int ng, long NN, double* Y, hipStream_t s);
// kp_apply with caller workspace Z, P (k x n x n each); skipped when any of
// flags[0..nflags) is nonzero.
void launch_kp_apply_ws(const double* Ax, const double* Ay, int n, int k, int transpose,
                        const double* X, double* Y, double* Z, double* P, const int* flags,
                        int nflags, hipStream_t s);

}  // namespace kpsb
