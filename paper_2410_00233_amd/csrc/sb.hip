// Split Bregman TV deblurring (paper, Algorithms 3 and 4) with the CGLS inner
// solve of Algorithm 5 on the augmented system A-hat = [A_k; lam (L_x (x) I);
// lam (I (x) L_y)] (eq. "agu A"), all in FP64.
//
// Images are n x n row-major (row vertical). With x = vec(X) column-major:
//   (L_x (x) I) x = vec(X L^T)  -> (X L^T)[r][c] = (X[r][c] - X[r][c+1]) / 2
//   (I (x) L_y) x = vec(L X)    -> (L X)[r][c]   = (X[r][c] - X[r+1][c]) / 2
// with L = bidiag(1, -1)/2 square, last row (0 .. 0 1)/2 (eq. "deriv"; the
// square reading P = N), and the adjoints (Y L)[r][c] = (Y[r][c] - Y[r][c-1])/2,
// (L^T Y)[r][c] = (Y[r][c] - Y[r-1][c])/2.
//
// Every kernel is one pass over the image; reductions write kRedBlocks FP64
// partials that the next kernel adds in a fixed order. Data-dependent stopping
// (RC_CGLS < tau_cgls, RC_SB < tau_sb) sets device flags that turn the rest of
// the queued kernels into no-ops, so the host never waits on a scalar.
#include "common.h"
#include "sb.h"
#include "partials.h"

namespace kpsb {

__device__ __forceinline__ double dLx(const double* X, int n, int r, int c) {
  double v = 0.5 * X[(long)r * n + c];
  if (c + 1 < n) v -= 0.5 * X[(long)r * n + c + 1];
  return v;
}
__device__ __forceinline__ double dLy(const double* X, int n, int r, int c) {
  double v = 0.5 * X[(long)r * n + c];
  if (r + 1 < n) v -= 0.5 * X[(long)(r + 1) * n + c];
  return v;
}
__device__ __forceinline__ double dLxT(const double* Y, int n, int r, int c) {
  double v = 0.5 * Y[(long)r * n + c];
  if (c >= 1) v -= 0.5 * Y[(long)r * n + c - 1];
  return v;
}
__device__ __forceinline__ double dLyT(const double* Y, int n, int r, int c) {
  double v = 0.5 * Y[(long)r * n + c];
  if (r >= 1) v -= 0.5 * Y[(long)(r - 1) * n + c];
  return v;
}

__device__ __forceinline__ double sb_wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// sum over the 256 threads; result broadcast to the block
__device__ __forceinline__ double sb_block_sum(double v, double* sh) {
  v = sb_wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  const double r = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return r;
}

// sum of partial slot q (stride 4) over the kRedBlocks partials
__device__ __forceinline__ double sb_partials(const double* part, int q, double* sh) {
  return sb_block_sum(part[threadIdx.x * 4 + q], sh);
}

__device__ __forceinline__ bool sb_skip(const SBDev& d, int levels) {
  for (int i = 0; i < levels; ++i)
    if (d.flags[i]) return true;
  return false;
}

#define SB_ROWS                                                   \
  const long NN = (long)d.n * d.n;                                \
  const long chunk = (NN + gridDim.x - 1) / gridDim.x;            \
  const long lo = (long)blockIdx.x * chunk;                       \
  const long hi = lo + chunk < NN ? lo + chunk : NN;

// r1 = b, r2 = lam (dx - gx), r3 = lam (dy - gy), x = 0 (CGLS restarts at 0)
__global__ void __launch_bounds__(256) sb_rhs_kernel(SBDev d) {
  if (sb_skip(d, 1)) return;
  SB_ROWS
  for (long e = lo + threadIdx.x; e < hi; e += 256) {
    d.r1[e] = d.b[e];
    d.r2[e] = d.lam * (d.dx[e] - d.gx[e]);
    d.r3[e] = d.lam * (d.dy[e] - d.gy[e]);
    d.x[e] = 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) d.flags[1] = 0;
}

// sum of the ng partial images at P (stride NN), fixed order
__device__ __forceinline__ double sb_sum_parts(const double* __restrict__ P, int ng, long NN,
                                               long e) {
  return add_partials_in_order(P[e], P + e, 1, ng, NN);
}

// f = T + lam (L_x^T r2 + L_y^T r3) with T the sum of ng partial images,
// partial ||f||^2 in slot 0
__global__ void __launch_bounds__(256) cgls_f_kernel(SBDev d, const double* __restrict__ T,
                                                     int ng, int levels) {
  if (sb_skip(d, levels)) return;
  __shared__ double sh[4];
  SB_ROWS
  double acc = 0.0;
  for (long e = lo + threadIdx.x; e < hi; e += 256) {
    const int r = (int)(e / d.n), c = (int)(e - (long)r * d.n);
    const double v = sb_sum_parts(T, ng, NN, e) +
                     d.lam * (dLxT(d.r2, d.n, r, c) + dLyT(d.r3, d.n, r, c));
    d.f[e] = v;
    acc += v * v;
  }
  acc = sb_block_sum(acc, sh);
  if (threadIdx.x == 0) d.part[blockIdx.x * 4 + 0] = acc;
}

// w = f, tau = ||f||^2 (start of CGLS)
__global__ void __launch_bounds__(256) cgls_w_init_kernel(SBDev d) {
  if (sb_skip(d, 1)) return;
  __shared__ double sh[4];
  const double tau = sb_partials(d.part, 0, sh);
  SB_ROWS
  for (long e = lo + threadIdx.x; e < hi; e += 256) d.w[e] = d.f[e];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    d.scal[0] = tau;
    if (tau == 0.0) d.flags[1] = 1;
  }
}

// z1 = A w (the sum of the ng partial images at P); partial
// ||z||^2 = ||A w||^2 + lam^2 (||L_x w||^2 + ||L_y w||^2) in slot 1
__global__ void __launch_bounds__(256) cgls_zn_kernel(SBDev d, const double* __restrict__ P,
                                                      int ng) {
  if (sb_skip(d, 2)) return;
  __shared__ double sh[4];
  SB_ROWS
  double acc = 0.0;
  for (long e = lo + threadIdx.x; e < hi; e += 256) {
    const int r = (int)(e / d.n), c = (int)(e - (long)r * d.n);
    const double z1 = sb_sum_parts(P, ng, NN, e);
    d.z1[e] = z1;
    const double lx = d.lam * dLx(d.w, d.n, r, c);
    const double ly = d.lam * dLy(d.w, d.n, r, c);
    acc += z1 * z1 + lx * lx + ly * ly;
  }
  acc = sb_block_sum(acc, sh);
  if (threadIdx.x == 0) d.part[blockIdx.x * 4 + 1] = acc;
}

// mu = tau / ||z||^2; x += mu w; r -= mu z; partials ||mu w||^2 (slot 2), ||x||^2 (3).
// The partial of ||z||^2, tau and the first pixel's operands (none depends on
// mu) are requested together, before the reduction's barriers.
__global__ void __launch_bounds__(256) cgls_xr_kernel(SBDev d) {
  if (sb_skip(d, 2)) return;
  __shared__ double sh[4];
  SB_ROWS
  const double pz = d.part[threadIdx.x * 4 + 1];
  const double tau = d.scal[0];
  const long e0 = lo + threadIdx.x;
  double we = 0.0, xe = 0.0, r1e = 0.0, z1e = 0.0, r2e = 0.0, r3e = 0.0, lxw = 0.0, lyw = 0.0;
  auto fetch = [&](long e) {
    const int r = (int)(e / d.n), c = (int)(e - (long)r * d.n);
    we = d.w[e];
    xe = d.x[e];
    r1e = d.r1[e];
    z1e = d.z1[e];
    r2e = d.r2[e];
    r3e = d.r3[e];
    lxw = dLx(d.w, d.n, r, c);
    lyw = dLy(d.w, d.n, r, c);
  };
  if (e0 < hi) fetch(e0);
  const double zz = sb_block_sum(pz, sh);
  const double mu = tau / zz;
  double a2 = 0.0, a3 = 0.0;
  for (long e = e0; e < hi; e += 256) {
    if (e != e0) fetch(e);
    const double xn = xe + mu * we;
    d.x[e] = xn;
    d.r1[e] = r1e - mu * z1e;
    d.r2[e] = r2e - mu * d.lam * lxw;
    d.r3[e] = r3e - mu * d.lam * lyw;
    a2 += (mu * we) * (mu * we);
    a3 += xn * xn;
  }
  a2 = sb_block_sum(a2, sh);
  a3 = sb_block_sum(a3, sh);
  if (threadIdx.x == 0) {
    d.part[blockIdx.x * 4 + 2] = a2;
    d.part[blockIdx.x * 4 + 3] = a3;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) d.scal[5] = tau;   // tau of this iteration
}

// tau' = ||f||^2, delta = tau'/tau, w = f + delta w; RC_CGLS into scal[3];
// block 0 counts the iteration and applies the stopping test. Blocks that
// start after the test has fired skip their w update, which the solve no
// longer reads (the next outer iteration restarts CGLS from w = f). The three
// partial slots, tau and the first pixel's f and w are requested together,
// before the reductions' barriers.
__global__ void __launch_bounds__(256) cgls_w_kernel(SBDev d) {
  if (sb_skip(d, 2)) return;
  __shared__ double sh[4];
  SB_ROWS
  const double p0 = d.part[threadIdx.x * 4 + 0];
  const double p2 = d.part[threadIdx.x * 4 + 2];
  const double p3 = d.part[threadIdx.x * 4 + 3];
  const double tau_old = d.scal[5];
  const long e0 = lo + threadIdx.x;
  double f0 = 0.0, w0 = 0.0;
  if (e0 < hi) {
    f0 = d.f[e0];
    w0 = d.w[e0];
  }
  const double tau_new = sb_block_sum(p0, sh);
  const double delta = tau_new / tau_old;
  if (e0 < hi) d.w[e0] = f0 + delta * w0;
  for (long e = e0 + 256; e < hi; e += 256) d.w[e] = d.f[e] + delta * d.w[e];
  const double s2 = sb_block_sum(p2, sh);
  const double s3 = sb_block_sum(p3, sh);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const double rc = s3 > 0.0 ? sqrt(s2) / sqrt(s3) : 0.0;
    d.scal[0] = tau_new;
    d.scal[3] = rc;
    d.flags[2] += 1;
    if ((d.tau_cgls > 0.0 && rc < d.tau_cgls) || tau_new == 0.0) d.flags[1] = 1;
  }
}

// c = L x + g, shrink, g = c - d; RC_SB partials; xprev = x
__global__ void __launch_bounds__(256) sb_shrink_kernel(SBDev d) {
  if (sb_skip(d, 1)) return;
  __shared__ double sh[4];
  SB_ROWS
  double a0 = 0.0, a1 = 0.0;
  for (long e = lo + threadIdx.x; e < hi; e += 256) {
    const int r = (int)(e / d.n), c = (int)(e - (long)r * d.n);
    const double cx = dLx(d.x, d.n, r, c) + d.gx[e];
    const double cy = dLy(d.x, d.n, r, c) + d.gy[e];
    double ddx, ddy;
    if (d.iso) {
      const double s = sqrt(cx * cx + cy * cy);
      const double sc = s > 0.0 ? fmax(s - d.thr, 0.0) / s : 0.0;
      ddx = cx * sc;
      ddy = cy * sc;
    } else {
      ddx = (cx > 0.0 ? 1.0 : (cx < 0.0 ? -1.0 : 0.0)) * fmax(fabs(cx) - d.thr, 0.0);
      ddy = (cy > 0.0 ? 1.0 : (cy < 0.0 ? -1.0 : 0.0)) * fmax(fabs(cy) - d.thr, 0.0);
    }
    d.dx[e] = ddx;
    d.dy[e] = ddy;
    d.gx[e] = cx - ddx;
    d.gy[e] = cy - ddy;
    const double xe = d.x[e], xp = d.xprev[e];
    a0 += (xe - xp) * (xe - xp);
    a1 += xp * xp;
    d.xprev[e] = xe;
  }
  a0 = sb_block_sum(a0, sh);
  a1 = sb_block_sum(a1, sh);
  if (threadIdx.x == 0) {
    d.part[blockIdx.x * 4 + 0] = a0;
    d.part[blockIdx.x * 4 + 1] = a1;
  }
}

__global__ void __launch_bounds__(256) sb_check_kernel(SBDev d) {
  if (sb_skip(d, 1)) return;
  __shared__ double sh[4];
  const double a0 = sb_partials(d.part, 0, sh);
  const double a1 = sb_partials(d.part, 1, sh);
  if (threadIdx.x == 0) {
    const double rc = a1 > 0.0 ? sqrt(a0 / a1) : 0.0;
    d.scal[2] = rc;
    d.flags[3] += 1;
    if (d.tau_sb > 0.0 && rc < d.tau_sb) d.flags[0] = 1;
  }
}

// ---------------------------------------------------------------------------
static dim3 grid_red() { return dim3(kRedBlocks); }

void sb_launch_rhs(const SBDev& d, hipStream_t s) {
  hipLaunchKernelGGL(sb_rhs_kernel, grid_red(), dim3(256), 0, s, d);
}
void sb_launch_f(const SBDev& d, const double* T, int ng, int levels, hipStream_t s) {
  hipLaunchKernelGGL(cgls_f_kernel, grid_red(), dim3(256), 0, s, d, T, ng, levels);
}
void sb_launch_w_init(const SBDev& d, hipStream_t s) {
  hipLaunchKernelGGL(cgls_w_init_kernel, grid_red(), dim3(256), 0, s, d);
}
void sb_launch_zn(const SBDev& d, const double* P, int ng, hipStream_t s) {
  hipLaunchKernelGGL(cgls_zn_kernel, grid_red(), dim3(256), 0, s, d, P, ng);
}
void sb_launch_xr(const SBDev& d, hipStream_t s) {
  hipLaunchKernelGGL(cgls_xr_kernel, grid_red(), dim3(256), 0, s, d);
}
void sb_launch_w(const SBDev& d, hipStream_t s) {
  hipLaunchKernelGGL(cgls_w_kernel, grid_red(), dim3(256), 0, s, d);
}
void sb_launch_shrink(const SBDev& d, hipStream_t s) {
  hipLaunchKernelGGL(sb_shrink_kernel, grid_red(), dim3(256), 0, s, d);
}
void sb_launch_check(const SBDev& d, hipStream_t s) {
  hipLaunchKernelGGL(sb_check_kernel, dim3(1), dim3(256), 0, s, d);
}

}  // namespace kpsb
