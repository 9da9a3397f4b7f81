// Small dense SVD in FP64 on one workgroup: one-sided (Hestenes) Jacobi with a
// round-robin pair ordering. Used for the (k_p+1) x k_p bidiagonal of
// Algorithm 1 ("svds" of C), for the k_p x k_p triangular factor that gives the
// SVD of H = Q^T B in Algorithm 2, and for the k x k factor of the
// Rayleigh-Ritz refinement. One-sided Jacobi is accurate to a small multiple of
// the unit roundoff relative to each singular value.
#include "common.h"

namespace kpsb {

constexpr int kJmax = 64;
constexpr int kJThreads = 1024;   // 16 waves: every pair of a round has its own wave
constexpr int kJWaves = kJThreads / 64;

__device__ __forceinline__ double jwave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ void __launch_bounds__(kJThreads)
jacobi_svd_kernel(const double* __restrict__ A, int m, int nc, double* __restrict__ U,
                  double* __restrict__ sig, double* __restrict__ V, int* __restrict__ sweeps_out) {
  __shared__ double W[kJmax * kJmax];    // columns of the working matrix (ld kJmax)
  __shared__ double Vs[kJmax * kJmax];   // accumulated right rotations (ld kJmax)
  __shared__ double nrm[kJmax];
  __shared__ int order[kJmax];
  __shared__ int rotated;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int nce = (nc + 1) & ~1;           // even number of columns (zero pad)

  for (int e = tid; e < kJmax * kJmax; e += kJThreads) {
    const int r = e % kJmax, c = e / kJmax;
    W[e] = (r < m && c < nc) ? A[r + (long)m * c] : 0.0;
    Vs[e] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  // Round-robin tournament: in round r of a sweep, position 0 holds column 0
  // and position i >= 1 holds column 1 + ((i - 1 - r) mod (nce - 1)) (column 0
  // fixed, the others rotated by one position per round; after nce - 1 rounds
  // the order is back to the start). Round r pairs positions k and nce - 1 - k.
  auto pos = [&](int i, int r) {
    if (i == 0) return 0;
    const int t = (i - 1 - r) % (nce - 1);
    return 1 + (t < 0 ? t + nce - 1 : t);
  };

  const double tol = 4.0 * 2.220446049250313e-16;
  int sweep = 0;
  for (; sweep < 60; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < nce - 1; ++round) {
      // the round's nce / 2 disjoint pairs, one per wave (they commute, so the
      // result does not depend on which wave takes which)
      for (int k = wave; k < nce / 2; k += kJWaves) {
        const int p = pos(k, round);
        const int q = pos(nce - 1 - k, round);
        const double wp = (lane < m) ? W[lane + kJmax * p] : 0.0;
        const double wq = (lane < m) ? W[lane + kJmax * q] : 0.0;
        const double alpha = jwave_sum(wp * wp);
        const double beta = jwave_sum(wq * wq);
        const double gamma = jwave_sum(wp * wq);
        if (gamma != 0.0 && fabs(gamma) > tol * sqrt(alpha * beta)) {
          const double zeta = (beta - alpha) / (2.0 * gamma);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t);
          const double s = c * t;
          if (lane < m) {
            W[lane + kJmax * p] = c * wp - s * wq;
            W[lane + kJmax * q] = s * wp + c * wq;
          }
          if (lane < nc) {
            const double vp = Vs[lane + kJmax * p];
            const double vq = Vs[lane + kJmax * q];
            Vs[lane + kJmax * p] = c * vp - s * vq;
            Vs[lane + kJmax * q] = s * vp + c * vq;
          }
          if (lane == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    const int any = rotated;
    __syncthreads();
    if (!any) break;
  }

  // singular values = column norms, then order descending (ties: lower index)
  for (int c = wave; c < nc; c += kJWaves) {
    const double w = (lane < m) ? W[lane + kJmax * c] : 0.0;
    const double s2 = jwave_sum(w * w);
    if (lane == 0) nrm[c] = sqrt(s2);
  }
  __syncthreads();
  if (tid < nc) {
    const double s = nrm[tid];
    int rank = 0;
    for (int i = 0; i < nc; ++i) {
      const double o = nrm[i];
      if (o > s || (o == s && i < tid)) ++rank;
    }
    order[rank] = tid;
  }
  __syncthreads();
  for (int e = tid; e < m * nc; e += kJThreads) {
    const int r = e % m, j = e / m;
    const int c = order[j];
    const double s = nrm[c];
    U[r + (long)m * j] = (s > 0.0) ? W[r + kJmax * c] / s : 0.0;
  }
  for (int e = tid; e < nc * nc; e += kJThreads) {
    const int r = e % nc, j = e / nc;
    V[r + (long)nc * j] = Vs[r + kJmax * order[j]];
  }
  if (tid < nc) sig[tid] = nrm[order[tid]];
  if (tid == 0 && sweeps_out) *sweeps_out = sweep;
}

void launch_jacobi_svd(const double* A, int m, int nc, double* U, double* sig, double* V,
                       int* sweeps, hipStream_t s) {
  hipLaunchKernelGGL(jacobi_svd_kernel, dim3(1), dim3(kJThreads), 0, s, A, m, nc, U, sig, V,
                     sweeps);
}

}  // namespace kpsb
