// Kronecker-sum apply (paper, eq. "KPAx"): array(A_k x) = sum_t Ay_t X Ax_t^T
// and its transpose sum_t Ay_t^T X Ax_t, in FP64 on MFMA
// (v_mfma_f64_16x16x4f64).
//
// Both products of a term are n x n x n GEMMs, batched over the k terms
// (grid.z = t): Z_t = X op(Ax_t), P_t = op(Ay_t) Z_t, then Y = sum_t P_t is
// reduced in a fixed order (deterministic). 2 * 2 k n^3 flops per apply.
#include "common.h"
#include "sb.h"

namespace kpsb {

struct GemmArgs {
  const double* A;
  long lda, sAz;
  int transA;      // A(m, kk) = transA ? A[kk*lda + m] : A[m*lda + kk]
  const double* B;
  long ldb, sBz;
  int transB;      // B(kk, c) = transB ? B[c*ldb + kk] : B[kk*ldb + c]
  double* C;
  long ldc, sCz;
  int M, N, K;
  const int* flags;  // skip when any of flags[0..nflags) is nonzero
  int nflags;
};

constexpr int kGT = 64;     // output tile
constexpr int kGK = 16;     // K tile
constexpr int kGP = 80;     // LDS row stride (doubles), bank-conflict padding

__global__ void __launch_bounds__(256) gemm_f64_kernel(GemmArgs g) {
  if (g.flags)
    for (int i = 0; i < g.nflags; ++i)
      if (g.flags[i]) return;
  __shared__ double As[kGK * kGP];
  __shared__ double Bs[kGK * kGP];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int m0 = blockIdx.x * kGT, n0 = blockIdx.y * kGT;
  const double* A = g.A + (long)blockIdx.z * g.sAz;
  const double* B = g.B + (long)blockIdx.z * g.sBz;
  double* C = g.C + (long)blockIdx.z * g.sCz;
  const int wm = wave & 1, wn = wave >> 1;
  doublex4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[i][j][e] = 0.0;

  for (int k0 = 0; k0 < g.K; k0 += kGK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;          // 0 .. 1023
      int mm, kk;
      if (g.transA) { mm = e & 63; kk = e >> 6; } else { kk = e & 15; mm = e >> 4; }
      const int m = m0 + mm, kg = k0 + kk;
      double v = 0.0;
      if (m < g.M && kg < g.K) v = g.transA ? A[(long)kg * g.lda + m] : A[(long)m * g.lda + kg];
      As[kk * kGP + mm] = v;
      int nn;
      if (g.transB) { kk = e & 15; nn = e >> 4; } else { nn = e & 63; kk = e >> 6; }
      const int c = n0 + nn, kb = k0 + kk;
      double u = 0.0;
      if (c < g.N && kb < g.K) u = g.transB ? B[(long)c * g.ldb + kb] : B[(long)kb * g.ldb + c];
      Bs[kk * kGP + nn] = u;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kGK / 4; ++s) {
      const int kk = 4 * s + (lane >> 4);
      double a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[kk * kGP + wm * 32 + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kk * kGP + wn * 32 + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // D layout of the FP64 MFMA: lane l, item e -> row l/16 + 4e, column l%16
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = m0 + wm * 32 + 16 * i + (lane >> 4) + 4 * e;
        const int c = n0 + wn * 32 + 16 * j + (lane & 15);
        if (m < g.M && c < g.N) C[(long)m * g.ldc + c] = acc[i][j][e];
      }
}

// Y[e] = sum_{t<k} P[t*NN + e]  (fixed order)
__global__ void sum_terms_kernel(const double* __restrict__ P, int k, long NN,
                                 double* __restrict__ Y, const int* __restrict__ flags,
                                 int nflags) {
  if (flags)
    for (int i = 0; i < nflags; ++i)
      if (flags[i]) return;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < NN;
       e += (long)gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int t = 0; t < k; ++t) v += P[(long)t * NN + e];
    Y[e] = v;
  }
}

static void gemm(const GemmArgs& g, int batch, hipStream_t s) {
  dim3 grid((g.M + kGT - 1) / kGT, (g.N + kGT - 1) / kGT, batch);
  hipLaunchKernelGGL(gemm_f64_kernel, grid, dim3(256), 0, s, g);
}

// Z (k x n x n) and P (k x n x n) are caller workspace.
void launch_kp_apply_ws(const double* Ax, const double* Ay, int n, int k, int transpose,
                        const double* X, double* Y, double* Z, double* P, const int* flags,
                        int nflags, hipStream_t s) {
  const long NN = (long)n * n;
  // Z_t = X * (transpose ? Ax_t : Ax_t^T)
  GemmArgs g1{X, n, 0, 0, Ax, n, NN, transpose ? 0 : 1, Z, n, NN, n, n, n, flags, nflags};
  gemm(g1, k, s);
  // P_t = (transpose ? Ay_t^T : Ay_t) * Z_t
  GemmArgs g2{Ay, n, NN, transpose ? 1 : 0, Z, n, NN, 0, P, n, NN, n, n, n, flags, nflags};
  gemm(g2, k, s);
  long blocks = (NN + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(sum_terms_kernel, dim3((int)blocks), dim3(256), 0, s, P, k, NN, Y, flags,
                     nflags);
}

}  // namespace kpsb
