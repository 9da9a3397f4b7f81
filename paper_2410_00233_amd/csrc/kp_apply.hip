// Kronecker-sum apply (paper, eq. "KPAx"): array(A_k x) = sum_t Ay_t X Ax_t^T
// and its transpose sum_t Ay_t^T X Ax_t, in FP64 on MFMA
// (v_mfma_f64_16x16x4f64).
//
// Two batched GEMMs over the k terms: Z_t = X op(Ax_t) (one output tile per
// workgroup and term), then the partial sums P_g = sum_{t in group g} op(Ay_t)
// Z_t, each workgroup accumulating the terms of its group in registers. The
// consumer adds the ngroups partials in a fixed order (deterministic). 4 k n^3
// flops per apply.
//
// GEMM kernel: a TM x TN output tile per 256-thread workgroup, each of the 4
// waves owning a (TM/2) x (TN/2) quadrant of 16 x 16 MFMA blocks; K tiles of KT
// staged through two LDS buffers, the next tile's global loads in flight in
// registers while the current one is multiplied (one barrier per K tile).
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
  int terms;       // number of terms t (A and B advance by sAz, sBz per term)
  int group;       // terms accumulated per workgroup (blockIdx.z = group index)
  const int* flags;  // skip when any of flags[0..nflags) is nonzero
  int nflags;
};

template <int TM, int TN, int KT>
struct GemmCfg {
  static constexpr int SA = TM + 16;   // LDS row strides (doubles): consecutive
  static constexpr int SB = TN + 16;   // rows 32 banks apart
  static constexpr int LA = TM * KT / 256;               // A elements per thread
  static constexpr int LB = TN * KT / 256;
  static constexpr int BI = TM / 32;                     // MFMA blocks per wave (rows)
  static constexpr int BJ = TN / 32;                     //                      (cols)
  static constexpr int LDS = 2 * KT * (SA + SB);         // doubles
};

template <int TM, int TN, int KT>
__global__ void __launch_bounds__(256) gemm_f64_kernel(GemmArgs g) {
  using Cfg = GemmCfg<TM, TN, KT>;
  if (g.flags)
    for (int i = 0; i < g.nflags; ++i)
      if (g.flags[i]) return;
  __shared__ double lds[Cfg::LDS];
  double* As = lds;                         // [2][KT][SA]
  double* Bs = lds + 2 * KT * Cfg::SA;      // [2][KT][SB]
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  // XCD-aware order: workgroups are dispatched to the 8 XCDs round-robin by
  // linear id; give each XCD a contiguous range of (tile, term) work so that
  // its L2 holds the operands of a few terms instead of all of them.
  const int gx = gridDim.x, gy = gridDim.y;
  const int total_wg = gx * gy * gridDim.z;
  const int lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const int per = total_wg / 8;
  const int ell = lin < per * 8 ? (lin % 8) * per + lin / 8 : lin;
  const int bx = ell % gx, by = (ell / gx) % gy, bz = ell / (gx * gy);
  const int m0 = bx * TM, n0 = by * TN;
  const int t_begin = bz * g.group;
  const int t_end = min(t_begin + g.group, g.terms);
  const int nK = (g.K + KT - 1) / KT;
  const int total = (t_end - t_begin) * nK;

  // Element e of a tile: along the contiguous global direction in runs of 4
  // (32-byte segments) when that direction is k, else along m (or n); the LDS
  // stores then hit at most two rows at once per bank.
  auto mapA = [&](int e, int& mm, int& kk) {
    if (g.transA) { mm = e % TM; kk = e / TM; }
    else { kk = (e & 3) + 4 * (e / (4 * TM)); mm = (e >> 2) % TM; }
  };
  auto mapB = [&](int e, int& nn, int& kk) {
    if (g.transB) { kk = (e & 3) + 4 * (e / (4 * TN)); nn = (e >> 2) % TN; }
    else { nn = e % TN; kk = e / TN; }
  };
  double ra[Cfg::LA], rb[Cfg::LB];
  auto load = [&](int it) {
    const int t = t_begin + it / nK;
    const int k0 = (it % nK) * KT;
    const double* A = g.A + (long)t * g.sAz;
    const double* B = g.B + (long)t * g.sBz;
#pragma unroll
    for (int q = 0; q < Cfg::LA; ++q) {
      int mm, kk;
      mapA(tid + 256 * q, mm, kk);
      const int m = m0 + mm, kg = k0 + kk;
      ra[q] = (m < g.M && kg < g.K) ? (g.transA ? A[(long)kg * g.lda + m] : A[(long)m * g.lda + kg])
                                    : 0.0;
    }
#pragma unroll
    for (int q = 0; q < Cfg::LB; ++q) {
      int nn, kk;
      mapB(tid + 256 * q, nn, kk);
      const int c = n0 + nn, kb = k0 + kk;
      rb[q] = (c < g.N && kb < g.K) ? (g.transB ? B[(long)c * g.ldb + kb] : B[(long)kb * g.ldb + c])
                                    : 0.0;
    }
  };
  auto store = [&](int buf) {
    double* as = As + buf * KT * Cfg::SA;
    double* bs = Bs + buf * KT * Cfg::SB;
#pragma unroll
    for (int q = 0; q < Cfg::LA; ++q) {
      int mm, kk;
      mapA(tid + 256 * q, mm, kk);
      as[kk * Cfg::SA + mm] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < Cfg::LB; ++q) {
      int nn, kk;
      mapB(tid + 256 * q, nn, kk);
      bs[kk * Cfg::SB + nn] = rb[q];
    }
  };

  doublex4 acc[Cfg::BI][Cfg::BJ];
#pragma unroll
  for (int i = 0; i < Cfg::BI; ++i)
#pragma unroll
    for (int j = 0; j < Cfg::BJ; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[i][j][e] = 0.0;

  if (total > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  for (int it = 0; it < total; ++it) {
    const int buf = it & 1;
    if (it + 1 < total) load(it + 1);
    const double* as = As + buf * KT * Cfg::SA;
    const double* bs = Bs + buf * KT * Cfg::SB;
#pragma unroll
    for (int s = 0; s < KT / 4; ++s) {
      const int kk = 4 * s + (lane >> 4);
      double a[Cfg::BI], b[Cfg::BJ];
#pragma unroll
      for (int i = 0; i < Cfg::BI; ++i) a[i] = as[kk * Cfg::SA + wm * (TM / 2) + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < Cfg::BJ; ++j) b[j] = bs[kk * Cfg::SB + wn * (TN / 2) + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < Cfg::BI; ++i)
#pragma unroll
        for (int j = 0; j < Cfg::BJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (it + 1 < total) store(buf ^ 1);
    __syncthreads();
  }
  // D layout of the FP64 MFMA: lane l, item e -> row l/16 + 4e, column l%16
  double* C = g.C + (long)bz * g.sCz;
#pragma unroll
  for (int i = 0; i < Cfg::BI; ++i)
#pragma unroll
    for (int j = 0; j < Cfg::BJ; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = m0 + wm * (TM / 2) + 16 * i + (lane >> 4) + 4 * e;
        const int c = n0 + wn * (TN / 2) + 16 * j + (lane & 15);
        if (m < g.M && c < g.N) C[(long)m * g.ldc + c] = acc[i][j][e];
      }
}

// Y[e] = sum_{g<ng} P[g*NN + e]  (fixed order)
__global__ void sum_terms_kernel(const double* __restrict__ P, int ng, long NN,
                                 double* __restrict__ Y, const int* __restrict__ flags,
                                 int nflags) {
  if (flags)
    for (int i = 0; i < nflags; ++i)
      if (flags[i]) return;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < NN;
       e += (long)gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int t = 0; t < ng; ++t) v += P[(long)t * NN + e];
    Y[e] = v;
  }
}

// Output tile and terms per workgroup for n x n images and k terms: 64 x 64
// tiles once they give at least 1024 workgroups per GEMM, else 32 x 32; the
// second GEMM accumulates `group` terms per workgroup while that still leaves
// about 1024 workgroups.
KpApplyPlan kp_apply_plan(int n, int k) {
  KpApplyPlan p;
  const long t64 = (long)((n + 63) / 64) * ((n + 63) / 64);
  const long t32 = (long)((n + 31) / 32) * ((n + 31) / 32);
  p.tile = t64 * k >= 1024 ? 64 : 32;
  const long tiles = p.tile == 64 ? t64 : t32;
  p.group = (int)std::max<long>(1, std::min<long>(k, tiles * k / 1024));
  p.ngroups = (k + p.group - 1) / p.group;
  return p;
}

template <int T, int KT>
static void gemm_launch(const GemmArgs& g, int zdim, hipStream_t s) {
  dim3 grid((g.M + T - 1) / T, (g.N + T - 1) / T, zdim);
  hipLaunchKernelGGL((gemm_f64_kernel<T, T, KT>), grid, dim3(256), 0, s, g);
}

// Launch variants (output tile, K tile), picked by the autotuner; the order of
// accumulation of every output element is the same in all of them.
static void gemm(const GemmArgs& g, int variant, int zdim, hipStream_t s) {
  switch (variant) {
    case 1: gemm_launch<32, 32>(g, zdim, s); break;
    case 2: gemm_launch<32, 16>(g, zdim, s); break;
    case 3: gemm_launch<64, 8>(g, zdim, s); break;   // half the LDS: twice the resident tiles
    default: gemm_launch<64, 16>(g, zdim, s); break;
  }
}

// Z (k x n x n) is workspace; P receives plan.ngroups partial images.
void launch_kp_apply_parts(const double* Ax, const double* Ay, int n, int k, int transpose,
                           const double* X, double* Z, double* P, const KpApplyPlan& plan,
                           const int* flags, int nflags, hipStream_t s) {
  const long NN = (long)n * n;
  // Z_t = X * (transpose ? Ax_t : Ax_t^T)
  GemmArgs g1{X, n, 0, 0, Ax, n, NN, transpose ? 0 : 1, Z, n, NN, n, n, n, k, 1, flags, nflags};
  // P_g = sum_{t in g} (transpose ? Ay_t^T : Ay_t) * Z_t
  GemmArgs g2{Ay, n, NN, transpose ? 1 : 0, Z, n, NN, 0, P, n, NN, n, n, n, k, plan.group,
              flags, nflags};
  const int v = tune_pick(kTuneApply, n, k, transpose, 4, [&](int vv) -> double {
    GemmArgs a = g1, b = g2;
    a.flags = b.flags = nullptr;   // the sample launches always run
    a.nflags = b.nflags = 0;
    return time_launches(s, 2, [&]() {
      gemm(a, vv, k, s);
      gemm(b, vv, plan.ngroups, s);
    });
  });
  gemm(g1, v, k, s);
  gemm(g2, v, plan.ngroups, s);
}

void launch_sum_parts(const double* P, int ng, long NN, double* Y, hipStream_t s) {
  long blocks = (NN + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(sum_terms_kernel, dim3((int)blocks), dim3(256), 0, s, P, ng, NN, Y,
                     (const int*)nullptr, 0);
}

void launch_kp_apply_ws(const double* Ax, const double* Ay, int n, int k, int transpose,
                        const double* X, double* Y, double* Z, double* P, const int* flags,
                        int nflags, hipStream_t s) {
  const KpApplyPlan plan = kp_apply_plan(n, k);
  launch_kp_apply_parts(Ax, Ay, n, k, transpose, X, Z, P, plan, flags, nflags, s);
  const long NN = (long)n * n;
  long blocks = (NN + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(sum_terms_kernel, dim3((int)blocks), dim3(256), 0, s, P, plan.ngroups, NN,
                     Y, flags, nflags);
}

}  // namespace kpsb
