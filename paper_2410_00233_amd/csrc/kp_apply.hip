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
// registers while the current one is multiplied (one barrier per K tile). Each
// operand is read from HBM / L2 along its contiguous direction in whole cache
// lines, whichever of m, n or k that is.
#include "common.h"
#include "sb.h"
#include "partials.h"

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
  // LDS layout of a staged tile (doubles). An operand contiguous along k in
  // global memory is loaded along k (16 lanes cover a 128-byte line) and staged
  // [m][k] with row stride KT + 1: the 16 rows of a fragment read then sit 2
  // banks apart. An operand contiguous along m (or n) is loaded along m and
  // staged [k][m] with row stride TM + 16.
  static constexpr int SKA = KT + 1, SMA = TM + 16;
  static constexpr int SKB = KT + 1, SNB = TN + 16;
  static constexpr int TILE_A = TM * SKA > KT * SMA ? TM * SKA : KT * SMA;
  static constexpr int TILE_B = TN * SKB > KT * SNB ? TN * SKB : KT * SNB;
  static constexpr int LA = TM * KT / 256;               // A elements per thread
  static constexpr int LB = TN * KT / 256;
  static constexpr int BI = TM / 32;                     // MFMA blocks per wave (rows)
  static constexpr int BJ = TN / 32;                     //                      (cols)
  static constexpr int LDS = 2 * (TILE_A + TILE_B);      // doubles
};

// AKC / BKC: A (B) contiguous along k in global memory (see GemmCfg).
// FULL: M, N, K are multiples of TM, TN, KT (no bounds checks; the general form
// zero-fills outside the operands). The term and K offset of the next tile to
// load advance incrementally, as do the per-thread load pointers, so a K step
// issues little besides its loads, LDS traffic and MFMAs. D: K tiles whose
// loads are in flight (a ring of D register slots, the K loop unrolled by D;
// past the last tile the last one is loaded again and never used).
template <int TM, int TN, int KT, bool AKC, bool BKC, bool FULL, int D>
__global__ void __launch_bounds__(256) gemm_f64_kernel(GemmArgs g) {
  using Cfg = GemmCfg<TM, TN, KT>;
  if (g.flags)
    for (int i = 0; i < g.nflags; ++i)
      if (g.flags[i]) return;
  __shared__ double lds[Cfg::LDS];
  double* As = lds;                         // [2][TILE_A]
  double* Bs = lds + 2 * Cfg::TILE_A;       // [2][TILE_B]
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

  // element e = tid + 256 q of a tile -> (row along m or n, kk), following the
  // contiguous direction; offsets in the tile (global) and in LDS
  auto mapA = [&](int e, int& mm, int& kk) {
    if (AKC) { mm = e / KT; kk = e % KT; }
    else { mm = e % TM; kk = e / TM; }
  };
  auto mapB = [&](int e, int& nn, int& kk) {
    if (BKC) { nn = e / KT; kk = e % KT; }
    else { nn = e % TN; kk = e / TN; }
  };
  auto offA = [](int mm, int kk) { return AKC ? mm * Cfg::SKA + kk : kk * Cfg::SMA + mm; };
  auto offB = [](int nn, int kk) { return BKC ? nn * Cfg::SKB + kk : kk * Cfg::SNB + nn; };
  const long lda = g.lda, ldb = g.ldb;
  long ga[Cfg::LA], gb[Cfg::LB];       // element offsets from the tile origin
  int la[Cfg::LA], lb[Cfg::LB];        // LDS offsets
  int ma[Cfg::LA], ka[Cfg::LA], nb_[Cfg::LB], kb_[Cfg::LB];
#pragma unroll
  for (int q = 0; q < Cfg::LA; ++q) {
    mapA(tid + 256 * q, ma[q], ka[q]);
    ga[q] = AKC ? (long)ma[q] * lda + ka[q] : (long)ka[q] * lda + ma[q];
    la[q] = offA(ma[q], ka[q]);
  }
#pragma unroll
  for (int q = 0; q < Cfg::LB; ++q) {
    mapB(tid + 256 * q, nb_[q], kb_[q]);
    gb[q] = BKC ? (long)nb_[q] * ldb + kb_[q] : (long)kb_[q] * ldb + nb_[q];
    lb[q] = offB(nb_[q], kb_[q]);
  }
  // tile origin of term t, K offset k0: A + t sAz + (AKC ? m0 lda + k0 : k0 lda + m0)
  const long a_step = AKC ? KT : (long)KT * lda;    // per K tile
  const long b_step = BKC ? KT : (long)KT * ldb;
  const double* a_org = g.A + (AKC ? (long)m0 * lda : m0);
  const double* b_org = g.B + (BKC ? (long)n0 * ldb : n0);
  int lt = t_begin, lk0 = 0;                        // the next tile to load
  int left = total;                                 // tiles not loaded yet
  const double* pa = a_org + (long)lt * g.sAz;
  const double* pb = b_org + (long)lt * g.sBz;
  double ra[D][Cfg::LA], rb[D][Cfg::LB];
  // loads the next tile into slot u (again the last one once all are loaded)
  auto load = [&](int u) {
#pragma unroll
    for (int q = 0; q < Cfg::LA; ++q) {
      if (FULL) ra[u][q] = pa[ga[q]];
      else ra[u][q] = (m0 + ma[q] < g.M && lk0 + ka[q] < g.K) ? pa[ga[q]] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < Cfg::LB; ++q) {
      if (FULL) rb[u][q] = pb[gb[q]];
      else rb[u][q] = (n0 + nb_[q] < g.N && lk0 + kb_[q] < g.K) ? pb[gb[q]] : 0.0;
    }
    if (--left > 0) {
      lk0 += KT;
      pa += a_step;
      pb += b_step;
      if (lk0 >= g.K) {                // next term
        lk0 = 0;
        ++lt;
        pa = a_org + (long)lt * g.sAz;
        pb = b_org + (long)lt * g.sBz;
      }
    } else {
      left = 0;
    }
  };
  auto store = [&](int buf, int u) {
    double* as = As + buf * Cfg::TILE_A;
    double* bs = Bs + buf * Cfg::TILE_B;
#pragma unroll
    for (int q = 0; q < Cfg::LA; ++q) as[la[q]] = ra[u][q];
#pragma unroll
    for (int q = 0; q < Cfg::LB; ++q) bs[lb[q]] = rb[u][q];
  };

  doublex4 acc[Cfg::BI][Cfg::BJ];
#pragma unroll
  for (int i = 0; i < Cfg::BI; ++i)
#pragma unroll
    for (int j = 0; j < Cfg::BJ; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[i][j][e] = 0.0;

  auto multiply = [&](int buf) {
    const double* as = As + buf * Cfg::TILE_A;
    const double* bs = Bs + buf * Cfg::TILE_B;
#pragma unroll
    for (int s = 0; s < KT / 4; ++s) {
      const int kk = 4 * s + (lane >> 4);
      double a[Cfg::BI], b[Cfg::BJ];
#pragma unroll
      for (int i = 0; i < Cfg::BI; ++i) a[i] = as[offA(wm * (TM / 2) + 16 * i + (lane & 15), kk)];
#pragma unroll
      for (int j = 0; j < Cfg::BJ; ++j) b[j] = bs[offB(wn * (TN / 2) + 16 * j + (lane & 15), kk)];
#pragma unroll
      for (int i = 0; i < Cfg::BI; ++i)
#pragma unroll
        for (int j = 0; j < Cfg::BJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  };

  if (total > 0) {
#pragma unroll
    for (int u = 0; u < D; ++u) load(u);
    store(0, 0);
    __syncthreads();
    int it0 = 0;
    for (; it0 + D <= total; it0 += D) {
#pragma unroll
      for (int u = 0; u < D; ++u) {
        const int it = it0 + u;
        load(u);                           // slot u held tile it, now in LDS
        multiply(it & 1);
        store((it + 1) & 1, (u + 1) % D);  // tile it + 1 (the last tile again at the end)
        __syncthreads();
      }
    }
#pragma unroll
    for (int u = 0; u + 1 < D; ++u) {      // the remaining total % D tiles
      const int it = it0 + u;
      if (it < total) {
        multiply(it & 1);
        if (it + 1 < total) store((it + 1) & 1, (u + 1) % D);
        __syncthreads();
      }
    }
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
        if (FULL || (m < g.M && c < g.N)) C[(long)m * g.ldc + c] = acc[i][j][e];
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
    Y[e] = add_partials_in_order(0.0, P + e, 0, ng, NN);
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

template <int T, int KT, int D, bool AKC, bool BKC>
static void gemm_launch2(const GemmArgs& g, int zdim, hipStream_t s) {
  dim3 grid((g.M + T - 1) / T, (g.N + T - 1) / T, zdim);
  const bool full = g.M % T == 0 && g.N % T == 0 && g.K % KT == 0;
  if (full)
    hipLaunchKernelGGL((gemm_f64_kernel<T, T, KT, AKC, BKC, true, D>), grid, dim3(256), 0, s, g);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<T, T, KT, AKC, BKC, false, D>), grid, dim3(256), 0, s, g);
}

// the operand layouts of the two GEMMs of an apply in either direction:
// (A, B) contiguous along k: (yes, yes), (yes, no) or (no, no)
template <int T, int KT, int D = 1>
static void gemm_launch(const GemmArgs& g, int zdim, hipStream_t s) {
  const bool akc = !g.transA, bkc = g.transB != 0;
  if (akc && bkc) gemm_launch2<T, KT, D, true, true>(g, zdim, s);
  else if (akc) gemm_launch2<T, KT, D, true, false>(g, zdim, s);
  else if (bkc) gemm_launch2<T, KT, D, false, true>(g, zdim, s);
  else gemm_launch2<T, KT, D, false, false>(g, zdim, s);
}

// Launch variants (output tile, K tile), picked by the autotuner; the order of
// accumulation of every output element is the same in all of them.
constexpr int kNumApplyVariants = 8;
static void gemm(const GemmArgs& g, int variant, int zdim, hipStream_t s) {
  switch (variant) {
    case 1: gemm_launch<32, 32>(g, zdim, s); break;
    case 2: gemm_launch<32, 16>(g, zdim, s); break;
    case 3: gemm_launch<64, 8>(g, zdim, s); break;   // half the LDS: twice the resident tiles
    case 4: gemm_launch<32, 16, 4>(g, zdim, s); break;
    case 5: gemm_launch<32, 32, 2>(g, zdim, s); break;
    case 6: gemm_launch<64, 16, 2>(g, zdim, s); break;
    case 7: gemm_launch<64, 8, 4>(g, zdim, s); break;
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
  const int v = tune_pick(kTuneApply, n, k, transpose, kNumApplyVariants, [&](int vv) -> double {
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
