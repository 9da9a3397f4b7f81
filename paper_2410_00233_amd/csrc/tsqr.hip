// Orthonormal basis of a tall N x m block (the RSVD range finder's QR after
// every product with B or B^T, section 2.3): Householder TSQR in FP64.
//
// The rows are split into P0 leaves of nearly equal height (at least m rows,
// at most rows_max). Each leaf is factored by one workgroup with the block's
// columns held in registers (wave w owns columns w, w + 16, ...; lane l rows
// l, l + 64, ...): for column j the owning wave forms the Householder
// reflector H_j = I - tau_j v_j v_j^T (v_j = 1 at row j; LAPACK's choice of
// sign, beta = -sign(alpha) ||x||) and stores v_j in LDS, and after one barrier
// every wave applies H_j to its own columns. The R factors of the leaves are
// then stacked `fan` at a time and factored the same way, one launch per tree
// level, up to a single root (the R of the whole block).
//
// Q is then formed from the root down, one launch per level: each node applies
// its reflectors, last to first, to [E; 0] held in registers (E the m x m
// block its parent handed down, I_m at the root) and hands each child its m
// rows; the leaves write their rows of Q. Column j of Q and row j of R are
// multiplied by the sign of R_jj, so that R has a non-negative diagonal.
//
// Every sum runs in a fixed order (DPP wave reductions, fixed loops, a fixed
// tree), so results are reproducible bit for bit.
#include "common.h"

namespace kpsb {

constexpr int kTsqrWaves = 16;
constexpr int kTsqrThreads = 64 * kTsqrWaves;
constexpr int kTsqrRegs = 16;           // doubles per lane: columns per wave x rows per lane
constexpr int kTsqrMaxLevels = 24;
constexpr size_t kTsqrLds = 160 * 1024 - 1024;   // under the 160 KB per workgroup

struct TsqrPlan {
  long N;
  int m;
  int cpw;                         // columns per wave (1, 2 or 4)
  int rows_max;                    // rows of a node (leaf or stacked R's)
  int fan;                         // children per tree node
  int levels;                      // node levels; level 0 = leaves, level levels-1 = the root
  int count[kTsqrMaxLevels];       // nodes per level
  long first[kTsqrMaxLevels];      // index of each level's first node
  long nodes;                      // nodes in all levels
  // workspace (doubles from the base): reflectors, tau, R factors, and the
  // m x m blocks E handed down to every node below the root
  long off_v, off_tau, off_r, off_e;
  size_t bytes;
};

// LDS of both kernels: a node's reflectors (rows_max x m), an m x m block and
// a few scalars
static size_t tsqr_lds_bytes(int rows_max, int m) {
  return 8 * ((size_t)rows_max * m + (size_t)m * m + 256);
}

static bool tsqr_make_plan(long N, int m, TsqrPlan* p) {
  if (m < 1 || m > 64 || N < m) return false;
  p->N = N;
  p->m = m;
  p->cpw = m <= 16 ? 1 : (m <= 32 ? 2 : 4);
  const int rpl = kTsqrRegs / p->cpw;
  const long lds_rows = (long)(kTsqrLds - tsqr_lds_bytes(0, m)) / (8L * m);
  p->rows_max = (int)std::min<long>(64L * rpl, lds_rows);
  p->fan = p->rows_max / m;
  if (p->fan < 2) return false;                 // (not reached for m <= 64)
  long P0 = (N + p->rows_max - 1) / p->rows_max;
  P0 = std::min(P0, N / m);                     // every leaf gets at least m rows
  int L = 0;
  long cnt = P0, nodes = 0;
  for (;;) {
    if (L == kTsqrMaxLevels) return false;
    p->count[L] = (int)cnt;
    p->first[L] = nodes;
    nodes += cnt;
    ++L;
    if (cnt == 1) break;
    cnt = (cnt + p->fan - 1) / p->fan;
  }
  p->levels = L;
  p->nodes = nodes;
  p->off_v = 0;
  p->off_tau = nodes * p->rows_max * (long)m;
  p->off_r = p->off_tau + nodes * (long)m;
  p->off_e = p->off_r + nodes * (long)m * m;
  p->bytes = (size_t)(p->off_e + nodes * (long)m * m) * 8;
  return true;
}

size_t tsqr_workspace_bytes(long N, int m) {
  TsqrPlan p;
  return tsqr_make_plan(N, m, &p) ? p.bytes : 0;
}

// v + DPP(v) on both 32-bit halves of a double; lanes the control leaves out
// (row_mask) add 0. With every row enabled no lane is left out, so the move
// needs no zeroed destination.
template <int CTRL, int ROWS>
__device__ __forceinline__ double tsqr_dpp_add(double v) {
  const long long b = __double_as_longlong(v);
  int lo, hi;
  if constexpr (ROWS == 0xf) {
    lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffff), CTRL, 0xf, 0xf, false);
    hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
  } else {
    lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, ROWS, 0xf, false);
    hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, false);
  }
  return v + __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the 64 lanes, returned to every lane: pairs, quads, halves and
// rows of 16 by DPP swaps, then rows 1 and 3 take row 0 / 2 (row_bcast:15),
// rows 2 and 3 take rows 0-1 (row_bcast:31); lane 63 then holds the sum.
__device__ __forceinline__ double tsqr_wave_sum(double v) {
  v = tsqr_dpp_add<0xB1, 0xf>(v);     // quad_perm [1,0,3,2]
  v = tsqr_dpp_add<0x4E, 0xf>(v);     // quad_perm [2,3,0,1]
  v = tsqr_dpp_add<0x141, 0xf>(v);    // row_half_mirror
  v = tsqr_dpp_add<0x140, 0xf>(v);    // row_mirror
  v = tsqr_dpp_add<0x142, 0xa>(v);    // row_bcast:15
  v = tsqr_dpp_add<0x143, 0xc>(v);    // row_bcast:31
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// lane `src` (wave-uniform) of a double
__device__ __forceinline__ double tsqr_readlane(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ long tsqr_leaf_row0(const TsqrPlan& p, long b) {
  return b * p.N / p.count[0];
}

// Factors the rows x m block held in x (wave w's q-th register column is
// column w + 16 q; row i = lane + 64 t). Leaves, in LDS, the reflectors in Vl
// (column j: zero above row j, 1 at row j, v below; zero from row `rows` to
// rows_max), R (upper triangle of the m x m column-major Rl) and tau.
template <int CPW>
__device__ void tsqr_factor_node(double (&x)[CPW][kTsqrRegs / CPW], int rows, int m, int ld,
                                 double* Vl, double* Rl, double* taul) {
  constexpr int RPL = kTsqrRegs / CPW;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = 0; j < m; ++j) {
    if (wave == j % kTsqrWaves) {
      const int qj = j / kTsqrWaves;
#pragma unroll
      for (int q = 0; q < CPW; ++q) {
        if (q != qj) continue;
        double ss = 0.0, xj = 0.0;
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          const int i = lane + 64 * t;
          const double v = x[q][t];
          if (i > j && i < rows) ss += v * v;
          if (t == j / 64) xj = v;
        }
        ss = tsqr_wave_sum(ss);
        const double alpha = tsqr_readlane(xj, j % 64);   // row j
        double tj = 0.0, beta = alpha, scale = 0.0;
        if (ss > 0.0) {
          const double nrm = sqrt(alpha * alpha + ss);
          beta = alpha >= 0.0 ? -nrm : nrm;
          // tau = (beta - alpha) / beta, scale = 1 / (alpha - beta), from one
          // reciprocal (the step's critical path)
          const double d = beta - alpha;
          const double r = 1.0 / (beta * d);
          tj = d * d * r;
          scale = -beta * r;
        }
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          const int i = lane + 64 * t;
          if (i >= ld) continue;
          double vi = 0.0;
          if (i > j && i < rows) {
            vi = x[q][t] * scale;
            x[q][t] = vi;
          } else if (i == j) {
            vi = 1.0;
            x[q][t] = beta;
          }
          Vl[i + j * ld] = vi;
        }
        if (lane == 0) {
          taul[j] = tj;
          Rl[j + j * m] = beta;
        }
      }
    }
    __syncthreads();
    const double tj = taul[j];
    const double* v = Vl + j * ld;
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
      const int c = wave + kTsqrWaves * q;
      if (c > j && c < m) {
        if (tj != 0.0) {
          // (v is zero above row j and from row `rows` on: no masks needed)
          double vr[RPL];
#pragma unroll
          for (int t = 0; t < RPL; ++t) vr[t] = lane + 64 * t < ld ? v[lane + 64 * t] : 0.0;
          double d = 0.0;
#pragma unroll
          for (int t = 0; t < RPL; ++t) d += vr[t] * x[q][t];
          const double f = tj * tsqr_wave_sum(d);
#pragma unroll
          for (int t = 0; t < RPL; ++t) x[q][t] -= f * vr[t];
        }
#pragma unroll
        for (int t = 0; t < RPL; ++t)
          if (lane + 64 * t == j) Rl[j + c * m] = x[q][t];
      }
    }
  }
  __syncthreads();
}

// writes the node's reflectors, tau and R (LDS) to its workspace slots
__device__ void tsqr_store_node(const TsqrPlan& p, long id, int rows, const double* Vl,
                                const double* Rl, const double* taul, double* ws) {
  const int m = p.m, ld = p.rows_max;
  double* V = ws + p.off_v + id * ld * (long)m;
  for (long e = threadIdx.x; e < (long)ld * m; e += blockDim.x) {
    const int i = (int)(e % ld);
    if (i < rows) V[e] = Vl[e];
  }
  double* R = ws + p.off_r + id * (long)m * m;
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
    const int a = e % m, b = e / m;
    R[e] = a <= b ? Rl[e] : 0.0;
  }
  for (int e = threadIdx.x; e < m; e += blockDim.x) ws[p.off_tau + id * m + e] = taul[e];
}

// One tree level: level 0 factors the leaves (rows of W), level l > 0 the
// stacks of their children's R factors. The root also writes Rout.
template <typename T, int CPW>
__global__ void __launch_bounds__(kTsqrThreads) tsqr_factor_kernel(const T* __restrict__ W,
                                                                     TsqrPlan p, int level,
                                                                     double* ws, double* Rout) {
  constexpr int RPL = kTsqrRegs / CPW;
  extern __shared__ double lds_t[];
  const int m = p.m, ld = p.rows_max;
  double* Vl = lds_t;                     // ld x m
  double* Rl = Vl + (long)ld * m;         // m x m
  double* taul = Rl + m * m;              // m
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long node = blockIdx.x;
  double x[CPW][RPL];
  int rows;
  if (level == 0) {
    const long r0 = tsqr_leaf_row0(p, node);
    rows = (int)(tsqr_leaf_row0(p, node + 1) - r0);
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
      const int c = wave + kTsqrWaves * q;
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int i = lane + 64 * t;
        x[q][t] = (c < m && i < rows) ? (double)W[r0 + i + (long)c * p.N] : 0.0;
      }
    }
  } else {
    const int nchild = (int)std::min<long>(p.fan, p.count[level - 1] - node * p.fan);
    rows = nchild * m;
    const double* Rc = ws + p.off_r + (p.first[level - 1] + node * p.fan) * (long)m * m;
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
      const int c = wave + kTsqrWaves * q;
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int i = lane + 64 * t;
        const int ch = i / m, r = i - ch * m;
        x[q][t] = (c < m && i < rows && r <= c) ? Rc[(long)ch * m * m + r + (long)c * m] : 0.0;
      }
    }
  }
  tsqr_factor_node<CPW>(x, rows, m, ld, Vl, Rl, taul);
  tsqr_store_node(p, p.first[level] + node, rows, Vl, Rl, taul, ws);
  if (level + 1 == p.levels && Rout) {   // the root: R with a non-negative diagonal
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
      const int r = e % m, c = e / m;
      const double d = Rl[r + r * m] < 0.0 ? -1.0 : 1.0;
      Rout[e] = r <= c ? d * Rl[e] : 0.0;
    }
  }
}

// Q from the root down, one tree level per launch: the workgroup of node
// (level, index) applies the node's reflectors, last to first, to [E; 0] (E:
// the m x m block its parent handed down, I_m at the root; each wave owns
// columns, registers hold the rows; reflectors read-only in LDS, so no barrier
// between them). Below the root it hands each child its m rows; at the leaves
// it writes its rows of Q, column j times the sign of the root's R_jj.
template <typename T, int CPW>
__global__ void __launch_bounds__(kTsqrThreads) tsqr_q_kernel(T* __restrict__ W, TsqrPlan p,
                                                                int level, double* ws) {
  constexpr int RPL = kTsqrRegs / CPW;
  extern __shared__ double lds_t[];
  const int m = p.m, ld = p.rows_max;
  double* Vl = lds_t;                     // ld x m
  double* taul = Vl + (long)ld * m;       // m
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long node = blockIdx.x;
  const long id = p.first[level] + node;
  const int rows = level == 0 ? (int)(tsqr_leaf_row0(p, node + 1) - tsqr_leaf_row0(p, node))
                              : (int)std::min<long>(p.fan, p.count[level - 1] - node * p.fan) * m;
  const double* V = ws + p.off_v + id * ld * (long)m;
  for (long e = threadIdx.x; e < (long)ld * m; e += blockDim.x) {
    const int i = (int)(e % ld), j = (int)(e / ld);
    Vl[e] = i == j ? 1.0 : (i > j && i < rows ? V[e] : 0.0);
  }
  for (int e = threadIdx.x; e < m; e += blockDim.x) taul[e] = ws[p.off_tau + id * m + e];
  const bool root = level + 1 == p.levels;
  const double* E = ws + p.off_e + id * (long)m * m;
  double x[CPW][RPL];
#pragma unroll
  for (int q = 0; q < CPW; ++q) {
    const int c = wave + kTsqrWaves * q;
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int i = lane + 64 * t;
      x[q][t] = (c < m && i < m) ? (root ? (i == c ? 1.0 : 0.0) : E[i + c * m]) : 0.0;
    }
  }
  __syncthreads();
  for (int j = m - 1; j >= 0; --j) {
    const double tj = taul[j];
    if (tj == 0.0) continue;
    // (v is zero above row j and from row `rows` on, as is x: no masks needed)
    const double* v = Vl + (long)j * ld;
    double vr[RPL];
#pragma unroll
    for (int t = 0; t < RPL; ++t) vr[t] = lane + 64 * t < ld ? v[lane + 64 * t] : 0.0;
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
      if (wave + kTsqrWaves * q < m) {
        double d = 0.0;
#pragma unroll
        for (int t = 0; t < RPL; ++t) d += vr[t] * x[q][t];
        const double f = tj * tsqr_wave_sum(d);
#pragma unroll
        for (int t = 0; t < RPL; ++t) x[q][t] -= f * vr[t];
      }
    }
  }
  if (level > 0) {
    // rows ch * m .. ch * m + m - 1 go to child ch (node * fan + ch)
    double* Ec = ws + p.off_e + (p.first[level - 1] + node * p.fan) * (long)m * m;
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
      const int c = wave + kTsqrWaves * q;
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int i = lane + 64 * t;
        if (c < m && i < rows) {
          const int ch = i / m, r = i - ch * m;
          Ec[(long)ch * m * m + r + (long)c * m] = x[q][t];
        }
      }
    }
  } else {
    const double* Rr = ws + p.off_r + p.first[p.levels - 1] * (long)m * m;
    const long r0 = tsqr_leaf_row0(p, node);
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
      const int c = wave + kTsqrWaves * q;
      if (c < m) {
        const double sg = Rr[c + (long)c * m] < 0.0 ? -1.0 : 1.0;
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          const int i = lane + 64 * t;
          if (i < rows) W[r0 + i + (long)c * p.N] = (T)(x[q][t] * sg);
        }
      }
    }
  }
}

template <typename T, int CPW>
static void tsqr_launch_cpw(const TsqrPlan& p, T* W, double* Rfac, double* ws, hipStream_t s) {
  const size_t lds = tsqr_lds_bytes(p.rows_max, p.m);
  (void)hipFuncSetAttribute((const void*)tsqr_factor_kernel<T, CPW>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  (void)hipFuncSetAttribute((const void*)tsqr_q_kernel<T, CPW>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  for (int l = 0; l < p.levels; ++l)
    hipLaunchKernelGGL((tsqr_factor_kernel<T, CPW>), dim3(p.count[l]), dim3(kTsqrThreads), lds, s,
                       W, p, l, ws, Rfac);
  for (int l = p.levels - 1; l >= 0; --l)
    hipLaunchKernelGGL((tsqr_q_kernel<T, CPW>), dim3(p.count[l]), dim3(kTsqrThreads), lds, s, W,
                       p, l, ws);
}

template <typename T>
bool launch_tsqr(T* W, long N, int m, double* Rfac, void* ws, hipStream_t s) {
  TsqrPlan p;
  if (!tsqr_make_plan(N, m, &p)) return false;
  double* w = static_cast<double*>(ws);
  if (p.cpw == 1) tsqr_launch_cpw<T, 1>(p, W, Rfac, w, s);
  else if (p.cpw == 2) tsqr_launch_cpw<T, 2>(p, W, Rfac, w, s);
  else tsqr_launch_cpw<T, 4>(p, W, Rfac, w, s);
  return true;
}

template bool launch_tsqr<float>(float*, long, int, double*, void*, hipStream_t);
template bool launch_tsqr<double>(double*, long, int, double*, void*, hipStream_t);

}  // namespace kpsb
