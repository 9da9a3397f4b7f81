// Generated-tile matrix-vector product y = R x - coef * z for the single-vector
// recurrences of Algorithm 1 (EGKB): s_j = B q_{j-1} - alpha_{j-1} s_{j-1} and
// q_j = B^T s_j - t_j q_{j-1}. Each generated entry of R is used once (one FMA
// per entry, no MFMA shape), so the kernels are bound by operand delivery and
// the vector FMA rate.
//
// FP64 kernel (the plain double-precision path): as in the block product, a
// workgroup owns 16 rows i in each of TJ row blocks j; the 16 + TJ - 1 grid
// rows they touch sit in LDS. x streams through LDS in chunks of kTKV entries
// (fixed c), double buffered. With 256 threads and 16*TJ rows,
// H = 256 / (16*TJ) threads share a row and split its K range.
// FP32 kernel: x in scalar registers, see rmat_gemv_sx_kernel below.
#include "common.h"

namespace kpsb {

constexpr int kTKV = 256;   // x entries staged per chunk (FP64 kernel)

// FP64 kernel: x chunks of kTKV entries, scalar LDS reads.
template <typename T, int TJ>
__global__ void __launch_bounds__(256)
rmat_gemv_kernel(const T* __restrict__ G, int ldg, int n, const T* __restrict__ x,
                 T* __restrict__ y, const T* __restrict__ z, double coef, int SW) {
  constexpr int SR = 16 + TJ - 1;
  constexpr int ROWS = 16 * TJ;
  constexpr int H = 256 / ROWS;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* slab = reinterpret_cast<T*>(lds_raw);
  T* xbuf = slab + SR * SW;                    // 2 x kTKV
  __shared__ double red[256];

  const int tid = threadIdx.x;
  const int n_it = (n + 15) >> 4;
  const int it = blockIdx.x % n_it;
  const int jt = blockIdx.x / n_it;
  const int i0 = it * 16;
  const int j0 = jt * TJ;
  const int g2 = 2 * n - 1;
  const int a0 = i0 - j0 - (TJ - 1) + n - 1;

  for (int al = 0; al < SR; ++al) {
    const int a = a0 + al;
    const bool rowok = (a >= 0) && (a < g2);
    const T* src = G + (long)(rowok ? a : 0) * ldg;
    for (int col = tid; col < SW; col += 256) {
      T v = (T)0;
      if (rowok && col < g2) v = src[col];
      slab[al * SW + col] = v;
    }
  }

  const int rr = tid % ROWS;          // row within the workgroup tile
  const int h = tid / ROWS;           // K split index
  const int li = rr & 15;
  const int jg = rr >> 4;
  const T* arow = slab + (li + (TJ - 1) - jg) * SW;

  const int nrc = (n + kTKV - 1) / kTKV;
  const int total = n * nrc;
  auto load = [&](int t) -> T {
    const int c = t / nrc;
    const int r = (t - c * nrc) * kTKV + tid;
    return (r < n) ? x[(long)n * c + r] : (T)0;
  };
  T st = load(0);
  xbuf[tid] = st;
  __syncthreads();

  double acc = 0.0;
  for (int t = 0; t < total; ++t) {
    if (t + 1 < total) st = load(t + 1);
    const int c = t / nrc;
    const int r0 = (t - c * nrc) * kTKV;
    const T* xs = xbuf + (t & 1) * kTKV;
    const T* ap = arow + (r0 - c + n - 1);
    const int kend = min(kTKV, n - r0);
    T part = (T)0;
#pragma unroll 8
    for (int k = h; k < kend; k += H) part += ap[k] * xs[k];
    acc += (double)part;
    if (t + 1 < total) xbuf[((t + 1) & 1) * kTKV + tid] = st;
    __syncthreads();
  }

  if (H > 1) {
    red[tid] = acc;
    __syncthreads();
    if (h == 0) {
      for (int q = 1; q < H; ++q) acc += red[tid + q * ROWS];
    }
  }
  if (h == 0) {
    const int i = i0 + li;
    const int j = j0 + jg;
    if (i < n && j < n) {
      const long row = i + (long)n * j;
      double v = acc;
      if (z) v -= coef * (double)z[row];
      y[row] = (T)v;
    }
  }
}

// ---------------------------------------------------------------------------
// FP32 matrix-vector product with x in scalar registers.
//
// All 64 lanes of a wave walk the same sequence of (r, c), so the x entries
// are the same for the whole wave and are read with scalar loads; each FMA
// takes x from an SGPR. A lane owns kSxP rows (i, j) of R and reuses every x
// entry for all of them. Row (i, j) of R is G[a][r - c + n - 1] with
// a = i - j + n - 1: for a chunk of kSxR consecutive r and c stepping down
// from n - 1, the needed grid entries slide up by one per step, so each row
// keeps a register window of its grid row, refilled with 4 entries per 4 steps
// (a ring of four 4-entry slots). The grid is read in transposed storage, one
// column per load: the 64 lanes of a wave need 19 consecutive rows a of the
// same column, one or two cache lines, where 16-byte loads along the rows would
// touch 19 lines per load (measured: the row-wise window loads halve the FMA
// rate; column-wise ones cost about a fifth). Every entry of R is still formed
// and multiplied (2 n^4 flops per product).
//
// x is first re-laid out (launch_gemv_xt) as xt[ch][u][q] = x[r + n c] with
// r = kSxR ch + q, c = n - 1 - u, zero for r >= n or u >= n, U = steps per
// chunk rounded up to 16; those zero steps and rows meet zero grid padding
// (a grid row carries at least 48 zero columns), so they add exact zeros.
// Workgroup: 16 i x 16 j rows; lane l owns i = i0 + l % 16 and
// j = j0 + l / 16 + 4 p (p < kSxP); its 4 waves take every 4th chunk of the same
// rows and their FP64 sums are added in a fixed order. Products of 8 steps are
// summed in FP32 per row and flushed into FP64.
constexpr int kSxR = 8;   // r entries per chunk

__global__ void gemv_xt_kernel(const float* __restrict__ x, int n, int U, int nch,
                               float* __restrict__ xt) {
  const long total = (long)nch * U * kSxR;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int q = (int)(e % kSxR);
    const long t = e / kSxR;
    const int u = (int)(t % U);
    const int ch = (int)(t / U);
    const int r = ch * kSxR + q;
    float v = 0.f;
    if (r < n && u < n) v = x[r + (long)n * (n - 1 - u)];
    xt[e] = v;
  }
}

// kSxP rows per lane; kSxV waves own different rows (4 kSxP j values each) and
// walk the same chunks at the same time (their x reads share the scalar cache);
// kSxW waves per row set split the chunks (r-parts).
//
// CMP (with box = the support box of G, see launch_grid_box): a workgroup
// whose grid rows all lie outside the box skips every chunk, and a chunk
// visits only the aligned runs of 4 step groups whose grid columns
// [r0 + 4g, r0 + 4g + 10] meet the box. The skipped products are exact zeros
// and the FP32 partial sums keep their 8-step pairing, so the result equals
// the dense one (finite x, up to the sign of zero).
//
// The x values of group g + 1 are requested right after the first product of
// group g: that product's wait covers every scalar load in flight (they may
// return out of order), so the next group's loads are issued only then and
// their latency hides behind the other 31 products of group g. Left to itself
// the compiler issues a run of groups' loads together and waits for all of
// them before the first group (same products, same order, same bits; 1.8 %
// slower dense and 35-40 % slower with a support box, where chunks are short).
template <int kSxP, int kSxV, int kSxW, bool CMP>
__global__ void __launch_bounds__(64 * kSxV * kSxW)
rmat_gemv_sx_kernel(const float* __restrict__ GT, int ldg, int n, const float* __restrict__ xt,
                    int U, float* __restrict__ y, const float* __restrict__ z, double coef,
                    const int* __restrict__ box) {
  __shared__ double red[kSxW][kSxV][kSxP][64];
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wave = wid / kSxV;          // r-part
  const int rw = wid % kSxV;            // row set
  const int n_it = (n + 15) >> 4;
  const int it = blockIdx.x % n_it, jt = blockIdx.x / n_it;
  const int i = it * 16 + (lane & 15);
  const int jb = (jt * kSxV + rw) * 4 * kSxP + (lane >> 4);
  // lane's grid row a = i - j + n - 1, read along its columns b in the
  // transposed storage (GT[b ldg + a]): the lanes of a wave read the 19
  // consecutive entries a of one column per load instead of 19 rows
  // Buffer loads over the ldg x ldg grid: the lane's row is a fixed byte offset,
  // the column a uniform (scalar) offset, so no per-load address arithmetic.
  // (lane offsets: the row, plus 0..3 columns; one scalar offset per slot)
  const int colb = 4 * ldg;   // bytes per grid column in the transposed storage
  int aoff[kSxP][4];
#pragma unroll
  for (int p = 0; p < kSxP; ++p) {
    const int j = jb + 4 * p;
    const bool ok = i < n && j < n;
#pragma unroll
    for (int k = 0; k < 4; ++k) aoff[p][k] = 4 * (ok ? i - j + n - 1 : 0) + k * colb;
  }
  const __amdgpu_buffer_rsrc_t grs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(GT), 0, (int)(4L * ldg * ldg), 0x00020000);
  auto ld1 = [&](int p, int k, int soff) {
    return __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(grs, aoff[p][k], soff, 0));
  };
  auto slot = [&](int p, int b) {   // entries b .. b + 3 of the lane's grid row
    const int s0 = b * colb;
    return make_float4(ld1(p, 0, s0), ld1(p, 1, s0), ld1(p, 2, s0), ld1(p, 3, s0));
  };
  const int nch = (n + kSxR - 1) / kSxR;
  const int ngrp = U / 4;                 // groups of 4 steps (multiple of 4)
  int bl = 0, bh = 0;
  bool active = true;
  if (CMP) {
    // grid rows of the workgroup: i in [16 it, 16 it + 15], j in [jw, jw + 4 kSxP kSxV - 1]
    const int jw = jt * kSxV * 4 * kSxP;
    const int amin = 16 * it - (jw + 4 * kSxP * kSxV - 1) + n - 1;
    const int amax = 16 * it + 15 - jw + n - 1;
    bl = box[2];
    bh = box[3];
    active = box[0] <= box[1] && bl <= bh && amin <= box[1] && amax >= box[0];
  }
  double acc[kSxP];
#pragma unroll
  for (int p = 0; p < kSxP; ++p) acc[p] = 0.0;
  for (int ch = wave; active && ch < nch; ch += kSxW) {
    const int r0 = ch * kSxR;
    int gbeg = 0, gend = ngrp;            // runs of 4 groups [gbeg, gend)
    if (CMP) {
      const int lo = bl - r0 - 10;          // 4 g >= lo  and  4 g <= bh - r0
      const int glo = lo <= 0 ? 0 : (lo + 3) / 4;
      const int ghi = bh - r0 < 0 ? -1 : (bh - r0) / 4;
      gbeg = (glo / 4) * 4;
      gend = min(ngrp, (ghi / 4) * 4 + 4);
      if (ghi < 0 || glo >= ngrp || gbeg >= gend) continue;
    }
    const float* xp = xt + (long)ch * U * kSxR;
    float pp[kSxP];
    {
      float4 S[kSxP][4];
#pragma unroll
      for (int p = 0; p < kSxP; ++p)
#pragma unroll
        for (int t = 0; t < 3; ++t)
          S[p][t] = slot(p, r0 + 4 * (gbeg + t));
      float xa[4 * kSxR], xb[4 * kSxR];
      auto ldx = [&](float (&d)[4 * kSxR], int g) {
        const float* src = xp + (long)g * 4 * kSxR;
#pragma unroll
        for (int e = 0; e < 4 * kSxR; ++e) d[e] = src[e];
      };
      ldx(xa, gbeg);
      for (int g0 = gbeg; g0 < gend; g0 += 4) {
#pragma unroll
        for (int gg = 0; gg < 4; ++gg) {
          const int g = g0 + gg;
          float(&xc)[4 * kSxR] = (gg & 1) ? xb : xa;
          float(&xn)[4 * kSxR] = (gg & 1) ? xa : xb;
#pragma unroll
          for (int p = 0; p < kSxP; ++p)
            S[p][(gg + 3) & 3] = slot(p, r0 + 4 * (g + 3));
          if ((gg & 1) == 0) {
#pragma unroll
            for (int p = 0; p < kSxP; ++p) pp[p] = 0.f;
          }
#pragma unroll
          for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int q = 0; q < kSxR; ++q) {
              const float xv = xc[v * kSxR + q];
              const int w = v + q;
              const int sl = (gg + (w >> 2)) & 3;
#pragma unroll
              for (int p = 0; p < kSxP; ++p) {
                const float4 sv = S[p][sl];
                const float gv = (w & 3) == 0 ? sv.x : (w & 3) == 1 ? sv.y : (w & 3) == 2 ? sv.z : sv.w;
                pp[p] = fmaf(gv, xv, pp[p]);
              }
              if (v == 0 && q == 0) {   // x of the next group (the last one reloads its own)
                __builtin_amdgcn_sched_barrier(0);
                ldx(xn, g + 1 < gend ? g + 1 : g);
                __builtin_amdgcn_sched_barrier(0);
              }
            }
          if (gg & 1) {
#pragma unroll
            for (int p = 0; p < kSxP; ++p) acc[p] += (double)pp[p];
          }
        }
      }
    }
  }
#pragma unroll
  for (int p = 0; p < kSxP; ++p) red[wave][rw][p][lane] = acc[p];
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int p = 0; p < kSxP; ++p) {
      const int j = jb + 4 * p;
      if (i < n && j < n) {
        double v = red[0][rw][p][lane];
#pragma unroll
        for (int w = 1; w < kSxW; ++w) v += red[w][rw][p][lane];
        const long row = i + (long)n * j;
        if (z) v -= coef * (double)z[row];
        y[row] = (float)v;
      }
    }
  }
}

int gemv_sx_steps(int n) { return ((n + 15) / 16) * 16; }
long gemv_sx_xt_len(int n) { return (long)((n + kSxR - 1) / kSxR) * gemv_sx_steps(n) * kSxR; }

void launch_rmat_gemv_sx(const float* G, int ldg, int n, const float* x, float* xt, float* y,
                         const float* z, double coef, hipStream_t s, const int* box) {
  const int U = gemv_sx_steps(n);
  const int nch = (n + kSxR - 1) / kSxR;
  const long tot = gemv_sx_xt_len(n);
  long blocks = (tot + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(gemv_xt_kernel, dim3((int)blocks), dim3(256), 0, s, x, n, U, nch, xt);
  // one row per lane, 8 waves splitting the chunks: the fastest of the shapes
  // measured (rows per lane 1-8, row-sharing waves 1-8, r-parts 1-16)
  constexpr int P = 1, V = 1, W = 8;
  const int grid = ((n + 15) / 16) * ((n + 4 * P * V - 1) / (4 * P * V));
  if (box)
    hipLaunchKernelGGL((rmat_gemv_sx_kernel<P, V, W, true>), dim3(grid), dim3(64 * V * W), 0, s,
                       G, ldg, n, xt, U, y, z, coef, box);
  else
    hipLaunchKernelGGL((rmat_gemv_sx_kernel<P, V, W, false>), dim3(grid), dim3(64 * V * W), 0, s,
                       G, ldg, n, xt, U, y, z, coef, box);
}

template <typename T>
static int gemv_stride(int n) {
  const int nrc = (n + kTKV - 1) / kTKV;
  const int W = nrc * kTKV + n - 1;
  return ((W + 31) / 32) * 32 + 1;
}

template <typename T>
static size_t gemv_lds(int n, int TJ) {
  return sizeof(T) * ((size_t)(16 + TJ - 1) * gemv_stride<T>(n) + 2 * (size_t)kTKV);
}

template <typename T>
bool plan_gemv(int n, size_t lds_limit, BlockPlan* plan) {
  static const int cand[] = {16, 8, 4, 2, 1};
  int forced = 0;
  if (const char* e = getenv("KPSB_GEMV_TJ")) forced = atoi(e);
  // the FP64 kernel's static reduction buffer (2 KB) shares the LDS budget
  size_t limit = lds_limit > 4096 ? lds_limit - 4096 : 0;
  for (int TJ : cand) {
    if (forced && TJ != forced) continue;
    size_t lds = gemv_lds<T>(n, TJ);
    if (lds <= limit) {
      plan->TJ = TJ;
      plan->SW = gemv_stride<T>(n);
      plan->lds = lds;
      plan->grid = ((n + 15) / 16) * ((n + TJ - 1) / TJ);
      return true;
    }
  }
  return false;
}
template bool plan_gemv<double>(int, size_t, BlockPlan*);

template <typename T, int TJ>
static void gemv_tj(const BlockPlan& p, const T* G, int ldg, int n, const T* x, T* y,
                    const T* z, double coef, hipStream_t s) {
  auto kern = rmat_gemv_kernel<T, TJ>;
  if (p.lds > 65536)
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)p.lds);
  hipLaunchKernelGGL(kern, dim3(p.grid), dim3(256), p.lds, s, G, ldg, n, x, y, z, coef, p.SW);
}

template <typename T>
void launch_rmat_gemv(const BlockPlan& p, const T* G, int ldg, int n, const T* x, T* y,
                      const T* z, double coef, hipStream_t s) {
  switch (p.TJ) {
    case 16: gemv_tj<T, 16>(p, G, ldg, n, x, y, z, coef, s); break;
    case 8: gemv_tj<T, 8>(p, G, ldg, n, x, y, z, coef, s); break;
    case 4: gemv_tj<T, 4>(p, G, ldg, n, x, y, z, coef, s); break;
    case 2: gemv_tj<T, 2>(p, G, ldg, n, x, y, z, coef, s); break;
    default: gemv_tj<T, 1>(p, G, ldg, n, x, y, z, coef, s); break;
  }
}
template void launch_rmat_gemv<double>(const BlockPlan&, const double*, int, int,
                                       const double*, double*, const double*, double,
                                       hipStream_t);

}  // namespace kpsb
