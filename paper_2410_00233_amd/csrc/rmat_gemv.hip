// Generated-tile matrix-vector product y = R x - coef * z for the single-vector
// recurrences of Algorithm 1 (EGKB): s_j = B q_{j-1} - alpha_{j-1} s_{j-1} and
// q_j = B^T s_j - t_j q_{j-1}. Each generated entry of R is used once, so this
// is bound by the rate at which the tile is read from LDS, not by MFMA.
//
// Layout as in the block product: a workgroup owns 16 rows i in each of TJ row
// blocks j; the 16 + TJ - 1 grid rows they touch sit in LDS. x streams through
// LDS in chunks of kTKV entries (fixed c), double buffered. With 256 threads and
// 16*TJ rows, H = 256 / (16*TJ) threads share a row and split its K range.
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

// FP32 kernel. For every column block c the staged x covers
// r in [r0_c, r0_c + LEN) with r0_c = -((n - 1 - c) mod 4), so the first slab
// column it meets, r0_c - c + n - 1, is a multiple of 4: both the slab row and
// the staged x are then read as aligned float4 (0.5 LDS reads per FMA). Entries
// with r outside [0, n) are staged as 0. Products of one c (LEN terms) are summed
// in FP32 and added into an FP64 accumulator.
template <int TJ, int NT>
__global__ void __launch_bounds__(NT)
rmat_gemv4_kernel(const float* __restrict__ G, int ldg, int n, const float* __restrict__ x,
                  float* __restrict__ y, const float* __restrict__ z, double coef, int SW,
                  int LEN) {
  constexpr int SR = 16 + TJ - 1;
  constexpr int ROWS = 16 * TJ;
  constexpr int H = NT / ROWS;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  float* slab = reinterpret_cast<float*>(lds_raw);
  float* xbuf = slab + SR * SW;                // 2 x LEN
  double* red = reinterpret_cast<double*>(xbuf + 2 * LEN);   // NT (H > 1)

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
    const float* src = G + (long)(rowok ? a : 0) * ldg;
    for (int col = tid; col < SW; col += NT) {
      float v = 0.f;
      if (rowok && col < g2) v = src[col];
      slab[al * SW + col] = v;
    }
  }

  const int rr = tid % ROWS;
  const int h = tid / ROWS;
  const int li = rr & 15;
  const int jg = rr >> 4;
  const float* arow = slab + (li + (TJ - 1) - jg) * SW;
  const int nv = LEN >> 2;                 // float4 per column block
  constexpr int MAXL = (2048 + NT - 1) / NT;   // staged x entries per thread (LEN <= 2048)
  float st[MAXL];
  auto load = [&](int c) {
    const int r0 = -((n - 1 - c) & 3);
#pragma unroll
    for (int m = 0; m < MAXL; ++m) {
      const int kk = tid + NT * m;
      const int r = r0 + kk;
      st[m] = (kk < LEN && r >= 0 && r < n) ? x[(long)n * c + r] : 0.f;
    }
  };
  auto store = [&](int buf) {
    float* xs = xbuf + buf * LEN;
#pragma unroll
    for (int m = 0; m < MAXL; ++m) {
      const int kk = tid + NT * m;
      if (kk < LEN) xs[kk] = st[m];
    }
  };
  load(0);
  store(0);
  __syncthreads();

  double acc = 0.0;
  for (int c = 0; c < n; ++c) {
    if (c + 1 < n) load(c + 1);
    const int base = -((n - 1 - c) & 3) - c + n - 1;      // multiple of 4
    const float4* ap = reinterpret_cast<const float4*>(arow + base);
    const float4* xs = reinterpret_cast<const float4*>(xbuf + (c & 1) * LEN);
    float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
#pragma unroll 4
    for (int v = h; v < nv; v += H) {
      const float4 a = ap[v];
      const float4 b = xs[v];
      p0 = fmaf(a.x, b.x, p0);
      p1 = fmaf(a.y, b.y, p1);
      p2 = fmaf(a.z, b.z, p2);
      p3 = fmaf(a.w, b.w, p3);
    }
    acc += (double)((p0 + p1) + (p2 + p3));
    if (c + 1 < n) store((c + 1) & 1);
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
      y[row] = (float)v;
    }
  }
}

static int gemv4_len(int n) { return ((n + 3 + 3) / 4) * 4; }

template <typename T>
static int gemv_stride(int n) {
  if (sizeof(T) == 4) {
    const int W = n + gemv4_len(n) - 1;           // largest slab column + 1
    return ((W + 63) / 64) * 64 + 4;               // multiple of 4 floats
  }
  const int nrc = (n + kTKV - 1) / kTKV;
  const int W = nrc * kTKV + n - 1;
  return ((W + 31) / 32) * 32 + 1;
}

constexpr int kGemvNT = 1024;   // threads of the FP32 kernel (H = 1024 / (16 TJ) per row)

template <typename T>
static size_t gemv_lds(int n, int TJ) {
  if (sizeof(T) == 4)
    return 4 * ((size_t)(16 + TJ - 1) * gemv_stride<T>(n) + 2 * (size_t)gemv4_len(n)) +
           8 * (size_t)kGemvNT;
  return sizeof(T) * ((size_t)(16 + TJ - 1) * gemv_stride<T>(n) + 2 * (size_t)kTKV);
}

template <typename T>
bool plan_gemv(int n, size_t lds_limit, BlockPlan* plan) {
  static const int cand[] = {16, 8, 4, 2, 1};
  int forced = 0;
  if (const char* e = getenv("KPSB_GEMV_TJ")) forced = atoi(e);
  if (sizeof(T) == 4 && gemv4_len(n) > 2048) return false;   // staged x per thread
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
template bool plan_gemv<float>(int, size_t, BlockPlan*);
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

template <int TJ>
static void gemv4_tj(const BlockPlan& p, const float* G, int ldg, int n, const float* x,
                     float* y, const float* z, double coef, hipStream_t s) {
  auto kern = rmat_gemv4_kernel<TJ, kGemvNT>;
  if (p.lds > 65536)
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)p.lds);
  hipLaunchKernelGGL(kern, dim3(p.grid), dim3(kGemvNT), p.lds, s, G, ldg, n, x, y, z, coef,
                     p.SW, gemv4_len(n));
}

template <>
void gemv_tj<float, 16>(const BlockPlan& p, const float* G, int ldg, int n, const float* x,
                        float* y, const float* z, double coef, hipStream_t s) {
  gemv4_tj<16>(p, G, ldg, n, x, y, z, coef, s);
}
template <>
void gemv_tj<float, 8>(const BlockPlan& p, const float* G, int ldg, int n, const float* x,
                       float* y, const float* z, double coef, hipStream_t s) {
  gemv4_tj<8>(p, G, ldg, n, x, y, z, coef, s);
}
template <>
void gemv_tj<float, 4>(const BlockPlan& p, const float* G, int ldg, int n, const float* x,
                       float* y, const float* z, double coef, hipStream_t s) {
  gemv4_tj<4>(p, G, ldg, n, x, y, z, coef, s);
}
template <>
void gemv_tj<float, 2>(const BlockPlan& p, const float* G, int ldg, int n, const float* x,
                       float* y, const float* z, double coef, hipStream_t s) {
  gemv4_tj<2>(p, G, ldg, n, x, y, z, coef, s);
}
template <>
void gemv_tj<float, 1>(const BlockPlan& p, const float* G, int ldg, int n, const float* x,
                       float* y, const float* z, double coef, hipStream_t s) {
  gemv4_tj<1>(p, G, ldg, n, x, y, z, coef, s);
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
template void launch_rmat_gemv<float>(const BlockPlan&, const float*, int, int, const float*,
                                      float*, const float*, double, hipStream_t);
template void launch_rmat_gemv<double>(const BlockPlan&, const double*, int, int,
                                       const double*, double*, const double*, double,
                                       hipStream_t);

}  // namespace kpsb
