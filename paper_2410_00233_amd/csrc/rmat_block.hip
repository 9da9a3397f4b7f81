// Generated-tile block product Y = R X with R = R(A) the rearranged blur
// (paper section 2.1; the dominant cost of Algorithms 1 and 2 per section 4.1).
//
// R is never stored. A workgroup owns 16 consecutive rows i in each of TJ
// consecutive row blocks j (R row i + n*j). Every entry of those rows is
// R[i + n*j, r + n*c] = G[i - j + n - 1][r - c + n - 1] (G = offset grid of the
// PSF), so the 16 + TJ - 1 grid rows they touch are copied once into LDS (the
// "slab") and every MFMA A-fragment is generated from the slab. The product is
// the full dense contraction over all n^2 columns of R: nothing is skipped or
// merged, whatever the PSF.
//
// X streams through LDS in K-tiles of TK entries (fixed c, r0 <= r < r0 + TK),
// double buffered, one barrier per tile. In FP32 the MFMA accumulators are
// added into FP64 registers after every column block c (n products), so the
// rounding error of the length-n^2 sums grows like sqrt(n), not sqrt(n^2). MFMA: v_mfma_f32_16x16x4f32 (FP32) or
// v_mfma_f64_16x16x4f64 (FP64). Fragment layout (checked on gfx950): A lane l
// holds row l%16, k = l/16; B lane l holds k = l/16, column l%16; D lane l
// holds column l%16 and, for item e = 0..3, row 4*(l/16) + e (FP32) or
// row l/16 + 4*e (FP64).
#include <algorithm>
#include <climits>

#include <type_traits>

#include "common.h"

namespace kpsb {

// ---------------------------------------------------------------------------
// Offset grid of one term: G[a][b] = sum over s1 in sh.sv, s2 in sh.su of
// P[cu + (b - (n-1)) + s2, cv + (a - (n-1)) + s1] (0 outside P), summed in FP64
// in the order of the shift lists and then rounded to T. The transposed grid
// swaps a and b. Zero boundary conditions: one shift 0 in each dimension.
__device__ __forceinline__ double grid_value(const double* __restrict__ psf, int pu, int pv,
                                             int cu, int cv, int n, int a, int b,
                                             const GridShifts& sh) {
  double v = 0.0;
  for (int x = 0; x < sh.nv; ++x) {
    const int w = cv + a - (n - 1) + sh.sv[x];
    if (w < 0 || w >= pv) continue;
    for (int y = 0; y < sh.nu; ++y) {
      const int u = cu + b - (n - 1) + sh.su[y];
      if (u >= 0 && u < pu) v += psf[(long)u * pv + w];
    }
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T from_double(double v) { return (T)v; }
template <>
__device__ __forceinline__ __hip_bfloat16 from_double<__hip_bfloat16>(double v) {
  return __float2bfloat16((float)v);
}
template <>
__device__ __forceinline__ __half from_double<__half>(double v) { return __float2half((float)v); }

template <typename T>
__global__ void build_grid_kernel(const double* __restrict__ psf, int pu, int pv, int cu,
                                  int cv, int n, int transpose, GridShifts sh,
                                  T* __restrict__ G, int ldg) {
  const int g2 = 2 * n - 1;
  const long total = (long)ldg * ldg;   // ldg x ldg: zero rows and columns beyond 2n - 1
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int a = (int)(e / ldg);
    const int b = (int)(e - (long)a * ldg);
    double v = 0.0;
    if (a < g2 && b < g2) v = transpose ? grid_value(psf, pu, pv, cu, cv, n, b, a, sh)
                                        : grid_value(psf, pu, pv, cu, cv, n, a, b, sh);
    G[e] = from_double<T>(v);
  }
}

// Two stages: kScaleParts workgroups write partial max|P| and sum|P| into
// scal[2 ..], one workgroup adds them in a fixed order (tree over the parts).
constexpr int kScaleParts = 256;

__device__ __forceinline__ void block_max_sum(double* sm, double* ss) {
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
      ss[threadIdx.x] += ss[threadIdx.x + w];
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256)
psf_scale_partial_kernel(const double* __restrict__ psf, long count, double* __restrict__ part) {
  __shared__ double sm[256];
  __shared__ double ss[256];
  double m = 0.0, t = 0.0;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < count; e += 256L * kScaleParts) {
    const double v = fabs(psf[e]);
    m = fmax(m, v);
    t += v;
  }
  sm[threadIdx.x] = m;
  ss[threadIdx.x] = t;
  __syncthreads();
  block_max_sum(sm, ss);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = sm[0];
    part[kScaleParts + blockIdx.x] = ss[0];
  }
}

__global__ void __launch_bounds__(256)
psf_scale_final_kernel(int nsum, double* __restrict__ scal) {
  __shared__ double sm[256];
  __shared__ double ss[256];
  const double* part = scal + 2;
  sm[threadIdx.x] = part[threadIdx.x];                 // kScaleParts == 256
  ss[threadIdx.x] = part[kScaleParts + threadIdx.x];
  __syncthreads();
  block_max_sum(sm, ss);
  if (threadIdx.x == 0) {
    double sc = 1.0;
    // a grid entry is a sum of at most nsum distinct PSF entries, so
    // min(nsum max|P|, sum|P|) bounds it (max|P| itself when nsum = 1)
    const double mx = nsum <= 1 ? sm[0] : fmin(nsum * sm[0], ss[0]);
    if (mx > 0.0) {
      int ex = 0;
      (void)frexp(1024.0 / mx, &ex);      // 1024 / mx = f 2^ex, f in [0.5, 1)
      sc = ldexp(1.0, ex - 1);            // largest 2^e <= 1024 / mx
    }
    scal[0] = sc;
    scal[1] = 1.0 / (sc * (double)(1 << kSplitXExp));
  }
}

int psf_split_scale_len() { return 2 + 2 * kScaleParts; }

void launch_psf_split_scale(const double* psf, long count, int nsum, double* scal,
                            hipStream_t s) {
  hipLaunchKernelGGL(psf_scale_partial_kernel, dim3(kScaleParts), dim3(256), 0, s, psf, count,
                     scal + 2);
  hipLaunchKernelGGL(psf_scale_final_kernel, dim3(1), dim3(256), 0, s, nsum, scal);
}

__device__ __forceinline__ __half d2h(double v) { return __half_raw{static_cast<_Float16>(v)}; }

__global__ void build_grid_split_kernel(const double* __restrict__ psf, int pu, int pv, int cu,
                                        int cv, int n, int transpose, GridShifts sh,
                                        const double* __restrict__ scal, int part,
                                        __half* __restrict__ G, int ldg) {
  const int g2 = 2 * n - 1;
  const long total = (long)g2 * ldg;
  const double sc = scal[0];
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int a = (int)(e / ldg);
    const int b = (int)(e - (long)a * ldg);
    double v = 0.0;
    if (b < g2) v = sc * (transpose ? grid_value(psf, pu, pv, cu, cv, n, b, a, sh)
                                    : grid_value(psf, pu, pv, cu, cv, n, a, b, sh));
    const __half h = d2h(v);
    G[e] = part == 0 ? h : d2h(v - (double)__half2float(h));
  }
}

void launch_build_grid_split(const double* psf, int pu, int pv, int cu, int cv, int n,
                             int transpose, const GridShifts& sh, const double* scal, int part,
                             __half* G, int ldg, hipStream_t s) {
  long total = (long)(2 * n - 1) * ldg;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(build_grid_split_kernel, dim3(blocks), dim3(256), 0, s, psf, pu, pv, cu,
                     cv, n, transpose, sh, scal, part, G, ldg);
}

template <typename T>
void launch_build_grid(const double* psf, int pu, int pv, int cu, int cv, int n,
                       int transpose, const GridShifts& sh, T* G, int ldg, hipStream_t s) {
  long total = (long)ldg * ldg;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(build_grid_kernel<T>, dim3(blocks), dim3(256), 0, s, psf, pu, pv, cu,
                     cv, n, transpose, sh, G, ldg);
}

// ---------------------------------------------------------------------------
// Terms of the reflexive operator: out[a + n b + ld col] = in[a + n (n-1-b) + ld col]
// (reversal of the block index b of every column).
template <typename T>
__global__ void flip_blocks_kernel(const T* __restrict__ in, T* __restrict__ out, int n,
                                   long ld, int ncols) {
  const long N = (long)n * n;
  const long total = N * ncols;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const long col = e / N;
    const long q = e - col * N;
    const long b = q / n;
    const long a = q - b * n;
    out[col * ld + q] = in[col * ld + a + (long)n * (n - 1 - b)];
  }
}

// Y = (Y + T1) + (T2 + T3)[flipped]: the four terms of a reflexive product.
template <typename T>
__global__ void combine_terms_kernel(T* __restrict__ Y, const T* __restrict__ T1,
                                     const T* __restrict__ T2, const T* __restrict__ T3, int n,
                                     long ld, int ncols) {
  const long N = (long)n * n;
  const long total = N * ncols;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const long col = e / N;
    const long q = e - col * N;
    const long b = q / n;
    const long a = q - b * n;
    const long f = col * ld + a + (long)n * (n - 1 - b);
    const long o = col * ld + q;
    Y[o] = (Y[o] + T1[o]) + (T2[f] + T3[f]);
  }
}

template <typename T>
void launch_flip_blocks(const T* in, T* out, int n, long ld, int ncols, hipStream_t s) {
  const long total = (long)n * n * ncols;
  int blocks = (int)std::min<long>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(flip_blocks_kernel<T>, dim3(blocks), dim3(256), 0, s, in, out, n, ld, ncols);
}

template <typename T>
void launch_combine_terms(T* Y, const T* T1, const T* T2, const T* T3, int n, long ld, int ncols,
                          hipStream_t s) {
  const long total = (long)n * n * ncols;
  int blocks = (int)std::min<long>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(combine_terms_kernel<T>, dim3(blocks), dim3(256), 0, s, Y, T1, T2, T3, n, ld,
                     ncols);
}
template void launch_flip_blocks<float>(const float*, float*, int, long, int, hipStream_t);
template void launch_flip_blocks<double>(const double*, double*, int, long, int, hipStream_t);
template void launch_combine_terms<float>(float*, const float*, const float*, const float*, int,
                                          long, int, hipStream_t);
template void launch_combine_terms<double>(double*, const double*, const double*, const double*,
                                           int, long, int, hipStream_t);
template void launch_build_grid<float>(const double*, int, int, int, int, int, int,
                                       const GridShifts&, float*, int, hipStream_t);
template void launch_build_grid<double>(const double*, int, int, int, int, int, int,
                                        const GridShifts&, double*, int, hipStream_t);
template void launch_build_grid<__hip_bfloat16>(const double*, int, int, int, int, int, int,
                                                const GridShifts&, __hip_bfloat16*, int,
                                                hipStream_t);
template void launch_build_grid<__half>(const double*, int, int, int, int, int, int,
                                        const GridShifts&, __half*, int, hipStream_t);

// ---------------------------------------------------------------------------
template <typename T> struct Vec4;
template <> struct Vec4<float> {
  typedef floatx4 type;
  static __device__ __forceinline__ int drow(int lk, int e) { return 4 * lk + e; }
};
template <> struct Vec4<double> {
  typedef doublex4 type;
  static __device__ __forceinline__ int drow(int lk, int e) { return lk + 4 * e; }
};

__device__ __forceinline__ floatx4 mfma16x16x4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ doublex4 mfma16x16x4(double a, double b, doublex4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kTK = 64;   // default K-tile (entries of r per staged X tile); 128, 176, 192 also built
constexpr int kKG = 16;   // K entries per group: 4 MFMA steps, 4 consecutive entries per lane

// Row stride (elements) of the transposed X tile in LDS. The 16-byte reads of a
// half-wave (16 row lanes x 2 lane groups 4 words apart) fall on distinct banks
// when the stride is 8 (mod 16) words (measured on gfx950: 128-bit reads are
// served 32 lanes at a time; 4 or 0 (mod 16) costs about 20 % more LDS
// cycles): KT + 8 floats. Doubles (lane groups 8 words apart) keep KT + 2.
template <typename T, int KT>
constexpr int x_stride() { return KT + (sizeof(T) == 4 ? 8 : 2); }

// K order. Column block c's range of r is shifted to start at r0(c) in {0,-1,-2,-3}
// so that every 16-entry group starts at a slab column that is a multiple of 4;
// in a group, lane group lk (= lane / 16) owns the 4 consecutive entries 4 lk .. 4 lk + 3
// and MFMA step u (0..3) multiplies entry 4 lk + u. Each lane then reads its A and
// B operands of a group with 16-byte LDS loads (four MFMA steps' worth), a quarter
// of the read instructions of one element per step. Entries with r outside [0, n)
// are staged as zero X. A tile is GPT = KT / 16 consecutive groups of one column
// block (the last tile of a block may hold fewer; the missing groups are skipped).
//
// box (optional, device): the rows [box[0], box[1]] and columns [box[2], box[3]]
// of G that hold its nonzero entries. With it, a workgroup whose grid rows are
// all outside writes zeros, and column block c visits only the groups whose
// grid columns r - c + n - 1 meet the box; every skipped product is an exact
// zero, so the result equals the dense one (for finite X, up to the sign of
// zero). Without it every entry of R is multiplied.
template <typename T, int TJ, int JB, int CB, bool CMP, int KT>
__device__ __forceinline__ void rmat_block_tile(const T* __restrict__ G, int ldg, int n,
                                                const T* __restrict__ X, long ldx,
                                                T* __restrict__ Y, long ldy, int ncols, int SW,
                                                int CP, const int* __restrict__ box, int bid,
                                                unsigned char* lds_raw) {
  constexpr int WAVES = (2 * TJ) / (JB * CB);
  constexpr int NT = 64 * WAVES;
  constexpr int SR = 16 + TJ - 1;
  constexpr int WC = 2 / CB;                 // waves along the 32 output columns
  constexpr int LPT = (KT * 32 + NT - 1) / NT;   // X elements staged per thread
  constexpr bool LFULL = (KT * 32) % NT == 0;    // else the last round is partial
  constexpr int GPT = KT / kKG;              // groups per tile
  constexpr int XT = x_stride<T, KT>();
  constexpr int VEC = 16 / (int)sizeof(T);   // elements per 16-byte LDS read
  typedef typename Vec4<T>::type acc_t;
  typedef T vec_t __attribute__((ext_vector_type(VEC)));

  T* slab = reinterpret_cast<T*>(lds_raw);
  T* xbuf = slab + SR * SW;                  // two transposed tiles of 32 x XT

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int n_it = (n + 15) >> 4;
  const int it = bid % n_it;
  const int jt = bid / n_it;
  const int i0 = it * 16;
  const int j0 = jt * TJ;
  const int g2 = 2 * n - 1;
  const int a0 = i0 - j0 - (TJ - 1) + n - 1;

  // grid columns that hold nonzeros (all of them without a box), and the
  // column blocks c whose r range [0, n) reaches them
  int bl = 0, bh = g2 - 1;
  bool active = true;
  if (CMP) {
    bl = box[2];
    bh = box[3];
    active = box[0] <= box[1] && bl <= bh && a0 <= box[1] && a0 + SR - 1 >= box[0];
  }
  const int c_lo = max(0, n - 1 - bh);
  const int c_hi = min(n - 1, 2 * n - 2 - bl);
  active = active && c_lo <= c_hi;

  // ---- slab: grid rows a0 .. a0 + SR - 1, zero outside the grid. Column
  // blocks c are processed in phases of CP; slab column s of a phase starting at
  // c0 holds grid column n - c0 - CP - 4 + s (a margin of 4 for r0(c) < 0).
  auto load_slab = [&](int c0) {
    const int cbase = n - c0 - CP - 4;
    for (int al = 0; al < SR; ++al) {
      const int a = a0 + al;
      const bool rowok = (a >= 0) && (a < g2);
      const T* src = G + (long)(rowok ? a : 0) * ldg;
      for (int col = tid; col < SW; col += NT) {
        const int gc = cbase + col;
        T v = (T)0;
        if (rowok && gc >= 0 && gc < g2) v = src[gc];
        slab[al * SW + col] = v;
      }
    }
  };

  // groups of column block c (with start r0) to visit: all those holding r < n,
  // or (with a box) those meeting r in [bl - n + 1 + c, bh - n + 1 + c]
  auto g_lo = [&](int c, int r0) { return CMP ? (max(r0, bl - n + 1 + c) - r0) / kKG : 0; };
  auto g_hi = [&](int c, int r0) {
    return (CMP ? min(n - 1, bh - n + 1 + c) - r0 : n - 1 - r0) / kKG;
  };

  // staged X element e = tid + NT m (e < 32 KT): column e / KT, entry e % KT of
  // the tile (a wave reads consecutive r and writes consecutive LDS words)
  T stage[LPT];
  auto load_tile = [&](int c, int r0, int gb, int gh) {
    const int rbase = r0 + kKG * gb;
    const int rend = r0 + kKG * (gh + 1);    // groups beyond gh are staged as zero
#pragma unroll
    for (int m = 0; m < LPT; ++m) {
      const int e = tid + NT * m;
      const int col = e / KT;
      const int r = rbase + e % KT;
      T v = (T)0;
      if ((LFULL || e < KT * 32) && col < ncols && r >= 0 && r < n && r < rend)
        v = X[(long)col * ldx + (long)n * c + r];
      stage[m] = v;
    }
  };
  auto store_tile = [&](int buf) {
    T* xs = xbuf + buf * (32 * XT);
#pragma unroll
    for (int m = 0; m < LPT; ++m) {
      const int e = tid + NT * m;
      if (LFULL || e < KT * 32) xs[(e / KT) * XT + e % KT] = stage[m];
    }
  };

  acc_t acc[JB][CB];
  double accd[JB][CB][4];
#pragma unroll
  for (int jb = 0; jb < JB; ++jb)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        acc[jb][cb][e] = (T)0;
        accd[jb][cb][e] = 0.0;
      }

  const int wc = wave % WC;
  const int wj = wave / WC;
  const int lrow = lane & 15;
  const int lk = lane >> 4;
  // slab row offset of every A fragment of this wave (independent of the tile)
  int arow[JB];
#pragma unroll
  for (int jb = 0; jb < JB; ++jb) arow[jb] = (lrow + (TJ - 1) - (wj * JB + jb)) * SW;

  // Operands of group g of a staged tile whose first group starts at slab column
  // colbase (a multiple of 4): each lane's 4 consecutive K entries, 16-byte reads.
  // nb (a compile-time count): the column blocks of the wave that hold columns
  // (CB, or 1 when a launch with CB = 2 has at most 16 columns: the second
  // block's operands and MFMAs are skipped, its outputs are not written)
  auto read_group = [&](auto nb, const T* xs, int colbase, int g, T (&a)[JB][4],
                        T (&b)[CB][4]) {
    constexpr int NB = decltype(nb)::value;
#pragma unroll
    for (int h = 0; h < 4 / VEC; ++h) {
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) {
        const vec_t v = *reinterpret_cast<const vec_t*>(
            slab + arow[jb] + colbase + kKG * g + 4 * lk + VEC * h);
#pragma unroll
        for (int u = 0; u < VEC; ++u) a[jb][VEC * h + u] = v[u];
      }
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        const vec_t v = *reinterpret_cast<const vec_t*>(
            xs + ((wc * CB + cb) * 16 + lrow) * XT + kKG * g + 4 * lk + VEC * h);
#pragma unroll
        for (int u = 0; u < VEC; ++u) b[cb][VEC * h + u] = v[u];
      }
    }
  };
  auto mma_group = [&](auto nb, const T (&a)[JB][4], const T (&b)[CB][4]) {
    constexpr int NB = decltype(nb)::value;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int jb = 0; jb < JB; ++jb)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
          acc[jb][cb] = mfma16x16x4(a[jb][u], b[cb][u], acc[jb][cb]);
  };
  // The reads of group g + 1 are issued before the MFMAs of group g: a full
  // tile in straight-line code; the last tile of a column block, which may hold
  // fewer groups, in a loop over pairs of groups with the same overlap.
  auto mma_tile = [&](auto nb, const T* xs, int colbase, int ng) {
    if (ng == GPT) {
      T a0[JB][4], b0[CB][4], a1[JB][4], b1[CB][4];
      read_group(nb, xs, colbase, 0, a0, b0);
#pragma unroll
      for (int g = 0; g < GPT; g += 2) {
        if (g + 1 < GPT) read_group(nb, xs, colbase, g + 1, a1, b1);
        __builtin_amdgcn_sched_barrier(0);
        mma_group(nb, a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        if (g + 1 < GPT) {
          if (g + 2 < GPT) read_group(nb, xs, colbase, g + 2, a0, b0);
          __builtin_amdgcn_sched_barrier(0);
          mma_group(nb, a1, b1);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    } else if (ng > 0) {
      T a0[JB][4], b0[CB][4], a1[JB][4], b1[CB][4];
      read_group(nb, xs, colbase, 0, a0, b0);
#pragma unroll 1
      for (int g = 0; g < ng; g += 2) {
        if (g + 1 < ng) read_group(nb, xs, colbase, g + 1, a1, b1);
        mma_group(nb, a0, b0);
        if (g + 1 < ng) {
          if (g + 2 < ng) read_group(nb, xs, colbase, g + 2, a0, b0);
          mma_group(nb, a1, b1);
        }
      }
    }
  };

  auto main_loop = [&](auto nb) {
  if (active) {   // uniform over the workgroup: every barrier below is reached by all
    // state: column block c, its position cpos in the phase [c0, c0 + CP), its
    // shift r0, the current tile's first group gb and the block's last group gh
    int c = c_lo;
    int cpos = c_lo % CP;
    int c0 = c_lo - cpos;
    int r0 = -((CP + 3 - cpos) & 3);
    int gb = g_lo(c, r0), gh = g_hi(c, r0);
    load_slab(c0);
    load_tile(c, r0, gb, gh);
    store_tile(0);
    __syncthreads();

    for (int q = 0;; ++q) {
      // the next tile: the next groups of c, else the first of c + 1
      int cn = c, cposn = cpos, r0n = r0, gbn = gb + GPT, ghn = gh;
      if (gbn > gh) {
        cn = c + 1;
        cposn = cpos + 1 == CP ? 0 : cpos + 1;
        r0n = -((CP + 3 - cposn) & 3);
        if (cn <= c_hi) {
          gbn = g_lo(cn, r0n);
          ghn = g_hi(cn, r0n);
        }
      }
      const bool more = cn <= c_hi;
      if (more) load_tile(cn, r0n, gbn, ghn);
      // slab column of the tile's first group: r0 + 16 gb - c + c0 + CP - 1 + 4
      mma_tile(nb, xbuf + (q & 1) * (32 * XT), r0 + kKG * gb - cpos + CP + 3,
               min(GPT, gh - gb + 1));
      if (more) store_tile((q + 1) & 1);
      __syncthreads();
      if (cn != c) {
        if (sizeof(T) == 4) {   // end of column block c: fold into the FP64 accumulators
#pragma unroll
          for (int jb = 0; jb < JB; ++jb)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                accd[jb][cb][e] += (double)acc[jb][cb][e];
                acc[jb][cb][e] = (T)0;
              }
        }
        if (!more) break;
        if (cposn == 0) {   // next phase: every wave is past the last tile's barrier
          c0 = cn;
          load_slab(c0);
          __syncthreads();
        }
      }
      c = cn;
      cpos = cposn;
      r0 = r0n;
      gb = gbn;
      gh = ghn;
    }
  }
  };
  if constexpr (CB == 2) {
    if (ncols <= 16) main_loop(std::integral_constant<int, 1>{});
    else main_loop(std::integral_constant<int, 2>{});
  } else {
    main_loop(std::integral_constant<int, CB>{});
  }

  // ---- epilogue -----------------------------------------------------------
#pragma unroll
  for (int jb = 0; jb < JB; ++jb) {
    const int j = j0 + wj * JB + jb;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const int col = (wc * CB + cb) * 16 + lrow;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = i0 + Vec4<T>::drow(lk, e);
        const double v = (sizeof(T) == 4) ? accd[jb][cb][e] : (double)acc[jb][cb][e];
        if (i < n && j < n && col < ncols) Y[(long)col * ldy + i + (long)n * j] = (T)v;
      }
    }
  }
}

// One workgroup per tile (16 rows i x TJ row blocks j of R).
template <typename T, int TJ, int JB, int CB, bool CMP, int KT>
__global__ void __launch_bounds__(64 * (2 * TJ) / (JB * CB))
rmat_block_kernel(const T* __restrict__ G, int ldg, int n, const T* __restrict__ X, long ldx,
                  T* __restrict__ Y, long ldy, int ncols, int SW, int CP,
                  const int* __restrict__ box) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  rmat_block_tile<T, TJ, JB, CB, CMP, KT>(G, ldg, n, X, ldx, Y, ldy, ncols, SW, CP, box,
                                          blockIdx.x, lds_raw);
}

// Persistent form for many products at once (batched KP-SVD): the tiles of all
// jobs form one list, job d owning items [jobs[d].first, jobs[d].first +
// jobs[d].tiles); each workgroup takes the next item from the shared counter
// (an atomic add by one thread, handed to the others through LDS) until the
// list is exhausted, so every workgroup leaves the loop. A tile is computed by
// the same code as in rmat_block_kernel, so each product's bits equal its
// single launch's.
template <typename T, int TJ, int JB, int CB, int KT>
__global__ void __launch_bounds__(64 * (2 * TJ) / (JB * CB))
rmat_block_persistent_kernel(const BlockJob* __restrict__ jobs, int njobs, int total,
                             int* __restrict__ counter) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ int item_s;
  for (;;) {
    if (threadIdx.x == 0) item_s = atomicAdd(counter, 1);
    __syncthreads();
    // the item and everything derived from it are uniform: keep them in SGPRs
    const int item = __builtin_amdgcn_readfirstlane(item_s);
    __syncthreads();                       // read by all before the next fetch
    if (item >= total) break;
    int lo = 0, hi = njobs - 1;            // the job holding the item
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (jobs[mid].first <= item) lo = mid;
      else hi = mid - 1;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    const BlockJob& jb = jobs[lo];
    rmat_block_tile<T, TJ, JB, CB, false, KT>(static_cast<const T*>(jb.G), jb.ldg, jb.n,
                                              static_cast<const T*>(jb.X), jb.ldx,
                                              static_cast<T*>(jb.Y), jb.ldy, jb.ncols, jb.SW,
                                              jb.CP, nullptr, item - jb.first, lds_raw);
    __syncthreads();                       // the slab and X buffers are free again
  }
}

// Slab row stride for phases of CP column blocks: the groups of a column block
// span 16 ntc entries (ntc = ceil((n + 3) / 16)), c spans CP values and the slab
// has a margin of 4, so a row needs 16 ntc + CP + 3 columns; padded so that the
// 16-byte reads of a half-wave fall on distinct banks (8 (mod 16) floats, as
// for the X tile; 2 (mod 32) doubles).
template <typename T>
static int slab_stride(int n, int CP, int TK) {
  (void)TK;
  const int ntc = (n + 3 + kKG - 1) / kKG;
  const int W = kKG * ntc + CP + 3;
  if (sizeof(T) == 4) return ((W + 15) / 16) * 16 + 8;     // 8 (mod 16) floats
  return ((W + 31) / 32) * 32 + 2;                         // 2 (mod 32) doubles
}

template <typename T>
static size_t block_lds(int n, int TJ, int CP, int TK) {
  const int XT = TK + (sizeof(T) == 4 ? 8 : 2);   // x_stride<T, TK>()
  return sizeof(T) * ((size_t)(16 + TJ - 1) * slab_stride<T>(n, CP, TK) + 2 * 32 * (size_t)XT);
}

// The largest row-block count TJ whose slab fits the LDS with whole column
// blocks in one phase or, for large n, in phases of CP >= 16 column blocks
// (the slab is reloaded per phase: (n / CP) x SR rows per workgroup).
template <typename T>
bool plan_block_tj(int n, size_t lds_limit, int TJ, BlockPlan* plan, int TK) {
  int cp_max = n;
  if (const char* e = getenv("KPSB_BLOCK_CP")) cp_max = std::max(1, std::min(n, atoi(e)));
  for (int CP = cp_max; CP >= 1; CP = (CP > 16 ? (CP + 1) / 2 : 0)) {
    const size_t lds = block_lds<T>(n, TJ, CP, TK);
    if (lds <= lds_limit) {
      plan->TJ = TJ;
      plan->CP = CP;
      plan->SW = slab_stride<T>(n, CP, TK);
      plan->TK = TK;
      plan->lds = lds;
      plan->grid = ((n + 15) / 16) * ((n + TJ - 1) / TJ);
      plan->waves = 0;
      plan->grid_limit = 0;
      return true;
    }
    if (CP <= 16) break;
  }
  return false;
}

template <typename T>
bool plan_block(int n, size_t lds_limit, BlockPlan* plan) {
  static const int cand[] = {16, 8, 4, 2, 1};
  int forced = 0;
  if (const char* e = getenv("KPSB_BLOCK_TJ")) forced = atoi(e);
  for (int TJ : cand) {
    if (forced && TJ != forced) continue;
    if (plan_block_tj<T>(n, lds_limit, TJ, plan)) return true;
  }
  return false;
}
template bool plan_block<float>(int, size_t, BlockPlan*);
template bool plan_block<double>(int, size_t, BlockPlan*);
template bool plan_block_tj<float>(int, size_t, int, BlockPlan*, int);
template bool plan_block_tj<double>(int, size_t, int, BlockPlan*, int);

template <typename T, int TJ, int JB, int CB, int KT = kTK>
static void launch_tj(const BlockPlan& p, const T* G, int ldg, int n, const T* X, long ldx,
                      T* Y, long ldy, int ncols, hipStream_t s, const int* box) {
  auto kern = box ? rmat_block_kernel<T, TJ, JB, CB, true, KT>
                  : rmat_block_kernel<T, TJ, JB, CB, false, KT>;
  constexpr int threads = 64 * (2 * TJ) / (JB * CB);
  if (p.lds > 65536)
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)p.lds);
  const int grid = p.grid_limit > 0 && p.grid_limit < p.grid ? p.grid_limit : p.grid;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), p.lds, s, G, ldg, n, X, ldx, Y, ldy,
                     ncols, p.SW, p.CP, box);
}

template <typename T>
void launch_rmat_block(const BlockPlan& p, const T* G, int ldg, int n, const T* X, long ldx,
                       T* Y, long ldy, int ncols, hipStream_t s, const int* box) {
  // waves per workgroup: TJ = 16 -> 16 (JB = 1) or 8 (JB = 2); TJ = 8 -> 8 (CB = 2)
  // or 16 (CB = 1); TJ = 12 -> 12 (K tiles of 128 or 176 only: a grid of
  // whole rounds of 256 workgroups where 8 and 16 leave a partial one, e.g.
  // 768 tiles at n = 384); chosen by the autotuner, 16 and 8 by default; K
  // tiles of 64 or (these shapes) 128, 176 or 192 entries (fewer tiles, so
  // fewer barriers, per column block; larger X buffers). 176 = 11 groups
  // splits the 33 groups of a column block whose r range starts below 0 into
  // three full tiles (at n = 512; 192 leaves a last tile of 9).
  if (p.TK == 176) {
    if (p.TJ == 16 && p.waves == 8)
      launch_tj<T, 16, 2, 2, 176>(p, G, ldg, n, X, ldx, Y, ldy, ncols, s, box);
    else if (p.TJ == 16)
      launch_tj<T, 16, 1, 2, 176>(p, G, ldg, n, X, ldx, Y, ldy, ncols, s, box);
    else if (p.TJ == 12)
      launch_tj<T, 12, 1, 2, 176>(p, G, ldg, n, X, ldx, Y, ldy, ncols, s, box);
    else if (p.TJ == 8 && p.waves == 16)
      launch_tj<T, 8, 1, 1, 176>(p, G, ldg, n, X, ldx, Y, ldy, ncols, s, box);
    else
      launch_tj<T, 8, 1, 2, 176>(p, G, ldg, n, X, ldx, Y, ldy, ncols, s, box);
    return;
  }
  if (p.TK == 192) {
    if (p.TJ == 16 && p.waves == 8)
      launch_tj<T, 16, 2, 2, 192>(p, G, ldg, n, X, ldx, Y, ldy, ncols, s, box);
    else if (p.TJ == 16)
      launch_tj<T, 16, 1, 2, 192>(p, G, ldg, n, X, ldx, Y, ldy, ncols, s, box);
    else if (p.TJ == 8 && p.waves == 16)
      launch_tj<T, 8, 1, 1, 192>(p, G, ldg, n, X, ldx, Y, ldy, ncols, s, box);
    else
      launch_tj<T, 8, 1, 2, 192>(p, G, ldg, n, X, ldx, Y, ldy, ncols, s, box);
    return;
  }
  if (p.TK == 128) {
    if (p.TJ == 16 && p.waves == 8)
      launch_tj<T, 16, 2, 2, 128>(p, G, ldg, n, X, ldx, Y, ldy, ncols, s, box);
    else if (p.TJ == 16)
      launch_tj<T, 16, 1, 2, 128>(p, G, ldg, n, X, ldx, Y, ldy, ncols, s, box);
    else if (p.TJ == 12)
      launch_tj<T, 12, 1, 2, 128>(p, G, ldg, n, X, ldx, Y, ldy, ncols, s, box);
    else if (p.TJ == 8 && p.waves == 16)
      launch_tj<T, 8, 1, 1, 128>(p, G, ldg, n, X, ldx, Y, ldy, ncols, s, box);
    else
      launch_tj<T, 8, 1, 2, 128>(p, G, ldg, n, X, ldx, Y, ldy, ncols, s, box);
    return;
  }
  if (p.TJ == 16 && p.waves == 8) {
    launch_tj<T, 16, 2, 2>(p, G, ldg, n, X, ldx, Y, ldy, ncols, s, box);
    return;
  }
  if (p.TJ == 8 && p.waves == 16) {
    launch_tj<T, 8, 1, 1>(p, G, ldg, n, X, ldx, Y, ldy, ncols, s, box);
    return;
  }
  switch (p.TJ) {
    case 16: launch_tj<T, 16, 1, 2>(p, G, ldg, n, X, ldx, Y, ldy, ncols, s, box); break;
    case 8: launch_tj<T, 8, 1, 2>(p, G, ldg, n, X, ldx, Y, ldy, ncols, s, box); break;
    case 4: launch_tj<T, 4, 1, 2>(p, G, ldg, n, X, ldx, Y, ldy, ncols, s, box); break;
    case 2: launch_tj<T, 2, 1, 1>(p, G, ldg, n, X, ldx, Y, ldy, ncols, s, box); break;
    default: launch_tj<T, 1, 1, 1>(p, G, ldg, n, X, ldx, Y, ldy, ncols, s, box); break;
  }
}
template void launch_rmat_block<float>(const BlockPlan&, const float*, int, int, const float*,
                                       long, float*, long, int, hipStream_t, const int*);
template void launch_rmat_block<double>(const BlockPlan&, const double*, int, int,
                                        const double*, long, double*, long, int, hipStream_t,
                                        const int*);

template <int TJ, int JB, int CB, int KT>
static void launch_persistent_tj(const BlockJob* jobs, int njobs, int total, int* counter,
                                 size_t lds, int grid, hipStream_t s) {
  auto kern = rmat_block_persistent_kernel<float, TJ, JB, CB, KT>;
  constexpr int threads = 64 * (2 * TJ) / (JB * CB);
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), lds, s, jobs, njobs, total, counter);
}

// shapes of 16 row blocks (8 or 16 waves) or 8 (8 or 16 waves) only
template <int KT>
static void launch_persistent_tk(const BlockPlan& p, const BlockJob* jobs, int njobs, int total,
                                 int* counter, size_t lds, int grid, hipStream_t s) {
  if (p.TJ == 16 && p.waves == 8)
    launch_persistent_tj<16, 2, 2, KT>(jobs, njobs, total, counter, lds, grid, s);
  else if (p.TJ == 16)
    launch_persistent_tj<16, 1, 2, KT>(jobs, njobs, total, counter, lds, grid, s);
  else if (p.TJ == 8 && p.waves == 16)
    launch_persistent_tj<8, 1, 1, KT>(jobs, njobs, total, counter, lds, grid, s);
  else
    launch_persistent_tj<8, 1, 2, KT>(jobs, njobs, total, counter, lds, grid, s);
}

void launch_rmat_block_persistent(const BlockPlan& shape, const BlockJob* jobs, int njobs,
                                  int total, int* counter, size_t lds, int grid, hipStream_t s) {
  launch_fill_int(counter, 1, 0, s);
  switch (shape.TK) {
    case 176: launch_persistent_tk<176>(shape, jobs, njobs, total, counter, lds, grid, s); break;
    case 192: launch_persistent_tk<192>(shape, jobs, njobs, total, counter, lds, grid, s); break;
    case 128: launch_persistent_tk<128>(shape, jobs, njobs, total, counter, lds, grid, s); break;
    default: launch_persistent_tk<64>(shape, jobs, njobs, total, counter, lds, grid, s); break;
  }
}

// Rows and columns of a grid that hold nonzero entries (support box for the
// block kernel): partial boxes of kBoxBlocks workgroups, then one reduction.
// box = {a_lo, a_hi, b_lo, b_hi}; an all-zero grid gives a_lo > a_hi.
constexpr int kBoxBlocks = 64;
template <typename T>
__global__ void grid_box_partial_kernel(const T* __restrict__ G, int ldg, int n,
                                        int* __restrict__ part) {
  const int g2 = 2 * n - 1;
  int alo = INT_MAX, ahi = -1, blo = INT_MAX, bhi = -1;
  for (int a = blockIdx.x; a < g2; a += gridDim.x) {
    const T* row = G + (long)a * ldg;
    for (int b = threadIdx.x; b < g2; b += blockDim.x) {
      if ((double)row[b] != 0.0) {
        alo = min(alo, a);
        ahi = max(ahi, a);
        blo = min(blo, b);
        bhi = max(bhi, b);
      }
    }
  }
  __shared__ int sh[4][256];
  sh[0][threadIdx.x] = alo;
  sh[1][threadIdx.x] = ahi;
  sh[2][threadIdx.x] = blo;
  sh[3][threadIdx.x] = bhi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sh[0][threadIdx.x] = min(sh[0][threadIdx.x], sh[0][threadIdx.x + w]);
      sh[1][threadIdx.x] = max(sh[1][threadIdx.x], sh[1][threadIdx.x + w]);
      sh[2][threadIdx.x] = min(sh[2][threadIdx.x], sh[2][threadIdx.x + w]);
      sh[3][threadIdx.x] = max(sh[3][threadIdx.x], sh[3][threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void grid_box_final_kernel(const int* __restrict__ part, int nparts,
                                      int* __restrict__ box) {
  if (threadIdx.x != 0) return;
  int alo = INT_MAX, ahi = -1, blo = INT_MAX, bhi = -1;
  for (int p = 0; p < nparts; ++p) {
    alo = min(alo, part[4 * p]);
    ahi = max(ahi, part[4 * p + 1]);
    blo = min(blo, part[4 * p + 2]);
    bhi = max(bhi, part[4 * p + 3]);
  }
  box[0] = alo;
  box[1] = ahi;
  box[2] = blo;
  box[3] = bhi;
}

template <typename T>
void launch_grid_box(const T* G, int ldg, int n, int* part, int* box, hipStream_t s) {
  hipLaunchKernelGGL(grid_box_partial_kernel<T>, dim3(kBoxBlocks), dim3(256), 0, s, G, ldg, n,
                     part);
  hipLaunchKernelGGL(grid_box_final_kernel, dim3(1), dim3(64), 0, s, part, kBoxBlocks, box);
}
int grid_box_parts() { return kBoxBlocks * 4; }
template void launch_grid_box<float>(const float*, int, int, int*, int*, hipStream_t);
template void launch_grid_box<double>(const double*, int, int, int*, int*, hipStream_t);
template void launch_grid_box<__hip_bfloat16>(const __hip_bfloat16*, int, int, int*, int*,
                                              hipStream_t);
template void launch_grid_box<__half>(const __half*, int, int, int*, int*, hipStream_t);

}  // namespace kpsb
