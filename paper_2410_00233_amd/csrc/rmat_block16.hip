// Generated-tile block product Y = R X with 16-bit inputs (BF16 or FP16) and
// FP32 accumulation on v_mfma_f32_16x16x32_{bf16,f16}: the reduced-precision
// mode of the block products (precision subsystem; accuracy is won back by the
// Rayleigh-Ritz refinement in the RSVD driver).
//
// Layout as in the FP32 kernel: a workgroup owns 16 rows i in each of TJ row
// blocks j and keeps the 16 + TJ - 1 grid rows they touch in LDS (16-bit). The
// MFMA takes 8 consecutive K entries per lane (A lane l: row l%16,
// k = 8*(l/16) + 0..7; B lane l: column l%16, same k; D lane l item e: row
// 4*(l/16) + e, column l%16 -- checked on gfx950). To read those 8 entries as
// one aligned 16-byte LDS load, the K range of column block c is shifted to
// r in [r0_c, r0_c + LEN) with r0_c = -((n - 1 - c) mod 8): its first slab
// column r0_c - c + n - 1 is then a multiple of 8. Entries with r outside
// [0, n) are staged as 0 (LEN = n + 7 rounded up to 32: at most 39 extra
// zero products per column block). X arrives already converted to 16 bits.
//
// Accumulation: the MFMA's FP32 accumulators take the whole sum (FOLD = false:
// the 16-bit products, whose operand rounding, 2^-9 relative, dwarfs FP32
// summation error), or are folded into FP64 accumulators at the end of every
// column block (FOLD = true: the split-FP16 refinement product, which must
// keep FP32-level accuracy; 64 more registers per 32 outputs per lane and
// about 15 % of the kernel time at n = 512).
#include "common.h"

namespace kpsb {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <typename H> struct Mfma16;
template <> struct Mfma16<__hip_bfloat16> {
  typedef bf16x8 vec;
  static __device__ __forceinline__ floatx4 mma(vec a, vec b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma16<__half> {
  typedef f16x8 vec;
  static __device__ __forceinline__ floatx4 mma(vec a, vec b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

constexpr int kKS = 32;      // K entries per MFMA step
constexpr int kSPT = 8;      // MFMA K steps per staged tile (one barrier per tile; 4 measured slower)
// LDS row stride of the staged X tile (16-bit elements): 136 words, 8 (mod 16),
// so that the 16-byte fragment reads of a half-wave fall on distinct banks
constexpr int kXS16 = kKS * kSPT + 16;

// X16 is the pre-shifted 16-bit copy of X (launch_to16_shifted): column `col`,
// K step ks = c * (LEN/32) + tt holds the 32 entries r0_c + 32 tt + (0..31) of
// column block c at X16[col * ldx + 32 ks + (0..31)], zero outside [0, n). A tile
// is kSPT consecutive K steps (it may span two column blocks).
template <typename H, int TJ, int JB, int CB, bool FOLD>
__global__ void __launch_bounds__(64 * (2 * TJ) / (JB * CB))
rmat_block16_kernel(const H* __restrict__ G, int ldg, int n, const H* __restrict__ X, long ldx,
                    float* __restrict__ Y, long ldy, int ncols, int SW, int LEN, int CP,
                    const double* __restrict__ inv_scale, int accumulate) {
  constexpr int WAVES = (2 * TJ) / (JB * CB);
  constexpr int NT = 64 * WAVES;
  constexpr int SR = 16 + TJ - 1;
  constexpr int WC = 2 / CB;
  constexpr int TILE = kKS * kSPT;                    // K entries per staged tile
  constexpr int CPC = TILE / 8;                       // 16-byte chunks per column of a tile
  constexpr int V8 = 32 * CPC;                        // 16-byte chunks per tile
  constexpr int LPT = (V8 + NT - 1) / NT;
  typedef typename Mfma16<H>::vec vec;
  typedef unsigned short u16;

  extern __shared__ __align__(16) unsigned char lds_raw[];
  u16* slab = reinterpret_cast<u16*>(lds_raw);
  u16* xbuf = slab + SR * SW;                       // 2 x 32 columns x kXS16
  const u16* Gb = reinterpret_cast<const u16*>(G);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int n_it = (n + 15) >> 4;
  const int it = blockIdx.x % n_it;
  const int jt = blockIdx.x / n_it;
  const int i0 = it * 16;
  const int j0 = jt * TJ;
  const int g2 = 2 * n - 1;
  const int a0 = i0 - j0 - (TJ - 1) + n - 1;

  // Slab phases: column blocks c in [c0, c0 + CP) need the grid columns from
  // gcol0 = floor8(n - 1 - (c_last) - 7) on (slab column s holds grid column
  // gcol0 + s); CP * ntc is a multiple of kSPT, so a tile never spans two
  // phases, and the slab is reloaded between tiles.
  int gcol0 = 0;
  auto load_slab = [&](int c0) {
    const int c1 = min(c0 + CP, n);
    gcol0 = (n - 1 - (c1 - 1) - 7) & ~7;
    for (int al = 0; al < SR; ++al) {
      const int a = a0 + al;
      const bool rowok = (a >= 0) && (a < g2);
      const u16* src = Gb + (long)(rowok ? a : 0) * ldg;
      for (int col = tid; col < SW; col += NT) {
        const int gc = gcol0 + col;
        u16 v = 0;
        if (rowok && gc >= 0 && gc < g2) v = src[gc];
        slab[al * SW + col] = v;
      }
    }
  };
  load_slab(0);

  const int ntc = LEN / kKS;                   // K steps per column block
  const int total_ks = n * ntc;
  const int ntiles = (total_ks + kSPT - 1) / kSPT;
  const long xlen = (long)total_ks * kKS;      // valid entries per column of X16
  uint4 stage[LPT];
  auto load_tile = [&](int t, uint4* dst) {
#pragma unroll
    for (int m = 0; m < LPT; ++m) {
      const int e = tid + NT * m;              // 16-byte chunk: column e / CPC, part e % CPC
      const int col = e / CPC;
      const long off = (long)t * TILE + (e % CPC) * 8;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (e < V8 && col < ncols && off < xlen)
        v = *reinterpret_cast<const uint4*>(reinterpret_cast<const u16*>(X) + (long)col * ldx + off);
      dst[m] = v;
    }
  };
  auto store_tile = [&](int buf) {
    u16* xs = xbuf + buf * (32 * kXS16);
#pragma unroll
    for (int m = 0; m < LPT; ++m) {
      const int e = tid + NT * m;
      if (e < V8) *reinterpret_cast<uint4*>(xs + (e / CPC) * kXS16 + (e % CPC) * 8) = stage[m];
    }
  };

  floatx4 acc[JB][CB];
  double accd[JB][CB][4];
#pragma unroll
  for (int jb = 0; jb < JB; ++jb)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        acc[jb][cb][e] = 0.f;
        accd[jb][cb][e] = 0.0;
      }

  const int wc = wave % WC;
  const int wj = wave / WC;
  const int lrow = lane & 15;
  const int lg = lane >> 4;                    // k group: entries 8*lg .. 8*lg + 7
  int arow[JB];
#pragma unroll
  for (int jb = 0; jb < JB; ++jb) arow[jb] = (lrow + (TJ - 1) - (wj * JB + jb)) * SW;

  load_tile(0, stage);
  store_tile(0);
  __syncthreads();

  // (c, tt) of K step ks = c * ntc + tt, advanced step by step (no division)
  int c = 0, tt = 0;
  for (int t = 0; t < ntiles; ++t) {
    if (t + 1 < ntiles) load_tile(t + 1, stage);
    const u16* xs = xbuf + (t & 1) * (32 * kXS16);
#pragma unroll
    for (int s = 0; s < kSPT; ++s) {
      const int ks = t * kSPT + s;
      if (ks < total_ks) {
        const int colbase = -((n - 1 - c) & 7) - c + n - 1 + tt * kKS - gcol0;   // multiple of 8
        vec bfr[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
          bfr[cb] = *reinterpret_cast<const vec*>(xs + ((wc * CB + cb) * 16 + lrow) * kXS16 +
                                                  s * kKS + 8 * lg);
#pragma unroll
        for (int jb = 0; jb < JB; ++jb) {
          const vec afr = *reinterpret_cast<const vec*>(slab + arow[jb] + colbase + 8 * lg);
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) acc[jb][cb] = Mfma16<H>::mma(afr, bfr[cb], acc[jb][cb]);
        }
        if (tt == ntc - 1) {       // end of column block c
          if constexpr (FOLD) {
#pragma unroll
            for (int jb = 0; jb < JB; ++jb)
#pragma unroll
              for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                  accd[jb][cb][e] += (double)acc[jb][cb][e];
                  acc[jb][cb][e] = 0.f;
                }
          }
          tt = 0;
          ++c;
        } else {
          ++tt;
        }
      }
    }
    if (t + 1 < ntiles) store_tile((t + 1) & 1);
    __syncthreads();
    const int ks_next = (t + 1) * kSPT;
    if (ks_next < total_ks && ks_next % (CP * ntc) == 0) {   // next phase (c = ks_next / ntc)
      load_slab(ks_next / ntc);
      __syncthreads();
    }
  }

  const double osc = inv_scale ? *inv_scale : 1.0;   // undo the operands' power-of-2 scaling
#pragma unroll
  for (int jb = 0; jb < JB; ++jb) {
    const int j = j0 + wj * JB + jb;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const int col = (wc * CB + cb) * 16 + lrow;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = i0 + 4 * lg + e;
        if (i < n && j < n && col < ncols) {
          float* yp = Y + (long)col * ldy + i + (long)n * j;
          const double v = (FOLD ? accd[jb][cb][e] : (double)acc[jb][cb][e]) * osc;
          *yp = accumulate ? (float)((double)*yp + v) : (float)v;
        }
      }
    }
  }
}

static int len16(int n) { return ((n + 7 + kKS - 1) / kKS) * kKS; }

// Slab row stride for phases of CP column blocks: a phase spans at most
// min(CP, n) + LEN + 13 grid columns from its 8-aligned start.
static int stride16(int n, int CP) {
  const int W = std::min(CP, n) + len16(n) + 16;
  return ((W + 31) / 32) * 32 + 16;        // 8 (mod 16) words: distinct banks per half-wave
}

static size_t lds16(int n, int TJ, int CP) {
  return 2 * ((size_t)(16 + TJ - 1) * stride16(n, CP) + 2 * 32 * kXS16);
}

// Length (16-bit elements) of one column of the pre-shifted X16 copy, padded to
// whole tiles so that tile loads never leave the buffer.
long x16_column_len(int n) {
  const long total = (long)n * len16(n);
  const long tile = kKS * kSPT;
  return ((total + tile - 1) / tile) * tile;
}

// One phase (CP = n) if the slab fits, else phases of CP column blocks, CP a
// multiple of kSPT (so phases start on tile boundaries), halved until it fits.
bool plan_block16_tj(int n, size_t lds_limit, int TJ, BlockPlan* plan) {
  int CP = n;
  if (lds16(n, TJ, CP) > lds_limit) {
    CP = 512;
    while (CP >= 16 && (CP >= n || lds16(n, TJ, CP) > lds_limit)) CP /= 2;
    if (CP < 16) return false;
  }
  const size_t lds = lds16(n, TJ, CP);
  plan->TJ = TJ;
  plan->CP = CP;
  plan->SW = stride16(n, CP);
  plan->lds = lds;
  plan->grid = ((n + 15) / 16) * ((n + TJ - 1) / TJ);
  plan->waves = 0;
  plan->grid_limit = 0;
  return true;
}

bool plan_block16(int n, size_t lds_limit, BlockPlan* plan) {
  static const int cand[] = {32, 16, 8, 4};
  int forced = 0;
  if (const char* e = getenv("KPSB_BLOCK16_TJ")) forced = atoi(e);
  for (int TJ : cand) {
    if (forced && TJ != forced) continue;
    if (plan_block16_tj(n, lds_limit, TJ, plan)) return true;
  }
  return false;
}

template <typename H, int TJ, int JB, int CB>
static void launch16_tj(const BlockPlan& p, const H* G, int ldg, int n, const H* X, long ldx,
                        float* Y, long ldy, int ncols, const double* inv_scale, int accumulate,
                        bool fold, hipStream_t s) {
  auto kern = fold ? rmat_block16_kernel<H, TJ, JB, CB, true> : rmat_block16_kernel<H, TJ, JB, CB, false>;
  constexpr int threads = 64 * (2 * TJ) / (JB * CB);
  if (p.lds > 65536)
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)p.lds);
  const int grid = p.grid_limit > 0 && p.grid_limit < p.grid ? p.grid_limit : p.grid;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), p.lds, s, G, ldg, n, X, ldx, Y, ldy,
                     ncols, p.SW, len16(n), p.CP, inv_scale, accumulate);
}

template <typename H>
void launch_rmat_block16(const BlockPlan& p, const H* G16, int ldg, int n, const H* X16,
                         long ldx, float* Y, long ldy, int ncols, hipStream_t s,
                         const double* inv_scale, int accumulate, bool fold) {
  // waves per workgroup (p.waves, 0 = the default): more waves hide the LDS
  // latency of the fragment reads better, fewer row blocks per wave read more
  // LDS per MFMA; chosen by the autotuner
  if (p.TJ == 64 && p.waves == 8) {
    launch16_tj<H, 64, 8, 2>(p, G16, ldg, n, X16, ldx, Y, ldy, ncols, inv_scale, accumulate, fold, s);
    return;
  }
  if (p.TJ == 64) {
    launch16_tj<H, 64, 4, 2>(p, G16, ldg, n, X16, ldx, Y, ldy, ncols, inv_scale, accumulate, fold, s);
    return;
  }
  if (p.TJ == 32 && p.waves == 16) {
    launch16_tj<H, 32, 2, 2>(p, G16, ldg, n, X16, ldx, Y, ldy, ncols, inv_scale, accumulate, fold, s);
    return;
  }
  if (p.TJ == 16 && p.waves == 8) {
    launch16_tj<H, 16, 2, 2>(p, G16, ldg, n, X16, ldx, Y, ldy, ncols, inv_scale, accumulate, fold, s);
    return;
  }
  if (p.TJ == 16 && p.waves == 16) {
    launch16_tj<H, 16, 1, 2>(p, G16, ldg, n, X16, ldx, Y, ldy, ncols, inv_scale, accumulate, fold, s);
    return;
  }
  switch (p.TJ) {
    case 32: launch16_tj<H, 32, 4, 2>(p, G16, ldg, n, X16, ldx, Y, ldy, ncols, inv_scale, accumulate, fold, s); break;
    case 16: launch16_tj<H, 16, 4, 2>(p, G16, ldg, n, X16, ldx, Y, ldy, ncols, inv_scale, accumulate, fold, s); break;
    case 8: launch16_tj<H, 8, 2, 2>(p, G16, ldg, n, X16, ldx, Y, ldy, ncols, inv_scale, accumulate, fold, s); break;
    default: launch16_tj<H, 4, 1, 2>(p, G16, ldg, n, X16, ldx, Y, ldy, ncols, inv_scale, accumulate, fold, s); break;
  }
}
template void launch_rmat_block16<__hip_bfloat16>(const BlockPlan&, const __hip_bfloat16*, int,
                                                  int, const __hip_bfloat16*, long, float*,
                                                  long, int, hipStream_t, const double*, int,
                                                  bool);
template void launch_rmat_block16<__half>(const BlockPlan&, const __half*, int, int,
                                          const __half*, long, float*, long, int, hipStream_t,
                                          const double*, int, bool);

// FP32 X (N x ncols, ld ldx) -> pre-shifted 16-bit copy (see rmat_block16_kernel):
// out[col * ldo + c * LEN + kk] = X[col * ldx + c * n + r0_c + kk] for
// 0 <= r0_c + kk < n, else 0; r0_c = -((n - 1 - c) mod 8). Round to nearest even.
__device__ __forceinline__ void cvt16(float v, __hip_bfloat16* o) { *o = __float2bfloat16(v); }
__device__ __forceinline__ void cvt16(float v, __half* o) { *o = __float2half(v); }
template <typename H>
__global__ void to16_shifted_kernel(const float* __restrict__ in, long ldx, int n, int ncols,
                                    int LEN, H* __restrict__ out, long ldo) {
  const long per_col = (long)n * LEN;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)ldo * ncols;
       e += (long)gridDim.x * blockDim.x) {
    const int col = (int)(e / ldo);
    const long o = e - (long)col * ldo;
    float v = 0.f;
    if (o < per_col) {
      const int c = (int)(o / LEN);
      const int kk = (int)(o - (long)c * LEN);
      const int r = -((n - 1 - c) & 7) + kk;
      if (r >= 0 && r < n) v = in[(long)col * ldx + (long)n * c + r];
    }
    cvt16(v, out + e);
  }
}
template <typename H>
void launch_to16_shifted(const float* in, long ldx, int n, int ncols, H* out, long ldo,
                         hipStream_t s) {
  hipLaunchKernelGGL(to16_shifted_kernel<H>, dim3(2048), dim3(256), 0, s, in, ldx, n, ncols,
                     len16(n), out, ldo);
}
template void launch_to16_shifted<__hip_bfloat16>(const float*, long, int, int, __hip_bfloat16*,
                                                  long, hipStream_t);
template void launch_to16_shifted<__half>(const float*, long, int, int, __half*, long, hipStream_t);

// Two-term FP16 split of the pre-shifted copy: with v' = v * 2^kSplitXExp,
// hi = fp16(v') and lo = fp16(v' - hi) (the residual is exact in FP32), so
// hi + lo carries about 22 significant bits of v. Columns of unit norm have
// |v| <= 1, i.e. |v'| <= 2048, inside FP16's range; the scaling keeps their
// entries away from FP16's subnormal range.
__global__ void to16_split_kernel(const float* __restrict__ in, long ldx, int n, int ncols,
                                  int LEN, __half* __restrict__ hi, __half* __restrict__ lo,
                                  long ldo) {
  const long per_col = (long)n * LEN;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)ldo * ncols;
       e += (long)gridDim.x * blockDim.x) {
    const int col = (int)(e / ldo);
    const long o = e - (long)col * ldo;
    float v = 0.f;
    if (o < per_col) {
      const int c = (int)(o / LEN);
      const int kk = (int)(o - (long)c * LEN);
      const int r = -((n - 1 - c) & 7) + kk;
      if (r >= 0 && r < n) v = in[(long)col * ldx + (long)n * c + r];
    }
    const float vs = v * (float)(1 << kSplitXExp);
    const __half h = __float2half(vs);
    hi[e] = h;
    lo[e] = __float2half(vs - __half2float(h));
  }
}
void launch_to16_split(const float* in, long ldx, int n, int ncols, __half* hi, __half* lo,
                       long ldo, hipStream_t s) {
  hipLaunchKernelGGL(to16_split_kernel, dim3(2048), dim3(256), 0, s, in, ldx, n, ncols,
                     len16(n), hi, lo, ldo);
}

}  // namespace kpsb
