// Vector kernels for Gram-Schmidt reorthogonalization, norms and the small
// tall-skinny products of the KP-SVD drivers. Every reduction writes a fixed
// number (kRedBlocks) of FP64 partial sums that consumers add in a fixed order,
// so results are deterministic run to run.
#include "common.h"

namespace kpsb {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Block-wide sum over 256 threads; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return r;
}

// Sum of the kRedBlocks partials (stride `stride`, offset `off`), identical in
// every block that calls it. Result broadcast to the whole block.
__device__ __forceinline__ double reduce_partials_block(const double* p, int stride, int off,
                                                        double* sh) {
  double v = p[(long)threadIdx.x * stride + off];   // kRedThreads == kRedBlocks
  v = block_sum(v, sh);
  if (threadIdx.x == 0) sh[4] = v;
  __syncthreads();
  double r = sh[4];
  __syncthreads();
  return r;
}

__device__ __forceinline__ void row_range(long N, long* lo, long* hi) {
  long chunk = (N + gridDim.x - 1) / gridDim.x;
  *lo = (long)blockIdx.x * chunk;
  *hi = *lo + chunk < N ? *lo + chunk : N;
}

// Vector paths (16-byte loads of VEC = 16 / sizeof(T) consecutive rows): taken
// when N, the leading dimension and the pointers allow them. The block's row
// range is then a multiple of VEC long (the last block's ends at N).
template <typename T> struct Vec16 {
  static constexpr int VEC = 16 / (int)sizeof(T);
  typedef T type __attribute__((ext_vector_type(VEC)));
};

__device__ __forceinline__ void row_range_vec(long N, int VEC, long* lo, long* hi) {
  const long nv = N / VEC;
  const long chunk = ((nv + gridDim.x - 1) / gridDim.x) * VEC;
  *lo = (long)blockIdx.x * chunk;
  *hi = *lo + chunk < N ? *lo + chunk : N;
  if (*lo > N) *lo = N;
}

template <typename T>
static bool vec_ok(long N, long ld, const void* a, const void* b) {
  constexpr int VEC = Vec16<T>::VEC;
  return N % VEC == 0 && ld % VEC == 0 && (uintptr_t)a % 16 == 0 && (uintptr_t)b % 16 == 0;
}

// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
multidot_kernel(const T* __restrict__ V, long ldv, int m, const T* __restrict__ w, long N,
                double* __restrict__ partials, const int* __restrict__ pred) {
  if (pred && *pred == 0) return;
  __shared__ double sh[8][4];
  long lo, hi;
  row_range(N, &lo, &hi);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int g = 0; g < m; g += 8) {
    double acc[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) acc[e] = 0.0;
    for (long r = lo + threadIdx.x; r < hi; r += 256) {
      const double wr = (double)w[r];
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (g + e < m) acc[e] += (double)V[(long)(g + e) * ldv + r] * wr;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      double v = wave_sum(acc[e]);
      if (lane == 0) sh[e][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < 8 && g + threadIdx.x < m) {
      const int e = threadIdx.x;
      partials[(long)blockIdx.x * m + g + e] = sh[e][0] + sh[e][1] + sh[e][2] + sh[e][3];
    }
    __syncthreads();
  }
}

// Vector form: wave q of the block takes the columns q, q + 4, q + 8, ... over
// the block's whole row range (lane l: rows lo + VEC (l + 64 t)), eight
// columns' loads in flight, and writes their block partials from a wave
// reduction (no barrier). w is read by every wave (served by the cache).
template <typename T>
__global__ void __launch_bounds__(256)
multidot_vec_kernel(const T* __restrict__ V, long ldv, int m, const T* __restrict__ w, long N,
                    double* __restrict__ partials, const int* __restrict__ pred) {
  if (pred && *pred == 0) return;
  constexpr int VEC = Vec16<T>::VEC;
  typedef typename Vec16<T>::type vec_t;
  constexpr int CG = 8;                       // columns per round of loads
  long lo, hi;
  row_range_vec(N, VEC, &lo, &hi);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c0 = wave; c0 < m; c0 += 4 * CG) {   // columns c0 + 4 e, e < CG
    double acc[CG];
#pragma unroll
    for (int e = 0; e < CG; ++e) acc[e] = 0.0;
    for (long r = lo + (long)VEC * lane; r < hi; r += 64L * VEC) {
      const vec_t wv = *reinterpret_cast<const vec_t*>(w + r);
      vec_t vv[CG];
#pragma unroll
      for (int e = 0; e < CG; ++e)
        if (c0 + 4 * e < m)
          vv[e] = *reinterpret_cast<const vec_t*>(V + (long)(c0 + 4 * e) * ldv + r);
#pragma unroll
      for (int e = 0; e < CG; ++e)
        if (c0 + 4 * e < m) {
          double t = 0.0;
#pragma unroll
          for (int u = 0; u < VEC; ++u) t += (double)vv[e][u] * (double)wv[u];
          acc[e] += t;
        }
    }
#pragma unroll
    for (int e = 0; e < CG; ++e) {
      const double v = wave_sum(acc[e]);
      if (lane == 0 && c0 + 4 * e < m) partials[(long)blockIdx.x * m + c0 + 4 * e] = v;
    }
  }
}

template <typename T>
void launch_multidot(const T* V, long ldv, int m, const T* w, long N, double* partials,
                     hipStream_t s, const int* pred) {
  if (vec_ok<T>(N, ldv, V, w))
    hipLaunchKernelGGL(multidot_vec_kernel<T>, dim3(kRedBlocks), dim3(256), 0, s, V, ldv, m, w,
                       N, partials, pred);
  else
    hipLaunchKernelGGL(multidot_kernel<T>, dim3(kRedBlocks), dim3(256), 0, s, V, ldv, m, w, N,
                       partials, pred);
}
template void launch_multidot<float>(const float*, long, int, const float*, long, double*,
                                     hipStream_t, const int*);
template void launch_multidot<double>(const double*, long, int, const double*, long,
                                      double*, hipStream_t, const int*);

// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
reduce_partials_kernel(const double* __restrict__ partials, int m, double* __restrict__ h,
                       int accumulate, const int* __restrict__ pred) {
  if (pred && *pred == 0) return;
  __shared__ double sh[8];
  // block i reduces column i
  const int i = blockIdx.x;
  double v = partials[(long)threadIdx.x * m + i];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) h[i] = accumulate ? h[i] + v : v;
}

void launch_reduce_partials(const double* partials, int m, double* h, int accumulate,
                            hipStream_t s, const int* pred) {
  if (m <= 0) return;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(m), dim3(kRedThreads), 0, s, partials, m,
                     h, accumulate, pred);
}

// ---------------------------------------------------------------------------
// Coefficients of a projection into hs[0..m): h itself, or (partials != NULL)
// the sums over the kRedBlocks multidot partials (layout [block][m]), added in
// a fixed order (lane l: blocks l, l + 64, l + 128, l + 192, then a wave sum),
// so every block holds the same values. Block 0 then stores them in h_out
// and/or adds them into h_add. Ends with a barrier.
__device__ __forceinline__ void load_coefs(const double* __restrict__ h,
                                           const double* __restrict__ partials, int m,
                                           double* __restrict__ h_out,
                                           double* __restrict__ h_add, double* hs) {
  if (partials) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = wave; i < m; i += 4) {
      double v = 0.0;
      for (int t = 0; t < kRedBlocks; t += 64) v += partials[(long)(t + lane) * m + i];
      v = wave_sum(v);
      if (lane == 0) hs[i] = v;
    }
  } else if ((int)threadIdx.x < m) {
    hs[threadIdx.x] = h[threadIdx.x];
  }
  __syncthreads();
  if (blockIdx.x == 0 && (int)threadIdx.x < m) {
    if (h_out) h_out[threadIdx.x] = hs[threadIdx.x];
    if (h_add) h_add[threadIdx.x] += hs[threadIdx.x];
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
project_out_kernel(T* __restrict__ w, const T* __restrict__ V, long ldv, int m,
                   const double* __restrict__ h, const double* __restrict__ partials,
                   double* __restrict__ h_out, double* __restrict__ h_add, long N,
                   double* __restrict__ nrm_partials, const int* __restrict__ pred) {
  if (pred && *pred == 0) return;
  __shared__ double hs[64];
  __shared__ double sh[8];
  load_coefs(h, partials, m, h_out, h_add, hs);
  long lo, hi;
  row_range(N, &lo, &hi);
  double nrm = 0.0;
  for (long r = lo + threadIdx.x; r < hi; r += 256) {
    double v = (double)w[r];
    for (int i = 0; i < m; ++i) v -= hs[i] * (double)V[(long)i * ldv + r];
    const T vt = (T)v;
    w[r] = vt;
    nrm += (double)vt * (double)vt;
  }
  nrm = block_sum(nrm, sh);
  if (threadIdx.x == 0 && nrm_partials) nrm_partials[blockIdx.x] = nrm;
}

// Vector form: VEC rows per thread, the columns in rounds of 16 loads in flight.
template <typename T>
__global__ void __launch_bounds__(256)
project_out_vec_kernel(T* __restrict__ w, const T* __restrict__ V, long ldv, int m,
                       const double* __restrict__ h, const double* __restrict__ partials,
                       double* __restrict__ h_out, double* __restrict__ h_add, long N,
                       double* __restrict__ nrm_partials, const int* __restrict__ pred) {
  if (pred && *pred == 0) return;
  constexpr int VEC = Vec16<T>::VEC;
  typedef typename Vec16<T>::type vec_t;
  constexpr int CG = 16;
  __shared__ double hs[64];
  __shared__ double sh[8];
  load_coefs(h, partials, m, h_out, h_add, hs);
  long lo, hi;
  row_range_vec(N, VEC, &lo, &hi);
  double nrm = 0.0;
  for (long r = lo + (long)VEC * threadIdx.x; r < hi; r += 256L * VEC) {
    const vec_t wv = *reinterpret_cast<const vec_t*>(w + r);
    double v[VEC];
#pragma unroll
    for (int u = 0; u < VEC; ++u) v[u] = (double)wv[u];
    for (int i0 = 0; i0 < m; i0 += CG) {
      vec_t vv[CG];
#pragma unroll
      for (int e = 0; e < CG; ++e)
        if (i0 + e < m) vv[e] = *reinterpret_cast<const vec_t*>(V + (long)(i0 + e) * ldv + r);
#pragma unroll
      for (int e = 0; e < CG; ++e)
        if (i0 + e < m) {
#pragma unroll
          for (int u = 0; u < VEC; ++u) v[u] -= hs[i0 + e] * (double)vv[e][u];
        }
    }
    vec_t o;
#pragma unroll
    for (int u = 0; u < VEC; ++u) {
      o[u] = (T)v[u];
      nrm += (double)o[u] * (double)o[u];
    }
    *reinterpret_cast<vec_t*>(w + r) = o;
  }
  nrm = block_sum(nrm, sh);
  if (threadIdx.x == 0 && nrm_partials) nrm_partials[blockIdx.x] = nrm;
}

template <typename T>
static void project_out_any(T* w, const T* V, long ldv, int m, const double* h,
                            const double* partials, double* h_out, double* h_add, long N,
                            double* nrm_partials, hipStream_t s, const int* pred) {
  if (vec_ok<T>(N, ldv, V, w))
    hipLaunchKernelGGL(project_out_vec_kernel<T>, dim3(kRedBlocks), dim3(256), 0, s, w, V, ldv,
                       m, h, partials, h_out, h_add, N, nrm_partials, pred);
  else
    hipLaunchKernelGGL(project_out_kernel<T>, dim3(kRedBlocks), dim3(256), 0, s, w, V, ldv, m,
                       h, partials, h_out, h_add, N, nrm_partials, pred);
}
template <typename T>
void launch_project_out_red(T* w, const T* V, long ldv, int m, const double* partials,
                            double* h_out, double* h_add, long N, double* nrm_partials,
                            hipStream_t s, const int* pred) {
  project_out_any<T>(w, V, ldv, m, nullptr, partials, h_out, h_add, N, nrm_partials, s, pred);
}
template void launch_project_out_red<float>(float*, const float*, long, int, const double*,
                                            double*, double*, long, double*, hipStream_t,
                                            const int*);
template void launch_project_out_red<double>(double*, const double*, long, int, const double*,
                                             double*, double*, long, double*, hipStream_t,
                                             const int*);

// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
norm2_partials_kernel(const T* __restrict__ w, long N, double* __restrict__ nrm_partials) {
  __shared__ double sh[8];
  long lo, hi;
  row_range(N, &lo, &hi);
  double nrm = 0.0;
  for (long r = lo + threadIdx.x; r < hi; r += 256) {
    const double v = (double)w[r];
    nrm += v * v;
  }
  nrm = block_sum(nrm, sh);
  if (threadIdx.x == 0) nrm_partials[blockIdx.x] = nrm;
}

template <typename T>
__global__ void __launch_bounds__(256)
norm2_partials_vec_kernel(const T* __restrict__ w, long N, double* __restrict__ nrm_partials) {
  constexpr int VEC = Vec16<T>::VEC;
  typedef typename Vec16<T>::type vec_t;
  __shared__ double sh[8];
  long lo, hi;
  row_range_vec(N, VEC, &lo, &hi);
  double nrm = 0.0;
  for (long r = lo + (long)VEC * threadIdx.x; r < hi; r += 256L * VEC) {
    const vec_t v = *reinterpret_cast<const vec_t*>(w + r);
#pragma unroll
    for (int u = 0; u < VEC; ++u) nrm += (double)v[u] * (double)v[u];
  }
  nrm = block_sum(nrm, sh);
  if (threadIdx.x == 0) nrm_partials[blockIdx.x] = nrm;
}

template <typename T>
void launch_norm2_partials(const T* w, long N, double* nrm_partials, hipStream_t s) {
  if (vec_ok<T>(N, 0, w, w))
    hipLaunchKernelGGL(norm2_partials_vec_kernel<T>, dim3(kRedBlocks), dim3(256), 0, s, w, N,
                       nrm_partials);
  else
    hipLaunchKernelGGL(norm2_partials_kernel<T>, dim3(kRedBlocks), dim3(256), 0, s, w, N,
                       nrm_partials);
}
template void launch_norm2_partials<float>(const float*, long, double*, hipStream_t);
template void launch_norm2_partials<double>(const double*, long, double*, hipStream_t);

// ---------------------------------------------------------------------------
template <typename T>
__global__ void scale_kernel(T* __restrict__ w, long N, double factor) {
  for (long r = blockIdx.x * (long)blockDim.x + threadIdx.x; r < N;
       r += (long)gridDim.x * blockDim.x)
    w[r] = (T)((double)w[r] * factor);
}
template <typename T>
void launch_scale(T* w, long N, double factor, hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel<T>, dim3(1024), dim3(256), 0, s, w, N, factor);
}
template void launch_scale<float>(float*, long, double, hipStream_t);
template void launch_scale<double>(double*, long, double, hipStream_t);

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11) + Box-Muller. Normal number e of
// (seed, stream): block counter (e/2 low, e/2 high, stream, 0), key (seed low,
// seed high); words (w0, w1) and (w2, w3) make two 53-bit uniforms ua, ub;
// r = sqrt(-2 log(1 - ua)), t = 2 pi ub; even e -> r cos t, odd e -> r sin t.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd > 0) { k0 += W0; k1 += W1; }
    const uint32_t hi0 = __umulhi(M0, c[0]), lo0 = M0 * c[0];
    const uint32_t hi1 = __umulhi(M1, c[2]), lo1 = M1 * c[2];
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
  }
}

template <typename T>
__global__ void philox_normals_kernel(T* __restrict__ out, long N, uint64_t seed,
                                      uint32_t stream_id, const int* __restrict__ pred) {
  if (pred && *pred == 0) return;
  const long nblk = (N + 1) / 2;
  for (long b = blockIdx.x * (long)blockDim.x + threadIdx.x; b < nblk;
       b += (long)gridDim.x * blockDim.x) {
    uint32_t c[4] = {(uint32_t)(b & 0xffffffffu), (uint32_t)((uint64_t)b >> 32), stream_id, 0u};
    philox4x32_10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
    const double two53 = 1.1102230246251565e-16;   // 2^-53
    const double ua = ((double)(c[0] >> 5) * 67108864.0 + (double)(c[1] >> 6)) * two53;
    const double ub = ((double)(c[2] >> 5) * 67108864.0 + (double)(c[3] >> 6)) * two53;
    const double r = sqrt(-2.0 * log(1.0 - ua));
    const double t = 6.283185307179586 * ub;
    out[2 * b] = (T)(r * cos(t));
    if (2 * b + 1 < N) out[2 * b + 1] = (T)(r * sin(t));
  }
}

template <typename T>
void launch_philox_normals(T* out, long N, uint64_t seed, uint32_t stream_id, hipStream_t s,
                           const int* pred) {
  hipLaunchKernelGGL(philox_normals_kernel<T>, dim3(1024), dim3(256), 0, s, out, N, seed,
                     stream_id, pred);
}
template void launch_philox_normals<float>(float*, long, uint64_t, uint32_t, hipStream_t,
                                           const int*);
template void launch_philox_normals<double>(double*, long, uint64_t, uint32_t, hipStream_t,
                                            const int*);

// ---------------------------------------------------------------------------
template <typename S, typename D>
__global__ void convert_kernel(const S* __restrict__ in, D* __restrict__ out, long N) {
  for (long r = blockIdx.x * (long)blockDim.x + threadIdx.x; r < N;
       r += (long)gridDim.x * blockDim.x)
    out[r] = (D)in[r];
}
template <typename S, typename D>
void launch_convert(const S* in, D* out, long N, hipStream_t s) {
  hipLaunchKernelGGL((convert_kernel<S, D>), dim3(1024), dim3(256), 0, s, in, out, N);
}
template void launch_convert<double, float>(const double*, float*, long, hipStream_t);
template void launch_convert<float, double>(const float*, double*, long, hipStream_t);
template void launch_convert<double, double>(const double*, double*, long, hipStream_t);
template void launch_convert<float, float>(const float*, float*, long, hipStream_t);

// ---------------------------------------------------------------------------
// out[:, t] = sum_i V[:, i] * C[i + ldc*t]   (FP64 accumulation)
template <typename T, typename O>
__global__ void __launch_bounds__(256)
small_gemm_kernel(const T* __restrict__ V, long ldv, int m, const double* __restrict__ C,
                  int ldc, int k, long N, O* __restrict__ out, long ldo) {
  __shared__ double Cs[64 * 64];
  for (int e = threadIdx.x; e < m * k; e += 256) {
    const int i = e % m, t = e / m;
    Cs[i + 64 * t] = C[i + (long)ldc * t];
  }
  __syncthreads();
  for (long r = blockIdx.x * (long)blockDim.x + threadIdx.x; r < N;
       r += (long)gridDim.x * blockDim.x) {
    for (int t0 = 0; t0 < k; t0 += 8) {
      double acc[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) acc[e] = 0.0;
      for (int i = 0; i < m; ++i) {
        const double v = (double)V[(long)i * ldv + r];
#pragma unroll
        for (int e = 0; e < 8; ++e) acc[e] += v * Cs[i + 64 * (t0 + e < k ? t0 + e : 0)];
      }
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (t0 + e < k) out[(long)(t0 + e) * ldo + r] = (O)acc[e];
    }
  }
}

template <typename T, typename O>
void launch_small_gemm(const T* V, long ldv, int m, const double* C, int ldc, int k, long N,
                       O* out, long ldo, hipStream_t s) {
  long blocks = (N + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL((small_gemm_kernel<T, O>), dim3((int)blocks), dim3(256), 0, s, V, ldv, m,
                     C, ldc, k, N, out, ldo);
}
template void launch_small_gemm<float, float>(const float*, long, int, const double*, int, int,
                                              long, float*, long, hipStream_t);
template void launch_small_gemm<float, double>(const float*, long, int, const double*, int,
                                               int, long, double*, long, hipStream_t);
template void launch_small_gemm<double, double>(const double*, long, int, const double*, int,
                                                int, long, double*, long, hipStream_t);
template void launch_small_gemm<double, float>(const double*, long, int, const double*, int,
                                               int, long, float*, long, hipStream_t);

}  // namespace kpsb
