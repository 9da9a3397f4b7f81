// The explicit-matrix path: R(A) formed by reordering a dense blur matrix A
// held in HBM (the paper's own pipeline stores A and rearranges it,
// section 2.1, eq. "initial rearrange A"), and the products with the stored
// R used by the KP-SVD drivers, as well as A x for split Bregman with A itself
// (the paper's method (i) of Table 1). Works for any A (any boundary
// condition, spatially variant blur); R is N x N with N = n^2, so the path
// needs 2 N^2 elements of HBM (A and R) and every product streams R from HBM.
//
// Layouts: A and R are row-major N x N. X, Y blocks are column-major N x b.
#include "common.h"

namespace kpsb {

// R[i + n j, r + n c] = A[r + n i, c + n j]: row (i + n j) of R is the column-
// major vec of block A_{i,j}. One workgroup per (block, 32 x 32 sub-tile),
// transposed through LDS so that both the read (along c) and the write
// (along r) are contiguous.
template <typename T>
__global__ void __launch_bounds__(256)
reorder_kernel(const T* __restrict__ A, T* __restrict__ R, int n) {
  __shared__ T tile[32][33];
  const long N = (long)n * n;
  const int tpb = (n + 31) / 32;                 // 32-wide sub-tiles per block side
  const long blk = blockIdx.x / (tpb * tpb);     // block index i + n j
  const int sub = blockIdx.x % (tpb * tpb);
  const int i = (int)(blk % n), j = (int)(blk / n);
  const int r0 = (sub % tpb) * 32, c0 = (sub / tpb) * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  for (int rr = ty; rr < 32; rr += 8) {         // read rows r of the block, c contiguous
    const int r = r0 + rr, c = c0 + tx;
    tile[rr][tx] = (r < n && c < n) ? A[(long)(r + (long)n * i) * N + c + (long)n * j] : (T)0;
  }
  __syncthreads();
  for (int cc = ty; cc < 32; cc += 8) {         // write R row blk, r contiguous
    const int c = c0 + cc, r = r0 + tx;
    if (r < n && c < n) R[blk * N + r + (long)n * c] = tile[tx][cc];
  }
}

template <typename T>
void launch_reorder(const T* A, T* R, int n, hipStream_t s) {
  const int tpb = (n + 31) / 32;
  const long grid = (long)n * n * tpb * tpb;
  hipLaunchKernelGGL(reorder_kernel<T>, dim3((unsigned)grid), dim3(256), 0, s, A, R, n);
}
template void launch_reorder<float>(const float*, float*, int, hipStream_t);
template void launch_reorder<double>(const double*, double*, int, hipStream_t);

// Explicit blur matrix from a PSF: A[r + n i, c + n j] = sum over the images
// c~ of c and j~ of j of P[cu + r - c~, cv + i - j~], where the images are c
// itself (zero boundary conditions, bc = 0), c + 2n m and -1 - c + 2n m for
// m = -1, 0, 1 (reflexive, bc = 1: the image extended by reflection about the
// edge of its last pixel, x[-1-k] = x[k], x[n+k] = x[n-1-k]) or c + n m for
// m = -2 .. 2 (periodic, bc = 2). One thread per entry, FP64 sums.
__device__ __forceinline__ int image_of(int bc, int k, int a, int n) {
  if (bc == 1) return a < 3 ? k + 2 * n * (a - 1) : -1 - k + 2 * n * (a - 4);
  if (bc == 2) return k + n * (a - 2);
  return k;
}

template <typename T>
__global__ void blur_matrix_kernel(const double* __restrict__ psf, int pu, int pv, int cu,
                                   int cv, int n, int bc, T* __restrict__ A) {
  const long N = (long)n * n;
  const int nim = bc == 1 ? 6 : (bc == 2 ? 5 : 1);
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < N * N;
       e += (long)gridDim.x * blockDim.x) {
    const long p = e / N, q = e - p * N;
    const int r = (int)(p % n), i = (int)(p / n);
    const int c = (int)(q % n), j = (int)(q / n);
    double v = 0.0;
    for (int a = 0; a < nim; ++a) {
      const int w = cv + i - image_of(bc, j, a, n);
      if (w < 0 || w >= pv) continue;
      for (int b = 0; b < nim; ++b) {
        const int u = cu + r - image_of(bc, c, b, n);
        if (u >= 0 && u < pu) v += psf[(long)u * pv + w];
      }
    }
    A[e] = (T)v;
  }
}

template <typename T>
void launch_blur_matrix(const double* psf, int pu, int pv, int cu, int cv, int n, int bc, T* A,
                        hipStream_t s) {
  hipLaunchKernelGGL(blur_matrix_kernel<T>, dim3(8192), dim3(256), 0, s, psf, pu, pv, cu, cv, n,
                     bc, A);
}
template void launch_blur_matrix<float>(const double*, int, int, int, int, int, int, float*,
                                        hipStream_t);
template void launch_blur_matrix<double>(const double*, int, int, int, int, int, int, double*,
                                         hipStream_t);

// ---------------------------------------------------------------------------
// y = M x - coef z with M = R (transpose = 0) or R^T, R row-major N x N; FP64
// accumulation. Row product: one wave per row, coalesced along the row.
__device__ __forceinline__ bool any_flag(const int* flags, int nflags) {
  if (flags)
    for (int i = 0; i < nflags; ++i)
      if (flags[i]) return true;
  return false;
}

constexpr int kGvInFlight = 4;   // 16-byte loads in flight per thread

// Row product (R x): one wave per row. With `vec` (N % VEC == 0, R and x
// 16-byte aligned) rows are read with 16-byte loads of VEC elements,
// kGvInFlight of them in flight per lane, into as many FP64 partial sums added
// in a fixed order; otherwise one element per load.
template <typename T>
__device__ __forceinline__ double dot_vec(const T* __restrict__ a, const T* __restrict__ b, long i) {
  constexpr int VEC = 16 / (int)sizeof(T);
  typedef T vec_t __attribute__((ext_vector_type(VEC)));
  const vec_t va = reinterpret_cast<const vec_t*>(a)[i];
  const vec_t vb = reinterpret_cast<const vec_t*>(b)[i];
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < VEC; ++u) s += (double)va[u] * (double)vb[u];
  return s;
}

template <typename T>
__global__ void __launch_bounds__(256)
stored_gemv_rows_kernel(const T* __restrict__ R, long N, const T* __restrict__ x,
                        T* __restrict__ y, const T* __restrict__ z, double coef, int vec,
                        const int* __restrict__ flags, int nflags) {
  if (any_flag(flags, nflags)) return;
  constexpr int VEC = 16 / (int)sizeof(T);
  const int lane = threadIdx.x & 63;
  const long row = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= N) return;
  const T* rp = R + row * N;
  double acc;
  if (vec) {
    const long NV = N / VEC;
    double a[kGvInFlight];
#pragma unroll
    for (int q = 0; q < kGvInFlight; ++q) a[q] = 0.0;
    long c = lane;
    for (; c + 64 * (kGvInFlight - 1) < NV; c += 64 * kGvInFlight) {
#pragma unroll
      for (int q = 0; q < kGvInFlight; ++q) a[q] += dot_vec<T>(rp, x, c + 64 * q);
    }
    for (; c < NV; c += 64) a[0] += dot_vec<T>(rp, x, c);
    acc = 0.0;
#pragma unroll
    for (int q = 0; q < kGvInFlight; ++q) acc += a[q];
  } else {
    acc = 0.0;
    for (long c = lane; c < N; c += 64) acc += (double)rp[c] * (double)x[c];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) {
    double v = acc;
    if (z) v -= coef * (double)z[row];
    y[row] = (T)v;
  }
}

// Column product (R^T w): workgroup (strip of 256 x VEC columns, row chunk)
// writes a partial sum per column; with `vec` (N % VEC == 0, R 16-byte aligned)
// each thread reads a 16-byte vector of VEC columns per row (kGvInFlight
// rows in flight), otherwise one column. The chunks are then added in a fixed order.
constexpr int kGvChunks = 32;
template <typename T>
__global__ void __launch_bounds__(256)
stored_gemv_cols_kernel(const T* __restrict__ R, long N, const T* __restrict__ w,
                        double* __restrict__ part, int vec, const int* __restrict__ flags,
                        int nflags) {
  if (any_flag(flags, nflags)) return;
  constexpr int VEC = 16 / (int)sizeof(T);
  typedef T vec_t __attribute__((ext_vector_type(VEC)));
  const int chunk = blockIdx.y;
  const long rows = (N + kGvChunks - 1) / kGvChunks;
  const long r0 = chunk * rows, r1 = r0 + rows < N ? r0 + rows : N;
  if (vec) {
    const long cv = (long)blockIdx.x * 256 + threadIdx.x;   // vector column
    if (cv * VEC >= N) return;
    double acc[VEC];
#pragma unroll
    for (int u = 0; u < VEC; ++u) acc[u] = 0.0;
    long r = r0;
    for (; r + kGvInFlight - 1 < r1; r += kGvInFlight) {
      vec_t v[kGvInFlight];
#pragma unroll
      for (int q = 0; q < kGvInFlight; ++q)
        v[q] = reinterpret_cast<const vec_t*>(R + (r + q) * N)[cv];
#pragma unroll
      for (int q = 0; q < kGvInFlight; ++q) {
        const double wr = (double)w[r + q];
#pragma unroll
        for (int u = 0; u < VEC; ++u) acc[u] += (double)v[q][u] * wr;
      }
    }
    for (; r < r1; ++r) {
      const vec_t v = reinterpret_cast<const vec_t*>(R + r * N)[cv];
      const double wr = (double)w[r];
#pragma unroll
      for (int u = 0; u < VEC; ++u) acc[u] += (double)v[u] * wr;
    }
#pragma unroll
    for (int u = 0; u < VEC; ++u) part[(long)chunk * N + cv * VEC + u] = acc[u];
    return;
  }
  const long col = (long)blockIdx.x * 256 + threadIdx.x;
  if (col >= N) return;
  double acc = 0.0;
  for (long r = r0; r < r1; ++r) acc += (double)R[r * N + col] * (double)w[r];
  part[(long)chunk * N + col] = acc;
}

template <typename T>
__global__ void stored_gemv_sum_kernel(const double* __restrict__ part, long N,
                                       T* __restrict__ y, const T* __restrict__ z, double coef,
                                       const int* __restrict__ flags, int nflags) {
  if (any_flag(flags, nflags)) return;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < N;
       e += (long)gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int ch = 0; ch < kGvChunks; ++ch) v += part[(long)ch * N + e];
    if (z) v -= coef * (double)z[e];
    y[e] = (T)v;
  }
}

long stored_gemv_ws(long N) { return (long)kGvChunks * N; }

template <typename T>
void launch_stored_gemv(const T* R, long N, int transpose, const T* x, T* y, const T* z,
                        double coef, double* ws, hipStream_t s, const int* flags, int nflags) {
  constexpr int VEC = 16 / (int)sizeof(T);
  const bool aligned = N % VEC == 0 && (uintptr_t)R % 16 == 0;
  if (!transpose) {
    const int vec = aligned && (uintptr_t)x % 16 == 0;
    hipLaunchKernelGGL(stored_gemv_rows_kernel<T>, dim3((unsigned)((N + 3) / 4)), dim3(256), 0,
                       s, R, N, x, y, z, coef, vec, flags, nflags);
    return;
  }
  const long ncv = aligned ? N / VEC : N;     // threads along the columns
  hipLaunchKernelGGL(stored_gemv_cols_kernel<T>, dim3((unsigned)((ncv + 255) / 256), kGvChunks),
                     dim3(256), 0, s, R, N, x, ws, (int)aligned, flags, nflags);
  long blocks = (N + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(stored_gemv_sum_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, ws, N,
                     y, z, coef, flags, nflags);
}
template void launch_stored_gemv<float>(const float*, long, int, const float*, float*,
                                        const float*, double, double*, hipStream_t, const int*,
                                        int);
template void launch_stored_gemv<double>(const double*, long, int, const double*, double*,
                                         const double*, double, double*, hipStream_t,
                                         const int*, int);

// out[r + n c] = in[r n + c]: an n x n image (row-major) to its column-major
// vec and back (the same map); skipped when a flag is set.
__global__ void transpose_image_kernel(const double* __restrict__ in, double* __restrict__ out,
                                       int n, const int* __restrict__ flags, int nflags) {
  if (any_flag(flags, nflags)) return;
  __shared__ double tile[32][33];
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int rr = ty; rr < 32; rr += 8) {
    const int r = r0 + rr, c = c0 + tx;
    tile[rr][tx] = (r < n && c < n) ? in[(long)r * n + c] : 0.0;
  }
  __syncthreads();
  for (int cc = ty; cc < 32; cc += 8) {
    const int c = c0 + cc, r = r0 + tx;
    if (r < n && c < n) out[r + (long)n * c] = tile[tx][cc];
  }
}

void launch_transpose_image(const double* in, double* out, int n, const int* flags, int nflags,
                            hipStream_t s) {
  const int t = (n + 31) / 32;
  hipLaunchKernelGGL(transpose_image_kernel, dim3(t, t), dim3(256), 0, s, in, out, n, flags,
                     nflags);
}

// ---------------------------------------------------------------------------
// Y = op(R) X for up to 32 columns on MFMA: a workgroup owns 64 rows of op(R)
// (4 waves x 16 rows, each wave 2 x 16 columns) and streams K in tiles of 64:
// the 64 x 64 tile of op(R) (read along R's rows in both orientations, stored
// k-major in LDS) and the 64 x 32 tile of X. R is read once per product; FP32
// accumulators are flushed into FP64 after every K tile.
template <typename T> struct MfmaT;
template <> struct MfmaT<float> {
  typedef floatx4 acc;
  static __device__ __forceinline__ acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int drow(int lk, int e) { return 4 * lk + e; }
};
template <> struct MfmaT<double> {
  typedef doublex4 acc;
  static __device__ __forceinline__ acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int drow(int lk, int e) { return lk + 4 * e; }
};

constexpr int kSgM = 64, kSgK = 64, kSgAS = kSgM + 1, kSgXS = 32 + 1;

template <typename T>
__global__ void __launch_bounds__(256)
stored_block_kernel(const T* __restrict__ R, long N, int transpose, const T* __restrict__ X,
                    T* __restrict__ Y, int ncols) {
  __shared__ T As[kSgK][kSgAS];   // As[k][m] = op(R)[m0 + m][k0 + k]
  __shared__ T Xs[kSgK][kSgXS];   // Xs[k][col] = X[k0 + k, col]
  typedef typename MfmaT<T>::acc acc_t;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long m0 = (long)blockIdx.x * kSgM;
  const int lrow = lane & 15, lk = lane >> 4;
  acc_t acc[2];
  double accd[2][4];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      acc[cb][e] = (T)0;
      accd[cb][e] = 0.0;
    }
  for (long k0 = 0; k0 < N; k0 += kSgK) {
    // op(R) tile: 64 x 64 elements, 16 per thread, contiguous along R's rows
#pragma unroll 4
    for (int q = 0; q < (kSgM * kSgK) / 256; ++q) {
      const int e = tid + 256 * q;
      const int fast = e & 63, slow = e >> 6;
      T v = (T)0;
      if (!transpose) {            // op(R)[m][k] = R[m0 + slow][k0 + fast]
        const long m = m0 + slow, k = k0 + fast;
        if (m < N && k < N) v = R[m * N + k];
        As[fast][slow] = v;
      } else {                     // op(R)[m][k] = R[k0 + slow][m0 + fast]
        const long k = k0 + slow, m = m0 + fast;
        if (m < N && k < N) v = R[k * N + m];
        As[slow][fast] = v;
      }
    }
#pragma unroll
    for (int q = 0; q < (kSgK * 32) / 256; ++q) {
      const int e = tid + 256 * q;
      const int kk = e & 63, col = e >> 6;
      const long k = k0 + kk;
      Xs[kk][col] = (col < ncols && k < N) ? X[(long)col * N + k] : (T)0;
    }
    __syncthreads();
#pragma unroll
    for (int s4 = 0; s4 < kSgK / 4; ++s4) {
      const int kk = 4 * s4 + lk;
      const T a = As[kk][wave * 16 + lrow];
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) acc[cb] = MfmaT<T>::mma(a, Xs[kk][cb * 16 + lrow], acc[cb]);
    }
    __syncthreads();
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        accd[cb][e] += (double)acc[cb][e];
        acc[cb][e] = (T)0;
      }
  }
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const int col = cb * 16 + lrow;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const long m = m0 + wave * 16 + MfmaT<T>::drow(lk, e);
      if (m < N && col < ncols) Y[(long)col * N + m] = (T)accd[cb][e];
    }
  }
}

template <typename T>
void launch_stored_block(const T* R, long N, int transpose, const T* X, T* Y, int ncols,
                         hipStream_t s) {
  hipLaunchKernelGGL(stored_block_kernel<T>, dim3((unsigned)((N + kSgM - 1) / kSgM)), dim3(256),
                     0, s, R, N, transpose, X, Y, ncols);
}
template void launch_stored_block<float>(const float*, long, int, const float*, float*, int,
                                         hipStream_t);
template void launch_stored_block<double>(const double*, long, int, const double*, double*,
                                          int, hipStream_t);

}  // namespace kpsb
