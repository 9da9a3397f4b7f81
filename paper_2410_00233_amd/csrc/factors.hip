// Kronecker factors from the truncated SVD of R(A) (paper, eq. "KP approx" and
// section "The Cost of forming the terms in KP"): Ax_t = sigma_t array(u_t, n, n),
// Ay_t = array(v_t, n, n), with array() the column-major reshape, written
// row-major. The sign of each pair (u_t, v_t) is fixed so that the entry of v_t
// with the largest magnitude (lowest index on ties) is positive.
#include "common.h"

namespace kpsb {

// block t finds argmax_r |V[r, t]| (lowest r on ties); 1024 threads, four
// loads in flight per thread
template <typename T>
__global__ void __launch_bounds__(1024)
argmax_abs_kernel(const T* __restrict__ V, long ldv, long N, int* __restrict__ out) {
  __shared__ double bv[1024];
  __shared__ long bi[1024];
  const int t = blockIdx.x;
  double best = -1.0;
  long besti = 0;
  for (long r0 = threadIdx.x; r0 < N; r0 += 4 * 1024) {
    double a[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long r = r0 + 1024L * u;
      a[u] = r < N ? fabs((double)V[(long)t * ldv + r]) : -1.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)    // increasing r; strictly greater keeps the lowest
      if (a[u] > best) { best = a[u]; besti = r0 + 1024L * u; }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = besti;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      const double o = bv[threadIdx.x + off];
      const long oi = bi[threadIdx.x + off];
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[t] = (int)bi[0];
}

// Tiled transpose: vec index a + n*b -> row-major [a][b].
template <typename T, typename O>
__global__ void __launch_bounds__(256)
write_factor_kernel(const T* __restrict__ U, const T* __restrict__ V, long ldu, int n,
                    const double* __restrict__ sigma, const int* __restrict__ amax,
                    O* __restrict__ Ax, O* __restrict__ Ay) {
  __shared__ double tu[32][33];
  __shared__ double tv[32][33];
  const int t = blockIdx.z;
  const int a0 = blockIdx.x * 32, b0 = blockIdx.y * 32;
  const long NN = (long)n * n;
  const double vmax = (double)V[(long)t * ldu + amax[t]];
  const double sgn = vmax < 0.0 ? -1.0 : 1.0;
  const double su = sgn * sigma[t];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  // read: consecutive a (vec index a + n b) -> coalesced
  for (int yy = ty; yy < 32; yy += 8) {
    const int a = a0 + tx, b = b0 + yy;
    double u = 0.0, v = 0.0;
    if (a < n && b < n) {
      u = (double)U[(long)t * ldu + a + (long)n * b];
      v = (double)V[(long)t * ldu + a + (long)n * b];
    }
    tu[yy][tx] = u;
    tv[yy][tx] = v;
  }
  __syncthreads();
  // write: consecutive b in row a -> coalesced
  for (int yy = ty; yy < 32; yy += 8) {
    const int a = a0 + yy, b = b0 + tx;
    if (a < n && b < n) {
      Ax[(long)t * NN + (long)a * n + b] = (O)(su * tu[tx][yy]);
      Ay[(long)t * NN + (long)a * n + b] = (O)(sgn * tv[tx][yy]);
    }
  }
}

template <typename T, typename O>
void launch_form_factors(const T* U, const T* V, long ldu, int n, int k, const double* sigma,
                         O* Ax, O* Ay, int* argmax_scratch, hipStream_t s) {
  if (k <= 0) return;
  hipLaunchKernelGGL(argmax_abs_kernel<T>, dim3(k), dim3(1024), 0, s, V, ldu, (long)n * n,
                     argmax_scratch);
  dim3 grid((n + 31) / 32, (n + 31) / 32, k);
  hipLaunchKernelGGL((write_factor_kernel<T, O>), grid, dim3(256), 0, s, U, V, ldu, n, sigma,
                     argmax_scratch, Ax, Ay);
}
template void launch_form_factors<float, float>(const float*, const float*, long, int, int,
                                                const double*, float*, float*, int*,
                                                hipStream_t);
template void launch_form_factors<float, double>(const float*, const float*, long, int, int,
                                                 const double*, double*, double*, int*,
                                                 hipStream_t);
template void launch_form_factors<double, double>(const double*, const double*, long, int, int,
                                                  const double*, double*, double*, int*,
                                                  hipStream_t);
template void launch_form_factors<double, float>(const double*, const double*, long, int, int,
                                                 const double*, float*, float*, int*,
                                                 hipStream_t);

}  // namespace kpsb
