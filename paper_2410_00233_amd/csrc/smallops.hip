// Tiny single-workgroup helpers used between the Gram-Schmidt passes and the
// small SVDs (bookkeeping of the triangular factor, transposes).
#include "common.h"

namespace kpsb {

// out (nc x m, ld nc) = in^T (in: m x nc, ld m)
__global__ void transpose_small_kernel(const double* __restrict__ in, int m, int nc,
                                       double* __restrict__ out) {
  for (int e = threadIdx.x; e < m * nc; e += blockDim.x) {
    const int r = e % m, c = e / m;
    out[c + (long)nc * r] = in[e];
  }
}
void launch_transpose_small(const double* in, int m, int nc, double* out, hipStream_t s) {
  hipLaunchKernelGGL(transpose_small_kernel, dim3(1), dim3(256), 0, s, in, m, nc, out);
}

// fill a small FP64 array
__global__ void fill_small_kernel(double* __restrict__ p, int m, double v) {
  for (int e = threadIdx.x; e < m; e += blockDim.x) p[e] = v;
}
void launch_fill_small(double* p, int m, double v, hipStream_t s) {
  hipLaunchKernelGGL(fill_small_kernel, dim3(1), dim3(256), 0, s, p, m, v);
}

void launch_fill_int(int* p, int n, int v, hipStream_t s);

// *flag |= 1 if any entry of p is NaN or infinite (caller zeroes *flag first)
__global__ void count_nonfinite_kernel(const double* __restrict__ p, long n, int* __restrict__ flag) {
  int mine = 0;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n;
       e += (long)gridDim.x * blockDim.x)
    if (!isfinite(p[e])) mine = 1;
  if (__any(mine) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}
void launch_count_nonfinite(const double* p, long n, int* flag, hipStream_t s) {
  launch_fill_int(flag, 1, 0, s);
  long blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(count_nonfinite_kernel, dim3((int)blocks), dim3(256), 0, s, p, n, flag);
}

// grid-stride fills (graph-capture safe, unlike memset nodes)
__global__ void fill_kernel(double* __restrict__ p, long n, double v) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n;
       e += (long)gridDim.x * blockDim.x)
    p[e] = v;
}
void launch_fill(double* p, long n, double v, hipStream_t s) {
  long blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(fill_kernel, dim3((int)blocks), dim3(256), 0, s, p, n, v);
}
__global__ void fill_int_kernel(int* __restrict__ p, int n, int v) {
  for (int e = threadIdx.x; e < n; e += blockDim.x) p[e] = v;
}
void launch_fill_int(int* p, int n, int v, hipStream_t s) {
  hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, s, p, n, v);
}

}  // namespace kpsb
