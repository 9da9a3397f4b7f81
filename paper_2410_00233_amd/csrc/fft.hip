// The blur A applied through two-dimensional FFTs: for a spatially invariant
// blur, A x is a convolution of the PSF with the image extended beyond its
// edges by the boundary conditions (the BTTB structure noted in section 1 of
// the paper), so split Bregman can use A itself (the paper's method (i) of
// Table 1) at O(n^2 log n) per product instead of a stored N x N matrix.
//
// With E the extended image (E[e][f] = x at the pixel whose image is
// (e + cu - pu + 1, f + cv - pv + 1), or 0 where there is none: zero boundary
// conditions take the pixel itself, periodic ones the pixel modulo n,
// reflexive ones its reflection about the edge of the last pixel),
//   (A x)[r][i] = sum_{u,v} P[u][v] E[r + pu - 1 - u][i + pv - 1 - v],
// the rows pu - 1 .. pu + n - 2 (columns likewise) of the linear convolution
// P * E, exact in a circular convolution of size M1 x M2 >= (n + pu - 1) x
// (n + pv - 1). A^T y is the adjoint chain: y placed at those rows and
// columns, correlated with P (the conjugate spectrum), and folded back onto
// the pixels (each pixel sums the entries of its images).
//
// Images are n x n FP64, row-major (pixel (r, i) at r n + i: r vertical, the
// PSF's first index u; i horizontal, its second index v). The spectrum S holds
// rows of the row transforms (M2/2 + 1 complex entries each, the real input's
// half spectrum); the column pass works on CB columns at a time in LDS and
// writes back in place. Radix-4 (plus one radix-2 pass for odd log2 M) DIF
// forward and DIT inverse transforms in LDS: the DIF output is in bit-reversed
// order and the spectrum of P is stored in that order, so the product with it
// needs no permutation and the DIT inverse returns natural order.
#include "common.h"

namespace kpsb {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a times -i (forward) or +i (inverse): W_4^1 of the transform's sign
__device__ __forceinline__ double2 mul_w4(double2 a, bool inv) {
  return inv ? double2{-a.y, a.x} : double2{a.y, -a.x};
}

// W_m^p = exp(-+ 2 pi i p / m) from the table tw[j] = exp(-2 pi i j / kFftMaxLen)
__device__ __forceinline__ double2 twid(const double2* __restrict__ tw, int p, int m, bool inv) {
  double2 w = tw[p * (kFftMaxLen / m)];
  if (inv) w.y = -w.y;
  return w;
}

__device__ __forceinline__ bool fft_skip(const int* flags, int nflags) {
  if (flags)
    for (int i = 0; i < nflags; ++i)
      if (flags[i]) return true;
  return false;
}

__device__ __forceinline__ int bitrev(int k, int lg) { return (int)(__brev((unsigned)k) >> (32 - lg)); }

// Decimation in frequency over nb sequences of length L = 2^lg in LDS (buf +
// b L): natural order in, bit-reversed order out. Ends with a barrier.
__device__ void fft_dif(double2* buf, int nb, int lg, const double2* __restrict__ tw, bool inv) {
  const int L = 1 << lg;
  int blk = L;                                   // current block size
  for (; blk >= 4; blk >>= 2) {                  // radix 4: half-sizes blk/2 and blk/4
    const int q = blk >> 2, per = L >> 2;
    for (int t = threadIdx.x; t < nb * per; t += blockDim.x) {
      const int b = t / per, u = t - b * per;
      const int g = u / q, p = u - g * q;
      double2* x = buf + b * L + g * blk + p;
      const double2 a0 = x[0], a1 = x[q], a2 = x[2 * q], a3 = x[3 * q];
      const double2 w = twid(tw, p, blk, inv);                   // W_{4q}^p
      const double2 s0 = cadd(a0, a2), d0 = cmul(csub(a0, a2), w);
      const double2 s1 = cadd(a1, a3), d1 = cmul(mul_w4(csub(a1, a3), inv), w);  // W_{4q}^{p+q}
      const double2 w2 = cmul(w, w);                             // W_{2q}^p
      x[0] = cadd(s0, s1);
      x[q] = cmul(csub(s0, s1), w2);
      x[2 * q] = cadd(d0, d1);
      x[3 * q] = cmul(csub(d0, d1), w2);
    }
    __syncthreads();
  }
  if (blk == 2) {                                // odd lg: the last stage, half-size 1
    const int per = L >> 1;
    for (int t = threadIdx.x; t < nb * per; t += blockDim.x) {
      const int b = t / per, u = t - b * per;
      double2* x = buf + b * L + 2 * u;
      const double2 a0 = x[0], a1 = x[1];
      x[0] = cadd(a0, a1);
      x[1] = csub(a0, a1);
    }
    __syncthreads();
  }
}

// Decimation in time: bit-reversed order in, natural order out. Ends with a
// barrier.
__device__ void fft_dit(double2* buf, int nb, int lg, const double2* __restrict__ tw, bool inv) {
  const int L = 1 << lg;
  int blk = 1;
  if (lg & 1) {                                  // odd lg: the first stage, half-size 1
    const int per = L >> 1;
    for (int t = threadIdx.x; t < nb * per; t += blockDim.x) {
      const int b = t / per, u = t - b * per;
      double2* x = buf + b * L + 2 * u;
      const double2 a0 = x[0], a1 = x[1];
      x[0] = cadd(a0, a1);
      x[1] = csub(a0, a1);
    }
    __syncthreads();
    blk = 2;
  }
  for (; blk < L; blk <<= 2) {                   // radix 4: half-sizes q = blk, then 2q
    const int q = blk, per = L >> 2;
    for (int t = threadIdx.x; t < nb * per; t += blockDim.x) {
      const int b = t / per, u = t - b * per;
      const int g = u / q, p = u - g * q;
      double2* x = buf + b * L + g * 4 * q + p;
      const double2 a0 = x[0], a1 = x[q], a2 = x[2 * q], a3 = x[3 * q];
      const double2 w = twid(tw, p, 4 * q, inv);                 // W_{4q}^p
      const double2 w2 = cmul(w, w);                             // W_{2q}^p
      const double2 t1 = cmul(a1, w2), t3 = cmul(a3, w2);
      const double2 s0 = cadd(a0, t1), s1 = csub(a0, t1);
      const double2 d0 = cmul(cadd(a2, t3), w);
      const double2 d1 = cmul(mul_w4(csub(a2, t3), inv), w);     // W_{4q}^{p+q}
      x[0] = cadd(s0, d0);
      x[2 * q] = csub(s0, d0);
      x[q] = cadd(s1, d1);
      x[3 * q] = csub(s1, d1);
    }
    __syncthreads();
  }
}

// The pixel whose image is the extended coordinate ct (-1: none), per the
// boundary conditions.
__device__ __forceinline__ int ext_source(int bc, int ct, int n) {
  if (bc == 1) {                                 // reflexive: period 2n, mirrored half
    int t = ct % (2 * n);
    if (t < 0) t += 2 * n;
    return t < n ? t : 2 * n - 1 - t;
  }
  if (bc == 2) {                                 // periodic
    int t = ct % n;
    return t < 0 ? t + n : t;
  }
  return (ct >= 0 && ct < n) ? ct : -1;
}

__global__ void fft_twiddle_kernel(double2* tw) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= kFftMaxLen) return;
  double sn, cs;
  sincospi(2.0 * (double)j / (double)kFftMaxLen, &sn, &cs);
  tw[j] = {cs, -sn};
}

// Row transforms of row pairs (a + i b packed into one complex transform,
// separated by the Hermitian symmetry of real input). mode 0: rows of the
// extended image of `src` (rows r0 .. r0 + nrows - 1 of E); 1: the n x n
// image `src` placed at rows and columns pu - 1 .. (the adjoint of the crop);
// 2: the PSF at the origin. Writes S rows r0 .. r0 + nrows - 1.
__global__ void __launch_bounds__(1024)
fft_rows_fwd_kernel(FftConv p, int mode, const double* __restrict__ src, int r0, int nrows,
                    const int* __restrict__ flags, int nflags) {
  if (fft_skip(flags, nflags)) return;
  extern __shared__ double2 sbuf[];
  const int M = 1 << p.l2, RP = p.rp;
  const int pair0 = blockIdx.x * RP;
  for (int idx = threadIdx.x; idx < RP * M; idx += blockDim.x) {
    const int j = idx >> p.l2, t = idx & (M - 1);
    const int ra = r0 + 2 * (pair0 + j);
    double v[2] = {0.0, 0.0};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int row = ra + h;
      if (row >= r0 + nrows) continue;
      if (mode == 0) {
        if (t < p.e2) {
          const int sr = ext_source(p.bc, row + p.cu - p.pu + 1, p.n);
          const int sc = ext_source(p.bc, t + p.cv - p.pv + 1, p.n);
          if (sr >= 0 && sc >= 0) v[h] = src[(long)sr * p.n + sc];
        }
      } else if (mode == 1) {
        const int rr = row - (p.pu - 1), cc = t - (p.pv - 1);
        if (rr >= 0 && rr < p.n && cc >= 0 && cc < p.n) v[h] = src[(long)rr * p.n + cc];
      } else {
        if (row < p.pu && t < p.pv) v[h] = src[(long)row * p.pv + t];
      }
    }
    sbuf[idx] = {v[0], v[1]};
  }
  __syncthreads();
  fft_dif(sbuf, RP, p.l2, p.tw, false);
  const int h2 = (M >> 1) + 1;
  for (int idx = threadIdx.x; idx < RP * h2; idx += blockDim.x) {
    const int j = idx / h2, k = idx - j * h2;
    const int ra = r0 + 2 * (pair0 + j);
    if (ra >= r0 + nrows) continue;
    const double2 zk = sbuf[j * M + bitrev(k, p.l2)];
    const double2 zm = sbuf[j * M + bitrev((M - k) & (M - 1), p.l2)];
    p.S[(long)ra * p.ls + k] = {0.5 * (zk.x + zm.x), 0.5 * (zk.y - zm.y)};
    if (ra + 1 < r0 + nrows) p.S[(long)(ra + 1) * p.ls + k] = {0.5 * (zk.y + zm.y), 0.5 * (zm.x - zk.x)};
  }
}

// Column transforms of CB columns per workgroup: rows rin0 .. rin1 - 1 of S in
// (the others zero), forward transform; mode 2 stores it as the PSF spectrum
// H (bit-reversed order, column-major: H[k M1 + pos]); modes 0 / 1 multiply by
// H / conj(H), transform back and write rows rout0 .. rout1 - 1 of S.
__global__ void __launch_bounds__(1024)
fft_cols_kernel(FftConv p, int mode, int rin0, int rin1, int rout0, int rout1,
                const int* __restrict__ flags, int nflags) {
  if (fft_skip(flags, nflags)) return;
  extern __shared__ double2 sbuf[];
  const int M = 1 << p.l1, CB = p.cb;
  const int h2 = ((1 << p.l2) >> 1) + 1;
  // Workgroups go to the 8 XCDs round-robin by id, while the CB columns of a
  // workgroup fill only part of each 128-byte line of S: give each XCD a
  // contiguous range of column groups, so the groups that share a line meet
  // in one L2 (the tail beyond a multiple of 8 keeps its order).
  const int per = gridDim.x >> 3;
  const int bid = blockIdx.x;
  const int grp = bid < (per << 3) ? (bid & 7) * per + (bid >> 3) : bid;
  const int k0 = grp * CB;
  for (int idx = threadIdx.x; idx < CB * M; idx += blockDim.x) {
    const int b = idx % CB, q = idx / CB;
    double2 v = {0.0, 0.0};
    if (q >= rin0 && q < rin1 && k0 + b < h2) v = p.S[(long)q * p.ls + k0 + b];
    sbuf[b * M + q] = v;
  }
  __syncthreads();
  fft_dif(sbuf, CB, p.l1, p.tw, false);
  if (mode == 2) {
    for (int idx = threadIdx.x; idx < CB * M; idx += blockDim.x) {
      const int b = idx >> p.l1, pos = idx & (M - 1);
      if (k0 + b < h2) p.H[(long)(k0 + b) * M + pos] = sbuf[idx];
    }
    return;
  }
  for (int idx = threadIdx.x; idx < CB * M; idx += blockDim.x) {
    const int b = idx >> p.l1, pos = idx & (M - 1);
    if (k0 + b >= h2) continue;
    double2 hv = p.H[(long)(k0 + b) * M + pos];
    if (mode == 1) hv.y = -hv.y;
    sbuf[idx] = cmul(sbuf[idx], hv);
  }
  __syncthreads();
  fft_dit(sbuf, CB, p.l1, p.tw, true);
  for (int idx = threadIdx.x; idx < CB * M; idx += blockDim.x) {
    const int b = idx % CB, q = idx / CB;
    if (q >= rout0 && q < rout1 && k0 + b < h2) p.S[(long)q * p.ls + k0 + b] = sbuf[b * M + q];
  }
}

// Inverse row transforms of row pairs of S (rows r0 .. r0 + nrows - 1), scaled
// by 1 / (M1 M2). mode 0: out[(row - o1) n + (t - o2)] for the rows and
// columns that land in the n x n image; 1: out[row e2 + t], t < e2 (the
// correlation on the extended grid, folded afterwards).
__global__ void __launch_bounds__(1024)
fft_rows_inv_kernel(FftConv p, int mode, int r0, int nrows, int o1, int o2,
                    double* __restrict__ out, const int* __restrict__ flags, int nflags) {
  if (fft_skip(flags, nflags)) return;
  extern __shared__ double2 sbuf[];
  const int M = 1 << p.l2, RP = p.rp, h2 = (M >> 1) + 1;
  const int pair0 = blockIdx.x * RP;
  for (int idx = threadIdx.x; idx < RP * M; idx += blockDim.x) {
    const int j = idx >> p.l2, k = idx & (M - 1);
    const int ra = r0 + 2 * (pair0 + j);
    double2 xa = {0.0, 0.0}, xb = {0.0, 0.0};
    if (ra < r0 + nrows) {
      const bool lo = k < h2;
      const int kk = lo ? k : M - k;
      xa = p.S[(long)ra * p.ls + kk];
      if (ra + 1 < r0 + nrows) xb = p.S[(long)(ra + 1) * p.ls + kk];
      if (!lo) {
        xa.y = -xa.y;
        xb.y = -xb.y;
      }
    }
    sbuf[j * M + bitrev(k, p.l2)] = {xa.x - xb.y, xa.y + xb.x};
  }
  __syncthreads();
  fft_dit(sbuf, RP, p.l2, p.tw, true);
  const double scale = 1.0 / ((double)(1 << p.l1) * (double)M);
  for (int idx = threadIdx.x; idx < RP * M; idx += blockDim.x) {
    const int j = idx >> p.l2, t = idx & (M - 1);
    const int ra = r0 + 2 * (pair0 + j);
    const double2 z = sbuf[idx];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int row = ra + h;
      if (row >= r0 + nrows) continue;
      const double v = (h ? z.y : z.x) * scale;
      if (mode == 0) {
        const int rr = row - o1, cc = t - o2;
        if (rr >= 0 && rr < p.n && cc >= 0 && cc < p.n) out[(long)rr * p.n + cc] = v;
      } else if (t < p.e2) {
        out[(long)row * p.e2 + t] = v;
      }
    }
  }
}

// Extended coordinates (offset so that 0 is the first extended index) whose
// source pixel is r: its images within [0, ext). At most 14 (reflexive, PSFs
// reaching <= 2n pixels from their centre).
__device__ __forceinline__ int ext_images(int bc, int r, int n, int shift, int ext, int* out) {
  int cnt = 0;
  if (bc == 0) {
    const int e = r + shift;
    if (e >= 0 && e < ext) out[cnt++] = e;
    return cnt;
  }
  for (int m = -3; m <= 3; ++m) {
    if (bc == 2) {
      const int e = r + n * m + shift;
      if (e >= 0 && e < ext) out[cnt++] = e;
    } else {
      const int e1 = r + 2 * n * m + shift, e2 = -1 - r + 2 * n * m + shift;
      if (e1 >= 0 && e1 < ext) out[cnt++] = e1;
      if (e2 >= 0 && e2 < ext) out[cnt++] = e2;
    }
  }
  return cnt;
}

// x[r][c] = sum over the extended entries G[e][f] whose source pixel is (r, c).
__global__ void __launch_bounds__(256)
fft_fold_kernel(FftConv p, const double* __restrict__ G, double* __restrict__ x,
                const int* __restrict__ flags, int nflags) {
  if (fft_skip(flags, nflags)) return;
  const long NN = (long)p.n * p.n;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= NN) return;
  const int r = (int)(idx / p.n), c = (int)(idx - (long)r * p.n);
  int er[16], ec[16];
  const int nr = ext_images(p.bc, r, p.n, p.pu - 1 - p.cu, p.e1, er);
  const int nc = ext_images(p.bc, c, p.n, p.pv - 1 - p.cv, p.e2, ec);
  double s = 0.0;
  for (int a = 0; a < nr; ++a)
    for (int b = 0; b < nc; ++b) s += G[(long)er[a] * p.e2 + ec[b]];
  x[idx] = s;
}

static size_t rows_lds(const FftConv& p) { return (size_t)p.rp * (1u << p.l2) * sizeof(double2); }
// Threads per workgroup of a pass over sequences of length 2^lg: from 1024
// entries up a workgroup holds one sequence, and more threads per sequence
// shorten each stage between barriers (n = 512, length 2048: 256 threads ran
// the CGLS iteration through FFTs in 168 us, 512 in 149, 1024 in 158; length
// 4096: A X 0.48 / 0.41 / 0.39 ms).
static int fft_threads(int lg) { return lg >= 12 ? 1024 : lg >= 10 ? 512 : 256; }
static size_t cols_lds(const FftConv& p) { return (size_t)p.cb * (1u << p.l1) * sizeof(double2); }

void fft_set_lds_limits() {
  static const bool once = [] {
    (void)hipFuncSetAttribute((const void*)fft_cols_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
    (void)hipFuncSetAttribute((const void*)fft_rows_fwd_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024);
    (void)hipFuncSetAttribute((const void*)fft_rows_inv_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024);
    return true;
  }();
  (void)once;
}

void launch_fft_twiddles(double2* tw, hipStream_t s) {
  fft_twiddle_kernel<<<(kFftMaxLen + 255) / 256, 256, 0, s>>>(tw);
}

void launch_fft_psf_spectrum(const FftConv& p, const double* psf, hipStream_t s) {
  const int pairs = (p.pu + 1) / 2;
  const int h2 = ((1 << p.l2) >> 1) + 1;
  fft_rows_fwd_kernel<<<(pairs + p.rp - 1) / p.rp, fft_threads(p.l2), rows_lds(p), s>>>(p, 2, psf, 0, p.pu,
                                                                          nullptr, 0);
  fft_cols_kernel<<<(h2 + p.cb - 1) / p.cb, fft_threads(p.l1), cols_lds(p), s>>>(p, 2, 0, p.pu, 0, 0, nullptr, 0);
}

void launch_fft_conv(const FftConv& p, int transpose, const double* X, double* Y,
                     const int* flags, int nflags, hipStream_t s) {
  const int h2 = ((1 << p.l2) >> 1) + 1;
  const int cgrid = (h2 + p.cb - 1) / p.cb;
  const int n = p.n;
  auto rgrid = [&](int rows) { return ((rows + 1) / 2 + p.rp - 1) / p.rp; };
  if (!transpose) {
    fft_rows_fwd_kernel<<<rgrid(p.e1), fft_threads(p.l2), rows_lds(p), s>>>(p, 0, X, 0, p.e1, flags, nflags);
    fft_cols_kernel<<<cgrid, fft_threads(p.l1), cols_lds(p), s>>>(p, 0, 0, p.e1, p.pu - 1, p.pu - 1 + n, flags,
                                                    nflags);
    fft_rows_inv_kernel<<<rgrid(n), fft_threads(p.l2), rows_lds(p), s>>>(p, 0, p.pu - 1, n, p.pu - 1, p.pv - 1,
                                                           Y, flags, nflags);
    return;
  }
  fft_rows_fwd_kernel<<<rgrid(n), fft_threads(p.l2), rows_lds(p), s>>>(p, 1, X, p.pu - 1, n, flags, nflags);
  if (p.bc == 0) {   // one image per pixel: the fold is the crop at the centre's offset
    const int o1 = p.pu - 1 - p.cu, o2 = p.pv - 1 - p.cv;
    fft_cols_kernel<<<cgrid, fft_threads(p.l1), cols_lds(p), s>>>(p, 1, p.pu - 1, p.pu - 1 + n, o1, o1 + n, flags,
                                                    nflags);
    fft_rows_inv_kernel<<<rgrid(n), fft_threads(p.l2), rows_lds(p), s>>>(p, 0, o1, n, o1, o2, Y, flags, nflags);
    return;
  }
  fft_cols_kernel<<<cgrid, fft_threads(p.l1), cols_lds(p), s>>>(p, 1, p.pu - 1, p.pu - 1 + n, 0, p.e1, flags,
                                                  nflags);
  fft_rows_inv_kernel<<<rgrid(p.e1), fft_threads(p.l2), rows_lds(p), s>>>(p, 1, 0, p.e1, 0, 0, p.G, flags,
                                                            nflags);
  const long NN = (long)n * n;
  fft_fold_kernel<<<(unsigned)((NN + 255) / 256), 256, 0, s>>>(p, p.G, Y, flags, nflags);
}

}  // namespace kpsb
