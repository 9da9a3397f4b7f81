// Internal declarations shared by the HIP kernels and the host drivers.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <functional>
#include <string>

namespace kpsb {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// Number of partial sums written by the reduction kernels (fixed, so that
// every reduction adds in the same order on every call: deterministic).
constexpr int kRedBlocks = 256;
constexpr int kRedThreads = 256;

// Offset grid of the PSF in the order R(A) uses it:
//   G[a][b] = P[cu + (b - (n-1)), cv + (a - (n-1))],  a, b in [0, 2n-1),
// so that R[i + n*j, r + n*c] = G[i - j + n - 1][r - c + n - 1]. The grid of
// R(A)^T is G^T (the blur with PSF P^T and swapped centre).
//
// Boundary conditions other than zero add the PSF at shifted offsets: the grid
// of a term is G[a][b] = sum over s1 in sv, s2 in su of
// P[cu + (b - (n-1)) + s2, cv + (a - (n-1)) + s1] (periodic: shifts n m,
// m = -2..2, in both dimensions; reflexive: the even shifts 2n m or the odd
// shifts n - 2n m, m = -1..1, per dimension; RmatTerms in api.cpp lists them).
struct GridShifts {
  int nv = 1, nu = 1;
  int sv[5] = {0, 0, 0, 0, 0};
  int su[5] = {0, 0, 0, 0, 0};
};
// G: ldg x ldg, ldg = grid_ld(n); the entries of rows or columns beyond 2n - 1
// are zero (so the grid may also be read column by column past its edge).
template <typename T>
void launch_build_grid(const double* psf, int pu, int pv, int cu, int cv, int n,
                       int transpose, const GridShifts& sh, T* G, int ldg, hipStream_t s);
// out = in with the block index b of each length-n^2 column reversed
// (entry a + n b <- a + n (n-1-b)); Y = (Y + T1) + flip(T2 + T3) entrywise.
template <typename T>
void launch_flip_blocks(const T* in, T* out, int n, long ld, int ncols, hipStream_t s);
template <typename T>
void launch_combine_terms(T* Y, const T* T1, const T* T2, const T* T3, int n, long ld, int ncols,
                          hipStream_t s);

// ---- generated-tile products (rmat_block.hip / rmat_gemv.hip) --------------
struct BlockPlan {
  int TJ;      // j-blocks (16 rows each) per workgroup
  int CP = 0;  // column blocks per slab phase (FP32/FP64 block product)
  int SW;      // LDS slab row stride (elements)
  size_t lds;  // dynamic LDS bytes
  int grid;    // workgroups
  int waves = 0;       // waves per workgroup (0: the default for TJ)
  int TK = 64;         // K-tile entries (FP32/FP64 block product: 64, 128, 176 or 192)
  int grid_limit = 0;  // > 0: launch only the first grid_limit workgroups (tuning samples)
};
// One product of a persistent block launch (launch_rmat_block_persistent): the
// arguments of launch_rmat_block for op(R) X of one problem (up to 32 columns),
// its tile count (grid of its own plan) and the index of its first tile in the
// launch's list.
struct BlockJob {
  const void* G;
  const void* X;
  void* Y;
  long ldx, ldy;
  int ldg, n, ncols, SW, CP, tiles, first, pad;
};
template <typename T>
bool plan_block(int n, size_t lds_limit, BlockPlan* plan);
// The plan with exactly TJ row blocks per workgroup (false if it cannot fit).
template <typename T>
bool plan_block_tj(int n, size_t lds_limit, int TJ, BlockPlan* plan, int TK = 64);
// box (device, optional): the support box of G from launch_grid_box; tiles
// outside it are skipped (same result for finite X).
template <typename T>
void launch_rmat_block(const BlockPlan& plan, const T* G, int ldg, int n, const T* X,
                       long ldx, T* Y, long ldy, int ncols, hipStream_t s,
                       const int* box = nullptr);
// box = {a_lo, a_hi, b_lo, b_hi}: the rows and columns of G holding its nonzero
// entries (a_lo > a_hi for an all-zero grid); part: grid_box_parts() ints.
template <typename T>
void launch_grid_box(const T* G, int ldg, int n, int* part, int* box, hipStream_t s);
int grid_box_parts();

// 16-bit-input variant (H = __hip_bfloat16 or __half): 16-bit grid and X,
// FP32 accumulation, FP32 output. X16 is the pre-shifted 16-bit copy made by
// launch_to16_shifted, x16_column_len(n) elements per column.
bool plan_block16(int n, size_t lds_limit, BlockPlan* plan);
bool plan_block16_tj(int n, size_t lds_limit, int TJ, BlockPlan* plan);
// inv_scale (device, may be null) multiplies the result (undoes power-of-2
// operand scaling); accumulate != 0 adds the result into Y. fold: the FP32
// partial sums go into FP64 accumulators once per column block of R (the
// split-FP16 product, which must keep FP32-level accuracy); otherwise the
// MFMA's FP32 accumulator takes the whole sum.
template <typename H>
void launch_rmat_block16(const BlockPlan& plan, const H* G16, int ldg, int n, const H* X16,
                         long ldx, float* Y, long ldy, int ncols, hipStream_t s,
                         const double* inv_scale = nullptr, int accumulate = 0, bool fold = false);

// Split FP16 operands of the refinement product (FP32-level accuracy from three
// FP16 products): X scaled by 2^kSplitXExp into hi + lo; the grid scaled by a
// power of two computed on the device (launch_psf_split_scale) into hi + lo.
constexpr int kSplitXExp = 11;
void launch_to16_split(const float* in, long ldx, int n, int ncols, __half* hi, __half* lo,
                       long ldo, hipStream_t s);
// scal[0] = 2^e with e the largest integer such that m * 2^e <= 1024, where m
// bounds every grid entry (max|P| when nsum = 1; min(nsum max|P|, sum|P|) for
// grids summing up to nsum PSF entries); scal[1] = 1 / (scal[0] * 2^kSplitXExp).
// scal holds psf_split_scale_len() doubles (the rest: partial maxima and sums).
// Device only, no host sync.
void launch_psf_split_scale(const double* psf, long count, int nsum, double* scal,
                            hipStream_t s);
int psf_split_scale_len();
// FP16 grid of the scaled PSF: part 0 = fp16(G s), part 1 = fp16(G s - part 0).
void launch_build_grid_split(const double* psf, int pu, int pv, int cu, int cv, int n,
                             int transpose, const GridShifts& sh, const double* scal, int part,
                             __half* G, int ldg, hipStream_t s);
long x16_column_len(int n);
template <typename H>
void launch_to16_shifted(const float* in, long ldx, int n, int ncols, H* out, long ldo,
                         hipStream_t s);

// Grid row stride for n: the 2n - 1 entries of a row plus at least 48 zero
// columns (read by the scalar-x matrix-vector kernel), a multiple of 8.
inline int grid_ld(int n) { return ((2 * n - 1 + 48) + 7) & ~7; }

// FP32 y = R x - coef * z with x in scalar registers; xt is workspace of
// gemv_sx_xt_len(n) floats. GT is the TRANSPOSE of the grid of R (entry (a, b)
// at GT[b * ldg + a]), ldg x ldg with ldg = grid_ld(n) (launch_build_grid).
long gemv_sx_xt_len(int n);
void launch_rmat_gemv_sx(const float* G, int ldg, int n, const float* x, float* xt, float* y,
                         const float* z, double coef, hipStream_t s, const int* box = nullptr);

template <typename T>
bool plan_gemv(int n, size_t lds_limit, BlockPlan* plan);
// y = R x - coef * z   (z may be null)
template <typename T>
void launch_rmat_gemv(const BlockPlan& plan, const T* G, int ldg, int n, const T* x,
                      T* y, const T* z, double coef, hipStream_t s);

// ---- explicit-matrix path (stored.hip) --------------------------------------
// A (N x N row-major) of the blur with PSF psf (device) and boundary
// conditions bc (0 zero, 1 reflexive)
template <typename T>
void launch_blur_matrix(const double* psf, int pu, int pv, int cu, int cv, int n, int bc, T* A,
                        hipStream_t s);
// R[i + n j, r + n c] = A[r + n i, c + n j] (A, R row-major N x N, N = n^2)
template <typename T>
void launch_reorder(const T* A, T* R, int n, hipStream_t s);
// y = op(R) x - coef z (op = R or R^T); ws: stored_gemv_ws(N) doubles
long stored_gemv_ws(long N);
template <typename T>
void launch_stored_gemv(const T* R, long N, int transpose, const T* x, T* y, const T* z,
                        double coef, double* ws, hipStream_t s, const int* flags = nullptr,
                        int nflags = 0);
// out[r + n c] = in[r n + c] (row-major image <-> column-major vec); skipped
// when any of flags[0..nflags) is set
void launch_transpose_image(const double* in, double* out, int n, const int* flags, int nflags,
                            hipStream_t s);
// Y = op(R) X, X and Y column-major N x ncols (ncols <= 32)
template <typename T>
void launch_stored_block(const T* R, long N, int transpose, const T* X, T* Y, int ncols,
                         hipStream_t s);

// All jobs' tiles in one launch of `grid` workgroups, each taking tiles from
// *counter (reset to 0 here, on the stream) until none is left. The launch shape
// (TJ, waves, TK of `shape`) is shared by the jobs; each job's SW / CP come from
// its own plan with that shape; lds: the largest job's dynamic LDS. jobs and
// counter: device memory.
void launch_rmat_block_persistent(const BlockPlan& shape, const BlockJob* jobs, int njobs,
                                  int total, int* counter, size_t lds, int grid, hipStream_t s);

// ---- autotuner (tune.cpp) ---------------------------------------------------
constexpr int kTuneBlock = 1;     // FP32 / FP64 block product: (TJ, waves)
constexpr int kTuneBlock16 = 2;   // 16-bit block product: TJ
constexpr int kTuneApply = 3;     // FP64 Kronecker apply GEMMs: (tile, K tile)
bool tune_enabled();   // KPSB_AUTOTUNE=0 keeps every operation at its variant 0
// Average ms of `reps` launches after one warm-up (hipEvents on s; synchronizes).
double time_launches(hipStream_t s, int reps, const std::function<void()>& launch);
// The variant of (op, n, a, b) to use: on first use, cost(v) is evaluated for
// every v < ncand (negative = not applicable) and the cheapest is kept.
int tune_pick(int op, int n, int a, int b, int ncand, const std::function<double(int)>& cost);
// Whether (op, n, a, b) on the current device has its variant chosen already
// (true when autotuning is off).
bool tune_known(int op, int n, int a, int b);
std::string tune_table();   // JSON list of the choices and measured costs
// While set on the calling thread, tune_pick times nothing: it returns the
// variant already chosen for the key, else variant 0 (without recording it).
void tune_set_no_timing(bool on);

// ---- static device scratch (noalloc.hip) -----------------------------------
size_t scratch_capacity();   // bytes
// Device address of `device`'s copy of the scratch array (call with that device
// current); looked up once per device, then cached.
hipError_t scratch_address(int device, void** out);

// ---- vector kernels (blas1.hip) --------------------------------------------
// partials[b * m + i] = sum over rows of block b of V[:, i] . w  (FP64 accum)
template <typename T>
// Kernels taking `pred` do nothing when pred != nullptr and *pred == 0 (device-side
// predication of data-dependent branches, no host synchronization).
void launch_multidot(const T* V, long ldv, int m, const T* w, long N, double* partials,
                     hipStream_t s, const int* pred = nullptr);
// h[i] (+)= sum_b partials[b*m + i]; if accumulate != 0 adds into h
void launch_reduce_partials(const double* partials, int m, double* h, int accumulate,
                            hipStream_t s, const int* pred = nullptr);
// w -= V h (m columns) with h = the sums of the launch_multidot partials
// (layout [block][m]), formed in every block; block 0 stores h in h_out and/or
// adds it into h_add (either may be NULL). Replaces a reduce_partials launch
// before the projection.
template <typename T>
void launch_project_out_red(T* w, const T* V, long ldv, int m, const double* partials,
                            double* h_out, double* h_add, long N, double* nrm_partials,
                            hipStream_t s, const int* pred = nullptr);
// nrm_partials[b] = block partial of ||w||^2
template <typename T>
void launch_norm2_partials(const T* w, long N, double* nrm_partials, hipStream_t s);
template <typename T>
void launch_scale(T* w, long N, double factor, hipStream_t s);
// out[e] = Philox normal number e of (seed, stream)
template <typename T>
void launch_philox_normals(T* out, long N, uint64_t seed, uint32_t stream_id,
                           hipStream_t s, const int* pred = nullptr);
template <typename S, typename D>
void launch_convert(const S* in, D* out, long N, hipStream_t s);
// out = V * C (V: N x m column-major ld ldv; C: m x k column-major FP64, ld ldc)
template <typename T, typename O>
void launch_small_gemm(const T* V, long ldv, int m, const double* C, int ldc, int k,
                       long N, O* out, long ldo, hipStream_t s);

// ---- single-workgroup helpers (smallops.hip) ---------------------------------
void launch_transpose_small(const double* in, int m, int nc, double* out, hipStream_t s);
// Householder TSQR of a tall N x m block (tsqr.hip): W <- Q with orthonormal
// columns and, if Rfac != NULL, Rfac <- R (m x m column-major, non-negative
// diagonal), W = Q R. Needs 1 <= m <= 64 and N >= m (else returns false and
// launches nothing); ws holds tsqr_workspace_bytes(N, m) bytes.
size_t tsqr_workspace_bytes(long N, int m);
template <typename T>
bool launch_tsqr(T* W, long N, int m, double* Rfac, void* ws, hipStream_t s);
void launch_fill_small(double* p, int m, double v, hipStream_t s);
void launch_fill(double* p, long n, double v, hipStream_t s);
void launch_fill_int(int* p, int n, int v, hipStream_t s);
void launch_count_nonfinite(const double* p, long n, int* flag, hipStream_t s);

// ---- small dense SVD (jacobi.hip) ------------------------------------------
// One-sided Jacobi SVD of an m x nc FP64 matrix (m >= nc, column-major, ld m,
// m <= 64, nc <= 64): U (m x nc), sig (nc, descending), V (nc x nc).
void launch_jacobi_svd(const double* A, int m, int nc, double* U, double* sig,
                       double* V, int* sweeps, hipStream_t s);

// ---- Kronecker factors (factors.hip) ---------------------------------------
// For t < k: find the index of the largest |v_t| (lowest on ties), then write
// Ax_t = sgn * sigma_t * array(u_t) and Ay_t = sgn * array(v_t) row-major.
template <typename T, typename O>
void launch_form_factors(const T* U, const T* V, long ldu, int n, int k,
                         const double* sigma, O* Ax, O* Ay, int* argmax_scratch,
                         hipStream_t s);

// ---- the blur through two-dimensional FFTs (fft.hip) -----------------------
// A x and A^T y of a spatially invariant blur with its boundary conditions as
// a circular convolution of size M1 x M2 (powers of two, 8 .. kFftMaxLen) of
// the extended image; fields set by fft_conv_plan in api.cpp.
constexpr int kFftMaxLen = 4096;
struct FftConv {
  int n, pu, pv, cu, cv, bc;
  int e1, e2;        // extended extents n + pu - 1, n + pv - 1
  int l1, l2;        // log2 M1, log2 M2
  int ls;            // row stride of S (complex entries), >= M2 / 2 + 1
  int rp;            // row pairs per workgroup of the row passes
  int cb;            // columns per workgroup of the column pass
  const double2* tw; // exp(-2 pi i j / kFftMaxLen), j < kFftMaxLen
  double2* S;        // e1 x ls: half spectra of the row transforms
  double2* H;        // (M2 / 2 + 1) x M1: spectrum of P, bit-reversed columns
  double* G;         // e1 x e2 (adjoint with non-zero boundary conditions)
};
void launch_fft_twiddles(double2* tw, hipStream_t s);
// H from the device PSF (pu x pv row-major); uses S.
void launch_fft_psf_spectrum(const FftConv& p, const double* psf, hipStream_t s);
// Y = A X (transpose 0) or A^T X, n x n row-major images; skipped when any of
// flags[0..nflags) is nonzero. Uses S (and G).
void launch_fft_conv(const FftConv& p, int transpose, const double* X, double* Y,
                     const int* flags, int nflags, hipStream_t s);
// the column pass's dynamic LDS above 64 KB (once per process)
void fft_set_lds_limits();

}  // namespace kpsb
