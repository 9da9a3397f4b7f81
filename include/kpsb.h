/*
 * kpsb.h -- C ABI of libkpsb.so: Kronecker-product SVD of the rearranged blur
 * matrix R(A) and split Bregman deblurring on AMD Instinct MI355X (gfx950).
 *
 * Method: Alsubhi & Renaut, "Split Bregman isotropic and anisotropic image
 * deblurring with Kronecker product sum approximations using single precision
 * enlarged-GKB or RSVD", arXiv 2410.00233.
 *
 * General rules
 *  - Every entry point returns kp_status and never aborts or throws; on an
 *    error kp_last_error(ctx) returns a description. Arguments are validated
 *    before any device work is queued.
 *  - "device" pointers are HIP device allocations owned by the caller; "host"
 *    pointers are ordinary host memory owned by the caller. The library never
 *    frees caller memory; it owns only the workspace inside its kp_ctx.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream). Device
 *    outputs are stream-ordered. Calls that return host outputs (sigma, k,
 *    statistics, diagnostics) synchronize `stream` before returning.
 *  - One kp_ctx per host thread; a context is not safe for concurrent use.
 *  - Images: an n x n image is stored row-major, X[row*n + col], row vertical.
 *    The paper's vec is column-major: pixel (r, c) is entry r + n*c.
 *    Vectors in the row or column space of R(A) (length n^2, Krylov bases,
 *    sketches) are stored in that vec order; a block of b such vectors is
 *    column-major with leading dimension n^2.
 *  - Blur model (paper, eq. "forward problem", zero boundary conditions):
 *    A[r + n*i, c + n*j] = P[cu + r - c, cv + i - j] (0 outside P), and the
 *    rearrangement of section 2.1 (eq. "initial rearrange A") gives
 *    R[i + n*j, r + n*c] = P[cu + r - c, cv + i - j]. R(A) is never stored: its
 *    tiles are generated from P on the device.
 */
#ifndef KPSB_H
#define KPSB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KP_OK = 0,
  KP_E_INVAL = 1,       /* invalid argument (nothing was queued)              */
  KP_E_NOMEM = 2,       /* workspace would exceed the context's HBM budget    */
  KP_E_DEVICE = 3,      /* a HIP runtime call failed                           */
  KP_E_NUMERIC = 4,     /* non-finite value met (e.g. NaN in the PSF)          */
  KP_E_BUSY = 5,        /* server queue full (nothing was queued)              */
  KP_E_TIMEOUT = 6,     /* kp_server_wait timed out; the request still runs     */
  KP_E_CANCELLED = 7,   /* stopped by kp_cancel / kp_server_cancel; outputs are
                           undefined (work already queued still completes)    */
  KP_W_BREAKDOWN = 100  /* result valid; a Lanczos breakdown was deflated     */
} kp_status;

/* KP_F16X3 (RSVD only): every product with R or R^T as three FP16 products of
 * two-term FP16 splits of R and of the input (R_hi X_hi + R_hi X_lo + R_lo X_hi,
 * FP32 accumulation, the main term folded into FP64 per column block): about
 * 2^-22 relative, FP32-level accuracy on the 16-bit matrix cores. */
typedef enum { KP_F64 = 0, KP_F32 = 1, KP_BF16 = 2, KP_F16 = 3, KP_F16X3 = 4 } kp_prec;

/* KP-SVD method: Algorithm 1 (EGKB) or Algorithm 2 (RSVD). */
typedef enum { KP_METHOD_GKB = 0, KP_METHOD_RSVD = 1 } kp_method;

typedef struct kp_ctx kp_ctx;

/* Boundary conditions of the blur: how the image is extended beyond its
 * edges. Zero: by zeros (R[i+n*j, r+n*c] = P[cu+r-c, cv+i-j], section 2.1).
 * Reflexive: by reflection about the edge of the last pixel, x[-1-k] = x[k],
 * x[n+k] = x[n-1-k] (the paper's "Medium" example). Periodic: x[k+n] = x[k].
 * Then A[r + n*i, c + n*j] = sum over the images c~ of c and j~ of j of
 * P[cu + r - c~, cv + i - j~], with images k + 2n m and -1 - k + 2n m
 * (m = -1, 0, 1) for reflexive and k + n m (m = -2 .. 2) for periodic: exact
 * for PSFs that reach at most 2n pixels from their centre (required). */
typedef enum { KP_BC_ZERO = 0, KP_BC_REFLEXIVE = 1, KP_BC_PERIODIC = 2 } kp_bc;

/* The blur: PSF P (pu x pv, row-major FP64, P[u*pv + v] with u the vertical
 * offset) with centre (cu, cv), acting on n x n images with boundary
 * conditions bc (kp_bc). `psf` is HOST memory, or DEVICE memory when
 * psf_on_device = 1. Requirements: 2 <= n <= 2048, pu, pv >= 1,
 * 0 <= cu < pu, 0 <= cv < pv, every P entry finite (checked on the host, or on
 * the device for a device PSF; KP_E_NUMERIC otherwise); for bc != KP_BC_ZERO
 * cu, pu-1-cu, cv, pv-1-cv <= 2n.
 * R(A) is generated from the PSF: one term for zero and periodic boundary
 * conditions (periodic: a grid summing the PSF at shifts of n), four for
 * reflexive ones (the mirrored images become Toeplitz terms after reversing
 * the block index j or c), so every product with a reflexive R(A) executes four
 * generated products. */
typedef struct {
  int32_t n;
  const double* psf;
  int32_t pu, pv, cu, cv;
  int32_t psf_on_device;
  int32_t bc;           /* kp_bc */
  int32_t compact;      /* 1: the block products skip the tiles of R(A) that lie
                           outside the rows and columns its PSF grid (in the
                           working precision) can reach: an all-zero row tile is
                           written as zeros, and only the K tiles whose offsets
                           meet the PSF's support are multiplied. Every skipped
                           product is an exact zero, so the result equals the
                           dense product for finite X (up to the sign of zero).
                           Applies to the FP32/FP64 block products and the FP32
                           matrix-vector product (the 16-bit and FP64
                           matrix-vector kernels stay dense). 0: the dense
                           product (the paper's cost model).                  */
} kp_blur;

/* Enlarged Golub-Kahan bidiagonalization (paper, Algorithm 1). */
typedef struct {
  int32_t k;            /* target rank (upper bound when auto_k = 1)               */
  int32_t p;            /* enlargement: k_p = k + p Lanczos steps                  */
  int32_t k_min;        /* stopping test only for steps j > k_min                 */
  int32_t auto_k;       /* 1: choose k by the nu rule (eq. "stopnu")              */
  double tau;           /* tau_EGKB of the nu rule (0: only the "nu rises" clause) */
  int32_t literal_init; /* 1: printed init zeta_1 = 1, nu_2 = 100                  */
  int32_t reorth;       /* 0: one-sided (q_j against Q), 1: full (also s_j vs S)   */
  kp_prec prec;         /* KP_F32 (paper's SP) or KP_F64                           */
  uint64_t seed;        /* Philox seed for the start vector (if y0 == NULL) and
                           for breakdown restart vectors                           */
  const double* y0;     /* optional HOST start vector y, length n^2 (vec order);
                           with block = b >= 1 the start block, n^2 x b
                           column-major                                            */
  double bd_rel;        /* breakdown when t_j or alpha_j is 0 or <= bd_rel times the
                           largest entry of the bidiagonal so far; 0 selects
                           100 * unit roundoff of `prec`                           */
  int32_t block;        /* 0: Algorithm 1 (one start vector). b >= 1: the block
                           Golub-Kahan bidiagonalization with b start vectors
                           (Golub, Luk & Overton 1981), the block analogue of
                           Algorithm 1 with full reorthogonalization, run for
                           ceil((k+p)/b) = nb blocks; needs (nb+1) b <= 64
                           (reorth is ignored). auto_k applies the nu rule
                           once per block J with zeta_J = the geometric mean of
                           alpha t over the block's columns (alpha = diagonal of
                           L_J, t = stored norms of the block's left vectors),
                           tested for J >= 2, J b > k_min; when it fires,
                           k = min(J b, k) and nb = ceil((k+p)/b). At b = 1
                           this is Algorithm 1's rule.
                           Without y0 column c of the start block is Philox
                           stream 0 (c = 0) or 2^31 + c. A breakdown of column m
                           of the left (right) basis is restarted from stream
                           2(m+1) (2(m+1)+1) and reported with break_side 0 (1)
                           and break_step m; diag.kp = nb b, diag.alpha/t are not
                           written, basis_u holds n^2 x (nb+1) b and basis_v
                           n^2 x nb b                                              */
} kp_gkb_opts;

/* Randomized SVD (paper, Algorithm 2) with orthonormalization after every
 * application of R or R^T. */
typedef struct {
  int32_t k, p, q;      /* rank, oversampling, power iterations                    */
  kp_prec prec;         /* KP_F32, KP_F64, KP_BF16 / KP_F16 (block products in
                           16-bit inputs with FP32 accumulation) or KP_F16X3
                           (split-FP16 products, FP32-level accuracy)              */
  int32_t refine;       /* 1: second reorthogonalization + Rayleigh-Ritz refinement
                           of the rank-k factors with an FP32 product W = R V;
                           2: the same with W from three FP16 MFMA products of
                           two-term FP16 splits of R and V (about 2^-22 relative,
                           FP32-level); 0: none                                    */
  uint64_t seed;        /* Philox seed for F when F == NULL                        */
  const double* F;      /* optional HOST sketch, n^2 x (k+p) column-major          */
} kp_rsvd_opts;

/* Diagnostics (all HOST, all optional). */
typedef struct {
  int32_t cap;          /* capacity of alpha / t (>= k_p + 1)                      */
  double* alpha;        /* out: alpha_1..alpha_kp                                  */
  double* t;            /* out: t_1..t_{kp+1}                                      */
  int32_t kp;           /* out: final k_p                                          */
  int32_t nbreak;       /* out: number of deflated breakdowns                      */
  int32_t break_side[128]; /* out: 0 = s-vector, 1 = q-vector, per event (at most
                            2 k_p + 1 events can occur)                            */
  int32_t break_step[128]; /* out: step j of each event                            */
  double ms_total;      /* out: wall time of the call (device, hipEvent)           */
  void* basis_u;        /* optional DEVICE out: left basis S (EGKB) or Y (RSVD),
                           n^2 x (k_p+1) resp. n^2 x k_p, column-major, in the
                           working precision                                       */
  void* basis_v;        /* optional DEVICE out: right basis Q (EGKB, n^2 x k_p)    */
} kp_diag;

/* Kronecker factors (paper, eq. "KP approx"): A ~ sum_t Ax_t (x) Ay_t with
 * Ax_t = sigma_t * array(u_t, n, n), Ay_t = array(v_t, n, n), array column-major;
 * each factor is stored row-major n x n at offset t*n*n. Signs are fixed so that
 * the largest-magnitude entry of v_t (lowest index on ties) is positive. */
typedef struct {
  int32_t n, k_cap;     /* in: image size and capacity (terms) of the buffers      */
  int32_t k;            /* out: number of terms produced                           */
  double* sigma;        /* HOST out [k_cap], descending                            */
  void* Ax;             /* DEVICE out, k_cap * n * n                               */
  void* Ay;             /* DEVICE out, k_cap * n * n                               */
  kp_prec factor_prec;  /* KP_F64 or KP_F32 element type of Ax / Ay                */
  kp_diag* diag;        /* optional                                                */
} kp_factors;

/* Split Bregman parameters (paper, Algorithms 3-5, lambda_x = lambda_y,
 * beta_x = beta_y). tau_sb = 0 / tau_cgls = 0 mean fixed iteration counts. */
typedef struct {
  double lambda, beta;
  int32_t L_max, I_max;
  double tau_sb, tau_cgls;
} sb_opts;

typedef struct {
  int32_t l_end;        /* outer iterations performed                              */
  int32_t iota_total;   /* total CGLS iterations                                   */
  double rc_sb;         /* last RC_SB                                              */
  int32_t graph_replays; /* CGLS iterations run as replays of a captured HIP graph
                            (8 per replay; 0 when the eager launches ran)           */
  int32_t reserved;
} sb_stats;

/* Per-kernel-class timing (tracing). While enabled, every launch of the FP32 /
 * FP64 generated-tile block product (class 0), the matrix-vector product
 * (class 1), the Kronecker-apply GEMMs (class 2) and the 16-bit block product
 * (class 3) is bracketed with hipEvents on the stream of the call;
 * kp_prof_read synchronizes the device and returns, per class, the summed event
 * time, the launch count and the algorithmic flops of those launches (2 n^4 per
 * column for R products, 4 k n^3 per apply). */
typedef struct {
  double ms[4];
  int64_t launches[4];
  double flops[4];
} kp_prof;

/* Context: binds `device`, owns a workspace that never exceeds
 * hbm_budget_bytes (0 = 90% of the device's free memory). */
kp_status kp_ctx_create(int device, size_t hbm_budget_bytes, kp_ctx** out);
kp_status kp_ctx_destroy(kp_ctx* ctx);
const char* kp_last_error(const kp_ctx* ctx);
/* Cancellation token of a context, callable from any thread: the KP-SVD or
 * split Bregman call in progress on ctx returns KP_E_CANCELLED at its next
 * cancellation point (every Lanczos step of Algorithm 1, every block of the
 * block variant, every pass of Algorithm 2, every outer iteration of
 * Algorithms 3-4 and every 8 CGLS iterations), leaving its outputs undefined.
 * The request is consumed by the call it stops; made while no call is in
 * progress, it stops the next one at its first cancellation point. On the
 * context of kp_svd_batched it stops the problems in progress and marks those
 * not started KP_E_CANCELLED. */
kp_status kp_cancel(kp_ctx* ctx);
/* Bytes of device workspace the context holds now (HOST out): the buffers its
 * calls have grown, kept between calls and freed by kp_ctx_destroy. */
kp_status kp_ctx_workspace(const kp_ctx* ctx, size_t* held);
kp_status kp_prof_enable(kp_ctx* ctx, int enable);
/* Reads (and, if reset != 0, clears) the accumulated timings. */
kp_status kp_prof_read(kp_ctx* ctx, kp_prof* out, int reset);
/* Library version string (static storage). */
const char* kp_version(void);
/* Autotuner report: the launch variant chosen for every (operation, size) met so
 * far in this process and the measured cost of each candidate (for the block
 * products the sample launch's time scaled to the whole launch by rounds of
 * resident workgroups, ms; ms per apply for the Kronecker GEMMs), as JSON
 * text. The first call of an operation at a new size times its candidates on
 * the call's stream (one warm-up and two sample launches each, more when a
 * launch is shorter than 0.1 ms) and keeps the fastest; all candidates give
 * bitwise-identical results. KPSB_AUTOTUNE=0 in
 * the environment keeps every operation at its first variant. out: HOST buffer
 * of cap bytes, NUL-terminated, truncated if short. */
kp_status kp_tune_report(char* out, size_t cap);

/* Y = R X (transpose = 0) or Y = R^T X (transpose = 1), the dense product with
 * generated tiles of R(A) (the dominant step of both Algorithms 1 and 2,
 * section 4.1). X, Y: DEVICE, n^2 x ncols column-major (ld = n^2).
 * prec: KP_F32 (float X, Y; FP32 MFMA), KP_F64 (double; FP64 MFMA), KP_BF16 /
 * KP_F16 (float X, Y; R tile and X rounded to 16 bits, FP32 accumulation).
 * ncols == 1 uses the matrix-vector kernel of Algorithm 1. */
kp_status kp_rmat_apply(kp_ctx* ctx, const kp_blur* blur, int transpose, kp_prec prec,
                        int32_t ncols, const void* X, void* Y, void* stream);

/* kp_rmat_apply for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same product, kernels and bits as kp_rmat_apply with the same arguments, but
 * every workspace buffer (PSF copy, grids of R and R^T, support boxes, staging
 * vector, term buffers) is carved from a static device array of 64 MiB that
 * the library holds on each GPU it runs on until the process ends; the call
 * makes no hipMalloc / hipFree and times no autotuner candidates (a launch shape
 * not chosen yet in the process takes the tuner's first variant, which gives
 * the same bits). prec: KP_F32 or KP_F64 (KP_E_INVAL otherwise). A product whose
 * workspace exceeds the array (PSF entries x 8 + 2 grids of
 * (2n + 48)^2 elements + ..., e.g. n = 512 with a full (2n-1)^2 PSF needs about
 * 18 MB in FP32 and 27 MB in FP64) is refused with KP_E_NOMEM before anything
 * is queued. Every call on one GPU, from any context, uses that GPU's one array,
 * which keeps the last call's contents: calls that overlap on a GPU (other
 * threads, other streams not ordered with this one) race and give undefined
 * results. */
kp_status kp_rmat_apply_noalloc(kp_ctx* ctx, const kp_blur* blur, int transpose, kp_prec prec,
                                int32_t ncols, const void* X, void* Y, void* stream);

/* Rank-k KP-SVD of R(A) by EGKB (Algorithm 1). Writes out->k terms. Returns
 * KP_W_BREAKDOWN when a breakdown was deflated (result still valid). */
kp_status kp_svd_gkb(kp_ctx* ctx, const kp_blur* blur, const kp_gkb_opts* opts,
                     kp_factors* out, void* stream);

/* Rank-k KP-SVD of R(A) by RSVD (Algorithm 2). */
kp_status kp_svd_rsvd(kp_ctx* ctx, const kp_blur* blur, const kp_rsvd_opts* opts,
                      kp_factors* out, void* stream);

/* array(A_k x) = sum_t Ay_t X Ax_t^T (transpose = 0) or
 * array(A_k^T x) = sum_t Ay_t^T X Ax_t (transpose = 1) (paper, eq. "KPAx").
 * f: KP_F64 factors (device); X, Y: DEVICE n x n row-major FP64. */
kp_status kp_apply(kp_ctx* ctx, const kp_factors* f, int transpose, const double* X,
                   double* Y, void* stream);

/* Split Bregman anisotropic (Algorithm 3) / isotropic (Algorithm 4) TV
 * deblurring with A replaced by A_k, CGLS inner solves (Algorithm 5), all FP64.
 * b, x: DEVICE n x n row-major FP64; f: KP_F64 factors. stats: HOST, optional. */
kp_status sb_solve_aniso(kp_ctx* ctx, const kp_factors* f, const double* b,
                         const sb_opts* opts, double* x, sb_stats* stats, void* stream);
kp_status sb_solve_iso(kp_ctx* ctx, const kp_factors* f, const double* b,
                       const sb_opts* opts, double* x, sb_stats* stats, void* stream);

/* ---------------------------------------------------------------------------
 * Batched KP-SVD: many independent problems (different n, PSF, method, rank).
 *
 * Problem i is (blurs[i], method[i], opts[i], out[i]) with opts[i] pointing to
 * a kp_gkb_opts (method KP_METHOD_GKB) or a kp_rsvd_opts (KP_METHOD_RSVD); each
 * is exactly the problem of the single call kp_svd_gkb / kp_svd_rsvd with the
 * same arguments and gives the same result (same kernels, same reduction
 * order). The problems run concurrently on `nworkers` worker contexts
 * (0 selects 4; at most 16), each with its own stream and workspace charged to
 * ctx's HBM budget; workers take problems largest first (estimated time).
 * Problems whose launch shapes the autotuner has not chosen yet (a size not
 * seen before in the process) run first, one at a time, so that the tuner
 * times its candidates on an otherwise idle GPU. Every
 * worker stream first waits for the work already queued on `stream`, and
 * `stream` waits for all workers at the end. The call returns when every
 * problem is finished (host outputs written).
 * status: optional HOST out [nprob], the status of each problem.
 * Returns KP_OK when every problem returned KP_OK, KP_W_BREAKDOWN when some
 * returned that warning and none failed, otherwise the status of the failing
 * problem with the lowest index (kp_last_error names it). */
kp_status kp_svd_batched(kp_ctx* ctx, int32_t nprob, const kp_blur* blurs,
                         const int32_t* method, const void* const* opts, kp_factors* out,
                         kp_status* status, int32_t nworkers, void* stream);

/* One split Bregman problem of sb_solve_batched: exactly the arguments of a
 * single sb_solve_iso (iso = 1, Algorithm 4) or sb_solve_aniso (iso = 0,
 * Algorithm 3) call. f: KP_F64 factors (device); b, x: DEVICE n x n row-major
 * FP64, b and x not aliased and no x shared by two problems. */
typedef struct {
  const kp_factors* f;
  const double* b;
  double* x;
  sb_opts opts;
  int32_t iso;
  int32_t reserved;
} sb_problem;

/* Batched split Bregman (Algorithms 3-5): the problems run concurrently on
 * `nworkers` worker contexts (0 selects 4; at most 16; the workers of
 * kp_svd_batched), largest first (n^3 k L_max I_max), each exactly as its
 * single call (same kernels and reduction order, so the same bits; HIP-graph
 * replays of the CGLS iterations where the single call uses them). Problems
 * whose Kronecker-apply launch shape is not tuned yet run first, one at a
 * time. Every worker stream first waits for the work queued on `stream`, and
 * `stream` waits for all of them at the end; the call returns when every
 * problem is finished. stats, status: optional HOST out [nprob]. Returns as
 * kp_svd_batched; kp_cancel on ctx stops the problems in progress and marks
 * those not started KP_E_CANCELLED. */
kp_status sb_solve_batched(kp_ctx* ctx, int32_t nprob, const sb_problem* probs,
                           sb_stats* stats, kp_status* status, int32_t nworkers, void* stream);

/* ---------------------------------------------------------------------------
 * Deblurring server: a request loop that runs split Bregman solves
 * (Algorithms 3-5) of different sizes concurrently, keeps the Kronecker factors
 * of recurring PSFs resident in HBM, and admits queued requests as solve slots
 * and memory free up (continuous batching: a request that arrives while others
 * run starts as soon as a slot and its memory footprint are available, and its
 * kernels overlap theirs on the device).
 *
 * Admission. A request's footprint is its solve workspace plus, on a factor
 * cache miss, its KP-SVD workspace and the new cache entry. Requests are taken
 * in arrival order; one that does not fit may be passed by later ones that do,
 * at most 8 times, after which it blocks the queue until it fits. Least
 * recently used factor sets that no running request holds are evicted when
 * memory or the entry limit requires. A request whose footprint alone exceeds
 * the budget is refused by kp_server_submit (KP_E_NOMEM).
 *
 * Tuning. A request that would make the autotuner choose a launch shape (the
 * first factor computation at a new size, or the first solve at a new size and
 * rank) waits until the running requests have finished and runs alone; the
 * others wait for it. This happens once per shape in the process.
 *
 * Results. Each request runs on one worker with its own stream and workspace,
 * so its output does not depend on what else runs (the same kernels and
 * reduction order as sb_solve_iso / sb_solve_aniso with the same factors). */
typedef struct kp_server kp_server;

typedef struct {
  int32_t slots;            /* concurrent solves (worker streams), 0 = 4, at most 16 */
  size_t hbm_budget_bytes;  /* admission budget for factor cache and workspaces;
                               0 = what the context's budget has left               */
  int32_t max_pending;      /* queued (not yet admitted) requests; 0 = 4096         */
  int32_t cache_entries;    /* resident factor sets; 0 = 64                         */
} kp_server_cfg;

typedef struct {
  uint64_t psf_key;         /* nonzero: factors are cached under (psf_key, n, method,
                               options); the key must identify the PSF and start
                               data. 0: factors are computed for this request only */
  kp_blur blur;             /* read only on a cache miss                             */
  int32_t method;           /* kp_method used on a miss                              */
  kp_gkb_opts gkb;          /* options when method == KP_METHOD_GKB                  */
  kp_rsvd_opts rsvd;        /* options when method == KP_METHOD_RSVD                 */
  int32_t k_cap;            /* terms kept (>= the method's k)                        */
  int32_t iso;              /* 1: isotropic (Algorithm 4), 0: anisotropic (Alg. 3)   */
  sb_opts sb;
  const double* b;          /* DEVICE n x n row-major blurred image, fully written
                               before submit                                         */
  double* x;                /* DEVICE n x n row-major output                         */
} kp_request;

typedef struct {
  kp_status status;
  sb_stats stats;
  int32_t k;                /* Kronecker terms used                                  */
  int32_t cache_hit;        /* 1 when the factors were resident                      */
  double queue_ms;          /* submit -> admitted (host clock)                       */
  double factor_ms;         /* KP-SVD time on a miss, else 0                         */
  double solve_ms;          /* split Bregman time                                    */
  double total_ms;          /* submit -> result complete                             */
  char msg[160];            /* error text when status is an error                    */
} kp_result;

/* Creates a server on ctx's device with cfg->slots worker threads. ctx must
 * outlive the server; the server does not use ctx's workspace. */
kp_status kp_server_create(kp_ctx* ctx, const kp_server_cfg* cfg, kp_server** out);
/* Queues a request (copied; the pointers it holds, including the host PSF and
 * y0 / F, must stay valid until kp_server_wait has returned its result).
 * Non-blocking. *ticket identifies the request for kp_server_wait. */
kp_status kp_server_submit(kp_server* srv, const kp_request* req, uint64_t* ticket);
/* Waits up to timeout_s seconds (< 0: no limit) for a request. On completion
 * fills *res (HOST), forgets the ticket and returns KP_OK (the request's own
 * status is res->status); x is then complete in device memory. Returns
 * KP_E_TIMEOUT if the request is still queued or running, KP_E_INVAL for an
 * unknown ticket. */
kp_status kp_server_wait(kp_server* srv, uint64_t ticket, double timeout_s, kp_result* res);
/* Server counters (HOST): [0] submitted, [1] completed, [2] cache hits,
 * [3] cache misses, [4] evictions, [5] bypasses of a blocked request,
 * [6] peak concurrently running requests, [7] resident factor sets. */
kp_status kp_server_stats(kp_server* srv, int64_t out[8]);
/* Cancels a request: a queued one is removed and completes at once with status
 * KP_E_CANCELLED; a running one stops at its next cancellation point (see
 * kp_cancel) with that status, its factors, if it was computing them, not
 * cached. A request that has finished keeps its result. The ticket must still
 * be collected with kp_server_wait. KP_E_INVAL for an unknown ticket. */
kp_status kp_server_cancel(kp_server* srv, uint64_t ticket);
/* Admission footprint of a request (HOST out, bytes): out[0] bounds the split
 * Bregman workspace (sb_solve_iso / sb_solve_aniso with k_cap terms), out[1]
 * the KP-SVD workspace of a factor-cache miss (kp_svd_gkb / kp_svd_rsvd with the
 * request's options), out[2] is the factor set (2 k_cap n^2 doubles). A request
 * is admitted when out[0] (a cache hit) or out[0] + out[1] + out[2] (a miss)
 * fits beside what is committed. Needs only the request's sizes and options;
 * KP_E_INVAL for a NULL argument, n outside [2, 2048], k_cap outside [1, 64] or
 * an unknown method. */
kp_status kp_request_footprint(const kp_request* req, size_t out[3]);
/* Finishes every submitted request, then frees the server's memory. */
kp_status kp_server_destroy(kp_server* srv);

/* ---------------------------------------------------------------------------
 * Explicit-matrix path: the paper's own pipeline stores the blur matrix A and
 * reorders it into R(A) (section 2.1, eq. "initial rearrange A"); this path
 * serves any A (any boundary condition, e.g. reflexive, or a spatially variant
 * blur). A and R are N x N with N = n^2 (2 <= n <= 1024), row-major, FP32
 * (KP_F32) or FP64 (KP_F64), DEVICE memory owned by the caller; every product
 * streams the stored R from HBM.
 *
 * R[i + n*j, r + n*c] = A[r + n*i, c + n*j]. A and R must not overlap. */
/* The explicit A of a blur with its boundary conditions (blur->bc, kp_bc):
 * A[r + n*i, c + n*j] = sum over the images c~ of c and j~ of j of
 * P[cu + r - c~, cv + i - j~] (zero: only c~ = c, j~ = j). */
kp_status kp_blur_matrix(kp_ctx* ctx, const kp_blur* blur, kp_prec prec, void* A, void* stream);
kp_status kp_rmat_reorder(kp_ctx* ctx, int32_t n, kp_prec prec, const void* A, void* R,
                          void* stream);
/* Y = R X or R^T X with the stored R (X, Y: DEVICE N x ncols column-major;
 * ncols == 1 uses the matrix-vector kernels). */
kp_status kp_rmat_apply_stored(kp_ctx* ctx, int32_t n, kp_prec prec, const void* R,
                               int transpose, int32_t ncols, const void* X, void* Y,
                               void* stream);
/* KP-SVD by EGKB (Algorithm 1) / RSVD (Algorithm 2) of a stored R; the element
 * type of R is opts->prec (KP_F32 or KP_F64; RSVD's 16-bit modes and the
 * split-FP16 refinement need a PSF and are not available here: refine = 2
 * uses the FP32 product). Same outputs and conventions as kp_svd_gkb /
 * kp_svd_rsvd. */
kp_status kp_svd_gkb_stored(kp_ctx* ctx, int32_t n, const void* R, const kp_gkb_opts* opts,
                            kp_factors* out, void* stream);
kp_status kp_svd_rsvd_stored(kp_ctx* ctx, int32_t n, const void* R, const kp_rsvd_opts* opts,
                             kp_factors* out, void* stream);
/* Split Bregman (Algorithms 3 / 4 with CGLS, Algorithm 5) with A itself in
 * place of A_k: the paper's method (i) of Table 1, against which it measures
 * the speed-up of the Kronecker approximation. A: DEVICE N x N row-major FP64
 * acting on the column-major vec of an image; b, x: DEVICE n x n row-major
 * images. */
kp_status sb_solve_aniso_direct(kp_ctx* ctx, int32_t n, const double* A, const double* b,
                                const sb_opts* opts, double* x, sb_stats* stats, void* stream);
kp_status sb_solve_iso_direct(kp_ctx* ctx, int32_t n, const double* A, const double* b,
                              const sb_opts* opts, double* x, sb_stats* stats, void* stream);

/* ---------------------------------------------------------------------------
 * The blur A through two-dimensional FFTs. For a spatially invariant blur A x
 * is a convolution, so A (the BTTB matrix of section 1 for zero boundary
 * conditions, and its reflexive and periodic counterparts) is applied without
 * being stored: the image is extended by its boundary conditions, convolved
 * with the PSF in a circular convolution of size M1 x M2 (the powers of two
 * >= n + pu - 1 and >= n + pv - 1, at most 4096), and cropped; A^T places,
 * correlates and folds each extended entry back onto its source pixel. FP64
 * throughout, O(n^2 log n) per product; equal to the product with the matrix
 * kp_blur_matrix builds up to FFT rounding (about 1e-15 relative).
 *
 * Y = A X (transpose = 0) or A^T X for the blur `blur` (PSF, centre, boundary
 * conditions; blur->compact is ignored). X, Y: DEVICE n x n row-major FP64
 * images (pixel (r, i) at r n + i; r pairs with the PSF's first index),
 * distinct. KP_E_INVAL for a bad blur, NULL or aliased images, or
 * n + pu - 1 or n + pv - 1 above 4096; KP_E_NUMERIC for a non-finite PSF
 * entry. Uses the context's workspace. Every call computes the PSF's
 * spectrum afresh (a row and a column pass over the PSF, about half the cost
 * of the product at n = 512); the solves below compute it once per solve. */
kp_status kp_blur_apply(kp_ctx* ctx, const kp_blur* blur, int transpose, const double* X,
                        double* Y, void* stream);
/* Split Bregman (Algorithms 3 / 4 with CGLS, Algorithm 5) with A itself
 * applied through kp_blur_apply's FFT products: the paper's method (i) of
 * Table 1 without a stored A, for any n the FFT sizes allow. Same options,
 * statistics, image layout and statuses as sb_solve_iso / sb_solve_aniso; the
 * same restored image as sb_solve_iso_direct / sb_solve_aniso_direct with the
 * explicit A up to rounding. */
kp_status sb_solve_aniso_fft(kp_ctx* ctx, const kp_blur* blur, const double* b,
                             const sb_opts* opts, double* x, sb_stats* stats, void* stream);
kp_status sb_solve_iso_fft(kp_ctx* ctx, const kp_blur* blur, const double* b,
                           const sb_opts* opts, double* x, sb_stats* stats, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* KPSB_H */
