// C ABI of libkpsb.so: argument validation, workspace, and the host drivers of
// the KP-SVD (Algorithms 1 and 2 of Alsubhi & Renaut, arXiv 2410.00233) and of
// split Bregman deblurring (Algorithms 3-5). Every arithmetic step runs in the
// HIP kernels of this library; the host only sequences them, keeps the scalar
// recurrences of Algorithm 1 and takes the data-dependent decisions (nu rule,
// breakdown) exactly as the algorithm states them.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <type_traits>
#include <string>
#include <vector>

#include "common.h"
#include "ctx.h"
#include "kpsb.h"
#include "sb.h"

using namespace kpsb;


namespace {

kp_status set_err(kp_ctx* c, kp_status st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

#define KP_HIP(c, expr)                                                              \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return set_err((c), KP_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define KP_TRY(expr)                \
  do {                              \
    kp_status st_ = (expr);         \
    if (st_ != KP_OK) return st_;   \
  } while (0)

kp_status check_launch(kp_ctx* c, const char* where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_err(c, KP_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
  return KP_OK;
}

// Cancellation point (host side, between launches): a pending kp_cancel ends
// the call with KP_E_CANCELLED; work already queued still runs to completion on
// the stream, and the call's outputs are undefined.
kp_status check_cancel(kp_ctx* c) {
  if (c->parent) {
    if (c->parent->cancel.load(std::memory_order_acquire) == 0) return KP_OK;
  } else if (c->cancel.exchange(0, std::memory_order_acq_rel) == 0) {
    return KP_OK;
  }
  return set_err(c, KP_E_CANCELLED, "cancelled by kp_cancel");
}

// Workspace buffer `name` of at least `bytes` (contents undefined).
// Host-side fault injection for tests of the error paths: with
// KPSB_FAULT_INJECT=alloc:N in the environment, the N-th workspace allocation
// counted from when the variable took its current value fails as if hipMalloc
// had failed (KP_E_NOMEM; nothing is allocated).
bool inject_alloc_fault() {
  static std::mutex mu;
  static std::string spec;
  static long count = 0;
  const char* e = getenv("KPSB_FAULT_INJECT");
  const std::string now = e ? e : "";
  std::lock_guard<std::mutex> lk(mu);
  if (now != spec) {
    spec = now;
    count = 0;
  }
  if (spec.compare(0, 6, "alloc:") != 0) return false;
  const long target = atol(spec.c_str() + 6);
  return ++count == target;
}

// set while this thread captures a graph (and holds capture_mutex() shared)
thread_local bool t_capturing = false;

kp_status ws(kp_ctx* c, const std::string& name, size_t bytes, void** out) {
  if (c->arena_base) {   // allocation-free mode: carve from the caller's scratch
    const size_t need = (bytes + 255) & ~(size_t)255;
    if (c->arena_used + need > c->arena_cap)
      return set_err(c, KP_E_NOMEM, "workspace '" + name + "' does not fit the static scratch (" +
                                        std::to_string(c->arena_cap) + " bytes)");
    *out = c->arena_base + c->arena_used;
    c->arena_used += need;
    return KP_OK;
  }
  auto& b = c->bufs[name];
  if (b.bytes >= bytes && b.p) {
    *out = b.p;
    return KP_OK;
  }
  bytes = (bytes + 255) & ~(size_t)255;
  kp_pool& pool = *c->pool;
  {
    std::lock_guard<std::mutex> lk(pool.m);
    if (pool.used - b.bytes + bytes > pool.budget)
      return set_err(c, KP_E_NOMEM, "workspace '" + name + "' of " + std::to_string(bytes) +
                                        " bytes exceeds the HBM budget (" +
                                        std::to_string(pool.budget) + " bytes, " +
                                        std::to_string(pool.used) + " in use)");
    pool.used += bytes;   // reserve before allocating
  }
  auto unreserve = [&](size_t v) {
    std::lock_guard<std::mutex> lk(pool.m);
    pool.used -= v;
  };
  if (b.p) {
    if (t_capturing) {   // this thread holds the capture lock shared
      unreserve(bytes);
      return set_err(c, KP_E_DEVICE, "workspace '" + name + "' would grow during a graph capture");
    }
    std::unique_lock<std::shared_mutex> nocap(capture_mutex());
    hipError_t e1 = hipDeviceSynchronize();
    hipError_t e2 = e1 == hipSuccess ? hipFree(b.p) : e1;
    if (e2 != hipSuccess) {
      unreserve(bytes);
      return set_err(c, KP_E_DEVICE, std::string("freeing workspace: ") + hipGetErrorString(e2));
    }
    unreserve(b.bytes);
    b.p = nullptr;
    b.bytes = 0;
  }
  void* p = nullptr;
  hipError_t e = inject_alloc_fault() ? hipErrorOutOfMemory : hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    unreserve(bytes);
    return set_err(c, KP_E_NOMEM, "hipMalloc of workspace '" + name + "' failed");
  }
  b.p = p;
  b.bytes = bytes;
  *out = p;
  return KP_OK;
}

template <typename T>
kp_status wsT(kp_ctx* c, const std::string& name, size_t count, T** out) {
  void* p = nullptr;
  KP_TRY(ws(c, name, count * sizeof(T), &p));
  *out = static_cast<T*>(p);
  return KP_OK;
}

kp_status validate_blur(kp_ctx* c, const kp_blur* b) {
  if (!b) return set_err(c, KP_E_INVAL, "blur is NULL");
  if (b->n < 2 || b->n > 2048) return set_err(c, KP_E_INVAL, "n must be in [2, 2048]");
  if (!b->psf) return set_err(c, KP_E_INVAL, "psf is NULL");
  if (b->pu < 1 || b->pv < 1) return set_err(c, KP_E_INVAL, "psf dimensions must be >= 1");
  if (b->cu < 0 || b->cu >= b->pu || b->cv < 0 || b->cv >= b->pv)
    return set_err(c, KP_E_INVAL, "psf centre outside the psf array");
  if ((long)b->pu * b->pv > (1L << 26)) return set_err(c, KP_E_INVAL, "psf too large");
  if (b->psf_on_device != 0 && b->psf_on_device != 1)
    return set_err(c, KP_E_INVAL, "psf_on_device must be 0 or 1");
  if (b->compact != 0 && b->compact != 1) return set_err(c, KP_E_INVAL, "compact must be 0 or 1");
  if (b->bc != KP_BC_ZERO && b->bc != KP_BC_REFLEXIVE && b->bc != KP_BC_PERIODIC)
    return set_err(c, KP_E_INVAL, "bc must be KP_BC_ZERO, KP_BC_REFLEXIVE or KP_BC_PERIODIC");
  if (b->bc != KP_BC_ZERO) {
    const long reach = 2L * b->n;
    if (b->cu > reach || b->pu - 1 - b->cu > reach || b->cv > reach || b->pv - 1 - b->cv > reach)
      return set_err(c, KP_E_INVAL,
                     "with reflexive or periodic boundary conditions the PSF may reach at most "
                     "2n pixels from its centre");
  }
  if (!b->psf_on_device)
    for (long e = 0; e < (long)b->pu * b->pv; ++e)
      if (!std::isfinite(b->psf[e])) return set_err(c, KP_E_NUMERIC, "psf has a non-finite entry");
  return KP_OK;
}

template <typename T> const char* tname();
template <> const char* tname<float>() { return "f32"; }
template <> const char* tname<double>() { return "f64"; }
template <> const char* tname<__hip_bfloat16>() { return "bf16"; }
template <> const char* tname<__half>() { return "f16"; }

// Terms of R(A) for the boundary conditions of a blur (every term is a
// generated operator over its own offset grid). Zero: R = R(G). Periodic: the
// images j + n m of the extended image only shift the offsets i - j (and
// r - c) by multiples of n, so R = R(G_per) is one term whose grid sums the
// PSF at those shifts. Reflexive: the images j + 2n m keep the Toeplitz form
// (even shifts 2n m), while the mirrored images -1 - j + 2n m depend on i + j;
// reversing the block index, j -> n-1-j, turns them into offsets i - j shifted
// by n - 2n m (odd shifts). With J the reversal of the block index of a
// length-n^2 vector (a + n b -> a + n (n-1-b)),
//   R = R(G_ee) + R(G_eo) J + J R(G_oe) + J R(G_oo) J,
// the first letter naming the shifts of the i - j offsets, the second those of
// the r - c offsets; R^T = sum_t J^{fu} R(G_t)^T J^{fv}. The image sets are
// m = -1..1 (reflexive) and m = -2..2 (periodic): exact for PSFs that reach at
// most 2n pixels from their centre.
struct RmatTerms {
  int nterm = 1;
  GridShifts sh[4];
  int fv[4] = {0, 0, 0, 0};   // term t reverses the row blocks j of R
  int fu[4] = {0, 0, 0, 0};   // term t reverses the column blocks c of R
  int nsum_max() const {
    int m = 1;
    for (int t = 0; t < nterm; ++t) m = std::max(m, sh[t].nv * sh[t].nu);
    return m;
  }
};

RmatTerms make_terms(int bc, int n) {
  RmatTerms r;
  if (bc == KP_BC_PERIODIC) {
    GridShifts g;
    g.nv = g.nu = 5;
    for (int m = -2; m <= 2; ++m) g.sv[m + 2] = g.su[m + 2] = -n * m;
    r.sh[0] = g;
  } else if (bc == KP_BC_REFLEXIVE) {
    int even[3], odd[3];
    for (int m = -1; m <= 1; ++m) {
      even[m + 1] = -2 * n * m;
      odd[m + 1] = n - 2 * n * m;
    }
    r.nterm = 4;
    for (int t = 0; t < 4; ++t) {
      r.fv[t] = t >> 1;
      r.fu[t] = t & 1;
      GridShifts& g = r.sh[t];
      g.nv = g.nu = 3;
      for (int x = 0; x < 3; ++x) {
        g.sv[x] = r.fv[t] ? odd[x] : even[x];
        g.su[x] = r.fu[t] ? odd[x] : even[x];
      }
    }
  }
  return r;
}

template <typename T>
struct Grids {
  T* G = nullptr;    // grid of R (term 0)
  T* Gt = nullptr;   // grid of R^T (term 0)
  int ldg = 0;
  RmatTerms terms;
  T* Gs[4] = {nullptr, nullptr, nullptr, nullptr};    // grid of term t
  T* Gts[4] = {nullptr, nullptr, nullptr, nullptr};   // its transpose
  // support boxes of Gs[t] / Gts[t] (device; null: dense products)
  int* box[4] = {nullptr, nullptr, nullptr, nullptr};
  int* boxt[4] = {nullptr, nullptr, nullptr, nullptr};
  Grids term(int t) const {
    Grids g;
    g.G = g.Gs[0] = Gs[t];
    g.Gt = g.Gts[0] = Gts[t];
    g.box[0] = box[t];
    g.boxt[0] = boxt[t];
    g.ldg = ldg;
    return g;
  }
};

// Device copy of the PSF: uploaded from the host, or (device PSF) used in place
// after a device-side finiteness check.
kp_status upload_psf(kp_ctx* c, const kp_blur* b, hipStream_t s, double** dpsf) {
  const long cnt = (long)b->pu * b->pv;
  if (b->psf_on_device) {
    int* flag = nullptr;
    KP_TRY(wsT(c, "psf_flag", 4, &flag));
    launch_count_nonfinite(b->psf, cnt, flag, s);
    KP_TRY(check_launch(c, "psf check"));
    KP_HIP(c, hipMemcpyAsync(c->pinned + 16, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    KP_HIP(c, hipStreamSynchronize(s));
    if (*reinterpret_cast<int*>(c->pinned + 16) != 0)
      return set_err(c, KP_E_NUMERIC, "psf has a non-finite entry");
    *dpsf = const_cast<double*>(b->psf);
    return KP_OK;
  }
  KP_TRY(wsT(c, "psf", (size_t)cnt, dpsf));
  KP_HIP(c, hipMemcpyAsync(*dpsf, b->psf, sizeof(double) * cnt, hipMemcpyHostToDevice, s));
  return KP_OK;
}

template <typename T>
kp_status build_grids(kp_ctx* c, const kp_blur* b, const double* dpsf, hipStream_t s,
                      Grids<T>* g) {
  const int n = b->n;
  g->ldg = grid_ld(n);
  g->terms = make_terms(b->bc, n);
  const size_t cnt = (size_t)g->ldg * g->ldg;   // square: see launch_build_grid
  for (int t = 0; t < g->terms.nterm; ++t) {
    const std::string sfx = std::string(tname<T>()) + (t ? "_" + std::to_string(t) : "");
    KP_TRY(wsT(c, "G_" + sfx, cnt, &g->Gs[t]));
    KP_TRY(wsT(c, "Gt_" + sfx, cnt, &g->Gts[t]));
    launch_build_grid<T>(dpsf, b->pu, b->pv, b->cu, b->cv, n, 0, g->terms.sh[t], g->Gs[t],
                         g->ldg, s);
    launch_build_grid<T>(dpsf, b->pu, b->pv, b->cu, b->cv, n, 1, g->terms.sh[t], g->Gts[t],
                         g->ldg, s);
    if (b->compact) {
      int* part = nullptr;
      KP_TRY(wsT(c, "gbox_part", (size_t)grid_box_parts(), &part));
      KP_TRY(wsT(c, "gbox_" + sfx, 8, &g->box[t]));
      g->boxt[t] = g->box[t] + 4;
      launch_grid_box<T>(g->Gs[t], g->ldg, n, part, g->box[t], s);
      launch_grid_box<T>(g->Gts[t], g->ldg, n, part, g->boxt[t], s);
    }
  }
  g->G = g->Gs[0];
  g->Gt = g->Gts[0];
  return check_launch(c, "build_grid");
}

// Y = sum over the terms of J^{out} op(R_t) J^{in} X (see RmatTerms): prod(t, in,
// out, first) computes one term's product into out (first: the term written
// straight into Y, which alone carries any extra operand of the product).
// One term: prod(0, X, Y, true). Four terms: X reversed once into a
// workspace, the three other terms into workspaces, then one combining pass.
template <typename B, typename F>
kp_status multi_term(kp_ctx* c, const RmatTerms& tm, int n, int tr, const B* X, B* Y,
                     int ncols, hipStream_t s, F prod) {
  if (tm.nterm == 1) return prod(0, X, Y, true);
  const long N = (long)n * n;
  const size_t cnt = (size_t)N * ncols;
  B *Xf = nullptr, *T1 = nullptr, *T2 = nullptr, *T3 = nullptr;
  KP_TRY(wsT(c, std::string("terms_x_") + tname<B>(), cnt, &Xf));
  KP_TRY(wsT(c, std::string("terms_1_") + tname<B>(), cnt, &T1));
  KP_TRY(wsT(c, std::string("terms_2_") + tname<B>(), cnt, &T2));
  KP_TRY(wsT(c, std::string("terms_3_") + tname<B>(), cnt, &T3));
  launch_flip_blocks<B>(X, Xf, n, N, ncols, s);
  for (int t = 0; t < tm.nterm; ++t) {
    const int fo = tr ? tm.fu[t] : tm.fv[t];
    const int fi = tr ? tm.fv[t] : tm.fu[t];
    B* dst = !fo ? (!fi ? Y : T1) : (!fi ? T2 : T3);
    KP_TRY(prod(t, fi ? Xf : X, dst, dst == Y));
  }
  launch_combine_terms<B>(Y, T1, T2, T3, n, N, ncols, s);
  return check_launch(c, "combine_terms");
}

template <typename T>
kp_status prep_grids(kp_ctx* c, const kp_blur* b, hipStream_t s, Grids<T>* g) {
  double* dpsf = nullptr;
  KP_TRY(upload_psf(c, b, s, &dpsf));
  return build_grids<T>(c, b, dpsf, s, g);
}

// Tracing: bracket a launch with events when the context profiles.
struct ProfScope {
  kp_ctx* c;
  hipStream_t s;
  kp_ctx::Rec r{};
  bool on;
  ProfScope(kp_ctx* ctx, hipStream_t st, int cls, double flops) : c(ctx), s(st), on(ctx->prof) {
    if (!on) return;
    r.cls = cls;
    r.flops = flops;
    if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) {
      on = false;
      return;
    }
    (void)hipEventRecord(r.a, s);
  }
  ~ProfScope() {
    if (!on) return;
    (void)hipEventRecord(r.b, s);
    c->recs.push_back(r);
  }
};

// Autotuned launch shapes of the block products: the cost of a variant is the
// time of a sample launch (the first 1024 workgroups, or the whole grid if
// smaller) scaled to the whole launch by rounds of resident workgroups (a
// partial last round costs a whole one): ms * ceil(grid / res) /
// ceil(sample / res), res = 256 CUs x the workgroups the LDS lets share a CU.
constexpr int kSampleWG = 1024;
struct BlockVariant {
  int TJ, waves, TK;
};
constexpr BlockVariant kBlockVariants[] = {{16, 16, 64},  {16, 8, 64},  {8, 8, 64},  {8, 16, 64},
                                           {16, 16, 128}, {16, 8, 128}, {8, 8, 128}, {8, 16, 128},
                                           {16, 16, 192}, {16, 8, 192}, {8, 8, 192}, {8, 16, 192},
                                           {16, 16, 176}, {16, 8, 176}, {8, 8, 176}, {8, 16, 176},
                                           {12, 12, 176}, {12, 12, 128}};
constexpr int kNumBlockVariants = 18;

double launch_estimate(double sample_ms, int grid, size_t lds, size_t lds_cap, int threads) {
  const int sample = std::min(grid, kSampleWG);
  const int by_lds = lds > 0 ? (int)std::max<size_t>(1, lds_cap / lds) : 8;
  const int by_waves = std::max(1, 32 / std::max(1, threads / 64));   // 32 waves per CU
  const long res = 256L * std::max(1, std::min(by_lds, by_waves));
  const long r_all = (grid + res - 1) / res, r_sample = (sample + res - 1) / res;
  return sample_ms * (double)r_all / (double)r_sample;
}
struct Block16Variant {
  int TJ, waves;
};
constexpr Block16Variant kBlock16Variants[] = {{32, 8}, {16, 4}, {32, 16}, {16, 8}, {16, 16},
                                               {64, 16}, {64, 8}};
constexpr int kNumBlock16Variants = 7;

template <typename T>
kp_status choose_block_plan(kp_ctx* c, const Grids<T>& g, int n, const T* X, T* Y, int nc,
                            hipStream_t s, BlockPlan* bp) {
  const long N = (long)n * n;
  const int v = tune_pick(kTuneBlock, n, (int)sizeof(T), 0, kNumBlockVariants,
                          [&](int k) -> double {
    BlockPlan p;
    if (!plan_block_tj<T>(n, c->lds_limit, kBlockVariants[k].TJ, &p, kBlockVariants[k].TK))
      return -1.0;
    p.waves = kBlockVariants[k].waves;
    p.grid_limit = std::min(p.grid, kSampleWG);
    const double ms = time_launches(s, 2, [&]() {
      launch_rmat_block<T>(p, g.G, g.ldg, n, X, N, Y, N, nc, s);
    });
    return ms < 0 ? -1.0 : launch_estimate(ms, p.grid, p.lds, c->lds_limit, 64 * p.waves);
  });
  if (!plan_block_tj<T>(n, c->lds_limit, kBlockVariants[v].TJ, bp, kBlockVariants[v].TK)) {
    if (!plan_block<T>(n, c->lds_limit, bp))
      return set_err(c, KP_E_INVAL, "no block-product tiling fits the LDS at this n");
    return KP_OK;
  }
  bp->waves = kBlockVariants[v].waves;
  return KP_OK;
}

// Y = R X (or R^T X) for any number of columns (groups of 32 per launch), one
// term.
template <typename T>
kp_status block_product1(kp_ctx* c, const Grids<T>& g, int n, int transpose, const T* X,
                         T* Y, int ncols, hipStream_t s) {
  if constexpr (std::is_same<T, float>::value) {
    if (c->batch && !(transpose ? g.boxt[0] : g.box[0]))   // lockstep batch: one launch for all
      return batch_block_product(c, transpose ? g.Gt : g.G, g.ldg, n, X, Y, ncols, s);
  }
  BlockPlan bp;
  KP_TRY(choose_block_plan<T>(c, g, n, X, Y, std::min(ncols, 32), s, &bp));
  const long N = (long)n * n;
  for (int c0 = 0; c0 < ncols; c0 += 32) {
    const int nc = ncols - c0 < 32 ? ncols - c0 : 32;
    ProfScope ps(c, s, 0, 2.0 * (double)N * (double)N * nc);
    launch_rmat_block<T>(bp, transpose ? g.Gt : g.G, g.ldg, n, X + N * c0, N, Y + N * c0, N,
                         nc, s, transpose ? g.boxt[0] : g.box[0]);
  }
  return check_launch(c, "rmat_block");
}

template <typename H>
kp_status choose_block16_plan(kp_ctx* c, const Grids<H>& g, int n, const H* X16, long ld16,
                              float* Y, int nc, hipStream_t s, BlockPlan* bp) {
  const long N = (long)n * n;
  const int v = tune_pick(kTuneBlock16, n, std::is_same<H, __half>::value ? KP_F16 : KP_BF16, 0,
                          kNumBlock16Variants,
                          [&](int k) -> double {
    BlockPlan p;
    if (!plan_block16_tj(n, c->lds_limit, kBlock16Variants[k].TJ, &p)) return -1.0;
    p.waves = kBlock16Variants[k].waves;
    p.grid_limit = std::min(p.grid, kSampleWG);
    const double ms = time_launches(s, 2, [&]() {
      launch_rmat_block16<H>(p, g.G, g.ldg, n, X16, ld16, Y, N, nc, s);
    });
    return ms < 0 ? -1.0 : launch_estimate(ms, p.grid, p.lds, c->lds_limit, 64 * p.waves);
  });
  if (plan_block16_tj(n, c->lds_limit, kBlock16Variants[v].TJ, bp)) {
    bp->waves = kBlock16Variants[v].waves;
    return KP_OK;
  }
  if (!plan_block16(n, c->lds_limit, bp))
    return set_err(c, KP_E_INVAL, "no 16-bit block-product tiling fits the LDS at this n");
  return KP_OK;
}

// Y = R X with 16-bit inputs (H = __hip_bfloat16 or __half) and FP32 output; X is
// rounded to H into a workspace copy first.
template <typename H>
kp_status block_product16_1(kp_ctx* c, const Grids<H>& g, int n, int transpose, const float* X,
                            float* Y, int ncols, hipStream_t s) {
  const long N = (long)n * n;
  const long ld16 = x16_column_len(n);
  H* X16 = nullptr;
  KP_TRY(wsT(c, "x16", (size_t)ld16 * ncols, &X16));
  launch_to16_shifted<H>(X, N, n, ncols, X16, ld16, s);
  BlockPlan bp;
  KP_TRY(choose_block16_plan<H>(c, g, n, X16, ld16, Y, std::min(ncols, 32), s, &bp));
  for (int c0 = 0; c0 < ncols; c0 += 32) {
    const int nc = ncols - c0 < 32 ? ncols - c0 : 32;
    ProfScope ps(c, s, 3, 2.0 * (double)N * (double)N * nc);
    launch_rmat_block16<H>(bp, transpose ? g.Gt : g.G, g.ldg, n, X16 + ld16 * c0, ld16,
                           Y + N * c0, N, nc, s);
  }
  return check_launch(c, "rmat_block16");
}

// W = R V (ncols columns, FP32 in and out) to about FP32 accuracy from three
// FP16 MFMA products: with R s = G_hi + G_lo and V 2^kSplitXExp = V_hi + V_lo
// (two-term FP16 splits, power-of-2 scalings), W = (G_hi V_hi + G_hi V_lo +
// G_lo V_hi) / (s 2^kSplitXExp); the dropped G_lo V_lo term is about 2^-22 of
// the product. Accumulated in FP64 inside each product, in FP32 across them.
kp_status split16_product(kp_ctx* c, const kp_blur* b, const double* dpsf, int n, int tr,
                          const float* V, float* W, int ncols, hipStream_t s) {
  BlockPlan bp;
  bool planned = false;
  const long N = (long)n * n;
  const int ldg = grid_ld(n);
  const size_t gcount = (size_t)(2 * n - 1) * ldg;
  const RmatTerms tm = make_terms(b->bc, n);
  double* scal = nullptr;
  __half *Ghi = nullptr, *Glo = nullptr, *Xhi = nullptr, *Xlo = nullptr;
  KP_TRY(wsT(c, "split_scal", (size_t)psf_split_scale_len(), &scal));
  KP_TRY(wsT(c, "G_split_hi", gcount, &Ghi));
  KP_TRY(wsT(c, "G_split_lo", gcount, &Glo));
  const long ld16 = x16_column_len(n);
  KP_TRY(wsT(c, "x_split_hi", (size_t)ld16 * ncols, &Xhi));
  KP_TRY(wsT(c, "x_split_lo", (size_t)ld16 * ncols, &Xlo));
  launch_psf_split_scale(dpsf, (long)b->pu * b->pv, tm.nsum_max(), scal, s);
  // the terms run one after another on the stream, so one hi/lo grid pair serves all
  return multi_term<float>(c, tm, n, tr, V, W, ncols, s,
                           [&](int t, const float* in, float* out, bool) -> kp_status {
    launch_build_grid_split(dpsf, b->pu, b->pv, b->cu, b->cv, n, tr, tm.sh[t], scal, 0, Ghi, ldg, s);
    launch_build_grid_split(dpsf, b->pu, b->pv, b->cu, b->cv, n, tr, tm.sh[t], scal, 1, Glo, ldg, s);
    launch_to16_split(in, N, n, ncols, Xhi, Xlo, ld16, s);
    if (!planned) {   // the tuned 16-bit launch shape (its samples write `out` first)
      Grids<__half> gg;
      gg.G = gg.Gs[0] = Ghi;
      gg.ldg = ldg;
      KP_TRY(choose_block16_plan<__half>(c, gg, n, Xhi, ld16, out, std::min(ncols, 32), s, &bp));
      planned = true;
    }
    // only the main term needs the FP64 fold: the two correction terms are
    // 2^-11 of it, so their FP32 accumulation error is that much smaller too
    for (int c0 = 0; c0 < ncols; c0 += 32) {
      const int nc = ncols - c0 < 32 ? ncols - c0 : 32;
      float* Wc = out + N * c0;
      launch_rmat_block16<__half>(bp, Ghi, ldg, n, Xhi + ld16 * c0, ld16, Wc, N, nc, s, scal + 1, 0, true);
      launch_rmat_block16<__half>(bp, Ghi, ldg, n, Xlo + ld16 * c0, ld16, Wc, N, nc, s, scal + 1, 1, false);
      launch_rmat_block16<__half>(bp, Glo, ldg, n, Xhi + ld16 * c0, ld16, Wc, N, nc, s, scal + 1, 1, false);
    }
    return check_launch(c, "split16_product");
  });
}

template <typename T>
kp_status gemv_product1(kp_ctx* c, const Grids<T>& g, int n, int transpose, const T* x, T* y,
                        const T* z, double coef, hipStream_t s) {
  const double NN = (double)n * n;
  if constexpr (std::is_same<T, float>::value) {
    // the kernel addresses the ldg x ldg grid through a buffer resource whose
    // size is a 32-bit byte count (n <= 2048 keeps it under 69 MB)
    if (4L * g.ldg * g.ldg > 0x7fffffffL)
      return set_err(c, KP_E_INVAL, "grid too large for the matrix-vector kernel");
    float* xt = nullptr;
    KP_TRY(wsT(c, "gemv_xt", (size_t)gemv_sx_xt_len(n), &xt));
    ProfScope ps(c, s, 1, 2.0 * NN * NN);
    // the kernel reads the grid of op(R) column by column: from the transposed
    // grid's rows
    launch_rmat_gemv_sx(transpose ? g.G : g.Gt, g.ldg, n, x, xt, y, z, coef, s,
                        transpose ? g.boxt[0] : g.box[0]);
    return check_launch(c, "rmat_gemv_sx");
  }
  BlockPlan gp;
  if (!plan_gemv<T>(n, c->lds_limit, &gp))
    return set_err(c, KP_E_INVAL, "no matrix-vector tiling fits the LDS at this n");
  {
    ProfScope ps(c, s, 1, 2.0 * NN * NN);
    launch_rmat_gemv<T>(gp, transpose ? g.Gt : g.G, g.ldg, n, x, y, z, coef, s);
  }
  return check_launch(c, "rmat_gemv");
}

// Products over all terms of R (boundary conditions; see RmatTerms).
template <typename T>
kp_status block_product(kp_ctx* c, const Grids<T>& g, int n, int tr, const T* X, T* Y,
                        int ncols, hipStream_t s) {
  return multi_term<T>(c, g.terms, n, tr, X, Y, ncols, s,
                       [&](int t, const T* in, T* out, bool) -> kp_status {
    return block_product1<T>(c, g.term(t), n, tr, in, out, ncols, s);
  });
}

template <typename H>
kp_status block_product16(kp_ctx* c, const Grids<H>& g, int n, int tr, const float* X,
                          float* Y, int ncols, hipStream_t s) {
  return multi_term<float>(c, g.terms, n, tr, X, Y, ncols, s,
                           [&](int t, const float* in, float* out, bool) -> kp_status {
    return block_product16_1<H>(c, g.term(t), n, tr, in, out, ncols, s);
  });
}

// y = R x - coef z (or R^T x - coef z; z may be null).
template <typename T>
kp_status gemv_product(kp_ctx* c, const Grids<T>& g, int n, int tr, const T* x, T* y,
                       const T* z, double coef, hipStream_t s) {
  return multi_term<T>(c, g.terms, n, tr, x, y, 1, s,
                       [&](int t, const T* in, T* out, bool first) -> kp_status {
    return gemv_product1<T>(c, g.term(t), n, tr, in, out, first ? z : nullptr,
                            first ? coef : 0.0, s);
  });
}

// Shared scratch of the vector kernels.
struct Scratch {
  double* partials = nullptr;   // kRedBlocks * 64
  double* nrmp = nullptr;       // kRedBlocks
  double* h = nullptr;          // 4 x 64 coefficient vectors
  double* scal = nullptr;       // 8 scalars
  int* flag = nullptr;          // device predicate
  int* flags = nullptr;         // 64 per-column predicates
};

kp_status get_scratch(kp_ctx* c, Scratch* sc) {
  KP_TRY(wsT(c, "partials", (size_t)kRedBlocks * 64, &sc->partials));
  KP_TRY(wsT(c, "nrmp", (size_t)kRedBlocks, &sc->nrmp));
  KP_TRY(wsT(c, "hvec", 4 * 64, &sc->h));
  KP_TRY(wsT(c, "scal", 8, &sc->scal));
  KP_TRY(wsT(c, "flag", 4, &sc->flag));
  KP_TRY(wsT(c, "flags", 64, &sc->flags));
  return KP_OK;
}

// ||w||^2 from kRedBlocks partials, read back to the host (synchronizes s).
kp_status read_norm(kp_ctx* c, const Scratch& sc, hipStream_t s, double* out) {
  launch_reduce_partials(sc.nrmp, 1, sc.scal, 0, s);
  KP_TRY(check_launch(c, "reduce_partials"));
  KP_HIP(c, hipMemcpyAsync(c->pinned, sc.scal, sizeof(double), hipMemcpyDeviceToHost, s));
  KP_HIP(c, hipStreamSynchronize(s));
  *out = std::sqrt(c->pinned[0]);
  return KP_OK;
}

// Classical Gram-Schmidt, two passes, of w against the m columns of V; leaves
// the partial sums of ||w||^2 in sc.nrmp.
template <typename T>
void cgs2(const Scratch& sc, T* w, const T* V, long ldv, int m, long N, hipStream_t s) {
  if (m == 0) {
    launch_norm2_partials<T>(w, N, sc.nrmp, s);
    return;
  }
  for (int pass = 0; pass < 2; ++pass) {
    launch_multidot<T>(V, ldv, m, w, N, sc.partials, s);
    launch_project_out_red<T>(w, V, ldv, m, sc.partials, sc.h, nullptr, N, sc.nrmp, s);
  }
}

// Orthonormal basis of the N x m block W in place (Householder TSQR), with its R
// factor in Rfac when that is not NULL.
template <typename T>
kp_status tsqr_qr(kp_ctx* c, T* W, long N, int m, double* Rfac, hipStream_t s) {
  const size_t bytes = tsqr_workspace_bytes(N, m);
  if (!bytes) return set_err(c, KP_E_INVAL, "QR of an N x m block needs 1 <= m <= 64, N >= m");
  void* w = nullptr;
  KP_TRY(ws(c, "tsqr", bytes, &w));
  launch_tsqr<T>(W, N, m, Rfac, w, s);
  return check_launch(c, "tsqr");
}

// Upload an N x m FP64 host block into device type T (through a staging buffer).
template <typename T>
kp_status upload_block(kp_ctx* c, const double* host, long count, T* dst, hipStream_t s) {
  double* stage = nullptr;
  KP_TRY(wsT(c, "stage64", (size_t)count, &stage));
  KP_HIP(c, hipMemcpyAsync(stage, host, sizeof(double) * count, hipMemcpyHostToDevice, s));
  launch_convert<double, T>(stage, dst, count, s);
  return check_launch(c, "convert");
}

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t s;
  explicit Timer(hipStream_t st) : s(st) {
    if (hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
      (void)hipEventRecord(a, s);
  }
  double stop() {
    float ms = 0.f;
    if (a && b) {
      (void)hipEventRecord(b, s);
      (void)hipEventSynchronize(b);
      (void)hipEventElapsedTime(&ms, a, b);
    }
    return ms;
  }
  ~Timer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

kp_status validate_factors_out(kp_ctx* c, const kp_factors* f, int n) {
  if (!f) return set_err(c, KP_E_INVAL, "factors is NULL");
  if (f->n != n) return set_err(c, KP_E_INVAL, "factors.n differs from blur.n");
  if (!f->sigma || !f->Ax || !f->Ay) return set_err(c, KP_E_INVAL, "factors buffers are NULL");
  if (f->factor_prec != KP_F64 && f->factor_prec != KP_F32)
    return set_err(c, KP_E_INVAL, "factor_prec must be KP_F64 or KP_F32");
  return KP_OK;
}

// Form Kronecker factors from left/right singular vector blocks (FP64, N x k).
kp_status write_factors(kp_ctx* c, const double* Ud, const double* Vd, const double* sig_dev,
                        int n, int k, kp_factors* f, hipStream_t s) {
  int* amax = nullptr;
  KP_TRY(wsT(c, "argmax", 64, &amax));
  const long N = (long)n * n;
  if (f->factor_prec == KP_F64)
    launch_form_factors<double, double>(Ud, Vd, N, n, k, sig_dev, (double*)f->Ax,
                                        (double*)f->Ay, amax, s);
  else
    launch_form_factors<double, float>(Ud, Vd, N, n, k, sig_dev, (float*)f->Ax,
                                       (float*)f->Ay, amax, s);
  return check_launch(c, "form_factors");
}

// ---------------------------------------------------------------------------
// The matrix B = R(A) of the KP-SVD drivers: generated tile by tile from a PSF
// (a blur with zero boundary conditions), or stored in HBM as an N x N
// row-major matrix (the reordered explicit A of any blur).
template <typename T>
struct RmatOp {
  int n = 0;
  const kp_blur* blur = nullptr;   // generated
  const double* dpsf = nullptr;
  Grids<T> g;
  const T* R = nullptr;            // stored
  double* gv_ws = nullptr;         // stored R^T x partial sums

  kp_status gemv(kp_ctx* c, int tr, const T* x, T* y, const T* z, double coef,
                 hipStream_t s) const {
    if (R) {
      const double NN = (double)n * n;
      ProfScope ps(c, s, 1, 2.0 * NN * NN);
      launch_stored_gemv<T>(R, (long)n * n, tr, x, y, z, coef, gv_ws, s);
      return check_launch(c, "stored_gemv");
    }
    return gemv_product<T>(c, g, n, tr, x, y, z, coef, s);
  }
  kp_status block(kp_ctx* c, int tr, const T* X, T* Y, int ncols, hipStream_t s) const {
    if (R) {
      const long N = (long)n * n;
      for (int c0 = 0; c0 < ncols; c0 += 32) {
        const int nc = ncols - c0 < 32 ? ncols - c0 : 32;
        ProfScope ps(c, s, 0, 2.0 * (double)N * (double)N * nc);
        launch_stored_block<T>(R, N, tr, X + N * c0, Y + N * c0, nc, s);
      }
      return check_launch(c, "stored_block");
    }
    return block_product<T>(c, g, n, tr, X, Y, ncols, s);
  }
};

template <typename T>
kp_status make_generated_op(kp_ctx* c, const kp_blur* b, hipStream_t s, RmatOp<T>* op) {
  op->n = b->n;
  op->blur = b;
  KP_TRY(upload_psf(c, b, s, const_cast<double**>(&op->dpsf)));
  return build_grids<T>(c, b, op->dpsf, s, &op->g);
}

template <typename T>
kp_status make_stored_op(kp_ctx* c, int n, const T* R, RmatOp<T>* op) {
  op->n = n;
  op->R = R;
  return wsT(c, "stored_gv", (size_t)stored_gemv_ws((long)n * n), &op->gv_ws);
}

// ---------------------------------------------------------------------------
// EGKB (Algorithm 1). Readings as in the oracle: nu_{j+1} = sqrt(zeta_j
// zeta_{j-1}); zeta_1 = alpha_1 t_1, nu_2 = +inf (or the printed 1 and 100);
// j = 2 .. k_p + 1; the nu test fires at most once, for j > k_min and
// j - 1 != k_p, setting k = min(j, k_in); U_k = S_{k_p+1} U_C[:, :k]; a
// breakdown stores 0 and restarts with a Philox vector (stream 2j for s_j,
// 2j + 1 for q_j) orthogonalized against the basis.
template <typename T>
kp_status egkb_impl(kp_ctx* c, const RmatOp<T>& op, const kp_gkb_opts* o, kp_factors* f,
                    hipStream_t s) {
  Timer timer(s);
  const int n = op.n;
  const long N = (long)n * n;
  int k = o->k;
  const int p = o->p;
  const int k_in = k;
  int kp = k + p;
  const int kp0 = kp;
  const double u = (sizeof(T) == 4) ? std::ldexp(1.0, -24) : std::ldexp(1.0, -53);
  const double bd_rel = o->bd_rel > 0 ? o->bd_rel : 1e2 * u;

  Scratch sc;
  KP_TRY(get_scratch(c, &sc));
  T *S = nullptr, *Q = nullptr;
  KP_TRY(wsT(c, std::string("egkbS_") + tname<T>(), (size_t)N * (kp0 + 1), &S));
  KP_TRY(wsT(c, std::string("egkbQ_") + tname<T>(), (size_t)N * kp0, &Q));

  std::vector<double> alpha, t;
  std::vector<std::pair<int, int>> breaks;
  // breakdown: the value is 0 or at most bd_rel times the largest entry of C
  // accepted so far (t_1 = ||y|| is not an entry of C and is excluded)
  auto is_bd = [&](double val, double scale) { return val <= bd_rel * scale || val == 0.0; };

  // restart vector for side (0 = s, 1 = q) at step j into w, CGS2 against V[:, :m]
  auto restart = [&](int side, int j, T* w, const T* V, int m) -> kp_status {
    launch_philox_normals<T>(w, N, o->seed, (uint32_t)(2 * j + side), s);
    cgs2<T>(sc, w, V, N, m, N, s);
    double nr = 0;
    KP_TRY(read_norm(c, sc, s, &nr));
    if (nr > 0) launch_scale<T>(w, N, 1.0 / nr, s);
    breaks.push_back({side, j});
    return check_launch(c, "restart");
  };

  // start vector y -> s_1 = y / t_1
  if (o->y0) {
    KP_TRY(upload_block<T>(c, o->y0, N, S, s));
  } else {
    launch_philox_normals<T>(S, N, o->seed, 0u, s);
  }
  launch_norm2_partials<T>(S, N, sc.nrmp, s);
  double t1 = 0;
  KP_TRY(read_norm(c, sc, s, &t1));
  if (!(t1 > 0) || !std::isfinite(t1)) return set_err(c, KP_E_INVAL, "start vector has zero or non-finite norm");
  launch_scale<T>(S, N, 1.0 / t1, s);
  t.push_back(t1);

  // q = B^T s_1, alpha_1 = ||q||
  KP_TRY(op.gemv(c, 1, S, Q, nullptr, 0.0, s));
  launch_norm2_partials<T>(Q, N, sc.nrmp, s);
  double a1 = 0;
  KP_TRY(read_norm(c, sc, s, &a1));
  if (!std::isfinite(a1)) return set_err(c, KP_E_NUMERIC, "non-finite alpha_1");
  if (is_bd(a1, 0.0)) {
    a1 = 0.0;
    KP_TRY(restart(1, 1, Q, Q, 0));
  } else {
    launch_scale<T>(Q, N, 1.0 / a1, s);
  }
  alpha.push_back(a1);
  std::map<int, double> zeta, nu;
  zeta[1] = o->literal_init ? 1.0 : a1 * t1;
  nu[2] = o->literal_init ? 100.0 : INFINITY;
  double scale = a1;
  bool fired = false;

  for (int j = 2; j <= kp + 1; ++j) {
    KP_TRY(check_cancel(c));
    T* sj = S + N * (j - 1);
    const T* sprev = S + N * (j - 2);
    const T* qprev = Q + N * (j - 2);
    // s_j = B q_{j-1} - alpha_{j-1} s_{j-1}
    KP_TRY(op.gemv(c, 0, qprev, sj, sprev, alpha.back(), s));
    if (o->reorth == 1)
      cgs2<T>(sc, sj, S, N, j - 1, N, s);
    else
      launch_norm2_partials<T>(sj, N, sc.nrmp, s);
    double tj = 0;
    KP_TRY(read_norm(c, sc, s, &tj));
    if (!std::isfinite(tj)) return set_err(c, KP_E_NUMERIC, "non-finite t_j");
    if (is_bd(tj, scale)) {
      tj = 0.0;
      KP_TRY(restart(0, j, sj, S, j - 1));
    } else {
      launch_scale<T>(sj, N, 1.0 / tj, s);
    }
    t.push_back(tj);
    scale = std::max(scale, tj);
    if (j <= kp) {
      T* qj = Q + N * (j - 1);
      // q_j = B^T s_j - t_j q_{j-1}, reorthogonalized against Q (step 6)
      KP_TRY(op.gemv(c, 1, sj, qj, qprev, tj, s));
      cgs2<T>(sc, qj, Q, N, j - 1, N, s);
      double aj = 0;
      KP_TRY(read_norm(c, sc, s, &aj));
      if (!std::isfinite(aj)) return set_err(c, KP_E_NUMERIC, "non-finite alpha_j");
      if (is_bd(aj, scale)) {
        aj = 0.0;
        KP_TRY(restart(1, j, qj, Q, j - 1));
      } else {
        launch_scale<T>(qj, N, 1.0 / aj, s);
      }
      alpha.push_back(aj);
      scale = std::max(scale, aj);
      zeta[j] = aj * tj;
      nu[j + 1] = std::sqrt(zeta[j] * zeta[j - 1]);
      if (o->auto_k && !fired && j > o->k_min && (j - 1) != kp) {
        if (nu[j + 1] > nu[j] || nu[j] < o->tau) {
          fired = true;
          k = std::min(j, k_in);
          kp = k + p;
        }
      }
    }
  }
  KP_TRY(check_launch(c, "egkb loop"));

  // C ((kp+1) x kp lower bidiagonal) and its SVD in FP64 on the device
  std::vector<double> C((size_t)(kp + 1) * kp, 0.0);
  for (int i = 0; i < kp; ++i) {
    C[i + (size_t)(kp + 1) * i] = alpha[i];
    C[i + 1 + (size_t)(kp + 1) * i] = t[i + 1];
  }
  double *dC, *Uc, *sig, *Vc;
  int* sweeps;
  KP_TRY(wsT(c, "smallA", 64 * 64, &dC));
  KP_TRY(wsT(c, "smallU", 64 * 64, &Uc));
  KP_TRY(wsT(c, "smallS", 64, &sig));
  KP_TRY(wsT(c, "smallV", 64 * 64, &Vc));
  KP_TRY(wsT(c, "sweeps", 4, &sweeps));
  KP_HIP(c, hipMemcpyAsync(dC, C.data(), sizeof(double) * C.size(), hipMemcpyHostToDevice, s));
  launch_jacobi_svd(dC, kp + 1, kp, Uc, sig, Vc, sweeps, s);
  KP_TRY(check_launch(c, "jacobi_svd"));

  const int kout = std::min(k, f->k_cap);
  double *Ud, *Vd;
  KP_TRY(wsT(c, "Ud", (size_t)N * kout, &Ud));
  KP_TRY(wsT(c, "Vd", (size_t)N * kout, &Vd));
  launch_small_gemm<T, double>(S, N, kp + 1, Uc, kp + 1, kout, N, Ud, N, s);
  launch_small_gemm<T, double>(Q, N, kp, Vc, kp, kout, N, Vd, N, s);
  KP_TRY(check_launch(c, "small_gemm"));
  KP_TRY(write_factors(c, Ud, Vd, sig, n, kout, f, s));
  KP_HIP(c, hipMemcpyAsync(c->pinned, sig, sizeof(double) * kout, hipMemcpyDeviceToHost, s));
  if (f->diag && f->diag->basis_u)
    KP_HIP(c, hipMemcpyAsync(f->diag->basis_u, S, sizeof(T) * N * (kp + 1),
                             hipMemcpyDeviceToDevice, s));
  if (f->diag && f->diag->basis_v)
    KP_HIP(c, hipMemcpyAsync(f->diag->basis_v, Q, sizeof(T) * N * kp, hipMemcpyDeviceToDevice, s));
  KP_HIP(c, hipStreamSynchronize(s));
  for (int i = 0; i < kout; ++i) f->sigma[i] = c->pinned[i];
  f->k = kout;
  if (kp_diag* d = f->diag) {
    for (int i = 0; i < kp && i < d->cap; ++i) if (d->alpha) d->alpha[i] = alpha[i];
    for (int i = 0; i < kp + 1 && i < d->cap; ++i) if (d->t) d->t[i] = t[i];
    d->kp = kp;
    d->nbreak = (int)breaks.size();
    for (int i = 0; i < (int)breaks.size() && i < 128; ++i) {
      d->break_side[i] = breaks[i].first;
      d->break_step[i] = breaks[i].second;
    }
    d->ms_total = timer.stop();
  }
  return breaks.empty() ? KP_OK : KP_W_BREAKDOWN;
}

// ---------------------------------------------------------------------------
// Block Golub-Kahan bidiagonalization (Golub, Luk & Overton 1981) with b start
// vectors: the block analogue of Algorithm 1 with full reorthogonalization.
// U_1 = orth(Y); for j = 1 .. nb: V_j L_j^T = B^T U_j - V_{j-1} R_{j-1}^T and
// U_{j+1} R_j = B V_j - U_j L_j, so that B [V_1 .. V_nb] = [U_1 .. U_nb+1] C with
// C block lower bidiagonal ((nb+1) b x nb b). Every new block is orthonormalized
// column by column with two classical Gram-Schmidt passes against all earlier
// vectors of its basis; the summed coefficients on the block's own earlier
// columns and the column norms are the entries of L_j^T (resp. R_j). Each
// column's norm is read back to take the breakdown decision of Algorithm 1
// (0, or at most bd_rel times the largest norm so far in C); a broken-down
// column stores 0 and is replaced by a Philox vector (stream 2(m+1) for column m
// of U, 2(m+1)+1 for column m of V) orthogonalized twice against its basis. The
// products with B and B^T are block products of b columns (the MFMA kernels),
// which is what the block form buys over Algorithm 1's matrix-vector products.
template <typename T>
kp_status egkb_block_impl(kp_ctx* c, const RmatOp<T>& op, const kp_gkb_opts* o, kp_factors* f,
                          hipStream_t s) {
  Timer timer(s);
  const int n = op.n;
  const long N = (long)n * n;
  const int b = o->block;
  const int k_in = o->k;
  int k = o->k;
  int nb = (o->k + o->p + b - 1) / b;
  const int nb0 = nb;
  const int kp0 = nb0 * b;
  const int rows0 = kp0 + b;          // C is allocated for the initial k_p
  const double u = (sizeof(T) == 4) ? std::ldexp(1.0, -24) : std::ldexp(1.0, -53);
  const double bd_rel = o->bd_rel > 0 ? o->bd_rel : 1e2 * u;

  Scratch sc;
  KP_TRY(get_scratch(c, &sc));
  double* hcol = sc.h;
  double* h2 = sc.h + 64;
  T *U = nullptr, *V = nullptr;
  KP_TRY(wsT(c, std::string("egkbS_") + tname<T>(), (size_t)N * rows0, &U));
  KP_TRY(wsT(c, std::string("egkbQ_") + tname<T>(), (size_t)N * kp0, &V));

  std::vector<double> C((size_t)rows0 * kp0, 0.0);
  std::vector<double> tcol;            // stored norm of every U column, in order
  std::map<int, double> zeta, nu;
  bool fired = false;
  std::vector<std::pair<int, int>> breaks;
  double scale = 0.0;

  // Column m of basis B0 (ld N) against its m predecessors, two CGS passes;
  // returns the norm and the coefficients on the last `nown` predecessors.
  auto gs_column = [&](T* B0, int m, int nown, double* own, double* nr) -> kp_status {
    T* w = B0 + N * m;
    if (m == 0) {
      launch_norm2_partials<T>(w, N, sc.nrmp, s);
    } else {
      launch_multidot<T>(B0, N, m, w, N, sc.partials, s);
      launch_project_out_red<T>(w, B0, N, m, sc.partials, hcol, nullptr, N, nullptr, s);
      launch_multidot<T>(B0, N, m, w, N, sc.partials, s);
      launch_project_out_red<T>(w, B0, N, m, sc.partials, h2, hcol, N, sc.nrmp, s);
    }
    launch_reduce_partials(sc.nrmp, 1, sc.scal, 0, s);
    KP_TRY(check_launch(c, "block_gs"));
    KP_HIP(c, hipMemcpyAsync(c->pinned, sc.scal, sizeof(double), hipMemcpyDeviceToHost, s));
    if (nown > 0)
      KP_HIP(c, hipMemcpyAsync(c->pinned + 1, hcol + (m - nown), sizeof(double) * nown,
                               hipMemcpyDeviceToHost, s));
    KP_HIP(c, hipStreamSynchronize(s));
    *nr = std::sqrt(c->pinned[0]);
    for (int i = 0; i < nown; ++i) own[i] = c->pinned[1 + i];
    return KP_OK;
  };

  // Orthonormalize column m (side 0 = U, 1 = V); *diag = stored norm.
  auto new_column = [&](T* B0, int m, int nown, int side, bool in_c, double* own,
                        double* diag) -> kp_status {
    double nr = 0.0;
    KP_TRY(gs_column(B0, m, nown, own, &nr));
    if (!std::isfinite(nr)) return set_err(c, KP_E_NUMERIC, "non-finite block column norm");
    T* w = B0 + N * m;
    if (nr == 0.0 || (in_c && nr <= bd_rel * scale)) {
      breaks.push_back({side, m});
      launch_philox_normals<T>(w, N, o->seed, (uint32_t)(2 * (m + 1) + side), s);
      cgs2<T>(sc, w, B0, N, m, N, s);
      double g = 0.0;
      KP_TRY(read_norm(c, sc, s, &g));
      if (g > 0) launch_scale<T>(w, N, 1.0 / g, s);
      *diag = 0.0;
    } else {
      launch_scale<T>(w, N, 1.0 / nr, s);
      *diag = nr;
      if (in_c) scale = std::max(scale, nr);
    }
    return check_launch(c, "block_column");
  };

  auto product = [&](int tr, const T* X, T* Y) -> kp_status {
    return b == 1 ? op.gemv(c, tr, X, Y, nullptr, 0.0, s) : op.block(c, tr, X, Y, b, s);
  };

  // start block U_1 = orth(Y) (its own triangular factor is not part of C)
  if (o->y0) {
    KP_TRY(upload_block<T>(c, o->y0, N * b, U, s));
  } else {
    for (int col = 0; col < b; ++col)
      launch_philox_normals<T>(U + N * col, N, o->seed, col == 0 ? 0u : 0x80000000u + col, s);
  }
  double own[64], d = 0.0;
  for (int col = 0; col < b; ++col) {
    KP_TRY(new_column(U, col, 0, 0, false, own, &d));
    tcol.push_back(d);
  }

  for (int j = 0; j < nb; ++j) {
    KP_TRY(check_cancel(c));
    const long jb = (long)j * b;
    // V_{j+1} L^T = B^T U_{j+1} (minus the earlier V, through the Gram-Schmidt)
    KP_TRY(product(1, U + N * jb, V + N * jb));
    double logsum = 0.0;
    for (int col = 0; col < b; ++col) {
      KP_TRY(new_column(V, (int)jb + col, col, 1, true, own, &d));
      for (int r = 0; r < col; ++r) C[(jb + col) + (size_t)rows0 * (jb + r)] = own[r];
      C[(jb + col) + (size_t)rows0 * (jb + col)] = d;
      logsum += std::log(d * tcol[jb + col]);     // -inf for a stored 0
    }
    // stopping rule of Algorithm 1 with one value per block: zeta_J = the
    // geometric mean of alpha t over the block's columns
    const int J = j + 1;
    zeta[J] = std::exp(logsum / b);
    if (J == 1) {
      if (o->literal_init) zeta[1] = 1.0;
      nu[2] = o->literal_init ? 100.0 : INFINITY;
    } else {
      nu[J + 1] = std::sqrt(zeta[J] * zeta[J - 1]);
      if (o->auto_k && !fired && J * b > o->k_min && (nu[J + 1] > nu[J] || nu[J] < o->tau)) {
        fired = true;
        k = std::min(J * b, k_in);
        nb = (k + o->p + b - 1) / b;
      }
    }
    // U_{j+2} R = B V_{j+1} (minus the earlier U)
    const long ub = jb + b;
    KP_TRY(product(0, V + N * jb, U + N * ub));
    for (int col = 0; col < b; ++col) {
      KP_TRY(new_column(U, (int)ub + col, col, 0, true, own, &d));
      for (int r = 0; r < col; ++r) C[(ub + r) + (size_t)rows0 * (jb + col)] = own[r];
      C[(ub + col) + (size_t)rows0 * (jb + col)] = d;
      tcol.push_back(d);
    }
  }
  KP_TRY(check_launch(c, "block egkb loop"));
  // the leading (nb+1) b x nb b part of C (nb may have shrunk by the rule)
  const int kp = nb * b;
  const int rows = kp + b;
  if (rows != rows0) {
    std::vector<double> Cc((size_t)rows * kp);
    for (int col = 0; col < kp; ++col)
      for (int r = 0; r < rows; ++r) Cc[r + (size_t)rows * col] = C[r + (size_t)rows0 * col];
    C.swap(Cc);
  }

  double *dC, *Uc, *sig, *Vc;
  int* sweeps;
  KP_TRY(wsT(c, "smallA", 64 * 64, &dC));
  KP_TRY(wsT(c, "smallU", 64 * 64, &Uc));
  KP_TRY(wsT(c, "smallS", 64, &sig));
  KP_TRY(wsT(c, "smallV", 64 * 64, &Vc));
  KP_TRY(wsT(c, "sweeps", 4, &sweeps));
  KP_HIP(c, hipMemcpyAsync(dC, C.data(), sizeof(double) * C.size(), hipMemcpyHostToDevice, s));
  launch_jacobi_svd(dC, rows, kp, Uc, sig, Vc, sweeps, s);
  KP_TRY(check_launch(c, "jacobi_svd"));

  const int kout = std::min(k, f->k_cap);
  double *Ud, *Vd;
  KP_TRY(wsT(c, "Ud", (size_t)N * kout, &Ud));
  KP_TRY(wsT(c, "Vd", (size_t)N * kout, &Vd));
  launch_small_gemm<T, double>(U, N, rows, Uc, rows, kout, N, Ud, N, s);
  launch_small_gemm<T, double>(V, N, kp, Vc, kp, kout, N, Vd, N, s);
  KP_TRY(check_launch(c, "small_gemm"));
  KP_TRY(write_factors(c, Ud, Vd, sig, n, kout, f, s));
  KP_HIP(c, hipMemcpyAsync(c->pinned, sig, sizeof(double) * kout, hipMemcpyDeviceToHost, s));
  if (f->diag && f->diag->basis_u)
    KP_HIP(c, hipMemcpyAsync(f->diag->basis_u, U, sizeof(T) * N * rows, hipMemcpyDeviceToDevice, s));
  if (f->diag && f->diag->basis_v)
    KP_HIP(c, hipMemcpyAsync(f->diag->basis_v, V, sizeof(T) * N * kp, hipMemcpyDeviceToDevice, s));
  KP_HIP(c, hipStreamSynchronize(s));
  for (int i = 0; i < kout; ++i) f->sigma[i] = c->pinned[i];
  f->k = kout;
  if (kp_diag* dg = f->diag) {
    dg->kp = kp;
    dg->nbreak = (int)breaks.size();
    for (int i = 0; i < (int)breaks.size() && i < 128; ++i) {
      dg->break_side[i] = breaks[i].first;
      dg->break_step[i] = breaks[i].second;
    }
    dg->ms_total = timer.stop();
  }
  return breaks.empty() ? KP_OK : KP_W_BREAKDOWN;
}

template <typename T>
kp_status gkb_run(kp_ctx* c, const RmatOp<T>& op, const kp_gkb_opts* o, kp_factors* f,
                  hipStream_t s) {
  return o->block >= 1 ? egkb_block_impl<T>(c, op, o, f, s) : egkb_impl<T>(c, op, o, f, s);
}

// ---------------------------------------------------------------------------
// RSVD (Algorithm 2): Y = orth(B F); q times Z = orth(B^T Y), Y = orth(B Z);
// H^T = B^T Y = Q_h R_h (Householder TSQR), R_h^T = U_r S V_r^T (Jacobi), so
// H = U_r S (Q_h V_r)^T: U_k = Y U_r[:, :k], V_k = Q_h V_r[:, :k].
// With KP_BF16 / KP_F16 every product with B runs on the 16-bit kernel (vectors
// stay FP32). The optional refinement reorthogonalizes V_k once more, forms
// W = B V_k with the FP32 (FP64) kernel and takes the SVD of W through its QR:
// W = Q_w R_w, R_w = U_w S Z^T, so the triplets become (Q_w U_w, S, V_k Z)
// (one-sided Rayleigh-Ritz on range(V_k)).
template <typename T>
kp_status rsvd_impl(kp_ctx* c, const RmatOp<T>& op, const kp_rsvd_opts* o, kp_factors* f,
                    hipStream_t s) {
  Timer timer(s);
  const int n = op.n;
  const long N = (long)n * n;
  const int k = o->k;
  const int kp = o->k + o->p;
  const kp_prec pp = o->prec;
  const kp_blur* b = op.blur;            // generated operator only (16-bit modes)
  Grids<__hip_bfloat16> gb;
  Grids<__half> gh;
  if (pp == KP_BF16) KP_TRY(build_grids<__hip_bfloat16>(c, b, op.dpsf, s, &gb));
  if (pp == KP_F16) KP_TRY(build_grids<__half>(c, b, op.dpsf, s, &gh));
  auto prod = [&](int tr, const T* X, T* Yo, int nc) -> kp_status {
    if constexpr (std::is_same<T, float>::value) {
      if (pp == KP_BF16) return block_product16<__hip_bfloat16>(c, gb, n, tr, X, Yo, nc, s);
      if (pp == KP_F16) return block_product16<__half>(c, gh, n, tr, X, Yo, nc, s);
      if (pp == KP_F16X3) return split16_product(c, b, op.dpsf, n, tr, X, Yo, nc, s);
    }
    return op.block(c, tr, X, Yo, nc, s);
  };
  T *Y = nullptr, *Z = nullptr;
  KP_TRY(wsT(c, std::string("rsvdY_") + tname<T>(), (size_t)N * kp, &Y));
  KP_TRY(wsT(c, std::string("rsvdZ_") + tname<T>(), (size_t)N * kp, &Z));
  if (o->F) {
    KP_TRY(upload_block<T>(c, o->F, N * kp, Z, s));
  } else {
    for (int col = 0; col < kp; ++col)
      launch_philox_normals<T>(Z + N * col, N, o->seed, 0x40000000u + (uint32_t)col, s);
  }
  auto qr = [&](T* Wb, int mm, double* Rf) { return tsqr_qr<T>(c, Wb, N, mm, Rf, s); };
  KP_TRY(prod(0, Z, Y, kp));
  KP_TRY(qr(Y, kp, nullptr));
  for (int it = 0; it < o->q; ++it) {
    KP_TRY(check_cancel(c));
    KP_TRY(prod(1, Y, Z, kp));
    KP_TRY(qr(Z, kp, nullptr));
    KP_TRY(prod(0, Z, Y, kp));
    KP_TRY(qr(Y, kp, nullptr));
  }
  if (f->diag && f->diag->basis_u)
    KP_HIP(c, hipMemcpyAsync(f->diag->basis_u, Y, sizeof(T) * N * kp, hipMemcpyDeviceToDevice, s));
  KP_TRY(check_cancel(c));
  KP_TRY(prod(1, Y, Z, kp));   // H^T
  double *Rh, *RhT, *Ur, *sig, *Vr;
  int* sweeps;
  KP_TRY(wsT(c, "smallR", 64 * 64, &Rh));
  KP_TRY(wsT(c, "smallA", 64 * 64, &RhT));
  KP_TRY(wsT(c, "smallU", 64 * 64, &Ur));
  KP_TRY(wsT(c, "smallS", 64, &sig));
  KP_TRY(wsT(c, "smallV", 64 * 64, &Vr));
  KP_TRY(wsT(c, "sweeps", 4, &sweeps));
  KP_TRY(qr(Z, kp, Rh));
  launch_transpose_small(Rh, kp, kp, RhT, s);
  launch_jacobi_svd(RhT, kp, kp, Ur, sig, Vr, sweeps, s);
  KP_TRY(check_launch(c, "jacobi_svd"));
  const int kout = std::min(k, f->k_cap);
  double *Ud, *Vd;
  KP_TRY(wsT(c, "Ud", (size_t)N * kout, &Ud));
  KP_TRY(wsT(c, "Vd", (size_t)N * kout, &Vd));
  launch_small_gemm<T, double>(Y, N, kp, Ur, kp, kout, N, Ud, N, s);
  launch_small_gemm<T, double>(Z, N, kp, Vr, kp, kout, N, Vd, N, s);
  KP_TRY(check_launch(c, "small_gemm"));
  if (o->refine) {
    T* Vf = Y;   // N x kout, reuses the sketch buffers
    T* W = Z;
    launch_convert<double, T>(Vd, Vf, N * kout, s);
    KP_TRY(qr(Vf, kout, nullptr));
    if constexpr (std::is_same<T, float>::value) {
      if ((o->refine == 2 || pp == KP_F16X3) && b)
        KP_TRY(split16_product(c, b, op.dpsf, n, 0, Vf, W, kout, s));
      else KP_TRY(op.block(c, 0, Vf, W, kout, s));
    } else {
      KP_TRY(op.block(c, 0, Vf, W, kout, s));
    }
    KP_TRY(qr(W, kout, Rh));
    launch_jacobi_svd(Rh, kout, kout, Ur, sig, Vr, sweeps, s);
    launch_small_gemm<T, double>(W, N, kout, Ur, kout, kout, N, Ud, N, s);
    launch_small_gemm<T, double>(Vf, N, kout, Vr, kout, kout, N, Vd, N, s);
    KP_TRY(check_launch(c, "refine"));
  }
  KP_TRY(write_factors(c, Ud, Vd, sig, n, kout, f, s));
  KP_HIP(c, hipMemcpyAsync(c->pinned, sig, sizeof(double) * kout, hipMemcpyDeviceToHost, s));
  KP_HIP(c, hipStreamSynchronize(s));
  for (int i = 0; i < kout; ++i) f->sigma[i] = c->pinned[i];
  f->k = kout;
  if (kp_diag* d = f->diag) {
    d->kp = kp;
    d->nbreak = 0;
    d->ms_total = timer.stop();
  }
  return KP_OK;
}

kp_status validate_apply_factors(kp_ctx* c, const kp_factors* f) {
  if (!f) return set_err(c, KP_E_INVAL, "factors is NULL");
  if (f->n < 2 || f->n > 8192) return set_err(c, KP_E_INVAL, "factors.n must be in [2, 8192]");
  if (f->k < 1 || f->k > f->k_cap) return set_err(c, KP_E_INVAL, "need 1 <= factors.k <= k_cap");
  if (!f->Ax || !f->Ay) return set_err(c, KP_E_INVAL, "factor buffers are NULL");
  if (f->factor_prec != KP_F64) return set_err(c, KP_E_INVAL, "kp_apply / sb_solve need KP_F64 factors");
  return KP_OK;
}

// Split Bregman (Algorithm 3 if iso == 0, Algorithm 4 if iso == 1) with CGLS
// (Algorithm 5). x^(0) = b enters only RC_SB of the first outer iteration; CGLS
// starts every outer iteration from 0. The host queues L_max x I_max
// iterations; device flags turn the remainder into no-ops once RC_CGLS <
// tau_cgls (per outer iteration) or RC_SB < tau_sb, and the host polls the
// flags every few iterations to stop queueing.
// The blur operator of a split Bregman solve: the Kronecker sum A_k (factors)
// or an explicit N x N matrix A in HBM (the paper's method (i) of Table 1).
// apply(tr, v, P, flags, s) enqueues op(A) v as `ngroups` partial images in P.
// The blur's FFT products (fft.hip): padded sizes, workspace, the twiddle
// table and the spectrum of P, enqueued on s.
kp_status fft_conv_plan(kp_ctx* c, const kp_blur* b, hipStream_t s, FftConv* p) {
  const int n = b->n;
  p->n = n;
  p->pu = b->pu;
  p->pv = b->pv;
  p->cu = b->cu;
  p->cv = b->cv;
  p->bc = b->bc;
  p->e1 = n + b->pu - 1;
  p->e2 = n + b->pv - 1;
  auto lg = [](int e) {
    int l = 3;
    while ((1 << l) < e) ++l;
    return l;
  };
  if (p->e1 > kFftMaxLen || p->e2 > kFftMaxLen)
    return set_err(c, KP_E_INVAL, "FFT blur products need n + pu - 1 and n + pv - 1 <= 4096");
  p->l1 = lg(p->e1);
  p->l2 = lg(p->e2);
  const int M1 = 1 << p->l1, M2 = 1 << p->l2, h2 = M2 / 2 + 1;
  p->ls = (h2 + 15) & ~15;
  // one sequence (row pair, column) per workgroup from length 512 up: the
  // padded sizes leave only a few hundred sequences per pass, and more
  // workgroups beat longer ones (n = 256, M = 1024: 4 columns and 2 row
  // pairs per workgroup ran the CGLS iteration in 122 us, one each in 86 us)
  p->rp = std::max(1, 512 / M2);
  p->cb = std::max(1, 512 / M1);
  double2* tw = nullptr;
  KP_TRY(wsT(c, "fft_tw", (size_t)kFftMaxLen, &tw));
  p->tw = tw;
  KP_TRY(wsT(c, "fft_S", (size_t)p->e1 * p->ls, &p->S));
  KP_TRY(wsT(c, "fft_H", (size_t)h2 * M1, &p->H));
  p->G = nullptr;
  if (p->bc != KP_BC_ZERO) KP_TRY(wsT(c, "fft_G", (size_t)p->e1 * p->e2, &p->G));
  double* dpsf = nullptr;
  KP_TRY(upload_psf(c, b, s, &dpsf));
  fft_set_lds_limits();
  launch_fft_twiddles(tw, s);
  launch_fft_psf_spectrum(*p, dpsf, s);
  return check_launch(c, "fft plan");
}

struct SbOp {
  int n = 0;
  const kp_factors* f = nullptr;
  const double* A = nullptr;
  const FftConv* fc = nullptr;
  KpApplyPlan plan;
  double *Z = nullptr, *gv = nullptr, *tv = nullptr, *ty = nullptr;
  int ngroups() const { return (A || fc) ? 1 : plan.ngroups; }
  void apply(int tr, const double* v, double* P, const int* flags, int nflags,
             hipStream_t s) const {
    if (fc) {
      launch_fft_conv(*fc, tr, v, P, flags, nflags, s);
      return;
    }
    if (A) {
      // images are row-major (pixel (r, c) at r n + c); A acts on vec (r + n c)
      launch_transpose_image(v, tv, n, flags, nflags, s);
      launch_stored_gemv<double>(A, (long)n * n, tr, tv, ty, nullptr, 0.0, gv, s, flags, nflags);
      launch_transpose_image(ty, P, n, flags, nflags, s);
      return;
    }
    launch_kp_apply_parts((const double*)f->Ax, (const double*)f->Ay, n, f->k, tr, v, Z, P,
                          plan, flags, nflags, s);
  }
};

kp_status sb_check_opts(kp_ctx* c, const double* b, const sb_opts* o, double* x) {
  if (!b || !x || !o) return set_err(c, KP_E_INVAL, "b, x or opts is NULL");
  if (b == x) return set_err(c, KP_E_INVAL, "b and x must not alias");
  if (!(o->lambda > 0) || !(o->beta > 0) || !std::isfinite(o->lambda) || !std::isfinite(o->beta))
    return set_err(c, KP_E_INVAL, "lambda and beta must be positive and finite");
  if (o->L_max < 1 || o->I_max < 1) return set_err(c, KP_E_INVAL, "L_max and I_max must be >= 1");
  if (o->tau_sb < 0 || o->tau_cgls < 0) return set_err(c, KP_E_INVAL, "tolerances must be >= 0");
  return KP_OK;
}

kp_status sb_solve_impl(kp_ctx* c, SbOp& op, const double* b, const sb_opts* o, double* x,
                        sb_stats* st, hipStream_t s, int iso) {
  KP_HIP(c, hipSetDevice(c->device));
  Timer timer(s);
  const int n = op.n;
  const long NN = (long)n * n;
  double* img = nullptr;
  KP_TRY(wsT(c, "sb_img", (size_t)14 * NN, &img));
  double *P, *part, *scal;
  int* flags;
  if (op.fc) {
    KP_TRY(wsT(c, "kpP", (size_t)NN, &P));
  } else if (op.A) {
    KP_TRY(wsT(c, "kpP", (size_t)NN, &P));
    KP_TRY(wsT(c, "sb_gv", (size_t)stored_gemv_ws(NN), &op.gv));
    KP_TRY(wsT(c, "sb_tv", (size_t)2 * NN, &op.tv));
    op.ty = op.tv + NN;
  } else {
    KP_TRY(wsT(c, "kpZ", (size_t)op.f->k * NN, &op.Z));
    KP_TRY(wsT(c, "kpP", (size_t)op.f->k * NN, &P));
    op.plan = kp_apply_plan(n, op.f->k);
  }
  KP_TRY(wsT(c, "sb_part", (size_t)kRedBlocks * 4, &part));
  KP_TRY(wsT(c, "sb_scal", 8, &scal));
  KP_TRY(wsT(c, "sb_flags", 4, &flags));
  SBDev d;
  d.n = n;
  d.lam = o->lambda;
  d.thr = o->beta / (o->lambda * o->lambda);     // 1 / gamma, gamma = lambda^2 / beta
  d.iso = iso;
  d.tau_cgls = o->tau_cgls;
  d.tau_sb = o->tau_sb;
  d.b = b;
  double* AtB = img;
  d.AtB = AtB;
  d.x = img + NN;
  d.xprev = img + 2 * NN;
  d.r1 = img + 3 * NN;
  d.r2 = img + 4 * NN;
  d.r3 = img + 5 * NN;
  d.w = img + 6 * NN;
  d.f = img + 7 * NN;
  d.z1 = img + 8 * NN;
  d.t1 = img + 9 * NN;
  d.dx = img + 10 * NN;
  d.dy = img + 11 * NN;
  d.gx = img + 12 * NN;
  d.gy = img + 13 * NN;
  d.part = part;
  d.scal = scal;
  d.flags = flags;
  launch_fill(d.dx, 4 * NN, 0.0, s);                 // dx, dy, gx, gy (contiguous)
  launch_fill_small(scal, 8, 0.0, s);
  launch_fill_int(flags, 4, 0, s);
  KP_HIP(c, hipMemcpyAsync(d.xprev, b, sizeof(double) * NN, hipMemcpyDeviceToDevice, s));
  const char* genv = getenv("KPSB_SB_GRAPH");
  const bool use_graph = genv ? atoi(genv) == 1 : n <= 160;
  // the captured iterations must not reach the autotuner's timed samples: one
  // forward apply (overwritten below) settles the forward launch beforehand
  if (use_graph) op.apply(0, b, P, nullptr, 0, s);
  op.apply(1, b, P, nullptr, 0, s);
  launch_sum_parts(P, op.ngroups(), NN, AtB, s);
  KP_TRY(check_launch(c, "sb init"));
  const int poll = 8;
  int* hflags = reinterpret_cast<int*>(c->pinned);
  auto read_flags = [&]() -> kp_status {
    KP_HIP(c, hipMemcpyAsync(hflags, flags, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    KP_HIP(c, hipStreamSynchronize(s));
    return KP_OK;
  };
  const int ng = op.ngroups();
  auto cgls_iteration = [&](hipStream_t st) {
    op.apply(0, d.w, P, flags, 2, st);
    sb_launch_zn(d, P, ng, st);
    sb_launch_xr(d, st);
    op.apply(1, d.r1, P, flags, 2, st);
    sb_launch_f(d, P, ng, 2, st);
    sb_launch_w(d, st);
  };
  // `poll` CGLS iterations (8 x 8 kernels) are captured once per solve as a HIP
  // graph and replayed between the host's flag polls (finished iterations are
  // no-ops on the device either way); captured on a private stream (the
  // caller's may be the null stream) in thread-local mode, replayed on the
  // caller's stream. Used where launch latency dominates: n <= 160 (at n = 128,
  // 53.6 vs 56.7 us per iteration including the capture; equal at n >= 256).
  // KPSB_SB_GRAPH=1 / 0 forces it on / off.
  hipGraphExec_t chunk = nullptr;
  if (use_graph && o->I_max >= poll) {
    hipStream_t cs = nullptr;
    KP_HIP(c, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t gr = nullptr;
    hipError_t e;
    {
      std::shared_lock<std::shared_mutex> cap(capture_mutex());
      t_capturing = true;
      e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        for (int i = 0; i < poll; ++i) cgls_iteration(cs);
        e = hipStreamEndCapture(cs, &gr);
      }
      t_capturing = false;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&chunk, gr, nullptr, nullptr, 0);
    if (gr) (void)hipGraphDestroy(gr);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {   // no graph: the same kernels are launched one by one
      (void)hipGetLastError();
      if (chunk) (void)hipGraphExecDestroy(chunk);
      chunk = nullptr;
    }
  }
  struct ExecGuard {
    hipGraphExec_t& g;
    ~ExecGuard() {
      if (g) (void)hipGraphExecDestroy(g);
    }
  } guard{chunk};
  int replays = 0;
  for (int ell = 0; ell < o->L_max; ++ell) {
    KP_TRY(check_cancel(c));
    sb_launch_rhs(d, s);
    sb_launch_f(d, AtB, 1, 1, s);
    sb_launch_w_init(d, s);
    for (int it = 0; it < o->I_max;) {
      if (chunk && it + poll <= o->I_max) {
        KP_HIP(c, hipGraphLaunch(chunk, s));
        it += poll;
        ++replays;
      } else {
        cgls_iteration(s);
        it += 1;
      }
      if (it % poll == 0 && it < o->I_max) KP_TRY(check_cancel(c));
      if (o->tau_cgls > 0 && it % poll == 0 && it < o->I_max) {
        KP_TRY(check_launch(c, "cgls"));
        KP_TRY(read_flags());
        if (hflags[0] || hflags[1]) break;
      }
    }
    sb_launch_shrink(d, s);
    sb_launch_check(d, s);
    KP_TRY(check_launch(c, "sb iteration"));
    if (o->tau_sb > 0) {
      KP_TRY(read_flags());
      if (hflags[0]) break;
    }
  }
  KP_HIP(c, hipMemcpyAsync(x, d.x, sizeof(double) * NN, hipMemcpyDeviceToDevice, s));
  KP_TRY(read_flags());
  double rc = 0.0;
  KP_HIP(c, hipMemcpyAsync(c->pinned + 8, scal + 2, sizeof(double), hipMemcpyDeviceToHost, s));
  KP_HIP(c, hipStreamSynchronize(s));
  rc = c->pinned[8];
  if (st) {
    st->l_end = hflags[3];
    st->iota_total = hflags[2];
    st->rc_sb = rc;
    st->graph_replays = replays;
    st->reserved = 0;
  }
  (void)timer;
  return KP_OK;
}

kp_status sb_solve(kp_ctx* c, const kp_factors* f, const double* b, const sb_opts* o, double* x,
                   sb_stats* st, hipStream_t s, int iso) {
  KP_TRY(validate_apply_factors(c, f));
  KP_TRY(sb_check_opts(c, b, o, x));
  SbOp op;
  op.n = f->n;
  op.f = f;
  return sb_solve_impl(c, op, b, o, x, st, s, iso);
}

kp_status sb_solve_direct(kp_ctx* c, int n, const double* A, const double* b, const sb_opts* o,
                          double* x, sb_stats* st, hipStream_t s, int iso) {
  if (n < 2 || n > 1024) return set_err(c, KP_E_INVAL, "n must be in [2, 1024]");
  if (!A) return set_err(c, KP_E_INVAL, "A is NULL");
  KP_TRY(sb_check_opts(c, b, o, x));
  SbOp op;
  op.n = n;
  op.A = A;
  return sb_solve_impl(c, op, b, o, x, st, s, iso);
}

kp_status sb_solve_fft(kp_ctx* c, const kp_blur* bl, const double* b, const sb_opts* o,
                       double* x, sb_stats* st, hipStream_t s, int iso) {
  KP_TRY(validate_blur(c, bl));
  KP_TRY(sb_check_opts(c, b, o, x));
  KP_HIP(c, hipSetDevice(c->device));
  FftConv fc;
  KP_TRY(fft_conv_plan(c, bl, s, &fc));
  SbOp op;
  op.n = bl->n;
  op.fc = &fc;
  return sb_solve_impl(c, op, b, o, x, st, s, iso);
}

}  // namespace

namespace kpsb {

kp_ctx* ctx_new(int device, std::shared_ptr<kp_pool> pool, size_t budget) {
  if (hipSetDevice(device) != hipSuccess) return nullptr;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return nullptr;
  kp_ctx* c = new kp_ctx();
  c->device = device;
  c->lds_limit = prop.sharedMemPerBlock;
  if (prop.maxSharedMemoryPerMultiProcessor > 0 &&
      (size_t)prop.maxSharedMemoryPerMultiProcessor < c->lds_limit)
    c->lds_limit = prop.maxSharedMemoryPerMultiProcessor;
  if (pool) {
    c->pool = std::move(pool);
  } else {
    size_t freeb = 0, totalb = 0;
    if (hipMemGetInfo(&freeb, &totalb) != hipSuccess) {
      delete c;
      return nullptr;
    }
    c->pool = std::make_shared<kp_pool>();
    c->pool->budget = budget ? budget : (size_t)(0.9 * (double)freeb);
  }
  if (hipHostMalloc((void**)&c->pinned, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    delete c;
    return nullptr;
  }
  return c;
}

bool tuned_block_shape(kp_ctx* c, int n, BlockPlan* shape) {
  tune_set_no_timing(true);
  const int v = tune_pick(kTuneBlock, n, (int)sizeof(float), 0, kNumBlockVariants,
                          [](int) { return -1.0; });
  tune_set_no_timing(false);
  if (!plan_block_tj<float>(n, c->lds_limit, kBlockVariants[v].TJ, shape, kBlockVariants[v].TK))
    return false;
  shape->waves = kBlockVariants[v].waves;
  return true;
}

std::shared_mutex& capture_mutex() {
  static std::shared_mutex m;
  return m;
}

size_t ctx_held(const kp_ctx* c) {
  size_t h = 0;
  for (auto& kv : c->bufs) h += kv.second.bytes;
  return h;
}

void ctx_trim(kp_ctx* c) {
  (void)hipSetDevice(c->device);
  size_t freed = 0;
  {
    std::unique_lock<std::shared_mutex> nocap(capture_mutex());
    (void)hipDeviceSynchronize();
    for (auto& kv : c->bufs)
      if (kv.second.p) {
        (void)hipFree(kv.second.p);
        freed += kv.second.bytes;
      }
  }
  c->bufs.clear();
  std::lock_guard<std::mutex> lk(c->pool->m);
  c->pool->used -= freed;
}

void ctx_free(kp_ctx* c) {
  for (kp_ctx* w : c->workers) ctx_free(w);
  c->workers.clear();
  ctx_trim(c);
  std::unique_lock<std::shared_mutex> nocap(capture_mutex());
  if (c->pinned) (void)hipHostFree(c->pinned);
  for (auto& r : c->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
  delete c;
}

}  // namespace kpsb

// ===========================================================================
extern "C" {

const char* kp_version(void) { return "kpsb 0.1 (gfx950)"; }

kp_status kp_tune_report(char* out, size_t cap) {
  if (!out || cap == 0) return KP_E_INVAL;
  const std::string t = tune_table();
  const size_t m = t.size() < cap - 1 ? t.size() : cap - 1;
  std::memcpy(out, t.data(), m);
  out[m] = 0;
  return KP_OK;
}

kp_status kp_ctx_create(int device, size_t hbm_budget_bytes, kp_ctx** out) {
  if (!out) return KP_E_INVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return KP_E_DEVICE;
  kp_ctx* c = ctx_new(device, nullptr, hbm_budget_bytes);
  if (!c) return KP_E_DEVICE;
  // the device address of this device's static scratch (device current here)
  if (scratch_address(device, &c->scratch) != hipSuccess) {
    ctx_free(c);
    return KP_E_DEVICE;
  }
  *out = c;
  return KP_OK;
}

kp_status kp_ctx_destroy(kp_ctx* c) {
  if (!c) return KP_E_INVAL;
  ctx_free(c);
  return KP_OK;
}

const char* kp_last_error(const kp_ctx* c) { return c ? c->err.c_str() : "null context"; }

kp_status kp_cancel(kp_ctx* c) {
  if (!c) return KP_E_INVAL;
  c->cancel.store(1, std::memory_order_release);
  return KP_OK;
}

kp_status kp_ctx_workspace(const kp_ctx* c, size_t* held) {
  if (!c || !held) return KP_E_INVAL;
  *held = ctx_held(c);
  return KP_OK;
}

kp_status kp_prof_enable(kp_ctx* c, int enable) {
  if (!c) return KP_E_INVAL;
  c->prof = enable != 0;
  for (kp_ctx* w : c->workers) w->prof = c->prof;
  return KP_OK;
}

namespace {
void prof_collect(kp_ctx* c, kp_ctx* into) {
  for (auto& r : c->recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      into->acc_ms[r.cls] += ms;
      into->acc_n[r.cls] += 1;
      into->acc_flops[r.cls] += r.flops;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  c->recs.clear();
}
}  // namespace

kp_status kp_prof_read(kp_ctx* c, kp_prof* out, int reset) {
  if (!c || !out) return KP_E_INVAL;
  KP_HIP(c, hipSetDevice(c->device));
  {
    std::unique_lock<std::shared_mutex> nocap(capture_mutex());
    KP_HIP(c, hipDeviceSynchronize());
  }
  prof_collect(c, c);
  for (kp_ctx* w : c->workers) prof_collect(w, c);
  for (int i = 0; i < 4; ++i) {
    out->ms[i] = c->acc_ms[i];
    out->launches[i] = c->acc_n[i];
    out->flops[i] = c->acc_flops[i];
    if (reset) {
      c->acc_ms[i] = 0;
      c->acc_n[i] = 0;
      c->acc_flops[i] = 0;
    }
  }
  return KP_OK;
}

namespace {
kp_status check_rmat_apply(kp_ctx* c, const kp_blur* b, int32_t ncols, const void* X, void* Y) {
  KP_TRY(validate_blur(c, b));
  if (ncols < 1 || ncols > 4096) return set_err(c, KP_E_INVAL, "ncols must be in [1, 4096]");
  if (!X || !Y) return set_err(c, KP_E_INVAL, "X or Y is NULL");
  if (X == Y) return set_err(c, KP_E_INVAL, "X and Y must not alias");
  return KP_OK;
}

// The workspace an FP32 / FP64 kp_rmat_apply requests, in the order and the
// 256-byte granules in which ws() carves it: the PSF copy (or the finiteness
// flag of a device PSF), per term the grids of R and R^T (with compaction their
// support boxes and the box reduction's partials; for one FP32 column the
// matrix-vector kernel's staging vector), and with several terms the reversed
// input and three term outputs of multi_term.
size_t rmat_apply_ws_bytes(const kp_blur* b, kp_prec prec, int ncols) {
  auto r = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const int n = b->n;
  const size_t es = prec == KP_F64 ? sizeof(double) : sizeof(float);
  const RmatTerms tm = make_terms(b->bc, n);
  const size_t ldg = (size_t)grid_ld(n);
  size_t need = b->psf_on_device ? r(4 * sizeof(int)) : r(sizeof(double) * b->pu * b->pv);
  for (int t = 0; t < tm.nterm; ++t) {
    need += 2 * r(ldg * ldg * es);
    if (b->compact) need += r(sizeof(int) * (size_t)grid_box_parts()) + r(8 * sizeof(int));
    if (ncols == 1 && prec == KP_F32) need += r(sizeof(float) * (size_t)gemv_sx_xt_len(n));
  }
  if (tm.nterm > 1) need += 4 * r((size_t)n * n * ncols * es);
  return need;
}

kp_status rmat_apply_body(kp_ctx* c, const kp_blur* b, int transpose, kp_prec prec,
                          int32_t ncols, const void* X, void* Y, hipStream_t s) {
  KP_HIP(c, hipSetDevice(c->device));
  const int n = b->n;
  if (prec == KP_F32) {
    Grids<float> g;
    KP_TRY(prep_grids<float>(c, b, s, &g));
    if (ncols == 1)
      return gemv_product<float>(c, g, n, transpose, (const float*)X, (float*)Y, nullptr, 0.0, s);
    return block_product<float>(c, g, n, transpose, (const float*)X, (float*)Y, ncols, s);
  }
  if (prec == KP_F64) {
    Grids<double> g;
    KP_TRY(prep_grids<double>(c, b, s, &g));
    if (ncols == 1)
      return gemv_product<double>(c, g, n, transpose, (const double*)X, (double*)Y, nullptr,
                                  0.0, s);
    return block_product<double>(c, g, n, transpose, (const double*)X, (double*)Y, ncols, s);
  }
  if (prec == KP_BF16 || prec == KP_F16) {
    double* dpsf = nullptr;
    KP_TRY(upload_psf(c, b, s, &dpsf));
    if (prec == KP_BF16) {
      Grids<__hip_bfloat16> g;
      KP_TRY(build_grids<__hip_bfloat16>(c, b, dpsf, s, &g));
      return block_product16<__hip_bfloat16>(c, g, n, transpose, (const float*)X, (float*)Y, ncols, s);
    }
    Grids<__half> g;
    KP_TRY(build_grids<__half>(c, b, dpsf, s, &g));
    return block_product16<__half>(c, g, n, transpose, (const float*)X, (float*)Y, ncols, s);
  }
  return set_err(c, KP_E_INVAL, "precision not supported by kp_rmat_apply");
}

// Workspace requests of the context come from the static scratch while alive;
// the autotuner times nothing meanwhile.
struct ArenaScope {
  kp_ctx* c;
  ArenaScope(kp_ctx* ctx, void* base, size_t cap) : c(ctx) {
    c->arena_base = static_cast<char*>(base);
    c->arena_cap = cap;
    c->arena_used = 0;
    tune_set_no_timing(true);
  }
  ~ArenaScope() {
    c->arena_base = nullptr;
    c->arena_cap = c->arena_used = 0;
    tune_set_no_timing(false);
  }
};
}  // namespace

kp_status kp_rmat_apply(kp_ctx* c, const kp_blur* b, int transpose, kp_prec prec, int32_t ncols,
                        const void* X, void* Y, void* stream) {
  if (!c) return KP_E_INVAL;
  KP_TRY(check_rmat_apply(c, b, ncols, X, Y));
  return rmat_apply_body(c, b, transpose, prec, ncols, X, Y, (hipStream_t)stream);
}

kp_status kp_rmat_apply_noalloc(kp_ctx* c, const kp_blur* b, int transpose, kp_prec prec,
                                int32_t ncols, const void* X, void* Y, void* stream) {
  if (!c) return KP_E_INVAL;
  KP_TRY(check_rmat_apply(c, b, ncols, X, Y));
  if (prec != KP_F32 && prec != KP_F64)
    return set_err(c, KP_E_INVAL, "kp_rmat_apply_noalloc supports KP_F32 and KP_F64");
  if (!c->scratch) return set_err(c, KP_E_DEVICE, "the static scratch of this device is unavailable");
  const size_t need = rmat_apply_ws_bytes(b, prec, ncols);
  if (need > scratch_capacity())
    return set_err(c, KP_E_NOMEM, "this product needs " + std::to_string(need) +
                                      " bytes of scratch; the static scratch holds " +
                                      std::to_string(scratch_capacity()));
  ArenaScope arena(c, c->scratch, scratch_capacity());
  return rmat_apply_body(c, b, transpose, prec, ncols, X, Y, (hipStream_t)stream);
}

namespace {
kp_status check_gkb(kp_ctx* c, const kp_gkb_opts* o, kp_factors* f, int n) {
  if (!o) return set_err(c, KP_E_INVAL, "opts is NULL");
  KP_TRY(validate_factors_out(c, f, n));
  const long N = (long)n * n;
  if (o->k < 1 || o->p < 0) return set_err(c, KP_E_INVAL, "need k >= 1 and p >= 0");
  if (o->k + o->p + 1 > 64) return set_err(c, KP_E_INVAL, "k + p must be <= 63");
  if (o->k + o->p + 1 > N) return set_err(c, KP_E_INVAL, "k + p must be < n^2");
  if (o->reorth != 0 && o->reorth != 1) return set_err(c, KP_E_INVAL, "reorth must be 0 or 1");
  if (f->k_cap < 1) return set_err(c, KP_E_INVAL, "factors.k_cap must be >= 1");
  if (o->block < 0) return set_err(c, KP_E_INVAL, "block must be >= 0");
  long ny = N;
  if (o->block >= 1) {
    const long b = o->block;
    const long nb = (o->k + o->p + b - 1) / b;
    if ((nb + 1) * b > 64)
      return set_err(c, KP_E_INVAL, "block GKB needs (ceil((k+p)/b) + 1) * b <= 64");
    if ((nb + 1) * b > N) return set_err(c, KP_E_INVAL, "block GKB needs (nb + 1) * b <= n^2");
    ny = N * b;
  }
  if (o->y0)
    for (long e = 0; e < ny; ++e)
      if (!std::isfinite(o->y0[e])) return set_err(c, KP_E_NUMERIC, "y0 has a non-finite entry");
  if (o->prec != KP_F32 && o->prec != KP_F64)
    return set_err(c, KP_E_INVAL, "EGKB precision must be KP_F32 or KP_F64");
  return KP_OK;
}

kp_status check_rsvd(kp_ctx* c, const kp_rsvd_opts* o, kp_factors* f, int n) {
  if (!o) return set_err(c, KP_E_INVAL, "opts is NULL");
  KP_TRY(validate_factors_out(c, f, n));
  const long N = (long)n * n;
  if (o->k < 1 || o->p < 0 || o->q < 0) return set_err(c, KP_E_INVAL, "need k >= 1, p >= 0, q >= 0");
  if (o->k + o->p > 64) return set_err(c, KP_E_INVAL, "k + p must be <= 64");
  if (o->k + o->p > N) return set_err(c, KP_E_INVAL, "k + p must be <= n^2");
  if (f->k_cap < 1) return set_err(c, KP_E_INVAL, "factors.k_cap must be >= 1");
  if (o->refine < 0 || o->refine > 2) return set_err(c, KP_E_INVAL, "refine must be 0, 1 or 2");
  if (o->F)
    for (long e = 0; e < N * (o->k + o->p); ++e)
      if (!std::isfinite(o->F[e])) return set_err(c, KP_E_NUMERIC, "F has a non-finite entry");
  if (o->prec != KP_F32 && o->prec != KP_F64 && o->prec != KP_BF16 && o->prec != KP_F16 &&
      o->prec != KP_F16X3)
    return set_err(c, KP_E_INVAL, "unknown RSVD precision");
  return KP_OK;
}

kp_status check_stored(kp_ctx* c, int n, const void* R, kp_prec prec) {
  if (n < 2 || n > 1024) return set_err(c, KP_E_INVAL, "n must be in [2, 1024]");
  if (!R) return set_err(c, KP_E_INVAL, "R is NULL");
  if (prec != KP_F32 && prec != KP_F64)
    return set_err(c, KP_E_INVAL, "a stored R is KP_F32 or KP_F64");
  return KP_OK;
}
}  // namespace

kp_status kp_svd_gkb(kp_ctx* c, const kp_blur* b, const kp_gkb_opts* o, kp_factors* f,
                     void* stream) {
  if (!c) return KP_E_INVAL;
  KP_TRY(validate_blur(c, b));
  KP_TRY(check_gkb(c, o, f, b->n));
  KP_HIP(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  if (o->prec == KP_F32) {
    RmatOp<float> op;
    KP_TRY(make_generated_op<float>(c, b, s, &op));
    return gkb_run<float>(c, op, o, f, s);
  }
  RmatOp<double> op;
  KP_TRY(make_generated_op<double>(c, b, s, &op));
  return gkb_run<double>(c, op, o, f, s);
}

kp_status kp_svd_rsvd(kp_ctx* c, const kp_blur* b, const kp_rsvd_opts* o, kp_factors* f,
                      void* stream) {
  if (!c) return KP_E_INVAL;
  KP_TRY(validate_blur(c, b));
  KP_TRY(check_rsvd(c, o, f, b->n));
  KP_HIP(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  if (o->prec == KP_F64) {
    RmatOp<double> op;
    KP_TRY(make_generated_op<double>(c, b, s, &op));
    return rsvd_impl<double>(c, op, o, f, s);
  }
  RmatOp<float> op;
  KP_TRY(make_generated_op<float>(c, b, s, &op));
  return rsvd_impl<float>(c, op, o, f, s);
}

kp_status kp_blur_matrix(kp_ctx* c, const kp_blur* b, kp_prec prec, void* A, void* stream) {
  if (!c) return KP_E_INVAL;
  KP_TRY(validate_blur(c, b));
  KP_TRY(check_stored(c, b->n, A, prec));
  const int bc = b->bc;
  KP_HIP(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  double* dpsf = nullptr;
  KP_TRY(upload_psf(c, b, s, &dpsf));
  if (prec == KP_F64)
    launch_blur_matrix<double>(dpsf, b->pu, b->pv, b->cu, b->cv, b->n, bc, (double*)A, s);
  else
    launch_blur_matrix<float>(dpsf, b->pu, b->pv, b->cu, b->cv, b->n, bc, (float*)A, s);
  return check_launch(c, "blur_matrix");
}

kp_status kp_rmat_reorder(kp_ctx* c, int32_t n, kp_prec prec, const void* A, void* R,
                          void* stream) {
  if (!c) return KP_E_INVAL;
  KP_TRY(check_stored(c, n, R, prec));
  if (!A) return set_err(c, KP_E_INVAL, "A is NULL");
  const size_t bytes = (size_t)n * n * (size_t)n * n * (prec == KP_F64 ? 8 : 4);
  const char* a = (const char*)A;
  const char* r = (const char*)R;
  if (a < r + bytes && r < a + bytes) return set_err(c, KP_E_INVAL, "A and R overlap");
  KP_HIP(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  if (prec == KP_F64) launch_reorder<double>((const double*)A, (double*)R, n, s);
  else launch_reorder<float>((const float*)A, (float*)R, n, s);
  return check_launch(c, "reorder");
}

kp_status kp_rmat_apply_stored(kp_ctx* c, int32_t n, kp_prec prec, const void* R, int transpose,
                               int32_t ncols, const void* X, void* Y, void* stream) {
  if (!c) return KP_E_INVAL;
  KP_TRY(check_stored(c, n, R, prec));
  if (ncols < 1 || ncols > 4096) return set_err(c, KP_E_INVAL, "ncols must be in [1, 4096]");
  if (!X || !Y) return set_err(c, KP_E_INVAL, "X or Y is NULL");
  if (X == Y) return set_err(c, KP_E_INVAL, "X and Y must not alias");
  KP_HIP(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  if (prec == KP_F64) {
    RmatOp<double> op;
    KP_TRY(make_stored_op<double>(c, n, (const double*)R, &op));
    return ncols == 1 ? op.gemv(c, transpose, (const double*)X, (double*)Y, nullptr, 0.0, s)
                      : op.block(c, transpose, (const double*)X, (double*)Y, ncols, s);
  }
  RmatOp<float> op;
  KP_TRY(make_stored_op<float>(c, n, (const float*)R, &op));
  return ncols == 1 ? op.gemv(c, transpose, (const float*)X, (float*)Y, nullptr, 0.0, s)
                    : op.block(c, transpose, (const float*)X, (float*)Y, ncols, s);
}

kp_status kp_svd_gkb_stored(kp_ctx* c, int32_t n, const void* R, const kp_gkb_opts* o,
                            kp_factors* f, void* stream) {
  if (!c) return KP_E_INVAL;
  KP_TRY(check_gkb(c, o, f, n));
  KP_TRY(check_stored(c, n, R, o->prec));
  KP_HIP(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  if (o->prec == KP_F32) {
    RmatOp<float> op;
    KP_TRY(make_stored_op<float>(c, n, (const float*)R, &op));
    return gkb_run<float>(c, op, o, f, s);
  }
  RmatOp<double> op;
  KP_TRY(make_stored_op<double>(c, n, (const double*)R, &op));
  return gkb_run<double>(c, op, o, f, s);
}

kp_status kp_svd_rsvd_stored(kp_ctx* c, int32_t n, const void* R, const kp_rsvd_opts* o,
                             kp_factors* f, void* stream) {
  if (!c) return KP_E_INVAL;
  KP_TRY(check_rsvd(c, o, f, n));
  KP_TRY(check_stored(c, n, R, o->prec));
  KP_HIP(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  if (o->prec == KP_F32) {
    RmatOp<float> op;
    KP_TRY(make_stored_op<float>(c, n, (const float*)R, &op));
    return rsvd_impl<float>(c, op, o, f, s);
  }
  RmatOp<double> op;
  KP_TRY(make_stored_op<double>(c, n, (const double*)R, &op));
  return rsvd_impl<double>(c, op, o, f, s);
}

kp_status kp_apply(kp_ctx* c, const kp_factors* f, int transpose, const double* X, double* Y,
                   void* stream) {
  if (!c) return KP_E_INVAL;
  KP_TRY(validate_apply_factors(c, f));
  if (!X || !Y) return set_err(c, KP_E_INVAL, "X or Y is NULL");
  if (X == Y) return set_err(c, KP_E_INVAL, "X and Y must not alias");
  KP_HIP(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  const int n = f->n, k = f->k;
  double *Z, *P;
  KP_TRY(wsT(c, "kpZ", (size_t)k * n * n, &Z));
  KP_TRY(wsT(c, "kpP", (size_t)k * n * n, &P));
  {
    ProfScope ps(c, s, 2, 4.0 * k * (double)n * n * n);
    launch_kp_apply_ws((const double*)f->Ax, (const double*)f->Ay, n, k, transpose, X, Y, Z, P,
                       nullptr, 0, s);
  }
  return check_launch(c, "kp_apply");
}

kp_status sb_solve_aniso(kp_ctx* c, const kp_factors* f, const double* b, const sb_opts* o,
                         double* x, sb_stats* st, void* stream) {
  if (!c) return KP_E_INVAL;
  return sb_solve(c, f, b, o, x, st, (hipStream_t)stream, 0);
}

kp_status sb_solve_iso(kp_ctx* c, const kp_factors* f, const double* b, const sb_opts* o,
                       double* x, sb_stats* st, void* stream) {
  if (!c) return KP_E_INVAL;
  return sb_solve(c, f, b, o, x, st, (hipStream_t)stream, 1);
}

kp_status sb_solve_aniso_direct(kp_ctx* c, int32_t n, const double* A, const double* b,
                                const sb_opts* o, double* x, sb_stats* st, void* stream) {
  if (!c) return KP_E_INVAL;
  return sb_solve_direct(c, n, A, b, o, x, st, (hipStream_t)stream, 0);
}

kp_status sb_solve_iso_direct(kp_ctx* c, int32_t n, const double* A, const double* b,
                              const sb_opts* o, double* x, sb_stats* st, void* stream) {
  if (!c) return KP_E_INVAL;
  return sb_solve_direct(c, n, A, b, o, x, st, (hipStream_t)stream, 1);
}

kp_status kp_blur_apply(kp_ctx* c, const kp_blur* b, int transpose, const double* X, double* Y,
                        void* stream) {
  if (!c) return KP_E_INVAL;
  KP_TRY(validate_blur(c, b));
  if (transpose != 0 && transpose != 1) return set_err(c, KP_E_INVAL, "transpose must be 0 or 1");
  if (!X || !Y) return set_err(c, KP_E_INVAL, "X or Y is NULL");
  if (X == Y) return set_err(c, KP_E_INVAL, "X and Y must not alias");
  KP_HIP(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  FftConv fc;
  KP_TRY(fft_conv_plan(c, b, s, &fc));
  launch_fft_conv(fc, transpose, X, Y, nullptr, 0, s);
  return check_launch(c, "blur_apply");
}

kp_status sb_solve_aniso_fft(kp_ctx* c, const kp_blur* blur, const double* b, const sb_opts* o,
                             double* x, sb_stats* st, void* stream) {
  if (!c) return KP_E_INVAL;
  return sb_solve_fft(c, blur, b, o, x, st, (hipStream_t)stream, 0);
}

kp_status sb_solve_iso_fft(kp_ctx* c, const kp_blur* blur, const double* b, const sb_opts* o,
                           double* x, sb_stats* st, void* stream) {
  if (!c) return KP_E_INVAL;
  return sb_solve_fft(c, blur, b, o, x, st, (hipStream_t)stream, 1);
}

}  // extern "C"
