// Concurrent runtime of libkpsb: the batched KP-SVD call and the deblurring
// request server. Both run independent problems on worker contexts, each with
// its own HIP stream and workspace, from host threads of their own, so the
// kernels of different problems overlap on the device while each problem
// executes exactly the sequence of its single-problem entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "common.h"
#include "ctx.h"
#include "kpsb.h"

using namespace kpsb;

namespace {

kp_status fail(kp_ctx* c, kp_status st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

// Makes sure `c` has at least `nw` worker contexts (sharing c's HBM budget),
// each with a non-blocking stream of default priority.
kp_status ensure_workers(kp_ctx* c, int nw) {
  while ((int)c->workers.size() < nw) {
    kp_ctx* w = ctx_new(c->device, c->pool, 0);
    if (!w) return fail(c, KP_E_DEVICE, "creating a worker context failed");
    if (hipStreamCreateWithFlags(&w->own_stream, hipStreamNonBlocking) != hipSuccess) {
      ctx_free(w);
      return fail(c, KP_E_DEVICE, "creating a worker stream failed");
    }
    w->prof = c->prof;
    w->parent = c;   // a kp_cancel of c reaches the problems in progress
    c->workers.push_back(w);
  }
  return KP_OK;
}

int rank_of(int32_t method, const void* opts) {
  if (!opts) return 0;
  if (method == KP_METHOD_GKB) {
    auto* o = static_cast<const kp_gkb_opts*>(opts);
    return o->k + o->p;
  }
  auto* o = static_cast<const kp_rsvd_opts*>(opts);
  return o->k + o->p;
}

// Estimated device time of a problem, for largest-first ordering: R products
// cost 2 n^4 per column (four generated products for reflexive boundary
// conditions); the single-vector products of EGKB run about three times slower
// per flop than the block products of RSVD.
double est_cost(const kp_blur& b, int32_t method, const void* opts) {
  const double n4 = std::pow((double)b.n, 4.0) * (b.bc == KP_BC_REFLEXIVE ? 4.0 : 1.0);
  const int kp = rank_of(method, opts);
  if (method == KP_METHOD_GKB) {
    const bool blk = opts && static_cast<const kp_gkb_opts*>(opts)->block >= 1;
    return (blk ? 1.6 : 3.0) * 4.0 * n4 * kp;
  }
  const int q = opts ? static_cast<const kp_rsvd_opts*>(opts)->q : 1;
  return (4.0 * q + 4.0) * n4 * kp;
}

// Problems of a batch whose products can share the persistent launch: RSVD in
// FP32 (every product a generated-tile FP32 block product) without support
// compaction. KPSB_BATCH_PERSISTENT=0 runs every problem on its own launches.
bool lockstep_eligible(const kp_blur& b, int32_t method, const void* opts) {
  const char* e = getenv("KPSB_BATCH_PERSISTENT");
  if (e && atoi(e) == 0) return false;
  if (method != KP_METHOD_RSVD || !opts || b.compact) return false;
  const kp_rsvd_opts* o = static_cast<const kp_rsvd_opts*>(opts);
  return o->prec == KP_F32;
}

kp_status run_one(kp_ctx* w, const kp_blur* b, int32_t method, const void* opts, kp_factors* f) {
  if (method == KP_METHOD_GKB)
    return kp_svd_gkb(w, b, static_cast<const kp_gkb_opts*>(opts), f, w->own_stream);
  if (method == KP_METHOD_RSVD)
    return kp_svd_rsvd(w, b, static_cast<const kp_rsvd_opts*>(opts), f, w->own_stream);
  return fail(w, KP_E_INVAL, "method must be KP_METHOD_GKB or KP_METHOD_RSVD");
}

bool is_error(kp_status s) { return s != KP_OK && s != KP_W_BREAKDOWN; }

// Whether a KP-SVD would pick a launch shape the autotuner has not chosen yet:
// its first call times candidate launches, which must not share the GPU with
// other problems' work or the samples measure the contention.
bool needs_tuning(const kp_blur& b, int32_t method, const void* opts) {
  if (!opts) return false;
  if (method == KP_METHOD_GKB) {
    const kp_gkb_opts* o = static_cast<const kp_gkb_opts*>(opts);
    if (o->block < 1) return false;   // matrix-vector products: not tuned
    return !tune_known(kTuneBlock, b.n, o->prec == KP_F64 ? 8 : 4, 0);
  }
  const kp_rsvd_opts* o = static_cast<const kp_rsvd_opts*>(opts);
  // the 16-bit tuner is keyed on the element type (KP_BF16 / KP_F16); the
  // split-FP16 products (KP_F16X3, and the refinement product of refine = 2 in
  // the FP32-vector modes) tune the FP16 kernel
  const bool split16 = (o->refine == 2 && o->prec != KP_F64) || o->prec == KP_F16X3;
  if (split16 && !tune_known(kTuneBlock16, b.n, KP_F16, 0)) return true;
  if (o->prec == KP_F16X3) return false;   // every product is a split-FP16 one
  if (o->prec == KP_BF16 || o->prec == KP_F16)
    return !tune_known(kTuneBlock16, b.n, o->prec, 0) ||
           (o->refine == 1 && !tune_known(kTuneBlock, b.n, 4, 0));
  return !tune_known(kTuneBlock, b.n, o->prec == KP_F64 ? 8 : 4, 0);
}

bool apply_needs_tuning(int n, int k) {
  return !tune_known(kTuneApply, n, k, 0) || !tune_known(kTuneApply, n, k, 1);
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

// ===========================================================================
// Lockstep product batch: the FP32 block products of the problems in flight
// are gathered and run as one persistent launch. Each problem's thread hands
// over its product (with an event marking its input ready on its stream) and
// waits; the thread whose request completes the set (every problem in flight
// has one pending, or has left) launches, and every stream then waits for the
// launch's completion event.
struct kp_batch {
  kp_ctx* parent = nullptr;
  BlockPlan shape;                 // TJ, waves, TK shared by every product
  hipStream_t stream = nullptr;    // the persistent launches
  std::mutex m;
  std::condition_variable cv;
  int active = 0;                  // threads that may still hand over a product
  uint64_t phase = 0;
  struct Req {
    hipEvent_t ready;
    std::vector<BlockJob> jobs;
    size_t lds;
  };
  std::vector<Req> pending;
  std::vector<BlockJob> host_jobs;
  BlockJob* djobs = nullptr;
  int djobs_cap = 0;
  int* counter = nullptr;
  hipEvent_t done = nullptr;       // completion of the latest launch
  kp_status err = KP_OK;
  std::string msg;
  int64_t launches = 0, products = 0;
};

namespace {

// Launches the pending products (caller holds b->m).
void batch_launch_locked(kp_batch* b) {
  b->host_jobs.clear();
  size_t lds = 0;
  for (auto& r : b->pending) {
    if (b->err == KP_OK && hipStreamWaitEvent(b->stream, r.ready, 0) != hipSuccess) {
      b->err = KP_E_DEVICE;
      b->msg = "hipStreamWaitEvent failed";
    }
    (void)hipEventDestroy(r.ready);
    for (auto& j : r.jobs) b->host_jobs.push_back(j);
    lds = std::max(lds, r.lds);
  }
  // largest tiles first (a tile's work grows as n^2), so that the small ones
  // fill in at the end
  std::stable_sort(b->host_jobs.begin(), b->host_jobs.end(),
                   [](const BlockJob& x, const BlockJob& y) { return x.n > y.n; });
  int total = 0;
  for (auto& j : b->host_jobs) {
    j.first = total;
    total += j.tiles;
  }
  const int nj = (int)b->host_jobs.size();
  if (b->err == KP_OK && nj > b->djobs_cap) {
    if (b->djobs) {
      (void)hipStreamSynchronize(b->stream);
      std::unique_lock<std::shared_mutex> nocap(capture_mutex());
      (void)hipFree(b->djobs);
      b->djobs = nullptr;
    }
    const int cap = std::max(64, 2 * nj);
    if (hipMalloc((void**)&b->djobs, sizeof(BlockJob) * cap) != hipSuccess) {
      (void)hipGetLastError();
      b->err = KP_E_NOMEM;
      b->msg = "allocating the batch's job list failed";
    } else {
      b->djobs_cap = cap;
    }
  }
  if (b->err == KP_OK && nj > 0) {
    // pageable source: the copy has consumed host_jobs when the call returns
    if (hipMemcpyAsync(b->djobs, b->host_jobs.data(), sizeof(BlockJob) * nj,
                       hipMemcpyHostToDevice, b->stream) != hipSuccess) {
      b->err = KP_E_DEVICE;
      b->msg = "copying the batch's job list failed";
    } else {
      const int per_cu = lds <= 78 * 1024 ? 2 : 1;
      const int grid = std::min(total, 256 * per_cu);
      hipEvent_t e0 = nullptr, e1 = nullptr;
      const bool prof = b->parent->prof && hipEventCreate(&e0) == hipSuccess &&
                        hipEventCreate(&e1) == hipSuccess;
      if (prof) (void)hipEventRecord(e0, b->stream);
      launch_rmat_block_persistent(b->shape, b->djobs, nj, total, b->counter, lds, grid,
                                   b->stream);
      if (prof) {
        (void)hipEventRecord(e1, b->stream);
        double fl = 0.0;
        for (auto& j : b->host_jobs) {
          const double N = (double)j.n * j.n;
          fl += 2.0 * N * N * j.ncols;
        }
        b->parent->recs.push_back(kp_ctx::Rec{e0, e1, 0, fl});
      }
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) {
        b->err = KP_E_DEVICE;
        b->msg = std::string("persistent block launch: ") + hipGetErrorString(e);
      }
      b->launches += 1;
      b->products += (int64_t)b->pending.size();
    }
  }
  if (hipEventRecord(b->done, b->stream) != hipSuccess && b->err == KP_OK) {
    b->err = KP_E_DEVICE;
    b->msg = "hipEventRecord failed";
  }
  b->pending.clear();
  b->phase += 1;
  b->cv.notify_all();
}

// A thread of the batch has no more products to hand over.
void batch_leave(kp_batch* b) {
  std::lock_guard<std::mutex> lk(b->m);
  b->active -= 1;
  if (!b->pending.empty() && (int)b->pending.size() == b->active) batch_launch_locked(b);
}

}  // namespace

namespace kpsb {

kp_status batch_block_product(kp_ctx* c, const float* G, int ldg, int n, const float* X,
                              float* Y, int ncols, hipStream_t s) {
  kp_batch* b = c->batch;
  BlockPlan p;   // (room for the persistent kernel's own LDS word)
  if (!plan_block_tj<float>(n, c->lds_limit - 64, b->shape.TJ, &p, b->shape.TK))
    return fail(c, KP_E_INVAL, "the batch's launch shape does not fit this n");
  kp_batch::Req r;
  r.lds = p.lds;
  const long N = (long)n * n;
  for (int c0 = 0; c0 < ncols; c0 += 32) {
    BlockJob j;
    std::memset(&j, 0, sizeof(j));
    j.G = G;
    j.X = X + N * c0;
    j.Y = Y + N * c0;
    j.ldx = j.ldy = N;
    j.ldg = ldg;
    j.n = n;
    j.ncols = std::min(32, ncols - c0);
    j.SW = p.SW;
    j.CP = p.CP;
    j.tiles = p.grid;
    r.jobs.push_back(j);
  }
  if (hipEventCreateWithFlags(&r.ready, hipEventDisableTiming) != hipSuccess)
    return fail(c, KP_E_DEVICE, "hipEventCreate failed");
  if (hipEventRecord(r.ready, s) != hipSuccess) {
    (void)hipEventDestroy(r.ready);
    return fail(c, KP_E_DEVICE, "hipEventRecord failed");
  }
  std::unique_lock<std::mutex> lk(b->m);
  b->pending.push_back(std::move(r));
  const uint64_t my = b->phase;
  if ((int)b->pending.size() == b->active) batch_launch_locked(b);
  else b->cv.wait(lk, [&] { return b->phase != my; });
  if (b->err != KP_OK) return fail(c, b->err, b->msg);
  // b->done still marks this phase's launch: the next one needs this thread's
  // next product
  if (hipStreamWaitEvent(s, b->done, 0) != hipSuccess)
    return fail(c, KP_E_DEVICE, "hipStreamWaitEvent failed");
  return KP_OK;
}

}  // namespace kpsb

// ===========================================================================
// Deblurring server
// ===========================================================================
namespace {

// Allowance for the small buffers of a solve or a KP-SVD (reduction partials,
// flags and scalars, the small SVD's matrices, support boxes): well under it.
constexpr size_t kSlack = 1u << 20;

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// Workspace of split Bregman on n x n images with k terms: 14 images, the
// Kronecker-apply intermediates (2 k images), and small buffers.
size_t sb_bytes(int n, int k) {
  const size_t NN = (size_t)n * n;
  return round256(14 * NN * 8) + 2 * round256((size_t)k * NN * 8) + kSlack;
}

// Workspace of a KP-SVD (upper bound): the R grids in every precision the
// method touches, the Krylov or sketch bases, the FP64 singular-vector blocks
// and the staging of a host start vector or sketch.
size_t svd_bytes(const kp_request& r) {
  const int n = r.blur.n;
  const size_t N = (size_t)n * n;
  const size_t grid = (size_t)grid_ld(n) * (size_t)grid_ld(n);
  size_t b = round256((size_t)r.blur.pu * r.blur.pv * 8);
  // reflexive boundary conditions: four grid pairs, the reversed input and
  // three term outputs of the widest product
  const size_t terms = r.blur.bc == KP_BC_REFLEXIVE ? 4 : 1;
  if (r.method == KP_METHOD_GKB) {
    const size_t es = r.gkb.prec == KP_F64 ? 8 : 4;
    int ucols = r.gkb.k + r.gkb.p + 1, vcols = r.gkb.k + r.gkb.p, wide = 1;
    if (r.gkb.block >= 1) {
      const int bs = r.gkb.block, nb = (r.gkb.k + r.gkb.p + bs - 1) / bs;
      ucols = (nb + 1) * bs;
      vcols = nb * bs;
      wide = bs;
    }
    b += 2 * terms * round256(grid * es);
    b += round256(N * ucols * es) + round256(N * vcols * es);
    b += 2 * round256(N * (size_t)r.k_cap * 8);
    if (terms > 1) b += 4 * round256(N * wide * es);
    if (r.gkb.y0) b += round256(N * (r.gkb.block >= 1 ? r.gkb.block : 1) * 8);
    // staging vector of the FP32 matrix-vector kernel (Algorithm 1, b = 1)
    if (r.gkb.block < 1 && es == 4) b += round256((size_t)gemv_sx_xt_len(n) * 4);
  } else {
    const size_t es = r.rsvd.prec == KP_F64 ? 8 : 4;
    const int kp = r.rsvd.k + r.rsvd.p;
    const size_t x16 = (size_t)x16_column_len(n);
    b += 2 * terms * round256(grid * es);
    if (r.rsvd.prec == KP_BF16 || r.rsvd.prec == KP_F16) {
      b += 2 * terms * round256(grid * 2);
      b += round256(x16 * kp * 2);            // 16-bit copy of the product's input
    }
    b += 2 * round256(N * kp * es);           // sketch / range bases Y, Z
    b += round256(tsqr_workspace_bytes((long)N, kp));   // the QR's reflectors and R factors
    b += 2 * round256(N * (size_t)r.k_cap * 8);
    if (terms > 1) b += 4 * round256(N * kp * es);
    if (r.rsvd.F) b += round256(N * kp * 8);
    if (r.rsvd.prec == KP_F16X3) {
      // split-FP16 products: hi / lo FP16 grids and hi / lo FP16 inputs of k + p
      // columns (also used by the refinement)
      b += 2 * round256((size_t)(2 * n - 1) * grid_ld(n) * 2);
      b += 2 * round256(x16 * (size_t)kp * 2);
    } else if (r.rsvd.refine == 2 && r.rsvd.prec != KP_F64) {
      // split-FP16 refinement: hi / lo FP16 grids and hi / lo FP16 inputs
      b += 2 * round256((size_t)(2 * n - 1) * grid_ld(n) * 2);
      b += 2 * round256(x16 * (size_t)r.rsvd.k * 2);
    }
  }
  return b + kSlack;
}

size_t factor_bytes(int n, int k_cap) { return 2 * round256((size_t)k_cap * n * n * 8); }

struct CacheKey {
  uint64_t psf_key;
  int32_t n, method, k, p, q, prec, refine, reorth, auto_k, k_min, literal_init, k_cap, bc, block;
  uint64_t seed;
  double tau, bd_rel;
  bool operator<(const CacheKey& o) const { return std::memcmp(this, &o, sizeof(CacheKey)) < 0; }
};

CacheKey key_of(const kp_request& r) {
  CacheKey k;
  std::memset(&k, 0, sizeof(k));   // padding participates in the ordering
  k.psf_key = r.psf_key;
  k.n = r.blur.n;
  k.bc = r.blur.bc;
  k.method = r.method;
  k.k_cap = r.k_cap;
  if (r.method == KP_METHOD_GKB) {
    k.k = r.gkb.k;
    k.p = r.gkb.p;
    k.prec = r.gkb.prec;
    k.reorth = r.gkb.reorth;
    k.auto_k = r.gkb.auto_k;
    k.k_min = r.gkb.k_min;
    k.literal_init = r.gkb.literal_init;
    k.seed = r.gkb.seed;
    k.tau = r.gkb.tau;
    k.bd_rel = r.gkb.bd_rel;
    k.block = r.gkb.block;
  } else {
    k.k = r.rsvd.k;
    k.p = r.rsvd.p;
    k.q = r.rsvd.q;
    k.prec = r.rsvd.prec;
    k.refine = r.rsvd.refine;
    k.seed = r.rsvd.seed;
  }
  return k;
}

struct Entry {
  int n = 0, k_cap = 0, k = 0;
  double* Ax = nullptr;
  double* Ay = nullptr;
  std::vector<double> sigma;
  size_t bytes = 0;
  int refs = 0;            // running requests using it
  bool ready = false;      // factors computed
  bool failed = false;
  uint64_t last_use = 0;
};

struct Job {
  uint64_t ticket = 0;
  kp_request req{};
  std::chrono::steady_clock::time_point t_submit;
  int bypassed = 0;
  bool cacheable = false;
  CacheKey key{};
};

}  // namespace

struct kp_server {
  kp_ctx* ctx = nullptr;             // the creating context (device, error text)
  std::shared_ptr<kp_pool> pool;     // the server's own budget
  int slots = 4;
  int max_pending = 4096;
  int cache_cap = 64;
  std::vector<kp_ctx*> workers;
  std::vector<size_t> running_ws;    // footprint of the request a worker runs (0 idle)
  std::vector<uint64_t> running_ticket;   // ticket a worker runs (0 idle)
  std::vector<std::thread> threads;

  std::mutex m;
  std::condition_variable cv_work;   // workers: new work or memory freed
  std::condition_variable cv_done;   // waiters: a result is ready
  std::deque<Job> queue;
  std::map<CacheKey, Entry> cache;
  size_t cache_bytes = 0;
  std::map<uint64_t, kp_result> done;
  std::map<uint64_t, bool> live;     // tickets submitted and not yet collected
  uint64_t next_ticket = 1;
  uint64_t use_clock = 0;
  bool stop = false;
  int running = 0;
  int64_t counters[8] = {0, 0, 0, 0, 0, 0, 0, 0};

  // Tuning gate: jobs run under it shared; a job that would make the autotuner
  // time candidate launches (a new size or rank) runs under it exclusively, so
  // that no other job's GPU work is in flight while the samples are timed.
  // Waiting exclusive jobs hold back new shared ones.
  std::mutex gm;
  std::condition_variable gcv;
  int gshared = 0;
  int gwait = 0;
  bool gexcl = false;
};

namespace {

void gate_enter(kp_server* s, bool excl) {
  std::unique_lock<std::mutex> lk(s->gm);
  if (excl) {
    s->gwait += 1;
    s->gcv.wait(lk, [&] { return !s->gexcl && s->gshared == 0; });
    s->gwait -= 1;
    s->gexcl = true;
  } else {
    s->gcv.wait(lk, [&] { return !s->gexcl && s->gwait == 0; });
    s->gshared += 1;
  }
}

void gate_leave(kp_server* s, bool excl) {
  {
    std::lock_guard<std::mutex> lk(s->gm);
    if (excl) s->gexcl = false;
    else s->gshared -= 1;
  }
  s->gcv.notify_all();
}

// Bytes committed by everything except worker `w`: resident or reserved
// factor sets, the reservations of running workers and (if count_idle) the
// workspace that idle workers still hold. Caller holds s->m.
size_t committed_except_locked(const kp_server* s, int w, bool count_idle) {
  size_t t = s->cache_bytes;
  for (int o = 0; o < (int)s->workers.size(); ++o) {
    if (o == w) continue;
    if (s->running_ws[o]) t += s->running_ws[o];
    else if (count_idle) t += ctx_held(s->workers[o]);
  }
  return t;
}

// Frees the least recently used factor set that no request uses. Caller holds
// s->m. Returns false when there is none.
bool evict_one_locked(kp_server* s) {
  auto victim = s->cache.end();
  for (auto it = s->cache.begin(); it != s->cache.end(); ++it)
    if (it->second.refs == 0 && it->second.ready &&
        (victim == s->cache.end() || it->second.last_use < victim->second.last_use))
      victim = it;
  if (victim == s->cache.end()) return false;
  (void)hipSetDevice(s->ctx->device);
  {
    std::unique_lock<std::shared_mutex> nocap(capture_mutex());
    (void)hipFree(victim->second.Ax);
    (void)hipFree(victim->second.Ay);
  }
  s->cache_bytes -= victim->second.bytes;
  {
    std::lock_guard<std::mutex> lk(s->pool->m);
    s->pool->used -= victim->second.bytes;
  }
  s->cache.erase(victim);
  s->counters[4] += 1;
  return true;
}

// Reserves `need` bytes (workspace growth plus new factors) for a request on
// idle worker w: first with every workspace kept, then with the workspace of
// idle workers released, then after evicting unused factor sets. Caller holds
// s->m. On success *reserved is the worker's reservation.
bool reserve_locked(kp_server* s, int w, size_t need_ws, size_t need_new, bool new_entry,
                    size_t* reserved) {
  const size_t B = s->pool->budget;
  if (new_entry)
    while ((int)s->cache.size() >= s->cache_cap)
      if (!evict_one_locked(s)) return false;
  const size_t held = ctx_held(s->workers[w]);
  if (committed_except_locked(s, w, true) + held + need_ws + need_new <= B) {
    *reserved = held + need_ws;
    return true;
  }
  for (;;) {
    if (committed_except_locked(s, w, false) + need_ws + need_new <= B) {
      for (int o = 0; o < (int)s->workers.size(); ++o)
        if (o == w || s->running_ws[o] == 0) ctx_trim(s->workers[o]);
      *reserved = need_ws;
      return true;
    }
    if (!evict_one_locked(s)) return false;
  }
}

// Picks the next admissible job for worker `w` (caller holds s->m): the first
// queued job whose factors are not being computed by another request and
// whose footprint fits; a job passed over 8 times blocks the jobs behind it.
bool take_job_locked(kp_server* s, int w, Job* out, Entry** entry, bool* hit) {
  for (size_t qi = 0; qi < s->queue.size(); ++qi) {
    Job& j = s->queue[qi];
    Entry* e = nullptr;
    bool is_hit = false;
    if (j.cacheable) {
      auto it = s->cache.find(j.key);
      if (it != s->cache.end()) {
        if (!it->second.ready) {        // being computed by another request
          if (j.bypassed >= 8) return false;
          continue;
        }
        e = &it->second;
        is_hit = true;
      }
    }
    const size_t need_ws = sb_bytes(j.req.blur.n, j.req.k_cap) + (is_hit ? 0 : svd_bytes(j.req));
    const size_t fb = is_hit ? 0 : factor_bytes(j.req.blur.n, j.req.k_cap);
    const bool new_entry = !is_hit && j.cacheable;
    size_t reserved = 0;
    if (is_hit) e->refs += 1;          // keep it from being evicted while reserving
    const bool ok = reserve_locked(s, w, need_ws, fb, new_entry, &reserved);
    if (is_hit) e->refs -= 1;
    if (!ok) {
      if (j.bypassed >= 8) return false;
      continue;
    }
    for (size_t pj = 0; pj < qi; ++pj) {
      s->queue[pj].bypassed += 1;
      s->counters[5] += 1;
    }
    *out = j;
    s->queue.erase(s->queue.begin() + qi);
    *hit = is_hit;
    if (is_hit) {
      e->refs += 1;
      e->last_use = ++s->use_clock;
      *entry = e;
      s->running_ws[w] = reserved;
    } else if (new_entry) {
      Entry ne;
      ne.n = out->req.blur.n;
      ne.k_cap = out->req.k_cap;
      ne.bytes = fb;
      ne.refs = 1;
      ne.last_use = ++s->use_clock;
      auto ins = s->cache.emplace(out->key, std::move(ne));
      s->cache_bytes += fb;            // reserved now, allocated by the worker
      *entry = &ins.first->second;
      s->running_ws[w] = reserved;
    } else {
      *entry = nullptr;
      s->running_ws[w] = reserved + fb;   // private factors of this request
    }
    if (s->running_ws[w] == 0) s->running_ws[w] = 1;   // nonzero marks "running"
    return true;
  }
  return false;
}

void finish_locked(kp_server* s, uint64_t ticket, const kp_result& r) {
  s->done[ticket] = r;
  s->counters[1] += 1;
  s->cv_done.notify_all();
}

void set_msg(kp_result* r, const char* msg) {
  std::snprintf(r->msg, sizeof(r->msg), "%s", msg ? msg : "");
}

void worker_loop(kp_server* s, int w) {
  kp_ctx* wc = s->workers[w];
  (void)hipSetDevice(wc->device);
  for (;;) {
    Job job;
    Entry* e = nullptr;
    bool hit = false;
    {
      std::unique_lock<std::mutex> lk(s->m);
      for (;;) {
        if (take_job_locked(s, w, &job, &e, &hit)) break;
        if (s->stop && s->queue.empty()) return;
        s->cv_work.wait(lk);
      }
      s->running += 1;
      s->running_ticket[w] = job.ticket;
      s->counters[6] = std::max<int64_t>(s->counters[6], s->running);
      s->counters[hit ? 2 : 3] += 1;
    }
    kp_result res;
    std::memset(&res, 0, sizeof(res));
    res.queue_ms = ms_since(job.t_submit);
    res.cache_hit = hit ? 1 : 0;
    const kp_request& r = job.req;
    const int n = r.blur.n;
    kp_status st = KP_OK;
    const void* ropts = r.method == KP_METHOD_GKB ? (const void*)&r.gkb : (const void*)&r.rsvd;
    bool excl = (!hit && needs_tuning(r.blur, r.method, ropts)) ||
                (hit && apply_needs_tuning(n, e->k));
    gate_enter(s, excl);
    // factors: resident, or computed into a cache entry / a private buffer
    double* Ax = nullptr;
    double* Ay = nullptr;
    int k = 0;
    std::vector<double> sigma;
    if (hit) {
      Ax = e->Ax;
      Ay = e->Ay;
      k = e->k;
    } else {
      const auto t0 = std::chrono::steady_clock::now();
      const size_t fb = (size_t)r.k_cap * n * n * sizeof(double);
      hipError_t e1 = hipMalloc((void**)&Ax, fb);
      hipError_t e2 = e1 == hipSuccess ? hipMalloc((void**)&Ay, fb) : e1;
      if (e2 != hipSuccess) {
        (void)hipGetLastError();
        st = KP_E_NOMEM;
        set_msg(&res, "allocating Kronecker factors failed");
      } else {
        std::lock_guard<std::mutex> lk(s->pool->m);
        s->pool->used += factor_bytes(n, r.k_cap);
      }
      if (st == KP_OK) {
        sigma.assign(r.k_cap, 0.0);
        kp_factors f;
        std::memset(&f, 0, sizeof(f));
        f.n = n;
        f.k_cap = r.k_cap;
        f.sigma = sigma.data();
        f.Ax = Ax;
        f.Ay = Ay;
        f.factor_prec = KP_F64;
        st = run_one(wc, &r.blur, r.method, ropts, &f);
        if (st == KP_W_BREAKDOWN) st = KP_OK;
        if (is_error(st)) set_msg(&res, wc->err.c_str());
        k = f.k;
      }
      res.factor_ms = ms_since(t0);
      std::lock_guard<std::mutex> lk(s->m);
      if (e) {
        if (st == KP_OK) {
          e->Ax = Ax;
          e->Ay = Ay;
          e->k = k;
          e->sigma = sigma;
          e->ready = true;
        } else {
          e->failed = true;
        }
        s->cv_work.notify_all();   // requests waiting for these factors
      }
    }
    if (st == KP_OK) {
      kp_factors f;
      std::memset(&f, 0, sizeof(f));
      f.n = n;
      f.k_cap = r.k_cap;
      f.k = k;
      f.sigma = hit ? e->sigma.data() : sigma.data();
      f.Ax = Ax;
      f.Ay = Ay;
      f.factor_prec = KP_F64;
      if (!excl && apply_needs_tuning(n, k)) {   // finish this job alone
        (void)hipStreamSynchronize(wc->own_stream);
        gate_leave(s, false);
        excl = true;
        gate_enter(s, true);
      }
      const auto t1 = std::chrono::steady_clock::now();
      st = r.iso ? sb_solve_iso(wc, &f, r.b, &r.sb, r.x, &res.stats, wc->own_stream)
                 : sb_solve_aniso(wc, &f, r.b, &r.sb, r.x, &res.stats, wc->own_stream);
      if (st == KP_OK && hipStreamSynchronize(wc->own_stream) != hipSuccess) {
        st = KP_E_DEVICE;
        set_msg(&res, "stream synchronization failed");
      }
      if (is_error(st) && res.msg[0] == 0) set_msg(&res, wc->err.c_str());
      res.solve_ms = ms_since(t1);
    }
    res.k = k;
    res.status = st;
    res.total_ms = ms_since(job.t_submit);
    std::vector<void*> to_free;
    size_t unpool = 0;
    {
      std::lock_guard<std::mutex> lk(s->m);
      if (e) {
        e->refs -= 1;
        if (e->failed && e->refs == 0) {   // drop the failed entry and its reservation
          for (auto it = s->cache.begin(); it != s->cache.end(); ++it)
            if (&it->second == e) {
              s->cache_bytes -= e->bytes;
              s->cache.erase(it);
              break;
            }
          if (Ax && Ay) unpool = factor_bytes(n, r.k_cap);
          to_free = {Ax, Ay};
        }
      } else {                             // private factors of this request
        if (Ax && Ay) unpool = factor_bytes(n, r.k_cap);
        to_free = {Ax, Ay};
      }
    }
    (void)hipStreamSynchronize(wc->own_stream);
    gate_leave(s, excl);
    if (!to_free.empty()) {
      {
        std::unique_lock<std::shared_mutex> nocap(capture_mutex());
        for (void* p : to_free)
          if (p) (void)hipFree(p);
      }
      std::lock_guard<std::mutex> lp(s->pool->m);
      s->pool->used -= unpool;
    }
    {
      std::lock_guard<std::mutex> lk(s->m);
      s->running_ws[w] = 0;
      s->running_ticket[w] = 0;
      wc->cancel.store(0);   // a cancel that came after the job's last check
      s->running -= 1;
      finish_locked(s, job.ticket, res);
    }
    s->cv_work.notify_all();
  }
}

kp_status check_request(kp_server* s, const kp_request* r, std::string* why) {
  if (!r) return *why = "request is NULL", KP_E_INVAL;
  if (!r->b || !r->x) return *why = "b or x is NULL", KP_E_INVAL;
  if (r->b == r->x) return *why = "b and x must not alias", KP_E_INVAL;
  if (r->blur.n < 2 || r->blur.n > 2048) return *why = "n must be in [2, 2048]", KP_E_INVAL;
  if (!r->blur.psf) return *why = "psf is NULL", KP_E_INVAL;
  if (r->method != KP_METHOD_GKB && r->method != KP_METHOD_RSVD)
    return *why = "method must be KP_METHOD_GKB or KP_METHOD_RSVD", KP_E_INVAL;
  const int k = r->method == KP_METHOD_GKB ? r->gkb.k : r->rsvd.k;
  if (r->k_cap < 1 || r->k_cap < k || r->k_cap > 64)
    return *why = "k_cap must be in [k, 64]", KP_E_INVAL;
  if (r->iso != 0 && r->iso != 1) return *why = "iso must be 0 or 1", KP_E_INVAL;
  if (!(r->sb.lambda > 0) || !(r->sb.beta > 0) || r->sb.L_max < 1 || r->sb.I_max < 1 ||
      r->sb.tau_sb < 0 || r->sb.tau_cgls < 0)
    return *why = "invalid split Bregman options", KP_E_INVAL;
  const size_t need = sb_bytes(r->blur.n, r->k_cap) + svd_bytes(*r) + factor_bytes(r->blur.n, r->k_cap);
  if (need > s->pool->budget)
    return *why = "request footprint " + std::to_string(need) + " exceeds the server budget " +
                  std::to_string(s->pool->budget), KP_E_NOMEM;
  return KP_OK;
}

}  // namespace

// ===========================================================================
extern "C" {

kp_status kp_request_footprint(const kp_request* r, size_t out[3]) {
  if (!r || !out) return KP_E_INVAL;
  if (r->blur.n < 2 || r->blur.n > 2048 || r->k_cap < 1 || r->k_cap > 64) return KP_E_INVAL;
  if (r->method != KP_METHOD_GKB && r->method != KP_METHOD_RSVD) return KP_E_INVAL;
  out[0] = sb_bytes(r->blur.n, r->k_cap);
  out[1] = svd_bytes(*r);
  out[2] = factor_bytes(r->blur.n, r->k_cap);
  return KP_OK;
}

kp_status kp_svd_batched(kp_ctx* c, int32_t nprob, const kp_blur* blurs, const int32_t* method,
                         const void* const* opts, kp_factors* out, kp_status* status,
                         int32_t nworkers, void* stream) {
  if (!c) return KP_E_INVAL;
  if (nprob < 0) return fail(c, KP_E_INVAL, "nprob must be >= 0");
  if (nprob == 0) return KP_OK;
  if (!blurs || !method || !opts || !out) return fail(c, KP_E_INVAL, "blurs, method, opts or out is NULL");
  if (nworkers < 0 || nworkers > 16) return fail(c, KP_E_INVAL, "nworkers must be in [0, 16]");
  for (int i = 0; i < nprob; ++i)
    if (method[i] != KP_METHOD_GKB && method[i] != KP_METHOD_RSVD)
      return fail(c, KP_E_INVAL, "problem " + std::to_string(i) + ": unknown method");
  const int nw = std::min<int>(nworkers ? nworkers : 4, nprob);
  // problems in flight in the lockstep group (each on its own worker)
  int n_lock = 0;
  for (int i = 0; i < nprob; ++i) n_lock += lockstep_eligible(blurs[i], method[i], opts[i]) ? 1 : 0;
  const int g_lock = n_lock >= 2 ? std::min<int>(nworkers ? nworkers : 16, n_lock) : 0;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KP_E_DEVICE, "hipSetDevice failed");
  kp_status st = ensure_workers(c, std::max(nw, g_lock));
  if (st != KP_OK) return st;
  const int nw_all = std::max(nw, g_lock);
  hipStream_t s = (hipStream_t)stream;
  // workers start after the work already queued on the caller's stream
  hipEvent_t start;
  if (hipEventCreateWithFlags(&start, hipEventDisableTiming) != hipSuccess)
    return fail(c, KP_E_DEVICE, "hipEventCreate failed");
  if (hipEventRecord(start, s) != hipSuccess) {
    (void)hipEventDestroy(start);
    return fail(c, KP_E_DEVICE, "hipEventRecord failed");
  }
  std::vector<int> order(nprob);
  for (int i = 0; i < nprob; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return est_cost(blurs[a], method[a], opts[a]) > est_cost(blurs[b], method[b], opts[b]);
  });
  std::vector<kp_status> res(nprob, KP_OK);
  std::vector<std::string> msg(nprob);
  // Problems that would tune a launch shape run first, one at a time on worker
  // 0 before the others start (the tuner then times its candidates on an
  // otherwise idle GPU); the rest are shared out. Results do not depend on it.
  std::vector<char> done(nprob, 0);
  for (int wi = 0; wi < nw_all; ++wi)
    (void)hipStreamWaitEvent(c->workers[wi]->own_stream, start, 0);
  for (int t = 0; t < nprob; ++t) {
    const int i = order[t];
    if (!needs_tuning(blurs[i], method[i], opts[i])) continue;
    kp_ctx* w = c->workers[0];
    (void)hipSetDevice(w->device);
    if (c->cancel.load(std::memory_order_acquire)) {
      res[i] = KP_E_CANCELLED;
      msg[i] = "cancelled before it started";
    } else {
      res[i] = run_one(w, &blurs[i], method[i], opts[i], &out[i]);
      if (is_error(res[i])) msg[i] = w->err;
    }
    done[i] = 1;
  }
  // Lockstep group: the eligible problems not run yet, largest first, g_lock at
  // a time; their products run as persistent launches of the batch.
  std::vector<int> lock_list;
  for (int t = 0; t < nprob; ++t)
    if (!done[order[t]] && g_lock > 0 && lockstep_eligible(blurs[order[t]], method[order[t]], opts[order[t]]))
      lock_list.push_back(order[t]);
  hipEvent_t lock_done = nullptr;
  if (lock_list.size() >= 2) {
    kp_batch b;
    b.parent = c;
    int n_max = 0;
    for (int i : lock_list) n_max = std::max(n_max, blurs[i].n);
    // the tuned shape of the largest n, except that 16-row-block tiles run with
    // 8 waves and K tiles of at most 176 entries: in the persistent loop the
    // 16-wave form (at most 128 registers per lane) would spill
    bool ok = tuned_block_shape(c, n_max, &b.shape);
    if (ok && b.shape.TJ == 12)   // the persistent kernel is built for 16 and 8 row blocks
      ok = plan_block_tj<float>(n_max, c->lds_limit, 16, &b.shape, b.shape.TK);
    if (ok && b.shape.TJ == 16) {
      b.shape.waves = 8;
      if (b.shape.TK == 192) b.shape.TK = 176;
    }
    ok = ok &&
              hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&b.done, hipEventDisableTiming) == hipSuccess &&
              hipMalloc((void**)&b.counter, sizeof(int)) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      for (int i : lock_list) {   // fall back to separate launches
        (void)i;
      }
      lock_list.clear();
    } else {
      (void)hipStreamWaitEvent(b.stream, start, 0);
      const int G = std::min<int>(g_lock, (int)lock_list.size());
      b.active = G;
      std::atomic<int> next_l{0};
      auto body_l = [&](int wi) {
        kp_ctx* w = c->workers[wi];
        (void)hipSetDevice(w->device);
        w->batch = &b;
        for (;;) {
          const int t = next_l.fetch_add(1);
          if (t >= (int)lock_list.size()) break;
          const int i = lock_list[t];
          if (c->cancel.load(std::memory_order_acquire)) {
            res[i] = KP_E_CANCELLED;
            msg[i] = "cancelled before it started";
          } else {
            res[i] = run_one(w, &blurs[i], method[i], opts[i], &out[i]);
            if (is_error(res[i])) msg[i] = w->err;
          }
          done[i] = 1;
        }
        w->batch = nullptr;
        batch_leave(&b);
      };
      std::vector<std::thread> thl;
      for (int wi = 1; wi < G; ++wi) thl.emplace_back(body_l, wi);
      body_l(0);
      for (auto& t : thl) t.join();
      if (hipEventCreateWithFlags(&lock_done, hipEventDisableTiming) == hipSuccess)
        (void)hipEventRecord(lock_done, b.stream);
    }
    if (b.stream) (void)hipStreamSynchronize(b.stream);
    {
      std::unique_lock<std::shared_mutex> nocap(capture_mutex());
      if (b.djobs) (void)hipFree(b.djobs);
      if (b.counter) (void)hipFree(b.counter);
    }
    if (b.done) (void)hipEventDestroy(b.done);
    if (b.stream) (void)hipStreamDestroy(b.stream);
    c->batch_launches = b.launches;
    c->batch_products = b.products;
  }

  std::atomic<int> next{0};
  std::vector<hipEvent_t> fin(nw_all, nullptr);
  auto body = [&](int wi) {
    kp_ctx* w = c->workers[wi];
    (void)hipSetDevice(w->device);
    for (;;) {
      const int t = next.fetch_add(1);
      if (t >= nprob) break;
      const int i = order[t];
      if (done[i]) continue;
      if (c->cancel.load(std::memory_order_acquire)) {
        res[i] = KP_E_CANCELLED;
        msg[i] = "cancelled before it started";
        continue;
      }
      res[i] = run_one(w, &blurs[i], method[i], opts[i], &out[i]);
      if (is_error(res[i])) msg[i] = w->err;
    }
    if (hipEventCreateWithFlags(&fin[wi], hipEventDisableTiming) == hipSuccess)
      (void)hipEventRecord(fin[wi], w->own_stream);
  };
  std::vector<std::thread> th;
  for (int wi = 1; wi < nw; ++wi) th.emplace_back(body, wi);
  body(0);
  for (auto& t : th) t.join();
  for (int wi = nw; wi < nw_all; ++wi)   // workers of the lockstep group only
    if (hipEventCreateWithFlags(&fin[wi], hipEventDisableTiming) == hipSuccess)
      (void)hipEventRecord(fin[wi], c->workers[wi]->own_stream);
  for (int wi = 0; wi < nw_all; ++wi)
    if (fin[wi]) {
      (void)hipStreamWaitEvent(s, fin[wi], 0);
      (void)hipEventDestroy(fin[wi]);
    }
  if (lock_done) {
    (void)hipStreamWaitEvent(s, lock_done, 0);
    (void)hipEventDestroy(lock_done);
  }
  (void)hipEventDestroy(start);
  // a cancel request that stopped problems is consumed by this call
  if (std::find(res.begin(), res.end(), KP_E_CANCELLED) != res.end()) c->cancel.store(0);
  kp_status worst = KP_OK;
  for (int i = 0; i < nprob; ++i) {
    if (status) status[i] = res[i];
    if (is_error(res[i]) && !is_error(worst)) {
      worst = res[i];
      c->err = "problem " + std::to_string(i) + ": " + msg[i];
    } else if (res[i] == KP_W_BREAKDOWN && worst == KP_OK) {
      worst = KP_W_BREAKDOWN;
    }
  }
  return worst;
}

kp_status sb_solve_batched(kp_ctx* c, int32_t nprob, const sb_problem* probs, sb_stats* stats,
                           kp_status* status, int32_t nworkers, void* stream) {
  if (!c) return KP_E_INVAL;
  if (nprob < 0) return fail(c, KP_E_INVAL, "nprob must be >= 0");
  if (nprob == 0) return KP_OK;
  if (!probs) return fail(c, KP_E_INVAL, "probs is NULL");
  if (nworkers < 0 || nworkers > 16) return fail(c, KP_E_INVAL, "nworkers must be in [0, 16]");
  for (int i = 0; i < nprob; ++i)
    if (!probs[i].f || !probs[i].b || !probs[i].x)
      return fail(c, KP_E_INVAL, "problem " + std::to_string(i) + ": f, b or x is NULL");
  const int nw = std::min<int>(nworkers ? nworkers : 4, nprob);
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KP_E_DEVICE, "hipSetDevice failed");
  kp_status st = ensure_workers(c, nw);
  if (st != KP_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t start;
  if (hipEventCreateWithFlags(&start, hipEventDisableTiming) != hipSuccess)
    return fail(c, KP_E_DEVICE, "hipEventCreate failed");
  if (hipEventRecord(start, s) != hipSuccess) {
    (void)hipEventDestroy(start);
    return fail(c, KP_E_DEVICE, "hipEventRecord failed");
  }
  for (int wi = 0; wi < nw; ++wi) (void)hipStreamWaitEvent(c->workers[wi]->own_stream, start, 0);
  // largest first: 4 k n^3 flops per apply, two applies per CGLS iteration
  auto cost = [&](int i) {
    const double n = probs[i].f->n;
    return n * n * n * (double)probs[i].f->k * probs[i].opts.L_max * probs[i].opts.I_max;
  };
  std::vector<int> order(nprob);
  for (int i = 0; i < nprob; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
  std::vector<kp_status> res(nprob, KP_OK);
  std::vector<std::string> msg(nprob);
  std::vector<sb_stats> st_out(nprob);
  std::vector<char> done(nprob, 0);
  auto run = [&](kp_ctx* w, int i) {
    if (c->cancel.load(std::memory_order_acquire)) {
      res[i] = KP_E_CANCELLED;
      msg[i] = "cancelled before it started";
      return;
    }
    std::memset(&st_out[i], 0, sizeof(sb_stats));
    const sb_problem& pr = probs[i];
    res[i] = pr.iso ? sb_solve_iso(w, pr.f, pr.b, &pr.opts, pr.x, &st_out[i], w->own_stream)
                    : sb_solve_aniso(w, pr.f, pr.b, &pr.opts, pr.x, &st_out[i], w->own_stream);
    if (is_error(res[i])) msg[i] = w->err;
  };
  // sizes whose apply GEMMs are not tuned yet: alone on worker 0 first
  for (int t = 0; t < nprob; ++t) {
    const int i = order[t];
    if (!apply_needs_tuning(probs[i].f->n, probs[i].f->k)) continue;
    kp_ctx* w = c->workers[0];
    (void)hipSetDevice(w->device);
    run(w, i);
    (void)hipStreamSynchronize(w->own_stream);
    done[i] = 1;
  }
  std::atomic<int> next{0};
  std::vector<hipEvent_t> fin(nw, nullptr);
  auto body = [&](int wi) {
    kp_ctx* w = c->workers[wi];
    (void)hipSetDevice(w->device);
    for (;;) {
      const int t = next.fetch_add(1);
      if (t >= nprob) break;
      const int i = order[t];
      if (!done[i]) run(w, i);
    }
    if (hipEventCreateWithFlags(&fin[wi], hipEventDisableTiming) == hipSuccess)
      (void)hipEventRecord(fin[wi], w->own_stream);
  };
  std::vector<std::thread> th;
  for (int wi = 1; wi < nw; ++wi) th.emplace_back(body, wi);
  body(0);
  for (auto& t : th) t.join();
  for (int wi = 0; wi < nw; ++wi)
    if (fin[wi]) {
      (void)hipStreamWaitEvent(s, fin[wi], 0);
      (void)hipEventDestroy(fin[wi]);
    }
  (void)hipEventDestroy(start);
  if (std::find(res.begin(), res.end(), KP_E_CANCELLED) != res.end()) c->cancel.store(0);
  kp_status worst = KP_OK;
  for (int i = 0; i < nprob; ++i) {
    if (status) status[i] = res[i];
    if (stats) stats[i] = st_out[i];
    if (is_error(res[i]) && !is_error(worst)) {
      worst = res[i];
      c->err = "problem " + std::to_string(i) + ": " + msg[i];
    } else if (res[i] == KP_W_BREAKDOWN && worst == KP_OK) {
      worst = KP_W_BREAKDOWN;
    }
  }
  return worst;
}

kp_status kp_server_create(kp_ctx* c, const kp_server_cfg* cfg, kp_server** out) {
  if (!c) return KP_E_INVAL;
  if (!cfg || !out) return fail(c, KP_E_INVAL, "cfg or out is NULL");
  *out = nullptr;
  if (cfg->slots < 0 || cfg->slots > 16) return fail(c, KP_E_INVAL, "slots must be in [0, 16]");
  if (cfg->max_pending < 0 || cfg->cache_entries < 0)
    return fail(c, KP_E_INVAL, "max_pending and cache_entries must be >= 0");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KP_E_DEVICE, "hipSetDevice failed");
  size_t left;
  {
    std::lock_guard<std::mutex> lk(c->pool->m);
    left = c->pool->budget > c->pool->used ? c->pool->budget - c->pool->used : 0;
  }
  const size_t budget = cfg->hbm_budget_bytes ? std::min(cfg->hbm_budget_bytes, left) : left;
  auto* s = new kp_server();
  s->ctx = c;
  s->pool = std::make_shared<kp_pool>();
  s->pool->budget = budget;
  s->slots = cfg->slots ? cfg->slots : 4;
  s->max_pending = cfg->max_pending ? cfg->max_pending : 4096;
  s->cache_cap = cfg->cache_entries ? cfg->cache_entries : 64;
  for (int w = 0; w < s->slots; ++w) {
    kp_ctx* wc = ctx_new(c->device, s->pool, 0);
    if (!wc || hipStreamCreateWithFlags(&wc->own_stream, hipStreamNonBlocking) != hipSuccess) {
      if (wc) ctx_free(wc);
      for (kp_ctx* x : s->workers) ctx_free(x);
      delete s;
      return fail(c, KP_E_DEVICE, "creating a server worker failed");
    }
    s->workers.push_back(wc);
  }
  s->running_ws.assign(s->slots, 0);
  s->running_ticket.assign(s->slots, 0);
  for (int w = 0; w < s->slots; ++w) s->threads.emplace_back(worker_loop, s, w);
  *out = s;
  return KP_OK;
}

kp_status kp_server_submit(kp_server* s, const kp_request* r, uint64_t* ticket) {
  if (!s || !ticket) return KP_E_INVAL;
  std::string why;
  kp_status st = check_request(s, r, &why);
  if (st != KP_OK) return fail(s->ctx, st, why);
  std::lock_guard<std::mutex> lk(s->m);
  if (s->stop) return fail(s->ctx, KP_E_INVAL, "server is shutting down");
  if ((int)s->queue.size() >= s->max_pending) return fail(s->ctx, KP_E_BUSY, "server queue is full");
  Job j;
  j.ticket = s->next_ticket++;
  j.req = *r;
  j.t_submit = std::chrono::steady_clock::now();
  j.cacheable = r->psf_key != 0;
  if (j.cacheable) j.key = key_of(*r);
  s->queue.push_back(j);
  s->live[j.ticket] = true;
  s->counters[0] += 1;
  *ticket = j.ticket;
  s->cv_work.notify_all();
  return KP_OK;
}

kp_status kp_server_wait(kp_server* s, uint64_t ticket, double timeout_s, kp_result* res) {
  if (!s || !res) return KP_E_INVAL;
  std::unique_lock<std::mutex> lk(s->m);
  if (!s->live.count(ticket)) return fail(s->ctx, KP_E_INVAL, "unknown ticket");
  auto ready = [&]() { return s->done.count(ticket) != 0; };
  if (timeout_s < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
    return KP_E_TIMEOUT;
  }
  *res = s->done[ticket];
  s->done.erase(ticket);
  s->live.erase(ticket);
  return KP_OK;
}

kp_status kp_server_cancel(kp_server* s, uint64_t ticket) {
  if (!s) return KP_E_INVAL;
  std::lock_guard<std::mutex> lk(s->m);
  if (!s->live.count(ticket)) return fail(s->ctx, KP_E_INVAL, "unknown ticket");
  if (s->done.count(ticket)) return KP_OK;   // finished already
  for (auto it = s->queue.begin(); it != s->queue.end(); ++it) {
    if (it->ticket != ticket) continue;
    kp_result r;
    std::memset(&r, 0, sizeof(r));
    r.status = KP_E_CANCELLED;
    set_msg(&r, "cancelled before it started");
    r.queue_ms = r.total_ms = ms_since(it->t_submit);
    s->queue.erase(it);
    finish_locked(s, ticket, r);
    s->cv_work.notify_all();   // the jobs it held back
    return KP_OK;
  }
  for (size_t w = 0; w < s->workers.size(); ++w)
    if (s->running_ticket[w] == ticket) s->workers[w]->cancel.store(1, std::memory_order_release);
  return KP_OK;
}

kp_status kp_server_stats(kp_server* s, int64_t out[8]) {
  if (!s || !out) return KP_E_INVAL;
  std::lock_guard<std::mutex> lk(s->m);
  for (int i = 0; i < 8; ++i) out[i] = s->counters[i];
  out[7] = (int64_t)s->cache.size();
  return KP_OK;
}

kp_status kp_server_destroy(kp_server* s) {
  if (!s) return KP_E_INVAL;
  {
    std::lock_guard<std::mutex> lk(s->m);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->threads) t.join();
  (void)hipSetDevice(s->ctx->device);
  {
    std::unique_lock<std::shared_mutex> nocap(capture_mutex());
    (void)hipDeviceSynchronize();
    for (auto& kv : s->cache) {
      if (kv.second.Ax) (void)hipFree(kv.second.Ax);
      if (kv.second.Ay) (void)hipFree(kv.second.Ay);
    }
  }
  for (kp_ctx* w : s->workers) ctx_free(w);
  delete s;
  return KP_OK;
}

}  // extern "C"
