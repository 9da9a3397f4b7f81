// Internal definition of kp_ctx, shared by the entry points (api.cpp) and the
// concurrent runtime (runtime.cpp: batched KP-SVD and the request server).
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <shared_mutex>
#include <string>
#include <vector>

#include "common.h"
#include "kpsb.h"

struct kp_batch;   // lockstep product batch of kp_svd_batched (runtime.cpp)

// HBM budget shared by a context and the worker contexts it spawns: every
// workspace allocation of any of them is charged here.
struct kp_pool {
  std::mutex m;
  size_t budget = 0;
  size_t used = 0;
};

struct kp_ctx {
  int device = 0;
  std::shared_ptr<kp_pool> pool;
  size_t lds_limit = 65536;
  std::string err;
  struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
  };
  std::map<std::string, Buf> bufs;
  double* pinned = nullptr;   // host readback buffer (64 doubles)
  // tracing: event pairs around product launches (see kp_prof_read)
  bool prof = false;
  struct Rec {
    hipEvent_t a, b;
    int cls;
    double flops;
  };
  std::vector<Rec> recs;
  double acc_ms[4] = {0, 0, 0, 0};
  int64_t acc_n[4] = {0, 0, 0, 0};
  double acc_flops[4] = {0, 0, 0, 0};
  // worker contexts (each with its own workspace and stream) used by the
  // batched call; created on first use and kept with their workspaces.
  std::vector<kp_ctx*> workers;
  hipStream_t own_stream = nullptr;   // set for worker contexts only
  // Allocation-free mode (kp_rmat_apply_noalloc): while arena_base is set, every
  // workspace request is carved, in order, from arena_base[0, arena_cap) and
  // nothing is allocated or freed.
  char* arena_base = nullptr;
  size_t arena_cap = 0, arena_used = 0;
  void* scratch = nullptr;   // this device's static scratch array (device address)
  // Cancellation (kp_cancel): set from any thread, consumed by the call it
  // stops. A worker of a batched call watches its parent's flag instead (the
  // batched call consumes it).
  std::atomic<int> cancel{0};
  kp_ctx* parent = nullptr;
  // Set on a worker that runs a problem of a lockstep batch: its generated-tile
  // FP32 block products are handed to the batch, which runs the products of all
  // problems in flight as one persistent launch.
  kp_batch* batch = nullptr;
  // persistent launches and products of the last kp_svd_batched call
  int64_t batch_launches = 0, batch_products = 0;
};

namespace kpsb {

// HIP refuses calls that synchronize the whole device (hipDeviceSynchronize,
// hipFree) while any stream of the process is capturing a graph, whatever the
// capture mode. Graph captures hold this lock shared; code that frees device
// memory or synchronizes the device holds it exclusively.
std::shared_mutex& capture_mutex();

// Creates a context bound to `device` that charges `pool` (the parent's, or a
// new one when pool is empty). Returns nullptr on a device error.
kp_ctx* ctx_new(int device, std::shared_ptr<kp_pool> pool, size_t budget);
// Frees a context's workspace, pinned buffer, events, workers and stream.
void ctx_free(kp_ctx* c);
// Frees every workspace buffer of `c` (after synchronizing the device).
void ctx_trim(kp_ctx* c);
// Bytes of workspace currently held by `c` itself.
size_t ctx_held(const kp_ctx* c);
// Y = op(R) X (FP32, ncols columns) through the lockstep batch of c (c->batch
// set): queued with the products of the other problems in flight, which run as
// one persistent launch; on return `s` waits for that launch. G: the grid of
// op(R) (ldg x ldg).
kp_status batch_block_product(kp_ctx* c, const float* G, int ldg, int n, const float* X,
                              float* Y, int ncols, hipStream_t s);
// The FP32 block-product launch shape the autotuner chose for n (its first
// variant if it has not chosen one), without timing anything.
bool tuned_block_shape(kp_ctx* c, int n, BlockPlan* shape);

}  // namespace kpsb
