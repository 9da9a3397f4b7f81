// Autotuner of the kernels' launch shapes. For a given (operation, problem
// shape) the first call times every candidate variant with hipEvents on the
// caller's stream and keeps the fastest for the rest of the process. The
// variants of one operation differ only in how the work is distributed over
// workgroups and waves; every output element is accumulated in the same order,
// so the results do not depend on the choice (checked by the tests).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "common.h"

namespace kpsb {

namespace {

struct Choice {
  int variant = 0;
  std::vector<double> ms;   // measured cost per candidate (< 0: not applicable)
};

std::mutex g_mu;
thread_local bool t_no_timing = false;
std::map<std::tuple<int, int, int, int, int>, Choice> g_table;

const char* op_name(int op) {
  switch (op) {
    case kTuneBlock: return "block32";
    case kTuneBlock16: return "block16";
    case kTuneApply: return "kp_apply";
    default: return "?";
  }
}

}  // namespace

bool tune_enabled() {
  const char* e = getenv("KPSB_AUTOTUNE");
  return !(e && atoi(e) == 0);
}

double time_launches(hipStream_t s, int reps, const std::function<void()>& launch) {
  // a stream under graph capture cannot be timed: no sample is launched
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) {
    (void)hipGetLastError();
    return -1.0;
  }
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    if (a) (void)hipEventDestroy(a);
    (void)hipGetLastError();
    return -1.0;
  }
  auto timed = [&](int r_count) -> double {
    (void)hipEventRecord(a, s);
    for (int r = 0; r < r_count; ++r) launch();
    (void)hipEventRecord(b, s);
    float ms = -1.f;
    if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess)
      ms = -1.f;
    return ms < 0 ? -1.0 : (double)ms / r_count;
  };
  launch();                                 // warm-up (instruction cache, clocks)
  double per = timed(reps);
  // short launches: time again over at least 0.5 ms of them (up to 32), so that
  // the candidates of a small size are not told apart by timer noise
  if (per >= 0 && per < 0.1) {
    const int more = (int)std::min(32.0, std::max((double)reps, std::ceil(0.5 / std::max(per, 1e-3))));
    if (more > reps) per = timed(more);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipGetLastError();
  return per;
}

bool tune_known(int op, int n, int a, int b) {
  if (!tune_enabled()) return true;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_mu);
  return g_table.count(std::make_tuple(op, dev, n, a, b)) != 0;
}

void tune_set_no_timing(bool on) { t_no_timing = on; }

int tune_pick(int op, int n, int a, int b, int ncand, const std::function<double(int)>& cost) {
  if (t_no_timing) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_table.find(std::make_tuple(op, dev, n, a, b));
    return it != g_table.end() ? it->second.variant : 0;
  }
  // KPSB_TUNE_FORCE=v pins every operation to its variant v when that variant
  // applies (used to check that all variants agree bit for bit)
  if (const char* f = getenv("KPSB_TUNE_FORCE")) {
    const int v = atoi(f);
    if (v >= 0 && v < ncand && cost(v) >= 0) return v;
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  const auto key = std::make_tuple(op, dev, n, a, b);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_table.find(key);
    if (it != g_table.end()) return it->second.variant;
  }
  Choice ch;
  if (!tune_enabled()) {
    ch.ms.assign(ncand, -1.0);
  } else {
    double best = -1.0;
    for (int v = 0; v < ncand; ++v) {
      const double m = cost(v);
      ch.ms.push_back(m);
      if (m >= 0 && (best < 0 || m < best)) {
        best = m;
        ch.variant = v;
      }
    }
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (tune_enabled() && !ch.ms.empty() && ch.variant == 0 && !(ch.ms[0] >= 0)) {
    // no sample could be timed (for instance under graph capture): variant 0,
    // not remembered, so that a later call on an ordinary stream tunes the key
    auto it = g_table.find(key);
    return it != g_table.end() ? it->second.variant : 0;
  }
  auto ins = g_table.emplace(key, ch);   // a concurrent tuner of the same key may have won
  return ins.first->second.variant;
}

std::string tune_table() {
  std::lock_guard<std::mutex> lk(g_mu);
  std::string out = "[";
  bool first = true;
  for (const auto& kv : g_table) {
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s{\"op\":\"%s\",\"n\":%d,\"a\":%d,\"b\":%d,\"variant\":%d,\"ms\":[",
                  first ? "" : ",", op_name(std::get<0>(kv.first)), std::get<2>(kv.first),
                  std::get<3>(kv.first), std::get<4>(kv.first), kv.second.variant);
    out += buf;
    for (size_t i = 0; i < kv.second.ms.size(); ++i) {
      std::snprintf(buf, sizeof(buf), "%s%.5g", i ? "," : "", kv.second.ms[i]);
      out += buf;
    }
    out += "]}";
    first = false;
  }
  return out + "]";
}

}  // namespace kpsb
