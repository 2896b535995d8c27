// Host runtime shared by the entry points: the plan object and a cache of
// captured HIP graphs for multi-step runs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <mutex>
#include <vector>

#include "plan.hpp"

namespace stencil {

// Captured launches of one run (key: two pointers and a step count).
struct GraphEntry {
  const void* k0 = nullptr;
  const void* k1 = nullptr;
  int64_t steps = 0;
  hipGraphExec_t exec = nullptr;
  uint64_t last_use = 0;
};

// A small LRU cache of instantiated graphs.  run() records the launches that
// enqueue(stream) makes on a private capture stream the first time a key is
// seen and replays the instantiated graph on `s` afterwards.  It declines
// (STENCIL_EUNSUPPORTED, nothing enqueued) when steps is outside
// [kMinSteps, kMaxSteps], when the caller is capturing `s` (its own graph then
// records the eager launches), or with STENCIL_NO_GRAPH=1 in the environment.
class GraphCache {
 public:
  static constexpr size_t kEntries = 4;
  static constexpr int64_t kMinSteps = 2;
  static constexpr int64_t kMaxSteps = 4096;

  ~GraphCache() {
    for (GraphEntry& g : entries_)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (capture_) (void)hipStreamDestroy(capture_);
  }

  template <class Enqueue>
  stencil_status_t run(const void* k0, const void* k1, int64_t steps, hipStream_t s, Enqueue enqueue) {
    if (steps < kMinSteps || steps > kMaxSteps) return STENCIL_EUNSUPPORTED;
    const char* off = std::getenv("STENCIL_NO_GRAPH");
    if (off && off[0] == '1') return STENCIL_EUNSUPPORTED;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) return STENCIL_EHIP;
    if (cs != hipStreamCaptureStatusNone) return STENCIL_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(mu_);
    GraphEntry* hit = nullptr;
    for (GraphEntry& g : entries_)
      if (g.k0 == k0 && g.k1 == k1 && g.steps == steps) hit = &g;
    if (!hit) {
      if (!capture_ && hipStreamCreateWithFlags(&capture_, hipStreamNonBlocking) != hipSuccess) return STENCIL_EHIP;
      if (hipStreamBeginCapture(capture_, hipStreamCaptureModeRelaxed) != hipSuccess) return STENCIL_EHIP;
      const stencil_status_t st = enqueue(capture_);
      hipGraph_t graph = nullptr;
      const hipError_t e = hipStreamEndCapture(capture_, &graph);
      if (st != STENCIL_OK || e != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        return st != STENCIL_OK ? st : STENCIL_EHIP;
      }
      hipGraphExec_t exec = nullptr;
      const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) return STENCIL_EHIP;
      if (entries_.size() >= kEntries) {
        size_t victim = 0;
        for (size_t k = 1; k < entries_.size(); ++k)
          if (entries_[k].last_use < entries_[victim].last_use) victim = k;
        (void)hipGraphExecDestroy(entries_[victim].exec);
        entries_.erase(entries_.begin() + victim);
      }
      GraphEntry g;
      g.k0 = k0;
      g.k1 = k1;
      g.steps = steps;
      g.exec = exec;
      entries_.push_back(g);
      hit = &entries_.back();
    }
    hit->last_use = ++clock_;
    return hipGraphLaunch(hit->exec, s) == hipSuccess ? STENCIL_OK : STENCIL_EHIP;
  }

 private:
  std::mutex mu_;
  std::vector<GraphEntry> entries_;
  hipStream_t capture_ = nullptr;
  uint64_t clock_ = 0;
};

}  // namespace stencil

struct stencil_plan_s {
  stencil::Resolved rs;
  int device = -1;
  stencil::GraphCache graphs;
  void* d_frag = nullptr;
  void* d_coef = nullptr;
  void* d_zeros = nullptr;
  size_t grid_bytes = 0;
};

namespace stencil {

inline bool overlaps(const void* a, const void* b, size_t n) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + n && y < x + n;
}

inline stencil_status_t check_device(int device) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return STENCIL_EHIP;
  return dev == device ? STENCIL_OK : STENCIL_EINVAL;
}

// The resolved plan's args with the two buffers and the launch's step count
// filled in, its kernel picked (by `pick`, else the plan's own picker) and the
// decomposition applied.
inline Kernel plan_kernel(const Resolved& rs, const void* in, void* out, KArgs* a, int fused = 1,
                          Picker pick = nullptr) {
  *a = rs.args;
  a->in = in;
  a->out = out;
  a->steps = fused;
  return (pick ? pick : rs.pick)(*a, rs.chunk_req);
}

// One launch: one step, or `fused` steps of a time-blocked plan.
inline stencil_status_t launch_one(const Resolved& rs, const void* in, void* out, hipStream_t s, int fused = 1) {
  KArgs a;
  const Kernel k = plan_kernel(rs, in, out, &a, fused);
  // a time-blocked 3D or outer-product launch needs 16-byte aligned buffers
  if (!k.launch && (rs.family == FAM_TB3D || (rs.family == FAM_MFMA2D && rs.time_block > 1))) return STENCIL_EINVAL;
  if (!k.launch || k.items < 1 || k.items > (int64_t(1) << 31) - 1) return STENCIL_EINTERNAL;
  return k.launch(a, (unsigned)k.items, s) == hipSuccess ? STENCIL_OK : STENCIL_EHIP;
}

// Launches of a run of `steps` steps (up to time_block steps each).
inline int64_t launch_count(const Resolved& rs, int64_t steps) {
  const int64_t tb = rs.time_block;
  return (steps + tb - 1) / tb;
}

// The launches of `steps` Jacobi steps, ping-ponging between buf0 and buf1.
inline stencil_status_t launch_steps(const Resolved& rs, void* buf0, void* buf1, int64_t steps, hipStream_t s) {
  void* buf[2] = {buf0, buf1};
  const int64_t tb = rs.time_block;
  int64_t t = 0;
  for (int64_t k = 0; t < steps; ++k) {
    const int fused = (int)(steps - t < tb ? steps - t : tb);
    const stencil_status_t st = launch_one(rs, buf[k & 1], buf[(k + 1) & 1], s, fused);
    if (st != STENCIL_OK) return st;
    t += fused;
  }
  return STENCIL_OK;
}

// Grid bytes of a descriptor (validated: dims >= 1, dtype F32 / F64).
inline size_t grid_bytes_of(const stencil_desc_t* d) {
  int64_t npts = 1;
  for (int k = 0; k < d->ndim; ++k) npts *= d->dims[k];
  return (size_t)npts * (d->dtype == STENCIL_F64 ? 8 : 4);
}

}  // namespace stencil
