// Serving loop with continuous batching (declared in stencil.h).
//
// Requests (a descriptor, an input and an output buffer, a step count) wait
// in a FIFO.  Each tick admits requests from the head of the queue while their
// device footprint fits the server's arena, then advances every resident
// request: each kernel group (the batched kernels of stencil_batch_*) gets k
// persistent launches, k chosen so that cheap groups do several steps in the
// time the costliest group does one (estimated from the plans' bytes and
// flops per point), and a grid takes part in its first min(k, steps left)
// launches.  A request that has done its steps is copied to its output buffer
// and leaves; its arena block is reused by later requests (stream order keeps
// the reuse behind the copy).
// No device allocation or free happens after creation: hipFree synchronises
// the device and would stall the pipeline.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "runtime.hpp"

using namespace stencil;

namespace {

constexpr size_t kAlign = 256;

// First-fit allocator over one device allocation, with coalescing frees.
class Arena {
 public:
  bool init(size_t bytes) {
    bytes = bytes / kAlign * kAlign;
    if (bytes == 0 || hipMalloc(&base_, bytes) != hipSuccess) return false;
    size_ = bytes;
    free_[0] = bytes;
    return true;
  }
  ~Arena() {
    if (base_) (void)hipFree(base_);
  }
  // offset of a block of `bytes`, or SIZE_MAX
  size_t alloc(size_t bytes) {
    bytes = (bytes + kAlign - 1) / kAlign * kAlign;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > bytes) free_[off + bytes] = len - bytes;
      used_[off] = bytes;
      return off;
    }
    return SIZE_MAX;
  }
  void release(size_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return;
    size_t len = u->second;
    used_.erase(u);
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + len == next->first) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += len;
        return;
      }
    }
    free_[off] = len;
  }
  char* ptr(size_t off) const { return static_cast<char*>(base_) + off; }
  size_t size() const { return size_; }
  size_t in_use() const {
    size_t s = 0;
    for (const auto& u : used_) s += u.second;
    return s;
  }

 private:
  void* base_ = nullptr;
  size_t size_ = 0;
  std::map<size_t, size_t> free_, used_;
};

struct Request {
  int64_t id = 0;
  Resolved rs;
  size_t grid_bytes = 0;
  double step_cost = 0.0;  // estimated seconds per step
  const void* input = nullptr;
  void* output = nullptr;
  int64_t steps = 0, done = 0;
  int32_t limit = 0;       // steps in the current tick
  size_t arena_off = SIZE_MAX;
  KArgs args{};            // buffers 0 / 1 in in / out
  Kernel kernel;
};

struct Slot {  // pinned staging for the operand upload of one request
  void* host = nullptr;
  hipEvent_t ready = nullptr;  // last copy from this slot
};

constexpr size_t kSlotBytes = 64 * 1024;
constexpr int kSlots = 64;

}  // namespace

struct stencil_server_s {
  int device = -1;
  hipStream_t stream = nullptr;
  Arena arena;
  int32_t max_active = 0;
  int32_t max_inflight = 4;
  int cus = 0;
  int64_t next_id = 1;
  int64_t tick = 0;
  std::deque<Request*> queue;
  std::vector<Request*> active;
  struct Group {
    Kernel k;
    int32_t first_entry = 0, ngrids = 0;
    int64_t total = 0;
    unsigned blocks = 0;
    int32_t launches = 1;
  };
  std::vector<Group> groups;
  static constexpr int kTables = 8;     // ring of work tables, one per tick in flight
  void* d_tables[kTables] = {};
  BatchGrid* h_tables[kTables] = {};    // pinned
  hipEvent_t table_free[kTables] = {};
  size_t table_cap = 0;                 // entries per table buffer
  int cur_table = 0;
  std::vector<Slot> slots;
  int next_slot = 0;
  std::vector<hipStream_t> side;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  std::deque<std::pair<hipEvent_t, std::vector<int64_t>>> pending;  // tick events and ids retired then
  std::vector<hipEvent_t> event_pool;
  std::deque<hipEvent_t> inflight;      // one event per recent tick (backpressure)

  ~stencil_server_s() {
    if (stream) (void)hipStreamSynchronize(stream);
    for (Request* r : queue) delete r;
    for (Request* r : active) delete r;
    for (auto& p : pending) (void)hipEventDestroy(p.first);
    for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : inflight) (void)hipEventDestroy(e);
    for (Slot& s : slots) {
      if (s.host) (void)hipHostFree(s.host);
      if (s.ready) (void)hipEventDestroy(s.ready);
    }
    for (int k = 0; k < kTables; ++k) {
      if (d_tables[k]) (void)hipFree(d_tables[k]);
      if (h_tables[k]) (void)hipHostFree(h_tables[k]);
      if (table_free[k]) (void)hipEventDestroy(table_free[k]);
    }
    for (hipStream_t s : side) (void)hipStreamDestroy(s);
    for (hipEvent_t e : join) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
    if (stream) (void)hipStreamDestroy(stream);
  }

  hipEvent_t get_event() {
    if (!event_pool.empty()) {
      hipEvent_t e = event_pool.back();
      event_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
  }
};

namespace {

// Device footprint of a request: two grids, operand fragments, dense
// coefficients and a zero line, each 256-byte aligned.
size_t footprint(const Request& r) {
  auto up = [](size_t v) { return (v + kAlign - 1) / kAlign * kAlign; };
  return 2 * up(r.grid_bytes) + up(r.rs.frag.size()) + up(r.rs.coef.size()) + kAlign;
}

stencil_status_t admit(stencil_server_s* s, Request* r) {
  auto up = [](size_t v) { return (v + kAlign - 1) / kAlign * kAlign; };
  char* base = s->arena.ptr(r->arena_off);
  char* b0 = base;
  char* b1 = b0 + up(r->grid_bytes);
  char* frag = b1 + up(r->grid_bytes);
  char* coef = frag + up(r->rs.frag.size());
  char* zeros = coef + up(r->rs.coef.size());
  // operands and the zero line through a pinned staging slot; operands larger
  // than a slot go straight from the request's own (pageable) host copies,
  // which the request keeps until it retires
  const size_t fb = r->rs.frag.size(), cb = r->rs.coef.size();
  const bool staged = fb + cb + kAlign <= kSlotBytes;
  Slot& sl = s->slots[s->next_slot];
  s->next_slot = (s->next_slot + 1) % kSlots;
  if (hipEventSynchronize(sl.ready) != hipSuccess) return STENCIL_EHIP;
  char* h = static_cast<char*>(sl.host);
  if (staged) {
    if (fb) std::memcpy(h, r->rs.frag.data(), fb);
    std::memcpy(h + fb, r->rs.coef.data(), cb);
    std::memset(h + fb + cb, 0, kAlign);
    if ((fb && hipMemcpyAsync(frag, h, fb, hipMemcpyHostToDevice, s->stream) != hipSuccess) ||
        hipMemcpyAsync(coef, h + fb, cb, hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemcpyAsync(zeros, h + fb + cb, kAlign, hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipEventRecord(sl.ready, s->stream) != hipSuccess)
      return STENCIL_EHIP;
  } else {
    std::memset(h, 0, kAlign);
    if ((fb && hipMemcpyAsync(frag, r->rs.frag.data(), fb, hipMemcpyHostToDevice, s->stream) != hipSuccess) ||
        hipMemcpyAsync(coef, r->rs.coef.data(), cb, hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemcpyAsync(zeros, h, kAlign, hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipEventRecord(sl.ready, s->stream) != hipSuccess)
      return STENCIL_EHIP;
  }
  if (hipMemcpyAsync(b0, r->input, r->grid_bytes, hipMemcpyDeviceToDevice, s->stream) != hipSuccess)
    return STENCIL_EHIP;
  KArgs a = r->rs.args;
  a.frag = fb ? frag : nullptr;
  a.coef = coef;
  a.zeros = zeros;
  a.in = b0;
  a.out = b1;
  r->kernel = r->rs.pick(a, r->rs.chunk_req);
  if (!r->kernel.launch_batch || r->kernel.items < 1) return STENCIL_EINTERNAL;
  r->args = a;
  // rough cost model: HBM bytes at 5 TB/s plus executed flops at 50 TFLOP/s
  const double pts = (double)r->grid_bytes / (r->rs.info.dtype == STENCIL_F64 ? 8.0 : 4.0);
  r->step_cost = pts * (r->rs.info.bytes_per_point / 5.0e12 + r->rs.info.executed_flops_per_point / 50.0e12);
  return STENCIL_OK;
}

stencil_status_t rebuild_tables(stencil_server_s* s) {
  s->groups.clear();
  std::map<const void*, size_t> by_kernel;
  std::vector<std::vector<Request*>> members;
  for (Request* r : s->active) {
    auto it = by_kernel.find(r->kernel.batch_id);
    if (it == by_kernel.end()) {
      it = by_kernel.emplace(r->kernel.batch_id, s->groups.size()).first;
      s->groups.emplace_back();
      s->groups.back().k = r->kernel;
      members.emplace_back();
    }
    members[it->second].push_back(r);
  }
  const size_t n = s->active.size();
  if (n > s->table_cap) {
    // grow the table buffers (after all work that read them)
    if (hipStreamSynchronize(s->stream) != hipSuccess) return STENCIL_EHIP;
    size_t cap = std::max<size_t>(n, 2 * s->table_cap);
    for (int k = 0; k < stencil_server_s::kTables; ++k) {
      if (s->d_tables[k]) (void)hipFree(s->d_tables[k]);
      if (s->h_tables[k]) (void)hipHostFree(s->h_tables[k]);
      s->d_tables[k] = nullptr;
      s->h_tables[k] = nullptr;
      if (hipMalloc(&s->d_tables[k], cap * sizeof(BatchGrid)) != hipSuccess ||
          hipHostMalloc((void**)&s->h_tables[k], cap * sizeof(BatchGrid)) != hipSuccess)
        return STENCIL_ENOMEM;
    }
    s->table_cap = cap;
  }
  const int k = (s->cur_table + 1) % stencil_server_s::kTables;
  if (hipEventSynchronize(s->table_free[k]) != hipSuccess) return STENCIL_EHIP;
  // launches per group: the costliest group does one step per tick (at least
  // 100 us of estimated work), cheaper groups up to 64
  std::vector<double> cost(s->groups.size(), 4.0e-6);
  for (size_t g = 0; g < s->groups.size(); ++g)
    for (Request* r : members[g]) cost[g] += r->step_cost;
  double tau = 100.0e-6;
  for (double c : cost) tau = std::max(tau, c);
  BatchGrid* h = s->h_tables[k];
  int32_t e = 0;
  for (size_t g = 0; g < s->groups.size(); ++g) {
    auto& G = s->groups[g];
    G.first_entry = e;
    G.ngrids = (int32_t)members[g].size();
    G.total = 0;
    G.launches = (int32_t)std::min(64.0, std::max(1.0, std::floor(tau / cost[g])));
    int32_t most = 1;
    for (Request* r : members[g]) {
      r->limit = (int32_t)std::min<int64_t>(G.launches, r->steps - r->done);
      most = std::max(most, r->limit);
      std::memset(&h[e], 0, sizeof(BatchGrid));
      h[e].args = r->args;
      h[e].first = (int32_t)G.total;
      h[e].phase = (int32_t)(r->done & 1);
      h[e].limit = r->limit;
      G.total += r->kernel.items;
      ++e;
    }
    G.launches = most;
    if (G.total > (int64_t(1) << 31) - 1) return STENCIL_EUNSUPPORTED;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, G.k.batch_id, G.k.threads, 0) != hipSuccess || occ < 1)
      occ = 1;
    G.blocks = (unsigned)std::min<int64_t>(G.total, (int64_t)occ * s->cus);
  }
  if (e && hipMemcpyAsync(s->d_tables[k], h, (size_t)e * sizeof(BatchGrid), hipMemcpyHostToDevice, s->stream) !=
               hipSuccess)
    return STENCIL_EHIP;
  s->cur_table = k;
  while (s->side.size() + 1 < s->groups.size()) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return STENCIL_EHIP;
    s->side.push_back(st);
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return STENCIL_EHIP;
    s->join.push_back(ev);
  }
  return STENCIL_OK;
}

stencil_status_t launch_tick(stencil_server_s* s) {
  const size_t ng = s->groups.size();
  if (ng == 0) return STENCIL_OK;
  const BatchGrid* table = static_cast<const BatchGrid*>(s->d_tables[s->cur_table]);
  if (ng > 1) {
    if (hipEventRecord(s->fork, s->stream) != hipSuccess) return STENCIL_EHIP;
    for (size_t g = 1; g < ng; ++g)
      if (hipStreamWaitEvent(s->side[g - 1], s->fork, 0) != hipSuccess) return STENCIL_EHIP;
  }
  for (size_t g = 0; g < ng; ++g) {
    const auto& G = s->groups[g];
    for (int32_t j = 0; j < G.launches; ++j) {
      BatchArgs b;
      b.table = table + G.first_entry;
      b.ngrids = G.ngrids;
      b.total = (int32_t)G.total;
      b.launch = j;
      b.pad = 0;
      if (G.k.launch_batch(b, G.blocks, g == 0 ? s->stream : s->side[g - 1]) != hipSuccess) return STENCIL_EHIP;
    }
  }
  for (size_t g = 1; g < ng; ++g) {
    if (hipEventRecord(s->join[g - 1], s->side[g - 1]) != hipSuccess) return STENCIL_EHIP;
    if (hipStreamWaitEvent(s->stream, s->join[g - 1], 0) != hipSuccess) return STENCIL_EHIP;
  }
  return hipEventRecord(s->table_free[s->cur_table], s->stream) == hipSuccess ? STENCIL_OK : STENCIL_EHIP;
}

}  // namespace

extern "C" {

stencil_status_t stencil_server_create(const stencil_server_config_t* cfg, stencil_server_t* out) {
  if (!out) return STENCIL_EINVAL;
  *out = nullptr;
  if (!cfg || cfg->arena_bytes < (int64_t)kAlign || cfg->max_active < 0 || cfg->max_inflight_ticks < 0)
    return STENCIL_EINVAL;
  stencil_server_s* s = nullptr;
  try {
    s = new (std::nothrow) stencil_server_s();
    if (!s) return STENCIL_ENOMEM;
    if (hipGetDevice(&s->device) != hipSuccess ||
        hipDeviceGetAttribute(&s->cus, hipDeviceAttributeMultiprocessorCount, s->device) != hipSuccess ||
        hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s->fork, hipEventDisableTiming) != hipSuccess) {
      delete s;
      return STENCIL_EHIP;
    }
    if (!s->arena.init((size_t)cfg->arena_bytes)) {
      delete s;
      return STENCIL_ENOMEM;
    }
    s->max_active = cfg->max_active;
    s->max_inflight = cfg->max_inflight_ticks > 0 ? cfg->max_inflight_ticks : 4;
    s->slots.resize(kSlots);
    for (Slot& sl : s->slots) {
      if (hipHostMalloc(&sl.host, kSlotBytes) != hipSuccess) {
        delete s;
        return STENCIL_ENOMEM;
      }
      if (hipEventCreateWithFlags(&sl.ready, hipEventDisableTiming) != hipSuccess) {
        delete s;
        return STENCIL_EHIP;
      }
    }
    for (int k = 0; k < stencil_server_s::kTables; ++k)
      if (hipEventCreateWithFlags(&s->table_free[k], hipEventDisableTiming) != hipSuccess) {
        delete s;
        return STENCIL_EHIP;
      }
    *out = s;
    return STENCIL_OK;
  } catch (...) {
    delete s;
    return STENCIL_EINTERNAL;
  }
}

stencil_status_t stencil_server_stream(stencil_server_t server, void** stream) {
  if (!server || !stream) return STENCIL_EINVAL;
  *stream = server->stream;
  return STENCIL_OK;
}

stencil_status_t stencil_server_submit(stencil_server_t s, const stencil_desc_t* desc, const void* input,
                                       void* output, int64_t steps, int64_t* id) {
  if (!s || !desc || !input || !output || steps < 0) return STENCIL_EINVAL;
  Request* r = nullptr;
  try {
    const stencil_status_t d = check_device(s->device);
    if (d != STENCIL_OK) return d;
    if (desc->time_block > 1) return STENCIL_EUNSUPPORTED;
    r = new (std::nothrow) Request();
    if (!r) return STENCIL_ENOMEM;
    const int st = resolve_plan(desc, &r->rs, true);
    if (st != STENCIL_OK) {
      delete r;
      return (stencil_status_t)st;
    }
    int64_t npts = 1;
    for (int k = 0; k < desc->ndim; ++k) npts *= desc->dims[k];
    r->grid_bytes = (size_t)npts * (desc->dtype == STENCIL_F64 ? 8 : 4);
    if (overlaps(input, output, r->grid_bytes)) {
      delete r;
      return STENCIL_EALIAS;
    }
    if (footprint(*r) > s->arena.size()) {
      delete r;
      return STENCIL_ENOMEM;  // can never be admitted
    }
    r->input = input;
    r->output = output;
    r->steps = steps;
    r->id = s->next_id++;
    s->queue.push_back(r);
    if (id) *id = r->id;
    return STENCIL_OK;
  } catch (...) {
    delete r;
    return STENCIL_EINTERNAL;
  }
}

stencil_status_t stencil_server_tick(stencil_server_t s, stencil_server_stats_t* stats) {
  if (!s) return STENCIL_EINVAL;
  try {
    const stencil_status_t d = check_device(s->device);
    if (d != STENCIL_OK) return d;
    std::vector<int64_t> retired;
    // 1) admission, FIFO
    while (!s->queue.empty() && (s->max_active == 0 || (int32_t)s->active.size() < s->max_active)) {
      Request* r = s->queue.front();
      const size_t off = s->arena.alloc(footprint(*r));
      if (off == SIZE_MAX) break;
      s->queue.pop_front();
      r->arena_off = off;
      const stencil_status_t st = admit(s, r);
      if (st != STENCIL_OK) {
        s->arena.release(off);
        delete r;
        return st;
      }
      if (r->steps == 0) {  // nothing to compute: the input is the result
        if (hipMemcpyAsync(r->output, r->input, r->grid_bytes, hipMemcpyDeviceToDevice, s->stream) != hipSuccess)
          return STENCIL_EHIP;
        retired.push_back(r->id);
        s->arena.release(off);
        delete r;
        continue;
      }
      s->active.push_back(r);
    }
    // 2) advance every resident request (a fresh work table each tick)
    if (!s->active.empty()) {
      stencil_status_t st = rebuild_tables(s);
      if (st == STENCIL_OK) st = launch_tick(s);
      if (st != STENCIL_OK) return st;
    }
    // 3) retire finished requests
    std::vector<Request*> keep;
    keep.reserve(s->active.size());
    for (Request* r : s->active) {
      r->done += r->limit;
      if (r->done < r->steps) {
        keep.push_back(r);
        continue;
      }
      const void* fin = (r->steps & 1) ? r->args.out : r->args.in;
      if (hipMemcpyAsync(r->output, fin, r->grid_bytes, hipMemcpyDeviceToDevice, s->stream) != hipSuccess)
        return STENCIL_EHIP;
      retired.push_back(r->id);
      s->arena.release(r->arena_off);
      delete r;
    }
    s->active.swap(keep);
    ++s->tick;
    // 4) completion event; bounded ticks in flight
    if (!retired.empty()) {
      hipEvent_t ev = s->get_event();
      if (!ev || hipEventRecord(ev, s->stream) != hipSuccess) return STENCIL_EHIP;
      s->pending.emplace_back(ev, retired);
    }
    hipEvent_t tick_ev = s->get_event();
    if (!tick_ev || hipEventRecord(tick_ev, s->stream) != hipSuccess) return STENCIL_EHIP;
    s->inflight.push_back(tick_ev);
    while ((int32_t)s->inflight.size() > s->max_inflight) {
      hipEvent_t old = s->inflight.front();
      s->inflight.pop_front();
      if (hipEventSynchronize(old) != hipSuccess) return STENCIL_EHIP;
      s->event_pool.push_back(old);
    }
    if (stats) {
      stats->active = (int32_t)s->active.size();
      stats->queued = (int32_t)s->queue.size();
      stats->groups = (int32_t)s->groups.size();
      stats->retired = (int32_t)retired.size();
      stats->tick = s->tick;
      stats->arena_in_use = (int64_t)s->arena.in_use();
    }
    return STENCIL_OK;
  } catch (...) {
    return STENCIL_EINTERNAL;
  }
}

stencil_status_t stencil_server_cancel(stencil_server_t s, int64_t id) {
  if (!s || id < 1) return STENCIL_EINVAL;
  try {
    // still queued: nothing of it reached the device
    for (auto it = s->queue.begin(); it != s->queue.end(); ++it) {
      if ((*it)->id != id) continue;
      delete *it;
      s->queue.erase(it);
      return STENCIL_OK;
    }
    // resident: no further launch or copy is enqueued for it; work already
    // enqueued on the server's stream still reads its arena block, and any
    // later use of the block (a new admission) is enqueued behind that work
    for (auto it = s->active.begin(); it != s->active.end(); ++it) {
      if ((*it)->id != id) continue;
      s->arena.release((*it)->arena_off);
      delete *it;
      s->active.erase(it);
      return STENCIL_OK;
    }
    return STENCIL_EINVAL;  // unknown, finished or already cancelled
  } catch (...) {
    return STENCIL_EINTERNAL;
  }
}

stencil_status_t stencil_server_poll(stencil_server_t s, int64_t* ids, int32_t capacity, int32_t* count) {
  if (!s || !count || capacity < 0 || (capacity > 0 && !ids)) return STENCIL_EINVAL;
  try {
    int32_t n = 0;
    while (!s->pending.empty()) {
      auto& front = s->pending.front();
      const hipError_t q = hipEventQuery(front.first);
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess) return STENCIL_EHIP;
      if (n + (int32_t)front.second.size() > capacity) break;
      for (int64_t v : front.second) ids[n++] = v;
      s->event_pool.push_back(front.first);
      s->pending.pop_front();
    }
    *count = n;
    return STENCIL_OK;
  } catch (...) {
    return STENCIL_EINTERNAL;
  }
}

stencil_status_t stencil_server_destroy(stencil_server_t s) {
  try {
    delete s;
    return STENCIL_OK;
  } catch (...) {
    return STENCIL_EINTERNAL;
  }
}

}  // extern "C"
