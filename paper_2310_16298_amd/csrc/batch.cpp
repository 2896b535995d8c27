// Batched launch: many grids of uneven sizes advanced together, one
// persistent launch per kernel group and step (declared in stencil.h).
#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "runtime.hpp"

using namespace stencil;

namespace {

struct Group {
  Kernel k;                     // shared kernel (items = 0 here; per grid in the table)
  std::vector<BatchGrid> grids;
  int64_t total = 0;            // work items over the group's grids
  unsigned blocks = 0;          // persistent workgroups of one launch
  const BatchGrid* d_table = nullptr;
};

}  // namespace

struct stencil_batch_s {
  int device = -1;
  int32_t count = 0;
  std::vector<Group> groups;
  void* d_tables = nullptr;
  std::vector<hipStream_t> side;  // one stream per group beyond the first
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  GraphCache graphs;

  ~stencil_batch_s() {
    for (hipStream_t s : side) (void)hipStreamDestroy(s);
    for (hipEvent_t e : join) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
    if (d_tables) (void)hipFree(d_tables);
  }
};

namespace {

stencil_status_t launch_group(const Group& g, int parity, hipStream_t s) {
  BatchArgs b;
  b.table = g.d_table;
  b.ngrids = (int32_t)g.grids.size();
  b.total = (int32_t)g.total;
  b.launch = parity & 1;
  b.pad = 0;
  return g.k.launch_batch(b, g.blocks, s) == hipSuccess ? STENCIL_OK : STENCIL_EHIP;
}

// Steps t = 0 .. steps-1 of every group; groups run on parallel streams
// forked from and joined back into `s`.
stencil_status_t enqueue_batch(stencil_batch_s* b, int64_t steps, hipStream_t s) {
  const size_t ng = b->groups.size();
  if (ng > 1) {
    if (hipEventRecord(b->fork, s) != hipSuccess) return STENCIL_EHIP;
    for (size_t g = 1; g < ng; ++g)
      if (hipStreamWaitEvent(b->side[g - 1], b->fork, 0) != hipSuccess) return STENCIL_EHIP;
  }
  for (int64_t t = 0; t < steps; ++t)
    for (size_t g = 0; g < ng; ++g) {
      const stencil_status_t st = launch_group(b->groups[g], (int)(t & 1), g == 0 ? s : b->side[g - 1]);
      if (st != STENCIL_OK) return st;
    }
  for (size_t g = 1; g < ng; ++g) {
    if (hipEventRecord(b->join[g - 1], b->side[g - 1]) != hipSuccess) return STENCIL_EHIP;
    if (hipStreamWaitEvent(s, b->join[g - 1], 0) != hipSuccess) return STENCIL_EHIP;
  }
  return STENCIL_OK;
}

struct Span {
  uintptr_t lo, hi;
};

}  // namespace

extern "C" {

stencil_status_t stencil_batch_create(const stencil_plan_t* plans, void* const* buf0, void* const* buf1,
                                      int32_t count, stencil_batch_t* out) {
  if (!out) return STENCIL_EINVAL;
  *out = nullptr;
  if (!plans || !buf0 || !buf1 || count < 1) return STENCIL_EINVAL;
  stencil_batch_s* b = nullptr;
  try {
    int device = -1;
    if (hipGetDevice(&device) != hipSuccess) return STENCIL_EHIP;
    std::vector<Span> spans;
    spans.reserve(2 * (size_t)count);
    for (int32_t i = 0; i < count; ++i) {
      const stencil_plan_s* p = plans[i];
      if (!p || !buf0[i] || !buf1[i]) return STENCIL_EINVAL;
      if (p->device != device) return STENCIL_EINVAL;
      // an explicit time block is rejected; one the library chose runs one
      // step per launch here (the plan's picker gives the one-step kernel)
      if (p->rs.time_block > 1 && !p->rs.tb_auto) return STENCIL_EUNSUPPORTED;
      spans.push_back({(uintptr_t)buf0[i], (uintptr_t)buf0[i] + p->grid_bytes});
      spans.push_back({(uintptr_t)buf1[i], (uintptr_t)buf1[i] + p->grid_bytes});
    }
    std::sort(spans.begin(), spans.end(), [](const Span& x, const Span& y) { return x.lo < y.lo; });
    for (size_t k = 1; k < spans.size(); ++k)
      if (spans[k].lo < spans[k - 1].hi) return STENCIL_EALIAS;

    b = new (std::nothrow) stencil_batch_s();
    if (!b) return STENCIL_ENOMEM;
    b->device = device;
    b->count = count;
    std::map<const void*, size_t> by_kernel;
    for (int32_t i = 0; i < count; ++i) {
      KArgs a;
      const Kernel k = plan_kernel(plans[i]->rs, buf0[i], buf1[i], &a);
      if (!k.launch || k.items < 1) {
        delete b;
        return STENCIL_EINTERNAL;
      }
      auto it = by_kernel.find(k.batch_id);
      if (it == by_kernel.end()) {
        it = by_kernel.emplace(k.batch_id, b->groups.size()).first;
        b->groups.emplace_back();
        b->groups.back().k = k;
      }
      Group& g = b->groups[it->second];
      BatchGrid e;
      std::memset(&e, 0, sizeof(e));
      e.args = a;
      e.first = (int32_t)g.total;
      e.phase = 0;
      e.limit = 2;  // launches 0 and 1 (the step parity) always advance every grid
      g.grids.push_back(e);
      g.total += k.items;
      if (g.total > (int64_t(1) << 31) - 1) {
        delete b;
        return STENCIL_EUNSUPPORTED;
      }
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
      delete b;
      return STENCIL_EHIP;
    }
    size_t table_entries = 0;
    for (Group& g : b->groups) {
      int occ = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, g.k.batch_id, g.k.threads, 0) != hipSuccess || occ < 1)
        occ = 1;
      const int64_t cap = (int64_t)occ * cus;
      g.blocks = (unsigned)std::min<int64_t>(g.total, cap);
      table_entries += g.grids.size();
    }
    if (hipMalloc(&b->d_tables, table_entries * sizeof(BatchGrid)) != hipSuccess) {
      delete b;
      return STENCIL_ENOMEM;
    }
    std::vector<BatchGrid> host;
    host.reserve(table_entries);
    for (Group& g : b->groups) {
      g.d_table = reinterpret_cast<const BatchGrid*>(b->d_tables) + host.size();
      host.insert(host.end(), g.grids.begin(), g.grids.end());
    }
    if (hipMemcpy(b->d_tables, host.data(), host.size() * sizeof(BatchGrid), hipMemcpyHostToDevice) != hipSuccess) {
      delete b;
      return STENCIL_EHIP;
    }
    if (b->groups.size() > 1) {
      if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess) {
        delete b;
        return STENCIL_EHIP;
      }
      for (size_t g = 1; g < b->groups.size(); ++g) {
        hipStream_t s = nullptr;
        hipEvent_t e = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
          delete b;
          return STENCIL_EHIP;
        }
        b->side.push_back(s);
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
          delete b;
          return STENCIL_EHIP;
        }
        b->join.push_back(e);
      }
    }
    *out = b;
    return STENCIL_OK;
  } catch (const std::bad_alloc&) {
    delete b;
    return STENCIL_ENOMEM;
  } catch (...) {
    delete b;
    return STENCIL_EINTERNAL;
  }
}

stencil_status_t stencil_batch_run_steps(stencil_batch_t batch, int64_t steps, void* stream, int32_t* result_index) {
  if (!batch || steps < 0) return STENCIL_EINVAL;
  try {
    const stencil_status_t d = check_device(batch->device);
    if (d != STENCIL_OK) return d;
    const hipStream_t s = (hipStream_t)stream;
    stencil_status_t st = batch->graphs.run(batch, nullptr, steps, s, [&](hipStream_t cs) {
      return enqueue_batch(batch, steps, cs);
    });
    if (st == STENCIL_EUNSUPPORTED) st = enqueue_batch(batch, steps, s);
    if (st != STENCIL_OK) return st;
    if (result_index) *result_index = (int32_t)(steps & 1);
    return STENCIL_OK;
  } catch (...) {
    return STENCIL_EINTERNAL;
  }
}

stencil_status_t stencil_batch_info(stencil_batch_t batch, int32_t* groups, int64_t* items, int64_t* blocks) {
  if (!batch) return STENCIL_EINVAL;
  int64_t it = 0, bl = 0;
  for (const Group& g : batch->groups) {
    it += g.total;
    bl += g.blocks;
  }
  if (groups) *groups = (int32_t)batch->groups.size();
  if (items) *items = it;
  if (blocks) *blocks = bl;
  return STENCIL_OK;
}

stencil_status_t stencil_batch_destroy(stencil_batch_t batch) {
  try {
    delete batch;
    return STENCIL_OK;
  } catch (...) {
    return STENCIL_EINTERNAL;
  }
}

}  // extern "C"
