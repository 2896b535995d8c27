// Batched launch: many grids of uneven sizes advanced together, one
// persistent launch per kernel group and step (declared in stencil.h).
#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <tuple>
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

// The grids whose plans the library time-blocked (time block T) with the
// same T-step kernel.  A run advances them in launches of at most T steps:
// by_size[s] lists the groups (one per kernel) that advance s steps in one
// launch, s = 1 .. T (s = 1: the plans' one-step kernels).
struct TbClass {
  int T = 1;
  std::vector<std::vector<size_t>> by_size;
};

// Launch sizes of a class's run of `steps` steps: the fewest launches of at
// most T steps whose count has the parity of `steps` (every grid of the
// batch then ends in buffer steps % 2), sizes as even as possible.
std::vector<int> tb_schedule(int64_t steps, int T) {
  std::vector<int> sizes;
  if (steps <= 0) return sizes;
  int64_t L = (steps + T - 1) / T;
  if ((L & 1) != (steps & 1)) ++L;  // L <= steps: steps >= 2 whenever the parity needs one more launch
  const int64_t base = steps / L, extra = steps % L;
  for (int64_t l = 0; l < L; ++l) sizes.push_back((int)(base + (l < extra ? 1 : 0)));
  return sizes;
}

}  // namespace

struct stencil_batch_s {
  int device = -1;
  int32_t count = 0;
  std::vector<Group> groups;
  std::vector<size_t> plain;      // groups of one step per launch: `steps` launches each
  std::vector<TbClass> classes;   // time-blocked grids
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

// Steps t = 0 .. steps-1 of every plain group, the scheduled launches of
// every time-blocked class; each plain group and each class on its own
// stream, forked from and joined back into `s`.
stencil_status_t enqueue_batch(stencil_batch_s* b, int64_t steps, hipStream_t s) {
  const size_t slots = b->plain.size() + b->classes.size();
  if (slots > 1) {
    if (hipEventRecord(b->fork, s) != hipSuccess) return STENCIL_EHIP;
    for (size_t k = 1; k < slots; ++k)
      if (hipStreamWaitEvent(b->side[k - 1], b->fork, 0) != hipSuccess) return STENCIL_EHIP;
  }
  size_t slot = 0;
  for (size_t gi : b->plain) {
    const hipStream_t st = slot == 0 ? s : b->side[slot - 1];
    ++slot;
    for (int64_t t = 0; t < steps; ++t) {
      const stencil_status_t e = launch_group(b->groups[gi], (int)(t & 1), st);
      if (e != STENCIL_OK) return e;
    }
  }
  for (const TbClass& c : b->classes) {
    const hipStream_t st = slot == 0 ? s : b->side[slot - 1];
    ++slot;
    const std::vector<int> sizes = tb_schedule(steps, c.T);
    for (size_t l = 0; l < sizes.size(); ++l)
      for (size_t gi : c.by_size[sizes[l]]) {
        const stencil_status_t e = launch_group(b->groups[gi], (int)(l & 1), st);
        if (e != STENCIL_OK) return e;
      }
  }
  for (size_t k = 1; k < slots; ++k) {
    if (hipEventRecord(b->join[k - 1], b->side[k - 1]) != hipSuccess) return STENCIL_EHIP;
    if (hipStreamWaitEvent(s, b->join[k - 1], 0) != hipSuccess) return STENCIL_EHIP;
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
      // an explicit time block is rejected; one the library chose advances
      // its grid up to T steps per launch (a time-blocked class below)
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
    std::map<const void*, size_t> by_kernel;                       // plain group by batched kernel
    std::map<std::pair<const void*, int>, size_t> by_class;         // class by (T-step kernel, T)
    std::map<std::tuple<size_t, int, const void*>, size_t> by_cgroup;  // group by (class, size, kernel)
    auto add_grid = [&](size_t gi, const KArgs& a, const Kernel& k) {
      Group& g = b->groups[gi];
      BatchGrid e;
      std::memset(&e, 0, sizeof(e));
      e.args = a;
      e.first = (int32_t)g.total;
      e.phase = 0;
      e.limit = 2;  // launches 0 and 1 (the launch parity) always advance every grid
      g.grids.push_back(e);
      g.total += k.items;
      return g.total <= (int64_t(1) << 31) - 1;
    };
    auto new_group = [&](const Kernel& k) {
      b->groups.emplace_back();
      b->groups.back().k = k;
      return b->groups.size() - 1;
    };
    for (int32_t i = 0; i < count; ++i) {
      const Resolved& rs = plans[i]->rs;
      const int T = rs.tb_auto ? rs.time_block : 1;
      bool placed = false;
      if (T > 1) {
        // the kernels of launches of 1 .. T steps, picked for a grid among
        // many; a grid whose buffers do not take a time-blocked kernel, or
        // that has none there, runs one step per launch
        std::vector<Kernel> ks(T + 1);
        std::vector<KArgs> as(T + 1);
        bool ok = true;
        for (int sz = 1; sz <= T && ok; ++sz) {
          ks[sz] = plan_kernel(rs, buf0[i], buf1[i], &as[sz], sz, rs.pick_batch);
          ok = ks[sz].launch && ks[sz].items >= 1;
        }
        if (ok) {
          auto cit = by_class.find({ks[T].batch_id, T});
          if (cit == by_class.end()) {
            cit = by_class.emplace(std::make_pair(ks[T].batch_id, T), b->classes.size()).first;
            b->classes.emplace_back();
            b->classes.back().T = T;
            b->classes.back().by_size.resize(T + 1);
          }
          const size_t ci = cit->second;
          for (int sz = 1; sz <= T; ++sz) {
            auto git = by_cgroup.find({ci, sz, ks[sz].batch_id});
            if (git == by_cgroup.end()) {
              git = by_cgroup.emplace(std::make_tuple(ci, sz, ks[sz].batch_id), new_group(ks[sz])).first;
              b->classes[ci].by_size[sz].push_back(git->second);
            }
            if (!add_grid(git->second, as[sz], ks[sz])) {
              delete b;
              return STENCIL_EUNSUPPORTED;
            }
          }
          placed = true;
        }
      }
      if (placed) continue;
      KArgs a;
      const Kernel k = plan_kernel(rs, buf0[i], buf1[i], &a);
      if (!k.launch || k.items < 1) {
        delete b;
        return STENCIL_EINTERNAL;
      }
      auto it = by_kernel.find(k.batch_id);
      if (it == by_kernel.end()) {
        it = by_kernel.emplace(k.batch_id, new_group(k)).first;
        b->plain.push_back(it->second);
      }
      if (!add_grid(it->second, a, k)) {
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
    const size_t slots = b->plain.size() + b->classes.size();
    if (slots > 1) {
      if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess) {
        delete b;
        return STENCIL_EHIP;
      }
      for (size_t g = 1; g < slots; ++g) {
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
