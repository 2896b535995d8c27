// Kernel selection and launch for one grid or a batch of grids.
//
// A picker chooses the kernel instantiation for a grid's extents and buffer
// pointers (direct-to-LDS windows need 16-byte lines), fills the grid's work
// decomposition into its KArgs and returns the kernel with its number of work
// items.  Each kernel body has two entry points: NAME_kernel(KArgs) covers one
// grid with one workgroup per item, NAME_batch(BatchArgs) loops persistently
// over the items of all grids in a table (compiled apart, so the single-grid
// kernel keeps its own register allocation).
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace stencil {

typedef hipError_t (*SingleLaunch)(const KArgs& a, unsigned blocks, hipStream_t s);
typedef hipError_t (*BatchLaunch)(const BatchArgs& b, unsigned blocks, hipStream_t s);

struct Kernel {
  SingleLaunch launch = nullptr;       // one grid: one workgroup per item
  BatchLaunch launch_batch = nullptr;  // persistent loop over a table of grids
  const void* single_id = nullptr;     // the single-grid __global__ function: occupancy queries
  const void* batch_id = nullptr;      // the batched __global__ function: grouping and occupancy queries
  int64_t items = 0;                   // work items (workgroup tiles) of the grid
  int threads = 256;                   // threads per workgroup (both entry points)
};

// chunk: requested rows (2D) / planes (3D) per work item, 0 = library choice.
typedef Kernel (*Picker)(KArgs& a, int32_t chunk);

// Workgroups of `threads` threads of `kernel` resident on one CU of the
// current device at once, and the device's CU count; 0 if the runtime cannot
// tell.  Cached per device and kernel (occupancy.cpp; a kernel is always
// launched with one workgroup size).
struct Residency {
  int per_cu = 0;
  int cus = 0;
};
Residency resident_workgroups(const void* kernel, int threads = 256);

template <auto K, int NT = 256>
hipError_t launch_single(const KArgs& a, unsigned blocks, hipStream_t s) {
  KArgs ka = a;
  void* args[] = {&ka};
  return hipLaunchKernel(reinterpret_cast<const void*>(K), dim3(blocks), dim3(NT), args, 0, s);
}

template <auto K, int NT = 256>
hipError_t launch_batched(const BatchArgs& b, unsigned blocks, hipStream_t s) {
  BatchArgs kb = b;
  void* args[] = {&kb};
  return hipLaunchKernel(reinterpret_cast<const void*>(K), dim3(blocks), dim3(NT), args, 0, s);
}

// NT: the kernels' workgroup size (their __launch_bounds__)
template <auto KS, auto KB, int NT = 256>
inline Kernel kernel_of(int64_t items) {
  Kernel k;
  k.launch = launch_single<KS, NT>;
  k.launch_batch = launch_batched<KB, NT>;
  k.threads = NT;
  k.single_id = reinterpret_cast<const void*>(KS);
  k.batch_id = reinterpret_cast<const void*>(KB);
  k.items = items;
  return k;
}

}  // namespace stencil
