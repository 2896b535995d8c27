// Resident workgroups per CU of a kernel and the CU count of a device, cached.
#include <map>
#include <mutex>
#include <utility>

#include "launch.hpp"

namespace stencil {

Residency resident_workgroups(const void* kernel, int threads) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, Residency> cache;
  int dev = -1;
  if (!kernel || hipGetDevice(&dev) != hipSuccess) return Residency{};
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_pair(dev, kernel);
  const auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int occ = 0, cus = 0;
  Residency r;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, threads, 0) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && occ > 0 && cus > 0) {
    r.per_cu = occ;
    r.cus = cus;
  }
  cache[key] = r;
  return r;
}

}  // namespace stencil
