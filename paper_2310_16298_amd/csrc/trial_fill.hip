// Seeded fill of the autotuner's trial grids.  Matrix-core and vector-ALU
// bound kernels draw less power on all-zero operands and hold a higher clock
// there (on MI355X the n = 4 box outer products ran 13-15 % faster on a zeroed
// 8192^2 grid than on random data), so trials run on values spread over
// [-1, 1) as a real state would be.
#include "plan.hpp"

namespace stencil {

// 64-bit finaliser of the SplitMix64 generator (Steele, Lea and Flood, 2014)
__device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <typename T>
__global__ __launch_bounds__(256) void trial_fill_kernel(T* __restrict__ p, int64_t n, uint64_t seed) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint64_t h = mix64(seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1));
    // top 53 bits as a fraction in [0, 1), mapped to [-1, 1)
    const double u = (double)(h >> 11) * 0x1.0p-53;
    p[i] = (T)(2.0 * u - 1.0);
  }
}

hipError_t launch_trial_fill(void* p, int dtype, int64_t n, uint64_t seed, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (dtype == STENCIL_F64)
    trial_fill_kernel<double><<<dim3((unsigned)blocks), dim3(256), 0, s>>>((double*)p, n, seed);
  else
    trial_fill_kernel<float><<<dim3((unsigned)blocks), dim3(256), 0, s>>>((float*)p, n, seed);
  return hipGetLastError();
}

}  // namespace stencil
