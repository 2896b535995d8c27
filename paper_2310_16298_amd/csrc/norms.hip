// Error norms of a state against an FP64 reference (drift check).
#include "plan.hpp"

namespace stencil {

__global__ void norms_init(double* out) {
  if (threadIdx.x < 3) out[threadIdx.x] = 0.0;
}

template <typename T>
__global__ __launch_bounds__(256) void norms_kernel(const T* __restrict__ a, const double* __restrict__ ref,
                                                    int64_t n, double* out) {
  __shared__ double s_d2[256], s_r2[256], s_mx[256];
  double d2 = 0.0, r2 = 0.0, mx = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double r = ref[i];
    const double d = (double)a[i] - r;
    d2 += d * d;
    r2 += r * r;
    mx = d != d ? INFINITY : fmax(mx, fabs(d));  // a NaN state reads as an infinite error
  }
  s_d2[threadIdx.x] = d2;
  s_r2[threadIdx.x] = r2;
  s_mx[threadIdx.x] = mx;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s_d2[threadIdx.x] += s_d2[threadIdx.x + off];
      s_r2[threadIdx.x] += s_r2[threadIdx.x + off];
      s_mx[threadIdx.x] = fmax(s_mx[threadIdx.x], s_mx[threadIdx.x + off]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&out[0], s_d2[0]);
    atomicAdd(&out[1], s_r2[0]);
    // non-negative doubles order like their bit patterns
    atomicMax(reinterpret_cast<unsigned long long*>(&out[2]), (unsigned long long)__double_as_longlong(s_mx[0]));
  }
}

hipError_t launch_error_norms(const void* a, int a_dtype, const double* ref, int64_t n, double* out,
                              hipStream_t s) {
  norms_init<<<1, 64, 0, s>>>(out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n == 0) return e;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (a_dtype == STENCIL_F64)
    norms_kernel<double><<<dim3((unsigned)blocks), dim3(256), 0, s>>>((const double*)a, ref, n, out);
  else
    norms_kernel<float><<<dim3((unsigned)blocks), dim3(256), 0, s>>>((const float*)a, ref, n, out);
  return hipGetLastError();
}

}  // namespace stencil
