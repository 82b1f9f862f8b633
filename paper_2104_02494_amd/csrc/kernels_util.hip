// kernels_util.hip -- small utility kernels shared by the entry points.
#include "internal.hpp"

namespace bkry {

__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t* p, int64_t count, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, int64_t count, uint32_t v, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  int64_t g = (count + 255) / 256;
  if (g > 1024) g = 1024;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)g), dim3(256), 0, st, p, count, v);
  return hipGetLastError();
}

}  // namespace bkry
