// kernels_transpose.hip -- transpose of a square CSR matrix (for adjoint
// solves with A^T).  Counting sort: per-column counts (integer atomics),
// one exclusive scan, scatter with per-column cursors, then each row of A^T
// is sorted by its column index, which makes the result independent of the
// order in which the atomics were served.  Integer results are exact.
#include "common.hpp"
#include "internal.hpp"

namespace bkry {

namespace {
constexpr int kTB = 256;
constexpr int kScan = 1024;

size_t a256(size_t x) { return (x + 255) / 256 * 256; }

// flag[0] != 0: malformed input (index out of range, rowptr not monotone)
__global__ __launch_bounds__(kTB) void tr_count_kernel(int64_t n, int64_t nnz, const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ colind, int32_t* cnt,
                                                        int32_t* flag) {
  for (int64_t i = blockIdx.x * (int64_t)kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB) {
    int64_t k0 = rowptr[i], k1 = rowptr[i + 1];
    if (k1 < k0 || (i == 0 && k0 != 0) || (i == n - 1 && k1 != nnz)) flag[0] = 1;
    if (k0 < 0) k0 = 0;
    if (k1 > nnz) k1 = nnz;
    for (int64_t k = k0; k < k1; ++k) {
      const int32_t j = colind[k];
      if ((uint32_t)j < (uint64_t)n)
        atomicAdd(&cnt[j + 1], 1);
      else
        flag[0] = 1;
    }
  }
}

// In-place inclusive scan of a[0..m) by one workgroup (chunk per thread).
__global__ __launch_bounds__(kScan) void tr_scan_kernel(int64_t m, int32_t* a) {
  __shared__ int64_t sums[kScan];
  const int64_t chunk = (m + kScan - 1) / kScan;
  const int64_t b = threadIdx.x * chunk, e = (b + chunk < m) ? b + chunk : m;
  int64_t acc = 0;
  for (int64_t i = b; i < e; ++i) acc += a[i];
  sums[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int t = 0; t < kScan; ++t) {
      const int64_t v = sums[t];
      sums[t] = run;
      run += v;
    }
  }
  __syncthreads();
  int64_t run = sums[threadIdx.x];
  for (int64_t i = b; i < e; ++i) {
    run += a[i];
    a[i] = (int32_t)run;
  }
}

__global__ __launch_bounds__(kTB) void tr_scatter_kernel(int64_t n, int64_t nnz, const int32_t* __restrict__ rowptr,
                                                          const int32_t* __restrict__ colind,
                                                          const double* __restrict__ val, int32_t* cursor,
                                                          int32_t* __restrict__ colindT, double* __restrict__ valT,
                                                          int32_t* __restrict__ permT, int32_t* flag) {
  for (int64_t i = blockIdx.x * (int64_t)kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB) {
    int64_t k0 = rowptr[i], k1 = rowptr[i + 1];
    if (k0 < 0) k0 = 0;
    if (k1 > nnz) k1 = nnz;
    for (int64_t k = k0; k < k1; ++k) {
      const int32_t j = colind[k];
      if ((uint32_t)j >= (uint64_t)n) continue;
      const int32_t t = atomicAdd(&cursor[j], 1);
      if (t < 0 || t >= nnz) {
        flag[0] = 1;
        continue;
      }
      colindT[t] = (int32_t)i;
      valT[t] = val[k];
      permT[t] = (int32_t)k;
    }
  }
}

__global__ __launch_bounds__(kTB) void tr_sort_kernel(int64_t n, int64_t nnz, const int32_t* __restrict__ rowptrT,
                                                       int32_t* __restrict__ colindT, double* __restrict__ valT,
                                                       int32_t* __restrict__ permT) {
  for (int64_t j = blockIdx.x * (int64_t)kTB + threadIdx.x; j < n; j += (int64_t)gridDim.x * kTB) {
    int64_t b = rowptrT[j], e = rowptrT[j + 1];
    if (b < 0) b = 0;
    if (e > nnz) e = nnz;
    for (int64_t x = b + 1; x < e; ++x) {
      const int32_t c = colindT[x];
      const double v = valT[x];
      const int32_t p = permT[x];
      int64_t y = x - 1;
      while (y >= b && colindT[y] > c) {
        colindT[y + 1] = colindT[y];
        valT[y + 1] = valT[y];
        permT[y + 1] = permT[y];
        --y;
      }
      colindT[y + 1] = c;
      valT[y + 1] = v;
      permT[y + 1] = p;
    }
  }
}

unsigned grid_for(int64_t n) {
  int64_t b = (n + kTB - 1) / kTB;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (unsigned)b;
}
}  // namespace

size_t csr_transpose_ws_bytes(int64_t n) { return 256 + a256(sizeof(int32_t) * (size_t)(n + 1)); }

hipError_t csr_transpose_run(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colind,
                             const double* val, int32_t* rowptrT, int32_t* colindT, double* valT, int32_t* permT,
                             void* ws, hipStream_t st) {
  int32_t* flag = static_cast<int32_t*>(ws);
  int32_t* cursor = reinterpret_cast<int32_t*>(static_cast<char*>(ws) + 256);
  hipError_t e = hipMemsetAsync(flag, 0, sizeof(int32_t), st);
  if (e == hipSuccess) e = hipMemsetAsync(rowptrT, 0, sizeof(int32_t) * (size_t)(n + 1), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(tr_count_kernel, dim3(grid_for(n)), dim3(kTB), 0, st, n, nnz, rowptr, colind, rowptrT, flag);
  hipLaunchKernelGGL(tr_scan_kernel, dim3(1), dim3(kScan), 0, st, n + 1, rowptrT);
  e = hipMemcpyAsync(cursor, rowptrT, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  if (nnz > 0) {
    hipLaunchKernelGGL(tr_scatter_kernel, dim3(grid_for(n)), dim3(kTB), 0, st, n, nnz, rowptr, colind, val, cursor,
                       colindT, valT, permT, flag);
    hipLaunchKernelGGL(tr_sort_kernel, dim3(grid_for(n)), dim3(kTB), 0, st, n, nnz, rowptrT, colindT, valT, permT);
  }
  return hipGetLastError();
}

}  // namespace bkry
