// kernels_ell.hip -- padded row-major (ELL) copy of a CSR matrix for the
// SpMM of the solvers.  Row i's entries go to [i*W, i*W + W) in storage
// order, or with its first diagonal entry moved to the front (the solvers'
// copies: the fused SpMM and Gram then reads a row's own X values from the
// diagonal's gather); the tail of a shorter row is padding (column -1, value
// 0).  A column index outside [0, n) is reported through `bad` and stored as
// padding.
#include "common.hpp"
#include "internal.hpp"

namespace bkry {

// Longest row (entries after clamping the row pointers to [0, nnz]).  A
// wavefront posts its maximum only if it exceeds the value already there: on
// rows of similar length almost no wavefront then issues the atomic, which
// the L2 would otherwise serialise (one per wavefront on one address).
__global__ __launch_bounds__(kBlock) void ell_width_kernel(int64_t n, int64_t nnz, const int32_t* __restrict__ rowptr,
                                                            int32_t* wmax) {
  int m = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    int64_t k0 = rowptr[i], k1 = rowptr[i + 1];
    k0 = k0 < 0 ? 0 : (k0 > nnz ? nnz : k0);
    k1 = k1 < 0 ? 0 : (k1 > nnz ? nnz : k1);
    const int64_t len = k1 - k0;
    if (len > m) m = len > 0x7fffffff ? 0x7fffffff : (int)len;
  }
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) m = max(m, __shfl_xor(m, d));
  if ((threadIdx.x & (kWave - 1)) == 0 && m > 0 && m > __hip_atomic_load(wmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    atomicMax(wmax, m);
}

// Offset of row i's first diagonal entry in [k0, k1) (-1: none).  The
// column indices are read eight at a time, from clamped indexes, so that a
// row waits for one round trip per eight entries.
__device__ __forceinline__ int ell_diag_pos(int64_t i, int64_t k0, int64_t k1, const int32_t* __restrict__ colind) {
  constexpr int kB = 8;
  for (int64_t kb = k0; kb < k1; kb += kB) {
    int32_t cc[kB];
#pragma unroll
    for (int e = 0; e < kB; ++e) cc[e] = colind[kb + e < k1 ? kb + e : k1 - 1];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int e = 0; e < kB; ++e)
      if (kb + e < k1 && cc[e] == i) return (int)(kb + e - k0);
  }
  return -1;
}

// One thread per padded entry (row-major), so the writes are coalesced.
// nodiag not null: slot 0 takes the row's first diagonal entry (at offset d),
// slots 1 .. d the entries before it, the others stay where they are.
template <typename Tin, typename T>
__global__ __launch_bounds__(kBlock) void ell_fill_kernel(int64_t n, int64_t nnz, const int32_t* __restrict__ rowptr,
                                                           const int32_t* __restrict__ colind,
                                                           const Tin* __restrict__ val, int W,
                                                           int32_t* __restrict__ ecol, T* __restrict__ eval,
                                                           int32_t* bad, int32_t* nodiag) {
  const int64_t total = n * (int64_t)W;
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < total; t += (int64_t)gridDim.x * kBlock) {
    const int64_t i = t / W;
    const int u = (int)(t - i * W);
    int64_t k0 = rowptr[i], k1 = rowptr[i + 1];
    k0 = k0 < 0 ? 0 : (k0 > nnz ? nnz : k0);
    k1 = k1 < 0 ? 0 : (k1 > nnz ? nnz : k1);
    int src = u;  // offset in the CSR row of the entry stored at slot u
    if (nodiag) {
      const int d = ell_diag_pos(i, k0, k1, colind);
      if (d < 0 && u == 0) *nodiag = 1;
      if (d > 0) src = u == 0 ? d : (u <= d ? u - 1 : u);
    }
    int32_t j = -1;
    T a = T(0);
    if (k0 + src < k1) {
      const int32_t cj = colind[k0 + src];
      if ((uint32_t)cj < (uint64_t)n) {
        j = cj;
        a = (T)val[k0 + src];
      } else if (bad) {
        *bad = 1;
      }
    }
    ecol[t] = j;
    eval[t] = a;
  }
}

// minv[i] = 1 / A_ii (Jacobi preconditioner).  A row without a diagonal
// entry, or with a diagonal that is not positive and finite, sets *bad = 1
// (its minv is set to 0).  Duplicate diagonal entries are summed.
__global__ __launch_bounds__(kBlock) void jacobi_minv_kernel(int64_t n, int64_t nnz, const int32_t* __restrict__ rowptr,
                                                              const int32_t* __restrict__ colind,
                                                              const double* __restrict__ val, double* minv,
                                                              int32_t* bad) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    int64_t k0 = rowptr[i], k1 = rowptr[i + 1];
    k0 = k0 < 0 ? 0 : (k0 > nnz ? nnz : k0);
    k1 = k1 < 0 ? 0 : (k1 > nnz ? nnz : k1);
    double d = 0.0;
    bool seen = false;
    for (int64_t k = k0; k < k1; ++k)
      if (colind[k] == i) {
        d += val[k];
        seen = true;
      }
    const bool ok = seen && d > 0.0 && isfinite(d);
    minv[i] = ok ? 1.0 / d : 0.0;
    if (!ok) *bad = 1;
  }
}

hipError_t launch_jacobi_minv(const CsrView& A, double* minv, int32_t* bad, hipStream_t st) {
  if (A.n <= 0) return hipSuccess;
  int64_t blocks = (A.n + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(jacobi_minv_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, st, A.n, A.nnz, A.rowptr, A.colind,
                     static_cast<const double*>(A.val), minv, bad);
  return hipGetLastError();
}

int ell_chunk(int s, int elem_bytes) {
  const int lpr = spmm_lanes_per_row(s, elem_bytes);
  return lpr * ell_entries_per_lane(lpr);
}

hipError_t launch_ell_width(const CsrView& A, int32_t* wmax, hipStream_t st) {
  int64_t blocks = (A.n + kBlock - 1) / kBlock;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  hipError_t e = hipMemsetAsync(wmax, 0, sizeof(int32_t), st);
  if (e != hipSuccess) return e;
  if (A.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(ell_width_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, st, A.n, A.nnz, A.rowptr, wmax);
  return hipGetLastError();
}

template <typename Tin, typename T>
hipError_t launch_ell_fill(const CsrView& A, const Tin* val, int W, int32_t* ecol, T* eval, int32_t* bad,
                           int32_t* nodiag, hipStream_t st) {
  const int64_t total = A.n * (int64_t)W;
  if (total <= 0) return hipSuccess;
  int64_t blocks = (total + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL((ell_fill_kernel<Tin, T>), dim3((unsigned)blocks), dim3(kBlock), 0, st, A.n, A.nnz, A.rowptr,
                     A.colind, val, W, ecol, eval, bad, nodiag);
  return hipGetLastError();
}

template hipError_t launch_ell_fill<double, double>(const CsrView&, const double*, int, int32_t*, double*,
                                                    int32_t*, int32_t*, hipStream_t);
template hipError_t launch_ell_fill<double, float>(const CsrView&, const double*, int, int32_t*, float*, int32_t*,
                                                   int32_t*, hipStream_t);
template hipError_t launch_ell_fill<float, float>(const CsrView&, const float*, int, int32_t*, float*, int32_t*,
                                                  int32_t*, hipStream_t);

}  // namespace bkry
