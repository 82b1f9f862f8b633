// kernels_bicgstab.hip -- block combinations of block BiCGStab (Ch. 6):
// Y = A0 + X1 C1 (+ X2 C2) for n x s blocks and s x s FP64 coefficient
// matrices, e.g. S = R - Q lambda, X = X + P (lambda sigma) + S (omega sigma)
// and P' = R + P beta - Q (omega beta).
//
// One thread per element (i, j): it reads row i of X1 (and X2) and column j
// of the coefficients (LDS), so the s threads of a row share its loads
// through the L1; the block's rows stream through once (grid-stride).
#include "common.hpp"
#include "internal.hpp"

namespace bkry {

template <typename T, bool TWO>
__global__ __launch_bounds__(kBlock) void lincomb_kernel(int64_t n, int s, const T* A0,
                                                          const T* __restrict__ X1, const double* __restrict__ C1,
                                                          const T* __restrict__ X2, const double* __restrict__ C2,
                                                          T* Y, const int32_t* done) {
  __shared__ double c1[kMaxS * kMaxS], c2[TWO ? kMaxS * kMaxS : 1];
  if (done && *done) return;
  for (int t = threadIdx.x; t < s * s; t += kBlock) {
    c1[t] = C1[t];
    if constexpr (TWO) c2[t] = C2[t];
  }
  __syncthreads();
  const int64_t total = n * s;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < total; e += (int64_t)gridDim.x * kBlock) {
    const int64_t i = e / s;
    const int j = (int)(e - i * s);
    const T* x1 = X1 + i * s;
    double acc = (double)A0[e];
    for (int k = 0; k < s; ++k) acc = fma((double)x1[k], c1[k * s + j], acc);
    if constexpr (TWO) {
      const T* x2 = X2 + i * s;
      for (int k = 0; k < s; ++k) acc = fma((double)x2[k], c2[k * s + j], acc);
    }
    Y[e] = (T)acc;
  }
}

template <typename T>
hipError_t launch_lincomb(int64_t n, int s, const T* A0, const T* X1, const double* C1, const T* X2,
                          const double* C2, T* Y, const int32_t* done, hipStream_t st) {
  if (s < 1 || s > kMaxS) return hipErrorInvalidValue;
  const int64_t total = n * s;
  if (total <= 0) return hipSuccess;
  int64_t blocks = (total + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  if (X2)
    hipLaunchKernelGGL((lincomb_kernel<T, true>), dim3((unsigned)blocks), dim3(kBlock), 0, st, n, s, A0, X1, C1, X2,
                       C2, Y, done);
  else
    hipLaunchKernelGGL((lincomb_kernel<T, false>), dim3((unsigned)blocks), dim3(kBlock), 0, st, n, s, A0, X1, C1,
                       X2, C2, Y, done);
  return hipGetLastError();
}

// The three combinations that end an iteration once omega and beta are known
// (X += P (lambda sigma) + S (omega sigma), R = S - omega U, P' = R + P beta -
// Q (omega beta)) run as one pass in the row-slot layout of the streaming
// kernels (bc_tail_rs_kernel, kernels_block.hip).
hipError_t launch_bc_tail(int64_t n, int s, double* X, const double* P, const double* S, const double* U,
                          const double* Q, double* R, double* Pn, const double* lamsig, const BcAux* x,
                          const int32_t* done, hipStream_t st) {
  if (s < 1 || s > kMaxS) return hipErrorInvalidValue;
  if (n <= 0) return hipSuccess;
  return launch_bc_tail_rs(n, s, X, P, S, U, Q, R, Pn, lamsig, x->omsig, x->negomI, x->pbeta, x->qbeta, done, st);
}

template hipError_t launch_lincomb<double>(int64_t, int, const double*, const double*, const double*, const double*,
                                           const double*, double*, const int32_t*, hipStream_t);

}  // namespace bkry
