// kernels_block.hip -- HBM-streaming kernels over n x s row-major blocks.
//
//   spmm          BOP, Y = A X (Ch. 3, kernel BOP), optionally fused with the
//                 Gram partials of <X, Y> (the alpha BDOT of block CG) or with
//                 the residual R = B - A X and its Gram partials;
//   gram          BDOT X^T Y, batched over several X blocks (block Gram-Schmidt);
//   cg_update     R~ = R - Q lambda fused with the Gram partials of R~
//                 (BAXPY + BDOT fusion of the two-reduction BCG, Ch. 8);
//   cg_pupdate    X += P (lambda sigma) and P = R + P beta in one pass;
//   block_combine Y +-= sum_j X_j C_j (Gram-Schmidt update, GMRes solution);
//   sddmm         sampled products on the CSR pattern;
//   casts / column scalings for the normalisers and iterative refinement.
//
// All kernels are bandwidth-bound (arithmetic intensity <= s/4 flop/byte in
// FP64, below the MI355X ridge of ~10).  Each lane streams 16-byte vectors.
// Gram matrices: per-lane register accumulation, a fixed butterfly over the
// row slots of a wavefront, a fixed-order sum over the wavefronts of a
// workgroup, one s x s partial per workgroup; then a small reduction kernel
// (at most 16 workgroups per Gram) sums contiguous slices of the partials and
// its last workgroup to finish adds the slice sums in slice order.  Which
// workgroup arrives last does not change the order of any sum, so results
// are deterministic.  The producers themselves need no grid-wide fences.
// Only integer counters use atomics; no floating-point atomics anywhere.
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"

namespace bkry {

template <int V>
using IC = std::integral_constant<int, V>;

// Calls f(IC<S>, IC<VEC>) for the block width s: powers of two use 16-byte
// vectors, other widths run one element per lane in the next power of two.
template <typename T, typename F>
hipError_t dispatch_s(int s, F&& f) {
  constexpr int vm = 16 / (int)sizeof(T);
  switch (s) {
    case 1: return f(IC<1>{}, IC<1>{});
    case 2: return f(IC<2>{}, IC<(2 < vm ? 2 : vm)>{});
    case 4: return f(IC<4>{}, IC<(4 < vm ? 4 : vm)>{});
    case 8: return f(IC<8>{}, IC<vm>{});
    case 16: return f(IC<16>{}, IC<vm>{});
    case 32: return f(IC<32>{}, IC<vm>{});
    default: break;
  }
  if (s == 3) return f(IC<4>{}, IC<1>{});
  if (s >= 5 && s <= 7) return f(IC<8>{}, IC<1>{});
  if (s >= 9 && s <= 15) return f(IC<16>{}, IC<1>{});
  if (s >= 17 && s <= 31) return f(IC<32>{}, IC<1>{});
  return hipErrorInvalidValue;
}

static int next_pow2(int s) {
  int S = 1;
  while (S < s) S <<= 1;
  return S;
}

int stream_grid(int64_t n, int s, int elem_bytes) {
  int S = next_pow2(s);
  int vm = 16 / elem_bytes;
  int VEC = (S == s) ? (S < vm ? S : vm) : 1;
  int LPR = S / VEC;
  int RPB = (kBlock / kWave) * (kWave / LPR);
  int64_t need = (n + RPB - 1) / RPB;
  int cap = (S <= 16) ? 1024 : 512;
  int64_t g = need < cap ? need : cap;
  g = (g + 7) / 8 * 8;
  return (int)(g < 8 ? 8 : g);
}

// Gather the full row (S values) held in chunks by the LPR lanes of a row
// slot and accumulate acc[a][b] += mine[a] * row[b] for a in the lane's own
// chunk.  All 64 lanes must execute this (the row slot's lanes are the
// shuffle sources).
template <typename T, int S, int VEC>
__device__ __forceinline__ void gram_row(T (&acc)[VEC][S], const vec_t<T, VEC>& mine, const vec_t<T, VEC>& other,
                                         int lane) {
  constexpr int LPR = S / VEC;
  const int base = lane & ~(LPR - 1);
#pragma unroll
  for (int cc = 0; cc < LPR; ++cc) {
    T o[VEC];
#pragma unroll
    for (int w = 0; w < VEC; ++w) o[w] = __shfl(other.v[w], base | cc);
#pragma unroll
    for (int a = 0; a < VEC; ++a)
#pragma unroll
      for (int w = 0; w < VEC; ++w) acc[a][cc * VEC + w] += mine.v[a] * o[w];
  }
}

// out[w] = sum_b row[b] * C[b][col0 + w] with the row gathered from the row
// slot's lanes and C an S x S matrix (stride S) in LDS.
template <typename T, int S, int VEC>
__device__ __forceinline__ void row_times(T (&out)[VEC], const vec_t<T, VEC>& mine, const T* C, int col0, int lane) {
  constexpr int LPR = S / VEC;
  const int base = lane & ~(LPR - 1);
#pragma unroll
  for (int w = 0; w < VEC; ++w) out[w] = T(0);
#pragma unroll
  for (int cc = 0; cc < LPR; ++cc) {
#pragma unroll
    for (int w2 = 0; w2 < VEC; ++w2) {
      T o = __shfl(mine.v[w2], base | cc);
      const T* crow = C + (cc * VEC + w2) * S + col0;
#pragma unroll
      for (int w = 0; w < VEC; ++w) out[w] += o * crow[w];
    }
  }
}

// Reduce per-lane Gram accumulators of a workgroup into its s x s partial
// (partial + ((blockIdx.y * gridDim.x + blockIdx.x) * s * s)).
template <typename T, int S, int VEC>
__device__ __forceinline__ void gram_store(T (&acc)[VEC][S], int s, T* partial, T* sh /* [NW][S*S] */) {
  constexpr int LPR = S / VEC;
  constexpr int NW = kBlock / kWave;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int c = lane % LPR;
#pragma unroll
  for (int a = 0; a < VEC; ++a)
#pragma unroll
    for (int b = 0; b < S; ++b) acc[a][b] = rowslot_sum<T, LPR>(acc[a][b]);
  if (lane < LPR) {
#pragma unroll
    for (int a = 0; a < VEC; ++a)
#pragma unroll
      for (int b = 0; b < S; ++b) sh[wave * S * S + (c * VEC + a) * S + b] = acc[a][b];
  }
  __syncthreads();
  T* pblk = partial + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * s * s;
  for (int t = threadIdx.x; t < s * s; t += kBlock) {
    int a = t / s, b = t % s;
    T sum = T(0);
#pragma unroll
    for (int w = 0; w < NW; ++w) sum += sh[w * S * S + a * S + b];
    pblk[t] = sum;
  }
}

// ------------------------------------------------------------ reduction --
// grid (ns, batch): workgroup (sl, y) sums partials [b0, b1) of slice y in
// block order into red.gpart[y][sl]; the last workgroup of slice y to finish
// adds the ns slice sums in order into red.G[y].  Only ns <= 16 workgroups
// take part, so the device-scope fences of the hand-off are cheap.
template <typename T>
__global__ __launch_bounds__(kBlock) void reduce_kernel(int ss, const T* __restrict__ partial, int nblk, Red red,
                                                         const int32_t* gate, const int32_t* fire) {
  __shared__ double sh[kBlock];
  __shared__ int last;
  if ((gate && *gate) || (fire && !*fire)) return;
  const int ns = gridDim.x, sl = blockIdx.x, y = blockIdx.y;
  const T* P = partial + (int64_t)y * nblk * ss;
  const int b0 = (int)((int64_t)nblk * sl / ns), b1 = (int)((int64_t)nblk * (sl + 1) / ns);
  double* slices = red.gpart + (int64_t)y * ns * ss;
  const int EB = ss < kBlock ? ss : kBlock;  // entries per pass
  const int SUB = kBlock / EB;                // sub-slices per entry
  const int t = threadIdx.x, te = t % EB, sub = t / EB;
  for (int base = 0; base < ss; base += EB) {
    const int e = base + te;
    double acc = 0.0;
    if (sub < SUB && e < ss)
      for (int b = b0 + sub; b < b1; b += SUB) acc += (double)P[(int64_t)b * ss + e];
    sh[t] = acc;
    __syncthreads();
    if (t < EB && e < ss) {
      double v = 0.0;
      for (int k = 0; k < SUB; ++k) v += sh[k * EB + t];
      slices[(int64_t)sl * ss + e] = v;
    }
    __syncthreads();
  }
  uint32_t* cnt = red.cnt + (int64_t)y * kCntStride;
  __threadfence();
  __syncthreads();
  if (t == 0) last = (atomicAdd(cnt, 1u) == (uint32_t)(ns - 1));
  __syncthreads();
  if (!last) return;
  __threadfence();
  double* G = red.G + (int64_t)y * ss;
  for (int e = t; e < ss; e += kBlock) {
    double v = 0.0;
    for (int k = 0; k < ns; ++k) v += slices[(int64_t)k * ss + e];
    G[e] = v;
  }
  if (t == 0) *cnt = 0;
}

static hipError_t launch_reduce(int s, const void* partial, bool f32, int nblk, int batch, Red red,
                                const int32_t* gate, const int32_t* fire, hipStream_t st) {
  const int ns = nblk < 16 ? nblk : 16;
  dim3 grid(ns, batch);
  if (f32)
    hipLaunchKernelGGL(reduce_kernel<float>, grid, dim3(kBlock), 0, st, s * s, static_cast<const float*>(partial),
                       nblk, red, gate, fire);
  else
    hipLaunchKernelGGL(reduce_kernel<double>, grid, dim3(kBlock), 0, st, s * s,
                       static_cast<const double*>(partial), nblk, red, gate, fire);
  return hipGetLastError();
}

// ------------------------------------------------------------------ SpMM --
// MODE 0: Y = A X.  MODE 1: Y = A X and Gram partials of X_own^T Y.
// MODE 2: Y = B - A X and Gram partials of Y^T Y.
template <typename T, int S, int VEC, int MODE>
__global__ __launch_bounds__(kBlock) void spmm_kernel(int64_t n, int64_t nnz, const int32_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ colind,
                                                       const T* __restrict__ val, int s, const T* __restrict__ X,
                                                       T* __restrict__ Y, const T* __restrict__ B,
                                                       T* __restrict__ partial, int32_t* bad,
                                                       const int32_t* done) {
  using L = Layout<T, S, VEC>;
  constexpr int NW = kBlock / kWave;
  constexpr int RPB = NW * L::RPW;
  constexpr int U = 8;
  constexpr int GA = MODE ? VEC : 1;
  constexpr int GB = MODE ? S : 1;
  __shared__ T sh[MODE ? NW * S * S : 1];
  if (done && *done) return;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r = lane / L::LPR, c = lane % L::LPR;
  const int col0 = c * VEC;
  const bool active = col0 < s;
  int64_t r0, r1;
  block_rows(n, blockIdx.x, gridDim.x, RPB, r0, r1);
  T gacc[GA][GB];
#pragma unroll
  for (int a = 0; a < GA; ++a)
#pragma unroll
    for (int b = 0; b < GB; ++b) gacc[a][b] = T(0);
  bool badidx = false;

  for (int64_t base = r0; base < r1; base += RPB) {
    const int64_t row = base + wave * L::RPW + r;
    const bool rv = row < r1 && active;
    vec_t<T, VEC> acc = zero_vec<T, VEC>();
    if (rv) {
      int64_t k0 = rowptr[row], k1 = rowptr[row + 1];
      if (k0 < 0) k0 = 0;
      if (k1 > nnz) k1 = nnz;
      for (int64_t k = k0; k < k1; k += U) {
        int jj[U];
        T aa[U];
        bool okk[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          okk[u] = (k + u) < k1;
          jj[u] = okk[u] ? colind[k + u] : 0;
          aa[u] = okk[u] ? val[k + u] : T(0);
        }
        vec_t<T, VEC> xx[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const bool okj = (uint32_t)jj[u] < (uint64_t)n;
          badidx |= okk[u] && !okj;
          xx[u] = (okk[u] && okj) ? load_vec<T, VEC>(X + (int64_t)jj[u] * s + col0) : zero_vec<T, VEC>();
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int w = 0; w < VEC; ++w) acc.v[w] += aa[u] * xx[u].v[w];
      }
      if (MODE == 2) {
        vec_t<T, VEC> b = load_vec<T, VEC>(B + row * s + col0);
#pragma unroll
        for (int w = 0; w < VEC; ++w) acc.v[w] = b.v[w] - acc.v[w];
      }
      store_vec<T, VEC>(Y + row * s + col0, acc);
    }
    if constexpr (MODE == 1) {
      vec_t<T, VEC> own = rv ? load_vec<T, VEC>(X + row * s + col0) : zero_vec<T, VEC>();
      gram_row<T, S, VEC>(gacc, own, acc, lane);
    } else if constexpr (MODE == 2) {
      gram_row<T, S, VEC>(gacc, acc, acc, lane);
    }
  }
  if (badidx && bad) *bad = 1;
  if constexpr (MODE != 0) gram_store<T, S, VEC>(gacc, s, partial, sh);
}

template <typename T>
hipError_t launch_spmm(const CsrView& A, int s, const T* X, T* Y, const T* B, int mode, T* partial, int nblk,
                       Red red, int32_t* bad, const int32_t* done, hipStream_t st) {
  hipError_t e = dispatch_s<T>(s, [&](auto S_, auto V_) -> hipError_t {
    constexpr int S = decltype(S_)::value, V = decltype(V_)::value;
    const T* val = static_cast<const T*>(A.val);
    if (mode == 0)
      hipLaunchKernelGGL((spmm_kernel<T, S, V, 0>), dim3(nblk), dim3(kBlock), 0, st, A.n, A.nnz, A.rowptr,
                         A.colind, val, s, X, Y, B, partial, bad, done);
    else if (mode == 1)
      hipLaunchKernelGGL((spmm_kernel<T, S, V, 1>), dim3(nblk), dim3(kBlock), 0, st, A.n, A.nnz, A.rowptr,
                         A.colind, val, s, X, Y, B, partial, bad, done);
    else
      hipLaunchKernelGGL((spmm_kernel<T, S, V, 2>), dim3(nblk), dim3(kBlock), 0, st, A.n, A.nnz, A.rowptr,
                         A.colind, val, s, X, Y, B, partial, bad, done);
    return hipGetLastError();
  });
  if (e != hipSuccess || mode == 0) return e;
  return launch_reduce(s, partial, sizeof(T) == 4, nblk, 1, red, done, nullptr, st);
}

// ------------------------------------------------------------------ Gram --
// blockIdx.y selects X_j = X + j * n * s; partial[(j * gridDim.x + blk) * s*s].
template <typename T, int S, int VEC>
__global__ __launch_bounds__(kBlock) void gram_kernel(int64_t n, int s, const T* __restrict__ X,
                                                       const T* __restrict__ Y, T* __restrict__ partial,
                                                       const int32_t* done, const int32_t* fire) {
  using L = Layout<T, S, VEC>;
  constexpr int NW = kBlock / kWave;
  constexpr int RPB = NW * L::RPW;
  __shared__ T sh[NW * S * S];
  if ((done && *done) || (fire && !*fire)) return;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r = lane / L::LPR, c = lane % L::LPR;
  const int col0 = c * VEC;
  const bool active = col0 < s;
  const T* Xj = X + (int64_t)blockIdx.y * n * s;
  int64_t r0, r1;
  block_rows(n, blockIdx.x, gridDim.x, RPB, r0, r1);
  T gacc[VEC][S];
#pragma unroll
  for (int a = 0; a < VEC; ++a)
#pragma unroll
    for (int b = 0; b < S; ++b) gacc[a][b] = T(0);
  for (int64_t base = r0; base < r1; base += RPB) {
    const int64_t row = base + wave * L::RPW + r;
    const bool rv = row < r1 && active;
    vec_t<T, VEC> x = rv ? load_vec<T, VEC>(Xj + row * s + col0) : zero_vec<T, VEC>();
    vec_t<T, VEC> y = rv ? load_vec<T, VEC>(Y + row * s + col0) : zero_vec<T, VEC>();
    gram_row<T, S, VEC>(gacc, x, y, lane);
  }
  gram_store<T, S, VEC>(gacc, s, partial, sh);
}

template <typename T>
hipError_t launch_gram(int64_t n, int s, const T* X, int nx, const T* Y, T* partial, int nblk, Red red,
                       const int32_t* done, hipStream_t st, const int32_t* fire) {
  if (nx <= 0) return hipSuccess;
  if (nx > kMaxBatch) return hipErrorInvalidValue;
  hipError_t e = dispatch_s<T>(s, [&](auto S_, auto V_) -> hipError_t {
    constexpr int S = decltype(S_)::value, V = decltype(V_)::value;
    hipLaunchKernelGGL((gram_kernel<T, S, V>), dim3(nblk, nx), dim3(kBlock), 0, st, n, s, X, Y, partial, done, fire);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  return launch_reduce(s, partial, sizeof(T) == 4, nblk, nx, red, done, fire, st);
}

// ---------------------------------------------------------- CG updates --
template <typename T>
__device__ __forceinline__ const T* ctl_mat(const CgCtl* ctl, int which);
template <>
__device__ __forceinline__ const double* ctl_mat<double>(const CgCtl* ctl, int which) {
  return which == 0 ? ctl->lam : which == 1 ? ctl->lamsig : ctl->beta;
}
template <>
__device__ __forceinline__ const float* ctl_mat<float>(const CgCtl* ctl, int which) {
  return which == 0 ? ctl->lam_f : which == 1 ? ctl->lamsig_f : ctl->beta_f;
}

// copy an s x s matrix (stride s) into an S x S LDS array padded with zeros
template <typename T, int S>
__device__ __forceinline__ void load_coeff(T* dst, const T* src, int s) {
  for (int t = threadIdx.x; t < S * S; t += kBlock) {
    int a = t / S, b = t % S;
    dst[t] = (a < s && b < s) ? src[a * s + b] : T(0);
  }
}

// R~ = R - Q lambda (in place in R); Gram partials of R~^T R~.
template <typename T, int S, int VEC>
__global__ __launch_bounds__(kBlock) void cg_update_kernel(int64_t n, int s, T* __restrict__ R,
                                                            const T* __restrict__ Q, const CgCtl* ctl,
                                                            T* __restrict__ partial) {
  using L = Layout<T, S, VEC>;
  constexpr int NW = kBlock / kWave;
  constexpr int RPB = NW * L::RPW;
  __shared__ T lam[S * S];
  __shared__ T sh[NW * S * S];
  if (ctl->gate) return;
  load_coeff<T, S>(lam, ctl_mat<T>(ctl, 0), s);
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r = lane / L::LPR, c = lane % L::LPR;
  const int col0 = c * VEC;
  const bool active = col0 < s;
  int64_t r0, r1;
  block_rows(n, blockIdx.x, gridDim.x, RPB, r0, r1);
  T gacc[VEC][S];
#pragma unroll
  for (int a = 0; a < VEC; ++a)
#pragma unroll
    for (int b = 0; b < S; ++b) gacc[a][b] = T(0);
  for (int64_t base = r0; base < r1; base += RPB) {
    const int64_t row = base + wave * L::RPW + r;
    const bool rv = row < r1 && active;
    vec_t<T, VEC> q = rv ? load_vec<T, VEC>(Q + row * s + col0) : zero_vec<T, VEC>();
    vec_t<T, VEC> rr = rv ? load_vec<T, VEC>(R + row * s + col0) : zero_vec<T, VEC>();
    T ql[VEC];
    row_times<T, S, VEC>(ql, q, lam, col0, lane);
    vec_t<T, VEC> out;
#pragma unroll
    for (int w = 0; w < VEC; ++w) out.v[w] = rr.v[w] - ql[w];
    if (rv) store_vec<T, VEC>(R + row * s + col0, out);
    gram_row<T, S, VEC>(gacc, out, out, lane);
  }
  gram_store<T, S, VEC>(gacc, s, partial, sh);
}

template <typename T>
hipError_t launch_cg_update(int64_t n, int s, T* R, const T* Q, const CgCtl* ctl, T* partial, int nblk, Red red,
                            hipStream_t st) {
  hipError_t e = dispatch_s<T>(s, [&](auto S_, auto V_) -> hipError_t {
    constexpr int S = decltype(S_)::value, V = decltype(V_)::value;
    hipLaunchKernelGGL((cg_update_kernel<T, S, V>), dim3(nblk), dim3(kBlock), 0, st, n, s, R, Q, ctl, partial);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  return launch_reduce(s, partial, sizeof(T) == 4, nblk, 1, red, &ctl->gate, nullptr, st);
}

// X += P (lambda sigma); unless the solve has ended: P = R + P beta.
template <typename T, int S, int VEC>
__global__ __launch_bounds__(kBlock) void cg_pupdate_kernel(int64_t n, int s, T* __restrict__ X,
                                                             T* __restrict__ P, const T* __restrict__ R,
                                                             const CgCtl* ctl) {
  using L = Layout<T, S, VEC>;
  constexpr int NW = kBlock / kWave;
  constexpr int RPB = NW * L::RPW;
  __shared__ T ls[S * S];
  __shared__ T bt[S * S];
  if (!ctl->x_pending || ctl->suspended) return;
  const bool pdir = !ctl->done;
  load_coeff<T, S>(ls, ctl_mat<T>(ctl, 1), s);
  load_coeff<T, S>(bt, ctl_mat<T>(ctl, 2), s);
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r = lane / L::LPR, c = lane % L::LPR;
  const int col0 = c * VEC;
  const bool active = col0 < s;
  int64_t r0, r1;
  block_rows(n, blockIdx.x, gridDim.x, RPB, r0, r1);
  for (int64_t base = r0; base < r1; base += RPB) {
    const int64_t row = base + wave * L::RPW + r;
    const bool rv = row < r1 && active;
    vec_t<T, VEC> p = rv ? load_vec<T, VEC>(P + row * s + col0) : zero_vec<T, VEC>();
    vec_t<T, VEC> x = rv ? load_vec<T, VEC>(X + row * s + col0) : zero_vec<T, VEC>();
    T dx[VEC];
    row_times<T, S, VEC>(dx, p, ls, col0, lane);
#pragma unroll
    for (int w = 0; w < VEC; ++w) x.v[w] += dx[w];
    if (rv) store_vec<T, VEC>(X + row * s + col0, x);
    if (pdir) {
      vec_t<T, VEC> rr = rv ? load_vec<T, VEC>(R + row * s + col0) : zero_vec<T, VEC>();
      T pb[VEC];
      row_times<T, S, VEC>(pb, p, bt, col0, lane);
#pragma unroll
      for (int w = 0; w < VEC; ++w) rr.v[w] += pb[w];
      if (rv) store_vec<T, VEC>(P + row * s + col0, rr);
    }
  }
}

template <typename T>
hipError_t launch_cg_pupdate(int64_t n, int s, T* X, T* P, const T* R, const CgCtl* ctl, hipStream_t st) {
  int nblk = stream_grid(n, s, sizeof(T));
  return dispatch_s<T>(s, [&](auto S_, auto V_) -> hipError_t {
    constexpr int S = decltype(S_)::value, V = decltype(V_)::value;
    hipLaunchKernelGGL((cg_pupdate_kernel<T, S, V>), dim3(nblk), dim3(kBlock), 0, st, n, s, X, P, R, ctl);
    return hipGetLastError();
  });
}

// ----------------------------------------------------- block combination --
// Y = Y + sign * sum_{j < nx} X_j C_j; C_j (s x s FP64, stride s) staged in
// LDS in chunks of JC blocks.
template <typename T, int S, int VEC>
__global__ __launch_bounds__(kBlock) void combine_kernel(int64_t n, int s, const T* __restrict__ X, int nx,
                                                          const double* __restrict__ C, double sign,
                                                          T* __restrict__ Y, const int32_t* done) {
  using L = Layout<T, S, VEC>;
  constexpr int NW = kBlock / kWave;
  constexpr int RPB = NW * L::RPW;
  constexpr int JC = (4096 / (S * S)) < 1 ? 1 : (4096 / (S * S));
  __shared__ T cs[JC * S * S];
  if (done && *done) return;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r = lane / L::LPR, c = lane % L::LPR;
  const int col0 = c * VEC;
  const bool active = col0 < s;
  int64_t r0, r1;
  block_rows(n, blockIdx.x, gridDim.x, RPB, r0, r1);
  for (int64_t base = r0; base < r1; base += RPB) {
    const int64_t row = base + wave * L::RPW + r;
    const bool rv = row < r1 && active;
    T acc[VEC];
#pragma unroll
    for (int w = 0; w < VEC; ++w) acc[w] = T(0);
    for (int j0 = 0; j0 < nx; j0 += JC) {
      const int jn = (nx - j0) < JC ? (nx - j0) : JC;
      __syncthreads();
      for (int t = threadIdx.x; t < jn * S * S; t += kBlock) {
        int jj = t / (S * S), e = t % (S * S), a = e / S, b = e % S;
        cs[t] = (a < s && b < s) ? (T)(sign * C[(int64_t)(j0 + jj) * s * s + a * s + b]) : T(0);
      }
      __syncthreads();
      for (int jj = 0; jj < jn; ++jj) {
        const T* Xj = X + (int64_t)(j0 + jj) * n * s;
        vec_t<T, VEC> x = rv ? load_vec<T, VEC>(Xj + row * s + col0) : zero_vec<T, VEC>();
        T d[VEC];
        row_times<T, S, VEC>(d, x, cs + jj * S * S, col0, lane);
#pragma unroll
        for (int w = 0; w < VEC; ++w) acc[w] += d[w];
      }
    }
    if (rv) {
      vec_t<T, VEC> y = load_vec<T, VEC>(Y + row * s + col0);
#pragma unroll
      for (int w = 0; w < VEC; ++w) y.v[w] += acc[w];
      store_vec<T, VEC>(Y + row * s + col0, y);
    }
  }
}

template <typename T>
hipError_t launch_block_combine(int64_t n, int s, const T* X, int nx, const double* C, double sign, T* Y,
                                const int32_t* done, hipStream_t st) {
  if (nx <= 0) return hipSuccess;
  int nblk = stream_grid(n, s, sizeof(T));
  return dispatch_s<T>(s, [&](auto S_, auto V_) -> hipError_t {
    constexpr int S = decltype(S_)::value, V = decltype(V_)::value;
    hipLaunchKernelGGL((combine_kernel<T, S, V>), dim3(nblk), dim3(kBlock), 0, st, n, s, X, nx, C, sign, Y,
                       done);
    return hipGetLastError();
  });
}

// ----------------------------------------------------------------- SDDMM --
template <typename T, int S, int VEC>
__global__ __launch_bounds__(kBlock) void sddmm_kernel(int64_t n, int64_t nnz, const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ colind, int s, T alpha,
                                                        const T* __restrict__ Lm, const T* __restrict__ X,
                                                        T* __restrict__ out, int32_t* bad) {
  using L = Layout<T, S, VEC>;
  constexpr int NW = kBlock / kWave;
  constexpr int RPB = NW * L::RPW;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r = lane / L::LPR, c = lane % L::LPR;
  const int col0 = c * VEC;
  const bool active = col0 < s;
  int64_t r0, r1;
  block_rows(n, blockIdx.x, gridDim.x, RPB, r0, r1);
  bool badidx = false;
  for (int64_t base = r0; base < r1; base += RPB) {
    const int64_t row = base + wave * L::RPW + r;
    if (row >= r1) continue;  // whole row slot leaves together
    vec_t<T, VEC> l = active ? load_vec<T, VEC>(Lm + row * s + col0) : zero_vec<T, VEC>();
    int64_t k0 = rowptr[row], k1 = rowptr[row + 1];
    if (k0 < 0) k0 = 0;
    if (k1 > nnz) k1 = nnz;
    for (int64_t k = k0; k < k1; ++k) {
      const int j = colind[k];
      const bool okj = (uint32_t)j < (uint64_t)n;
      badidx |= !okj;
      vec_t<T, VEC> x = (okj && active) ? load_vec<T, VEC>(X + (int64_t)j * s + col0) : zero_vec<T, VEC>();
      T d = T(0);
#pragma unroll
      for (int w = 0; w < VEC; ++w) d += l.v[w] * x.v[w];
      d = rowgroup_sum<T, L::LPR>(d);
      if (c == 0) out[k] = alpha * d;
    }
  }
  if (badidx && bad) *bad = 1;
}

template <typename T>
hipError_t launch_sddmm(const CsrView& A, int s, double alpha, const T* Lm, const T* X, T* out, int32_t* bad,
                        hipStream_t st) {
  int nblk = stream_grid(A.n, s, sizeof(T));
  return dispatch_s<T>(s, [&](auto S_, auto V_) -> hipError_t {
    constexpr int S = decltype(S_)::value, V = decltype(V_)::value;
    hipLaunchKernelGGL((sddmm_kernel<T, S, V>), dim3(nblk), dim3(kBlock), 0, st, A.n, A.nnz, A.rowptr, A.colind, s,
                       (T)alpha, Lm, X, out, bad);
    return hipGetLastError();
  });
}

// ------------------------------------------------- elementwise helpers --
// Y[i][j] = X[i][j] / d[j] if d[j] > 0, else the unit vector e_z(j) with
// z(j) = 0 (parallel normaliser) or j (global normaliser).
template <typename T>
__global__ __launch_bounds__(kBlock) void colscale_kernel(int64_t n, int s, const T* __restrict__ X,
                                                           T* __restrict__ Y, const double* __restrict__ d,
                                                           int global_kind, const int32_t* gd, const int32_t* gf) {
  if (gd && *gd) return;
  if (gf && !*gf) return;
  const int64_t total = n * s;
  for (int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x; t < total; t += (int64_t)gridDim.x * kBlock) {
    const int64_t i = t / s;
    const int j = (int)(t % s);
    const double dj = d[j];
    const int64_t z = global_kind ? j : 0;
    Y[t] = dj > 0.0 ? (T)((double)X[t] / dj) : (T)(i == z ? 1.0 : 0.0);
  }
}

template <typename T>
hipError_t launch_colscale(int64_t n, int s, const T* X, T* Y, const double* d, int global_kind,
                           const int32_t* gate_done, const int32_t* gate_fire, hipStream_t st) {
  int64_t blocks = (n * s + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(colscale_kernel<T>, dim3((unsigned)blocks), dim3(kBlock), 0, st, n, s, X, Y, d, global_kind,
                     gate_done, gate_fire);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void cast_scale_kernel(int64_t n, int s, const double* __restrict__ R,
                                                             const double* __restrict__ scale,
                                                             float* __restrict__ out) {
  const int64_t total = n * s;
  for (int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x; t < total; t += (int64_t)gridDim.x * kBlock) {
    const double sc = scale[t % s];
    out[t] = sc > 0.0 ? (float)(R[t] / sc) : 0.0f;
  }
}

hipError_t launch_cast_scale_f32(int64_t n, int s, const double* R, const double* scale, float* out,
                                 hipStream_t st) {
  int64_t blocks = (n * s + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(cast_scale_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, st, n, s, R, scale, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void accum_scaled_kernel(int64_t n, int s, const float* __restrict__ D,
                                                               const double* __restrict__ scale,
                                                               double* __restrict__ X) {
  const int64_t total = n * s;
  for (int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x; t < total; t += (int64_t)gridDim.x * kBlock)
    X[t] += (double)D[t] * scale[t % s];
}

hipError_t launch_accum_scaled(int64_t n, int s, const float* D, const double* scale, double* X, hipStream_t st) {
  int64_t blocks = (n * s + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(accum_scaled_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, st, n, s, D, scale, X);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void cast_f32_kernel(int64_t count, const double* __restrict__ in,
                                                           float* __restrict__ out) {
  for (int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x; t < count; t += (int64_t)gridDim.x * kBlock)
    out[t] = (float)in[t];
}

hipError_t launch_cast_f32(int64_t count, const double* in, float* out, hipStream_t st) {
  int64_t blocks = (count + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(cast_f32_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, st, count, in, out);
  return hipGetLastError();
}

// ------------------------------------------------------ instantiations --
#define BKRY_INST(T)                                                                                              \
  template hipError_t launch_spmm<T>(const CsrView&, int, const T*, T*, const T*, int, T*, int, Red, int32_t*,     \
                                     const int32_t*, hipStream_t);                                                 \
  template hipError_t launch_gram<T>(int64_t, int, const T*, int, const T*, T*, int, Red, const int32_t*,          \
                                     hipStream_t, const int32_t*);                                                 \
  template hipError_t launch_cg_update<T>(int64_t, int, T*, const T*, const CgCtl*, T*, int, Red, hipStream_t);    \
  template hipError_t launch_cg_pupdate<T>(int64_t, int, T*, T*, const T*, const CgCtl*, hipStream_t);             \
  template hipError_t launch_block_combine<T>(int64_t, int, const T*, int, const double*, double, T*,               \
                                              const int32_t*, hipStream_t);                                        \
  template hipError_t launch_colscale<T>(int64_t, int, const T*, T*, const double*, int, const int32_t*,           \
                                         const int32_t*, hipStream_t);                                             \
  template hipError_t launch_sddmm<T>(const CsrView&, int, double, const T*, const T*, T*, int32_t*, hipStream_t);

BKRY_INST(double)
BKRY_INST(float)

}  // namespace bkry
