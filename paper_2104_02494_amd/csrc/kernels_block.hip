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

// Non-zeros per SpMM load batch of the CSR kernel.
constexpr int kUnroll = 8;
// Workgroups per gang of the ELL SpMM (see gang_rows).
constexpr int kGang = 8;
// Chunks of a row whose matrix entries the ELL SpMM requests ahead (rows of
// more than one chunk).
constexpr int kPfChunks = 3;


// Store of a streaming output.
template <typename T, int N>
__device__ __forceinline__ void store_out(T* p, const vec_t<T, N>& x) {
  store_vec<T, N>(p, x);
}
// Store of a streaming output with the non-temporal hint.  On MI355X this
// is faster for the SpMM output and the direction update (measured), and
// slower for the in-place residual update, which keeps store_out.
template <typename T, int N>
__device__ __forceinline__ void store_nt(T* p, const vec_t<T, N>& x) {
#pragma unroll
  for (int i = 0; i < N; ++i) __builtin_nontemporal_store(x.v[i], p + i);
}

static int next_pow2(int s) {
  int S = 1;
  while (S < s) S <<= 1;
  return S;
}

// VEC chosen by dispatch_s for width s and element size (host mirror).
static int vec_for(int s, int elem_bytes) {
  const int v16 = 16 / elem_bytes;
  switch (s) {
    case 1: return 1;
    case 2: return 2;
    case 4: return 4;
    case 8: return v16;
    case 16:
    case 32: return v16;
    default: return 1;
  }
}

int spmm_lanes_per_row(int s, int elem_bytes) { return next_pow2(s) / vec_for(s, elem_bytes); }

// Launch width of a streaming kernel without Gram partials: wider, since no
// reduction has to read one partial per workgroup.
static int stream_grid_wide(int64_t n, int s, int elem_bytes) {
  const int S = next_pow2(s);
  const int RPB = (kBlock / kWave) * (kWave / (S / vec_for(s, elem_bytes)));
  int64_t g = (n + RPB - 1) / RPB;
  if (g > 4096) g = 4096;
  g = (g + 7) / 8 * 8;
  return (int)(g < 8 ? 8 : g);
}

int stream_grid(int64_t n, int s, int elem_bytes) {
  int S = next_pow2(s);
  int VEC = vec_for(s, elem_bytes);
  int LPR = S / VEC;
  int RPB = (kBlock / kWave) * (kWave / LPR);
  int64_t need = (n + RPB - 1) / RPB;
  int cap = (S <= 16) ? 1024 : 512;
  int64_t g = need < cap ? need : cap;
  g = (g + 7) / 8 * 8;
  return (int)(g < 8 ? 8 : g);
}

// Row slots of 8 or more lanes (S = 16, 32 with 16-byte chunks, and the
// one-element layouts of the odd widths) share rows through LDS: each lane
// stores its chunk, then every lane reads the whole row with vector loads
// that all lanes of the slot issue together (broadcast reads).  That replaces
// S cross-lane permutes per row, whose latency serialised the wide kernels.
// The slot's lanes are in one wavefront, whose LDS accesses execute in order,
// so no barrier is needed.  Each row slot of the workgroup owns S entries.
template <typename T, int S, int VEC>
__device__ __forceinline__ const T* lds_row(const vec_t<T, VEC>& v) {
  constexpr int LPR = S / VEC;
  __shared__ __align__(16) T rows[kBlock / LPR * S];
  T* r = rows + (threadIdx.x / LPR) * S;
  store_vec<T, VEC>(r + (threadIdx.x % LPR) * VEC, v);
  __builtin_amdgcn_wave_barrier();
  return r;
}

// Gather the full row (S values) held in chunks by the LPR lanes of a row
// slot and accumulate acc[a][b] += mine[a] * row[b] for a in the lane's own
// chunk.  All 64 lanes must execute this (the row slot's lanes are the
// sources); for LPR <= 4 the values move by DPP quad permutations, wider
// slots go through LDS (lds_row).
template <typename T, int S, int VEC>
__device__ __forceinline__ void gram_row(T (&acc)[VEC][S], const vec_t<T, VEC>& mine, const vec_t<T, VEC>& other,
                                         int lane) {
  constexpr int LPR = S / VEC;
  (void)lane;
  if constexpr (LPR >= 8) {
    const T* r = lds_row<T, S, VEC>(other);
#pragma unroll
    for (int b0 = 0; b0 < S; b0 += 2) {
      const vec_t<T, 2> o = load_vec<T, 2>(r + b0);
#pragma unroll
      for (int a = 0; a < VEC; ++a) {
        acc[a][b0] += mine.v[a] * o.v[0];
        acc[a][b0 + 1] += mine.v[a] * o.v[1];
      }
    }
  } else {
    static_for<LPR>([&](auto cc_) {
      constexpr int cc = decltype(cc_)::value;
      T o[VEC];
#pragma unroll
      for (int w = 0; w < VEC; ++w) o[w] = group_bcast<LPR, cc>(other.v[w]);
#pragma unroll
      for (int a = 0; a < VEC; ++a)
#pragma unroll
        for (int w = 0; w < VEC; ++w) acc[a][cc * VEC + w] += mine.v[a] * o[w];
    });
  }
}

// out[w] += sum_b row[b] * C[b][col0 + w] (one fused multiply-add per term, b
// in order) with the row gathered from the row slot's lanes and C an S x S
// matrix (stride S) in LDS.
template <typename T, int S, int VEC>
__device__ __forceinline__ void row_times_acc(T (&out)[VEC], const vec_t<T, VEC>& mine, const T* C, int col0) {
  constexpr int LPR = S / VEC;
  if constexpr (LPR >= 8) {
    const T* r = lds_row<T, S, VEC>(mine);
#pragma unroll
    for (int b0 = 0; b0 < S; b0 += 2) {
      const vec_t<T, 2> o = load_vec<T, 2>(r + b0);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const T* crow = C + (b0 + h) * S + col0;
#pragma unroll
        for (int w = 0; w < VEC; ++w) out[w] = fma(o.v[h], crow[w], out[w]);
      }
    }
  } else {
    static_for<LPR>([&](auto cc_) {
      constexpr int cc = decltype(cc_)::value;
#pragma unroll
      for (int w2 = 0; w2 < VEC; ++w2) {
        const T o = group_bcast<LPR, cc>(mine.v[w2]);
        const T* crow = C + (cc * VEC + w2) * S + col0;
#pragma unroll
        for (int w = 0; w < VEC; ++w) out[w] = fma(o, crow[w], out[w]);
      }
    });
  }
}

// out[w] = sum_b row[b] * C[b][col0 + w] with the row gathered from the row
// slot's lanes and C an S x S matrix (stride S) in LDS.
template <typename T, int S, int VEC>
__device__ __forceinline__ void row_times(T (&out)[VEC], const vec_t<T, VEC>& mine, const T* C, int col0, int lane) {
  constexpr int LPR = S / VEC;
  (void)lane;
#pragma unroll
  for (int w = 0; w < VEC; ++w) out[w] = T(0);
  if constexpr (LPR >= 8) {
    const T* r = lds_row<T, S, VEC>(mine);
#pragma unroll
    for (int b0 = 0; b0 < S; b0 += 2) {
      const vec_t<T, 2> o = load_vec<T, 2>(r + b0);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const T* crow = C + (b0 + h) * S + col0;
#pragma unroll
        for (int w = 0; w < VEC; ++w) out[w] += o.v[h] * crow[w];
      }
    }
  } else {
    static_for<LPR>([&](auto cc_) {
      constexpr int cc = decltype(cc_)::value;
#pragma unroll
      for (int w2 = 0; w2 < VEC; ++w2) {
        const T o = group_bcast<LPR, cc>(mine.v[w2]);
        const T* crow = C + (cc * VEC + w2) * S + col0;
#pragma unroll
        for (int w = 0; w < VEC; ++w) out[w] += o * crow[w];
      }
    });
  }
}

// Reduce per-lane Gram accumulators of a workgroup into its s x s partial
// (partial + ((blockIdx.y * gridDim.x + blockIdx.x) * s * s)).
// Reduce the per-lane Gram accumulators of the workgroup and write its s x s
// partial of batch slice `slice` (partial[(slice * gridDim.x + blockIdx.x) *
// s * s]).  Safe to call several times in a row (LDS is reused).
template <typename T, int S, int VEC>
__device__ __forceinline__ void gram_store(T (&acc)[VEC][S], int s, T* partial, T* sh /* [NW][S*S] */,
                                           int64_t slice = 0, int64_t pstride = 0) {
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
  T* pblk = partial + (slice * gridDim.x + blockIdx.x) * (pstride > 0 ? pstride : (int64_t)s * s);
  for (int t = threadIdx.x; t < s * s; t += kBlock) {
    int a = t / s, b = t % s;
    T sum = T(0);
#pragma unroll
    for (int w = 0; w < NW; ++w) sum += sh[w * S * S + a * S + b];
    pblk[t] = sum;
  }
  __syncthreads();
}

// ------------------------------------------------------------------ SpMM --
// MODE 0: Y = A X.  MODE 1: Y = A X and Gram partials of X_own^T Y.
// MODE 2: Y = B - A X and Gram partials of Y^T Y.  Every product term is an
// explicit fused multiply-add in storage order, so the CSR and ELL kernels
// round identically.
//
// CSR kernel, software-pipelined: the row pointers of tile i+2 and the first
// kUnroll non-zeros of tile i+1 are loaded while the X rows of tile i are
// gathered, so one memory round trip per tile is exposed instead of three.
template <typename T, int S, int VEC, int MODE>
__global__ __launch_bounds__(kBlock) void spmm_csr_kernel(int64_t n, int64_t nnz, const int32_t* __restrict__ rowptr,
                                                          const int32_t* __restrict__ colind,
                                                          const T* __restrict__ val, int s, const T* __restrict__ X,
                                                          T* __restrict__ Y, const T* __restrict__ B,
                                                          T* __restrict__ partial, int32_t* bad,
                                                          const int32_t* done, int64_t pstride) {
  using L = Layout<T, S, VEC>;
  constexpr int NW = kBlock / kWave;
  constexpr int RPB = NW * L::RPW;
  constexpr int U = kUnroll;
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
  const int64_t step = RPB;
  T gacc[GA][GB];
#pragma unroll
  for (int a = 0; a < GA; ++a)
#pragma unroll
    for (int b = 0; b < GB; ++b) gacc[a][b] = T(0);
  bool badidx = false;
  const int64_t roff = wave * L::RPW + r;

  // row extent [k0, k1) clamped to [0, nnz]; empty for rows outside the slice
  auto ld_rp = [&](int64_t rw, int64_t& k0, int64_t& k1) {
    k0 = 0;
    k1 = 0;
    if (rw < r1 && active) {
      k0 = rowptr[rw];
      k1 = rowptr[rw + 1];
      k0 = k0 < 0 ? 0 : k0;
      k1 = k1 > nnz ? nnz : k1;
    }
  };
  // first U entries of [k0, k1): returns how many are present
  auto ld_chunk = [&](int64_t k0, int64_t k1, int (&jj)[U], T (&aa)[U]) -> int {
    const int64_t m = k1 - k0;
    const int cnt = m <= 0 ? 0 : (m < U ? (int)m : U);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      jj[u] = u < cnt ? colind[k0 + u] : 0;
      aa[u] = u < cnt ? val[k0 + u] : T(0);
    }
    return cnt;
  };

  int64_t k0c, k1c, k0n, k1n;
  ld_rp(r0 + roff, k0c, k1c);
  ld_rp(r0 + roff + step, k0n, k1n);
  int cj[U];
  T ca[U];
  int cc = ld_chunk(k0c, k1c, cj, ca);
  for (int64_t base = r0; base < r1; base += step) {
    const int64_t row = base + roff;
    const bool rv = row < r1 && active;
    int64_t k0nn, k1nn;
    ld_rp(row + 2 * step, k0nn, k1nn);
    int nj[U];
    T na[U];
    const int nc = ld_chunk(k0n, k1n, nj, na);
    vec_t<T, VEC> xx[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool okj = (uint32_t)cj[u] < (uint64_t)n;
      badidx |= (u < cc) && !okj;
      xx[u] = (u < cc && okj) ? load_vec<T, VEC>(X + (int64_t)cj[u] * s + col0) : zero_vec<T, VEC>();
    }
    vec_t<T, VEC> own = zero_vec<T, VEC>();
    if (MODE == 1 && rv) own = load_vec<T, VEC>(X + row * s + col0);
    if (MODE == 2 && rv) own = load_vec<T, VEC>(B + row * s + col0);
    vec_t<T, VEC> acc = zero_vec<T, VEC>();
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int w = 0; w < VEC; ++w) acc.v[w] = fma(ca[u], xx[u].v[w], acc.v[w]);
    // rows longer than U: remaining entries without pipelining
    for (int64_t k = k0c + U; k < k1c; k += U) {
      int jj[U];
      T aa[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool ok = (k + u) < k1c;
        jj[u] = ok ? colind[k + u] : 0;
        aa[u] = ok ? val[k + u] : T(0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool ok = (k + u) < k1c;
        const bool okj = (uint32_t)jj[u] < (uint64_t)n;
        badidx |= ok && !okj;
        xx[u] = (ok && okj) ? load_vec<T, VEC>(X + (int64_t)jj[u] * s + col0) : zero_vec<T, VEC>();
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int w = 0; w < VEC; ++w) acc.v[w] = fma(aa[u], xx[u].v[w], acc.v[w]);
    }
    if (MODE == 2) {
#pragma unroll
      for (int w = 0; w < VEC; ++w) acc.v[w] = own.v[w] - acc.v[w];
    }
    if (rv) store_nt<T, VEC>(Y + row * s + col0, acc);
    if constexpr (MODE == 1) {
      gram_row<T, S, VEC>(gacc, own, acc, lane);
    } else if constexpr (MODE == 2) {
      gram_row<T, S, VEC>(gacc, acc, acc, lane);
    }
    k0c = k0n;
    k1c = k1n;
    k0n = k0nn;
    k1n = k1nn;
    cc = nc;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      cj[u] = nj[u];
      ca[u] = na[u];
    }
  }
  if (badidx && bad) *bad = 1;
  if constexpr (MODE != 0) gram_store<T, S, VEC>(gacc, s, partial, sh, 0, pstride);
}

// SpMM on the padded row-major (ELL) copy of A: row i's entries sit at
// [i*W, i*W + W), padding marked by column -1.  The LPR lanes of a row load a
// chunk of C = LPR*E consecutive entries with one E-wide load each (so the
// matrix stream is read with fully coalesced loads and no row pointers), and
// the entries are passed around the row group with lane permutations before
// the gathers.  The first chunk of the next tile is loaded while the current
// tile gathers.  Entries are summed in storage order, padding contributing
// nothing: on a copy in CSR order the result equals the CSR kernel's bit for
// bit.  The solvers' copies hold each row's diagonal entry in slot 0 (diag0):
// the Gram X^T (A X) of MODE 1 then takes the row's own X values from that
// entry's gather instead of loading them a second time.
//
// Cache use: every matrix line is consumed by one load, so the matrix stream
// is read with the non-temporal hint and leaves the L2 to the gathered X
// rows; gangs of kGang workgroups sweep one row range together (gang_rows),
// so an XCD runs few concurrent row fronts and the X rows that neighbouring
// rows share (a banded or stencil pattern) are still in its L2 when reused.
template <typename T, int S, int VEC, int MODE, bool PF = false>
__global__ __launch_bounds__(kBlock) void spmm_ell_kernel(int64_t n, int W, const int32_t* __restrict__ ecol,
                                                           const T* __restrict__ eval, int s,
                                                           const T* __restrict__ X, T* __restrict__ Y,
                                                           const T* __restrict__ B, T* __restrict__ partial,
                                                           const int32_t* done, int64_t pstride, int diag0) {
  using L = Layout<T, S, VEC>;
  constexpr int LPR = L::LPR;
  constexpr int E = ell_entries_per_lane(LPR);
  constexpr int C = LPR * E;
  constexpr int NW = kBlock / kWave;
  constexpr int RPB = NW * L::RPW;
  constexpr int GA = MODE ? VEC : 1;
  constexpr int GB = MODE ? S : 1;
  __shared__ T sh[MODE ? NW * S * S : 1];
  if (done && *done) return;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r = lane / LPR, c = lane % LPR;
  const int col0 = c * VEC;
  const bool active = col0 < s;
  int64_t r0, r1, step;
  gang_rows(n, blockIdx.x, gridDim.x, RPB, kGang, r0, r1, step);
  T gacc[GA][GB];
#pragma unroll
  for (int a = 0; a < GA; ++a)
#pragma unroll
    for (int b = 0; b < GB; ++b) gacc[a][b] = T(0);
  const int64_t roff = wave * L::RPW + r;
  const int nch = W / C;

  // this lane's E entries of chunk j of row rw (padding outside the range)
  auto ld = [&](int64_t rw, int j, vec_t<int32_t, E>& cj, vec_t<T, E>& ca) {
    if (rw < r1) {
      const int64_t k = rw * W + (int64_t)j * C + c * E;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        cj.v[e] = __builtin_nontemporal_load(ecol + k + e);
        ca.v[e] = __builtin_nontemporal_load(eval + k + e);
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        cj.v[e] = -1;
        ca.v[e] = T(0);
      }
    }
  };
  // acc += sum over the chunk's C entries, in storage order
  // (slots of 8 or more lanes share the chunk's entries through LDS, as
  // lds_row does for rows); with take, first = the X values of entry 0
  auto chunk = [&](const vec_t<int32_t, E>& cj, const vec_t<T, E>& ca, bool rv, vec_t<T, VEC>& acc, bool take,
                   vec_t<T, VEC>& first) {
    int jj[C];
    T aa[C];
    if constexpr (LPR >= 8) {
      __shared__ __align__(16) int32_t js[kBlock / LPR * C];
      __shared__ __align__(16) T as[kBlock / LPR * C];
      const int base = (threadIdx.x / LPR) * C;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        js[base + c * E + e] = cj.v[e];
        as[base + c * E + e] = ca.v[e];
      }
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int u = 0; u < C; u += 4) {
        const vec_t<int32_t, 4> q = load_vec<int32_t, 4>(js + base + u);
#pragma unroll
        for (int h = 0; h < 4; ++h) jj[u + h] = q.v[h];
      }
#pragma unroll
      for (int u = 0; u < C; u += 2) {
        const vec_t<T, 2> q = load_vec<T, 2>(as + base + u);
        aa[u] = q.v[0];
        aa[u + 1] = q.v[1];
      }
    } else {
      static_for<C>([&](auto u_) {
        constexpr int u = decltype(u_)::value;
        jj[u] = group_bcast<LPR, u / E>(cj.v[u % E]);
        aa[u] = group_bcast<LPR, u / E>(ca.v[u % E]);
      });
    }
    vec_t<T, VEC> xx[C];
#pragma unroll
    for (int u = 0; u < C; ++u) {
      const bool ok = rv && (uint32_t)jj[u] < (uint64_t)n;
      xx[u] = ok ? load_vec<T, VEC>(X + (int64_t)jj[u] * s + col0) : zero_vec<T, VEC>();
      if (!ok) aa[u] = T(0);
    }
    if (take) {
#pragma unroll
      for (int w = 0; w < VEC; ++w) first.v[w] = xx[0].v[w];
    }
#pragma unroll
    for (int u = 0; u < C; ++u)
#pragma unroll
      for (int w = 0; w < VEC; ++w) acc.v[w] = fma(aa[u], xx[u].v[w], acc.v[w]);
  };
  // MODE 1 on a diagonal-first copy: the own rows come from the first gather
  const bool own_first = MODE == 1 && diag0;
  // FP32 entries up to 16 columns: chunks 1 .. kPfChunks of the next tile are
  // requested with its chunk 0, during this tile's gathers (for FP64 entries
  // the extra registers would cost a wavefront per SIMD)
  constexpr bool NEXT = PF && sizeof(T) == 4 && S <= 16;

  vec_t<int32_t, E> cj, nj;
  vec_t<T, E> ca, na;
  vec_t<int32_t, E> pj[kPfChunks], qj[kPfChunks];
  vec_t<T, E> pa[kPfChunks], qa[kPfChunks];
  ld(r0 + roff, 0, cj, ca);
  if constexpr (NEXT) {
#pragma unroll
    for (int q = 0; q < kPfChunks; ++q)
      if (1 + q < nch) ld(r0 + roff, 1 + q, pj[q], pa[q]);
  }
  for (int64_t base = r0; base < r1; base += step) {
    const int64_t row = base + roff;
    const bool rv = row < r1 && active;
    ld(row + step, 0, nj, na);
    vec_t<T, VEC> own = zero_vec<T, VEC>();
    if (MODE == 1 && rv && !own_first) own = load_vec<T, VEC>(X + row * s + col0);
    if (MODE == 2 && rv) own = load_vec<T, VEC>(B + row * s + col0);
    vec_t<T, VEC> acc = zero_vec<T, VEC>();
    if constexpr (NEXT) {
      // this tile's chunks 1 .. kPfChunks arrived during the previous tile;
      // the next tile's are requested now
#pragma unroll
      for (int q = 0; q < kPfChunks; ++q)
        if (1 + q < nch) ld(row + step, 1 + q, qj[q], qa[q]);
      chunk(cj, ca, rv, acc, own_first, own);
#pragma unroll
      for (int q = 0; q < kPfChunks; ++q)
        if (1 + q < nch) chunk(pj[q], pa[q], rv, acc, false, own);
      for (int j = 1 + kPfChunks; j < nch; ++j) {
        vec_t<int32_t, E> kj;
        vec_t<T, E> ka;
        ld(row, j, kj, ka);
        chunk(kj, ka, rv, acc, false, own);
      }
#pragma unroll
      for (int q = 0; q < kPfChunks; ++q) {
        pj[q] = qj[q];
        pa[q] = qa[q];
      }
    } else if constexpr (PF) {
      // rows of several chunks (wide stencils): the entries of chunks 1 ..
      // kPfChunks are requested before the first chunk's gathers, so a row
      // waits for its matrix entries once instead of once per chunk
      vec_t<int32_t, E> rj[kPfChunks];
      vec_t<T, E> ra[kPfChunks];
#pragma unroll
      for (int q = 0; q < kPfChunks; ++q)
        if (1 + q < nch) ld(row, 1 + q, rj[q], ra[q]);
      chunk(cj, ca, rv, acc, own_first, own);
#pragma unroll
      for (int q = 0; q < kPfChunks; ++q)
        if (1 + q < nch) chunk(rj[q], ra[q], rv, acc, false, own);
      for (int j = 1 + kPfChunks; j < nch; ++j) {
        vec_t<int32_t, E> kj;
        vec_t<T, E> ka;
        ld(row, j, kj, ka);
        chunk(kj, ka, rv, acc, false, own);
      }
    } else {
      chunk(cj, ca, rv, acc, own_first, own);
      for (int j = 1; j < nch; ++j) {
        vec_t<int32_t, E> kj;
        vec_t<T, E> ka;
        ld(row, j, kj, ka);
        chunk(kj, ka, rv, acc, false, own);
      }
    }
    if (MODE == 2) {
#pragma unroll
      for (int w = 0; w < VEC; ++w) acc.v[w] = own.v[w] - acc.v[w];
    }
    if (rv) store_nt<T, VEC>(Y + row * s + col0, acc);
    if constexpr (MODE == 1) {
      gram_row<T, S, VEC>(gacc, own, acc, lane);
    } else if constexpr (MODE == 2) {
      gram_row<T, S, VEC>(gacc, acc, acc, lane);
    }
    cj = nj;
    ca = na;
  }
  if constexpr (MODE != 0) gram_store<T, S, VEC>(gacc, s, partial, sh, 0, pstride);
}

// Workgroups of kernel K that the device holds at once (cached per kernel).
template <auto K>
static int resident_blocks() {
  static int cached = 0;
  if (cached == 0) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, K, kBlock, 0) != hipSuccess || per <= 0 || cus <= 0) {
      (void)hipGetLastError();
      return 1 << 30;
    }
    cached = per * cus;
  }
  return cached;
}

// Launch width of a streaming kernel: the requested width, capped so that
// every workgroup is resident (a workgroup owns a contiguous row range, so a
// second round of workgroups would only lengthen the tail), a multiple of 8.
template <auto K>
static int fit_grid(int nblk) {
  const int cap = resident_blocks<K>() / 8 * 8;
  return (cap >= 8 && nblk > cap) ? cap : nblk;
}

// Whether the ELL rows of width W span several chunks (the prefetching
// form of the ELL SpMM).
template <int S, int V>
static bool ell_prefetch(int W) {
  constexpr int LPR = S / V;
  return W / (LPR * ell_entries_per_lane(LPR)) > 1;
}

template <typename T>
hipError_t launch_spmm(const CsrView& A, int s, const T* X, T* Y, const T* B, int mode, T* partial, int nblk,
                       Red red, int32_t* bad, const int32_t* done, hipStream_t st, Epi epi, hipEvent_t ev_after,
                       int gram_slot, int ngram) {
  if constexpr (sizeof(T) == 8) {
    // wide blocks: the plain product, then X^T Y on the matrix cores (the
    // fused Gram's s x s per row is the larger cost at these widths)
    if (mode == 1 && ngram <= 1 && gram_slot == 0 && wide_mfma(s)) {
      hipError_t e = launch_spmm<T>(A, s, X, Y, B, 0, nullptr, nblk, red, bad, done, st, Epi{}, nullptr, 0, 1);
      if (e == hipSuccess) e = launch_gram_mfma(A.n, s, X, Y, partial, nblk, done, nullptr, st);
      if (e == hipSuccess && ev_after) e = hipEventRecord(ev_after, st);
      if (e != hipSuccess) return e;
      return launch_reduce(s, partial, false, nblk, 1, red, done, nullptr, epi, st);
    }
  }
  T* const pbase = partial;
  const int64_t pstride = ngram > 1 ? (int64_t)ngram * s * s : 0;
  partial += (int64_t)gram_slot * s * s;
  hipError_t e = dispatch_s<T>(s, [&](auto S_, auto V_) -> hipError_t {
    constexpr int S = decltype(S_)::value, V = decltype(V_)::value;
    const T* val = static_cast<const T*>(A.val);
    if (A.ell_w > 0) {
      const T* ev = static_cast<const T*>(A.ell_val);
      auto go = [&](auto PF_) {
        constexpr bool PF = decltype(PF_)::value;
        if (mode == 0) {
          nblk = fit_grid<spmm_ell_kernel<T, S, V, 0, PF>>(nblk);
          hipLaunchKernelGGL((spmm_ell_kernel<T, S, V, 0, PF>), dim3(nblk), dim3(kBlock), 0, st, A.n, A.ell_w,
                             A.ell_col, ev, s, X, Y, B, partial, done, pstride, 0);
        } else if (mode == 1) {
          nblk = fit_grid<spmm_ell_kernel<T, S, V, 1, PF>>(nblk);
          hipLaunchKernelGGL((spmm_ell_kernel<T, S, V, 1, PF>), dim3(nblk), dim3(kBlock), 0, st, A.n, A.ell_w,
                             A.ell_col, ev, s, X, Y, B, partial, done, pstride, A.ell_diag0 ? 1 : 0);
        } else {
          nblk = fit_grid<spmm_ell_kernel<T, S, V, 2, PF>>(nblk);
          hipLaunchKernelGGL((spmm_ell_kernel<T, S, V, 2, PF>), dim3(nblk), dim3(kBlock), 0, st, A.n, A.ell_w,
                             A.ell_col, ev, s, X, Y, B, partial, done, pstride, 0);
        }
      };
      if (ell_prefetch<S, V>(A.ell_w))
        go(std::true_type{});
      else
        go(std::false_type{});
      return hipGetLastError();
    }
    if (mode == 0)
      nblk = fit_grid<spmm_csr_kernel<T, S, V, 0>>(nblk);
    else if (mode == 1)
      nblk = fit_grid<spmm_csr_kernel<T, S, V, 1>>(nblk);
    else
      nblk = fit_grid<spmm_csr_kernel<T, S, V, 2>>(nblk);
    if (mode == 0)
      hipLaunchKernelGGL((spmm_csr_kernel<T, S, V, 0>), dim3(nblk), dim3(kBlock), 0, st, A.n, A.nnz, A.rowptr,
                         A.colind, val, s, X, Y, B, partial, bad, done, pstride);
    else if (mode == 1)
      hipLaunchKernelGGL((spmm_csr_kernel<T, S, V, 1>), dim3(nblk), dim3(kBlock), 0, st, A.n, A.nnz, A.rowptr,
                         A.colind, val, s, X, Y, B, partial, bad, done, pstride);
    else
      hipLaunchKernelGGL((spmm_csr_kernel<T, S, V, 2>), dim3(nblk), dim3(kBlock), 0, st, A.n, A.nnz, A.rowptr,
                         A.colind, val, s, X, Y, B, partial, bad, done, pstride);
    return hipGetLastError();
  });
  if (e == hipSuccess && ev_after) e = hipEventRecord(ev_after, st);
  if (e != hipSuccess || mode == 0) return e;
  return launch_reduce(s, pbase, sizeof(T) == 4, nblk, 1, red, done, nullptr, epi, st);
}

// Workgroups launch_spmm uses for a requested nblk (its kernels' residency cap).
template <typename T>
int spmm_grid(const CsrView& A, int s, int mode, int nblk) {
  int out = nblk;
  (void)dispatch_s<T>(s, [&](auto S_, auto V_) -> hipError_t {
    constexpr int S = decltype(S_)::value, V = decltype(V_)::value;
    if (A.ell_w > 0 && ell_prefetch<S, V>(A.ell_w))
      out = mode == 0 ? fit_grid<spmm_ell_kernel<T, S, V, 0, true>>(nblk)
                      : (mode == 1 ? fit_grid<spmm_ell_kernel<T, S, V, 1, true>>(nblk)
                                   : fit_grid<spmm_ell_kernel<T, S, V, 2, true>>(nblk));
    else if (A.ell_w > 0)
      out = mode == 0 ? fit_grid<spmm_ell_kernel<T, S, V, 0>>(nblk)
                      : (mode == 1 ? fit_grid<spmm_ell_kernel<T, S, V, 1>>(nblk)
                                   : fit_grid<spmm_ell_kernel<T, S, V, 2>>(nblk));
    else
      out = mode == 0 ? fit_grid<spmm_csr_kernel<T, S, V, 0>>(nblk)
                      : (mode == 1 ? fit_grid<spmm_csr_kernel<T, S, V, 1>>(nblk)
                                   : fit_grid<spmm_csr_kernel<T, S, V, 2>>(nblk));
    return hipSuccess;
  });
  return out;
}

// ------------------------------------------------------------------ Gram --
// Batch slice j < nx: X_j^T Y with X_j = X + j * n * s, into
// partial[(j * gridDim.x + blk) * s*s].  A workgroup computes JB consecutive
// slices (blockIdx.y = slice / JB), so Y is read once per JB blocks X_j.
template <typename T, int S, int VEC, int JB>
__global__ __launch_bounds__(kBlock) void gram_kernel(int64_t n, int s, const T* __restrict__ X, int nx,
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
  const int j0 = blockIdx.y * JB;
  const int jn = (nx - j0) < JB ? (nx - j0) : JB;
  int64_t r0, r1;
  int64_t rstep;
  stream_rows(n, RPB, r0, r1, rstep);
  T gacc[JB][VEC][S];
#pragma unroll
  for (int jj = 0; jj < JB; ++jj)
#pragma unroll
    for (int a = 0; a < VEC; ++a)
#pragma unroll
      for (int b = 0; b < S; ++b) gacc[jj][a][b] = T(0);
  for (int64_t base = r0; base < r1; base += rstep) {
    const int64_t row = base + wave * L::RPW + r;
    const bool rv = row < r1 && active;
    vec_t<T, VEC> y = rv ? load_vec<T, VEC>(Y + row * s + col0) : zero_vec<T, VEC>();
    vec_t<T, VEC> x[JB];
#pragma unroll
    for (int jj = 0; jj < JB; ++jj)
      x[jj] = (rv && jj < jn) ? load_vec<T, VEC>(X + (int64_t)(j0 + jj) * n * s + row * s + col0)
                              : zero_vec<T, VEC>();
#pragma unroll
    for (int jj = 0; jj < JB; ++jj) gram_row<T, S, VEC>(gacc[jj], x[jj], y, lane);
  }
#pragma unroll
  for (int jj = 0; jj < JB; ++jj)
    if (jj < jn) gram_store<T, S, VEC>(gacc[jj], s, partial, sh, j0 + jj);
}

// Slices computed per workgroup for width S (bounded by the registers of
// the Gram accumulators).
template <int S>
constexpr int gram_jb() {
  return S <= 8 ? 4 : (S <= 16 ? 2 : 1);
}

template <typename T>
hipError_t launch_gram(int64_t n, int s, const T* X, int nx, const T* Y, T* partial, int nblk, Red red,
                       const int32_t* done, hipStream_t st, const int32_t* fire) {
  if (nx <= 0) return hipSuccess;
  if (nx > kMaxBatch) return hipErrorInvalidValue;
  if constexpr (sizeof(T) == 8) {
    // widths 9..32 in FP64: matrix cores
    if (nx == 1 && mfma_width(s)) {
      hipError_t e = launch_gram_mfma(n, s, X, Y, partial, nblk, done, fire, st);
      if (e != hipSuccess) return e;
      return launch_reduce(s, partial, false, nblk, 1, red, done, fire, Epi{}, st);
    }
  }
  hipError_t e = dispatch_s<T>(s, [&](auto S_, auto V_) -> hipError_t {
    constexpr int S = decltype(S_)::value, V = decltype(V_)::value;
    if (nx == 1) {
      hipLaunchKernelGGL((gram_kernel<T, S, V, 1>), dim3(nblk, 1), dim3(kBlock), 0, st, n, s, X, nx, Y, partial,
                         done, fire);
    } else {
      // batched: about 2048 workgroups in all (each grid row re-reads Y, and
      // every workgroup adds nx partials to the reduction), a multiple of 8
      constexpr int JB = gram_jb<S>();
      const int gy = (nx + JB - 1) / JB;
      int nb = 2048 / gy / 8 * 8;
      if (nb < 64) nb = 64;
      if (nb < nblk) nblk = nb;
      hipLaunchKernelGGL((gram_kernel<T, S, V, JB>), dim3(nblk, gy), dim3(kBlock), 0, st, n, s, X, nx, Y, partial,
                         done, fire);
    }
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  return launch_reduce(s, partial, sizeof(T) == 4, nblk, nx, red, done, fire, Epi{}, st);
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

// load_coeff in two halves, so that the loads of several coefficient
// matrices are in flight together: the entries (clamped indexes, always a
// valid address) into registers, then (zero outside s x s) into LDS.
template <typename T, int S>
struct CoeffRegs {
  T v[(S * S + kBlock - 1) / kBlock];
};
template <typename T, int S>
__device__ __forceinline__ void coeff_load(CoeffRegs<T, S>& r, const T* src, int s) {
#pragma unroll
  for (int u = 0; u < (S * S + kBlock - 1) / kBlock; ++u) {
    const int t = min((int)threadIdx.x + u * kBlock, S * S - 1), a = t / S, b = t % S;
    r.v[u] = src[min(a, s - 1) * s + min(b, s - 1)];
  }
}
template <typename T, int S>
__device__ __forceinline__ void coeff_store(T* dst, const CoeffRegs<T, S>& r, int s) {
#pragma unroll
  for (int u = 0; u < (S * S + kBlock - 1) / kBlock; ++u) {
    const int t = (int)threadIdx.x + u * kBlock, a = t / S, b = t % S;
    if (t < S * S) dst[t] = (a < s && b < s) ? r.v[u] : T(0);
  }
}

// R~ = R - Q lambda (in place in R); Gram partials of R~^T R~, and with
// PC also of R~^T M^-1 R~ (M^-1 = diag(minv)), stored side by side.
template <typename T, int S, int VEC, bool PC>
__global__ __launch_bounds__(kBlock) void cg_update_kernel(int64_t n, int s, T* __restrict__ R,
                                                            const T* __restrict__ Q, const CgCtl* ctl,
                                                            T* __restrict__ partial,
                                                            const double* __restrict__ minv, int64_t pstride) {
  using L = Layout<T, S, VEC>;
  constexpr int NW = kBlock / kWave;
  constexpr int RPB = NW * L::RPW;
  __shared__ T lam[S * S];
  __shared__ T sh[NW * S * S];
  // the gate and the coefficients are requested together
  const int32_t gate = ctl->gate;
  CoeffRegs<T, S> rl;
  coeff_load<T, S>(rl, ctl_mat<T>(ctl, 0), s);
  if (gate) return;
  coeff_store<T, S>(lam, rl, s);
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r = lane / L::LPR, c = lane % L::LPR;
  const int col0 = c * VEC;
  const bool active = col0 < s;
  int64_t r0, r1;
  int64_t rstep;
  stream_rows(n, RPB, r0, r1, rstep);
  T gacc[VEC][S];
  T gacc2[PC ? VEC : 1][PC ? S : 1];
#pragma unroll
  for (int a = 0; a < VEC; ++a)
#pragma unroll
    for (int b = 0; b < S; ++b) gacc[a][b] = T(0);
  if constexpr (PC) {
#pragma unroll
    for (int a = 0; a < VEC; ++a)
#pragma unroll
      for (int b = 0; b < S; ++b) gacc2[a][b] = T(0);
  }
  for (int64_t base = r0; base < r1; base += rstep) {
    const int64_t row = base + wave * L::RPW + r;
    const bool rv = row < r1 && active;
    vec_t<T, VEC> q = rv ? load_vec<T, VEC>(Q + row * s + col0) : zero_vec<T, VEC>();
    vec_t<T, VEC> rr = rv ? load_vec<T, VEC>(R + row * s + col0) : zero_vec<T, VEC>();
    T ql[VEC];
    row_times<T, S, VEC>(ql, q, lam, col0, lane);
    vec_t<T, VEC> out;
#pragma unroll
    for (int w = 0; w < VEC; ++w) out.v[w] = rr.v[w] - ql[w];
    if (rv) store_out<T, VEC>(R + row * s + col0, out);
    gram_row<T, S, VEC>(gacc, out, out, lane);
    if constexpr (PC) {
      const T m = rv ? (T)minv[row] : T(0);
      vec_t<T, VEC> z;
#pragma unroll
      for (int w = 0; w < VEC; ++w) z.v[w] = m * out.v[w];
      gram_row<T, S, VEC>(gacc2, z, out, lane);
    }
  }
  if constexpr (PC) {
    gram_store<T, S, VEC>(gacc, s, partial, sh, 0, 2 * (int64_t)s * s);
    gram_store<T, S, VEC>(gacc2, s, partial + (int64_t)s * s, sh, 0, 2 * (int64_t)s * s);
  } else {
    gram_store<T, S, VEC>(gacc, s, partial, sh, 0, pstride);
  }
}

template <typename T>
hipError_t launch_cg_update(int64_t n, int s, T* R, const T* Q, const CgCtl* ctl, T* partial, int nblk, Red red,
                            hipStream_t st, Epi epi, hipEvent_t ev_after, const double* minv) {
  if (minv && (sizeof(T) != 8 || epi.kind != EPI_CG_RHO_M)) return hipErrorInvalidValue;
  hipError_t e;
  if constexpr (sizeof(T) == 8) {
    if (wide_mfma(s))
      e = launch_cg_update_mfma(n, s, R, Q, ctl, partial, nblk, minv, 0, st);
    else
      e = hipErrorNotSupported;
  } else {
    e = hipErrorNotSupported;
  }
  if (e == hipErrorNotSupported)
    e = dispatch_s<T>(s, [&](auto S_, auto V_) -> hipError_t {
      constexpr int S = decltype(S_)::value, V0 = decltype(V_)::value;
      // FP32 at 16 columns: 2 values per lane (8 lanes per row) instead of
      // 4, which halves the per-lane Gram accumulators (73 instead of 150
      // VGPRs, 6 instead of 3 workgroups per CU; 36 against 42 us at 96^3);
      // the s x s partial it writes is the same
      constexpr int V = (sizeof(T) == 4 && S == 16 && V0 == 4) ? 2 : V0;
      if (minv)
        hipLaunchKernelGGL((cg_update_kernel<T, S, V, true>), dim3(nblk), dim3(kBlock), 0, st, n, s, R, Q, ctl,
                           partial, minv, (int64_t)0);
      else
        hipLaunchKernelGGL((cg_update_kernel<T, S, V, false>), dim3(nblk), dim3(kBlock), 0, st, n, s, R, Q, ctl,
                           partial, minv, (int64_t)0);
      return hipGetLastError();
    });
  if (e == hipSuccess && ev_after) e = hipEventRecord(ev_after, st);
  if (e != hipSuccess) return e;
  return launch_reduce(s, partial, sizeof(T) == 4, nblk, 1, red, &ctl->gate, nullptr, epi, st);
}

hipError_t launch_cg_update_partials(int64_t n, int s, double* R, const double* Q, const CgCtl* ctl, double* partial,
                                     int nblk, int64_t pstride, hipStream_t st) {
  if (wide_mfma(s)) return launch_cg_update_mfma(n, s, R, Q, ctl, partial, nblk, nullptr, pstride, st);
  return dispatch_s<double>(s, [&](auto S_, auto V_) -> hipError_t {
    constexpr int S = decltype(S_)::value, V = decltype(V_)::value;
    hipLaunchKernelGGL((cg_update_kernel<double, S, V, false>), dim3(nblk), dim3(kBlock), 0, st, n, s, R, Q, ctl,
                       partial, (const double*)nullptr, pstride);
    return hipGetLastError();
  });
}

// Gram partials X^T Y (no reduction) at stride pstride per workgroup.
template <int S, int VEC>
__global__ __launch_bounds__(kBlock) void gram_pair_kernel(int64_t n, int s, const double* __restrict__ X,
                                                            const double* __restrict__ Y,
                                                            double* __restrict__ partial, int64_t pstride,
                                                            const int32_t* skip_a, const int32_t* skip_b) {
  using T = double;
  using L = Layout<T, S, VEC>;
  constexpr int NW = kBlock / kWave;
  constexpr int RPB = NW * L::RPW;
  __shared__ T sh[NW * S * S];
  if ((skip_a && *skip_a) || (skip_b && *skip_b)) return;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r = lane / L::LPR, c = lane % L::LPR;
  const int col0 = c * VEC;
  const bool active = col0 < s;
  int64_t r0, r1, rstep;
  stream_rows(n, RPB, r0, r1, rstep);
  T gacc[VEC][S];
#pragma unroll
  for (int a = 0; a < VEC; ++a)
#pragma unroll
    for (int b = 0; b < S; ++b) gacc[a][b] = T(0);
  for (int64_t base = r0; base < r1; base += rstep) {
    const int64_t row = base + wave * L::RPW + r;
    const bool rv = row < r1 && active;
    const vec_t<T, VEC> x = rv ? load_vec<T, VEC>(X + row * s + col0) : zero_vec<T, VEC>();
    const vec_t<T, VEC> y = rv ? load_vec<T, VEC>(Y + row * s + col0) : zero_vec<T, VEC>();
    gram_row<T, S, VEC>(gacc, x, y, lane);
  }
  gram_store<T, S, VEC>(gacc, s, partial, sh, 0, pstride);
}

hipError_t launch_gram_partials(int64_t n, int s, const double* X, const double* Y, double* partial, int nblk,
                                int64_t pstride, const int32_t* skip_a, const int32_t* skip_b, hipStream_t st) {
  return dispatch_s<double>(s, [&](auto S_, auto V_) -> hipError_t {
    constexpr int S = decltype(S_)::value, V = decltype(V_)::value;
    hipLaunchKernelGGL((gram_pair_kernel<S, V>), dim3(nblk), dim3(kBlock), 0, st, n, s, X, Y, partial, pstride,
                       skip_a, skip_b);
    return hipGetLastError();
  });
}

// Direction update of block CG with the X update deferred by one iteration:
// the term P_k (lambda sigma)_k of an iteration whose predecessor's term was
// already added is held back and added together with the next one, so X is
// read and written every other iteration.  Once the solve has ended every
// owed term is added.  Unless it has ended, P_{k+1} = R + P_k beta goes into
// Pn, which holds P_{k-1} on entry (each lane reads its P_{k-1} entries
// before it overwrites them).
template <typename T>
__device__ __forceinline__ const T* ctl_prev(const CgCtl* ctl);
template <>
__device__ __forceinline__ const double* ctl_prev<double>(const CgCtl* ctl) {
  return ctl->lamsig_prev;
}
template <>
__device__ __forceinline__ const float* ctl_prev<float>(const CgCtl* ctl) {
  return ctl->lamsig_prev_f;
}

template <typename T, int S, int VEC, bool PC>
__global__ __launch_bounds__(kBlock) void cg_pupdate_kernel(int64_t n, int s, T* __restrict__ X,
                                                             const T* __restrict__ P, T* __restrict__ Pn,
                                                             const T* __restrict__ R, const CgCtl* ctl,
                                                             const double* __restrict__ minv) {
  using L = Layout<T, S, VEC>;
  constexpr int NW = kBlock / kWave;
  constexpr int RPB = NW * L::RPW;
  __shared__ T ls[S * S], lp[S * S], bt[S * S];
  // the control words, then every coefficient matrix, requested before the
  // first wait for them
  const int32_t susp = ctl->suspended, dn = ctl->done, xp = ctl->x_pending, xd = ctl->xdef_in;
  if (susp) return;
  const bool done = dn != 0;
  const bool xk = xp != 0;   // this iteration's alpha step ran
  const bool xin = xd != 0;  // the previous P's term is owed
  if (!xk && !xin) return;
  const bool flush = done || xin;
  const bool addk = xk && flush;
  const bool pdir = xk && !done;
  CoeffRegs<T, S> rls, rlp, rbt;
  if (addk) coeff_load<T, S>(rls, ctl_mat<T>(ctl, 1), s);
  if (xin) coeff_load<T, S>(rlp, ctl_prev<T>(ctl), s);
  if (pdir) coeff_load<T, S>(rbt, ctl_mat<T>(ctl, 2), s);
  if (addk) coeff_store<T, S>(ls, rls, s);
  if (xin) coeff_store<T, S>(lp, rlp, s);
  if (pdir) coeff_store<T, S>(bt, rbt, s);
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r = lane / L::LPR, c = lane % L::LPR;
  const int col0 = c * VEC;
  const bool active = col0 < s;
  int64_t r0, r1;
  int64_t rstep;
  stream_rows(n, RPB, r0, r1, rstep);
  for (int64_t base = r0; base < r1; base += rstep) {
    const int64_t row = base + wave * L::RPW + r;
    const bool rv = row < r1 && active;
    const vec_t<T, VEC> p = rv ? load_vec<T, VEC>(P + row * s + col0) : zero_vec<T, VEC>();
    if (flush) {
      vec_t<T, VEC> x = rv ? load_vec<T, VEC>(X + row * s + col0) : zero_vec<T, VEC>();
      if (xin) {
        const vec_t<T, VEC> pp = rv ? load_vec<T, VEC>(Pn + row * s + col0) : zero_vec<T, VEC>();
        T dx[VEC];
        row_times<T, S, VEC>(dx, pp, lp, col0, lane);
#pragma unroll
        for (int w = 0; w < VEC; ++w) x.v[w] += dx[w];
      }
      if (addk) {
        T dx[VEC];
        row_times<T, S, VEC>(dx, p, ls, col0, lane);
#pragma unroll
        for (int w = 0; w < VEC; ++w) x.v[w] += dx[w];
      }
      if (rv) store_nt<T, VEC>(X + row * s + col0, x);
    }
    if (pdir) {
      vec_t<T, VEC> rr = rv ? load_vec<T, VEC>(R + row * s + col0) : zero_vec<T, VEC>();
      if constexpr (PC) {
        const T m = rv ? (T)minv[row] : T(0);
#pragma unroll
        for (int w = 0; w < VEC; ++w) rr.v[w] = m * rr.v[w];
      }
      T pb[VEC];
      row_times<T, S, VEC>(pb, p, bt, col0, lane);
#pragma unroll
      for (int w = 0; w < VEC; ++w) rr.v[w] += pb[w];
      if (rv) store_nt<T, VEC>(Pn + row * s + col0, rr);
    }
  }
}

template <typename T>
hipError_t launch_cg_pupdate(int64_t n, int s, T* X, const T* P, T* Pn, const T* R, const CgCtl* ctl,
                             hipStream_t st, const double* minv) {
  if (minv && sizeof(T) != 8) return hipErrorInvalidValue;
  int nblk = stream_grid_wide(n, s, sizeof(T));
  if constexpr (sizeof(T) == 8) {
    if (wide_mfma(s)) return launch_cg_pupdate_mfma(n, s, X, P, Pn, R, ctl, nblk, minv, st);
  }
  return dispatch_s<T>(s, [&](auto S_, auto V_) -> hipError_t {
    constexpr int S = decltype(S_)::value, V = decltype(V_)::value;
    if (minv)
      hipLaunchKernelGGL((cg_pupdate_kernel<T, S, V, true>), dim3(nblk), dim3(kBlock), 0, st, n, s, X, P, Pn, R,
                         ctl, minv);
    else
      hipLaunchKernelGGL((cg_pupdate_kernel<T, S, V, false>), dim3(nblk), dim3(kBlock), 0, st, n, s, X, P, Pn, R,
                         ctl, minv);
    return hipGetLastError();
  });
}

// ------------------------------------------------------------ Gropp BCG --
// Residual pass of Gropp's block CG with a diagonal preconditioner: R~ = R -
// Q lambda and Z = Z - V lambda with V = M^-1 Q formed row by row (the
// recurrence that replaces Z = M^-1 R~), both in place, with the Gram
// partials of R~^T R~ (stopping norms) and Z^T R~ (rho') side by side at
// stride 2 s^2, the layout the preconditioned rho reduction reads.
template <int S, int VEC>
__global__ __launch_bounds__(kBlock) void gropp_update_kernel(int64_t n, int s, double* __restrict__ R,
                                                               const double* __restrict__ Q, double* __restrict__ Z,
                                                               const CgCtl* ctl, double* __restrict__ partial,
                                                               const double* __restrict__ minv) {
  using T = double;
  using L = Layout<T, S, VEC>;
  constexpr int NW = kBlock / kWave;
  constexpr int RPB = NW * L::RPW;
  __shared__ T lam[S * S];
  __shared__ T sh[NW * S * S];
  const int32_t gate = ctl->gate;
  CoeffRegs<T, S> rl;
  coeff_load<T, S>(rl, ctl->lam, s);
  if (gate) return;
  coeff_store<T, S>(lam, rl, s);
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r = lane / L::LPR, c = lane % L::LPR;
  const int col0 = c * VEC;
  const bool active = col0 < s;
  int64_t r0, r1, rstep;
  stream_rows(n, RPB, r0, r1, rstep);
  T gacc[VEC][S], gacc2[VEC][S];
#pragma unroll
  for (int a = 0; a < VEC; ++a)
#pragma unroll
    for (int b = 0; b < S; ++b) gacc[a][b] = gacc2[a][b] = T(0);
  for (int64_t base = r0; base < r1; base += rstep) {
    const int64_t row = base + wave * L::RPW + r;
    const bool rv = row < r1 && active;
    const vec_t<T, VEC> q = rv ? load_vec<T, VEC>(Q + row * s + col0) : zero_vec<T, VEC>();
    const vec_t<T, VEC> rr = rv ? load_vec<T, VEC>(R + row * s + col0) : zero_vec<T, VEC>();
    vec_t<T, VEC> z = rv ? load_vec<T, VEC>(Z + row * s + col0) : zero_vec<T, VEC>();
    const T m = rv ? minv[row] : T(0);
    vec_t<T, VEC> v;
#pragma unroll
    for (int w = 0; w < VEC; ++w) v.v[w] = m * q.v[w];
    T ql[VEC], vl[VEC];
    row_times<T, S, VEC>(ql, q, lam, col0, lane);
    row_times<T, S, VEC>(vl, v, lam, col0, lane);
    vec_t<T, VEC> out;
#pragma unroll
    for (int w = 0; w < VEC; ++w) {
      out.v[w] = rr.v[w] - ql[w];
      z.v[w] = z.v[w] - vl[w];
    }
    if (rv) {
      store_vec<T, VEC>(R + row * s + col0, out);
      store_vec<T, VEC>(Z + row * s + col0, z);
    }
    gram_row<T, S, VEC>(gacc, out, out, lane);
    gram_row<T, S, VEC>(gacc2, z, out, lane);
  }
  gram_store<T, S, VEC>(gacc, s, partial, sh, 0, 2 * (int64_t)s * s);
  gram_store<T, S, VEC>(gacc2, s, partial + (int64_t)s * s, sh, 0, 2 * (int64_t)s * s);
}

hipError_t launch_gropp_update(int64_t n, int s, double* R, const double* Q, double* Z, const CgCtl* ctl,
                               double* partial, int nblk, const double* minv, hipStream_t st) {
  return dispatch_s<double>(s, [&](auto S_, auto V_) -> hipError_t {
    constexpr int S = decltype(S_)::value, V = decltype(V_)::value;
    hipLaunchKernelGGL((gropp_update_kernel<S, V>), dim3(nblk), dim3(kBlock), 0, st, n, s, R, Q, Z, ctl, partial,
                       minv);
    return hipGetLastError();
  });
}

// Direction pass of Gropp's block CG: the X update of cg_pupdate_kernel
// (deferred by one iteration, same gating), P_{k+1} = Z + P_k beta into Pn
// (which holds P_{k-1}), Q = U + Q beta in place, and the Gram partials of
// P_{k+1}^T Q_{k+1} (the next alpha).
template <int S, int VEC>
__global__ __launch_bounds__(kBlock) void gropp_dir_kernel(int64_t n, int s, double* __restrict__ X,
                                                            const double* __restrict__ P, double* __restrict__ Pn,
                                                            const double* __restrict__ Z,
                                                            const double* __restrict__ U, double* __restrict__ Q,
                                                            const CgCtl* ctl, double* __restrict__ partial) {
  using T = double;
  using L = Layout<T, S, VEC>;
  constexpr int NW = kBlock / kWave;
  constexpr int RPB = NW * L::RPW;
  __shared__ T ls[S * S], lp[S * S], bt[S * S];
  __shared__ T sh[NW * S * S];
  const int32_t susp = ctl->suspended, dn = ctl->done, xp = ctl->x_pending, xd = ctl->xdef_in;
  if (susp) return;
  const bool done = dn != 0;
  const bool xk = xp != 0;
  const bool xin = xd != 0;
  if (!xk && !xin) return;
  const bool flush = done || xin;
  const bool addk = xk && flush;
  const bool pdir = xk && !done;
  CoeffRegs<T, S> rls, rlp, rbt;
  if (addk) coeff_load<T, S>(rls, ctl->lamsig, s);
  if (xin) coeff_load<T, S>(rlp, ctl->lamsig_prev, s);
  if (pdir) coeff_load<T, S>(rbt, ctl->beta, s);
  if (addk) coeff_store<T, S>(ls, rls, s);
  if (xin) coeff_store<T, S>(lp, rlp, s);
  if (pdir) coeff_store<T, S>(bt, rbt, s);
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r = lane / L::LPR, c = lane % L::LPR;
  const int col0 = c * VEC;
  const bool active = col0 < s;
  int64_t r0, r1, rstep;
  stream_rows(n, RPB, r0, r1, rstep);
  T gacc[VEC][S];
#pragma unroll
  for (int a = 0; a < VEC; ++a)
#pragma unroll
    for (int b = 0; b < S; ++b) gacc[a][b] = T(0);
  for (int64_t base = r0; base < r1; base += rstep) {
    const int64_t row = base + wave * L::RPW + r;
    const bool rv = row < r1 && active;
    const vec_t<T, VEC> p = rv ? load_vec<T, VEC>(P + row * s + col0) : zero_vec<T, VEC>();
    if (flush) {
      vec_t<T, VEC> x = rv ? load_vec<T, VEC>(X + row * s + col0) : zero_vec<T, VEC>();
      if (xin) {
        const vec_t<T, VEC> pp = rv ? load_vec<T, VEC>(Pn + row * s + col0) : zero_vec<T, VEC>();
        T dx[VEC];
        row_times<T, S, VEC>(dx, pp, lp, col0, lane);
#pragma unroll
        for (int w = 0; w < VEC; ++w) x.v[w] += dx[w];
      }
      if (addk) {
        T dx[VEC];
        row_times<T, S, VEC>(dx, p, ls, col0, lane);
#pragma unroll
        for (int w = 0; w < VEC; ++w) x.v[w] += dx[w];
      }
      if (rv) store_vec<T, VEC>(X + row * s + col0, x);
    }
    if (pdir) {
      vec_t<T, VEC> pn = rv ? load_vec<T, VEC>(Z + row * s + col0) : zero_vec<T, VEC>();
      vec_t<T, VEC> qn = rv ? load_vec<T, VEC>(U + row * s + col0) : zero_vec<T, VEC>();
      const vec_t<T, VEC> q = rv ? load_vec<T, VEC>(Q + row * s + col0) : zero_vec<T, VEC>();
      T pb[VEC], qb[VEC];
      row_times<T, S, VEC>(pb, p, bt, col0, lane);
      row_times<T, S, VEC>(qb, q, bt, col0, lane);
#pragma unroll
      for (int w = 0; w < VEC; ++w) {
        pn.v[w] += pb[w];
        qn.v[w] += qb[w];
      }
      if (rv) {
        store_vec<T, VEC>(Pn + row * s + col0, pn);
        store_vec<T, VEC>(Q + row * s + col0, qn);
      }
      gram_row<T, S, VEC>(gacc, pn, qn, lane);
    }
  }
  if (pdir) gram_store<T, S, VEC>(gacc, s, partial, sh);
}

hipError_t launch_gropp_dir(int64_t n, int s, double* X, const double* P, double* Pn, const double* Z,
                            const double* U, double* Q, const CgCtl* ctl, double* partial, int nblk, hipStream_t st) {
  return dispatch_s<double>(s, [&](auto S_, auto V_) -> hipError_t {
    constexpr int S = decltype(S_)::value, V = decltype(V_)::value;
    hipLaunchKernelGGL((gropp_dir_kernel<S, V>), dim3(nblk), dim3(kBlock), 0, st, n, s, X, P, Pn, Z, U, Q, ctl,
                       partial);
    return hipGetLastError();
  });
}

// ------------------------------------------------------ block BiCGStab --
// The three combinations that end a block BiCGStab iteration once omega and
// beta are known, in one pass over the rows in the streaming layout:
// X += P (lambda sigma) + S (omega sigma), R = S - omega U,
// P' = R + P beta - Q (omega beta).  Each entry runs the same fused
// multiply-adds, in the same order, as the one-thread-per-entry combinations.
template <int S_, int VEC>
__global__ __launch_bounds__(kBlock) void bc_tail_rs_kernel(int64_t n, int s, double* __restrict__ X,
                                                             const double* __restrict__ P,
                                                             const double* __restrict__ Sb,
                                                             const double* __restrict__ U,
                                                             const double* __restrict__ Q, double* __restrict__ R,
                                                             double* __restrict__ Pn, const double* lamsig,
                                                             const double* omsig, const double* negomI,
                                                             const double* pbeta, const double* qbeta,
                                                             const int32_t* done) {
  using T = double;
  using L = Layout<T, S_, VEC>;
  constexpr int S = S_;
  constexpr int NW = kBlock / kWave;
  constexpr int RPB = NW * L::RPW;
  __shared__ T cl[S * S], co[S * S], cu[S * S], cp[S * S], cq[S * S];
  // the gate and the five coefficient matrices are requested together
  const int32_t dn = done ? *done : 0;
  CoeffRegs<T, S> rl, ro, ru, rp, rq;
  coeff_load<T, S>(rl, lamsig, s);
  coeff_load<T, S>(ro, omsig, s);
  coeff_load<T, S>(ru, negomI, s);
  coeff_load<T, S>(rp, pbeta, s);
  coeff_load<T, S>(rq, qbeta, s);
  if (dn) return;
  coeff_store<T, S>(cl, rl, s);
  coeff_store<T, S>(co, ro, s);
  coeff_store<T, S>(cu, ru, s);
  coeff_store<T, S>(cp, rp, s);
  coeff_store<T, S>(cq, rq, s);
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r = lane / L::LPR, c = lane % L::LPR;
  const int col0 = c * VEC;
  const bool active = col0 < s;
  int64_t r0, r1, rstep;
  stream_rows(n, RPB, r0, r1, rstep);
  for (int64_t base = r0; base < r1; base += rstep) {
    const int64_t row = base + wave * L::RPW + r;
    const bool rv = row < r1 && active;
    const int64_t o = row * s + col0;
    const vec_t<T, VEC> p = rv ? load_vec<T, VEC>(P + o) : zero_vec<T, VEC>();
    const vec_t<T, VEC> sr = rv ? load_vec<T, VEC>(Sb + o) : zero_vec<T, VEC>();
    const vec_t<T, VEC> u = rv ? load_vec<T, VEC>(U + o) : zero_vec<T, VEC>();
    const vec_t<T, VEC> q = rv ? load_vec<T, VEC>(Q + o) : zero_vec<T, VEC>();
    vec_t<T, VEC> x = rv ? load_vec<T, VEC>(X + o) : zero_vec<T, VEC>();
    row_times_acc<T, S, VEC>(x.v, p, cl, col0);
    row_times_acc<T, S, VEC>(x.v, sr, co, col0);
    vec_t<T, VEC> rn = sr;
    row_times_acc<T, S, VEC>(rn.v, u, cu, col0);
    vec_t<T, VEC> pn = rn;
    row_times_acc<T, S, VEC>(pn.v, p, cp, col0);
    row_times_acc<T, S, VEC>(pn.v, q, cq, col0);
    if (rv) {
      store_nt<T, VEC>(X + o, x);
      store_out<T, VEC>(R + o, rn);
      store_nt<T, VEC>(Pn + o, pn);
    }
  }
}

hipError_t launch_bc_tail_rs(int64_t n, int s, double* X, const double* P, const double* S, const double* U,
                             const double* Q, double* R, double* Pn, const double* lamsig, const double* omsig,
                             const double* negomI, const double* pbeta, const double* qbeta, const int32_t* done,
                             hipStream_t st) {
  const int nblk = stream_grid_wide(n, s, sizeof(double));
  return dispatch_s<double>(s, [&](auto S_, auto V_) -> hipError_t {
    constexpr int SS = decltype(S_)::value, V = decltype(V_)::value;
    hipLaunchKernelGGL((bc_tail_rs_kernel<SS, V>), dim3(nblk), dim3(kBlock), 0, st, n, s, X, P, S, U, Q, R, Pn,
                       lamsig, omsig, negomI, pbeta, qbeta, done);
    return hipGetLastError();
  });
}

// ------------------------------------------------- one-reduction block CG --
// Fused pass of iteration k of the one-reduction block CG (MODE 0), the Gram
// of a re-normalised residual (MODE 1) and the final owed X term (MODE 2);
// see launch_cg1r_pass.  Every update is row-local, so P, Q, R and X are
// overwritten in place.  X takes the terms of two iterations every other
// iteration: the odd iteration k adds P_{k-1} (lambda sigma)_{k-1}, read
// anyway for the direction update, and P_k (lambda sigma)_k.
template <int S, int VEC, int MODE>
__global__ __launch_bounds__(kBlock) void cg1r_pass_kernel(int64_t n, int s, double* __restrict__ R,
                                                            const double* __restrict__ U, double* __restrict__ P,
                                                            double* __restrict__ Q, double* __restrict__ X,
                                                            const CgCtl* ctl, double* __restrict__ partial, int k) {
  using T = double;
  using L = Layout<T, S, VEC>;
  constexpr int NW = kBlock / kWave;
  constexpr int RPB = NW * L::RPW;
  __shared__ T lam[MODE == 0 ? S * S : 1], bt[MODE == 0 ? S * S : 1], cs[MODE != 1 ? S * S : 1],
      cp[MODE == 0 ? S * S : 1];
  __shared__ T sh[MODE != 2 ? NW * S * S : 1];
  // MODE 2 runs after the end; MODE 1 with k < 0 (the initial residual)
  // does not depend on a re-normalisation decision
  // the control words, then the coefficient matrices, requested before the
  // first wait for them
  const int32_t cdone = ctl->done, liter = ctl->lam_iter, cfire = ctl->fire;
  if (MODE != 2 && cdone) return;
  if (MODE == 0 && liter != k) return;
  if (MODE == 1 && k >= 0 && !cfire) return;
  const bool first = k == 0, xodd = (k & 1) != 0;
  const bool gram = MODE == 1 || (MODE == 0 && !cfire);
  if constexpr (MODE == 0) {
    CoeffRegs<T, S> rl, rb, rs, rp;
    coeff_load<T, S>(rl, ctl->lam, s);
    if (!first) coeff_load<T, S>(rb, ctl->beta, s);
    if (xodd) {
      coeff_load<T, S>(rs, ctl->lamsig, s);
      coeff_load<T, S>(rp, ctl->lamsig_prev, s);
    }
    coeff_store<T, S>(lam, rl, s);
    if (!first) coeff_store<T, S>(bt, rb, s);
    if (xodd) {
      coeff_store<T, S>(cs, rs, s);
      coeff_store<T, S>(cp, rp, s);
    }
  } else if constexpr (MODE == 2) {
    load_coeff<T, S>(cs, ctl->lamsig, s);
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r = lane / L::LPR, c = lane % L::LPR;
  const int col0 = c * VEC;
  const bool active = col0 < s;
  int64_t r0, r1;
  int64_t rstep;
  stream_rows(n, RPB, r0, r1, rstep);
  T gacc[MODE != 2 ? VEC : 1][MODE != 2 ? S : 1];
  if constexpr (MODE != 2) {
#pragma unroll
    for (int a = 0; a < VEC; ++a)
#pragma unroll
      for (int b = 0; b < S; ++b) gacc[a][b] = T(0);
  }
  for (int64_t base = r0; base < r1; base += rstep) {
    const int64_t row = base + wave * L::RPW + r;
    const bool rv = row < r1 && active;
    const int64_t o = row * s + col0;
    if constexpr (MODE == 2) {
      const vec_t<T, VEC> p = rv ? load_vec<T, VEC>(P + o) : zero_vec<T, VEC>();
      vec_t<T, VEC> x = rv ? load_vec<T, VEC>(X + o) : zero_vec<T, VEC>();
      T dx[VEC];
      row_times<T, S, VEC>(dx, p, cs, col0, lane);
#pragma unroll
      for (int w = 0; w < VEC; ++w) x.v[w] += dx[w];
      if (rv) store_nt<T, VEC>(X + o, x);
    } else if constexpr (MODE == 1) {
      const vec_t<T, VEC> rr = rv ? load_vec<T, VEC>(R + o) : zero_vec<T, VEC>();
      gram_row<T, S, VEC>(gacc, rr, rr, lane);
    } else {
      const vec_t<T, VEC> rr = rv ? load_vec<T, VEC>(R + o) : zero_vec<T, VEC>();
      const vec_t<T, VEC> u = rv ? load_vec<T, VEC>(U + o) : zero_vec<T, VEC>();
      vec_t<T, VEC> p = rr, q = u;
      vec_t<T, VEC> po = zero_vec<T, VEC>();
      if (!first) {
        po = rv ? load_vec<T, VEC>(P + o) : zero_vec<T, VEC>();
        const vec_t<T, VEC> qo = rv ? load_vec<T, VEC>(Q + o) : zero_vec<T, VEC>();
        T pb[VEC], qb[VEC];
        row_times<T, S, VEC>(pb, po, bt, col0, lane);
        row_times<T, S, VEC>(qb, qo, bt, col0, lane);
#pragma unroll
        for (int w = 0; w < VEC; ++w) {
          p.v[w] += pb[w];
          q.v[w] += qb[w];
        }
      }
      if (xodd) {
        vec_t<T, VEC> x = rv ? load_vec<T, VEC>(X + o) : zero_vec<T, VEC>();
        T d1[VEC], d2[VEC];
        row_times<T, S, VEC>(d1, po, cp, col0, lane);
        row_times<T, S, VEC>(d2, p, cs, col0, lane);
#pragma unroll
        for (int w = 0; w < VEC; ++w) x.v[w] += d1[w] + d2[w];
        if (rv) store_nt<T, VEC>(X + o, x);
      }
      T ql[VEC];
      row_times<T, S, VEC>(ql, q, lam, col0, lane);
      vec_t<T, VEC> rn;
#pragma unroll
      for (int w = 0; w < VEC; ++w) rn.v[w] = rr.v[w] - ql[w];
      if (rv) {
        store_out<T, VEC>(P + o, p);
        store_out<T, VEC>(Q + o, q);
        store_out<T, VEC>(R + o, rn);
      }
      if (gram) gram_row<T, S, VEC>(gacc, rn, rn, lane);
    }
  }
  if constexpr (MODE != 2)
    if (gram) gram_store<T, S, VEC>(gacc, s, partial, sh, 0, 2 * (int64_t)s * s);
}

hipError_t launch_cg1r_pass(int64_t n, int s, double* R, const double* U, double* P, double* Q, double* X,
                            const CgCtl* ctl, double* partial, int nblk, int k, int mode, hipStream_t st) {
  if (mode < 0 || mode > 2) return hipErrorInvalidValue;
  return dispatch_s<double>(s, [&](auto S_, auto V_) -> hipError_t {
    constexpr int S = decltype(S_)::value, V = decltype(V_)::value;
    if (mode == 0)
      hipLaunchKernelGGL((cg1r_pass_kernel<S, V, 0>), dim3(nblk), dim3(kBlock), 0, st, n, s, R, U, P, Q, X, ctl,
                         partial, k);
    else if (mode == 1)
      hipLaunchKernelGGL((cg1r_pass_kernel<S, V, 1>), dim3(nblk), dim3(kBlock), 0, st, n, s, R, U, P, Q, X, ctl,
                         partial, k);
    else
      hipLaunchKernelGGL((cg1r_pass_kernel<S, V, 2>), dim3(nblk), dim3(kBlock), 0, st, n, s, R, U, P, Q, X, ctl,
                         partial, k);
    return hipGetLastError();
  });
}

// Z = M^-1 R, M^-1 = diag(minv): one thread per element (the row of an
// element is its index divided by s).
template <typename T>
__global__ __launch_bounds__(kBlock) void row_scale_kernel(int64_t n, int s, const double* __restrict__ minv,
                                                            const T* __restrict__ R, T* __restrict__ Z,
                                                            const int32_t* done, const int32_t* fire) {
  if ((done && *done) || (fire && !*fire)) return;
  const int64_t total = n * s;
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < total; t += (int64_t)gridDim.x * kBlock)
    Z[t] = (T)minv[t / s] * R[t];
}

template <typename T>
hipError_t launch_row_scale(int64_t n, int s, const double* minv, const T* R, T* Z, const int32_t* done,
                            const int32_t* fire, hipStream_t st) {
  const int64_t total = n * s;
  if (total <= 0) return hipSuccess;
  int64_t blocks = (total + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL((row_scale_kernel<T>), dim3((unsigned)blocks), dim3(kBlock), 0, st, n, s, minv, R, Z, done,
                     fire);
  return hipGetLastError();
}

// ------------------------------------------------------ row products --
// X = X C in place (C s x s FP64, applied to each row), optionally with the
// Gram partials of the result (GRAM = 1).  Runs only if gf is null or *gf.
template <typename T, int S, int VEC, int GRAM>
__global__ __launch_bounds__(kBlock) void rowmul_kernel(int64_t n, int s, T* __restrict__ X,
                                                         const double* __restrict__ C, T* __restrict__ partial,
                                                         const int32_t* gf) {
  using L = Layout<T, S, VEC>;
  constexpr int NW = kBlock / kWave;
  constexpr int RPB = NW * L::RPW;
  __shared__ T cm[S * S];
  __shared__ T sh[GRAM ? NW * S * S : 1];
  if (gf && !*gf) return;
  for (int t = threadIdx.x; t < S * S; t += kBlock) {
    const int a = t / S, b = t % S;
    cm[t] = (a < s && b < s) ? (T)C[a * s + b] : T(0);
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r = lane / L::LPR, c = lane % L::LPR;
  const int col0 = c * VEC;
  const bool active = col0 < s;
  int64_t r0, r1;
  int64_t rstep;
  stream_rows(n, RPB, r0, r1, rstep);
  T gacc[GRAM ? VEC : 1][GRAM ? S : 1];
#pragma unroll
  for (int a = 0; a < (GRAM ? VEC : 1); ++a)
#pragma unroll
    for (int b = 0; b < (GRAM ? S : 1); ++b) gacc[a][b] = T(0);
  for (int64_t base = r0; base < r1; base += rstep) {
    const int64_t row = base + wave * L::RPW + r;
    const bool rv = row < r1 && active;
    vec_t<T, VEC> x = rv ? load_vec<T, VEC>(X + row * s + col0) : zero_vec<T, VEC>();
    T y[VEC];
    row_times<T, S, VEC>(y, x, cm, col0, lane);
    vec_t<T, VEC> out;
#pragma unroll
    for (int w = 0; w < VEC; ++w) out.v[w] = y[w];
    if (rv) store_out<T, VEC>(X + row * s + col0, out);
    if constexpr (GRAM) gram_row<T, S, VEC>(gacc, out, out, lane);
  }
  if constexpr (GRAM) gram_store<T, S, VEC>(gacc, s, partial, sh);
}

template <typename T>
hipError_t launch_rowmul(int64_t n, int s, T* X, const double* C, bool gram, T* partial, int nblk, Red red,
                         const int32_t* gf, hipStream_t st) {
  if constexpr (sizeof(T) == 8) {
    // widths 9..32 in FP64: matrix cores
    if (mfma_width(s)) {
      hipError_t e = launch_rowmul_mfma(n, s, X, C, gram, partial, nblk, gf, st);
      if (e != hipSuccess || !gram) return e;
      return launch_reduce(s, partial, false, nblk, 1, red, nullptr, gf, Epi{}, st);
    }
  }
  hipError_t e = dispatch_s<T>(s, [&](auto S_, auto V_) -> hipError_t {
    constexpr int S = decltype(S_)::value, V = decltype(V_)::value;
    if (gram)
      hipLaunchKernelGGL((rowmul_kernel<T, S, V, 1>), dim3(nblk), dim3(kBlock), 0, st, n, s, X, C, partial, gf);
    else
      hipLaunchKernelGGL((rowmul_kernel<T, S, V, 0>), dim3(nblk), dim3(kBlock), 0, st, n, s, X, C, partial, gf);
    return hipGetLastError();
  });
  if (e != hipSuccess || !gram) return e;
  return launch_reduce(s, partial, sizeof(T) == 4, nblk, 1, red, nullptr, gf, Epi{}, st);
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
  int64_t rstep;
  stream_rows(n, RPB, r0, r1, rstep);
  auto load_cs = [&](int j0, int jn) {
    for (int t = threadIdx.x; t < jn * S * S; t += kBlock) {
      int jj = t / (S * S), e = t % (S * S), a = e / S, b = e % S;
      cs[t] = (a < s && b < s) ? (T)(sign * C[(int64_t)(j0 + jj) * s * s + a * s + b]) : T(0);
    }
  };
  // all coefficient blocks fit (the usual case): load them once per workgroup
  const bool once = nx <= JC;
  if (once) {
    load_cs(0, nx);
    __syncthreads();
  }
  for (int64_t base = r0; base < r1; base += rstep) {
    const int64_t row = base + wave * L::RPW + r;
    const bool rv = row < r1 && active;
    T acc[VEC];
#pragma unroll
    for (int w = 0; w < VEC; ++w) acc[w] = T(0);
    for (int j0 = 0; j0 < nx; j0 += JC) {
      const int jn = (nx - j0) < JC ? (nx - j0) : JC;
      if (!once) {
        __syncthreads();
        load_cs(j0, jn);
        __syncthreads();
      }
      // rows of four blocks are loaded before their products, so one memory
      // round trip covers four terms; the terms are still added in order
      for (int jb = 0; jb < jn; jb += 4) {
        vec_t<T, VEC> x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const T* Xj = X + (int64_t)(j0 + jb + u) * n * s;
          x[u] = (rv && jb + u < jn) ? load_vec<T, VEC>(Xj + row * s + col0) : zero_vec<T, VEC>();
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (jb + u < jn) {
            T d[VEC];
            row_times<T, S, VEC>(d, x[u], cs + (jb + u) * S * S, col0, lane);
#pragma unroll
            for (int w = 0; w < VEC; ++w) acc[w] += d[w];
          }
        }
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
  int nblk = stream_grid_wide(n, s, sizeof(T));
  return dispatch_s<T>(s, [&](auto S_, auto V_) -> hipError_t {
    constexpr int S = decltype(S_)::value, V = decltype(V_)::value;
    hipLaunchKernelGGL((combine_kernel<T, S, V>), dim3(nblk), dim3(kBlock), 0, st, n, s, X, nx, C, sign, Y,
                       done);
    return hipGetLastError();
  });
}

// ------------------------------------------- pipelined Gram-Schmidt pass --
// One pass of the pipelined Gram-Schmidt orthogonalisation (Ch. 9): with the
// window w, the inner product of basis block g = u + w is taken with W as it
// stands right before the update with basis block u is subtracted.  The pass
// applies the updates u0 .. u0 + nu - 1 (their coefficients C_u, s x s, are
// known from earlier passes) row by row, and for the first ng of them
// accumulates V_{g0 + j}^T W^(u0 + j) (g0 = u0 + w) before update j, so W is
// read and written once for nu updates and ng inner products:
//   q = W_row;  for j < nu:  [j < ng] G_{g0+j} += V_{g0+j,row}^T q;  q -= V_{u0+j,row} C_{u0+j}
// Each update is subtracted on its own, as the listing's loop does.  Gram
// partials as gram_kernel's (slice j: partial[(j * gridDim.x + blk) s^2]).
template <int S, int VEC, int NU>
__global__ __launch_bounds__(kBlock) void pgs_pass_kernel(int64_t n, int s, const double* __restrict__ V,
                                                           double* __restrict__ W, int u0, int nu,
                                                           const double* __restrict__ C, int g0, int ng,
                                                           double* __restrict__ partial, const int32_t* done) {
  using L = Layout<double, S, VEC>;
  constexpr int NW = kBlock / kWave;
  constexpr int RPB = NW * L::RPW;
  __shared__ double cs[NU * S * S];
  __shared__ double sh[NW * S * S];
  if (done && *done) return;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r = lane / L::LPR, c = lane % L::LPR;
  const int col0 = c * VEC;
  const bool active = col0 < s;
  for (int t = threadIdx.x; t < nu * S * S; t += kBlock) {
    const int j = t / (S * S), e = t % (S * S), a = e / S, b = e % S;
    cs[t] = (a < s && b < s) ? C[(int64_t)(u0 + j) * s * s + a * s + b] : 0.0;
  }
  __syncthreads();
  int64_t r0, r1, rstep;
  stream_rows(n, RPB, r0, r1, rstep);
  double gacc[NU][VEC][S];
#pragma unroll
  for (int j = 0; j < NU; ++j)
#pragma unroll
    for (int a = 0; a < VEC; ++a)
#pragma unroll
      for (int b = 0; b < S; ++b) gacc[j][a][b] = 0.0;
  const int64_t blk = n * (int64_t)s;
  for (int64_t base = r0; base < r1; base += rstep) {
    const int64_t row = base + wave * L::RPW + r;
    const bool rv = row < r1 && active;
    vec_t<double, VEC> q = rv ? load_vec<double, VEC>(W + row * s + col0) : zero_vec<double, VEC>();
    vec_t<double, VEC> vu[NU], vg[NU];
#pragma unroll
    for (int j = 0; j < NU; ++j) {
      vu[j] = (rv && j < nu) ? load_vec<double, VEC>(V + (u0 + j) * blk + row * s + col0) : zero_vec<double, VEC>();
      vg[j] = (rv && j < ng) ? load_vec<double, VEC>(V + (g0 + j) * blk + row * s + col0) : zero_vec<double, VEC>();
    }
#pragma unroll
    for (int j = 0; j < NU; ++j) {
      if (j < ng) gram_row<double, S, VEC>(gacc[j], vg[j], q, lane);
      if (j < nu) {
        double d[VEC];
        row_times<double, S, VEC>(d, vu[j], cs + j * S * S, col0, lane);
#pragma unroll
        for (int w = 0; w < VEC; ++w) q.v[w] -= d[w];
      }
    }
    if (rv) store_vec<double, VEC>(W + row * s + col0, q);
  }
#pragma unroll
  for (int j = 0; j < NU; ++j)
    if (j < ng) gram_store<double, S, VEC>(gacc[j], s, partial, sh, j);
}

int pgs_max_updates(int s) {
  int nu = 1;
  (void)dispatch_s<double>(s, [&](auto S_, auto) -> hipError_t {
    nu = gram_jb<decltype(S_)::value>();
    return hipSuccess;
  });
  return nu;
}

hipError_t launch_pgs_pass(int64_t n, int s, const double* V, double* W, int u0, int nu, const double* C, int g0,
                           int ng, double* partial, int nblk, const int32_t* done, hipStream_t st) {
  if (nu <= 0 || ng > nu || nu > pgs_max_updates(s)) return hipErrorInvalidValue;
  return dispatch_s<double>(s, [&](auto S_, auto V_) -> hipError_t {
    constexpr int S = decltype(S_)::value, VV = decltype(V_)::value;
    constexpr int NU = gram_jb<S>();
    hipLaunchKernelGGL((pgs_pass_kernel<S, VV, NU>), dim3(nblk), dim3(kBlock), 0, st, n, s, V, W, u0, nu, C, g0, ng,
                       partial, done);
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
                                     const int32_t*, hipStream_t, Epi, hipEvent_t, int, int);                      \
  template int spmm_grid<T>(const CsrView&, int, int, int);                                                       \
  template hipError_t launch_gram<T>(int64_t, int, const T*, int, const T*, T*, int, Red, const int32_t*,          \
                                     hipStream_t, const int32_t*);                                                 \
  template hipError_t launch_cg_update<T>(int64_t, int, T*, const T*, const CgCtl*, T*, int, Red, hipStream_t,    \
                                          Epi, hipEvent_t, const double*);                                         \
  template hipError_t launch_cg_pupdate<T>(int64_t, int, T*, const T*, T*, const T*, const CgCtl*, hipStream_t,   \
                                           const double*);                                                         \
  template hipError_t launch_row_scale<T>(int64_t, int, const double*, const T*, T*, const int32_t*,              \
                                          const int32_t*, hipStream_t);                                            \
  template hipError_t launch_rowmul<T>(int64_t, int, T*, const double*, bool, T*, int, Red, const int32_t*,        \
                                       hipStream_t);                                                               \
  template hipError_t launch_block_combine<T>(int64_t, int, const T*, int, const double*, double, T*,               \
                                              const int32_t*, hipStream_t);                                        \
  template hipError_t launch_colscale<T>(int64_t, int, const T*, T*, const double*, int, const int32_t*,           \
                                         const int32_t*, hipStream_t);                                             \
  template hipError_t launch_sddmm<T>(const CsrView&, int, double, const T*, const T*, T*, int32_t*, hipStream_t);

BKRY_INST(double)
BKRY_INST(float)

}  // namespace bkry
