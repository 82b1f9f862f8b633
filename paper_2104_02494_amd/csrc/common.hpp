// common.hpp -- device helpers shared by the block Krylov kernels (gfx950).
//
// Lane layout used by every n x s block kernel ("row-interleaved" blocks):
// a wavefront of 64 lanes is split into RPW row slots of LPR = S / VEC lanes;
// lane (r, c) owns columns [c*VEC, c*VEC + VEC) of one row and moves them with
// one VEC-wide load (16 bytes for FP64 VEC = 2 and FP32 VEC = 4), so the LPR
// lanes of a row read or write the row's S*sizeof(T) bytes contiguously.  The
// full row, when a lane needs it (Gram updates, block products), is gathered
// from the row's other lanes with wavefront shuffles.  S is a power of two
// <= 32; a runtime s <= S gives the active columns (VEC = 1 when s != S).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace bkry {

constexpr int kWave = 64;

template <typename T, int N>
struct alignas(sizeof(T) * N) vec_t {
  T v[N];
};

template <typename T, int N>
__device__ __forceinline__ vec_t<T, N> load_vec(const T* p) {
  return *reinterpret_cast<const vec_t<T, N>*>(p);
}

template <typename T, int N>
__device__ __forceinline__ void store_vec(T* p, const vec_t<T, N>& x) {
  *reinterpret_cast<vec_t<T, N>*>(p) = x;
}

template <typename T, int N>
__device__ __forceinline__ vec_t<T, N> zero_vec() {
  vec_t<T, N> z;
#pragma unroll
  for (int i = 0; i < N; ++i) z.v[i] = T(0);
  return z;
}

template <int V>
using IC = std::integral_constant<int, V>;

// Calls f(IC<S>, IC<VEC>) for the block width s.  Widths 1, 2 and 4 give a
// lane a whole row; 8, 16 and 32 move 16 bytes per lane; other widths run one
// element per lane in the next power of two.
template <typename T, typename F>
hipError_t dispatch_s(int s, F&& f) {
  constexpr int v16 = 16 / (int)sizeof(T);
  switch (s) {
    case 1: return f(IC<1>{}, IC<1>{});
    case 2: return f(IC<2>{}, IC<2>{});
    case 4: return f(IC<4>{}, IC<4>{});
    case 8: return f(IC<8>{}, IC<v16>{});
    case 16: return f(IC<16>{}, IC<v16>{});
    case 32: return f(IC<32>{}, IC<v16>{});
    default: break;
  }
  if (s == 3) return f(IC<4>{}, IC<1>{});
  if (s >= 5 && s <= 7) return f(IC<8>{}, IC<1>{});
  if (s >= 9 && s <= 15) return f(IC<16>{}, IC<1>{});
  if (s >= 17 && s <= 31) return f(IC<32>{}, IC<1>{});
  return hipErrorInvalidValue;
}

// Compile-time layout of a block kernel for element type T and width S.
template <typename T, int S_, int VEC_>
struct Layout {
  static constexpr int S = S_;
  static constexpr int VEC = VEC_;
  static constexpr int LPR = S / VEC;          // lanes per row
  static constexpr int RPW = kWave / LPR;      // rows per wavefront
  static_assert(S % VEC == 0 && LPR <= kWave, "bad layout");
};

// Sum over all 64 lanes; every lane receives the total.  Fixed butterfly
// order, so the result is the same on every call.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) v += __shfl_xor(v, d);
  return v;
}

// Sum over the lanes that share the low log2(LPR) lane bits (the row slots
// of one column chunk): after this, every lane holds the sum over all row
// slots of its chunk.
template <typename T, int LPR>
__device__ __forceinline__ T rowslot_sum(T v) {
#pragma unroll
  for (int d = LPR; d < kWave; d <<= 1) v += __shfl_xor(v, d);
  return v;
}

// Sum over the LPR lanes of one row (the column chunks of a row).
template <typename T, int LPR>
__device__ __forceinline__ T rowgroup_sum(T v) {
#pragma unroll
  for (int d = 1; d < LPR; d <<= 1) v += __shfl_xor(v, d);
  return v;
}

// f(integral_constant<int, I>) for I = 0 .. N-1, unrolled at compile time.
template <int I, int N, typename F>
__device__ __forceinline__ void static_for_impl(F& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for_impl<I + 1, N>(f);
  }
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl<0, N>(f);
}

// Entries of the padded (ELL) matrix copy that each lane of an LPR-lane row
// group loads per chunk; a chunk holds LPR * E consecutive entries of a row.
constexpr int ell_entries_per_lane(int LPR) { return LPR <= 4 ? 2 : 1; }

// Value held by lane K (0 <= K < LPR) of the caller's LPR-lane row group.
// LPR <= 4 uses a DPP quad permutation (no LDS traffic); wider groups use a
// cross-lane permute.  Every lane of the wavefront must execute it.
template <int LPR, int K>
__device__ __forceinline__ int group_bcast(int v) {
  static_assert(K >= 0 && K < LPR, "lane out of group");
  if constexpr (LPR == 1) {
    return v;
  } else if constexpr (LPR == 2) {
    return __builtin_amdgcn_update_dpp(0, v, K | (K << 2) | ((2 + K) << 4) | ((2 + K) << 6), 0xF, 0xF, false);
  } else if constexpr (LPR == 4) {
    return __builtin_amdgcn_update_dpp(0, v, K * 0x55, 0xF, 0xF, false);
  } else {
    return __shfl(v, (int)(threadIdx.x & (kWave - 1) & ~(LPR - 1)) + K);
  }
}
template <int LPR, int K>
__device__ __forceinline__ float group_bcast(float v) {
  return __int_as_float(group_bcast<LPR, K>(__float_as_int(v)));
}
template <int LPR, int K>
__device__ __forceinline__ double group_bcast(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = group_bcast<LPR, K>((int)(b & 0xffffffffLL));
  const int hi = group_bcast<LPR, K>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Contiguous row range of block `blk` out of `nblk`, rounded to `step` rows,
// with the block index remapped so that consecutive row ranges stay on one
// XCD (workgroups are dealt round-robin over the 8 XCDs; each XCD has its
// own L2, which then sees neighbouring rows of the gathered operand).
// The remap is a bijection of [0, nblk) only when nblk is a multiple of 8;
// otherwise blocks keep their own index.
__device__ __forceinline__ void block_rows(int64_t n, int blk, int nblk, int step, int64_t& r0, int64_t& r1) {
  int logical = (nblk % 8 == 0) ? (blk % 8) * (nblk / 8) + blk / 8 : blk;
  int64_t per = (n + nblk - 1) / nblk;
  per = (per + step - 1) / step * step;
  r0 = (int64_t)logical * per;
  r1 = r0 + per;
  if (r1 > n) r1 = n;
  if (r0 > n) r0 = n;
}

// Rows of a streaming kernel (no reuse between rows): workgroups take the
// tiles of step0 rows in turn (grid-stride), so the whole launch sweeps the
// block as one front; the workgroup visits rows r0, r0 + step, ... below r1.
// On MI355X this streams about 7 % faster than one contiguous range per
// workgroup (fewer concurrent DRAM streams).
__device__ __forceinline__ void stream_rows(int64_t n, int step0, int64_t& r0, int64_t& r1, int64_t& step) {
  r0 = (int64_t)blockIdx.x * step0;
  r1 = n;
  step = (int64_t)gridDim.x * step0;
}

// Row range of a workgroup that belongs to a gang of G workgroups on one XCD
// (workgroups blk = x, x + 8, x + 16, ... run on XCD x): the gang owns one
// contiguous range and its members take turns on consecutive tiles of
// `step0` rows, so the gang sweeps its range as one front.  The workgroup
// starts at r0 (its first tile) and advances by `step` = G * step0; r1 bounds
// the gang's range.  Gangs of one XCD own adjacent ranges.  When the launch
// width is not a multiple of 8 * G, this is block_rows with step = step0.
__device__ __forceinline__ void gang_rows(int64_t n, int blk, int nblk, int step0, int G, int64_t& r0, int64_t& r1,
                                          int64_t& step) {
  if (G <= 1 || nblk % (8 * G) != 0) {
    block_rows(n, blk, nblk, step0, r0, r1);
    step = step0;
    return;
  }
  const int per_xcd = nblk / 8, xcd = blk % 8, local = blk / 8;
  const int nstreams = nblk / G;
  const int stream = xcd * (per_xcd / G) + local / G, sub = local % G;
  int64_t per = (n + nstreams - 1) / nstreams;
  per = (per + step0 - 1) / step0 * step0;
  int64_t g0 = (int64_t)stream * per;
  r1 = g0 + per;
  if (r1 > n) r1 = n;
  r0 = g0 + (int64_t)sub * step0;
  if (r0 > r1) r0 = r1;
  step = (int64_t)G * step0;
}

}  // namespace bkry
