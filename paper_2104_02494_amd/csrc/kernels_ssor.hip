// kernels_ssor.hip -- multicolour SSOR preconditioner: the colouring (Jones-
// Plassmann rounds), the rows bucketed by colour, and the forward / backward
// colour sweeps on n x s row-major blocks.
//
// With the rows ordered by colour and A = L + D + U split in that order (L:
// entries whose column has a smaller colour),
//   M = (D + omega L) D^-1 (D + omega U) / (omega (2 - omega)),
// and Z = M^-1 R is a forward sweep y = (D + omega L)^-1 R (colours upwards)
// followed by a backward sweep Z = (D + omega U)^-1 (omega (2 - omega) D y)
// (colours downwards, in place over y).  Rows of one colour share no entry,
// so one launch per colour and sweep updates all of its rows independently.
#include "common.hpp"
#include "internal.hpp"

namespace bkry {

namespace {

// v beats u: higher priority, ties to the smaller row index.
__device__ __forceinline__ bool beats(uint32_t pv, int64_t v, uint32_t pu, int64_t u) {
  return pv > pu || (pv == pu && v < u);
}

}  // namespace

// One Jones-Plassmann round r: an uncoloured row that beats every neighbour
// still uncoloured at the start of the round takes the smallest colour held
// by no neighbour coloured in an earlier round.  state[v] = -1 (uncoloured)
// or (round << 16) | colour; a neighbour coloured in this same round counts
// as uncoloured (it beats v then, so v is not a local maximum anyway, and the
// decision does not depend on whether its store is visible yet).  The result
// equals the greedy colouring in priority order.  more[r] = 1 if a row is
// still uncoloured after the round.
// A column index outside [0, n) sets *bad and is ignored.
// Row pointers are clamped to [0, nnz].
__global__ __launch_bounds__(kBlock) void jp_round_kernel(int64_t n, int64_t nnz, const int32_t* __restrict__ rowptr,
                                                           const int32_t* __restrict__ colind,
                                                           const uint32_t* __restrict__ prio, int32_t* state,
                                                           int round, int32_t* more, int32_t* bad) {
  bool left = false;
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock) {
    if (state[v] >= 0) continue;
    const int64_t k0 = min(max((int64_t)rowptr[v], (int64_t)0), nnz);
    const int64_t k1 = min(max((int64_t)rowptr[v + 1], (int64_t)0), nnz);
    const uint32_t pv = prio[v];
    bool top = true;
    for (int64_t k = k0; k < k1 && top; ++k) {
      const int32_t u = colind[k];
      if (u == v) continue;
      if ((uint32_t)u >= (uint64_t)n) {
        *bad = 1;
        continue;
      }
      const int32_t su = __hip_atomic_load(state + u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (su < 0 || (su >> 16) == round) top = !beats(prio[u], u, pv, v);
    }
    if (!top) {
      left = true;
      continue;
    }
    int c = -1;
    for (int base = 0; c < 0; base += 64) {
      uint64_t used = 0;
      for (int64_t k = k0; k < k1; ++k) {
        const int32_t u = colind[k];
        if (u == v || (uint32_t)u >= (uint64_t)n) continue;
        const int32_t su = __hip_atomic_load(state + u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (su < 0 || (su >> 16) >= round) continue;
        const int cu = su & 0xffff;
        if (cu >= base && cu < base + 64) used |= 1ull << (cu - base);
      }
      if (~used != 0ull) c = base + __builtin_ctzll(~used);
    }
    // more colours than the packing holds are reported by the check (colour
    // kMaxColors or above)
    if (c > 0xffff) c = 0xffff;
    __hip_atomic_store(state + v, (round << 16) | c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (__any(left ? 1 : 0) && (threadIdx.x & (kWave - 1)) == 0) more[round] = 1;
}

// colors[v] = colour of state[v]; ncolors (atomic max); colour counts.
__global__ __launch_bounds__(kBlock) void jp_final_kernel(int64_t n, const int32_t* __restrict__ state,
                                                           int32_t* __restrict__ colors, int32_t* ncolors) {
  int m = 0;
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock) {
    const int c = state[v] & 0xffff;
    colors[v] = c;
    m = max(m, c + 1);
  }
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) m = max(m, __shfl_xor(m, d));
  if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(ncolors, m);
}

static int grid_for(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b > 4096) b = 4096;
  return (int)(b < 1 ? 1 : b);
}

hipError_t launch_jp_round(const CsrView& A, const uint32_t* prio, int32_t* state, int round, int32_t* more,
                           int32_t* bad, hipStream_t st) {
  hipLaunchKernelGGL(jp_round_kernel, dim3(grid_for(A.n)), dim3(kBlock), 0, st, A.n, A.nnz, A.rowptr, A.colind,
                     prio, state, round, more, bad);
  return hipGetLastError();
}

hipError_t launch_jp_final(int64_t n, const int32_t* state, int32_t* colors, int32_t* ncolors, hipStream_t st) {
  hipLaunchKernelGGL(jp_final_kernel, dim3(grid_for(n)), dim3(kBlock), 0, st, n, state, colors, ncolors);
  return hipGetLastError();
}

// Checks a colouring against A and prepares the sweeps: bad[0] = 1 for a
// colour outside [0, kMaxColors), bad[1] = 1 for two coupled rows of one
// colour, a column index outside [0, n) or row pointers that are not
// non-decreasing within [0, nnz] (the sweeps then never run), bad[2] = 1 for
// a row without a positive finite diagonal; d[i] = sum of the diagonal
// entries of row i; ncolors (atomic max) and count[c] (atomic adds).
__global__ __launch_bounds__(kBlock) void ssor_check_kernel(int64_t n, int64_t nnz, const int32_t* __restrict__ rowptr,
                                                             const int32_t* __restrict__ colind,
                                                             const double* __restrict__ val,
                                                             const int32_t* __restrict__ colors, double* d,
                                                             int32_t* ncolors, int32_t* count, int32_t* bad) {
  int m = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    const int32_t ci = colors[i];
    if (ci < 0 || ci >= kMaxColors) {
      bad[0] = 1;
      d[i] = 0.0;
      continue;
    }
    m = max(m, ci + 1);
    atomicAdd(count + ci, 1);
    const int64_t k0 = rowptr[i], k1 = rowptr[i + 1];
    if (k0 < 0 || k1 < k0 || k1 > nnz) {
      bad[1] = 1;
      d[i] = 0.0;
      continue;
    }
    double di = 0.0;
    for (int64_t k = k0; k < k1; ++k) {
      const int32_t j = colind[k];
      if ((uint32_t)j >= (uint64_t)n) {
        bad[1] = 1;
      } else if (j == i) {
        di += val[k];
      } else if (colors[j] == ci) {
        bad[1] = 1;
      }
    }
    if (!(di > 0.0) || !isfinite(di)) bad[2] = 1;
    d[i] = di;
  }
#pragma unroll
  for (int dd = 1; dd < kWave; dd <<= 1) m = max(m, __shfl_xor(m, dd));
  if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(ncolors, m);
}

// off[c] = sum of count[0..c) (one thread; ncolors is small).
__global__ void ssor_offsets_kernel(const int32_t* count, const int32_t* ncolors, int32_t* off, int32_t* cursor) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int acc = 0;
  const int nc = *ncolors;
  for (int c = 0; c < nc; ++c) {
    off[c] = acc;
    cursor[c] = 0;
    acc += count[c];
  }
  off[nc] = acc;
}

// perm[off[c] + slot] = i for the rows i of colour c (slot order is
// arbitrary: the rows of one colour are independent).
__global__ __launch_bounds__(kBlock) void ssor_bucket_kernel(int64_t n, const int32_t* __restrict__ colors,
                                                              const int32_t* __restrict__ off, int32_t* cursor,
                                                              int32_t* __restrict__ perm) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    const int32_t c = colors[i];
    perm[off[c] + atomicAdd(cursor + c, 1)] = (int32_t)i;
  }
}

hipError_t launch_ssor_check(const CsrView& A, const int32_t* colors, double* d, int32_t* ncolors, int32_t* count,
                             int32_t* bad, hipStream_t st) {
  hipLaunchKernelGGL(ssor_check_kernel, dim3(grid_for(A.n)), dim3(kBlock), 0, st, A.n, A.nnz, A.rowptr, A.colind,
                     static_cast<const double*>(A.val), colors, d, ncolors, count, bad);
  return hipGetLastError();
}

hipError_t launch_ssor_bucket(int64_t n, const int32_t* colors, const int32_t* count, const int32_t* ncolors,
                              int32_t* off, int32_t* cursor, int32_t* perm, hipStream_t st) {
  hipLaunchKernelGGL(ssor_offsets_kernel, dim3(1), dim3(64), 0, st, count, ncolors, off, cursor);
  hipLaunchKernelGGL(ssor_bucket_kernel, dim3(grid_for(n)), dim3(kBlock), 0, st, n, colors, off, cursor, perm);
  return hipGetLastError();
}

// One colour of a sweep, in the row-slot layout of the streaming kernels
// (a row held by LPR = S / VEC lanes, VEC contiguous columns each).  Forward
// (BACK = false): Z_i = (R_i - omega sum_{colour(j) < c} a_ij Z_j) / d_i.
// Backward: Z_i = (f d_i Z_i - omega sum_{colour(j) > c} a_ij Z_j) / d_i with
// f = omega (2 - omega).  The lanes of a row slot read its entries together
// (one load per row slot) and VEC consecutive values of each gathered row.
template <bool BACK, int S, int VEC>
__global__ __launch_bounds__(kBlock) void ssor_sweep_kernel(int s, const int32_t* __restrict__ rowptr,
                                                             const int32_t* __restrict__ colind,
                                                             const double* __restrict__ val,
                                                             const int32_t* __restrict__ colors,
                                                             const double* __restrict__ d,
                                                             const int32_t* __restrict__ perm,
                                                             const int32_t* __restrict__ off, int c, double omega,
                                                             const double* __restrict__ R, double* Z,
                                                             const int32_t* skip_a, const int32_t* skip_b,
                                                             const int32_t* need) {
  using L = Layout<double, S, VEC>;
  constexpr int NW = kBlock / kWave;
  constexpr int RPB = NW * L::RPW;
  if ((skip_a && *skip_a) || (skip_b && *skip_b) || (need && !*need)) return;
  const int64_t o0 = off[c], cnt = (int64_t)off[c + 1] - o0;
  const double f = omega * (2.0 - omega);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int col0 = (lane % L::LPR) * VEC;
  if (col0 >= s) return;
  for (int64_t base = (int64_t)blockIdx.x * RPB; base < cnt; base += (int64_t)gridDim.x * RPB) {
    const int64_t r = base + wave * L::RPW + lane / L::LPR;
    if (r >= cnt) continue;
    const int64_t i = perm[o0 + r];
    const double di = d[i];
    vec_t<double, VEC> acc;
    if (BACK) {
      acc = load_vec<double, VEC>(Z + i * s + col0);
#pragma unroll
      for (int w = 0; w < VEC; ++w) acc.v[w] = (f * di) * acc.v[w];
    } else {
      acc = load_vec<double, VEC>(R + i * s + col0);
    }
    const int32_t k1 = rowptr[i + 1];
    for (int32_t k = rowptr[i]; k < k1; ++k) {
      const int32_t j = colind[k];
      const int32_t cj = colors[j];
      if (BACK ? cj > c : cj < c) {
        const double a = -(omega * val[k]);
        const vec_t<double, VEC> zj = load_vec<double, VEC>(Z + (int64_t)j * s + col0);
#pragma unroll
        for (int w = 0; w < VEC; ++w) acc.v[w] = fma(a, zj.v[w], acc.v[w]);
      }
    }
#pragma unroll
    for (int w = 0; w < VEC; ++w) acc.v[w] = acc.v[w] / di;
    store_vec<double, VEC>(Z + i * s + col0, acc);
  }
}

hipError_t launch_ssor_apply(const SsorPlan& m, int s, const double* R, double* Z, const int32_t* skip_a,
                             const int32_t* skip_b, const int32_t* need, hipStream_t st) {
  const double* val = static_cast<const double*>(m.A.val);
  return dispatch_s<double>(s, [&](auto S_, auto V_) -> hipError_t {
    constexpr int S = decltype(S_)::value, V = decltype(V_)::value;
    using L = Layout<double, S, V>;
    constexpr int RPB = (kBlock / kWave) * L::RPW;
    int64_t b = (m.count_max + RPB - 1) / RPB;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    for (int pass = 0; pass < 2; ++pass)
      for (int k = 0; k < m.ncolors; ++k) {
        const int c = pass == 0 ? k : m.ncolors - 1 - k;
        if (pass == 0)
          hipLaunchKernelGGL((ssor_sweep_kernel<false, S, V>), dim3((unsigned)b), dim3(kBlock), 0, st, s,
                             m.A.rowptr, m.A.colind, val, m.colors, m.d, m.perm, m.off, c, m.omega, R, Z, skip_a,
                             skip_b, need);
        else
          hipLaunchKernelGGL((ssor_sweep_kernel<true, S, V>), dim3((unsigned)b), dim3(kBlock), 0, st, s,
                             m.A.rowptr, m.A.colind, val, m.colors, m.d, m.perm, m.off, c, m.omega, R, Z, skip_a,
                             skip_b, need);
      }
    return hipGetLastError();
  });
}

}  // namespace bkry
