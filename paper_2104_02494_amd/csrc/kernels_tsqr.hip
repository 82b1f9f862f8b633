// kernels_tsqr.hip -- normaliser Norm_S(X) = (Q, N) (Definition "normalizer",
// Ch. 3) by tall-skinny Householder QR (Section "The TSQR Algorithm", Ch. 7).
//
// The paper's TSQR splits the rows over processes, QR-factors each slab,
// gathers the R factors, QR-factors their stack and scatters the
// corrections back.  On one GPU the "processes" are workgroup row tiles and
// the gather is a tree of workgroups:
//
//   leaf   each workgroup factors a 256-row tile of one column group with
//          Householder reflections (thread t holds row t in registers); the
//          reflectors overwrite the tile in place, the g x g R goes to a
//          small FP64 buffer;
//   tree   stacks of 256/g R factors are factored the same way in FP64,
//          level by level, until one R remains;
//   root   diag(R) >= 0 by a sign flip, which also seeds the Q formation;
//   down   each tree tile applies its reflectors to [M; 0] (M its incoming
//          g x g factor), producing the factors of the level below;
//   apply  each leaf tile applies its reflectors to [M; 0] and writes its
//          rows of Q over the reflectors.
//
// Householder (not Cholesky-based) keeps the normaliser defined for rank-
// deficient blocks: a zero sub-column gives the identity reflector and Q
// stays orthonormal, gaining artificial directions.  Block-parallel runs one
// independent TSQR per column group (grid.y); the parallel and global
// normalisers need only column norms.
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"

namespace bkry {

constexpr int kTileRows = 256;  // rows per tile = threads per workgroup
constexpr int kTW = kTileRows / kWave;

// Row loads of the tile kernels in two halves: row_issue loads the G
// entries of row p (of the valid fallback row q when !ok; columns past g
// clamped), so that several rows' loads are in flight together; row_mask
// then zeroes what lies outside (consuming each value through an empty asm,
// so that the compiler cannot move a load under the bounds test and wait
// for it there).
template <typename U, int G>
__device__ __forceinline__ void row_issue(U (&v)[G], const U* p, const U* q, bool ok, int g) {
  const U* r = ok ? p : q;
#pragma unroll
  for (int c = 0; c < G; ++c) v[c] = r[c < g ? c : g - 1];
}
template <typename T, typename U, int G>
__device__ __forceinline__ void row_mask(T (&x)[G], U (&v)[G], bool ok, int g) {
#pragma unroll
  for (int c = 0; c < G; ++c) {
    U w = v[c];
    asm volatile("" : "+v"(w));
    x[c] = (ok && c < g) ? (T)w : T(0);
  }
}

template <int V>
using ICt = std::integral_constant<int, V>;

template <typename F>
hipError_t dispatch_g(int g, F&& f) {
  if (g <= 2) return f(ICt<2>{});
  if (g <= 4) return f(ICt<4>{});
  if (g <= 8) return f(ICt<8>{});
  if (g <= 16) return f(ICt<16>{});
  if (g <= 32) return f(ICt<32>{});
  return hipErrorInvalidValue;
}

__device__ __forceinline__ bool gate_closed(const int32_t* gd, const int32_t* gf) {
  return (gd && *gd) || (gf && !*gf);
}

// Block-wide sums of the entries lo <= c < G of v (every thread receives
// them), fixed order: butterfly inside each wavefront, then waves 0..3.
template <typename CT, int G>
__device__ __forceinline__ void tile_sum(CT (&v)[G], int lo, CT* lds) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
  for (int c = 0; c < G; ++c)
    if (c >= lo) v[c] = wave_sum(v[c]);
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < G; ++c)
      if (c >= lo) lds[wave * G + c] = v[c];
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < G; ++c)
    if (c >= lo) v[c] = ((lds[c] + lds[G + c]) + lds[2 * G + c]) + lds[3 * G + c];
  __syncthreads();
}

// Householder QR of the tile whose row t is x (Golub & Van Loan "house",
// R_jj = mu >= 0 for non-zero sub-columns).  On exit, x holds the reflector
// entries below the diagonal and R on and above it; beta[j] in LDS.  The
// column loop is unrolled by template recursion so that x stays in
// registers (static indices).
template <typename CT, int G, int J>
__device__ __forceinline__ void factor_step(CT (&x)[G], int g, CT* lds, CT* beta) {
  if constexpr (J < G) {
    if (J < g) {
      const int t = threadIdx.x;
      CT sv[2] = {(t > J) ? x[J] * x[J] : CT(0), (t == J) ? x[J] : CT(0)};
      tile_sum<CT, 2>(sv, 0, lds);
      const CT sig = sv[0], x1 = sv[1];
      CT b = CT(0), v1 = CT(1), mu = x1;
      if (sig != CT(0)) {
        mu = sqrt(x1 * x1 + sig);
        v1 = (x1 <= CT(0)) ? (x1 - mu) : (-sig / (x1 + mu));
        b = CT(2) * v1 * v1 / (sig + v1 * v1);
      }
      const CT vt = (t == J) ? CT(1) : ((t > J && sig != CT(0)) ? x[J] / v1 : CT(0));
      if (b != CT(0)) {
        CT w[G];
#pragma unroll
        for (int c = 0; c < G; ++c) w[c] = (c > J) ? vt * x[c] : CT(0);
        tile_sum<CT, G>(w, J + 1, lds);
#pragma unroll
        for (int c = 0; c < G; ++c)
          if (c > J) x[c] -= b * vt * w[c];
      }
      if (t > J) x[J] = vt;
      if (t == J) x[J] = mu;
      if (t == 0) beta[J] = b;
      factor_step<CT, G, J + 1>(x, g, lds, beta);
    }
  }
}

template <typename CT, int G>
__device__ void tile_factor(CT (&x)[G], int g, CT* lds, CT* beta) {
  factor_step<CT, G, 0>(x, g, lds, beta);
  __syncthreads();
}

// z <- H_0 H_1 ... H_{g-1} z for the tile's reflectors (row t of the
// reflector storage is v; row t of the operand is z), J = g-1 down to 0.
template <typename CT, int G, int J>
__device__ __forceinline__ void apply_step(CT (&z)[G], const CT (&v)[G], int g, const CT* beta, CT* lds) {
  if constexpr (J >= 0) {
    if (J < g) {
      const CT b = beta[J];
      if (b != CT(0)) {
        const int t = threadIdx.x;
        const CT vt = (t == J) ? CT(1) : (t > J ? v[J] : CT(0));
        CT w[G];
#pragma unroll
        for (int c = 0; c < G; ++c) w[c] = vt * z[c];
        tile_sum<CT, G>(w, 0, lds);
#pragma unroll
        for (int c = 0; c < G; ++c) z[c] -= b * vt * w[c];
      }
    }
    apply_step<CT, G, J - 1>(z, v, g, beta, lds);
  }
}

template <typename CT, int G>
__device__ void tile_apply(CT (&z)[G], const CT (&v)[G], int g, const CT* beta, CT* lds) {
  apply_step<CT, G, G - 1>(z, v, g, beta, lds);
}

// ------------------------------------------------------------------ leaf --
template <typename T, int G>
__global__ __launch_bounds__(kTileRows) void tsqr_leaf_kernel(int64_t n, int s, int g, T* __restrict__ X,
                                                               double* __restrict__ Rb, T* __restrict__ betas,
                                                               int ntile, const int32_t* gd, const int32_t* gf) {
  __shared__ T lds[kTW * G];
  __shared__ T beta[G];
  if (gate_closed(gd, gf)) return;
  const int t = threadIdx.x, tile = blockIdx.x, grp = blockIdx.y;
  const int64_t row = (int64_t)tile * kTileRows + t;
  T* base = X + row * s + grp * g;
  T x[G], xr[G];
  row_issue<T, G>(xr, base, X + grp * g, row < n, g);
  __builtin_amdgcn_sched_barrier(0);
  row_mask<T, T, G>(x, xr, row < n, g);
  tile_factor<T, G>(x, g, lds, beta);
  if (row < n) {
#pragma unroll
    for (int c = 0; c < G; ++c)
      if (c < g) base[c] = x[c];
  }
  const int64_t id = (int64_t)grp * ntile + tile;
  if (t < g) {
#pragma unroll
    for (int c = 0; c < G; ++c)
      if (c < g) Rb[id * g * g + t * g + c] = (c >= t) ? (double)x[c] : 0.0;
    betas[id * g + t] = beta[t];
  }
}

// ------------------------------------------------------------------ tree --
// Tiles of nr = 256/g stacked R factors (rows ridx*g .. ridx*g + g - 1).
template <int G>
__global__ __launch_bounds__(kTileRows) void tsqr_tree_kernel(int g, int cnt_in, double* __restrict__ Rin,
                                                               int cnt_out, double* __restrict__ Rout,
                                                               double* __restrict__ betas, const int32_t* gd,
                                                               const int32_t* gf) {
  __shared__ double lds[kTW * G];
  __shared__ double beta[G];
  if (gate_closed(gd, gf)) return;
  const int t = threadIdx.x, tile = blockIdx.x, grp = blockIdx.y;
  const int nr = kTileRows / g;
  const int ridx = tile * nr + t / g, rrow = t % g;
  const bool valid = t < nr * g && ridx < cnt_in;
  double* src = Rin + ((int64_t)grp * cnt_in + ridx) * g * g + rrow * g;
  double x[G], xr[G];
  row_issue<double, G>(xr, src, Rin, valid, g);
  __builtin_amdgcn_sched_barrier(0);
  row_mask<double, double, G>(x, xr, valid, g);
  tile_factor<double, G>(x, g, lds, beta);
  if (valid) {
#pragma unroll
    for (int c = 0; c < G; ++c)
      if (c < g) src[c] = x[c];
  }
  const int64_t id = (int64_t)grp * cnt_out + tile;
  if (t < g) {
#pragma unroll
    for (int c = 0; c < G; ++c)
      if (c < g) Rout[id * g * g + t * g + c] = (c >= t) ? x[c] : 0.0;
    betas[id * g + t] = beta[t];
  }
}

// ------------------------------------------------------------------ root --
// N block of the group = D R with D = sign(diag R) (sign 0 = +1); M = D.
__global__ void tsqr_root_kernel(int s, int g, const double* __restrict__ R, double* __restrict__ N,
                                 double* __restrict__ M, const int32_t* gd, const int32_t* gf) {
  if (gate_closed(gd, gf)) return;
  const int grp = blockIdx.x, o = grp * g;
  const double* Rg = R + (int64_t)grp * g * g;
  for (int t = threadIdx.x; t < g * s; t += blockDim.x) {
    const int i = t / s, c = t % s;
    const double d = Rg[i * g + i] < 0.0 ? -1.0 : 1.0;
    double v = 0.0;
    if (c >= o && c < o + g && c - o >= i) v = d * Rg[i * g + (c - o)];
    N[(o + i) * s + c] = v;
    if (c < g) M[(int64_t)grp * g * g + i * g + c] = (i == c) ? d : 0.0;
  }
}

// ------------------------------------------------------------------ down --
template <int G>
__global__ __launch_bounds__(kTileRows) void tsqr_down_kernel(int g, int cnt_in, const double* __restrict__ Rin,
                                                               const double* __restrict__ betas, int cnt_k,
                                                               const double* __restrict__ Mk,
                                                               double* __restrict__ Mbelow, const int32_t* gd,
                                                               const int32_t* gf) {
  __shared__ double lds[kTW * G];
  __shared__ double beta[G];
  if (gate_closed(gd, gf)) return;
  const int t = threadIdx.x, tile = blockIdx.x, grp = blockIdx.y;
  const int nr = kTileRows / g;
  const int ridx = tile * nr + t / g, rrow = t % g;
  const bool valid = t < nr * g && ridx < cnt_in;
  const int64_t id = (int64_t)grp * cnt_k + tile;
  const double* src = Rin + ((int64_t)grp * cnt_in + ridx) * g * g + rrow * g;
  double v[G], z[G], vr[G], zr[G];
  row_issue<double, G>(vr, src, Rin, valid, g);
  row_issue<double, G>(zr, Mk + id * g * g + t * g, Mk + id * g * g, t < g, g);
  if (t < g) beta[t] = betas[id * g + t];
  __builtin_amdgcn_sched_barrier(0);
  row_mask<double, double, G>(v, vr, valid, g);
  row_mask<double, double, G>(z, zr, t < g, g);
  __syncthreads();
  tile_apply<double, G>(z, v, g, beta, lds);
  if (valid) {
    double* dst = Mbelow + ((int64_t)grp * cnt_in + ridx) * g * g + rrow * g;
#pragma unroll
    for (int c = 0; c < G; ++c)
      if (c < g) dst[c] = z[c];
  }
}

// ----------------------------------------------------------------- apply --
template <typename T, int G>
__global__ __launch_bounds__(kTileRows) void tsqr_apply_kernel(int64_t n, int s, int g, T* __restrict__ X,
                                                                const T* __restrict__ betas,
                                                                const double* __restrict__ M0, int ntile,
                                                                const int32_t* gd, const int32_t* gf) {
  __shared__ T lds[kTW * G];
  __shared__ T beta[G];
  if (gate_closed(gd, gf)) return;
  const int t = threadIdx.x, tile = blockIdx.x, grp = blockIdx.y;
  const int64_t row = (int64_t)tile * kTileRows + t;
  const int64_t id = (int64_t)grp * ntile + tile;
  T* base = X + row * s + grp * g;
  T v[G], z[G], vr[G];
  double zr[G];
  row_issue<T, G>(vr, base, X + grp * g, row < n, g);
  row_issue<double, G>(zr, M0 + id * g * g + t * g, M0 + id * g * g, t < g, g);
  if (t < g) beta[t] = betas[id * g + t];
  __builtin_amdgcn_sched_barrier(0);
  row_mask<T, T, G>(v, vr, row < n, g);
  row_mask<T, double, G>(z, zr, t < g, g);
  __syncthreads();
  tile_apply<T, G>(z, v, g, beta, lds);
  if (row < n) {
#pragma unroll
    for (int c = 0; c < G; ++c)
      if (c < g) base[c] = z[c];
  }
}

// ---------------------------------------------------------------- driver --
namespace {

struct TsqrPlan {
  int g = 0, ngrp = 0, L = 0;
  int cnt[40];
  size_t off_betas_leaf = 0, off_R[40], off_bt[40], off_M[40], total = 0;
};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

template <typename T>
TsqrPlan make_plan(int64_t n, const Sub& sub) {
  TsqrPlan p;
  p.g = sub.g;
  p.ngrp = sub.s / sub.g;
  const int nr = kTileRows / p.g;
  p.cnt[0] = (int)((n + kTileRows - 1) / kTileRows);
  p.L = 0;
  while (p.cnt[p.L] > 1) {
    p.cnt[p.L + 1] = (p.cnt[p.L] + nr - 1) / nr;
    p.L++;
  }
  size_t off = 0;
  p.off_betas_leaf = off;
  off += align256(sizeof(T) * (size_t)p.ngrp * p.cnt[0] * p.g);
  for (int k = 0; k <= p.L; ++k) {
    p.off_R[k] = off;
    off += align256(sizeof(double) * (size_t)p.ngrp * p.cnt[k] * p.g * p.g);
    p.off_M[k] = off;
    off += align256(sizeof(double) * (size_t)p.ngrp * p.cnt[k] * p.g * p.g);
    p.off_bt[k] = off;
    off += align256(sizeof(double) * (size_t)p.ngrp * p.cnt[k] * p.g);
  }
  p.total = off;
  return p;
}

bool uses_norms(const Sub& sub) { return sub.kind == PARALLEL || sub.kind == GLOBAL || sub.g == 1; }

template <typename T>
size_t norms_ws(int64_t n, const Sub& sub) {
  const int nblk = stream_grid(n, sub.s, sizeof(T));
  return align256(sizeof(T) * (size_t)nblk * sub.s * sub.s) + align256(sizeof(double) * sub.s * sub.s) +
         align256(sizeof(double) * sub.s) + align256(sizeof(double) * red_gpart_count(nblk, sub.s));
}

}  // namespace

// Workspace of the CholeskyQR2 path (placed before the Householder plan).
template <typename T>
size_t cholqr_ws(int64_t n, const Sub& sub) {
  const int s = sub.s;
  const int nblk = stream_grid(n, s, sizeof(T));
  return align256(sizeof(T) * (size_t)nblk * s * s) + align256(sizeof(double) * red_gpart_count(nblk, s)) +
         4 * align256(sizeof(double) * s * s) + align256(4 * sizeof(int32_t));
}

// Block-global: rho (g x g) and the column divisors ahead of the workspace of
// the block normaliser of the (n q) x g stacked view.
static size_t bg_head(const Sub& sub) { return align256(sizeof(double) * sub.g * sub.g) + align256(sizeof(double) * sub.s); }

size_t tsqr_workspace_bytes(int64_t n, Sub sub) {
  if (sub.kind == BGLOBAL) return bg_head(sub) + tsqr_workspace_bytes(n * (sub.s / sub.g), Sub{BLOCK, sub.g, sub.g});
  if (uses_norms(sub)) return norms_ws<double>(n, sub);
  size_t a = cholqr_ws<double>(n, sub) + make_plan<double>(n, sub).total;
  size_t b = cholqr_ws<float>(n, sub) + make_plan<float>(n, sub).total;
  return a > b ? a : b;
}

// Householder TSQR of X (in place: Q over X) with the normaliser into N.
template <typename T>
static hipError_t hh_tsqr(int64_t n, const Sub& sub, T* X, double* N, char* w, const int32_t* gd,
                          const int32_t* gf, hipStream_t st) {
  const int s = sub.s;
  const TsqrPlan p = make_plan<T>(n, sub);
  const int g = p.g;
  T* betas_leaf = reinterpret_cast<T*>(w + p.off_betas_leaf);
  auto R = [&](int k) { return reinterpret_cast<double*>(w + p.off_R[k]); };
  auto M = [&](int k) { return reinterpret_cast<double*>(w + p.off_M[k]); };
  auto BT = [&](int k) { return reinterpret_cast<double*>(w + p.off_bt[k]); };
  return dispatch_g(g, [&](auto G_) -> hipError_t {
    constexpr int G = decltype(G_)::value;
    hipLaunchKernelGGL((tsqr_leaf_kernel<T, G>), dim3(p.cnt[0], p.ngrp), dim3(kTileRows), 0, st, n, s, g, X, R(0),
                       betas_leaf, p.cnt[0], gd, gf);
    for (int k = 1; k <= p.L; ++k)
      hipLaunchKernelGGL((tsqr_tree_kernel<G>), dim3(p.cnt[k], p.ngrp), dim3(kTileRows), 0, st, g, p.cnt[k - 1],
                         R(k - 1), p.cnt[k], R(k), BT(k), gd, gf);
    hipLaunchKernelGGL(tsqr_root_kernel, dim3(p.ngrp), dim3(256), 0, st, s, g, R(p.L), N, M(p.L), gd, gf);
    for (int k = p.L; k >= 1; --k)
      hipLaunchKernelGGL((tsqr_down_kernel<G>), dim3(p.cnt[k], p.ngrp), dim3(kTileRows), 0, st, g, p.cnt[k - 1],
                         R(k - 1), BT(k), p.cnt[k], M(k), M(k - 1), gd, gf);
    hipLaunchKernelGGL((tsqr_apply_kernel<T, G>), dim3(p.cnt[0], p.ngrp), dim3(kTileRows), 0, st, n, s, g, X,
                       betas_leaf, M(0), p.cnt[0], gd, gf);
    return hipGetLastError();
  });
}

// Block / hybrid normaliser (FP64 blocks).  For a well-conditioned block the unique QR
// with positive diagonal is reached by CholeskyQR2: Y = X R1^-1 with R1 from
// the Cholesky of X^T X, then Q = Y R2^-1 with R2 from the Cholesky of
// Y^T Y, N = R2 R1 (five block passes, no per-column synchronisation).  When
// the first Cholesky fails or its pivots spread by more than a factor
// 1/ratio within a group (X near rank-deficient), or Y^T Y is not near I, the
// Householder TSQR runs instead, on X or on Y, and N = R_householder R1;
// that path keeps the normaliser defined for rank-deficient blocks.  All
// branches are decided on the device (plan flags), so no host round trip.
template <typename T>
hipError_t tsqr_run(int64_t n, Sub sub, T* X, double* N, void* ws, uint32_t* cnt, const int32_t* gd,
                    const int32_t* gf, hipStream_t st, int32_t* plan_ext, bool fallback) {
  char* w = static_cast<char*>(ws);
  const int s = sub.s;
  if (sub.kind == BGLOBAL) {
    // Row r of the n x s row-major block, cut into q rows of width g, is row r
    // of every group X_1, ..., X_q: the buffer read as (n q) x g is a row
    // permutation of the stacked [X_1; ...; X_q], whose QR (Q rho) has the
    // same rho and the rows of Q permuted alike.  Y = sqrt(q) Q.
    const int g = sub.g, q = s / g;
    double* rho = reinterpret_cast<double*>(w);
    double* d = reinterpret_cast<double*>(w + align256(sizeof(double) * g * g));
    hipError_t e = tsqr_run<T>(n * q, Sub{BLOCK, g, g}, X, rho, w + bg_head(sub), cnt, gd, gf, st, plan_ext, fallback);
    if (e == hipSuccess) e = launch_bg_expand(rho, sub, N, d, gd, gf, st);
    if (e == hipSuccess) e = launch_colscale<T>(n, s, X, X, d, 0, gd, gf, st);
    return e;
  }
  if (uses_norms(sub)) {
    const int nblk = stream_grid(n, s, sizeof(T));
    T* part = reinterpret_cast<T*>(w);
    w += align256(sizeof(T) * (size_t)nblk * s * s);
    double* G = reinterpret_cast<double*>(w);
    w += align256(sizeof(double) * s * s);
    double* d = reinterpret_cast<double*>(w);
    w += align256(sizeof(double) * s);
    double* gpart = reinterpret_cast<double*>(w);
    Sub ns = sub;
    if (ns.kind == HYBRID) ns.kind = PARALLEL;
    hipError_t e = launch_gram<T>(n, s, X, 1, X, part, nblk, Red{G, gpart, cnt}, gd, st, gf);
    if (e == hipSuccess) e = launch_norm_diag(G, ns, d, N, gd, gf, st);
    if (e == hipSuccess) e = launch_colscale<T>(n, s, X, X, d, ns.kind == GLOBAL, gd, gf, st);
    return e;
  }
  if constexpr (sizeof(T) == 4) {
    // FP32 blocks (the inner solve of iterative refinement): CholeskyQR in
    // FP32 loses orthogonality to kappa^2 u32 and slowed the inner solves
    // down; the Householder TSQR (FP64 R combine) is kept there.
    return hh_tsqr<T>(n, sub, X, N, w + cholqr_ws<T>(n, sub), gd, gf, st);
  }
  const int nblk = stream_grid(n, s, sizeof(T));
  T* part = reinterpret_cast<T*>(w);
  w += align256(sizeof(T) * (size_t)nblk * s * s);
  double* gpart = reinterpret_cast<double*>(w);
  w += align256(sizeof(double) * red_gpart_count(nblk, s));
  double* G = reinterpret_cast<double*>(w);
  w += align256(sizeof(double) * s * s);
  double* R1 = reinterpret_cast<double*>(w);
  w += align256(sizeof(double) * s * s);
  double* Rinv = reinterpret_cast<double*>(w);
  w += align256(sizeof(double) * s * s);
  double* Nh = reinterpret_cast<double*>(w);
  w += align256(sizeof(double) * s * s);
  int32_t* plan = plan_ext ? plan_ext : reinterpret_cast<int32_t*>(w);
  w += align256(4 * sizeof(int32_t));
  const double ratio = sizeof(T) == 8 ? 1e-6 : 3e-3;
  const Red red{G, gpart, cnt};
  hipError_t e = launch_gram<T>(n, s, X, 1, X, part, nblk, red, gd, st, gf);
  if (e == hipSuccess) e = launch_cholqr(1, G, sub, R1, Rinv, N, plan, ratio, gd, gf, st);
  if (e == hipSuccess) e = launch_rowmul<T>(n, s, X, Rinv, true, part, nblk, red, plan + 0, st);
  if (e == hipSuccess) e = launch_cholqr(2, G, sub, R1, Rinv, N, plan, ratio, nullptr, nullptr, st);
  if (e == hipSuccess) e = launch_rowmul<T>(n, s, X, Rinv, false, part, nblk, Red{}, plan + 1, st);
  if (!fallback) return e;
  if (e == hipSuccess) e = hh_tsqr<T>(n, sub, X, Nh, w, nullptr, plan + 2, st);
  if (e == hipSuccess) e = launch_cholqr_compose(Nh, R1, N, sub, plan, st);
  return e;
}

template hipError_t tsqr_run<double>(int64_t, Sub, double*, double*, void*, uint32_t*, const int32_t*,
                                     const int32_t*, hipStream_t, int32_t*, bool);
template hipError_t tsqr_run<float>(int64_t, Sub, float*, double*, void*, uint32_t*, const int32_t*,
                                    const int32_t*, hipStream_t, int32_t*, bool);

}  // namespace bkry
