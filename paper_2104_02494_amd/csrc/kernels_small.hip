// kernels_small.hip -- the p x p coefficient algebra, on the device, FP64.
//
// One workgroup of one wavefront (64 threads) works on matrices in LDS
// (p <= 32); with a single wavefront the workgroup barriers are nearly free.
// Keeping this on the device lets a whole block CG iteration (or GMRes step)
// be enqueued without a host round trip; the host reads back only a few flags.
//
//   cg_init / cg_alpha / cg_rho / cg_reortho_fin   the coefficient steps of
//       the adaptive block CG (Algorithm "BCG Method with Adaptive Residual
//       Re-Orthonormalization", Ch. 4): alpha, lambda = alpha^-1 rho,
//       lambda sigma, the kappa_D test, the column-norm stopping test,
//       beta = rho^-1 gamma^T rho', sigma = gamma sigma;
//   norm_diag    normaliser of the parallel / global subalgebras;
//   gm_*         block GMRes: generalised Givens rotations of the block
//       Hessenberg column, the sigma update, the residual test and the block
//       back-substitution (Algorithm "Block GMRes Method", Ch. 5);
//   ir_check     stopping test and column scales of iterative refinement.
//
// Cholesky solves run on the projected (S-structured) matrices; since the
// entries outside the subalgebra's blocks are exact zeros, the factorisation
// of the whole p x p matrix equals one factorisation per S-block.
#include <float.h>
#include <math.h>

#include "common.hpp"
#include "internal.hpp"

namespace bkry {

constexpr int kSB = 64;         // threads of the small-algebra workgroups (one wavefront)
constexpr int kSS = kMaxS * kMaxS;

// Register tile (SM >= s) of the Cholesky solves for width s.
template <typename F>
static hipError_t dispatch_sm(int s, F&& f) {
  if (s <= 8) return f(std::integral_constant<int, 8>{});
  if (s <= 16) return f(std::integral_constant<int, 16>{});
  return f(std::integral_constant<int, 32>{});
}

__device__ __forceinline__ int tid() { return threadIdx.x; }

// Ordering point between the lanes of the workgroup's single wavefront for
// data exchanged through LDS only: the wavefront's LDS accesses are carried
// out in program order, so no workgroup barrier (and no wait for outstanding
// accesses) is needed, only a point the compiler does not move accesses
// across.  Not for data exchanged through global memory.
__device__ __forceinline__ void sm_wave_sync() { __builtin_amdgcn_wave_barrier(); }

// t / d and t % d for 0 <= t < 2048 and 1 <= d <= 32 by one multiply: with
// m = ceil(2^16 / d), e = m d - 2^16 <= d - 1, t m / 2^16 = t / d + t e / (d
// 2^16) and t e <= 2047 * 31 < 2^16, so the floor is t / d's (the loops over
// s x s entries would otherwise run two integer divisions, some 40
// instructions, per entry).
struct SmDiv {
  int d, m;
  __device__ explicit SmDiv(int d_) : d(d_), m((65536 + d_ - 1) / d_) {}
  __device__ int q(int t) const { return (t * m) >> 16; }
  __device__ int r(int t) const { return t - q(t) * d; }
};

// Value of v in the lane given by the DPP control CTRL (within rows of 16).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Reductions over the workgroup's single wavefront (every lane receives the
// same result, in a fixed order): inside each row of 16 lanes by DPP
// exchanges (neighbours, pairs, mirrored halves, mirrored rows; each step
// adds two equal partial sums, so all lanes of a row agree), then the four
// row results read from lanes 0, 16, 32, 48 and combined in row order.  All
// 64 lanes must execute it.
__device__ __forceinline__ double wsum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return ((readlane_f64(v, 0) + readlane_f64(v, 16)) + readlane_f64(v, 32)) + readlane_f64(v, 48);
}
__device__ __forceinline__ double wmax(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));
  v = fmax(v, dpp_f64<0x4E>(v));
  v = fmax(v, dpp_f64<0x141>(v));
  v = fmax(v, dpp_f64<0x140>(v));
  return fmax(fmax(readlane_f64(v, 0), readlane_f64(v, 16)), fmax(readlane_f64(v, 32), readlane_f64(v, 48)));
}
__device__ __forceinline__ bool wany(bool b) { return __any(b ? 1 : 0) != 0; }

// dst[0 .. count) = src[0 .. count) (LDS or global, not overlapping), in
// batches of U entries per lane whose loads (clamped indexes) are all issued
// before the batch's stores: from global memory a batch costs one round trip,
// where the plain loop waited for every entry.
template <int U>
__device__ __forceinline__ void sm_copy_batched(double* dst, const double* src, int count) {
  for (int base = 0; base < count; base += U * kSB) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = base + tid() + u * kSB;
      v[u] = src[t < count ? t : count - 1];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = base + tid() + u * kSB;
      if (t < count) dst[t] = v[u];
    }
  }
}
__device__ __forceinline__ void sm_copy(double* dst, const double* src, int count) {
  if (count <= kSB) {  // one entry per lane (s <= 8)
    if (tid() < count) dst[tid()] = src[tid()];
  } else if (count <= 4 * kSB) {
    sm_copy_batched<4>(dst, src, count);
  } else {
    sm_copy_batched<8>(dst, src, count);
  }
}

// dst = src (count <= N entries, typically global memory into LDS) with every
// lane's loads issued before its first store: one memory round trip instead
// of one per kSB entries (a copy loop waits for each load before its store).
template <int N, typename T>
__device__ __forceinline__ void sm_fetch(T* dst, const T* src, int count) {
  constexpr int U = (N + kSB - 1) / kSB;
  T v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int t = tid() + u * kSB;
    if (u * kSB < count) v[u] = src[t < count ? t : count - 1];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int t = tid() + u * kSB;
    if (t < count) dst[t] = v[u];
  }
}

// sm_fetch in two halves (registers in between), so that the loads of
// several blocks, and other loads, are in flight before the first wait.
template <int N, typename T>
struct SmRegs {
  T v[(N + kSB - 1) / kSB];
};
template <int N, typename T>
__device__ __forceinline__ void sm_load(SmRegs<N, T>& r, const T* src, int count) {
#pragma unroll
  for (int u = 0; u < (N + kSB - 1) / kSB; ++u) {
    const int t = tid() + u * kSB;
    if (u * kSB < count) r.v[u] = src[t < count ? t : count - 1];
  }
}
template <int N, typename T>
__device__ __forceinline__ void sm_store(T* dst, const SmRegs<N, T>& r, int count) {
#pragma unroll
  for (int u = 0; u < (N + kSB - 1) / kSB; ++u) {
    const int t = tid() + u * kSB;
    if (t < count) dst[t] = r.v[u];
  }
}

__device__ __forceinline__ void sm_eye(double* M, int s) {
  const SmDiv ds(s);
  for (int t = tid(); t < s * s; t += kSB) M[t] = (ds.q(t) == ds.r(t)) ? 1.0 : 0.0;
}

// Projection onto the subalgebra (zero outside the g x g diagonal blocks;
// global: tr/s * I; block-global: the mean of the q diagonal blocks on every
// diagonal block).
__device__ __forceinline__ void sm_project(double* M, const Sub& sub, double* scratch1) {
  const int s = sub.s;
  const SmDiv ds(s), dg(sub.g);
  __syncthreads();
  if (sub.kind == BGLOBAL) {
    // g <= s/2 <= 16: each lane owns at most 256/kSB entries of the g x g mean
    constexpr int kPer = (kMaxS / 2) * (kMaxS / 2) / kSB;
    const int g = sub.g, q = s / g;
    double v[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid() + u * kSB;
      double acc = 0.0;
      if (e < g * g) {
        const int a = dg.q(e), b = dg.r(e);
        for (int k = 0; k < q; ++k) acc += M[(k * g + a) * s + k * g + b];
      }
      v[u] = acc / (double)q;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid() + u * kSB;
      if (e < g * g) {
        const int a = dg.q(e), b = dg.r(e);
        for (int k = 0; k < q; ++k) M[(k * g + a) * s + k * g + b] = v[u];
      }
    }
    for (int t = tid(); t < s * s; t += kSB)
      if (dg.q(ds.q(t)) != dg.q(ds.r(t))) M[t] = 0.0;
  } else if (sub.kind == GLOBAL) {
    double d = 0.0;
    for (int a = tid(); a < s; a += kSB) d += M[a * s + a];
    const double v = wsum(d) / (double)s;
    __syncthreads();
    for (int t = tid(); t < s * s; t += kSB) M[t] = (ds.q(t) == ds.r(t)) ? v : 0.0;
  } else if (sub.g < s) {  // block with g = s: nothing lies outside the one block
    for (int t = tid(); t < s * s; t += kSB)
      if (dg.q(ds.q(t)) != dg.q(ds.r(t))) M[t] = 0.0;
  }
  __syncthreads();
}

// FP64 16 x 16 x 4 product on the matrix cores, D = A B + C: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] and holds D[4 v + l / 16][l % 16]
// in element v (the layout measured on gfx950).
typedef double mf_d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ mf_d4 mf_mma(double a, double b, mf_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// An empty asm statement that makes x opaque to the compiler: a value used
// only in one arm of a lane-dependent selection is then not sunk into a
// divergent branch of its own (every lane of a wavefront would run all arms
// in turn), and a guarded load is issued unconditionally.
__device__ __forceinline__ void mf_opaque(double& x) { asm volatile("" : "+v"(x)); }

// C = A B (transA: C = A^T B); C must not alias A or B.  Above 16 columns
// on the matrix cores: 2 x 2 tiles of 16 x 16, 8 steps of k each; entries
// past s are read (they stay inside the kMaxS^2 arrays) and replaced by zero.
// Up to 16 columns each entry of C is one lane's dot product in k order.
__device__ __forceinline__ void sm_mm(double* C, const double* A, const double* B, int s, bool transA) {
  __syncthreads();
  if (s > 16) {
    const int l = tid(), lr = l / 16, lc = l % 16;
    mf_d4 acc[2][2];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = mf_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const int k = 4 * kk + lr;
      double a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int i = 16 * t + lc;
        double av = transA ? A[k * s + i] : A[i * s + k], bv = B[k * s + i];
        mf_opaque(av);
        mf_opaque(bv);
        a[t] = (i < s && k < s) ? av : 0.0;
        b[t] = (i < s && k < s) ? bv : 0.0;
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = mf_mma(a[ti], b[tj], acc[ti][tj]);
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * ti + 4 * v + lr, j = 16 * tj + lc;
          if (i < s && j < s) C[i * s + j] = acc[ti][tj][v];
        }
    __syncthreads();
    return;
  }
  for (int t = tid(); t < s * s; t += kSB) {
    const int i = t / s, j = t % s;
    double acc = 0.0;
    for (int k = 0; k < s; ++k) acc += (transA ? A[k * s + i] : A[i * s + k]) * B[k * s + j];
    C[t] = acc;
  }
  __syncthreads();
}

// kappa_D(A) = kappa(D^-1/2 A D^-1/2) (Definition "Diagonally scaled condition
// number", Ch. 4) from the eigenvalues of the scaled matrix by the parallel
// (round-robin) cyclic Jacobi method.  Infinity if a diagonal entry or the
// smallest eigenvalue is not positive.
__device__ __forceinline__ double sm_kappaD(const double* A, int s, double* M, double* T, double* rc, double* rs, int* partner,
                            int* first, double* red) {
  const int sp = s + (s & 1);
  __syncthreads();
  if (tid() == 0) {
    int bad = 0;
    for (int i = 0; i < s; ++i) bad |= !(A[i * s + i] > 0.0);
    red[0] = bad;
  }
  __syncthreads();
  if (red[0] != 0.0) return INFINITY;
  for (int e = tid(); e < sp * sp; e += kSB) {
    const int i = e / sp, j = e % sp;
    M[e] = (i < s && j < s) ? A[i * s + j] / sqrt(A[i * s + i] * A[j * s + j]) : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    double offl = 0.0, totl = 0.0;
    for (int e = tid(); e < sp * sp; e += kSB) {
      const double v = M[e] * M[e];
      totl += v;
      if (e / sp != e % sp) offl += v;
    }
    const double off = wsum(offl), tot = wsum(totl);
    if (off == 0.0 || off <= 1e-30 * tot) break;
    for (int round = 0; round < sp - 1; ++round) {
      if (tid() < sp / 2) {
        const int pa = tid(), pb = sp - 1 - tid();
        int p = pa == 0 ? 0 : 1 + (pa - 1 + round) % (sp - 1);
        int q = pb == 0 ? 0 : 1 + (pb - 1 + round) % (sp - 1);
        if (p > q) {
          int tmp = p;
          p = q;
          q = tmp;
        }
        double c = 1.0, sn = 0.0;
        const double apq = M[p * sp + q];
        if (q < s && apq != 0.0) {
          const double tau = (M[q * sp + q] - M[p * sp + p]) / (2.0 * apq);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          sn = t * c;
        }
        rc[p] = c;
        rs[p] = sn;
        partner[p] = q;
        first[p] = 1;
        rc[q] = c;
        rs[q] = sn;
        partner[q] = p;
        first[q] = 0;
      }
      __syncthreads();
      for (int e = tid(); e < sp * sp; e += kSB) {  // T = M J
        const int i = e / sp, j = e % sp, jp = partner[j];
        const double c = rc[j], sn = rs[j];
        T[e] = first[j] ? c * M[i * sp + j] - sn * M[i * sp + jp] : sn * M[i * sp + jp] + c * M[i * sp + j];
      }
      __syncthreads();
      for (int e = tid(); e < sp * sp; e += kSB) {  // M = J^T T
        const int i = e / sp, j = e % sp, ip = partner[i];
        const double c = rc[i], sn = rs[i];
        M[e] = first[i] ? c * T[i * sp + j] - sn * T[ip * sp + j] : sn * T[ip * sp + j] + c * T[i * sp + j];
      }
      __syncthreads();
    }
  }
  __syncthreads();
  if (tid() == 0) {
    double lo = M[0], hi = M[0];
    for (int i = 1; i < s; ++i) {
      lo = fmin(lo, M[i * sp + i]);
      hi = fmax(hi, M[i * sp + i]);
    }
    red[2] = (lo > 0.0) ? hi / lo : INFINITY;
  }
  __syncthreads();
  return red[2];
}

// ---------------------------------------- register-resident Cholesky --
// Value of v in lane `lane` (uniform result; the lane need not be active).
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// In-register Cholesky of A (s x s, s <= SM, LDS): on return lane i holds
// row i of L in l (entries above the diagonal are left over from A) and
// rinv[k] = 1 / L_kk in every lane.  False (uniformly) on a non-positive or
// non-finite pivot.
// With sa, sh given, the matrix factored is sa A + sh I.
// EX: s == SM, known at compile time (every size guard folds away, which
// keeps the unrolled code of the widest factor small enough for the
// instruction cache).
template <int SM, bool EX>
__device__ __forceinline__ bool rf_factor(const double* A, int s, double (&l)[SM], double (&rinv)[SM],
                                          double sa = 1.0, double sh = 0.0) {
  if constexpr (EX) s = SM;
  const int t = tid();
#pragma unroll
  for (int j = 0; j < SM; ++j) l[j] = (t < s && j < s) ? fma(sa, A[t * s + j], t == j ? sh : 0.0) : 0.0;
#pragma unroll
  for (int k = 0; k < SM; ++k) {
    rinv[k] = 0.0;
    if (k < s) {
      const double d = readlane_d(l[k], k);
      if (!(d > 0.0) || !isfinite(d)) return false;
      // pivot reciprocal d^-1/2 first, L_kk = d d^-1/2 (no division)
      rinv[k] = rsqrt(d);
      const double lkk = d * rinv[k];
      if (t == k)
        l[k] = lkk;
      else if (t > k)
        l[k] = l[k] * rinv[k];
#pragma unroll
      for (int j = k + 1; j < SM; ++j) {
        if (j < s) {
          const double ljk = readlane_d(l[k], j);
          if (t >= j) l[j] = fma(-l[k], ljk, l[j]);
        }
      }
    }
  }
  return true;
}

// Column t of L^-1 (lane t) by forward substitution.
template <int SM, bool EX>
__device__ __forceinline__ void rf_linv_column(const double (&l)[SM], const double (&rinv)[SM], int s,
                                               double (&y)[SM]) {
  if constexpr (EX) s = SM;
  const int t = tid();
#pragma unroll
  for (int i = 0; i < SM; ++i) {
    if (i < s) {
      double acc = (i == t) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < i; ++k) acc = fma(-readlane_d(l[k], i), y[k], acc);
      y[i] = acc * rinv[i];
    } else {
      y[i] = 0.0;
    }
  }
}

// X = A^-1 B for SPD A (s x s, s <= SM, LDS) through A = L L^T, and, if Linv
// is not null, Linv = L^-1 (LDS; zero above the diagonal).  The factor lives
// in registers, lane i holding row i; each right-hand side column lives in
// the registers of its own lane; entries of L reach the other lanes by lane
// reads, so the whole factor-and-solve runs without LDS round trips.  The
// pivots' reciprocal square roots are formed once, so there is no division.
// Returns false (uniformly) on a non-positive or non-finite pivot.
template <int SM, bool EX>
__device__ __forceinline__ bool rf_cholesky_solve_x(const double* A, const double* B, double* X, double* Linv, int s) {
  if constexpr (EX) s = SM;
  __syncthreads();
  const int t = tid();
  double l[SM], rinv[SM];
  if (!rf_factor<SM, EX>(A, s, l, rinv)) return false;
  double x[SM];
#pragma unroll
  for (int i = 0; i < SM; ++i) x[i] = (t < s && i < s) ? B[i * s + t] : 0.0;
#pragma unroll
  for (int i = 0; i < SM; ++i) {  // L y = b
    if (i < s) {
      double acc = x[i];
#pragma unroll
      for (int k = 0; k < i; ++k) acc = fma(-readlane_d(l[k], i), x[k], acc);
      x[i] = acc * rinv[i];
    }
  }
#pragma unroll
  for (int i = SM - 1; i >= 0; --i) {  // L^T x = y
    if (i < s) {
      double acc = x[i];
#pragma unroll
      for (int k = i + 1; k < SM; ++k)
        if (k < s) acc = fma(-readlane_d(l[i], k), x[k], acc);
      x[i] = acc * rinv[i];
    }
  }
  if (t < s) {
#pragma unroll
    for (int i = 0; i < SM; ++i)
      if (i < s) X[i * s + t] = x[i];
  }
  if (Linv) {
    double y[SM];
    rf_linv_column<SM, EX>(l, rinv, s, y);
    if (t < s) {
#pragma unroll
      for (int i = 0; i < SM; ++i)
        if (i < s) Linv[i * s + t] = y[i];
    }
  }
  __syncthreads();
  return true;
}
template <int SM>
__device__ __forceinline__ bool lc_cholesky_solve(const double* A, const double* B, double* X, double* Linv, int s);
template <int SM>
__device__ __forceinline__ bool rf_cholesky_solve(const double* A, const double* B, double* X, double* Linv, int s) {
  if constexpr (SM >= 16) {
    return lc_cholesky_solve<SM>(A, B, X, Linv, s);
  } else {
    return s == SM ? rf_cholesky_solve_x<SM, true>(A, B, X, Linv, s)
                   : rf_cholesky_solve_x<SM, false>(A, B, X, Linv, s);
  }
}

// A = L L^T with L and L^-1 stored (LDS, zero above the diagonal).
template <int SM, bool EX>
__device__ __forceinline__ bool rf_cholesky_factor_x(const double* A, double* Lo, double* Linv, int s) {
  if constexpr (EX) s = SM;
  __syncthreads();
  const int t = tid();
  double l[SM], rinv[SM];
  if (!rf_factor<SM, EX>(A, s, l, rinv)) return false;
  if (t < s) {
#pragma unroll
    for (int j = 0; j < SM; ++j)
      if (j < s) Lo[t * s + j] = (j <= t) ? l[j] : 0.0;
  }
  double y[SM];
  rf_linv_column<SM, EX>(l, rinv, s, y);
  if (t < s) {
#pragma unroll
    for (int i = 0; i < SM; ++i)
      if (i < s) Linv[i * s + t] = y[i];
  }
  __syncthreads();
  return true;
}
template <int SM>
__device__ __forceinline__ bool lc_cholesky_factor(const double* A, double* Lo, double* Linv, int s);
template <int SM>
__device__ __forceinline__ bool rf_cholesky_factor(const double* A, double* Lo, double* Linv, int s) {
  if constexpr (SM >= 16) {
    return lc_cholesky_factor<SM>(A, Lo, Linv, s);
  } else {
    return s == SM ? rf_cholesky_factor_x<SM, true>(A, Lo, Linv, s)
                   : rf_cholesky_factor_x<SM, false>(A, Lo, Linv, s);
  }
}

// Whether sa A + sh I (A symmetric s x s, LDS) is positive definite, by
// attempting its Cholesky factorisation (uniform result).
template <int SM>
__device__ __forceinline__ bool lc_definite(const double* A, int s, double sa, double sh);
template <int SM>
__device__ __forceinline__ bool rf_definite(const double* A, int s, double sa, double sh) {
  if constexpr (SM >= 16) {
    return lc_definite<SM>(A, s, sa, sh);
  } else {
    double l[SM], rinv[SM];
    return s == SM ? rf_factor<SM, true>(A, s, l, rinv, sa, sh) : rf_factor<SM, false>(A, s, l, rinv, sa, sh);
  }
}

// ------------------------------------------------------ wide helpers --
// For widths 16 and 32 the register forms above unroll into tens of
// thousands of instructions (each entry of L reaches the other lanes by two
// lane reads, one step after the other), which the coefficient steps would
// stream through the instruction cache on every call.  The wide forms below
// spread every vector over all 64 lanes and exchange through LDS.
template <int SM>
struct Seg {
  static constexpr int NQ = kSB / SM;  // lanes per row
  static constexpr int RW = SM / NQ;   // entries per lane
  // segment stride in doubles: the NQ segments read by one instruction start
  // 16 bytes apart modulo the bank width, so their 16-byte reads do not collide
  static constexpr int ST = RW + 2;
  static constexpr int LEN = NQ * ST;
  __device__ static constexpr int at(int i) { return (i / RW) * ST + i % RW; }
};

template <int SM>
struct PowLds {
  __align__(16) double xs[Seg<SM>::LEN];  // the iterate, segmented
  double part[kSB];                       // partial row sums
};

template <int SM>
__device__ __forceinline__ PowLds<SM>* pow_lds() {
  __shared__ PowLds<SM> w;
  return &w;
}

__device__ __forceinline__ void st2(double* p, double a, double b) {
  *reinterpret_cast<double2*>(p) = make_double2(a, b);
}
__device__ __forceinline__ double2 ld2(const double* p) { return *reinterpret_cast<const double2*>(p); }

// ------------------------------ blocked Cholesky on the matrix cores (wide) --
// The same factorisation in blocks of 4 columns, so a width-32 matrix takes 8
// dependent steps instead of 32, each a handful of instructions plus a few
// v_mfma_f64_16x16x4f64 products.  The trailing matrix and the right-hand
// sides stay in accumulator layout for the whole factorisation (lane l holds
// entries (16 a + 4 v + l / 16, 16 b + l % 16) of tile (a, b), v = 0..3).
// Block step K (columns 4K .. 4K + 3):
//   the panel (those 4 columns) goes through LDS into row layout; every lane
//   factors the 4 x 4 diagonal block, D = L_KK L_KK^T, and forms W = L_KK^-1
//   (pivot reciprocals d^-1/2, L_kk = d * d^-1/2); lane (k = l / 16, row r)
//   forms its panel entry L[r][4K + k] = sum_m P[r][m] W[k][m], which is at
//   once the A operand (rows) and the B operand (columns) of the rank-4
//   update of the trailing matrix, A -= L_K L_K^T, one product per tile;
//   the right-hand sides' rows 4K .. 4K + 3 become Y_K = W B_K (forward
//   substitution) and the rows below lose L_K Y_K, one product per tile.
// The back substitution L^T X = Y runs the same blocks from the last up:
// X_K = W^T Y_K, then the rows above lose L_K^T X_K.  Rows and columns past
// s are padded with the identity (right-hand sides with zeros), so no step
// depends on s.  A single wavefront's LDS accesses are carried out in program
// order, so the exchanges need no barrier.

template <int SM>
struct MfLds {
  __align__(16) double Pn[SM * 4];       // panel rows (row-major, 4 columns)
  __align__(16) double Yb[2 * SM * 4];   // the block's right-hand-side rows, by column
  __align__(16) double Ws[SM / 4 * 16];  // W = L_KK^-1 of every diagonal block (row-major 4 x 4)
  double Ls[SM * (SM + 1)];              // L, rows padded to SM + 1
};

template <int SM>
__device__ __forceinline__ MfLds<SM>* mf_lds() {
  __shared__ MfLds<SM> w;
  return &w;
}

// d = L L^T for the 4 x 4 block d (row-major, lower part read): L and
// W = L^-1 (row-major, zero above the diagonal).  bad: a pivot that is not
// positive or not finite.
__device__ __forceinline__ void mf_diag4(const double (&d)[16], double (&L)[16], double (&W)[16], bool& bad) {
#pragma unroll
  for (int i = 0; i < 16; ++i) L[i] = W[i] = 0.0;
  double p = d[0];
  bad |= !(p > 0.0) || !isfinite(p);
  const double r0 = rsqrt(p);
  L[0] = p * r0;
  L[4] = d[4] * r0;
  L[8] = d[8] * r0;
  L[12] = d[12] * r0;
  p = fma(-L[4], L[4], d[5]);
  bad |= !(p > 0.0) || !isfinite(p);
  const double r1 = rsqrt(p);
  L[5] = p * r1;
  L[9] = fma(-L[8], L[4], d[9]) * r1;
  L[13] = fma(-L[12], L[4], d[13]) * r1;
  p = fma(-L[9], L[9], fma(-L[8], L[8], d[10]));
  bad |= !(p > 0.0) || !isfinite(p);
  const double r2 = rsqrt(p);
  L[10] = p * r2;
  L[14] = fma(-L[13], L[9], fma(-L[12], L[8], d[14])) * r2;
  p = fma(-L[14], L[14], fma(-L[13], L[13], fma(-L[12], L[12], d[15])));
  bad |= !(p > 0.0) || !isfinite(p);
  const double r3 = rsqrt(p);
  L[15] = p * r3;
  W[0] = r0;
  W[5] = r1;
  W[10] = r2;
  W[15] = r3;
  W[4] = -(L[4] * r0) * r1;
  W[9] = -(L[9] * r1) * r2;
  W[14] = -(L[14] * r2) * r3;
  W[8] = -fma(L[9], W[4], L[8] * r0) * r2;
  W[13] = -fma(L[14], W[9], L[13] * r1) * r3;
  W[12] = -fma(L[14], W[8], fma(L[13], W[4], L[12] * r0)) * r3;
}

// Element k (0..3, this lane's) of the four values v[0..3], by selects (the
// values are made opaque first, see mf_opaque).
__device__ __forceinline__ double mf_pick(double (&v)[4], int k) {
#pragma unroll
  for (int i = 0; i < 4; ++i) mf_opaque(v[i]);
  const double lo = (k & 1) ? v[1] : v[0], hi = (k & 1) ? v[3] : v[2];
  return (k & 2) ? hi : lo;
}

// sa A + sh I = L L^T (A: s x s in LDS); RHS: X = (sa A + sh I)^-1 B (BACK)
// or Y = L^-1 B (no BACK) into X; INV: Linv = L^-1; LO: Lo = L (zero above the
// diagonal).  All s x s, row-major, in LDS, in arrays of at least SM x SM
// entries (the loads are not guarded); X may alias B.  False (uniformly) on a
// pivot that is not positive or not finite.
template <int SM, bool RHS, bool INV, bool BACK, bool LO>
__device__ __forceinline__ bool mf_chol(const double* A, int s, double sa, double sh, const double* B, double* X,
                                        double* Linv, double* Lo) {
  constexpr int NT = SM / 16, NB = SM / 4;
  constexpr int NR = RHS ? NT : 0, NC = NR + (INV ? NT : 0), NCA = NC > 0 ? NC : 1;
  constexpr bool KEEP_L = BACK || LO;
  MfLds<SM>* w = mf_lds<SM>();
  const int l = tid(), lr = l / 16, lc = l % 16;
  mf_d4 at[NT][NT];
  mf_d4 bt[NT][NCA];
  __syncthreads();
  static_for<NT>([&](auto A_) {
    constexpr int a = decltype(A_)::value;
    static_for<NT>([&](auto B_) {
      constexpr int b = decltype(B_)::value;
      if constexpr (b <= a) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          // the load is unconditional (r s + c < SM^2 stays inside the
          // caller's s x s <= SM x SM array) so no load waits in a branch
          const int r = 16 * a + 4 * v + lr, c = 16 * b + lc;
          double av = A[r * s + c];
          mf_opaque(av);
          at[a][b][v] = (r < s && c < s) ? fma(sa, av, r == c ? sh : 0.0) : (r == c ? 1.0 : 0.0);
        }
      }
    });
    static_for<NCA>([&](auto C_) {
      constexpr int cc = decltype(C_)::value;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * a + 4 * v + lr;
        if constexpr (cc < NR) {
          const int c = 16 * cc + lc;
          double bv = B[r * s + c];
          mf_opaque(bv);
          bt[a][cc][v] = (r < s && c < s) ? bv : 0.0;
        } else {
          bt[a][cc][v] = (r == 16 * (cc - NR) + lc) ? 1.0 : 0.0;
        }
      }
    });
  });
  __syncthreads();
  bool bad = false;
  static_for<NB>([&](auto K_) {
    constexpr int K = decltype(K_)::value, ta = K / 4, kb = K % 4;
    // publish the panel and the block's right-hand-side rows
    if (lc / 4 == kb) {
      static_for<NT>([&](auto A_) {
        constexpr int a = decltype(A_)::value;
        if constexpr (a >= ta) {
#pragma unroll
          for (int v = 0; v < 4; ++v) w->Pn[(16 * a + 4 * v + lr) * 4 + lc % 4] = at[a][ta][v];
        }
      });
    }
    if constexpr (NC > 0) {
#pragma unroll
      for (int c = 0; c < NC; ++c) w->Yb[(16 * c + lc) * 4 + lr] = bt[ta][c][kb];
    }
    __builtin_amdgcn_wave_barrier();
    double d[16];
#pragma unroll
    for (int i = 0; i < 16; i += 2) {
      const double2 q = ld2(w->Pn + 16 * K + i);
      d[i] = q.x;
      d[i + 1] = q.y;
    }
    double pr[NT][4];
    static_for<NT>([&](auto A_) {
      constexpr int a = decltype(A_)::value;
      if constexpr (a >= ta) {
        const double2 q0 = ld2(w->Pn + (16 * a + lc) * 4), q1 = ld2(w->Pn + (16 * a + lc) * 4 + 2);
        pr[a][0] = q0.x;
        pr[a][1] = q0.y;
        pr[a][2] = q1.x;
        pr[a][3] = q1.y;
      }
    });
    double yb[NCA][4];
    if constexpr (NC > 0) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const double2 q0 = ld2(w->Yb + (16 * c + lc) * 4), q1 = ld2(w->Yb + (16 * c + lc) * 4 + 2);
        yb[c][0] = q0.x;
        yb[c][1] = q0.y;
        yb[c][2] = q1.x;
        yb[c][3] = q1.y;
      }
    }
    double L4[16], W4[16];
    mf_diag4(d, L4, W4, bad);
    // this lane's panel entries L[16 a + lc][4K + lr]: the rows of the block
    // take L_KK itself, the rows above it zero
    double lv[NT], op[NT];
    static_for<NT>([&](auto A_) {
      constexpr int a = decltype(A_)::value;
      if constexpr (a < ta) {
        lv[a] = 0.0;
        op[a] = 0.0;
      } else {
        double pl[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          double x = pr[a][0] * W4[4 * k];
#pragma unroll
          for (int m = 1; m <= k; ++m) x = fma(pr[a][m], W4[4 * k + m], x);
          pl[k] = x;
        }
        const int r = 16 * a + lc;
        const double trail = mf_pick(pl, lr);
        if constexpr (a == ta && LO) {
          // the block's own rows take L_KK as factored (only the stored L
          // reads them)
          const int rr = (r - 4 * K) & 3;  // the block row, on the block's rows
          double lrow[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            double col[4] = {L4[k], L4[4 + k], L4[8 + k], L4[12 + k]};
            lrow[k] = mf_pick(col, rr);
          }
          double x = mf_pick(lrow, lr);
          x = (r >= 4 * K + 4) ? trail : x;
          lv[a] = (r < 4 * K) ? 0.0 : x;
        } else {
          lv[a] = (a == ta && r < 4 * K) ? 0.0 : trail;
        }
        op[a] = (r < 4 * K + 4) ? 0.0 : trail;
      }
    });
    if constexpr (KEEP_L) {
      static_for<NT>([&](auto A_) {
        constexpr int a = decltype(A_)::value;
        if constexpr (a >= ta) w->Ls[(16 * a + lc) * (SM + 1) + 4 * K + lr] = lv[a];
      });
    }
    if constexpr (BACK) {
      if (l == 0) {
#pragma unroll
        for (int i = 0; i < 16; i += 2) st2(w->Ws + 16 * K + i, W4[i], W4[i + 1]);
      }
    }
    // rank-4 update of the trailing matrix
    static_for<NT>([&](auto A_) {
      constexpr int a = decltype(A_)::value;
      static_for<NT>([&](auto B_) {
        constexpr int b = decltype(B_)::value;
        if constexpr (a >= ta && b >= ta && b <= a) at[a][b] = mf_mma(-op[a], op[b], at[a][b]);
      });
    });
    // forward substitution: Y_K = W B_K, then the rows below
    if constexpr (NC > 0) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        double yk[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          double x = W4[4 * k] * yb[c][0];
#pragma unroll
          for (int m = 1; m <= k; ++m) x = fma(W4[4 * k + m], yb[c][m], x);
          yk[k] = x;
        }
        const double y = mf_pick(yk, lr);
        bt[ta][c][kb] = y;
        static_for<NT>([&](auto A_) {
          constexpr int a = decltype(A_)::value;
          if constexpr (a >= ta) bt[a][c] = mf_mma(-op[a], y, bt[a][c]);
        });
      }
    }
  });
  if (bad) {
    __syncthreads();
    return false;
  }
  if constexpr (INV) {
    static_for<NT>([&](auto A_) {
      constexpr int a = decltype(A_)::value;
#pragma unroll
      for (int c = 0; c < NT; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * a + 4 * v + lr, cl = 16 * c + lc;
          if (r < s && cl < s) Linv[r * s + cl] = bt[a][NR + c][v];
        }
    });
  }
  if constexpr (BACK) {
    static_for<NB>([&](auto J_) {
      constexpr int K = NB - 1 - decltype(J_)::value, ta = K / 4, kb = K % 4;
#pragma unroll
      for (int c = 0; c < NR; ++c) w->Yb[(16 * c + lc) * 4 + lr] = bt[ta][c][kb];
      __builtin_amdgcn_wave_barrier();
      double W4[16];
#pragma unroll
      for (int i = 0; i < 16; i += 2) {
        const double2 q = ld2(w->Ws + 16 * K + i);
        W4[i] = q.x;
        W4[i + 1] = q.y;
      }
      double op[NT];
      static_for<NT>([&](auto A_) {
        constexpr int a = decltype(A_)::value;
        if constexpr (a <= ta) {
          const int r = 16 * a + lc;
          const double v = w->Ls[(4 * K + lr) * (SM + 1) + r];
          op[a] = (r < 4 * K) ? v : 0.0;
        }
      });
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        const double2 q0 = ld2(w->Yb + (16 * c + lc) * 4), q1 = ld2(w->Yb + (16 * c + lc) * 4 + 2);
        const double y[4] = {q0.x, q0.y, q1.x, q1.y};
        double xk[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          double x = W4[12 + k] * y[3];
#pragma unroll
          for (int m = 2; m >= k; --m) x = fma(W4[4 * m + k], y[m], x);
          xk[k] = x;
        }
        const double x = mf_pick(xk, lr);
        bt[ta][c][kb] = x;
        static_for<NT>([&](auto A_) {
          constexpr int a = decltype(A_)::value;
          if constexpr (a <= ta) bt[a][c] = mf_mma(-op[a], x, bt[a][c]);
        });
      }
    });
  }
  if constexpr (RHS) {
    __syncthreads();
    static_for<NT>([&](auto A_) {
      constexpr int a = decltype(A_)::value;
#pragma unroll
      for (int c = 0; c < NR; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * a + 4 * v + lr, cl = 16 * c + lc;
          if (r < s && cl < s) X[r * s + cl] = bt[a][c][v];
        }
    });
  }
  if constexpr (LO) {
    __syncthreads();
    const SmDiv ds(s);
    for (int e = tid(); e < s * s; e += kSB) {
      const int i = ds.q(e), j = ds.r(e);
      Lo[e] = (j <= i) ? w->Ls[i * (SM + 1) + j] : 0.0;
    }
  }
  __syncthreads();
  return true;
}

// X = A^-1 B (and Linv = L^-1 if not null) for SPD A, all s x s in LDS.
template <int SM>
__device__ __forceinline__ bool lc_cholesky_solve(const double* A, const double* B, double* X, double* Linv, int s) {
  if (Linv) return mf_chol<SM, true, true, true, false>(A, s, 1.0, 0.0, B, X, Linv, nullptr);
  return mf_chol<SM, true, false, true, false>(A, s, 1.0, 0.0, B, X, nullptr, nullptr);
}

// A = L L^T with L (zero above the diagonal) and L^-1 stored, s x s in LDS.
template <int SM>
__device__ __forceinline__ bool lc_cholesky_factor(const double* A, double* Lo, double* Linv, int s) {
  return mf_chol<SM, false, true, false, true>(A, s, 1.0, 0.0, nullptr, nullptr, Linv, Lo);
}

template <int SM>
__device__ __forceinline__ bool lc_definite(const double* A, int s, double sa, double sh) {
  return mf_chol<SM, false, false, false, false>(A, s, sa, sh, nullptr, nullptr, nullptr, nullptr);
}

// Largest eigenvalue of the symmetric tridiagonal matrix with diagonal
// a[0 .. j) and off-diagonal b[0 .. j - 1) (LDS, read alike by all lanes),
// from below: bisection on Sturm counts (the negative pivots of the LDL^T
// factorisation of T - sigma I count the eigenvalues below sigma), with the
// 64 lanes testing 64 shifts of the bracket at once, so that each pass
// narrows it 65-fold; four passes from the Gershgorin interval.  Returns the
// lower end of the final bracket.
__device__ __forceinline__ double tridiag_lmax(const double* a, const double* b, int j) {
  double lo = a[0], hi = a[0];
  for (int i = 0; i < j; ++i) {
    const double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < j ? fabs(b[i]) : 0.0);
    lo = fmin(lo, a[i] - r);
    hi = fmax(hi, a[i] + r);
  }
  const double pivmin = 1e-290 + 1e-30 * (hi - lo);
  const int t = tid();
  for (int pass = 0; pass < 4; ++pass) {
    const double w = (hi - lo) / 65.0;
    const double sg = lo + w * (t + 1);
    int cnt = 0;
    double d = 1.0;
    for (int i = 0; i < j; ++i) {
      const double bb = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
      d = (a[i] - sg) - bb / d;
      if (fabs(d) < pivmin) d = -pivmin;
      cnt += d < 0.0 ? 1 : 0;
    }
    // the smallest shift with all j eigenvalues below it bounds lambda_max
    const unsigned long long m = __ballot(cnt == j);
    if (m == 0) {
      lo += 64.0 * w;
    } else {
      const int k = __builtin_ctzll(m);
      hi = lo + w * (k + 1);
      lo += w * k;
    }
  }
  return lo;
}

// Lanczos estimate of lambda_max of the symmetric s x s matrix A (LDS) from
// the normalised all-ones vector: the largest eigenvalue of the Lanczos
// tridiagonal matrix T_j (a Ritz value, so at most lambda_max up to
// rounding), taken every four steps from j = 8 until it changes by at most
// 1e-6 relative, the subspace is invariant, or j = s (T_s has the spectrum
// of A).  Far fewer matrix-vector products than the power iteration where
// the largest eigenvalues are close.  Uniform result.  The owner of row i
// is lane i; for SM >= 16 the matrix sits in registers by row segments (lane
// (q, i) holding row i, columns [q RW, q RW + RW)) and the vector in LDS,
// for SM <= 8 lane i holds row i and the vector moves by lane reads.  A
// single wavefront's LDS accesses are carried out in program order, so the
// exchanges need no barrier.
template <int SM>
__device__ __forceinline__ double lanczos_lmax(const double* A, int s) {
  __shared__ double ta[kMaxS], tb[kMaxS];
  const int t = tid();
  constexpr bool WIDE = SM >= 16;
  using G = Seg<WIDE ? SM : 16>;
  const int i = WIDE ? t % SM : t, q = WIDE ? t / SM : 0, c0 = q * G::RW;
  constexpr int NR = WIDE ? G::RW : SM;
  double m[NR];
#pragma unroll
  for (int u = 0; u < NR; ++u) {
    const int c = WIDE ? c0 + u : u;
    m[u] = (i < s && c < s) ? A[i * s + c] : 0.0;
  }
  PowLds<WIDE ? SM : 16>* w = nullptr;
  if constexpr (WIDE) w = pow_lds<SM>();
  __syncthreads();
  // y = (A x)_i on every lane of row i (x held by the owner lanes, zero elsewhere)
  auto matvec = [&](double x) {
    double y = 0.0;
    if constexpr (WIDE) {
      if (q == 0) w->xs[G::at(i)] = x;
      __builtin_amdgcn_wave_barrier();
      const double* seg = w->xs + q * G::ST;
      double p0 = 0.0, p1 = 0.0;
#pragma unroll
      for (int u = 0; u < NR; u += 2) {
        const double2 v = ld2(seg + u);
        p0 = fma(m[u], v.x, p0);
        p1 = fma(m[u + 1], v.y, p1);
      }
      w->part[t] = p0 + p1;
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int h = 0; h < G::NQ; ++h) y += w->part[h * SM + i];
      __builtin_amdgcn_wave_barrier();
    } else {
#pragma unroll
      for (int c = 0; c < NR; ++c) y = fma(m[c], readlane_d(x, c), y);
    }
    return y;
  };
  const bool own = WIDE ? (q == 0 && i < s) : (t < s);
  double v = own ? 1.0 / sqrt((double)s) : 0.0, vp = 0.0, bprev = 0.0, anorm = 0.0;
  double theta = 0.0, prev = 0.0;
  bool have = false;
  for (int j = 1; j <= s; ++j) {
    double y = matvec(v);
    y = own ? y - bprev * vp : 0.0;
    const double al = wsum(y * v);
    y = own ? y - al * v : 0.0;
    const double bt = sqrt(wsum(y * y));
    if (t == 0) {
      ta[j - 1] = al;
      tb[j - 1] = bt;
    }
    __builtin_amdgcn_wave_barrier();
    anorm = fmax(anorm, fabs(al) + bt + bprev);
    const bool last = j == s || !(bt > 1e-14 * anorm);
    if (last || (j >= 8 && j % 4 == 0)) {
      theta = tridiag_lmax(ta, tb, j);
      if (last || (have && fabs(theta - prev) <= 1e-6 * fabs(theta))) break;
      prev = theta;
      have = true;
    }
    vp = v;
    v = y / bt;
    bprev = bt;
  }
  __syncthreads();
  return theta;
}

// The re-orthonormalisation is decided per iteration (the L^-1 bound of the
// kappa_D test is needed) only for 0 < eta < inf, eta sqrt(eps) <= 1, g > 1.
// The control block's scalars that a coefficient step reads, loaded in one
// batch at its start (the control block is written during the step, so the
// compiler cannot keep its fields in scalar loads, and every separate read
// would cost a memory round trip before its use).
struct CgHead {
  int32_t s, kind, g, fire, iters, maxit, hist_cap, dynamic, xdef_pend, lam_iter;
  double tol, eta, sqrt_eps;
};
__device__ __forceinline__ CgHead cg_head(const CgCtl* c) {
  CgHead h;
  h.s = c->s;
  h.kind = c->kind;
  h.g = c->g;
  h.fire = c->fire;
  h.iters = c->iters;
  h.maxit = c->maxit;
  h.hist_cap = c->hist_cap;
  h.dynamic = c->dynamic;
  h.xdef_pend = c->xdef_pend;
  h.lam_iter = c->lam_iter;
  h.tol = c->tol;
  h.eta = c->eta;
  h.sqrt_eps = c->sqrt_eps;
  return h;
}

__device__ __forceinline__ bool reortho_dynamic(const CgHead& h) {
  return h.eta > 0.0 && !isinf(h.eta) && !(h.eta * h.sqrt_eps > 1.0) && h.g > 1;
}

// The kappa_D test of the iteration.  T holds L^-1 (alpha = L L^T) whenever
// reortho_dynamic(c); it is then overwritten.
// Re-orthonormalisation test: fire iff eta * kappa_D(alpha) * sqrt(eps) > 1
// (eta = 0 never, eta = infinity always); kappa_D equals 1 for the diagonal
// subalgebras.  T holds L^-1 for the Cholesky factor L of alpha.  The
// decision is the one kappa_D itself gives; it is reached, cheapest first, by
// guaranteed bounds on kappa_D, by definiteness tests of shifted copies of
// M = D^-1/2 alpha D^-1/2, and only when both leave it open by the Jacobi
// eigenvalues of M.
template <int SM>
__device__ __forceinline__ bool reortho_test(CgCtl* c, const CgHead& h, const double* alpha, double* M, double* T,
                                             double* rc, double* rs, int* partner, int* first, double* red) {
  if (!(h.eta > 0.0)) return false;
  if (isinf(h.eta)) return true;
  const int s = h.s;
  if (h.eta * h.sqrt_eps > 1.0) return true;  // kappa_D >= 1
  if (h.g <= 1) return false;                 // kappa_D = 1
  __syncthreads();
  // Guaranteed bounds on kappa_D = lambda_max(M) / lambda_min(M) for
  // M = D^-1/2 alpha D^-1/2 = L_M L_M^T, L_M^-1 = L^-1 D^1/2 (T holds L^-1):
  //   above: lambda_max <= min(|M|_F, |M|_inf) and
  //          1 / lambda_min = |L_M^-1|_2^2 <= min(|L_M^-1|_F^2, |L_M^-1|_1 |L_M^-1|_inf);
  //   below: lambda_max >= max(1, 1^T M 1 / s) (unit diagonal, Rayleigh
  //          quotient) and 1 / lambda_min >= max_i (M^-1)_ii.
  // The eigenvalues are computed only when the bounds leave the decision open.
  // (rc, rs: the square roots of alpha's diagonal and their reciprocals; the
  // slack of 1e-12 in the tests below covers the few roundings of each entry)
  const int t = tid();
  for (int i = t; i < s; i += kSB) {
    const double si = sqrt(alpha[i * s + i]);
    rc[i] = si;
    rs[i] = 1.0 / si;
  }
  __syncthreads();
  double fm = 0.0, li = 0.0;
  const SmDiv ds(s);
  for (int e = t; e < s * s; e += kSB) {
    const int i = ds.q(e), j = ds.r(e);
    const double m = alpha[e] * rs[i] * rs[j], u = T[e] * rc[j];
    fm += m * m;
    li += u * u;
  }
  double rowM = 0.0, sumM = 0.0, rowL = 0.0, colL = 0.0, dinv = 0.0;
  if (t < s) {
    const double st = rc[t], rt = rs[t];
#pragma unroll 4
    for (int j = 0; j < s; ++j) {
      const double mtj = alpha[t * s + j] * rt * rs[j];
      rowM += fabs(mtj);
      sumM += mtj;
      rowL += fabs(T[t * s + j] * rc[j]);  // row t of L_M^-1
      const double ljt = T[j * s + t] * st;  // column t of L_M^-1
      colL += fabs(ljt);
      dinv += ljt * ljt;
    }
  }
  const double nF = sqrt(wsum(fm)), nInf = wmax(rowM);
  const double ub = fmin(nF * wsum(li), fmin(nF, nInf) * wmax(colL) * wmax(rowL));
  const double es = h.eta * h.sqrt_eps;
  if (isfinite(ub) && ub * (1.0 + 1e-12) * es <= 1.0) return false;
  const double lmax_lo = fmax(1.0, wsum(sumM) / s), lmax_hi = fmin(nF, nInf);
  const double lb = lmax_lo * wmax(dinv);
  if (isfinite(lb) && lb * (1.0 - 1e-12) * es > 1.0) return true;
  // Definiteness tests, with tau = 1 / es, which bound lambda_min exactly:
  // M - l/tau I positive definite gives lambda_min > l/tau, not positive
  // definite lambda_min <= l/tau.  First against the bounds on lambda_max
  // above (M - lmax_hi/tau I positive definite: does not fire; M -
  // lmax_lo/tau I not positive definite: fires), which decides every
  // kappa_D farther from the threshold than their ratio; then with
  // theta <= lambda_max < mu (Lanczos estimate, then mu I - M positive
  // definite): M - theta/tau I not positive definite fires, M - mu/tau I
  // positive definite does not.  Only a lambda_min between the last two
  // shifts is left to the eigenvalues.
  for (int e = tid(); e < s * s; e += kSB) {
    const int i = ds.q(e), j = ds.r(e);
    M[e] = alpha[e] * rs[i] * rs[j];
  }
  __syncthreads();
  if (isfinite(lmax_hi) && rf_definite<SM>(M, s, 1.0, -lmax_hi * es)) return false;
  if (isfinite(lmax_lo) && !rf_definite<SM>(M, s, 1.0, -lmax_lo * es)) return true;
  const double theta = lanczos_lmax<SM>(M, s), mu = theta * (1.0 + 1e-3);
  if (theta > 0.0 && isfinite(theta) && rf_definite<SM>(M, s, -1.0, mu)) {
    if (!rf_definite<SM>(M, s, 1.0, -theta * es)) return true;
    if (rf_definite<SM>(M, s, 1.0, -mu * es)) return false;
  }
  __syncthreads();
  const double kd = sm_kappaD(alpha, s, M, T, rc, rs, partner, first, red);
  if (tid() == 0) c->kd_jacobi += 1;
  return h.eta * kd * h.sqrt_eps > 1.0;
}

__device__ __forceinline__ void store_coeff(double* d64, float* d32, const double* src, int s) {
  for (int t = tid(); t < s * s; t += kSB) {
    d64[t] = src[t];
    d32[t] = (float)src[t];
  }
}

__device__ __forceinline__ bool all_finite(const double* M, int count, double* red) {
  (void)red;
  __syncthreads();
  bool bad = false;
  for (int t = tid(); t < count; t += kSB) bad |= !isfinite(M[t]);
  return !wany(bad);
}

// ------------------------------------------------------------ projection --
__global__ __launch_bounds__(kSB) void project_kernel(const double* G, double* out, Sub sub, const int32_t* gate) {
  __shared__ double M[kSS];
  __shared__ double red[4];
  if (gate && *gate) return;
  const int ss = sub.s * sub.s;
  sm_copy(M, G + (int64_t)blockIdx.x * ss, ss);
  sm_project(M, sub, red);
  sm_copy(out + (int64_t)blockIdx.x * ss, M, ss);
}

hipError_t launch_project_batched(const double* G, double* out, Sub sub, int batch, const int32_t* gate,
                                  hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(project_kernel, dim3(batch), dim3(kSB), 0, st, G, out, sub, gate);
  return hipGetLastError();
}

hipError_t launch_project(const double* G, double* out, Sub sub, hipStream_t st) {
  return launch_project_batched(G, out, sub, 1, nullptr, st);
}

// --------------------------------------------------------------- CG steps --
// G_R0 (non-null): Gram of R0 = B - A X0 -> initial column norms, sigma = I
// when no normalisation follows.  G_rho (non-null): Gram of the (normalised)
// residual -> rho = <R, R>_S.
__global__ __launch_bounds__(kSB) void cg_init_kernel(CgCtl* c, const double* G_R0, const double* G_rho) {
  __shared__ double M[kSS];
  __shared__ double red[4];
  const int s = c->s;
  const Sub sub{c->kind, s, c->g};
  if (G_R0) {
    if (tid() == 0) {
      int allzero = 1;
      for (int i = 0; i < s; ++i) {
        const double nr = sqrt(G_R0[i * s + i]);
        c->r0n[i] = nr;
        c->relres[i] = nr > 0.0 ? 1.0 : 0.0;
        allzero &= (nr == 0.0);
      }
      c->iters = 0;
      c->status = 0;
      c->fire = 0;
      c->x_pending = 0;
      c->converged = allzero;
      c->done = allzero;
      c->gate = allzero;
      c->suspended = 0;
      c->kd_jacobi = 0;
      c->xdef_in = 0;
      c->xdef_pend = 0;
      c->lam_iter = -1;
      c->nreorth = (c->eta > 0.0 && !allzero) ? 1 : 0;
      c->bad_index = 0;
    }
    if (!(c->eta > 0.0)) sm_eye(c->sigma, s);
    for (int t = tid(); t < s * s; t += kSB) c->gamma[t] = (t / s == t % s) ? 1.0 : 0.0;
  }
  if (G_rho) {
    __syncthreads();
    if (c->done) return;
    sm_copy(M, G_rho, s * s);
    sm_project(M, sub, red);
    if (!all_finite(M, s * s, red)) {
      if (tid() == 0) {
        c->status = -3;
        c->done = 1;
        c->gate = 1;
      }
      return;
    }
    sm_copy(c->rho, M, s * s);
  }
}

hipError_t launch_cg_init(CgCtl* ctl, const double* G_R0, const double* G_rho, hipStream_t st) {
  hipLaunchKernelGGL(cg_init_kernel, dim3(1), dim3(kSB), 0, st, ctl, G_R0, G_rho);
  return hipGetLastError();
}

// alpha = <P, Q>_S; lambda = alpha^-1 rho; lambda sigma; the kappa_D test.
// Runs only while the solve is live and not suspended (the caller checks).
// rho_l, sigma_l: copies of c->rho and c->sigma (LDS, loaded by the caller).
// PART: kAlphaAll does everything; a launch of two workgroups splits the
// step into kAlphaCoef (lambda, lambda sigma, the deferred X bookkeeping;
// every failure is reported there) and kAlphaKappa (the kappa_D test on its
// own factorisation of the same alpha, writing only the fire flag), which
// run side by side: neither output depends on the other.
constexpr int kAlphaAll = 0, kAlphaCoef = 1, kAlphaKappa = 2;
template <int SM, int PART = kAlphaAll>
__device__ __forceinline__ void cg_alpha_body(CgCtl* c, const CgHead& h, const double* G, const double* rho_l,
                                              const double* sigma_l) {
  __shared__ double Al[kSS], Lm[kSS], LS[kSS], W[kSS], T[kSS];
  __shared__ double rc[kMaxS], rs[kMaxS], red[4];
  __shared__ int partner[kMaxS], first[kMaxS];
  const int s = h.s;
  const Sub sub{h.kind, s, h.g};
  if constexpr (PART == kAlphaKappa) {
    sm_copy(Al, G, s * s);
    sm_project(Al, sub, red);
    if (!all_finite(Al, s * s, red)) return;  // reported by the other part
    // L^-1 for the bounds (W serves as scratch for L); a failed
    // factorisation is reported by the other part
    if (reortho_dynamic(h) && !rf_cholesky_factor<SM>(Al, W, T, s)) return;
    const bool fire = reortho_test<SM>(c, h, Al, W, T, rc, rs, partner, first, red);
    if (tid() == 0) c->fire = fire ? 1 : 0;
    return;
  }
  // deferred X update: if the previous iteration's term is still owed, keep
  // its lambda sigma; this iteration's update then adds both, otherwise it
  // defers its own term
  // (the copy is loaded here and stored before the new lambda sigma, so
  // that no wait for it falls on the critical path)
  const int xin = h.xdef_pend;
  SmRegs<SM * SM, double> r_ls;
  SmRegs<SM * SM, float> r_lsf;
  if (xin) {
    sm_load(r_ls, c->lamsig, s * s);
    sm_load(r_lsf, c->lamsig_f, s * s);
  }
  auto keep_prev = [&] {
    if (xin) {
      sm_store(c->lamsig_prev, r_ls, s * s);
      sm_store(c->lamsig_prev_f, r_lsf, s * s);
    }
  };
  __syncthreads();
  if (tid() == 0) {
    c->xdef_in = xin;
    c->xdef_pend = xin ? 0 : 1;
  }
  sm_copy(Al, G, s * s);
  sm_project(Al, sub, red);
  bool ok = all_finite(Al, s * s, red);
  if (!ok) {
    keep_prev();
    if (tid() == 0) {
      c->status = -3;
      c->done = 1;
      c->gate = 1;
      c->x_pending = 0;
    }
    return;
  }
  // lambda = alpha^-1 rho, and L^-1 when the kappa_D test needs its bound
  if (!rf_cholesky_solve<SM>(Al, rho_l, Lm, (PART == kAlphaAll && reortho_dynamic(h)) ? T : nullptr, s)) {
    keep_prev();
    if (tid() == 0) {
      c->status = -2;
      c->done = 1;
      c->gate = 1;
      c->x_pending = 0;
    }
    return;
  }
  sm_mm(LS, Lm, sigma_l, s, false);  // lambda sigma
  // the coefficients go to global memory after the kappa_D test: a workgroup
  // barrier after a global store waits for the store
  bool fire = false;
  if constexpr (PART == kAlphaAll) fire = reortho_test<SM>(c, h, Al, W, T, rc, rs, partner, first, red);
  keep_prev();
  __syncthreads();
  store_coeff(c->lam, c->lam_f, Lm, s);
  store_coeff(c->lamsig, c->lamsig_f, LS, s);
  sm_copy(c->alpha, Al, s * s);
  if (tid() == 0) {
    if constexpr (PART == kAlphaAll) c->fire = fire ? 1 : 0;
    c->x_pending = 1;
  }
}

// G = R~^T R~ (full).  Column norms of the true residual R~ sigma, stopping
// test, and (no normalisation this iteration) rho' = <Z, R~>_S and
// beta = rho^-1 rho', Z = M^-1 R~ (Gz = R~^T M^-1 R~, or null for M = I).  Runs only while the iteration is live (the caller
// checks the gate).
// rho_l, sigma_l, r0n_l: copies of c->rho, c->sigma and c->r0n (LDS).
template <int SM>
__device__ __forceinline__ void cg_rho_body(CgCtl* c, const CgHead& h, const double* G, double* hist, const double* rho_l,
                                            const double* sigma_l, const double* r0n_l, const double* Gz) {
  __shared__ double Gm[kSS], T1[kSS], Bt[kSS];
  __shared__ double red[4];
  __shared__ int flag[1];
  const int s = h.s;
  const Sub sub{h.kind, s, h.g};
  const double* Sg = sigma_l;
  sm_copy(Gm, G, s * s);
  sm_mm(T1, Gm, Sg, s, false);  // G sigma
  // column norms of R~ sigma: sqrt(diag(sigma^T G sigma)), one lane per column
  double rel = 0.0;
  bool nanl = false;
  for (int i = tid(); i < s; i += kSB) {
    double acc = 0.0;
#pragma unroll 8
    for (int a = 0; a < s; ++a) acc += Sg[a * s + i] * T1[a * s + i];
    const double cn = sqrt(fmax(acc, 0.0));
    const double r = r0n_l[i] > 0.0 ? cn / r0n_l[i] : 0.0;
    nanl |= !isfinite(acc);
    c->relres[i] = r;
    rel = fmax(rel, r);
  }
  const double m = wmax(rel);
  const bool nan = wany(nanl);
  if (tid() == 0) {
    const int it = h.iters;
    if (hist && it < h.hist_cap) hist[it] = nan ? NAN : m;
    c->iters = it + 1;
    if (h.fire) c->nreorth += 1;
    int state = 0;  // 0 continue, 1 ended
    if (nan) {
      c->status = -3;
      state = 1;
    } else if (m <= h.tol) {
      c->converged = 1;
      state = 1;
    } else if (it + 1 >= h.maxit) {
      state = 1;
    }
    c->done = state;
    // a dynamically decided re-normalisation suspends the iteration; the host
    // launches it at its next read-back
    const int susp = (!state && h.fire && h.dynamic) ? 1 : 0;
    c->suspended = susp;
    c->gate = state | susp;
    flag[0] = state;
  }
  __syncthreads();
  if (flag[0] || h.fire) return;
  // rho' = <Z, R~>_S, beta = rho^-1 rho' (gamma = I); Z = R~ unless a
  // preconditioner's Gram Gz = R~^T M^-1 R~ is given
  if (Gz) {
    __syncthreads();
    sm_copy(Gm, Gz, s * s);
  }
  sm_project(Gm, sub, red);
  if (!rf_cholesky_solve<SM>(rho_l, Gm, Bt, nullptr, s)) {
    if (tid() == 0) {
      c->status = -2;
      c->done = 1;
      c->gate = 1;
    }
    return;
  }
  store_coeff(c->beta, c->beta_f, Bt, s);
  sm_copy(c->rho, Gm, s * s);
}

// One-reduction block CG (alg:1R-CG, Ch. 8): the coefficient step of
// iteration k from the Grams of R-bar^k, G = [R^T R | R^T A R] (full, s x s
// each).  k > 0: column norms of R-bar^k sigma^k and the stopping test
// (iteration k ends there), beta^{k-1} = rho^-1 gamma^T rho^k (gamma = I
// unless iteration k-1 re-normalised) and alpha^k = delta^k - beta^T alpha
// beta; k = 0: alpha^0 = delta^0.  Then lambda^k = alpha^-1 rho^k, lambda
// sigma (the previous one kept for the X update) and the kappa_D test of
// alpha^k, which decides whether R~^{k+1} is re-normalised.
// rho_l, sigma_l, r0n_l: copies of c->rho, c->sigma and c->r0n (LDS).
template <int SM>
__device__ __forceinline__ void cg1r_body(CgCtl* c, const CgHead& h, const double* G, double* hist, const double* rho_l,
                                          const double* sigma_l, const double* r0n_l) {
  __shared__ double Rh[kSS], Dl[kSS], T1[kSS], Bt[kSS], Al[kSS], Lm[kSS], W[kSS], Tt[kSS];
  __shared__ double rc[kMaxS], rs[kMaxS], red[4];
  __shared__ int partner[kMaxS], first[kMaxS], flag[1];
  const int s = h.s, ss = s * s;
  const Sub sub{h.kind, s, h.g};
  const int k = h.lam_iter + 1;
  auto fail = [&](int status) {
    if (tid() == 0) {
      c->status = status;
      c->done = 1;
      c->gate = 1;
    }
  };
  if (k > 0) {
    sm_mm(T1, G, sigma_l, s, false);  // G sigma
    double rel = 0.0;
    bool nanl = false;
    for (int i = tid(); i < s; i += kSB) {
      double acc = 0.0;
      for (int a = 0; a < s; ++a) acc += sigma_l[a * s + i] * T1[a * s + i];
      const double cn = sqrt(fmax(acc, 0.0));
      const double r = r0n_l[i] > 0.0 ? cn / r0n_l[i] : 0.0;
      nanl |= !isfinite(acc);
      c->relres[i] = r;
      rel = fmax(rel, r);
    }
    const double m = wmax(rel);
    const bool nan = wany(nanl);
    if (tid() == 0) {
      if (hist && k - 1 < h.hist_cap) hist[k - 1] = nan ? NAN : m;
      c->iters = k;
      int state = 0;
      if (nan) {
        c->status = -3;
        state = 1;
      } else if (m <= h.tol) {
        c->converged = 1;
        state = 1;
      } else if (k >= h.maxit) {
        state = 1;
      }
      c->done = state;
      c->gate = state;
      flag[0] = state;
    }
    __syncthreads();
    if (flag[0]) return;
  }
  sm_copy(Rh, G, ss);
  sm_project(Rh, sub, red);
  sm_copy(Dl, G + ss, ss);
  sm_project(Dl, sub, red);
  if (!all_finite(Rh, ss, red) || !all_finite(Dl, ss, red)) return fail(-3);
  if (k > 0) {
    if (h.fire) {  // gamma^T rho'
      sm_copy(W, c->gamma, ss);
      sm_mm(T1, W, Rh, s, true);
    } else {
      sm_copy(T1, Rh, ss);
    }
    if (!rf_cholesky_solve<SM>(rho_l, T1, Bt, nullptr, s)) return fail(-2);
    sm_copy(W, c->alpha, ss);
    sm_mm(T1, W, Bt, s, false);  // alpha beta
    sm_mm(Tt, Bt, T1, s, true);  // beta^T alpha beta
    for (int t = tid(); t < ss; t += kSB) Al[t] = Dl[t] - Tt[t];
  } else {
    for (int t = tid(); t < ss; t += kSB) {
      Bt[t] = 0.0;
      Al[t] = Dl[t];
    }
  }
  if (!all_finite(Al, ss, red)) return fail(-3);
  if (!rf_cholesky_solve<SM>(Al, Rh, Lm, reortho_dynamic(h) ? Tt : nullptr, s)) return fail(-2);
  sm_mm(T1, Lm, sigma_l, s, false);  // lambda sigma
  // global stores after the kappa_D test (see cg_alpha_body)
  const bool fire = reortho_test<SM>(c, h, Al, W, Tt, rc, rs, partner, first, red);
  __syncthreads();
  sm_fetch<kSS>(c->lamsig_prev, c->lamsig, ss);
  store_coeff(c->lam, c->lam_f, Lm, s);
  store_coeff(c->lamsig, c->lamsig_f, T1, s);
  store_coeff(c->beta, c->beta_f, Bt, s);
  sm_copy(c->alpha, Al, ss);
  sm_copy(c->rho, Rh, ss);
  if (tid() == 0) {
    c->fire = fire ? 1 : 0;
    c->lam_iter = k;
    // a dynamically decided re-normalisation suspends the iteration after
    // its fused pass; the host launches it at its next read-back
    const int susp = (fire && h.dynamic) ? 1 : 0;
    c->suspended = susp;
    c->gate = susp;
  }
}

// After R~^{k+1} was re-normalised (gamma in c->gamma): sigma = gamma sigma,
// count it, resume.
__global__ __launch_bounds__(kSB) void cg1r_fin_kernel(CgCtl* c) {
  __shared__ double Ga[kSS], Sg[kSS], T1[kSS];
  if (c->done || !c->fire) return;
  const int s = c->s;
  sm_copy(Ga, c->gamma, s * s);
  sm_copy(Sg, c->sigma, s * s);
  sm_mm(T1, Ga, Sg, s, false);
  sm_copy(c->sigma, T1, s * s);
  __syncthreads();
  if (tid() == 0) {
    c->nreorth += 1;
    c->suspended = 0;
    c->gate = 0;
  }
}

hipError_t launch_cg1r_fin(CgCtl* ctl, int s, hipStream_t st) {
  (void)s;
  hipLaunchKernelGGL(cg1r_fin_kernel, dim3(1), dim3(kSB), 0, st, ctl);
  return hipGetLastError();
}

// --------------------------------------------------- Gram reduction --
// grid (ns, batch), one wavefront per workgroup: workgroup (sl, y) sums the
// partials [b0, b1) of batch slice y in block order into red.gpart[y][sl];
// the last workgroup of slice y to finish adds the ns slice sums in slice
// order into red.G[y] and then runs the epilogue EPI on it.  Which workgroup
// finishes last does not change the order of any sum, so the result is
// deterministic.  Only the <= kMaxSlices workgroups of a slice take part in
// the hand-off, so its device-scope fences are cheap.
// Sum of p[b * stride], b < count, in order; the loads of a batch of 32 are
// all issued before the first add, so a batch costs one memory round trip.
template <typename T>
__device__ __forceinline__ double sum_strided(const T* __restrict__ p, int64_t stride, int count) {
  constexpr int K = 32;
  double acc = 0.0;
  for (int b = 0; b < count; b += K) {
    // unconditional loads (indexes past the end re-read the last partial and
    // are not added): a load under a branch would be waited for on its own
    T v[K];
#pragma unroll
    for (int u = 0; u < K; ++u) v[u] = p[(int64_t)min(b + u, count - 1) * stride];
    // keep the scheduler from moving the first adds (and so the first
    // wait) in between the loads: all K are in flight before the first wait
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < K; ++u)
      if (b + u < count) acc += (double)v[u];
  }
  return acc;
}

// Plain reductions (no epilogue) run four wavefronts per workgroup, so that
// wide Grams (s = 32: 1024 entries per partial) are summed by 256 lanes;
// the CG epilogues need a single wavefront.
constexpr int kRedPlain = 256;

// ng: Grams per partial of a plain reduction (EPI_NONE); the epilogue kinds
// fix their own.
template <typename T, int EPI, int SM>
__global__ __launch_bounds__(EPI == EPI_NONE ? kRedPlain : kSB) void reduce_kernel(
    int s, const T* __restrict__ partial, int nblk, Red red, const int32_t* gate, const int32_t* fire, CgCtl* c,
    double* hist, int ng) {
  constexpr int NTH = EPI == EPI_NONE ? kRedPlain : kSB;
  constexpr bool RHO = EPI == EPI_CG_RHO || EPI == EPI_CG_RHO_M;
  constexpr bool NORMS = RHO || EPI == EPI_CG_1R;
  constexpr int NG = (EPI == EPI_CG_RHO_M || EPI == EPI_CG_1R) ? 2 : 1;  // Grams per partial
  __shared__ int last;
  __shared__ double pre_rho[EPI != EPI_NONE ? kSS : 1], pre_sig[EPI != EPI_NONE ? kSS : 1];
  __shared__ double pre_r0n[NORMS ? kMaxS : 1];
  const int ss = s * s, m = (EPI == EPI_NONE ? ng : NG) * ss;
  // Every load of the prologue is issued before the first wait: the control
  // words and the epilogue's inputs from the control block (kept in
  // registers; only the last workgroup stores them to LDS), then, once the
  // gate is known, the partials.
  SmRegs<SM * SM, double> r_rho, r_sig;
  SmRegs<SM, double> r_r0n;
  int32_t cdone = 0, cgate = 0, gv = 0, fv = 1;
  CgHead h{};
  if constexpr (EPI != EPI_NONE) {
    if constexpr (EPI == EPI_CG_ALPHA) cdone = c->done;
    cgate = c->gate;
    h = cg_head(c);
    sm_load(r_rho, c->rho, ss);
    sm_load(r_sig, c->sigma, ss);
    if constexpr (NORMS) sm_load(r_r0n, c->r0n, s);
  } else {
    if (gate) gv = *gate;
    if (fire) fv = *fire;
  }
  if constexpr (EPI == EPI_CG_ALPHA) {
    if (cdone) {  // ended: nothing of this iteration reaches X (owed terms were added)
      if (blockIdx.x == 0 && tid() == 0) {
        c->x_pending = 0;
        c->xdef_in = 0;
      }
      return;
    }
    if (cgate) return;  // suspended: the iteration waits for its re-normalisation
  } else if constexpr (NORMS) {
    if (cgate) return;
  } else {
    if (gv || !fv) return;
  }
  const int ns = gridDim.x, sl = blockIdx.x, y = blockIdx.y;
  const T* P = partial + (int64_t)y * nblk * m;
  const int b0 = (int)((int64_t)nblk * sl / ns), b1 = (int)((int64_t)nblk * (sl + 1) / ns);
  double* slices = red.gpart + (int64_t)y * ns * m;
  for (int e = tid(); e < m; e += NTH) slices[(int64_t)sl * m + e] = sum_strided<T>(P + (int64_t)b0 * m + e, m, b1 - b0);
  uint32_t* cnt = red.cnt + (int64_t)y * kCntStride;
  __threadfence();
  __syncthreads();
  if (tid() == 0) last = (atomicAdd(cnt, 1u) == (uint32_t)(ns - 1));
  __syncthreads();
  if (!last) return;
  __threadfence();
  double* G = red.G + (int64_t)y * m;
  __shared__ double Gl[EPI != EPI_NONE ? NG * kSS : 1];
  for (int e = tid(); e < m; e += NTH) {
    const double v = sum_strided<double>(slices + e, m, ns);
    G[e] = v;
    if constexpr (EPI != EPI_NONE) Gl[e] = v;
  }
  if (tid() == 0) *cnt = 0;
  if constexpr (EPI != EPI_NONE) {
    sm_store(pre_rho, r_rho, ss);
    sm_store(pre_sig, r_sig, ss);
    if constexpr (NORMS) sm_store(pre_r0n, r_r0n, s);
  }
  if constexpr (EPI == EPI_CG_ALPHA) {
    __syncthreads();
    cg_alpha_body<SM>(c, h, Gl, pre_rho, pre_sig);
  } else if constexpr (RHO) {
    __syncthreads();
    cg_rho_body<SM>(c, h, Gl, hist, pre_rho, pre_sig, pre_r0n, NG == 2 ? Gl + ss : nullptr);
  } else if constexpr (EPI == EPI_CG_1R) {
    __syncthreads();
    cg1r_body<SM>(c, h, Gl, hist, pre_rho, pre_sig, pre_r0n);
  }
}

// The coefficient step of a CG reduction in a launch of its own, after a
// plain reduction into G (wide Grams: the plain reduction's four wavefronts
// sum s x s partials of s > 16 several times faster than the single
// wavefront an epilogue runs on).  Same gating and inputs as the fused form.
template <int EPI, int SM>
__global__ __launch_bounds__(kSB) void cg_epi_kernel(int s, const double* G, CgCtl* c, double* hist) {
  constexpr bool RHO = EPI == EPI_CG_RHO || EPI == EPI_CG_RHO_M;
  constexpr int NG = (EPI == EPI_CG_RHO_M || EPI == EPI_CG_1R) ? 2 : 1;
  __shared__ double pre_rho[kSS], pre_sig[kSS], pre_r0n[kMaxS], Gl[NG * kSS];
  // the control words and every input block are requested before the first
  // wait (s = c->s, passed by the host)
  const int ss = s * s;
  const int32_t cdone = EPI == EPI_CG_ALPHA ? c->done : 0, cgate = c->gate;
  const CgHead h = cg_head(c);
  SmRegs<SM * SM, double> r_rho, r_sig;
  SmRegs<SM, double> r_r0n;
  SmRegs<NG * SM * SM, double> r_g;
  sm_load(r_rho, c->rho, ss);
  sm_load(r_sig, c->sigma, ss);
  sm_load(r_r0n, c->r0n, s);
  sm_load(r_g, G, NG * ss);
  if constexpr (EPI == EPI_CG_ALPHA) {
    if (cdone) {
      if (blockIdx.x == 0 && tid() == 0) {
        c->x_pending = 0;
        c->xdef_in = 0;
      }
      return;
    }
  }
  if (cgate) return;
  sm_store(pre_rho, r_rho, ss);
  sm_store(pre_sig, r_sig, ss);
  sm_store(pre_r0n, r_r0n, s);
  sm_store(Gl, r_g, NG * ss);
  __syncthreads();
  if constexpr (EPI == EPI_CG_ALPHA) {
    // launched with two workgroups: the coefficients and the kappa_D test
    // side by side
    if (blockIdx.x == 0)
      cg_alpha_body<SM, kAlphaCoef>(c, h, Gl, pre_rho, pre_sig);
    else
      cg_alpha_body<SM, kAlphaKappa>(c, h, Gl, pre_rho, pre_sig);
  } else if constexpr (RHO) {
    cg_rho_body<SM>(c, h, Gl, hist, pre_rho, pre_sig, pre_r0n, NG == 2 ? Gl + ss : nullptr);
  } else {
    cg1r_body<SM>(c, h, Gl, hist, pre_rho, pre_sig, pre_r0n);
  }
}

// About 32 partials per reduction workgroup (one batch of loads), at most
// kMaxSlices workgroups.
static int reduce_slices(int nblk) {
  int ns = (nblk + 31) / 32;
  if (ns < 1) ns = 1;
  if (ns > kMaxSlices) ns = kMaxSlices;
  return ns;
}

// Plain reduction of partials of m >= 64 entries (s x s Grams from s = 8
// up): workgroup (x, y) owns entries [x kWideE, x kWideE + kWideE) of
// batch slice y, its threads being kWideE entries x kWideL partial lanes;
// lane q sums the partials q, q + kWideL, ... in order (one batch of loads
// for up to 32 of them), and the kWideL lane sums are added in lane order
// into red.G.  Every workgroup writes its own entries, so there is no
// hand-off between workgroups; the summation order is fixed, so the result
// is deterministic.  Gated like the plain form of reduce_kernel.
constexpr int kWideE = 16, kWideL = kRedPlain / kWideE;

template <typename T>
__global__ __launch_bounds__(kRedPlain) void reduce_wide_kernel(int m, const T* __restrict__ partial, int nblk,
                                                                 Red red, const int32_t* gate, const int32_t* fire) {
  __shared__ double part[kRedPlain];
  if ((gate && *gate) || (fire && !*fire)) return;
  const int y = blockIdx.y, x = threadIdx.x % kWideE, q = threadIdx.x / kWideE;
  const int e = blockIdx.x * kWideE + x;
  const T* P = partial + (int64_t)y * nblk * m;
  double acc = 0.0;
  if (e < m && q < nblk) acc = sum_strided<T>(P + (int64_t)q * m + e, (int64_t)kWideL * m, (nblk - q + kWideL - 1) / kWideL);
  part[threadIdx.x] = acc;
  __syncthreads();
  if (q == 0 && e < m) {
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < kWideL; ++k) v += part[k * kWideE + x];
    red.G[(int64_t)y * m + e] = v;
  }
}

template <typename T>
static void launch_reduce_plain(int m, const T* partial, int nblk, int batch, Red red, const int32_t* gate,
                                const int32_t* fire, int s, int ng, hipStream_t st) {
  if (m >= 64) {
    hipLaunchKernelGGL(reduce_wide_kernel<T>, dim3((m + kWideE - 1) / kWideE, batch), dim3(kRedPlain), 0, st, m,
                       partial, nblk, red, gate, fire);
  } else {
    dim3 grid(reduce_slices(nblk), batch);
    hipLaunchKernelGGL((reduce_kernel<T, EPI_NONE, 8>), grid, dim3(kRedPlain), 0, st, s, partial, nblk, red, gate,
                       fire, nullptr, nullptr, ng);
  }
}

template <typename T>
static hipError_t launch_reduce_t(int s, const T* partial, int nblk, int batch, Red red, const int32_t* gate,
                                  const int32_t* fire, Epi epi, hipStream_t st) {
  dim3 grid(reduce_slices(nblk), batch);
  if (epi.kind == EPI_NONE) {
    launch_reduce_plain<T>(s * s, partial, nblk, batch, red, gate, fire, s, 1, st);
    return hipGetLastError();
  }
  if (batch != 1 || !epi.ctl ||
      (epi.kind != EPI_CG_ALPHA && epi.kind != EPI_CG_RHO && epi.kind != EPI_CG_RHO_M && epi.kind != EPI_CG_1R))
    return hipErrorInvalidValue;
  if ((epi.kind == EPI_CG_RHO_M || epi.kind == EPI_CG_1R) && sizeof(T) != 8) return hipErrorInvalidValue;
  if (s >= 16) {
    // wide Grams (256 entries and more): plain reduction (gated like the
    // epilogue), then the coefficient step in its own single-wavefront
    // launch; the fused form's single wavefront would sum the partials in
    // s^2 / 64 dependent batches
    const int ng = (epi.kind == EPI_CG_RHO_M || epi.kind == EPI_CG_1R) ? 2 : 1;
    launch_reduce_plain<T>(ng * s * s, partial, nblk, 1, red, &epi.ctl->gate, nullptr, s, ng, st);
    auto go = [&](auto SM_) {
      constexpr int SM = decltype(SM_)::value;
      if (epi.kind == EPI_CG_ALPHA)
        hipLaunchKernelGGL((cg_epi_kernel<EPI_CG_ALPHA, SM>), dim3(2), dim3(kSB), 0, st, s, red.G, epi.ctl, epi.hist);
      else if (epi.kind == EPI_CG_RHO)
        hipLaunchKernelGGL((cg_epi_kernel<EPI_CG_RHO, SM>), dim3(1), dim3(kSB), 0, st, s, red.G, epi.ctl, epi.hist);
      else if (epi.kind == EPI_CG_RHO_M)
        hipLaunchKernelGGL((cg_epi_kernel<EPI_CG_RHO_M, SM>), dim3(1), dim3(kSB), 0, st, s, red.G, epi.ctl,
                           epi.hist);
      else
        hipLaunchKernelGGL((cg_epi_kernel<EPI_CG_1R, SM>), dim3(1), dim3(kSB), 0, st, s, red.G, epi.ctl, epi.hist);
    };
    if (s > 16)
      go(std::integral_constant<int, 32>{});
    else
      go(std::integral_constant<int, 16>{});
    return hipGetLastError();
  }
  return dispatch_sm(s, [&](auto SM_) -> hipError_t {
    constexpr int SM = decltype(SM_)::value;
    if (epi.kind == EPI_CG_ALPHA)
      hipLaunchKernelGGL((reduce_kernel<T, EPI_CG_ALPHA, SM>), grid, dim3(kSB), 0, st, s, partial, nblk, red, gate,
                         fire, epi.ctl, epi.hist, 1);
    else if (epi.kind == EPI_CG_RHO)
      hipLaunchKernelGGL((reduce_kernel<T, EPI_CG_RHO, SM>), grid, dim3(kSB), 0, st, s, partial, nblk, red, gate,
                         fire, epi.ctl, epi.hist, 1);
    else if constexpr (sizeof(T) == 8) {
      if (epi.kind == EPI_CG_RHO_M)
        hipLaunchKernelGGL((reduce_kernel<T, EPI_CG_RHO_M, SM>), grid, dim3(kSB), 0, st, s, partial, nblk, red, gate,
                           fire, epi.ctl, epi.hist, 1);
      else
        hipLaunchKernelGGL((reduce_kernel<T, EPI_CG_1R, SM>), grid, dim3(kSB), 0, st, s, partial, nblk, red, gate,
                           fire, epi.ctl, epi.hist, 1);
    } else {
      return hipErrorInvalidValue;
    }
    return hipGetLastError();
  });
}

hipError_t launch_reduce(int s, const void* partial, bool f32, int nblk, int batch, Red red, const int32_t* gate,
                         const int32_t* fire, Epi epi, hipStream_t st) {
  if (f32) return launch_reduce_t<float>(s, static_cast<const float*>(partial), nblk, batch, red, gate, fire, epi, st);
  return launch_reduce_t<double>(s, static_cast<const double*>(partial), nblk, batch, red, gate, fire, epi, st);
}

// After the residual was normalised, R~ = R-bar gamma: sigma = gamma sigma,
// rho' = <R-bar, R-bar>_S (G is the Gram of R-bar), beta = rho^-1 gamma^T rho'.
template <int SM>
__global__ __launch_bounds__(kSB) void cg_reortho_fin_kernel(CgCtl* c, const double* G) {
  __shared__ double Gm[kSS], Ga[kSS], Sg[kSS], T1[kSS], L[kSS], Bt[kSS];
  __shared__ double red[4];
  if (c->done || !c->fire) return;
  const int s = c->s;
  const Sub sub{c->kind, s, c->g};
  sm_copy(Ga, c->gamma, s * s);
  sm_copy(Sg, c->sigma, s * s);
  sm_mm(T1, Ga, Sg, s, false);
  sm_copy(c->sigma, T1, s * s);
  sm_copy(Gm, G, s * s);
  sm_project(Gm, sub, red);
  sm_mm(T1, Ga, Gm, s, true);  // gamma^T rho'
  sm_copy(L, c->rho, s * s);
  if (!rf_cholesky_solve<SM>(L, T1, Bt, nullptr, s)) {
    if (tid() == 0) {
      c->status = -2;
      c->done = 1;
      c->gate = 1;
      c->suspended = 0;  // the X update of this iteration still runs
    }
    return;
  }
  store_coeff(c->beta, c->beta_f, Bt, s);
  sm_copy(c->rho, Gm, s * s);
  __syncthreads();
  if (tid() == 0) {
    c->suspended = 0;
    c->gate = c->done;
  }
}

hipError_t launch_cg_reortho_fin(CgCtl* ctl, int s, const double* G, hipStream_t st) {
  return dispatch_sm(s, [&](auto SM_) -> hipError_t {
    constexpr int SM = decltype(SM_)::value;
    hipLaunchKernelGGL(cg_reortho_fin_kernel<SM>, dim3(1), dim3(kSB), 0, st, ctl, G);
    return hipGetLastError();
  });
}

// ------------------------------------------------------ block BiCGStab --
// X = A^-1 B inside the subalgebra for a general A (s x s in LDS, already
// projected, so its off-block entries are zero and the elimination stays
// inside each S-block) by Gaussian elimination with partial pivoting: the
// pivot is the first row of largest magnitude at or below the diagonal.  A
// and B are overwritten.  False (uniformly) on a zero or non-finite pivot.
__device__ __forceinline__ bool sm_lu_solve(double* A, double* B, double* X, int s, int* piv_sh) {
  for (int c = 0; c < s; ++c) {
    __syncthreads();
    if (tid() == 0) {
      int p = c;
      double best = fabs(A[c * s + c]);
      for (int i = c + 1; i < s; ++i)
        if (fabs(A[i * s + c]) > best) {
          best = fabs(A[i * s + c]);
          p = i;
        }
      piv_sh[0] = p;
    }
    __syncthreads();
    const int p = piv_sh[0];
    const double pv = A[p * s + c];
    if (!(pv != 0.0) || !isfinite(pv)) return false;
    if (p != c)
      for (int j = tid(); j < s; j += kSB) {
        double t = A[c * s + j];
        A[c * s + j] = A[p * s + j];
        A[p * s + j] = t;
        t = B[c * s + j];
        B[c * s + j] = B[p * s + j];
        B[p * s + j] = t;
      }
    __syncthreads();
    // rows below c: lane i computes its multiplier, then updates its row
    for (int i = c + 1 + tid(); i < s; i += kSB) {
      const double f = A[i * s + c] / A[c * s + c];
      for (int j = c; j < s; ++j) A[i * s + j] -= f * A[c * s + j];
      for (int j = 0; j < s; ++j) B[i * s + j] -= f * B[c * s + j];
    }
  }
  __syncthreads();
  for (int col = tid(); col < s; col += kSB)
    for (int i = s - 1; i >= 0; --i) {
      double sum = B[i * s + col];
      for (int k = i + 1; k < s; ++k) sum -= A[i * s + k] * X[k * s + col];
      X[i * s + col] = sum / A[i * s + i];
    }
  __syncthreads();
  return true;
}

__device__ __forceinline__ void bc_fail(CgCtl* c, int status) {
  if (tid() == 0) {
    c->status = status;
    c->done = 1;
    c->fire = 0;
  }
}

template <int SM>
__global__ __launch_bounds__(kSB) void bc_lambda_kernel(CgCtl* c, BcAux* x, const double* Gqr, const double* Grr) {
  __shared__ double Am[kSS], Bm[kSS], Lm[kSS], Sg[kSS], T1[kSS], Lo[kSS], Li[kSS], W[kSS];
  __shared__ double rc[kMaxS], rs[kMaxS], red[4];
  __shared__ int partner[kMaxS], first[kMaxS], piv[1];
  const int32_t cdone = c->done;
  const CgHead h = cg_head(c);  // before any write to the control block
  if (cdone) return;
  const int s = h.s, ss = s * s;
  const Sub sub{h.kind, s, h.g};
  // a = <R~0, Q>_S = proj((Q^T R~0)^T), <R~0, R>_S likewise
  for (int t = tid(); t < ss; t += kSB) {
    const int i = t / s, j = t % s;
    Am[t] = Gqr[j * s + i];
    Bm[t] = Gqr[ss + j * s + i];
  }
  sm_project(Am, sub, red);
  sm_project(Bm, sub, red);
  if (!all_finite(Am, ss, red) || !all_finite(Bm, ss, red)) {
    bc_fail(c, -3);
    return;
  }
  sm_copy(x->a, Am, ss);
  if (!sm_lu_solve(Am, Bm, Lm, s, piv)) {
    bc_fail(c, -2);
    return;
  }
  sm_copy(Sg, c->sigma, ss);
  sm_mm(T1, Lm, Sg, s, false);  // lambda sigma
  for (int t = tid(); t < ss; t += kSB) {
    x->neglam[t] = -Lm[t];
    c->lamsig[t] = T1[t];
  }
  // re-orthonormalisation test on kappa_D(<R, R>_S)
  for (int t = tid(); t < ss; t += kSB) W[t] = Grr[t];
  sm_project(W, sub, red);
  sm_copy(Am, W, ss);
  __syncthreads();
  bool fire;
  if (rf_cholesky_factor<SM>(Am, Lo, Li, s))
    fire = reortho_test<SM>(c, h, Am, W, Li, rc, rs, partner, first, red);
  else
    fire = h.eta > 0.0;  // not positive definite: kappa_D = infinity
  __syncthreads();
  if (tid() == 0) {
    c->fire = fire ? 1 : 0;
    if (fire) c->nreorth += 1;
  }
}

__global__ __launch_bounds__(kSB) void bc_sigma_kernel(CgCtl* c) {
  __shared__ double Ga[kSS], Sg[kSS], T1[kSS];
  if (c->done || !c->fire) return;
  const int s = c->s;
  sm_copy(Ga, c->gamma, s * s);
  sm_copy(Sg, c->sigma, s * s);
  sm_mm(T1, Ga, Sg, s, false);
  sm_copy(c->sigma, T1, s * s);
}

__global__ __launch_bounds__(kSB) void bc_omega_kernel(CgCtl* c, BcAux* x, const double* G3) {
  __shared__ double Am[kSS], Bm[kSS], Bt[kSS], Sg[kSS];
  __shared__ double red[4];
  __shared__ int piv[1];
  if (c->done) return;
  const int s = c->s, ss = s * s;
  const Sub sub{c->kind, s, c->g};
  double us = 0.0, uu = 0.0;
  for (int i = tid(); i < s; i += kSB) {
    us += G3[i * s + i];
    uu += G3[ss + i * s + i];
  }
  us = wsum(us);
  uu = wsum(uu);
  if (!isfinite(us) || !isfinite(uu)) {
    bc_fail(c, -3);
    return;
  }
  if (!(uu > 0.0)) {
    bc_fail(c, -2);
    return;
  }
  const double om = us / uu;
  sm_copy(Am, x->a, ss);
  for (int t = tid(); t < ss; t += kSB) Bm[t] = G3[2 * ss + t];  // <R~0, U> = R~0^T U
  sm_project(Bm, sub, red);
  if (!sm_lu_solve(Am, Bm, Bt, s, piv)) {
    bc_fail(c, -2);
    return;
  }
  sm_copy(Sg, c->sigma, ss);
  for (int t = tid(); t < ss; t += kSB) {
    const double b = -Bt[t];
    x->pbeta[t] = b;
    x->qbeta[t] = -om * b;
    x->omsig[t] = om * Sg[t];
    x->negomI[t] = (t / s == t % s) ? -om : 0.0;
  }
  if (tid() == 0) x->omega = om;
}

__global__ __launch_bounds__(kSB) void bc_stop_kernel(CgCtl* c, const double* Grr, double* hist) {
  __shared__ double Gm[kSS], Sg[kSS], T1[kSS];
  const int32_t cdone = c->done;
  const CgHead h = cg_head(c);  // before any write to the control block
  if (cdone) return;
  const int s = h.s;
  const double r0i = tid() < s ? c->r0n[tid()] : 0.0;
  sm_copy(Gm, Grr, s * s);
  sm_copy(Sg, c->sigma, s * s);
  sm_mm(T1, Gm, Sg, s, false);  // G sigma
  double rel = 0.0;
  bool nanl = false;
  for (int i = tid(); i < s; i += kSB) {
    double acc = 0.0;
#pragma unroll 8
    for (int a = 0; a < s; ++a) acc += Sg[a * s + i] * T1[a * s + i];
    const double r = r0i > 0.0 ? sqrt(fmax(acc, 0.0)) / r0i : 0.0;
    nanl |= !isfinite(acc);
    c->relres[i] = r;
    rel = fmax(rel, r);
  }
  const double m = wmax(rel);
  const bool nan = wany(nanl);
  if (tid() == 0) {
    const int it = h.iters;
    if (hist && it < h.hist_cap) hist[it] = nan ? NAN : m;
    c->iters = it + 1;
    if (nan) {
      c->status = -3;
      c->done = 1;
    } else if (m <= h.tol) {
      c->converged = 1;
      c->done = 1;
    } else if (it + 1 >= h.maxit) {
      c->done = 1;
    }
  }
}

hipError_t launch_bc_lambda(CgCtl* ctl, BcAux* aux, int s, const double* Gqr, const double* Grr, hipStream_t st) {
  return dispatch_sm(s, [&](auto SM_) -> hipError_t {
    constexpr int SM = decltype(SM_)::value;
    hipLaunchKernelGGL(bc_lambda_kernel<SM>, dim3(1), dim3(kSB), 0, st, ctl, aux, Gqr, Grr);
    return hipGetLastError();
  });
}

hipError_t launch_bc_sigma(CgCtl* ctl, hipStream_t st) {
  hipLaunchKernelGGL(bc_sigma_kernel, dim3(1), dim3(kSB), 0, st, ctl);
  return hipGetLastError();
}

hipError_t launch_bc_omega(CgCtl* ctl, BcAux* aux, const double* G3, hipStream_t st) {
  hipLaunchKernelGGL(bc_omega_kernel, dim3(1), dim3(kSB), 0, st, ctl, aux, G3);
  return hipGetLastError();
}

hipError_t launch_bc_stop(CgCtl* ctl, const double* Grr, double* hist, hipStream_t st) {
  hipLaunchKernelGGL(bc_stop_kernel, dim3(1), dim3(kSB), 0, st, ctl, Grr, hist);
  return hipGetLastError();
}

// ------------------------------------------------------------ CholeskyQR --
// One factorisation step of the block / hybrid normaliser by CholeskyQR2 (see
// launch_cholqr in internal.hpp for the plan flags).  G is the full Gram of
// the block; its projection onto the subalgebra is block diagonal, so one
// Cholesky of the whole matrix is one Cholesky per column group.
template <int SM>
__global__ __launch_bounds__(kSB) void cholqr_kernel(int stage, const double* G, Sub sub, double* R1, double* Rinv,
                                                      double* N, int32_t* plan, double ratio_min, const int32_t* gd,
                                                      const int32_t* gf) {
  __shared__ double Gm[kSS], L[kSS], Li[kSS], R1l[kSS];
  __shared__ double red[4];
  const int s = sub.s, t = tid();
  // the gates and the plan flag are read in one batch
  const int32_t gdv = gd ? *gd : 0, gfv = gf ? *gf : 1, p0 = plan[0];
  if (stage == 1) {
    if (gdv || !gfv) {
      if (t == 0) {
        plan[0] = 0;
        plan[1] = 0;
        plan[2] = 0;
      }
      return;
    }
  } else if (!p0) {
    return;
  }
  sm_copy(Gm, G, s * s);
  sm_project(Gm, sub, red);
  bool ok = all_finite(Gm, s * s, red);
  if (stage == 2 && ok) {
    // Y^T Y within rounding of I (every entry of each group's Gram within
    // 8 s eps of the identity): Y is already orthonormal to that level, the
    // second pass would change it by about as much, so it is skipped:
    // Q = Y, N = R1 (three block passes in all instead of five)
    bool off = false;
    const double tau = 8.0 * s * DBL_EPSILON;
    for (int e = t; e < s * s; e += kSB) {
      const int i = e / s, j = e % s;
      if (i / sub.g == j / sub.g) off |= !(fabs(Gm[e] - (i == j ? 1.0 : 0.0)) <= tau);
    }
    if (!wany(off)) {
      for (int e = t; e < s * s; e += kSB) N[e] = R1[e];
      if (t == 0) {
        plan[1] = 0;
        plan[2] = 0;
      }
      return;
    }
  }
  if (ok) ok = rf_cholesky_factor<SM>(Gm, L, Li, s);
  if (ok) {
    bool bad = false;
    if (stage == 1) {
      // kappa(X) >= max_j L_jj / min_j L_jj within a group: refuse ratios
      // beyond what one Cholesky of the Gram can resolve
      if (t < s) {
        const int g0 = (t / sub.g) * sub.g;
        double mx = 0.0;
        for (int j = g0; j < g0 + sub.g; ++j) mx = fmax(mx, L[j * s + j]);
        bad = !(L[t * s + t] >= ratio_min * mx);
      }
    } else {
      // Y^T Y must be near the identity for the second pass to finish
      for (int e = t; e < s * s; e += kSB) {
        const int i = e / s, j = e % s;
        if (i / sub.g == j / sub.g) bad |= !(fabs(Gm[e] - (i == j ? 1.0 : 0.0)) <= 0.5);
      }
    }
    ok = !wany(bad);
  }
  __syncthreads();
  if (stage == 1) {
    for (int e = t; e < s * s; e += kSB) {
      const int i = e / s, j = e % s;
      const double id = (i == j) ? 1.0 : 0.0;
      R1[e] = ok ? L[j * s + i] : id;    // R1 = L^T
      Rinv[e] = ok ? Li[j * s + i] : id; // R1^-1 = (L^-1)^T
    }
    if (t == 0) {
      plan[0] = ok ? 1 : 0;
      plan[1] = 0;
      plan[2] = ok ? 0 : 1;
    }
  } else {
    if (ok) {
      sm_copy(R1l, R1, s * s);
      __syncthreads();
      for (int e = t; e < s * s; e += kSB) {
        const int i = e / s, j = e % s;
        Rinv[e] = Li[j * s + i];
        double acc = 0.0;  // (L^T R1)_ij
        for (int k = 0; k < s; ++k) acc = fma(L[k * s + i], R1l[k * s + j], acc);
        N[e] = acc;
      }
    }
    if (t == 0) {
      plan[1] = ok ? 1 : 0;
      plan[2] = ok ? 0 : 1;
    }
  }
}

__global__ __launch_bounds__(kSB) void cholqr_compose_kernel(const double* Nh, const double* R1, double* N, int s,
                                                              const int32_t* plan) {
  if (!plan[2]) return;
  for (int e = tid(); e < s * s; e += kSB) {
    const int i = e / s, j = e % s;
    double acc = 0.0;
    for (int k = 0; k < s; ++k) acc = fma(Nh[i * s + k], R1[k * s + j], acc);
    N[e] = acc;
  }
}

hipError_t launch_cholqr(int stage, const double* G, Sub sub, double* R1, double* Rinv, double* N, int32_t* plan,
                         double ratio_min, const int32_t* gd, const int32_t* gf, hipStream_t st) {
  return dispatch_sm(sub.s, [&](auto SM_) -> hipError_t {
    constexpr int SM = decltype(SM_)::value;
    hipLaunchKernelGGL(cholqr_kernel<SM>, dim3(1), dim3(kSB), 0, st, stage, G, sub, R1, Rinv, N, plan, ratio_min,
                       gd, gf);
    return hipGetLastError();
  });
}

hipError_t launch_cholqr_compose(const double* Nh, const double* R1, double* N, Sub sub, const int32_t* plan,
                                 hipStream_t st) {
  hipLaunchKernelGGL(cholqr_compose_kernel, dim3(1), dim3(kSB), 0, st, Nh, R1, N, sub.s, plan);
  return hipGetLastError();
}

// Normaliser of the parallel (N = diag(|x_j|)) and global (N = |X|_F/sqrt(p) I)
// subalgebras from the Gram matrix G of X.
__global__ __launch_bounds__(kSB) void norm_diag_kernel(const double* G, Sub sub, double* d, double* N,
                                                         const int32_t* gd, const int32_t* gf) {
  if (gd && *gd) return;
  if (gf && !*gf) return;
  const int s = sub.s;
  __shared__ double cg[1];
  if (tid() == 0) {
    double ss = 0.0;
    for (int j = 0; j < s; ++j) ss += G[j * s + j];
    cg[0] = sqrt(ss) / sqrt((double)s);
  }
  __syncthreads();
  for (int t = tid(); t < s * s; t += kSB) {
    const int i = t / s, j = t % s;
    const double dj = sub.kind == GLOBAL ? cg[0] : sqrt(G[j * s + j]);
    if (i == 0) d[j] = dj;
    N[t] = (i == j) ? dj : 0.0;
  }
}

hipError_t launch_norm_diag(const double* G, Sub sub, double* d, double* out_N, const int32_t* gate_done,
                            const int32_t* gate_fire, hipStream_t st) {
  hipLaunchKernelGGL(norm_diag_kernel, dim3(1), dim3(kSB), 0, st, G, sub, d, out_N, gate_done, gate_fire);
  return hipGetLastError();
}

// Block-global normaliser from the R factor rho (g x g) of the stacked
// groups: N = I_q (x) rho / sqrt(q), and d[j] = 1/sqrt(q) (the column divisor
// that turns the stacked Q into Y = sqrt(q) Q).
__global__ __launch_bounds__(kSB) void bg_expand_kernel(const double* rho, Sub sub, double* N, double* d,
                                                        const int32_t* gd, const int32_t* gf) {
  if (gd && *gd) return;
  if (gf && !*gf) return;
  const int s = sub.s, g = sub.g;
  const double rq = sqrt((double)(s / g));
  for (int t = tid(); t < s * s; t += kSB) {
    const int i = t / s, j = t % s;
    N[t] = (i / g == j / g) ? rho[(i % g) * g + j % g] / rq : 0.0;
  }
  for (int j = tid(); j < s; j += kSB) d[j] = 1.0 / rq;
}

hipError_t launch_bg_expand(const double* rho, Sub sub, double* N, double* d, const int32_t* gate_done,
                            const int32_t* gate_fire, hipStream_t st) {
  hipLaunchKernelGGL(bg_expand_kernel, dim3(1), dim3(kSB), 0, st, rho, sub, N, d, gate_done, gate_fire);
  return hipGetLastError();
}

// ------------------------------------------------------------------ GMRes --
// Full QR of the rows x cols matrix M (row stride cols, rows <= 64) by
// Householder reflections: R in the upper triangle of M, the full rows x rows
// orthogonal Q (row stride rows) with M_in = Q [R; 0].
// GC > 0: cols = GC and rows = 2 GC known at compile time (every loop
// unrolled without guards, so no load waits inside a branch); GC = 0: any
// cols <= SM, rows = 2 cols.
template <int SM, int GC = 0>
__device__ __forceinline__ void sm_house_full(double* M, int rows, int cols, double* Q, double* beta) {
  // rows <= 2 SM <= kSB (lane t holds row t of the reflected column), cols <= SM
  constexpr int RM = 2 * SM;
  if constexpr (GC > 0) {
    rows = 2 * GC;
    cols = GC;
  }
  const int t = tid();
#pragma unroll
  for (int j = 0; j < (GC > 0 ? GC : SM); ++j) {
    if (GC == 0 && j >= cols) break;
    sm_wave_sync();
    const double xi = (t > j && t < rows) ? M[t * cols + j] : 0.0;
    const double sig = wsum(xi * xi);
    const double x1 = M[j * cols + j];
    double b = 0.0, v1 = 1.0, mu = 0.0;
    if (sig != 0.0) {
      mu = sqrt(x1 * x1 + sig);
      v1 = (x1 <= 0.0) ? (x1 - mu) : (-sig / (x1 + mu));
      b = 2.0 * v1 * v1 / (sig + v1 * v1);
    }
    sm_wave_sync();
    if (sig != 0.0) {
      if (t > j && t < rows) M[t * cols + j] = xi / v1;
      if (t == j) M[j * cols + j] = mu;
    }
    if (t == 0) beta[j] = b;
    sm_wave_sync();
    if (b != 0.0) {
      // the two columns are read into registers before any store: a store
      // to column cc might alias a later load of column j for all the
      // compiler knows, which would order every load after the stores
      for (int cc = j + 1 + t; cc < cols; cc += kSB) {
        double vj[RM], vc[RM];
#pragma unroll
        for (int i = 0; i < RM; ++i) {
          const int r = j + i;
          vj[i] = (r < rows) ? M[r * cols + j] : 0.0;
          vc[i] = (r < rows) ? M[r * cols + cc] : 0.0;
        }
        double w = vc[0];
#pragma unroll
        for (int i = 1; i < RM; ++i) w += vj[i] * vc[i];
        M[j * cols + cc] = vc[0] - b * w;
#pragma unroll
        for (int i = 1; i < RM; ++i) {
          const int r = j + i;
          if (r < rows) M[r * cols + cc] = vc[i] - b * vj[i] * w;
        }
      }
    }
  }
  sm_wave_sync();
  for (int e = t; e < rows * rows; e += kSB) Q[e] = 0.0;
  sm_wave_sync();
  if (t < rows) Q[t * rows + t] = 1.0;
#pragma unroll
  for (int jj = (GC > 0 ? GC : SM) - 1; jj >= 0; --jj) {
    const int j = (GC > 0) ? jj : jj - (SM - cols);
    if (j < 0) continue;
    sm_wave_sync();
    const double b = beta[j];
    if (b == 0.0) continue;
    if (t < rows) {
      const int cc = t;
      double vj[RM], vc[RM];
#pragma unroll
      for (int i = 0; i < RM; ++i) {
        const int r = j + i;
        vj[i] = (r < rows && i > 0) ? M[r * cols + j] : 0.0;
        vc[i] = (r < rows) ? Q[r * rows + cc] : 0.0;
      }
      double w = vc[0];
#pragma unroll
      for (int i = 1; i < RM; ++i) w += vj[i] * vc[i];
      Q[j * rows + cc] = vc[0] - b * w;
#pragma unroll
      for (int i = 1; i < RM; ++i) {
        const int r = j + i;
        if (r < rows) Q[r * rows + cc] = vc[i] - b * vj[i] * w;
      }
    }
  }
  sm_wave_sync();
}

// [x; y] <- Om^T [x; y] for S-elements x, y (s x s, row stride s), Om the
// per-group 2g x 2g factors stored consecutively.
template <int SM, int GC = 0>
__device__ __forceinline__ void sm_apply_givens_T(const double* Om, double* x, double* y, int s, int g, double* tmp) {
  if constexpr (GC > 0) g = GC;
  const int ngrp = s / g, m2 = 2 * g;
  __syncthreads();
  for (int e = tid(); e < ngrp * m2 * g; e += kSB) {
    const int grp = e / (m2 * g), rem = e % (m2 * g), i = rem / g, cc = rem % g;
    const double* O = Om + (int64_t)grp * m2 * m2;
    const int o = grp * g;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < 2 * (GC > 0 ? GC : SM); ++k) {
      if (GC > 0 || k < m2) {
        const double col = k < g ? x[(o + k) * s + o + cc] : y[(o + k - g) * s + o + cc];
        acc += O[k * m2 + i] * col;
      }
    }
    tmp[e] = acc;
  }
  __syncthreads();
  for (int e = tid(); e < ngrp * m2 * g; e += kSB) {
    const int grp = e / (m2 * g), rem = e % (m2 * g), i = rem / g, cc = rem % g;
    const int o = grp * g;
    if (i < g)
      x[(o + i) * s + o + cc] = tmp[e];
    else
      y[(o + i - g) * s + o + cc] = tmp[e];
  }
  __syncthreads();
}

__global__ __launch_bounds__(kSB) void gm_cycle_init_kernel(GmCtl* c, double* sig, const double* sigma0,
                                                             const double* G_R, int first) {
  const int s = c->s, m = c->m, ss = s * s;
  if (first && tid() == 0) {
    double f = 0.0;
    for (int i = 0; i < s; ++i) {
      c->r0n[i] = sqrt(G_R[i * s + i]);
      f += G_R[i * s + i];
    }
    c->r0F = sqrt(f);
    c->total = 0;
    c->status = 0;
    c->converged = (f == 0.0);
    c->bad_index = 0;
  }
  __syncthreads();
  for (int t = tid(); t < (m + 1) * ss; t += kSB) sig[t] = t < ss ? sigma0[t] : 0.0;
  if (tid() == 0) {
    c->kend = 0;
    c->done = c->converged;
  }
}

hipError_t launch_gm_cycle_init(GmCtl* ctl, double* sig, const double* sigma0, const double* G_R, int first,
                                hipStream_t st) {
  hipLaunchKernelGGL(gm_cycle_init_kernel, dim3(1), dim3(kSB), 0, st, ctl, sig, sigma0, G_R, first);
  return hipGetLastError();
}

// Step k of a cycle: the new Hessenberg column h_jk = H1_j + H2_j (the two
// Gram-Schmidt passes) for j <= k and gamma = h_{k+1,k}.
// Rotations staged in LDS at once (width <= 8, k <= kGmStage): the factor of
// each previous rotation and the next block, kGmStage x (4 g^2 + s^2) <= 40 x
// 320 entries.
constexpr int kGmStage = 40;

template <int SM>
__global__ __launch_bounds__(kSB) void gm_step_kernel(GmCtl* c, int k, double* H, double* sig, double* Om,
                                                       const double* H1, const double* H2, const double* gamma,
                                                       double* hist) {
  constexpr int NO = 4 * SM * SM;  // entries of one rotation's factors (ngrp m2^2 <= (2 SM)^2)
  constexpr bool STAGE = SM <= 8;
  __shared__ double Qf[NO], tmp[2 * SM * SM], gm[SM * SM], xs[SM * SM], ys[SM * SM];
  __shared__ double stage[STAGE ? kGmStage * (NO + SM * SM) : 1];
  // staged: the rotated blocks j < k of the new column, written to H once
  // after the rotations (a workgroup barrier after a global store waits for
  // the store, which would expose one memory round trip per rotation)
  __shared__ double hrot[STAGE ? kGmStage * SM * SM : 1];
  __shared__ double beta[SM];
  double* M = tmp;  // the Householder input is not live while rotations use tmp
  if (c->done) return;
  const int s = c->s, g = c->g, m = c->m, ss = s * s, ngrp = s / g, m2 = 2 * g;
  const int t0 = tid();
  const int no = ngrp * m2 * m2, ne = ngrp * m2 * g;
  const bool staged = STAGE && k <= kGmStage;
  // The new column, h_jk = H1_j + H2_j for j <= k (blocks j < k are replaced
  // by their rotated values below); with staging, also every previous
  // rotation's factor and block j + 1 of the new column into LDS.  Loads in
  // chunks of U per lane, all issued before the chunk's stores: the loads
  // are unconditional (indexes past the end re-read the last entry) and a
  // scheduling barrier keeps them ahead of the first use, so a chunk costs
  // one memory round trip.
  {
    constexpr int U = 16;
    const int total = (k + 1) * ss;
    for (int base = 0; base < total; base += U * kSB) {
      double a[U], b[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int t = min(base + t0 + u * kSB, total - 1);
        a[u] = H1[t];
        b[u] = H2[t];
      }
      __builtin_amdgcn_sched_barrier(0);
      // block j and entry e of t = base + t0 + u kSB, advanced by kSB per
      // u (one division per batch instead of one per entry)
      int j = (base + t0) / ss, e = base + t0 - j * ss;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int t = base + t0 + u * kSB;
        const double v = a[u] + b[u];
        if (t < total) {
          H[((int64_t)j * m + k) * ss + e] = v;
          if (staged && j >= 1) stage[(j - 1) * (NO + SM * SM) + NO + e] = v;
        }
        e += kSB;
        while (e >= ss) {
          e -= ss;
          ++j;
        }
      }
    }
    if (staged) {
      const int tot = k * no;
      for (int base = 0; base < tot; base += U * kSB) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = Om[min(base + t0 + u * kSB, tot - 1)];
        __builtin_amdgcn_sched_barrier(0);
        int j = (base + t0) / no, e = base + t0 - j * no;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int t = base + t0 + u * kSB;
          if (t < tot) stage[j * (NO + SM * SM) + e] = v[u];
          e += kSB;
          while (e >= no) {
            e -= no;
            ++j;
          }
        }
      }
    }
  }
  sm_copy(gm, gamma, ss);
  for (int e = t0; e < ss; e += kSB) xs[e] = H1[e] + H2[e];
  // Rotations of the previous steps, j = 0 .. k-1: x carries block j of the
  // new column, y receives block j+1.  Unstaged, the factor of rotation j+1
  // and block j+2 are loaded into registers while rotation j is applied, so
  // memory latency is exposed about once per rotation.
  constexpr int RO = (NO + kSB - 1) / kSB;       // factor entries per lane (m2 = 2g <= 2s)
  constexpr int RS = (SM * SM + kSB - 1) / kSB;  // block entries per lane
  constexpr int RN = (2 * SM * SM + kSB - 1) / kSB;  // rotated entries per lane
  const SmDiv dg(g);
  const bool full = g == SM && s == SM;  // one group of full width: m2 = 2 SM
  double opre[RO], ypre[RS];
  auto load_next = [&](int j) {
#pragma unroll
    for (int r = 0; r < RO; ++r) {
      const int e = t0 + r * kSB;
      opre[r] = (j < k && e < no) ? Om[(int64_t)j * no + e] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      const int e = t0 + r * kSB;
      ypre[r] = (j < k && e < ss) ? H1[(int64_t)(j + 1) * ss + e] + H2[(int64_t)(j + 1) * ss + e] : 0.0;
    }
  };
  if (!staged) load_next(0);
  if (staged && full) __syncthreads();  // the staged data, before the LDS-only rotations
  for (int j = 0; j < k; ++j) {
    if (staged && full)
      sm_wave_sync();
    else
      __syncthreads();
    const double* O0 = Qf;
    const double* Y = ys;
    if constexpr (SM == 8) {
      if (staged && full) {
        // [x; y] <- O^T [x; y] (16 x 8) as four 16 x 16 x 4 products on the
        // matrix cores (lane layout of mf_mma): A[i][q] = O[q][i], B[q][c] =
        // row q of [x; y] (columns 8 .. 15 zero), D[i][c] = the rotated row i
        const double* O = stage + j * (NO + SM * SM);
        const double* Ys = O + NO;
        const int lr = t0 / 16, lc = t0 % 16;
        mf_d4 acc = mf_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int q = 4 * kk + lr;
          const double a = O[q * 16 + lc];
          double bv = 0.0;
          if (lc < 8) bv = q < 8 ? xs[q * 8 + lc] : Ys[(q - 8) * 8 + lc];
          acc = mf_mma(a, bv, acc);
        }
        sm_wave_sync();
        if (lc < 8) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = 4 * v + lr;
            if (i < 8)
              hrot[j * SM * SM + i * 8 + lc] = acc[v];
            else
              xs[(i - 8) * 8 + lc] = acc[v];
          }
        }
        continue;
      }
    }
    if (staged) {
      O0 = stage + j * (NO + SM * SM);
      Y = O0 + NO;
    } else {
#pragma unroll
      for (int r = 0; r < RO; ++r) {
        const int e = t0 + r * kSB;
        if (e < no) Qf[e] = opre[r];
      }
#pragma unroll
      for (int r = 0; r < RS; ++r) {
        const int e = t0 + r * kSB;
        if (e < ss) ys[e] = ypre[r];
      }
      __syncthreads();
      load_next(j + 1);
    }
    double out[RN];
#pragma unroll
    for (int r = 0; r < RN; ++r) {
      const int e = t0 + r * kSB;
      out[r] = 0.0;
      if (e < ne) {
        const int ge = dg.q(e), grp = dg.q(ge) / 2, i = ge - grp * m2, cc = e - ge * g;
        const double* O = O0 + grp * m2 * m2;
        const int o = grp * g;
        double acc = 0.0;
        // compile-time trip count (m2 <= 2 SM; exactly 2 SM when g = SM):
        // every LDS load of the product is issued before the first add
        if (full) {
#pragma unroll
          for (int q = 0; q < 2 * SM; ++q) {
            const double col = q < SM ? xs[q * s + cc] : Y[(q - SM) * s + cc];
            acc += O[q * 2 * SM + i] * col;
          }
        } else {
#pragma unroll
          for (int q = 0; q < 2 * SM; ++q) {
            if (q < m2) {
              const double col = q < g ? xs[(o + q) * s + o + cc] : Y[(o + q - g) * s + o + cc];
              acc += O[q * m2 + i] * col;
            }
          }
        }
        out[r] = acc;
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RN; ++r) {
      const int e = t0 + r * kSB;
      if (e < ne) {
        const int ge = dg.q(e), grp = dg.q(ge) / 2, i = ge - grp * m2, cc = e - ge * g;
        const int o = grp * g;
        if (i >= g)
          xs[(o + i - g) * s + o + cc] = out[r];
        else if (staged)
          hrot[j * SM * SM + (o + i) * s + o + cc] = out[r];
        else
          H[((int64_t)j * m + k) * ss + (o + i) * s + o + cc] = out[r];
      }
    }
  }
  if (staged) {
    __syncthreads();
    // blocks j < k of the new column: the rotated group entries (the rest of
    // each block keeps the value written above)
    if (full) {
      // one group of full width: the rotated part of block j is all of it
#pragma unroll 4
      for (int j = 0; j < k; ++j) {
        double* Hj = H + ((int64_t)j * m + k) * ss;
        const double* hj = hrot + j * SM * SM;
        for (int e = t0; e < ss; e += kSB) Hj[e] = hj[e];
      }
    } else {
      for (int j = 0; j < k; ++j) {
        double* Hj = H + ((int64_t)j * m + k) * ss;
        const double* hj = hrot + j * SM * SM;
        for (int e = t0; e < ne; e += kSB) {
          const int ge = dg.q(e), grp = dg.q(ge) / 2, i = ge - grp * m2, cc = e - ge * g;
          const int o = grp * g;
          if (i < g) Hj[(o + i) * s + o + cc] = hj[(o + i) * s + o + cc];
        }
      }
    }
  }
  __syncthreads();
  double* hkk = H + ((int64_t)k * m + k) * ss;
  for (int e = t0; e < ss; e += kSB) hkk[e] = xs[e];
  __syncthreads();
  double* Omk = Om + (int64_t)k * ngrp * m2 * m2;
  if (g == 1) {
    // 2 x 1 Householder per column
    for (int grp = tid(); grp < ngrp; grp += kSB) {
      const double x1 = xs[grp * s + grp], x2 = gm[grp * s + grp];
      const double sg = x2 * x2;
      double* O = Omk + grp * 4;
      if (sg == 0.0) {
        O[0] = 1.0; O[1] = 0.0; O[2] = 0.0; O[3] = 1.0;
      } else {
        const double mu = sqrt(x1 * x1 + sg);
        const double v1 = (x1 <= 0.0) ? (x1 - mu) : (-sg / (x1 + mu));
        const double b = 2.0 * v1 * v1 / (sg + v1 * v1);
        const double v2 = x2 / v1;
        O[0] = 1.0 - b; O[1] = -b * v2; O[2] = -b * v2; O[3] = 1.0 - b * v2 * v2;
        hkk[grp * s + grp] = mu;
      }
    }
  } else {
    for (int grp = 0; grp < ngrp; ++grp) {
      const int o = grp * g;
      __syncthreads();
      for (int t = tid(); t < m2 * g; t += kSB) {
        const int i = t / g, cc = t % g;
        M[t] = i < g ? xs[(o + i) * s + o + cc] : gm[(o + i - g) * s + o + cc];
      }
      if (g == SM)
        sm_house_full<SM, SM>(M, m2, g, Qf, beta);
      else
        sm_house_full<SM>(M, m2, g, Qf, beta);
      for (int t = tid(); t < m2 * m2; t += kSB) Omk[grp * m2 * m2 + t] = Qf[t];
      for (int t = tid(); t < g * g; t += kSB) {
        const int i = t / g, cc = t % g;
        hkk[(o + i) * s + o + cc] = cc >= i ? M[i * g + cc] : 0.0;
      }
    }
  }
  __syncthreads();
  // sigma_k and sigma_{k+1} are rotated in LDS (xs and ys are free by now)
  sm_fetch<SM * SM>(xs, sig + (int64_t)k * ss, ss);
  sm_fetch<SM * SM>(ys, sig + (int64_t)(k + 1) * ss, ss);
  if (g == SM)
    sm_apply_givens_T<SM, SM>(Omk, xs, ys, s, g, tmp);
  else
    sm_apply_givens_T<SM>(Omk, xs, ys, s, g, tmp);
  for (int e = t0; e < ss; e += kSB) {
    sig[(int64_t)k * ss + e] = xs[e];
    sig[(int64_t)(k + 1) * ss + e] = ys[e];
  }
  // residual measure from sigma_{k+1}: column norms (lane i: column i), or
  // the Frobenius norm for the global subalgebras
  double meas;
  bool nan;
  {
    const double* sk = ys;
    double acc = 0.0;
    if (t0 < s) {
#pragma unroll 8
      for (int a = 0; a < s; ++a) acc += sk[a * s + t0] * sk[a * s + t0];
    }
    if (c->kind == GLOBAL || c->kind == BGLOBAL) {
      const double f = wsum(acc);
      meas = sqrt(f) / c->r0F;
      nan = !isfinite(f);
    } else {
      const double rel = (t0 < s && c->r0n[t0] > 0.0) ? sqrt(acc) / c->r0n[t0] : 0.0;
      meas = wmax(rel);
      nan = wany(!isfinite(acc));
    }
  }
  if (tid() == 0) {
    const int tot = c->total;
    if (hist && tot < c->hist_cap) hist[tot] = nan ? NAN : meas;
    c->total = tot + 1;
    c->kend = k + 1;
    if (nan) {
      c->status = -3;
      c->done = 1;
    } else if (meas <= c->tol) {
      c->converged = 1;
      c->done = 1;
    } else if (tot + 1 >= c->maxit) {
      c->done = 1;
    }
  }
}

hipError_t launch_gm_step(GmCtl* ctl, int s, int k, double* H, double* sig, double* Om, const double* H1,
                          const double* H2, const double* gamma, double* hist, hipStream_t st) {
  return dispatch_sm(s, [&](auto SM_) -> hipError_t {
    constexpr int SM = decltype(SM_)::value;
    hipLaunchKernelGGL(gm_step_kernel<SM>, dim3(1), dim3(kSB), 0, st, ctl, k, H, sig, Om, H1, H2, gamma, hist);
    return hipGetLastError();
  });
}

// zeta_l = R_ll^-1 (sigma_l - sum_{j>l} H_lj zeta_j), l = kend-1 .. 0; a zero
// pivot gives a zero component.
__global__ __launch_bounds__(kSB) void gm_backsub_kernel(GmCtl* c, const double* H, const double* sig,
                                                          double* zeta) {
  __shared__ double tmp[kSS];
  const int s = c->s, g = c->g, m = c->m, ss = s * s, kend = c->kend;
  for (int l = kend - 1; l >= 0; --l) {
    __syncthreads();
    for (int t = tid(); t < ss; t += kSB) {
      const int a = t / s, b = t % s;
      double acc = sig[(int64_t)l * ss + t];
      for (int j = l + 1; j < kend; ++j) {
        const double* hl = H + ((int64_t)l * m + j) * ss;
        const double* zj = zeta + (int64_t)j * ss;
        double d = 0.0;
        for (int cc = 0; cc < s; ++cc) d += hl[a * s + cc] * zj[cc * s + b];
        acc -= d;
      }
      tmp[t] = acc;
    }
    __syncthreads();
    const double* T = H + ((int64_t)l * m + l) * ss;
    double* z = zeta + (int64_t)l * ss;
    for (int t = tid(); t < ss; t += kSB) z[t] = 0.0;
    __syncthreads();
    for (int e = tid(); e < s; e += kSB) {  // thread per (group, column): e = o + b
      const int grp = e / g, b = e % g, o = grp * g;
      for (int a = g - 1; a >= 0; --a) {
        double acc = tmp[(o + a) * s + o + b];
        for (int cc = a + 1; cc < g; ++cc) acc -= T[(o + a) * s + o + cc] * z[(o + cc) * s + o + b];
        const double piv = T[(o + a) * s + o + a];
        z[(o + a) * s + o + b] = piv != 0.0 ? acc / piv : 0.0;
      }
    }
  }
}

// The same back substitution for widths s <= 8 and kend <= kGmStage, right-
// looking: once zeta_j is known, every right-hand side l < j loses H_lj
// zeta_j.  The right-hand sides stay in LDS; lane q < s^2 holds entry q of
// every block, and the blocks H_lj, l < j, of the next step are loaded into
// registers while this step runs, so each step waits for memory about once
// (the left-looking form above waits for every block it reads).
__global__ __launch_bounds__(kSB) void gm_backsub8_kernel(GmCtl* c, const double* H, const double* sig,
                                                           double* zeta) {
  constexpr int SS = 64, NB = kGmStage;
  __shared__ double rhs[NB * SS], hb[NB * SS], zj[SS], zl[NB * SS];
  const int s = c->s, g = c->g, m = c->m, ss = s * s, kend = c->kend;
  const int q = tid();
  const bool own = q < ss;
  if (kend <= 0) return;
  // loads are unconditional (indexes outside the used range re-read a valid
  // entry, never stored), so that all of a batch are in flight at once
  const int qq = own ? q : 0;
  double hv[NB];
  auto load_col = [&](int j) {  // H_lj, l <= j, entry q
#pragma unroll
    for (int l = 0; l < NB; ++l) hv[l] = H[((int64_t)(l <= j ? l : j) * m + j) * ss + qq];
  };
  load_col(kend - 1);
  {
    double sv[NB];
#pragma unroll
    for (int l = 0; l < NB; ++l) sv[l] = sig[(int64_t)(l < kend ? l : kend - 1) * ss + qq];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int l = 0; l < NB; ++l)
      if (own && l < kend) rhs[l * SS + q] = sv[l];
  }
#pragma unroll
  for (int l = 0; l < NB; ++l)
    if (own && l < kend) hb[l * SS + q] = hv[l];
  for (int j = kend - 1; j >= 0; --j) {
    __syncthreads();
    if (j > 0) load_col(j - 1);
    // zeta_j = R_jj^-1 rhs_j per (group, column): thread e = o + b
    if (own) zj[q] = 0.0;
    __syncthreads();
    const double* T = hb + j * SS;
    const double* r = rhs + j * SS;
    for (int e = q; e < s; e += kSB) {
      const int grp = e / g, b = e % g, o = grp * g;
      for (int a = g - 1; a >= 0; --a) {
        double acc = r[(o + a) * s + o + b];
        for (int cc = a + 1; cc < g; ++cc) acc -= T[(o + a) * s + o + cc] * zj[(o + cc) * s + o + b];
        const double piv = T[(o + a) * s + o + a];
        zj[(o + a) * s + o + b] = piv != 0.0 ? acc / piv : 0.0;
      }
    }
    __syncthreads();
    if (own) {
      zl[j * SS + q] = zj[q];  // written to zeta at the end (see hrot in gm_step_kernel)
      // rhs_l -= H_lj zeta_j, l < j: entry q = (a, b) of every block
      const int a = q / s, b = q - a * s;
      for (int l = 0; l < j; ++l) {
        double d = 0.0;
        for (int cc = 0; cc < s; ++cc) d += hb[l * SS + a * s + cc] * zj[cc * s + b];
        rhs[l * SS + q] -= d;
      }
    }
    __syncthreads();
    if (j > 0) {
#pragma unroll
      for (int l = 0; l < NB; ++l)
        if (own && l < j) hb[l * SS + q] = hv[l];
    }
  }
  __syncthreads();
  if (own)
    for (int l = 0; l < kend; ++l) zeta[(int64_t)l * ss + q] = zl[l * SS + q];
}

hipError_t launch_gm_backsub(GmCtl* ctl, int s, int kend, const double* H, const double* sig, double* zeta,
                             hipStream_t st) {
  if (s <= 8 && kend <= kGmStage)
    hipLaunchKernelGGL(gm_backsub8_kernel, dim3(1), dim3(kSB), 0, st, ctl, H, sig, zeta);
  else
    hipLaunchKernelGGL(gm_backsub_kernel, dim3(1), dim3(kSB), 0, st, ctl, H, sig, zeta);
  return hipGetLastError();
}

// ---------------------------------------------------- iterative refinement --
// From the Gram G of the FP64 residual: column norms -> scale, relative
// residuals (r0n is set on the first call), flag[0] = converged,
// flag[1] = non-finite.
__global__ __launch_bounds__(kSB) void ir_check_kernel(int s, const double* G, double* r0n, double* scale,
                                                        double* relres, int32_t* flag, double tol, int first) {
  if (tid() != 0) return;
  double m = 0.0;
  int nan = 0;
  for (int i = 0; i < s; ++i) {
    const double g = G[i * s + i];
    nan |= !isfinite(g);
    const double cn = sqrt(fmax(g, 0.0));
    if (first) r0n[i] = cn;
    scale[i] = cn;
    const double rel = r0n[i] > 0.0 ? cn / r0n[i] : 0.0;
    relres[i] = rel;
    m = fmax(m, rel);
  }
  flag[0] = (m <= tol) ? 1 : 0;
  flag[1] = nan;
}

hipError_t launch_ir_check(int s, const double* G, double* r0n, double* scale, double* relres, int32_t* flag,
                           double tol, int first, hipStream_t st) {
  hipLaunchKernelGGL(ir_check_kernel, dim3(1), dim3(kSB), 0, st, s, G, r0n, scale, relres, flag, tol, first);
  return hipGetLastError();
}

}  // namespace bkry
