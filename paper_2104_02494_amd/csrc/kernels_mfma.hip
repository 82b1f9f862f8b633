// kernels_mfma.hip -- FP64 Gram and row-product kernels on the matrix cores
// (v_mfma_f64_16x16x4f64) for block widths s = 9..32 (padded to S = 16 or
// 32 columns, the columns past s masked).
//
// These are the dense contractions of the normaliser (Definition
// "normalizer", Ch. 3; CholeskyQR2 with the Householder TSQR of Ch. 7 as the
// fallback): G = X^T Y over all n rows, and X = X C for an s x s matrix C
// (optionally with the Gram of the result).  At s = 32 the vector versions
// hold 32-column accumulators per lane and exchange every row across 16
// lanes; the matrix cores take the operands in a fixed lane layout instead.
//
// Lane layout of one 16 x 16 x 4 FP64 product D += A B (64 lanes, measured
// on gfx950): lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and
// holds D[4 v + l / 16][l % 16] in accumulator element v = 0..3.
//
// A wavefront handles tiles of rows (k-steps of 4 rows; 16 rows in the row
// product, 32 or 64 in the Gram); a workgroup of four wavefronts sweeps the
// rows grid-stride and writes one s x s partial (row-major, stride s) like
// the vector Gram kernels, so the same fixed-order reduction follows.
#include "common.hpp"
#include "internal.hpp"

namespace bkry {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kMW = kBlock / kWave;  // wavefronts per workgroup
constexpr int kTile = 16;            // rows per wavefront tile

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Entries (4 kk + lr, 16 tj + lc) of the s x s matrix C (zero outside s x s)
// for every k-step kk and tile tj, scaled by sign.  The loads read clamped
// indexes, are all issued before a scheduling barrier and are consumed
// through an empty asm, so the compiler can neither put a load under the
// bounds test nor wait for one before the next is issued: the operands cost
// one memory round trip.
template <int NK, int NT>
__device__ __forceinline__ void coeff_operand(const double* C, int s, double sign, int lr, int lc,
                                              double (&cb)[NK][NT]) {
#pragma unroll
  for (int kk = 0; kk < NK; ++kk)
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) cb[kk][tj] = C[min(4 * kk + lr, s - 1) * s + min(16 * tj + lc, s - 1)];
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int kk = 0; kk < NK; ++kk)
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) {
      double v = cb[kk][tj];
      asm volatile("" : "+v"(v));
      cb[kk][tj] = (4 * kk + lr < s && 16 * tj + lc < s) ? sign * v : 0.0;
    }
}

// Sum the wavefronts' S x S tiles (acc[ti][tj], lane layout above) into the
// workgroup's partial.  sh: kMW * S * S doubles of LDS.
// pstride: distance of consecutive workgroups' partials (0: s * s).  Safe to
// call twice in a row (the LDS is reused after a barrier).
template <int S>
__device__ __forceinline__ void mfma_gram_store(const d4 (&acc)[S / 16][S / 16], int s, double* partial,
                                                double* sh, int64_t pstride = 0) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  __syncthreads();
#pragma unroll
  for (int ti = 0; ti < S / 16; ++ti)
#pragma unroll
    for (int tj = 0; tj < S / 16; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        sh[wave * S * S + (16 * ti + 4 * v + lane / 16) * S + 16 * tj + lane % 16] = acc[ti][tj][v];
  __syncthreads();
  double* pblk = partial + (int64_t)blockIdx.x * (pstride > 0 ? pstride : (int64_t)s * s);
  for (int t = threadIdx.x; t < s * s; t += kBlock) {
    const int a = t / s, b = t % s;
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < kMW; ++w) sum += sh[w * S * S + a * S + b];
    pblk[t] = sum;
  }
}

// G partials of X^T Y (X, Y: n x s, row stride s).  A wavefront takes
// KS k-steps (4 KS rows) per sweep step and issues all their loads before
// the products, so that enough bytes are in flight; with SYM (Y == X) only
// X is loaded and only the tiles ti <= tj are formed (the rest mirrored).
template <int S, bool SYM>
__global__ __launch_bounds__(kBlock) void gram_mfma_kernel(int64_t n, int s, const double* __restrict__ X,
                                                            const double* __restrict__ Y,
                                                            double* __restrict__ partial, const int32_t* done,
                                                            const int32_t* fire) {
  constexpr int NT = S / 16, KS = SYM ? 16 : 8;
  constexpr int RW = 4 * KS;  // rows per wavefront and sweep step
  __shared__ double sh[kMW * S * S];
  if ((done && *done) || (fire && !*fire)) return;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int lr = lane / 16, lc = lane % 16;  // row within a k-step, column within a tile
  d4 acc[NT][NT];
#pragma unroll
  for (int ti = 0; ti < NT; ++ti)
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) acc[ti][tj] = d4{0.0, 0.0, 0.0, 0.0};
  const int64_t step = (int64_t)gridDim.x * kMW * RW;
  for (int64_t base = ((int64_t)blockIdx.x * kMW + wave) * RW; base < n; base += step) {
    double a[KS][NT], b[SYM ? 1 : KS][SYM ? 1 : NT];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int64_t row = base + 4 * ks + lr;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int col = 16 * t + lc;
        const bool ok = row < n && col < s;
        const int64_t k = ok ? row * s + col : 0;
        a[ks][t] = ok ? X[k] : 0.0;
        if constexpr (!SYM) b[ks][t] = ok ? Y[k] : 0.0;
      }
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int tj = 0; tj < NT; ++tj) {
          if constexpr (SYM) {
            if (tj >= ti) acc[ti][tj] = mfma(a[ks][ti], a[ks][tj], acc[ti][tj]);
          } else {
            acc[ti][tj] = mfma(a[ks][ti], b[ks][tj], acc[ti][tj]);
          }
        }
  }
  if constexpr (SYM) {
    // tile (tj, ti) = tile (ti, tj)^T: write the upper tiles, mirror in LDS
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int tj = 0; tj < NT; ++tj)
        if (tj >= ti)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = 16 * ti + 4 * v + lr, j = 16 * tj + lc;
            sh[wave * S * S + i * S + j] = acc[ti][tj][v];
            if (tj > ti) sh[wave * S * S + j * S + i] = acc[ti][tj][v];
          }
    __syncthreads();
    double* pblk = partial + (int64_t)blockIdx.x * s * s;
    for (int t = threadIdx.x; t < s * s; t += kBlock) {
      const int i = t / s, j = t % s;
      double sum = 0.0;
#pragma unroll
      for (int w = 0; w < kMW; ++w) sum += sh[w * S * S + i * S + j];
      pblk[t] = sum;
    }
  } else {
    mfma_gram_store<S>(acc, s, partial, sh);
  }
}

// X = X C in place (C: s x s FP64, stride s); with GRAM also the partials of
// the result's Gram.  Each wavefront reads its rows completely before it
// writes them, and no two wavefronts share rows.
template <int S, bool GRAM>
__global__ __launch_bounds__(kBlock) void rowmul_mfma_kernel(int64_t n, int s, double* __restrict__ X,
                                                              const double* __restrict__ C,
                                                              double* __restrict__ partial, const int32_t* gf) {
  constexpr int NT = S / 16, NK = S / 4;
  __shared__ double sh[GRAM ? kMW * S * S : 1];
  if (gf && !*gf) return;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int lr = lane / 16, lc = lane % 16;
  // B operands: C[4 kk + lr][16 tj + lc], zero outside s x s
  double cb[NK][NT];
  coeff_operand<NK, NT>(C, s, 1.0, lr, lc, cb);
  d4 g[GRAM ? NT : 1][GRAM ? NT : 1];
  if constexpr (GRAM) {
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int tj = 0; tj < NT; ++tj) g[ti][tj] = d4{0.0, 0.0, 0.0, 0.0};
  }
  constexpr int TR = GRAM ? 2 : 1;  // 16-row tiles per wavefront and sweep step (measured best)
  const int64_t step = (int64_t)gridDim.x * kMW * kTile * TR;
  for (int64_t base = ((int64_t)blockIdx.x * kMW + wave) * kTile * TR; base < n; base += step) {
    // A operands: X[tb + lc][4 kk + lr] for the tiles tb = base + 16 tr; all
    // loads of the step are issued before the products
    double xa[TR][NK];
#pragma unroll
    for (int tr = 0; tr < TR; ++tr) {
      const int64_t arow = base + kTile * tr + lc;
#pragma unroll
      for (int kk = 0; kk < NK; ++kk) {
        const int col = 4 * kk + lr;
        const bool ok = arow < n && col < s;
        xa[tr][kk] = ok ? X[ok ? arow * s + col : 0] : 0.0;
      }
    }
#pragma unroll
    for (int tr = 0; tr < TR; ++tr) {
      const int64_t tb = base + kTile * tr;
      d4 y[NT];
#pragma unroll
      for (int tj = 0; tj < NT; ++tj) {
        y[tj] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) y[tj] = mfma(xa[tr][kk], cb[kk][tj], y[tj]);
      }
      // y[tj][v] = result at row tb + 4 v + lr, column 16 tj + lc
#pragma unroll
      for (int tj = 0; tj < NT; ++tj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t row = tb + 4 * v + lr;
          const int col = 16 * tj + lc;
          if (row < n && col < s) X[row * s + col] = y[tj][v];
        }
      if constexpr (GRAM) {
        // the result tile in accumulator layout is already the operand
        // layout of k-step v (rows tb + 4 v .. + 3): rows past n are zero
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int ti = 0; ti < NT; ++ti)
#pragma unroll
            for (int tj = 0; tj < NT; ++tj) g[ti][tj] = mfma(y[ti][v], y[tj][v], g[ti][tj]);
      }
    }
  }
  if constexpr (GRAM) mfma_gram_store<S>(g, s, partial, sh);
}

// ------------------------------------------------ block CG streaming steps --
// The residual and direction updates of block CG for wide blocks, with every
// n x s times s x s product on the matrix cores (same operand layouts as
// rowmul_mfma_kernel: a 16-row tile of a block as the A operand, the s x s
// coefficients as B, the result in accumulator layout, which is also the
// layout in which the added block is loaded and the result stored).  A
// product accumulates onto the block it updates, so R - Q lambda is formed
// as R + Q (-lambda) in one chain of fused products.

// A 16-row tile tb of block Y (row stride s) as A operands (column 4 kk + lr
// of row tb + lc) and in accumulator layout (row tb + 4 v + lr, column
// 16 tj + lc); rows past n and columns past s read as zero.
template <int NK>
__device__ __forceinline__ void tile_operand(const double* __restrict__ Y, int64_t n, int s, int64_t tb, int lr,
                                             int lc, double (&a)[NK]) {
  const int64_t row = tb + lc;
#pragma unroll
  for (int kk = 0; kk < NK; ++kk) {
    const int col = 4 * kk + lr;
    const bool ok = row < n && col < s;
    a[kk] = ok ? Y[row * s + col] : 0.0;
  }
}
template <int NT>
__device__ __forceinline__ void tile_acc_load(const double* __restrict__ Y, int64_t n, int s, int64_t tb, int lr,
                                              int lc, d4 (&y)[NT]) {
#pragma unroll
  for (int tj = 0; tj < NT; ++tj)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = tb + 4 * v + lr;
      const int col = 16 * tj + lc;
      const bool ok = row < n && col < s;
      y[tj][v] = ok ? Y[row * s + col] : 0.0;
    }
}
template <int NT>
__device__ __forceinline__ void tile_acc_store(double* __restrict__ Y, int64_t n, int s, int64_t tb, int lr, int lc,
                                               const d4 (&y)[NT]) {
#pragma unroll
  for (int tj = 0; tj < NT; ++tj)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = tb + 4 * v + lr;
      const int col = 16 * tj + lc;
      if (row < n && col < s) __builtin_nontemporal_store(y[tj][v], Y + row * s + col);
    }
}
template <int NK, int NT>
__device__ __forceinline__ void tile_product_acc(const double (&a)[NK], const double (&cb)[NK][NT], d4 (&y)[NT]) {
#pragma unroll
  for (int tj = 0; tj < NT; ++tj)
#pragma unroll
    for (int kk = 0; kk < NK; ++kk) y[tj] = mfma(a[kk], cb[kk][tj], y[tj]);
}

// R~ = R - Q lambda (in place), Gram partials of R~^T R~ and, with PC, of
// R~^T M^-1 R~ at stride pstride (the same partials as cg_update_kernel).
template <int S, bool PC>
__global__ __launch_bounds__(kBlock) void cg_update_mfma_kernel(int64_t n, int s, double* __restrict__ R,
                                                                 const double* __restrict__ Q, const CgCtl* ctl,
                                                                 double* __restrict__ partial,
                                                                 const double* __restrict__ minv, int64_t pstride) {
  constexpr int NT = S / 16, NK = S / 4;
  __shared__ double sh[kMW * S * S];
  if (ctl->gate) return;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int lr = lane / 16, lc = lane % 16;
  double cb[NK][NT];
  coeff_operand<NK, NT>(ctl->lam, s, -1.0, lr, lc, cb);
  d4 g[NT][NT], g2[PC ? NT : 1][PC ? NT : 1];
#pragma unroll
  for (int ti = 0; ti < NT; ++ti)
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) {
      g[ti][tj] = d4{0.0, 0.0, 0.0, 0.0};
      if constexpr (PC) g2[ti][tj] = d4{0.0, 0.0, 0.0, 0.0};
    }
  const int64_t step = (int64_t)gridDim.x * kMW * kTile;
  for (int64_t tb = ((int64_t)blockIdx.x * kMW + wave) * kTile; tb < n; tb += step) {
    double qa[NK];
    d4 y[NT];
    tile_operand<NK>(Q, n, s, tb, lr, lc, qa);
    tile_acc_load<NT>(R, n, s, tb, lr, lc, y);
    tile_product_acc<NK, NT>(qa, cb, y);
#pragma unroll
    for (int tj = 0; tj < NT; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = tb + 4 * v + lr;
        const int col = 16 * tj + lc;
        if (row < n && col < s) R[row * s + col] = y[tj][v];
      }
    // accumulator layout = operand layout of k-step v (rows tb + 4 v ..)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double z[NT];
      if constexpr (PC) {
        const int64_t row = tb + 4 * v + lr;
        const double m = row < n ? minv[row] : 0.0;
#pragma unroll
        for (int ti = 0; ti < NT; ++ti) z[ti] = m * y[ti][v];
      }
#pragma unroll
      for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int tj = 0; tj < NT; ++tj) {
          g[ti][tj] = mfma(y[ti][v], y[tj][v], g[ti][tj]);
          if constexpr (PC) g2[ti][tj] = mfma(z[ti], y[tj][v], g2[ti][tj]);
        }
    }
  }
  if constexpr (PC) {
    mfma_gram_store<S>(g, s, partial, sh, 2 * (int64_t)s * s);
    mfma_gram_store<S>(g2, s, partial + (int64_t)s * s, sh, 2 * (int64_t)s * s);
  } else {
    mfma_gram_store<S>(g, s, partial, sh, pstride);
  }
}

// The direction update of cg_pupdate_kernel (same gating and deferred X
// update): X += P_{k-1} (lambda sigma)_{k-1} [owed] + P_k (lambda sigma)_k
// [when flushed]; P_{k+1} = M^-1 R + P_k beta into Pn (which holds P_{k-1}:
// every tile reads its P_{k-1} rows before it overwrites them).
template <int S, bool PC>
__global__ __launch_bounds__(kBlock) void cg_pupdate_mfma_kernel(int64_t n, int s, double* __restrict__ X,
                                                                  const double* __restrict__ P,
                                                                  double* __restrict__ Pn,
                                                                  const double* __restrict__ R, const CgCtl* ctl,
                                                                  const double* __restrict__ minv) {
  constexpr int NT = S / 16, NK = S / 4;
  if (ctl->suspended) return;
  const bool done = ctl->done != 0;
  const bool xk = ctl->x_pending != 0;
  const bool xin = ctl->xdef_in != 0;
  if (!xk && !xin) return;
  const bool flush = done || xin;
  const bool addk = xk && flush;
  const bool pdir = xk && !done;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int lr = lane / 16, lc = lane % 16;
  double cls[NK][NT], clp[NK][NT], cbt[NK][NT];
  if (addk) coeff_operand<NK, NT>(ctl->lamsig, s, 1.0, lr, lc, cls);
  if (xin) coeff_operand<NK, NT>(ctl->lamsig_prev, s, 1.0, lr, lc, clp);
  if (pdir) coeff_operand<NK, NT>(ctl->beta, s, 1.0, lr, lc, cbt);
  const int64_t step = (int64_t)gridDim.x * kMW * kTile;
  for (int64_t tb = ((int64_t)blockIdx.x * kMW + wave) * kTile; tb < n; tb += step) {
    double pa[NK];
    tile_operand<NK>(P, n, s, tb, lr, lc, pa);
    if (flush) {
      d4 x[NT];
      tile_acc_load<NT>(X, n, s, tb, lr, lc, x);
      if (xin) {
        double ppa[NK];
        tile_operand<NK>(Pn, n, s, tb, lr, lc, ppa);
        tile_product_acc<NK, NT>(ppa, clp, x);
      }
      if (addk) tile_product_acc<NK, NT>(pa, cls, x);
      tile_acc_store<NT>(X, n, s, tb, lr, lc, x);
    }
    if (pdir) {
      d4 r[NT];
      tile_acc_load<NT>(R, n, s, tb, lr, lc, r);
      if constexpr (PC) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t row = tb + 4 * v + lr;
          const double m = row < n ? minv[row] : 0.0;
#pragma unroll
          for (int tj = 0; tj < NT; ++tj) r[tj][v] = m * r[tj][v];
        }
      }
      tile_product_acc<NK, NT>(pa, cbt, r);
      tile_acc_store<NT>(Pn, n, s, tb, lr, lc, r);
    }
  }
}

}  // namespace

bool mfma_width(int s) { return s > 8 && s <= 32; }

hipError_t launch_gram_mfma(int64_t n, int s, const double* X, const double* Y, double* partial, int nblk,
                            const int32_t* done, const int32_t* fire, hipStream_t st) {
  if (!mfma_width(s)) return hipErrorInvalidValue;
  const bool sym = X == Y;
  if (s <= 16) {
    if (sym)
      hipLaunchKernelGGL((gram_mfma_kernel<16, true>), dim3(nblk), dim3(kBlock), 0, st, n, s, X, Y, partial, done,
                         fire);
    else
      hipLaunchKernelGGL((gram_mfma_kernel<16, false>), dim3(nblk), dim3(kBlock), 0, st, n, s, X, Y, partial, done,
                         fire);
  } else {
    if (sym)
      hipLaunchKernelGGL((gram_mfma_kernel<32, true>), dim3(nblk), dim3(kBlock), 0, st, n, s, X, Y, partial, done,
                         fire);
    else
      hipLaunchKernelGGL((gram_mfma_kernel<32, false>), dim3(nblk), dim3(kBlock), 0, st, n, s, X, Y, partial, done,
                         fire);
  }
  return hipGetLastError();
}

hipError_t launch_rowmul_mfma(int64_t n, int s, double* X, const double* C, bool gram, double* partial, int nblk,
                              const int32_t* gf, hipStream_t st) {
  if (!mfma_width(s)) return hipErrorInvalidValue;
  if (s <= 16) {
    if (gram)
      hipLaunchKernelGGL((rowmul_mfma_kernel<16, true>), dim3(nblk), dim3(kBlock), 0, st, n, s, X, C, partial, gf);
    else
      hipLaunchKernelGGL((rowmul_mfma_kernel<16, false>), dim3(nblk), dim3(kBlock), 0, st, n, s, X, C, partial, gf);
  } else {
    if (gram)
      hipLaunchKernelGGL((rowmul_mfma_kernel<32, true>), dim3(nblk), dim3(kBlock), 0, st, n, s, X, C, partial, gf);
    else
      hipLaunchKernelGGL((rowmul_mfma_kernel<32, false>), dim3(nblk), dim3(kBlock), 0, st, n, s, X, C, partial, gf);
  }
  return hipGetLastError();
}

hipError_t launch_cg_update_mfma(int64_t n, int s, double* R, const double* Q, const CgCtl* ctl, double* partial,
                                 int nblk, const double* minv, int64_t pstride, hipStream_t st) {
  if (!mfma_width(s)) return hipErrorInvalidValue;
  auto go = [&](auto S_) {
    constexpr int S = decltype(S_)::value;
    if (minv)
      hipLaunchKernelGGL((cg_update_mfma_kernel<S, true>), dim3(nblk), dim3(kBlock), 0, st, n, s, R, Q, ctl, partial,
                         minv, pstride);
    else
      hipLaunchKernelGGL((cg_update_mfma_kernel<S, false>), dim3(nblk), dim3(kBlock), 0, st, n, s, R, Q, ctl,
                         partial, minv, pstride);
  };
  if (s <= 16)
    go(std::integral_constant<int, 16>{});
  else
    go(std::integral_constant<int, 32>{});
  return hipGetLastError();
}

hipError_t launch_cg_pupdate_mfma(int64_t n, int s, double* X, const double* P, double* Pn, const double* R,
                                  const CgCtl* ctl, int nblk, const double* minv, hipStream_t st) {
  if (!mfma_width(s)) return hipErrorInvalidValue;
  auto go = [&](auto S_) {
    constexpr int S = decltype(S_)::value;
    if (minv)
      hipLaunchKernelGGL((cg_pupdate_mfma_kernel<S, true>), dim3(nblk), dim3(kBlock), 0, st, n, s, X, P, Pn, R, ctl,
                         minv);
    else
      hipLaunchKernelGGL((cg_pupdate_mfma_kernel<S, false>), dim3(nblk), dim3(kBlock), 0, st, n, s, X, P, Pn, R,
                         ctl, minv);
  };
  if (s <= 16)
    go(std::integral_constant<int, 16>{});
  else
    go(std::integral_constant<int, 32>{});
  return hipGetLastError();
}

}  // namespace bkry
