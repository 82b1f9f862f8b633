/*
 * bkry.h -- C ABI of the MI355X block Krylov library (libbkry.so).
 *
 * Solves A X = B for a sparse n x n matrix A in CSR form and p right-hand
 * sides (the block system of Ch. 3, "A General Block Krylov Framework", of
 * N.-A. Dreier, "Hardware-Oriented Krylov Methods for High-Performance
 * Computing", arXiv 2104.02494), over a chosen *-subalgebra S of R^{p x p}.
 *
 * Conventions shared by every entry point:
 *  - Pointers are DEVICE pointers (memory of the handle's device) unless a
 *    comment marks them [host].  The caller owns every buffer it passes; the
 *    library owns only its internal workspace, which lives as long as the
 *    handle.
 *  - Block vectors are n x p, row-major ("row-interleaved": element (i,j) at
 *    i*p + j), FP64 unless the name says _f32; 16-byte aligned base pointers.
 *  - CSR is 0-based with int32 row pointers and column indices, columns
 *    sorted or not, nnz < 2^31.  Kernels never read outside [0, nnz) or
 *    outside the n rows of a block even for malformed index data; a column
 *    index outside [0, n) makes the call fail with BKRY_E_INVALID (reported
 *    by the solvers, and by bkry_last_error after a bkry_synchronize for the
 *    asynchronous kernels).
 *  - 1 <= p <= 32.  Every call is ordered on the handle's stream.  bkry_spmm,
 *    bkry_bdot, bkry_tsqr and bkry_sddmm are asynchronous; the solvers and
 *    bkry_csr_transpose return when their result is complete.
 *  - Every function returns a status code; no C++ exception crosses the ABI.
 *    The last failure's message is available from bkry_last_error.
 *  - Results are deterministic: reductions run in a fixed order, with no
 *    floating-point atomics, so repeated calls give identical bits.
 */
#ifndef BKRY_H
#define BKRY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define BKRY_OK 0
#define BKRY_NOT_CONVERGED 1 /* iteration cap reached; X holds the last iterate, info is valid */
#define BKRY_E_INVALID (-1)  /* bad size, null pointer, p % q != 0, p > 32, bad CSR index */
#define BKRY_E_BREAKDOWN (-2) /* a Cholesky pivot of alpha or rho was not positive (A not SPD,
                                 or a rank-deficient residual without re-orthonormalisation) */
#define BKRY_E_NONFINITE (-3) /* a non-finite value appeared in the block coefficients */
#define BKRY_E_HIP (-4)       /* HIP runtime error */
#define BKRY_E_ALLOC (-5)     /* device memory allocation failed */

/* *-subalgebras (Definitions "elementary *-subalgebras" and "Relevant
 * *-subalgebras", Ch. 3):
 *   BKRY_PARALLEL  diagonal matrices, <X,Y> = diag(X^T Y)  (columns independent);
 *   BKRY_GLOBAL    multiples of I, <X,Y> = tr(X^T Y)/p * I;
 *   BKRY_BLOCK     all p x p matrices, <X,Y> = X^T Y;
 *   BKRY_HYBRID    block-parallel with q contiguous column groups of width p/q,
 *                  <X,Y> = blockdiag(X_1^T Y_1, ..., X_q^T Y_q);
 *   BKRY_BLOCK_GLOBAL  block-global, q contiguous column groups of width g = p/q,
 *                  <X,Y> = I_q (x) (1/q) sum_i X_i^T Y_i; its normaliser is the
 *                  QR of the stacked [X_1; ...; X_q] = Q rho with Y_i = sqrt(q) Q_i
 *                  and N = I_q (x) rho / sqrt(q).  q = 1 is BKRY_BLOCK and q = p
 *                  is BKRY_GLOBAL (the call runs those).                     */
#define BKRY_PARALLEL 0
#define BKRY_GLOBAL 1
#define BKRY_BLOCK 2
#define BKRY_HYBRID 3
#define BKRY_BLOCK_GLOBAL 4

/* arithmetic of a CG solve */
#define BKRY_F64 0    /* everything in FP64 */
#define BKRY_F32_IR 1 /* FP32 inner block CG (SpMM, BDOT, BAXPY, TSQR tiles in FP32,
                         p x p algebra and TSQR R-combine in FP64) inside FP64
                         iterative refinement on the true residual */

typedef struct bkry_handle_s* bkry_handle;

typedef struct {
  int32_t kind; /* BKRY_PARALLEL / GLOBAL / BLOCK / HYBRID / BLOCK_GLOBAL */
  int32_t q;    /* number of column groups for BKRY_HYBRID and BKRY_BLOCK_GLOBAL (p % q == 0);
                   ignored otherwise */
} bkry_subalg;

typedef struct {
  int64_t n;
  int64_t nnz;
  const int32_t* rowptr; /* [n+1] */
  const int32_t* colind; /* [nnz] */
  const double* val;     /* [nnz] */
} bkry_csr;

typedef struct {
  /* inputs (0 / NULL select the default) */
  double inner_tol;     /* BKRY_F32_IR: relative tolerance of each inner solve (default 1e-5) */
  int32_t max_outer;    /* BKRY_F32_IR: cap on refinement steps (default 30) */
  int32_t hist_cap;     /* capacity of hist */
  double* hist;         /* [host] per iteration: max_i relative residual of column i */
  double* relres;       /* [host] p entries: final relative column residuals (recursive) */
  double* true_relres;  /* [host] p entries: final |B_i - A X_i| / |R0_i|, recomputed in FP64 */
  /* outputs */
  int32_t iters;        /* block iterations (CG) or Arnoldi steps (GMRes), inner total for IR */
  int32_t reorth;       /* normalisations of the residual (CG) */
  int32_t outer_iters;  /* refinement steps (IR) or restart cycles (GMRes) */
  int32_t converged;    /* 1 if every column met the tolerance */
  int32_t hist_len;     /* entries written to hist */
  int32_t pad_;
  double seconds;       /* wall time of the solve */
} bkry_info;

/* Create a handle on HIP device `device` that orders all work on `stream`
 * (a hipStream_t; NULL = the null stream).  The handle is not thread-safe. */
int bkry_create(bkry_handle* h, int device, void* stream);
int bkry_destroy(bkry_handle h);
int bkry_set_stream(bkry_handle h, void* stream);
/* Wait for the handle's stream and report a pending asynchronous error. */
int bkry_synchronize(bkry_handle h);
/* Message of the last failing call on this handle (valid until the next call). */
const char* bkry_last_error(bkry_handle h);

/* Kernel timing (measurement support, not part of the method): bits 0-7 of
 * `enable` are a mask of kernel ids (bit k times id k; 0 turns timing off,
 * 0xF times all four), bits 8-15 an optional sampling stride N (time one
 * launch in N of each kernel; 0 or 1 times every launch).  The block CG
 * driver brackets each selected launch of a streaming kernel with HIP events
 * on the handle's stream and accumulates the elapsed times (each event pair
 * adds a few microseconds to the solve).  Kernel
 * ids: 0 SpMM fused with the alpha Gram partials, 1 residual update fused
 * with the Gram partials of R~ (for 0 and 1 the Gram reductions and
 * coefficient steps that follow are not included), 2 direction update
 * (X and P), 3 whole re-normalisation (TSQR, Gram, coefficients).  bkry_profile_read returns the total milliseconds and
 * the number of timed launches of one kernel id, optionally resetting them. */
int bkry_profile(bkry_handle h, int enable);
int bkry_profile_read(bkry_handle h, int32_t kernel, double* total_ms, int64_t* launches, int32_t reset);

/* Matrix format that the SpMM streams (measurement and testing support; the
 * arithmetic is the same): BKRY_FMT_AUTO (default) lets the solvers stream a
 * padded row-major copy of A (ELL: every row padded to the longest row,
 * rounded up to a multiple of 2, 4 or 8 entries by p), built in the handle's
 * workspace at the start of each solve, when that copy costs at most 25 %
 * more bytes per product than CSR, and streams CSR otherwise and in
 * bkry_spmm; BKRY_FMT_CSR always streams CSR; BKRY_FMT_ELL always streams
 * the ELL copy (bkry_spmm and bkry_spmm_f32 then build it on every call and
 * return when it is built).  bkry_spmm and bkry_spmm_f32 sum each row's
 * entries in CSR order in either format, so their results are bit-identical
 * across formats.  The solvers' ELL copy holds each row's first diagonal
 * entry in slot 0 (the fused product and Gram reads a row's own values from
 * that entry's gather) and the other entries in CSR order, so a solve through
 * it agrees with a CSR solve to rounding, not bit for bit. */
#define BKRY_FMT_AUTO 0
#define BKRY_FMT_CSR 1
#define BKRY_FMT_ELL 2
int bkry_set_spmm_format(bkry_handle h, int32_t format);

/* BOP (Ch. 3, Performance Analysis): Y = A X for n x p blocks.  Each output
 * entry is summed over the row's non-zeros in storage order. */
int bkry_spmm(bkry_handle h, const bkry_csr* A, int32_t p, const double* X, double* Y);
/* FP32 BOP with FP32 accumulation (the inner kernel of BKRY_F32_IR). */
int bkry_spmm_f32(bkry_handle h, int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colind,
                  const float* val, int32_t p, const float* X, float* Y);

/* BDOT (Ch. 3, block inner product): G = <X, Y>_S, a p x p row-major device
 * array; entries outside the subalgebra's pattern are zero. */
int bkry_bdot(bkry_handle h, int64_t n, int32_t p, bkry_subalg S, const double* X, const double* Y, double* G);
/* FP32 BDOT with FP32 accumulation inside each workgroup; G in FP64. */
int bkry_bdot_f32(bkry_handle h, int64_t n, int32_t p, bkry_subalg S, const float* X, const float* Y, double* G);

/* bkry_bdot for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops): the same kernels and the same result,
 * bit for bit, but the partial Grams, slice sums and reduction counter live
 * in a fixed 5 MiB scratch array per GPU (held until the process ends)
 * instead of the handle's workspace, so the call allocates nothing (the
 * handle must have been created beforehand).  Every call on one GPU shares
 * that GPU's array: calls that overlap on one GPU (several handles or
 * streams) race and must be serialised by the caller.  The counter is
 * cleared by a kernel on each call.  Asynchronous on the handle's stream.
 * BKRY_E_INVALID if the call would need more scratch than the array holds
 * (not reachable for p <= 32). */
int bkry_bdot_noalloc(bkry_handle h, int64_t n, int32_t p, bkry_subalg S, const double* X, const double* Y,
                      double* G);

/* Normaliser / S-QR decomposition (Definition "normalizer", Ch. 3; TSQR,
 * Ch. 7): X = Q R with <Q,Q>_S = I and R in S upper triangular per S-block,
 * diag(R) >= 0; Q overwrites X, R (p x p) goes to device memory.  Block and
 * hybrid: CholeskyQR2 by default (R1 = chol(X^T X) per group, Y = X R1^-1,
 * R2 = chol(Y^T Y), Q = Y R2^-1, R = R2 R1); the second pass is skipped when
 * Y^T Y is already within rounding of I (Q = Y, R = R1).  When the first
 * Cholesky fails or its pivots spread by more than 1e6 within a group (X
 * near rank-deficient), or Y^T Y is not near I, a Householder tall-skinny QR
 * (tile QRs, a tree of R combines, Q formation) runs instead, on X or on Y
 * with R = R_householder R1.  All of this is decided on the device.
 * For full-rank X the result is the unique QR with diag(R) > 0 up to
 * rounding.  Block-global: the same QR of the q stacked column groups.
 * Parallel normalises columns and global scales by |X|_F / sqrt(p).
 * Rank-deficient X is allowed: Q is still S-orthonormal.
 * Requires n >= p (block/global) or n >= p/q (hybrid). */
int bkry_tsqr(bkry_handle h, int64_t n, int32_t p, bkry_subalg S, double* X_inout_Q, double* R);

/* Block CG with adaptive residual re-orthonormalisation (Algorithm "BCG
 * Method with Adaptive Residual Re-Orthonormalization", Ch. 4) for SPD A,
 * without preconditioner.  X holds X0 on entry and the solution on exit.
 * Stops when max_i |R_i| / |R0_i| <= tol (recursive residual) or after maxit
 * iterations.  The residual is re-normalised in iteration k when
 * eta * kappa_D(alpha_k) * sqrt(eps) > 1 (eps of the working precision);
 * eta = 0 never, eta = INFINITY always.  prec = BKRY_F64 or BKRY_F32_IR.
 * With BKRY_F32_IR an inner FP32 solve that breaks down or meets non-finite
 * values ends the refinement with that status if it made no progress or the
 * previous inner solve failed the same way; a refinement that ends
 * unconverged after such an inner failure returns its status instead of
 * BKRY_NOT_CONVERGED.  info [host] may be NULL. */
int bkry_cg_solve(bkry_handle h, const bkry_csr* A, int32_t p, bkry_subalg S, const double* B, double* X,
                  double tol, int32_t maxit, double eta, int32_t prec, bkry_info* info);

/* Preconditioned block CG (the same algorithm with a preconditioner M: the
 * search directions start from and are updated with Z = M^-1 R-bar, and
 * rho = <Z, R-bar>_S) for a diagonal SPD M given by minv [device, n
 * doubles, 8-byte aligned, caller-owned]: minv[i] = (M^-1)_ii > 0.  FP64;
 * otherwise as bkry_cg_solve (the stopping test uses the unpreconditioned
 * residual R).  Non-finite or non-positive entries of minv are not checked
 * and end in BKRY_E_BREAKDOWN or BKRY_E_NONFINITE. */
int bkry_pcg_solve(bkry_handle h, const bkry_csr* A, int32_t p, bkry_subalg S, const double* B, double* X,
                   const double* minv, double tol, int32_t maxit, double eta, bkry_info* info);

/* Multicolour ordering for the SSOR preconditioner: colors[i] [device, n
 * int32, caller-owned] = the greedy colouring of the graph of A in order of
 * decreasing prio[i] [device, n uint32] (ties: smaller row first), computed by
 * parallel Jones-Plassmann rounds; *ncolors [host] = number of colours.  The
 * pattern of A must be symmetric (the SSOR calls reject a colouring that
 * leaves two coupled rows in one colour).  Values of A are not read.
 * BKRY_E_INVALID for a column index outside [0, n) or more than 4096
 * colours. */
int bkry_color(bkry_handle h, const bkry_csr* A, const uint32_t* prio, int32_t* colors, int32_t* ncolors);

/* Multicolour SSOR preconditioner (the SSOR-type preconditioners of the
 * experiments, Ch. 4): with the rows ordered by colour and A = L + D + U in
 * that order (L: entries whose column has a smaller colour),
 * M = (D + omega L) D^-1 (D + omega U) / (omega (2 - omega)), SPD for SPD A and
 * 0 < omega < 2.  Z = M^-1 R by a forward and a backward colour sweep (one
 * launch per colour and sweep).  R, Z [device, n x p row-major FP64, no
 * aliasing]; colors [device, n int32] as from bkry_color.  BKRY_E_INVALID if
 * two coupled rows share a colour, a colour is outside [0, 4096), a diagonal
 * entry is missing or not positive, or omega is outside (0, 2). */
int bkry_ssor_apply(bkry_handle h, const bkry_csr* A, int32_t p, const int32_t* colors, double omega,
                    const double* R, double* Z);

/* Block CG with adaptive residual re-orthonormalisation preconditioned by the
 * multicolour SSOR of bkry_ssor_apply (colors, omega as there); FP64;
 * otherwise as bkry_pcg_solve.  The stopping test uses the unpreconditioned
 * residual. */
int bkry_pcg_ssor_solve(bkry_handle h, const bkry_csr* A, int32_t p, bkry_subalg S, const double* B, double* X,
                        const int32_t* colors, double omega, double tol, int32_t maxit, double eta,
                        bkry_info* info);

/* Block CG with one reduction per iteration (Algorithm "BCG with One
 * Reduction", Ch. 8): the same iteration as bkry_cg_solve in exact
 * arithmetic, with U = A R-bar formed right after the residual update,
 * Q = A P carried by Q = U + Q beta and alpha by alpha' = delta -
 * beta^T alpha beta (delta = <R-bar, U>_S), so that the residual norms, rho
 * and delta of an iteration share one reduction.  Needs two more n x p
 * blocks of workspace than bkry_cg_solve.  FP64, M = I; arguments, stopping
 * test, re-normalisation rule and info as bkry_cg_solve (prec is FP64). */
int bkry_cg1r_solve(bkry_handle h, const bkry_csr* A, int32_t p, bkry_subalg S, const double* B, double* X,
                    double tol, int32_t maxit, double eta, bkry_info* info);

/* Gropp's block CG (Algorithm "Gropp's BCG", Ch. 8): the iteration of
 * bkry_pcg_solve (minv [device, n doubles, 8-byte aligned] = diag(M^-1) of a
 * diagonal SPD preconditioner) or, with minv = NULL, of bkry_cg_solve, with
 * Q = A P carried by the recurrence Q = U + Q beta (U = A Z) and Z = M^-1
 * R-bar by Z = Z - M^-1 Q lambda (Z = M^-1 R-bar formed anew after a
 * re-normalisation), so that U = A Z no longer waits for the reduction of
 * rho' (the overlap the method is built for).  Needs one (M = I) or two more
 * n x p blocks of workspace than bkry_cg_solve.  FP64; arguments, stopping
 * test, re-normalisation rule and info as bkry_cg_solve. */
int bkry_gropp_solve(bkry_handle h, const bkry_csr* A, int32_t p, bkry_subalg S, const double* B, double* X,
                     const double* minv, double tol, int32_t maxit, double eta, bkry_info* info);

/* Jacobi preconditioner of bkry_pcg_solve: minv[i] = 1 / A_ii [device, n
 * doubles, caller-owned].  BKRY_E_INVALID if a row has no diagonal entry or
 * its diagonal is not positive and finite (duplicates are summed).
 * Synchronous. */
int bkry_jacobi_minv(bkry_handle h, const bkry_csr* A, double* minv);

/* Block BiCGStab with adaptive residual re-orthonormalisation (Algorithm
 * "BBiCGStab with Adaptive Residual Re-Orthonormalization", Ch. 6) for
 * general (non-symmetric) A, without preconditioner; shadow residual R~0 =
 * the initial (normalised) residual.  Coefficient systems are solved per
 * S-block by LU with partial pivoting; omega minimises the Frobenius norm of
 * the transformed residual.  The residual is re-normalised in iteration k
 * when eta * kappa_D(<R_k, R_k>_S) * sqrt(eps) > 1 (eta = 0 never,
 * INFINITY always).  Stops when max_i |R_i| / |R0_i| <= tol (recursive
 * residual R^ sigma) or after maxit iterations; info->true_relres holds the
 * FP64 true residual.  When the recursion meets tol but the FP64 true
 * residual does not (BiCGStab's residual gap), the iteration is restarted
 * from the current X with a new normalised and shadow residual and the first
 * start's stopping denominators, at most 10 times within maxit iterations in
 * all (info->outer_iters = restarts); info->converged (and BKRY_OK) means
 * the FP64 true residual meets tol.  A zero pivot or <U, U>_F = 0 is
 * BKRY_E_BREAKDOWN.
 * FP64; X holds X0 on entry; info [host] may be NULL. */
int bkry_bicgstab_solve(bkry_handle h, const bkry_csr* A, int32_t p, bkry_subalg S, const double* B, double* X,
                        double tol, int32_t maxit, double eta, bkry_info* info);

/* Restarted block GMRes (Algorithm "Block GMRes Method", Ch. 5): block
 * Arnoldi with classical Gram-Schmidt applied twice (Algorithm "classical
 * Gram-Schmidt", Ch. 9) and TSQR normalisation of each new block, generalised
 * Givens rotations on the block Hessenberg matrix, restart length `restart`.
 * maxit counts Arnoldi steps over all cycles.  Stops when every column's
 * relative residual is <= tol (Frobenius form for BKRY_GLOBAL).  Requires
 * n >= p. */
int bkry_gmres_solve(bkry_handle h, const bkry_csr* A, int32_t p, bkry_subalg S, const double* B, double* X,
                     double tol, int32_t maxit, int32_t restart, bkry_info* info);

/* Restarted block GMRes as bkry_gmres_solve, with the pipelined Gram-Schmidt
 * orthogonalisation of window r >= 1 (Algorithm "Pipelined Gram-Schmidt
 * Orthogonalization", Ch. 9) in every Arnoldi step instead of classical
 * Gram-Schmidt applied twice: the inner product with basis block i is taken
 * after the updates with blocks 0 .. i - r - 1 (window min(r, k) in step k;
 * r >= restart - 1 is classical Gram-Schmidt applied once).  Each pass over W
 * subtracts up to min(r, 4 / 2 / 1 for p <= 8 / 16 / 32) updates and takes
 * the inner products of as many blocks, so a step moves about half the block
 * traffic of the default at large r; stability decreases as r grows (the
 * text's trade-off).  BKRY_E_INVALID for r < 1; otherwise as bkry_gmres_solve. */
int bkry_gmres_pipelined_solve(bkry_handle h, const bkry_csr* A, int32_t p, bkry_subalg S, const double* B,
                               double* X, double tol, int32_t maxit, int32_t restart, int32_t r, bkry_info* info);

/* Sampled product on the pattern of A: out_val[k] = alpha * sum_c L[i][c] X[j][c]
 * for the k-th stored entry (i, j).  With L the adjoint solution and
 * alpha = -1 this is the gradient of a loss with respect to the values of A. */
int bkry_sddmm(bkry_handle h, const bkry_csr* pattern, int32_t p, double alpha, const double* L, const double* X,
               double* out_val);

/* Transpose of a square CSR matrix (counting sort; rows of A^T list their
 * columns in ascending order).  rowptrT [n+1], colindT/valT/permT [nnz];
 * permT[t] is the position in A of entry t of A^T.  Synchronous. */
int bkry_csr_transpose(bkry_handle h, const bkry_csr* A, int32_t* rowptrT, int32_t* colindT, double* valT,
                       int32_t* permT);

#ifdef __cplusplus
}
#endif
#endif /* BKRY_H */
