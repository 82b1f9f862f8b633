// internal.hpp -- host-side interfaces between the translation units of
// libbkry.so (kernel launchers, device control blocks, workspace).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace bkry {

constexpr int kMaxS = 32;
constexpr int kBlock = 256;  // threads per workgroup of the streaming kernels

enum Kind { PARALLEL = 0, GLOBAL = 1, BLOCK = 2, HYBRID = 3, BGLOBAL = 4 };

// Subalgebra in the library's terms: group width g (block: s, hybrid and
// block-global: s/q, parallel and global: 1) plus the kind (global differs
// from parallel, and block-global from hybrid, only in the projection and the
// normaliser).
struct Sub {
  int kind;
  int s;
  int g;
};

// Target of the Gram reductions: the producer writes one s x s partial per
// workgroup; the reduction kernel (<= kMaxSlices workgroups per batch slice)
// writes slice sums to gpart and the final FP64 Gram to G.  cnt holds one
// zeroed counter per batch slice (left zero).
struct Red {
  double* G;
  double* gpart;
  uint32_t* cnt;
};
constexpr int kCntStride = 64;    // counters reserved per batch slice
constexpr int kMaxBatch = 256;    // batch slices of one launch
constexpr int kMaxSlices = 64;    // reduction workgroups per batch slice
inline size_t red_gpart_count(int nblk, int s) {
  (void)nblk;
  return (size_t)kMaxSlices * s * s;
}

// A sparse matrix as the kernels see it: CSR, plus optionally a padded
// row-major copy (ELL, row width ell_w > 0) that the SpMM then reads instead.
struct CsrView {
  int64_t n, nnz;
  const int32_t* rowptr;
  const int32_t* colind;
  const void* val;                  // double or float, by the launcher's T
  int ell_w = 0;                    // 0: no ELL copy
  const int32_t* ell_col = nullptr; // [n * ell_w], padding -1
  const void* ell_val = nullptr;    // [n * ell_w], element type of val
  bool ell_diag0 = false;           // slot 0 of every ELL row holds its diagonal entry
};

// Device control block of a block CG solve.  The integer header is read back
// by the host to steer the loop; everything else stays on the device.
struct CgCtl {
  int32_t done;       // 1: the solve has ended (converged, cap, breakdown)
  int32_t status;     // 0, or -2 breakdown, -3 non-finite
  int32_t converged;
  int32_t fire;       // re-orthonormalise in this iteration
  int32_t x_pending;  // the X update of this iteration is still due
  int32_t iters;
  int32_t nreorth;
  int32_t maxit;
  int32_t s, kind, g, hist_cap;
  int32_t bad_index;  // a CSR column index was out of range
  int32_t gate;       // streaming kernels skip while set (done or suspended)
  int32_t suspended;  // the iteration waits for a re-normalisation launched by the host
  int32_t dynamic;    // the re-orthonormalisation test is decided per iteration
  int32_t kd_jacobi;  // iterations whose kappa_D needed the Jacobi eigenvalues
  int32_t xdef_in;    // this iteration's direction update owes X the previous P's term
  int32_t xdef_pend;  // after this iteration's update, P's term is owed to X
  int32_t lam_iter;   // one-reduction CG: iteration whose lambda was computed last (-1: none)
  int32_t pad_[4];
  double tol, eta, sqrt_eps, pad2_;
  double r0n[kMaxS];
  double relres[kMaxS];
  double alpha[kMaxS * kMaxS];
  double rho[kMaxS * kMaxS];
  double lam[kMaxS * kMaxS];
  double lamsig[kMaxS * kMaxS];
  double sigma[kMaxS * kMaxS];
  double gamma[kMaxS * kMaxS];
  double beta[kMaxS * kMaxS];
  float lam_f[kMaxS * kMaxS];
  float lamsig_f[kMaxS * kMaxS];
  float beta_f[kMaxS * kMaxS];
  double lamsig_prev[kMaxS * kMaxS];  // lambda sigma of the iteration whose X term is owed
  float lamsig_prev_f[kMaxS * kMaxS];
};
constexpr int kCtlHeaderInts = 24;

// Coefficients of block BiCGStab beside its CgCtl (which holds the header,
// sigma, gamma, lambda sigma, r0n and relres): a = <R~0, Q^>_S of the
// iteration, and the s x s multipliers of its block combinations.
struct BcAux {
  double a[kMaxS * kMaxS];
  double neglam[kMaxS * kMaxS];  // -lambda
  double omsig[kMaxS * kMaxS];   // omega sigma
  double negomI[kMaxS * kMaxS];  // -omega I
  double pbeta[kMaxS * kMaxS];   // beta
  double qbeta[kMaxS * kMaxS];   // -omega beta
  double omega, pad_[7];
};

// Device control block of a block GMRes solve (per-cycle arrays live in
// separate workspace buffers: H, sig, Om, zeta).
struct GmCtl {
  int32_t done;       // cycle finished (converged or step cap)
  int32_t status;
  int32_t converged;
  int32_t kend;       // steps taken in the current cycle
  int32_t total;      // Arnoldi steps over all cycles
  int32_t maxit;
  int32_t s, kind, g, m, hist_cap, bad_index;
  int32_t pad_[4];
  double tol, r0F, pad2_[2];
  double r0n[kMaxS];
};

// Work that the last workgroup of a Gram reduction does once G is complete:
// nothing, or the coefficient step of block CG that consumes this Gram
// (EPI_CG_ALPHA after the SpMM, EPI_CG_RHO after the residual update), so
// that no separate launch is needed.  The CG epilogues gate themselves on
// the control block (the reduction's gate / fire arguments are then unused).
// EPI_CG_RHO_M: the residual update of the preconditioned CG, whose
// partials hold two Grams per workgroup ([R~^T R~ | R~^T M^-1 R~], 2*s*s
// entries); red.G then receives both.
// EPI_CG_1R: the one reduction of an iteration of the one-reduction block CG,
// partials [R^T R | R^T A R] (2*s*s entries) written by two producers (the
// fused update pass and the SpMM); its epilogue does the whole coefficient
// step.
enum EpiKind { EPI_NONE = 0, EPI_CG_ALPHA = 1, EPI_CG_RHO = 2, EPI_CG_RHO_M = 3, EPI_CG_1R = 4 };
struct Epi {
  int kind = EPI_NONE;
  CgCtl* ctl = nullptr;
  double* hist = nullptr;  // EPI_CG_RHO: per-iteration residual history (device)
};

// Reduce `batch` slices of nblk partials (T = double or float) into red.G;
// run only if *gate == 0 and *fire != 0 (null: no condition).
hipError_t launch_reduce(int s, const void* partial, bool f32, int nblk, int batch, Red red, const int32_t* gate,
                         const int32_t* fire, Epi epi, hipStream_t st);

// ---------------------------------------------------------------- grids ----
// Number of workgroups of the streaming block kernels for n rows of width s
// (a multiple of 8 so that the XCD-contiguous row mapping is a bijection).
int stream_grid(int64_t n, int s, int elem_bytes);

// ------------------------------------------------------- block kernels ----
// SpMM modes: 0 Y = A X; 1 also the Gram X^T Y (X the own rows) into red.G;
// 2 Y = B - A X and the Gram Y^T Y into red.G.  partial: nblk*s*s of T.
// ev_after (optional): recorded on st right after the streaming kernel,
// before its reduction (kernel timing).
// gram_slot / ngram: the Gram partial of workgroup b goes to
// partial + (b * ngram + gram_slot) * s*s (several Grams per partial, the
// others written by other kernels); the reduction then reads ngram Grams per
// partial from `partial`.  nblk may be lowered to what the kernel keeps
// resident (spmm_grid gives the value used).
template <typename T>
hipError_t launch_spmm(const CsrView& A, int s, const T* X, T* Y, const T* B, int mode, T* partial,
                       int nblk, Red red, int32_t* bad, const int32_t* gate, hipStream_t st, Epi epi = Epi{},
                       hipEvent_t ev_after = nullptr, int gram_slot = 0, int ngram = 1);
template <typename T>
int spmm_grid(const CsrView& A, int s, int mode, int nblk);

// Gram X_j^T Y for X_j = X + j*n*s, j < nx, into red.G + j*s*s (batched:
// partial, gpart and counters are per slice).  Optional second gate `fire`:
// run only if *fire != 0.
template <typename T>
hipError_t launch_gram(int64_t n, int s, const T* X, int nx, const T* Y, T* partial, int nblk, Red red,
                       const int32_t* gate, hipStream_t st, const int32_t* fire = nullptr);

// FP64 Gram X^T Y and row product X = X C on the matrix cores (widths
// 8 < s <= 32; kernels_mfma.hip); same partial layout as the vector kernels
// (one s x s partial per workgroup, nblk workgroups).
bool mfma_width(int s);
// Gropp's block CG (FP64): the residual pass with the Z recurrence and the
// Grams R~^T R~, Z^T R~ (stride 2 s^2), and the direction pass (X update as
// the block CG direction update, P_{k+1} = Z + P_k beta into Pn, Q = U + Q
// beta, Gram partials of P_{k+1}^T Q_{k+1}).  Partials only: the caller
// reduces them.
hipError_t launch_gropp_update(int64_t n, int s, double* R, const double* Q, double* Z, const CgCtl* ctl,
                               double* partial, int nblk, const double* minv, hipStream_t st);
hipError_t launch_gropp_dir(int64_t n, int s, double* X, const double* P, double* Pn, const double* Z,
                            const double* U, double* Q, const CgCtl* ctl, double* partial, int nblk, hipStream_t st);
// Widths whose CG streaming steps (residual and direction updates, the
// SpMM's alpha Gram) run on the matrix cores in FP64.
inline bool wide_mfma(int s) { return s > 16 && s <= 32; }
hipError_t launch_cg_update_mfma(int64_t n, int s, double* R, const double* Q, const CgCtl* ctl, double* partial,
                                 int nblk, const double* minv, int64_t pstride, hipStream_t st);
hipError_t launch_cg_pupdate_mfma(int64_t n, int s, double* X, const double* P, double* Pn, const double* R,
                                  const CgCtl* ctl, int nblk, const double* minv, hipStream_t st);
hipError_t launch_gram_mfma(int64_t n, int s, const double* X, const double* Y, double* partial, int nblk,
                            const int32_t* done, const int32_t* fire, hipStream_t st);
hipError_t launch_rowmul_mfma(int64_t n, int s, double* X, const double* C, bool gram, double* partial, int nblk,
                              const int32_t* gf, hipStream_t st);

// CG residual update R~ = R - Q lambda (in place in R) and the Gram of R~ into
// red.G.  With minv (the diagonal of M^-1, n entries; FP64 only), also the
// Gram R~^T M^-1 R~ (partials of 2*s*s entries, epi kind EPI_CG_RHO_M).
template <typename T>
hipError_t launch_cg_update(int64_t n, int s, T* R, const T* Q, const CgCtl* ctl, T* partial, int nblk, Red red,
                            hipStream_t st, Epi epi = Epi{}, hipEvent_t ev_after = nullptr,
                            const double* minv = nullptr);

// CG direction update.  X receives the terms P_k (lambda sigma)_k every other
// iteration, two at a time (P_{k-1} and P_k), and all owed terms once the
// solve has ended; unless it has ended, Pn = R + P beta, where Pn holds
// P_{k-1} on entry (read first, row by row) and P_{k+1} on exit.
// With minv (diagonal of M^-1), Pn = M^-1 R + P beta.
template <typename T>
hipError_t launch_cg_pupdate(int64_t n, int s, T* X, const T* P, T* Pn, const T* R, const CgCtl* ctl,
                             hipStream_t st, const double* minv = nullptr);

// Z = M^-1 R for the diagonal M^-1 = diag(minv); runs only if *done == 0
// and (fire null or *fire != 0).
template <typename T>
hipError_t launch_row_scale(int64_t n, int s, const double* minv, const T* R, T* Z, const int32_t* done,
                            const int32_t* fire, hipStream_t st);

// X = X C in place (C s x s FP64); with gram, also the Gram X^T X of the
// result into red.G.  Runs only if gf is null or *gf != 0.
template <typename T>
hipError_t launch_rowmul(int64_t n, int s, T* X, const double* C, bool gram, T* partial, int nblk, Red red,
                         const int32_t* gf, hipStream_t st);

// Pipelined Gram-Schmidt pass (see pgs_pass_kernel): updates u0 .. u0+nu-1
// of W with the basis blocks of V and coefficients C (block u at C + u s^2),
// Gram partials of V_{g0+j}^T W for j < ng taken before update j.  At most
// pgs_max_updates(s) updates per pass; nblk as for launch_gram.
int pgs_max_updates(int s);
hipError_t launch_pgs_pass(int64_t n, int s, const double* V, double* W, int u0, int nu, const double* C, int g0,
                           int ng, double* partial, int nblk, const int32_t* done, hipStream_t st);

// Y = X C (+ Y if accumulate) for a list of blocks: Y op= sum_j X_j C_j,
// X_j = X + j*n*s, C_j s x s FP64 at C + j*s*s; sign = +1 or -1.
template <typename T>
hipError_t launch_block_combine(int64_t n, int s, const T* X, int nx, const double* C, double sign, T* Y,
                                const int32_t* done, hipStream_t st);

// Column scaling used by the parallel / global normalisers: Y[i][j] = X[i][j] / d[j]
// where d[j] > 0, else e_(zero_row(j)) with zero_row = 0 (parallel) or j (global).
template <typename T>
hipError_t launch_colscale(int64_t n, int s, const T* X, T* Y, const double* d, int global_kind,
                           const int32_t* gate_done, const int32_t* gate_fire, hipStream_t st);

hipError_t launch_cast_scale_f32(int64_t n, int s, const double* R, const double* scale, float* out,
                                 hipStream_t st);
hipError_t launch_accum_scaled(int64_t n, int s, const float* D, const double* scale, double* X,
                               hipStream_t st);
hipError_t launch_cast_f32(int64_t count, const double* in, float* out, hipStream_t st);

template <typename T>
hipError_t launch_sddmm(const CsrView& A, int s, double alpha, const T* L, const T* X, T* out, int32_t* bad,
                        hipStream_t st);

// ----------------------------------------------------- small algebra ----
// Single-workgroup kernels on the p x p coefficients (FP64).
hipError_t launch_project(const double* G, double* out, Sub sub, hipStream_t st);
// p[0, count) = v (a kernel, so that the call can be captured in a graph).
hipError_t launch_fill_u32(uint32_t* p, int64_t count, uint32_t v, hipStream_t st);
hipError_t launch_cg_init(CgCtl* ctl, const double* G_R0, const double* G_rho, hipStream_t st);
hipError_t launch_cg_reortho_fin(CgCtl* ctl, int s, const double* G, hipStream_t st);

// ------------------------------------------------- multicolour SSOR ----
constexpr int kMaxColors = 4096;
// The preconditioner of one solve: A (FP64 CSR), its colouring, the
// diagonal d, the rows bucketed by colour (perm[off[c] .. off[c+1]) hold the
// rows of colour c) and omega.
struct SsorPlan {
  CsrView A;
  const int32_t* colors = nullptr;
  const double* d = nullptr;
  const int32_t* perm = nullptr;
  const int32_t* off = nullptr;
  int ncolors = 0;
  int64_t count_max = 0;  // rows of the largest colour
  double omega = 1.0;
};
// One Jones-Plassmann round (state: -1 or (round << 16) | colour; more[round]
// = 1 if a row is left uncoloured; bad = 1 for a column index outside [0, n)).
hipError_t launch_jp_round(const CsrView& A, const uint32_t* prio, int32_t* state, int round, int32_t* more,
                           int32_t* bad, hipStream_t st);
hipError_t launch_jp_final(int64_t n, const int32_t* state, int32_t* colors, int32_t* ncolors, hipStream_t st);
// Colouring check (bad[0]: colour outside [0, kMaxColors); bad[1]: coupled
// rows of one colour or a bad column index; bad[2]: a row without a positive
// diagonal), diagonal d, ncolors (atomic max, zeroed by the caller) and
// colour counts (zeroed by the caller).
hipError_t launch_ssor_check(const CsrView& A, const int32_t* colors, double* d, int32_t* ncolors, int32_t* count,
                             int32_t* bad, hipStream_t st);
hipError_t launch_ssor_bucket(int64_t n, const int32_t* colors, const int32_t* count, const int32_t* ncolors,
                              int32_t* off, int32_t* cursor, int32_t* perm, hipStream_t st);
// Z = M^-1 R (Z must not alias R); skipped if *skip_a or *skip_b, or if
// need is given and *need == 0 (null pointers: no condition).
hipError_t launch_ssor_apply(const SsorPlan& m, int s, const double* R, double* Z, const int32_t* skip_a,
                             const int32_t* skip_b, const int32_t* need, hipStream_t st);
// Gram partials X^T Y into partial (stride pstride per workgroup), no
// reduction; skipped like launch_ssor_apply.
hipError_t launch_gram_partials(int64_t n, int s, const double* X, const double* Y, double* partial, int nblk,
                                int64_t pstride, const int32_t* skip_a, const int32_t* skip_b, hipStream_t st);
// R~ = R - Q lambda with the Gram partials of R~ at stride pstride, without
// the reduction (FP64).
hipError_t launch_cg_update_partials(int64_t n, int s, double* R, const double* Q, const CgCtl* ctl, double* partial,
                                     int nblk, int64_t pstride, hipStream_t st);

// One-reduction block CG.  Fused pass of iteration k (runs only if lambda^k
// was computed and the solve is live): P = R + P beta, Q = U + Q beta
// (P = R, Q = U for k = 0), for odd k X += P_old (lambda sigma)_{k-1} +
// P (lambda sigma)_k, R = R - Q lambda and, unless the residual is
// re-normalised next, the Gram partials of R into slot 0 of 2.
// mode 1: only the Gram partials of R (after a re-normalisation of iteration
// k, or unconditionally for k < 0).
// mode 2: X += P (lambda sigma) (the term an even last iteration owes X;
// runs also after the end).
hipError_t launch_cg1r_pass(int64_t n, int s, double* R, const double* U, double* P, double* Q, double* X,
                            const CgCtl* ctl, double* partial, int nblk, int k, int mode, hipStream_t st);
// After the residual was re-normalised: sigma = gamma sigma, the count, and
// the iteration resumes.
hipError_t launch_cg1r_fin(CgCtl* ctl, int s, hipStream_t st);
// Normaliser coefficients for parallel / global: from the Gram G of X, write
// the column divisors d and N (p x p) to `out_N` (gated like the CG kernels).
// N = I_q (x) rho / sqrt(q) from the g x g rho; d[j] = 1/sqrt(q).
hipError_t launch_bg_expand(const double* rho, Sub sub, double* N, double* d, const int32_t* gate_done,
                            const int32_t* gate_fire, hipStream_t st);
hipError_t launch_norm_diag(const double* G, Sub sub, double* d, double* out_N, const int32_t* gate_done,
                            const int32_t* gate_fire, hipStream_t st);

// CholeskyQR steps of the block / hybrid normaliser (plan: [0] the first
// Cholesky of X^T X succeeded, [1] the second succeeded, [2] the Householder
// TSQR must run instead).  stage 1 factors G = X^T X: R1 and Rinv = R1^-1,
// or R1 = I and plan[2] = 1; it runs only if the gates gd / gf are open, and
// otherwise clears the plan.  stage 2 (only if plan[0]) factors G = Y^T Y
// of Y = X R1^-1: Rinv = R2^-1 and N = R2 R1, or plan[2] = 1; when G is
// already within 8 s eps of the identity it sets N = R1 and clears plan[1]
// (Q = Y, no second row product).  ratio_min is
// the smallest accepted ratio of the diagonal entries of R1 within a group.
hipError_t launch_cholqr(int stage, const double* G, Sub sub, double* R1, double* Rinv, double* N, int32_t* plan,
                         double ratio_min, const int32_t* gd, const int32_t* gf, hipStream_t st);
// N = Nh R1 (block-diagonal upper triangular factors) if plan[2].
hipError_t launch_cholqr_compose(const double* Nh, const double* R1, double* N, Sub sub, const int32_t* plan,
                                 hipStream_t st);

// GMRes small kernels
hipError_t launch_gm_step(GmCtl* ctl, int s, int k, double* H, double* sig, double* Om, const double* H1,
                          const double* H2, const double* gamma, double* hist, hipStream_t st);
hipError_t launch_project_batched(const double* G, double* out, Sub sub, int batch, const int32_t* gate,
                                  hipStream_t st);
hipError_t launch_ir_check(int s, const double* G, double* r0n, double* scale, double* relres, int32_t* flag,
                           double tol, int first, hipStream_t st);
hipError_t launch_gm_backsub(GmCtl* ctl, int s, int kend, const double* H, const double* sig, double* zeta,
                             hipStream_t st);
hipError_t launch_gm_cycle_init(GmCtl* ctl, double* sig, const double* sigma0, const double* G_R,
                                int first_cycle, hipStream_t st);

// ------------------------------------------------------------ ELL copy ----
// Lanes per row of the streaming kernels for width s (element size in bytes).
int spmm_lanes_per_row(int s, int elem_bytes);
// ELL row widths are multiples of this chunk for width s.
int ell_chunk(int s, int elem_bytes);
// *wmax = longest row of A (enqueued on st; the caller reads it back).
hipError_t launch_ell_width(const CsrView& A, int32_t* wmax, hipStream_t st);
// Fill the ELL copy (row width W >= longest row) from A's CSR arrays with
// values `val` converted to T; bad column indices set *bad = 1.  nodiag not
// null: every row's first diagonal entry goes to slot 0 (the entries before
// it move up by one); a row without one keeps CSR order and sets
// *nodiag = 1 (the copy then does not qualify as diagonal first).
template <typename Tin, typename T>
hipError_t launch_ell_fill(const CsrView& A, const Tin* val, int W, int32_t* ecol, T* eval, int32_t* bad,
                           int32_t* nodiag, hipStream_t st);

// minv[i] = 1 / A_ii (FP64 values); a missing, non-positive or non-finite
// diagonal sets *bad = 1.
hipError_t launch_jacobi_minv(const CsrView& A, double* minv, int32_t* bad, hipStream_t st);

// ------------------------------------------------------ block BiCGStab ----
// Coefficient steps of block BiCGStab (single-wavefront kernels, each a no-op
// once ctl->done is set).  bc_lambda: from Gqr = [Q^T R~0 | R^T R~0] and
// Grr = R^T R: a, lambda = a^-1 <R~0, R>_S (per-S-block LU with partial
// pivoting), -lambda, lambda sigma and the re-orthonormalisation test on
// kappa_D(<R, R>_S).  bc_sigma: sigma = gamma sigma when the test fired.
// bc_omega: from G3 = [S^T U | U^T U | R~0^T U]: omega = <U, S>_F / <U, U>_F,
// beta = -a^-1 <R~0, U>_S and the combination multipliers.  bc_stop: column
// norms of R sigma from Grr, stopping test, history, iteration count.
hipError_t launch_bc_lambda(CgCtl* ctl, BcAux* aux, int s, const double* Gqr, const double* Grr, hipStream_t st);
hipError_t launch_bc_sigma(CgCtl* ctl, hipStream_t st);
hipError_t launch_bc_omega(CgCtl* ctl, BcAux* aux, const double* G3, hipStream_t st);
hipError_t launch_bc_stop(CgCtl* ctl, const double* Grr, double* hist, hipStream_t st);
// Y = A0 + X1 C1 (+ X2 C2) for n x s blocks (C: s x s FP64, device); Y may
// alias A0 but neither X.  Runs only if *done == 0 (done may be null).
// X += P (lambda sigma) + S (omega sigma), R = S - omega U, P' = R + P beta -
// Q (omega beta) in one pass (the coefficients from lamsig and x).
hipError_t launch_bc_tail(int64_t n, int s, double* X, const double* P, const double* S, const double* U,
                          const double* Q, double* R, double* Pn, const double* lamsig, const BcAux* x,
                          const int32_t* done, hipStream_t st);
// The same pass in the row-slot layout of the streaming kernels (kernels_block.hip).
hipError_t launch_bc_tail_rs(int64_t n, int s, double* X, const double* P, const double* S, const double* U,
                             const double* Q, double* R, double* Pn, const double* lamsig, const double* omsig,
                             const double* negomI, const double* pbeta, const double* qbeta, const int32_t* done,
                             hipStream_t st);
template <typename T>
hipError_t launch_lincomb(int64_t n, int s, const T* A0, const T* X1, const double* C1, const T* X2,
                          const double* C2, T* Y, const int32_t* done, hipStream_t st);

// ---------------------------------------------------------------- TSQR ----
// Workspace (bytes) needed by tsqr_run for n rows, width s, subalgebra sub.
size_t tsqr_workspace_bytes(int64_t n, Sub sub);
// Normalise X (n x s, row stride s, element T) in place; N (s x s FP64,
// device) receives the normaliser.  gate_done / gate_fire (may be null): run
// only if *gate_done == 0 and *gate_fire != 0.  plan (4 device ints, may be
// null): where the CholeskyQR path records its decisions (plan[2] != 0: the
// Householder fallback was needed); fallback = false: the fallback launches
// are not enqueued, so with plan[2] != 0 the result is not the normaliser
// and the caller redoes the work with fallback = true.
template <typename T>
hipError_t tsqr_run(int64_t n, Sub sub, T* X, double* N, void* ws, uint32_t* cnt, const int32_t* gate_done,
                    const int32_t* gate_fire, hipStream_t st, int32_t* plan = nullptr, bool fallback = true);

// -------------------------------------------------------- transpose ----
hipError_t csr_transpose_run(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colind,
                             const double* val, int32_t* rowptrT, int32_t* colindT, double* valT,
                             int32_t* permT, void* ws, hipStream_t st);
size_t csr_transpose_ws_bytes(int64_t n);

}  // namespace bkry
