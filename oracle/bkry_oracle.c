/*
 * bkry_oracle.c -- plain, slow, FP64 CPU oracle for the block Krylov hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library: it is written directly from
 * the thesis (Dreier, "Hardware-Oriented Krylov Methods for High-Performance
 * Computing", arXiv 2104.02494), in plain loops, without blocking, fusion or
 * reordering, so that it can be checked against the text by eye.
 *
 * Conventions: block vectors are n x s row-major ("row-interleaved"), element
 * (i,j) at X[i*ld + j]; CSR is 0-based with int32 indices; every s x s
 * element of a *-subalgebra is a dense row-major s x s array.  Build with
 * -O2 -ffp-contract=off so that no multiply-add is fused.
 *
 * Status codes: 0 ok, 1 not converged, -1 invalid argument, -2 breakdown
 * (a Cholesky pivot <= 0), -3 non-finite value.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_PARALLEL = 0, OR_GLOBAL = 1, OR_BLOCK = 2, OR_HYBRID = 3, OR_BGLOBAL = 4 };
enum { OR_OK = 0, OR_NOT_CONVERGED = 1, OR_E_INVALID = -1, OR_E_BREAKDOWN = -2, OR_E_NONFINITE = -3 };

typedef int64_t i64;

/* ------------------------------------------------------------------------ */
/* Subalgebra bookkeeping (Definitions "elementary *-subalgebras" and        */
/* "Relevant *-subalgebras", Ch. 3).  "hybrid" is the block-parallel         */
/* subalgebra with q contiguous column groups of width g = s/q.              */
/* ------------------------------------------------------------------------ */
static int group_width(int s, int kind, int q) {
  switch (kind) {
    case OR_BLOCK: return s;
    case OR_HYBRID: return (q > 0 && s % q == 0) ? s / q : -1;
    case OR_BGLOBAL: return (q > 0 && s % q == 0) ? s / q : -1;
    case OR_PARALLEL: return 1;
    case OR_GLOBAL: return 1;
    default: return -1;
  }
}

static int valid_subalg(int s, int kind, int q) {
  if (s < 1) return 0;
  return group_width(s, kind, q) > 0;
}

/* ------------------------------------------------------------------------ */
/* BOP: Y = A X for CSR A (Ch. 3, Performance Analysis, kernel BOP).          */
/* Each entry is summed in CSR order.                                        */
/* ------------------------------------------------------------------------ */
void or_spmm(i64 n, const int32_t* rowptr, const int32_t* colind, const double* val, int s,
             const double* X, double* Y) {
  for (i64 i = 0; i < n; ++i) {
    for (int j = 0; j < s; ++j) {
      double acc = 0.0;
      for (i64 k = rowptr[i]; k < rowptr[i + 1]; ++k) acc += val[k] * X[(i64)colind[k] * s + j];
      Y[i * s + j] = acc;
    }
  }
}

/* R = B - A X */
void or_residual(i64 n, const int32_t* rowptr, const int32_t* colind, const double* val, int s,
                 const double* B, const double* X, double* R) {
  or_spmm(n, rowptr, colind, val, s, X, R);
  for (i64 t = 0; t < n * s; ++t) R[t] = B[t] - R[t];
}

/* Full Gram matrix G = X^T Y (s x s), rows summed in ascending order.  Every
 * entry is its own running sum over the rows; the rows are visited once, in
 * order, so the blocks are read row by row. */
void or_gram(i64 n, int s, const double* X, i64 ldx, const double* Y, i64 ldy, double* G) {
  for (int t = 0; t < s * s; ++t) G[t] = 0.0;
  for (i64 i = 0; i < n; ++i)
    for (int a = 0; a < s; ++a)
      for (int b = 0; b < s; ++b) G[a * s + b] += X[i * ldx + a] * Y[i * ldy + b];
}

/* Projection of a full Gram matrix onto the subalgebra, which turns X^T Y into
 * the block inner product of that subalgebra:
 *   block:    X^T Y;
 *   hybrid:   only the q diagonal g x g blocks are kept;
 *   parallel: only the diagonal is kept;
 *   global:   (tr(X^T Y) / s) * I.  The printed definition has no 1/s; the
 *             normality axiom tr<X,Y> = <X,Y>_F requires it;
 *   block-global (q groups of width g): the mean (1/q) sum_i X_i^T Y_i of
 *             the diagonal g x g blocks, repeated on every diagonal block
 *             (I_q (x) ...), per Definition "Relevant *-subalgebras". */
void or_project(int s, int kind, int q, double* G) {
  int g = group_width(s, kind, q);
  if (kind == OR_GLOBAL) {
    double tr = 0.0;
    for (int a = 0; a < s; ++a) tr += G[a * s + a];
    tr /= (double)s;
    for (int a = 0; a < s; ++a)
      for (int b = 0; b < s; ++b) G[a * s + b] = (a == b) ? tr : 0.0;
    return;
  }
  if (kind == OR_BGLOBAL) {
    /* block-global: (1/q) sum_i X_i^T Y_i on every diagonal g x g block */
    double avg[64 * 64];
    for (int a = 0; a < g; ++a)
      for (int b = 0; b < g; ++b) {
        double acc = 0.0;
        for (int grp = 0; grp < s / g; ++grp) acc += G[(grp * g + a) * s + grp * g + b];
        avg[a * g + b] = acc / (double)(s / g);
      }
    for (int a = 0; a < s; ++a)
      for (int b = 0; b < s; ++b) G[a * s + b] = (a / g == b / g) ? avg[(a % g) * g + b % g] : 0.0;
    return;
  }
  for (int a = 0; a < s; ++a)
    for (int b = 0; b < s; ++b)
      if (a / g != b / g) G[a * s + b] = 0.0;
}

/* BDOT: the block inner product <X, Y>_S (Ch. 3, kernel BDOT). */
int or_bdot(i64 n, int s, int kind, int q, const double* X, const double* Y, double* G) {
  if (!valid_subalg(s, kind, q)) return OR_E_INVALID;
  or_gram(n, s, X, s, Y, s, G);
  or_project(s, kind, q, G);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Householder thin QR (Golub & Van Loan, "house" + backward accumulation),  */
/* the method the thesis uses for the normaliser (Ch. 3, normaliser remark).  */
/* X is m x c (row stride ldx), m >= c.  Outputs Q (m x c, stride ldq) with   */
/* Q^T Q = I and R (c x c, upper triangular) with diag(R) >= 0.  A zero       */
/* sub-column gives the identity reflector, so rank-deficient X still yields */
/* an orthonormal Q (the completion is whatever the reflectors produce).     */
/* ------------------------------------------------------------------------ */
int or_householder_qr(i64 m, int c, const double* X, i64 ldx, double* Q, i64 ldq, double* R) {
  if (m < c || c < 1) return OR_E_INVALID;
  double* A = (double*)malloc(sizeof(double) * (size_t)(m * c));
  double* beta = (double*)malloc(sizeof(double) * (size_t)c);
  double* w = (double*)malloc(sizeof(double) * (size_t)c);
  if (!A || !beta || !w) { free(A); free(beta); free(w); return OR_E_INVALID; }
  for (i64 i = 0; i < m; ++i)
    for (int j = 0; j < c; ++j) A[i * c + j] = X[i * ldx + j];

  for (int j = 0; j < c; ++j) {
    double x1 = A[(i64)j * c + j];
    double sig = 0.0;
    for (i64 i = j + 1; i < m; ++i) sig += A[i * c + j] * A[i * c + j];
    if (sig == 0.0) {
      beta[j] = 0.0; /* identity reflector; R_jj = x1 */
      continue;
    }
    double mu = sqrt(x1 * x1 + sig);
    double v1 = (x1 <= 0.0) ? (x1 - mu) : (-sig / (x1 + mu));
    beta[j] = 2.0 * v1 * v1 / (sig + v1 * v1);
    for (i64 i = j + 1; i < m; ++i) A[i * c + j] /= v1; /* v = [1; x(2:)/v1] */
    A[(i64)j * c + j] = mu;
    /* apply H_j = I - beta v v^T to the trailing columns: w_cc = v^T a_cc
     * (a running sum over the rows in ascending order per column), then
     * a_cc -= beta v w_cc */
    for (int cc = j + 1; cc < c; ++cc) w[cc] = A[(i64)j * c + cc];
    for (i64 i = j + 1; i < m; ++i)
      for (int cc = j + 1; cc < c; ++cc) w[cc] += A[i * c + j] * A[i * c + cc];
    for (int cc = j + 1; cc < c; ++cc) A[(i64)j * c + cc] -= beta[j] * w[cc];
    for (i64 i = j + 1; i < m; ++i)
      for (int cc = j + 1; cc < c; ++cc) A[i * c + cc] -= beta[j] * A[i * c + j] * w[cc];
  }
  for (int a = 0; a < c; ++a)
    for (int b = 0; b < c; ++b) R[a * c + b] = (b >= a) ? A[(i64)a * c + b] : 0.0;

  /* Q = H_0 H_1 ... H_{c-1} [I_c; 0], accumulated from the last reflector. */
  for (i64 i = 0; i < m; ++i)
    for (int j = 0; j < c; ++j) Q[i * ldq + j] = (i == j) ? 1.0 : 0.0;
  for (int j = c - 1; j >= 0; --j) {
    if (beta[j] == 0.0) continue;
    for (int cc = j; cc < c; ++cc) w[cc] = Q[(i64)j * ldq + cc];
    for (i64 i = j + 1; i < m; ++i)
      for (int cc = j; cc < c; ++cc) w[cc] += A[i * c + j] * Q[i * ldq + cc];
    for (int cc = j; cc < c; ++cc) Q[(i64)j * ldq + cc] -= beta[j] * w[cc];
    for (i64 i = j + 1; i < m; ++i)
      for (int cc = j; cc < c; ++cc) Q[i * ldq + cc] -= beta[j] * A[i * c + j] * w[cc];
  }
  /* canonical signs: diag(R) >= 0 */
  for (int j = 0; j < c; ++j) {
    if (R[j * c + j] < 0.0) {
      for (int b = j; b < c; ++b) R[j * c + b] = -R[j * c + b];
      for (i64 i = 0; i < m; ++i) Q[i * ldq + j] = -Q[i * ldq + j];
    }
  }
  free(A);
  free(beta);
  free(w);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Normaliser Norm_S(X): X = Y N with <Y,Y>_S = I and N in S (Definition     */
/* "normalizer", Ch. 3), computed by Householder QR for every X including    */
/* rank-deficient ones.                                                      */
/*   block:    N = R of the QR of X;                                         */
/*   hybrid:   one QR per column group, N block diagonal;                    */
/*   block-global: QR of the groups stacked vertically, N = I (x) rho/sqrt q;*/
/*   parallel: N_jj = |x_j|, y_j = x_j / N_jj, and y_j = e_1 for x_j = 0;    */
/*   global:   N = c I with c = |X|_F / sqrt(s), Y = X / c; for X = 0 the     */
/*             columns of Y are e_1, ..., e_s.                               */
/* Y may alias X.                                                            */
/* ------------------------------------------------------------------------ */
int or_normalize(i64 n, int s, int kind, int q, const double* X, double* Y, double* N) {
  int g = group_width(s, kind, q);
  if (g < 1 || n < g || (kind == OR_GLOBAL && n < s)) return OR_E_INVALID;
  for (int t = 0; t < s * s; ++t) N[t] = 0.0;
  if (kind == OR_PARALLEL) {
    for (int j = 0; j < s; ++j) {
      double ss = 0.0;
      for (i64 i = 0; i < n; ++i) ss += X[i * s + j] * X[i * s + j];
      double nrm = sqrt(ss);
      N[j * s + j] = nrm;
      for (i64 i = 0; i < n; ++i) Y[i * s + j] = (nrm > 0.0) ? X[i * s + j] / nrm : (i == 0 ? 1.0 : 0.0);
    }
    return OR_OK;
  }
  if (kind == OR_GLOBAL) {
    double ss = 0.0;
    for (i64 t = 0; t < n * s; ++t) ss += X[t] * X[t];
    double c = sqrt(ss) / sqrt((double)s);
    for (int j = 0; j < s; ++j) N[j * s + j] = c;
    for (i64 i = 0; i < n; ++i)
      for (int j = 0; j < s; ++j) Y[i * s + j] = (c > 0.0) ? X[i * s + j] / c : (i == j ? 1.0 : 0.0);
    return OR_OK;
  }
  if (kind == OR_BGLOBAL) {
    /* QR of the stacked [X_1; ...; X_q] (qn x g) = Y~ rho, N = I (x) rho/sqrt(q),
     * Y_i = sqrt(q) Y~_i (the block-global example of Ch. 3) */
    const int nq = s / g;
    double* Xs = (double*)malloc(sizeof(double) * (size_t)(n * s));
    double* Qs = (double*)malloc(sizeof(double) * (size_t)(n * s));
    double* Rs = (double*)malloc(sizeof(double) * (size_t)(g * g));
    if (!Xs || !Qs || !Rs) { free(Xs); free(Qs); free(Rs); return OR_E_INVALID; }
    for (int grp = 0; grp < nq; ++grp)
      for (i64 i = 0; i < n; ++i)
        for (int j = 0; j < g; ++j) Xs[((i64)grp * n + i) * g + j] = X[i * s + grp * g + j];
    int st = or_householder_qr(n * nq, g, Xs, g, Qs, g, Rs);
    if (st != OR_OK) { free(Xs); free(Qs); free(Rs); return st; }
    const double rq = sqrt((double)nq);
    for (int grp = 0; grp < nq; ++grp) {
      for (i64 i = 0; i < n; ++i)
        for (int j = 0; j < g; ++j) Y[i * s + grp * g + j] = rq * Qs[((i64)grp * n + i) * g + j];
      for (int a = 0; a < g; ++a)
        for (int b = 0; b < g; ++b) N[(grp * g + a) * s + grp * g + b] = Rs[a * g + b] / rq;
    }
    free(Xs); free(Qs); free(Rs);
    return OR_OK;
  }
  double* Qg = (double*)malloc(sizeof(double) * (size_t)(n * g));
  double* Rg = (double*)malloc(sizeof(double) * (size_t)(g * g));
  if (!Qg || !Rg) { free(Qg); free(Rg); return OR_E_INVALID; }
  for (int grp = 0; grp < s / g; ++grp) {
    int st = or_householder_qr(n, g, X + grp * g, s, Qg, g, Rg);
    if (st != OR_OK) { free(Qg); free(Rg); return st; }
    for (i64 i = 0; i < n; ++i)
      for (int j = 0; j < g; ++j) Y[i * s + grp * g + j] = Qg[i * g + j];
    for (int a = 0; a < g; ++a)
      for (int b = 0; b < g; ++b) N[(grp * g + a) * s + grp * g + b] = Rg[a * g + b];
  }
  free(Qg);
  free(Rg);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Solve A X = B inside the subalgebra, A symmetric positive definite in S   */
/* (alpha and rho of the block CG are SPD by block positive definiteness,    */
/* Definition "BSA/BPD", Ch. 3).  One Cholesky factorisation per S-block;    */
/* no pivoting.  A non-positive or non-finite pivot is a breakdown.  Only    */
/* the S-blocks of B are used; X is returned in S.                           */
/* ------------------------------------------------------------------------ */
int or_chol_solve(int s, int kind, int q, const double* A, const double* B, double* X) {
  int g = group_width(s, kind, q);
  if (g < 1) return OR_E_INVALID;
  double L[64 * 64];
  if (g > 64) return OR_E_INVALID;
  for (int t = 0; t < s * s; ++t) X[t] = 0.0;
  for (int grp = 0; grp < s / g; ++grp) {
    int o = grp * g;
    for (int j = 0; j < g; ++j) {
      for (int i = j; i < g; ++i) {
        double sum = A[(o + i) * s + o + j];
        for (int k = 0; k < j; ++k) sum -= L[i * g + k] * L[j * g + k];
        if (i == j) {
          if (!(sum > 0.0) || !isfinite(sum)) return OR_E_BREAKDOWN;
          L[j * g + j] = sqrt(sum);
        } else {
          L[i * g + j] = sum / L[j * g + j];
        }
      }
    }
    for (int col = 0; col < g; ++col) {
      double y[64];
      for (int i = 0; i < g; ++i) { /* L y = b */
        double sum = B[(o + i) * s + o + col];
        for (int k = 0; k < i; ++k) sum -= L[i * g + k] * y[k];
        y[i] = sum / L[i * g + i];
      }
      for (int i = g - 1; i >= 0; --i) { /* L^T x = y */
        double sum = y[i];
        for (int k = i + 1; k < g; ++k) sum -= L[k * g + i] * X[(o + k) * s + o + col];
        X[(o + i) * s + o + col] = sum / L[i * g + i];
      }
    }
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Eigenvalues of a symmetric s x s matrix by the cyclic Jacobi method       */
/* (Golub & Van Loan, cyclic-by-row with the symmetric 2x2 Schur step).      */
/* ------------------------------------------------------------------------ */
int or_sym_eigenvalues(int s, const double* Ain, double* ev) {
  if (s < 1 || s > 64) return OR_E_INVALID;
  double A[64 * 64];
  for (int t = 0; t < s * s; ++t) A[t] = Ain[t];
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < s; ++i)
      for (int j = 0; j < s; ++j) {
        tot += A[i * s + j] * A[i * s + j];
        if (i != j) off += A[i * s + j] * A[i * s + j];
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < s - 1; ++p)
      for (int qq = p + 1; qq < s; ++qq) {
        double apq = A[p * s + qq];
        if (apq == 0.0) continue;
        double tau = (A[qq * s + qq] - A[p * s + p]) / (2.0 * apq);
        double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        double c = 1.0 / sqrt(1.0 + t * t), sn = t * c;
        for (int k = 0; k < s; ++k) { /* A <- A J (columns p, q) */
          double akp = A[k * s + p], akq = A[k * s + qq];
          A[k * s + p] = c * akp - sn * akq;
          A[k * s + qq] = sn * akp + c * akq;
        }
        for (int k = 0; k < s; ++k) { /* A <- J^T A (rows p, q) */
          double apk = A[p * s + k], aqk = A[qq * s + k];
          A[p * s + k] = c * apk - sn * aqk;
          A[qq * s + k] = sn * apk + c * aqk;
        }
      }
  }
  for (int i = 0; i < s; ++i) ev[i] = A[i * s + i];
  return OR_OK;
}

/* Diagonally scaled condition number kappa_D(alpha) = kappa(D^-1/2 alpha D^-1/2),
 * D = diag(alpha) (Definition "Diagonally scaled condition number", Ch. 4).
 * Infinity if a diagonal entry or the smallest eigenvalue is not positive. */
double or_kappa_D(int s, const double* alpha) {
  double S[64 * 64] = {0.0}, ev[64] = {0.0};
  if (s < 1 || s > 64) return INFINITY;
  for (int i = 0; i < s; ++i)
    if (!(alpha[i * s + i] > 0.0)) return INFINITY;
  for (int i = 0; i < s; ++i)
    for (int j = 0; j < s; ++j) S[i * s + j] = alpha[i * s + j] / sqrt(alpha[i * s + i] * alpha[j * s + j]);
  or_sym_eigenvalues(s, S, ev);
  double lo = ev[0], hi = ev[0];
  for (int i = 1; i < s; ++i) {
    if (ev[i] < lo) lo = ev[i];
    if (ev[i] > hi) hi = ev[i];
  }
  if (!(lo > 0.0)) return INFINITY;
  return hi / lo;
}

/* Re-orthonormalisation test of the adaptive block CG.  The printed test
 * "eta * kappa_D > sqrt(eps)" fires for every eta >= 1e-8; the reading used
 * here, which is consistent with the iteration/re-orthonormalisation counts
 * the thesis reports for both precisions and with "no re-orthonormalization
 * in the parallel case", is: fire iff eta * kappa_D * sqrt(eps) > 1, with
 * eta = 0 never and eta = infinity always firing. */
int or_reortho_fires(double eta, double kappaD, double eps) {
  if (eta <= 0.0) return 0;
  if (isinf(eta)) return 1;
  return eta * kappaD * sqrt(eps) > 1.0;
}

/* small dense helpers (row-major s x s) */
static void mm(int s, const double* A, const double* B, double* C) { /* C = A B */
  for (int i = 0; i < s; ++i)
    for (int j = 0; j < s; ++j) {
      double acc = 0.0;
      for (int k = 0; k < s; ++k) acc += A[i * s + k] * B[k * s + j];
      C[i * s + j] = acc;
    }
}
static void mtm(int s, const double* A, const double* B, double* C) { /* C = A^T B */
  for (int i = 0; i < s; ++i)
    for (int j = 0; j < s; ++j) {
      double acc = 0.0;
      for (int k = 0; k < s; ++k) acc += A[k * s + i] * B[k * s + j];
      C[i * s + j] = acc;
    }
}
static void eye(int s, double* A) {
  for (int i = 0; i < s; ++i)
    for (int j = 0; j < s; ++j) A[i * s + j] = (i == j) ? 1.0 : 0.0;
}
/* Y += X c  (X, Y n x s; c s x s) */
static void block_axpy(i64 n, int s, const double* X, const double* c, double* Y) {
  for (i64 i = 0; i < n; ++i)
    for (int j = 0; j < s; ++j) {
      double acc = 0.0;
      for (int k = 0; k < s; ++k) acc += X[i * s + k] * c[k * s + j];
      Y[i * s + j] += acc;
    }
}
/* Y -= X c */
static void block_axmy(i64 n, int s, const double* X, const double* c, double* Y) {
  for (i64 i = 0; i < n; ++i)
    for (int j = 0; j < s; ++j) {
      double acc = 0.0;
      for (int k = 0; k < s; ++k) acc += X[i * s + k] * c[k * s + j];
      Y[i * s + j] -= acc;
    }
}
static void column_norms(i64 n, int s, const double* X, double* out) {
  for (int j = 0; j < s; ++j) out[j] = 0.0;
  for (i64 i = 0; i < n; ++i)
    for (int j = 0; j < s; ++j) out[j] += X[i * s + j] * X[i * s + j];
  for (int j = 0; j < s; ++j) out[j] = sqrt(out[j]);
}
/* max_i num_i / den_i over columns with den_i > 0 (a column whose initial
 * residual is zero counts as converged) */
static double max_rel(int s, const double* num, const double* den, double* rel) {
  double m = 0.0;
  for (int i = 0; i < s; ++i) {
    double r = (den[i] > 0.0) ? num[i] / den[i] : 0.0;
    if (rel) rel[i] = r;
    if (r > m || isnan(r)) m = isnan(r) ? NAN : r;
  }
  return m;
}

/* Z = M^-1 R for a diagonal M (row i scaled by minv[i]); minv = NULL: copy. */
static void apply_minv(i64 n, int s, const double* minv, const double* R, double* Z) {
  for (i64 i = 0; i < n; ++i)
    for (int j = 0; j < s; ++j) Z[i * s + j] = minv ? minv[i] * R[i * s + j] : R[i * s + j];
}

/* ------------------------------------------------------------------------ */
/* Multicolour ordering for SSOR: the greedy colouring in order of           */
/* decreasing priority (ties: smaller row index first).  Each row takes the  */
/* smallest colour that no already coloured neighbour (an off-diagonal       */
/* column of its row) holds.  For a symmetric pattern this is the colouring  */
/* the parallel Jones-Plassmann rounds produce with the same priorities.     */
/* Returns the number of colours, or OR_E_INVALID (bad column index).        */
/* ------------------------------------------------------------------------ */
static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

int or_color_greedy(i64 n, const int32_t* rowptr, const int32_t* colind, const uint32_t* prio, int32_t* colors) {
  uint64_t* key = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
  int32_t* mark = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 2));
  if (!key || !mark) { free(key); free(mark); return OR_E_INVALID; }
  for (i64 i = 0; i < n; ++i) {
    key[i] = ((uint64_t)(~prio[i]) << 32) | (uint64_t)i;  /* ascending key = priority descending */
    colors[i] = -1;
  }
  qsort(key, (size_t)n, sizeof(uint64_t), cmp_u64);
  for (i64 i = 0; i < n + 2; ++i) mark[i] = -1;
  int ncol = 0, st = OR_OK;
  for (i64 t = 0; t < n; ++t) {
    const i64 v = (i64)(key[t] & 0xffffffffu);
    for (int32_t k = rowptr[v]; k < rowptr[v + 1]; ++k) {
      const int32_t u = colind[k];
      if (u < 0 || u >= n) { st = OR_E_INVALID; goto out; }
      if (u != v && colors[u] >= 0) mark[colors[u]] = (int32_t)v;
    }
    int c = 0;
    while (mark[c] == (int32_t)v) ++c;
    colors[v] = c;
    if (c + 1 > ncol) ncol = c + 1;
  }
out:
  free(key);
  free(mark);
  return st != OR_OK ? st : ncol;
}

/* Multicolour symmetric SOR preconditioner (the SSOR-type preconditioners of */
/* the experiments, Ch. 4), on the rows ordered by colour: with A = L + D + U */
/* split in that order (L: entries whose column has a smaller colour),        */
/*   M = (D + omega L) D^-1 (D + omega U) / (omega (2 - omega)),              */
/* SPD for SPD A and 0 < omega < 2.  Z = M^-1 R by a forward sweep           */
/* y = (D + omega L)^-1 R, colour by colour upwards, then a backward sweep    */
/* Z = (D + omega U)^-1 (omega (2 - omega) D y), colour by colour downwards   */
/* (Z computed in place over y).  Rows of one colour share no entry, so each  */
/* row only reads finished values.  Duplicate diagonal entries are summed.    */
/* OR_E_INVALID: a row without a positive diagonal, or two coupled rows of   */
/* one colour.                                                               */
int or_ssor_apply(i64 n, const int32_t* rowptr, const int32_t* colind, const double* val, const int32_t* colors,
                  int ncolors, double omega, int s, const double* R, double* Z) {
  double* d = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  if (!d) return OR_E_INVALID;
  for (i64 i = 0; i < n; ++i) {
    double di = 0.0;
    for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
      const int32_t j = colind[k];
      if (j == i) di += val[k];
      else if (colors[j] == colors[i]) { free(d); return OR_E_INVALID; }
    }
    if (!(di > 0.0)) { free(d); return OR_E_INVALID; }
    d[i] = di;
  }
  for (int c = 0; c < ncolors; ++c)
    for (i64 i = 0; i < n; ++i) {
      if (colors[i] != c) continue;
      for (int col = 0; col < s; ++col) {
        double acc = R[i * s + col];
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
          if (colors[colind[k]] < c) acc -= (omega * val[k]) * Z[(i64)colind[k] * s + col];
        Z[i * s + col] = acc / d[i];
      }
    }
  const double f = omega * (2.0 - omega);
  for (int c = ncolors - 1; c >= 0; --c)
    for (i64 i = 0; i < n; ++i) {
      if (colors[i] != c) continue;
      for (int col = 0; col < s; ++col) {
        double acc = (f * d[i]) * Z[i * s + col];
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
          if (colors[colind[k]] > c) acc -= (omega * val[k]) * Z[(i64)colind[k] * s + col];
        Z[i * s + col] = acc / d[i];
      }
    }
  free(d);
  return OR_OK;
}

/* The preconditioner of the block CG: diagonal (minv, NULL = identity) or    */
/* multicolour SSOR (ssor non-NULL).                                          */
typedef struct {
  const int32_t* rowptr;
  const int32_t* colind;
  const double* val;
  const int32_t* colors;
  int ncolors;
  double omega;
} or_ssor_t;

static void apply_prec(i64 n, int s, const double* minv, const or_ssor_t* ss, const double* R, double* Z) {
  if (ss) (void)or_ssor_apply(n, ss->rowptr, ss->colind, ss->val, ss->colors, ss->ncolors, ss->omega, s, R, Z);
  else apply_minv(n, s, minv, R, Z);
}

/* ------------------------------------------------------------------------ */
/* Block CG with adaptive residual re-orthonormalisation (Algorithm          */
/* "BCG Method with Adaptive Residual Re-Orthonormalization", Ch. 4) with a  */
/* diagonal preconditioner M: minv[i] = (M^-1)_ii, or minv = NULL for M = I  */
/* (then Z = R-bar is a plain copy and rho = <R-bar, R-bar>_S).              */
/*                                                                          */
/*   R0 = B - A X0                                                           */
/*   (R-bar, sigma) = Norm_S(R0) if eta > 0, else (R0, I)                    */
/*   P = M^-1 R-bar, rho = <P, R-bar>_S                                      */
/*   repeat: Q = A P; alpha = <P,Q>_S; lambda = alpha^-1 rho;                */
/*           X += P lambda sigma; R~ = R-bar - Q lambda;                     */
/*           if the test fires: (R-bar, gamma) = Norm_S(R~), sigma = gamma sigma */
/*           else R-bar = R~, gamma = I;                                     */
/*           stop if max_i |(R-bar sigma)_i| / |R0_i| <= tol;                */
/*           Z = M^-1 R-bar; rho' = <Z, R-bar>_S; beta = rho^-1 gamma^T rho'; */
/*           P = Z + P beta; rho = rho'.                                     */
/*                                                                          */
/* The stopping norm is the maximum column 2-norm (the thesis' choice),      */
/* taken relative to the initial residual column.  After a normalisation the */
/* column norms are those of sigma (exact for block, hybrid and parallel);   */
/* for global they are computed from R-bar sigma.  If every initial column   */
/* is zero the solve returns immediately.                                    */
/*                                                                          */
/* info[0] = iterations, info[1] = normalisations (the initial one included),*/
/* info[2] = converged.  relres[s] = final recursive relative column norms.  */
/* hist (optional, cap entries) = max relative column norm per iteration.    */
/* Pk/Rk (optional, cap_blocks n x s blocks) record P^k and the true residual */
/* R^k = R-bar^k sigma^k for k = 0, 1, ... (for invariant checks).           */
/* ------------------------------------------------------------------------ */
static int bcg_impl(i64 n, const int32_t* rowptr, const int32_t* colind, const double* val, int s, int kind, int q,
                    const double* B, double* X, double tol, int maxit, double eta, double eps, int32_t* info,
                    double* relres, double* hist, int hist_cap, double* Pk, double* Rk, int cap_blocks,
                    const double* minv, const or_ssor_t* ssor) {
  if (!valid_subalg(s, kind, q) || s > 64 || n < group_width(s, kind, q)) return OR_E_INVALID;
  size_t blk = (size_t)(n * s);
  double* R = (double*)calloc(blk, sizeof(double));
  double* P = (double*)calloc(blk, sizeof(double));
  double* Qb = (double*)calloc(blk, sizeof(double));
  double* T = (double*)calloc(blk, sizeof(double));
  if (!R || !P || !Qb || !T) { free(R); free(P); free(Qb); free(T); return OR_E_INVALID; }
  size_t ss = (size_t)s * s;
  double sigma[64 * 64], alpha[64 * 64], rho[64 * 64], rho_new[64 * 64], lambda[64 * 64], tmp[64 * 64];
  double gamma[64 * 64], beta[64 * 64], r0n[64], cn[64], rel[64];
  int st = OR_OK, iters = 0, nro = 0, conv = 0;

  or_residual(n, rowptr, colind, val, s, B, X, R);
  column_norms(n, s, R, r0n);
  for (int i = 0; i < s; ++i) rel[i] = (r0n[i] > 0.0) ? 1.0 : 0.0;
  {
    int allzero = 1;
    for (int i = 0; i < s; ++i) allzero &= (r0n[i] == 0.0);
    if (allzero) {
      conv = 1;
      for (int i = 0; i < s; ++i) rel[i] = 0.0;
      goto done;
    }
  }
  if (eta > 0.0) {
    st = or_normalize(n, s, kind, q, R, R, sigma);
    if (st != OR_OK) goto done;
    nro++;
  } else {
    eye(s, sigma);
  }
  apply_prec(n, s, minv, ssor, R, P);                 /* P = M^-1 R-bar */
  or_bdot(n, s, kind, q, P, R, rho);

  for (int k = 0; k < maxit; ++k) {
    if (Pk && k < cap_blocks) memcpy(Pk + (size_t)k * blk, P, blk * sizeof(double));
    if (Rk && k < cap_blocks) {
      memset(T, 0, blk * sizeof(double));
      block_axpy(n, s, R, sigma, T);
      memcpy(Rk + (size_t)k * blk, T, blk * sizeof(double));
    }
    or_spmm(n, rowptr, colind, val, s, P, Qb);        /* Q = A P */
    or_bdot(n, s, kind, q, P, Qb, alpha);             /* alpha = <P, Q>_S */
    for (size_t t = 0; t < ss; ++t)
      if (!isfinite(alpha[t])) { st = OR_E_NONFINITE; goto done; }
    st = or_chol_solve(s, kind, q, alpha, rho, lambda); /* lambda = alpha^-1 rho */
    if (st != OR_OK) goto done;
    mm(s, lambda, sigma, tmp);                        /* X += P (lambda sigma) */
    block_axpy(n, s, P, tmp, X);
    block_axmy(n, s, Qb, lambda, R);                  /* R~ = R-bar - Q lambda */
    iters = k + 1;
    int fire = or_reortho_fires(eta, or_kappa_D(s, alpha), eps);
    if (fire) {
      st = or_normalize(n, s, kind, q, R, R, gamma);  /* (R-bar, gamma) = Norm_S(R~) */
      if (st != OR_OK) goto done;
      nro++;
      mm(s, gamma, sigma, tmp);                       /* sigma = gamma sigma */
      memcpy(sigma, tmp, ss * sizeof(double));
      if (kind != OR_GLOBAL && kind != OR_BGLOBAL) {
        for (int i = 0; i < s; ++i) {
          double acc = 0.0;
          for (int a = 0; a < s; ++a) acc += sigma[a * s + i] * sigma[a * s + i];
          cn[i] = sqrt(acc);
        }
      } else {
        memset(T, 0, blk * sizeof(double));
        block_axpy(n, s, R, sigma, T);
        column_norms(n, s, T, cn);
      }
    } else {
      eye(s, gamma);
      memset(T, 0, blk * sizeof(double));
      block_axpy(n, s, R, sigma, T);
      column_norms(n, s, T, cn);
    }
    double m = max_rel(s, cn, r0n, rel);
    if (hist && k < hist_cap) hist[k] = m;
    if (isnan(m)) { st = OR_E_NONFINITE; goto done; }
    if (m <= tol) { conv = 1; break; }
    apply_prec(n, s, minv, ssor, R, T);               /* Z = M^-1 R-bar */
    or_bdot(n, s, kind, q, T, R, rho_new);            /* rho' = <Z, R-bar>_S */
    mtm(s, gamma, rho_new, tmp);                      /* beta = rho^-1 gamma^T rho' */
    st = or_chol_solve(s, kind, q, rho, tmp, beta);
    if (st != OR_OK) goto done;
    block_axpy(n, s, P, beta, T);                     /* P = Z + P beta */
    memcpy(P, T, blk * sizeof(double));
    memcpy(rho, rho_new, ss * sizeof(double));
  }
done:
  if (info) { info[0] = iters; info[1] = nro; info[2] = conv; }
  if (relres) for (int i = 0; i < s; ++i) relres[i] = rel[i];
  free(R); free(P); free(Qb); free(T);
  if (st != OR_OK) return st;
  return conv ? OR_OK : OR_NOT_CONVERGED;
}

int or_bcg(i64 n, const int32_t* rowptr, const int32_t* colind, const double* val, int s, int kind, int q,
           const double* B, double* X, double tol, int maxit, double eta, double eps, int32_t* info,
           double* relres, double* hist, int hist_cap, double* Pk, double* Rk, int cap_blocks, const double* minv) {
  return bcg_impl(n, rowptr, colind, val, s, kind, q, B, X, tol, maxit, eta, eps, info, relres, hist, hist_cap, Pk,
                  Rk, cap_blocks, minv, NULL);
}

/* The same block CG preconditioned by multicolour SSOR (or_ssor_apply) with */
/* the given colouring and omega.                                             */
int or_bcg_ssor(i64 n, const int32_t* rowptr, const int32_t* colind, const double* val, int s, int kind, int q,
                const double* B, double* X, double tol, int maxit, double eta, double eps, int32_t* info,
                double* relres, double* hist, int hist_cap, const int32_t* colors, int ncolors, double omega) {
  const or_ssor_t ss = {rowptr, colind, val, colors, ncolors, omega};
  double* T = (double*)calloc((size_t)(n * s), sizeof(double));
  double* Zt = (double*)calloc((size_t)(n * s), sizeof(double));
  if (!T || !Zt) { free(T); free(Zt); return OR_E_INVALID; }
  int st = or_ssor_apply(n, rowptr, colind, val, colors, ncolors, omega, s, T, Zt);  /* validates the colouring */
  free(T); free(Zt);
  if (st != OR_OK) return st;
  return bcg_impl(n, rowptr, colind, val, s, kind, q, B, X, tol, maxit, eta, eps, info, relres, hist, hist_cap, NULL,
                  NULL, 0, NULL, &ss);
}

/* ------------------------------------------------------------------------ */
/* Block CG with one reduction per iteration (alg:1R-CG, Ch. 8, "Fusing      */
/* Inner Block Products"): the auxiliary block U = A Z is formed right after */
/* the preconditioner, Q = A P is carried by the recursion Q = U + Q beta,   */
/* and alpha by alpha' = delta - beta^T alpha beta with delta = <Z, U>_S     */
/* (the derivation around eq. alpha_k+1), so rho', delta and the residual    */
/* norm can share one reduction.  In exact arithmetic the iterates are those */
/* of alg:bcgaro.  Same arguments, outputs and stopping test as or_bcg (the  */
/* column norms after a re-normalisation, and all norms of the global and    */
/* block-global subalgebras, as there).                                      */
/* ------------------------------------------------------------------------ */
/* ------------------------------------------------------------------------ */
/* Gropp's block CG (Algorithm "Gropp's BCG", Ch. 8) with a diagonal         */
/* preconditioner M (minv = diag(M^-1); NULL: M = I).  Besides P, Q = A P    */
/* and R-bar it carries Z = M^-1 R-bar, V = M^-1 Q and U = A Z, and updates  */
/* Q = U + Q beta and, unless the residual is re-normalised, Z = Z - V       */
/* lambda by recurrences instead of forming A P and M^-1 R-bar anew; after a */
/* re-normalisation Z = M^-1 R-bar is formed directly, as the listing says.  */
/* The reductions (alpha; rho' and the stopping norms) and the updates are   */
/* taken in the listing's order; the stopping test and its norms are those   */
/* of the other block CG forms here (readings as in or_bcg).                 */
/* ------------------------------------------------------------------------ */
int or_bcg_gropp(i64 n, const int32_t* rowptr, const int32_t* colind, const double* val, int s, int kind, int q,
                 const double* B, double* X, double tol, int maxit, double eta, double eps, int32_t* info,
                 double* relres, double* hist, int hist_cap, const double* minv) {
  if (!valid_subalg(s, kind, q) || s > 64 || n < group_width(s, kind, q)) return OR_E_INVALID;
  size_t blk = (size_t)(n * s);
  double* R = (double*)calloc(blk, sizeof(double));
  double* P = (double*)calloc(blk, sizeof(double));
  double* Qb = (double*)calloc(blk, sizeof(double));
  double* Z = (double*)calloc(blk, sizeof(double));
  double* V = (double*)calloc(blk, sizeof(double));
  double* U = (double*)calloc(blk, sizeof(double));
  double* T = (double*)calloc(blk, sizeof(double));
  if (!R || !P || !Qb || !Z || !V || !U || !T) {
    free(R); free(P); free(Qb); free(Z); free(V); free(U); free(T);
    return OR_E_INVALID;
  }
  size_t ss = (size_t)s * s;
  double sigma[64 * 64], alpha[64 * 64], rho[64 * 64], rho_new[64 * 64], lambda[64 * 64];
  double gamma[64 * 64], beta[64 * 64], tmp[64 * 64], lamsig[64 * 64];
  double r0n[64], cn[64], rel[64];
  int st = OR_OK, iters = 0, nro = 0, conv = 0;

  or_residual(n, rowptr, colind, val, s, B, X, R);
  column_norms(n, s, R, r0n);
  for (int i = 0; i < s; ++i) rel[i] = (r0n[i] > 0.0) ? 1.0 : 0.0;
  {
    int allzero = 1;
    for (int i = 0; i < s; ++i) allzero &= (r0n[i] == 0.0);
    if (allzero) {
      conv = 1;
      for (int i = 0; i < s; ++i) rel[i] = 0.0;
      goto done;
    }
  }
  if (eta > 0.0) {
    st = or_normalize(n, s, kind, q, R, R, sigma);
    if (st != OR_OK) goto done;
    nro++;
  } else {
    eye(s, sigma);
  }
  apply_minv(n, s, minv, R, P);                       /* P^0 = M^-1 R-bar^0 */
  or_spmm(n, rowptr, colind, val, s, P, Qb);          /* Q^0 = A P^0 */
  memcpy(Z, P, blk * sizeof(double));                 /* Z^0 = P^0 */
  or_bdot(n, s, kind, q, P, R, rho);                  /* rho^0 = <P^0, R-bar^0>_S */

  for (int k = 0; k < maxit; ++k) {
    or_bdot(n, s, kind, q, P, Qb, alpha);             /* alpha = <P, Q>_S */
    apply_minv(n, s, minv, Qb, V);                    /* V = M^-1 Q */
    for (size_t t = 0; t < ss; ++t)
      if (!isfinite(alpha[t])) { st = OR_E_NONFINITE; goto done; }
    st = or_chol_solve(s, kind, q, alpha, rho, lambda); /* lambda = alpha^-1 rho */
    if (st != OR_OK) goto done;
    block_axmy(n, s, Qb, lambda, R);                  /* R~ = R-bar - Q lambda */
    mm(s, lambda, sigma, lamsig);                     /* lambda sigma (before sigma changes) */
    iters = k + 1;
    int fire = or_reortho_fires(eta, or_kappa_D(s, alpha), eps);
    if (fire) {
      st = or_normalize(n, s, kind, q, R, R, gamma);  /* (R-bar, gamma) = Norm_S(R~) */
      if (st != OR_OK) goto done;
      nro++;
      mm(s, gamma, sigma, tmp);                       /* sigma = gamma sigma */
      memcpy(sigma, tmp, ss * sizeof(double));
      if (kind != OR_GLOBAL && kind != OR_BGLOBAL) {
        for (int i = 0; i < s; ++i) {
          double acc = 0.0;
          for (int a = 0; a < s; ++a) acc += sigma[a * s + i] * sigma[a * s + i];
          cn[i] = sqrt(acc);
        }
      } else {
        memset(T, 0, blk * sizeof(double));
        block_axpy(n, s, R, sigma, T);
        column_norms(n, s, T, cn);
      }
      apply_minv(n, s, minv, R, Z);                   /* Z = M^-1 R-bar */
    } else {
      eye(s, gamma);
      memset(T, 0, blk * sizeof(double));
      block_axpy(n, s, R, sigma, T);
      column_norms(n, s, T, cn);
      block_axmy(n, s, V, lambda, Z);                 /* Z = Z - V lambda */
    }
    block_axpy(n, s, P, lamsig, X);                   /* X += P lambda sigma */
    or_bdot(n, s, kind, q, Z, R, rho_new);            /* rho' = <Z, R-bar>_S */
    or_spmm(n, rowptr, colind, val, s, Z, U);         /* U = A Z */
    double m = max_rel(s, cn, r0n, rel);
    if (hist && k < hist_cap) hist[k] = m;
    if (isnan(m)) { st = OR_E_NONFINITE; goto done; }
    if (m <= tol) { conv = 1; break; }
    mtm(s, gamma, rho_new, tmp);                      /* beta = rho^-1 gamma^T rho' */
    st = or_chol_solve(s, kind, q, rho, tmp, beta);
    if (st != OR_OK) goto done;
    memcpy(T, Z, blk * sizeof(double));               /* P = Z + P beta */
    block_axpy(n, s, P, beta, T);
    memcpy(P, T, blk * sizeof(double));
    memcpy(T, U, blk * sizeof(double));               /* Q = U + Q beta */
    block_axpy(n, s, Qb, beta, T);
    memcpy(Qb, T, blk * sizeof(double));
    memcpy(rho, rho_new, ss * sizeof(double));
  }
done:
  if (info) { info[0] = iters; info[1] = nro; info[2] = conv; }
  if (relres) for (int i = 0; i < s; ++i) relres[i] = rel[i];
  free(R); free(P); free(Qb); free(Z); free(V); free(U); free(T);
  if (st != OR_OK) return st;
  return conv ? OR_OK : OR_NOT_CONVERGED;
}

int or_bcg1r(i64 n, const int32_t* rowptr, const int32_t* colind, const double* val, int s, int kind, int q,
             const double* B, double* X, double tol, int maxit, double eta, double eps, int32_t* info,
             double* relres, double* hist, int hist_cap, const double* minv) {
  if (!valid_subalg(s, kind, q) || s > 64 || n < group_width(s, kind, q)) return OR_E_INVALID;
  size_t blk = (size_t)(n * s);
  double* R = (double*)calloc(blk, sizeof(double));
  double* P = (double*)calloc(blk, sizeof(double));
  double* Qb = (double*)calloc(blk, sizeof(double));
  double* Z = (double*)calloc(blk, sizeof(double));
  double* U = (double*)calloc(blk, sizeof(double));
  double* T = (double*)calloc(blk, sizeof(double));
  if (!R || !P || !Qb || !Z || !U || !T) {
    free(R); free(P); free(Qb); free(Z); free(U); free(T);
    return OR_E_INVALID;
  }
  size_t ss = (size_t)s * s;
  double sigma[64 * 64], alpha[64 * 64], rho[64 * 64], rho_new[64 * 64], delta[64 * 64], lambda[64 * 64];
  double gamma[64 * 64], beta[64 * 64], tmp[64 * 64], tmp2[64 * 64], lamsig[64 * 64];
  double r0n[64], cn[64], rel[64];
  int st = OR_OK, iters = 0, nro = 0, conv = 0;

  or_residual(n, rowptr, colind, val, s, B, X, R);
  column_norms(n, s, R, r0n);
  for (int i = 0; i < s; ++i) rel[i] = (r0n[i] > 0.0) ? 1.0 : 0.0;
  {
    int allzero = 1;
    for (int i = 0; i < s; ++i) allzero &= (r0n[i] == 0.0);
    if (allzero) {
      conv = 1;
      for (int i = 0; i < s; ++i) rel[i] = 0.0;
      goto done;
    }
  }
  if (eta > 0.0) {
    st = or_normalize(n, s, kind, q, R, R, sigma);
    if (st != OR_OK) goto done;
    nro++;
  } else {
    eye(s, sigma);
  }
  apply_minv(n, s, minv, R, P);                       /* P^0 = M^-1 R-bar^0 */
  or_bdot(n, s, kind, q, P, R, rho);                  /* rho^0 = <P^0, R-bar^0>_S */
  or_spmm(n, rowptr, colind, val, s, P, Qb);          /* Q^0 = A P^0 */
  or_bdot(n, s, kind, q, P, Qb, alpha);               /* alpha^0 = <P^0, Q^0>_S */

  for (int k = 0; k < maxit; ++k) {
    for (size_t t = 0; t < ss; ++t)
      if (!isfinite(alpha[t])) { st = OR_E_NONFINITE; goto done; }
    st = or_chol_solve(s, kind, q, alpha, rho, lambda); /* lambda = alpha^-1 rho */
    if (st != OR_OK) goto done;
    block_axmy(n, s, Qb, lambda, R);                  /* R~ = R-bar - Q lambda */
    mm(s, lambda, sigma, lamsig);                     /* lambda^k sigma^k (before sigma changes) */
    iters = k + 1;
    int fire = or_reortho_fires(eta, or_kappa_D(s, alpha), eps);
    if (fire) {
      st = or_normalize(n, s, kind, q, R, R, gamma);  /* (R-bar, gamma) = Norm_S(R~) */
      if (st != OR_OK) goto done;
      nro++;
      mm(s, gamma, sigma, tmp);                       /* sigma = gamma sigma */
      memcpy(sigma, tmp, ss * sizeof(double));
      if (kind != OR_GLOBAL && kind != OR_BGLOBAL) {
        for (int i = 0; i < s; ++i) {
          double acc = 0.0;
          for (int a = 0; a < s; ++a) acc += sigma[a * s + i] * sigma[a * s + i];
          cn[i] = sqrt(acc);
        }
      } else {
        memset(T, 0, blk * sizeof(double));
        block_axpy(n, s, R, sigma, T);
        column_norms(n, s, T, cn);
      }
    } else {
      eye(s, gamma);
      memset(T, 0, blk * sizeof(double));
      block_axpy(n, s, R, sigma, T);
      column_norms(n, s, T, cn);
    }
    block_axpy(n, s, P, lamsig, X);                   /* X += P lambda sigma */
    apply_minv(n, s, minv, R, Z);                     /* Z = M^-1 R-bar */
    or_bdot(n, s, kind, q, Z, R, rho_new);            /* rho' = <Z, R-bar>_S */
    or_spmm(n, rowptr, colind, val, s, Z, U);         /* U = A Z */
    or_bdot(n, s, kind, q, Z, U, delta);              /* delta = <Z, U>_S */
    double m = max_rel(s, cn, r0n, rel);
    if (hist && k < hist_cap) hist[k] = m;
    if (isnan(m)) { st = OR_E_NONFINITE; goto done; }
    if (m <= tol) { conv = 1; break; }
    mtm(s, gamma, rho_new, tmp);                      /* beta = rho^-1 gamma^T rho' */
    st = or_chol_solve(s, kind, q, rho, tmp, beta);
    if (st != OR_OK) goto done;
    memcpy(T, Z, blk * sizeof(double));               /* P = Z + P beta */
    block_axpy(n, s, P, beta, T);
    memcpy(P, T, blk * sizeof(double));
    memcpy(T, U, blk * sizeof(double));               /* Q = U + Q beta */
    block_axpy(n, s, Qb, beta, T);
    memcpy(Qb, T, blk * sizeof(double));
    mm(s, alpha, beta, tmp);                          /* alpha = delta - beta^T alpha beta */
    mtm(s, beta, tmp, tmp2);
    for (size_t t = 0; t < ss; ++t) alpha[t] = delta[t] - tmp2[t];
    memcpy(rho, rho_new, ss * sizeof(double));
  }
done:
  if (info) { info[0] = iters; info[1] = nro; info[2] = conv; }
  if (relres) for (int i = 0; i < s; ++i) relres[i] = rel[i];
  free(R); free(P); free(Qb); free(Z); free(U); free(T);
  if (st != OR_OK) return st;
  return conv ? OR_OK : OR_NOT_CONVERGED;
}

/* ------------------------------------------------------------------------ */
/* Solve A X = B inside the subalgebra for a general (non-symmetric) A in S  */
/* by Gaussian elimination with partial pivoting per S-block (the           */
/* coefficient systems of block BiCGStab, Ch. 6).  A zero pivot is a         */
/* breakdown.  Only the S-blocks of B are used; X is returned in S.          */
/* ------------------------------------------------------------------------ */
int or_lu_solve(int s, int kind, int q, const double* A, const double* B, double* X) {
  int g = group_width(s, kind, q);
  if (g < 1 || g > 64) return OR_E_INVALID;
  double M[64 * 64], Y[64 * 64];
  for (int t = 0; t < s * s; ++t) X[t] = 0.0;
  for (int grp = 0; grp < s / g; ++grp) {
    int o = grp * g;
    for (int i = 0; i < g; ++i)
      for (int j = 0; j < g; ++j) {
        M[i * g + j] = A[(o + i) * s + o + j];
        Y[i * g + j] = B[(o + i) * s + o + j];
      }
    for (int c = 0; c < g; ++c) {
      int piv = c;
      for (int i = c + 1; i < g; ++i)
        if (fabs(M[i * g + c]) > fabs(M[piv * g + c])) piv = i;
      if (!(M[piv * g + c] != 0.0) || !isfinite(M[piv * g + c])) return OR_E_BREAKDOWN;
      if (piv != c)
        for (int j = 0; j < g; ++j) {
          double t = M[c * g + j]; M[c * g + j] = M[piv * g + j]; M[piv * g + j] = t;
          t = Y[c * g + j]; Y[c * g + j] = Y[piv * g + j]; Y[piv * g + j] = t;
        }
      for (int i = c + 1; i < g; ++i) {
        double f = M[i * g + c] / M[c * g + c];
        for (int j = c; j < g; ++j) M[i * g + j] -= f * M[c * g + j];
        for (int j = 0; j < g; ++j) Y[i * g + j] -= f * Y[c * g + j];
      }
    }
    for (int col = 0; col < g; ++col)
      for (int i = g - 1; i >= 0; --i) {
        double sum = Y[i * g + col];
        for (int k = i + 1; k < g; ++k) sum -= M[i * g + k] * X[(o + k) * s + o + col];
        X[(o + i) * s + o + col] = sum / M[i * g + i];
      }
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Block BiCGStab with adaptive residual re-orthonormalisation (Algorithm    */
/* "BBiCGStab with Adaptive Residual Re-Orthonormalization", Ch. 6) without  */
/* preconditioner (M = I, so Z = Q, V = R-hat and T = S-hat after a          */
/* re-normalisation), shadow residual R~0 = P-hat^0:                         */
/*                                                                          */
/*   R0 = B - A X0; (R^, sigma) = Norm_S(R0) if eta > 0, else (R0, I)        */
/*   P^ = R^, R~0 = P^, V^ = P^                                              */
/*   repeat: Q^ = A P^; a = <R~0, Q^>_S; lambda = a^-1 <R~0, R^>_S;          */
/*           Z^ = Q^; S^ = R^ - Q^ lambda; X += P^ lambda sigma;             */
/*           if eta kappa_D(<R^, R^>_S) sqrt(eps) > 1:                       */
/*              (S^, gamma) = Norm_S(S^), sigma = gamma sigma, T^ = S^       */
/*           else T^ = V^ - Z^ lambda;                                       */
/*           U^ = A T^; omega = <U^, S^>_F / <U^, U^>_F;                     */
/*           X += omega T^ sigma; R^ = S^ - omega U^;                        */
/*           stop if max_i |(R^ sigma)_i| / |R0_i| <= tol;                   */
/*           V^ = R^; beta = -a^-1 <R~0, U^>_S; P^ = V^ + (P^ - omega Z^) beta. */
/*                                                                          */
/* sigma in the two X updates is the current one: after a re-normalisation  */
/* T^ carries the new transformation (T = T^ gamma sigma), so the second     */
/* update uses the updated sigma (reading of the listing, which writes       */
/* sigma^k).  <.,.>_F is the Frobenius inner product sum_ij X_ij Y_ij.       */
/* info[0] = iterations, info[1] = normalisations (the initial one included),*/
/* info[2] = converged.                                                      */
/* ------------------------------------------------------------------------ */
/* r0n_fixed (NULL: the column norms of B - A X0): the denominators of the
 * stopping test, kept from an earlier run when the iteration is restarted. */
static int bbicgstab_impl(i64 n, const int32_t* rowptr, const int32_t* colind, const double* val, int s, int kind,
                          int q, const double* B, double* X, double tol, int maxit, double eta, double eps,
                          int32_t* info, double* relres, double* hist, int hist_cap, const double* r0n_fixed,
                          double* r0n_out) {
  if (!valid_subalg(s, kind, q) || s > 64 || n < group_width(s, kind, q)) return OR_E_INVALID;
  size_t blk = (size_t)(n * s), ss = (size_t)s * s;
  double* R = (double*)calloc(blk, sizeof(double));
  double* P = (double*)calloc(blk, sizeof(double));
  double* Rt = (double*)calloc(blk, sizeof(double));
  double* Q = (double*)calloc(blk, sizeof(double));
  double* S = (double*)calloc(blk, sizeof(double));
  double* T = (double*)calloc(blk, sizeof(double));
  double* U = (double*)calloc(blk, sizeof(double));
  double* W = (double*)calloc(blk, sizeof(double));
  if (!R || !P || !Rt || !Q || !S || !T || !U || !W) {
    free(R); free(P); free(Rt); free(Q); free(S); free(T); free(U); free(W);
    return OR_E_INVALID;
  }
  double sigma[64 * 64], a[64 * 64], g[64 * 64], lambda[64 * 64], beta[64 * 64], gamma[64 * 64], tmp[64 * 64];
  double r0n[64], cn[64], rel[64];
  int st = OR_OK, iters = 0, nro = 0, conv = 0;

  or_residual(n, rowptr, colind, val, s, B, X, R);
  column_norms(n, s, R, r0n);
  {
    int allzero = 1;
    for (int i = 0; i < s; ++i) allzero &= (r0n[i] == 0.0);
    if (r0n_fixed)
      for (int i = 0; i < s; ++i) r0n[i] = r0n_fixed[i];
    if (r0n_out)
      for (int i = 0; i < s; ++i) r0n_out[i] = r0n[i];
    for (int i = 0; i < s; ++i) rel[i] = (r0n[i] > 0.0) ? 1.0 : 0.0;
    if (allzero) {
      conv = 1;
      for (int i = 0; i < s; ++i) rel[i] = 0.0;
      goto done;
    }
  }
  if (eta > 0.0) {
    st = or_normalize(n, s, kind, q, R, R, sigma);
    if (st != OR_OK) goto done;
    nro++;
  } else {
    eye(s, sigma);
  }
  memcpy(P, R, blk * sizeof(double));                  /* P^ = R^ (M = I)  */
  memcpy(Rt, P, blk * sizeof(double));                 /* R~0 = P^         */

  for (int k = 0; k < maxit; ++k) {
    or_spmm(n, rowptr, colind, val, s, P, Q);          /* Q^ = A P^ */
    or_bdot(n, s, kind, q, Rt, Q, a);                  /* a = <R~0, Q^>_S */
    or_bdot(n, s, kind, q, Rt, R, g);                  /* <R~0, R^>_S */
    for (size_t t = 0; t < ss; ++t)
      if (!isfinite(a[t]) || !isfinite(g[t])) { st = OR_E_NONFINITE; goto done; }
    st = or_lu_solve(s, kind, q, a, g, lambda);        /* lambda = a^-1 <R~0, R^>_S */
    if (st != OR_OK) goto done;
    memcpy(S, R, blk * sizeof(double));                /* S^ = R^ - Q^ lambda */
    block_axmy(n, s, Q, lambda, S);
    mm(s, lambda, sigma, tmp);                         /* X += P^ lambda sigma */
    block_axpy(n, s, P, tmp, X);
    or_bdot(n, s, kind, q, R, R, g);                   /* test on <R^, R^>_S */
    int fire = or_reortho_fires(eta, or_kappa_D(s, g), eps);
    if (fire) {
      st = or_normalize(n, s, kind, q, S, S, gamma);   /* (S^, gamma) = Norm_S(S^) */
      if (st != OR_OK) goto done;
      nro++;
      mm(s, gamma, sigma, tmp);                        /* sigma = gamma sigma */
      memcpy(sigma, tmp, ss * sizeof(double));
      memcpy(T, S, blk * sizeof(double));              /* T^ = M^-1 S^ */
    } else {
      memcpy(T, R, blk * sizeof(double));              /* T^ = V^ - Z^ lambda, V^ = R^, Z^ = Q^ */
      block_axmy(n, s, Q, lambda, T);
    }
    or_spmm(n, rowptr, colind, val, s, T, U);          /* U^ = A T^ */
    double us = 0.0, uu = 0.0;
    for (size_t t = 0; t < blk; ++t) {
      us += U[t] * S[t];
      uu += U[t] * U[t];
    }
    if (!(uu > 0.0) || !isfinite(uu) || !isfinite(us)) { st = (uu == 0.0) ? OR_E_BREAKDOWN : OR_E_NONFINITE; goto done; }
    const double omega = us / uu;
    for (int i = 0; i < s; ++i)                        /* X += omega T^ sigma */
      for (int j = 0; j < s; ++j) tmp[i * s + j] = omega * sigma[i * s + j];
    block_axpy(n, s, T, tmp, X);
    for (size_t t = 0; t < blk; ++t) R[t] = S[t] - omega * U[t]; /* R^ = S^ - omega U^ */
    iters = k + 1;
    memset(W, 0, blk * sizeof(double));                /* stopping test on R^ sigma */
    block_axpy(n, s, R, sigma, W);
    column_norms(n, s, W, cn);
    double m = max_rel(s, cn, r0n, rel);
    if (hist && k < hist_cap) hist[k] = m;
    if (isnan(m)) { st = OR_E_NONFINITE; goto done; }
    if (m <= tol) { conv = 1; break; }
    or_bdot(n, s, kind, q, Rt, U, g);                  /* beta = -a^-1 <R~0, U^>_S */
    st = or_lu_solve(s, kind, q, a, g, beta);
    if (st != OR_OK) goto done;
    for (size_t t = 0; t < ss; ++t) beta[t] = -beta[t];
    for (size_t t = 0; t < blk; ++t) W[t] = P[t] - omega * Q[t]; /* P^ = V^ + (P^ - omega Z^) beta */
    memcpy(P, R, blk * sizeof(double));
    block_axpy(n, s, W, beta, P);
  }
done:
  if (info) { info[0] = iters; info[1] = nro; info[2] = conv; }
  if (relres) for (int i = 0; i < s; ++i) relres[i] = rel[i];
  free(R); free(P); free(Rt); free(Q); free(S); free(T); free(U); free(W);
  if (st != OR_OK) return st;
  return conv ? OR_OK : OR_NOT_CONVERGED;
}

int or_bbicgstab(i64 n, const int32_t* rowptr, const int32_t* colind, const double* val, int s, int kind, int q,
                 const double* B, double* X, double tol, int maxit, double eta, double eps, int32_t* info,
                 double* relres, double* hist, int hist_cap) {
  return bbicgstab_impl(n, rowptr, colind, val, s, kind, q, B, X, tol, maxit, eta, eps, info, relres, hist,
                        hist_cap, NULL, NULL);
}

/* Block BiCGStab restarted on the true residual (a reading beyond the
 * listing, which stops on the recursive residual R^ sigma): when the
 * recursion meets tol but the true residual B - A X does not (the residual
 * gap of BiCGStab), the iteration starts again from the current X (new
 * residual, normalised, and new shadow residual), with the stopping test's
 * denominators kept from the first start; at most max_restarts times, the
 * iterations of all runs counting against maxit.  info[3] = restarts;
 * converged only if the true residual meets tol. */
int or_bbicgstab_restarted(i64 n, const int32_t* rowptr, const int32_t* colind, const double* val, int s,
                           int kind, int q, const double* B, double* X, double tol, int maxit, double eta,
                           double eps, int max_restarts, int32_t* info, double* relres, double* hist,
                           int hist_cap) {
  if (!valid_subalg(s, kind, q) || s > 64 || n < group_width(s, kind, q) || max_restarts < 0) return OR_E_INVALID;
  double r0n[64], cn[64], rel[64];
  double* R = (double*)malloc(sizeof(double) * (size_t)(n * s));
  if (!R) return OR_E_INVALID;
  int32_t sub[4];
  int total = 0, nro = 0, restarts = 0, conv = 0, st = OR_OK;
  for (;;) {
    const int used = total;
    st = bbicgstab_impl(n, rowptr, colind, val, s, kind, q, B, X, tol, maxit - used, eta, eps, sub, rel,
                        hist ? hist + (used < hist_cap ? used : hist_cap) : NULL,
                        hist_cap > used ? hist_cap - used : 0, restarts ? r0n : NULL, restarts ? NULL : r0n);
    total += sub[0];
    nro += sub[1];
    if (st != OR_OK && st != OR_NOT_CONVERGED) break;
    if (!sub[2]) break;                                 /* stopped at maxit */
    or_residual(n, rowptr, colind, val, s, B, X, R);    /* true residual */
    column_norms(n, s, R, cn);
    double m = max_rel(s, cn, r0n, rel);
    if (m <= tol) { conv = 1; break; }
    if (restarts == max_restarts || total >= maxit) break;
    restarts++;
  }
  if (info) { info[0] = total; info[1] = nro; info[2] = conv; info[3] = restarts; }
  if (relres) for (int i = 0; i < s; ++i) relres[i] = rel[i];
  free(R);
  if (st != OR_OK && st != OR_NOT_CONVERGED) return st;
  return conv ? OR_OK : OR_NOT_CONVERGED;
}

/* ------------------------------------------------------------------------ */
/* Block Arnoldi step with modified Gram-Schmidt (Algorithm "Block Arnoldi    */
/* Method", Ch. 5).  Given S-orthonormal V_0..V_k (each n x s, consecutive), */
/* computes W = A V_k, h_jk = <V_j, W>_S and W -= V_j h_jk for j = 0..k in   */
/* turn, then (V_{k+1}, gamma) = Norm_S(W).  The printed step stores         */
/* eta = -<V_j, W> and adds V_j eta while the normaliser returns a positive  */
/* sub-diagonal; the Hessenberg matrix is kept consistent here by storing    */
/* +<V_j, W> and subtracting (as in Gram-Schmidt).  h has k+2 entries.        */
/* ------------------------------------------------------------------------ */
static int arnoldi_step(i64 n, const int32_t* rowptr, const int32_t* colind, const double* val, int s,
                        int kind, int q, double* V, int k, double* h /* (k+2) s x s */) {
  size_t blk = (size_t)(n * s), ss = (size_t)s * s;
  double* W = V + (size_t)(k + 1) * blk;
  or_spmm(n, rowptr, colind, val, s, V + (size_t)k * blk, W);
  for (int j = 0; j <= k; ++j) {
    or_bdot(n, s, kind, q, V + (size_t)j * blk, W, h + (size_t)j * ss);
    block_axmy(n, s, V + (size_t)j * blk, h + (size_t)j * ss, W);
  }
  return or_normalize(n, s, kind, q, W, W, h + (size_t)(k + 1) * ss);
}

/* ------------------------------------------------------------------------ */
/* Block Arnoldi step with the pipelined Gram-Schmidt orthogonalisation of   */
/* Ch. 9 (Algorithm "Pipelined Gram-Schmidt Orthogonalization") with window  */
/* r: the inner products of the first r basis blocks are formed first; then  */
/* each further inner product h_i = <V_i, W>_S is formed before the update   */
/* with basis block i - r is subtracted; the last r updates follow; finally  */
/* (V_{k+1}, gamma) = Norm_S(W).  Readings: the window is min(r, k) (the     */
/* listing asks for 1 <= r <= k); the closing loop subtracts the blocks      */
/* k - r + 1 .. k, the ones the middle loop has not subtracted (the printed  */
/* lower bound k - r would subtract block k - r twice; with k - r + 1, r = 0 */
/* is modified and r = k classical Gram-Schmidt, as the text states); h_i =  */
/* <V_i, W>_S as for modified Gram-Schmidt above.                            */
/* ------------------------------------------------------------------------ */
static int arnoldi_step_pipelined(i64 n, const int32_t* rowptr, const int32_t* colind, const double* val, int s,
                                  int kind, int q, double* V, int k, int r, double* h /* (k+2) s x s */) {
  size_t blk = (size_t)(n * s), ss = (size_t)s * s;
  double* W = V + (size_t)(k + 1) * blk;
  const int w = r < k ? r : k;
  or_spmm(n, rowptr, colind, val, s, V + (size_t)k * blk, W);
  for (int i = 0; i < w; ++i) or_bdot(n, s, kind, q, V + (size_t)i * blk, W, h + (size_t)i * ss);
  for (int i = w; i <= k; ++i) {
    or_bdot(n, s, kind, q, V + (size_t)i * blk, W, h + (size_t)i * ss);
    block_axmy(n, s, V + (size_t)(i - w) * blk, h + (size_t)(i - w) * ss, W);
  }
  for (int i = k - w + 1; i <= k; ++i) block_axmy(n, s, V + (size_t)i * blk, h + (size_t)i * ss, W);
  return or_normalize(n, s, kind, q, W, W, h + (size_t)(k + 1) * ss);
}

/* Block Arnoldi with m steps from V0 = Norm_S(R) (for the Arnoldi relation
 * checks).  V gets m+1 blocks; H ((m+1) x m S-elements, entry (j,k) at
 * H[(j*m + k) * s*s]) the block Hessenberg matrix with A V~ = V H. */
int or_block_arnoldi(i64 n, const int32_t* rowptr, const int32_t* colind, const double* val, int s, int kind,
                     int q, const double* R, int m, double* V, double* H, double* sigma0) {
  if (!valid_subalg(s, kind, q) || s > 64) return OR_E_INVALID;
  size_t ss = (size_t)s * s;
  int st = or_normalize(n, s, kind, q, R, V, sigma0);
  if (st != OR_OK) return st;
  double* h = (double*)malloc(sizeof(double) * (size_t)(m + 1) * ss);
  memset(H, 0, sizeof(double) * (size_t)(m + 1) * m * ss);
  for (int k = 0; k < m; ++k) {
    st = arnoldi_step(n, rowptr, colind, val, s, kind, q, V, k, h);
    if (st != OR_OK) break;
    for (int j = 0; j <= k + 1; ++j) memcpy(H + ((size_t)j * m + k) * ss, h + (size_t)j * ss, ss * sizeof(double));
  }
  free(h);
  return st;
}

/* Full QR of the 2g x g matrix [top; bot] (each g x g, row stride s, taken
 * from the S-block at offset o): [top; bot] = Om [rho; 0] with Om (2g x 2g)
 * orthogonal, the generalised Givens rotation of the block GMRes method.
 * Om is returned explicitly (row-major 2g x 2g); rho replaces top and zero
 * replaces bot. */
static void block_givens(int s, int g, int o, double* top, double* bot, double* Om) {
  int m2 = 2 * g;
  double M[128 * 64];
  double Qf[128 * 128];
  double beta[64];
  for (int i = 0; i < g; ++i)
    for (int j = 0; j < g; ++j) {
      M[i * g + j] = top[(o + i) * s + o + j];
      M[(g + i) * g + j] = bot[(o + i) * s + o + j];
    }
  for (int j = 0; j < g; ++j) {
    double x1 = M[j * g + j], sig = 0.0;
    for (int i = j + 1; i < m2; ++i) sig += M[i * g + j] * M[i * g + j];
    if (sig == 0.0) { beta[j] = 0.0; continue; }
    double mu = sqrt(x1 * x1 + sig);
    double v1 = (x1 <= 0.0) ? (x1 - mu) : (-sig / (x1 + mu));
    beta[j] = 2.0 * v1 * v1 / (sig + v1 * v1);
    for (int i = j + 1; i < m2; ++i) M[i * g + j] /= v1;
    M[j * g + j] = mu;
    for (int c = j + 1; c < g; ++c) {
      double w = M[j * g + c];
      for (int i = j + 1; i < m2; ++i) w += M[i * g + j] * M[i * g + c];
      M[j * g + c] -= beta[j] * w;
      for (int i = j + 1; i < m2; ++i) M[i * g + c] -= beta[j] * M[i * g + j] * w;
    }
  }
  /* full Q = H_0 ... H_{g-1} (2g x 2g) */
  for (int i = 0; i < m2; ++i)
    for (int j = 0; j < m2; ++j) Qf[i * m2 + j] = (i == j) ? 1.0 : 0.0;
  for (int j = g - 1; j >= 0; --j) {
    if (beta[j] == 0.0) continue;
    for (int c = 0; c < m2; ++c) {
      double w = Qf[j * m2 + c];
      for (int i = j + 1; i < m2; ++i) w += M[i * g + j] * Qf[i * m2 + c];
      Qf[j * m2 + c] -= beta[j] * w;
      for (int i = j + 1; i < m2; ++i) Qf[i * m2 + c] -= beta[j] * M[i * g + j] * w;
    }
  }
  for (int i = 0; i < g; ++i)
    for (int j = 0; j < g; ++j) {
      top[(o + i) * s + o + j] = (j >= i) ? M[i * g + j] : 0.0;
      bot[(o + i) * s + o + j] = 0.0;
    }
  memcpy(Om, Qf, sizeof(double) * (size_t)m2 * m2);
}

/* [x; y] <- Om^T [x; y] per S-block, for s x s S-elements x, y. */
static void apply_givens_T(int s, int g, const double* Om /* per group 2g x 2g */, double* x, double* y) {
  int m2 = 2 * g;
  double col[128], out[128];
  for (int grp = 0; grp < s / g; ++grp) {
    const double* O = Om + (size_t)grp * m2 * m2;
    int o = grp * g;
    for (int c = 0; c < g; ++c) {
      for (int i = 0; i < g; ++i) {
        col[i] = x[(o + i) * s + o + c];
        col[g + i] = y[(o + i) * s + o + c];
      }
      for (int i = 0; i < m2; ++i) {
        double acc = 0.0;
        for (int k = 0; k < m2; ++k) acc += O[k * m2 + i] * col[k];
        out[i] = acc;
      }
      for (int i = 0; i < g; ++i) {
        x[(o + i) * s + o + c] = out[i];
        y[(o + i) * s + o + c] = out[g + i];
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Restarted block GMRes (Algorithm "Block GMRes Method", Ch. 5) with MGS    */
/* block Arnoldi, the generalised Givens rotations applied on the fly to the */
/* Hessenberg column and to sigma, block back-substitution and restart.      */
/*                                                                          */
/* Readings: the Hessenberg entries are +<V_j, W>_S (see arnoldi_step); the  */
/* back-substitution runs over the steps actually taken in the cycle; the    */
/* step count limit maxit counts Arnoldi steps over all cycles; the stopping */
/* test is max_i |sigma^{k+1} e_i| / |R0_i| <= tol for block, hybrid and     */
/* parallel (these are the residual column norms) and, for global, the       */
/* Frobenius form |sigma^{k+1}|_F / |R0|_F <= tol.  A zero pivot in the back */
/* substitution gives a zero component.                                      */
/*                                                                          */
/* info[0] = Arnoldi steps, info[1] = cycles, info[2] = converged.           */
/* relres[s] = true relative column residuals at exit; hist = per step       */
/* residual measure.                                                         */
/* ------------------------------------------------------------------------ */
/* orth < 0: modified Gram-Schmidt; orth = r >= 0: pipelined Gram-Schmidt
 * with window r (r = 0 is modified Gram-Schmidt again, r >= restart - 1
 * classical Gram-Schmidt). */
static int bgmres_impl(i64 n, const int32_t* rowptr, const int32_t* colind, const double* val, int s, int kind,
                       int q, const double* B, double* X, double tol, int maxit, int restart, int orth,
                       int32_t* info, double* relres, double* hist, int hist_cap) {
  int g = group_width(s, kind, q);
  if (g < 1 || s > 64 || restart < 1 || n < s) return OR_E_INVALID;
  int m = restart, ngrp = s / g;
  size_t blk = (size_t)(n * s), ss = (size_t)s * s;
  double* V = (double*)malloc(sizeof(double) * (size_t)(m + 1) * blk);
  double* R = (double*)malloc(sizeof(double) * blk);
  double* H = (double*)malloc(sizeof(double) * (size_t)(m + 1) * m * ss);
  double* sig = (double*)malloc(sizeof(double) * (size_t)(m + 1) * ss);
  double* Om = (double*)malloc(sizeof(double) * (size_t)m * ngrp * 4 * g * g);
  double* zeta = (double*)malloc(sizeof(double) * (size_t)m * ss);
  double* h = (double*)malloc(sizeof(double) * (size_t)(m + 1) * ss);
  if (!V || !R || !H || !sig || !Om || !zeta || !h) {
    free(V); free(R); free(H); free(sig); free(Om); free(zeta); free(h);
    return OR_E_INVALID;
  }
  double r0n[64], cn[64], rel[64], tmp[64 * 64], r0F = 0.0;
  int st = OR_OK, total = 0, cycles = 0, conv = 0;

  or_residual(n, rowptr, colind, val, s, B, X, R);
  column_norms(n, s, R, r0n);
  for (int i = 0; i < s; ++i) r0F += r0n[i] * r0n[i];
  r0F = sqrt(r0F);
  if (r0F == 0.0) { conv = 1; goto finish; }

  while (1) {
    cycles++;
    or_residual(n, rowptr, colind, val, s, B, X, R);
    memset(sig, 0, sizeof(double) * (size_t)(m + 1) * ss);
    memset(H, 0, sizeof(double) * (size_t)(m + 1) * m * ss);
    st = or_normalize(n, s, kind, q, R, V, sig); /* V^0 sigma^0 = Norm_S(R0) */
    if (st != OR_OK) goto finish;
    int kend = 0;
    for (int k = 0; k < m; ++k) {
      st = orth < 0 ? arnoldi_step(n, rowptr, colind, val, s, kind, q, V, k, h)
                    : arnoldi_step_pipelined(n, rowptr, colind, val, s, kind, q, V, k, orth, h);
      if (st != OR_OK) goto finish;
      for (int j = 0; j <= k; ++j) memcpy(H + ((size_t)j * m + k) * ss, h + (size_t)j * ss, ss * sizeof(double));
      double* gam = h + (size_t)(k + 1) * ss;
      for (int j = 0; j < k; ++j) /* apply the previous rotations to column k */
        apply_givens_T(s, g, Om + (size_t)j * ngrp * 4 * g * g, H + ((size_t)j * m + k) * ss,
                       H + ((size_t)(j + 1) * m + k) * ss);
      for (int grp = 0; grp < ngrp; ++grp) /* Q_k [eta_kk; 0] = [eta_kk; gamma] */
        block_givens(s, g, grp * g, H + ((size_t)k * m + k) * ss, gam,
                     Om + ((size_t)k * ngrp + grp) * 4 * g * g);
      apply_givens_T(s, g, Om + (size_t)k * ngrp * 4 * g * g, sig + (size_t)k * ss, sig + (size_t)(k + 1) * ss);
      total++;
      kend = k + 1;
      const double* sk = sig + (size_t)(k + 1) * ss;
      double meas;
      if (kind == OR_GLOBAL || kind == OR_BGLOBAL) {
        double f = 0.0;
        for (size_t t = 0; t < ss; ++t) f += sk[t] * sk[t];
        meas = sqrt(f) / r0F;
      } else {
        for (int i = 0; i < s; ++i) {
          double acc = 0.0;
          for (int a = 0; a < s; ++a) acc += sk[a * s + i] * sk[a * s + i];
          cn[i] = sqrt(acc);
        }
        meas = max_rel(s, cn, r0n, NULL);
      }
      if (hist && total - 1 < hist_cap) hist[total - 1] = meas;
      if (isnan(meas)) { st = OR_E_NONFINITE; goto finish; }
      if (meas <= tol) { conv = 1; break; }
      if (total >= maxit) break;
    }
    /* back-substitution: zeta_l = eta_ll^-1 (sigma_l - sum_{j>l} eta_lj zeta_j) */
    for (int l = kend - 1; l >= 0; --l) {
      memcpy(tmp, sig + (size_t)l * ss, ss * sizeof(double));
      for (int j = l + 1; j < kend; ++j) {
        const double* hl = H + ((size_t)l * m + j) * ss;
        const double* zj = zeta + (size_t)j * ss;
        for (int a = 0; a < s; ++a)
          for (int b = 0; b < s; ++b) {
            double acc = 0.0;
            for (int c = 0; c < s; ++c) acc += hl[a * s + c] * zj[c * s + b];
            tmp[a * s + b] -= acc;
          }
      }
      const double* T = H + ((size_t)l * m + l) * ss; /* upper triangular per S-block */
      double* z = zeta + (size_t)l * ss;
      memset(z, 0, ss * sizeof(double));
      for (int grp = 0; grp < ngrp; ++grp) {
        int o = grp * g;
        for (int b = 0; b < g; ++b)
          for (int a = g - 1; a >= 0; --a) {
            double acc = tmp[(o + a) * s + o + b];
            for (int c = a + 1; c < g; ++c) acc -= T[(o + a) * s + o + c] * z[(o + c) * s + o + b];
            double piv = T[(o + a) * s + o + a];
            z[(o + a) * s + o + b] = (piv != 0.0) ? acc / piv : 0.0;
          }
      }
    }
    for (int j = 0; j < kend; ++j) block_axpy(n, s, V + (size_t)j * blk, zeta + (size_t)j * ss, X);
    if (conv || total >= maxit) break;
  }
finish:
  or_residual(n, rowptr, colind, val, s, B, X, R);
  column_norms(n, s, R, cn);
  max_rel(s, cn, r0n, rel);
  if (relres) for (int i = 0; i < s; ++i) relres[i] = rel[i];
  if (info) { info[0] = total; info[1] = cycles; info[2] = conv; }
  free(V); free(R); free(H); free(sig); free(Om); free(zeta); free(h);
  if (st != OR_OK) return st;
  return conv ? OR_OK : OR_NOT_CONVERGED;
}

int or_bgmres(i64 n, const int32_t* rowptr, const int32_t* colind, const double* val, int s, int kind, int q,
              const double* B, double* X, double tol, int maxit, int restart, int32_t* info, double* relres,
              double* hist, int hist_cap) {
  return bgmres_impl(n, rowptr, colind, val, s, kind, q, B, X, tol, maxit, restart, -1, info, relres, hist,
                     hist_cap);
}

/* Block GMRes with the pipelined Gram-Schmidt orthogonalisation of window r
 * (Ch. 9) in every Arnoldi step. */
int or_bgmres_pipelined(i64 n, const int32_t* rowptr, const int32_t* colind, const double* val, int s, int kind,
                        int q, const double* B, double* X, double tol, int maxit, int restart, int r,
                        int32_t* info, double* relres, double* hist, int hist_cap) {
  if (r < 0) return OR_E_INVALID;
  return bgmres_impl(n, rowptr, colind, val, s, kind, q, B, X, tol, maxit, restart, r, info, relres, hist,
                     hist_cap);
}

/* Block Arnoldi (m steps from V0 = Norm_S(R)) with the pipelined
 * Gram-Schmidt of window r; V, H, sigma0 as or_block_arnoldi. */
int or_block_arnoldi_pipelined(i64 n, const int32_t* rowptr, const int32_t* colind, const double* val, int s,
                               int kind, int q, const double* R, int m, int r, double* V, double* H,
                               double* sigma0) {
  if (!valid_subalg(s, kind, q) || s > 64 || r < 0) return OR_E_INVALID;
  size_t ss = (size_t)s * s;
  int st = or_normalize(n, s, kind, q, R, V, sigma0);
  if (st != OR_OK) return st;
  double* h = (double*)malloc(sizeof(double) * (size_t)(m + 1) * ss);
  memset(H, 0, sizeof(double) * (size_t)(m + 1) * m * ss);
  for (int k = 0; k < m; ++k) {
    st = arnoldi_step_pipelined(n, rowptr, colind, val, s, kind, q, V, k, r, h);
    if (st != OR_OK) break;
    for (int j = 0; j <= k + 1; ++j) memcpy(H + ((size_t)j * m + k) * ss, h + (size_t)j * ss, ss * sizeof(double));
  }
  free(h);
  return st;
}

/* ------------------------------------------------------------------------ */
/* Sampled dense-dense product on the pattern of A:                          */
/*   out[k] = alpha * sum_c L[i][c] * X[colind[k]][c]  for k in row i.       */
/* With alpha = -1, L = Lambda (adjoint solution) and X the forward solution */
/* this is dL/dval = -(Lambda X^T) restricted to the pattern of A.           */
/* ------------------------------------------------------------------------ */
void or_sddmm(i64 n, const int32_t* rowptr, const int32_t* colind, int s, double alpha, const double* L,
              const double* X, double* out) {
  for (i64 i = 0; i < n; ++i)
    for (i64 k = rowptr[i]; k < rowptr[i + 1]; ++k) {
      double acc = 0.0;
      for (int c = 0; c < s; ++c) acc += L[i * s + c] * X[(i64)colind[k] * s + c];
      out[k] = alpha * acc;
    }
}

/* Transpose of a square CSR matrix by a stable counting sort over the
 * entries in storage order: rows of A^T list their columns ascending.
 * permT[t] = index in A of entry t of A^T. */
void or_csr_transpose(i64 n, const int32_t* rowptr, const int32_t* colind, const double* val, int32_t* rowptrT,
                      int32_t* colindT, double* valT, int32_t* permT) {
  i64 nnz = rowptr[n];
  for (i64 j = 0; j <= n; ++j) rowptrT[j] = 0;
  for (i64 k = 0; k < nnz; ++k) rowptrT[colind[k] + 1]++;
  for (i64 j = 0; j < n; ++j) rowptrT[j + 1] += rowptrT[j];
  int32_t* cur = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  for (i64 j = 0; j <= n; ++j) cur[j] = rowptrT[j];
  for (i64 i = 0; i < n; ++i)
    for (i64 k = rowptr[i]; k < rowptr[i + 1]; ++k) {
      int32_t t = cur[colind[k]]++;
      colindT[t] = (int32_t)i;
      valT[t] = val[k];
      permT[t] = (int32_t)k;
    }
  free(cur);
}

double or_eps_f64(void) { return DBL_EPSILON; }
double or_eps_f32(void) { return (double)FLT_EPSILON; }
