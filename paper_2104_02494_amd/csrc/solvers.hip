// solvers.hip -- host drivers of the block solvers.  Every arithmetic step
// runs in the kernels; the host enqueues them on one stream and reads back
// only the few integers of a control block (once per batch of iterations for
// CG, once per cycle for GMRes, once per refinement step for IR).
#include <float.h>
#include <math.h>
#include <stddef.h>
#include <string.h>

#include "solvers.hpp"

#include <utility>
#include <vector>

namespace bkry {

#define BK_TRY(x)                       \
  do {                                  \
    hipError_t e_ = (x);                \
    if (e_ != hipSuccess) return e_;    \
  } while (0)

// ------------------------------------------------------------ kernel timing --
hipError_t prof_init(Prof* p) {
  for (int k = 0; k < PROF_N; ++k) {
    p->used[k] = 0;
    p->ms[k] = 0.0;
    p->cnt[k] = 0;
    p->dropped[k] = 0;
    for (int e = 0; e < 2; ++e)
      for (int i = 0; i < kProfSlots; ++i) BK_TRY(hipEventCreate(&p->ev[k][e][i]));
  }
  return hipSuccess;
}

void prof_destroy(Prof* p) {
  for (int k = 0; k < PROF_N; ++k)
    for (int e = 0; e < 2; ++e)
      for (int i = 0; i < kProfSlots; ++i) (void)hipEventDestroy(p->ev[k][e][i]);
}

hipError_t prof_flush(Prof* p, const int* live) {
  if (!p) return hipSuccess;
  for (int k = 0; k < PROF_N; ++k) {
    const int lim = live ? live[k] : 0x7fffffff;
    for (int i = 0; i < p->used[k]; ++i) {
      if (p->iter[k][i] >= 0 && p->iter[k][i] >= lim) {
        p->dropped[k] += 1;
        continue;
      }
      float ms = 0.0f;
      BK_TRY(hipEventElapsedTime(&ms, p->ev[k][0][i], p->ev[k][1][i]));
      p->ms[k] += ms;
      p->cnt[k] += 1;
    }
    p->used[k] = 0;
  }
  return hipSuccess;
}

namespace {
// Records the start event on construction and the end event on destruction,
// unless the timed launcher records the end event itself (end()).
struct ProfScope {
  Prof* p;
  int k;
  hipStream_t st;
  bool handed = false;
  // iter: the solver iteration the launch belongs to (-1: always live).
  ProfScope(Prof* p_, int k_, hipStream_t st_, int iter = -1)
      : p((p_ && (p_->mask >> k_ & 1) && p_->seen[k_]++ % p_->every == 0) ? p_ : nullptr), k(k_), st(st_) {
    if (p && p->used[k] < kProfSlots) {
      p->iter[k][p->used[k]] = iter;
      (void)hipEventRecord(p->ev[k][0][p->used[k]], st);
    }
  }
  // End event for a launcher to record after its streaming kernel (or null).
  hipEvent_t end() {
    if (!(p && p->used[k] < kProfSlots)) return nullptr;
    handed = true;
    return p->ev[k][1][p->used[k]];
  }
  ~ProfScope() {
    if (p && p->used[k] < kProfSlots) {
      if (!handed) (void)hipEventRecord(p->ev[k][1][p->used[k]], st);
      p->used[k] += 1;
    }
  }
};
}  // namespace

// ---------------------------------------------------------------- block CG --
template <typename T>
CgBufs<T> carve_cg(Carver& c, int64_t n, Sub sub, int hist_cap, uint32_t* cnt) {
  const int s = sub.s;
  const int nblk = stream_grid(n, s, sizeof(T));
  CgBufs<T> b;
  b.P = c.take<T>((size_t)n * s);
  b.P2 = c.take<T>((size_t)n * s);
  b.Q = c.take<T>((size_t)n * s);
  b.R = c.take<T>((size_t)n * s);
  // room for two Grams per workgroup (the preconditioned residual update)
  b.partial = c.take<T>((size_t)2 * nblk * s * s);
  b.gpart = c.take<double>(2 * red_gpart_count(nblk, s));
  b.Ga = c.take<double>((size_t)s * s);
  b.Gr = c.take<double>((size_t)2 * s * s);
  b.Gq = c.take<double>((size_t)s * s);
  b.hist = c.take<double>((size_t)(hist_cap > 0 ? hist_cap : 1));
  b.ctl = c.take<CgCtl>(1);
  b.tsqr_ws = c.take<char>(tsqr_workspace_bytes(n, sub));
  b.cnt = cnt;
  return b;
}

// Re-normalisation of the residual (R-bar, gamma) = Norm_S(R~), then
// sigma = gamma sigma, rho' and beta (cg_reortho_fin); runs only while the
// solve is live and the re-orthonormalisation test fired.
// With a preconditioner, rho' = <M^-1 R-bar, R-bar>_S (Z = M^-1 R-bar goes
// through Q, which is free at this point of the iteration).
template <typename T>
static hipError_t cg_normalise(int64_t n, Sub sub, const CgBufs<T>& b, int nblk, hipStream_t st, Prof* prof,
                               const double* minv) {
  CgCtl* c = b.ctl;
  ProfScope ps(prof, PROF_CG_NORMALISE, st);
  BK_TRY(tsqr_run<T>(n, sub, b.R, c->gamma, b.tsqr_ws, b.cnt, &c->done, &c->fire, st));
  const T* Z = b.R;
  if (minv) {
    BK_TRY(launch_row_scale<T>(n, sub.s, minv, b.R, b.Q, &c->done, &c->fire, st));
    Z = b.Q;
  }
  BK_TRY(launch_gram<T>(n, sub.s, Z, 1, b.R, b.partial, nblk, Red{b.Gq, b.gpart, b.cnt}, &c->done, st, &c->fire));
  return launch_cg_reortho_fin(c, sub.s, b.Gq, st);
}

template <typename T>
hipError_t cg_run(const CsrView& A, Sub sub, const T* B, T* X, double tol, int maxit, double eta, double eps,
                  int hist_cap, const CgBufs<T>& b, hipStream_t st, int32_t* hflags, CgResult& res, Prof* prof,
                  const double* minv) {
  if (minv && sizeof(T) != 8) return hipErrorInvalidValue;
  const int64_t n = A.n;
  const int s = sub.s;
  const int nblk = stream_grid(n, s, sizeof(T));
  CgCtl* c = b.ctl;
  int32_t* done = &c->done;
  int32_t* gate = &c->gate;
  const Red ra{b.Ga, b.gpart, b.cnt}, rr{b.Gr, b.gpart, b.cnt};

  // The test eta kappa_D sqrt(eps) > 1 never fires for eta = 0 and always
  // fires for eta = inf or eta sqrt(eps) > 1 (kappa_D >= 1); for the diagonal
  // subalgebras kappa_D = 1.  Only the remaining cases are decided per
  // iteration on the device.
  const bool always = eta > 0.0 && (isinf(eta) || eta * sqrt(eps) > 1.0);
  const bool dynamic = eta > 0.0 && !always && sub.g > 1;

  // control header, staged through pinned memory
  CgCtl* h = reinterpret_cast<CgCtl*>(hflags + 64);
  static_assert(offsetof(CgCtl, r0n) <= (kHostFlagsInts - 64) * sizeof(int32_t), "header too large");
  memset(h, 0, offsetof(CgCtl, r0n));
  h->maxit = maxit;
  h->s = s;
  h->kind = sub.kind;
  h->g = sub.g;
  h->hist_cap = hist_cap;
  h->dynamic = dynamic ? 1 : 0;
  h->tol = tol;
  h->eta = eta;
  h->sqrt_eps = sqrt(eps);
  BK_TRY(hipMemcpyAsync(c, h, offsetof(CgCtl, r0n), hipMemcpyHostToDevice, st));

  // R0 = B - A X0 with its Gram matrix; initial normalisation; P = R; rho.
  BK_TRY(launch_spmm<T>(A, s, X, b.R, B, 2, b.partial, nblk, ra, &c->bad_index, nullptr, st));
  BK_TRY(launch_cg_init(c, b.Ga, nullptr, st));
  if (eta > 0.0) BK_TRY(tsqr_run<T>(n, sub, b.R, c->sigma, b.tsqr_ws, b.cnt, done, nullptr, st));
  if (minv) {
    // P = M^-1 R-bar, rho = <P, R-bar>_S
    BK_TRY(launch_row_scale<T>(n, s, minv, b.R, b.P, nullptr, nullptr, st));
    BK_TRY(launch_gram<T>(n, s, b.P, 1, b.R, b.partial, nblk, rr, done, st));
    BK_TRY(launch_cg_init(c, nullptr, b.Gr, st));
  } else {
    BK_TRY(launch_gram<T>(n, s, b.R, 1, b.R, b.partial, nblk, rr, done, st));
    BK_TRY(launch_cg_init(c, nullptr, b.Gr, st));
    BK_TRY(hipMemcpyAsync(b.P, b.R, sizeof(T) * (size_t)n * s, hipMemcpyDeviceToDevice, st));
  }

  const CgCtl* hc = reinterpret_cast<const CgCtl*>(hflags);
  // P_k lives in pbuf[k % 2]; the direction update writes P_{k+1} over
  // P_{k-1} (the X update is deferred by one iteration, see cg_pupdate_kernel)
  T* const pbuf[2] = {b.P, b.P2};
  int k = 0;  // iteration the next enqueued kernels belong to
  int batch = 4, last_iters = -1;
  while (maxit > 0) {
    for (int it = 0; it < batch; ++it, ++k) {
      T* const Pk = pbuf[k & 1];
      T* const Pn = pbuf[(k + 1) & 1];
      {
        // Q = A P and alpha = <P, Q>_S; the reduction's last workgroup
        // computes lambda, lambda sigma and the re-orthonormalisation test
        ProfScope ps(prof, PROF_CG_SPMM, st, k);
        BK_TRY(launch_spmm<T>(A, s, Pk, b.Q, nullptr, 1, b.partial, nblk, ra, &c->bad_index, gate, st,
                              Epi{EPI_CG_ALPHA, c, nullptr}, ps.end()));
      }
      {
        // R~ = R - Q lambda and its Gram; then the stopping test, rho' and beta
        ProfScope ps(prof, PROF_CG_UPDATE, st, k);
        BK_TRY(launch_cg_update<T>(n, s, b.R, b.Q, c, b.partial, nblk, rr, st,
                                   Epi{minv ? EPI_CG_RHO_M : EPI_CG_RHO, c, b.hist}, ps.end(), minv));
      }
      if (always) BK_TRY(cg_normalise<T>(n, sub, b, nblk, st, prof, minv));
      {
        ProfScope ps(prof, PROF_CG_PUPDATE, st, k);
        BK_TRY(launch_cg_pupdate<T>(n, s, X, Pk, Pn, b.R, c, st, minv));
      }
    }
    BK_TRY(hipMemcpyAsync(hflags, c, kCtlHeaderInts * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    BK_TRY(hipStreamSynchronize(st));
    {
      // two-reduction loop: iteration iters-1 is the last whose SpMM and
      // residual update ran; a suspended iteration's direction update waits
      const int it = hc->iters, itp = hc->suspended ? hc->iters - 1 : hc->iters;
      const int live[PROF_N] = {it, it, itp, 0x7fffffff};
      BK_TRY(prof_flush(prof, live));
    }
    if (hc->done) break;
    if (hc->suspended) {
      // iteration iters-1 waits for its re-normalisation (the later kernels
      // of the batch were gated off): run it, finish the iteration's
      // direction update, continue with short batches
      const int ks = hc->iters - 1;
      BK_TRY(cg_normalise<T>(n, sub, b, nblk, st, prof, minv));
      {
        ProfScope ps(prof, PROF_CG_PUPDATE, st);
        BK_TRY(launch_cg_pupdate<T>(n, s, X, pbuf[ks & 1], pbuf[(ks + 1) & 1], b.R, c, st, minv));
      }
      k = ks + 1;
      batch = 2;
    } else {
      if (hc->iters == last_iters) break;  // no progress (cannot happen while live)
      if (batch < 32) batch *= 2;
    }
    last_iters = hc->iters;
  }
  BK_TRY(hipMemcpyAsync(hflags, c, kCtlHeaderInts * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  BK_TRY(hipStreamSynchronize(st));
  res.status = hc->status;
  res.iters = hc->iters;
  res.nreorth = hc->nreorth;
  res.converged = hc->converged;
  res.bad_index = hc->bad_index;
  res.kd_jacobi = hc->kd_jacobi;
  return hipSuccess;
}

template CgBufs<double> carve_cg<double>(Carver&, int64_t, Sub, int, uint32_t*);
template CgBufs<float> carve_cg<float>(Carver&, int64_t, Sub, int, uint32_t*);
template hipError_t cg_run<double>(const CsrView&, Sub, const double*, double*, double, int, double, double, int,
                                   const CgBufs<double>&, hipStream_t, int32_t*, CgResult&, Prof*, const double*);
template hipError_t cg_run<float>(const CsrView&, Sub, const float*, float*, double, int, double, double, int,
                                  const CgBufs<float>&, hipStream_t, int32_t*, CgResult&, Prof*, const double*);

// ---------------------------------------------------------- Gropp BCG --
// Re-normalisation of R~ inside Gropp's block CG: (R-bar, gamma) =
// Norm_S(R~), then Z = M^-1 R-bar directly (Z aliases R for M = I), rho' =
// <Z, R-bar>_S and the coefficient step that finishes it (sigma, beta).
static hipError_t gropp_normalise(int64_t n, Sub sub, const CgBufs<double>& b, double* Z, int nblk, hipStream_t st,
                                  Prof* prof, const double* minv) {
  CgCtl* c = b.ctl;
  ProfScope ps(prof, PROF_CG_NORMALISE, st);
  BK_TRY(tsqr_run<double>(n, sub, b.R, c->gamma, b.tsqr_ws, b.cnt, &c->done, &c->fire, st));
  if (minv) BK_TRY(launch_row_scale<double>(n, sub.s, minv, b.R, Z, &c->done, &c->fire, st));
  BK_TRY(launch_gram<double>(n, sub.s, Z, 1, b.R, b.partial, nblk, Red{b.Gq, b.gpart, b.cnt}, &c->done, st,
                             &c->fire));
  return launch_cg_reortho_fin(c, sub.s, b.Gq, st);
}

hipError_t gropp_run(const CsrView& A, Sub sub, const double* B, double* X, double tol, int maxit, double eta,
                     int hist_cap, const CgBufs<double>& b, double* U, double* Zbuf, hipStream_t st, int32_t* hflags,
                     CgResult& res, Prof* prof, const double* minv) {
  const int64_t n = A.n;
  const int s = sub.s;
  const size_t blk = (size_t)n * s;
  const double eps = DBL_EPSILON;
  const int nblk = stream_grid(n, s, sizeof(double));
  CgCtl* c = b.ctl;
  int32_t* gate = &c->gate;
  const Red ra{b.Ga, b.gpart, b.cnt}, rr{b.Gr, b.gpart, b.cnt};
  const bool always = eta > 0.0 && (isinf(eta) || eta * sqrt(eps) > 1.0);
  const bool dynamic = eta > 0.0 && !always && sub.g > 1;
  // Z = M^-1 R-bar is carried by its recurrence; for M = I the recurrence
  // repeats the residual update operation for operation, so Z is R-bar
  double* Z = minv ? Zbuf : b.R;

  CgCtl* h = reinterpret_cast<CgCtl*>(hflags + 64);
  memset(h, 0, offsetof(CgCtl, r0n));
  h->maxit = maxit;
  h->s = s;
  h->kind = sub.kind;
  h->g = sub.g;
  h->hist_cap = hist_cap;
  h->dynamic = dynamic ? 1 : 0;
  h->tol = tol;
  h->eta = eta;
  h->sqrt_eps = sqrt(eps);
  BK_TRY(hipMemcpyAsync(c, h, offsetof(CgCtl, r0n), hipMemcpyHostToDevice, st));

  // R0 = B - A X0; normalisation; P0 = Z0 = M^-1 R-bar; rho = <P0, R-bar>_S;
  // Q0 = A P0; alpha = <P0, Q0>_S and its coefficient step (lambda)
  BK_TRY(launch_spmm<double>(A, s, X, b.R, B, 2, b.partial, nblk, ra, &c->bad_index, nullptr, st));
  BK_TRY(launch_cg_init(c, b.Ga, nullptr, st));
  if (eta > 0.0) BK_TRY(tsqr_run<double>(n, sub, b.R, c->sigma, b.tsqr_ws, b.cnt, &c->done, nullptr, st));
  if (minv) {
    BK_TRY(launch_row_scale<double>(n, s, minv, b.R, b.P, nullptr, nullptr, st));
    BK_TRY(hipMemcpyAsync(Z, b.P, sizeof(double) * blk, hipMemcpyDeviceToDevice, st));
  } else {
    BK_TRY(hipMemcpyAsync(b.P, b.R, sizeof(double) * blk, hipMemcpyDeviceToDevice, st));
  }
  BK_TRY(launch_gram<double>(n, s, b.P, 1, b.R, b.partial, nblk, rr, &c->done, st));
  BK_TRY(launch_cg_init(c, nullptr, b.Gr, st));
  BK_TRY(launch_spmm<double>(A, s, b.P, b.Q, nullptr, 0, nullptr, nblk, ra, &c->bad_index, &c->done, st));
  BK_TRY(launch_gram_partials(n, s, b.P, b.Q, b.partial, nblk, 0, &c->done, nullptr, st));
  BK_TRY(launch_reduce(s, b.partial, false, nblk, 1, ra, gate, nullptr, Epi{EPI_CG_ALPHA, c, nullptr}, st));

  const CgCtl* hc = reinterpret_cast<const CgCtl*>(hflags);
  // P_k lives in pbuf[k % 2] (the direction pass writes P_{k+1} over
  // P_{k-1}, whose term the deferred X update reads first)
  double* const pbuf[2] = {b.P, b.P2};
  // the rest of iteration k after its residual pass (and, if it fired, its
  // re-normalisation): U = A Z, the direction pass and the next alpha
  auto tail = [&](int k) -> hipError_t {
    {
      ProfScope ps(prof, PROF_CG_SPMM, st, k);
      BK_TRY(launch_spmm<double>(A, s, Z, U, nullptr, 0, nullptr, nblk, ra, &c->bad_index, gate, st, Epi{},
                                 ps.end()));
    }
    {
      ProfScope ps(prof, PROF_CG_PUPDATE, st, k);
      BK_TRY(launch_gropp_dir(n, s, X, pbuf[k & 1], pbuf[(k + 1) & 1], Z, U, b.Q, c, b.partial, nblk, st));
    }
    return launch_reduce(s, b.partial, false, nblk, 1, ra, gate, nullptr, Epi{EPI_CG_ALPHA, c, nullptr}, st);
  };
  int k = 0, batch = 4, last_iters = -1;
  while (maxit > 0) {
    for (int it = 0; it < batch; ++it, ++k) {
      {
        // R~ = R-bar - Q lambda (and Z = Z - M^-1 Q lambda); stopping test,
        // rho' = <Z, R~>_S and beta in the reduction's coefficient step
        ProfScope ps(prof, PROF_CG_UPDATE, st, k);
        if (minv) {
          BK_TRY(launch_gropp_update(n, s, b.R, b.Q, Z, c, b.partial, nblk, minv, st));
          BK_TRY(launch_reduce(s, b.partial, false, nblk, 1, rr, gate, nullptr, Epi{EPI_CG_RHO_M, c, b.hist}, st));
        } else {
          BK_TRY(launch_cg_update<double>(n, s, b.R, b.Q, c, b.partial, nblk, rr, st, Epi{EPI_CG_RHO, c, b.hist},
                                          nullptr, nullptr));
        }
      }
      if (always) BK_TRY(gropp_normalise(n, sub, b, Z, nblk, st, prof, minv));
      BK_TRY(tail(k));
    }
    BK_TRY(hipMemcpyAsync(hflags, c, kCtlHeaderInts * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    BK_TRY(hipStreamSynchronize(st));
    {
      const int it = hc->iters, itp = hc->suspended ? hc->iters - 1 : hc->iters;
      const int live[PROF_N] = {itp, it, itp, 0x7fffffff};
      BK_TRY(prof_flush(prof, live));
    }
    if (hc->done) break;
    if (hc->suspended) {
      // iteration iters-1 waits for its re-normalisation: run it and the
      // rest of that iteration, then continue with short batches
      const int ks = hc->iters - 1;
      BK_TRY(gropp_normalise(n, sub, b, Z, nblk, st, prof, minv));
      BK_TRY(tail(ks));
      k = ks + 1;
      batch = 2;
    } else {
      if (hc->iters == last_iters) break;
      if (batch < 32) batch *= 2;
    }
    last_iters = hc->iters;
  }
  BK_TRY(hipMemcpyAsync(hflags, c, kCtlHeaderInts * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  BK_TRY(hipStreamSynchronize(st));
  res.status = hc->status;
  res.iters = hc->iters;
  res.nreorth = hc->nreorth;
  res.converged = hc->converged;
  res.bad_index = hc->bad_index;
  res.kd_jacobi = hc->kd_jacobi;
  return hipSuccess;
}

// ------------------------------------------------------ multicolour SSOR --
SsorWs ssor_carve(Carver& c, int64_t n) {
  SsorWs w;
  w.d = c.take<double>((size_t)n);
  w.perm = c.take<int32_t>((size_t)n);
  w.off = c.take<int32_t>(kMaxColors + 1);
  w.cursor = c.take<int32_t>(kMaxColors);
  w.count = c.take<int32_t>(kMaxColors);
  w.misc = c.take<int32_t>(4);  // ncolors, bad[3]
  return w;
}

hipError_t ssor_plan_build(const CsrView& A, const int32_t* colors, double omega, const SsorWs& w, hipStream_t st,
                           SsorPlan& plan, int& err) {
  err = 0;
  BK_TRY(hipMemsetAsync(w.count, 0, sizeof(int32_t) * kMaxColors, st));
  BK_TRY(hipMemsetAsync(w.misc, 0, sizeof(int32_t) * 4, st));
  BK_TRY(launch_ssor_check(A, colors, w.d, w.misc, w.count, w.misc + 1, st));
  int32_t misc[4];
  BK_TRY(hipMemcpyAsync(misc, w.misc, sizeof(misc), hipMemcpyDeviceToHost, st));
  BK_TRY(hipStreamSynchronize(st));
  if (misc[1]) err = 1;
  else if (misc[2]) err = 2;
  else if (misc[3]) err = 3;
  if (err) return hipSuccess;
  const int nc = misc[0];
  BK_TRY(launch_ssor_bucket(A.n, colors, w.count, w.misc, w.off, w.cursor, w.perm, st));
  static thread_local int32_t cnt[kMaxColors];
  BK_TRY(hipMemcpyAsync(cnt, w.count, sizeof(int32_t) * nc, hipMemcpyDeviceToHost, st));
  BK_TRY(hipStreamSynchronize(st));
  int64_t cmax = 0;
  for (int c = 0; c < nc; ++c) cmax = cnt[c] > cmax ? cnt[c] : cmax;
  plan.A = A;
  plan.colors = colors;
  plan.d = w.d;
  plan.perm = w.perm;
  plan.off = w.off;
  plan.ncolors = nc;
  plan.count_max = cmax;
  plan.omega = omega;
  return hipSuccess;
}

// Re-normalisation with the SSOR preconditioner: (R-bar, gamma) = Norm_S(R~),
// Z = M^-1 R-bar into Q, rho' = <Z, R-bar>_S, then sigma, beta (cg_reortho_fin).
static hipError_t ssor_normalise(int64_t n, Sub sub, const CgBufs<double>& b, const SsorPlan& m, int nblk,
                                 hipStream_t st, Prof* prof) {
  CgCtl* c = b.ctl;
  ProfScope ps(prof, PROF_CG_NORMALISE, st);
  BK_TRY(tsqr_run<double>(n, sub, b.R, c->gamma, b.tsqr_ws, b.cnt, &c->done, &c->fire, st));
  BK_TRY(launch_ssor_apply(m, sub.s, b.R, b.Q, &c->done, nullptr, &c->fire, st));
  BK_TRY(launch_gram<double>(n, sub.s, b.Q, 1, b.R, b.partial, nblk, Red{b.Gq, b.gpart, b.cnt}, &c->done, st,
                             &c->fire));
  return launch_cg_reortho_fin(c, sub.s, b.Gq, st);
}

hipError_t pcg_ssor_run(const CsrView& A, Sub sub, const double* B, double* X, double tol, int maxit, double eta,
                        int hist_cap, const CgBufs<double>& b, const SsorPlan& m, hipStream_t st, int32_t* hflags,
                        CgResult& res, Prof* prof) {
  const int64_t n = A.n;
  const int s = sub.s;
  const double eps = DBL_EPSILON;
  const int nblk = stream_grid(n, s, sizeof(double));
  const int64_t ss = (int64_t)s * s;
  CgCtl* c = b.ctl;
  int32_t* done = &c->done;
  int32_t* gate = &c->gate;
  const Red ra{b.Ga, b.gpart, b.cnt}, rr{b.Gr, b.gpart, b.cnt};
  const bool always = eta > 0.0 && (isinf(eta) || eta * sqrt(eps) > 1.0);
  const bool dynamic = eta > 0.0 && !always && sub.g > 1;

  CgCtl* h = reinterpret_cast<CgCtl*>(hflags + 64);
  memset(h, 0, offsetof(CgCtl, r0n));
  h->maxit = maxit;
  h->s = s;
  h->kind = sub.kind;
  h->g = sub.g;
  h->hist_cap = hist_cap;
  h->dynamic = dynamic ? 1 : 0;
  h->tol = tol;
  h->eta = eta;
  h->sqrt_eps = sqrt(eps);
  BK_TRY(hipMemcpyAsync(c, h, offsetof(CgCtl, r0n), hipMemcpyHostToDevice, st));

  // R0 = B - A X0; initial normalisation; P = M^-1 R-bar, rho = <P, R-bar>_S
  BK_TRY(launch_spmm<double>(A, s, X, b.R, B, 2, b.partial, nblk, ra, &c->bad_index, nullptr, st));
  BK_TRY(launch_cg_init(c, b.Ga, nullptr, st));
  if (eta > 0.0) BK_TRY(tsqr_run<double>(n, sub, b.R, c->sigma, b.tsqr_ws, b.cnt, done, nullptr, st));
  BK_TRY(launch_ssor_apply(m, s, b.R, b.P, done, nullptr, nullptr, st));
  BK_TRY(launch_gram<double>(n, s, b.P, 1, b.R, b.partial, nblk, rr, done, st));
  BK_TRY(launch_cg_init(c, nullptr, b.Gr, st));

  const CgCtl* hc = reinterpret_cast<const CgCtl*>(hflags);
  double* const pbuf[2] = {b.P, b.P2};
  int k = 0, batch = 4, last_iters = -1;
  while (maxit > 0) {
    for (int it = 0; it < batch; ++it, ++k) {
      double* const Pk = pbuf[k & 1];
      double* const Pn = pbuf[(k + 1) & 1];
      {
        ProfScope ps(prof, PROF_CG_SPMM, st, k);
        BK_TRY(launch_spmm<double>(A, s, Pk, b.Q, nullptr, 1, b.partial, nblk, ra, &c->bad_index, gate, st,
                                   Epi{EPI_CG_ALPHA, c, nullptr}, ps.end()));
      }
      {
        // R~ = R - Q lambda (Gram of R~ into the first half of each partial);
        // unless R~ is re-normalised, Z = M^-1 R~ into Q and <Z, R~> into the
        // second half; one reduction for both (stopping test, rho', beta)
        ProfScope ps(prof, PROF_CG_UPDATE, st, k);
        BK_TRY(launch_cg_update_partials(n, s, b.R, b.Q, c, b.partial, nblk, 2 * ss, st));
        BK_TRY(launch_ssor_apply(m, s, b.R, b.Q, gate, &c->fire, nullptr, st));
        BK_TRY(launch_gram_partials(n, s, b.Q, b.R, b.partial + ss, nblk, 2 * ss, gate, &c->fire, st));
        BK_TRY(launch_reduce(s, b.partial, false, nblk, 1, rr, gate, nullptr, Epi{EPI_CG_RHO_M, c, b.hist}, st));
      }
      if (always) BK_TRY(ssor_normalise(n, sub, b, m, nblk, st, prof));
      {
        ProfScope ps(prof, PROF_CG_PUPDATE, st, k);
        BK_TRY(launch_cg_pupdate<double>(n, s, X, Pk, Pn, b.Q, c, st, nullptr));
      }
    }
    BK_TRY(hipMemcpyAsync(hflags, c, kCtlHeaderInts * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    BK_TRY(hipStreamSynchronize(st));
    {
      // two-reduction loop: iteration iters-1 is the last whose SpMM and
      // residual update ran; a suspended iteration's direction update waits
      const int it = hc->iters, itp = hc->suspended ? hc->iters - 1 : hc->iters;
      const int live[PROF_N] = {it, it, itp, 0x7fffffff};
      BK_TRY(prof_flush(prof, live));
    }
    if (hc->done) break;
    if (hc->suspended) {
      const int ks = hc->iters - 1;
      BK_TRY(ssor_normalise(n, sub, b, m, nblk, st, prof));
      {
        ProfScope ps(prof, PROF_CG_PUPDATE, st);
        BK_TRY(launch_cg_pupdate<double>(n, s, X, pbuf[ks & 1], pbuf[(ks + 1) & 1], b.Q, c, st, nullptr));
      }
      k = ks + 1;
      batch = 2;
    } else {
      if (hc->iters == last_iters) break;
      if (batch < 32) batch *= 2;
    }
    last_iters = hc->iters;
  }
  BK_TRY(hipMemcpyAsync(hflags, c, kCtlHeaderInts * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  BK_TRY(hipStreamSynchronize(st));
  res.status = hc->status;
  res.iters = hc->iters;
  res.nreorth = hc->nreorth;
  res.converged = hc->converged;
  res.bad_index = hc->bad_index;
  res.kd_jacobi = hc->kd_jacobi;
  return hipSuccess;
}

// ------------------------------------------------- one-reduction block CG --
// Per iteration k: the SpMM U = A R-bar^k writes the Gram partials R^T U
// into slot 1 of the partials whose slot 0 the previous fused pass filled
// with R^T R; the one reduction's epilogue runs the whole coefficient step
// (cg1r_body); the fused pass updates P, Q, X and R-bar (and the next slot
// 0).  Three launches and one reduction per iteration.
static hipError_t cg1r_normalise(int64_t n, Sub sub, const CgBufs<double>& b, int nblk, int k, hipStream_t st,
                                 Prof* prof) {
  CgCtl* c = b.ctl;
  ProfScope ps(prof, PROF_CG_NORMALISE, st);
  BK_TRY(tsqr_run<double>(n, sub, b.R, c->gamma, b.tsqr_ws, b.cnt, &c->done, &c->fire, st));
  BK_TRY(launch_cg1r_fin(c, sub.s, st));
  return launch_cg1r_pass(n, sub.s, b.R, b.P2, b.P, b.Q, nullptr, c, b.partial, nblk, k, 1, st);
}

hipError_t cg1r_run(const CsrView& A, Sub sub, const double* B, double* X, double tol, int maxit, double eta,
                    int hist_cap, const CgBufs<double>& b, hipStream_t st, int32_t* hflags, CgResult& res,
                    Prof* prof) {
  const int64_t n = A.n;
  const int s = sub.s;
  const double eps = DBL_EPSILON;
  // the fused pass and the SpMM write the two halves of one partial per
  // workgroup: both run on the SpMM's grid
  const int nblk = spmm_grid<double>(A, s, 1, stream_grid(n, s, sizeof(double)));
  CgCtl* c = b.ctl;
  int32_t* gate = &c->gate;
  const bool always = eta > 0.0 && (isinf(eta) || eta * sqrt(eps) > 1.0);
  const bool dynamic = eta > 0.0 && !always && sub.g > 1;

  CgCtl* h = reinterpret_cast<CgCtl*>(hflags + 64);
  memset(h, 0, offsetof(CgCtl, r0n));
  h->maxit = maxit;
  h->s = s;
  h->kind = sub.kind;
  h->g = sub.g;
  h->hist_cap = hist_cap;
  h->dynamic = dynamic ? 1 : 0;
  h->tol = tol;
  h->eta = eta;
  h->sqrt_eps = sqrt(eps);
  BK_TRY(hipMemcpyAsync(c, h, offsetof(CgCtl, r0n), hipMemcpyHostToDevice, st));

  // R0 = B - A X0 and its column norms; initial normalisation; slot 0 of the
  // partials: the Gram of R-bar^0
  BK_TRY(launch_spmm<double>(A, s, X, b.R, B, 2, b.partial, stream_grid(n, s, sizeof(double)),
                             Red{b.Ga, b.gpart, b.cnt}, &c->bad_index, nullptr, st));
  BK_TRY(launch_cg_init(c, b.Ga, nullptr, st));
  if (eta > 0.0) BK_TRY(tsqr_run<double>(n, sub, b.R, c->sigma, b.tsqr_ws, b.cnt, &c->done, nullptr, st));
  BK_TRY(launch_cg1r_pass(n, s, b.R, b.P2, b.P, b.Q, X, c, b.partial, nblk, -1, 1, st));

  const CgCtl* hc = reinterpret_cast<const CgCtl*>(hflags);
  const Red red{b.Gr, b.gpart, b.cnt};
  int k = 0, batch = 4, last_iters = -1;
  while (maxit > 0) {
    for (int it = 0; it < batch; ++it, ++k) {
      {
        ProfScope ps(prof, PROF_CG_SPMM, st, k);
        BK_TRY(launch_spmm<double>(A, s, b.R, b.P2, nullptr, 1, b.partial, nblk, red, &c->bad_index, gate, st,
                                   Epi{EPI_CG_1R, c, b.hist}, ps.end(), 1, 2));
      }
      {
        ProfScope ps(prof, PROF_CG_UPDATE, st, k);
        BK_TRY(launch_cg1r_pass(n, s, b.R, b.P2, b.P, b.Q, X, c, b.partial, nblk, k, 0, st));
      }
      if (always) BK_TRY(cg1r_normalise(n, sub, b, nblk, k, st, prof));
    }
    BK_TRY(hipMemcpyAsync(hflags, c, kCtlHeaderInts * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    BK_TRY(hipStreamSynchronize(st));
    {
      // one-reduction loop: the SpMM of iteration iters decided the end (or
      // the suspension); the fused pass of that iteration ran unless it ended
      const int it = hc->iters + 1, itp = hc->done ? hc->iters : hc->iters + 1;
      const int live[PROF_N] = {it, itp, 0x7fffffff, 0x7fffffff};
      BK_TRY(prof_flush(prof, live));
    }
    if (hc->done) break;
    if (hc->suspended) {
      // iteration j fired: its fused pass ran, the later kernels of the batch
      // were gated off; re-normalise R~^{j+1} and resume at iteration j + 1
      const int j = hc->lam_iter;
      BK_TRY(cg1r_normalise(n, sub, b, nblk, j, st, prof));
      k = j + 1;
      batch = 2;
    } else {
      if (hc->iters == last_iters && hc->lam_iter + 1 == k) {
        // no progress although live (cannot happen): stop
        break;
      }
      if (batch < 32) batch *= 2;
    }
    last_iters = hc->iters;
  }
  BK_TRY(hipMemcpyAsync(hflags, c, kCtlHeaderInts * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  BK_TRY(hipStreamSynchronize(st));
  // an even last iteration j deferred its X term P_j (lambda sigma)_j
  const int j = hc->lam_iter;
  if (j >= 0 && (j & 1) == 0) {
    BK_TRY(launch_cg1r_pass(n, s, b.R, b.P2, b.P, b.Q, X, c, b.partial, nblk, j, 2, st));
    BK_TRY(hipStreamSynchronize(st));
  }
  res.status = hc->status;
  res.iters = hc->iters;
  res.nreorth = hc->nreorth;
  res.converged = hc->converged;
  res.bad_index = hc->bad_index;
  res.kd_jacobi = hc->kd_jacobi;
  return hipSuccess;
}

// ------------------------------------------------------ block BiCGStab --
BcBufs carve_bc(Carver& c, int64_t n, Sub sub, int hist_cap, uint32_t* cnt) {
  const int s = sub.s;
  const int nblk = stream_grid(n, s, sizeof(double));
  const size_t blk = (size_t)n * s;
  BcBufs b;
  b.P = c.take<double>(blk);
  b.Pn = c.take<double>(blk);
  b.W2 = c.take<double>(2 * blk);
  b.W3 = c.take<double>(3 * blk);
  b.partial = c.take<double>((size_t)3 * nblk * s * s);
  b.gpart = c.take<double>(3 * red_gpart_count(nblk, s));
  b.G = c.take<double>((size_t)3 * s * s);
  b.Grr = c.take<double>((size_t)s * s);
  b.hist = c.take<double>((size_t)(hist_cap > 0 ? hist_cap : 1));
  b.ctl = c.take<CgCtl>(1);
  b.aux = c.take<BcAux>(1);
  b.tsqr_ws = c.take<char>(tsqr_workspace_bytes(n, sub));
  b.cnt = cnt;
  return b;
}

// One iteration of Algorithm "BBiCGStab with Adaptive Residual
// Re-Orthonormalization" (Ch. 6) with M = I, as a sequence of launches that
// all become no-ops once ctl->done is set:
//   Q = A P; [Q^T R~0 | R^T R~0]; lambda, kappa_D test (bc_lambda);
//   S = R - Q lambda; if the test fired: (S, gamma) = Norm_S(S), sigma =
//   gamma sigma (T = S either way, M = I); U = A S;
//   [S^T U | U^T U | R~0^T U]; omega, beta (bc_omega);
//   X += P (lambda sigma_old) + S (omega sigma); R = S - omega U;
//   R^T R and the stopping test (bc_stop); P' = R + P beta - Q (omega beta).
// lambda sigma is formed before sigma changes, omega sigma after (the X
// update by T carries the new transformation).
hipError_t bc_run(const CsrView& A, Sub sub, const double* B, double* X, double tol, int maxit, double eta,
                  int hist_cap, const BcBufs& b, hipStream_t st, int32_t* hflags, BcResult& res,
                  const double* r0n_fixed) {
  const int64_t n = A.n;
  const int s = sub.s;
  const size_t blk = (size_t)n * s;
  const int nblk = stream_grid(n, s, sizeof(double));
  CgCtl* c = b.ctl;
  BcAux* x = b.aux;
  int32_t* done = &c->done;
  double* Q = b.W2;
  double* R = b.W2 + blk;
  double* S = b.W3;
  double* U = b.W3 + blk;
  double* Rt = b.W3 + 2 * blk;
  const Red red{b.G, b.gpart, b.cnt}, rrr{b.Grr, b.gpart, b.cnt};

  CgCtl* h = reinterpret_cast<CgCtl*>(hflags + 64);
  memset(h, 0, offsetof(CgCtl, r0n));
  h->maxit = maxit;
  h->s = s;
  h->kind = sub.kind;
  h->g = sub.g;
  h->hist_cap = hist_cap;
  h->tol = tol;
  h->eta = eta;
  h->sqrt_eps = sqrt(DBL_EPSILON);
  BK_TRY(hipMemcpyAsync(c, h, offsetof(CgCtl, r0n), hipMemcpyHostToDevice, st));

  // R0 = B - A X0 and its Gram; initial normalisation; P = R, R~0 = P
  BK_TRY(launch_spmm<double>(A, s, X, R, B, 2, b.partial, nblk, rrr, &c->bad_index, nullptr, st));
  BK_TRY(launch_cg_init(c, b.Grr, nullptr, st));
  // a restart keeps the stopping test's denominators of the first start
  if (r0n_fixed) BK_TRY(hipMemcpyAsync(c->r0n, r0n_fixed, sizeof(double) * s, hipMemcpyDeviceToDevice, st));
  if (eta > 0.0) {
    BK_TRY(tsqr_run<double>(n, sub, R, c->sigma, b.tsqr_ws, b.cnt, done, nullptr, st));
    BK_TRY(launch_gram<double>(n, s, R, 1, R, b.partial, nblk, rrr, done, st));
  }
  BK_TRY(hipMemcpyAsync(b.P, R, sizeof(double) * blk, hipMemcpyDeviceToDevice, st));
  BK_TRY(hipMemcpyAsync(Rt, R, sizeof(double) * blk, hipMemcpyDeviceToDevice, st));

  const CgCtl* hc = reinterpret_cast<const CgCtl*>(hflags);
  double* P = b.P;
  double* Pn = b.Pn;
  int batch = 4;
  while (maxit > 0) {
    for (int it = 0; it < batch; ++it) {
      BK_TRY(launch_spmm<double>(A, s, P, Q, nullptr, 0, nullptr, nblk, red, &c->bad_index, done, st));
      BK_TRY(launch_gram<double>(n, s, Q, 2, Rt, b.partial, nblk, red, done, st));  // Q^T R~0, R^T R~0
      BK_TRY(launch_bc_lambda(c, x, s, b.G, b.Grr, st));
      BK_TRY(launch_lincomb<double>(n, s, R, Q, x->neglam, nullptr, nullptr, S, done, st));
      BK_TRY(tsqr_run<double>(n, sub, S, c->gamma, b.tsqr_ws, b.cnt, done, &c->fire, st));
      BK_TRY(launch_bc_sigma(c, st));
      BK_TRY(launch_spmm<double>(A, s, S, U, nullptr, 0, nullptr, nblk, red, &c->bad_index, done, st));
      BK_TRY(launch_gram<double>(n, s, S, 3, U, b.partial, nblk, red, done, st));  // S^T U, U^T U, R~0^T U
      BK_TRY(launch_bc_omega(c, x, b.G, st));
      // X, R and P' in one pass (P' of the last iteration is never used)
      BK_TRY(launch_bc_tail(n, s, X, P, S, U, Q, R, Pn, c->lamsig, x, done, st));
      BK_TRY(launch_gram<double>(n, s, R, 1, R, b.partial, nblk, rrr, done, st));
      BK_TRY(launch_bc_stop(c, b.Grr, b.hist, st));
      std::swap(P, Pn);
    }
    BK_TRY(hipMemcpyAsync(hflags, c, kCtlHeaderInts * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    BK_TRY(hipStreamSynchronize(st));
    if (hc->done) break;
    if (batch < 32) batch *= 2;
  }
  BK_TRY(hipMemcpyAsync(hflags, c, kCtlHeaderInts * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  BK_TRY(hipStreamSynchronize(st));
  res.status = hc->status;
  res.iters = hc->iters;
  res.nreorth = hc->nreorth;
  res.converged = hc->converged;
  res.bad_index = hc->bad_index;
  return hipSuccess;
}

// ------------------------------------------------------ true residuals --
hipError_t true_relres(const CsrView& A, int s, const double* B, const double* X, double* R, double* partial,
                       double* gpart, uint32_t* cnt, double* G, const double* r0n, double* relres, int32_t* flag,
                       double* scale_scratch, hipStream_t st) {
  const int nblk = stream_grid(A.n, s, sizeof(double));
  BK_TRY(launch_spmm<double>(A, s, X, R, B, 2, partial, nblk, Red{G, gpart, cnt}, nullptr, nullptr, st));
  return launch_ir_check(s, G, const_cast<double*>(r0n), scale_scratch, relres, flag, 0.0, 0, st);
}

// ------------------------------------------------ iterative refinement --
IrBufs carve_ir(Carver& c, int64_t n, int64_t nnz, Sub sub, uint32_t* cnt) {
  const int s = sub.s;
  const int nblk = stream_grid(n, s, sizeof(double));
  IrBufs b;
  b.A32 = c.take<float>((size_t)(nnz > 0 ? nnz : 1));
  b.R32 = c.take<float>((size_t)n * s);
  b.X32 = c.take<float>((size_t)n * s);
  b.R64 = c.take<double>((size_t)n * s);
  b.partial = c.take<double>((size_t)nblk * s * s);
  b.gpart = c.take<double>(red_gpart_count(nblk, s));
  b.G = c.take<double>((size_t)s * s);
  b.r0n = c.take<double>(kMaxS);
  b.scale = c.take<double>(kMaxS);
  b.relres = c.take<double>(kMaxS);
  b.flag = c.take<int32_t>(4);
  b.cnt = cnt;
  b.cg = carve_cg<float>(c, n, sub, 0, cnt);
  return b;
}

// Mixed precision: the FP64 residual R = B - A X is scaled column-wise to unit
// norm, rounded to FP32, and an FP32 block CG solves A D = R/|R| to the inner
// tolerance; X += D |R| in FP64; repeat until the FP64 residual meets tol.
hipError_t ir_run(const CsrView& A, Sub sub, const double* B, double* X, double tol, int maxit, double eta,
                  double inner_tol, int max_outer, double* hist_host, int hist_cap, const IrBufs& b, hipStream_t st,
                  int32_t* hflags, double* relres_host, IrResult& res, Prof* prof) {
  const int64_t n = A.n;
  const int s = sub.s;
  const int nblk = stream_grid(n, s, sizeof(double));
  BK_TRY(launch_cast_f32(A.nnz, static_cast<const double*>(A.val), b.A32, st));
  CsrView A32 = A;
  A32.val = b.A32;
  A32.ell_w = b.ell_w;
  A32.ell_col = b.ell_col;
  A32.ell_val = b.ell_val;
  A32.ell_diag0 = b.ell_diag0;
  int32_t* dflag = b.flag;
  BK_TRY(hipMemsetAsync(dflag, 0, 4 * sizeof(int32_t), st));
  for (int outer = 0;; ++outer) {
    BK_TRY(launch_spmm<double>(A, s, X, b.R64, B, 2, b.partial, nblk, Red{b.G, b.gpart, b.cnt}, dflag + 2, nullptr,
                               st));
    BK_TRY(launch_ir_check(s, b.G, b.r0n, b.scale, b.relres, dflag, tol, outer == 0, st));
    BK_TRY(hipMemcpyAsync(hflags, dflag, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    BK_TRY(hipMemcpyAsync(relres_host, b.relres, s * sizeof(double), hipMemcpyDeviceToHost, st));
    BK_TRY(hipStreamSynchronize(st));
    double m = 0.0;
    for (int i = 0; i < s; ++i) m = fmax(m, relres_host[i]);
    if (outer > 0 && res.hist_len < hist_cap && hist_host) hist_host[res.hist_len++] = m;
    res.outer = outer;
    res.bad_index = hflags[2];
    if (hflags[2]) return hipSuccess;
    if (hflags[1]) {
      res.status = -3;
      return hipSuccess;
    }
    if (hflags[0]) {
      res.converged = 1;
      return hipSuccess;
    }
    if (outer >= max_outer) {
      res.status = res.inner_status;
      return hipSuccess;
    }
    BK_TRY(launch_cast_scale_f32(n, s, b.R64, b.scale, b.R32, st));
    BK_TRY(hipMemsetAsync(b.X32, 0, sizeof(float) * (size_t)n * s, st));
    CgResult r;
    BK_TRY(cg_run<float>(A32, sub, b.R32, b.X32, inner_tol, maxit, eta, (double)FLT_EPSILON, 0, b.cg, st, hflags, r,
                         prof));
    res.inner_iters += r.iters;
    res.nreorth += r.nreorth;
    if (r.bad_index) {
      res.bad_index = 1;
      return hipSuccess;
    }
    // An inner breakdown or non-finite value ends the refinement when the
    // inner solve made no progress, or when the previous outer step's inner
    // solve failed the same way; otherwise its partial correction is kept and
    // the failure is remembered (and reported if the refinement ends
    // unconverged).
    if (r.status != 0 && (r.iters <= 1 || r.status == res.inner_status)) {
      res.status = r.status;
      res.inner_status = r.status;
      return hipSuccess;
    }
    res.inner_status = r.status;
    BK_TRY(launch_accum_scaled(n, s, b.X32, b.scale, X, st));
  }
}

// ------------------------------------------------------------ block GMRes --
GmBufs carve_gm(Carver& c, int64_t n, Sub sub, int m, int hist_cap, uint32_t* cnt) {
  const int s = sub.s, ss = s * s;
  const int nblk = stream_grid(n, s, sizeof(double));
  GmBufs b;
  b.V = c.take<double>((size_t)(m + 1) * n * s);
  b.partial = c.take<double>((size_t)(m + 1) * nblk * ss);
  b.gpart = c.take<double>((size_t)(m + 1) * red_gpart_count(nblk, s));
  b.Gb = c.take<double>((size_t)(m + 1) * ss);
  b.H1 = c.take<double>((size_t)(m + 1) * ss);
  b.H2 = c.take<double>((size_t)(m + 1) * ss);
  b.H = c.take<double>((size_t)(m + 1) * m * ss);
  b.sig = c.take<double>((size_t)(m + 1) * ss);
  b.Om = c.take<double>((size_t)m * 4 * ss);
  b.zeta = c.take<double>((size_t)m * ss);
  b.sigma0 = c.take<double>((size_t)ss);
  b.gam = c.take<double>((size_t)ss);
  b.hist = c.take<double>((size_t)(hist_cap > 0 ? hist_cap : 1));
  b.relres = c.take<double>(kMaxS);
  b.flag = c.take<int32_t>(4);
  b.plans = c.take<int32_t>((size_t)4 * (m + 1));
  b.ctl = c.take<GmCtl>(1);
  b.tsqr_ws = c.take<char>(tsqr_workspace_bytes(n, sub));
  b.cnt = cnt;
  return b;
}

hipError_t gm_run(const CsrView& A, Sub sub, const double* B, double* X, double tol, int maxit, int m,
                  int hist_cap, const GmBufs& b, hipStream_t st, int32_t* hflags, GmResult& res, int orth) {
  const int64_t n = A.n;
  const int s = sub.s;
  const size_t blk = (size_t)n * s;
  const int nblk = stream_grid(n, s, sizeof(double));
  const Red red{b.Gb, b.gpart, b.cnt};
  // The block subalgebra's projection is the identity: its batched Grams are
  // reduced straight into H instead of through Gb and a projection launch.
  const bool proj_id = sub.kind == BLOCK;
  auto red_to = [&](double* target) { return proj_id ? Red{target, b.gpart, b.cnt} : red; };
  GmCtl* c = b.ctl;
  int32_t* done = &c->done;
  GmCtl* h = reinterpret_cast<GmCtl*>(hflags + 64);
  memset(h, 0, sizeof(GmCtl));
  h->maxit = maxit;
  h->s = s;
  h->kind = sub.kind;
  h->g = sub.g;
  h->m = m;
  h->hist_cap = hist_cap;
  h->tol = tol;
  BK_TRY(hipMemcpyAsync(c, h, sizeof(GmCtl), hipMemcpyHostToDevice, st));
  const size_t ss = (size_t)s * s;
  // the step kernel adds the coefficients of two passes; the pipelined
  // orthogonalisation has one, so the second stays zero
  if (orth > 0) BK_TRY(hipMemsetAsync(b.H2, 0, sizeof(double) * (size_t)(m + 1) * ss, st));
  const int lmax = pgs_max_updates(s);
  // The Arnoldi normalisers are enqueued without the Householder fallback
  // of CholeskyQR (its launches, gated off when unused, cost more than the
  // rest of the normaliser at this width); each step records its CholeskyQR
  // decisions, and a cycle in which one step needed the fallback is redone
  // with it, from the control block as it was before the cycle.
  GmCtl before;
  std::vector<int32_t> hplans((size_t)4 * (m + 1));
  bool safe = false;
  for (int cycle = 0;; ++cycle) {
    if (cycle > 0 || safe) BK_TRY(hipMemcpyAsync(&before, c, sizeof(GmCtl), hipMemcpyDeviceToHost, st));
    BK_TRY(hipStreamSynchronize(st));
    if (cycle == 0 && !safe) before = *h;
    BK_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(b.plans), 4 * (m + 1), 0u, st));
    // R = B - A X into V_0, its Gram; V_0 sigma_0 = Norm_S(R)
    BK_TRY(launch_spmm<double>(A, s, X, b.V, B, 2, b.partial, nblk, red, &c->bad_index, nullptr, st));
    BK_TRY(tsqr_run<double>(n, sub, b.V, b.sigma0, b.tsqr_ws, b.cnt, nullptr, nullptr, st));
    BK_TRY(launch_gm_cycle_init(c, b.sig, b.sigma0, b.Gb, cycle == 0, st));
    for (int k = 0; k < m; ++k) {
      double* Vk = b.V + (size_t)k * blk;
      double* W = b.V + (size_t)(k + 1) * blk;
      BK_TRY(launch_spmm<double>(A, s, Vk, W, nullptr, 0, nullptr, nblk, red, &c->bad_index, done, st));
      if (orth > 0) {
        // pipelined Gram-Schmidt, window w: H_i = <V_i, W>_S for i < w from
        // W as it comes; then passes of at most min(w, lmax) updates, each
        // taking the inner products of the blocks w places further on
        const int w = orth < k ? (orth > 0 ? orth : 1) : (k > 0 ? k : 1);
        const int L = w < lmax ? w : lmax;
        BK_TRY(launch_gram<double>(n, s, b.V, w < k + 1 ? w : k + 1, W, b.partial, nblk, red_to(b.H1), done, st));
        if (!proj_id) BK_TRY(launch_project_batched(b.Gb, b.H1, sub, w < k + 1 ? w : k + 1, done, st));
        for (int u0 = 0; u0 <= k; u0 += L) {
          const int nu = (k + 1 - u0) < L ? (k + 1 - u0) : L;
          const int g0 = u0 + w;
          const int ng = g0 > k ? 0 : ((k + 1 - g0) < nu ? (k + 1 - g0) : nu);
          BK_TRY(launch_pgs_pass(n, s, b.V, W, u0, nu, b.H1, g0, ng, b.partial, nblk, done, st));
          if (ng > 0) {
            BK_TRY(launch_reduce(s, b.partial, false, nblk, ng, red_to(b.H1 + (size_t)g0 * ss), done, nullptr,
                                 Epi{}, st));
            if (!proj_id) BK_TRY(launch_project_batched(b.Gb, b.H1 + (size_t)g0 * ss, sub, ng, done, st));
          }
        }
      } else {
        // classical Gram-Schmidt, twice: H_j = <V_j, W>_S, W -= sum_j V_j H_j
        double* Hp[2] = {b.H1, b.H2};
        for (int pass = 0; pass < 2; ++pass) {
          BK_TRY(launch_gram<double>(n, s, b.V, k + 1, W, b.partial, nblk, red_to(Hp[pass]), done, st));
          if (!proj_id) BK_TRY(launch_project_batched(b.Gb, Hp[pass], sub, k + 1, done, st));
          BK_TRY(launch_block_combine<double>(n, s, b.V, k + 1, Hp[pass], -1.0, W, done, st));
        }
      }
      BK_TRY(tsqr_run<double>(n, sub, W, b.gam, b.tsqr_ws, b.cnt, done, nullptr, st, b.plans + 4 * k, safe));
      BK_TRY(launch_gm_step(c, s, k, b.H, b.sig, b.Om, b.H1, b.H2, b.gam, b.hist, st));
    }
    BK_TRY(hipMemcpyAsync(hflags, c, 16 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if (!safe)
      BK_TRY(hipMemcpyAsync(hplans.data(), b.plans, sizeof(int32_t) * 4 * m, hipMemcpyDeviceToHost, st));
    BK_TRY(hipStreamSynchronize(st));
    if (!safe) {
      bool redo = false;
      for (int k = 0; k < m; ++k) redo |= hplans[(size_t)4 * k + 2] != 0;
      if (redo) {
        // restore the control block and run this cycle again with the fallback
        BK_TRY(hipMemcpyAsync(c, &before, sizeof(GmCtl), hipMemcpyHostToDevice, st));
        safe = true;
        --cycle;
        continue;
      }
    }
    safe = false;
    const GmCtl* hc = reinterpret_cast<const GmCtl*>(hflags);
    const int kend = hc->kend;
    res.status = hc->status;
    res.converged = hc->converged;
    res.steps = hc->total;
    res.cycles = cycle + (kend > 0 ? 1 : 0);
    res.bad_index = hc->bad_index;
    if (res.bad_index || res.status) return hipSuccess;
    if (kend > 0) {
      BK_TRY(launch_gm_backsub(c, s, kend, b.H, b.sig, b.zeta, st));
      BK_TRY(launch_block_combine<double>(n, s, b.V, kend, b.zeta, 1.0, X, nullptr, st));
    }
    if (res.converged || res.steps >= maxit || kend == 0) break;
  }
  return hipSuccess;
}

}  // namespace bkry
