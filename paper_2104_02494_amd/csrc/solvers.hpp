// solvers.hpp -- workspace layout and drivers of the block solvers.
#pragma once

#include <stddef.h>

#include "internal.hpp"

namespace bkry {

// Carves 256-byte aligned buffers out of one workspace; with base == nullptr
// it only counts the bytes.
struct Carver {
  char* base = nullptr;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += (count * sizeof(T) + 255) / 256 * 256;
    return p;
  }
};

// Optional timing of the solver's streaming kernels with HIP events recorded
// on the solver's stream around each launch (kernel ids below).
enum ProfKernel { PROF_CG_SPMM = 0, PROF_CG_UPDATE = 1, PROF_CG_PUPDATE = 2, PROF_CG_NORMALISE = 3, PROF_N = 4 };
constexpr int kProfSlots = 64;
struct Prof {
  hipEvent_t ev[PROF_N][2][kProfSlots];
  int used[PROF_N];
  int iter[PROF_N][kProfSlots];  // iteration of the timed launch (-1: always live)
  double ms[PROF_N];
  long long cnt[PROF_N];
  long long dropped[PROF_N];     // timed launches discarded as gated off
  int mask = (1 << PROF_N) - 1;  // kernel ids that are timed (bit k = id k)
  int every = 1;                  // time one launch in `every` of each kernel
  long long seen[PROF_N] = {};    // launches seen per kernel id
};
hipError_t prof_init(Prof* p);
void prof_destroy(Prof* p);
// Accumulates the recorded pairs (the stream must have been synchronised).
// live (null: every launch counts): per kernel id, the first iteration whose
// launches found the solve ended or suspended and returned at once; timings
// of launches of iterations >= live[id] are discarded, so averages cover
// only launches that did the work.
hipError_t prof_flush(Prof* p, const int* live = nullptr);

// Pinned host staging area shared by the drivers: ints [0, 64) receive
// read-backs, ints [64, 256) stage uploads.
constexpr int kHostFlagsInts = 256;

// Zeroed reduction counters owned by the handle (kMaxBatch slices).
constexpr size_t kCounterInts = (size_t)kMaxBatch * kCntStride;

template <typename T>
struct CgBufs {
  T *P = nullptr, *P2 = nullptr, *Q = nullptr, *R = nullptr, *partial = nullptr;
  double *Ga = nullptr, *Gr = nullptr, *Gq = nullptr, *gpart = nullptr, *hist = nullptr;
  CgCtl* ctl = nullptr;
  void* tsqr_ws = nullptr;
  uint32_t* cnt = nullptr;
};

template <typename T>
CgBufs<T> carve_cg(Carver& c, int64_t n, Sub sub, int hist_cap, uint32_t* cnt);

struct CgResult {
  int status = 0;  // 0, -2 breakdown, -3 non-finite
  int iters = 0, nreorth = 0, converged = 0, bad_index = 0, kd_jacobi = 0;
};

// Block CG in element type T (FP64 or FP32 streaming kernels; p x p algebra in
// FP64).  X holds X0 on entry.  eps is the machine epsilon of T.  minv (FP64
// only; device, n entries): the diagonal of M^-1 of a diagonal preconditioner
// M (null: M = I).
template <typename T>
hipError_t cg_run(const CsrView& A, Sub sub, const T* B, T* X, double tol, int maxit, double eta, double eps,
                  int hist_cap, const CgBufs<T>& b, hipStream_t st, int32_t* hflags, CgResult& res,
                  Prof* prof = nullptr, const double* minv = nullptr);

// Block CG with one reduction per iteration (alg:1R-CG), FP64, M = I.  Uses
// the CgBufs of the same n and sub: R holds R-bar, P2 holds U = A R-bar.
hipError_t cg1r_run(const CsrView& A, Sub sub, const double* B, double* X, double tol, int maxit, double eta,
                    int hist_cap, const CgBufs<double>& b, hipStream_t st, int32_t* hflags, CgResult& res,
                    Prof* prof = nullptr);

// Gropp's block CG (alg:gropps_block_cg, Ch. 8), FP64, with a diagonal
// preconditioner (minv) or M = I: the CgBufs of the same n and sub plus two
// n x s blocks, U = A Z and Z = M^-1 R-bar (unused for M = I).
hipError_t gropp_run(const CsrView& A, Sub sub, const double* B, double* X, double tol, int maxit, double eta,
                     int hist_cap, const CgBufs<double>& b, double* U, double* Zbuf, hipStream_t st, int32_t* hflags,
                     CgResult& res, Prof* prof = nullptr, const double* minv = nullptr);

// Workspace of a multicolour SSOR plan (ssor_carve) and its construction:
// checks the colouring against A (err: 0, or 1 colour out of range, 2 coupled
// rows of one colour or a bad column index, 3 a row without a positive
// diagonal), the diagonal, the rows bucketed by colour.  Synchronises st.
struct SsorWs {
  double* d = nullptr;
  int32_t *perm = nullptr, *off = nullptr, *cursor = nullptr, *count = nullptr, *misc = nullptr;
};
SsorWs ssor_carve(Carver& c, int64_t n);
hipError_t ssor_plan_build(const CsrView& A, const int32_t* colors, double omega, const SsorWs& w, hipStream_t st,
                           SsorPlan& plan, int& err);

// Block CG preconditioned by multicolour SSOR (FP64): as cg_run with Z =
// M^-1 R-bar from the colour sweeps (Z goes through Q, which is free after
// the residual update).
hipError_t pcg_ssor_run(const CsrView& A, Sub sub, const double* B, double* X, double tol, int maxit, double eta,
                        int hist_cap, const CgBufs<double>& b, const SsorPlan& m, hipStream_t st, int32_t* hflags,
                        CgResult& res, Prof* prof = nullptr);

struct IrBufs {
  float *A32 = nullptr, *R32 = nullptr, *X32 = nullptr;
  double *R64 = nullptr, *partial = nullptr, *gpart = nullptr, *G = nullptr, *r0n = nullptr, *scale = nullptr;
  double* relres = nullptr;
  int32_t* flag = nullptr;
  uint32_t* cnt = nullptr;
  CgBufs<float> cg;
  // optional FP32 ELL copy of A for the inner solves (filled by the caller)
  int ell_w = 0;
  const int32_t* ell_col = nullptr;
  const float* ell_val = nullptr;
  bool ell_diag0 = false;  // slot 0 of every ELL row holds its diagonal entry
};
IrBufs carve_ir(Carver& c, int64_t n, int64_t nnz, Sub sub, uint32_t* cnt);

struct IrResult {
  int status = 0, converged = 0, outer = 0, inner_iters = 0, nreorth = 0, bad_index = 0, hist_len = 0;
  int inner_status = 0;  // status of the last inner solve (0, -2 breakdown, -3 non-finite)
};
hipError_t ir_run(const CsrView& A, Sub sub, const double* B, double* X, double tol, int maxit, double eta,
                  double inner_tol, int max_outer, double* hist_host, int hist_cap, const IrBufs& b, hipStream_t st,
                  int32_t* hflags, double* relres_host, IrResult& res, Prof* prof = nullptr);

struct GmBufs {
  double *V = nullptr, *partial = nullptr, *gpart = nullptr, *Gb = nullptr, *H1 = nullptr, *H2 = nullptr;
  double *H = nullptr, *sig = nullptr, *Om = nullptr, *zeta = nullptr, *sigma0 = nullptr, *gam = nullptr;
  double *hist = nullptr, *relres = nullptr;
  int32_t* flag = nullptr;
  int32_t* plans = nullptr;  // the CholeskyQR decisions of each Arnoldi step, 4 ints each
  GmCtl* ctl = nullptr;
  void* tsqr_ws = nullptr;
  uint32_t* cnt = nullptr;
};
GmBufs carve_gm(Carver& c, int64_t n, Sub sub, int m, int hist_cap, uint32_t* cnt);

struct GmResult {
  int status = 0, converged = 0, steps = 0, cycles = 0, bad_index = 0;
};
// orth = 0: classical Gram-Schmidt applied twice; orth = r >= 1: the
// pipelined Gram-Schmidt of window r (Ch. 9).
hipError_t gm_run(const CsrView& A, Sub sub, const double* B, double* X, double tol, int maxit, int m,
                  int hist_cap, const GmBufs& b, hipStream_t st, int32_t* hflags, GmResult& res, int orth = 0);

// ------------------------------------------------------ block BiCGStab --
struct BcBufs {
  double *P = nullptr, *Pn = nullptr;
  double* W2 = nullptr;  // [Q | R]: 2 blocks
  double* W3 = nullptr;  // [S | U | R~0]: 3 blocks
  double *partial = nullptr, *gpart = nullptr, *G = nullptr, *Grr = nullptr, *hist = nullptr;
  CgCtl* ctl = nullptr;
  BcAux* aux = nullptr;
  void* tsqr_ws = nullptr;
  uint32_t* cnt = nullptr;
};
BcBufs carve_bc(Carver& c, int64_t n, Sub sub, int hist_cap, uint32_t* cnt);

struct BcResult {
  int status = 0, iters = 0, nreorth = 0, converged = 0, bad_index = 0;
};

// Block BiCGStab with adaptive residual re-orthonormalisation (FP64, M = I).
// X holds X0 on entry.
// r0n_fixed (device, s doubles, or null): stopping-test denominators kept
// from an earlier start (a restart on the true residual).
hipError_t bc_run(const CsrView& A, Sub sub, const double* B, double* X, double tol, int maxit, double eta,
                  int hist_cap, const BcBufs& b, hipStream_t st, int32_t* hflags, BcResult& res,
                  const double* r0n_fixed = nullptr);

// True relative column residuals |B_i - A X_i| / r0n_i (FP64) into relres
// (device); R (n x s), partial, gpart, G and scale_scratch are scratch.
hipError_t true_relres(const CsrView& A, int s, const double* B, const double* X, double* R, double* partial,
                       double* gpart, uint32_t* cnt, double* G, const double* r0n, double* relres, int32_t* flag,
                       double* scale_scratch, hipStream_t st);

}  // namespace bkry
