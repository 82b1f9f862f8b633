// api.hip -- the C ABI of libbkry.so (declared in include/bkry.h).
//
// The handle owns a growable device workspace, a pinned host staging area
// and the stream; every entry point validates its arguments on the host
// (sizes, pointers, subalgebra), sets the device, and then only enqueues
// kernels.  No C++ exception crosses the ABI.
#include <float.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <mutex>
#include <new>
#include <string>

#include "bkry.h"
#include "solvers.hpp"

using namespace bkry;

struct bkry_handle_s {
  int device = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_cap = 0;
  int32_t* hflags = nullptr;  // pinned host, kHostFlagsInts
  int32_t* dflags = nullptr;  // device: [0] bad CSR index seen by an asynchronous kernel,
                              // [1] longest CSR row, [2] bad index seen while building an ELL copy,
                              // [3] row without a diagonal entry seen while building a solver's ELL copy,
                              // [4] bad diagonal seen by bkry_jacobi_minv
  uint32_t* cnt = nullptr;    // device: zeroed grid-reduction counters (left zero by every kernel)
  Prof* prof = nullptr;       // kernel timing, when enabled
  int32_t spmm_format = BKRY_FMT_AUTO;
  std::string err;
};

namespace {

int fail(bkry_handle h, int code, const std::string& msg) {
  if (h) h->err = msg;
  return code;
}

int hip_fail(bkry_handle h, hipError_t e, const char* where) {
  return fail(h, BKRY_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define API_HIP(x, where)                           \
  do {                                              \
    hipError_t e_ = (x);                            \
    if (e_ != hipSuccess) return hip_fail(h, e_, where); \
  } while (0)

CsrView view(const bkry_csr* A) { return CsrView{A->n, A->nnz, A->rowptr, A->colind, A->val}; }

int ensure_ws(bkry_handle h, size_t bytes) {
  if (bytes <= h->ws_cap) return BKRY_OK;
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "workspace sync");
  if (h->ws) (void)hipFree(h->ws);
  h->ws = nullptr;
  h->ws_cap = 0;
  size_t want = bytes + bytes / 8;
  e = hipMalloc(reinterpret_cast<void**>(&h->ws), want);
  if (e != hipSuccess) {
    h->ws = nullptr;
    (void)hipGetLastError();
    return fail(h, BKRY_E_ALLOC, "workspace allocation of " + std::to_string(want) + " bytes failed");
  }
  h->ws_cap = want;
  return BKRY_OK;
}

int begin(bkry_handle h) {
  if (!h) return BKRY_E_INVALID;
  h->err.clear();
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return hip_fail(h, e, "hipSetDevice");
  return BKRY_OK;
}

// Validates p and the subalgebra; fills sub.
int check_sub(bkry_handle h, int32_t p, bkry_subalg S, Sub& sub) {
  if (p < 1 || p > kMaxS) return fail(h, BKRY_E_INVALID, "p must be in [1, 32]");
  sub.s = p;
  sub.kind = S.kind;
  switch (S.kind) {
    case BKRY_BLOCK: sub.g = p; break;
    case BKRY_PARALLEL:
    case BKRY_GLOBAL: sub.g = 1; break;
    case BKRY_HYBRID:
      if (S.q < 1 || p % S.q != 0) return fail(h, BKRY_E_INVALID, "hybrid subalgebra needs q >= 1 dividing p");
      sub.g = p / S.q;
      break;
    case BKRY_BLOCK_GLOBAL:
      if (S.q < 1 || p % S.q != 0) return fail(h, BKRY_E_INVALID, "block-global subalgebra needs q >= 1 dividing p");
      sub.g = p / S.q;
      // one group is the block subalgebra, groups of one column the global one
      sub.kind = sub.g == p ? BLOCK : (sub.g == 1 ? GLOBAL : BGLOBAL);
      break;
    default: return fail(h, BKRY_E_INVALID, "unknown subalgebra kind");
  }
  return BKRY_OK;
}

int check_csr(bkry_handle h, const bkry_csr* A, bool need_val) {
  if (!A) return fail(h, BKRY_E_INVALID, "null CSR descriptor");
  if (A->n < 1) return fail(h, BKRY_E_INVALID, "n must be >= 1");
  if (A->nnz < 0 || A->nnz >= (int64_t)1 << 31) return fail(h, BKRY_E_INVALID, "nnz must be in [0, 2^31)");
  if (A->n >= (int64_t)1 << 31) return fail(h, BKRY_E_INVALID, "n must be < 2^31");
  if (!A->rowptr) return fail(h, BKRY_E_INVALID, "null rowptr");
  if (A->nnz > 0 && (!A->colind || (need_val && !A->val))) return fail(h, BKRY_E_INVALID, "null colind/val");
  return BKRY_OK;
}

// Row width of the ELL copy of A that this call streams (0: stream CSR).
// AUTO picks ELL for the solvers when the padded copy costs at most 25 %
// more bytes per SpMM than CSR; bkry_spmm uses ELL only when it is forced.
int ell_width_for(bkry_handle h, const bkry_csr* A, int p, int elem_bytes, bool solver, int& W) {
  W = 0;
  if (h->spmm_format == BKRY_FMT_CSR || (h->spmm_format == BKRY_FMT_AUTO && !solver)) return BKRY_OK;
  API_HIP(launch_ell_width(view(A), h->dflags + 1, h->stream), "ell width");
  API_HIP(hipMemcpyAsync(h->hflags, h->dflags + 1, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream), "ell width");
  API_HIP(hipStreamSynchronize(h->stream), "ell width");
  const int64_t wmax = h->hflags[0] > 1 ? h->hflags[0] : 1;
  const int64_t C = ell_chunk(p, elem_bytes);
  const int64_t Wc = (wmax + C - 1) / C * C;
  if (h->spmm_format == BKRY_FMT_AUTO) {
    const double n = (double)A->n, eb = elem_bytes;
    const double csr = 4.0 * (n + 1) + (double)A->nnz * (4.0 + eb) + 2.0 * n * p * eb;
    const double ell = n * (double)Wc * (4.0 + eb) + 2.0 * n * p * eb;
    if (ell > 1.25 * csr) return BKRY_OK;
  }
  if (Wc > (1 << 20)) return fail(h, BKRY_E_INVALID, "ELL row width too large");
  W = (int)Wc;
  return BKRY_OK;
}

// Fill the ELL copy (width W) of A with values val and attach it to v;
// synchronous, so that a bad column index is reported here.  The solvers'
// copies (diag_first) hold each row's diagonal entry in slot 0 when every row
// has one (v.ell_diag0), else CSR order.
template <typename Tin, typename T>
int ell_build(bkry_handle h, const bkry_csr* A, const Tin* val, int W, int32_t* ecol, T* eval, CsrView& v,
              bool diag_first) {
  if (W <= 0) return BKRY_OK;
  API_HIP(hipMemsetAsync(h->dflags + 2, 0, 2 * sizeof(int32_t), h->stream), "ell fill");
  API_HIP((launch_ell_fill<Tin, T>(view(A), val, W, ecol, eval, h->dflags + 2, diag_first ? h->dflags + 3 : nullptr,
                                   h->stream)),
          "ell fill");
  API_HIP(hipMemcpyAsync(h->hflags, h->dflags + 2, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream),
          "ell fill");
  API_HIP(hipStreamSynchronize(h->stream), "ell fill");
  if (h->hflags[0]) return fail(h, BKRY_E_INVALID, "a CSR column index was outside [0, n)");
  v.ell_w = W;
  v.ell_col = ecol;
  v.ell_val = eval;
  v.ell_diag0 = diag_first && h->hflags[1] == 0;
  return BKRY_OK;
}

bool misaligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) != 0; }

int check_blocks(bkry_handle h, std::initializer_list<const void*> ptrs) {
  for (const void* p : ptrs) {
    if (!p) return fail(h, BKRY_E_INVALID, "null block pointer");
    if (misaligned(p)) return fail(h, BKRY_E_INVALID, "block pointers must be 16-byte aligned");
  }
  return BKRY_OK;
}


int status_of(int st, bkry_handle h) {
  if (st == -2) return fail(h, BKRY_E_BREAKDOWN, "breakdown: a Cholesky pivot of alpha or rho was not positive");
  if (st == -3) return fail(h, BKRY_E_NONFINITE, "non-finite value in the block coefficients");
  return BKRY_OK;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

template <typename T>
int bdot_impl(bkry_handle h, int64_t n, int32_t p, bkry_subalg S, const T* X, const T* Y, double* G) {
  int rc = begin(h);
  Sub sub;
  if (!rc) rc = check_sub(h, p, S, sub);
  if (!rc && n < 1) rc = fail(h, BKRY_E_INVALID, "n must be >= 1");
  if (!rc) rc = check_blocks(h, {X, Y});
  if (!rc && !G) rc = fail(h, BKRY_E_INVALID, "null G");
  if (rc) return rc;
  const int nblk = stream_grid(n, p, sizeof(T));
  Carver c;
  c.take<T>((size_t)nblk * p * p);
  c.take<double>(red_gpart_count(nblk, p));
  c.take<double>((size_t)p * p);
  rc = ensure_ws(h, c.off);
  if (rc) return rc;
  Carver w{h->ws};
  T* part = w.take<T>((size_t)nblk * p * p);
  double* gpart = w.take<double>(red_gpart_count(nblk, p));
  double* Gf = w.take<double>((size_t)p * p);
  API_HIP(launch_gram<T>(n, p, X, 1, Y, part, nblk, Red{Gf, gpart, h->cnt}, nullptr, h->stream), "bdot");
  API_HIP(launch_project(Gf, G, sub, h->stream), "bdot");
  return BKRY_OK;
}

// ------------------------------------------------ allocation-free scratch --
// Device memory of the allocation-free entry points: one fixed array per GPU,
// held for the life of the process.  Host code never passes `scratch` itself
// to a kernel (in host code it names a host-side stand-in); it uses the
// device address resolved once per device by resolve_scratch.
constexpr size_t kScratchBytes = (size_t)5 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};

// With `device` current: the device address of this GPU's scratch array.
hipError_t resolve_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return hipSuccess;
  char* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(reinterpret_cast<void**>(&ptr), HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch[device] = ptr;
  return hipSuccess;
}

char* scratch_of(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (device >= 0 && device < kMaxDevices) ? g_scratch[device] : nullptr;
}

}  // namespace

extern "C" {

int bkry_create(bkry_handle* out, int device, void* stream) {
  if (!out) return BKRY_E_INVALID;
  *out = nullptr;
  bkry_handle h = new (std::nothrow) bkry_handle_s();
  if (!h) return BKRY_E_ALLOC;
  h->device = device;
  h->stream = static_cast<hipStream_t>(stream);
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&h->hflags), kHostFlagsInts * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&h->dflags), 64 * sizeof(int32_t));
  if (e == hipSuccess) e = hipMemsetAsync(h->dflags, 0, 64 * sizeof(int32_t), h->stream);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&h->cnt), kCounterInts * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemsetAsync(h->cnt, 0, kCounterInts * sizeof(uint32_t), h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess) e = resolve_scratch(device);
  if (e != hipSuccess) {
    if (h->hflags) (void)hipHostFree(h->hflags);
    if (h->dflags) (void)hipFree(h->dflags);
    if (h->cnt) (void)hipFree(h->cnt);
    delete h;
    return BKRY_E_HIP;
  }
  *out = h;
  return BKRY_OK;
}

int bkry_destroy(bkry_handle h) {
  if (!h) return BKRY_E_INVALID;
  (void)hipSetDevice(h->device);
  (void)hipStreamSynchronize(h->stream);
  if (h->ws) (void)hipFree(h->ws);
  if (h->dflags) (void)hipFree(h->dflags);
  if (h->cnt) (void)hipFree(h->cnt);
  if (h->hflags) (void)hipHostFree(h->hflags);
  if (h->prof) {
    prof_destroy(h->prof);
    delete h->prof;
  }
  delete h;
  return BKRY_OK;
}

int bkry_set_stream(bkry_handle h, void* stream) {
  int rc = begin(h);
  if (rc) return rc;
  h->stream = static_cast<hipStream_t>(stream);
  return BKRY_OK;
}

const char* bkry_last_error(bkry_handle h) { return h ? h->err.c_str() : "null handle"; }

int bkry_synchronize(bkry_handle h) {
  int rc = begin(h);
  if (rc) return rc;
  API_HIP(hipMemcpyAsync(h->hflags, h->dflags, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream), "sync");
  API_HIP(hipStreamSynchronize(h->stream), "sync");
  if (h->hflags[0]) {
    API_HIP(hipMemsetAsync(h->dflags, 0, sizeof(int32_t), h->stream), "sync");
    API_HIP(hipStreamSynchronize(h->stream), "sync");
    return fail(h, BKRY_E_INVALID, "a CSR column index was outside [0, n)");
  }
  return BKRY_OK;
}

int bkry_profile(bkry_handle h, int enable) {
  int rc = begin(h);
  if (rc) return rc;
  const int mask = enable & 0xFF, every = (enable >> 8) & 0xFF;
  if (mask & ~((1 << PROF_N) - 1) || (enable >> 16)) return fail(h, BKRY_E_INVALID, "bad kernel timing mask");
  if (enable && !h->prof) {
    h->prof = new (std::nothrow) Prof();
    if (!h->prof) return fail(h, BKRY_E_ALLOC, "profile state");
    API_HIP(prof_init(h->prof), "profile");
  }
  if (enable) {
    h->prof->mask = mask;
    h->prof->every = every > 1 ? every : 1;
  } else if (h->prof) {
    API_HIP(hipStreamSynchronize(h->stream), "profile");
    prof_destroy(h->prof);
    delete h->prof;
    h->prof = nullptr;
  }
  return BKRY_OK;
}

int bkry_profile_read(bkry_handle h, int32_t kernel, double* total_ms, int64_t* launches, int32_t reset) {
  int rc = begin(h);
  if (rc) return rc;
  if (!h->prof) return fail(h, BKRY_E_INVALID, "kernel timing is not enabled");
  if (kernel < 0 || kernel >= PROF_N) return fail(h, BKRY_E_INVALID, "unknown kernel id");
  if (total_ms) *total_ms = h->prof->ms[kernel];
  if (launches) *launches = h->prof->cnt[kernel];
  if (reset) {
    h->prof->ms[kernel] = 0.0;
    h->prof->cnt[kernel] = 0;
    h->prof->dropped[kernel] = 0;
  }
  return BKRY_OK;
}

int bkry_set_spmm_format(bkry_handle h, int32_t format) {
  int rc = begin(h);
  if (rc) return rc;
  if (format != BKRY_FMT_AUTO && format != BKRY_FMT_CSR && format != BKRY_FMT_ELL)
    return fail(h, BKRY_E_INVALID, "unknown SpMM format");
  h->spmm_format = format;
  return BKRY_OK;
}

int bkry_spmm(bkry_handle h, const bkry_csr* A, int32_t p, const double* X, double* Y) {
  int rc = begin(h);
  if (!rc) rc = check_csr(h, A, true);
  if (!rc && (p < 1 || p > kMaxS)) rc = fail(h, BKRY_E_INVALID, "p must be in [1, 32]");
  if (!rc) rc = check_blocks(h, {X, Y});
  if (rc) return rc;
  int W = 0;
  rc = ell_width_for(h, A, p, sizeof(double), false, W);
  if (rc) return rc;
  CsrView v = view(A);
  if (W > 0) {
    Carver c;
    c.take<int32_t>((size_t)A->n * W);
    c.take<double>((size_t)A->n * W);
    rc = ensure_ws(h, c.off);
    if (rc) return rc;
    Carver w{h->ws};
    int32_t* ecol = w.take<int32_t>((size_t)A->n * W);
    double* eval = w.take<double>((size_t)A->n * W);
    rc = ell_build<double, double>(h, A, A->val, W, ecol, eval, v, false);
    if (rc) return rc;
  }
  const int nblk = stream_grid(A->n, p, sizeof(double));
  API_HIP(launch_spmm<double>(v, p, X, Y, nullptr, 0, nullptr, nblk, Red{}, h->dflags, nullptr, h->stream), "spmm");
  return BKRY_OK;
}

int bkry_spmm_f32(bkry_handle h, int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colind,
                  const float* val, int32_t p, const float* X, float* Y) {
  bkry_csr A{n, nnz, rowptr, colind, nullptr};
  int rc = begin(h);
  if (!rc) rc = check_csr(h, &A, false);
  if (!rc && nnz > 0 && !val) rc = fail(h, BKRY_E_INVALID, "null val");
  if (!rc && (p < 1 || p > kMaxS)) rc = fail(h, BKRY_E_INVALID, "p must be in [1, 32]");
  if (!rc) rc = check_blocks(h, {X, Y});
  if (rc) return rc;
  CsrView v{n, nnz, rowptr, colind, val};
  int W = 0;
  rc = ell_width_for(h, &A, p, sizeof(float), false, W);
  if (rc) return rc;
  if (W > 0) {
    Carver c;
    c.take<int32_t>((size_t)n * W);
    c.take<float>((size_t)n * W);
    rc = ensure_ws(h, c.off);
    if (rc) return rc;
    Carver w{h->ws};
    int32_t* ecol = w.take<int32_t>((size_t)n * W);
    float* eval = w.take<float>((size_t)n * W);
    rc = ell_build<float, float>(h, &A, val, W, ecol, eval, v, false);
    if (rc) return rc;
  }
  const int nblk = stream_grid(n, p, sizeof(float));
  API_HIP(launch_spmm<float>(v, p, X, Y, nullptr, 0, nullptr, nblk, Red{}, h->dflags, nullptr, h->stream),
          "spmm_f32");
  return BKRY_OK;
}

int bkry_bdot(bkry_handle h, int64_t n, int32_t p, bkry_subalg S, const double* X, const double* Y, double* G) {
  return bdot_impl<double>(h, n, p, S, X, Y, G);
}

int bkry_bdot_f32(bkry_handle h, int64_t n, int32_t p, bkry_subalg S, const float* X, const float* Y, double* G) {
  return bdot_impl<float>(h, n, p, S, X, Y, G);
}

int bkry_bdot_noalloc(bkry_handle h, int64_t n, int32_t p, bkry_subalg S, const double* X, const double* Y,
                      double* G) {
  int rc = begin(h);
  Sub sub;
  if (!rc) rc = check_sub(h, p, S, sub);
  if (!rc && n < 1) rc = fail(h, BKRY_E_INVALID, "n must be >= 1");
  if (!rc) rc = check_blocks(h, {X, Y});
  if (!rc && !G) rc = fail(h, BKRY_E_INVALID, "null G");
  if (rc) return rc;
  char* base = scratch_of(h->device);
  if (!base) return fail(h, BKRY_E_HIP, "bdot_noalloc: the scratch array of this device was not resolved");
  // the same partials, slice sums and Gram as bkry_bdot, plus one counter
  // slice, carved from the device's scratch array
  const int nblk = stream_grid(n, p, sizeof(double));
  Carver c;
  c.take<double>((size_t)nblk * p * p);
  c.take<double>(red_gpart_count(nblk, p));
  c.take<double>((size_t)p * p);
  c.take<uint32_t>(kCntStride);
  if (c.off > kScratchBytes)
    return fail(h, BKRY_E_INVALID, "bdot_noalloc needs " + std::to_string(c.off) + " bytes of scratch, more than the " +
                                       std::to_string(kScratchBytes) + " it holds");
  Carver w{base};
  double* part = w.take<double>((size_t)nblk * p * p);
  double* gpart = w.take<double>(red_gpart_count(nblk, p));
  double* Gf = w.take<double>((size_t)p * p);
  uint32_t* cnt = w.take<uint32_t>(kCntStride);
  // the reduction's hand-off counter must start at zero; a fill kernel (not
  // a memset) keeps the call capturable in a HIP graph
  API_HIP(launch_fill_u32(cnt, kCntStride, 0u, h->stream), "bdot_noalloc");
  API_HIP(launch_gram<double>(n, p, X, 1, Y, part, nblk, Red{Gf, gpart, cnt}, nullptr, h->stream), "bdot_noalloc");
  API_HIP(launch_project(Gf, G, sub, h->stream), "bdot_noalloc");
  return BKRY_OK;
}

int bkry_tsqr(bkry_handle h, int64_t n, int32_t p, bkry_subalg S, double* X, double* R) {
  int rc = begin(h);
  Sub sub;
  if (!rc) rc = check_sub(h, p, S, sub);
  if (!rc && (n < sub.g || (sub.kind == GLOBAL && n < p)))
    rc = fail(h, BKRY_E_INVALID, "the normaliser needs n >= p (block, global) or n >= p/q (hybrid, block-global)");
  if (!rc) rc = check_blocks(h, {X});
  if (!rc && !R) rc = fail(h, BKRY_E_INVALID, "null R");
  if (rc) return rc;
  rc = ensure_ws(h, tsqr_workspace_bytes(n, sub));
  if (rc) return rc;
  API_HIP(tsqr_run<double>(n, sub, X, R, h->ws, h->cnt, nullptr, nullptr, h->stream), "tsqr");
  return BKRY_OK;
}

namespace {
int ssor_fail(bkry_handle h, int err) {
  if (err == 1) return fail(h, BKRY_E_INVALID, "a colour is outside [0, 4096)");
  if (err == 2) return fail(h, BKRY_E_INVALID, "two rows of one colour are coupled (not a colouring of A), or a "
                                               "column index is outside [0, n)");
  return fail(h, BKRY_E_INVALID, "a diagonal entry of A is missing, not positive or not finite");
}

int cg_solve_impl(bkry_handle h, const bkry_csr* A, int32_t p, bkry_subalg S, const double* B, double* X,
                  double tol, int32_t maxit, double eta, int32_t prec, const double* minv, bkry_info* info,
                  bool one_reduction = false, const int32_t* ssor_colors = nullptr, double omega = 1.0,
                  bool gropp = false) {
  int rc = begin(h);
  Sub sub;
  if (!rc) rc = check_csr(h, A, true);
  if (!rc) rc = check_sub(h, p, S, sub);
  if (!rc) rc = check_blocks(h, {B, X});
  if (!rc && minv && prec != BKRY_F64) rc = fail(h, BKRY_E_INVALID, "the preconditioned solve runs in FP64");
  if (!rc && !(tol >= 0.0)) rc = fail(h, BKRY_E_INVALID, "tol must be >= 0");
  if (!rc && maxit < 0) rc = fail(h, BKRY_E_INVALID, "maxit must be >= 0");
  if (!rc && !(eta >= 0.0)) rc = fail(h, BKRY_E_INVALID, "eta must be >= 0");
  if (!rc && prec != BKRY_F64 && prec != BKRY_F32_IR) rc = fail(h, BKRY_E_INVALID, "unknown precision");
  if (!rc && eta > 0.0 && (A->n < sub.g || (sub.kind == GLOBAL && A->n < p)))
    rc = fail(h, BKRY_E_INVALID, "re-orthonormalisation needs n >= p (block, global) or n >= p/q (hybrid)");
  if (rc) return rc;
  const double t0 = now_s();
  const int64_t n = A->n;
  const int hist_cap = (info && info->hist && info->hist_cap > 0) ? info->hist_cap : 0;
  double relres[kMaxS], trel[kMaxS];
  int status = 0, iters = 0, nre = 0, outer = 0, conv = 0, bad = 0, hist_len = 0;
  int W = 0;
  rc = ell_width_for(h, A, p, prec == BKRY_F64 ? sizeof(double) : sizeof(float), true, W);
  if (rc) return rc;
  const size_t ne = (size_t)n * W;
  if (prec == BKRY_F64) {
    Carver c;
    carve_cg<double>(c, n, sub, hist_cap, h->cnt);
    c.take<double>(kMaxS);
    c.take<double>(kMaxS);
    c.take<int32_t>(4);
    c.take<int32_t>(ne);
    c.take<double>(ne);
    if (ssor_colors) ssor_carve(c, n);
    if (gropp) {
      c.take<double>((size_t)n * p);
      if (minv) c.take<double>((size_t)n * p);
    }
    rc = ensure_ws(h, c.off);
    if (rc) return rc;
    Carver w{h->ws};
    CgBufs<double> cb = carve_cg<double>(w, n, sub, hist_cap, h->cnt);
    double* trr = w.take<double>(kMaxS);
    double* tsc = w.take<double>(kMaxS);
    int32_t* tfl = w.take<int32_t>(4);
    int32_t* ecol = w.take<int32_t>(ne);
    double* eval = w.take<double>(ne);
    SsorWs sw;
    if (ssor_colors) sw = ssor_carve(w, n);
    double* gU = gropp ? w.take<double>((size_t)n * p) : nullptr;
    double* gZ = (gropp && minv) ? w.take<double>((size_t)n * p) : nullptr;
    CsrView v = view(A);
    rc = ell_build<double, double>(h, A, A->val, W, ecol, eval, v, true);
    if (rc) return rc;
    SsorPlan plan;
    if (ssor_colors) {
      int err = 0;
      API_HIP(ssor_plan_build(v, ssor_colors, omega, sw, h->stream, plan, err), "ssor plan");
      if (err) return ssor_fail(h, err);
    }
    CgResult r;
    hipError_t e = gropp ? gropp_run(v, sub, B, X, tol, maxit, eta, hist_cap, cb, gU, gZ, h->stream, h->hflags, r,
                                     h->prof, minv)
                   : ssor_colors ? pcg_ssor_run(v, sub, B, X, tol, maxit, eta, hist_cap, cb, plan, h->stream,
                                                h->hflags, r, h->prof)
                   : one_reduction
                       ? cg1r_run(v, sub, B, X, tol, maxit, eta, hist_cap, cb, h->stream, h->hflags, r, h->prof)
                       : cg_run<double>(v, sub, B, X, tol, maxit, eta, DBL_EPSILON, hist_cap, cb, h->stream,
                                        h->hflags, r, h->prof, minv);
    if (e != hipSuccess) return hip_fail(h, e, "cg_solve");
    status = r.status;
    iters = r.iters;
    nre = r.nreorth;
    conv = r.converged;
    bad = r.bad_index;
    hist_len = iters < hist_cap ? iters : hist_cap;
    API_HIP(hipMemcpyAsync(relres, cb.ctl->relres, sizeof(double) * p, hipMemcpyDeviceToHost, h->stream), "cg");
    if (hist_len > 0)
      API_HIP(hipMemcpyAsync(info->hist, cb.hist, sizeof(double) * hist_len, hipMemcpyDeviceToHost, h->stream), "cg");
    API_HIP(true_relres(v, p, B, X, cb.Q, cb.partial, cb.gpart, h->cnt, cb.Ga, cb.ctl->r0n, trr, tfl, tsc, h->stream),
            "cg");
    API_HIP(hipMemcpyAsync(trel, trr, sizeof(double) * p, hipMemcpyDeviceToHost, h->stream), "cg");
    API_HIP(hipStreamSynchronize(h->stream), "cg");
  } else {
    Carver c;
    carve_ir(c, n, A->nnz, sub, h->cnt);
    c.take<double>(kMaxS);
    c.take<double>(kMaxS);
    c.take<int32_t>(4);
    c.take<int32_t>(ne);
    c.take<float>(ne);
    rc = ensure_ws(h, c.off);
    if (rc) return rc;
    Carver w{h->ws};
    IrBufs ib = carve_ir(w, n, A->nnz, sub, h->cnt);
    double* trr = w.take<double>(kMaxS);
    double* tsc = w.take<double>(kMaxS);
    int32_t* tfl = w.take<int32_t>(4);
    int32_t* ecol = w.take<int32_t>(ne);
    float* eval = w.take<float>(ne);
    CsrView v32 = view(A);
    rc = ell_build<double, float>(h, A, A->val, W, ecol, eval, v32, true);
    if (rc) return rc;
    ib.ell_w = v32.ell_w;
    ib.ell_col = v32.ell_col;
    ib.ell_val = static_cast<const float*>(v32.ell_val);
    ib.ell_diag0 = v32.ell_diag0;
    const double itol = (info && info->inner_tol > 0.0) ? info->inner_tol : 1e-5;
    const int mo = (info && info->max_outer > 0) ? info->max_outer : 30;
    IrResult r;
    hipError_t e = ir_run(view(A), sub, B, X, tol, maxit, eta, itol, mo, info ? info->hist : nullptr, hist_cap, ib,
                          h->stream, h->hflags, relres, r, h->prof);
    if (e != hipSuccess) return hip_fail(h, e, "cg_solve (FP32 refinement)");
    status = r.status;
    iters = r.inner_iters;
    nre = r.nreorth;
    outer = r.outer;
    conv = r.converged;
    bad = r.bad_index;
    hist_len = r.hist_len;
    API_HIP(true_relres(view(A), p, B, X, ib.R64, ib.partial, ib.gpart, h->cnt, ib.G, ib.r0n, trr, tfl, tsc,
                        h->stream),
            "ir");
    API_HIP(hipMemcpyAsync(trel, trr, sizeof(double) * p, hipMemcpyDeviceToHost, h->stream), "ir");
    API_HIP(hipStreamSynchronize(h->stream), "ir");
  }
  if (info) {
    info->iters = iters;
    info->reorth = nre;
    info->outer_iters = outer;
    info->converged = conv;
    info->hist_len = hist_len;
    info->seconds = now_s() - t0;
    if (info->relres) memcpy(info->relres, relres, sizeof(double) * p);
    if (info->true_relres) memcpy(info->true_relres, trel, sizeof(double) * p);
  }
  if (bad) return fail(h, BKRY_E_INVALID, "a CSR column index was outside [0, n)");
  rc = status_of(status, h);
  if (rc) return rc;
  return conv ? BKRY_OK : BKRY_NOT_CONVERGED;
}
}  // namespace

int bkry_cg_solve(bkry_handle h, const bkry_csr* A, int32_t p, bkry_subalg S, const double* B, double* X,
                  double tol, int32_t maxit, double eta, int32_t prec, bkry_info* info) {
  return cg_solve_impl(h, A, p, S, B, X, tol, maxit, eta, prec, nullptr, info);
}

int bkry_cg1r_solve(bkry_handle h, const bkry_csr* A, int32_t p, bkry_subalg S, const double* B, double* X,
                    double tol, int32_t maxit, double eta, bkry_info* info) {
  return cg_solve_impl(h, A, p, S, B, X, tol, maxit, eta, BKRY_F64, nullptr, info, true);
}

int bkry_pcg_ssor_solve(bkry_handle h, const bkry_csr* A, int32_t p, bkry_subalg S, const double* B, double* X,
                        const int32_t* colors, double omega, double tol, int32_t maxit, double eta,
                        bkry_info* info) {
  if (!h) return BKRY_E_INVALID;
  if (!colors) return fail(h, BKRY_E_INVALID, "null colors");
  if (!(omega > 0.0 && omega < 2.0)) return fail(h, BKRY_E_INVALID, "omega must be in (0, 2)");
  return cg_solve_impl(h, A, p, S, B, X, tol, maxit, eta, BKRY_F64, nullptr, info, false, colors, omega);
}

int bkry_color(bkry_handle h, const bkry_csr* A, const uint32_t* prio, int32_t* colors, int32_t* ncolors) {
  int rc = begin(h);
  if (!rc) rc = check_csr(h, A, false);
  if (!rc && (!prio || !colors || !ncolors)) rc = fail(h, BKRY_E_INVALID, "null prio, colors or ncolors");
  if (rc) return rc;
  constexpr int kMaxRounds = 4096;
  const int64_t n = A->n;
  Carver c;
  c.take<int32_t>((size_t)n);
  c.take<int32_t>(kMaxRounds);
  c.take<int32_t>(4);
  rc = ensure_ws(h, c.off);
  if (rc) return rc;
  Carver w{h->ws};
  int32_t* state = w.take<int32_t>((size_t)n);
  int32_t* more = w.take<int32_t>(kMaxRounds);
  int32_t* misc = w.take<int32_t>(4);
  API_HIP(hipMemsetAsync(state, 0xff, sizeof(int32_t) * (size_t)n, h->stream), "color");
  API_HIP(hipMemsetAsync(more, 0, sizeof(int32_t) * kMaxRounds, h->stream), "color");
  API_HIP(hipMemsetAsync(misc, 0, sizeof(int32_t) * 4, h->stream), "color");
  const CsrView v = view(A);
  int r = 0;
  bool finished = false;
  while (r < kMaxRounds && !finished) {
    const int r1 = r + 16 < kMaxRounds ? r + 16 : kMaxRounds;
    for (; r < r1; ++r) API_HIP(launch_jp_round(v, prio, state, r, more, misc + 1, h->stream), "color");
    API_HIP(hipMemcpyAsync(h->hflags, more + r - 1, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream), "color");
    API_HIP(hipMemcpyAsync(h->hflags + 1, misc + 1, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream), "color");
    API_HIP(hipStreamSynchronize(h->stream), "color");
    if (h->hflags[1]) return fail(h, BKRY_E_INVALID, "a CSR column index was outside [0, n)");
    finished = h->hflags[0] == 0;
  }
  if (!finished) return fail(h, BKRY_E_INVALID, "the colouring did not finish within 4096 rounds");
  API_HIP(launch_jp_final(n, state, colors, misc, h->stream), "color");
  API_HIP(hipMemcpyAsync(h->hflags, misc, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream), "color");
  API_HIP(hipStreamSynchronize(h->stream), "color");
  *ncolors = h->hflags[0];
  if (*ncolors > kMaxColors) return fail(h, BKRY_E_INVALID, "more than 4096 colours");
  return BKRY_OK;
}

int bkry_ssor_apply(bkry_handle h, const bkry_csr* A, int32_t p, const int32_t* colors, double omega,
                    const double* R, double* Z) {
  int rc = begin(h);
  if (!rc) rc = check_csr(h, A, true);
  if (!rc && (p < 1 || p > kMaxS)) rc = fail(h, BKRY_E_INVALID, "p must be in [1, 32]");
  if (!rc) rc = check_blocks(h, {R, Z});
  if (!rc && !colors) rc = fail(h, BKRY_E_INVALID, "null colors");
  if (!rc && R == Z) rc = fail(h, BKRY_E_INVALID, "Z must not alias R");
  if (!rc && !(omega > 0.0 && omega < 2.0)) rc = fail(h, BKRY_E_INVALID, "omega must be in (0, 2)");
  if (rc) return rc;
  Carver c;
  ssor_carve(c, A->n);
  rc = ensure_ws(h, c.off);
  if (rc) return rc;
  Carver w{h->ws};
  const SsorWs sw = ssor_carve(w, A->n);
  SsorPlan plan;
  int err = 0;
  API_HIP(ssor_plan_build(view(A), colors, omega, sw, h->stream, plan, err), "ssor plan");
  if (err) return ssor_fail(h, err);
  API_HIP(launch_ssor_apply(plan, p, R, Z, nullptr, nullptr, nullptr, h->stream), "ssor apply");
  API_HIP(hipStreamSynchronize(h->stream), "ssor apply");
  return BKRY_OK;
}

int bkry_gropp_solve(bkry_handle h, const bkry_csr* A, int32_t p, bkry_subalg S, const double* B, double* X,
                     const double* minv, double tol, int32_t maxit, double eta, bkry_info* info) {
  if (!h) return BKRY_E_INVALID;
  if (minv && (reinterpret_cast<uintptr_t>(minv) & 7) != 0)
    return fail(h, BKRY_E_INVALID, "minv must be 8-byte aligned");
  return cg_solve_impl(h, A, p, S, B, X, tol, maxit, eta, BKRY_F64, minv, info, false, nullptr, 1.0, true);
}

int bkry_pcg_solve(bkry_handle h, const bkry_csr* A, int32_t p, bkry_subalg S, const double* B, double* X,
                   const double* minv, double tol, int32_t maxit, double eta, bkry_info* info) {
  if (!h) return BKRY_E_INVALID;
  if (!minv) return fail(h, BKRY_E_INVALID, "null minv");
  if ((reinterpret_cast<uintptr_t>(minv) & 7) != 0) return fail(h, BKRY_E_INVALID, "minv must be 8-byte aligned");
  return cg_solve_impl(h, A, p, S, B, X, tol, maxit, eta, BKRY_F64, minv, info);
}

int bkry_jacobi_minv(bkry_handle h, const bkry_csr* A, double* minv) {
  int rc = begin(h);
  if (!rc) rc = check_csr(h, A, true);
  if (!rc && !minv) rc = fail(h, BKRY_E_INVALID, "null minv");
  if (rc) return rc;
  API_HIP(hipMemsetAsync(h->dflags + 4, 0, sizeof(int32_t), h->stream), "jacobi");
  API_HIP(launch_jacobi_minv(view(A), minv, h->dflags + 4, h->stream), "jacobi");
  API_HIP(hipMemcpyAsync(h->hflags, h->dflags + 4, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream), "jacobi");
  API_HIP(hipStreamSynchronize(h->stream), "jacobi");
  if (h->hflags[0]) return fail(h, BKRY_E_INVALID, "a diagonal entry of A is missing, not positive or not finite");
  return BKRY_OK;
}

}  // extern "C"

namespace {
int gmres_impl(bkry_handle h, const bkry_csr* A, int32_t p, bkry_subalg S, const double* B, double* X, double tol,
               int32_t maxit, int32_t restart, int32_t orth, bkry_info* info) {
  int rc = begin(h);
  Sub sub;
  if (!rc) rc = check_csr(h, A, true);
  if (!rc) rc = check_sub(h, p, S, sub);
  if (!rc) rc = check_blocks(h, {B, X});
  if (!rc && !(tol >= 0.0)) rc = fail(h, BKRY_E_INVALID, "tol must be >= 0");
  if (!rc && maxit < 0) rc = fail(h, BKRY_E_INVALID, "maxit must be >= 0");
  if (!rc && (restart < 1 || restart > 200)) rc = fail(h, BKRY_E_INVALID, "restart must be in [1, 200]");
  if (!rc && A->n < p) rc = fail(h, BKRY_E_INVALID, "block GMRes needs n >= p");
  if (rc) return rc;
  const double t0 = now_s();
  const int64_t n = A->n;
  const int hist_cap = (info && info->hist && info->hist_cap > 0) ? info->hist_cap : 0;
  int W = 0;
  rc = ell_width_for(h, A, p, sizeof(double), true, W);
  if (rc) return rc;
  const size_t ne = (size_t)n * W;
  Carver c;
  carve_gm(c, n, sub, restart, hist_cap, h->cnt);
  c.take<double>(kMaxS);
  c.take<double>(kMaxS);
  c.take<int32_t>(ne);
  c.take<double>(ne);
  rc = ensure_ws(h, c.off);
  if (rc) return rc;
  Carver w{h->ws};
  GmBufs gb = carve_gm(w, n, sub, restart, hist_cap, h->cnt);
  double* trr = w.take<double>(kMaxS);
  double* tsc = w.take<double>(kMaxS);
  int32_t* ecol = w.take<int32_t>(ne);
  double* eval = w.take<double>(ne);
  CsrView v = view(A);
  rc = ell_build<double, double>(h, A, A->val, W, ecol, eval, v, true);
  if (rc) return rc;
  GmResult r;
  if (maxit > 0) {
    hipError_t e = gm_run(v, sub, B, X, tol, maxit, restart, hist_cap, gb, h->stream, h->hflags, r, orth);
    if (e != hipSuccess) return hip_fail(h, e, "gmres_solve");
  } else {
    // no step allowed: only the initial residual norms
    const int nblk = stream_grid(n, p, sizeof(double));
    API_HIP(launch_spmm<double>(v, p, X, gb.V, B, 2, gb.partial, nblk, Red{gb.Gb, gb.gpart, h->cnt}, nullptr,
                                nullptr, h->stream),
            "gmres");
    API_HIP(launch_gm_cycle_init(gb.ctl, gb.sig, gb.Gb, gb.Gb, 1, h->stream), "gmres");
    API_HIP(hipMemcpyAsync(h->hflags, gb.ctl, 16 * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream), "gmres");
    API_HIP(hipStreamSynchronize(h->stream), "gmres");
    r.converged = reinterpret_cast<GmCtl*>(h->hflags)->converged;
  }
  double trel[kMaxS];
  API_HIP(true_relres(v, p, B, X, gb.V, gb.partial, gb.gpart, h->cnt, gb.Gb, gb.ctl->r0n, trr, gb.flag, tsc,
                      h->stream),
          "gmres");
  API_HIP(hipMemcpyAsync(trel, trr, sizeof(double) * p, hipMemcpyDeviceToHost, h->stream), "gmres");
  const int hist_len = r.steps < hist_cap ? r.steps : hist_cap;
  if (hist_len > 0)
    API_HIP(hipMemcpyAsync(info->hist, gb.hist, sizeof(double) * hist_len, hipMemcpyDeviceToHost, h->stream), "gmres");
  API_HIP(hipStreamSynchronize(h->stream), "gmres");
  if (info) {
    info->iters = r.steps;
    info->reorth = 0;
    info->outer_iters = r.cycles;
    info->converged = r.converged;
    info->hist_len = hist_len;
    info->seconds = now_s() - t0;
    if (info->relres) memcpy(info->relres, trel, sizeof(double) * p);
    if (info->true_relres) memcpy(info->true_relres, trel, sizeof(double) * p);
  }
  if (r.bad_index) return fail(h, BKRY_E_INVALID, "a CSR column index was outside [0, n)");
  rc = status_of(r.status, h);
  if (rc) return rc;
  return r.converged ? BKRY_OK : BKRY_NOT_CONVERGED;
}
}  // namespace

extern "C" {

int bkry_gmres_solve(bkry_handle h, const bkry_csr* A, int32_t p, bkry_subalg S, const double* B, double* X,
                     double tol, int32_t maxit, int32_t restart, bkry_info* info) {
  return gmres_impl(h, A, p, S, B, X, tol, maxit, restart, 0, info);
}

int bkry_gmres_pipelined_solve(bkry_handle h, const bkry_csr* A, int32_t p, bkry_subalg S, const double* B,
                               double* X, double tol, int32_t maxit, int32_t restart, int32_t r, bkry_info* info) {
  if (h && r < 1) {
    h->err = "the pipelined Gram-Schmidt window r must be >= 1";
    return BKRY_E_INVALID;
  }
  return gmres_impl(h, A, p, S, B, X, tol, maxit, restart, r, info);
}

int bkry_bicgstab_solve(bkry_handle h, const bkry_csr* A, int32_t p, bkry_subalg S, const double* B, double* X,
                        double tol, int32_t maxit, double eta, bkry_info* info) {
  int rc = begin(h);
  Sub sub;
  if (!rc) rc = check_csr(h, A, true);
  if (!rc) rc = check_sub(h, p, S, sub);
  if (!rc) rc = check_blocks(h, {B, X});
  if (!rc && !(tol >= 0.0)) rc = fail(h, BKRY_E_INVALID, "tol must be >= 0");
  if (!rc && maxit < 0) rc = fail(h, BKRY_E_INVALID, "maxit must be >= 0");
  if (!rc && !(eta >= 0.0)) rc = fail(h, BKRY_E_INVALID, "eta must be >= 0");
  if (!rc && (A->n < sub.g || (sub.kind == GLOBAL && A->n < p)))
    rc = fail(h, BKRY_E_INVALID, "block BiCGStab needs n >= p (block, global) or n >= p/q (hybrid)");
  if (rc) return rc;
  const double t0 = now_s();
  const int64_t n = A->n;
  const int hist_cap = (info && info->hist && info->hist_cap > 0) ? info->hist_cap : 0;
  int W = 0;
  rc = ell_width_for(h, A, p, sizeof(double), true, W);
  if (rc) return rc;
  const size_t ne = (size_t)n * W;
  Carver c;
  carve_bc(c, n, sub, hist_cap, h->cnt);
  c.take<double>(kMaxS);
  c.take<double>(kMaxS);
  c.take<int32_t>(4);
  c.take<int32_t>(ne);
  c.take<double>(ne);
  c.take<double>(kMaxS);
  rc = ensure_ws(h, c.off);
  if (rc) return rc;
  Carver w{h->ws};
  BcBufs bb = carve_bc(w, n, sub, hist_cap, h->cnt);
  double* trr = w.take<double>(kMaxS);
  double* tsc = w.take<double>(kMaxS);
  int32_t* tfl = w.take<int32_t>(4);
  int32_t* ecol = w.take<int32_t>(ne);
  double* eval = w.take<double>(ne);
  double* r0save = w.take<double>(kMaxS);
  CsrView v = view(A);
  rc = ell_build<double, double>(h, A, A->val, W, ecol, eval, v, true);
  if (rc) return rc;
  // The recursion's residual can drift from the true one (BiCGStab's residual
  // gap).  When the recursion meets tol but the FP64 true residual does not,
  // the iteration is restarted from the current X (new normalised residual
  // and shadow residual, the first start's stopping denominators), at most
  // kBcRestarts times within maxit; converged means the true residual meets
  // tol.
  constexpr int kBcRestarts = 10;
  BcResult r;
  double relres[kMaxS], trel[kMaxS];
  int total = 0, nre = 0, restarts = 0;
  for (;;) {
    const int used = total;
    BcBufs bbr = bb;
    bbr.hist = bb.hist + (used < hist_cap ? used : hist_cap);
    const int cap_r = hist_cap > used ? hist_cap - used : 0;
    hipError_t e = bc_run(v, sub, B, X, tol, maxit - used, eta, cap_r, bbr, h->stream, h->hflags, r,
                          restarts ? r0save : nullptr);
    if (e != hipSuccess) return hip_fail(h, e, "bicgstab_solve");
    total += r.iters;
    nre += r.nreorth;
    if (!restarts)
      API_HIP(hipMemcpyAsync(r0save, bb.ctl->r0n, sizeof(double) * p, hipMemcpyDeviceToDevice, h->stream), "bicgstab");
    API_HIP(hipMemcpyAsync(relres, bb.ctl->relres, sizeof(double) * p, hipMemcpyDeviceToHost, h->stream),
            "bicgstab");
    API_HIP(true_relres(v, p, B, X, bb.W3, bb.partial, bb.gpart, h->cnt, bb.G, bb.ctl->r0n, trr, tfl, tsc,
                        h->stream),
            "bicgstab");
    API_HIP(hipMemcpyAsync(trel, trr, sizeof(double) * p, hipMemcpyDeviceToHost, h->stream), "bicgstab");
    API_HIP(hipStreamSynchronize(h->stream), "bicgstab");
    if (r.bad_index || r.status || !r.converged || tol == 0.0) break;
    double tmax = 0.0;
    for (int i = 0; i < p; ++i) tmax = trel[i] > tmax ? trel[i] : tmax;
    if (tmax <= tol) break;
    r.converged = 0;
    if (restarts == kBcRestarts || total >= maxit) break;
    ++restarts;
  }
  r.iters = total;
  r.nreorth = nre;
  const int hist_len = r.iters < hist_cap ? r.iters : hist_cap;
  if (hist_len > 0)
    API_HIP(hipMemcpyAsync(info->hist, bb.hist, sizeof(double) * hist_len, hipMemcpyDeviceToHost, h->stream),
            "bicgstab");
  API_HIP(hipStreamSynchronize(h->stream), "bicgstab");
  if (info) {
    info->iters = r.iters;
    info->reorth = r.nreorth;
    info->outer_iters = restarts;
    info->converged = r.converged;
    info->hist_len = hist_len;
    info->seconds = now_s() - t0;
    if (info->relres) memcpy(info->relres, relres, sizeof(double) * p);
    if (info->true_relres) memcpy(info->true_relres, trel, sizeof(double) * p);
  }
  if (r.bad_index) return fail(h, BKRY_E_INVALID, "a CSR column index was outside [0, n)");
  rc = status_of(r.status, h);
  if (rc) return rc;
  return r.converged ? BKRY_OK : BKRY_NOT_CONVERGED;
}

int bkry_sddmm(bkry_handle h, const bkry_csr* pattern, int32_t p, double alpha, const double* L, const double* X,
               double* out_val) {
  int rc = begin(h);
  if (!rc) rc = check_csr(h, pattern, false);
  if (!rc && (p < 1 || p > kMaxS)) rc = fail(h, BKRY_E_INVALID, "p must be in [1, 32]");
  if (!rc) rc = check_blocks(h, {L, X});
  if (!rc && pattern->nnz > 0 && !out_val) rc = fail(h, BKRY_E_INVALID, "null out_val");
  if (rc) return rc;
  if (pattern->nnz == 0) return BKRY_OK;
  API_HIP(launch_sddmm<double>(view(pattern), p, alpha, L, X, out_val, h->dflags, h->stream), "sddmm");
  return BKRY_OK;
}

int bkry_csr_transpose(bkry_handle h, const bkry_csr* A, int32_t* rowptrT, int32_t* colindT, double* valT,
                       int32_t* permT) {
  int rc = begin(h);
  if (!rc) rc = check_csr(h, A, true);
  if (!rc && (!rowptrT || (A->nnz > 0 && (!colindT || !valT || !permT))))
    rc = fail(h, BKRY_E_INVALID, "null output pointer");
  if (rc) return rc;
  rc = ensure_ws(h, csr_transpose_ws_bytes(A->n));
  if (rc) return rc;
  API_HIP(csr_transpose_run(A->n, A->nnz, A->rowptr, A->colind, A->val, rowptrT, colindT, valT, permT, h->ws,
                            h->stream),
          "csr_transpose");
  API_HIP(hipMemcpyAsync(h->hflags, h->ws, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream), "csr_transpose");
  API_HIP(hipStreamSynchronize(h->stream), "csr_transpose");
  if (h->hflags[0]) return fail(h, BKRY_E_INVALID, "a CSR column index was outside [0, n)");
  return BKRY_OK;
}

}  // extern "C"
