// C ABI of the library (declared in include/hopf.h): argument checking,
// problem setup, tiling of query columns, workspace management, launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <map>
#include <string>
#include <vector>

#include "../../include/hopf.h"
#include "backward.hpp"
#include "checks.hpp"
#include "common.hpp"
#include "dense.hpp"
#include "control.hpp"
#include "diag.hpp"
#include "rotate.hpp"
#include "setup.hpp"

using namespace hopf;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static hopf_status fail(hopf_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}
#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess)                                                                \
      return fail(_e == hipErrorOutOfMemory ? HOPF_ENOMEM : HOPF_EDEVICE, "%s: %s (%s:%d)", \
                  #expr, hipGetErrorString(_e), __FILE__, __LINE__);                     \
  } while (0)

extern "C" const char* hopf_last_error(void) { return g_err.c_str(); }
extern "C" const char* hopf_version(void) { return "hopf-mi355x 0.1 (gfx950)"; }

// Deterministic scheduling of the dense kernels (read when a launch, or a plan, is built).
static std::atomic<int> g_deterministic{0};
extern "C" hopf_status hopf_set_deterministic(int32_t on) {
  if (on != 0 && on != 1) return fail(HOPF_EINVAL, "hopf_set_deterministic: on must be 0 or 1 (got %d)", (int)on);
  g_deterministic.store(on);
  return HOPF_OK;
}
extern "C" int32_t hopf_get_deterministic(void) { return g_deterministic.load(); }

// ---------------------------------------------------------------------------
// problem handle
// ---------------------------------------------------------------------------
struct hopf_problem {
  int device = 0;
  int n = 0, n_pad = 0, K = 1, level_set = 0, hkind = 0, precision = 0, diagonal = 0, max_iter = 1;
  int jkind = 0;  // hopf_jkind
  double lambda = 1.0, tol = 0.0;
  double* d_w = nullptr;        // n_pad
  float* d_wf = nullptr;        // n_pad, FP32 copy
  double* d_centres = nullptr;  // K*n_pad (null if all centres are 0 and K == 1)
  double* d_Md = nullptr;       // n_pad^2
  float* d_Mf = nullptr;        // n_pad^2 (F32 precision)
  __bf16* d_Mb = nullptr;       // n_pad^2 (BF16_REFINED precision)
  int8_t* d_Mq = nullptr;       // BF16_REFINED: M in integer slices for the exact anchor products
  int32_t* d_Mqe = nullptr;     // their row exponents
  double* d_adiag = nullptr;    // n (diagonal A)
  double* d_drift = nullptr;    // n (HOPF_H_LINCTRL: the drift diagonal)
  double* d_minv = nullptr;     // n (diagonal A)
  // HOPF_H_AL2: eigenvectors P of HA (n x n, FP64); the problem is held in HA's eigenbasis
  // (A' = P^T A P, weights = eigenvalues, centres P^T c) and points are rotated in and out
  double* d_HP = nullptr;
  float* d_Af = nullptr;          // dense A (n x n, FP32, original basis) for the control read-out
  double* d_centres0 = nullptr;   // HOPF_H_AL2: the centres in the original basis (K x n_pad)
  unsigned long long* d_iter_total = nullptr;  // passes of the dense kernels over all columns
};

// ---------------------------------------------------------------------------
// per-device workspace
// ---------------------------------------------------------------------------
// chunk counters of a workspace or plan: one per kernel class of a call, and the per-thread
// kernel's point queue in the last
constexpr int kMaxClasses = 64;
constexpr int kCounters = kMaxClasses + 1;

struct Workspace {
  std::mutex mu;
  float* state = nullptr; size_t state_bytes = 0;
  double* state64 = nullptr; size_t state64_bytes = 0;
  unsigned char* best = nullptr; size_t best_bytes = 0;   // per-point best value (double) + copy (int32)
  int* counter = nullptr;
  unsigned char* meta = nullptr; size_t meta_bytes = 0;
  double* scratch = nullptr; size_t scratch_bytes = 0;
  float* rot = nullptr; size_t rot_bytes = 0;              // rotated points of HOPF_H_AL2 problems
  unsigned char* pinned = nullptr; size_t pinned_bytes = 0;
  hipEvent_t ev = nullptr;
  bool ev_pending = false;
  int ncu = 0;
};
static Workspace g_ws[64];

static hopf_status ws_grow(void** p, size_t* cur, size_t need) {
  if (need <= *cur) return HOPF_OK;
  size_t sz = std::max(need, *cur + *cur / 4);
  if (*p) {
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipFree(*p));
    *p = nullptr; *cur = 0;
  }
  HIP_TRY(hipMalloc(p, sz));
  *cur = sz;
  return HOPF_OK;
}

static hopf_status ws_get(int dev, Workspace** out) {
  if (dev < 0 || dev >= 64) return fail(HOPF_EDEVICE, "device index %d out of range", dev);
  Workspace* w = &g_ws[dev];
  if (w->ncu == 0) {
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      return fail(HOPF_EDEVICE, "device %d is %s, this library is built for gfx950", dev, prop.gcnArchName);
    w->ncu = prop.multiProcessorCount;
    HIP_TRY(hipEventCreateWithFlags(&w->ev, hipEventDisableTiming));
  }
  *out = w;
  return HOPF_OK;
}

// Upload small metadata (problem views, tile lists) through a pinned staging buffer.
// The staging buffer is reused only after the previous upload has been consumed.
static hopf_status ws_upload(Workspace* w, const void* src, size_t bytes, hipStream_t stream, void** dst) {
  if (w->ev_pending) { HIP_TRY(hipEventSynchronize(w->ev)); w->ev_pending = false; }
  if (bytes > w->pinned_bytes) {
    if (w->pinned) HIP_TRY(hipHostFree(w->pinned));
    w->pinned = nullptr;
    size_t sz = std::max(bytes, (size_t)1 << 16);
    HIP_TRY(hipHostMalloc((void**)&w->pinned, sz, hipHostMallocDefault));
    w->pinned_bytes = sz;
  }
  hopf_status st = ws_grow((void**)&w->meta, &w->meta_bytes, bytes);
  if (st) return st;
  std::memcpy(w->pinned, src, bytes);
  HIP_TRY(hipMemcpyAsync(w->meta, w->pinned, bytes, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipEventRecord(w->ev, stream));
  w->ev_pending = true;
  *dst = w->meta;
  return HOPF_OK;
}

static int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return v ? std::atoi(v) : dflt;
}

// ---------------------------------------------------------------------------
// create / destroy
// ---------------------------------------------------------------------------
static hopf_status validate(const hopf_problem_desc* d) {
  char why[512];
  const hopf_status st = check_desc(d, why, sizeof why);
  return st ? fail(st, "%s", why) : HOPF_OK;
}

static hopf_status validate_columns(int64_t npts, int32_t K) {
  char why[256];
  const hopf_status st = check_columns(npts, K, why, sizeof why);
  return st ? fail(st, "%s", why) : HOPF_OK;
}

// Device memory of problems (their matrices and set-up temporaries).  Freed blocks are kept per
// device and exact size, up to kBlockCache bytes per device, and handed out again: creating a
// problem of a size created before then costs no hipMalloc (a large one costs tens of
// microseconds, and a problem takes about a dozen).  A block is cached only after the device has
// finished its queued work (the implicit synchronisation of hipFree, kept), so no pending kernel
// can still read it when it is handed out again.
namespace {
struct LiveBlock { int dev; size_t bytes; };
std::mutex g_blk_mu;
std::unordered_map<void*, LiveBlock> g_blk_live;
std::multimap<std::pair<int, size_t>, void*> g_blk_free;
size_t g_blk_cached[64] = {};
constexpr size_t kBlockCache = size_t(1) << 30;
}  // namespace

static hipError_t dmalloc_raw(void** p, size_t bytes) {
  *p = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev >= 0 && dev < 64 && bytes > 0) {
    std::lock_guard<std::mutex> g(g_blk_mu);
    auto it = g_blk_free.find({dev, bytes});
    if (it != g_blk_free.end()) {
      *p = it->second;
      g_blk_free.erase(it);
      g_blk_cached[dev] -= bytes;
      g_blk_live[*p] = {dev, bytes};
      return hipSuccess;
    }
  }
  e = hipMalloc(p, bytes);
  if (e != hipSuccess) { *p = nullptr; return e; }
  if (*p && dev >= 0 && dev < 64) {
    std::lock_guard<std::mutex> g(g_blk_mu);
    g_blk_live[*p] = {dev, bytes};
  }
  return hipSuccess;
}
template <typename T>
static hipError_t dmalloc(T** p, size_t bytes) {
  void* v = nullptr;
  const hipError_t e = dmalloc_raw(&v, bytes);
  *p = (T*)v;
  return e;
}
static void dfree(void* p) {
  if (!p) return;
  LiveBlock b{};
  {
    std::lock_guard<std::mutex> g(g_blk_mu);
    auto it = g_blk_live.find(p);
    if (it == g_blk_live.end()) { (void)hipFree(p); return; }
    b = it->second;
    g_blk_live.erase(it);
  }
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) cur = b.dev;
  if (cur != b.dev) (void)hipSetDevice(b.dev);
  const hipError_t e = hipDeviceSynchronize();
  if (cur != b.dev) (void)hipSetDevice(cur);
  if (e == hipSuccess) {
    std::lock_guard<std::mutex> g(g_blk_mu);
    if (g_blk_cached[b.dev] + b.bytes <= kBlockCache) {
      g_blk_free.insert({{b.dev, b.bytes}, p});
      g_blk_cached[b.dev] += b.bytes;
      return;
    }
  }
  (void)hipFree(p);
}

static void free_problem(hopf_problem* p) {
  dfree(p->d_w); dfree(p->d_wf); dfree(p->d_centres); dfree(p->d_Md); dfree(p->d_Mf); dfree(p->d_Mb);
  dfree(p->d_Mq); dfree(p->d_Mqe); dfree(p->d_drift);
  dfree(p->d_adiag); dfree(p->d_minv); dfree(p->d_HP); dfree(p->d_Af); dfree(p->d_centres0);
  dfree(p->d_iter_total);
  delete p;
}

// HOPF_H_AL2 on the per-thread path: HA = P diag(sig) P^T on the device (Jacobi, FP64) into
// p->d_HP, and sig as the problem's weights; the problem stays in the caller's basis.
static hopf_status eig_HA(hopf_problem* p, const hopf_problem_desc* d, hipStream_t stream) {
  const int n = p->n;
  const size_t nn = (size_t)n * n;
  double *dHA = nullptr, *sig = nullptr;
  int* sweeps = nullptr;
  auto cleanup = [&]() { dfree(dHA); dfree(sig); dfree(sweeps); };
  if (dmalloc(&p->d_HP, sizeof(double) * nn) || dmalloc(&dHA, sizeof(double) * nn) ||
      dmalloc(&sig, sizeof(double) * n) || dmalloc(&sweeps, sizeof(int))) {
    cleanup();
    return fail(HOPF_ENOMEM, "hipMalloc HA eigenbasis");
  }
  hipError_t e = hipMemcpy(dHA, d->HA, sizeof(double) * nn, hipMemcpyHostToDevice);
  if (!e) e = launch_jacobi_eig(dHA, n, p->d_HP, sig, sweeps, stream);
  if (!e) e = launch_set_weights(sig, n, p->n_pad, p->d_w, p->d_wf, stream);
  std::vector<double> hs(n);
  if (!e) e = hipStreamSynchronize(stream);
  if (!e) e = hipMemcpy(hs.data(), sig, sizeof(double) * n, hipMemcpyDeviceToHost);
  cleanup();
  if (e) return fail(HOPF_EDEVICE, "HA eigenbasis: %s", hipGetErrorString(e));
  for (int i = 0; i < n; ++i)
    if (!(hs[i] > 0.0)) return fail(HOPF_ENOTSPD, "HA is not positive definite (eigenvalue %g)", hs[i]);
  return HOPF_OK;
}

// HOPF_H_AL2: HA = P diag(sig) P^T on the device (Jacobi, FP64); the problem is moved into that
// basis in place: A (device, n x n) <- P^T A P, weights <- sig, centres <- P^T c.  Synchronises
// to check that HA is positive definite.
static hopf_status rotate_problem(hopf_problem* p, const hopf_problem_desc* d, double* dA, hipStream_t stream) {
  const int n = p->n;
  double *dHA = nullptr, *sig = nullptr, *T = nullptr, *A2 = nullptr, *C2 = nullptr;
  int* sweeps = nullptr;
  auto cleanup = [&]() { dfree(dHA); dfree(sig); dfree(T); dfree(A2); dfree(C2); dfree(sweeps); };
  const size_t nn = (size_t)n * n;
  if (dmalloc(&p->d_HP, sizeof(double) * nn) || dmalloc(&dHA, sizeof(double) * nn) ||
      dmalloc(&sig, sizeof(double) * n) || dmalloc(&T, sizeof(double) * nn) ||
      dmalloc(&A2, sizeof(double) * nn) || dmalloc(&sweeps, sizeof(int))) {
    cleanup();
    return fail(HOPF_ENOMEM, "hipMalloc HA eigenbasis");
  }
  hipError_t e = hipMemcpy(dHA, d->HA, sizeof(double) * nn, hipMemcpyHostToDevice);
  if (!e) e = launch_jacobi_eig(dHA, n, p->d_HP, sig, sweeps, stream);
  if (!e) e = launch_congruence(dA, p->d_HP, n, T, A2, stream);
  if (!e) e = hipMemcpyAsync(dA, A2, sizeof(double) * nn, hipMemcpyDeviceToDevice, stream);
  if (!e) e = launch_set_weights(sig, n, p->n_pad, p->d_w, p->d_wf, stream);
  if (!e && p->d_centres) {
    const size_t cb = sizeof(double) * (size_t)p->K * p->n_pad;
    if (dmalloc(&C2, cb)) { cleanup(); return fail(HOPF_ENOMEM, "hipMalloc centres"); }
    e = hipMemsetAsync(C2, 0, cb, stream);
    if (!e) e = launch_rotate_centres(p->d_centres, C2, p->n_pad, p->d_HP, n, p->K, stream);
    if (!e) e = hipMemcpyAsync(p->d_centres, C2, cb, hipMemcpyDeviceToDevice, stream);
  }
  std::vector<double> hs(n);
  int hsw = 0;
  if (!e) e = hipStreamSynchronize(stream);
  if (!e) e = hipMemcpy(hs.data(), sig, sizeof(double) * n, hipMemcpyDeviceToHost);
  if (!e) e = hipMemcpy(&hsw, sweeps, sizeof(int), hipMemcpyDeviceToHost);
  cleanup();
  if (e) return fail(HOPF_EDEVICE, "HA eigenbasis: %s", hipGetErrorString(e));
  for (int i = 0; i < n; ++i)
    if (!(hs[i] > 0.0)) return fail(HOPF_ENOTSPD, "HA is not positive definite (eigenvalue %g)", hs[i]);
  (void)hsw;
  return HOPF_OK;
}

static hopf_status create_one(const hopf_problem_desc* d, hipStream_t stream, hopf_problem** out,
                              std::vector<double*>* pending_S) {
  hopf_status st = validate(d);
  if (st) return st;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  Workspace* w;
  if ((st = ws_get(dev, &w))) return st;
  hopf_problem* p = new hopf_problem;
  p->device = dev;
  p->n = d->n; p->K = d->K; p->level_set = d->level_set ? 1 : 0; p->hkind = d->hkind;
  p->precision = d->precision; p->lambda = d->lambda; p->tol = d->tol; p->max_iter = d->max_iter;
  const bool al2 = d->hkind == HOPF_H_AL2;
  p->jkind = d->jkind;
  // HOPF_H_AL2 in FP64 stays in the caller's basis on the per-thread path (the prox rotates);
  // otherwise it is solved in HA's eigenbasis, where A is dense
  const bool al2_rot = al2 && d->precision != HOPF_F64;
  p->diagonal = (!al2_rot && (p->jkind != HOPF_J_QUADRATIC || d->A == nullptr || d->A_is_diagonal)) ? 1 : 0;
  const int n = d->n;
  const int n_pad = (n + 31) / 32 * 32;
  p->n_pad = n_pad;
  auto bail = [&](hopf_status s) { free_problem(p); return s; };
  std::vector<double> hw(n_pad, 0.0);
  for (int i = 0; i < n; ++i) hw[i] = d->w ? d->w[i] : 1.0;
  hipError_t e = dmalloc(&p->d_w, sizeof(double) * n_pad);
  if (e) return bail(fail(HOPF_ENOMEM, "hipMalloc w"));
  e = hipMemcpy(p->d_w, hw.data(), sizeof(double) * n_pad, hipMemcpyHostToDevice);
  if (e) return bail(fail(HOPF_EDEVICE, "copy w: %s", hipGetErrorString(e)));
  {
    std::vector<float> hwf(n_pad);
    for (int i = 0; i < n_pad; ++i) hwf[i] = (float)hw[i];
    if (dmalloc(&p->d_wf, sizeof(float) * n_pad)) return bail(fail(HOPF_ENOMEM, "hipMalloc wf"));
    if (hipMemcpy(p->d_wf, hwf.data(), sizeof(float) * n_pad, hipMemcpyHostToDevice))
      return bail(fail(HOPF_EDEVICE, "copy wf"));
  }
  if (dmalloc(&p->d_iter_total, sizeof(unsigned long long))) return bail(fail(HOPF_ENOMEM, "hipMalloc counter"));
  if (d->hkind == HOPF_H_LINCTRL) {
    if (dmalloc(&p->d_drift, sizeof(double) * n)) return bail(fail(HOPF_ENOMEM, "hipMalloc drift"));
    if (hipMemcpy(p->d_drift, d->drift, sizeof(double) * n, hipMemcpyHostToDevice))
      return bail(fail(HOPF_EDEVICE, "copy drift"));
  }
  if (hipMemset(p->d_iter_total, 0, sizeof(unsigned long long))) return bail(fail(HOPF_EDEVICE, "clear counter"));
  if (d->centres) {
    std::vector<double> hc((size_t)d->K * n_pad, 0.0);
    for (int k = 0; k < d->K; ++k)
      for (int i = 0; i < n; ++i) hc[(size_t)k * n_pad + i] = d->centres[(size_t)k * n + i];
    if (dmalloc(&p->d_centres, sizeof(double) * hc.size())) return bail(fail(HOPF_ENOMEM, "hipMalloc centres"));
    if (hipMemcpy(p->d_centres, hc.data(), sizeof(double) * hc.size(), hipMemcpyHostToDevice))
      return bail(fail(HOPF_EDEVICE, "copy centres"));
  }
  const size_t mm = (size_t)n_pad * n_pad;
  if (dmalloc(&p->d_Md, sizeof(double) * mm)) return bail(fail(HOPF_ENOMEM, "hipMalloc M (FP64)"));
  if (d->precision != HOPF_BF16_REFINED && dmalloc(&p->d_Mf, sizeof(float) * mm))
    return bail(fail(HOPF_ENOMEM, "hipMalloc M (FP32)"));
  if (d->precision == HOPF_BF16_REFINED && dmalloc(&p->d_Mb, sizeof(__bf16) * mm))
    return bail(fail(HOPF_ENOMEM, "hipMalloc M (BF16)"));
  // integer slices of M for the exact anchor products of the refined tile solver (BF16 or FP32
  // increments); also for a diagonal problem that hopf_eval runs per thread, since a ragged batch
  // runs it in the dense kernels
  if (d->precision != HOPF_F64 &&
      (dmalloc(&p->d_Mq, (size_t)kSlices * n_pad * pad64(n_pad)) || dmalloc(&p->d_Mqe, sizeof(int32_t) * n_pad)))
    return bail(fail(HOPF_ENOMEM, "hipMalloc M (slices)"));
  if (p->diagonal) {
    std::vector<double> a(n, 1.0);  // unused by the squared-norm initial data
    if (d->A && p->jkind == HOPF_J_QUADRATIC) for (int i = 0; i < n; ++i) a[i] = d->A[i];
    if (dmalloc(&p->d_adiag, sizeof(double) * n) || dmalloc(&p->d_minv, sizeof(double) * n))
      return bail(fail(HOPF_ENOMEM, "hipMalloc diagonal"));
    if (hipMemcpy(p->d_adiag, a.data(), sizeof(double) * n, hipMemcpyHostToDevice))
      return bail(fail(HOPF_EDEVICE, "copy A"));
    e = launch_diag_inverse(p->d_adiag, n, n_pad, d->lambda, p->d_Md, p->d_Mf, p->d_Mb, p->d_minv, stream);
    if (!e && p->d_Mq) e = launch_slice_rows(p->d_Md, n_pad, p->d_Mq, p->d_Mqe, stream);
    if (e) return bail(fail(HOPF_EDEVICE, "diag inverse: %s", hipGetErrorString(e)));
    if (al2) {  // HA = P diag(sig) P^T (FP64 Jacobi on the device); the weights become sig
      if ((st = eig_HA(p, d, stream))) return bail(st);
    }
  } else {
    // A + lambda I in FP64 on the device; the Gauss-Jordan batch is run by the caller
    double* dA = nullptr;
    double* S = nullptr;
    if (dmalloc(&dA, sizeof(double) * (size_t)n * n) || dmalloc(&S, sizeof(double) * mm)) {
      dfree(dA);
      return bail(fail(HOPF_ENOMEM, "hipMalloc setup"));
    }
    std::vector<double> hA;
    const double* srcA = d->A;
    if (al2 && (d->A == nullptr || d->A_is_diagonal)) {  // the rotated problem is dense
      hA.assign((size_t)n * n, 0.0);
      for (int i = 0; i < n; ++i) hA[(size_t)i * n + i] = d->A ? d->A[i] : 1.0;
      srcA = hA.data();
    }
    if (hipMemcpy(dA, srcA, sizeof(double) * (size_t)n * n, hipMemcpyHostToDevice)) {
      dfree(dA); dfree(S);
      return bail(fail(HOPF_EDEVICE, "copy A"));
    }
    {  // FP32 copy of A in the caller's basis (before any rotation), for the control read-out
      const int64_t nn = (int64_t)n * n;
      if (dmalloc(&p->d_Af, sizeof(float) * nn) || launch_to_f32(dA, p->d_Af, nn, stream)) {
        dfree(dA); dfree(S);
        return bail(fail(HOPF_ENOMEM, "FP32 copy of A"));
      }
    }
    if (al2 && p->d_centres) {
      const size_t cb = sizeof(double) * (size_t)p->K * n_pad;
      if (dmalloc(&p->d_centres0, cb) || hipMemcpy(p->d_centres0, p->d_centres, cb, hipMemcpyDeviceToDevice)) {
        dfree(dA); dfree(S);
        return bail(fail(HOPF_ENOMEM, "copy of the centres"));
      }
    }
    if (al2) {
      hopf_status rs = rotate_problem(p, d, dA, stream);
      if (rs) { dfree(dA); dfree(S); return bail(rs); }
    }
    e = launch_build_shifted(dA, n, n_pad, d->lambda, S, stream);
    hipStreamSynchronize(stream);
    dfree(dA);
    if (e) { dfree(S); return bail(fail(HOPF_EDEVICE, "build A + lambda I: %s", hipGetErrorString(e))); }
    pending_S->push_back(S);
  }
  *out = p;
  return HOPF_OK;
}

// Runs the batched block Gauss-Jordan inverse for the dense problems of `probs`
// (pending_S[i] belongs to the i-th dense problem in order), writes the M copies.
static hopf_status factor_batch(std::vector<hopf_problem*>& dense, std::vector<double*>& S,
                                hipStream_t stream) {
  const int np = (int)dense.size();
  if (np == 0) return HOPF_OK;
  std::vector<int> order(np);
  for (int i = 0; i < np; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return dense[a]->n_pad > dense[b]->n_pad; });
  std::vector<SetupProb> hp(np);
  std::vector<int> nblocks(np);
  size_t scratch = 0;
  for (int r = 0; r < np; ++r) scratch += 32 * 32 + 2 * (size_t)dense[order[r]]->n_pad * 32;
  double* d_scr = nullptr;
  int* d_status = nullptr;
  SetupProb* d_probs = nullptr;
  const int steps = dense[order[0]]->n_pad / 32;
  int* d_prefix = nullptr;
  std::vector<int> h_prefix((size_t)steps * 2 * (np + 1));
  auto cleanup = [&]() {
    dfree(d_scr); dfree(d_status); dfree(d_probs); dfree(d_prefix);
  };
  if (dmalloc(&d_scr, sizeof(double) * scratch) || dmalloc(&d_status, sizeof(int) * np) ||
      dmalloc(&d_probs, sizeof(SetupProb) * np) ||
      dmalloc(&d_prefix, sizeof(int) * h_prefix.size())) {
    cleanup();
    return fail(HOPF_ENOMEM, "hipMalloc setup scratch");
  }
  double* q = d_scr;
  for (int r = 0; r < np; ++r) {
    hopf_problem* p = dense[order[r]];
    SetupProb& sp = hp[r];
    sp.S = S[order[r]]; sp.n_pad = p->n_pad; sp.status = d_status + r;
    sp.P = q; q += 32 * 32;
    sp.T = q; q += (size_t)p->n_pad * 32;
    sp.R = q; q += (size_t)p->n_pad * 32;
    nblocks[r] = p->n_pad / 32;
  }
  hipError_t e = hipMemsetAsync(d_status, 0, sizeof(int) * np, stream);
  if (!e) e = hipMemcpyAsync(d_probs, hp.data(), sizeof(SetupProb) * np, hipMemcpyHostToDevice, stream);
  if (!e) e = run_gauss_jordan(d_probs, nblocks.data(), np, d_prefix, h_prefix.data(), stream);
  for (int r = 0; r < np && !e; ++r) {
    hopf_problem* p = dense[order[r]];
    e = launch_finalize_copies(S[order[r]], p->n, p->n_pad, p->d_Md, p->d_Mf, p->d_Mb, stream);
    if (!e && p->d_Mq) e = launch_slice_rows(p->d_Md, p->n_pad, p->d_Mq, p->d_Mqe, stream);
  }
  std::vector<int> status(np, 0);
  if (!e) e = hipMemcpyAsync(status.data(), d_status, sizeof(int) * np, hipMemcpyDeviceToHost, stream);
  if (!e) e = hipStreamSynchronize(stream);
  cleanup();
  if (e) return fail(HOPF_EDEVICE, "factorisation: %s", hipGetErrorString(e));
  for (int r = 0; r < np; ++r)
    if (status[r]) return fail(HOPF_ENOTSPD, "A + lambda I is not positive definite (problem %d)", order[r]);
  return HOPF_OK;
}

extern "C" hopf_status hopf_problem_create(const hopf_problem_desc* desc, void* stream, hopf_problem_t* out) {
  if (!out) return fail(HOPF_EINVAL, "out is NULL");
  *out = nullptr;
  return hopf_problem_create_batch(1, desc, stream, out);
}

extern "C" hopf_status hopf_problem_create_batch(int32_t nprob, const hopf_problem_desc* descs, void* stream,
                                                 hopf_problem_t* out) {
  if (nprob < 0 || (nprob > 0 && (!descs || !out))) return fail(HOPF_EINVAL, "bad batch arguments");
  hipStream_t s = (hipStream_t)stream;
  std::vector<hopf_problem*> made, dense;
  std::vector<double*> S;
  for (int i = 0; i < nprob; ++i) out[i] = nullptr;
  auto undo = [&]() {
    for (double* x : S) dfree(x);
    for (hopf_problem* p : made) free_problem(p);
  };
  for (int i = 0; i < nprob; ++i) {
    hopf_problem* p = nullptr;
    size_t before = S.size();
    hopf_status st = create_one(&descs[i], s, &p, &S);
    if (st) {
      std::string m = g_err;
      undo();
      return fail(st, "problem %d: %s", i, m.c_str());
    }
    made.push_back(p);
    if (S.size() > before) dense.push_back(p);
  }
  hopf_status st = factor_batch(dense, S, s);
  for (double* x : S) dfree(x);
  S.clear();
  if (st) {
    std::string m = g_err;
    for (hopf_problem* p : made) free_problem(p);
    return fail(st, "%s", m.c_str());
  }
  for (int i = 0; i < nprob; ++i) out[i] = made[i];
  return HOPF_OK;
}

extern "C" hopf_status hopf_problem_destroy(hopf_problem_t p) {
  if (!p) return HOPF_OK;
  hipDeviceSynchronize();
  free_problem(p);
  return HOPF_OK;
}

extern "C" hopf_status hopf_problem_info(hopf_problem_t p, int32_t* n, int32_t* n_pad, int32_t* K,
                                         int32_t* precision) {
  if (!p) return fail(HOPF_EINVAL, "problem is NULL");
  if (n) *n = p->n;
  if (n_pad) *n_pad = p->n_pad;
  if (K) *K = p->K;
  if (precision) *precision = p->precision;
  return HOPF_OK;
}

extern "C" hopf_status hopf_problem_iterations(hopf_problem_t p, int64_t* total, int32_t reset) {
  if (!p || !total) return fail(HOPF_EINVAL, "NULL argument");
  unsigned long long v = 0;
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(&v, p->d_iter_total, sizeof v, hipMemcpyDeviceToHost));
  *total = (int64_t)v;
  if (reset) HIP_TRY(hipMemset(p->d_iter_total, 0, sizeof v));
  return HOPF_OK;
}

extern "C" hopf_status hopf_problem_get_inverse(hopf_problem_t p, double* out) {
  if (!p || !out) return fail(HOPF_EINVAL, "NULL argument");
  std::vector<double> h((size_t)p->n_pad * p->n_pad);
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(h.data(), p->d_Md, sizeof(double) * h.size(), hipMemcpyDeviceToHost));
  for (int i = 0; i < p->n; ++i)
    for (int j = 0; j < p->n; ++j) out[(size_t)i * p->n + j] = h[(size_t)i * p->n_pad + j];
  return HOPF_OK;
}

// ---------------------------------------------------------------------------
// dense launches (one problem or a ragged batch)
// ---------------------------------------------------------------------------
struct DenseCall {
  hopf_problem* p;
  DenseProb view;
};

// A dense call split into kernel classes (one persistent launch each, by launch shape): every
// class has its own metadata (problem views, then chunks of whole points), staging and chunk
// counter, so the classes are enqueued back to back without the host waiting between them.
struct DenseClass {
  int key = 0;              // kSmallClass + kind of H, kRsClass or 100000 wl + 10000 ks + 100 pt + 10 occ + nw
  DenseVariant var{};
  bool small = false, rs = false;
  int nchunks = 0, grid = 0, max_npad = 32;
  size_t lds = 0;
  int64_t ws_per_wg = 0, ws64_per_wg = 0;
  size_t views_off = 0, chunks_off = 0;    // bytes into the metadata blob
  size_t state_off = 0, state64_off = 0;   // floats / doubles into the staging
  std::vector<int> members;                // call indices, in view order
  std::vector<DenseChunk> chunks;
};
struct DensePlan {
  int mode = 0, distance = 0;
  int anchor_every = 32, anchor_wait = 0, rs_anchor_every = 24, small_anchor_every = 32, small_anchor_wait = 0;
  int det = 0;  // fixed chunk schedule (hopf_set_deterministic)
  std::vector<DenseClass> cls;
  size_t blob_bytes = 0, state_floats = 0, state64_doubles = 0;
  int64_t total_pts = 0;
};
constexpr int kSmallClass = 1 << 20, kRsClass = 1 << 21;

static void plan_dense(const std::vector<DenseCall>& calls, int mode, int distance, int ncu, DensePlan* P) {
  P->mode = mode; P->distance = distance;
  P->det = g_deterministic.load();
  P->anchor_every = std::max(1, env_int("HOPF_ANCHOR_EVERY", 32));
  // an anchor is also taken as soon as this many columns of a tile wait for one (0: never)
  P->anchor_wait = std::max(0, env_int("HOPF_ANCHOR_WAIT", 0));
  // the on-chip kernel's anchors cost about ten of its passes: every 24 passes gave the fewest
  // cycles on n = 1024 (16: more anchors than iterations saved, 32 and above: more iterations)
  P->rs_anchor_every = std::max(1, env_int("HOPF_RS_ANCHOR_EVERY", 24));
  P->small_anchor_every = std::max(1, env_int("HOPF_SMALL_ANCHOR_EVERY", 32));
  P->small_anchor_wait = std::max(0, env_int("HOPF_SMALL_ANCHOR_WAIT", 0));
  const bool use_small = env_int("HOPF_SMALL", 1) != 0;
  static const bool use_rs = env_int("HOPF_RS", 1) != 0;
  auto class_of = [&](const hopf_problem* p) -> int {
    if (use_small && dense_small_fits(mode, p->n_pad, distance)) return kSmallClass + dense_small_kind(p->hkind);
    if (use_rs && dense_rs_fits(mode, p->n_pad, p->K, p->hkind, distance)) return kRsClass;
    const DenseVariant v = dense_variant(mode, p->n_pad);
    // sqrt(<p, D p>) (also HA's, solved in its eigenbasis) needs the tile kernel's multiplier phase
    const int wl = (p->hkind == HOPF_H_WL2 || p->hkind == HOPF_H_AL2) && !distance ? 1 : 0;
    return 100000 * wl + 10000 * v.ks + 100 * v.pt + 10 * v.occ + v.nw;
  };
  P->total_pts = 0;
  for (auto& c : calls) P->total_pts += c.view.npts;
  std::vector<int> keys;
  for (auto& c : calls) {
    const int key = class_of(c.p);
    if (c.view.npts > 0 && std::find(keys.begin(), keys.end(), key) == keys.end()) keys.push_back(key);
  }
  std::sort(keys.begin(), keys.end());
  size_t off = 0, st = 0, st64 = 0;
  for (int key : keys) {
    DenseClass C;
    C.key = key;
    C.small = key >= kSmallClass && key < kSmallClass + 3;  // + the kind of H
    C.rs = key == kRsClass;
    C.var = C.small ? DenseVariant{dense_small_cols(), dense_small_occupancy(), 4, 1}
          : C.rs    ? DenseVariant{dense_rs_cols(), 1, 4, 1}
                    : DenseVariant{(key % 10000) / 100, (key / 10) % 10, key % 10, (key / 10000) % 10, key / 100000};
    std::vector<std::pair<double, int>> order;  // (cost, view index)
    for (int i = 0; i < (int)calls.size(); ++i) {
      const DenseCall& c = calls[i];
      if (class_of(c.p) != key || c.view.npts == 0) continue;
      order.push_back({(double)c.p->n_pad * c.p->n_pad * c.p->K * (double)c.view.npts, (int)C.members.size()});
      C.members.push_back(i);
      C.max_npad = std::max(C.max_npad, c.p->n_pad);
    }
    // largest problems first; chunks of whole points, about one tile of columns each
    std::stable_sort(order.begin(), order.end(), [](const std::pair<double, int>& x, const std::pair<double, int>& y) {
      return x.first > y.first;
    });
    for (auto& o : order) {
      const DenseProb& v = calls[C.members[o.second]].view;
      const int ppc = std::max(1, C.var.pt / v.K);
      for (int64_t p0 = 0; p0 < v.npts; p0 += ppc) {
        DenseChunk ch;
        ch.prob = o.second;
        ch.col0 = (int)(p0 * v.K);
        ch.ncols = (int)(std::min<int64_t>(ppc, v.npts - p0) * v.K);
        ch.pad = 0;
        C.chunks.push_back(ch);
      }
    }
    C.nchunks = (int)C.chunks.size();
    // the small kernel: four independent waves per workgroup, each taking chunks
    C.grid = C.small ? std::min((C.nchunks + 3) / 4, C.var.occ * ncu) : std::min(C.nchunks, C.var.occ * ncu);
    // the tile kernel's staging: z^a, dz, e^a, p (and the split contraction's partial products)
    C.ws_per_wg = C.small ? 0
                : C.rs    ? dense_rs_ws_floats(C.max_npad)
                          : (C.var.ks == 2 ? 5 : 4) * (int64_t)C.var.pt * C.max_npad;
    // FP64 anchor staging, then its integer slices (kSlices x pt x pad64 bytes)
    C.ws64_per_wg = (int64_t)C.var.pt * C.max_npad + (int64_t)kSlices * C.var.pt * pad64(C.max_npad) / 8;
    if (C.rs)
      C.lds = dense_rs_lds_bytes(C.max_npad);
    else if (!C.small)
      for (int i : C.members) C.lds = std::max(C.lds, dense_lds_bytes(mode, calls[i].p->n_pad));
    C.views_off = off;
    off += (sizeof(DenseProb) * C.members.size() + 255) / 256 * 256;
    C.chunks_off = off;
    off += (sizeof(DenseChunk) * C.chunks.size() + 255) / 256 * 256;
    C.state_off = st;
    st += (size_t)C.ws_per_wg * C.grid;
    C.state64_off = st64;
    st64 += (size_t)C.ws64_per_wg * C.grid;
    P->cls.push_back(std::move(C));
  }
  P->blob_bytes = std::max<size_t>(off, 256);
  P->state_floats = std::max<size_t>(st, 1);
  P->state64_doubles = std::max<size_t>(st64, 1);
}

// Fills the metadata blob: the views (with their per-point best arrays, bestv/bestk of
// total_pts entries in call order) and the chunks of every class.
static void plan_blob(const DensePlan& P, std::vector<DenseCall>& calls, double* bestv, int32_t* bestk,
                      std::vector<unsigned char>* blob) {
  int64_t o = 0;
  for (auto& c : calls) { c.view.bestv = bestv + o; c.view.bestk = bestk + o; o += c.view.npts; }
  blob->assign(P.blob_bytes, 0);
  for (const DenseClass& C : P.cls) {
    for (size_t m = 0; m < C.members.size(); ++m)
      std::memcpy(blob->data() + C.views_off + m * sizeof(DenseProb), &calls[C.members[m]].view, sizeof(DenseProb));
    if (!C.chunks.empty())
      std::memcpy(blob->data() + C.chunks_off, C.chunks.data(), sizeof(DenseChunk) * C.chunks.size());
  }
}

// Enqueues every class: the resets of its chunk counter and best arrays (kernels), then its
// persistent launch.  No host synchronisation, no allocation.
static hopf_status plan_launch(const DensePlan& P, const std::vector<DenseCall>& calls, const unsigned char* meta,
                               float* state, double* state64, int* counters, hipStream_t stream) {
  for (size_t ci = 0; ci < P.cls.size(); ++ci) {
    const DenseClass& C = P.cls[ci];
    int* counter = counters + ci;
    for (int i : C.members) {
      const DenseProb& v = calls[i].view;
      hipError_t e = launch_reset(counter, v.bestv, v.bestk, v.npts, stream);
      if (e) return fail(HOPF_EDEVICE, "reset launch: %s", hipGetErrorString(e));
    }
    const DenseProb* dv = (const DenseProb*)(meta + C.views_off);
    const DenseChunk* dc = (const DenseChunk*)(meta + C.chunks_off);
    float* ws = state + C.state_off;
    double* ws64 = state64 + C.state64_off;
    hipError_t e =
        C.small ? launch_dense_small(C.max_npad, P.mode == 2, C.key - kSmallClass, dv, dc, C.nchunks, counter, C.grid,
                                     P.small_anchor_every, P.small_anchor_wait, P.det, stream)
        : C.rs  ? launch_dense_rs(C.max_npad, dv, dc, C.nchunks, counter, ws64, C.ws64_per_wg, ws, C.ws_per_wg, C.grid,
                                  C.lds, P.rs_anchor_every, P.anchor_wait, P.det, stream)
                : launch_dense(P.mode, C.var, dv, dc, C.nchunks, counter, ws, ws64, C.ws_per_wg, C.ws64_per_wg, C.grid,
                               C.lds, P.distance, P.anchor_every, P.anchor_wait, P.det, stream);
    if (e) return fail(HOPF_EDEVICE, "dense launch: %s", hipGetErrorString(e));
  }
  return HOPF_OK;
}

static hopf_status run_dense(std::vector<DenseCall>& calls, int mode, int distance, hipStream_t stream) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  Workspace* w;
  hopf_status st = ws_get(dev, &w);
  if (st) return st;
  std::lock_guard<std::mutex> lk(w->mu);
  DensePlan P;
  plan_dense(calls, mode, distance, w->ncu, &P);
  if (P.cls.empty()) return HOPF_OK;
  if ((int)P.cls.size() > kMaxClasses) return fail(HOPF_EINVAL, "too many kernel classes in one call");
  if (!w->counter) HIP_TRY(hipMalloc(&w->counter, sizeof(int) * kCounters));
  const size_t nb = (size_t)std::max<int64_t>(P.total_pts, 1);
  if ((st = ws_grow((void**)&w->best, &w->best_bytes, (sizeof(double) + sizeof(int32_t)) * nb))) return st;
  if ((st = ws_grow((void**)&w->state, &w->state_bytes, sizeof(float) * P.state_floats))) return st;
  if ((st = ws_grow((void**)&w->state64, &w->state64_bytes, sizeof(double) * P.state64_doubles))) return st;
  std::vector<unsigned char> blob;
  plan_blob(P, calls, (double*)w->best, (int32_t*)(w->best + sizeof(double) * nb), &blob);
  void* dmeta = nullptr;
  if ((st = ws_upload(w, blob.data(), blob.size(), stream, &dmeta))) return st;
  return plan_launch(P, calls, (const unsigned char*)dmeta, w->state, w->state64, w->counter, stream);
}

static DenseProb make_view(hopf_problem* p) {
  DenseProb v;
  std::memset(&v, 0, sizeof v);
  v.n = p->n; v.n_pad = p->n_pad; v.K = p->K; v.level_set = p->level_set;
  v.hkind = p->hkind == HOPF_H_AL2 ? HK_WL2 : p->hkind;  // in HA's eigenbasis
  v.max_iter = p->max_iter; v.lambda = p->lambda; v.tol = p->tol;
  v.Mb = p->d_Mb; v.Mf = p->d_Mf; v.Md = p->d_Md; v.Mq = p->d_Mq; v.Mqe = p->d_Mqe; v.w = p->d_w; v.wf = p->d_wf; v.centres = p->d_centres;
  v.max_newton = 50;
  v.iter_total = p->d_iter_total;
  return v;
}

// Solver mode of a precision: 1 BF16 increments on exact anchors; 2 FP32 increments on exact
// anchors (HOPF_F32; HOPF_F32_PLAIN=1 selects 0, the plain FP32 iteration, for comparison).
static int mode_for(int precision) {
  if (precision == HOPF_BF16_REFINED) return 1;
  static const bool plain = env_int("HOPF_F32_PLAIN", 0) != 0;
  return plain ? 0 : 2;
}
static int mode_of(hopf_problem* p) { return mode_for(p->precision); }

// Points of HOPF_H_AL2 problems are solved in HA's eigenbasis: their x (or y) is rotated into a
// workspace buffer before the solve, and the solver's gradient (or closest point) is rotated back
// into the caller's buffer after it.
struct RotBack {
  const float* q; float* dst; const double* P; int n; int64_t npts;
};
static hopf_status rotate_calls_in(std::vector<DenseCall>& calls, hipStream_t stream, std::vector<RotBack>* back) {
  size_t need = 0;
  for (auto& c : calls)
    if (c.p->hkind == HOPF_H_AL2) need += 2 * (size_t)c.view.npts * c.p->n;
  if (need == 0) return HOPF_OK;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  Workspace* w;
  hopf_status st = ws_get(dev, &w);
  if (st) return st;
  {
    std::lock_guard<std::mutex> lk(w->mu);
    if ((st = ws_grow((void**)&w->rot, &w->rot_bytes, sizeof(float) * need))) return st;
  }
  float* q = w->rot;
  for (auto& c : calls) {
    if (c.p->hkind != HOPF_H_AL2 || c.view.npts == 0) continue;
    const int n = c.p->n;
    float* xr = q; q += (size_t)c.view.npts * n;
    float* qr = q; q += (size_t)c.view.npts * n;
    hipError_t e = launch_rotate_points_in(c.view.x, xr, c.p->d_HP, n, c.view.npts, stream);
    if (e) return fail(HOPF_EDEVICE, "rotate points: %s", hipGetErrorString(e));
    back->push_back(RotBack{qr, c.view.grad, c.p->d_HP, n, c.view.npts});
    c.view.x = xr;
    c.view.grad = qr;
  }
  return HOPF_OK;
}
static hopf_status rotate_calls_out(const std::vector<RotBack>& back, hipStream_t stream) {
  for (const RotBack& b : back) {
    hipError_t e = launch_rotate_points_out(b.q, b.dst, b.P, b.n, b.npts, stream);
    if (e) return fail(HOPF_EDEVICE, "rotate points back: %s", hipGetErrorString(e));
  }
  return HOPF_OK;
}
static hopf_status run_dense_rotated(std::vector<DenseCall>& calls, int mode, int distance, hipStream_t stream) {
  std::vector<RotBack> back;
  hopf_status st = rotate_calls_in(calls, stream, &back);
  if (!st) st = run_dense(calls, mode, distance, stream);
  if (!st) st = rotate_calls_out(back, stream);
  return st;
}

extern "C" hopf_status hopf_eval(hopf_problem_t p, int64_t npts, const void* x, const void* t, void* phi,
                                 void* grad, void* dphidt, int32_t* iters, int32_t* kstar, void* stream) {
  if (!p) return fail(HOPF_EINVAL, "problem is NULL");
  if (hopf_status cs = validate_columns(npts, p->K)) return cs;
  if (npts == 0) return HOPF_OK;
  if (!x || !t || !phi || !grad || !dphidt) return fail(HOPF_EINVAL, "NULL array argument");
  hipStream_t s = (hipStream_t)stream;
  if (p->diagonal && p->n <= kDiagMaxN) {
    DiagProb dp;
    dp.n = p->n; dp.ld = p->n_pad; dp.K = p->K; dp.level_set = p->level_set; dp.hkind = p->hkind;
    dp.jkind = p->jkind;
    dp.max_iter = p->max_iter; dp.lambda = p->lambda; dp.tol = p->tol;
    dp.minv = p->d_minv; dp.adiag = p->d_adiag; dp.w = p->d_w; dp.centres = p->d_centres;
    dp.P = p->hkind == HOPF_H_AL2 ? p->d_HP : nullptr;
    dp.drift = p->d_drift;
    dp.x = x; dp.t = t; dp.npts = npts; dp.phi = phi; dp.grad = grad; dp.dphidt = dphidt;
    dp.iters = iters; dp.kstar = kstar;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    Workspace* w;
    hopf_status st = ws_get(dev, &w);
    if (st) return st;
    {
      std::lock_guard<std::mutex> lk(w->mu);
      if (!w->counter) HIP_TRY(hipMalloc(&w->counter, sizeof(int) * kCounters));
    }
    // the last counter slot is the per-thread kernel's point queue (the tile kernels use the first)
    hipError_t e = launch_diag(dp, p->precision == HOPF_F64, w->counter + kMaxClasses, w->ncu, s);
    if (e) return fail(HOPF_EDEVICE, "diag launch: %s", hipGetErrorString(e));
    return HOPF_OK;
  }
  std::vector<DenseCall> calls(1);
  calls[0].p = p;
  DenseProb& v = calls[0].view;
  v = make_view(p);
  v.x = (const float*)x; v.t = (const float*)t; v.npts = npts;
  v.phi = (float*)phi; v.grad = (float*)grad; v.dphidt = (float*)dphidt; v.iters = iters; v.kstar = kstar;
  return run_dense_rotated(calls, mode_of(p), 0, s);
}

extern "C" hopf_status hopf_control(hopf_problem_t p, int64_t npts, const void* x, const void* t, const void* grad,
                                    const int32_t* kstar, void* beta, void* xT, void* stream) {
  if (!p) return fail(HOPF_EINVAL, "problem is NULL");
  if (p->jkind != HOPF_J_QUADRATIC) return fail(HOPF_EINVAL, "the control read-out needs the quadratic J");
  if (p->hkind == HOPF_H_LINCTRL)
    return fail(HOPF_EINVAL, "the control read-out is for time-independent Hamiltonians");
  if (npts < 0) return fail(HOPF_EINVAL, "npts < 0");
  if (npts == 0) return HOPF_OK;
  if (!x || !t || !grad || !beta || !xT) return fail(HOPF_EINVAL, "NULL array argument");
  if (p->K > 1 && !kstar) return fail(HOPF_EINVAL, "kstar is required when K > 1");
  ControlArgs a;
  a.n = p->n; a.npts = npts; a.kstar = kstar;
  a.Af = p->diagonal ? nullptr : p->d_Af;
  a.adiag = p->d_adiag;
  a.centres = p->d_centres0 ? p->d_centres0 : p->d_centres;
  a.ldc = p->n_pad;
  hipError_t e = launch_control(a, p->precision == HOPF_F64, x, t, grad, beta, xT, (hipStream_t)stream);
  if (e) return fail(HOPF_EDEVICE, "control launch: %s", hipGetErrorString(e));
  return HOPF_OK;
}

extern "C" hopf_status hopf_max_over_hamiltonians(int32_t k, int64_t npts, int32_t n, int32_t f64,
                                                  const void* const* phis, const void* const* grads,
                                                  const void* const* dphidts, void* phi, void* grad, void* dphidt,
                                                  int32_t* istar, void* stream) {
  if (k < 1 || k > kMaxHamiltonians) return fail(HOPF_EINVAL, "k = %d outside [1, %d]", k, kMaxHamiltonians);
  if (npts < 0 || n < 1) return fail(HOPF_EINVAL, "bad sizes");
  if (npts == 0) return HOPF_OK;
  if (!phis || !grads || !dphidts || !phi || !grad || !dphidt) return fail(HOPF_EINVAL, "NULL array argument");
  MaxHArgs a;
  a.k = k; a.n = n; a.npts = npts;
  for (int i = 0; i < k; ++i) {
    if (!phis[i] || !grads[i] || !dphidts[i]) return fail(HOPF_EINVAL, "NULL input %d", i);
    a.phi[i] = phis[i]; a.grad[i] = grads[i]; a.dphidt[i] = dphidts[i];
  }
  hipError_t e = launch_max_h(a, f64 != 0, phi, grad, dphidt, istar, (hipStream_t)stream);
  if (e) return fail(HOPF_EDEVICE, "max launch: %s", hipGetErrorString(e));
  return HOPF_OK;
}

extern "C" hopf_status hopf_closest_point(hopf_problem_t p, int64_t npts, const void* y, double s_tol,
                                          void* dist, void* cp, int32_t* kstar, int32_t* inside,
                                          int32_t* newton, void* stream) {
  if (!p) return fail(HOPF_EINVAL, "problem is NULL");
  if (!p->level_set) return fail(HOPF_EINVAL, "closest point needs an ellipsoid level-set problem (level_set = 1)");
  if (p->jkind != HOPF_J_QUADRATIC) return fail(HOPF_EINVAL, "closest point needs the quadratic J (ellipsoids)");
  if (p->precision == HOPF_F64) return fail(HOPF_EINVAL, "closest point needs HOPF_F32 or HOPF_BF16_REFINED");
  if (!(s_tol > 0.0) || !std::isfinite(s_tol)) return fail(HOPF_EINVAL, "s_tol must be finite and > 0");
  if (hopf_status cs = validate_columns(npts, p->K)) return cs;
  if (npts == 0) return HOPF_OK;
  if (!y || !dist || !cp || !kstar) return fail(HOPF_EINVAL, "NULL array argument");
  std::vector<DenseCall> calls(1);
  calls[0].p = p;
  DenseProb& v = calls[0].view;
  v = make_view(p);
  v.x = (const float*)y; v.npts = npts; v.grad = (float*)cp; v.kstar = kstar;
  v.dist = (float*)dist; v.inside = inside; v.newton = newton; v.s_tol = s_tol;
  return run_dense_rotated(calls, mode_of(p), 1, (hipStream_t)stream);
}

// The calls of a ragged evaluation (the argument checks of hopf_eval_ragged).
static hopf_status ragged_calls(int32_t nprob, const hopf_problem_t* probs, const int64_t* pt_offset,
                                const void* x_packed, const void* t, void* phi, void* grad_packed, void* dphidt,
                                int32_t* iters, int32_t* kstar, std::vector<DenseCall>* calls, int* prec_out) {
  if (nprob < 0 || (nprob > 0 && (!probs || !pt_offset))) return fail(HOPF_EINVAL, "bad ragged arguments");
  if (nprob == 0) return HOPF_OK;
  if (!x_packed || !t || !phi || !grad_packed || !dphidt) return fail(HOPF_EINVAL, "NULL array argument");
  const int prec = probs[0] ? probs[0]->precision : -1;
  if (pt_offset[0] != 0) return fail(HOPF_EINVAL, "pt_offset[0] must be 0");
  int64_t xoff = 0;
  for (int q = 0; q < nprob; ++q) {
    hopf_problem* p = probs[q];
    if (!p) return fail(HOPF_EINVAL, "problem %d is NULL", q);
    char why[256];
    if (hopf_status cs = check_ragged_member(q, p->precision, prec, p->hkind, p->jkind, p->n, why, sizeof why))
      return fail(cs, "%s", why);
    const int64_t np = pt_offset[q + 1] - pt_offset[q];
    if (np < 0) return fail(HOPF_EINVAL, "pt_offset must be nondecreasing");
    if (hopf_status cs = check_columns(np, p->K, why, sizeof why)) return fail(cs, "problem %d: %s", q, why);
    DenseCall c;
    c.p = p;
    c.view = make_view(p);
    const int64_t g0 = pt_offset[q];
    c.view.x = (const float*)x_packed + xoff;
    c.view.t = (const float*)t + g0;
    c.view.npts = np;
    c.view.phi = (float*)phi + g0;
    c.view.grad = (float*)grad_packed + xoff;
    c.view.dphidt = (float*)dphidt + g0;
    c.view.iters = iters ? iters + g0 : nullptr;
    c.view.kstar = kstar ? kstar + g0 : nullptr;
    xoff += np * p->n;
    calls->push_back(c);
  }
  *prec_out = prec;
  return HOPF_OK;
}

extern "C" hopf_status hopf_eval_ragged(int32_t nprob, const hopf_problem_t* probs, const int64_t* pt_offset,
                                        const void* x_packed, const void* t, void* phi, void* grad_packed,
                                        void* dphidt, int32_t* iters, int32_t* kstar, void* stream) {
  std::vector<DenseCall> calls;
  int prec = 0;
  if (hopf_status st = ragged_calls(nprob, probs, pt_offset, x_packed, t, phi, grad_packed, dphidt, iters, kstar,
                                    &calls, &prec))
    return st;
  if (calls.empty()) return HOPF_OK;
  return run_dense_rotated(calls, mode_for(prec), 0, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// A ragged evaluation bound once to its arguments, relaunched by kernels alone
// ---------------------------------------------------------------------------
struct RotIn {
  const float* src; float* dst; const double* P; int n; int64_t npts;
};
struct hopf_ragged_plan {
  int device = 0;
  DensePlan P;
  std::vector<DenseCall> calls;
  std::vector<RotIn> rot_in;
  std::vector<RotBack> rot_back;
  unsigned char* meta = nullptr;
  float* state = nullptr;
  double* state64 = nullptr;
  unsigned char* best = nullptr;
  int* counters = nullptr;
  float* rot = nullptr;
};

static void free_plan(hopf_ragged_plan* pl) {
  hipFree(pl->meta); hipFree(pl->state); hipFree(pl->state64); hipFree(pl->best); hipFree(pl->counters);
  hipFree(pl->rot);
  delete pl;
}

extern "C" hopf_status hopf_ragged_plan_create(int32_t nprob, const hopf_problem_t* probs, const int64_t* pt_offset,
                                               const void* x_packed, const void* t, void* phi, void* grad_packed,
                                               void* dphidt, int32_t* iters, int32_t* kstar,
                                               hopf_ragged_plan_t* out) {
  if (!out) return fail(HOPF_EINVAL, "out is NULL");
  *out = nullptr;
  hopf_ragged_plan* pl = new hopf_ragged_plan();
  auto bail = [&](hopf_status st) { free_plan(pl); return st; };
  int prec = 0;
  if (hopf_status st = ragged_calls(nprob, probs, pt_offset, x_packed, t, phi, grad_packed, dphidt, iters, kstar,
                                    &pl->calls, &prec))
    return bail(st);
  if (hipGetDevice(&pl->device)) return bail(fail(HOPF_EDEVICE, "hipGetDevice"));
  Workspace* w;
  if (hopf_status st = ws_get(pl->device, &w)) return bail(st);
  // points of HOPF_H_AL2 problems are solved in HA's eigenbasis: buffers of the plan's own
  size_t need = 0;
  for (auto& c : pl->calls)
    if (c.p->hkind == HOPF_H_AL2) need += 2 * (size_t)c.view.npts * c.p->n;
  if (need && hipMalloc(&pl->rot, sizeof(float) * need)) return bail(fail(HOPF_ENOMEM, "hipMalloc rotations"));
  float* q = pl->rot;
  for (auto& c : pl->calls) {
    if (c.p->hkind != HOPF_H_AL2 || c.view.npts == 0) continue;
    const int n = c.p->n;
    float* xr = q; q += (size_t)c.view.npts * n;
    float* qr = q; q += (size_t)c.view.npts * n;
    pl->rot_in.push_back(RotIn{c.view.x, xr, c.p->d_HP, n, c.view.npts});
    pl->rot_back.push_back(RotBack{qr, c.view.grad, c.p->d_HP, n, c.view.npts});
    c.view.x = xr;
    c.view.grad = qr;
  }
  plan_dense(pl->calls, mode_for(prec), 0, w->ncu, &pl->P);
  if ((int)pl->P.cls.size() > kMaxClasses) return bail(fail(HOPF_EINVAL, "too many kernel classes in one call"));
  const size_t nb = (size_t)std::max<int64_t>(pl->P.total_pts, 1);
  if (hipMalloc(&pl->meta, pl->P.blob_bytes) || hipMalloc(&pl->state, sizeof(float) * pl->P.state_floats) ||
      hipMalloc(&pl->state64, sizeof(double) * pl->P.state64_doubles) ||
      hipMalloc(&pl->best, (sizeof(double) + sizeof(int32_t)) * nb) ||
      hipMalloc(&pl->counters, sizeof(int) * kMaxClasses))
    return bail(fail(HOPF_ENOMEM, "hipMalloc plan buffers"));
  std::vector<unsigned char> blob;
  plan_blob(pl->P, pl->calls, (double*)pl->best, (int32_t*)(pl->best + sizeof(double) * nb), &blob);
  if (hipMemcpy(pl->meta, blob.data(), blob.size(), hipMemcpyHostToDevice))
    return bail(fail(HOPF_EDEVICE, "upload plan metadata"));
  *out = pl;
  return HOPF_OK;
}

extern "C" hopf_status hopf_ragged_plan_launch(hopf_ragged_plan_t pl, void* stream) {
  if (!pl) return fail(HOPF_EINVAL, "plan is NULL");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != pl->device) return fail(HOPF_EINVAL, "the plan was made on device %d, the current device is %d",
                                     pl->device, dev);
  hipStream_t s = (hipStream_t)stream;
  for (const RotIn& r : pl->rot_in) {
    hipError_t e = launch_rotate_points_in(r.src, r.dst, r.P, r.n, r.npts, s);
    if (e) return fail(HOPF_EDEVICE, "rotate points: %s", hipGetErrorString(e));
  }
  if (hopf_status st = plan_launch(pl->P, pl->calls, pl->meta, pl->state, pl->state64, pl->counters, s)) return st;
  return rotate_calls_out(pl->rot_back, s);
}

extern "C" hopf_status hopf_ragged_plan_destroy(hopf_ragged_plan_t pl) {
  if (!pl) return HOPF_OK;
  hipDeviceSynchronize();
  free_plan(pl);
  return HOPF_OK;
}

extern "C" hopf_status hopf_closest_point_ragged(int32_t nprob, const hopf_problem_t* probs, const int64_t* pt_offset,
                                                 const void* y_packed, double s_tol, void* dist, void* cp_packed,
                                                 int32_t* kstar, int32_t* inside, int32_t* newton, void* stream) {
  if (nprob < 0 || (nprob > 0 && (!probs || !pt_offset))) return fail(HOPF_EINVAL, "bad ragged arguments");
  if (nprob == 0) return HOPF_OK;
  if (!(s_tol > 0.0) || !std::isfinite(s_tol)) return fail(HOPF_EINVAL, "s_tol must be finite and > 0");
  if (!y_packed || !dist || !cp_packed || !kstar) return fail(HOPF_EINVAL, "NULL array argument");
  if (pt_offset[0] != 0) return fail(HOPF_EINVAL, "pt_offset[0] must be 0");
  const int prec = probs[0] ? probs[0]->precision : -1;
  std::vector<DenseCall> calls;
  int64_t yoff = 0;
  for (int q = 0; q < nprob; ++q) {
    hopf_problem* p = probs[q];
    if (!p) return fail(HOPF_EINVAL, "problem %d is NULL", q);
    if (p->precision != prec) return fail(HOPF_EINVAL, "problem %d: problems of a ragged batch must share one precision", q);
    if (p->precision == HOPF_F64) return fail(HOPF_EINVAL, "problem %d: closest point needs HOPF_F32 or HOPF_BF16_REFINED", q);
    if (!p->level_set || p->jkind != HOPF_J_QUADRATIC)
      return fail(HOPF_EINVAL, "problem %d: closest point needs ellipsoid level sets (level_set = 1, quadratic J)", q);
    const int64_t np = pt_offset[q + 1] - pt_offset[q];
    if (np < 0) return fail(HOPF_EINVAL, "pt_offset must be nondecreasing");
    char why[256];
    if (hopf_status cs = check_columns(np, p->K, why, sizeof why)) return fail(cs, "problem %d: %s", q, why);
    DenseCall c;
    c.p = p;
    c.view = make_view(p);
    const int64_t g0 = pt_offset[q];
    c.view.x = (const float*)y_packed + yoff;
    c.view.npts = np;
    c.view.grad = (float*)cp_packed + yoff;
    c.view.dist = (float*)dist + g0;
    c.view.kstar = kstar + g0;
    c.view.inside = inside ? inside + g0 : nullptr;
    c.view.newton = newton ? newton + g0 : nullptr;
    c.view.s_tol = s_tol;
    yoff += np * p->n;
    calls.push_back(c);
  }
  return run_dense_rotated(calls, mode_for(prec), 1, (hipStream_t)stream);
}

extern "C" hopf_status hopf_backward(hopf_problem_t p, int64_t npts, const void* gphi, const void* grad_saved,
                                     const void* dphidt_saved, const int32_t* kstar_saved, void* gx, void* gt,
                                     void* gA, void* gc, void* stream) {
  if (!p) return fail(HOPF_EINVAL, "problem is NULL");
  if (p->precision == HOPF_F64) return fail(HOPF_EINVAL, "backward needs HOPF_F32 or HOPF_BF16_REFINED");
  if (npts < 0) return fail(HOPF_EINVAL, "npts < 0");
  if (npts > 0 && (!gphi || !grad_saved)) return fail(HOPF_EINVAL, "gphi and grad_saved are required");
  if (npts > 0 && gt && !dphidt_saved) return fail(HOPF_EINVAL, "gt needs dphidt_saved");
  if (npts > 0 && gc && p->K > 1 && !kstar_saved) return fail(HOPF_EINVAL, "gc needs kstar_saved when K > 1");
  if (gA && p->jkind != HOPF_J_QUADRATIC) return fail(HOPF_EINVAL, "gA needs the quadratic J");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  Workspace* w;
  hopf_status st = ws_get(dev, &w);
  if (st) return st;
  std::lock_guard<std::mutex> lk(w->mu);
  const BackwardPlan plan = backward_plan(npts, p->n, p->K, gA != nullptr, gc != nullptr, (size_t)-1);
  if ((st = ws_grow((void**)&w->scratch, &w->scratch_bytes, std::max<size_t>(plan.bytes_a + plan.bytes_c, 256))))
    return st;
  BackwardArgs a;
  a.npts = npts; a.n = p->n; a.K = p->K;
  a.g = (const float*)gphi; a.grad = (const float*)grad_saved; a.dphidt = (const float*)dphidt_saved;
  a.kstar = kstar_saved; a.gx = (float*)gx; a.gt = (float*)gt; a.gA = (float*)gA; a.gc = (float*)gc;
  hipError_t e = launch_backward(a, plan, w->scratch, (hipStream_t)stream);
  if (e) return fail(HOPF_EDEVICE, "backward launch: %s", hipGetErrorString(e));
  return HOPF_OK;
}

// ---------------------------------------------------------------------------
// backward without allocations: the split partials live in a fixed device array
// ---------------------------------------------------------------------------
// Every GPU the library runs on holds this array from the library's first use on it until the
// process ends.  Host code never passes the array's own name to a kernel (on the host it is a
// stand-in, not a device address): its device address is looked up once per device with
// hipGetSymbolAddress and only that address is used.
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
static void* g_scratch_ptr[64];
static std::mutex g_scratch_mu;

static hopf_status scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(HOPF_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return HOPF_OK;
}

extern "C" hopf_status hopf_backward_noalloc(hopf_problem_t p, int64_t npts, const void* gphi,
                                             const void* grad_saved, const void* dphidt_saved,
                                             const int32_t* kstar_saved, void* gx, void* gt, void* gA, void* gc,
                                             void* stream) {
  if (!p) return fail(HOPF_EINVAL, "problem is NULL");
  if (p->precision == HOPF_F64) return fail(HOPF_EINVAL, "backward needs HOPF_F32 or HOPF_BF16_REFINED");
  if (npts < 0) return fail(HOPF_EINVAL, "npts < 0");
  if (npts > 0 && (!gphi || !grad_saved)) return fail(HOPF_EINVAL, "gphi and grad_saved are required");
  if (npts > 0 && gt && !dphidt_saved) return fail(HOPF_EINVAL, "gt needs dphidt_saved");
  if (npts > 0 && gc && p->K > 1 && !kstar_saved) return fail(HOPF_EINVAL, "gc needs kstar_saved when K > 1");
  if (gA && p->jkind != HOPF_J_QUADRATIC) return fail(HOPF_EINVAL, "gA needs the quadratic J");
  const BackwardPlan plan = backward_plan(npts, p->n, p->K, gA != nullptr, gc != nullptr, kNoAllocScratchBytes);
  if (!plan.ok || plan.bytes_a + plan.bytes_c > kNoAllocScratchBytes)
    return fail(HOPF_EINVAL,
                "hopf_backward_noalloc: n = %d, K = %d needs more than its %zu-byte scratch (one split of the gA "
                "tiles takes %zu bytes); use hopf_backward",
                p->n, p->K, kNoAllocScratchBytes, (size_t)plan.ntl * 64 * 64 * sizeof(float));
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(HOPF_EDEVICE, "device index %d out of range", dev);
  void* ptr = nullptr;
  if (hopf_status st = scratch_address(dev, &ptr)) return st;
  BackwardArgs a;
  a.npts = npts; a.n = p->n; a.K = p->K;
  a.g = (const float*)gphi; a.grad = (const float*)grad_saved; a.dphidt = (const float*)dphidt_saved;
  a.kstar = kstar_saved; a.gx = (float*)gx; a.gt = (float*)gt; a.gA = (float*)gA; a.gc = (float*)gc;
  hipError_t e = launch_backward(a, plan, ptr, (hipStream_t)stream);
  if (e) return fail(HOPF_EDEVICE, "backward launch: %s", hipGetErrorString(e));
  return HOPF_OK;
}
