// Host-side argument checks of the C ABI (declarations and rules in checks.hpp).
#include "checks.hpp"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

namespace hopf {

static hopf_status say(hopf_status st, char* why, size_t len, const char* fmt, ...) {
  if (why && len > 0) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(why, len, fmt, ap);
    va_end(ap);
  }
  return st;
}

// Index of the first non-finite entry of a[0 .. m), or -1.  The scan accumulates a flag without
// branching (it vectorises); the index is searched only when the flag is set.
static int64_t first_nonfinite(const double* a, int64_t m) {
  int bad = 0;
  for (int64_t i = 0; i < m; ++i) bad |= std::isfinite(a[i]) ? 0 : 1;
  if (!bad) return -1;
  for (int64_t i = 0; i < m; ++i)
    if (!std::isfinite(a[i])) return i;
  return -1;
}

static bool differ(double a, double b) {
  return std::fabs(a - b) > 1e-12 * std::fmax(1.0, std::fmax(std::fabs(a), std::fabs(b)));
}

// Checks the row-major n x n matrix S in one pass: every entry finite, and S symmetric to a
// relative 1e-12.  The matrix is walked in 64 x 64 tiles of the lower block triangle; each
// mirrored upper tile is first copied transposed into a local buffer (row reads), so both
// operands of every comparison are read contiguously, every entry is read once, and the loops
// vectorise (a row-by-row scan reads the upper triangle with a stride of n doubles).  Block rows
// are dealt round-robin to up to 8 host threads from n = 768 (the pass is bound by memory
// bandwidth; below that the threads' start costs more than they save).  Returns 0, or 1 with *bad the first non-finite index, or 2 with (*bi, *bj) the
// first mismatch in row-major order of the lower triangle.
constexpr int kCheckTile = 64;

// Tiles of the block rows first, first + stride, ...: bit 0 set if an entry is not finite, bit 1
// if a pair differs.
static int check_rows(const double* S, int n, int first, int stride) {
  constexpr int kT = kCheckTile;
  double up[kT][kT];  // up[i - ib][j - jb] = S[j][i] (32 KiB)
  int nonfinite = 0, asym = 0;
  for (int ib = first * kT; ib < n; ib += stride * kT) {
    const int ie = std::min(n, ib + kT);
    for (int jb = 0; jb <= ib; jb += kT) {
      const int je = std::min(n, jb + kT);
      if (jb < ib) {
        for (int j = jb; j < je; ++j)
          for (int i = ib; i < ie; ++i) up[i - ib][j - jb] = S[(size_t)j * n + i];
        for (int i = ib; i < ie; ++i) {
          const double* row = S + (size_t)i * n;
          for (int j = jb; j < je; ++j) {
            const double a = row[j], b = up[i - ib][j - jb];
            nonfinite |= (std::isfinite(a) && std::isfinite(b)) ? 0 : 1;
            asym |= differ(a, b) ? 1 : 0;
          }
        }
      } else {  // a diagonal tile: both triangles are in it
        for (int i = ib; i < ie; ++i) {
          const double* row = S + (size_t)i * n;
          for (int j = jb; j < je; ++j) {
            nonfinite |= std::isfinite(row[j]) ? 0 : 1;
            if (j < i) asym |= differ(row[j], S[(size_t)j * n + i]) ? 1 : 0;
          }
        }
      }
    }
  }
  return nonfinite | (asym << 1);
}

static int check_dense(const double* S, int n, int64_t* bad, int* bi, int* bj) {
  const int nbr = (n + kCheckTile - 1) / kCheckTile;  // block rows
  int nt = 1;
  if (n >= 768) {
    const unsigned hc = std::thread::hardware_concurrency();
    nt = std::max(1, std::min({8, nbr, hc > 0 ? (int)hc : 1}));
  }
  int flags = 0;
  if (nt == 1) {
    flags = check_rows(S, n, 0, 1);
  } else {
    std::vector<int> part(nt, 0);
    std::vector<std::thread> pool;
    pool.reserve(nt - 1);
    // the block rows of a thread that could not be started are checked on this thread
    std::vector<char> started(nt, 0);
    for (int t = 1; t < nt; ++t) {
      try {
        pool.emplace_back([&part, S, n, t, nt] { part[t] = check_rows(S, n, t, nt); });
        started[t] = 1;
      } catch (...) {
      }
    }
    part[0] = check_rows(S, n, 0, nt);
    for (int t = 1; t < nt; ++t)
      if (!started[t]) part[t] = check_rows(S, n, t, nt);
    for (auto& th : pool) th.join();
    for (int f : part) flags |= f;
  }
  const int nonfinite = flags & 1, asym = flags & 2;
  if (nonfinite) { *bad = first_nonfinite(S, (int64_t)n * n); return 1; }
  if (!asym) return 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j)
      if (differ(S[(size_t)i * n + j], S[(size_t)j * n + i])) { *bi = i; *bj = j; return 2; }
  return 0;
}

hopf_status check_desc(const hopf_problem_desc* d, char* why, size_t len) {
  if (!d) return say(HOPF_EINVAL, why, len, "desc is NULL");
  if (d->n < 1 || d->n > kMaxN) return say(HOPF_EINVAL, why, len, "n = %d outside [1, %d]", d->n, kMaxN);
  if (d->K < 1 || d->K > kMaxK) return say(HOPF_EINVAL, why, len, "K = %d outside [1, %d]", d->K, kMaxK);
  if (!(d->lambda > 0.0) || !std::isfinite(d->lambda))
    return say(HOPF_EINVAL, why, len, "lambda must be finite and > 0");
  if (!(d->tol >= 0.0) || !std::isfinite(d->tol)) return say(HOPF_EINVAL, why, len, "tol must be finite and >= 0");
  if (d->max_iter < 1) return say(HOPF_EINVAL, why, len, "max_iter must be >= 1");
  // a C caller may store any int in the enum fields: read them as integers (loading an
  // out-of-range value through the C++ enum type would be undefined)
  int hk = 0, prec = 0;
  static_assert(sizeof(d->hkind) == sizeof(int) && sizeof(d->precision) == sizeof(int), "enum fields are ints");
  std::memcpy(&hk, &d->hkind, sizeof hk);
  std::memcpy(&prec, &d->precision, sizeof prec);
  if (hk < HOPF_H_WL1 || hk > HOPF_H_LINCTRL) return say(HOPF_EINVAL, why, len, "unknown hkind %d", hk);
  if (d->jkind < HOPF_J_QUADRATIC || d->jkind > HOPF_J_LINFSQ)
    return say(HOPF_EINVAL, why, len, "unknown jkind %d", (int)d->jkind);
  if (prec < HOPF_F64 || prec > HOPF_BF16_REFINED) return say(HOPF_EINVAL, why, len, "unknown precision %d", prec);
  const int n = d->n;
  if (d->w)
    for (int i = 0; i < n; ++i) {
      if (!(d->w[i] >= 0.0) || !std::isfinite(d->w[i]))
        return say(HOPF_EINVAL, why, len, "w[%d] must be finite and >= 0", i);
      if (d->hkind == HOPF_H_WL2 && !(d->w[i] > 0.0))
        return say(HOPF_EINVAL, why, len, "w[%d] must be > 0 for HOPF_H_WL2 (D = diag(w) positive definite)", i);
    }
  if (d->centres)
    for (int64_t i = 0; i < (int64_t)d->K * n; ++i)
      if (!std::isfinite(d->centres[i])) return say(HOPF_EINVAL, why, len, "centres[%lld] is not finite", (long long)i);
  const bool normsq = d->jkind != HOPF_J_QUADRATIC;
  const bool diag = normsq || d->A == nullptr || d->A_is_diagonal;
  if (d->A && !normsq) {
    if (d->A_is_diagonal) {
      const int64_t bad = first_nonfinite(d->A, n);
      if (bad >= 0) return say(HOPF_EINVAL, why, len, "A[%lld] is not finite", (long long)bad);
      for (int i = 0; i < n; ++i)
        if (!(d->A[i] > 0.0)) return say(HOPF_ENOTSPD, why, len, "diagonal A[%d] = %g is not > 0", i, d->A[i]);
    } else {
      int64_t bad = -1;
      int bi = 0, bj = 0;
      const int r = check_dense(d->A, n, &bad, &bi, &bj);
      if (r == 1) return say(HOPF_EINVAL, why, len, "A[%lld] is not finite", (long long)bad);
      if (r == 2) return say(HOPF_EINVAL, why, len, "A is not symmetric at (%d, %d)", bi, bj);
    }
  }
  if (d->precision == HOPF_F64 && !(diag && n <= kDiagMaxN))
    return say(HOPF_EINVAL, why, len,
               "HOPF_F64 supports diagonal A with n <= %d; use HOPF_F32 or HOPF_BF16_REFINED", kDiagMaxN);
  // the ellipsoid projection (whole-column reductions inside its Newton loop) runs in every kernel
  // of the quadratic J: per-thread (diagonal A), wave-local and tile kernels (dense A)
  // the breakpoint searches run in the per-thread kernel
  if (normsq && (n > kDiagMaxN || d->precision == HOPF_BF16_REFINED))
    return say(HOPF_EINVAL, why, len, "squared-norm J supports n <= %d with HOPF_F64 or HOPF_F32", kDiagMaxN);
  if (d->hkind == HOPF_H_LINF && !(diag && n <= kDiagMaxN && d->precision != HOPF_BF16_REFINED))
    return say(HOPF_EINVAL, why, len,
               "HOPF_H_LINF supports diagonal A or a squared-norm J, n <= %d, HOPF_F64 or HOPF_F32", kDiagMaxN);
  if (normsq && d->hkind == HOPF_H_AL2) return say(HOPF_EINVAL, why, len, "HOPF_H_AL2 needs the quadratic J");
  if (d->hkind == HOPF_H_LINCTRL) {
    // the per-point integrated weights run in the per-thread kernel only
    if (normsq || !diag || n > kDiagMaxN || d->precision == HOPF_BF16_REFINED)
      return say(HOPF_EINVAL, why, len, "HOPF_H_LINCTRL supports the quadratic J with diagonal A, n <= %d, "
                 "HOPF_F64 or HOPF_F32", kDiagMaxN);
    if (!d->drift) return say(HOPF_EINVAL, why, len, "HOPF_H_LINCTRL needs the drift diagonal");
    for (int i = 0; i < n; ++i)
      if (!std::isfinite(d->drift[i])) return say(HOPF_EINVAL, why, len, "drift[%d] is not finite", i);
  }
  if (d->hkind == HOPF_H_AL2) {
    // FP64: the per-thread kernel with diagonal A, the prox rotating into HA's eigenbasis; FP32 and
    // refined: solved in HA's eigenbasis, where A becomes dense, by the dense kernels
    const bool f64_diag = d->precision == HOPF_F64 && diag && n <= kDiagMaxN;
    if (!f64_diag && (d->precision == HOPF_F64 || n > kRotMaxN))
      return say(HOPF_EINVAL, why, len, "HOPF_H_AL2 supports HOPF_F64 with diagonal A and n <= %d, or HOPF_F32 "
                 "and HOPF_BF16_REFINED with n <= %d", kDiagMaxN, kRotMaxN);
    if (!d->HA) return say(HOPF_EINVAL, why, len, "HOPF_H_AL2 needs the matrix HA");
    int64_t bad = -1;
    int bi = 0, bj = 0;
    const int r = check_dense(d->HA, n, &bad, &bi, &bj);
    if (r == 1) return say(HOPF_EINVAL, why, len, "HA[%lld] is not finite", (long long)bad);
    if (r == 2) return say(HOPF_EINVAL, why, len, "HA is not symmetric at (%d, %d)", bi, bj);
  }
  return HOPF_OK;
}

hopf_status check_columns(int64_t npts, int32_t K, char* why, size_t len) {
  if (npts < 0) return say(HOPF_EINVAL, why, len, "npts < 0");
  if (K < 1) return say(HOPF_EINVAL, why, len, "K = %d < 1", K);
  if (npts > kMaxColumns / K)
    return say(HOPF_EINVAL, why, len, "npts * K = %lld * %d exceeds %lld (split the call)", (long long)npts, K,
               (long long)kMaxColumns);
  return HOPF_OK;
}

hopf_status check_ragged_member(int32_t q, int32_t precision, int32_t batch_precision, int32_t hkind, int32_t jkind,
                                int32_t n, char* why, size_t len) {
  if (precision != batch_precision)
    return say(HOPF_EINVAL, why, len, "problem %d: problems of a ragged batch must share one precision", q);
  if (precision == HOPF_F64)
    return say(HOPF_EINVAL, why, len, "problem %d: ragged batches need HOPF_F32 or HOPF_BF16_REFINED", q);
  if (jkind != HOPF_J_QUADRATIC || hkind == HOPF_H_LINF || hkind == HOPF_H_LINCTRL)
    return say(HOPF_EINVAL, why, len,
               "problem %d: squared-norm J, HOPF_H_LINF and HOPF_H_LINCTRL run per point (hopf_eval), not in "
               "ragged batches", q);
  (void)n;  // the ellipsoidal norms run in every dense kernel
  return HOPF_OK;
}

}  // namespace hopf
