// Per-thread Hopf solver for diagonal A: J(y) = 1/2 sum y_i^2 / a_i, so update (3.4a) is
// elementwise, v_i = (x'_i + lambda (d_i - b_i)) / (a_i + lambda); also for the squared-norm
// initial data 1/2 |y|_1^2 and 1/2 |y|_inf^2 (section 4.4), whose update (3.4a) is the prox of the
// squared dual norm, and for H = |p|_inf (section 4.2), both by a breakpoint search.  One thread
// per query point runs the split-Bregman updates (3.4a)-(3.4c) literally, in
// FP64 registers, with the paper's initial values (v0 = d0 = x', b0 = 0) and
// its stopping test (section 4.5: the three squared norms
// |v^k - v^{k-1}|^2, |d^k - d^{k-1}|^2, |d^k - v^k|^2 all <= tol), then takes
// the min over the K translated copies (section 2).  The path is bound by HBM
// traffic: it reads x and t once and writes phi, grad, dphidt once (for sqrt(<p, D p>) the prox
// runs a Newton loop per iteration and the path is bound by FP64 arithmetic instead).
#include <algorithm>
#include <cstdint>

#include "common.hpp"
#include "diag.hpp"

namespace hopf {

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// In place: z <- prox of theta sqrt(<., D .>), D = diag(w) (section 4.3): z minus its projection
// onto the Wulff ellipsoid sum y_i^2 / s_i <= 1, s_i = theta^2 w_i (eq. (prox-projection)).  Zero
// inside; otherwise z_i mu / (s_i + mu) with mu > 0 the root of phi(mu) = sum s_i z_i^2 /
// (s_i + mu)^2 = 1, by Newton on 1 / sqrt(phi) - 1 (concave and increasing: monotone from mu = 0,
// exact in one step when all s_i are equal) until the step is at FP64 rounding level.
template <int NMAX>
__device__ __forceinline__ void wl2_prox(int n, const double* w, double theta, double* z) {
  double q = 0.0;
#pragma unroll
  for (int i = 0; i < NMAX; ++i)
    if (i < n) q += z[i] * z[i] / (theta * theta * w[i]);
  if (!(q > 1.0)) {
#pragma unroll
    for (int i = 0; i < NMAX; ++i) z[i] = 0.0;
    return;
  }
  double mu = 0.0;
  for (int it = 0; it < 100; ++it) {
    double ph = 0.0, ps = 0.0;
#pragma unroll
    for (int i = 0; i < NMAX; ++i) {
      if (i >= n) continue;
      const double s = theta * theta * w[i], inv = 1.0 / (s + mu);
      const double e = s * z[i] * z[i] * inv * inv;
      ph += e;
      ps += e * inv;
    }
    const double step = ph * (sqrt(ph) - 1.0) / ps;
    if (!(step > 1e-15 * mu)) break;
    mu += step;
  }
#pragma unroll
  for (int i = 0; i < NMAX; ++i)
    if (i < n) z[i] = mu * z[i] / (theta * theta * w[i] + mu);
}

// The breakpoint problems of sections 4.2 and 4.4: the root mu of the decreasing, piecewise-affine
// f(mu) = a S(mu) - b mu - c, S(mu) = sum_i (u_i - mu)_+ (u_i = |z_i| >= 0, 0 beyond n), given
// f(0) > 0 > f(max u).  As in the paper, the breakpoints are sorted and searched: u is sorted in
// place, descending, by a bitonic network (all indices static, so nothing leaves registers); then
// S at the k-th largest breakpoint is P_k - k u_(k) with P_k the sum of the k larger ones, and
// since f increases along the descending breakpoints, the first with f >= 0 is the largest such
// one, L.  The root lies in the affine piece after L, whose active set is {i : u_i > L}, so
// a (sum_act u_i - m mu) - b mu - c = 0 gives mu directly.
template <int NMAX>
__device__ __forceinline__ double breakpoint_root(double* u, double a, double b, double c) {
  static_assert((NMAX & (NMAX - 1)) == 0, "the sorting network needs a power of two");
#pragma unroll
  for (int size = 2; size <= NMAX; size <<= 1)
#pragma unroll
    for (int stride = size / 2; stride > 0; stride >>= 1)
#pragma unroll
      for (int i = 0; i < NMAX; ++i) {
        const int l = i ^ stride;
        if (l > i) {
          const double x = u[i], y = u[l];
          const bool desc = (i & size) == 0 || size == NMAX;
          u[i] = desc ? fmax(x, y) : fmin(x, y);
          u[l] = desc ? fmin(x, y) : fmax(x, y);
        }
      }
  double L = 0.0, P = 0.0;
  bool found = false;
#pragma unroll
  for (int k = 0; k < NMAX; ++k) {
    if (!found && u[k] > 0.0 && a * (P - k * u[k]) - b * u[k] - c >= 0.0) { L = u[k]; found = true; }
    P += u[k];
  }
  double sa = 0.0, m = 0.0;
#pragma unroll
  for (int i = 0; i < NMAX; ++i)
    if (u[i] > L) { sa += u[i]; m += 1.0; }
  return (a * sa - c) / (a * m + b);
}

// prox of theta |.|_inf (section 4.2): z - pi(z), pi the projection onto the l1 ball of radius
// theta; 0 inside it, else clamp(z, -mu, mu) with |shrink1(z, mu)|_1 = theta.  In place.
template <int NMAX>
__device__ __forceinline__ void linf_prox(int n, double theta, double* z) {
  double u[NMAX], s1 = 0.0;
#pragma unroll
  for (int i = 0; i < NMAX; ++i) { u[i] = i < n ? fabs(z[i]) : 0.0; s1 += u[i]; }
  if (!(s1 > theta)) {
#pragma unroll
    for (int i = 0; i < NMAX; ++i) z[i] = 0.0;
    return;
  }
  const double mu = breakpoint_root<NMAX>(u, 1.0, 0.0, theta);
#pragma unroll
  for (int i = 0; i < NMAX; ++i) z[i] = fmin(fmax(z[i], -mu), mu);
}

// Update (3.4a) for a squared-norm J: v = prox of J* / lambda at w = d - b + x / lambda (in place).
// J* = 1/2 |.|_1^2 (J = 1/2 |.|_inf^2): shrink1(w, beta), beta = |shrink1(w, beta)|_1 / lambda
// (section 4.4).  J* = 1/2 |.|_inf^2 (J = 1/2 |.|_1^2): by Moreau's identity with the conjugate
// (lambda / 2) |.|_1^2, w - shrink1(w, beta) = clamp(w, -beta, beta), beta = lambda |shrink1(w, beta)|_1.
template <int NMAX>
__device__ __forceinline__ void normsq_vupdate(int n, int jkind, double lam, double* w) {
  double u[NMAX], s1 = 0.0;
#pragma unroll
  for (int i = 0; i < NMAX; ++i) { u[i] = i < n ? fabs(w[i]) : 0.0; s1 += u[i]; }
  if (!(s1 > 0.0)) return;  // w = 0: the prox is 0
  const double a = jkind == JK_LINFSQ ? 1.0 / lam : lam;
  const double beta = breakpoint_root<NMAX>(u, a, 1.0, 0.0);
#pragma unroll
  for (int i = 0; i < NMAX; ++i) {
    const double c = fmin(fmax(w[i], -beta), beta);
    w[i] = jkind == JK_LINFSQ ? w[i] - c : c;
  }
}

// A coefficient of the problem (the same for every thread), read once into scalar registers.  Read
// inside the iteration loops, such loads sit under per-coordinate branches and are not hoisted, so
// every iteration would wait for their latency.
__device__ __forceinline__ double uniform(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// The diagonal of M = (A + lambda I)^{-1} and the weights (1 without weights), coordinates >= n
// taking coordinate 0's values (never used).  Up to 16 coordinates they are held in (scalar)
// registers; beyond, registers are short and they stay in memory (cm, cw then point there).
constexpr int kCoefRegs = 16;
__constant__ double kOnes[32] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1,
                                 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
template <int NMAX>
struct DiagCoef {
  double m[NMAX <= kCoefRegs ? NMAX : 1], w[NMAX <= kCoefRegs ? NMAX : 1];
  const double* cm;
  const double* cw;
  __device__ __forceinline__ explicit DiagCoef(const DiagProb& pb) {
    if constexpr (NMAX <= kCoefRegs) {
      // all loads issued before any is used (unconditional, in-bounds indices), then moved to
      // scalar registers
      const double* pm = pb.minv ? pb.minv : kOnes;
      const double* pw = pb.w ? pb.w : kOnes;
      double tm[NMAX], tw[NMAX];
#pragma unroll
      for (int i = 0; i < NMAX; ++i) {
        const int ic = i < pb.n ? i : 0;
        tm[i] = pm[ic];
        tw[i] = pw[ic];
      }
#pragma unroll
      for (int i = 0; i < NMAX; ++i) {
        m[i] = uniform(tm[i]);
        w[i] = uniform(tw[i]);
      }
      cm = m;
      cw = w;
    } else {
      cm = pb.minv;
      cw = pb.w ? pb.w : kOnes;
    }
  }
};

// For the persistent kernel below: one split-Bregman iteration (3.4a)-(3.4c) of one point and
// copy, in place, for every kind of J and H of the per-thread path; returns the paper's stopping
// test (section 4.5).
template <int NMAX>
__device__ __forceinline__ bool sb_step(const DiagProb& pb, const double* cm, const double* cw, double th,
                                        const double* xp, double* v, double* d, double* b) {
  const int n = pb.n;
  const double lam = pb.lambda;
  const bool l1 = hk_has_l1(pb.hkind), l2 = hk_has_l2(pb.hkind), wl2 = pb.hkind == HK_WL2;
  double vn[NMAX], dn[NMAX];
  double ss = 0.0;
  if (pb.jkind == JK_QUAD) {
#pragma unroll
    for (int i = 0; i < NMAX; ++i)
      vn[i] = i < n ? cm[i] * (xp[i] + lam * (d[i] - b[i])) : 0.0;  // (3.4a)
  } else {
#pragma unroll
    for (int i = 0; i < NMAX; ++i) vn[i] = i < n ? d[i] - b[i] + xp[i] / lam : 0.0;
    normsq_vupdate<NMAX>(n, pb.jkind, lam, vn);                         // (3.4a), squared norm
  }
#pragma unroll
  for (int i = 0; i < NMAX; ++i) {
    if (i >= n) { dn[i] = 0.0; continue; }
    double z = vn[i] + b[i];
    double s = z;
    if (l1) {                                                 // (3.4b), shrink1
      double a = th * cw[i];
      double m = fabs(z) - a;
      s = m > 0.0 ? (z >= 0.0 ? m : -m) : 0.0;
    }
    dn[i] = s;
    ss += s * s;
  }
  if (l2) {                                                   // (3.4b), shrink2
    double nr = sqrt(ss);
    double f = nr > 0.0 ? fmax(nr - th, 0.0) / nr : 0.0;
#pragma unroll
    for (int i = 0; i < NMAX; ++i) dn[i] *= f;
  }
  if (wl2) wl2_prox<NMAX>(n, cw, th, dn);  // (3.4b), z - projection
  if (pb.hkind == HK_LINF) linf_prox<NMAX>(n, th, dn);       // (3.4b), z - l1-ball projection
  double r1 = 0.0, r2 = 0.0, r3 = 0.0;
#pragma unroll
  for (int i = 0; i < NMAX; ++i) {
    if (i >= n) continue;
    b[i] = b[i] + vn[i] - dn[i];                              // (3.4c)
    r1 += (vn[i] - v[i]) * (vn[i] - v[i]);
    r2 += (dn[i] - d[i]) * (dn[i] - d[i]);
    r3 += (dn[i] - vn[i]) * (dn[i] - vn[i]);
    v[i] = vn[i]; d[i] = dn[i];
  }
  return r1 <= pb.tol && r2 <= pb.tol && r3 <= pb.tol;
}

// phi_k = <x', d> - J*(d) - t H(d)  (- 1/2 for an ellipsoid level set); J*(d) = 1/2 sum a_i d_i^2,
// or the squared dual norm for the squared-norm initial data.  *H receives H(d).
template <int NMAX>
__device__ __forceinline__ double copy_value(const DiagProb& pb, const double* cw, double t, const double* xp,
                                             const double* d, double* Hout) {
  const int n = pb.n;
  const bool l1 = hk_has_l1(pb.hkind), l2 = hk_has_l2(pb.hkind), wl2 = pb.hkind == HK_WL2;
  const bool quad = pb.jkind == JK_QUAD;
  double xd = 0.0, q = 0.0, h1 = 0.0, h2 = 0.0, dmax = 0.0, dsum = 0.0;
  double av[NMAX <= kCoefRegs ? NMAX : 1];  // diagonal of A: all loads in flight together
  if constexpr (NMAX <= kCoefRegs) {
#pragma unroll
    for (int i = 0; i < NMAX; ++i) av[i] = quad ? pb.adiag[i < n ? i : 0] : 0.0;
  }
#pragma unroll
  for (int i = 0; i < NMAX; ++i) {
    if (i >= n) continue;
    xd += xp[i] * d[i];
    double ai;
    if constexpr (NMAX <= kCoefRegs) ai = av[i];
    else ai = quad ? pb.adiag[i] : 0.0;
    if (quad) q += ai * d[i] * d[i];
    const double wi = cw[i];
    h1 += wl2 ? wi * d[i] * d[i] : wi * fabs(d[i]);
    h2 += d[i] * d[i];
    dmax = fmax(dmax, fabs(d[i]));
    dsum += fabs(d[i]);
  }
  if (!quad) q = pb.jkind == JK_L1SQ ? dmax * dmax : dsum * dsum;
  const double H = pb.hkind == HK_LINF ? dmax : wl2 ? sqrt(h1) : (l1 ? h1 : 0.0) + (l2 ? sqrt(h2) : 0.0);
  *Hout = H;
  return xd - 0.5 * q - t * H - (pb.level_set ? 0.5 : 0.0);
}

template <int NMAX>
__device__ __forceinline__ void init_copy(const DiagProb& pb, const double* x, int k, double* xp, double* v,
                                          double* d, double* b) {
#pragma unroll
  for (int i = 0; i < NMAX; ++i) {
    xp[i] = (i < pb.n) ? x[i] - (pb.centres ? pb.centres[(size_t)k * pb.ld + i] : 0.0) : 0.0;
    v[i] = xp[i]; d[i] = xp[i]; b[i] = 0.0;
  }
}

// loads point j; false (and NaN outputs, iters = kstar = -1) for t <= 0 or non-finite input
template <typename T, int NMAX>
__device__ __forceinline__ bool load_point(const DiagProb& pb, int64_t j, double* x, double* t) {
  const int n = pb.n;
  const T* xj = (const T*)pb.x + j * n;
  *t = (double)((const T*)pb.t)[j];
  bool ok = *t > 0.0 && isfinite(*t);
#pragma unroll
  for (int i = 0; i < NMAX; ++i) x[i] = (double)xj[i < n ? i : 0];  // all loads in flight together
#pragma unroll
  for (int i = 0; i < NMAX; ++i) {
    if (i < n && !isfinite(x[i])) ok = false;
    x[i] = i < n ? x[i] : 0.0;
  }
  if (!ok) {
    const T qn = (T)__builtin_nan("");
    T* gj = (T*)pb.grad + j * n;
    ((T*)pb.phi)[j] = qn; ((T*)pb.dphidt)[j] = qn;
    for (int i = 0; i < n; ++i) gj[i] = qn;
    if (pb.iters) pb.iters[j] = -1;
    if (pb.kstar) pb.kstar[j] = -1;
  }
  return ok;
}

template <typename T, int NMAX>
__device__ __forceinline__ void store_point(const DiagProb& pb, int64_t j, double best, double bh, int kbest,
                                            int itbest, const double* pbest) {
  T* gj = (T*)pb.grad + j * pb.n;
  ((T*)pb.phi)[j] = (T)best;
  ((T*)pb.dphidt)[j] = (T)(-bh);
  for (int i = 0; i < pb.n; ++i) gj[i] = (T)pbest[i];
  if (pb.iters) pb.iters[j] = itbest;
  if (pb.kstar) pb.kstar[j] = kbest;
}

// One thread per point (the iteration counts of this family are short and uniform): the quadratic
// diagonal J with the weighted l1 / l2 norms, or (WL2) the ellipsoidal norm, whose projection is
// compiled only into that instance (it would otherwise hold registers, and so occupancy, from the
// memory-bound norms).  ONE: a single copy without a centre (the plain J), where the point's own
// x is the iteration's x' and p is written from the final iterate.
// ROT (with WL2): H = sqrt(<p, HA p>), the paper's |.|_A case of section 4.3, in the caller's
// basis: the prox rotates z into HA's eigenbasis (HA = P diag(sig) P^T; the weights are sig),
// projects there onto the diagonal ellipsoid and rotates back, P staged in LDS.
// LC: the time-dependent Hamiltonian of linear controls (section 2.2, extensions) with
// M = diag(drift), N = diag(w) and box controls, H(p, s) = sum_i e^{-s m_i} w_i |p_i|: the Hopf
// formula takes its integral over [0, t], sum_i W_i |p_i| with W_i = w_i (1 - e^{-t m_i}) / m_i,
// so a point is the weighted-l1 problem with the per-point weights W_i / t (thresholds W_i /
// lambda); dphi/dt = -H(p, t), the integrand at s = t.
template <typename T, int NMAX, bool WL2, bool ONE, bool ROT = false, bool LC = false>
__global__ void __launch_bounds__(kBlock) diag_kernel(DiagProb pb) {
  __shared__ double sP[ROT ? NMAX * NMAX : 1];
  if constexpr (ROT) {
    for (int e = threadIdx.x; e < pb.n * pb.n; e += blockDim.x) sP[e] = pb.P[e];
    __syncthreads();
  }
  // grid-stride over the points (loading the next point before solving the current one was
  // measured slower: the extra registers cost a wave per SIMD)
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int n = pb.n;
  const double lam = pb.lambda;
  const bool l1 = LC || (!WL2 && hk_has_l1(pb.hkind)), l2 = !LC && !WL2 && hk_has_l2(pb.hkind);
  constexpr bool wl2 = WL2;
  const DiagCoef<NMAX> coef(pb);
  const double* const cm = coef.cm;
  const double* const cw = coef.cw;
  T xs[NMAX], ts = (T)0;  // the loaded point (all loads in flight together)
  // rows of exactly NMAX values, 16-byte aligned: moved as 16-byte vectors (half or a quarter of
  // the memory instructions of element-wise accesses)
  constexpr int VW = 16 / (int)sizeof(T);  // values per 16-byte vector
  constexpr bool VEC = NMAX <= 16 && NMAX % VW == 0;  // (registers are short above 16)
  const bool vec = VEC && n == NMAX && ((uintptr_t)pb.x % 16) == 0 && ((uintptr_t)pb.grad % 16) == 0;
  auto issue = [&](int64_t jj) {
    const T* xj = (const T*)pb.x + jj * n;
    if (VEC && vec) {
#pragma unroll
      for (int q = 0; q < NMAX / VW; ++q) {
        const u32x4 w = ((const u32x4*)xj)[q];
        __builtin_memcpy(&xs[q * VW], &w, 16);
      }
    } else {
#pragma unroll
      for (int i = 0; i < NMAX; ++i) xs[i] = xj[i < n ? i : 0];
    }
    ts = ((const T*)pb.t)[jj];
  };
  auto store_row = [&](T* gj, const double* p) {
    if (VEC && vec) {
#pragma unroll
      for (int q = 0; q < NMAX / VW; ++q) {
        T v[VW];
#pragma unroll
        for (int e = 0; e < VW; ++e) v[e] = (T)p[q * VW + e];
        u32x4 w;
        __builtin_memcpy(&w, v, 16);
        ((u32x4*)gj)[q] = w;
      }
    } else {
      for (int i = 0; i < n; ++i) gj[i] = (T)p[i];
    }
  };
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < pb.npts; j += stride) {
    issue(j);
    double x[NMAX];
#pragma unroll
    for (int i = 0; i < NMAX; ++i) x[i] = (double)xs[i];
    const double t = (double)ts;
    bool ok = t > 0.0 && isfinite(t);
#pragma unroll
    for (int i = 0; i < NMAX; ++i) {
      if (i < n && !isfinite(x[i])) ok = false;
      x[i] = i < n ? x[i] : 0.0;
    }
    T* gj = (T*)pb.grad + j * n;
    if (!ok) {
      const T qn = (T)__builtin_nan("");
      ((T*)pb.phi)[j] = qn; ((T*)pb.dphidt)[j] = qn;
      for (int i = 0; i < n; ++i) gj[i] = qn;
      if (pb.iters) pb.iters[j] = -1;
      if (pb.kstar) pb.kstar[j] = -1;
      continue;
    }
    const double th = t / lam;
    // LC: the weights of the integrated Hamiltonian divided by t, lw_i = w_i (1 - e^{-x}) / x with
    // x = t m_i (1 at x = 0; expm1 keeps it accurate for small x)
    double lw[LC ? NMAX : 1];
    if constexpr (LC) {
      double dm[NMAX];
#pragma unroll
      for (int i = 0; i < NMAX; ++i) dm[i] = pb.drift[i < n ? i : 0];
#pragma unroll
      for (int i = 0; i < NMAX; ++i) {
        const double xm = t * dm[i];
        lw[i] = i < n ? cw[i] * (xm != 0.0 ? -expm1(-xm) / xm : 1.0) : 0.0;
      }
    }
    double best = 0.0, bh = 0.0;
    int kbest = -1, itbest = 0;
    double pbest[NMAX];
    for (int k = 0; k < (ONE ? 1 : pb.K); ++k) {
      double xp[NMAX], v[NMAX], d[NMAX], b[NMAX];
#pragma unroll
      for (int i = 0; i < NMAX; ++i) {
        xp[i] = (i < n) ? x[i] - (!ONE && pb.centres ? pb.centres[(size_t)k * pb.ld + i] : 0.0) : 0.0;
        v[i] = xp[i]; d[i] = xp[i]; b[i] = 0.0;
      }
      int it = 0;
      bool conv = false;
      while (it < pb.max_iter) {
        ++it;
        double vn[NMAX], dn[NMAX];
        double ss = 0.0;
#pragma unroll
        for (int i = 0; i < NMAX; ++i) {
          if (i >= n) { vn[i] = 0.0; dn[i] = 0.0; continue; }
          vn[i] = cm[i] * (xp[i] + lam * (d[i] - b[i]));        // (3.4a)
          double z = vn[i] + b[i];
          double s = z;
          if (l1) {                                                 // (3.4b), shrink1
            double a = th * (LC ? lw[i] : cw[i]);
            double m = fabs(z) - a;
            s = m > 0.0 ? (z >= 0.0 ? m : -m) : 0.0;
          }
          dn[i] = s;
          ss += s * s;
        }
        if (l2) {                                                   // (3.4b), shrink2
          double nr = sqrt(ss);
          double f = nr > 0.0 ? fmax(nr - th, 0.0) / nr : 0.0;
#pragma unroll
          for (int i = 0; i < NMAX; ++i) dn[i] *= f;
        }
        if constexpr (WL2 && !ROT) wl2_prox<NMAX>(n, cw, th, dn);  // (3.4b), z - projection
        if constexpr (ROT) {  // (3.4b) in HA's eigenbasis: P prox(P^T z)
          double zr[NMAX];
#pragma unroll
          for (int a = 0; a < NMAX; ++a) zr[a] = 0.0;
#pragma unroll
          for (int i = 0; i < NMAX; ++i) {  // static indices: the vectors stay in registers
            if (i >= n) continue;
#pragma unroll
            for (int a = 0; a < NMAX; ++a)
              if (a < n) zr[a] += sP[i * n + a] * dn[i];
          }
          wl2_prox<NMAX>(n, cw, th, zr);
#pragma unroll
          for (int i = 0; i < NMAX; ++i) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < NMAX; ++a)
              if (a < n) s += sP[i * n + a] * zr[a];
            dn[i] = i < n ? s : 0.0;
          }
        }
        double r1 = 0.0, r2 = 0.0, r3 = 0.0;
#pragma unroll
        for (int i = 0; i < NMAX; ++i) {
          if (i >= n) continue;
          b[i] = b[i] + vn[i] - dn[i];                              // (3.4c)
          r1 += (vn[i] - v[i]) * (vn[i] - v[i]);
          r2 += (dn[i] - d[i]) * (dn[i] - d[i]);
          r3 += (dn[i] - vn[i]) * (dn[i] - vn[i]);
          v[i] = vn[i]; d[i] = dn[i];
        }
        if (r1 <= pb.tol && r2 <= pb.tol && r3 <= pb.tol) { conv = true; break; }
      }
      // phi_k = <x', d> - 1/2 sum a_i d_i^2 - t H(d)  (- 1/2 for an ellipsoid level set)
      double xd = 0.0, q = 0.0, h1 = 0.0, h2 = 0.0, hnow = 0.0;
      double av[NMAX <= kCoefRegs ? NMAX : 1];  // diagonal of A: all loads in flight together
      if constexpr (NMAX <= kCoefRegs) {
#pragma unroll
        for (int i = 0; i < NMAX; ++i) av[i] = pb.adiag[i < n ? i : 0];
      }
#pragma unroll
      for (int i = 0; i < NMAX; ++i) {
        if (i >= n) continue;
        xd += xp[i] * d[i];
        double ai;
        if constexpr (NMAX <= kCoefRegs) ai = av[i];
        else ai = pb.adiag[i];
        q += ai * d[i] * d[i];
        const double wi = LC ? lw[i] : cw[i];
        if constexpr (LC) hnow += cw[i] * exp(-t * pb.drift[i]) * fabs(d[i]);  // H(d, t)
        if constexpr (ROT) {  // <d, HA d> = sum_a sig_a (P^T d)_a^2
          double s = 0.0;
#pragma unroll
          for (int k2 = 0; k2 < NMAX; ++k2)
            if (k2 < n) s += sP[k2 * n + i] * d[k2];
          h1 += wi * s * s;
        } else {
          h1 += wl2 ? wi * d[i] * d[i] : wi * fabs(d[i]);
        }
        h2 += d[i] * d[i];
      }
      const double H = wl2 ? sqrt(h1) : (l1 ? h1 : 0.0) + (l2 ? sqrt(h2) : 0.0);
      const double val = xd - 0.5 * q - t * H - (pb.level_set ? 0.5 : 0.0);
      if (kbest < 0 || val < best) {
        best = val; bh = LC ? hnow : H; kbest = k; itbest = conv ? it : -2;
        if constexpr (!ONE) {
#pragma unroll
          for (int i = 0; i < NMAX; ++i) pbest[i] = d[i];
        }
      }
      if constexpr (ONE) store_row(gj, d);
    }
    ((T*)pb.phi)[j] = (T)best;
    ((T*)pb.dphidt)[j] = (T)(-bh);
    if constexpr (!ONE) store_row(gj, pbest);
    if (pb.iters) pb.iters[j] = itbest;
    if (pb.kstar) pb.kstar[j] = kbest;
  }
}

// The squared-norm initial data and H = |.|_inf: iteration counts vary over orders of magnitude
// between points (the paper's ADMM is slow for these nonsmooth pairs), so one point per thread
// would keep a whole wave waiting for its slowest lane.  Here every lane runs its own state
// machine: each pass is one iteration of the lane's current (point, copy); a lane that finishes
// a copy evaluates it, moves to the next copy or writes the point and takes the next one from a
// global counter, without waiting for the rest of its wave.  The grid is persistent.
template <typename T, int NMAX>
__global__ void __launch_bounds__(kBlock) diag_ext_kernel(DiagProb pb, int* __restrict__ counter) {
  double x[NMAX], xp[NMAX], v[NMAX], d[NMAX], b[NMAX], pbest[NMAX];
  const DiagCoef<NMAX> coef(pb);
  const double* const cm = coef.cm;
  const double* const cw = coef.cw;
  double t = 0.0, th = 0.0, best = 0.0, bh = 0.0;
  int64_t j = -1;
  int k = 0, it = 0, kbest = -1, itbest = 0;
  bool have = false;
  auto fetch = [&]() {  // next valid point, or have = false
    while (true) {
      j = (int64_t)atomicAdd((unsigned int*)counter, 1u);  // unsigned: the overshoot past npts cannot wrap
      if (j >= pb.npts) { have = false; return; }
      if (load_point<T, NMAX>(pb, j, x, &t)) break;
    }
    have = true;
    th = t / pb.lambda;
    k = 0; it = 0; kbest = -1; itbest = 0; best = 0.0; bh = 0.0;
    init_copy<NMAX>(pb, x, 0, xp, v, d, b);
  };
  fetch();
  while (have) {
    ++it;
    const bool conv = sb_step<NMAX>(pb, cm, cw, th, xp, v, d, b);
    if (conv || it >= pb.max_iter) {
      double H;
      const double val = copy_value<NMAX>(pb, cw, t, xp, d, &H);
      if (kbest < 0 || val < best) {
        best = val; bh = H; kbest = k; itbest = conv ? it : -2;
#pragma unroll
        for (int i = 0; i < NMAX; ++i) pbest[i] = d[i];
      }
      if (++k < pb.K) {
        it = 0;
        init_copy<NMAX>(pb, x, k, xp, v, d, b);
      } else {
        store_point<T, NMAX>(pb, j, best, bh, kbest, itbest, pbest);
        fetch();
      }
    }
  }
}

template <typename T, int NMAX>
static hipError_t launch_n(const DiagProb& pb, bool ext, int* counter, int ncu, hipStream_t stream) {
  if (!ext) {
    // grid-stride: at most 8 workgroups per CU (the kernel's occupancy is lower), each thread then
    // takes several points
    const int64_t need = (pb.npts + kBlock - 1) / kBlock;
    const unsigned grid = (unsigned)std::min<int64_t>(need, (int64_t)8 * ncu);
    if (pb.hkind == HK_AL2)
      hipLaunchKernelGGL((diag_kernel<T, NMAX, true, false, true>), dim3(grid), dim3(kBlock), 0, stream, pb);
    else if (pb.hkind == HK_LINCTRL)
      hipLaunchKernelGGL((diag_kernel<T, NMAX, false, false, false, true>), dim3(grid), dim3(kBlock), 0, stream, pb);
    else if (pb.hkind == HK_WL2)
      hipLaunchKernelGGL((diag_kernel<T, NMAX, true, false>), dim3(grid), dim3(kBlock), 0, stream, pb);
    else if (pb.K == 1 && pb.centres == nullptr)
      hipLaunchKernelGGL((diag_kernel<T, NMAX, false, true>), dim3(grid), dim3(kBlock), 0, stream, pb);
    else
      hipLaunchKernelGGL((diag_kernel<T, NMAX, false, false>), dim3(grid), dim3(kBlock), 0, stream, pb);
  } else {
    // persistent: enough workgroups for the resident waves (at most 8 workgroups per CU)
    const int64_t need = (pb.npts + kBlock - 1) / kBlock;
    const unsigned grid = (unsigned)std::min<int64_t>(need, (int64_t)8 * ncu);
    hipError_t e = hipMemsetAsync(counter, 0, sizeof(int), stream);
    if (e) return e;
    hipLaunchKernelGGL((diag_ext_kernel<T, NMAX>), dim3(grid), dim3(kBlock), 0, stream, pb, counter);
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_t(const DiagProb& pb, bool ext, int* counter, int ncu, hipStream_t stream) {
  if (pb.n <= 8) return launch_n<T, 8>(pb, ext, counter, ncu, stream);
  if (pb.n <= 16) return launch_n<T, 16>(pb, ext, counter, ncu, stream);
  if (pb.n <= 32) return launch_n<T, 32>(pb, ext, counter, ncu, stream);
  return hipErrorInvalidValue;
}

hipError_t launch_diag(const DiagProb& pb, bool f64, int* counter, int ncu, hipStream_t stream) {
  if (pb.npts == 0) return hipSuccess;
  const bool ext = pb.jkind != JK_QUAD || pb.hkind == HK_LINF;
  if (ext && (!counter || pb.npts > INT32_MAX)) return hipErrorInvalidValue;
  if (pb.hkind == HK_AL2 && (!pb.P || ext)) return hipErrorInvalidValue;
  if (pb.hkind == HK_LINCTRL && (!pb.drift || ext)) return hipErrorInvalidValue;
  return f64 ? launch_t<double>(pb, ext, counter, ncu, stream) : launch_t<float>(pb, ext, counter, ncu, stream);
}

}  // namespace hopf
