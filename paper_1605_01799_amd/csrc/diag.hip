// Diagonal-A Hopf solver: J(y) = 1/2 sum y_i^2 / a_i, so update (3.4a) is
// elementwise, v_i = (x'_i + lambda (d_i - b_i)) / (a_i + lambda).  One thread
// per query point runs the split-Bregman updates (3.4a)-(3.4c) literally, in
// FP64 registers, with the paper's initial values (v0 = d0 = x', b0 = 0) and
// its stopping test (section 4.5: the three squared norms
// |v^k - v^{k-1}|^2, |d^k - d^{k-1}|^2, |d^k - v^k|^2 all <= tol), then takes
// the min over the K translated copies (section 2).  The path is bound by HBM
// traffic: it reads x and t once and writes phi, grad, dphidt once (for sqrt(<p, D p>) the prox
// runs a Newton loop per iteration and the path is bound by FP64 arithmetic instead).
#include "common.hpp"
#include "diag.hpp"

namespace hopf {

// In place: z <- prox of theta sqrt(<., D .>), D = diag(w) (section 4.4): z minus its projection
// onto the Wulff ellipsoid sum y_i^2 / s_i <= 1, s_i = theta^2 w_i (eq. (prox-projection)).  Zero
// inside; otherwise z_i mu / (s_i + mu) with mu > 0 the root of phi(mu) = sum s_i z_i^2 /
// (s_i + mu)^2 = 1, by Newton on 1 / sqrt(phi) - 1 (concave and increasing: monotone from mu = 0,
// exact in one step when all s_i are equal) until the step is at FP64 rounding level.
template <int NMAX>
__device__ __forceinline__ void wl2_prox(int n, const double* w, double theta, double* z) {
  double q = 0.0;
#pragma unroll
  for (int i = 0; i < NMAX; ++i)
    if (i < n) q += z[i] * z[i] / (theta * theta * (w ? w[i] : 1.0));
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
      const double s = theta * theta * (w ? w[i] : 1.0), inv = 1.0 / (s + mu);
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
    if (i < n) z[i] = mu * z[i] / (theta * theta * (w ? w[i] : 1.0) + mu);
}

template <typename T, int NMAX>
__global__ void __launch_bounds__(kBlock) diag_kernel(DiagProb pb) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= pb.npts) return;
  const int n = pb.n;
  const double lam = pb.lambda;
  const T* xj = (const T*)pb.x + j * n;
  const double t = (double)((const T*)pb.t)[j];
  double x[NMAX];
  bool ok = t > 0.0 && isfinite(t);
#pragma unroll
  for (int i = 0; i < NMAX; ++i) {
    x[i] = i < n ? (double)xj[i] : 0.0;
    if (i < n && !isfinite(x[i])) ok = false;
  }
  T* gj = (T*)pb.grad + j * n;
  if (!ok) {
    const T qn = (T)__builtin_nan("");
    ((T*)pb.phi)[j] = qn; ((T*)pb.dphidt)[j] = qn;
    for (int i = 0; i < n; ++i) gj[i] = qn;
    if (pb.iters) pb.iters[j] = -1;
    if (pb.kstar) pb.kstar[j] = -1;
    return;
  }
  const bool l1 = hk_has_l1(pb.hkind), l2 = hk_has_l2(pb.hkind), wl2 = pb.hkind == HK_WL2;
  const double th = t / lam;
  double best = 0.0, bh = 0.0;
  int kbest = -1, itbest = 0;
  double pbest[NMAX];
  for (int k = 0; k < pb.K; ++k) {
    double xp[NMAX], v[NMAX], d[NMAX], b[NMAX];
#pragma unroll
    for (int i = 0; i < NMAX; ++i) {
      xp[i] = (i < n) ? x[i] - (pb.centres ? pb.centres[(size_t)k * pb.ld + i] : 0.0) : 0.0;
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
        vn[i] = pb.minv[i] * (xp[i] + lam * (d[i] - b[i]));       // (3.4a)
        double z = vn[i] + b[i];
        double s = z;
        if (l1) {                                                 // (3.4b), shrink1
          double a = th * (pb.w ? pb.w[i] : 1.0);
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
      if (wl2) wl2_prox<NMAX>(n, pb.w, th, dn);                  // (3.4b), z - projection
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
    double xd = 0.0, q = 0.0, h1 = 0.0, h2 = 0.0;
#pragma unroll
    for (int i = 0; i < NMAX; ++i) {
      if (i >= n) continue;
      xd += xp[i] * d[i];
      q += pb.adiag[i] * d[i] * d[i];
      const double wi = pb.w ? pb.w[i] : 1.0;
      h1 += wl2 ? wi * d[i] * d[i] : wi * fabs(d[i]);
      h2 += d[i] * d[i];
    }
    const double H = wl2 ? sqrt(h1) : (l1 ? h1 : 0.0) + (l2 ? sqrt(h2) : 0.0);
    const double val = xd - 0.5 * q - t * H - (pb.level_set ? 0.5 : 0.0);
    if (kbest < 0 || val < best) {
      best = val; bh = H; kbest = k; itbest = conv ? it : -2;
#pragma unroll
      for (int i = 0; i < NMAX; ++i) pbest[i] = d[i];
    }
  }
  ((T*)pb.phi)[j] = (T)best;
  ((T*)pb.dphidt)[j] = (T)(-bh);
  for (int i = 0; i < n; ++i) gj[i] = (T)pbest[i];
  if (pb.iters) pb.iters[j] = itbest;
  if (pb.kstar) pb.kstar[j] = kbest;
}

template <typename T>
static hipError_t launch_t(const DiagProb& pb, hipStream_t stream) {
  const unsigned grid = (unsigned)((pb.npts + kBlock - 1) / kBlock);
  if (pb.n <= 8) hipLaunchKernelGGL((diag_kernel<T, 8>), dim3(grid), dim3(kBlock), 0, stream, pb);
  else if (pb.n <= 16) hipLaunchKernelGGL((diag_kernel<T, 16>), dim3(grid), dim3(kBlock), 0, stream, pb);
  else if (pb.n <= 32) hipLaunchKernelGGL((diag_kernel<T, 32>), dim3(grid), dim3(kBlock), 0, stream, pb);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_diag(const DiagProb& pb, bool f64, hipStream_t stream) {
  if (pb.npts == 0) return hipSuccess;
  return f64 ? launch_t<double>(pb, stream) : launch_t<float>(pb, stream);
}

}  // namespace hopf
