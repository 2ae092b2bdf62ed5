/*
 * Plain FP64 CPU oracle for Darbon & Osher, arXiv:1605.01799.
 *
 * TEST INFRASTRUCTURE ONLY (see hopf_oracle.h).  It is deliberately slow and
 * literal: one point at a time, dense triangular solves, the split-Bregman
 * updates in the order the paper gives them, Neumaier-compensated sums.
 */
#include "hopf_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Compensated summation (Neumaier).                                          */
/* ------------------------------------------------------------------------- */
typedef struct { double s, c; } ksum;
static void ks_add(ksum* k, double v) {
  double t = k->s + v;
  if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
  else k->c += (v - t) + k->s;
  k->s = t;
}
static double ks_val(const ksum* k) { return k->s + k->c; }

static double dot(int n, const double* a, const double* b) {
  ksum k = {0, 0};
  for (int i = 0; i < n; ++i) ks_add(&k, a[i] * b[i]);
  return ks_val(&k);
}
static double sqdist(int n, const double* a, const double* b) {
  ksum k = {0, 0};
  for (int i = 0; i < n; ++i) { double d = a[i] - b[i]; ks_add(&k, d * d); }
  return ks_val(&k);
}

/* ------------------------------------------------------------------------- */
/* Dense SPD factorisation and solves (used for the quadratic prox, which is  */
/* the resolvent (I + alpha A)^{-1} of section 4.1; here in the form          */
/* (A + lambda I)^{-1} that update (3.4a) needs).                             */
/* ------------------------------------------------------------------------- */
/* Cholesky of S = A + shift*I into lower-triangular L (row-major).  Returns -2 if not SPD. */
static int cholesky(int n, const double* A, double shift, double* L) {
  memset(L, 0, sizeof(double) * (size_t)n * n);
  for (int j = 0; j < n; ++j) {
    ksum k = {0, 0};
    ks_add(&k, A[(size_t)j * n + j] + shift);
    for (int m = 0; m < j; ++m) ks_add(&k, -L[(size_t)j * n + m] * L[(size_t)j * n + m]);
    double djj = ks_val(&k);
    if (!(djj > 0.0)) return -2;
    double ljj = sqrt(djj);
    L[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      ksum q = {0, 0};
      ks_add(&q, A[(size_t)i * n + j]);
      for (int m = 0; m < j; ++m) ks_add(&q, -L[(size_t)i * n + m] * L[(size_t)j * n + m]);
      L[(size_t)i * n + j] = ks_val(&q) / ljj;
    }
  }
  return 0;
}
/* Solve L L^T out = rhs. */
static void chol_solve(int n, const double* L, const double* rhs, double* tmp, double* out) {
  for (int i = 0; i < n; ++i) {
    ksum k = {0, 0};
    ks_add(&k, rhs[i]);
    for (int m = 0; m < i; ++m) ks_add(&k, -L[(size_t)i * n + m] * tmp[m]);
    tmp[i] = ks_val(&k) / L[(size_t)i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    ksum k = {0, 0};
    ks_add(&k, tmp[i]);
    for (int m = i + 1; m < n; ++m) ks_add(&k, -L[(size_t)m * n + i] * out[m]);
    out[i] = ks_val(&k) / L[(size_t)i * n + i];
  }
}
/* p^T A p */
static double quad(int n, const double* A, const double* p) {
  ksum k = {0, 0};
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) ks_add(&k, p[i] * A[(size_t)i * n + j] * p[j]);
  return ks_val(&k);
}

/* ------------------------------------------------------------------------- */
/* Hamiltonians and their proximal maps.                                      */
/* ------------------------------------------------------------------------- */
static double wgt(const double* w, int i) { return w ? w[i] : 1.0; }

/* Soft thresholding, eq. (shrink1_def) / section 4.1: sign(z)max(|z|-a,0), sign(0)=1. */
static double shrink1(double z, double a) {
  double m = fabs(z) - a;
  if (m <= 0.0) return 0.0;
  return z >= 0.0 ? m : -m;
}

/* H(p) for the supported family (support functions of a box, a ball, their Minkowski sum, and
 * of the ellipsoid sum y_i^2 / w_i <= 1: the norm sqrt(<p, D p>) with D = diag(w), section 4.3). */
static double ham(const oh_problem* pb, int hkind, const double* p) {
  const int n = pb->n;
  const double* w = pb->w;
  if (hkind == OH_AL2) return sqrt(quad(n, pb->HA, p)); /* sqrt(<p, HA p>) */
  if (hkind == OH_LINF) {
    double m = 0.0;
    for (int i = 0; i < n; ++i) m = fabs(p[i]) > m ? fabs(p[i]) : m;
    return m;
  }
  if (hkind == OH_WL2) {
    ksum k = {0, 0};
    for (int i = 0; i < n; ++i) ks_add(&k, wgt(w, i) * p[i] * p[i]);
    return sqrt(ks_val(&k));
  }
  double h = 0.0;
  if (hkind == OH_WL1 || hkind == OH_L2_WL1) {
    ksum k = {0, 0};
    for (int i = 0; i < n; ++i) ks_add(&k, wgt(w, i) * fabs(p[i]));
    h += ks_val(&k);
  }
  if (hkind == OH_L2 || hkind == OH_L2_WL1) h += sqrt(dot(n, p, p));
  return h;
}

/* d = argmin_d { theta*H(d) + 1/2 ||d - z||^2 }, i.e. update (3.4b) with theta = t/lambda.
 * WL1: componentwise shrink1 with thresholds theta*w_i (eq. shrink1_def).
 * L2:  shrink2(z, theta) (eq. shrink2_def).
 * L2 + WL1: shrink2(shrink1(z, theta*w), theta), the composition of the two maps
 * (the prox of a sum of a group norm and a separable norm that both act on
 * the same single group). */
/* prox of theta * sqrt(<., D .>), D = diag(w) > 0 (section 4.3).  By eq. (prox-projection) it is
 * z - pi_C(z), C the Wulff shape of theta H: the ellipsoid sum y_i^2 / s_i <= 1 with squared
 * semi-axes s_i = theta^2 w_i.  For z in C the prox is 0.  Otherwise the projection is
 * s_i z_i / (s_i + mu), with mu > 0 the Lagrange multiplier solving sum s_i z_i^2 / (s_i + mu)^2 = 1,
 * i.e. the minimiser of mu -> sum s_i z_i^2 / (s_i + mu) + mu, found as the paper does by Newton's
 * method from mu = 0 (here run until the step is at rounding level, not the paper's 1e-8).
 * Then d_i = z_i - s_i z_i / (s_i + mu) = mu z_i / (s_i + mu). */
static void prox_wl2(int n, const double* w, double theta, const double* z, double* d) {
  ksum q = {0, 0};
  for (int i = 0; i < n; ++i) ks_add(&q, z[i] * z[i] / (theta * theta * wgt(w, i)));
  if (ks_val(&q) <= 1.0) {
    for (int i = 0; i < n; ++i) d[i] = 0.0;
    return;
  }
  double mu = 0.0;
  for (int it = 0; it < 1000; ++it) {
    ksum g = {0, 0}, gp = {0, 0};  /* derivative and second derivative of the minimised function */
    ks_add(&g, 1.0);
    for (int i = 0; i < n; ++i) {
      const double s = theta * theta * wgt(w, i), den = s + mu;
      const double e = s * z[i] * z[i] / (den * den);
      ks_add(&g, -e);
      ks_add(&gp, 2.0 * e / den);
    }
    const double dmu = -ks_val(&g) / ks_val(&gp);
    if (!(dmu > 0.0)) break; /* increasing from the left until rounding stops it */
    mu += dmu;
    if (dmu <= 1e-16 * (mu > 1.0 ? mu : 1.0)) break;
  }
  for (int i = 0; i < n; ++i) {
    const double s = theta * theta * wgt(w, i);
    d[i] = mu * z[i] / (s + mu);
  }
}

/* prox of theta * sqrt(<., HA .>) for a full SPD HA = Q diag(sig) Q^T (section 4.3, the case
 * ||.||_A): the Wulff shape is the ellipsoid y^T HA^{-1} y <= 1 and, as the paper states, the
 * projection onto it is Q pi_D(Q^T w) with pi_D the projection onto the axis-aligned ellipsoid of
 * the eigenvalues; so d = z - Q pi_D(Q^T z) = Q (u - pi_D(u)), u = Q^T z, the diagonal prox in
 * the eigenbasis rotated back. */
static void prox_al2(int n, const double* Q, const double* sig, double theta, const double* z,
                     double* d, double* u, double* du) {
  for (int a = 0; a < n; ++a) {
    ksum k = {0, 0};
    for (int i = 0; i < n; ++i) ks_add(&k, Q[(size_t)i * n + a] * z[i]);
    u[a] = ks_val(&k);
  }
  prox_wl2(n, sig, theta, u, du);
  for (int i = 0; i < n; ++i) {
    ksum k = {0, 0};
    for (int a = 0; a < n; ++a) ks_add(&k, Q[(size_t)i * n + a] * du[a]);
    d[i] = ks_val(&k);
  }
}

/* The breakpoint method of sections 4.2 and 4.4 for a root of a decreasing, piecewise-affine
 * function f(mu) = a |shrink1(z, mu)|_1 - b mu - c on [0, max |z_i|], whose breakpoints are 0 and
 * the |z_i|: sort the breakpoints increasingly, find the two consecutive ones l_j, l_{j+1} with
 * f(l_j) >= 0 > f(l_{j+1}), and interpolate (f is affine between them).  The caller guarantees
 * f(0) >= 0 > f(max |z_i|).  `bp` holds n + 1 doubles. */
static double shrink1_norm(int n, const double* z, double mu) {
  ksum k = {0, 0};
  for (int i = 0; i < n; ++i) ks_add(&k, fabs(shrink1(z[i], mu)));
  return ks_val(&k);
}
static int cmp_double(const void* a, const void* b) {
  const double x = *(const double*)a, y = *(const double*)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}
static double breakpoint_root(int n, const double* z, double a, double b, double c, double* bp) {
  bp[0] = 0.0;
  for (int i = 0; i < n; ++i) bp[i + 1] = fabs(z[i]);
  qsort(bp, (size_t)n + 1, sizeof(double), cmp_double);
  double lo = bp[0], flo = a * shrink1_norm(n, z, lo) - b * lo - c;
  for (int j = 1; j <= n; ++j) {
    if (bp[j] == lo) continue;
    const double hi = bp[j], fhi = a * shrink1_norm(n, z, hi) - b * hi - c;
    if (fhi < 0.0) return lo + flo * (hi - lo) / (flo - fhi);
    lo = hi; flo = fhi;
  }
  return lo;
}

/* prox of theta |.|_inf (section 4.2): z - pi(z), pi the projection onto the l1 ball of radius
 * theta (the Wulff shape); 0 when |z|_1 <= theta, else z - shrink1(z, mu) with mu the root of
 * |shrink1(z, mu)|_1 = theta (eqs. projection_mu_linfty, condition_mu_linfty). */
static void prox_linf(int n, double theta, const double* z, double* d, double* bp) {
  ksum k = {0, 0};
  for (int i = 0; i < n; ++i) ks_add(&k, fabs(z[i]));
  if (ks_val(&k) <= theta) {
    for (int i = 0; i < n; ++i) d[i] = 0.0;
    return;
  }
  const double mu = breakpoint_root(n, z, 1.0, 0.0, theta, bp);
  for (int i = 0; i < n; ++i) d[i] = z[i] - shrink1(z[i], mu);
}

/* prox of (alpha / 2) |.|_1^2 (section 4.4): shrink1(z, beta) with beta = alpha |shrink1(z, beta)|_1
 * (eqs. optimality_beta_l1_2, prox_l1_2_with_beta), beta the root of the breakpoint function
 * alpha |shrink1(z, beta)|_1 - beta. */
static void prox_l1sq(int n, double alpha, const double* z, double* out, double* bp) {
  int nz = 0;
  for (int i = 0; i < n; ++i) nz |= z[i] != 0.0;
  const double beta = nz ? breakpoint_root(n, z, alpha, 1.0, 0.0, bp) : 0.0;
  for (int i = 0; i < n; ++i) out[i] = shrink1(z[i], beta);
}

/* prox of (alpha / 2) |.|_inf^2 by Moreau's identity with its conjugate (1 / (2 alpha)) |.|_1^2
 * (section 4.4; the printed form with alpha / 2 in both terms holds for alpha = 1 only):
 * z - prox_{(1 / (2 alpha)) |.|_1^2}(z). */
static void prox_linfsq(int n, double alpha, const double* z, double* out, double* bp, double* tmp) {
  prox_l1sq(n, 1.0 / alpha, z, tmp, bp);
  for (int i = 0; i < n; ++i) out[i] = z[i] - tmp[i];
}

static void prox_h(int n, int hkind, const double* w, double theta, const double* z, double* d) {
  if (hkind == OH_WL2) {
    prox_wl2(n, w, theta, z, d);
    return;
  }
  if (hkind == OH_WL1 || hkind == OH_L2_WL1) {
    for (int i = 0; i < n; ++i) d[i] = shrink1(z[i], theta * wgt(w, i));
  } else {
    memcpy(d, z, sizeof(double) * (size_t)n);
  }
  if (hkind == OH_L2 || hkind == OH_L2_WL1) {
    double nr = sqrt(dot(n, d, d));
    if (nr == 0.0) {
      for (int i = 0; i < n; ++i) d[i] = 0.0;
    } else {
      double f = (nr - theta > 0.0 ? nr - theta : 0.0) / nr;
      for (int i = 0; i < n; ++i) d[i] *= f;
    }
  }
}

/* ------------------------------------------------------------------------- */
/* One Hopf evaluation by split Bregman, eqs. (3.4a)-(3.4c), with the         */
/* initial values v0 = d0 = x', b0 = 0 and the stopping test of section 4.5   */
/* (all three squared norms <= tol).                                           */
/* ------------------------------------------------------------------------- */
typedef struct {
  int n;
  double *v, *d, *b, *rhs, *vn, *dn, *z, *tmp, *y, *t2, *bp;
} scratch;

static int scratch_alloc(scratch* s, int n) {
  s->n = n;
  double* buf = (double*)calloc((size_t)11 * n + 1, sizeof(double));
  if (!buf) return -1;
  s->v = buf; s->d = buf + n; s->b = buf + 2 * n; s->rhs = buf + 3 * n; s->vn = buf + 4 * n;
  s->dn = buf + 5 * n; s->z = buf + 6 * n; s->tmp = buf + 7 * n; s->y = buf + 8 * n;
  s->t2 = buf + 9 * n; s->bp = buf + 10 * n; /* bp: n + 1 breakpoints */
  return 0;
}

static double norm1(int n, const double* p) {
  ksum k = {0, 0};
  for (int i = 0; i < n; ++i) ks_add(&k, fabs(p[i]));
  return ks_val(&k);
}
static double norminf(int n, const double* p) {
  double m = 0.0;
  for (int i = 0; i < n; ++i) m = fabs(p[i]) > m ? fabs(p[i]) : m;
  return m;
}
static void scratch_free(scratch* s) { free(s->v); }

/* Solves min_p F(p) = 1/2 p^T A p + t H(p) - <xp, p>.  Writes p (= d^K) into out_p,
 * returns -F(p) (the Hopf value of eq. (3.3) without any constant offset).
 * *iters = number of v-updates, or -2 if max_iter was reached.
 * gap (nullable): J(xp - lambda b) + F(p) with J(y) = 1/2 y^T A^{-1} y (needs LA = chol(A)). */
static double hopf_solve(const oh_problem* pb, int hkind, const double* LS, const double* LA,
                         const double* xp, double t, scratch* s, double* out_p, int32_t* iters,
                         double* gap) {
  const int n = pb->n;
  const double lam = pb->lambda;
  memcpy(s->v, xp, sizeof(double) * (size_t)n);
  memcpy(s->d, xp, sizeof(double) * (size_t)n);
  memset(s->b, 0, sizeof(double) * (size_t)n);
  int k = 0, conv = 0;
  while (k < pb->max_iter) {
    ++k;
    /* (3.4a): v = argmin J*(v) - <x,v> + lambda/2 ||d - v - b||^2  <=>  (A + lambda I) v = x + lambda (d - b) */
    if (pb->jkind == OJ_QUAD) {
      for (int i = 0; i < n; ++i) s->rhs[i] = xp[i] + lam * (s->d[i] - s->b[i]);
      chol_solve(n, LS, s->rhs, s->tmp, s->vn);
    } else {
      /* the same minimisation for a squared-norm J* is the prox of (1 / lambda) J* at d - b + x / lambda */
      for (int i = 0; i < n; ++i) s->rhs[i] = s->d[i] - s->b[i] + xp[i] / lam;
      if (pb->jkind == OJ_L1SQ) prox_linfsq(n, 1.0 / lam, s->rhs, s->vn, s->bp, s->t2); /* J* = 1/2 |.|_inf^2 */
      else prox_l1sq(n, 1.0 / lam, s->rhs, s->vn, s->bp);                              /* J* = 1/2 |.|_1^2 */
    }
    /* (3.4b): d = prox_{(t/lambda) H}(v + b) */
    for (int i = 0; i < n; ++i) s->z[i] = s->vn[i] + s->b[i];
    const double theta = t / lam;
    if (hkind == OH_AL2) prox_al2(n, pb->HQ, pb->Hsig, theta, s->z, s->dn, s->tmp, s->y);
    else if (hkind == OH_LINF) prox_linf(n, theta, s->z, s->dn, s->bp);
    else prox_h(n, hkind, pb->w, theta, s->z, s->dn);
    /* (3.4c): b = b + v - d */
    for (int i = 0; i < n; ++i) s->b[i] = s->b[i] + s->vn[i] - s->dn[i];
    double r1 = sqdist(n, s->vn, s->v);
    double r2 = sqdist(n, s->dn, s->d);
    double r3 = sqdist(n, s->dn, s->vn);
    memcpy(s->v, s->vn, sizeof(double) * (size_t)n);
    memcpy(s->d, s->dn, sizeof(double) * (size_t)n);
    if (r1 <= pb->tol && r2 <= pb->tol && r3 <= pb->tol) { conv = 1; break; }
  }
  *iters = conv ? k : -2;
  const double* p = s->d;
  memcpy(out_p, p, sizeof(double) * (size_t)n);
  ksum F = {0, 0};
  if (pb->jkind == OJ_QUAD) ks_add(&F, 0.5 * quad(n, pb->A, p));
  else {
    const double q = pb->jkind == OJ_L1SQ ? norminf(n, p) : norm1(n, p); /* J* = 1/2 (dual norm)^2 */
    ks_add(&F, 0.5 * q * q);
  }
  ks_add(&F, t * ham(pb, hkind, p));
  ks_add(&F, -dot(n, xp, p));
  double Fv = ks_val(&F);
  if (gap) {
    /* Hopf-Lax feasible point y = x' - lambda b: lambda b / t lies in t^{-1} * t dH(d) within the Wulff shape. */
    for (int i = 0; i < n; ++i) s->y[i] = xp[i] - lam * s->b[i];
    double Jy;
    if (pb->jkind == OJ_QUAD) {
      chol_solve(n, LA, s->y, s->tmp, s->z); /* z = A^{-1} y */
      Jy = 0.5 * dot(n, s->y, s->z);
    } else {
      const double q = pb->jkind == OJ_L1SQ ? norm1(n, s->y) : norminf(n, s->y);
      Jy = 0.5 * q * q;
    }
    *gap = Jy + Fv;
  }
  return -Fv;
}

/* ------------------------------------------------------------------------- */
/* Threading over points.                                                     */
/* ------------------------------------------------------------------------- */
typedef struct {
  const oh_problem* pb;
  const double *LS, *LA;
  int64_t begin, end;
  const double *x, *t;
  double *phi, *grad, *dphidt, *gap;
  int32_t *iters, *kstar;
  int rc;
} eval_job;

static void* eval_worker(void* arg) {
  eval_job* J = (eval_job*)arg;
  const oh_problem* pb = J->pb;
  const int n = pb->n;
  scratch s;
  if (scratch_alloc(&s, n)) { J->rc = -1; return NULL; }
  double* xp = (double*)malloc(sizeof(double) * (size_t)n * 2);
  double* p = xp + n;
  for (int64_t j = J->begin; j < J->end; ++j) {
    const double* x = J->x + (size_t)j * n;
    double t = J->t[j];
    double best = INFINITY;
    int kb = -1;
    for (int k = 0; k < pb->K; ++k) {
      for (int i = 0; i < n; ++i) xp[i] = x[i] - (pb->centres ? pb->centres[(size_t)k * n + i] : 0.0);
      int32_t it;
      double g = 0.0;
      double val = hopf_solve(pb, pb->hkind, J->LS, J->LA, xp, t, &s, p, &it, J->gap ? &g : NULL);
      if (pb->level_set) val -= 0.5; /* J_k* carries the constant +1/2 */
      /* min over initial data (section 2): phi = min_k phi_k, lowest k on ties */
      if (val < best || kb < 0) {
        best = val; kb = k;
        memcpy(J->grad + (size_t)j * n, p, sizeof(double) * (size_t)n);
        J->iters[j] = it;
        if (J->gap) J->gap[j] = g;
      }
    }
    J->phi[j] = best;
    J->kstar[j] = kb;
    /* dphi/dt = -H(grad phi), from (1.1a) */
    J->dphidt[j] = -ham(pb, pb->hkind, J->grad + (size_t)j * n);
  }
  free(xp);
  scratch_free(&s);
  return NULL;
}

static int check_problem(const oh_problem* pb) {
  if (!pb || pb->n < 1 || !pb->A || pb->K < 1 || !(pb->lambda > 0) || pb->max_iter < 1) return -1;
  if (pb->hkind < OH_WL1 || pb->hkind > OH_LINF) return -1;
  if (pb->jkind < OJ_QUAD || pb->jkind > OJ_LINFSQ) return -1;
  if (pb->hkind == OH_AL2) {
    if (!pb->HA || !pb->HQ || !pb->Hsig) return -1;
    for (int i = 0; i < pb->n; ++i)
      if (!(pb->Hsig[i] > 0)) return -1;
  }
  if (pb->w)
    for (int i = 0; i < pb->n; ++i)
      if (!(pb->w[i] >= 0) || (pb->hkind == OH_WL2 && !(pb->w[i] > 0))) return -1;
  return 0;
}

int oh_eval(const oh_problem* pb, int64_t npts, const double* x, const double* t, double* phi,
            double* grad, double* dphidt, int32_t* iters, int32_t* kstar, double* gap,
            int nthreads) {
  if (check_problem(pb) || npts < 0) return -1;
  for (int64_t j = 0; j < npts; ++j)
    if (!(t[j] > 0)) return -1;
  const int n = pb->n;
  double* LS = (double*)malloc(sizeof(double) * (size_t)n * n * 2);
  double* LA = LS + (size_t)n * n;
  if (!LS) return -1;
  int rc = cholesky(n, pb->A, pb->lambda, LS);
  if (rc == 0 && gap) rc = cholesky(n, pb->A, 0.0, LA);
  if (rc) { free(LS); return rc; }
  if (nthreads < 1) nthreads = 1;
  if (nthreads > npts) nthreads = npts > 0 ? (int)npts : 1;
  eval_job* jobs = (eval_job*)calloc((size_t)nthreads, sizeof(eval_job));
  pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
  for (int i = 0; i < nthreads; ++i) {
    eval_job* J = &jobs[i];
    J->pb = pb; J->LS = LS; J->LA = LA; J->x = x; J->t = t;
    J->phi = phi; J->grad = grad; J->dphidt = dphidt; J->gap = gap; J->iters = iters; J->kstar = kstar;
    J->begin = npts * i / nthreads; J->end = npts * (i + 1) / nthreads;
    if (nthreads == 1) eval_worker(J);
    else pthread_create(&th[i], NULL, eval_worker, J);
  }
  rc = 0;
  for (int i = 0; i < nthreads; ++i) {
    if (nthreads > 1) pthread_join(th[i], NULL);
    if (jobs[i].rc) rc = jobs[i].rc;
  }
  free(jobs); free(th); free(LS);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Closest point / distance by the level-set route of section 3.2:            */
/* psi solves the eikonal equation with psi(.,0) = L_k (the quadratic level-  */
/* set function of ellipsoid k), psi(y, s) is a Hopf evaluation with          */
/* H = ||.||_2 (split Bregman (3.9) is (3.4) with H = ||.||_2), and Newton on */
/* s uses d psi / ds = -||grad_x psi|| (eq. Newton_zero).                     */
/* ------------------------------------------------------------------------- */
typedef struct {
  const oh_problem* pb;
  const double *LS, *LA;
  int64_t begin, end;
  const double* y;
  double s_tol;
  int32_t max_newton;
  double *dist, *cp;
  int32_t *kstar, *inside, *newton;
  int rc;
} dist_job;

static void* dist_worker(void* arg) {
  dist_job* J = (dist_job*)arg;
  const oh_problem* pb = J->pb;
  const int n = pb->n;
  scratch s;
  if (scratch_alloc(&s, n)) { J->rc = -1; return NULL; }
  double* buf = (double*)malloc(sizeof(double) * (size_t)n * 4);
  double *yp = buf, *g = buf + n, *p = buf + 2 * n, *tmp = buf + 3 * n;
  for (int64_t j = J->begin; j < J->end; ++j) {
    const double* y = J->y + (size_t)j * n;
    double best = INFINITY;
    int kb = -1, ins = 0, nb = 0;
    double* cpj = J->cp + (size_t)j * n;
    for (int k = 0; k < pb->K && !ins; ++k) {
      for (int i = 0; i < n; ++i) yp[i] = y[i] - (pb->centres ? pb->centres[(size_t)k * n + i] : 0.0);
      chol_solve(n, J->LA, yp, tmp, g); /* g = A^{-1}(y - c_k) = grad L_k(y) */
      double Ly = 0.5 * (dot(n, yp, g) - 1.0);
      if (Ly <= 0.0) { /* y lies in ellipsoid k: distance 0, closest point y */
        ins = 1; kb = k; best = 0.0;
        memcpy(cpj, y, sizeof(double) * (size_t)n);
        break;
      }
      double sv = Ly / sqrt(dot(n, g, g)); /* a lower bound of the distance */
      int l = 0;
      double pn = 0.0;
      while (l < J->max_newton) {
        ++l;
        int32_t it;
        double psi = hopf_solve(pb, OH_L2, J->LS, J->LA, yp, sv, &s, p, &it, NULL) - 0.5;
        pn = sqrt(dot(n, p, p));
        if (pn == 0.0) break;
        double ds = psi / pn; /* s_{l+1} = s_l - psi / (d psi/ds), d psi/ds = -||grad psi|| */
        sv += ds;
        if (fabs(ds) <= J->s_tol * (sv > 1.0 ? sv : 1.0)) break;
      }
      if (sv < best) {
        best = sv; kb = k; nb = l;
        /* pi(y) = y - s * grad psi / ||grad psi||  (eq. projection_when_s_known) */
        for (int i = 0; i < n; ++i) cpj[i] = y[i] - (pn > 0 ? sv * p[i] / pn : 0.0);
      }
    }
    J->dist[j] = best;
    J->kstar[j] = kb;
    J->inside[j] = ins;
    if (J->newton) J->newton[j] = nb;
  }
  free(buf);
  scratch_free(&s);
  return NULL;
}

int oh_distance_newton(const oh_problem* pb, int64_t npts, const double* y, double s_tol,
                       int32_t max_newton, double* dist, double* cp, int32_t* kstar,
                       int32_t* inside, int32_t* newton, int nthreads) {
  if (check_problem(pb) || npts < 0 || max_newton < 1) return -1;
  const int n = pb->n;
  double* LS = (double*)malloc(sizeof(double) * (size_t)n * n * 2);
  double* LA = LS + (size_t)n * n;
  int rc = cholesky(n, pb->A, pb->lambda, LS);
  if (rc == 0) rc = cholesky(n, pb->A, 0.0, LA);
  if (rc) { free(LS); return rc; }
  if (nthreads < 1) nthreads = 1;
  if (nthreads > npts) nthreads = npts > 0 ? (int)npts : 1;
  dist_job* jobs = (dist_job*)calloc((size_t)nthreads, sizeof(dist_job));
  pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
  for (int i = 0; i < nthreads; ++i) {
    dist_job* J = &jobs[i];
    J->pb = pb; J->LS = LS; J->LA = LA; J->y = y; J->s_tol = s_tol; J->max_newton = max_newton;
    J->dist = dist; J->cp = cp; J->kstar = kstar; J->inside = inside; J->newton = newton;
    J->begin = npts * i / nthreads; J->end = npts * (i + 1) / nthreads;
    if (nthreads == 1) dist_worker(J);
    else pthread_create(&th[i], NULL, dist_worker, J);
  }
  rc = 0;
  for (int i = 0; i < nthreads; ++i) {
    if (nthreads > 1) pthread_join(th[i], NULL);
    if (jobs[i].rc) rc = jobs[i].rc;
  }
  free(jobs); free(th); free(LS);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Textbook projection onto an ellipsoid (section 4.3): in the eigenbasis the  */
/* projection of u is sigma_i u_i / (sigma_i + mu) with mu > 0 the root of     */
/* sum sigma_i u_i^2 / (sigma_i + mu)^2 = 1, found by Newton from mu = 0.      */
/* ------------------------------------------------------------------------- */
int oh_distance_secular(int32_t n, const double* Q, const double* sigma, int32_t K,
                        const double* centres, int64_t npts, const double* y, double* dist,
                        double* cp, int32_t* kstar, int32_t* inside) {
  if (n < 1 || !Q || !sigma || K < 1 || npts < 0) return -1;
  for (int i = 0; i < n; ++i)
    if (!(sigma[i] > 0)) return -2;
  double* buf = (double*)malloc(sizeof(double) * (size_t)n * 3);
  double *u = buf, *us = buf + n, *col = buf + 2 * n;
  for (int64_t j = 0; j < npts; ++j) {
    const double* yj = y + (size_t)j * n;
    double* cpj = cp + (size_t)j * n;
    double best = INFINITY;
    int kb = -1, ins = 0;
    for (int k = 0; k < K && !ins; ++k) {
      const double* c = centres ? centres + (size_t)k * n : NULL;
      for (int a = 0; a < n; ++a) { /* u = Q^T (y - c) */
        ksum s = {0, 0};
        for (int i = 0; i < n; ++i) ks_add(&s, Q[(size_t)i * n + a] * (yj[i] - (c ? c[i] : 0.0)));
        u[a] = ks_val(&s);
      }
      ksum q = {0, 0};
      for (int a = 0; a < n; ++a) ks_add(&q, u[a] * u[a] / sigma[a]);
      if (ks_val(&q) <= 1.0) {
        ins = 1; kb = k; best = 0.0;
        memcpy(cpj, yj, sizeof(double) * (size_t)n);
        break;
      }
      double mu = 0.0;
      for (int it = 0; it < 500; ++it) {
        ksum g = {0, 0}, gp = {0, 0};
        ks_add(&g, -1.0);
        for (int a = 0; a < n; ++a) {
          double den = sigma[a] + mu;
          double e = sigma[a] * u[a] * u[a] / (den * den);
          ks_add(&g, e);
          ks_add(&gp, -2.0 * e / den);
        }
        double dmu = -ks_val(&g) / ks_val(&gp);
        mu += dmu;
        if (fabs(dmu) <= 1e-15 * (mu > 1.0 ? mu : 1.0)) break;
      }
      ksum d2 = {0, 0};
      for (int a = 0; a < n; ++a) {
        us[a] = sigma[a] * u[a] / (sigma[a] + mu);
        double e = u[a] - us[a];
        ks_add(&d2, e * e);
      }
      double dk = sqrt(ks_val(&d2));
      if (dk < best) {
        best = dk; kb = k;
        for (int i = 0; i < n; ++i) { /* cp = c + Q u* */
          for (int a = 0; a < n; ++a) col[a] = Q[(size_t)i * n + a];
          cpj[i] = (c ? c[i] : 0.0) + dot(n, col, us);
        }
      }
    }
    dist[j] = best; kstar[j] = kb; inside[j] = ins;
  }
  free(buf);
  return 0;
}
