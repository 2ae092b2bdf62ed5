/*
 * Plain FP64 CPU oracle for the Hopf-formula evaluation of Darbon & Osher,
 * "Algorithms for overcoming the curse of dimensionality for certain
 * Hamilton-Jacobi equations arising in control theory and elsewhere"
 * (arXiv:1605.01799).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this library; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the HIP library.
 *
 * Everything is double precision, one point at a time, in the order the paper
 * states the algorithm.  Dot products use Neumaier-compensated summation.
 */
#ifndef HOPF_ORACLE_H
#define HOPF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OH_WL1 = 0, OH_L2 = 1, OH_L2_WL1 = 2, OH_WL2 = 3, OH_AL2 = 4, OH_LINF = 5 };
/* initial data: quadratic 1/2 y^T A^{-1} y, or the squared norms of section 4.4 */
enum { OJ_QUAD = 0, OJ_L1SQ = 1, OJ_LINFSQ = 2 };

typedef struct {
  int32_t n;
  const double* A;        /* n*n row-major SPD; J(y) = 1/2 y^T A^{-1} y, so J*(p) = 1/2 p^T A p */
  int32_t K;              /* number of ellipsoids / translated copies of J (>= 1) */
  const double* centres;  /* K*n, or NULL (all centres 0) */
  int32_t level_set;      /* 1: J_k(y) = 1/2((y-c_k)^T A^{-1} (y-c_k) - 1) */
  int32_t hkind;          /* OH_WL1, OH_L2, OH_L2_WL1, OH_WL2, OH_AL2, OH_LINF (||p||_inf) */
  const double* w;        /* n weights >= 0 (> 0 for OH_WL2), or NULL (all 1) */
  double lambda;          /* split-Bregman penalty (paper: 1) */
  double tol;             /* stop when max of the three squared norms <= tol */
  int32_t max_iter;
  /* OH_AL2 only: H(p) = sqrt(p^T HA p) with HA (n*n row-major SPD) = HQ diag(Hsig) HQ^T
   * (HQ row-major, columns = eigenvectors); NULL otherwise */
  const double* HA;
  const double* HQ;
  const double* Hsig;
  /* OJ_QUAD: J(y) = 1/2 y^T A^{-1} y; OJ_L1SQ: J(y) = 1/2 |y|_1^2 (J*(p) = 1/2 |p|_inf^2);
   * OJ_LINFSQ: J(y) = 1/2 |y|_inf^2 (J*(p) = 1/2 |p|_1^2).  For the last two A is not used. */
  int32_t jkind;
} oh_problem;

/* Returns 0 on success, -1 on bad arguments, -2 if A + lambda I (or A) is not SPD.
 * Per point j (of npts): phi[j], grad[j*n..], dphidt[j], iters[j] (of the
 * attaining ellipsoid; -2 if the cap was hit), kstar[j] (lowest index attaining
 * the min).  gap (nullable): duality-gap certificate J(x'-lambda b) + F(d) of
 * the attaining ellipsoid.  nthreads <= 0 means 1. */
int oh_eval(const oh_problem* pb, int64_t npts, const double* x, const double* t,
            double* phi, double* grad, double* dphidt, int32_t* iters,
            int32_t* kstar, double* gap, int nthreads);

/* Distance from y to the union of the K ellipsoids {u : (u-c_k)^T A^{-1} (u-c_k) <= 1}
 * by the paper's level-set route: Newton on s for psi_k(y, s) = 0, each psi_k
 * evaluated by split Bregman with H = ||.||_2.  s_tol: stop at |ds| <= s_tol*max(1,s).
 * Outputs dist[j], cp[j*n..], kstar[j], inside[j] (1 if y is in the union), newton[j]
 * (Newton steps of the attaining ellipsoid). */
int oh_distance_newton(const oh_problem* pb, int64_t npts, const double* y,
                       double s_tol, int32_t max_newton,
                       double* dist, double* cp, int32_t* kstar, int32_t* inside,
                       int32_t* newton, int nthreads);

/* Distance to the same union by the textbook route: project u = Q^T (y - c_k)
 * onto the axis-aligned ellipsoid sum u_i^2 / sigma_i <= 1 through the
 * Lagrange-multiplier (secular) equation, Newton on mu from mu = 0.
 * Q (n*n row-major, columns = eigenvectors) and sigma (n) describe A = Q diag(sigma) Q^T. */
int oh_distance_secular(int32_t n, const double* Q, const double* sigma, int32_t K,
                        const double* centres, int64_t npts, const double* y,
                        double* dist, double* cp, int32_t* kstar, int32_t* inside);

#ifdef __cplusplus
}
#endif
#endif
