/*
 * hopf.h -- C ABI of the MI355X (gfx950) Hopf-formula library.
 *
 * Method: Darbon & Osher, "Algorithms for overcoming the curse of
 * dimensionality for certain Hamilton-Jacobi equations arising in control
 * theory and elsewhere", arXiv:1605.01799.
 *
 * For every query point (x, t) the library evaluates the Hopf formula
 * (eqs. (1.2)/(3.3))
 *     phi(x, t) = -min_p { J*(p) + t H(p) - <x, p> }
 * for the initial data J(y) = 1/2 y^T A^{-1} y (A symmetric positive definite,
 * so J*(p) = 1/2 p^T A p), or for the non-convex initial data
 * J = min_k J_k over K translated copies / ellipsoid level-set functions
 * (section 2, "min over initial data": phi = min_k phi_k), with the convex,
 * positively 1-homogeneous Hamiltonians H = sum_i w_i |p_i|, ||p||_2, or their
 * sum.  The minimiser is found by split Bregman (eqs. (3.4a)-(3.4c)); the
 * library returns phi, grad_x phi = p* (the minimiser, section 1) and
 * d phi / d t = -H(p*) (eq. (1.1a)).  It also computes the distance from a
 * point to a union of ellipsoids and the closest point on it (section 3.2,
 * level-set eikonal evaluation with Newton on s, eq. (Newton_zero)), and the
 * envelope-theorem gradients of phi with respect to x, t, A and the centres.
 *
 * Conventions (all entry points):
 *  - Host pointers are marked "host"; every other array argument is a DEVICE
 *    pointer owned by the caller (e.g. allocated by PyTorch).  The library
 *    owns only what a problem handle holds (the factored matrices on device)
 *    and an internal workspace per device (grown on demand with hipMalloc).
 *  - Array element type: double for precision HOPF_F64, float for HOPF_F32
 *    and HOPF_BF16_REFINED ("real" below).  Points are stored point-major:
 *    x[j*n + i] is coordinate i of point j.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Every call is
 *    stream-ordered: returning HOPF_OK means the work was enqueued, not that
 *    it finished.  Host arrays passed in are copied before the call returns.
 *  - Errors: argument checks happen synchronously on the host and return a
 *    status; no state is changed on error.  hopf_last_error() returns a
 *    thread-local description of the last non-OK status.  Per-point problems
 *    are reported in iters[]: >= 1 converged after that many v-updates, -2
 *    the iteration cap was hit, or (plain FP32 iteration only) the step norm stopped
 *    decreasing for 64 iterations before reaching tol, i.e. the iterate
 *    stalled at FP32 precision (outputs come from the last iterate), -1 a
 *    non-finite input, or t <= 0 or not finite (outputs are NaN).
 *  - Calls that share a problem handle may run concurrently on different
 *    streams; calls on one device share the workspace and are serialised by
 *    the library's per-device lock around enqueueing (not around execution:
 *    use one stream per device, or synchronise between streams).
 */
#ifndef HOPF_H
#define HOPF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HOPF_OK = 0,
  HOPF_EINVAL = -1,   /* bad argument */
  HOPF_ENOTSPD = -2,  /* A + lambda I (or A) is not symmetric positive definite */
  HOPF_ENOMEM = -3,   /* device allocation failed */
  HOPF_EDEVICE = -4   /* HIP runtime error or missing gfx950 device */
} hopf_status;

typedef enum {
  HOPF_H_WL1 = 0,     /* H(p) = sum_i w_i |p_i|            (support function of a box)  */
  HOPF_H_L2 = 1,      /* H(p) = ||p||_2                    (support function of a ball) */
  HOPF_H_L2_WL1 = 2,  /* H(p) = ||p||_2 + sum_i w_i |p_i|  (their Minkowski sum)        */
  HOPF_H_WL2 = 3,     /* H(p) = sqrt(sum_i w_i p_i^2), w_i > 0: the norm sqrt(<p, D p>),
                         D = diag(w), of section 4.3 (support function of the ellipsoid
                         sum_i y_i^2 / w_i <= 1).  Its prox is z minus the projection onto
                         that ellipsoid (eq. (prox-projection)), one Newton solve for the
                         Lagrange multiplier per iteration (in the refined modes: on the
                         multiplier's increment since the anchor, FP64 at the anchor).
                         Every precision and size of the quadratic J (HOPF_F64: diagonal
                         A with n <= 32, as for every H). */
  HOPF_H_AL2 = 4,     /* H(p) = sqrt(<p, HA p>) for a full SPD matrix HA (the norm ||.||_A of
                         section 4.3; HA in the descriptor).  The library diagonalises HA on the
                         device (HA = P diag(s) P^T, FP64 Jacobi) and holds the problem in that
                         basis, where H is HOPF_H_WL2 with weights s, A becomes P^T A P and the
                         centres P^T c; points are rotated in before the solve and gradients /
                         closest points rotated back after it.  HOPF_F32 and
                         HOPF_BF16_REFINED with n <= 64; HOPF_F64 with diagonal A and
                         n <= 32 (there the prox rotates, A stays diagonal). */
  HOPF_H_LINF = 5,    /* H(p) = ||p||_inf (section 4.2): its prox is z minus the projection onto
                         the l1 ball (the Wulff shape), found by a breakpoint search.  On the
                         per-thread path only: diagonal A or a squared-norm J, n <= 32. */
  HOPF_H_LINCTRL = 6  /* The time-dependent Hamiltonian of linear controls (section 2.2, "some
                         extensions"): the state follows dx/ds = M x + N beta(s), beta(s) in the
                         box [-1, 1]^n, with M = diag(drift) and N = diag(w) (w_i >= 0: the
                         box's half-widths scaled by |N_ii|).  In the variables z = e^{-sM} x,
                         H(p, s) = sum_i e^{-s m_i} w_i |p_i|, and the Hopf formula takes its
                         integral, phi(z, t) = -min_u (J*(u) + sum_i W_i(t) |u_i| - <z, u>),
                         W_i(t) = w_i (1 - e^{-t m_i}) / m_i (t w_i for m_i = 0).  The points
                         passed to hopf_eval are z; grad = the minimiser u*, dphidt =
                         -H(grad, t) (the Hamiltonian at time t).  Per-thread path only:
                         diagonal A (or A = I), n <= 32, HOPF_F64 or HOPF_F32, quadratic J;
                         not in ragged batches, no control read-out. */
} hopf_hkind;

/* Initial data J (section 4.4).  HOPF_J_QUADRATIC uses the descriptor's A; the squared norms
 * ignore A (it may be NULL), run on the per-thread path (n <= 32, HOPF_F64 or HOPF_F32) and take
 * update (3.4a) as the prox of J* (the squared dual norm) by a breakpoint search. */
typedef enum {
  HOPF_J_QUADRATIC = 0,  /* J(y) = 1/2 y^T A^{-1} y            (J*(p) = 1/2 p^T A p)      */
  HOPF_J_L1SQ = 1,       /* J(y) = 1/2 ||y||_1^2                (J*(p) = 1/2 ||p||_inf^2)  */
  HOPF_J_LINFSQ = 2      /* J(y) = 1/2 ||y||_inf^2              (J*(p) = 1/2 ||p||_1^2)    */
} hopf_jkind;

typedef enum {
  HOPF_F64 = 0,          /* double I/O and arithmetic (diagonal A only) */
  HOPF_F32 = 1,          /* float I/O; FP32 MFMA products and FP32 state on increments,
                            refined by exact anchor products every few iterations (FP64 MFMA
                            for n <= 64, integer slices above) */
  HOPF_BF16_REFINED = 2  /* float I/O; BF16 MFMA products on increments, refined by
                            anchor products every few iterations that are exact up to
                            ~2^-31 of the row and column scales (integer slices) */
} hopf_precision;

typedef struct {
  int32_t n;                 /* dimension, 1 <= n <= 2048 */
  const double* A;           /* host. n*n row-major SPD matrix, or n entries if A_is_diagonal.
                                NULL means A = I.  J(y) = 1/2 y^T A^{-1} y. */
  int32_t A_is_diagonal;     /* 1: A holds the n diagonal entries (elementwise path) */
  int32_t K;                 /* number of translated copies of J, K >= 1 */
  const double* centres;     /* host, K*n, or NULL (all centres 0) */
  int32_t level_set;         /* 1: J_k(y) = 1/2((y-c_k)^T A^{-1} (y-c_k) - 1), ellipsoid k */
  hopf_hkind hkind;
  const double* w;           /* host, n weights >= 0 (> 0 for HOPF_H_WL2), or NULL (all 1);
                                ignored for HOPF_H_L2 */
  double lambda;             /* split-Bregman penalty > 0 (the paper uses 1) */
  double tol;                /* stopping tolerance on squared norms (see hopf_eval) */
  int32_t max_iter;          /* iteration cap >= 1 */
  hopf_precision precision;
  const double* HA;          /* host, n*n row-major SPD matrix of H for HOPF_H_AL2; otherwise
                                ignored (may be NULL).  HOPF_ENOTSPD if it is not positive
                                definite. */
  int32_t jkind;             /* hopf_jkind; 0 (HOPF_J_QUADRATIC) keeps the A above.  Translated
                                copies (K, centres) apply to every kind: J_k = J(. - c_k). */
  const double* drift;       /* host, n diagonal entries of the drift matrix M for
                                HOPF_H_LINCTRL (finite, any sign); otherwise ignored (may be
                                NULL). */
} hopf_problem_desc;

typedef struct hopf_problem* hopf_problem_t;

/* Creates a problem: validates the descriptor, copies the host data, and
 * enqueues on `stream` the FP64 factorisation of A + lambda I on the device
 * (block Gauss-Jordan inverse M = (A + lambda I)^{-1} with a Cholesky test of
 * every pivot block; section 4.1 states that the quadratic prox is
 * (I + alpha A)^{-1}), followed by the rounded copies the kernels read.
 * Returns HOPF_ENOTSPD (after synchronising `stream`) if a pivot block is not
 * positive definite.  *out is owned by the caller until hopf_problem_destroy. */
hopf_status hopf_problem_create(const hopf_problem_desc* desc, void* stream, hopf_problem_t* out);

/* Creates nprob problems at once (descs[i] -> out[i]); the dense factorisations of
 * the batch run together (problems sorted by size, one launch sequence), which is
 * how a ragged batch of many problems should be set up.  On error no handle is
 * returned (all out[i] are NULL) and the message names the failing problem. */
hopf_status hopf_problem_create_batch(int32_t nprob, const hopf_problem_desc* descs, void* stream,
                                      hopf_problem_t* out);

/* Releases the device memory of a problem (synchronises the device first).  The library keeps
 * up to 1 GiB of such freed blocks per device and hands them out again to problems created later
 * with the same buffer sizes (no hipMalloc for a repeated set-up); beyond that they go back to
 * the device.  The kept blocks are held until the process ends. */
hopf_status hopf_problem_destroy(hopf_problem_t problem);

/* Evaluates npts points (eq. (3.3), split Bregman (3.4a)-(3.4c) with
 * v0 = d0 = x - c_k, b0 = 0).  Inputs: x (npts*n), t (npts, > 0).  Outputs:
 * phi (npts), grad (npts*n) = p* of the attaining copy, dphidt (npts) =
 * -H(p*), iters (npts, nullable), kstar (npts, nullable; lowest index
 * attaining the min over k).  npts * K must stay below 2^31 (HOPF_EINVAL
 * otherwise).  A point stops when the squared change of the
 * split-Bregman iterate between two iterations, summed over the last two
 * iterations as (sqrt(a) + sqrt(b))^2, is <= tol; this bounds all three
 * squared norms of the stopping test of section 4.5 by tol.  npts == 0 is a
 * no-op. */
hopf_status hopf_eval(hopf_problem_t problem, int64_t npts, const void* x, const void* t,
                      void* phi, void* grad, void* dphidt, int32_t* iters, int32_t* kstar,
                      void* stream);

/* Distance from each y (npts*n) to the union of the K ellipsoids
 * {u : (u-c_k)^T A^{-1} (u-c_k) <= 1} of the problem (level_set must be 1;
 * H = ||.||_2 is used whatever the problem's hkind), by Newton on s for
 * psi_k(y, s) = 0 with psi_k the eikonal Hopf evaluation (section 3.2).
 * Outputs: dist (npts), cp (npts*n) closest point, kstar (npts, nearest
 * ellipsoid), inside (npts, nullable: 1 if y lies in the union, then dist = 0
 * and cp = y), newton (npts, nullable: Newton steps of the nearest ellipsoid,
 * -2 if a cap was hit, -1 for a non-finite y).  s_tol: Newton stops when
 * |s_{l+1} - s_l| <= s_tol * max(1, s).  Every inner solve has its own
 * max_iter budget; a solve that hits it still gives
 * the Newton step, and the point is then reported with newton = -2.
 * npts * K must stay below 2^31 (HOPF_EINVAL otherwise). */
hopf_status hopf_closest_point(hopf_problem_t problem, int64_t npts, const void* y, double s_tol,
                               void* dist, void* cp, int32_t* kstar, int32_t* inside,
                               int32_t* newton, void* stream);

/* Ragged batch: nprob problems (any n, K, A, w; one precision for all, not
 * HOPF_F64; no HOPF_H_LINF or squared-norm J).  The problems are grouped into kernel
 * classes by padded size (the launch shape of each class); each class is one
 * persistent launch over its problems' points; the classes are enqueued
 * back to back on stream, each with its own metadata, staging and chunk counter in the
 * per-device workspace (no host wait between them; calls on one stream are ordered).  Every problem's npts * K must stay below 2^31.  pt_offset (host, nprob+1)
 * gives the points of problem q as [pt_offset[q], pt_offset[q+1]); x_packed
 * holds the points of problem q contiguously starting at element
 * sum_{r<q} (pt_offset[r+1]-pt_offset[r]) * n_r, and grad_packed likewise.
 * t, phi, dphidt, iters, kstar are indexed by the global point index. */
hopf_status hopf_eval_ragged(int32_t nprob, const hopf_problem_t* problems,
                             const int64_t* pt_offset, const void* x_packed, const void* t,
                             void* phi, void* grad_packed, void* dphidt, int32_t* iters,
                             int32_t* kstar, void* stream);

/* A ragged evaluation bound once to its arguments (a plan), for callers that relaunch the same
 * batch: hopf_ragged_plan_create checks and groups the problems exactly as hopf_eval_ragged (same
 * arguments and layouts; the device arrays are referenced, not copied, and must stay valid and
 * unmoved while the plan lives), allocates the plan's own metadata, staging and counters and
 * uploads the metadata (synchronously).  hopf_ragged_plan_launch then enqueues only kernels on
 * stream (the counters' and per-point bests' resets are kernels too): no allocation, no copy, no
 * host synchronisation, so it can be captured in a HIP graph and replayed; each launch evaluates
 * the points in place (results as hopf_eval_ragged, read from the arrays at launch time).  Launches
 * of one plan must not overlap (they share its staging), and it must be launched on the device it
 * was made on (HOPF_EINVAL otherwise).  hopf_ragged_plan_destroy synchronises the device and frees
 * the plan.  Errors: as hopf_eval_ragged; HOPF_ENOMEM; HOPF_EDEVICE. */
typedef struct hopf_ragged_plan* hopf_ragged_plan_t;
hopf_status hopf_ragged_plan_create(int32_t nprob, const hopf_problem_t* problems, const int64_t* pt_offset,
                                    const void* x_packed, const void* t, void* phi, void* grad_packed, void* dphidt,
                                    int32_t* iters, int32_t* kstar, hopf_ragged_plan_t* out);
hopf_status hopf_ragged_plan_launch(hopf_ragged_plan_t plan, void* stream);
hopf_status hopf_ragged_plan_destroy(hopf_ragged_plan_t plan);

/* Ragged batch of closest points and distances (section 3.2, the Newton iteration on s of
 * eq. Newton_zero, with the inner evaluations of section 3.1): hopf_closest_point over nprob
 * ellipsoid level-set problems (level_set = 1, quadratic J; one precision for all, not
 * HOPF_F64) in the launches of hopf_eval_ragged.  pt_offset as there; y_packed and cp_packed
 * hold the points of problem q contiguously (n_q floats each) in problem order; dist, kstar,
 * inside and newton are indexed by the global point index (inside, newton nullable).  Results
 * and errors as hopf_closest_point, per problem. */
hopf_status hopf_closest_point_ragged(int32_t nprob, const hopf_problem_t* problems, const int64_t* pt_offset,
                                      const void* y_packed, double s_tol, void* dist, void* cp_packed,
                                      int32_t* kstar, int32_t* inside, int32_t* newton, void* stream);

/* Envelope-theorem gradients of L = sum_j gphi_j phi_j (phi is the optimal
 * value of eq. (3.3), an objective affine in x, t, A and c_k at fixed p):
 *   gx[j] = gphi_j p*_j,  gt[j] = gphi_j dphidt_j (= -gphi_j H(p*_j)),
 *   gA = -1/2 sum_j gphi_j p*_j p*_j^T (n*n, row-major),
 *   gc[k] = -sum_{j: kstar_j = k} gphi_j p*_j (K*n).
 * grad_saved, dphidt_saved, kstar_saved are hopf_eval's outputs.  Any output
 * may be NULL.  gA and gc are overwritten (not accumulated).  kstar_saved may
 * be NULL when K == 1. */
hopf_status hopf_backward(hopf_problem_t problem, int64_t npts, const void* gphi,
                          const void* grad_saved, const void* dphidt_saved,
                          const int32_t* kstar_saved, void* gx, void* gt, void* gA, void* gc,
                          void* stream);

/* hopf_backward for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same arguments, results
 * and kernels, with the split partials of the sums in a fixed 32 MiB device array that
 * the library holds on every GPU it runs on until the process ends, instead of the
 * per-device workspace.  No device or host memory is allocated by this call.  The gA
 * partials of one point range take 16 KiB per 64 x 64 tile of gA's lower triangle and
 * must fit beside the gc partials (at most a quarter of the array), which holds for
 * n <= 3456 (every problem the library accepts, n <= 2048); larger sizes would return
 * HOPF_EINVAL.  Point counts are not limited: the number of point ranges is reduced to
 * what fits (results then differ from hopf_backward's only by the order of the sums;
 * for n <= 256 and K <= 8 the counts, and so the bits, are the same).  The array keeps the last call's
 * contents; every byte a call reads was written by that call.  Calls that overlap on one
 * GPU (several streams or threads) race on the array: serialise them. */
hopf_status hopf_backward_noalloc(hopf_problem_t problem, int64_t npts, const void* gphi,
                                  const void* grad_saved, const void* dphidt_saved,
                                  const int32_t* kstar_saved, void* gx, void* gt, void* gA, void* gc,
                                  void* stream);

/* Optimal-control read-out (section 2, optimal control): from the points x (npts*n), times t
 * (npts) and an evaluation's grad (npts*n, p*) and kstar (npts; nullable when K = 1), writes the
 * terminal value xT = c_k* + A p* (the Hopf-Lax minimiser, where p* is a subgradient of J_k*) and
 * the control beta = (x - xT) / t, which equals grad H(p*) wherever H is differentiable at p*
 * (otherwise it is the subgradient of H at p* that the optimality of p* selects).  Needs the
 * quadratic J; I/O in the problem's precision (double for HOPF_F64).  Points with kstar < 0
 * (invalid inputs) get NaN.  A dense A is held in FP32 for this read-out. */
hopf_status hopf_control(hopf_problem_t problem, int64_t npts, const void* x, const void* t, const void* grad,
                         const int32_t* kstar, void* beta, void* xT, void* stream);

/* The minimum of Hamiltonians (section 2, extensions): for one J and Hamiltonians H_1..H_k
 * (k <= 16), phi for H = min_i H_i is max_i phi_i.  Given the k evaluations of the same npts
 * points (host arrays of k device pointers: phi_i (npts), grad_i (npts*n), dphidt_i (npts)),
 * writes phi = max_i phi_i and the grad and dphidt of the attaining i (lowest index on ties), and
 * istar (npts, nullable).  f64 != 0: double arrays, else float. */
hopf_status hopf_max_over_hamiltonians(int32_t k, int64_t npts, int32_t n, int32_t f64, const void* const* phis,
                                       const void* const* grads, const void* const* dphidts, void* phi,
                                       void* grad, void* dphidt, int32_t* istar, void* stream);

/* Work done for the problem so far: *total = the number of split-Bregman passes (each one
 * product with M = (A + lambda I)^{-1}, the v-update of eq. (3.4a)) summed over every column the
 * dense solvers ran for it: every copy of a union of level sets (section 3.1), every Newton solve
 * of a distance (section 3.2), every call since creation or the last reset.  Counted on the device
 * when a column finishes; the diagonal per-thread path does not count (its per-point iteration
 * count is the total).  Synchronises the device.  reset != 0 then clears the count.
 * Errors: HOPF_EINVAL for a NULL argument, HOPF_EDEVICE. */
hopf_status hopf_problem_iterations(hopf_problem_t problem, int64_t* total, int32_t reset);

/* Device-side factor of the problem, for inspection and tests: copies
 * M = (A + lambda I)^{-1} (n*n, row-major, FP64) to the host array out.  For a HOPF_H_AL2
 * problem this is the factor of the problem in HA's eigenbasis, (P^T A P + lambda I)^{-1}. */
hopf_status hopf_problem_get_inverse(hopf_problem_t problem, double* out);

/* Problem dimension, padded dimension, K, precision; any pointer may be NULL. */
hopf_status hopf_problem_info(hopf_problem_t problem, int32_t* n, int32_t* n_pad, int32_t* K,
                              int32_t* precision);

/* Deterministic mode of the dense evaluations (hopf_eval, hopf_closest_point, their ragged
 * forms and plans; the per-point diagonal kernels are deterministic already): on = 1 makes
 * every later launch (a plan: every plan created later) give the same bits in every output,
 * run after run and replay after replay, for the same problems and arguments on the same
 * device; on = 0 (the default) restores the fastest schedule, whose results agree to the
 * parity tolerances but not bit for bit.  Split Bregman's points are independent (section 3),
 * but a dense workgroup iterates a tile of columns together and re-bases their anchors
 * together, so a column's rounding depends on the columns it shares a tile with; by default
 * workgroups take chunks of columns from a shared counter as they free up, which makes that
 * company depend on timing.  In deterministic mode workgroup (or wave) u of U takes the
 * chunks u, u + U, u + 2U, ... instead, which can leave some compute units idle at the end of
 * a launch.  The value sums are always added in a fixed order.  The setting is process-wide
 * (an atomic flag read when a launch or plan is built).  Errors: HOPF_EINVAL for on other
 * than 0 or 1. */
hopf_status hopf_set_deterministic(int32_t on);
/* The current setting (0 or 1). */
int32_t hopf_get_deterministic(void);

/* Thread-local message for the last non-OK status returned on this thread. */
const char* hopf_last_error(void);

/* Library version string. */
const char* hopf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HOPF_H */
