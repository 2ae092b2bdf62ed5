/* Driver of the FP64 oracle (oracle/hopf_oracle.c) for the sanitizer build of
 * tests/test_host_checks.py: gcc with the address and undefined-behaviour
 * sanitizers, every Hamiltonian and initial-data kind, unions, both distance
 * routes, one and several threads, on small seeded problems.  It checks only
 * that everything runs clean and returns finite values; the oracle's numbers
 * are pinned by tests/test_oracle_pins.py. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/hopf_oracle.h"

static unsigned long long rng_state = 160501799ull;
static double urand(void) { /* xorshift64*, uniform in [0, 1) */
  rng_state ^= rng_state >> 12; rng_state ^= rng_state << 25; rng_state ^= rng_state >> 27;
  return (double)((rng_state * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}

static int failures = 0;

static void check_finite(const char* name, const double* v, long m) {
  for (long i = 0; i < m; ++i)
    if (!isfinite(v[i])) { printf("FAIL %s: entry %ld not finite\n", name, i); ++failures; return; }
}

int main(void) {
  enum { N = 5, P = 7, K = 3 };
  double A[N * N], HA[N * N], HQ[N * N], Hsig[N], w[N], C[K * N], x[P * N], t[P];
  memset(A, 0, sizeof A); memset(HA, 0, sizeof HA); memset(HQ, 0, sizeof HQ);
  for (int i = 0; i < N; ++i) {
    for (int j = 0; j < N; ++j) A[i * N + j] = 0.1 / (1.0 + abs(i - j));
    A[i * N + i] = 1.0 + i;  /* diagonally dominant: SPD */
    HA[i * N + i] = Hsig[i] = 0.5 + 0.25 * i;
    HQ[i * N + i] = 1.0;
    w[i] = 0.5 + urand();
  }
  for (int i = 0; i < K * N; ++i) C[i] = 3.0 * (urand() - 0.5);
  for (int i = 0; i < P * N; ++i) x[i] = 4.0 * (urand() - 0.5);
  for (int j = 0; j < P; ++j) t[j] = 0.05 + 2.0 * urand();
  double phi[P], grad[P * N], dphidt[P], gap[P];
  int32_t iters[P], kstar[P];

  const int hk[] = {OH_WL1, OH_L2, OH_L2_WL1, OH_WL2, OH_AL2, OH_LINF};
  for (int a = 0; a < 6; ++a)
    for (int jk = 0; jk < 3; ++jk)
      for (int th = 1; th <= 3; th += 2) {
        if (jk != OJ_QUAD && hk[a] == OH_AL2) continue;
        oh_problem pb;
        memset(&pb, 0, sizeof pb);
        pb.n = N; pb.A = A; pb.K = K; pb.centres = C; pb.level_set = jk == OJ_QUAD; pb.hkind = hk[a];
        pb.w = w; pb.lambda = 1.0; pb.tol = 1e-24; pb.max_iter = 20000; pb.jkind = jk;
        if (hk[a] == OH_AL2) { pb.HA = HA; pb.HQ = HQ; pb.Hsig = Hsig; }
        const int rc = oh_eval(&pb, P, x, t, phi, grad, dphidt, iters, kstar, gap, th);
        char name[64];
        snprintf(name, sizeof name, "eval H=%d J=%d threads=%d", hk[a], jk, th);
        if (rc != 0) { printf("FAIL %s: rc %d\n", name, rc); ++failures; continue; }
        check_finite(name, phi, P); check_finite(name, grad, (long)P * N); check_finite(name, dphidt, P);
        printf("ok %s\n", name);
      }
  { /* distances to a union of ellipsoids: the level-set route and the secular equation */
    double dist[P], cp[P * N], dist2[P], cp2[P * N], Q[N * N], sig[N];
    int32_t ks[P], ins[P], nw[P], ks2[P], ins2[P];
    oh_problem pb;
    memset(&pb, 0, sizeof pb);
    memset(Q, 0, sizeof Q);
    for (int i = 0; i < N; ++i) { Q[i * N + i] = 1.0; sig[i] = 1.0 + i; }
    double Ad[N * N];
    memset(Ad, 0, sizeof Ad);
    for (int i = 0; i < N; ++i) Ad[i * N + i] = sig[i];
    pb.n = N; pb.A = Ad; pb.K = K; pb.centres = C; pb.level_set = 1; pb.hkind = OH_L2; pb.lambda = 1.0;
    pb.tol = 1e-24; pb.max_iter = 20000;
    for (int th = 1; th <= 2; ++th) {
      if (oh_distance_newton(&pb, P, x, 1e-12, 50, dist, cp, ks, ins, nw, th) != 0) { printf("FAIL newton\n"); ++failures; }
      check_finite("distance (Newton on s)", dist, P);
      check_finite("closest point (Newton on s)", cp, (long)P * N);
    }
    if (oh_distance_secular(N, Q, sig, K, C, P, x, dist2, cp2, ks2, ins2) != 0) { printf("FAIL secular\n"); ++failures; }
    check_finite("distance (secular)", dist2, P);
    printf("ok distances\n");
  }
  { /* rejected arguments do not touch the outputs */
    oh_problem pb;
    memset(&pb, 0, sizeof pb);
    pb.n = 0;
    if (oh_eval(&pb, P, x, t, phi, grad, dphidt, iters, kstar, gap, 1) == 0) { printf("FAIL n = 0 accepted\n"); ++failures; }
    printf("ok rejected arguments\n");
  }
  printf("%s: %d failure(s)\n", failures ? "FAILED" : "PASSED", failures);
  return failures ? 1 : 0;
}
