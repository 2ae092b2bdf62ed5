// Driver of the C ABI's host-side argument checks (paper_1605_01799_amd/csrc/checks.cpp), built by
// tests/test_host_checks.py with g++ under the address and undefined-behaviour sanitizers.  It never
// touches a GPU: every call here is pure host code.  Prints one line per case and exits non-zero
// on the first unexpected status.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../paper_1605_01799_amd/csrc/checks.hpp"

using namespace hopf;

static int failures = 0;

static void expect(const char* name, hopf_status got, hopf_status want, const char* why) {
  const bool ok = got == want;
  std::printf("%s %s: status %d (want %d)%s%s\n", ok ? "ok" : "FAIL", name, (int)got, (int)want, why[0] ? " -- " : "",
              why);
  if (!ok) ++failures;
}

static void expect_msg(const char* name, hopf_status got, hopf_status want, const char* why, const char* part) {
  expect(name, got, want, why);
  if (!std::strstr(why, part)) {
    std::printf("FAIL %s: the message does not name %s\n", name, part);
    ++failures;
  }
}

static hopf_problem_desc base(int n) {
  hopf_problem_desc d;
  std::memset(&d, 0, sizeof d);
  d.n = n; d.K = 1; d.hkind = HOPF_H_WL1; d.lambda = 1.0; d.tol = 1e-12; d.max_iter = 100;
  d.precision = HOPF_F32; d.jkind = HOPF_J_QUADRATIC;
  return d;
}

int main() {
  char why[512];
  // ---- descriptors
  {
    hopf_problem_desc d = base(8);
    why[0] = 0; expect("identity A, F32", check_desc(&d, why, sizeof why), HOPF_OK, why);
    why[0] = 0; expect("NULL descriptor", check_desc(nullptr, why, sizeof why), HOPF_EINVAL, why);
    d.n = 0; why[0] = 0; expect("n = 0", check_desc(&d, why, sizeof why), HOPF_EINVAL, why);
    d.n = kMaxN + 1; why[0] = 0; expect("n too large", check_desc(&d, why, sizeof why), HOPF_EINVAL, why);
    d = base(8); d.K = kMaxK + 1; why[0] = 0; expect("K too large", check_desc(&d, why, sizeof why), HOPF_EINVAL, why);
    d = base(8); d.lambda = 0.0; why[0] = 0; expect("lambda = 0", check_desc(&d, why, sizeof why), HOPF_EINVAL, why);
    d = base(8); d.lambda = NAN; why[0] = 0; expect("lambda NaN", check_desc(&d, why, sizeof why), HOPF_EINVAL, why);
    d = base(8); d.tol = -1.0; why[0] = 0; expect("tol < 0", check_desc(&d, why, sizeof why), HOPF_EINVAL, why);
    d = base(8); d.max_iter = 0; why[0] = 0; expect("max_iter = 0", check_desc(&d, why, sizeof why), HOPF_EINVAL, why);
    d = base(8); { const int bad = 17; std::memcpy(&d.hkind, &bad, sizeof bad); } why[0] = 0; expect("unknown hkind", check_desc(&d, why, sizeof why), HOPF_EINVAL, why);
    d = base(8); { const int bad = 9; std::memcpy(&d.precision, &bad, sizeof bad); } why[0] = 0;
    expect("unknown precision", check_desc(&d, why, sizeof why), HOPF_EINVAL, why);
  }
  {  // weights, centres, A
    std::vector<double> w(8, 1.0), c(16, 0.5), A(64, 0.0), Ad(8, 2.0);
    for (int i = 0; i < 8; ++i) A[i * 8 + i] = 2.0;
    hopf_problem_desc d = base(8);
    d.w = w.data(); d.A = A.data(); d.K = 2; d.centres = c.data();
    why[0] = 0; expect("dense A, K = 2", check_desc(&d, why, sizeof why), HOPF_OK, why);
    w[3] = -1.0; why[0] = 0; expect("negative weight", check_desc(&d, why, sizeof why), HOPF_EINVAL, why);
    w[3] = INFINITY; why[0] = 0; expect("infinite weight", check_desc(&d, why, sizeof why), HOPF_EINVAL, why);
    w[3] = 0.0; d.hkind = HOPF_H_WL2; why[0] = 0;
    expect("zero weight for sqrt(<p, D p>)", check_desc(&d, why, sizeof why), HOPF_EINVAL, why);
    w[3] = 1.0; d.hkind = HOPF_H_WL1; c[15] = NAN; why[0] = 0;
    expect("NaN centre (last entry)", check_desc(&d, why, sizeof why), HOPF_EINVAL, why);
    c[15] = 0.5; A[1] = 0.5; why[0] = 0; expect("asymmetric A", check_desc(&d, why, sizeof why), HOPF_EINVAL, why);
    A[8] = 0.5; why[0] = 0; expect("symmetric A again", check_desc(&d, why, sizeof why), HOPF_OK, why);
    A[63] = NAN; why[0] = 0; expect("NaN in A (last entry)", check_desc(&d, why, sizeof why), HOPF_EINVAL, why);
    A[63] = 2.0;
    d.A = Ad.data(); d.A_is_diagonal = 1; Ad[7] = 0.0; why[0] = 0;
    expect("diagonal A with a zero", check_desc(&d, why, sizeof why), HOPF_ENOTSPD, why);
  }
  {  // a dense A over several 64 x 64 tiles with a ragged last one (n = 200): the one-pass check
     // finds every entry and reports the first offence in row-major order
    const int n = 200;
    std::vector<double> A((size_t)n * n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j <= i; ++j) A[(size_t)i * n + j] = A[(size_t)j * n + i] = (i == j) ? n : 1.0 / (1 + i + j);
    hopf_problem_desc d = base(n);
    d.A = A.data();
    auto at = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
    why[0] = 0; expect("symmetric A, n = 200", check_desc(&d, why, sizeof why), HOPF_OK, why);
    at(150, 10) += 1e-6; why[0] = 0;
    expect_msg("asymmetric lower entry (150, 10)", check_desc(&d, why, sizeof why), HOPF_EINVAL, why, "(150, 10)");
    at(150, 10) = at(10, 150); at(10, 150) -= 1e-6; why[0] = 0;
    expect_msg("asymmetric upper entry (10, 150)", check_desc(&d, why, sizeof why), HOPF_EINVAL, why, "(150, 10)");
    at(199, 198) += 1.0; why[0] = 0;
    expect_msg("two mismatches: the first in row order", check_desc(&d, why, sizeof why), HOPF_EINVAL, why,
               "(150, 10)");
    at(10, 150) = at(150, 10); at(199, 198) = at(198, 199); at(3, 190) = NAN; why[0] = 0;
    expect_msg("NaN in the upper triangle", check_desc(&d, why, sizeof why), HOPF_EINVAL, why, "A[790]");
    at(3, 190) = at(190, 3); at(130, 130) = INFINITY; why[0] = 0;
    expect_msg("infinite diagonal entry", check_desc(&d, why, sizeof why), HOPF_EINVAL, why, "A[26130]");
    at(130, 130) = n; why[0] = 0;
    expect("symmetric A again, n = 200", check_desc(&d, why, sizeof why), HOPF_OK, why);
  }
  {  // n = 1000: the block rows are split over host threads; offences in rows of different threads
    const int n = 1000;
    std::vector<double> A((size_t)n * n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j <= i; ++j) A[(size_t)i * n + j] = A[(size_t)j * n + i] = (i == j) ? n : 1.0 / (1 + i + j);
    hopf_problem_desc d = base(n);
    d.A = A.data();
    auto at = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
    why[0] = 0; expect("symmetric A, n = 1000", check_desc(&d, why, sizeof why), HOPF_OK, why);
    at(900, 700) += 1e-3; at(999, 5) -= 1e-3; why[0] = 0;
    expect_msg("two mismatches, n = 1000", check_desc(&d, why, sizeof why), HOPF_EINVAL, why, "(900, 700)");
    at(900, 700) = at(700, 900); at(999, 5) = at(5, 999); at(640, 641) = INFINITY; at(80, 3) = NAN; why[0] = 0;
    expect_msg("two non-finite entries, n = 1000", check_desc(&d, why, sizeof why), HOPF_EINVAL, why, "A[80003]");
    at(640, 641) = at(641, 640); at(80, 3) = at(3, 80); why[0] = 0;
    expect("symmetric A again, n = 1000", check_desc(&d, why, sizeof why), HOPF_OK, why);
  }
  {  // (H, J, precision, n) combinations
    hopf_problem_desc d = base(33);
    d.precision = HOPF_F64; why[0] = 0;
    expect("F64 beyond the per-thread path", check_desc(&d, why, sizeof why), HOPF_EINVAL, why);
    d = base(65); d.hkind = HOPF_H_WL2; why[0] = 0;
    expect("sqrt(<p, D p>) at n = 65 (tile kernel)", check_desc(&d, why, sizeof why), HOPF_OK, why);
    std::vector<double> A(64 * 64, 0.0);
    for (int i = 0; i < 64; ++i) A[i * 64 + i] = 1.5;
    d = base(64); d.A = A.data(); d.hkind = HOPF_H_WL2; why[0] = 0;
    expect("sqrt(<p, D p>), dense n = 64, F32", check_desc(&d, why, sizeof why), HOPF_OK, why);
    d.precision = HOPF_BF16_REFINED; why[0] = 0;
    expect("sqrt(<p, D p>), dense, refined", check_desc(&d, why, sizeof why), HOPF_OK, why);
    d = base(16); d.hkind = HOPF_H_AL2; why[0] = 0;
    expect("sqrt(<p, HA p>) without HA", check_desc(&d, why, sizeof why), HOPF_EINVAL, why);
    {
      std::vector<double> HA(65 * 65, 0.0), HA16(16 * 16, 0.0);
      for (int i = 0; i < 65; ++i) HA[i * 65 + i] = 2.0;
      for (int i = 0; i < 16; ++i) HA16[i * 16 + i] = 2.0;
      d = base(16); d.hkind = HOPF_H_AL2; d.HA = HA16.data(); d.precision = HOPF_BF16_REFINED; why[0] = 0;
      expect("sqrt(<p, HA p>), refined, n = 16", check_desc(&d, why, sizeof why), HOPF_OK, why);
      d = base(65); d.hkind = HOPF_H_AL2; d.HA = HA.data(); why[0] = 0;
      expect("sqrt(<p, HA p>), n = 65", check_desc(&d, why, sizeof why), HOPF_OK, why);
      d.precision = HOPF_F64; why[0] = 0;
      expect("sqrt(<p, HA p>), F64 beyond the per-thread path", check_desc(&d, why, sizeof why), HOPF_EINVAL, why);
    }
    {  // the time-dependent H of linear controls: per-thread path only, needs the drift
      std::vector<double> drift(40, 0.5), Ad(40, 1.5), A8(64, 0.0);
      for (int i = 0; i < 8; ++i) A8[i * 8 + i] = 2.0;
      d = base(8); d.hkind = HOPF_H_LINCTRL; d.drift = drift.data(); d.precision = HOPF_F64; why[0] = 0;
      expect("linear controls, A = I, F64", check_desc(&d, why, sizeof why), HOPF_OK, why);
      d.A = Ad.data(); d.A_is_diagonal = 1; d.precision = HOPF_F32; why[0] = 0;
      expect("linear controls, diagonal A, F32", check_desc(&d, why, sizeof why), HOPF_OK, why);
      d.precision = HOPF_BF16_REFINED; why[0] = 0;
      expect("linear controls, refined", check_desc(&d, why, sizeof why), HOPF_EINVAL, why);
      d.precision = HOPF_F64; d.drift = nullptr; why[0] = 0;
      expect("linear controls without the drift", check_desc(&d, why, sizeof why), HOPF_EINVAL, why);
      d.drift = drift.data(); drift[7] = NAN; why[0] = 0;
      expect("linear controls, NaN drift (last entry)", check_desc(&d, why, sizeof why), HOPF_EINVAL, why);
      drift[7] = 0.5;
      d.A = A8.data(); d.A_is_diagonal = 0; why[0] = 0;
      expect("linear controls, dense A", check_desc(&d, why, sizeof why), HOPF_EINVAL, why);
      d = base(33); d.hkind = HOPF_H_LINCTRL; d.drift = drift.data(); d.A = Ad.data(); d.A_is_diagonal = 1;
      why[0] = 0;
      expect("linear controls, n = 33", check_desc(&d, why, sizeof why), HOPF_EINVAL, why);
    }
    d = base(16); d.jkind = HOPF_J_L1SQ; d.hkind = HOPF_H_LINF; why[0] = 0;
    expect("1/2 |y|_1^2 with |p|_inf", check_desc(&d, why, sizeof why), HOPF_OK, why);
    d.precision = HOPF_BF16_REFINED; why[0] = 0;
    expect("squared norm, refined", check_desc(&d, why, sizeof why), HOPF_EINVAL, why);
  }
  // ---- column counts: npts * K must fit the device's 32-bit column numbers
  {
    const int64_t lim = kMaxColumns;
    why[0] = 0; expect("npts = 0", check_columns(0, 1, why, sizeof why), HOPF_OK, why);
    why[0] = 0; expect("npts < 0", check_columns(-1, 1, why, sizeof why), HOPF_EINVAL, why);
    why[0] = 0; expect("npts = 2^31 - 1, K = 1", check_columns(lim, 1, why, sizeof why), HOPF_OK, why);
    why[0] = 0; expect("npts = 2^31, K = 1", check_columns(lim + 1, 1, why, sizeof why), HOPF_EINVAL, why);
    why[0] = 0; expect("npts * 8 just below 2^31", check_columns(lim / 8, 8, why, sizeof why), HOPF_OK, why);
    why[0] = 0; expect("npts * 8 at 2^31", check_columns(lim / 8 + 1, 8, why, sizeof why), HOPF_EINVAL, why);
    why[0] = 0; expect("npts * 64 overflowing int64 if multiplied", check_columns((int64_t)1 << 58, 64, why, sizeof why),
                       HOPF_EINVAL, why);
    why[0] = 0; expect("K = 0", check_columns(10, 0, why, sizeof why), HOPF_EINVAL, why);
  }
  // ---- ragged members
  {
    why[0] = 0;
    expect("ragged: F32 weighted l1", check_ragged_member(0, HOPF_F32, HOPF_F32, HOPF_H_WL1, HOPF_J_QUADRATIC, 500, why, sizeof why),
           HOPF_OK, why);
    why[0] = 0;
    expect("ragged: mixed precision", check_ragged_member(3, HOPF_F32, HOPF_BF16_REFINED, HOPF_H_WL1, HOPF_J_QUADRATIC, 8, why, sizeof why),
           HOPF_EINVAL, why);
    why[0] = 0;
    expect("ragged: F64", check_ragged_member(0, HOPF_F64, HOPF_F64, HOPF_H_WL1, HOPF_J_QUADRATIC, 8, why, sizeof why),
           HOPF_EINVAL, why);
    why[0] = 0;
    expect("ragged: sqrt(<p, D p>) refined",
           check_ragged_member(1, HOPF_BF16_REFINED, HOPF_BF16_REFINED, HOPF_H_WL2, HOPF_J_QUADRATIC, 8, why, sizeof why),
           HOPF_OK, why);
    why[0] = 0;
    expect("ragged: sqrt(<p, D p>) F32, n = 32",
           check_ragged_member(1, HOPF_F32, HOPF_F32, HOPF_H_WL2, HOPF_J_QUADRATIC, 32, why, sizeof why), HOPF_OK, why);
    why[0] = 0;
    expect("ragged: sqrt(<p, D p>) F32, n = 500",
           check_ragged_member(1, HOPF_F32, HOPF_F32, HOPF_H_WL2, HOPF_J_QUADRATIC, 500, why, sizeof why), HOPF_OK, why);
    why[0] = 0;
    expect("ragged: linear controls",
           check_ragged_member(1, HOPF_F32, HOPF_F32, HOPF_H_LINCTRL, HOPF_J_QUADRATIC, 8, why, sizeof why), HOPF_EINVAL, why);
    why[0] = 0;
    expect("ragged: |p|_inf", check_ragged_member(2, HOPF_F32, HOPF_F32, HOPF_H_LINF, HOPF_J_QUADRATIC, 8, why, sizeof why),
           HOPF_EINVAL, why);
  }
  // ---- a message buffer of length 1 and a NULL buffer are both safe
  {
    char one[1] = {'x'};
    expect("1-byte message buffer", check_columns(-1, 1, one, sizeof one), HOPF_EINVAL, "");
    if (one[0] != 0) { std::printf("FAIL 1-byte buffer not terminated\n"); ++failures; }
    expect("NULL message buffer", check_columns(-1, 1, nullptr, 0), HOPF_EINVAL, "");
  }
  std::printf("%s: %d failure(s)\n", failures ? "FAILED" : "PASSED", failures);
  return failures ? 1 : 0;
}
