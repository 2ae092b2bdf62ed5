#pragma once
#include "checks.hpp"
#include "common.hpp"

namespace hopf {


struct DiagProb {
  int n, ld, K, level_set, hkind, max_iter;  // ld: stride of the centre rows
  int jkind;              // JK_QUAD: J = 1/2 sum y_i^2 / a_i; JK_L1SQ, JK_LINFSQ: squared norms
  double lambda, tol;
  const double* minv;     // n: 1 / (a_i + lambda)
  const double* adiag;    // n: a_i
  const double* w;        // n or null
  const double* centres;  // K*ld or null
  const double* P;        // HK_AL2: eigenvectors of HA (n x n, row-major, columns the vectors); else null
  const double* drift;    // HK_LINCTRL: the n diagonal entries m_i of the drift matrix M; else null
  const void* x; const void* t;
  int64_t npts;
  void* phi; void* grad; void* dphidt; int32_t* iters; int32_t* kstar;
};

// counter: one device int of scratch (the persistent kernel's point queue; reset here on the
// stream), ncu: compute units of the device.
hipError_t launch_diag(const DiagProb& pb, bool f64, int* counter, int ncu, hipStream_t stream);

}  // namespace hopf
