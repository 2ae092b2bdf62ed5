#pragma once
#include "common.hpp"

namespace hopf {

struct BackwardArgs {
  int64_t npts;
  int n, K;
  const float* g; const float* grad; const float* dphidt; const int32_t* kstar;
  float* gx; float* gt; float* gA; float* gc;
};
// scratch: backward_splits(npts) * (n*n + K*n) doubles
int backward_splits(int64_t npts);
hipError_t launch_backward(const BackwardArgs& a, double* scratch, hipStream_t stream);

}  // namespace hopf
