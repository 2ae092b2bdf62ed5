#pragma once
#include <stddef.h>

#include "common.hpp"

namespace hopf {

struct BackwardArgs {
  int64_t npts;
  int n, K;
  const float* g; const float* grad; const float* dphidt; const int32_t* kstar;
  float* gx; float* gt; float* gA; float* gc;
};

// Split counts and scratch of one backward call: the gx / gt / gc pass runs splits_c workgroups
// (FP64 gc partials, bytes_c, at the start of the scratch), the gA GEMM splits_a point ranges of
// ntl lower 64 x 64 tiles (FP32 partials, bytes_a, after them).  The counts are reduced to fit
// cap_bytes; ok is false when even one split does not fit.
struct BackwardPlan {
  int ntl, splits_a, splits_c;
  size_t bytes_a, bytes_c;
  bool ok;
};
BackwardPlan backward_plan(int64_t npts, int n, int K, bool want_gA, bool want_gc, size_t cap_bytes);
hipError_t launch_backward(const BackwardArgs& a, const BackwardPlan& plan, void* scratch, hipStream_t stream);

}  // namespace hopf
