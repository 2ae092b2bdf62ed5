#pragma once
#include "common.hpp"

namespace hopf {

// The control read-out of one problem: x(T) = c_k* + A p*, beta = (x - x(T)) / t.
struct ControlArgs {
  int n = 0;
  int64_t npts = 0;
  const float* Af = nullptr;        // n x n FP32 row-major copy of A, or null for a diagonal A
  const double* adiag = nullptr;    // n (diagonal A)
  const double* centres = nullptr;  // K x ldc, or null
  int ldc = 0;
  const int32_t* kstar = nullptr;   // npts, or null (copy 0); a negative entry marks an invalid point
};

constexpr int kMaxHamiltonians = 16;

// max over k evaluations of the same points (phi_i, grad_i npts x n, dphidt_i)
struct MaxHArgs {
  const void* phi[kMaxHamiltonians];
  const void* grad[kMaxHamiltonians];
  const void* dphidt[kMaxHamiltonians];
  int k = 0;
  int n = 0;
  int64_t npts = 0;
};

hipError_t launch_control(const ControlArgs& a, bool f64, const void* x, const void* t, const void* p, void* beta,
                          void* xT, hipStream_t stream);
hipError_t launch_max_h(const MaxHArgs& a, bool f64, void* phi, void* grad, void* dphidt, int32_t* istar,
                        hipStream_t stream);

}  // namespace hopf
