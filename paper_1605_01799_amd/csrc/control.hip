// Read-outs on top of the evaluation (section 2):
//
//  * the optimal control and the terminal value.  For the quadratic initial data J_k(y) =
//    1/2 (y - c_k)^T A^{-1} (y - c_k) the Hopf-Lax minimiser ybar, the point where grad phi = p*
//    lies in dJ_k(ybar), is ybar = c_k + A p*; it is the terminal value x(T) of the optimal
//    trajectory, and the control is beta = (x - x(T)) / t (the paper's grad H(grad phi) wherever H
//    is differentiable at p*, otherwise the subgradient that the optimality of p* selects).
//  * the minimum of Hamiltonians: with one J and Hamiltonians H_1..H_k, phi for H = min_i H_i is
//    max_i phi_i, with the gradient and time derivative of the attaining i (the lowest on ties).
#include "common.hpp"
#include "control.hpp"

namespace hopf {

namespace {

// one thread per output coordinate (point j, row i); FP64 accumulation
template <typename T, bool DIAG>
__global__ void __launch_bounds__(kBlock) control_kernel(ControlArgs a, const T* __restrict__ x,
                                                         const T* __restrict__ t, const T* __restrict__ p,
                                                         T* __restrict__ beta, T* __restrict__ xT) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= a.npts * a.n) return;
  const int n = a.n;
  const int64_t j = e / n;
  const int i = (int)(e % n);
  const int k = a.kstar ? a.kstar[j] : 0;
  if (k < 0) {  // the point had no valid value (non-finite input or t <= 0)
    beta[e] = (T)__builtin_nan("");
    xT[e] = (T)__builtin_nan("");
    return;
  }
  const T* pj = p + j * n;
  double s;
  if (DIAG) {
    s = a.adiag[i] * (double)pj[i];
  } else {
    const float* Ai = a.Af + (size_t)i * n;
    s = 0.0;
    for (int m = 0; m < n; ++m) s += (double)Ai[m] * (double)pj[m];
  }
  const double y = (a.centres ? a.centres[(size_t)k * a.ldc + i] : 0.0) + s;
  xT[e] = (T)y;
  beta[e] = (T)(((double)x[e] - y) / (double)t[j]);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) max_h_kernel(MaxHArgs a, T* __restrict__ phi, T* __restrict__ grad,
                                                       T* __restrict__ dphidt, int32_t* __restrict__ istar) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= a.npts) return;
  int best = 0;
  T bv = ((const T*)a.phi[0])[j];
  for (int i = 1; i < a.k; ++i) {
    const T v = ((const T*)a.phi[i])[j];
    if (v > bv) { bv = v; best = i; }
  }
  phi[j] = bv;
  dphidt[j] = ((const T*)a.dphidt[best])[j];
  const T* g = (const T*)a.grad[best] + j * a.n;
  for (int i = 0; i < a.n; ++i) grad[j * a.n + i] = g[i];
  if (istar) istar[j] = best;
}

}  // namespace

hipError_t launch_control(const ControlArgs& a, bool f64, const void* x, const void* t, const void* p, void* beta,
                          void* xT, hipStream_t stream) {
  if (a.npts == 0) return hipSuccess;
  const unsigned grid = (unsigned)((a.npts * a.n + kBlock - 1) / kBlock);
  const bool diag = a.Af == nullptr;
  if (f64) {
    if (!diag) return hipErrorInvalidValue;  // FP64 problems are diagonal
    hipLaunchKernelGGL((control_kernel<double, true>), dim3(grid), dim3(kBlock), 0, stream, a, (const double*)x,
                       (const double*)t, (const double*)p, (double*)beta, (double*)xT);
  } else if (diag) {
    hipLaunchKernelGGL((control_kernel<float, true>), dim3(grid), dim3(kBlock), 0, stream, a, (const float*)x,
                       (const float*)t, (const float*)p, (float*)beta, (float*)xT);
  } else {
    hipLaunchKernelGGL((control_kernel<float, false>), dim3(grid), dim3(kBlock), 0, stream, a, (const float*)x,
                       (const float*)t, (const float*)p, (float*)beta, (float*)xT);
  }
  return hipGetLastError();
}

hipError_t launch_max_h(const MaxHArgs& a, bool f64, void* phi, void* grad, void* dphidt, int32_t* istar,
                        hipStream_t stream) {
  if (a.npts == 0) return hipSuccess;
  const unsigned grid = (unsigned)((a.npts + kBlock - 1) / kBlock);
  if (f64)
    hipLaunchKernelGGL((max_h_kernel<double>), dim3(grid), dim3(kBlock), 0, stream, a, (double*)phi, (double*)grad,
                       (double*)dphidt, istar);
  else
    hipLaunchKernelGGL((max_h_kernel<float>), dim3(grid), dim3(kBlock), 0, stream, a, (float*)phi, (float*)grad,
                       (float*)dphidt, istar);
  return hipGetLastError();
}

}  // namespace hopf
