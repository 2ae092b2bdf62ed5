#pragma once
#include "checks.hpp"
#include "common.hpp"

namespace hopf {


// HA (n x n, FP64, device) = P diag(sig) P^T; P row-major with the eigenvectors as columns.
// *sweeps receives the number of Jacobi sweeps taken.
hipError_t launch_jacobi_eig(const double* HA, int n, double* P, double* sig, int* sweeps, hipStream_t stream);
// out = P^T A P (n x n, FP64, symmetrised); T is n x n scratch.
hipError_t launch_congruence(const double* A, const double* P, int n, double* T, double* out, hipStream_t stream);
// w[i] = sig[i] for i < n, 0 up to n_pad; wf the FP32 copy.
hipError_t launch_set_weights(const double* sig, int n, int n_pad, double* w, float* wf, hipStream_t stream);
// K centres (row stride ld): out_k = P^T in_k.
hipError_t launch_rotate_centres(const double* in, double* out, int64_t ld, const double* P, int n, int K,
                                 hipStream_t stream);
// Points (npts x n, FP32): xr_j = P^T x_j, and back p_j = P q_j.
hipError_t launch_rotate_points_in(const float* x, float* xr, const double* P, int n, int64_t npts,
                                   hipStream_t stream);
hipError_t launch_rotate_points_out(const float* q, float* p, const double* P, int n, int64_t npts,
                                    hipStream_t stream);

}  // namespace hopf
