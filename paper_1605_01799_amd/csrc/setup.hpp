#pragma once
#include "common.hpp"

namespace hopf {

struct SetupProb {
  double* S;      // n_pad*n_pad working matrix (becomes the inverse)
  double* P;      // 32*32 pivot-block inverse
  double* T;      // n_pad*32 copy of the column panel
  double* R;      // 32*n_pad new row panel
  int* status;    // set to 1 if a pivot block is not positive definite
  int n_pad;
  int pad;
};

hipError_t run_gauss_jordan(const SetupProb* d_probs, const int* h_nblocks, int nprob, int* d_prefix,
                            int* h_prefix, hipStream_t stream);
hipError_t launch_build_shifted(const double* A, int n, int n_pad, double lambda, double* S,
                                hipStream_t stream);
// b = (float)a, m entries
hipError_t launch_to_f32(const double* a, float* b, int64_t m, hipStream_t stream);
hipError_t launch_finalize_copies(const double* S, int n, int n_pad, double* Md, float* Mf, __bf16* Mb,
                                  hipStream_t stream);
// Integer slices of M (refined mode): kSlices * n_pad * pad64(n_pad) bytes and n_pad exponents.
hipError_t launch_slice_rows(const double* Md, int n_pad, int8_t* Mq, int32_t* Mqe, hipStream_t stream);
hipError_t launch_diag_inverse(const double* a, int n, int n_pad, double lambda, double* Md, float* Mf,
                               __bf16* Mb, double* minv_diag, hipStream_t stream);

}  // namespace hopf
