// Per-problem FP64 setup: M = (A + lambda I)^{-1} on the device.
//
// Update (3.4a) is the resolvent of the quadratic J*(p) = 1/2 p^T A p, i.e. a
// solve with A + lambda I (section 4.1 gives the quadratic prox as
// (I + alpha A)^{-1}).  The solver applies it to many right-hand sides per
// iteration, so the inverse is formed once: block Gauss-Jordan elimination in
// FP64 on S = A + lambda I (symmetric positive definite, so no pivoting is
// needed and every pivot block is SPD), 32x32 blocks.  Each pivot block is
// inverted by Gauss-Jordan elimination, whose pivots double as the positive-
// definiteness test.  Problems of a batch are sorted by size so that the
// problems still active at step s form a prefix of the list.
#include "common.hpp"
#include "setup.hpp"

namespace hopf {

constexpr int NB = 32;

// Pivot block: P = S_KK^{-1} by Gauss-Jordan elimination without pivoting on the SPD block, one
// 256-thread workgroup per problem with the block in LDS (four entries per thread).  Step k turns
// column k into a unit column: with p = a_kk, a_kk <- 1/p, a_kj <- a_kj/p, a_ik <- -a_ik/p and
// a_ij <- a_ij - a_ik a_kj/p (i, j != k); after the NB steps the block holds its inverse.  The
// pivots p are the diagonal of the block's LDL^T factorisation, so all of them are positive
// exactly when the block is positive definite: that is the definiteness test (a failed pivot is
// replaced by 1 so that the rest stays finite, and the problem is flagged).
constexpr int kPivThreads = 256;
__global__ void __launch_bounds__(kPivThreads) gj_pivot_kernel(const SetupProb* probs, int nprob, int step) {
  const int q = blockIdx.x;
  if (q >= nprob) return;
  const SetupProb pb = probs[q];
  if (step * NB >= pb.n_pad) return;
  constexpr int kPer = NB * NB / kPivThreads;
  __shared__ double a[NB][NB + 1];
  __shared__ int bad;
  const int tid = threadIdx.x, k0 = step * NB;
  for (int e = tid; e < NB * NB; e += kPivThreads) {
    const int i = e / NB, j = e % NB;
    a[i][j] = pb.S[(size_t)(k0 + i) * pb.n_pad + k0 + j];
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int k = 0; k < NB; ++k) {
    double p = a[k][k];
    if (!(p > 0.0)) {
      p = 1.0;
      if (tid == 0) bad = 1;
    }
    const double ip = 1.0 / p;
    double v[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + kPivThreads * u, i = e / NB, j = e % NB;
      if (i == k) v[u] = (j == k) ? ip : a[k][j] * ip;
      else if (j == k) v[u] = -a[i][k] * ip;
      else v[u] = fma(-a[i][k], a[k][j] * ip, a[i][j]);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + kPivThreads * u;
      a[e / NB][e % NB] = v[u];
    }
    __syncthreads();
  }
  for (int e = tid; e < NB * NB; e += kPivThreads) pb.P[e] = a[e / NB][e % NB];
  if (tid == 0 && bad) *pb.status = 1;
}

// Panels: T = S[:, K] (copy of the old column panel), R = P * S[K, :] (new row panel).
// Grid: one workgroup per (problem, 32-block b) flattened; problems sorted by size.
__global__ void __launch_bounds__(kBlock) gj_panel_kernel(const SetupProb* probs, const int* blk_prefix,
                                                          int nactive, int step) {
  // find the problem of this block: blk_prefix[q] = sum_{r<q} nblocks_r over active problems
  int b = blockIdx.x;
  int lo = 0, hi = nactive;  // largest q with blk_prefix[q] <= b
  while (hi - lo > 1) { int mid = (lo + hi) / 2; if (blk_prefix[mid] <= b) lo = mid; else hi = mid; }
  const SetupProb pb = probs[lo];
  b -= blk_prefix[lo];
  const int ld = pb.n_pad, k0 = step * NB, r0 = b * NB;
  __shared__ double P[NB][NB + 1];
  __shared__ double Sk[NB][NB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < NB * NB; e += kBlock) {
    int i = e / NB, j = e % NB;
    P[i][j] = pb.P[i * NB + j];
    Sk[i][j] = pb.S[(size_t)(k0 + i) * ld + r0 + j];     // S[K rows][block b cols]
    pb.T[(size_t)(r0 + i) * NB + j] = pb.S[(size_t)(r0 + i) * ld + k0 + j];  // S[block b rows][K cols]
  }
  __syncthreads();
  for (int e = tid; e < NB * NB; e += kBlock) {
    int i = e / NB, j = e % NB;
    double s = 0.0;
    for (int m = 0; m < NB; ++m) s += P[i][m] * Sk[m][j];
    pb.R[(size_t)i * ld + r0 + j] = s;
  }
}

// Trailing update of every 32x32 tile (bi, bj):
//   bi != K, bj != K : S_ij -= T_i R_j ;  bj == K : S_iK = -T_i P ;  bi == K : S_Kj = R_j ;  S_KK = P.
__global__ void __launch_bounds__(kBlock) gj_update_kernel(const SetupProb* probs, const int* tile_prefix,
                                                           int nactive, int step) {
  int b = blockIdx.x;
  int lo = 0, hi = nactive;
  while (hi - lo > 1) { int mid = (lo + hi) / 2; if (tile_prefix[mid] <= b) lo = mid; else hi = mid; }
  const SetupProb pb = probs[lo];
  b -= tile_prefix[lo];
  const int ld = pb.n_pad, nb = pb.n_pad / NB, K = step;
  const int bi = b / nb, bj = b % nb;
  const int tid = threadIdx.x;
  __shared__ double Ti[NB][NB + 1];
  __shared__ double Rj[NB][NB + 1];
  if (bi == K && bj == K) {
    for (int e = tid; e < NB * NB; e += kBlock) {
      int i = e / NB, j = e % NB;
      pb.S[(size_t)(K * NB + i) * ld + K * NB + j] = pb.P[i * NB + j];
    }
    return;
  }
  if (bi == K) {
    for (int e = tid; e < NB * NB; e += kBlock) {
      int i = e / NB, j = e % NB;
      pb.S[(size_t)(K * NB + i) * ld + bj * NB + j] = pb.R[(size_t)i * ld + bj * NB + j];
    }
    return;
  }
  for (int e = tid; e < NB * NB; e += kBlock) {
    int i = e / NB, j = e % NB;
    Ti[i][j] = pb.T[(size_t)(bi * NB + i) * NB + j];
    Rj[i][j] = (bj == K) ? pb.P[i * NB + j] : pb.R[(size_t)i * ld + bj * NB + j];
  }
  __syncthreads();
  // T_i R_j by FP64 MFMA 16x16x4: wave w takes the 16 x 16 quadrant (w / 2, w % 2), eight k-steps.
  // Operands: A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k; the output's row i sits in lane
  // j + 16 (i % 4), register i / 4.
  static_assert(kBlock == 256 && NB == 32, "four waves, one 16 x 16 quadrant of the 32 x 32 tile each");
  const int wave = tid >> 6, l = tid & 63, wi = wave >> 1, wj = wave & 1;
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ks = 0; ks < NB / 4; ++ks)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Ti[16 * wi + (l & 15)][4 * ks + (l >> 4)],
                                              Rj[4 * ks + (l >> 4)][16 * wj + (l & 15)], acc, 0, 0, 0);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = 16 * wi + 4 * v + (l >> 4), j = 16 * wj + (l & 15);
    double* dst = &pb.S[(size_t)(bi * NB + i) * ld + bj * NB + j];
    *dst = (bj == K) ? -acc[v] : (*dst - acc[v]);
  }
}

// S = A + lambda I (identity on the padding) from a dense FP64 A (n x n, row-major).
__global__ void build_shifted_kernel(const double* A, int n, int n_pad, double lambda, double* S) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n_pad * n_pad) return;
  int i = (int)(e / n_pad), j = (int)(e % n_pad);
  double v;
  if (i < n && j < n) v = A[(size_t)i * n + j] + (i == j ? lambda : 0.0);
  else v = (i == j) ? 1.0 : 0.0;
  S[e] = v;
}

// M copies from the finished inverse: symmetrised, zero outside n x n.
__global__ void finalize_copies_kernel(const double* S, int n, int n_pad, double* Md, float* Mf,
                                       __bf16* Mb) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n_pad * n_pad) return;
  int i = (int)(e / n_pad), j = (int)(e % n_pad);
  double v = 0.0;
  if (i < n && j < n) v = 0.5 * (S[(size_t)i * n_pad + j] + S[(size_t)j * n_pad + i]);
  if (Md) Md[e] = v;
  if (Mf) Mf[mf_index(i, j, n_pad)] = (float)v;
  if (Mb) Mb[mb_index(i, j, n_pad)] = to_bf16((float)v);
}

// Integer slices of M for the refined solver's exact anchor products (layout and scale: the
// kSlices definitions).  One workgroup per row: its largest |M_ik| fixes the row exponent, then
// every entry is split by repeated scaling by 2^7 and rounding (each step exact in FP64).
__global__ void __launch_bounds__(kBlock) slice_rows_kernel(const double* Md, int n_pad, int8_t* Mq,
                                                            int32_t* Mqe) {
  __shared__ double red[kBlock];
  const int i = blockIdx.x, tid = threadIdx.x;
  const int n64 = pad64(n_pad), nks = n64 >> 6, RT = n_pad >> 4;
  const double* row = Md + (size_t)i * n_pad;
  double m = 0.0;
  for (int k = tid; k < n_pad; k += kBlock) m = fmax(m, fabs(row[k]));
  red[tid] = m;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
    __syncthreads();
  }
  const int ex = slice_exponent(red[0]);
  if (tid == 0) Mqe[i] = ex;
  const size_t slice_bytes = (size_t)n_pad * n64;
  for (int k = tid; k < n64; k += kBlock) {
    double x = k < n_pad ? ldexp(row[k], -ex) : 0.0;
    const size_t unit = ((size_t)(i >> 4) * nks + (k >> 6)) * 64 + (i & 15) + 16 * ((k & 63) >> 4);
    for (int a = 0; a < kSlices; ++a) {
      x *= 128.0;
      const double r = rint(x);
      x -= r;
      Mq[a * slice_bytes + unit * 16 + (k & 15)] = (int8_t)(int)r;
    }
  }
}

// Diagonal A: M = diag(1 / (a_i + lambda)).
__global__ void diag_inverse_kernel(const double* a, int n, int n_pad, double lambda, double* Md,
                                    float* Mf, __bf16* Mb, double* minv_diag) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n_pad * n_pad) return;
  int i = (int)(e / n_pad), j = (int)(e % n_pad);
  double v = (i == j && i < n) ? 1.0 / (a[i] + lambda) : 0.0;
  if (Md) Md[e] = v;
  if (Mf) Mf[mf_index(i, j, n_pad)] = (float)v;
  if (Mb) Mb[mb_index(i, j, n_pad)] = to_bf16((float)v);
  if (minv_diag && i == j && i < n) minv_diag[i] = v;
}

// ---------------------------------------------------------------------------
// Host driver for a batch of dense problems (already sorted by n_pad, descending).
// ---------------------------------------------------------------------------
hipError_t run_gauss_jordan(const SetupProb* d_probs, const int* h_nblocks, int nprob, int* d_prefix,
                            int* h_prefix, hipStream_t stream) {
  // h_prefix / d_prefix hold, for every step s, the block and tile prefix sums over the
  // problems still active at s (sizes: steps * 2 * (nprob + 1)).  One blocking copy.
  if (nprob == 0) return hipSuccess;
  const int max_steps = h_nblocks[0];
  const size_t stride = 2 * (size_t)(nprob + 1);
  for (int s = 0; s < max_steps; ++s) {
    int* hb = h_prefix + s * stride;
    int* ht = hb + nprob + 1;
    hb[0] = 0; ht[0] = 0;
    for (int q = 0; q < nprob; ++q) {
      int a = h_nblocks[q] > s ? 1 : 0;
      hb[q + 1] = hb[q] + a * h_nblocks[q];
      ht[q + 1] = ht[q] + a * h_nblocks[q] * h_nblocks[q];
    }
  }
  hipError_t e = hipMemcpyAsync(d_prefix, h_prefix, sizeof(int) * stride * max_steps,
                                hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(stream);  // h_prefix may be reused by the caller after return
  if (e != hipSuccess) return e;
  for (int s = 0; s < max_steps; ++s) {
    int nactive = 0;
    while (nactive < nprob && h_nblocks[nactive] > s) ++nactive;
    const int* hb = h_prefix + s * stride;
    const int* ht = hb + nprob + 1;
    const int* db = d_prefix + s * stride;
    const int* dt = db + nprob + 1;
    hipLaunchKernelGGL(gj_pivot_kernel, dim3(nactive), dim3(kPivThreads), 0, stream, d_probs, nactive, s);
    hipLaunchKernelGGL(gj_panel_kernel, dim3(hb[nactive]), dim3(kBlock), 0, stream, d_probs, db,
                       nactive, s);
    hipLaunchKernelGGL(gj_update_kernel, dim3(ht[nactive]), dim3(kBlock), 0, stream, d_probs, dt,
                       nactive, s);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

__global__ void to_f32_kernel(const double* __restrict__ a, float* __restrict__ b, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) b[i] = (float)a[i];
}

hipError_t launch_to_f32(const double* a, float* b, int64_t m, hipStream_t stream) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(to_f32_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, stream, a, b, m);
  return hipGetLastError();
}

hipError_t launch_build_shifted(const double* A, int n, int n_pad, double lambda, double* S,
                                hipStream_t stream) {
  int64_t tot = (int64_t)n_pad * n_pad;
  hipLaunchKernelGGL(build_shifted_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, stream,
                     A, n, n_pad, lambda, S);
  return hipGetLastError();
}

hipError_t launch_finalize_copies(const double* S, int n, int n_pad, double* Md, float* Mf, __bf16* Mb,
                                  hipStream_t stream) {
  int64_t tot = (int64_t)n_pad * n_pad;
  hipLaunchKernelGGL(finalize_copies_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, stream,
                     S, n, n_pad, Md, Mf, Mb);
  return hipGetLastError();
}

hipError_t launch_slice_rows(const double* Md, int n_pad, int8_t* Mq, int32_t* Mqe, hipStream_t stream) {
  hipLaunchKernelGGL(slice_rows_kernel, dim3((unsigned)n_pad), dim3(kBlock), 0, stream, Md, n_pad, Mq, Mqe);
  return hipGetLastError();
}

hipError_t launch_diag_inverse(const double* a, int n, int n_pad, double lambda, double* Md, float* Mf,
                               __bf16* Mb, double* minv_diag, hipStream_t stream) {
  int64_t tot = (int64_t)n_pad * n_pad;
  hipLaunchKernelGGL(diag_inverse_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, stream,
                     a, n, n_pad, lambda, Md, Mf, Mb, minv_diag);
  return hipGetLastError();
}

}  // namespace hopf
