// Envelope-theorem backward pass.  phi_j is the optimal value of eq. (3.3);
// at fixed p its objective J*(p) + t H(p) - <x, p> (with J_k*(p) =
// 1/2 p^T A p + <c_k, p> (+ 1/2)) is affine in x, t, A and c_k, so at the
// minimiser p*_j:
//   d phi/dx = p*,  d phi/dt = -H(p*),  d phi/dA = -1/2 p* p*^T,  d phi/dc_{k*} = -p*.
// gA and gc are sums over points: split over point ranges into FP64 partials,
// then reduced in a fixed order (deterministic).
#include "common.hpp"
#include "backward.hpp"

namespace hopf {

__global__ void bw_pointwise_kernel(int64_t npts, int n, const float* g, const float* grad,
                                    const float* dphidt, float* gx, float* gt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= npts * n) return;
  const int64_t j = e / n;
  if (gx) gx[e] = g[j] * grad[e];
  if (gt && e % n == 0) gt[j] = g[j] * dphidt[j];
}

// gA partial: tile (bi, bj) of 32x32, points [p0, p1) of split s.
constexpr int BT = 32;
__global__ void __launch_bounds__(kBlock) bw_gA_partial_kernel(int64_t npts, int n, int ntile, int64_t chunk,
                                                               const float* g, const float* grad,
                                                               double* part) {
  const int tile = blockIdx.x, split = blockIdx.y;
  const int bi = tile / ntile, bj = tile % ntile;
  const int64_t p0 = (int64_t)split * chunk;
  const int64_t p1 = p0 + chunk < npts ? p0 + chunk : npts;
  __shared__ float Pi[64][BT + 1];
  __shared__ float Pj[64][BT + 1];
  const int tid = threadIdx.x;
  const int ti = tid / 16, tj = tid % 16;  // each thread: rows 2ti..2ti+1, cols 2tj..2tj+1
  double acc[2][2] = {{0, 0}, {0, 0}};
  for (int64_t b0 = p0; b0 < p1; b0 += 64) {
    for (int e = tid; e < 64 * BT; e += kBlock) {
      const int pp = e / BT, q = e % BT;
      const int64_t j = b0 + pp;
      const int ii = bi * BT + q, jj = bj * BT + q;
      float gj = (j < p1) ? g[j] : 0.f;
      Pi[pp][q] = (j < p1 && ii < n) ? gj * grad[j * n + ii] : 0.f;
      Pj[pp][q] = (j < p1 && jj < n) ? grad[j * n + jj] : 0.f;
    }
    __syncthreads();
    for (int pp = 0; pp < 64; ++pp) {
      const double a0 = Pi[pp][2 * ti], a1 = Pi[pp][2 * ti + 1];
      const double b0v = Pj[pp][2 * tj], b1v = Pj[pp][2 * tj + 1];
      acc[0][0] += a0 * b0v; acc[0][1] += a0 * b1v;
      acc[1][0] += a1 * b0v; acc[1][1] += a1 * b1v;
    }
    __syncthreads();
  }
  const int64_t nn = (int64_t)n * n;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const int ii = bi * BT + 2 * ti + a, jj = bj * BT + 2 * tj + b;
      if (ii < n && jj < n) part[(int64_t)split * nn + (int64_t)ii * n + jj] = acc[a][b];
    }
}

__global__ void bw_reduce_kernel(int64_t m, int nsplit, const double* part, double scale, float* out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  double s = 0.0;
  for (int q = 0; q < nsplit; ++q) s += part[(int64_t)q * m + e];
  out[e] = (float)(scale * s);
}

// gc partial: per split s, per (k, i): sum over points j of the split with kstar_j == k of g_j p_ji.
// One pass over the points of the split: for K <= KMAX the K sums of coordinate i stay in
// registers (each point adds to the sum of its own attaining copy); larger K loop over k.
template <int KMAX>
__global__ void bw_gc_partial_kernel(int64_t npts, int n, int K, int64_t chunk, const float* g,
                                     const float* grad, const int32_t* kstar, double* part) {
  const int split = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t p0 = (int64_t)split * chunk;
  const int64_t p1 = p0 + chunk < npts ? p0 + chunk : npts;
  if (K <= KMAX) {
    double s[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) s[k] = 0.0;
    for (int64_t j = p0; j < p1; ++j) {
      const int kk = kstar ? kstar[j] : 0;
      const double v = (double)g[j] * (double)grad[j * n + i];
#pragma unroll
      for (int k = 0; k < KMAX; ++k) s[k] += (kk == k) ? v : 0.0;
    }
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
      if (k < K) part[((int64_t)split * K + k) * n + i] = s[k];
    return;
  }
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (int64_t j = p0; j < p1; ++j) {
      const int kk = kstar ? kstar[j] : 0;
      if (kk == k) s += (double)g[j] * (double)grad[j * n + i];
    }
    part[((int64_t)split * K + k) * n + i] = s;
  }
}

hipError_t launch_backward(const BackwardArgs& a, double* scratch, hipStream_t stream) {
  const int64_t npts = a.npts;
  const int n = a.n;
  if (npts == 0) {
    if (a.gA) { hipError_t e = hipMemsetAsync(a.gA, 0, sizeof(float) * n * n, stream); if (e) return e; }
    if (a.gc) { hipError_t e = hipMemsetAsync(a.gc, 0, sizeof(float) * a.K * n, stream); if (e) return e; }
    return hipSuccess;
  }
  if (a.gx || a.gt) {
    const int64_t tot = npts * n;
    hipLaunchKernelGGL(bw_pointwise_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, stream,
                       npts, n, a.g, a.grad, a.dphidt, a.gx, a.gt);
  }
  const int nsplit = backward_splits(npts);
  const int64_t chunk = (npts + nsplit - 1) / nsplit;
  if (a.gA) {
    const int ntile = (n + BT - 1) / BT;
    hipLaunchKernelGGL(bw_gA_partial_kernel, dim3(ntile * ntile, nsplit), dim3(kBlock), 0, stream, npts, n,
                       ntile, chunk, a.g, a.grad, scratch);
    const int64_t m = (int64_t)n * n;
    hipLaunchKernelGGL(bw_reduce_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, stream, m, nsplit,
                       scratch, -0.5, a.gA);
  }
  if (a.gc) {
    double* sc = scratch + (a.gA ? (size_t)nsplit * n * n : 0);
    hipLaunchKernelGGL(bw_gc_partial_kernel<8>, dim3((n + 255) / 256, nsplit), dim3(256), 0, stream, npts, n,
                       a.K, chunk, a.g, a.grad, a.kstar, sc);
    const int64_t m = (int64_t)a.K * n;
    hipLaunchKernelGGL(bw_reduce_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, stream, m, nsplit,
                       sc, -1.0, a.gc);
  }
  return hipGetLastError();
}

int backward_splits(int64_t npts) {
  int64_t s = (npts + 4095) / 4096;
  if (s < 1) s = 1;
  if (s > 256) s = 256;
  return (int)s;
}

}  // namespace hopf
