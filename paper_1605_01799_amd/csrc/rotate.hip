// The eigenbasis of the Hamiltonian's matrix for H(p) = sqrt(<p, HA p>) (section 4.3, the norm
// ||.||_A).  The paper projects onto the Wulff ellipsoid of HA as P pi_D(P^T w), HA = P D P^T.
// Here the rotation is applied to the whole problem once instead of twice per iteration: with
// p = P q,
//     J*(p) = 1/2 q^T (P^T A P) q,   H(p) = sqrt(q^T D q),   <x - c_k, p> = <P^T x - P^T c_k, q>,
// so the point is solved as the diagonal-weight problem (A' = P^T A P, w = diag D, x' = P^T x,
// c' = P^T c) and p = P q is rotated back.  phi and dphi/dt are invariant.
//
//  * jacobi_eig_kernel: HA = P diag(sig) P^T in FP64 by the cyclic Jacobi method, one workgroup,
//    the matrix and the accumulated rotations in LDS; each sweep visits every pair once in
//    m - 1 rounds of m / 2 disjoint rotations (round-robin order, m = n rounded up to even).
//  * congruence_kernel: A' = P^T A P (FP64, symmetrised).
//  * rotate_*: the per-point rotations (FP64 accumulation, P staged in LDS).
#include "common.hpp"
#include "rotate.hpp"

namespace hopf {

namespace {

constexpr int kJacobiMaxSweeps = 40;

__global__ void __launch_bounds__(kBlock) jacobi_eig_kernel(const double* __restrict__ HA, int n,
                                                            double* __restrict__ P, double* __restrict__ sig,
                                                            int* __restrict__ sweeps) {
  __shared__ double a[kRotMaxN][kRotMaxN + 1], v[kRotMaxN][kRotMaxN + 1];
  __shared__ double cs[kRotMaxN / 2][2];
  __shared__ int pq[kRotMaxN / 2][2];
  __shared__ double red[kBlock][2];
  __shared__ int done;
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += kBlock) {
    const int i = e / n, j = e % n;
    a[i][j] = 0.5 * (HA[(size_t)i * n + j] + HA[(size_t)j * n + i]);
    v[i][j] = i == j ? 1.0 : 0.0;
  }
  const int m = n + (n & 1);  // index n (odd n) is a dummy that pairs with nothing
  const int half = m / 2;
  __syncthreads();
  int sweep = 0;
  for (; sweep < kJacobiMaxSweeps; ++sweep) {
    // stop when the off-diagonal part is at FP64 rounding level of the diagonal
    double off = 0.0, dia = 0.0;
    for (int e = tid; e < n * n; e += kBlock) {
      const int i = e / n, j = e % n;
      const double x = a[i][j] * a[i][j];
      if (i == j) dia += x;
      else off += x;
    }
    red[tid][0] = off; red[tid][1] = dia;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
      if (tid < s) { red[tid][0] += red[tid + s][0]; red[tid][1] += red[tid + s][1]; }
      __syncthreads();
    }
    if (tid == 0) done = !(red[0][0] > 1e-30 * red[0][1]);
    __syncthreads();
    if (done) break;
    for (int r = 0; r < m - 1; ++r) {
      if (tid < half) {
        auto idx = [&](int k) { return k == 0 ? 0 : ((k - 1 + r) % (m - 1)) + 1; };
        const int p = idx(tid), q = idx(m - 1 - tid);
        double c = 1.0, s = 0.0;
        if (p < n && q < n && a[p][q] != 0.0) {
          // the rotation that zeroes a_pq: tan of its angle is the smaller root of
          // t^2 + 2 tau t - 1 = 0, tau = (a_qq - a_pp) / (2 a_pq)
          const double tau = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
        }
        pq[tid][0] = p; pq[tid][1] = q;
        cs[tid][0] = c; cs[tid][1] = s;
      }
      __syncthreads();
      // rows p, q of A <- J^T A (disjoint pairs touch disjoint rows)
      for (int e = tid; e < half * n; e += kBlock) {
        const int i = e / n, k = e % n;
        const int p = pq[i][0], q = pq[i][1];
        if (p >= n || q >= n) continue;
        const double c = cs[i][0], s = cs[i][1];
        const double x = a[p][k], y = a[q][k];
        a[p][k] = c * x - s * y;
        a[q][k] = s * x + c * y;
      }
      __syncthreads();
      // columns p, q of A <- A J and of V <- V J
      for (int e = tid; e < half * n; e += kBlock) {
        const int i = e / n, k = e % n;
        const int p = pq[i][0], q = pq[i][1];
        if (p >= n || q >= n) continue;
        const double c = cs[i][0], s = cs[i][1];
        const double x = a[k][p], y = a[k][q];
        a[k][p] = c * x - s * y;
        a[k][q] = s * x + c * y;
        const double vx = v[k][p], vy = v[k][q];
        v[k][p] = c * vx - s * vy;
        v[k][q] = s * vx + c * vy;
      }
      __syncthreads();
    }
  }
  for (int e = tid; e < n * n; e += kBlock) {
    const int i = e / n, j = e % n;
    P[(size_t)i * n + j] = v[i][j];
    if (i == j) sig[i] = a[i][i];
  }
  if (tid == 0) *sweeps = sweep;
}

// T = A P (pass 0) or out = sym(P^T T) (pass 1); one thread per output entry.
__global__ void __launch_bounds__(kBlock) congruence_kernel(const double* __restrict__ A,
                                                            const double* __restrict__ P, int n,
                                                            double* __restrict__ T, double* __restrict__ out,
                                                            int pass) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= n * n) return;
  const int i = e / n, j = e % n;
  if (pass == 0) {
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += A[(size_t)i * n + k] * P[(size_t)k * n + j];
    T[e] = s;
  } else {
    double s1 = 0.0, s2 = 0.0;
    for (int k = 0; k < n; ++k) {
      s1 += P[(size_t)k * n + i] * T[(size_t)k * n + j];
      s2 += P[(size_t)k * n + j] * T[(size_t)k * n + i];
    }
    out[e] = 0.5 * (s1 + s2);
  }
}

// w = sig (FP64 and FP32 copies, zero beyond n)
__global__ void set_weights_kernel(const double* __restrict__ sig, int n, int n_pad, double* __restrict__ w,
                                   float* __restrict__ wf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pad) return;
  const double s = i < n ? sig[i] : 0.0;
  w[i] = s;
  wf[i] = (float)s;
}

// rows of `in` (rows x n, stride ld_in) times P^T (TRANS: out_a = sum_i P_ia in_i) or P
// (out_i = sum_a P_ia in_a); FP64 accumulation, P staged in LDS; one thread per output entry.
template <typename TI, typename TO, bool TRANS>
__global__ void __launch_bounds__(kBlock) rotate_rows_kernel(const TI* __restrict__ in, int64_t ld_in,
                                                             TO* __restrict__ out, int64_t ld_out,
                                                             const double* __restrict__ P, int n, int64_t rows) {
  // P staged so that the threads of one point (consecutive output coordinates c) read
  // consecutive LDS words: as is for P^T (column c), transposed for P (row c)
  __shared__ double sP[kRotMaxN * kRotMaxN];
  for (int e = threadIdx.x; e < n * n; e += kBlock) sP[e] = TRANS ? P[e] : P[(e % n) * n + e / n];
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= rows * n) return;
  const int64_t j = e / n;
  const int c = (int)(e % n);
  const TI* x = in + j * ld_in;
  double s = 0.0;
  if (TRANS) {
    for (int i = 0; i < n; ++i) s += sP[i * n + c] * (double)x[i];
  } else {
    for (int a = 0; a < n; ++a) s += sP[a * n + c] * (double)x[a];
  }
  out[j * ld_out + c] = (TO)s;
}

template <typename TI, typename TO, bool TRANS>
hipError_t launch_rows(const TI* in, int64_t ld_in, TO* out, int64_t ld_out, const double* P, int n, int64_t rows,
                       hipStream_t stream) {
  if (rows == 0) return hipSuccess;
  if (n > kRotMaxN) return hipErrorInvalidValue;
  const int64_t tot = rows * n;
  hipLaunchKernelGGL((rotate_rows_kernel<TI, TO, TRANS>), dim3((unsigned)((tot + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, stream, in, ld_in, out, ld_out, P, n, rows);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_jacobi_eig(const double* HA, int n, double* P, double* sig, int* sweeps, hipStream_t stream) {
  if (n < 1 || n > kRotMaxN) return hipErrorInvalidValue;
  hipLaunchKernelGGL(jacobi_eig_kernel, dim3(1), dim3(kBlock), 0, stream, HA, n, P, sig, sweeps);
  return hipGetLastError();
}

hipError_t launch_congruence(const double* A, const double* P, int n, double* T, double* out, hipStream_t stream) {
  const unsigned g = (unsigned)((n * n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(congruence_kernel, dim3(g), dim3(kBlock), 0, stream, A, P, n, T, out, 0);
  hipLaunchKernelGGL(congruence_kernel, dim3(g), dim3(kBlock), 0, stream, A, P, n, T, out, 1);
  return hipGetLastError();
}

hipError_t launch_set_weights(const double* sig, int n, int n_pad, double* w, float* wf, hipStream_t stream) {
  hipLaunchKernelGGL(set_weights_kernel, dim3((n_pad + 63) / 64), dim3(64), 0, stream, sig, n, n_pad, w, wf);
  return hipGetLastError();
}

hipError_t launch_rotate_centres(const double* in, double* out, int64_t ld, const double* P, int n, int K,
                                 hipStream_t stream) {
  return launch_rows<double, double, true>(in, ld, out, ld, P, n, K, stream);
}

hipError_t launch_rotate_points_in(const float* x, float* xr, const double* P, int n, int64_t npts,
                                   hipStream_t stream) {
  return launch_rows<float, float, true>(x, n, xr, n, P, n, npts, stream);
}

hipError_t launch_rotate_points_out(const float* q, float* p, const double* P, int n, int64_t npts,
                                    hipStream_t stream) {
  return launch_rows<float, float, false>(q, n, p, n, P, n, npts, stream);
}

}  // namespace hopf
