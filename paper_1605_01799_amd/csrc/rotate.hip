// The eigenbasis of the Hamiltonian's matrix for H(p) = sqrt(<p, HA p>) (section 4.3, the norm
// ||.||_A).  The paper projects onto the Wulff ellipsoid of HA as P pi_D(P^T w), HA = P D P^T.
// Here the rotation is applied to the whole problem once instead of twice per iteration: with
// p = P q,
//     J*(p) = 1/2 q^T (P^T A P) q,   H(p) = sqrt(q^T D q),   <x - c_k, p> = <P^T x - P^T c_k, q>,
// so the point is solved as the diagonal-weight problem (A' = P^T A P, w = diag D, x' = P^T x,
// c' = P^T c) and p = P q is rotated back.  phi and dphi/dt are invariant.
//
//  * jacobi_eig_kernel: HA = P diag(sig) P^T in FP64 by the cyclic Jacobi method, one workgroup,
//    the matrix and the accumulated rotations in LDS (n <= kRotLdsN); each sweep visits every pair
//    once in m - 1 rounds of m / 2 disjoint rotations (round-robin order, m = n rounded up to even).
//  * jacobi_round_kernel (larger n): the same rounds with the matrix in global memory, one launch
//    per round over the whole device.
//  * congruence_kernel: A' = P^T A P (FP64, symmetrised).
//  * rotate_*: the per-point rotations (FP64 accumulation; P staged in LDS for n <= kRotLdsN, else
//    a tiled product over 64 x 64 output tiles).
#include <utility>

#include "common.hpp"
#include "rotate.hpp"

namespace hopf {

namespace {

constexpr int kJacobiMaxSweeps = 40;
constexpr int kRotLdsN = 64;  // the one-workgroup Jacobi and the LDS-staged rotations

__global__ void __launch_bounds__(kBlock) jacobi_eig_kernel(const double* __restrict__ HA, int n,
                                                            double* __restrict__ P, double* __restrict__ sig,
                                                            int* __restrict__ sweeps) {
  __shared__ double a[kRotLdsN][kRotLdsN + 1], v[kRotLdsN][kRotLdsN + 1];
  __shared__ double cs[kRotLdsN / 2][2];
  __shared__ int pq[kRotLdsN / 2][2];
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

// ---- the same method for larger n, the matrix in global memory
// Member k (0 <= k < m) of the round-robin schedule in round r: position 0 stays, the others turn.
__device__ __forceinline__ int rr_index(int k, int r, int m) { return k == 0 ? 0 : ((k - 1 + r) % (m - 1)) + 1; }
// The rotation of pair a in round r from the current matrix (identity for a pair with the dummy
// index n of odd n, or a zero off-diagonal entry); the same formula as the one-workgroup kernel.
__device__ __forceinline__ void rr_rotation(const double* A, int n, int m, int r, int a, int* p, int* q, double* c,
                                            double* s) {
  *p = rr_index(a, r, m);
  *q = rr_index(m - 1 - a, r, m);
  *c = 1.0; *s = 0.0;
  if (*p < n && *q < n) {
    const double apq = A[(size_t)*p * n + *q];
    if (apq != 0.0) {
      const double tau = (A[(size_t)*q * n + *q] - A[(size_t)*p * n + *p]) / (2.0 * apq);
      const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
      *c = 1.0 / sqrt(1.0 + t * t);
      *s = t * *c;
    }
  }
}
// One round: An = J^T A J and V <- V J for the round's m / 2 disjoint rotations J.  Entries e < h^2
// (h = m / 2) take the 2 x 2 block of rows {p_a, q_a} and columns {p_b, q_b} (a = e / h, b = e % h):
// rows rotated by pair a, then columns by pair b; entries h^2 + i h + a rotate row i of V in the
// columns of pair a.  A is only read, An only written, so blocks never see each other's output.
__global__ void __launch_bounds__(kBlock) jacobi_round_kernel(const double* __restrict__ A,
                                                              double* __restrict__ An,
                                                              double* __restrict__ V, int n, int m, int r) {
  const int h = m / 2;
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t nb = (int64_t)h * h;
  if (e < nb) {
    const int a = (int)(e / h), b = (int)(e % h);
    int pa, qa, pb, qb;
    double ca, sa, cb, sb;
    rr_rotation(A, n, m, r, a, &pa, &qa, &ca, &sa);
    rr_rotation(A, n, m, r, b, &pb, &qb, &cb, &sb);
    auto at = [&](int i, int j) { return (i < n && j < n) ? A[(size_t)i * n + j] : 0.0; };
    const double x00 = at(pa, pb), x01 = at(pa, qb), x10 = at(qa, pb), x11 = at(qa, qb);
    // rows: [p; q] <- [c p - s q; s p + c q]
    const double y00 = ca * x00 - sa * x10, y01 = ca * x01 - sa * x11;
    const double y10 = sa * x00 + ca * x10, y11 = sa * x01 + ca * x11;
    // columns likewise
    const double z00 = cb * y00 - sb * y01, z01 = sb * y00 + cb * y01;
    const double z10 = cb * y10 - sb * y11, z11 = sb * y10 + cb * y11;
    if (pa < n && pb < n) An[(size_t)pa * n + pb] = z00;
    if (pa < n && qb < n) An[(size_t)pa * n + qb] = z01;
    if (qa < n && pb < n) An[(size_t)qa * n + pb] = z10;
    if (qa < n && qb < n) An[(size_t)qa * n + qb] = z11;
  } else if (e < nb + (int64_t)n * h) {
    const int64_t f = e - nb;
    const int i = (int)(f / h), a = (int)(f % h);
    int p, q;
    double c, s;
    rr_rotation(A, n, m, r, a, &p, &q, &c, &s);
    if (p < n && q < n) {
      const double vx = V[(size_t)i * n + p], vy = V[(size_t)i * n + q];
      V[(size_t)i * n + p] = c * vx - s * vy;
      V[(size_t)i * n + q] = s * vx + c * vy;
    }
  }
}
// A = sym(HA), V = I
__global__ void jacobi_init_kernel(const double* __restrict__ HA, double* __restrict__ A, double* __restrict__ V,
                                   int n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int i = (int)(e / n), j = (int)(e % n);
  A[e] = 0.5 * (HA[(size_t)i * n + j] + HA[(size_t)j * n + i]);
  V[e] = i == j ? 1.0 : 0.0;
}
// sums[0] += off-diagonal squares, sums[1] += diagonal squares (sums cleared by the first thread
// of a separate launch)
__global__ void jacobi_clear_kernel(double* sums) {
  if (threadIdx.x < 2) sums[threadIdx.x] = 0.0;
}
__global__ void __launch_bounds__(kBlock) jacobi_norms_kernel(const double* __restrict__ A, int n,
                                                              double* __restrict__ sums) {
  __shared__ double red[kBlock][2];
  double off = 0.0, dia = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < (int64_t)n * n; e += (int64_t)gridDim.x * kBlock) {
    const double x = A[e] * A[e];
    if (e / n == e % n) dia += x;
    else off += x;
  }
  red[threadIdx.x][0] = off; red[threadIdx.x][1] = dia;
  __syncthreads();
  for (int k = kBlock / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) { red[threadIdx.x][0] += red[threadIdx.x + k][0]; red[threadIdx.x][1] += red[threadIdx.x + k][1]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) { atomicAdd(sums, red[0][0]); atomicAdd(sums + 1, red[0][1]); }
}
__global__ void jacobi_out_kernel(const double* __restrict__ A, const double* __restrict__ V, int n,
                                  double* __restrict__ P, double* __restrict__ sig) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  P[e] = V[e];
  if (e / n == e % n) sig[e / n] = A[e];
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
  __shared__ double sP[kRotLdsN * kRotLdsN];
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

// The same rotations for larger n: out (rows x n) = in B with B[k][c] = P[k n + c] (TRANS) or
// P[c n + k]; a 64 x 64 output tile per workgroup, 16-deep slabs of in and B staged in LDS (FP64),
// 4 x 4 outputs per thread.
template <typename TI, typename TO, bool TRANS>
__global__ void __launch_bounds__(kBlock) rotate_rows_tiled_kernel(const TI* __restrict__ in, int64_t ld_in,
                                                                   TO* __restrict__ out, int64_t ld_out,
                                                                   const double* __restrict__ P, int n,
                                                                   int64_t rows) {
  __shared__ double Xs[16][64 + 1], Bs[16][64 + 1];
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int c0 = blockIdx.y * 64;
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int k0 = 0; k0 < n; k0 += 16) {
    for (int e = tid; e < 64 * 16; e += kBlock) {  // 16 consecutive k of a row
      const int rr = e >> 4, kk = e & 15;
      const int64_t row = r0 + rr;
      const int k = k0 + kk;
      Xs[kk][rr] = (row < rows && k < n) ? (double)in[row * ld_in + k] : 0.0;
    }
    for (int e = tid; e < 16 * 64; e += kBlock) {
      int kk, cc;
      if (TRANS) { kk = e >> 6; cc = e & 63; }  // consecutive columns of a row of P
      else { cc = e >> 4; kk = e & 15; }        // consecutive k of a row of P
      const int k = k0 + kk, c = c0 + cc;
      Bs[kk][cc] = (k < n && c < n) ? (TRANS ? P[(size_t)k * n + c] : P[(size_t)c * n + k]) : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 16; ++kk) {
      double xv[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) { xv[i] = Xs[kk][tr + 16 * i]; bv[i] = Bs[kk][tc + 16 * i]; }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += xv[i] * bv[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t row = r0 + tr + 16 * i;
      const int c = c0 + tc + 16 * j;
      if (row < rows && c < n) out[row * ld_out + c] = (TO)acc[i][j];
    }
}

template <typename TI, typename TO, bool TRANS>
hipError_t launch_rows(const TI* in, int64_t ld_in, TO* out, int64_t ld_out, const double* P, int n, int64_t rows,
                       hipStream_t stream) {
  if (rows == 0) return hipSuccess;
  if (n > kRotMaxN) return hipErrorInvalidValue;
  if (n > kRotLdsN) {
    hipLaunchKernelGGL((rotate_rows_tiled_kernel<TI, TO, TRANS>), dim3((unsigned)((rows + 63) / 64), (n + 63) / 64),
                       dim3(kBlock), 0, stream, in, ld_in, out, ld_out, P, n, rows);
    return hipGetLastError();
  }
  const int64_t tot = rows * n;
  hipLaunchKernelGGL((rotate_rows_kernel<TI, TO, TRANS>), dim3((unsigned)((tot + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, stream, in, ld_in, out, ld_out, P, n, rows);
  return hipGetLastError();
}

}  // namespace

// Larger n: rounds launched from the host, the off-diagonal norm read back after every sweep
// (the same stopping rule as the one-workgroup kernel).  Synchronises the stream.
static hipError_t jacobi_eig_global(const double* HA, int n, double* P, double* sig, int* sweeps,
                                    hipStream_t stream) {
  double *A = nullptr, *An = nullptr, *V = nullptr, *sums = nullptr;
  const size_t nn = (size_t)n * n;
  hipError_t e = hipMalloc(&A, sizeof(double) * nn);
  if (!e) e = hipMalloc(&An, sizeof(double) * nn);
  if (!e) e = hipMalloc(&V, sizeof(double) * nn);
  if (!e) e = hipMalloc(&sums, sizeof(double) * 2);
  const unsigned gnn = (unsigned)((nn + kBlock - 1) / kBlock);
  const int m = n + (n & 1), h = m / 2;
  const int64_t work = (int64_t)h * h + (int64_t)n * h;
  const unsigned gr = (unsigned)((work + kBlock - 1) / kBlock);
  if (!e) {
    hipLaunchKernelGGL(jacobi_init_kernel, dim3(gnn), dim3(kBlock), 0, stream, HA, A, V, n);
    e = hipGetLastError();
  }
  int sweep = 0;
  for (; !e && sweep < kJacobiMaxSweeps; ++sweep) {
    double hs[2] = {0.0, 0.0};
    hipLaunchKernelGGL(jacobi_clear_kernel, dim3(1), dim3(64), 0, stream, sums);
    hipLaunchKernelGGL(jacobi_norms_kernel, dim3(256), dim3(kBlock), 0, stream, A, n, sums);
    e = hipGetLastError();
    if (!e) e = hipMemcpyAsync(hs, sums, sizeof hs, hipMemcpyDeviceToHost, stream);
    if (!e) e = hipStreamSynchronize(stream);
    if (e || !(hs[0] > 1e-30 * hs[1])) break;
    for (int r = 0; r < m - 1 && !e; ++r) {
      hipLaunchKernelGGL(jacobi_round_kernel, dim3(gr), dim3(kBlock), 0, stream, A, An, V, n, m, r);
      e = hipGetLastError();
      std::swap(A, An);
    }
  }
  if (!e) {
    hipLaunchKernelGGL(jacobi_out_kernel, dim3(gnn), dim3(kBlock), 0, stream, A, V, n, P, sig);
    e = hipGetLastError();
  }
  if (!e) e = hipMemcpyAsync(sweeps, &sweep, sizeof(int), hipMemcpyHostToDevice, stream);
  if (!e) e = hipStreamSynchronize(stream);
  hipFree(A); hipFree(An); hipFree(V); hipFree(sums);
  return e;
}

hipError_t launch_jacobi_eig(const double* HA, int n, double* P, double* sig, int* sweeps, hipStream_t stream) {
  if (n < 1 || n > kRotMaxN) return hipErrorInvalidValue;
  if (n > kRotLdsN) return jacobi_eig_global(HA, n, P, sig, sweeps, stream);
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
