// Envelope-theorem backward pass.  phi_j is the optimal value of eq. (3.3);
// at fixed p its objective J*(p) + t H(p) - <x, p> (with J_k*(p) =
// 1/2 p^T A p + <c_k, p> (+ 1/2)) is affine in x, t, A and c_k, so at the
// minimiser p*_j:
//   d phi/dx = p*,  d phi/dt = -H(p*),  d phi/dA = -1/2 p* p*^T,  d phi/dc_{k*} = -p*.
// For L = sum_j g_j phi_j:
//   gA = -1/2 P^T diag(g) P    (P: npts x n, the saved p* rows): one GEMM over the points, on
//        FP32 MFMA (16x16x4), split over point ranges into FP32 partials of 64 x 64 tiles of the
//        lower triangle (gA is symmetric), summed over the splits in FP64 in a fixed order;
//   gx, gt, gc: one pass over the p* rows writes gx = g_j p*_j and gt, and accumulates
//        gc_k = -sum_{j: k*_j = k} g_j p*_j per point range in FP64, summed in a fixed order.
// Both reductions are deterministic: a split's points and the order of every sum are fixed by
// the sizes and the split counts.
#include <algorithm>

#include "common.hpp"
#include "backward.hpp"

namespace hopf {

constexpr int kGT = 64;       // gA output tile (kGT x kGT), four waves of 32 x 32
constexpr int kGB = 64;       // points per LDS batch of the gA kernel
constexpr int kGLd = kGT + 4; // LDS row length (floats)
constexpr int kXcd = 8;       // workgroups are dealt to the 8 XCDs round robin

__global__ void bw_fill_kernel(float* __restrict__ p, int64_t m) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < m) p[e] = 0.f;
}

// Lower-triangle tile t -> (bi, bj), bi >= bj, t = bi (bi + 1) / 2 + bj.
__device__ __forceinline__ void tri_tile(int t, int* bi, int* bj) {
  int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  *bi = i;
  *bj = t - i * (i + 1) / 2;
}

// gA partials.  Workgroup b takes split s and lower tile t with all tiles of one split on one XCD
// (b % 8 = s % 8), so the split's p* rows are read from HBM once into that XCD's L2.
// part: [split][tile][64][64] FP32, rows/cols beyond n are zero.
// MFMA operand mapping (v_mfma_f32_16x16x4f32: A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k,
// D[i][j] in lane j + 16 (i / 4), register i % 4): k-slot g = lane / 16 of k-step s holds point
// 4 s + g of the batch; in a wave's 32 x 32 quadrant, sub-tile (ra, cb) row r is tile row
// 2 r + ra and column c is tile column 2 c + cb, so one float2 LDS read gives both sub-tiles'
// operands.
template <bool VEC>
__global__ void __launch_bounds__(kBlock) bw_gA_mfma_kernel(int64_t npts, int n, int ntl, int nsplit,
                                                            int64_t chunk, const float* __restrict__ g,
                                                            const float* __restrict__ P, float* __restrict__ part) {
  const int b = blockIdx.x;
  const int xcd = b % kXcd, q = b / kXcd;
  const int tile = q % ntl, split = (q / ntl) * kXcd + xcd;
  if (split >= nsplit) return;
  int bi, bj;
  tri_tile(tile, &bi, &bj);
  const int I0 = bi * kGT, J0 = bj * kGT;
  const int64_t p0 = (int64_t)split * chunk;
  const int64_t p1 = p0 + chunk < npts ? p0 + chunk : npts;

  __shared__ __attribute__((aligned(16))) float XI[kGB][kGLd];
  __shared__ __attribute__((aligned(16))) float XJ[kGB][kGLd];
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63;
  const int lr = l & 15, lg = l >> 4;
  const int wr = wave >> 1, wc = wave & 1;

  // staging: thread tid loads rows pp = tid / 16 + 16 u (u = 0..3) and columns 4 (tid % 16) .. + 3
  const int sc = 4 * (tid & 15), sr = tid >> 4;
  auto load = [&](int64_t b0, f32x4 (&ri)[4], f32x4 (&rj)[4]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t j = b0 + sr + 16 * u;
      f32x4 vi = {0.f, 0.f, 0.f, 0.f}, vj = {0.f, 0.f, 0.f, 0.f};
      if (j < p1) {
        const float gj = g[j];
        const float* row = P + j * (int64_t)n;
        if (VEC) {  // n % 4 == 0: whole float4 inside or outside the row
          if (I0 + sc < n) vi = *gp((const f32x4*)(row + I0 + sc)) * gj;
          if (J0 + sc < n) vj = *gp((const f32x4*)(row + J0 + sc));
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            if (I0 + sc + e < n) vi[e] = gj * row[I0 + sc + e];
            if (J0 + sc + e < n) vj[e] = row[J0 + sc + e];
          }
        }
      }
      ri[u] = vi; rj[u] = vj;
    }
  };

  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = f32x4{0.f, 0.f, 0.f, 0.f};

  f32x4 ri[4], rj[4];
  load(p0, ri, rj);
  for (int64_t b0 = p0; b0 < p1; b0 += kGB) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      *(f32x4*)&XI[sr + 16 * u][sc] = ri[u];
      *(f32x4*)&XJ[sr + 16 * u][sc] = rj[u];
    }
    __syncthreads();
    if (b0 + kGB < p1) load(b0 + kGB, ri, rj);  // the next batch is in flight during the products
#pragma unroll
    for (int s = 0; s < kGB / 4; ++s) {
      const int pp = 4 * s + lg;
      const float2 a = *(const float2*)&XI[pp][32 * wr + 2 * lr];
      const float2 bb = *(const float2*)&XJ[pp][32 * wc + 2 * lr];
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, bb.x, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, bb.y, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, bb.x, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, bb.y, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  float* dst = part + ((int64_t)split * ntl + tile) * (kGT * kGT);
#pragma unroll
  for (int ra = 0; ra < 2; ++ra)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int li = 32 * wr + 2 * (4 * lg + i) + ra;
        const int lj = 32 * wc + 2 * lr + cb;
        dst[li * kGT + lj] = acc[ra][cb][i];
      }
}

// gA = -1/2 (sum over splits of the lower tiles' partials, in FP64), mirrored into the upper
// triangle; one thread per element of the lower tiles (reads of consecutive elements).
__global__ void bw_gA_reduce_kernel(int n, int ntl, int nsplit, const float* __restrict__ part,
                                    float* __restrict__ gA) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)ntl * (kGT * kGT)) return;
  const int tile = (int)(e / (kGT * kGT)), r = (int)(e % (kGT * kGT));
  int bi, bj;
  tri_tile(tile, &bi, &bj);
  const int a = bi * kGT + r / kGT, b = bj * kGT + r % kGT;
  if (a >= n || b >= n) return;
  double s = 0.0;
  for (int q = 0; q < nsplit; ++q) s += (double)part[(int64_t)q * ntl * (kGT * kGT) + e];
  const float v = (float)(-0.5 * s);
  gA[(int64_t)a * n + b] = v;
  if (bi != bj) gA[(int64_t)b * n + a] = v;
}

// One pass over the p* rows of split blockIdx.x: gx = g_j p*_j, gt = g_j dphidt_j, and the sums
// of g_j p*_j by attaining copy (partials [split][k][i] in FP64).
// VEC (n % 4 == 0, n <= 1024, 16-byte aligned rows): a thread takes 4 consecutive coordinates of
// every 256/(n/4)-th row, with U rows' loads in flight, and sums in FP32 over its rows (at most a
// few hundred); the row lanes are combined in FP64 in a fixed order.  Otherwise a thread takes one
// coordinate (for n <= 256, 256/n point lanes; beyond, coordinates tid, tid + 256, ...).
template <int KMAX, bool VEC>
__global__ void __launch_bounds__(kBlock) bw_points_kernel(int64_t npts, int n, int K, int64_t chunk,
                                                           const float* __restrict__ g, const float* __restrict__ P,
                                                           const float* __restrict__ dphidt,
                                                           const int32_t* __restrict__ kstar, float* __restrict__ gx,
                                                           float* __restrict__ gt, double* __restrict__ partc) {
  const int split = blockIdx.x, tid = threadIdx.x;
  const int64_t p0 = (int64_t)split * chunk;
  const int64_t p1 = p0 + chunk < npts ? p0 + chunk : npts;
  const bool want_c = partc != nullptr;
  __shared__ double red[kBlock][4];
  if (VEC) {
    constexpr int U = 8;  // rows whose loads are in flight together
    const int q4 = n >> 2, rpw = kBlock / q4;
    const int c4 = tid % q4, rl = tid / q4;
    const bool act = rl < rpw;
    f32x4 s[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) s[k] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t jb = p0 + rl; jb < p1; jb += (int64_t)rpw * U) {
      f32x4 pv[U];
      float gv[U];
      int kv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t j = jb + (int64_t)u * rpw;
        const bool in = act && j < p1;
        gv[u] = in ? g[j] : 0.f;
        pv[u] = in ? *gp((const f32x4*)(P + j * (int64_t)n) + c4) : f32x4{0.f, 0.f, 0.f, 0.f};
        kv[u] = (in && kstar) ? kstar[j] : 0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t j = jb + (int64_t)u * rpw;
        if (!act || j >= p1) break;
        const f32x4 v = pv[u] * gv[u];
        if (gx) *gp((f32x4*)(gx + j * (int64_t)n) + c4) = v;
        if (gt && c4 == 0) gt[j] = gv[u] * dphidt[j];
        if (want_c) {
#pragma unroll
          for (int k = 0; k < KMAX; ++k)
            if (kv[u] == k) s[k] += v;
        }
      }
    }
    if (!want_c) return;
    for (int k = 0; k < K; ++k) {  // K <= KMAX on this path
      f32x4 sk = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < KMAX; ++kk)
        if (kk == k) sk = s[kk];
#pragma unroll
      for (int e = 0; e < 4; ++e) red[tid][e] = (double)sk[e];
      __syncthreads();
      if (tid < q4) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          double t = 0.0;
          for (int r = 0; r < rpw; ++r) t += red[r * q4 + tid][e];
          partc[((int64_t)split * K + k) * n + 4 * tid + e] = t;
        }
      }
      __syncthreads();
    }
    return;
  }
  if (n <= kBlock) {
    const int npl = kBlock / n;
    const int i = tid % n, pl = tid / n;
    double s[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) s[k] = 0.0;
    if (pl < npl) {
      constexpr int U = 8;
      for (int64_t jb = p0 + pl; jb < p1; jb += (int64_t)npl * U) {
        float gv[U], pv[U];
        int kv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t j = jb + (int64_t)u * npl;
          const bool in = j < p1;
          gv[u] = in ? g[j] : 0.f;
          pv[u] = in ? P[j * (int64_t)n + i] : 0.f;
          kv[u] = (in && kstar) ? kstar[j] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t j = jb + (int64_t)u * npl;
          if (j >= p1) break;
          const float v = gv[u] * pv[u];
          if (gx) gx[j * (int64_t)n + i] = v;
          if (gt && i == 0) gt[j] = gv[u] * dphidt[j];
          if (want_c) {
#pragma unroll
            for (int k = 0; k < KMAX; ++k) s[k] += (kv[u] == k) ? (double)v : 0.0;
          }
        }
      }
    }
    if (!want_c) return;
    if (K <= KMAX) {
      for (int k = 0; k < K; ++k) {
        red[tid][0] = s[k < KMAX ? k : 0];
        __syncthreads();
        if (tid < n) {
          double t = 0.0;
          for (int q = 0; q < npl; ++q) t += red[q * n + tid][0];
          partc[((int64_t)split * K + k) * n + tid] = t;
        }
        __syncthreads();
      }
      return;
    }
    // K > KMAX: one coordinate per thread, copies in an outer loop
    for (int k = 0; k < K; ++k) {
      for (int ii = tid; ii < n; ii += kBlock) {
        double t = 0.0;
        for (int64_t j = p0; j < p1; ++j)
          if ((kstar ? kstar[j] : 0) == k) t += (double)(g[j] * P[j * (int64_t)n + ii]);
        partc[((int64_t)split * K + k) * n + ii] = t;
      }
    }
    return;
  }
  for (int i0 = 0; i0 < n; i0 += kBlock) {
    const int i = i0 + tid;
    if (i >= n) break;
    double s[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) s[k] = 0.0;
    for (int64_t j = p0; j < p1; ++j) {
      const float gj = g[j];
      const float v = gj * P[j * (int64_t)n + i];
      if (gx) gx[j * (int64_t)n + i] = v;
      if (gt && i == 0) gt[j] = gj * dphidt[j];
      if (want_c && K <= KMAX) {
        const int kk = kstar ? kstar[j] : 0;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) s[k] += (kk == k) ? (double)v : 0.0;
      }
    }
    if (!want_c) continue;
    if (K <= KMAX) {
      for (int k = 0; k < K; ++k) partc[((int64_t)split * K + k) * n + i] = s[k];
    } else {
      for (int k = 0; k < K; ++k) {
        double t = 0.0;
        for (int64_t j = p0; j < p1; ++j)
          if ((kstar ? kstar[j] : 0) == k) t += (double)(g[j] * P[j * (int64_t)n + i]);
        partc[((int64_t)split * K + k) * n + i] = t;
      }
    }
  }
}

// gc = -(sum over splits, FP64, fixed order): a workgroup takes 16 consecutive outputs; its 16
// groups of 16 threads take the splits q = group, group + 16, ..., and the group sums are added
// in group order.
__global__ void __launch_bounds__(kBlock) bw_gc_reduce_kernel(int64_t m, int nsplit, const double* __restrict__ part,
                                                              float* __restrict__ gc) {
  const int tid = threadIdx.x, grp = tid >> 4;
  const int64_t e = (int64_t)blockIdx.x * 16 + (tid & 15);
  __shared__ double red[16][16];
  double s = 0.0;
  if (e < m)
    for (int q = grp; q < nsplit; q += 16) s += part[(int64_t)q * m + e];
  red[grp][tid & 15] = s;
  __syncthreads();
  if (tid < 16 && e < m) {
    double t = 0.0;
    for (int q = 0; q < 16; ++q) t += red[q][tid];
    gc[e] = (float)(-t);
  }
}

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

BackwardPlan backward_plan(int64_t npts, int n, int K, bool want_gA, bool want_gc, size_t cap_bytes) {
  BackwardPlan pl;
  const int T = (int)cdiv(n, kGT);
  pl.ntl = T * (T + 1) / 2;
  pl.splits_a = 0; pl.splits_c = 0; pl.bytes_a = 0; pl.bytes_c = 0; pl.ok = true;
  if (npts <= 0) return pl;
  const int64_t pts = npts;
  int sc = (int)std::min<int64_t>(std::max<int64_t>(cdiv(pts, 512), 1), 512);
  int sa = (int)std::min<int64_t>(std::max<int64_t>(cdiv(pts, 2048), 1), 128);
  const size_t per_c = sizeof(double) * (size_t)K * n;
  const size_t per_a = sizeof(float) * (size_t)pl.ntl * kGT * kGT;
  if (want_gc && (size_t)sc * per_c > cap_bytes / 4) sc = (int)std::max<size_t>(1, (cap_bytes / 4) / per_c);
  if (want_gc && (size_t)sc * per_c > cap_bytes) pl.ok = false;
  const size_t bc = want_gc ? (size_t)sc * per_c : 0;
  const size_t bc_al = (bc + 255) / 256 * 256;
  if (want_gA) {
    const size_t room = cap_bytes > bc_al ? cap_bytes - bc_al : 0;
    if ((size_t)sa * per_a > room) sa = (int)(room / per_a);
    if (sa < 1) { sa = 1; pl.ok = false; }
  }
  pl.splits_a = want_gA ? sa : 0;
  pl.splits_c = sc;  // also the gx / gt pass's workgroups
  pl.bytes_c = bc_al;
  pl.bytes_a = want_gA ? (size_t)sa * per_a : 0;
  return pl;
}

hipError_t launch_backward(const BackwardArgs& a, const BackwardPlan& pl, void* scratch, hipStream_t stream) {
  const int64_t npts = a.npts;
  const int n = a.n;
  if (npts == 0) {  // the sums over no points: zeros (a fill kernel, not a memset node)
    if (a.gA) {
      const int64_t m = (int64_t)n * n;
      hipLaunchKernelGGL(bw_fill_kernel, dim3((unsigned)cdiv(m, 256)), dim3(256), 0, stream, a.gA, m);
    }
    if (a.gc) {
      const int64_t m = (int64_t)a.K * n;
      hipLaunchKernelGGL(bw_fill_kernel, dim3((unsigned)cdiv(m, 256)), dim3(256), 0, stream, a.gc, m);
    }
    return hipGetLastError();
  }
  double* partc = a.gc ? (double*)scratch : nullptr;
  float* parta = (float*)((unsigned char*)scratch + pl.bytes_c);
  if (a.gx || a.gt || a.gc) {
    const int64_t chunk = cdiv(npts, pl.splits_c);
    const int nsc = (int)cdiv(npts, chunk);
    const bool vec = n % 4 == 0 && n <= 4 * kBlock && a.K <= 8 && (((uintptr_t)a.grad | (uintptr_t)a.gx) & 15) == 0;
    if (vec)
      hipLaunchKernelGGL((bw_points_kernel<8, true>), dim3(nsc), dim3(kBlock), 0, stream, npts, n, a.K, chunk, a.g,
                         a.grad, a.dphidt, a.kstar, a.gx, a.gt, partc);
    else
      hipLaunchKernelGGL((bw_points_kernel<8, false>), dim3(nsc), dim3(kBlock), 0, stream, npts, n, a.K, chunk, a.g,
                         a.grad, a.dphidt, a.kstar, a.gx, a.gt, partc);
    if (a.gc) {
      const int64_t m = (int64_t)a.K * n;
      hipLaunchKernelGGL(bw_gc_reduce_kernel, dim3((unsigned)cdiv(m, 16)), dim3(kBlock), 0, stream, m, nsc, partc,
                         a.gc);
    }
  }
  if (a.gA) {
    const int64_t chunk = cdiv(npts, pl.splits_a);
    const int nsa = (int)cdiv(npts, chunk);
    const int groups = (int)cdiv(nsa, kXcd);
    const unsigned grid = (unsigned)(groups * kXcd * pl.ntl);
    const bool vec = (n % 4) == 0 && (((uintptr_t)a.grad) & 15) == 0;
    if (vec)
      hipLaunchKernelGGL(bw_gA_mfma_kernel<true>, dim3(grid), dim3(kBlock), 0, stream, npts, n, pl.ntl, nsa, chunk,
                         a.g, a.grad, parta);
    else
      hipLaunchKernelGGL(bw_gA_mfma_kernel<false>, dim3(grid), dim3(kBlock), 0, stream, npts, n, pl.ntl, nsa, chunk,
                         a.g, a.grad, parta);
    const int64_t m = (int64_t)pl.ntl * kGT * kGT;
    hipLaunchKernelGGL(bw_gA_reduce_kernel, dim3((unsigned)cdiv(m, 256)), dim3(256), 0, stream, n, pl.ntl, nsa,
                       parta, a.gA);
  }
  return hipGetLastError();
}

}  // namespace hopf
