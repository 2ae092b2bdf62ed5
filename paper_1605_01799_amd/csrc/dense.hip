// Dense-A Hopf solver for gfx950: split Bregman (eqs. (3.4a)-(3.4c)) for a
// tile of query columns held by one workgroup, all iterations of the tile in
// one persistent launch.
//
// A "column" is one (point j, copy k) pair: x'_jk = x_j - c_k.  The three
// split-Bregman updates are carried in Douglas-Rachford form on the single
// vector z = v + b (v from (3.4a), b from (3.4c)):
//     d^k = prox_{(t/lambda) H}(z^k)           (3.4b)
//     r^k = x' + lambda (d^k - b^k) = x' + lambda (2 d^k - z^k)
//     v^{k+1} = M r^k,  M = (A + lambda I)^{-1}  (3.4a)
//     z^{k+1} = z^k - d^k + v^{k+1}              ((3.4c) folded in: b = z - d)
// The first iteration uses d^0 = x', b^0 = 0 (the paper's initial values),
// i.e. the identity in place of the prox.  The prox of the three supported
// Hamiltonians is gamma * shrink1(z, theta_i) with theta_i = (t/lambda) w_i
// (weights present) and gamma = max(|s|_2 - t/lambda, 0) / |s|_2 (l2 present),
// 1 otherwise (eqs. shrink1_def, shrink2_def; for l2 + weighted l1 the
// l2 shrink is applied to the l1-shrunk vector).
//
// v^{k+1} = M r^k is the hot contraction: one GEMM of the n x n matrix M with
// the n x P_t block of right-hand sides per iteration, on MFMA.  Two modes:
//   F32      z in FP32, FP32 MFMA (16x16x4) products on r.
//   REFINED  BF16 MFMA (16x16x32) products, FP32 accumulate, applied to the
//            INCREMENT r^k - r^a since an anchor state; the anchor product
//            v^a = M r^a is formed exactly with FP64 MFMA (16x16x4) every
//            `anchor_every` iterations.  The state is kept as an FP32 anchor
//            za plus an FP32 increment dz (z = za + dz), with ea = v^a - d^a
//            stored in FP32, so every rounding on the iteration path is
//            relative to a vanishing increment and the fixed point is the
//            FP64-exact one.  The first `warmup` iterations run plain BF16
//            products on the full r (no stopping allowed there).
// Values: phi = <x', d> - 1/2 d^T A d - t H(d) (- 1/2 for ellipsoid level
// sets) with d^T A d = (2 d - v)^T (r - lambda v) + O(|d - v|^2) because
// (A + lambda I) v = r: evaluated in the iteration after a column converged
// (after a fresh FP64 anchor in REFINED mode), so no product with A is needed.
// Distances (section 3.2): psi_k(y, s) is the same evaluation with H = |.|_2,
// t = s and the ellipsoid level set; Newton on s (eq. Newton_zero,
// d psi / ds = -|grad psi|) starts at s = 0 where psi = L_k(y) and grad psi =
// grad L_k(y), each Newton step warm-starting the inner iteration.
#include "common.hpp"
#include "dense.hpp"

namespace hopf {

constexpr int kMaxCols = 64;
constexpr int kNRed = 6;  // step^2, |s|^2 increment, <x',d>, (2d-v).(r-lam v), sum w|d|, |d|^2

struct ColShared {
  double t[kMaxCols], th1[kMaxCols], th2[kMaxCols], gam[kMaxCols], gama[kMaxCols], dgam[kMaxCols];
  double ssa2[kMaxCols], ssq[kMaxCols], prev[kMaxCols], s[kMaxCols], phi[kMaxCols], hp[kMaxCols];
  double pn[kMaxCols];
  int j[kMaxCols], k[kMaxCols], state[kMaxCols], iters[kMaxCols], newton[kMaxCols], flags[kMaxCols];
  double red[4][kMaxCols][kNRed];
  int ctl[8];
};
enum { FLAG_FIRST = 1, FLAG_CAPPED = 2, FLAG_INSIDE = 4, FLAG_NEWTON_CAP = 8 };
enum { CTL_ANCHOR = 0, CTL_PHASE = 1, CTL_LAST_ANCHOR = 2, CTL_FINISH = 3 };
enum { PHASE_WARMUP = 0, PHASE_DELTA = 1 };

__device__ __forceinline__ float clampf(float z, float lo, float hi) { return fminf(fmaxf(z, lo), hi); }
__device__ __forceinline__ float theta_i(double th1, const double* w, int i) { return (float)(th1 * w[i]); }
// shrink1 of an anchor value in FP64 with the FP64 threshold: the anchor reference d^a must be
// exact, since every increment of the following iterations is measured from it.
__device__ __forceinline__ double anchor_shrink(float za, double th1, const double* w, int i) {
  const double z = (double)za, th = th1 * w[i];
  return z - fmin(fmax(z, -th), th);
}

template <int MODE, int CT>
struct Dense {
  static constexpr int PT = 16 * CT;  // columns per tile
  static constexpr int RG = 4;        // row tiles per wave per pass

  // ---------------------------------------------------------------- GEMM pieces
  // acc[r][c] += M[16 rt_r .. , :] * B[:, 16 c ..] over the full contraction.
  static __device__ __forceinline__ void gemm_bf16(const __bf16* __restrict__ M, int n_pad,
                                                   const __bf16* B, int ldb, const int* rt, int nrt,
                                                   f32x4 (&acc)[RG][CT]) {
    const int l = threadIdx.x & 63;
    const int lr = l & 15, lg = l >> 4;
    const __bf16* arow[RG];
#pragma unroll
    for (int r = 0; r < RG; ++r) arow[r] = M + (size_t)(16 * (r < nrt ? rt[r] : 0) + lr) * n_pad + 8 * lg;
    const __bf16* bcol = B + lr * ldb + 8 * lg;
    bf16x8 a0[RG], a1[RG];
#pragma unroll
    for (int r = 0; r < RG; ++r) a0[r] = *(const bf16x8*)(arow[r]);
    for (int k0 = 0; k0 < n_pad; k0 += 32) {
      const bool more = k0 + 32 < n_pad;
#pragma unroll
      for (int r = 0; r < RG; ++r)
        if (more) a1[r] = *(const bf16x8*)(arow[r] + k0 + 32);
      bf16x8 b[CT];
#pragma unroll
      for (int c = 0; c < CT; ++c) b[c] = *(const bf16x8*)(bcol + 16 * c * ldb + k0);
#pragma unroll
      for (int r = 0; r < RG; ++r)
        if (r < nrt) {
#pragma unroll
          for (int c = 0; c < CT; ++c)
            acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0[r], b[c], acc[r][c], 0, 0, 0);
        }
#pragma unroll
      for (int r = 0; r < RG; ++r) a0[r] = a1[r];
    }
  }

  static __device__ __forceinline__ void gemm_f32(const float* __restrict__ M, int n_pad, const float* B,
                                                  int ldb, const int* rt, int nrt, f32x4 (&acc)[RG][CT]) {
    const int l = threadIdx.x & 63;
    const int lr = l & 15, lg = l >> 4;
    const float* arow[RG];
#pragma unroll
    for (int r = 0; r < RG; ++r) arow[r] = M + (size_t)(16 * (r < nrt ? rt[r] : 0) + lr) * n_pad + 4 * lg;
    const float* bcol = B + lr * ldb + 4 * lg;
    for (int k0 = 0; k0 < n_pad; k0 += 16) {
      f32x4 a[RG], b[CT];
#pragma unroll
      for (int r = 0; r < RG; ++r) a[r] = *(const f32x4*)(arow[r] + k0);
#pragma unroll
      for (int c = 0; c < CT; ++c) b[c] = *(const f32x4*)(bcol + 16 * c * ldb + k0);
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < RG; ++r)
          if (r < nrt) {
#pragma unroll
            for (int c = 0; c < CT; ++c)
              acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r][q], b[c][q], acc[r][c], 0, 0, 0);
          }
    }
  }

  // FP64: one 16-column block. A rows are loaded in the order 4(rho%4) + rho/4 so that the
  // output lands in the same lane layout as the FP32/BF16 16x16 products:
  // lane l, register i -> row 4(l/16) + i, column l%16.
  static __device__ __forceinline__ void gemm_f64(const double* __restrict__ M, int n_pad, const double* B,
                                                  int ldb, int bcols, const int* rt, int nrt,
                                                  f64x4 (&acc)[RG]) {
    const int l = threadIdx.x & 63;
    const int lr = l & 15, lg = l >> 4;
    const int arow_perm = 4 * (lr & 3) + (lr >> 2);
    const double* arow[RG];
#pragma unroll
    for (int r = 0; r < RG; ++r) arow[r] = M + (size_t)(16 * (r < nrt ? rt[r] : 0) + arow_perm) * n_pad + 4 * lg;
    const bool bon = lr < bcols;
    const double* bcol = B + lr * ldb + 4 * lg;
    for (int k0 = 0; k0 < n_pad; k0 += 16) {
      f64x4 a[RG], b;
#pragma unroll
      for (int r = 0; r < RG; ++r) a[r] = *(const f64x4*)(arow[r] + k0);
      if (bon) b = *(const f64x4*)(bcol + k0);
      else b = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < RG; ++r)
          if (r < nrt) acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r][q], b[q], acc[r], 0, 0, 0);
    }
  }
};

// Wave-level sum of a double across the 64 lanes (result in every lane).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <int MODE, int CT>
__global__ void __launch_bounds__(kBlock, 1)
dense_kernel(const DenseProb* __restrict__ probs, const DenseTile* __restrict__ tiles, int ntiles,
             float* __restrict__ ws, int64_t ws_per_wg, int distance, int warmup, int anchor_every) {
  using D = Dense<MODE, CT>;
  constexpr int PT = D::PT;
  constexpr int RG = D::RG;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  __shared__ ColShared S;

  const int tid = threadIdx.x;
  const int wave = tid >> 6, l = tid & 63;
  float* wsb = ws + (int64_t)blockIdx.x * ws_per_wg;

  for (int ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
    const DenseTile tile = tiles[ti];
    const DenseProb& pb = probs[tile.prob];
    const int n = pb.n, n_pad = pb.n_pad, K = pb.K;
    const double lam = pb.lambda;
    const bool has_l1 = !distance && hk_has_l1(pb.hkind);
    const bool has_l2 = distance || hk_has_l2(pb.hkind);
    const int ncols = tile.npt * K;
    float* za = wsb;
    float* dz = wsb + (int64_t)PT * n_pad;
    float* ea = wsb + 2 * (int64_t)PT * n_pad;
    float* pout = wsb + 3 * (int64_t)PT * n_pad;
    const int nq = n_pad >> 2;
    const int RT = n_pad >> 4;
    const float flam = (float)lam;

    // ---------------------------------------------------------------- column init
    if (tid < PT) {
      const int c = tid;
      int st = COL_EMPTY;
      if (c < ncols) {
        const int jj = tile.pt0 + c / K, kk = c % K;
        S.j[c] = jj; S.k[c] = kk;
        double tv = distance ? 0.0 : (double)pb.t[jj];
        S.t[c] = tv;
        st = (distance || tv > 0.0) ? COL_ACTIVE : COL_INVALID;
        S.th1[c] = has_l1 ? tv / lam : 0.0;
        S.th2[c] = (!distance && has_l2) ? tv / lam : 0.0;
      }
      S.state[c] = st;
      S.gam[c] = 1.0; S.gama[c] = 1.0; S.dgam[c] = 0.0; S.ssa2[c] = 0.0; S.ssq[c] = 0.0;
      S.prev[c] = 1e300; S.s[c] = 0.0; S.phi[c] = 0.0; S.hp[c] = 0.0; S.pn[c] = 0.0;
      S.iters[c] = 0; S.newton[c] = 0; S.flags[c] = FLAG_FIRST;
    }
    if (tid == 0) {
      S.ctl[CTL_ANCHOR] = 0; S.ctl[CTL_PHASE] = PHASE_WARMUP; S.ctl[CTL_LAST_ANCHOR] = 0;
      S.ctl[CTL_FINISH] = 0;
    }
    __syncthreads();
    // state init + finiteness check, one wave per column
    for (int c = wave; c < PT; c += 4) {
      const int st = S.state[c];
      bool bad = false;
      const double* cen = (pb.centres && st != COL_EMPTY) ? pb.centres + (size_t)S.k[c] * n_pad : nullptr;
      const float* xj = (st != COL_EMPTY) ? pb.x + (size_t)S.j[c] * n : nullptr;
      for (int i = l; i < n_pad; i += 64) {
        float v = 0.f;
        if (st != COL_EMPTY && i < n) {
          float xv = xj[i];
          if (!isfinite(xv)) bad = true;
          v = (float)((double)xv - (cen ? cen[i] : 0.0));
        }
        za[(size_t)c * n_pad + i] = (st == COL_ACTIVE) ? v : 0.f;
        dz[(size_t)c * n_pad + i] = 0.f;
        ea[(size_t)c * n_pad + i] = 0.f;
      }
      bool anybad = __any(bad);
      if (l == 0 && anybad && st == COL_ACTIVE) S.state[c] = COL_INVALID;
    }
    __syncthreads();

    int k_it = 0;
    while (true) {
      // ------------------------------------------------------------ anchor (REFINED)
      if (MODE == 1 && S.ctl[CTL_ANCHOR]) {
        const bool from_warmup = S.ctl[CTL_PHASE] == PHASE_WARMUP;
        // pass A: renormalise z = za + dz, anchor d^a = gamma^a shrink1(za), norms
        for (int c = wave; c < PT; c += 4) {
          const int st = S.state[c];
          if (st != COL_ACTIVE && st != COL_WAITING) continue;
          const double th1 = S.th1[c];
          double pss = 0.0, pinc = 0.0;
          for (int i = l; i < n_pad; i += 64) {
            const size_t e = (size_t)c * n_pad + i;
            double z = from_warmup ? (double)za[e] : (double)za[e] + (double)dz[e];
            float zan = (float)z;
            float dzn = (float)(z - (double)zan);
            za[e] = zan; dz[e] = dzn;
            float th = theta_i(th1, pb.w, i);
            float ca = clampf(zan, -th, th);
            float sa = zan - ca;
            float ds = dzn - clampf(dzn + sa, -th - ca, th - ca);
            const double sa64 = anchor_shrink(zan, th1, pb.w, i);
            pss += sa64 * sa64;
            pinc += (double)ds * (2.0 * (double)sa + (double)ds);
          }
          pss = wave_sum(pss); pinc = wave_sum(pinc);
          if (l == 0) {
            S.ssa2[c] = pss;
            double ssq = pss + pinc;
            S.ssq[c] = ssq;
            double ga = 1.0, g = 1.0;
            if (has_l2) {
              double na = sqrt(pss), nz = sqrt(fmax(ssq, 0.0)), th2 = S.th2[c];
              ga = na > 0.0 ? fmax(na - th2, 0.0) / na : 0.0;
              g = nz > 0.0 ? fmax(nz - th2, 0.0) / nz : 0.0;
            }
            if (S.flags[c] & FLAG_FIRST) { ga = 1.0; }  // cannot happen after warm-up; kept for max_iter < 1
            S.gama[c] = ga; S.gam[c] = g; S.dgam[c] = g - ga;
          }
        }
        __syncthreads();
        // pass B: v^a = M r^a in FP64, 16 (or 8) columns at a time; ea = v^a - d^a
        double* B64 = (double*)lds_raw;
        const int SB = n_pad <= 1024 ? 16 : 8;
        const int ldb64 = n_pad + 2;
        for (int c0 = 0; c0 < PT; c0 += SB) {
          bool any = false;
          for (int cc = 0; cc < SB; ++cc) {
            int st = S.state[c0 + cc];
            any |= (st == COL_ACTIVE || st == COL_WAITING);
          }
          if (!any) continue;
          for (int g = tid; g < SB * n_pad; g += kBlock) {
            const int cc = g / n_pad, i = g % n_pad, c = c0 + cc;
            const int st = S.state[c];
            double r = 0.0;
            if ((st == COL_ACTIVE || st == COL_WAITING) && i < n) {
              const size_t e = (size_t)c * n_pad + i;
              const float zan = za[e];
              const double sa64 = anchor_shrink(zan, S.th1[c], pb.w, i);
              double xp = (double)pb.x[(size_t)S.j[c] * n + i] - (pb.centres ? pb.centres[(size_t)S.k[c] * n_pad + i] : 0.0);
              r = xp + lam * (2.0 * S.gama[c] * sa64 - (double)zan);
            }
            B64[cc * ldb64 + i] = r;
          }
          __syncthreads();
          for (int rt0 = wave; rt0 < RT; rt0 += 4 * RG) {
            int rt[RG]; int nrt = 0;
#pragma unroll
            for (int r = 0; r < RG; ++r) { rt[r] = rt0 + 4 * r; if (rt[r] < RT) nrt = r + 1; }
            f64x4 acc[RG];
#pragma unroll
            for (int r = 0; r < RG; ++r) acc[r] = f64x4{0.0, 0.0, 0.0, 0.0};
            D::gemm_f64(pb.Md, n_pad, B64, ldb64, SB, rt, nrt, acc);
            const int cc = l & 15;
            const int c = c0 + cc;
            if (cc < SB) {
              const int st = S.state[c];
              if (st == COL_ACTIVE || st == COL_WAITING) {
                const double ga = S.gama[c];
#pragma unroll
                for (int r = 0; r < RG; ++r) {
                  if (r >= nrt) continue;
                  const int row0 = 16 * rt[r] + 4 * (l >> 4);
#pragma unroll
                  for (int i = 0; i < 4; ++i) {
                    const int row = row0 + i;
                    const size_t e = (size_t)c * n_pad + row;
                    const double sa64 = anchor_shrink(za[e], S.th1[c], pb.w, row);
                    ea[e] = (row < n) ? (float)(acc[r][i] - ga * sa64) : 0.f;
                  }
                }
              }
            }
          }
          __syncthreads();
        }
        if (tid < PT) {
          if (S.state[tid] == COL_WAITING) S.state[tid] = COL_PHI;
        }
        if (tid == 0) {
          S.ctl[CTL_ANCHOR] = 0; S.ctl[CTL_PHASE] = PHASE_DELTA; S.ctl[CTL_LAST_ANCHOR] = k_it;
        }
        __syncthreads();
      }
      if (MODE == 0 && tid < PT) {  // plain mode: converged columns are evaluated right away
        if (S.state[tid] == COL_WAITING) S.state[tid] = COL_PHI;
      }
      __syncthreads();
      // finished?
      if (tid == 0) {
        int live = 0;
        for (int c = 0; c < PT; ++c) {
          int st = S.state[c];
          live |= (st == COL_ACTIVE || st == COL_PHI || st == COL_WAITING);
        }
        S.ctl[CTL_FINISH] = !live;
      }
      __syncthreads();
      if (S.ctl[CTL_FINISH]) break;
      const bool delta = (MODE == 1) && S.ctl[CTL_PHASE] == PHASE_DELTA;

      // ------------------------------------------------------------ prologue: right-hand sides
      if (MODE == 1) {
        __bf16* B16 = (__bf16*)lds_raw;
        const int ldb = n_pad + 8;
        for (int g = tid; g < PT * nq; g += kBlock) {
          const int c = g / nq, i0 = (g % nq) * 4;
          const int st = S.state[c];
          float rv[4] = {0.f, 0.f, 0.f, 0.f};
          if (st == COL_ACTIVE || st == COL_PHI) {
            const size_t e = (size_t)c * n_pad + i0;
            const f32x4 zav = *(const f32x4*)(za + e);
            if (delta) {
              const f32x4 dzv = *(const f32x4*)(dz + e);
              const float gaf = (float)S.gama[c], dgf = (float)S.dgam[c];
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                float th = theta_i(S.th1[c], pb.w, i0 + q);
                float ca = clampf(zav[q], -th, th), sa = zav[q] - ca;
                float ds = dzv[q] - clampf(dzv[q] + sa, -th - ca, th - ca);
                float dd = gaf * ds + dgf * (sa + ds);
                rv[q] = flam * (2.f * dd - dzv[q]);
              }
            } else {
              const bool first = S.flags[c] & FLAG_FIRST;
              const float gf = (float)S.gam[c];
              const float* xj = pb.x + (size_t)S.j[c] * n;
              const double* cen = pb.centres ? pb.centres + (size_t)S.k[c] * n_pad : nullptr;
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int i = i0 + q;
                if (i >= n) continue;
                float z = zav[q];
                float d = z;
                if (!first) { float th = theta_i(S.th1[c], pb.w, i); d = gf * (z - clampf(z, -th, th)); }
                float xp = (float)((double)xj[i] - (cen ? cen[i] : 0.0));
                rv[q] = xp + flam * (2.f * d - z);
              }
            }
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) B16[c * ldb + i0 + q] = to_bf16(rv[q]);
        }
      } else {
        float* B32 = (float*)lds_raw;
        const int ldb = n_pad + 4;
        for (int g = tid; g < PT * nq; g += kBlock) {
          const int c = g / nq, i0 = (g % nq) * 4;
          const int st = S.state[c];
          f32x4 rv = {0.f, 0.f, 0.f, 0.f};
          if (st == COL_ACTIVE || st == COL_PHI) {
            const f32x4 zav = *(const f32x4*)(za + (size_t)c * n_pad + i0);
            const bool first = S.flags[c] & FLAG_FIRST;
            const float gf = (float)S.gam[c];
            const float* xj = pb.x + (size_t)S.j[c] * n;
            const double* cen = pb.centres ? pb.centres + (size_t)S.k[c] * n_pad : nullptr;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int i = i0 + q;
              if (i >= n) continue;
              float z = zav[q];
              float d = z;
              if (!first) { float th = theta_i(S.th1[c], pb.w, i); d = gf * (z - clampf(z, -th, th)); }
              float xp = (float)((double)xj[i] - (cen ? cen[i] : 0.0));
              rv[q] = xp + flam * (2.f * d - z);
            }
          }
          *(f32x4*)(B32 + c * ldb + i0) = rv;
        }
      }
      __syncthreads();

      // ------------------------------------------------------------ GEMM + epilogue
      double part[CT][kNRed];
#pragma unroll
      for (int c = 0; c < CT; ++c)
#pragma unroll
        for (int q = 0; q < kNRed; ++q) part[c][q] = 0.0;

      for (int rt0 = wave; rt0 < RT; rt0 += 4 * RG) {
        int rt[RG]; int nrt = 0;
#pragma unroll
        for (int r = 0; r < RG; ++r) { rt[r] = rt0 + 4 * r; if (rt[r] < RT) nrt = r + 1; }
        f32x4 acc[RG][CT];
#pragma unroll
        for (int r = 0; r < RG; ++r)
#pragma unroll
          for (int c = 0; c < CT; ++c) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
        if (MODE == 1) D::gemm_bf16(pb.Mb, n_pad, (const __bf16*)lds_raw, n_pad + 8, rt, nrt, acc);
        else D::gemm_f32(pb.Mf, n_pad, (const float*)lds_raw, n_pad + 4, rt, nrt, acc);

#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          const int c = 16 * ct + (l & 15);
          const int st = S.state[c];
          if (st != COL_ACTIVE && st != COL_PHI) continue;
          const bool first = S.flags[c] & FLAG_FIRST;
          const double th1 = S.th1[c];
#pragma unroll
          for (int r = 0; r < RG; ++r) {
            if (r >= nrt) continue;
            const int row0 = 16 * rt[r] + 4 * (l >> 4);
            const size_t e = (size_t)c * n_pad + row0;
            const f32x4 v = acc[r][ct];
            f32x4 zav = *(const f32x4*)(za + e);
            if (MODE == 1 && delta) {
              f32x4 dzv = *(const f32x4*)(dz + e);
              const f32x4 eav = *(const f32x4*)(ea + e);
              const float gaf = (float)S.gama[c], dgf = (float)S.dgam[c];
              // COL_PHI also takes the step: with the fresh anchor it re-runs the stopping test on an
              // exact product (a column that converged to a stale anchor's fixed point continues).
              f32x4 pv;
              const double ga = S.gama[c];
              const float* xj = pb.x + (size_t)S.j[c] * n;
              const double* cen = pb.centres ? pb.centres + (size_t)S.k[c] * n_pad : nullptr;
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int i = row0 + q;
                float th = theta_i(th1, pb.w, i);
                float ca = clampf(zav[q], -th, th), sa = zav[q] - ca;
                float lo = -th - ca, hi = th - ca;
                float ds = dzv[q] - clampf(dzv[q] + sa, lo, hi);
                float dd = gaf * ds + dgf * (sa + ds);
                float step = eav[q] + v[q] - dd;      // z^{k+1} - z^k
                float dzn = dzv[q] + step;
                float dsn = dzn - clampf(dzn + sa, lo, hi);
                part[ct][0] += (double)step * (double)step;
                part[ct][1] += (double)dsn * (2.0 * (double)sa + (double)dsn);
                if (st == COL_PHI) {  // value from the exact-product identity at the current iterate
                  double da = ga * anchor_shrink(zav[q], th1, pb.w, i);
                  double d = da + (double)dd;
                  double vv = (double)eav[q] + da + (double)v[q];
                  double xp = (i < n) ? (double)xj[i] - (cen ? cen[i] : 0.0) : 0.0;
                  double ra = xp + lam * (2.0 * da - (double)zav[q]);
                  double rr = ra + lam * (2.0 * (double)dd - (double)dzv[q]);
                  if (i >= n) d = 0.0;
                  part[ct][2] += xp * d;
                  part[ct][3] += (2.0 * d - vv) * (rr - lam * vv);
                  part[ct][4] += (i < n ? pb.w[i] : 0.0) * fabs(d);
                  part[ct][5] += d * d;
                  pv[q] = (float)d;
                }
                dzv[q] = dzn;
              }
              *(f32x4*)(dz + e) = dzv;
              if (st == COL_PHI) *(f32x4*)(pout + e) = pv;
            } else {
              // plain iteration (F32 mode, or the BF16 warm-up): z^{k+1} = z - d + v
              const float gf = (float)S.gam[c];
              if (st == COL_ACTIVE) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                  float th = theta_i(th1, pb.w, row0 + q);
                  float z = zav[q];
                  float d = first ? z : gf * (z - clampf(z, -th, th));
                  float zn = z - d + v[q];
                  float step = zn - z;
                  float sn = zn - clampf(zn, -th, th);
                  part[ct][0] += (double)step * (double)step;
                  part[ct][1] += (double)sn * (double)sn;
                  zav[q] = zn;
                }
                *(f32x4*)(za + e) = zav;
              } else if (MODE == 0) {  // COL_PHI in F32 mode: r is in LDS
                const float* B32 = (const float*)lds_raw;
                const int ldb = n_pad + 4;
                const float* xj = pb.x + (size_t)S.j[c] * n;
                const double* cen = pb.centres ? pb.centres + (size_t)S.k[c] * n_pad : nullptr;
                f32x4 pv;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                  const int i = row0 + q;
                  float th = theta_i(th1, pb.w, i);
                  float z = zav[q];
                  double d = (i < n) ? (double)(first ? z : gf * (z - clampf(z, -th, th))) : 0.0;
                  double vv = (double)v[q];
                  double rr = (double)B32[c * ldb + i];
                  double xp = (i < n) ? (double)xj[i] - (cen ? cen[i] : 0.0) : 0.0;
                  part[ct][2] += xp * d;
                  part[ct][3] += (2.0 * d - vv) * (rr - lam * vv);
                  part[ct][4] += (i < n ? pb.w[i] : 0.0) * fabs(d);
                  part[ct][5] += d * d;
                  pv[q] = (float)d;
                }
                *(f32x4*)(pout + e) = pv;
              }
            }
          }
        }
      }
      // reduce partials: over the 4 lane groups, then across waves through LDS
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int q = 0; q < kNRed; ++q) {
          double v = part[ct][q];
          v += __shfl_xor(v, 16);
          v += __shfl_xor(v, 32);
          if (l < 16) S.red[wave][16 * ct + l][q] = v;
        }
      __syncthreads();

      // ------------------------------------------------------------ per-column update
      if (tid < PT) {
        const int c = tid;
        const int st = S.state[c];
        double sm[kNRed];
#pragma unroll
        for (int q = 0; q < kNRed; ++q) sm[q] = S.red[0][c][q] + S.red[1][c][q] + S.red[2][c][q] + S.red[3][c][q];
        const bool stepped = st == COL_ACTIVE || (MODE == 1 && st == COL_PHI);
        bool evaluate = (MODE == 0 && st == COL_PHI);
        if (stepped) {
          S.iters[c] += 1;
          const double ssq = delta ? S.ssa2[c] + sm[1] : sm[1];
          S.ssq[c] = ssq;
          double g = 1.0;
          if (has_l2) {
            double nz = sqrt(fmax(ssq, 0.0));
            g = nz > 0.0 ? fmax(nz - S.th2[c], 0.0) / nz : 0.0;
          }
          S.gam[c] = g;
          S.dgam[c] = g - S.gama[c];
          S.flags[c] &= ~FLAG_FIRST;
          const bool can_stop = (MODE == 0) || delta;
          const double a = sqrt(sm[0]), b = sqrt(S.prev[c]);
          S.prev[c] = sm[0];
          const bool conv = can_stop && (a + b) * (a + b) <= pb.tol;
          const bool capped = S.iters[c] >= pb.max_iter;
          if (st == COL_ACTIVE) {
            if (conv) S.state[c] = COL_WAITING;
            else if (capped) { S.state[c] = COL_WAITING; S.flags[c] |= FLAG_CAPPED; }
          } else {
            if (capped && !conv) S.flags[c] |= FLAG_CAPPED;
            if (conv || (S.flags[c] & FLAG_CAPPED)) evaluate = true;
            else S.state[c] = COL_ACTIVE;
          }
        }
        if (evaluate) {
          const double tt = distance ? S.s[c] : S.t[c];
          const double pn = sqrt(sm[5]);
          const double H = (has_l1 ? sm[4] : 0.0) + (has_l2 ? pn : 0.0);
          const double val = sm[2] - 0.5 * sm[3] - tt * H - (pb.level_set ? 0.5 : 0.0);
          S.phi[c] = val; S.hp[c] = H; S.pn[c] = pn;
          if (!distance) {
            S.state[c] = COL_DONE;
          } else {
            if (S.s[c] == 0.0 && val <= 0.0) {  // psi(y, 0) = L_k(y) <= 0: y lies in ellipsoid k
              S.flags[c] |= FLAG_INSIDE; S.state[c] = COL_DONE;
            } else if (!(pn > 0.0) || (S.flags[c] & FLAG_CAPPED)) {
              S.state[c] = COL_DONE;
            } else {
              const double ds = val / pn;          // s_{l+1} = s_l - psi / (d psi / ds), d psi/ds = -|grad psi|
              const double sn = S.s[c] + ds;
              S.newton[c] += 1;
              S.s[c] = sn;
              if (fabs(ds) <= pb.s_tol * fmax(1.0, sn)) {
                S.state[c] = COL_DONE;
              } else if (S.newton[c] >= pb.max_newton) {
                S.flags[c] |= FLAG_NEWTON_CAP; S.state[c] = COL_DONE;
              } else {
                S.th2[c] = sn / lam;
                const double nz = sqrt(fmax(S.ssq[c], 0.0));
                const double g = nz > 0.0 ? fmax(nz - S.th2[c], 0.0) / nz : 0.0;
                S.gam[c] = g; S.dgam[c] = g - S.gama[c];
                S.prev[c] = 1e300;
                S.state[c] = COL_ACTIVE;
              }
            }
          }
        }
      }
      __syncthreads();
      if (tid == 0) {
        int nact = 0, nwait = 0;
        for (int c = 0; c < PT; ++c) {
          nact += S.state[c] == COL_ACTIVE;
          nwait += S.state[c] == COL_WAITING;
        }
        if (MODE == 1) {
          const int kn = k_it + 1;
          if (S.ctl[CTL_PHASE] == PHASE_WARMUP) {
            if (kn >= warmup || (nact == 0 && nwait > 0)) S.ctl[CTL_ANCHOR] = 1;
          } else {
            if ((nact > 0 && kn - S.ctl[CTL_LAST_ANCHOR] >= anchor_every) || (nwait > 0 && nact == 0))
              S.ctl[CTL_ANCHOR] = 1;
          }
        }
      }
      __syncthreads();
      ++k_it;
    }

    // ---------------------------------------------------------------- outputs (min over copies)
    const int npt = tile.npt;
    __shared__ int win[kMaxCols];
    if (tid < npt) {
      int best = -1;
      double bv = 0.0;
      bool inside = false;
      for (int kk = 0; kk < K; ++kk) {
        const int c = tid * K + kk;
        if (S.state[c] != COL_DONE) continue;
        if (distance) {
          if (S.flags[c] & FLAG_INSIDE) { if (!inside) { inside = true; best = c; } continue; }
          if (inside) continue;
          if (best < 0 || S.s[c] < bv) { best = c; bv = S.s[c]; }
        } else {
          if (best < 0 || S.phi[c] < bv) { best = c; bv = S.phi[c]; }
        }
      }
      win[tid] = best;
      const int64_t j = tile.pt0 + tid;
      const float qnan = __builtin_nanf("");
      if (!distance) {
        if (best < 0) {
          pb.phi[j] = qnan; pb.dphidt[j] = qnan;
          if (pb.iters) pb.iters[j] = -1;
          if (pb.kstar) pb.kstar[j] = -1;
        } else {
          pb.phi[j] = (float)S.phi[best];
          pb.dphidt[j] = (float)(-S.hp[best]);
          if (pb.iters) pb.iters[j] = (S.flags[best] & FLAG_CAPPED) ? -2 : S.iters[best];
          if (pb.kstar) pb.kstar[j] = best - tid * K;
        }
      } else {
        if (best < 0) {
          pb.dist[j] = qnan;
          if (pb.kstar) pb.kstar[j] = -1;
          if (pb.inside) pb.inside[j] = 0;
          if (pb.newton) pb.newton[j] = -1;
        } else {
          pb.dist[j] = inside ? 0.f : (float)S.s[best];
          if (pb.kstar) pb.kstar[j] = best - tid * K;
          if (pb.inside) pb.inside[j] = inside ? 1 : 0;
          if (pb.newton) pb.newton[j] = (S.flags[best] & (FLAG_CAPPED | FLAG_NEWTON_CAP)) ? -2 : S.newton[best];
        }
      }
    }
    __syncthreads();
    for (int g = tid; g < npt * n; g += kBlock) {
      const int p = g / n, i = g % n;
      const int c = win[p];
      const int64_t j = tile.pt0 + p;
      float v;
      if (c < 0) v = __builtin_nanf("");
      else if (!distance) v = pout[(size_t)c * n_pad + i];
      else {
        const float y = pb.x[(size_t)j * n + i];
        if (S.flags[c] & FLAG_INSIDE) v = y;
        else v = (float)((double)y - S.s[c] * (double)pout[(size_t)c * n_pad + i] / S.pn[c]);
      }
      pb.grad[(size_t)j * n + i] = v;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Host launcher
// ---------------------------------------------------------------------------
int dense_cols_per_tile(int mode, int n_pad) {
  if (mode == 1) return n_pad <= 1024 ? 64 : 32;
  if (n_pad <= 512) return 64;
  if (n_pad <= 1024) return 32;
  return 16;
}

size_t dense_lds_bytes(int mode, int n_pad) {
  const int pt = dense_cols_per_tile(mode, n_pad);
  size_t b;
  if (mode == 1) {
    size_t b16 = (size_t)pt * (n_pad + 8) * 2;
    size_t b64 = (size_t)(n_pad <= 1024 ? 16 : 8) * (n_pad + 2) * 8;
    b = b16 > b64 ? b16 : b64;
  } else {
    b = (size_t)pt * (n_pad + 4) * 4;
  }
  return b;
}

template <int MODE, int CT>
static hipError_t launch_t(const DenseProb* d_probs, const DenseTile* d_tiles, int ntiles, float* ws,
                           int64_t ws_per_wg, int grid, size_t lds, int distance, int warmup,
                           int anchor_every, hipStream_t stream) {
  auto kern = dense_kernel<MODE, CT>;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(136 * 1024));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), lds, stream, d_probs, d_tiles, ntiles, ws,
                     ws_per_wg, distance, warmup, anchor_every);
  return hipGetLastError();
}

hipError_t launch_dense(int mode, int cols_per_tile, const DenseProb* d_probs, const DenseTile* d_tiles,
                        int ntiles, float* ws, int64_t ws_per_wg, int grid, size_t lds, int distance,
                        int warmup, int anchor_every, hipStream_t stream) {
  const int ct = cols_per_tile / 16;
  if (mode == 1) {
    if (ct == 4) return launch_t<1, 4>(d_probs, d_tiles, ntiles, ws, ws_per_wg, grid, lds, distance, warmup, anchor_every, stream);
    if (ct == 2) return launch_t<1, 2>(d_probs, d_tiles, ntiles, ws, ws_per_wg, grid, lds, distance, warmup, anchor_every, stream);
    if (ct == 1) return launch_t<1, 1>(d_probs, d_tiles, ntiles, ws, ws_per_wg, grid, lds, distance, warmup, anchor_every, stream);
  } else {
    if (ct == 4) return launch_t<0, 4>(d_probs, d_tiles, ntiles, ws, ws_per_wg, grid, lds, distance, warmup, anchor_every, stream);
    if (ct == 2) return launch_t<0, 2>(d_probs, d_tiles, ntiles, ws, ws_per_wg, grid, lds, distance, warmup, anchor_every, stream);
    if (ct == 1) return launch_t<0, 1>(d_probs, d_tiles, ntiles, ws, ws_per_wg, grid, lds, distance, warmup, anchor_every, stream);
  }
  return hipErrorInvalidValue;
}

}  // namespace hopf
