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
// l2 shrink is applied to the l1-shrunk vector).  For H = sqrt(<p, D p>), D = diag(w) (section
// 4.3; also sqrt(<p, HA p>), solved in HA's eigenbasis), the prox is z minus the projection of z
// onto the Wulff ellipsoid sum y_i^2 / s_i <= 1, s_i = (t/lambda)^2 w_i:
//     d_i = mu z_i / (s_i + mu),  mu > 0 solving phi(mu) = sum_i s_i z_i^2 / (s_i + mu)^2 = 1,
// or d = 0 when z lies inside.  mu is found by Newton on 1/sqrt(phi) - 1 (concave, increasing),
// whose sums over the rows of a column are workgroup reductions: in FP64 from 0 at an anchor
// (mu^a of za), in FP32 warm-started in the plain iterations, and in REFINED mode two Newton
// steps per pass on the increment dmu = mu - mu^a written with products of increments (below).
//
// v^{k+1} = M r^k is the hot contraction: one GEMM of the n x n matrix M with
// the n x P_t block of right-hand sides per iteration, on MFMA.  Three modes:
//   F32      z in FP32, FP32 MFMA (16x16x4) products on r (the plain method).
//   F32 REFINED  as REFINED below with FP32 MFMA (16x16x4) products of FP32 increments.
//   REFINED  BF16 MFMA (16x16x32) products, FP32 accumulate, applied to the
//            INCREMENT r^k - r^a since an anchor state; the anchor product
//            v^a = M r^a is formed every `anchor_every` iterations from the
//            FP64 r^a, exactly up to ~2^-31 of its row and column scales, as
//            int8 MFMA (16x16x64) products of integer slices of M and r^a
//            with exact int32 accumulation.  The state is kept as an FP32
//            anchor za plus an FP32 increment dz (z = za + dz), with
//            ea = v^a - d^a stored in FP32, so every rounding on the iteration
//            path is relative to a vanishing increment and the fixed point is
//            that of the exact product.  The first `warmup` iterations run
//            plain BF16 products on the full r (no stopping allowed there).
// Values: phi = <x', d> - 1/2 d^T A d - t H(d) (- 1/2 for ellipsoid level
// sets) with d^T A d = (2 d - v)^T (r - lambda v) + O(|d - v|^2) because
// (A + lambda I) v = r: evaluated in the iteration after a column converged
// (after a fresh anchor in REFINED mode), so no product with A is needed.
// Distances (section 3.2): psi_k(y, s) is the same evaluation with H = |.|_2,
// t = s and the ellipsoid level set; Newton on s (eq. Newton_zero,
// d psi / ds = -|grad psi|) starts at s = 0 where psi = L_k(y) and grad psi =
// grad L_k(y), each Newton step warm-starting the inner iteration.
#include <cstdio>
#include <cstdlib>

#include "common.hpp"
#include "dense.hpp"
#include "dense_shared.hpp"

namespace hopf {

// sqrt(<p, D p>): the prox of z for multiplier mu (s = (t/lambda)^2 w_i), 0 inside the ellipsoid
__device__ __forceinline__ float wl2_d(float z, float s, float mu, bool inside) {
  return (inside || !(s > 0.f)) ? 0.f : mu * z * __builtin_amdgcn_rcpf(s + mu);
}
// its increment prox(za + dz) - prox(za) at mu = mu^a + dmu, from products of increments:
//   (mu dz (s + mu^a) + za s dmu) / ((s + mu)(s + mu^a)),  or -d^a when z lies inside
__device__ __forceinline__ float wl2_dd(float za, float dz, float s, float mua, float dm, bool ains, bool cin) {
  if (!(s > 0.f)) return 0.f;
  const float A = s + mua, mu = mua + dm, B = s + mu;
  if (cin) return ains ? 0.f : -mua * za * __builtin_amdgcn_rcpf(A);
  return (mu * dz * A + za * s * dm) * __builtin_amdgcn_rcpf(B * A);
}
// the anchor's d^a in FP64
__device__ __forceinline__ double wl2_da(float za, double s, double mua, bool ains) {
  return (ains || !(s > 0.0)) ? 0.0 : mua * (double)za / (s + mua);
}
constexpr int kWl2PlainNewton = 12;   // cap on a plain pass's Newton steps (warm-started)
constexpr int kWl2AnchorNewton = 100; // cap on an anchor's FP64 Newton steps (from 0)

// MODE 0: FP32 products; MODE 1: BF16 increments + exact anchors; MODE 2: FP32 increments + exact
// anchors.  CT column tiles of 16, RG row
// tiles per wave and product pass, NW waves per workgroup (the waves split the row tiles),
// OCC workgroups per CU.  With two waves per SIMD (NW = 8, or OCC = 2) each wave keeps at most
// 256 registers per lane, and one wave's products overlap another's epilogue.
// WL: every problem of the launch is H = sqrt(<p, D p>) (its multiplier phase compiled in).
template <int MODE, int CT, int RG, int OCC, int NW, int KS = 1, bool WL = false>
__global__ void __launch_bounds__(NW * 64, OCC)
dense_kernel(const DenseProb* __restrict__ probs, const DenseChunk* __restrict__ chunks, int nchunks,
             int* __restrict__ chunk_counter, float* __restrict__ ws, double* __restrict__ ws64,
             int64_t ws_per_wg, int64_t ws64_per_wg, int distance, int anchor_every, int anchor_wait, int det) {
  constexpr int PT = 16 * CT;
  static_assert(KS == 1 || MODE == 2, "the split contraction is for the FP32 refined mode");
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  __shared__ ColShared<PT, NW> S;
  __shared__ double red3[NW][PT];  // third partial of the multiplier sums (sqrt(<p, D p>))
  __shared__ int wsel[PT];         // columns in a multiplier solve: 1 plain, 2 increment, 3 anchor

  const int tid = threadIdx.x;
  const int wave = tid >> 6, l = tid & 63;
  float* const wsb = ws + (int64_t)blockIdx.x * ws_per_wg;

  if (tid < PT) { S.state[tid] = COL_EMPTY; S.fresh[tid] = 0; }
  if (tid == 0) {
    int taken = 0;
    const int c0 = next_chunk(chunk_counter, det, (int)blockIdx.x, (int)gridDim.x, taken);
    S.ctl[CTL_TAKEN] = taken;
    if (c0 >= nchunks) {
      S.ctl[CTL_EXIT] = 1;
    } else {
      S.ctl[CTL_EXIT] = 0;
      S.ctl[CTL_PROB] = chunks[c0].prob;
      S.ctl[CTL_NEXTCOL] = chunks[c0].col0;
      S.ctl[CTL_CHUNKEND] = chunks[c0].col0 + chunks[c0].ncols;
    }
    S.ctl[CTL_PENDING] = -1; S.ctl[CTL_NOMORE] = 0; S.ctl[CTL_ANCHOR] = 0; S.ctl[CTL_LAST_ANCHOR] = 0;
  }
  __syncthreads();
  if (S.ctl[CTL_EXIT]) return;

  int k_it = 0;
  while (true) {
    __syncthreads();  // every control word read in the previous pass is consumed before it changes
    const DenseProb pb = probs[S.ctl[CTL_PROB]];  // by value: fields stay in registers
    const int n = pb.n, n_pad = pb.n_pad, K = pb.K;
    const double lam = pb.lambda;
    const float flam = (float)lam;
    const bool has_l1 = !distance && hk_has_l1(pb.hkind);
    const bool has_l2 = distance || hk_has_l2(pb.hkind);
    const bool wl2 = WL && !distance;  // sqrt(<p, D p>) (HA's, in its eigenbasis)
    float* const za = wsb;
    float* const dz = wsb + (int64_t)PT * n_pad;
    float* const ea = wsb + 2 * (int64_t)PT * n_pad;
    float* const pout = wsb + 3 * (int64_t)PT * n_pad;
    float* const vpart = wsb + 4 * (int64_t)PT * n_pad;  // KS = 2: the first half's partial products
    const int nq = n_pad >> 2;
    const int RT = n_pad >> 4;

    // sqrt(<p, D p>): multiplier solves.  A sweep sums three terms over the rows of every column
    // with wsel != 0 (wave w takes the row tiles w, w + NW, ...; a lane's rows as in the epilogue)
    // into S.red[w][c][0..1] and red3[w][c]; then `update` (thread c of wave 0) takes the column
    // sums and says whether the column needs another sweep; at most `cap` sweeps.
    auto wl2_solve = [&](int cap, auto&& term, auto&& update) {
      for (int it = 0; it < cap; ++it) {
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          const int c = 16 * ct + (l & 15);
          double p[3] = {0.0, 0.0, 0.0};
          const int sel = wsel[c];
          if (sel)
            for (int rt = wave; rt < RT; rt += NW) term(c, sel, st_block(rt, ct, RT) + 4 * l, 16 * rt + 4 * (l >> 4), p);
#pragma unroll
          for (int q = 0; q < 3; ++q) { p[q] += __shfl_xor(p[q], 16); p[q] += __shfl_xor(p[q], 32); }
          if (l < 16) { S.red[wave][c][0] = p[0]; S.red[wave][c][1] = p[1]; red3[wave][c] = p[2]; }
        }
        __syncthreads();
        if (wave == 0) {
          bool more = false;
          if (tid < PT && wsel[tid]) {
            double q0 = 0.0, q1 = 0.0, q2 = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) { q0 += S.red[w][tid][0]; q1 += S.red[w][tid][1]; q2 += red3[w][tid]; }
            more = update(tid, it, q0, q1, q2, it + 1 == cap);
            if (!more) wsel[tid] = 0;
          }
          const bool any = __any(more);
          if (l == 0) S.ctl[CTL_WL2] = any ? 1 : 0;
        }
        __syncthreads();
        if (!S.ctl[CTL_WL2]) break;
      }
    };
    // an anchor: phi(mu; za) = sum s za^2 / (s + mu)^2 and -1/2 its derivative in FP64, and
    // sum za^2 / s (= phi(0; za): za lies inside when it is <= 1)
    auto term_anchor = [&](int c, int sel, size_t et, int row0, double* p) {
      const f32x4 zv = ld_nt4(za + et);
      const double th2 = S.th2[c], mu = S.gama[c];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double sv = th2 * *gp(pb.w + row0 + q);
        if (!(sv > 0.0)) continue;
        const double z = (double)zv[q], inv = 1.0 / (sv + mu), e = sv * z * z * inv * inv;
        p[0] += z * z / sv; p[1] += e; p[2] += e * inv;
      }
    };
    // Newton on 1/sqrt(phi) - 1 from mu = 0 (increasing monotonically to the root); FP64
    auto upd_anchor = [&](int c, int it, double qi, double ph, double ps, bool last) -> bool {
      if (it == 0 && !(qi > 1.0)) {  // za inside: d^a = 0
        S.gama[c] = 0.0; S.ssa2[c] = qi - 1.0; S.flags[c] |= FLAG_INSIDE | FLAG_CIN;
        return false;
      }
      const double mu = S.gama[c], stp = ph * (sqrt(ph) - 1.0) / ps;
      if (!(stp > 1e-15 * mu) || last) {  // phi(mu^a; za) - 1: the increments' reference
        S.ssa2[c] = ph - 1.0; S.flags[c] &= ~(FLAG_INSIDE | FLAG_CIN);
        return false;
      }
      S.gama[c] = mu + stp;
      return true;
    };
    // a pass, FP32 terms.  Plain (wsel 1): the sums of the anchor's form for z = za at mu.
    // Increment (wsel 2): sum z^2 / s, F(dmu) - (phi(mu^a; za) - 1) and -F'(dmu) / 2 with
    //   F(dmu) = sum s a b / ((s + mu)^2 (s + mu^a)^2) + phi(mu^a; za) - 1,
    //   a = dz (s + mu^a) - za dmu,  b = z (s + mu^a) + za (s + mu),  z = za + dz,
    // which is phi(mu; z) - 1 written with increments; F' = -2 sum s z^2 / (s + mu)^3.
    auto term_pass = [&](int c, int sel, size_t et, int row0, double* p) {
      const f32x4 zv = ld_nt4(za + et);
      const f32x4 dv = sel == 2 ? ld_nt4(dz + et) : f32x4{0.f, 0.f, 0.f, 0.f};
      const f32x4 wv = *gp((const f32x4*)(pb.wf + row0));
      const float th2f = (float)S.th2[c];
      float a0 = 0.f, a1 = 0.f, a2 = 0.f;
      if (sel == 1) {
        const float mu = (float)S.gam[c];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float sv = theta_f(th2f, wv[q]);
          if (!(sv > 0.f)) continue;
          const float z = zv[q], iB = __builtin_amdgcn_rcpf(sv + mu), e = sv * z * z * iB * iB;
          a0 += z * z * __builtin_amdgcn_rcpf(sv); a1 += e; a2 += e * iB;
        }
      } else {
        const float mua = (float)S.gama[c], dm = (float)S.dgam[c], mu = mua + dm;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float sv = theta_f(th2f, wv[q]);
          if (!(sv > 0.f)) continue;
          const float zA = zv[q], d = dv[q], z = zA + d, A = sv + mua, B = sv + mu;
          const float iA = __builtin_amdgcn_rcpf(A), iB = __builtin_amdgcn_rcpf(B);
          const float a = d * A - zA * dm, b = z * A + zA * B;
          a0 += z * z * __builtin_amdgcn_rcpf(sv);
          a1 += sv * a * b * (iB * iB) * (iA * iA);
          a2 += sv * z * z * (iB * iB * iB);
        }
      }
      p[0] += (double)a0; p[1] += (double)a1; p[2] += (double)a2;
    };
    // plain: warm-started Newton on 1/sqrt(phi) - 1 (a step from the right of the root lands
    // left of it, clamped at 0; from the left the steps increase monotonically); increment: two
    // Newton steps on F, warm-started from the last pass's dmu (mu stays >= 0)
    auto upd_pass = [&](int c, int it, double q0, double q1, double q2, bool last) -> bool {
      if (wsel[c] == 1) {
        if (it == 0) {
          if (!(q0 > 1.0)) { S.gam[c] = 0.0; S.flags[c] |= FLAG_CIN; return false; }
          S.flags[c] &= ~FLAG_CIN;
        }
        if (!(q2 > 0.0)) return false;
        const double stp = q1 * (sqrt(q1) - 1.0) / q2;
        const double mu = fmax(S.gam[c] + stp, 0.0);
        S.gam[c] = mu;
        return !last && fabs(stp) > (MODE == 0 ? 1e-6 : 1e-5) * mu;
      }
      if (it == 0) {
        if (!(q0 > 1.0)) S.flags[c] |= FLAG_CIN;
        else S.flags[c] &= ~FLAG_CIN;
      }
      if (!(S.flags[c] & FLAG_CIN) && q2 > 0.0)
        S.dgam[c] = fmax(S.dgam[c] + (q1 + S.ssa2[c]) / (2.0 * q2), -S.gama[c]);
      return it == 0 && !last;
    };

    // ================================================================ anchor (REFINED mode)
    if (MODE >= 1 && S.ctl[CTL_ANCHOR]) {
      // pass A (block order, as the epilogue): renormalise z = za + dz (za the nearest float, dz
      // the remainder), the exact anchor reference s_a in FP64, and the norms of the shrink2 factors
      {
        double pss[CT], pinc[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          pss[ct] = 0.0; pinc[ct] = 0.0;
          const int c = 16 * ct + (l & 15);
          const int st = S.state[c];
          if (st != COL_ACTIVE && st != COL_WAITING) continue;
          const double th1 = S.th1[c];
          constexpr int PB = (OCC == 2 || NW == 8) ? 2 : 4;  // row tiles whose loads are in flight together
          for (int rtb = wave; rtb < RT; rtb += NW * PB) {
            f32x4 zv[PB], dv[PB], wv[PB];
#pragma unroll
            for (int u = 0; u < PB; ++u) {
              const int rtc = (rtb + NW * u) < RT ? rtb + NW * u : 0;
              const size_t et = st_block(rtc, ct, RT) + 4 * l;
              zv[u] = ld_nt4(za + et); dv[u] = ld_nt4(dz + et);
              wv[u] = *gp((const f32x4*)(pb.wf + 16 * rtc + 4 * (l >> 4)));
            }
#pragma unroll
            for (int u = 0; u < PB; ++u) {
              const int rt = rtb + NW * u;
              if (rt >= RT) continue;  // wave-uniform
              const int row0 = 16 * rt + 4 * (l >> 4);
              const size_t et = st_block(rt, ct, RT) + 4 * l;
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const double z = (double)zv[u][q] + (double)dv[u][q];
                const float zan = (float)z;
                const float dzn = (float)(z - (double)zan);
                zv[u][q] = zan; dv[u][q] = dzn;
                const float th = theta_f((float)th1, wv[u][q]);
                const float ca = clampf(zan, -th, th), sa = zan - ca;
                const float ds = dzn - clampf(dzn + sa, -th - ca, th - ca);
                const double sa64 = anchor_shrink(zan, th1, pb.w, row0 + q);
                pss[ct] += sa64 * sa64;
                pinc[ct] += (double)ds * (2.0 * (double)sa + (double)ds);
              }
              st_nt4(za + et, zv[u]); st_nt4(dz + et, dv[u]);
            }
          }
        }
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          double a = pss[ct], b = pinc[ct];
          a += __shfl_xor(a, 16); a += __shfl_xor(a, 32);
          b += __shfl_xor(b, 16); b += __shfl_xor(b, 32);
          if (l < 16) { S.red[wave][16 * ct + l][0] = a; S.red[wave][16 * ct + l][1] = b; }
        }
        __syncthreads();
        if (tid < PT) {
          const int c = tid;
          const int st = S.state[c];
          if (st == COL_ACTIVE || st == COL_WAITING) {
            double pssc = 0.0, pincc = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) { pssc += S.red[w][c][0]; pincc += S.red[w][c][1]; }
            S.ssa2[c] = pssc;
            const double ssq = pssc + pincc;
            S.ssq[c] = ssq;
            double ga = 1.0, g = 1.0;
            if (has_l2) {
              const double na = sqrt(pssc), nz = sqrt(fmax(ssq, 0.0)), th2 = S.th2[c];
              ga = na > 0.0 ? fmax(na - th2, 0.0) / na : 0.0;
              g = nz > 0.0 ? fmax(nz - th2, 0.0) / nz : 0.0;
            }
            S.gama[c] = ga; S.gam[c] = g; S.dgam[c] = g - ga;
            S.phase[c] = PH_DELTA;
          }
        }
      }
      __syncthreads();
      if (wl2) {  // the anchor's multiplier mu^a of za (as renormalised above), in FP64
        if (tid < PT) {
          const int st = S.state[tid];
          const bool on = st == COL_ACTIVE || st == COL_WAITING;
          wsel[tid] = on ? 3 : 0;
          if (on) { S.gama[tid] = 0.0; S.dgam[tid] = 0.0; }
        }
        __syncthreads();
        wl2_solve(kWl2AnchorNewton, term_anchor, upd_anchor);
      }
      // v^a = M r^a; ea = v^a - d^a.  r^a = x' + lambda (2 d^a - z^a) is formed once per anchor in
      // FP64 (the workgroup's staging, column-major, n_pad per column) and the product is taken in
      // integer slices (the kSlices definitions): M and r^a are split into kSlices 7-bit slices
      // under per-row and per-column power-of-two scales, and the slice products with
      // a + b <= kSlices + 1 (1-based) are accumulated exactly.  The dropped pairs (a + b = 8:
      // five of them, each term below 2^-44 of 2^(e_i + f_c)) and the truncated slices (below
      // 2^-43 of the scale per entry) leave at most ~ 7 n_pad 2^-44 of 2^(e_i + f_c), about 2^-31
      // at n_pad = 1024, i.e. 2^-29 of max_k |M_ik| max_k |r_kc| in the worst case: far below what
      // the anchor has to resolve, while the int8 products run many times faster than FP64 ones.
      {
        double* const ra = ws64 + (int64_t)blockIdx.x * ws64_per_wg;
        const int n64 = pad64(n_pad);
        int8_t* const rq = (int8_t*)(ra + (size_t)PT * n_pad);  // kSlices x PT x n64 bytes
        double cmax[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          cmax[ct] = 0.0;
          const int c = 16 * ct + (l & 15);
          const int st = S.state[c];
          const bool on = st == COL_ACTIVE || st == COL_WAITING;
          const double th1 = S.th1[c], ga = S.gama[c], th2 = S.th2[c];
          const bool ains = S.flags[c] & FLAG_INSIDE;
          const HOPF_GLOBAL float* xj = gp(pb.x + (size_t)S.j[c] * n);
          const HOPF_GLOBAL double* cen = pb.centres ? gp(pb.centres + (size_t)S.k[c] * n_pad) : nullptr;
          constexpr int PB = (OCC == 2 || NW == 8) ? 2 : 4;  // row tiles whose loads are in flight together
          for (int rtb = wave; rtb < RT; rtb += NW * PB) {
            f32x4 zv[PB];
#pragma unroll
            for (int u = 0; u < PB; ++u) {
              const int rtc = (rtb + NW * u) < RT ? rtb + NW * u : 0;
              zv[u] = on ? ld_nt4(za + st_block(rtc, ct, RT) + 4 * l) : f32x4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int u = 0; u < PB; ++u) {
              const int rt = rtb + NW * u;
              if (rt >= RT) continue;  // wave-uniform
              const int row0 = 16 * rt + 4 * (l >> 4);
              double rv[4] = {0.0, 0.0, 0.0, 0.0};
              if (on) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                  const int row = row0 + q;
                  if (row < n) {
                    const double da = wl2 ? wl2_da(zv[u][q], th2 * *gp(pb.w + row), ga, ains)
                                          : ga * anchor_shrink(zv[u][q], th1, pb.w, row);
                    const double xp = (double)xj[row] - (cen ? cen[row] : 0.0);
                    rv[q] = xp + lam * (2.0 * da - (double)zv[u][q]);
                    cmax[ct] = fmax(cmax[ct], fabs(rv[q]));
                  }
                }
              }
              HOPF_GLOBAL double* dst = gp(ra + (size_t)c * n_pad + row0);
              *(HOPF_GLOBAL f64x2*)dst = f64x2{rv[0], rv[1]};
              *(HOPF_GLOBAL f64x2*)(dst + 2) = f64x2{rv[2], rv[3]};
            }
          }
        }
        // column scales: the largest |r^a| of each column, over the lane groups, then the waves
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          double m = cmax[ct];
          m = fmax(m, __shfl_xor(m, 16));
          m = fmax(m, __shfl_xor(m, 32));
          if (l < 16) S.red[wave][16 * ct + l][0] = m;
        }
        __syncthreads();  // the staging is complete (written and read by this workgroup only)
        if (tid < PT) {
          double m = 0.0;
#pragma unroll
          for (int w = 0; w < NW; ++w) m = fmax(m, S.red[w][tid][0]);
          S.rexp[tid] = slice_exponent(m);
        }
        __syncthreads();
        // the slices of r^a, [slice][column][k] with n64 bytes per column (zero beyond n_pad);
        // each thread takes 4 consecutive k of one column
        {
          const int q4 = n64 >> 2;
          for (int u = tid; u < PT * q4; u += NW * 64) {
            const int c = u / q4, k4 = 4 * (u - c * q4);
            const int fe = S.rexp[c];
            uint32_t word[kSlices];
#pragma unroll
            for (int s = 0; s < kSlices; ++s) word[s] = 0u;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int k = k4 + e;
              double x = k < n_pad ? ldexp(*gp(ra + (size_t)c * n_pad + k), -fe) : 0.0;
#pragma unroll
              for (int s = 0; s < kSlices; ++s) {
                x *= 128.0;
                const double r = rint(x);
                x -= r;
                word[s] |= (uint32_t)(uint8_t)(int8_t)(int)r << (8 * e);
              }
            }
#pragma unroll
            for (int s = 0; s < kSlices; ++s) *gp((uint32_t*)(rq + ((size_t)s * PT + c) * n64 + k4)) = word[s];
          }
        }
        // products, one row tile per wave and pass; the slices of r^a stream through LDS in blocks
        // of kbq rows of all PT columns (the BF16 right-hand-side buffer is free during an
        // anchor), and every wave takes part in every block, also one without a row tile
        const int kbq = anchor_kbq(n_pad), ldq = kbq + 16;
        int8_t* const Bq = (int8_t*)lds_raw;
        for (int rt0 = 0; rt0 < RT; rt0 += NW) {
          const int rt = rt0 + wave;
          const bool has = rt < RT;  // wave-uniform
          i32x4 acc[kSlices][CT];
#pragma unroll
          for (int s = 0; s < kSlices; ++s)
#pragma unroll
            for (int c = 0; c < CT; ++c) acc[s][c] = i32x4{0, 0, 0, 0};
          for (int k0 = 0; k0 < n64; k0 += kbq) {
            const int kb = n64 - k0 < kbq ? n64 - k0 : kbq;  // a multiple of 64
            const int hu = kb >> 4;                           // 16-byte units per slice and column
            __syncthreads();  // the slices are written (first block) or the previous block is consumed
            for (int u = tid; u < kSlices * PT * hu; u += NW * 64) {
              const int sc = u / hu, off = 16 * (u - sc * hu);  // sc = slice PT + column
              *(i32x4*)(Bq + sc * ldq + off) = *gp((const i32x4*)(rq + (size_t)sc * n64 + k0 + off));
            }
            __syncthreads();
            if (has) gemm_slices<CT>(pb.Mq, RT, n64 >> 6, rt, k0 >> 6, kb >> 6, Bq, ldq, acc);
          }
          if (!has) continue;  // after the last barrier of the pass
          const int row0 = 16 * rt + 4 * (l >> 4);
          int rexp_row[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) rexp_row[i] = *gp(pb.Mqe + row0 + i);
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            const int c = 16 * ct + (l & 15);
            const int st = S.state[c];
            if (st != COL_ACTIVE && st != COL_WAITING) continue;
            const double ga = S.gama[c];
            const int fe = S.rexp[c];
            f32x4 ev;
            const size_t et = st_block(rt, ct, RT) + 4 * l;
            const f32x4 zv = ld_nt4(za + et);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int row = row0 + i;
              double v = 0.0;  // smallest terms first
#pragma unroll
              for (int s = kSlices - 1; s >= 0; --s) v += ldexp((double)acc[s][ct][i], rexp_row[i] + fe - 7 * (s + 2));
              const double da = wl2 ? wl2_da(zv[i], S.th2[c] * *gp(pb.w + row), ga, S.flags[c] & FLAG_INSIDE)
                                    : ga * anchor_shrink(zv[i], S.th1[c], pb.w, row);
              ev[i] = (row < n) ? (float)(v - da) : 0.f;
            }
            st_nt4(ea + et, ev);
          }
        }
      }
      __syncthreads();
      if (tid < PT && S.state[tid] == COL_WAITING) S.state[tid] = COL_PHI;
      if (tid == 0) { S.ctl[CTL_ANCHOR] = 0; S.ctl[CTL_LAST_ANCHOR] = k_it; }
      __syncthreads();
    }
    if (MODE == 0) {  // plain mode: converged columns are evaluated right away
      if (tid < PT && S.state[tid] == COL_WAITING) S.state[tid] = COL_PHI;
      __syncthreads();
    }

    // ================================================================ flush finished slots
    // With one copy per point (and no distance), each finished slot writes its own scalars (its
    // p was written to the output by its value iteration); only invalid slots are left for the
    // copy pass below, which writes their NaN rows.
    // Otherwise thread 0 settles the outputs of every finished slot in slot order (the best copy
    // of a point so far, lowest copy index on ties), marking the slot whose p is to be written;
    // then all threads copy those vectors.  Copies of one point live in one workgroup, so the
    // best value of a point is only ever compared here, by this thread.
    const bool single = pb.K == 1 && !distance;
    if (single) {
      int nan_rows = 0;
      if (tid < PT) {
        const int c = tid;
        const int st = S.state[c];
        int better = 0;
        if (st == COL_DONE || st == COL_INVALID) {
          const int64_t j = S.j[c];
          if (pb.iter_total) atomicAdd(pb.iter_total, (unsigned long long)S.iters[c]);
          const float qnan = __builtin_nanf("");
          if (st == COL_INVALID) {
            better = 2;
            pb.phi[j] = qnan; pb.dphidt[j] = qnan;
            if (pb.iters) pb.iters[j] = -1;
            if (pb.kstar) pb.kstar[j] = -1;
          } else {
            pb.phi[j] = (float)S.phi[c];
            pb.dphidt[j] = (float)(-S.hp[c]);
            if (pb.iters) pb.iters[j] = (S.flags[c] & FLAG_CAPPED) ? -2 : S.iters[c];
            if (pb.kstar) pb.kstar[j] = 0;
            S.state[c] = COL_EMPTY;
          }
        }
        S.better[c] = better;
        nan_rows = better == 2;
      }
      if (tid == 0) S.ctl[CTL_BETTER] = 0;
      __syncthreads();
      if (nan_rows) S.ctl[CTL_BETTER] = 1;  // benign race: every writer stores 1
    } else if (tid == 0) {
      int any = 0;
      for (int c = 0; c < PT; ++c) {
        S.better[c] = 0;
        const int st = S.state[c];
        if (st != COL_DONE && st != COL_INVALID) continue;
        any = 1;
        if (pb.iter_total) atomicAdd(pb.iter_total, (unsigned long long)S.iters[c]);
        const int64_t j = S.j[c];
        const int kk = S.k[c];
        int better;
        if (st == COL_INVALID) {
          better = 2;
        } else {
          const double key = distance ? ((S.flags[c] & FLAG_INSIDE) ? -1.0 : S.s[c]) : S.phi[c];
          const int bk = pb.bestk[j];
          const double bv = pb.bestv[j];
          better = (bk < 0 || key < bv || (key == bv && kk < bk)) ? 1 : 0;
          if (better) { pb.bestv[j] = key; pb.bestk[j] = kk; }
        }
        if (better) {  // an earlier slot of this pass that wrote the same point is superseded
          for (int c2 = 0; c2 < c; ++c2)
            if (S.better[c2] && S.j[c2] == S.j[c]) S.better[c2] = 0;
        }
        S.better[c] = better;
        const float qnan = __builtin_nanf("");
        if (better == 2) {
          pb.bestk[j] = -2;
          if (!distance) {
            pb.phi[j] = qnan; pb.dphidt[j] = qnan;
            if (pb.iters) pb.iters[j] = -1;
            if (pb.kstar) pb.kstar[j] = -1;
          } else {
            pb.dist[j] = qnan;
            if (pb.kstar) pb.kstar[j] = -1;
            if (pb.inside) pb.inside[j] = 0;
            if (pb.newton) pb.newton[j] = -1;
          }
        } else if (better == 1) {
          if (!distance) {
            pb.phi[j] = (float)S.phi[c];
            pb.dphidt[j] = (float)(-S.hp[c]);
            if (pb.iters) pb.iters[j] = (S.flags[c] & FLAG_CAPPED) ? -2 : S.iters[c];
            if (pb.kstar) pb.kstar[j] = kk;
          } else {
            const bool ins = S.flags[c] & FLAG_INSIDE;
            pb.dist[j] = ins ? 0.f : (float)S.s[c];
            if (pb.kstar) pb.kstar[j] = kk;
            if (pb.inside) pb.inside[j] = ins ? 1 : 0;
            if (pb.newton) pb.newton[j] = (S.flags[c] & (FLAG_CAPPED | FLAG_NEWTON_CAP)) ? -2 : S.newton[c];
          }
        }
      }
      S.ctl[CTL_BETTER] = any;
    }
    __syncthreads();
    if (S.ctl[CTL_BETTER]) {
      for (int c = wave; c < PT; c += NW) {  // one wave per slot, lanes over coordinates
        const int better = S.better[c];
        if (!better) continue;
        const int64_t j = S.j[c];
        const bool ins = S.flags[c] & FLAG_INSIDE;
        const double sc = distance ? S.s[c] / S.pn[c] : 0.0;
        for (int i = l; i < n; i += 64) {
          float v;
          if (better == 2) v = __builtin_nanf("");
          else if (!distance) v = ld_nt(pout + (size_t)c * n_pad + i);
          else {
            const float y = pb.x[(size_t)j * n + i];
            v = ins ? y : (float)((double)y - sc * (double)ld_nt(pout + (size_t)c * n_pad + i));
          }
          pb.grad[(size_t)j * n + i] = v;
        }
      }
      __syncthreads();
      if (tid < PT && (S.state[tid] == COL_DONE || S.state[tid] == COL_INVALID)) S.state[tid] = COL_EMPTY;
      __syncthreads();
    }

    // ================================================================ refill empty slots
    if (tid == 0) {
      int prob = S.ctl[CTL_PROB], nextcol = S.ctl[CTL_NEXTCOL], cend = S.ctl[CTL_CHUNKEND];
      int pending = S.ctl[CTL_PENDING], nomore = S.ctl[CTL_NOMORE], taken = S.ctl[CTL_TAKEN];
      int live = 0;
      for (int c = 0; c < PT; ++c) {
        S.fresh[c] = 0;
        if (S.state[c] != COL_EMPTY) { ++live; continue; }
        while (nextcol >= cend && pending < 0 && !nomore) {
          const int nc = next_chunk(chunk_counter, det, (int)blockIdx.x, (int)gridDim.x, taken);
          if (nc >= nchunks) { nomore = 1; break; }
          if (chunks[nc].prob == prob) { nextcol = chunks[nc].col0; cend = nextcol + chunks[nc].ncols; }
          else pending = nc;
        }
        if (nextcol < cend) {
          const int col = nextcol++;
          S.col[c] = col; S.j[c] = col / K; S.k[c] = col % K;
          S.fresh[c] = 1;
          ++live;
        }
      }
      int exitf = 0;
      if (live == 0) {
        if (pending >= 0) {  // all slots drained: switch to the pending problem
          prob = chunks[pending].prob;
          nextcol = chunks[pending].col0;
          cend = nextcol + chunks[pending].ncols;
          pending = -1;
          S.ctl[CTL_ANY] = 1;  // ask for another refill pass with the new problem
        } else {
          exitf = 1;
          S.ctl[CTL_ANY] = 0;
        }
      } else {
        S.ctl[CTL_ANY] = 0;
      }
      S.ctl[CTL_PROB] = prob; S.ctl[CTL_NEXTCOL] = nextcol; S.ctl[CTL_CHUNKEND] = cend;
      S.ctl[CTL_PENDING] = pending; S.ctl[CTL_NOMORE] = nomore; S.ctl[CTL_EXIT] = exitf;
      S.ctl[CTL_TAKEN] = taken;
    }
    __syncthreads();
    if (S.ctl[CTL_EXIT]) break;
    if (S.ctl[CTL_ANY]) {  // problem switch: restart the loop body with the new problem's view
      if (tid == 0) { S.ctl[CTL_LAST_ANCHOR] = k_it; S.ctl[CTL_ANCHOR] = 0; }
      __syncthreads();
      continue;
    }
    // initialise the fresh slots: scalars ...
    if (tid < PT && S.fresh[tid]) {
      const int c = tid;
      const int64_t jj = S.j[c];
      const double tv = distance ? 0.0 : (double)pb.t[jj];
      S.t[c] = tv;
      S.state[c] = (distance || (tv > 0.0 && isfinite(tv))) ? COL_ACTIVE : COL_INVALID;
      S.th1[c] = has_l1 ? tv / lam : 0.0;
      S.th2[c] = (!distance && has_l2) ? tv / lam : 0.0;
      S.gam[c] = 1.0; S.gama[c] = 1.0; S.dgam[c] = 0.0; S.ssa2[c] = 0.0; S.ssq[c] = 0.0;
      if (wl2) { S.th2[c] = (tv / lam) * (tv / lam); S.gam[c] = 0.0; S.gama[c] = 0.0; }  // s_i = th2 w_i; mu
      S.prev[c] = 1e300; S.s[c] = 0.0; S.phi[c] = 0.0; S.hp[c] = 0.0; S.pn[c] = 0.0;
      S.best[c] = 1e300; S.stall[c] = 0;
      S.iters[c] = 0; S.newton[c] = 0; S.flags[c] = FLAG_FIRST; S.phase[c] = PH_WARMUP;
    }
    __syncthreads();
    // ... and state (one wave per slot; also the finiteness check)
    for (int c = wave; c < PT; c += NW) {
      if (!S.fresh[c]) continue;
      const int st = S.state[c];
      bool bad = false;
      const double* cen = pb.centres ? pb.centres + (size_t)S.k[c] * n_pad : nullptr;
      const float* xj = pb.x + (size_t)S.j[c] * n;
      for (int i = l; i < n_pad; i += 64) {
        float v = 0.f;
        if (i < n) {
          const float xv = xj[i];
          if (!isfinite(xv)) bad = true;
          v = (float)((double)xv - (cen ? cen[i] : 0.0));
        }
        // until the first anchor, ea holds x' (the right-hand side of the plain iterations)
        const size_t e = st_index(c, i, RT);
        const float v0 = (st == COL_ACTIVE) ? v : 0.f;
        st_nt(za + e, v0);
        st_nt(dz + e, 0.f);
        st_nt(ea + e, v0);
      }
      const bool anybad = __any(bad);
      if (l == 0 && anybad && st == COL_ACTIVE) S.state[c] = COL_INVALID;
    }
    __syncthreads();
    {  // anything to iterate?  (invalid slots are flushed at the top of the next pass)
      if (tid == 0) {
        int live = 0;
        for (int c = 0; c < PT; ++c) {
          const int st = S.state[c];
          live |= (st == COL_ACTIVE || st == COL_PHI) ? 1 : (st == COL_INVALID ? 2 : 0);
        }
        S.ctl[CTL_ANY] = live;
      }
      __syncthreads();
      if (!(S.ctl[CTL_ANY] & 1)) {
        if (S.ctl[CTL_ANY] & 2) continue;  // only invalid slots: flush them
        // only waiting slots remain: an anchor (REFINED) makes them evaluable
        if (tid == 0) S.ctl[CTL_ANCHOR] = 1;
        __syncthreads();
        continue;
      }
    }

    value_clear(S, tid);  // value sums of this pass (ordered before their updates by the barrier below)
    // ================================================================ prologue: right-hand sides
    // Block order: wave w takes the row tiles w, w+4, ... of every column tile; lane l works on
    // rows 16 rt + 4 (l/16) .. + 3 of column 16 ct + l%16, its block's contiguous 16 bytes.
    // With KS = 2 the right-hand sides of one half of the rows at a time: rows of row tiles
    // [rt_lo, rt_hi) at LDS rows from 16 rt_lo.
    const int ldb = MODE == 1 ? n_pad + 8 : n_pad / KS + 4;  // BF16 (MODE 1) or FP32 right-hand sides
    auto prologue = [&](int rt_lo, int rt_hi) {
      constexpr int PB = (OCC == 2 || NW == 8) ? 2 : 4;  // row tiles whose loads are in flight together
      const int kbase = 16 * rt_lo;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int c = 16 * ct + (l & 15);
        const int st = S.state[c];
        const bool on = st == COL_ACTIVE || st == COL_PHI;
        const bool deltac = MODE >= 1 && S.phase[c] == PH_DELTA;
        const bool first = S.flags[c] & FLAG_FIRST;
        const float gaf = (float)S.gama[c], dgf = (float)S.dgam[c], gf = (float)S.gam[c];
        const float th1f = (float)S.th1[c], th2f = (float)S.th2[c];
        const bool ains = S.flags[c] & FLAG_INSIDE, cin = S.flags[c] & FLAG_CIN;
        // batches of PB row tiles: all their state loads are in flight before any is used
        const float* sv_src = deltac ? dz : ea;  // increment (delta phase) or x' (plain)
        for (int rtb = rt_lo + wave; rtb < rt_hi; rtb += NW * PB) {
          f32x4 zv[PB], sv[PB], wv[PB];
#pragma unroll
          for (int u = 0; u < PB; ++u) {
            const int rt = rtb + NW * u;
            const int rtc = rt < rt_hi ? rt : rt_lo;  // in-bounds address; result not stored
            const size_t et = st_block(rtc, ct, RT) + 4 * l;
            if (on) {
              zv[u] = ld_nt4(za + et);
              sv[u] = ld_nt4(sv_src + et);
              wv[u] = *gp((const f32x4*)(pb.wf + 16 * rtc + 4 * (l >> 4)));
            } else {
              zv[u] = f32x4{0.f, 0.f, 0.f, 0.f}; sv[u] = zv[u]; wv[u] = zv[u];
            }
          }
#pragma unroll
          for (int u = 0; u < PB; ++u) {
            const int rt = rtb + NW * u;
            if (rt >= rt_hi) continue;  // wave-uniform
            const int row0 = 16 * rt + 4 * (l >> 4);
            f32x4 rv = {0.f, 0.f, 0.f, 0.f};
            if (on) {
              if (deltac) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                  const float th = theta_f(th1f, wv[u][q]);
                  const float ca = clampf(zv[u][q], -th, th), sa = zv[u][q] - ca;
                  const float ds = sv[u][q] - clampf(sv[u][q] + sa, -th - ca, th - ca);
                  const float dd = wl2 ? wl2_dd(zv[u][q], sv[u][q], theta_f(th2f, wv[u][q]), gaf, dgf, ains, cin)
                                       : gaf * ds + dgf * (sa + ds);
                  rv[q] = flam * (2.f * dd - sv[u][q]);
                }
              } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                  const float z = zv[u][q];
                  const float th = theta_f(th1f, wv[u][q]);
                  const float d = first ? z
                                  : (wl2 ? wl2_d(z, theta_f(th2f, wv[u][q]), gf, cin) : gf * (z - clampf(z, -th, th)));
                  rv[q] = sv[u][q] + flam * (2.f * d - z);
                }
              }
            }
            if (MODE == 1) {
              typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
              bf16x4 o;
#pragma unroll
              for (int q = 0; q < 4; ++q) o[q] = to_bf16(rv[q]);
              *(bf16x4*)((__bf16*)lds_raw + c * ldb + row0) = o;
            } else {
              *(f32x4*)((float*)lds_raw + c * ldb + row0 - kbase) = rv;
            }
          }
        }
      }
    };
    prologue(0, RT / KS);
    __syncthreads();

    // ================================================================ GEMM + epilogue
    float part[CT][2];  // this lane's step^2 and |s|^2 (increment) partials; value sums go to S.redv
#pragma unroll
    for (int c = 0; c < CT; ++c) { part[c][0] = 0.f; part[c][1] = 0.f; }
    // the column scalars of this lane's slots (columns 16 ct + l % 16) are read from LDS where
    // they are used: registers are kept for the products
    // (one 16-column tile: the FP32 refined shape of the largest sizes, whose M streams from
    // beyond L2, so six k-steps of fragments are kept in flight)
    constexpr int PFF = (MODE == 2 && CT == 1) ? 6 : 3;
    const int nks = n_pad >> 4;  // k-steps of the FP32 products
    if (KS == 2) {
      // the contraction over the first half of the rows for every row group, its partial products
      // to the staging (in the state's block layout), then the right-hand sides of the second half
      for (int rt0 = 0; rt0 < RT; rt0 += NW * RG) {
        int rt[RG]; int nrt = 0;
#pragma unroll
        for (int r = 0; r < RG; ++r) { rt[r] = rt0 + wave + NW * r; if (rt[r] < RT) nrt = r + 1; }
        f32x4 acc[RG][CT];
#pragma unroll
        for (int r = 0; r < RG; ++r)
#pragma unroll
          for (int c = 0; c < CT; ++c) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
        gemm_f32<RG, CT, PFF>(pb.Mf, n_pad, (const float*)lds_raw, ldb, rt, nrt, acc, 0, nks / 2);
#pragma unroll
        for (int r = 0; r < RG; ++r) {
          if (r >= nrt) continue;
#pragma unroll
          for (int c = 0; c < CT; ++c) st_nt4(vpart + st_block(rt[r], c, RT) + 4 * l, acc[r][c]);
        }
      }
      __syncthreads();
      prologue(RT / 2, RT);
      __syncthreads();
    }

    for (int rt0 = 0; rt0 < RT; rt0 += NW * RG) {
      int rt[RG]; int nrt = 0;
#pragma unroll
      for (int r = 0; r < RG; ++r) { rt[r] = rt0 + wave + NW * r; if (rt[r] < RT) nrt = r + 1; }
      f32x4 acc[RG][CT];
#pragma unroll
      for (int r = 0; r < RG; ++r)
#pragma unroll
        for (int c = 0; c < CT; ++c)
          acc[r][c] = (KS == 2 && r < nrt) ? ld_nt4(vpart + st_block(rt[r], c, RT) + 4 * l) : f32x4{0.f, 0.f, 0.f, 0.f};
      if (MODE == 1) gemm_bf16<RG, CT>(pb.Mb, n_pad, (const __bf16*)lds_raw, n_pad + 8, rt, nrt, acc);
      else gemm_f32<RG, CT, PFF>(pb.Mf, n_pad, (const float*)lds_raw, ldb, rt, nrt, acc, KS == 2 ? nks / 2 : 0,
                                 nks / KS);

#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int c = 16 * ct + (l & 15);
        const int st = S.state[c];
        if (st != COL_ACTIVE && st != COL_PHI) continue;
        const bool delta = MODE >= 1 && S.phase[c] == PH_DELTA;
        const float th1f = (float)S.th1[c], th2f = (float)S.th2[c];
        const bool ains = S.flags[c] & FLAG_INSIDE, cin = S.flags[c] & FLAG_CIN;
        // the state of all RG row tiles of this column is requested before any of it is used
        f32x4 zst[RG], dst[RG], est[RG], wst[RG];
#pragma unroll
        for (int r = 0; r < RG; ++r) {
          if (r >= nrt) continue;
          const int row0 = 16 * rt[r] + 4 * (l >> 4);
          const size_t et = st_block(rt[r], ct, RT) + 4 * l;
          zst[r] = ld_nt4(za + et);
          wst[r] = *gp((const f32x4*)(pb.wf + row0));
          if (delta) { dst[r] = ld_nt4(dz + et); est[r] = ld_nt4(ea + et); }
        }
#pragma unroll
        for (int r = 0; r < RG; ++r) {
          if (r >= nrt) continue;
          const int row0 = 16 * rt[r] + 4 * (l >> 4);
          const size_t e = (size_t)c * n_pad + row0;      // value staging: column-major
          const size_t et = st_block(rt[r], ct, RT) + 4 * l;  // state: block layout
          const f32x4 v = acc[r][ct];
          f32x4 zav = zst[r];
          if (delta) {
            // COL_PHI also takes the step: with the fresh anchor it re-runs the stopping test on an
            // exact product (a column that converged to a stale anchor's fixed point continues).
            f32x4 dzv = dst[r];
            const f32x4 eav = est[r];
            const float gaf = (float)S.gama[c], dgf = (float)S.dgam[c];
            float s0 = 0.f, s1 = 0.f;
            f32x4 ddv;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const float th = theta_f(th1f, wst[r][q]);
              const float ca = clampf(zav[q], -th, th), sa = zav[q] - ca;
              const float lo = -th - ca, hi = th - ca;
              const float ds = dzv[q] - clampf(dzv[q] + sa, lo, hi);
              const float dd = wl2 ? wl2_dd(zav[q], dzv[q], theta_f(th2f, wst[r][q]), gaf, dgf, ains, cin)
                                   : gaf * ds + dgf * (sa + ds);
              const float step = eav[q] + v[q] - dd;      // z^{k+1} - z^k
              const float dzn = dzv[q] + step;
              const float dsn = dzn - clampf(dzn + sa, lo, hi);
              s0 += step * step;
              s1 += dsn * (2.f * sa + dsn);
              ddv[q] = dd;
              dzv[q] = dzn;
            }
            part[ct][0] += s0;
            part[ct][1] += s1;
            if (st == COL_PHI) {  // value from the exact-product identity at the current iterate
              const double ga = S.gama[c], th1 = S.th1[c];
              const HOPF_GLOBAL float* xj = gp(pb.x + (size_t)S.j[c] * n);
              const double* cen = pb.centres ? pb.centres + (size_t)S.k[c] * n_pad : nullptr;
              const f32x4 dz0 = dst[r];
              f32x4 pv;
              double v2 = 0.0, v3 = 0.0, v4 = 0.0, v5 = 0.0;
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int i = row0 + q;
                const double da = wl2 ? wl2_da(zav[q], S.th2[c] * *gp(pb.w + i), ga, ains)
                                      : ga * anchor_shrink(zav[q], th1, pb.w, i);
                double d = da + (double)ddv[q];
                const double vv = (double)eav[q] + da + (double)v[q];
                const double xp = (i < n) ? (double)xj[i < n ? i : 0] - (cen ? *gp(cen + i) : 0.0) : 0.0;
                const double rr = xp + lam * (2.0 * da - (double)zav[q]) + lam * (2.0 * (double)ddv[q] - (double)dz0[q]);
                if (i >= n) d = 0.0;
                v2 += xp * d;
                v3 += (2.0 * d - vv) * (rr - lam * vv);
                v4 += wl2 ? *gp(pb.w + i) * d * d : (double)wst[r][q] * fabs(d);
                v5 += d * d;
                pv[q] = (float)d;
              }
              value_sums(S.redv[wave][c], v2, v3, v4, v5, l);
              if (single) store_grad(pb.grad + (size_t)S.j[c] * n, row0, n, pv);
              else st_nt4(pout + e, pv);
            }
            st_nt4(dz + et, dzv);
          } else {
            // plain iteration (F32 mode, or the BF16 warm-up): z^{k+1} = z - d + v
            const float gf = (float)S.gam[c];
            const bool first = S.flags[c] & FLAG_FIRST;
            if (st == COL_ACTIVE) {
              float s0 = 0.f, s1 = 0.f;
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const float th = theta_f(th1f, wst[r][q]);
                const float z = zav[q];
                const float d = first ? z
                                : (wl2 ? wl2_d(z, theta_f(th2f, wst[r][q]), gf, cin) : gf * (z - clampf(z, -th, th)));
                const float zn = z - d + v[q];
                const float step = zn - z;
                const float sn = zn - clampf(zn, -th, th);
                s0 += step * step;
                s1 += sn * sn;
                zav[q] = zn;
              }
              part[ct][0] += s0;
              part[ct][1] += s1;
              st_nt4(za + et, zav);
            } else if (MODE == 0) {  // COL_PHI in F32 mode: r is in LDS
              const float* B32 = (const float*)lds_raw;
              const int ldb = n_pad + 4;
              const HOPF_GLOBAL float* xj = gp(pb.x + (size_t)S.j[c] * n);
              const double* cen = pb.centres ? pb.centres + (size_t)S.k[c] * n_pad : nullptr;
              f32x4 pv;
              double v2 = 0.0, v3 = 0.0, v4 = 0.0, v5 = 0.0;
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int i = row0 + q;
                const float th = theta_f(th1f, wst[r][q]);
                const float z = zav[q];
                const float df = first ? z
                                 : (wl2 ? wl2_d(z, theta_f(th2f, wst[r][q]), gf, cin) : gf * (z - clampf(z, -th, th)));
                const double d = (i < n) ? (double)df : 0.0;
                const double vv = (double)v[q];
                const double rr = (double)B32[c * ldb + i];
                const double xp = (i < n) ? (double)xj[i < n ? i : 0] - (cen ? *gp(cen + i) : 0.0) : 0.0;
                v2 += xp * d;
                v3 += (2.0 * d - vv) * (rr - lam * vv);
                v4 += wl2 ? *gp(pb.w + (i < n ? i : 0)) * d * d : (double)wst[r][q] * fabs(d);
                v5 += d * d;
                pv[q] = (float)d;
              }
              value_sums(S.redv[wave][c], v2, v3, v4, v5, l);
              if (single) store_grad(pb.grad + (size_t)S.j[c] * n, row0, n, pv);
              else st_nt4(pout + e, pv);
            }
          }
        }
      }
    }
    // reduce the step partials: over the 4 lane groups, then across waves through LDS
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        double v = (double)part[ct][q];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        if (l < 16) S.red[wave][16 * ct + l][q] = v;
      }
    __syncthreads();

    // ================================================================ per-column update
    if (tid < PT) {
      const int c = tid;
      const int st = S.state[c];
      double sm[kNRed];
      sm[0] = 0.0; sm[1] = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) { sm[0] += S.red[w][c][0]; sm[1] += S.red[w][c][1]; }
#pragma unroll
      for (int q = 2; q < kNRed; ++q) sm[q] = value_total(S, c, q - 2);
      const bool delta = MODE >= 1 && S.phase[c] == PH_DELTA;
      const bool stepped = st == COL_ACTIVE || (MODE >= 1 && st == COL_PHI);
      bool evaluate = (MODE == 0 && st == COL_PHI);
      if (stepped) {
        S.iters[c] += 1;
        const double ssq = delta ? S.ssa2[c] + sm[1] : sm[1];
        S.ssq[c] = ssq;
        double g = 1.0;
        if (has_l2) {
          const double nz = sqrt(fmax(ssq, 0.0));
          g = nz > 0.0 ? fmax(nz - S.th2[c], 0.0) / nz : 0.0;
        }
        if (!wl2) {  // (for sqrt(<p, D p>) gam and dgam hold multipliers, set below)
          S.gam[c] = g;
          S.dgam[c] = g - S.gama[c];
        }
        S.flags[c] &= ~FLAG_FIRST;
        const bool can_stop = (MODE == 0) || delta;
        const double a = sqrt(sm[0]), b = sqrt(S.prev[c]);
        S.prev[c] = sm[0];
        const bool conv = can_stop && (a + b) * (a + b) <= pb.tol;
        bool stalled = false;
        if (MODE == 0) {
          if (sm[0] < S.best[c]) { S.best[c] = sm[0]; S.stall[c] = 0; }
          else stalled = ++S.stall[c] >= kStallIters;
        }
        const bool capped = S.iters[c] >= pb.max_iter || stalled;
        if (st == COL_ACTIVE) {
          if (conv) S.state[c] = COL_WAITING;
          else if (capped) { S.state[c] = COL_WAITING; S.flags[c] |= FLAG_SOLVE_CAP | FLAG_CAPPED; }
        } else {
          if (capped && !conv) S.flags[c] |= FLAG_SOLVE_CAP | FLAG_CAPPED;
          if (conv || (S.flags[c] & FLAG_SOLVE_CAP)) evaluate = true;
          else S.state[c] = COL_ACTIVE;
        }
      }
      if (evaluate) {
        const double tt = distance ? S.s[c] : S.t[c];
        const double pn = sqrt(sm[5]);
        const double H = wl2 ? sqrt(sm[4]) : (has_l1 ? sm[4] : 0.0) + (has_l2 ? pn : 0.0);
        const double val = sm[2] - 0.5 * sm[3] - tt * H - (pb.level_set ? 0.5 : 0.0);
        S.phi[c] = val; S.hp[c] = H; S.pn[c] = pn;
        if (!distance) {
          S.state[c] = COL_DONE;
        } else {
          if (S.s[c] == 0.0 && val <= 0.0) {  // psi(y, 0) = L_k(y) <= 0: y lies in ellipsoid k
            S.flags[c] |= FLAG_INSIDE; S.state[c] = COL_DONE;
          } else if (!(pn > 0.0)) {
            S.state[c] = COL_DONE;
          } else {
            const double ds = val / pn;  // s_{l+1} = s_l - psi / (d psi / ds), d psi/ds = -|grad psi|
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
              // a new solve: its own iteration budget and stall watch (a capped solve still
              // gives a usable psi and gradient, so Newton goes on and the result is flagged)
              if (pb.iter_total) atomicAdd(pb.iter_total, (unsigned long long)S.iters[c]);
              S.prev[c] = 1e300; S.best[c] = 1e300; S.stall[c] = 0; S.iters[c] = 0;
              S.flags[c] &= ~FLAG_SOLVE_CAP;
              S.state[c] = COL_ACTIVE;
            }
          }
        }
      }
    }
    __syncthreads();
    if (wl2) {  // the multipliers of the next pass's prox
      if (tid < PT) {
        const int st = S.state[tid];
        const bool go = st == COL_ACTIVE || (MODE == 0 && st == COL_WAITING);
        wsel[tid] = go ? ((MODE >= 1 && S.phase[tid] == PH_DELTA) ? 2 : 1) : 0;
      }
      __syncthreads();
      wl2_solve(kWl2PlainNewton, term_pass, upd_pass);
    }
    if (tid == 0) {
      int nact = 0, nwait = 0;
      for (int c = 0; c < PT; ++c) {
        nact += S.state[c] == COL_ACTIVE;
        nwait += S.state[c] == COL_WAITING;
      }
      if (MODE >= 1) {
        const int kn = k_it + 1;
        if ((nact > 0 && kn - S.ctl[CTL_LAST_ANCHOR] >= anchor_every) || (nwait > 0 && nact == 0) ||
            (anchor_wait > 0 && nwait >= anchor_wait))
          S.ctl[CTL_ANCHOR] = 1;
      }
    }
    __syncthreads();
    ++k_it;
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
// Launch shapes picked by the project's autotuner (autotune.py: every launchable shape timed on a
// synthetic union-of-level-sets workload per mode and padded size), {mode, largest n_pad, pt, occ, nw}.
struct TunedShape { int mode, npad_max, pt, occ, nw; };
static const TunedShape kTuned[] = {
#include "tune_table.inc"
};

// the largest dynamic LDS of the FP32 right-hand sides before the contraction is split in two
constexpr size_t kSplitLds = 136 * 1024;

static DenseVariant shape_of(int mode, int n_pad) {
  // HOPF_DENSE_VARIANT=pt:occ:nw forces a shape (the autotuner's sweeps), else the tuned table,
  // else the rules below
  if (const char* v = getenv("HOPF_DENSE_VARIANT")) {
    DenseVariant f{0, 0, 0, 1};
    if (sscanf(v, "%d:%d:%d", &f.pt, &f.occ, &f.nw) == 3 && f.pt > 0) return f;
  }
  for (const TunedShape& t : kTuned)
    if (t.mode == mode && n_pad <= t.npad_max) return DenseVariant{t.pt, t.occ, t.nw, 1};
  // refined mode up to n_pad = 1024: two 32-column workgroups of 4 waves per CU; FP32 modes
  // (plain and refined) by size
  if (mode == 1) {
    if (n_pad > 1024) return DenseVariant{32, 1, 4, 1};
    return DenseVariant{32, 2, 4, 1};
  }
  if (n_pad <= 512) return DenseVariant{64, 1, 4, 1};
  if (n_pad <= 1024) return DenseVariant{32, 1, 4, 1};
  return DenseVariant{16, 1, 4, 1};
}

DenseVariant dense_variant(int mode, int n_pad) {
  DenseVariant v = shape_of(mode, n_pad);
  v.ks = (mode == 2 && (size_t)v.pt * (n_pad + 4) * 4 > kSplitLds) ? 2 : 1;
  return v;
}

size_t dense_lds_bytes(int mode, int n_pad) {
  const DenseVariant v = dense_variant(mode, n_pad);
  const int pt = v.pt;
  // refined: the BF16 (FP32) right-hand sides, or a block of the anchor right-hand sides' slices
  if (mode == 1)
    return std::max((size_t)pt * (n_pad + 8) * 2, (size_t)kSlices * pt * (anchor_kbq(n_pad) + 16));
  if (mode == 2)
    return std::max((size_t)pt * (n_pad / v.ks + 4) * 4, (size_t)kSlices * pt * (anchor_kbq(n_pad) + 16));
  return (size_t)pt * (n_pad + 4) * 4;
}

__global__ void reset_call_kernel(int* counter, double* bestv, int32_t* bestk, int64_t npts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *counter = 0;
  if (i < npts) { bestv[i] = __builtin_inf(); bestk[i] = -1; }
}

hipError_t launch_reset(int* counter, double* bestv, int32_t* bestk, int64_t npts, hipStream_t stream) {
  const int64_t m = npts > 0 ? npts : 1;
  hipLaunchKernelGGL(reset_call_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, stream, counter, bestv,
                     bestk, npts);
  return hipGetLastError();
}

template <int MODE, int CT, int RG, int OCC, int NW, int KS = 1, bool WL = false>
static hipError_t launch_t(const DenseProb* d_probs, const DenseChunk* d_chunks, int nchunks, int* counter,
                           float* ws, double* ws64, int64_t ws_per_wg, int64_t ws64_per_wg, int grid, size_t lds,
                           int distance, int anchor_every, int anchor_wait, int det, hipStream_t stream) {
  auto kern = dense_kernel<MODE, CT, RG, OCC, NW, KS, WL>;
  static size_t attr_bytes[64] = {};  // dynamic LDS allowed so far, per device
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  if (lds > attr_bytes[dev]) {
    e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) {  // more LDS than a workgroup may have: report it without leaving it pending
      (void)hipGetLastError();
      return e;
    }
    attr_bytes[dev] = lds;
  }
  hipLaunchKernelGGL(kern, dim3(grid), dim3(NW * 64), lds, stream, d_probs, d_chunks, nchunks, counter, ws, ws64,
                     ws_per_wg, ws64_per_wg, distance, anchor_every, anchor_wait, det);
  return hipGetLastError();
}

template <bool WL>
static hipError_t launch_shape(int mode, DenseVariant var, const DenseProb* d_probs, const DenseChunk* d_chunks,
                               int nchunks, int* counter, float* ws, double* ws64, int64_t ws_per_wg,
                               int64_t ws64_per_wg, int grid, size_t lds, int distance, int anchor_every,
                               int anchor_wait, int det, hipStream_t stream) {
  const int ct = var.pt / 16, occ = var.occ, nw = var.nw;
#define HOPF_LAUNCH(M, C, R, O, W, K)                                                                            \
  return launch_t<M, C, R, O, W, K, WL>(d_probs, d_chunks, nchunks, counter, ws, ws64, ws_per_wg, ws64_per_wg, \
                                        grid, lds, distance, anchor_every, anchor_wait, det, stream)
  if (mode == 2 && var.ks == 2) {  // the split contraction
    if (ct == 4) HOPF_LAUNCH(2, 4, 4, 1, 4, 2);
    if (ct == 2) HOPF_LAUNCH(2, 2, 4, 1, 4, 2);
    return hipErrorInvalidValue;
  }
  if (var.ks != 1) return hipErrorInvalidValue;
  if (mode == 1) {
    if (nw == 8 && ct == 4) HOPF_LAUNCH(1, 4, 2, 1, 8, 1);
    if (occ == 2 && ct == 2) HOPF_LAUNCH(1, 2, 2, 2, 4, 1);
    if (occ == 1 && ct == 4) HOPF_LAUNCH(1, 4, 4, 1, 4, 1);
    if (occ == 1 && ct == 2) HOPF_LAUNCH(1, 2, 4, 1, 4, 1);
  } else if (mode == 2) {
    if (ct == 4) HOPF_LAUNCH(2, 4, 4, 1, 4, 1);
    if (ct == 2) HOPF_LAUNCH(2, 2, 4, 1, 4, 1);
    if (ct == 1) HOPF_LAUNCH(2, 1, 4, 1, 4, 1);
  } else {
    if (ct == 4) HOPF_LAUNCH(0, 4, 4, 1, 4, 1);
    if (ct == 2) HOPF_LAUNCH(0, 2, 4, 1, 4, 1);
    if (ct == 1) HOPF_LAUNCH(0, 1, 4, 1, 4, 1);
  }
#undef HOPF_LAUNCH
  return hipErrorInvalidValue;
}

hipError_t launch_dense(int mode, DenseVariant var, const DenseProb* d_probs, const DenseChunk* d_chunks,
                        int nchunks, int* counter, float* ws, double* ws64, int64_t ws_per_wg, int64_t ws64_per_wg,
                        int grid, size_t lds, int distance, int anchor_every, int anchor_wait, int det,
                        hipStream_t stream) {
  // sqrt(<p, D p>) problems run in instances with their multiplier phase, the others without it
  if (var.wl && !distance)
    return launch_shape<true>(mode, var, d_probs, d_chunks, nchunks, counter, ws, ws64, ws_per_wg, ws64_per_wg, grid,
                              lds, distance, anchor_every, anchor_wait, det, stream);
  return launch_shape<false>(mode, var, d_probs, d_chunks, nchunks, counter, ws, ws64, ws_per_wg, ws64_per_wg, grid,
                             lds, distance, anchor_every, anchor_wait, det, stream);
}

}  // namespace hopf
