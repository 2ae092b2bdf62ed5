// Small dense problems (n_pad <= 64), FP32 products: one wave per tile of 16 CT columns, with
// the whole iteration in registers and no workgroup barrier.
//
// Same method and arithmetic as the FP32 mode of the tile solver in dense.hip (split Bregman,
// eqs. (3.4a)-(3.4c), in Douglas-Rachford form on z = v + b; see that file).  What differs is
// where things live.  With n_pad = 16 RTM rows (RTM <= 4) a lane holds, for each of its CT
// columns 16 ct + l%16 (ct < CT), the rows 16 rt + 4 (l/16) + q (q = 0..3) of every row tile
// rt: the MFMA output layout.  The B operand of the 16x16x4 FP32 product for k-step kt (k = 16 kt + 4 (l/16)
// + q) is then exactly the lane's own right-hand side of row tile kt, and the A operand
// (M[16 rt + l%16][16 kt + 4 (l/16) + q]) is held for the whole problem in RTM x RTM registers
// of four floats (M is stored in that fragment order).  The product v = M r, the prox, the step
// norms (two lane shuffles per column) and the stopping decisions never leave the wave.
//
// Columns are (point, copy) pairs; a wave takes chunks of whole points from the launch's queue,
// so the copies of a point are settled by one wave, in column order.
#include <cstdint>
#include <type_traits>

#include "common.hpp"
#include "dense.hpp"
#include "dense_shared.hpp"

#ifndef SMALL_CT
#define SMALL_CT 1   // column tiles per wave
#define SMALL_OCC 2  // workgroups per CU
#endif

namespace hopf {

namespace {

// Sum over the four lanes of a column (l, l ^ 16, l ^ 32, l ^ 48), in FP64.
__device__ __forceinline__ double col_sum(float f) {
  double v = (double)f;
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

// The same in FP32 (the step norms, which only decide when to stop); the four lanes add in the
// same pairs and agree bit for bit.
__device__ __forceinline__ float col_sumf(float v) {
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

// clamp(z, lo, hi) for lo <= hi, one instruction
__device__ __forceinline__ float med3f(float z, float lo, float hi) { return __builtin_amdgcn_fmed3f(z, lo, hi); }

// prox of theta sqrt(<., D .>) at coordinate z with s = theta^2 w (see the pass below); the first
// pass of a solve has d = z
__device__ __forceinline__ float wl2_prox(float z, float s, float mu, bool first, bool inside) {
  return first ? z : ((inside || !(s > 0.f)) ? 0.f : mu * z * __builtin_amdgcn_rcpf(s + mu));
}
constexpr int kWl2Newton = 40;           // cap on the multiplier's Newton steps per pass
constexpr float kWl2Rel = 2.5e-7f;       // a step below this fraction of mu ends them

}  // namespace

// RTM row tiles (n_pad <= 16 RTM), CT column tiles per wave, OCC workgroups per CU.
template <int RTM, int CT, int OCC>
__global__ void __launch_bounds__(kBlock, OCC)
dense_small_kernel(const DenseProb* __restrict__ probs, const DenseChunk* __restrict__ chunks, int nchunks,
                   int* __restrict__ chunk_counter) {
  const int l = threadIdx.x & 63;
  const int lr = l & 15, lg = l >> 4;
  // wave-uniform values go through readfirstlane so that the queue state, the problem's scalars
  // and every branch on them live in scalar registers
  auto uni = [](int v) { return __builtin_amdgcn_readfirstlane(v); };

  // queue position of this wave
  int prob = -1, nextcol = 0, cend = 0, pending = -1, nomore = 0;
  {
    int c0 = 0;
    if (l == 0) c0 = atomicAdd(chunk_counter, 1);
    c0 = uni(__shfl(c0, 0));
    if (c0 >= nchunks) return;
    prob = uni(chunks[c0].prob); nextcol = uni(chunks[c0].col0); cend = nextcol + uni(chunks[c0].ncols);
  }

  // per-problem registers; rows and columns beyond n_pad (n_pad < 16 RTM) are zero in M, w and x',
  // so their coordinates stay zero and the products need no bounds
  DenseProb pb = probs[prob];
  f32x4 Mf[RTM][RTM];
  f32x4 wv[RTM];
  auto load_problem = [&]() {
    pb = probs[prob];
    const int nks = uni(pb.n_pad) >> 4;
#pragma unroll
    for (int rt = 0; rt < RTM; ++rt) {
      const int rtc = rt < nks ? rt : 0;
#pragma unroll
      for (int kt = 0; kt < RTM; ++kt) {
        const int ktc = kt < nks ? kt : 0;
        Mf[rt][kt] = (rt < nks && kt < nks) ? *gp((const f32x4*)pb.Mf + ((size_t)rtc * nks + ktc) * 64 + l)
                                            : f32x4{0.f, 0.f, 0.f, 0.f};
      }
      wv[rt] = rt < nks ? *gp((const f32x4*)(pb.wf + 16 * rtc + 4 * lg)) : f32x4{0.f, 0.f, 0.f, 0.f};
    }
  };
  load_problem();

  // per-column registers (column 16 ct + lr; replicated in the four lanes of the column)
  f32x4 z[RTM][CT], xp[RTM][CT];
  int st[CT], flags[CT], iters[CT], stall[CT], jj[CT], kk[CT];
  float thr[CT], gam[CT];  // t / lambda, the shrink2 factor
  float prev[CT], bst[CT];
  double phi[CT], hp[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    st[ct] = COL_EMPTY; flags[ct] = 0; iters[ct] = 0; stall[ct] = 0; jj[ct] = 0; kk[ct] = 0;
    thr[ct] = 0.f; gam[ct] = 1.f;
    prev[ct] = 3e38f; bst[ct] = 3e38f; phi[ct] = 0.0; hp[ct] = 0.0;
#pragma unroll
    for (int rt = 0; rt < RTM; ++rt) { z[rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f}; xp[rt][ct] = z[rt][ct]; }
  }

  while (true) {
    const int n = uni(pb.n), n_pad = uni(pb.n_pad), K = uni(pb.K), hkind = uni(pb.hkind);
    const int nrt = n_pad >> 4;
    const float flam = (float)pb.lambda;
    const bool has_l1 = hk_has_l1(hkind), has_l2 = hk_has_l2(hkind);

    // ============================================================ settle finished columns
    // Lanes 0..15 stand for the 16 columns of each tile in the ballots below (lane lr of row
    // group 0).  With one copy per point the finished columns write their results in parallel;
    // with several copies they are settled one at a time in column order (the per-point best is
    // read, compared and written back).
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const bool fin = st[ct] == COL_DONE || st[ct] == COL_INVALID;
      uint64_t fmask = __ballot(fin && lg == 0) & 0xffffull;
      if (!fmask) continue;
      if (K == 1) {
        if (fin) {  // the column's four lanes: its p rows; row group 0 also the scalars
          const int j = jj[ct];
          const bool bad = st[ct] == COL_INVALID;
          HOPF_GLOBAL float* g = gp(pb.grad + (size_t)j * n);
#pragma unroll
          for (int rt = 0; rt < RTM; ++rt) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int row = 16 * rt + 4 * lg + q;
              if (rt < nrt && row < n) g[row] = bad ? __builtin_nanf("") : z[rt][ct][q];
            }
          }
          if (lg == 0) {
            pb.phi[j] = bad ? __builtin_nanf("") : (float)phi[ct];
            pb.dphidt[j] = bad ? __builtin_nanf("") : (float)(-hp[ct]);
            if (pb.iters) pb.iters[j] = bad ? -1 : ((flags[ct] & FLAG_CAPPED) ? -2 : iters[ct]);
            if (pb.kstar) pb.kstar[j] = bad ? -1 : 0;
          }
          st[ct] = COL_EMPTY;
        }
        continue;
      }
      while (fmask) {  // in column order
        const int c0 = __builtin_ctzll(fmask);
        fmask &= fmask - 1;
        const int s = uni(__shfl(st[ct], c0));
        // the column's scalars, broadcast by every lane (no lane may be inactive in a shuffle)
        const int j = __shfl(jj[ct], c0), k = __shfl(kk[ct], c0);
        const double key = __shfl(phi[ct], c0), hpk = __shfl(hp[ct], c0);
        const int fl = __shfl(flags[ct], c0), itk = __shfl(iters[ct], c0);
        int better = 0;
        if (l == 0) {
          if (s == COL_INVALID) {
            better = 2;
            pb.bestk[j] = -2;
            pb.phi[j] = __builtin_nanf(""); pb.dphidt[j] = __builtin_nanf("");
            if (pb.iters) pb.iters[j] = -1;
            if (pb.kstar) pb.kstar[j] = -1;
          } else {
            const int bk = pb.bestk[j];
            const double bv = pb.bestv[j];
            better = (bk < 0 || key < bv || (key == bv && k < bk)) ? 1 : 0;
            if (better) {
              pb.bestv[j] = key; pb.bestk[j] = k;
              pb.phi[j] = (float)key;
              pb.dphidt[j] = (float)(-hpk);
              if (pb.iters) pb.iters[j] = (fl & FLAG_CAPPED) ? -2 : itk;
              if (pb.kstar) pb.kstar[j] = k;
            }
          }
        }
        better = uni(__shfl(better, 0));
        if (better && lr == c0) {  // the column's four lanes write p (kept in z) or NaN
          HOPF_GLOBAL float* g = gp(pb.grad + (size_t)j * n);
#pragma unroll
          for (int rt = 0; rt < RTM; ++rt) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int row = 16 * rt + 4 * lg + q;
              if (rt < nrt && row < n) g[row] = better == 2 ? __builtin_nanf("") : z[rt][ct][q];
            }
          }
        }
        if (lr == c0) st[ct] = COL_EMPTY;
      }
    }

    // ============================================================ refill empty columns
    // The queue positions are handed out in column order by a scalar loop; then every refilled
    // column loads its point at once (one memory latency per refill, whatever the count).
    int live = 0;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      uint64_t emask = __ballot(st[ct] == COL_EMPTY && lg == 0) & 0xffffull;
      if (emask != 0xffffull) live = 1;
      int mycol = -1;
      while (emask) {
        const int c0 = __builtin_ctzll(emask);
        emask &= emask - 1;
        while (nextcol >= cend && pending < 0 && !nomore) {
          int nc = 0;
          if (l == 0) nc = atomicAdd(chunk_counter, 1);
          nc = uni(__shfl(nc, 0));
          if (nc >= nchunks) { nomore = 1; break; }
          if (uni(chunks[nc].prob) == prob) { nextcol = uni(chunks[nc].col0); cend = nextcol + uni(chunks[nc].ncols); }
          else pending = nc;
        }
        if (nextcol >= cend) break;  // nothing more for this problem
        if (lr == c0) mycol = nextcol;
        ++nextcol;
        live = 1;
      }
      if (mycol >= 0) {  // the column's four lanes take the new (point, copy)
        const int j = mycol / K, k = mycol % K;
        jj[ct] = j; kk[ct] = k;
        const float tv = pb.t[j];
        const bool tok = tv > 0.f && isfinite(tv);
        thr[ct] = (float)((double)tv / pb.lambda);
        gam[ct] = 1.f; iters[ct] = 0; stall[ct] = 0; flags[ct] = FLAG_FIRST;
        prev[ct] = 3e38f; bst[ct] = 3e38f; phi[ct] = 0.0; hp[ct] = 0.0;
        const HOPF_GLOBAL float* xj = gp(pb.x + (size_t)j * n);
        const HOPF_GLOBAL double* cen = pb.centres ? gp(pb.centres + (size_t)k * n_pad) : nullptr;
        bool nf = false;
#pragma unroll
        for (int rt = 0; rt < RTM; ++rt) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int row = 16 * rt + 4 * lg + q;
            float v = 0.f;
            if (rt < nrt && row < n) {
              const float xv = xj[row];
              if (!isfinite(xv)) nf = true;
              v = (float)((double)xv - (cen ? cen[row] : 0.0));
            }
            xp[rt][ct][q] = v;
            z[rt][ct][q] = v;
          }
        }
        st[ct] = tok ? COL_ACTIVE : COL_INVALID;
        if (nf) st[ct] = COL_INVALID;  // combined over the column's lanes below
      }
    }
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {  // a non-finite coordinate in any lane of a column invalidates it
      int inv = st[ct] == COL_INVALID ? 1 : 0;
      inv |= __shfl_xor(inv, 16);
      inv |= __shfl_xor(inv, 32);
      if (inv && st[ct] == COL_ACTIVE) st[ct] = COL_INVALID;
    }
    if (!live) {
      if (pending >= 0) {  // drained: switch to the pending problem
        prob = uni(chunks[pending].prob); nextcol = uni(chunks[pending].col0);
        cend = nextcol + uni(chunks[pending].ncols);
        pending = -1;
        load_problem();
        continue;
      }
      break;
    }
    // only invalid columns left: settle them before iterating
    {
      int any_on = 0, any_inv = 0;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        any_on |= (st[ct] == COL_ACTIVE || st[ct] == COL_WAITING || st[ct] == COL_PHI) ? 1 : 0;
        any_inv |= st[ct] == COL_INVALID ? 1 : 0;
      }
      if (!__any(any_on)) {
        if (__any(any_inv)) continue;
      }
    }
    int phi_lane = 0;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      if (st[ct] == COL_WAITING) st[ct] = COL_PHI;  // converged: this pass evaluates the value
      phi_lane |= st[ct] == COL_PHI ? 1 : 0;
    }
    const bool any_phi = __any(phi_lane);

    // one pass of every column: the Hamiltonian's kind fixed at compile time, so that the pass is
    // straight-line code the scheduler can interleave (products of one row tile with the update
    // of the previous one)
    auto pass = [&](auto kindtag) {
      // KIND 0: weighted l1 (shrink1 only); 1: l2 or l2 + weighted l1 (shrink2 factor);
      // 2: sqrt(<p, D p>) (projection onto the Wulff ellipsoid)
      constexpr int KIND = decltype(kindtag)::value;
      constexpr bool HL2 = KIND == 1, WL2 = KIND == 2;
      // ---------------------------------------------------------- right-hand sides
      // d = prox of the current z (eq. (3.4b)); the first pass of a solve has d = z, which is the
      // same formula with threshold 0 and factor 1.  u = z - d is the C operand of the products,
      // so that they return the next z = z - d + M r directly (eq. (3.4a) in Douglas-Rachford
      // form); r = x' + lambda (2 d - z).  Columns that are not iterating compute garbage that is
      // never read (the product keeps columns apart).
      float thd[CT], gd[CT];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const bool first = flags[ct] & FLAG_FIRST;
        thd[ct] = (first || !has_l1) ? 0.f : thr[ct];
        gd[ct] = (first || !HL2) ? 1.f : gam[ct];
      }
      // sqrt(<p, D p>): prox_{theta H}(z) = z - pi(z), pi the projection onto the ellipsoid
      // sum y_i^2 / s_i <= 1 with s_i = theta^2 w_i (section 4.3, eq. (prox-projection)):
      // 0 for z inside, else d_i = mu z_i / (s_i + mu) with mu > 0 solving
      // phi(mu) = sum s_i z_i^2 / (s_i + mu)^2 = 1.  Newton runs on 1 / sqrt(phi) - 1 (concave and
      // increasing in mu, so from mu = 0 the steps increase monotonically to the root, exactly in
      // one step when all s_i are equal); every column of the wave iterates until its step is at
      // FP32 rounding level.
      float mu[CT], th2[CT];
      bool dz0[CT];  // d = 0 (z inside the ellipsoid)
      if (WL2) {
        bool go[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          const bool first = flags[ct] & FLAG_FIRST;
          const bool on = st[ct] == COL_ACTIVE || st[ct] == COL_PHI;
          th2[ct] = thr[ct] * thr[ct];
          float qa = 0.f;
#pragma unroll
          for (int rt = 0; rt < RTM; ++rt)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const float zz = z[rt][ct][q], sv = th2[ct] * wv[rt][q];
              qa += sv > 0.f ? zz * zz * __builtin_amdgcn_rcpf(sv) : 0.f;
            }
          const float qs = col_sumf(qa);
          dz0[ct] = !first && !(qs > 1.f);
          go[ct] = on && !first && !dz0[ct];
          mu[ct] = 0.f;
        }
        for (int it = 0; it < kWl2Newton; ++it) {
          int any = 0;
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            float pa = 0.f, pb3 = 0.f;
#pragma unroll
            for (int rt = 0; rt < RTM; ++rt)
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                // sv = 0 on padding rows: they contribute nothing (and rcp(0) must not reach a sum)
                const float zz = z[rt][ct][q], sv = th2[ct] * wv[rt][q];
                const float inv = sv > 0.f ? __builtin_amdgcn_rcpf(sv + mu[ct]) : 0.f;
                const float e = sv * zz * zz * inv * inv;
                pa += e;
                pb3 += e * inv;
              }
            const float ph = col_sumf(pa), ps = col_sumf(pb3);
            const float step = ph * (__builtin_sqrtf(ph) - 1.f) / ps;
            go[ct] = go[ct] && step > kWl2Rel * mu[ct];
            if (go[ct]) mu[ct] += step;
            any |= go[ct] ? 1 : 0;
          }
          if (!__any(any)) break;
        }
      }
      f32x4 r[RTM][CT], u[RTM][CT];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
#pragma unroll
        for (int rt = 0; rt < RTM; ++rt) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float zz = z[rt][ct][q];
            float d;
            if (WL2) {
              d = wl2_prox(zz, th2[ct] * wv[rt][q], mu[ct], flags[ct] & FLAG_FIRST, dz0[ct]);
            } else {
              const float th = theta_f(thd[ct], wv[rt][q]);
              d = (HL2 ? gd[ct] : 1.f) * (zz - med3f(zz, -th, th));
            }
            u[rt][ct][q] = zz - d;
            r[rt][ct][q] = xp[rt][ct][q] + flam * (2.f * d - zz);
          }
        }
      }
      if (any_phi) {  // the value pass needs the plain product M r
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int rt = 0; rt < RTM; ++rt)
#pragma unroll
            for (int q = 0; q < 4; ++q) u[rt][ct][q] = st[ct] == COL_PHI ? 0.f : u[rt][ct][q];
      }

      // ---------------------------------------------------------- products, then the step sums
      // (u becomes z - d + M r, or M r in a value pass)
#pragma unroll
      for (int rt = 0; rt < RTM; ++rt)
#pragma unroll
        for (int kt = 0; kt < RTM; ++kt)
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
              u[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(Mf[rt][kt][q], r[kt][ct][q], u[rt][ct], 0, 0, 0);

      float s0[CT], s1[CT];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const bool act = st[ct] == COL_ACTIVE;
        float a0 = 0.f, a1 = 0.f;
        const float thn = has_l1 ? thr[ct] : 0.f;
#pragma unroll
        for (int rt = 0; rt < RTM; ++rt) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float zn = u[rt][ct][q];
            const float step = zn - z[rt][ct][q];
            a0 += step * step;
            if (HL2) {  // |shrink1(z)|, for the shrink2 factor of the next pass
              const float th = theta_f(thn, wv[rt][q]);
              const float sn = zn - med3f(zn, -th, th);
              a1 += sn * sn;
            }
            z[rt][ct][q] = act ? zn : z[rt][ct][q];
          }
        }
        s0[ct] = col_sumf(a0);
        s1[ct] = HL2 ? col_sumf(a1) : 0.f;
      }

      // ---------------------------------------------------------- per-column update
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        if (st[ct] != COL_ACTIVE) continue;
        const double sm0 = (double)s0[ct];
        iters[ct] += 1;
        float g = 1.f;
        if (HL2) {
          const double nz = sqrt(fmax((double)s1[ct], 0.0));
          g = nz > 0.0 ? (float)(fmax(nz - (double)thr[ct], 0.0) / nz) : 0.f;
        }
        gam[ct] = g;
        flags[ct] &= ~FLAG_FIRST;
        // (|dz_k| + |dz_{k-1}|)^2 <= tol
        const double pv = (double)prev[ct];
        prev[ct] = (float)sm0;
        const bool conv = sm0 + pv + 2.0 * sqrt(sm0 * pv) <= pb.tol;
        bool stalled = false;
        if (sm0 < (double)bst[ct]) { bst[ct] = (float)sm0; stall[ct] = 0; }
        else stalled = ++stall[ct] >= kStallIters;
        const bool capped = iters[ct] >= pb.max_iter || stalled;
        if (conv) st[ct] = COL_WAITING;
        else if (capped) { st[ct] = COL_WAITING; flags[ct] |= FLAG_SOLVE_CAP | FLAG_CAPPED; }
      }

      // ---------------------------------------------------------- value pass (eq. (3.5))
      if (any_phi) {
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          const bool isphi = st[ct] == COL_PHI;
          float v2 = 0.f, v3 = 0.f, v4 = 0.f, v5 = 0.f;
#pragma unroll
          for (int rt = 0; rt < RTM; ++rt) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int row = 16 * rt + 4 * lg + q;
              const float zz = z[rt][ct][q];
              float d;
              if (WL2) {
                d = wl2_prox(zz, th2[ct] * wv[rt][q], mu[ct], flags[ct] & FLAG_FIRST, dz0[ct]);
              } else {
                const float th = theta_f(thd[ct], wv[rt][q]);
                d = (HL2 ? gd[ct] : 1.f) * (zz - med3f(zz, -th, th));
              }
              if (row >= n) d = 0.f;
              const float vv = u[rt][ct][q];
              const float rr = xp[rt][ct][q] + flam * (2.f * d - zz);
              v2 += xp[rt][ct][q] * d;
              v3 += (2.f * d - vv) * (rr - flam * vv);
              v4 += WL2 ? wv[rt][q] * d * d : wv[rt][q] * fabsf(d);
              v5 += d * d;
              z[rt][ct][q] = isphi ? d : zz;  // p replaces z
            }
          }
          const double sm2 = col_sum(v2), sm3 = col_sum(v3), sm4 = col_sum(v4), sm5 = col_sum(v5);
          if (isphi) {
            const double pn = sqrt(sm5);
            const double H = WL2 ? sqrt(sm4) : (has_l1 ? sm4 : 0.0) + (HL2 ? pn : 0.0);
            const double tv = (double)pb.t[jj[ct]];
            phi[ct] = sm2 - 0.5 * sm3 - tv * H - (pb.level_set ? 0.5 : 0.0);
            hp[ct] = H;
            st[ct] = COL_DONE;
          }
        }
      }
    };
    if (hkind == HK_WL2) pass(std::integral_constant<int, 2>{});
    else if (has_l2) pass(std::integral_constant<int, 1>{});
    else pass(std::integral_constant<int, 0>{});
  }
}

bool dense_small_fits(int mode, int n_pad, int distance) { return mode == 0 && !distance && n_pad <= 64; }

int dense_small_cols() { return 16 * SMALL_CT; }
int dense_small_occupancy() { return SMALL_OCC; }

hipError_t launch_dense_small(int n_pad, const DenseProb* d_probs, const DenseChunk* d_chunks, int nchunks,
                              int* counter, int grid, hipStream_t stream) {
  if (n_pad <= 32)
    hipLaunchKernelGGL((dense_small_kernel<2, SMALL_CT, SMALL_OCC>), dim3(grid), dim3(kBlock), 0, stream, d_probs,
                       d_chunks, nchunks, counter);
  else if (n_pad <= 64)
    hipLaunchKernelGGL((dense_small_kernel<4, SMALL_CT, SMALL_OCC>), dim3(grid), dim3(kBlock), 0, stream, d_probs,
                       d_chunks, nchunks, counter);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace hopf
