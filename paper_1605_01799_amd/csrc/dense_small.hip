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
//
// Refined FP32 (REF): plain FP32 products of the whole right-hand side stall at the FP32
// rounding floor of the fixed point (about kappa(A) u / (1 - rho)).  With REF the iteration is
// carried, as in the refined tile solver, on an anchor za and an increment dz (z = za + dz):
// every `anchor_every` passes (and when converged columns wait with nothing else iterating) the
// wave re-bases za <- za + dz and takes the anchor product v^a = M r^a of the FP64 right-hand
// side r^a = x' + lambda (2 d^a - za), d^a the prox of za with FP64 thresholds, in FP64 (FP64
// MFMA 16x16x4 on the FP64 copy of M), and keeps ea = v^a - d^a.  Between anchors a pass
// computes only increments in FP32: dd = prox(za + dz) - prox(za) from the anchor's shrink
// decomposition, dr = lambda (2 dd - dz), dv = M dr (FP32 MFMA), and dz <- dz + ea + dv - dd, so
// every rounding is relative to a vanishing increment and the fixed point is that of the exact
// product.  A column that passes the stopping test waits for the next anchor and is accepted only
// if the test still passes on the fresh anchor (its value pass).  For the ellipsoidal norm
// sqrt(<p, D p>) the prox is d = mu z / (s + mu) (section 4.3) with the multiplier mu of the
// projection: the anchor solves for mu^a in FP64, and a pass solves for the increment dmu of the
// multiplier by Newton on the difference phi(mu^a + dmu; za + dz) - phi(mu^a; za), whose terms
// are products of increments (so dmu is resolved relative to the increments), then
// dd = (mu dz (s + mu^a) + za s dmu) / ((s + mu)(s + mu^a)).
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
__device__ __forceinline__ double col_sum(double v) {
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

// RTM row tiles (n_pad <= 16 RTM), CT column tiles per wave, OCC workgroups per CU, REF the
// refined FP32 iteration (above).
// KS: the kinds of H of the launch's problems (0: weighted l1; 1: l2, l2 + weighted l1; 2:
// sqrt(<p, D p>)); only that pass is compiled in, so the simpler kinds keep their registers.
template <int RTM, int CT, int OCC, bool REF, int KS>
__global__ void __launch_bounds__(kBlock, OCC)
dense_small_kernel(const DenseProb* __restrict__ probs, const DenseChunk* __restrict__ chunks, int nchunks,
                   int* __restrict__ chunk_counter, int anchor_every, int anchor_wait, int det) {
  const int l = threadIdx.x & 63;
  const int lr = l & 15, lg = l >> 4;
  // wave-uniform values go through readfirstlane so that the queue state, the problem's scalars
  // and every branch on them live in scalar registers
  auto uni = [](int v) { return __builtin_amdgcn_readfirstlane(v); };

  // queue position of this wave
  int prob = -1, nextcol = 0, cend = 0, pending = -1, nomore = 0;
  // with det the waves take fixed chunks: wave unit of `units` (see next_chunk)
  const int units = (int)gridDim.x * (int)(blockDim.x >> 6);
  const int unit = (int)blockIdx.x * (int)(blockDim.x >> 6) + (int)(threadIdx.x >> 6);
  int taken = 0;  // (lane 0's count is the one used)
  {
    int c0 = 0;
    if (l == 0) c0 = next_chunk(chunk_counter, det, unit, units, taken);
    c0 = uni(__shfl(c0, 0));
    if (c0 >= nchunks) return;
    prob = uni(chunks[c0].prob); nextcol = uni(chunks[c0].col0); cend = nextcol + uni(chunks[c0].ncols);
  }

  // per-problem operands; rows and columns beyond n_pad (n_pad < 16 RTM) are zero in M, w and x',
  // so their coordinates stay zero and the products need no bounds.  M's fragments are held in
  // registers (plain) or, in the refined kernel (whose state takes more registers), in the wave's
  // own LDS region, each lane reading back only what it wrote; during an anchor that region
  // holds the FP64 staging of s^a (the shrink of za) and r^a, [rt * 4 + q][lane] each, and M is
  // reloaded after it.
  DenseProb pb = probs[prob];
  constexpr int RM = REF ? 1 : RTM;
  f32x4 Mf[RM][RM];
  constexpr int kRegion = REF ? (RTM * RTM * 16 > RTM * 4 * 16 ? RTM * RTM * 16 : RTM * 4 * 16) : 16;  // x 64 bytes
  __shared__ __attribute__((aligned(16))) unsigned char lds_small[REF ? 4 : 1][kRegion * 64];
  const int wave = REF ? (int)(threadIdx.x >> 6) : 0;
  f32x4* const Ms = (f32x4*)lds_small[wave];                    // [rt * RTM + kt][64]
  double* const sbuf = (double*)lds_small[wave];                // [rt * 4 + q][64]
  double* const rbuf = (double*)lds_small[wave] + RTM * 4 * 64;  // [rt * 4 + q][64]
  auto mfrag = [&](int rt, int kt) -> f32x4 {
    return REF ? Ms[(rt * RTM + kt) * 64 + l] : Mf[REF ? 0 : rt][REF ? 0 : kt];
  };
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
        const f32x4 m = (rt < nks && kt < nks) ? *gp((const f32x4*)pb.Mf + ((size_t)rtc * nks + ktc) * 64 + l)
                                               : f32x4{0.f, 0.f, 0.f, 0.f};
        if (REF) Ms[(rt * RTM + kt) * 64 + l] = m;
        else Mf[REF ? 0 : rt][REF ? 0 : kt] = m;
      }
      wv[rt] = rt < nks ? *gp((const f32x4*)(pb.wf + 16 * rtc + 4 * lg)) : f32x4{0.f, 0.f, 0.f, 0.f};
    }
  };
  load_problem();

  // per-column registers (column 16 ct + lr; replicated in the four lanes of the column).
  // Plain pass: z the iterate, xp = x' (FP32).  REF: z the anchor za, dz the increment, xp = x'
  // until the column's first pass and ea = v^a - d^a after it.  p replaces z once the value is taken.
  constexpr int RD = REF ? RTM : 1;
  f32x4 z[RTM][CT], xp[RTM][CT], dz[RD][CT];
  int st[CT], flags[CT], iters[CT], stall[CT], jj[CT], kk[CT];
  float thr[CT], gam[CT];  // t / lambda, the shrink2 factor
  float prev[CT], bst[CT];
  double phi[CT], hp[CT];
  double gama[CT], ssa2[CT];  // REF: the anchor's shrink2 factor and |shrink1(za)|^2 (FP64)
  float dgam[CT];             // REF: gam - gama
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    st[ct] = COL_EMPTY; flags[ct] = 0; iters[ct] = 0; stall[ct] = 0; jj[ct] = 0; kk[ct] = 0;
    thr[ct] = 0.f; gam[ct] = 1.f;
    prev[ct] = 3e38f; bst[ct] = 3e38f; phi[ct] = 0.0; hp[ct] = 0.0;
    gama[ct] = 1.0; ssa2[ct] = 0.0; dgam[ct] = 0.f;
#pragma unroll
    for (int rt = 0; rt < RTM; ++rt) { z[rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f}; xp[rt][ct] = z[rt][ct]; }
#pragma unroll
    for (int rt = 0; rt < RD; ++rt) dz[rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  int since = 0;  // REF: passes since the wave's last anchor

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
            if (pb.iter_total) atomicAdd(pb.iter_total, (unsigned long long)iters[ct]);
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
          if (pb.iter_total) atomicAdd(pb.iter_total, (unsigned long long)itk);
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
          if (l == 0) nc = next_chunk(chunk_counter, det, unit, units, taken);
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
        gama[ct] = 1.0; ssa2[ct] = 0.0; dgam[ct] = 0.f;
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
          if (REF) dz[rt < RD ? rt : 0][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
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
        since = 0;
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
    const bool refined = REF;
    int phi_lane = 0;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      if (!refined && st[ct] == COL_WAITING) st[ct] = COL_PHI;  // converged: this pass evaluates the value
      phi_lane |= st[ct] == COL_PHI ? 1 : 0;
    }
    const bool any_phi = !refined && __any(phi_lane);

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
        for (int kt = 0; kt < RTM; ++kt) {
          const f32x4 a = mfrag(rt, kt);
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
              u[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q], r[kt][ct][q], u[rt][ct], 0, 0, 0);
        }

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
    // ============================================================ refined pass (REF; l1 / l2 kinds)
    // Every column runs in increment form: za (z), dz, ea (xp).  A fresh column's first pass takes
    // its FP32 start: za = x', d^a = prox(za), r^a = x' + lambda (2 d^a - za) as the B operand and
    // -d^a as the C operand, so the product returns ea = M r^a - d^a (an FP32 estimate, replaced at
    // the column's first exact anchor), which is also its first increment.  Only columns anchored
    // exactly (FLAG_EXACT) may stop.
    // For the ellipsoidal norm (KIND 2) a column's gama holds the anchor's multiplier mu^a (FP64),
    // dgam the current increment dmu, ssa2 the anchor's residual phi(mu^a; za) - 1, and
    // FLAG_INSIDE (no distances here) that za lies inside the Wulff ellipsoid (d^a = 0).
    auto pass_ref = [&](auto kindtag) {
      constexpr int KIND = decltype(kindtag)::value;
      constexpr bool HL2 = KIND == 1, WL = KIND == 2;
      const double lam = pb.lambda;
      // row tile rt of a register array in a rolled loop (selects: the arrays stay in registers);
      // the rare blocks below (anchor, value terms) run one row tile at a time this way, so that
      // they add few live registers to the iteration's
      auto get4 = [&](const f32x4 (&a)[RTM][CT], int rt, int ct) -> f32x4 {
        f32x4 v = a[0][ct];
#pragma unroll
        for (int i = 1; i < RTM; ++i) v = rt == i ? a[i][ct] : v;
        return v;
      };
      auto set4 = [&](f32x4 (&a)[RTM][CT], int rt, int ct, f32x4 v) {
#pragma unroll
        for (int i = 0; i < RTM; ++i) a[i][ct] = rt == i ? v : a[i][ct];
      };
      auto getw = [&](int rt) -> f32x4 {
        f32x4 v = wv[0];
#pragma unroll
        for (int i = 1; i < RTM; ++i) v = rt == i ? wv[i] : v;
        return v;
      };

      // ---------------------------------------------------------- anchor
      {
        int nact = 0, nwait = 0;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          nact += __popcll(__ballot(st[ct] == COL_ACTIVE && lg == 0));
          nwait += __popcll(__ballot(st[ct] == COL_WAITING && lg == 0));
        }
        const bool take = (nact > 0 && since >= anchor_every) || (nwait > 0 && nact == 0) ||
                          (anchor_wait > 0 && nwait >= anchor_wait);
        if (take) {
          since = 0;
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            const bool on = (st[ct] == COL_ACTIVE && !(flags[ct] & FLAG_FIRST)) || st[ct] == COL_WAITING;
            const int j = jj[ct], k = kk[ct];
            const double tv = on ? (double)pb.t[j] : 0.0;
            const double th1 = has_l1 ? tv / lam : 0.0, th2 = HL2 ? tv / lam : 0.0;
            const double thw = tv / lam;  // WL: s_i = thw^2 w_i
            const float thn = has_l1 ? thr[ct] : 0.f;
            const HOPF_GLOBAL float* xj = gp(pb.x + (size_t)j * n);
            const HOPF_GLOBAL double* cen = pb.centres ? gp(pb.centres + (size_t)k * n_pad) : nullptr;
            // re-base z = za + dz (za the nearest float, dz the remainder); s^a = shrink1(za) with
            // FP64 thresholds, to the staging
            double pss = 0.0, pinc = 0.0;
#pragma unroll 1
            for (int rt = 0; rt < RTM; ++rt) {
              f32x4 zv = get4(z, rt, ct), dv = get4(dz, rt, ct);
              const f32x4 w4 = getw(rt);
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int row = 16 * rt + 4 * lg + q;
                const bool inb = on && rt < nrt && row < n;
                const double zd = (double)zv[q] + (double)dv[q];
                const float zan = (float)zd, dzn = (float)(zd - (double)zan);
                const float th = theta_f(thn, w4[q]);
                const float ca = med3f(zan, -th, th), sav = zan - ca;
                const float ds = dzn - med3f(dzn + sav, -th - ca, th - ca);
                const double sa = inb ? ((has_l1 && !WL) ? anchor_shrink(zan, th1, pb.w, row) : (double)zan) : 0.0;
                pss += sa * sa;
                pinc += inb ? (double)ds * (2.0 * (double)sav + (double)ds) : 0.0;
                if (on) { zv[q] = zan; dv[q] = dzn; }
                sbuf[(rt * 4 + q) * 64 + l] = sa;  // WL: za, replaced by d^a below
              }
              set4(z, rt, ct, zv); set4(dz, rt, ct, dv);
            }
            const double ssa = col_sum(pss), sinc = col_sum(pinc);
            double ga = 1.0, g = 1.0;
            if (HL2) {
              const double na = sqrt(ssa), nz = sqrt(fmax(ssa + sinc, 0.0));
              ga = na > 0.0 ? fmax(na - th2, 0.0) / na : 0.0;
              g = nz > 0.0 ? fmax(nz - th2, 0.0) / nz : 0.0;
            }
            if (WL) {
              // the projection of za onto sum y_i^2 / s_i <= 1 in FP64: inside, or mu^a > 0 solving
              // phi(mu) = sum s_i za_i^2 / (s_i + mu)^2 = 1 by Newton on 1 / sqrt(phi) - 1 from 0
              auto sums = [&](double mu, double* ph, double* ps, double* qi) {
                double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll 1
                for (int rt = 0; rt < nrt; ++rt) {
                  const f32x4 w4 = getw(rt);
                  (void)w4;
#pragma unroll
                  for (int q = 0; q < 4; ++q) {
                    const int row = 16 * rt + 4 * lg + q;
                    if (row >= n) continue;
                    const double zz = sbuf[(rt * 4 + q) * 64 + l];
                    const double sv = thw * thw * *gp(pb.w + row);
                    if (!(sv > 0.0)) continue;
                    const double inv = 1.0 / (sv + mu);
                    const double e = sv * zz * zz * inv * inv;
                    a += e; b += e * inv; c += zz * zz / sv;
                  }
                }
                *ph = col_sum(a); *ps = col_sum(b); *qi = col_sum(c);
              };
              double ph, ps, qi;
              sums(0.0, &ph, &ps, &qi);
              const bool ins = !(qi > 1.0);
              double mu = 0.0;
              if (!ins) {
                for (int it = 0; it < 100; ++it) {
                  const double stp = ph * (sqrt(ph) - 1.0) / ps;
                  if (!(stp > 1e-15 * mu)) break;
                  mu += stp;
                  sums(mu, &ph, &ps, &qi);
                }
              }
              if (on) {
                gama[ct] = mu; dgam[ct] = 0.f; ssa2[ct] = ins ? qi - 1.0 : ph - 1.0;
                flags[ct] = ins ? (flags[ct] | FLAG_INSIDE) : (flags[ct] & ~FLAG_INSIDE);
              }
              // d^a = mu^a za / (s + mu^a), or 0 inside
#pragma unroll 1
              for (int rt = 0; rt < RTM; ++rt) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                  const int row = 16 * rt + 4 * lg + q;
                  const double zz = sbuf[(rt * 4 + q) * 64 + l];
                  const double sv = (rt < nrt && row < n) ? thw * thw * *gp(pb.w + row) : 0.0;
                  sbuf[(rt * 4 + q) * 64 + l] = (ins || !(sv > 0.0)) ? 0.0 : mu * zz / (sv + mu);
                }
              }
              ga = 1.0;
            }
            if (on && !WL) { gama[ct] = ga; ssa2[ct] = ssa; gam[ct] = (float)g; dgam[ct] = (float)(g - ga); }
            // r^a = x' + lambda (2 d^a - za) in FP64 (d^a = ga s^a), the B operand of the FP64 products
#pragma unroll 1
            for (int rt = 0; rt < RTM; ++rt) {
              const f32x4 zv = get4(z, rt, ct);
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int row = 16 * rt + 4 * lg + q;
                const bool inb = on && rt < nrt && row < n;
                const double xpd = inb ? (double)xj[row] - (cen ? cen[row] : 0.0) : 0.0;
                const double sa = sbuf[(rt * 4 + q) * 64 + l];
                rbuf[(rt * 4 + q) * 64 + l] = inb ? xpd + lam * (2.0 * ga * sa - (double)zv[q]) : 0.0;
              }
            }
            // v^a = M r^a by FP64 MFMA 16x16x4.  Its operands are laid out as the FP32 product's (A[i][k]
            // in lane i + 16 k, B[k][j] in lane j + 16 k: B is the lane's own r^a row), but its output
            // row i sits in lane j + 16 (i % 4), register i / 4, where the FP32 product has lane
            // j + 16 (i / 4), register i % 4.  Feeding A's row i from M's row 16 rt + 4 (i % 4) + i / 4
            // puts row 4 (l / 16) + q of the tile into register q of lane l, the state's layout.
            // ea = v^a - d^a
#pragma unroll 1
            for (int rt = 0; rt < nrt; ++rt) {
              f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
              for (int kt = 0; kt < RTM; ++kt) {
                if (kt >= nrt) continue;  // wave-uniform
                const int arow = 16 * rt + 4 * (lr & 3) + (lr >> 2);
                const f64x4 a = *gp((const f64x4*)(pb.Md + (size_t)arow * n_pad + 16 * kt + 4 * lg));
#pragma unroll
                for (int q = 0; q < 4; ++q)
                  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], rbuf[(kt * 4 + q) * 64 + l], acc, 0, 0, 0);
              }
              f32x4 ev = get4(xp, rt, ct);
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int row = 16 * rt + 4 * lg + q;
                const double sa = sbuf[(rt * 4 + q) * 64 + l];
                if (on) ev[q] = row < n ? (float)(acc[q] - ga * sa) : 0.f;
              }
              set4(xp, rt, ct, ev);
            }
            if (on) flags[ct] |= FLAG_EXACT;
            if (st[ct] == COL_WAITING) st[ct] = COL_PHI;  // converged: this pass re-tests and evaluates
          }
          // M's FP32 fragments back into the wave's LDS region (zeros beyond n_pad: the staging
          // overwrote them too)
          const int nks = n_pad >> 4;
#pragma unroll
          for (int rt = 0; rt < RTM; ++rt)
#pragma unroll
            for (int kt = 0; kt < RTM; ++kt)
              Ms[(rt * RTM + kt) * 64 + l] = (rt < nks && kt < nks)
                                                 ? *gp((const f32x4*)pb.Mf + ((size_t)rt * nks + kt) * 64 + l)
                                                 : f32x4{0.f, 0.f, 0.f, 0.f};
        }
      }
      ++since;
      int phi_lane = 0, fresh_lane = 0;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        phi_lane |= st[ct] == COL_PHI ? 1 : 0;
        fresh_lane |= (st[ct] == COL_ACTIVE && (flags[ct] & FLAG_FIRST)) ? 1 : 0;
      }
      const bool any_phi = __any(phi_lane);

      // ---------------------------------------------------------- l2 factor of fresh columns' start
      if (HL2 && __any(fresh_lane)) {
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          const float thn = has_l1 ? thr[ct] : 0.f;
          float a = 0.f;
#pragma unroll
          for (int rt = 0; rt < RTM; ++rt)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const float th = theta_f(thn, wv[rt][q]);
              const float sa = z[rt][ct][q] - med3f(z[rt][ct][q], -th, th);
              a += sa * sa;
            }
          const double s = (double)col_sumf(a);
          if (st[ct] == COL_ACTIVE && (flags[ct] & FLAG_FIRST)) {
            const double na = sqrt(s);
            const double ga = na > 0.0 ? fmax(na - (double)thr[ct], 0.0) / na : 0.0;
            gama[ct] = ga; ssa2[ct] = s; gam[ct] = (float)ga; dgam[ct] = 0.f;
          }
        }
      }

      // ---------------------------------------------------------- ellipsoidal norm: multipliers
      // A fresh column's start: mu of za by FP32 Newton from 0 (its ea is an FP32 estimate anyway).
      // Every other column: whether z = za + dz is inside the Wulff ellipsoid (then d = 0), else the
      // increment dmu by two Newton steps, warm-started from the last pass, on
      //   F(dmu) = sum_i s_i a_i b_i / ((s_i + mu)^2 (s_i + mu^a)^2) + (phi(mu^a; za) - 1),
      //   a_i = dz_i (s_i + mu^a) - za_i dmu,  b_i = z_i (s_i + mu^a) + za_i (s_i + mu),
      // which is phi(mu; z) - 1 written with increments, F' = -2 sum_i s_i z_i^2 / (s_i + mu)^3.
      bool cin[CT];
      if (WL) {
        if (__any(fresh_lane)) {
          float mu[CT], th2[CT], ph[CT];
          bool go[CT], ins[CT];
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
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
            ins[ct] = !(qs > 1.f);
            go[ct] = (st[ct] == COL_ACTIVE && (flags[ct] & FLAG_FIRST)) && !ins[ct];
            mu[ct] = 0.f;
            ph[ct] = qs;
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
                  const float zz = z[rt][ct][q], sv = th2[ct] * wv[rt][q];
                  const float inv = sv > 0.f ? __builtin_amdgcn_rcpf(sv + mu[ct]) : 0.f;
                  const float e = sv * zz * zz * inv * inv;
                  pa += e;
                  pb3 += e * inv;
                }
              const float phs = col_sumf(pa), ps = col_sumf(pb3);
              const float stp = phs * (__builtin_sqrtf(phs) - 1.f) / ps;
              go[ct] = go[ct] && stp > kWl2Rel * mu[ct];
              if (go[ct]) { mu[ct] += stp; ph[ct] = phs; }
              any |= go[ct] ? 1 : 0;
            }
            if (!__any(any)) break;
          }
#pragma unroll
          for (int ct = 0; ct < CT; ++ct)
            if (st[ct] == COL_ACTIVE && (flags[ct] & FLAG_FIRST)) {
              gama[ct] = ins[ct] ? 0.0 : (double)mu[ct];
              dgam[ct] = 0.f;
              ssa2[ct] = 0.0;
              flags[ct] = ins[ct] ? (flags[ct] | FLAG_INSIDE) : (flags[ct] & ~FLAG_INSIDE);
            }
        }
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          const float th2 = thr[ct] * thr[ct];
          float qa = 0.f;
#pragma unroll
          for (int rt = 0; rt < RTM; ++rt)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const float zz = z[rt][ct][q] + dz[rt][ct][q], sv = th2 * wv[rt][q];
              qa += sv > 0.f ? zz * zz * __builtin_amdgcn_rcpf(sv) : 0.f;
            }
          cin[ct] = !(col_sumf(qa) > 1.f);
        }
#pragma unroll
        for (int it = 0; it < 2; ++it) {
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            const float th2 = thr[ct] * thr[ct];
            const float mua = (float)gama[ct], dm = dgam[ct], mu = mua + dm;
            float fa = 0.f, ga2 = 0.f;
#pragma unroll
            for (int rt = 0; rt < RTM; ++rt)
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const float sv = th2 * wv[rt][q];
                const float za = z[rt][ct][q], dzv = dz[rt][ct][q], zz = za + dzv;
                const float A = sv + mua, B = sv + mu;
                const float iA = sv > 0.f ? __builtin_amdgcn_rcpf(A) : 0.f;
                const float iB = sv > 0.f ? __builtin_amdgcn_rcpf(B) : 0.f;
                const float a = dzv * A - za * dm, b = zz * A + za * B;
                fa += sv * a * b * (iB * iB) * (iA * iA);
                ga2 += sv * zz * zz * (iB * iB * iB);
              }
            const float F = col_sumf(fa) + (float)ssa2[ct], G = col_sumf(ga2);
            const bool upd = !(flags[ct] & FLAG_FIRST) && !cin[ct] && G > 0.f;
            float dn = upd ? dm + F / (2.f * G) : dm;
            dn = fmaxf(dn, -mua);  // mu stays >= 0
            dgam[ct] = dn;
          }
        }
      }

      // ---------------------------------------------------------- right-hand sides
      // increment: dd = prox(za + dz) - prox(za) from za's shrink decomposition (exact in FP32 for
      // the shrink), r = lambda (2 dd - dz), u = dz + ea - dd: the products return the next dz;
      // a value pass takes u = 0 (the plain product)
      auto inc = [&](int ct, int rt, int q, float dzv, float* sa, float* lo, float* hi) -> float {
        const float za = z[rt][ct][q];
        if (WL) {  // dd = (mu dz (s + mu^a) + za s dmu) / ((s + mu)(s + mu^a)), or -d^a inside
          const float sv = thr[ct] * thr[ct] * wv[rt][q];
          const float mua = (float)gama[ct], dm = dgam[ct], mu = mua + dm;
          const float A = sv + mua, B = sv + mu;
          const bool ains = flags[ct] & FLAG_INSIDE;
          const float da = (ains || !(sv > 0.f)) ? 0.f : mua * za * __builtin_amdgcn_rcpf(A);
          const float inside_dd = -da;
          const float out_dd = sv > 0.f ? (mu * dzv * A + za * sv * dm) * __builtin_amdgcn_rcpf(B * A) : 0.f;
          *sa = da; *lo = 0.f; *hi = 0.f;  // sa returns d^a (FP32) for a fresh column's start
          return cin[ct] ? inside_dd : out_dd;
        }
        const float th = theta_f(has_l1 ? thr[ct] : 0.f, wv[rt][q]);
        const float ca = med3f(za, -th, th);
        *sa = za - ca; *lo = -th - ca; *hi = th - ca;
        const float ds = dzv - med3f(dzv + *sa, *lo, *hi);
        return HL2 ? (float)gama[ct] * ds + dgam[ct] * (*sa + ds) : ds;
      };
      f32x4 r[RTM][CT], u[RTM][CT];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const bool isphi = st[ct] == COL_PHI;
        const bool fresh = flags[ct] & FLAG_FIRST;
        const float gaf = (float)gama[ct];
#pragma unroll
        for (int rt = 0; rt < RTM; ++rt) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float dzv = dz[rt][ct][q];
            float sa, lo, hi;
            const float dd = inc(ct, rt, q, dzv, &sa, &lo, &hi);
            const float da = HL2 ? gaf * sa : sa;
            const float zz = z[rt][ct][q];
            r[rt][ct][q] = fresh ? xp[rt][ct][q] + flam * (2.f * da - zz) : flam * (2.f * dd - dzv);
            u[rt][ct][q] = fresh ? -da : (isphi ? 0.f : dzv + xp[rt][ct][q] - dd);
          }
        }
      }

      // ---------------------------------------------------------- products, then the step sums
#pragma unroll
      for (int rt = 0; rt < RTM; ++rt)
#pragma unroll
        for (int kt = 0; kt < RTM; ++kt) {
          const f32x4 a = mfrag(rt, kt);
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
              u[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q], r[kt][ct][q], u[rt][ct], 0, 0, 0);
        }

      float s0[CT], s1[CT];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const bool act = st[ct] == COL_ACTIVE;
        const bool isphi = st[ct] == COL_PHI;
        const bool fresh = flags[ct] & FLAG_FIRST;
        float a0 = 0.f, a1 = 0.f;
#pragma unroll
        for (int rt = 0; rt < RTM; ++rt) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float res = u[rt][ct][q];
            const float dzv = dz[rt][ct][q];
            float sa, lo, hi;
            const float dd = inc(ct, rt, q, dzv, &sa, &lo, &hi);
            const float dzn = isphi ? dzv + xp[rt][ct][q] + res - dd : res;
            const float step = dzn - dzv;
            a0 += step * step;
            if (HL2) {  // the shrink2 norm's increment (only the l2 kinds use it)
              const float dsn = dzn - med3f(dzn + sa, lo, hi);
              a1 += dsn * (2.f * sa + dsn);
            }
            if (act) {
              dz[rt][ct][q] = dzn;
              if (fresh) xp[rt][ct][q] = res;  // ea (FP32 estimate)
            }
          }
        }
        s0[ct] = col_sumf(a0);
        s1[ct] = HL2 ? col_sumf(a1) : 0.f;
      }

      // ---------------------------------------------------------- value terms (value passes)
      // From the exact-product identity at the current iterate, in FP64: d = d^a + dd,
      // v = v^a + dv (v^a = ea + d^a), r = r^a + dr; the pass's increment is applied here too.
      double v2s[CT], v3s[CT], v4s[CT], v5s[CT];
      f32x4 pd[RTM][CT];  // p of a value pass
      if (any_phi) {
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          const bool isphi = st[ct] == COL_PHI;
          double w2 = 0.0, w3 = 0.0, w4 = 0.0, w5 = 0.0;
          const HOPF_GLOBAL float* xj = gp(pb.x + (size_t)jj[ct] * n);
          const HOPF_GLOBAL double* cen = pb.centres ? gp(pb.centres + (size_t)kk[ct] * n_pad) : nullptr;
          const double th1 = has_l1 ? (double)pb.t[jj[ct]] / lam : 0.0;
          const double wl_th = (double)pb.t[jj[ct]] / lam;  // WL: s_i = wl_th^2 w_i
          const float thn = has_l1 ? thr[ct] : 0.f;
          const float gaf = (float)gama[ct];
#pragma unroll 1
          for (int rt = 0; rt < RTM; ++rt) {
            const f32x4 zv = get4(z, rt, ct), ev = get4(xp, rt, ct), uv = get4(u, rt, ct), w4v = getw(rt);
            f32x4 dv = get4(dz, rt, ct), pv;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int row = 16 * rt + 4 * lg + q;
              const bool inb = isphi && rt < nrt && row < n;
              const float dzv = dv[q], za = zv[q];
              float dd;
              double da;
              const double wr = inb ? *gp(pb.w + row) : 0.0;
              if (WL) {
                const float sv = thr[ct] * thr[ct] * w4v[q];
                const float mua = (float)gama[ct], dm = dgam[ct], mu = mua + dm;
                const float A = sv + mua, B = sv + mu;
                const bool ains = flags[ct] & FLAG_INSIDE;
                const float daf = (ains || !(sv > 0.f)) ? 0.f : mua * za * __builtin_amdgcn_rcpf(A);
                dd = cin[ct] ? -daf : (sv > 0.f ? (mu * dzv * A + za * sv * dm) * __builtin_amdgcn_rcpf(B * A) : 0.f);
                const double s64 = wl_th * wl_th * wr;
                da = (ains || !(s64 > 0.0)) ? 0.0 : gama[ct] * (double)za / (s64 + gama[ct]);
              } else {
                const float th = theta_f(thn, w4v[q]);
                const float ca = med3f(za, -th, th), sa = za - ca;
                const float ds = dzv - med3f(dzv + sa, -th - ca, th - ca);
                dd = HL2 ? gaf * ds + dgam[ct] * (sa + ds) : ds;
                da = gama[ct] * (has_l1 ? (double)za - fmin(fmax((double)za, -th1 * wr), th1 * wr) : (double)za);
              }
              const double d = inb ? da + (double)dd : 0.0;
              const double vv = (double)ev[q] + da + (double)uv[q];
              const double xpd = inb ? (double)xj[row] - (cen ? cen[row] : 0.0) : 0.0;
              const double rr = xpd + lam * (2.0 * da - (double)za) + lam * (2.0 * (double)dd - (double)dzv);
              w2 += xpd * d;
              w3 += (2.0 * d - vv) * (rr - lam * vv);
              w4 += WL ? wr * d * d : wr * fabs(d);
              w5 += d * d;
              pv[q] = (float)d;
              if (isphi) dv[q] = dzv + ev[q] + uv[q] - dd;
            }
            set4(pd, rt, ct, pv);
            set4(dz, rt, ct, dv);
          }
          v2s[ct] = col_sum(w2); v3s[ct] = col_sum(w3); v4s[ct] = col_sum(w4); v5s[ct] = col_sum(w5);
        }
      }

      // ---------------------------------------------------------- per-column update
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const bool isphi = st[ct] == COL_PHI;
        if (!(st[ct] == COL_ACTIVE || isphi)) continue;
        const double sm0 = (double)s0[ct];
        iters[ct] += 1;
        if (HL2) {
          const double nz = sqrt(fmax(ssa2[ct] + (double)s1[ct], 0.0));
          const double gg = nz > 0.0 ? fmax(nz - (double)thr[ct], 0.0) / nz : 0.0;
          gam[ct] = (float)gg;
          dgam[ct] = (float)(gg - gama[ct]);
        }
        flags[ct] &= ~FLAG_FIRST;
        // (|dz_k| + |dz_{k-1}|)^2 <= tol, on increments measured from an exact anchor
        const double pv = (double)prev[ct];
        prev[ct] = (float)sm0;
        const bool conv = (flags[ct] & FLAG_EXACT) && sm0 + pv + 2.0 * sqrt(sm0 * pv) <= pb.tol;
        const bool capped = iters[ct] >= pb.max_iter;
        if (!isphi) {
          if (conv) st[ct] = COL_WAITING;
          else if (capped) { st[ct] = COL_WAITING; flags[ct] |= FLAG_SOLVE_CAP | FLAG_CAPPED; }
        } else {
          if (capped && !conv) flags[ct] |= FLAG_SOLVE_CAP | FLAG_CAPPED;
          if (conv || (flags[ct] & FLAG_SOLVE_CAP)) {
            const double pn = sqrt(v5s[ct]);
            const double H = WL ? sqrt(v4s[ct]) : (has_l1 ? v4s[ct] : 0.0) + (HL2 ? pn : 0.0);
            const double tv = (double)pb.t[jj[ct]];
            phi[ct] = v2s[ct] - 0.5 * v3s[ct] - tv * H - (pb.level_set ? 0.5 : 0.0);
            hp[ct] = H;
            st[ct] = COL_DONE;
#pragma unroll
            for (int rt = 0; rt < RTM; ++rt) z[rt][ct] = pd[rt][ct];  // p replaces za
          } else {
            st[ct] = COL_ACTIVE;
          }
        }
      }
    };
    (void)hkind;
    if constexpr (REF) pass_ref(std::integral_constant<int, KS>{});
    else pass(std::integral_constant<int, KS>{});
  }
}

bool dense_small_fits(int mode, int n_pad, int distance) { return mode != 1 && !distance && n_pad <= 64; }

int dense_small_cols() { return 16 * SMALL_CT; }
int dense_small_occupancy() { return SMALL_OCC; }

int dense_small_kind(int hkind) { return hkind == HK_WL2 || hkind == HK_AL2 ? 2 : (hk_has_l2(hkind) ? 1 : 0); }

template <int KS>
static void launch_small_kind(int n_pad, bool refined, const DenseProb* d_probs, const DenseChunk* d_chunks,
                              int nchunks, int* counter, int grid, int anchor_every, int anchor_wait, int det,
                              hipStream_t stream) {
#define HOPF_SMALL(R, F)                                                                                        \
  hipLaunchKernelGGL((dense_small_kernel<R, SMALL_CT, SMALL_OCC, F, KS>), dim3(grid), dim3(kBlock), 0, stream, \
                     d_probs, d_chunks, nchunks, counter, anchor_every, anchor_wait, det)
  if (n_pad <= 32) {
    if (refined) HOPF_SMALL(2, true); else HOPF_SMALL(2, false);
  } else {
    if (refined) HOPF_SMALL(4, true); else HOPF_SMALL(4, false);
  }
#undef HOPF_SMALL
}

hipError_t launch_dense_small(int n_pad, bool refined, int kind, const DenseProb* d_probs, const DenseChunk* d_chunks,
                              int nchunks, int* counter, int grid, int anchor_every, int anchor_wait, int det,
                              hipStream_t stream) {
  if (n_pad > 64 || kind < 0 || kind > 2) return hipErrorInvalidValue;
  if (kind == 0) launch_small_kind<0>(n_pad, refined, d_probs, d_chunks, nchunks, counter, grid, anchor_every, anchor_wait, det, stream);
  else if (kind == 1) launch_small_kind<1>(n_pad, refined, d_probs, d_chunks, nchunks, counter, grid, anchor_every, anchor_wait, det, stream);
  else launch_small_kind<2>(n_pad, refined, d_probs, d_chunks, nchunks, counter, grid, anchor_every, anchor_wait, det, stream);
  return hipGetLastError();
}

}  // namespace hopf
