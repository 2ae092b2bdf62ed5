// Refined dense solver (BF16 increments on exact integer-sliced anchor products, as the refined
// mode of dense.hip) with the column iteration held on chip: one persistent workgroup of 8 waves
// per CU (two per SIMD) owns a tile of 32 columns (one point each, K = 1), and wave w owns the
// row tiles w, w + 8, w + 16, ... of every column.  The increment dz (FP32) stays in the owner
// wave's registers in the 16x16 MFMA output layout; ea = v^a - d^a (BF16 at n_pad > 512, else
// FP32) sits in LDS in the same layout; the anchor za (FP32), which changes only at anchors,
// lives in the workgroup's staging in global memory (L2-resident) and is read where a phase needs
// it.  The anchor has to be the nearest float of z: the products see only increments from it, so
// any remainder left in dz (a BF16 anchor, say) would enter every BF16 product and bound the
// accuracy at about 2^-18 of |z|.
// Per pass only M's BF16 fragments (L2-resident) and the anchors are streamed; at anchors, M's
// integer slices.
//
// The method is that of dense.hip (split Bregman, eqs. (3.4a)-(3.4c), in Douglas-Rachford form
// on z = v + b; the increment form of the refined mode).  A pass:
//   prologue  every wave forms, for its rows, dd = prox(za + dz) - prox(za) (from za's shrink
//             decomposition and the column's l2 factors) and dr = lambda (2 dd - dz), rounded to
//             BF16 into the right-hand-side buffer (a fresh column's first pass instead takes
//             r = x' + lambda (2 d^a - za), d^a the prox of za: its product gives an estimate of
//             ea, replaced at the column's first exact anchor);
//   products  v = M dr, BF16 MFMA 16x16x32 with FP32 accumulate, the wave's row tiles in groups
//             of four, M's fragments streamed kPF k-steps ahead (M is what a pass streams:
//             2 n_pad^2 bytes from L2 per 32 columns);
//   epilogue  step = ea + v - dd, dz += step, and the column partial sums (step^2 and the
//             increment of |shrink1(z)|^2), reduced over lane groups and then waves;
//   update    one thread per column: stopping test (only after an exact anchor), l2 factor,
//             the workgroup's anchor decision.
// Every `anchor_every` passes (and whenever only converged columns are left) an anchor re-bases
// za <- za + dz and takes v^a = M r^a exactly in integer slices (the kSlices definitions) of the
// FP64 r^a = x' + lambda (2 d^a - za), d^a with FP64 thresholds; a converged column is accepted
// only if the stopping test still passes in the pass right after it (its value pass, which also
// evaluates phi from the exact-product identity of dense.hip and writes p).
#include <algorithm>

#include "common.hpp"
#include "dense.hpp"
#include "dense_shared.hpp"

namespace hopf {

namespace {
constexpr int kNW = 8;          // waves per workgroup (two per SIMD)
constexpr int kCT = 2;          // column tiles of 16
constexpr int kPT = 16 * kCT;   // columns per workgroup
constexpr int kRG = 4;          // row tiles per product group
constexpr int kPF = 3;          // k-steps of M's fragments in flight
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f32x4 f4(bf16x4 v) { return f32x4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]}; }
__device__ __forceinline__ bf16x4 b4(f32x4 v) {
  return bf16x4{to_bf16(v[0]), to_bf16(v[1]), to_bf16(v[2]), to_bf16(v[3])};
}
// clamp of x to [lo, hi] (lo <= hi) in one instruction
__device__ __forceinline__ float med3f(float x, float lo, float hi) { return __builtin_amdgcn_fmed3f(x, lo, hi); }
// ea storage in LDS: FP32 or BF16
__device__ __forceinline__ f32x4 edec(f32x4 v) { return v; }
__device__ __forceinline__ f32x4 edec(bf16x4 v) { return f4(v); }
template <typename EV> __device__ __forceinline__ EV eenc(f32x4 v);
template <> __device__ __forceinline__ f32x4 eenc<f32x4>(f32x4 v) { return v; }
template <> __device__ __forceinline__ bf16x4 eenc<bf16x4>(f32x4 v) { return b4(v); }
}  // namespace

// RW: row tiles per wave (n_pad <= 16 NW RW).
template <int RW, typename EV>
__global__ void __launch_bounds__(kNW * 64, 1)
dense_rs_kernel(const DenseProb* __restrict__ probs, const DenseChunk* __restrict__ chunks, int nchunks,
                int* __restrict__ chunk_counter, double* __restrict__ ws64, int64_t ws64_per_wg,
                float* __restrict__ ws, int64_t ws_per_wg, int anchor_every, int anchor_wait, int det) {
  constexpr int NW = kNW, CT = kCT, PT = kPT;
  static_assert(PT <= 64, "the slot bookkeeping takes one lane of wave 0 per slot");
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  __shared__ ColShared<PT, NW> S;
  __shared__ __attribute__((aligned(16))) float Wl[1024];  // the problem's FP32 weights
  // LDS: ea (BF16, [wave][i][ct][lane] x 4) then the right-hand sides (BF16, [column][n_pad + 8]);
  // during an anchor the right-hand-side buffer holds blocks of r^a's slices
  EV* const Ebuf = (EV*)lds_raw;
  __bf16* const Bbuf = (__bf16*)(lds_raw + (size_t)NW * RW * CT * 64 * sizeof(EV));

  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  // Lane indices are re-derived at the start of every phase from an opaque copy of the thread
  // index, so that the addresses computed from them are recomputed (a few integer operations)
  // rather than kept in registers across the whole loop.
  int tid, l, lr, lg;
  auto lanes = [&]() {
    int t = (int)threadIdx.x;
    asm volatile("" : "+v"(t));
    tid = t; l = t & 63; lr = l & 15; lg = l >> 4;
  };
  lanes();
  auto eidx = [&](int i, int ct) { return ((wave * RW + i) * CT + ct) * 64 + l; };
  // float staging in global memory, [3][wave][i][ct][lane] x 4: slot 0 holds za, slot 1 dz during
  // anchors and value passes, slot 2 v of value passes
  float* const sst = ws + (int64_t)blockIdx.x * ws_per_wg;
  auto sidx = [&](int which, int i, int ct) {
    return ((((size_t)which * NW + wave) * RW + i) * CT + ct) * 256 + 4 * l;
  };

  f32x4 dz[RW][CT];
#pragma unroll
  for (int i = 0; i < RW; ++i)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      dz[i][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
      st_nt4(sst + sidx(0, i, ct), dz[i][ct]);
    }
  int wprob = -1;  // the problem whose weights are in Wl

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
    __syncthreads();
    lanes();
    const DenseProb pb = probs[S.ctl[CTL_PROB]];
    const int n = pb.n, n_pad = pb.n_pad;
    const double lam = pb.lambda;
    const float flam = (float)lam;
    const bool has_l1 = hk_has_l1(pb.hkind), has_l2 = hk_has_l2(pb.hkind);
    const int RT = n_pad >> 4;
    const int nrw = RT > wave ? (RT - wave + NW - 1) / NW : 0;  // row tiles of this wave
    const int ldb = n_pad + 8;
    if (S.ctl[CTL_PROB] != wprob) {  // workgroup-uniform
      for (int r = tid; r < n_pad; r += NW * 64) Wl[r] = pb.wf[r];
      wprob = S.ctl[CTL_PROB];
      __syncthreads();
    }

    // ============================================================ anchor
    if (S.ctl[CTL_ANCHOR]) {
      lanes();
      // A1: re-base z = za + dz (za the nearest float, dz the remainder), the FP64 shrink reference
      //     and the norms of the shrink2 factors
      {
        double pss[CT], pinc[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          pss[ct] = 0.0; pinc[ct] = 0.0;
          const int c = 16 * ct + lr;
          const int st = S.state[c];
          const bool on = (st == COL_ACTIVE && !S.fresh[c]) || st == COL_WAITING;
          const double th1 = S.th1[c];
          const float th1f = (float)th1;
#pragma unroll
          for (int i = 0; i < RW; ++i) {
            if (i >= nrw) continue;  // wave-uniform
            const int rt = wave + NW * i;
            const f32x4 wv = *(const f32x4*)(Wl + 16 * rt + 4 * lg);
            f32x4 zv = ld_nt4(sst + sidx(0, i, ct)), dv = dz[i][ct];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int row = 16 * rt + 4 * lg + q;
              const double z = (double)zv[q] + (double)dv[q];
              const float zan = (float)z;
              const float dzn = (float)(z - (double)zan);
              const float th = theta_f(th1f, wv[q]);
              const float ca = med3f(zan, -th, th), sa = zan - ca;
              const float ds = dzn - med3f(dzn + sa, -th - ca, th - ca);
              const double sa64 = row < n ? anchor_shrink(zan, th1, pb.w, row) : 0.0;
              if (on) {
                pss[ct] += sa64 * sa64;
                pinc[ct] += (double)ds * (2.0 * (double)sa + (double)ds);
                zv[q] = zan; dv[q] = dzn;
              }
            }
            st_nt4(sst + sidx(0, i, ct), zv);
            dz[i][ct] = dv;
            __builtin_amdgcn_sched_barrier(0);
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
          if ((st == COL_ACTIVE && !S.fresh[c]) || st == COL_WAITING) {
            double a = 0.0, b = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) { a += S.red[w][c][0]; b += S.red[w][c][1]; }
            S.ssa2[c] = a;
            const double ssq = a + b;
            double ga = 1.0, g = 1.0;
            if (has_l2) {
              const double na = sqrt(a), nz = sqrt(fmax(ssq, 0.0)), th2 = S.th2[c];
              ga = na > 0.0 ? fmax(na - th2, 0.0) / na : 0.0;
              g = nz > 0.0 ? fmax(nz - th2, 0.0) / nz : 0.0;
            }
            S.gama[c] = ga; S.gam[c] = g; S.dgam[c] = g - ga;
          }
        }
        __syncthreads();
      }
      lanes();
      // A2: dz to the staging (the registers are needed below), r^a = x' + lambda (2 d^a - za) in
      //     FP64 in registers, its column maxima, then its integer slices ([slice][column][k])
      //     straight from the registers: a lane's four rows of a column make one 32-bit word
#pragma unroll
      for (int i = 0; i < RW; ++i)  // every slot, so that none of the registers stays live
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) st_nt4(sst + sidx(1, i, ct), dz[i][ct]);
      const int n64 = pad64(n_pad);
      int8_t* const rq = (int8_t*)(ws64 + (int64_t)blockIdx.x * ws64_per_wg);
      {
        double rv[RW][CT][4];
        double cmax[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          cmax[ct] = 0.0;
          const int c = 16 * ct + lr;
          const int st = S.state[c];
          const bool on = (st == COL_ACTIVE && !S.fresh[c]) || st == COL_WAITING;
          const double th1 = S.th1[c], ga = S.gama[c];
          const HOPF_GLOBAL float* xj = gp(pb.x + (size_t)S.j[c] * n);
          const HOPF_GLOBAL double* cen = pb.centres ? gp(pb.centres) : nullptr;
#pragma unroll
          for (int i = 0; i < RW; ++i) {
#pragma unroll
            for (int q = 0; q < 4; ++q) rv[i][ct][q] = 0.0;
            if (i >= nrw) continue;
            const int row0 = 16 * (wave + NW * i) + 4 * lg;
            if (on) {
              const f32x4 zv = ld_nt4(sst + sidx(0, i, ct));
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int row = row0 + q;
                if (row < n) {
                  const double sa64 = anchor_shrink(zv[q], th1, pb.w, row);
                  const double xp = (double)xj[row] - (cen ? cen[row] : 0.0);
                  rv[i][ct][q] = xp + lam * (2.0 * ga * sa64 - (double)zv[q]);
                  cmax[ct] = fmax(cmax[ct], fabs(rv[i][ct][q]));
                }
              }
            }
          }
        }
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          double m = cmax[ct];
          m = fmax(m, __shfl_xor(m, 16));
          m = fmax(m, __shfl_xor(m, 32));
          if (l < 16) S.red[wave][16 * ct + l][0] = m;
        }
        __syncthreads();
        if (tid < PT) {
          double m = 0.0;
#pragma unroll
          for (int w = 0; w < NW; ++w) m = fmax(m, S.red[w][tid][0]);
          S.rexp[tid] = slice_exponent(m);
        }
        __syncthreads();
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          const int c = 16 * ct + lr;
          const int fe = S.rexp[c];
#pragma unroll
          for (int i = 0; i < RW; ++i) {
            if (i >= nrw) continue;
            const int row0 = 16 * (wave + NW * i) + 4 * lg;
            uint32_t word[kSlices];
#pragma unroll
            for (int s = 0; s < kSlices; ++s) word[s] = 0u;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              double x = ldexp(rv[i][ct][q], -fe);
#pragma unroll
              for (int s = 0; s < kSlices; ++s) {
                x *= 128.0;
                const double r = rint(x);
                x -= r;
                word[s] |= (uint32_t)(uint8_t)(int8_t)(int)r << (8 * q);
              }
            }
#pragma unroll
            for (int s = 0; s < kSlices; ++s) *gp((uint32_t*)(rq + ((size_t)s * PT + c) * n64 + row0)) = word[s];
          }
        }
        // rows n_pad .. n64 - 1 of the slices (a k-step of 64 reaches past n_pad): zero
        for (int u = tid; u < kSlices * PT * (n64 - n_pad) / 4; u += NW * 64) {
          const int w4 = (n64 - n_pad) / 4, sc = u / w4, k4 = n_pad + 4 * (u - sc * w4);
          *gp((uint32_t*)(rq + (size_t)sc * n64 + k4)) = 0u;
        }
      }
      lanes();
      // A3: products one row tile per wave and round, r^a's slices through LDS in blocks of kbq
      //     rows; ea = v^a - d^a into the LDS ea buffer
      {
        const int kbq = anchor_kbq(n_pad), ldq = kbq + 16;
        int8_t* const Bq = (int8_t*)Bbuf;
        for (int i = 0; i < RW; ++i) {  // rounds: row tile i of every wave
          const bool has = i < nrw;       // wave-uniform
          const int rt = wave + NW * i;
          i32x4 acc[kSlices][CT];
#pragma unroll
          for (int s = 0; s < kSlices; ++s)
#pragma unroll
            for (int c = 0; c < CT; ++c) acc[s][c] = i32x4{0, 0, 0, 0};
          for (int k0 = 0; k0 < n64; k0 += kbq) {
            const int kb = n64 - k0 < kbq ? n64 - k0 : kbq;
            const int hu = kb >> 4;
            __syncthreads();
            constexpr int kU = 6;  // 16-byte units in flight per thread
            for (int u0 = tid; u0 < kSlices * PT * hu; u0 += kU * NW * 64) {
              i32x4 t[kU];
#pragma unroll
              for (int e = 0; e < kU; ++e) {
                const int u = u0 + e * NW * 64;
                if (u < kSlices * PT * hu) {
                  const int sc = u / hu, off = 16 * (u - sc * hu);
                  t[e] = *gp((const i32x4*)(rq + (size_t)sc * n64 + k0 + off));
                }
              }
#pragma unroll
              for (int e = 0; e < kU; ++e) {
                const int u = u0 + e * NW * 64;
                if (u < kSlices * PT * hu) {
                  const int sc = u / hu, off = 16 * (u - sc * hu);
                  *(i32x4*)(Bq + sc * ldq + off) = t[e];
                }
              }
            }
            __syncthreads();
            if (has) gemm_slices<CT>(pb.Mq, RT, n64 >> 6, rt, k0 >> 6, kb >> 6, Bq, ldq, acc);
          }
          if (!has) continue;
          const int row0 = 16 * rt + 4 * lg;
          int rexp_row[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) rexp_row[q] = *gp(pb.Mqe + row0 + q);
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            const int c = 16 * ct + lr;
            const int st = S.state[c];
            if (!((st == COL_ACTIVE && !S.fresh[c]) || st == COL_WAITING)) continue;
            const double ga = S.gama[c], th1 = S.th1[c];
            const int fe = S.rexp[c];
            const f32x4 zv = ld_nt4(sst + sidx(0, i, ct));
            f32x4 ev;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int row = row0 + q;
              double v = 0.0;  // smallest terms first
#pragma unroll
              for (int s = kSlices - 1; s >= 0; --s) v += ldexp((double)acc[s][ct][q], rexp_row[q] + fe - 7 * (s + 2));
              const double sa64 = row < n ? anchor_shrink(zv[q], th1, pb.w, row) : 0.0;
              ev[q] = row < n ? (float)(v - ga * sa64) : 0.f;
            }
            Ebuf[eidx(i, ct)] = eenc<EV>(ev);
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < RW; ++i)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) dz[i][ct] = ld_nt4(sst + sidx(1, i, ct));
      if (tid < PT) {
        const int st = S.state[tid];
        if ((st == COL_ACTIVE && !S.fresh[tid]) || st == COL_WAITING) S.flags[tid] |= FLAG_EXACT;
        if (st == COL_WAITING) S.state[tid] = COL_PHI;
      }
      if (tid == 0) { S.ctl[CTL_ANCHOR] = 0; S.ctl[CTL_LAST_ANCHOR] = k_it; }
      __syncthreads();
    }

    lanes();
    // ============================================================ settle finished columns
    // p of a finished column was written to the output by its value pass; here its scalars, and
    // NaN rows for invalid inputs
    {
      int nan_rows = 0;
      if (tid < PT) {
        const int c = tid;
        const int st = S.state[c];
        S.better[c] = 0;
        if (st == COL_DONE || st == COL_INVALID) {
          const int64_t j = S.j[c];
          if (pb.iter_total) atomicAdd(pb.iter_total, (unsigned long long)S.iters[c]);
          if (st == COL_INVALID) {
            const float qnan = __builtin_nanf("");
            pb.phi[j] = qnan; pb.dphidt[j] = qnan;
            if (pb.iters) pb.iters[j] = -1;
            if (pb.kstar) pb.kstar[j] = -1;
            S.better[c] = 2;
            nan_rows = 1;
          } else {
            pb.phi[j] = (float)S.phi[c];
            pb.dphidt[j] = (float)(-S.hp[c]);
            if (pb.iters) pb.iters[j] = (S.flags[c] & FLAG_CAPPED) ? -2 : S.iters[c];
            if (pb.kstar) pb.kstar[j] = 0;
            S.state[c] = COL_EMPTY;
          }
        }
      }
      if (tid == 0) S.ctl[CTL_BETTER] = 0;
      __syncthreads();
      if (nan_rows) S.ctl[CTL_BETTER] = 1;  // benign race: every writer stores 1
      __syncthreads();
      if (S.ctl[CTL_BETTER]) {
        for (int c = wave; c < PT; c += NW) {
          if (S.better[c] != 2) continue;
          const int64_t j = S.j[c];
          for (int i = l; i < n; i += 64) pb.grad[(size_t)j * n + i] = __builtin_nanf("");
        }
        __syncthreads();
        if (tid < PT && S.state[tid] == COL_INVALID) S.state[tid] = COL_EMPTY;
        __syncthreads();
      }
    }

    // ============================================================ refill empty slots
    // wave 0, one lane per slot: when the current chunk has a column for every empty slot, the
    // slots take consecutive columns in slot order; otherwise lane 0 walks the slots and fetches
    // chunks
    bool refilled = false;
    if (wave == 0) {
      const int st = l < PT ? S.state[l] : COL_ACTIVE;
      if (l < PT) S.fresh[l] = 0;
      const uint64_t em = __ballot(st == COL_EMPTY);
      const int nempty = __popcll(em);
      const int nextcol = S.ctl[CTL_NEXTCOL], cend = S.ctl[CTL_CHUNKEND];
      if (nempty <= cend - nextcol) {  // wave-uniform
        if ((em >> l) & 1) {
          const int col = nextcol + __popcll(em & ((1ull << l) - 1));
          S.col[l] = col; S.j[l] = col; S.k[l] = 0;
          S.fresh[l] = 1;
        }
        if (l == 0) { S.ctl[CTL_NEXTCOL] = nextcol + nempty; S.ctl[CTL_ANY] = 0; S.ctl[CTL_EXIT] = 0; }
        refilled = true;
      }
    }
    if (tid == 0 && !refilled) {
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
          S.col[c] = col; S.j[c] = col; S.k[c] = 0;
          S.fresh[c] = 1;
          ++live;
        }
      }
      int exitf = 0;
      if (live == 0) {
        if (pending >= 0) {
          prob = chunks[pending].prob;
          nextcol = chunks[pending].col0;
          cend = nextcol + chunks[pending].ncols;
          pending = -1;
          S.ctl[CTL_ANY] = 1;
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
    // fresh slots: scalars, then their state (owner waves: za = x', dz = 0), the finiteness check
    // and the norm of shrink1(x') for the l2 factor of the first pass
    int any_fresh = 0;
    if (tid < PT && S.fresh[tid]) {
      const int c = tid;
      const double tv = (double)pb.t[S.j[c]];
      S.t[c] = tv;
      S.state[c] = (tv > 0.0 && isfinite(tv)) ? COL_ACTIVE : COL_INVALID;
      S.th1[c] = has_l1 ? tv / lam : 0.0;
      S.th2[c] = has_l2 ? tv / lam : 0.0;
      S.gam[c] = 1.0; S.gama[c] = 1.0; S.dgam[c] = 0.0; S.ssa2[c] = 0.0; S.ssq[c] = 0.0;
      S.prev[c] = 1e300; S.phi[c] = 0.0; S.hp[c] = 0.0; S.pn[c] = 0.0;
      S.iters[c] = 0; S.flags[c] = 0;
      S.ctl[CTL_ANY] = 1;
    }
    __syncthreads();
    any_fresh = S.ctl[CTL_ANY];
    if (any_fresh) {
      lanes();
      float ps[CT];
      int bad[CT];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        ps[ct] = 0.f; bad[ct] = 0;
        const int c = 16 * ct + lr;
        if (!S.fresh[c]) continue;
        const float th1f = (float)S.th1[c];
        const HOPF_GLOBAL float* xj = gp(pb.x + (size_t)S.j[c] * n);
        const HOPF_GLOBAL double* cen = pb.centres ? gp(pb.centres) : nullptr;
#pragma unroll
        for (int i = 0; i < RW; ++i) {
          if (i >= nrw) continue;
          const int rt = wave + NW * i;
          const f32x4 wv = *(const f32x4*)(Wl + 16 * rt + 4 * lg);
          f32x4 v = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int row = 16 * rt + 4 * lg + q;
            if (row < n) {
              const float xv = xj[row];
              if (!isfinite(xv)) bad[ct] = 1;
              const float xp = (float)((double)xv - (cen ? cen[row] : 0.0));
              v[q] = xp;
              const float th = theta_f(th1f, wv[q]);
              const float sa = xp - med3f(xp, -th, th);
              ps[ct] += sa * sa;
            }
          }
          st_nt4(sst + sidx(0, i, ct), v);
          dz[i][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
          __builtin_amdgcn_sched_barrier(0);
        }
      }
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        double a = (double)ps[ct];
        a += __shfl_xor(a, 16); a += __shfl_xor(a, 32);
        int b = bad[ct];
        b |= __shfl_xor(b, 16); b |= __shfl_xor(b, 32);
        if (l < 16) { S.red[wave][16 * ct + l][0] = a; S.red[wave][16 * ct + l][1] = (double)b; }
      }
      __syncthreads();
      if (tid < PT && S.fresh[tid]) {
        const int c = tid;
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) { a += S.red[w][c][0]; b += S.red[w][c][1]; }
        if (b > 0.0) S.state[c] = COL_INVALID;
        S.ssa2[c] = a;
        double ga = 1.0;
        if (has_l2) {
          const double na = sqrt(a);
          ga = na > 0.0 ? fmax(na - S.th2[c], 0.0) / na : 0.0;
        }
        S.gama[c] = ga; S.gam[c] = ga; S.dgam[c] = 0.0;
      }
      if (tid == 0) S.ctl[CTL_ANY] = 0;
      __syncthreads();
    }
    {  // anything to iterate? (wave 0, one lane per slot; also whether a value pass is due)
      if (wave == 0) {
        const int st = l < PT ? S.state[l] : COL_EMPTY;
        const uint64_t m_it = __ballot(st == COL_ACTIVE || st == COL_PHI);
        const uint64_t m_inv = __ballot(st == COL_INVALID), m_phi = __ballot(st == COL_PHI);
        if (l == 0) {
          S.ctl[CTL_ANY] = (m_it ? 1 : 0) | (m_inv ? 2 : 0);
          S.ctl[CTL_PHIPASS] = m_phi != 0;
        }
      }
      __syncthreads();
      if (!(S.ctl[CTL_ANY] & 1)) {
        if (S.ctl[CTL_ANY] & 2) continue;  // only invalid slots: flush them
        if (tid == 0) S.ctl[CTL_ANCHOR] = 1;  // only waiting slots: an anchor makes them evaluable
        __syncthreads();
        continue;
      }
    }
    value_clear(S, tid);

    lanes();
    // ============================================================ prologue: right-hand sides
    // dd = prox(za + dz) - prox(za): shrink1 increment ds from za's decomposition (ca = clamp(za),
    // sa = za - ca), then the l2 factors: dd = ga ds + (g - ga)(sa + ds).  Fresh columns:
    // r = x' + lambda (2 d^a - za) with d^a = ga sa (za = x').
    {
      // a wave with all RW row tiles (every wave once n_pad = 16 NW RW) runs the tiles without
      // branches between them, so their anchor loads are in flight together
      auto prologue_tile = [&](int i, int ct, int c, int onmask, bool fresh, float th1f, float gaf, float dgf,
                               f32x4 zv) {
        const int row0 = 16 * (wave + NW * i) + 4 * lg;
        const f32x4 wv = *(const f32x4*)(Wl + row0);
        bf16x4 o;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float zz = zv[q], dzv = dz[i][ct][q];
          const float th = theta_f(th1f, wv[q]);
          const float ca = med3f(zz, -th, th), sa = zz - ca;
          const float ds = dzv - med3f(dzv + sa, -th - ca, th - ca);
          const float dd = gaf * ds + dgf * (sa + ds);
          const float rn = flam * (2.f * dd - dzv), rf = zz + flam * (2.f * gaf * sa - zz);
          // columns not iterated get +0 (a bit mask: no branch per element)
          o[q] = to_bf16(__int_as_float(__float_as_int(fresh ? rf : rn) & onmask));
        }
        *(bf16x4*)(Bbuf + c * ldb + row0) = o;
      };
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int c = 16 * ct + lr;
        const int st = S.state[c];
        const int onmask = (st == COL_ACTIVE || st == COL_PHI) ? -1 : 0;
        const bool fresh = S.fresh[c];
        const float th1f = (float)S.th1[c], gaf = (float)S.gama[c], dgf = (float)S.dgam[c];
        if (nrw == RW) {
          f32x4 zl[RW];
#pragma unroll
          for (int i = 0; i < RW; ++i) zl[i] = ld_nt4(sst + sidx(0, i, ct));
#pragma unroll
          for (int i = 0; i < RW; ++i) prologue_tile(i, ct, c, onmask, fresh, th1f, gaf, dgf, zl[i]);
        } else {
#pragma unroll
          for (int i = 0; i < RW; ++i)
            if (i < nrw) prologue_tile(i, ct, c, onmask, fresh, th1f, gaf, dgf, ld_nt4(sst + sidx(0, i, ct)));
        }
      }
    }
    __syncthreads();

    // ============================================================ products + epilogue
    float part[CT][2];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) { part[ct][0] = 0.f; part[ct][1] = 0.f; }
#pragma unroll
    for (int i0 = 0; i0 < RW; i0 += kRG) {
      if (i0 >= nrw) continue;  // wave-uniform
      lanes();
      int rt[kRG];
      int nr = 0;
#pragma unroll
      for (int r = 0; r < kRG; ++r) { rt[r] = wave + NW * (i0 + r); if (i0 + r < nrw) nr = r + 1; }
      f32x4 acc[kRG][CT];
#pragma unroll
      for (int r = 0; r < kRG; ++r)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[r][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
      gemm_bf16<kRG, CT, kPF>(pb.Mb, n_pad, Bbuf, ldb, rt, nr, acc);
      __builtin_amdgcn_sched_barrier(0);
      // one row tile of one column tile; columns not iterated (empty, waiting, done) keep dz
      auto epi_tile = [&](int r, int ct, int st, bool fresh, float th1f, float gaf, float dgf, f32x4 zv, f32x4 eb) {
        const bool on = st == COL_ACTIVE || st == COL_PHI;
        const int i = i0 + r;
        const int row0 = 16 * rt[r] + 4 * lg;
        const f32x4 wv = *(const f32x4*)(Wl + row0);
        const f32x4 v = acc[r][ct];
        const f32x4 dz0 = dz[i][ct];
        f32x4 dv, enew;
        float s0 = 0.f, s1 = 0.f;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float th = theta_f(th1f, wv[q]);
          const float ca = med3f(zv[q], -th, th), sa = zv[q] - ca;
          const float lo = -th - ca, hi = th - ca;
          const float ds = dz0[q] - med3f(dz0[q] + sa, lo, hi);
          const float dd = gaf * ds + dgf * (sa + ds);
          // fresh: v is M r^a, so ea = v - d^a (estimate) and the first step is ea
          const float ef = v[q] - gaf * sa, sn = eb[q] + v[q] - dd;
          const float step = fresh ? ef : sn;
          const float dzn = dz0[q] + step;
          const float dsn = dzn - med3f(dzn + sa, lo, hi);
          s0 += step * step;
          s1 += dsn * (2.f * sa + dsn);
          dv[q] = on ? dzn : dz0[q];
          enew[q] = ef;
        }
        part[ct][0] += on ? s0 : 0.f;
        part[ct][1] += on ? s1 : 0.f;
        if (on && fresh) Ebuf[eidx(i, ct)] = eenc<EV>(enew);
        if (st == COL_PHI) {  // the value phase below takes it from here
          st_nt4(sst + sidx(1, i, ct), dz0);
          st_nt4(sst + sidx(2, i, ct), v);
        }
        dz[i][ct] = dv;
      };
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int c = 16 * ct + lr;
        const int st = S.state[c];
        const bool fresh = S.fresh[c];
        const float th1f = (float)S.th1[c], gaf = (float)S.gama[c], dgf = (float)S.dgam[c];
        if (nr == kRG) {  // the group's anchors and ea loaded together
          f32x4 zg[kRG];
          EV eg[kRG];
#pragma unroll
          for (int r = 0; r < kRG; ++r) { zg[r] = ld_nt4(sst + sidx(0, i0 + r, ct)); eg[r] = Ebuf[eidx(i0 + r, ct)]; }
#pragma unroll
          for (int r = 0; r < kRG; ++r) epi_tile(r, ct, st, fresh, th1f, gaf, dgf, zg[r], edec(eg[r]));
        } else {
#pragma unroll
          for (int r = 0; r < kRG; ++r)
            if (r < nr)
              epi_tile(r, ct, st, fresh, th1f, gaf, dgf, ld_nt4(sst + sidx(0, i0 + r, ct)),
                       edec(Ebuf[eidx(i0 + r, ct)]));
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    // ============================================================ value pass
    // phi from the exact-product identity at the iterate the pass started from, and p = d, for
    // the columns of a value pass: their (za, dz, v) were staged by the epilogue; dd is formed
    // again with the same arithmetic
    if (S.ctl[CTL_PHIPASS]) {
      lanes();
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int c = 16 * ct + lr;
        if (S.state[c] != COL_PHI) continue;
        const double ga = S.gama[c], th1 = S.th1[c];
        const float th1f = (float)th1, gaf = (float)ga, dgf = (float)S.dgam[c];
        const HOPF_GLOBAL float* xj = gp(pb.x + (size_t)S.j[c] * n);
        const HOPF_GLOBAL double* cen = pb.centres ? gp(pb.centres) : nullptr;
        double v2 = 0.0, v3 = 0.0, v4 = 0.0, v5 = 0.0;
        for (int i = 0; i < nrw; ++i) {
          const int row0 = 16 * (wave + NW * i) + 4 * lg;
          const f32x4 wv = *(const f32x4*)(Wl + row0);
          const f32x4 eb = edec(Ebuf[eidx(i, ct)]);
          const f32x4 zv = ld_nt4(sst + sidx(0, i, ct)), dz0 = ld_nt4(sst + sidx(1, i, ct));
          const f32x4 v = ld_nt4(sst + sidx(2, i, ct));
          f32x4 pv;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int row = row0 + q;
            const float th = theta_f(th1f, wv[q]);
            const float ca = med3f(zv[q], -th, th), sa = zv[q] - ca;
            const float ds = dz0[q] - med3f(dz0[q] + sa, -th - ca, th - ca);
            const float dd = gaf * ds + dgf * (sa + ds);
            const double da = ga * anchor_shrink(zv[q], th1, pb.w, row < n ? row : 0);
            double d = da + (double)dd;
            const double vv = (double)eb[q] + da + (double)v[q];
            const double xp = (row < n) ? (double)xj[row] - (cen ? cen[row] : 0.0) : 0.0;
            const double rr = xp + lam * (2.0 * da - (double)zv[q]) + lam * (2.0 * (double)dd - (double)dz0[q]);
            if (row >= n) d = 0.0;
            v2 += xp * d;
            v3 += (2.0 * d - vv) * (rr - lam * vv);
            v4 += (double)wv[q] * fabs(d);
            v5 += d * d;
            pv[q] = (float)d;
          }
          store_grad(pb.grad + (size_t)S.j[c] * n, row0, n, pv);
        }
        value_sums(S.redv[wave][c], v2, v3, v4, v5, l);
      }
    }
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

    lanes();
    // ============================================================ per-column update
    if (tid < PT) {
      const int c = tid;
      const int st = S.state[c];
      if (st == COL_ACTIVE || st == COL_PHI) {
        double sm0 = 0.0, sm1 = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) { sm0 += S.red[w][c][0]; sm1 += S.red[w][c][1]; }
        S.iters[c] += 1;
        const double ssq = S.ssa2[c] + sm1;
        S.ssq[c] = ssq;
        double g = 1.0;
        if (has_l2) {
          const double nz = sqrt(fmax(ssq, 0.0));
          g = nz > 0.0 ? fmax(nz - S.th2[c], 0.0) / nz : 0.0;
        }
        S.gam[c] = g;
        S.dgam[c] = g - S.gama[c];
        const double a = sqrt(sm0), b = sqrt(S.prev[c]);
        S.prev[c] = sm0;
        const bool conv = (S.flags[c] & FLAG_EXACT) && (a + b) * (a + b) <= pb.tol;
        const bool capped = S.iters[c] >= pb.max_iter;
        if (st == COL_ACTIVE) {
          if (conv) S.state[c] = COL_WAITING;
          else if (capped) { S.state[c] = COL_WAITING; S.flags[c] |= FLAG_SOLVE_CAP | FLAG_CAPPED; }
        } else {
          if (capped && !conv) S.flags[c] |= FLAG_SOLVE_CAP | FLAG_CAPPED;
          if (conv || (S.flags[c] & FLAG_SOLVE_CAP)) {
            const double pn = sqrt(value_total(S, c, 3));
            const double H = (has_l1 ? value_total(S, c, 2) : 0.0) + (has_l2 ? pn : 0.0);
            S.phi[c] = value_total(S, c, 0) - 0.5 * value_total(S, c, 1) - S.t[c] * H - (pb.level_set ? 0.5 : 0.0);
            S.hp[c] = H; S.pn[c] = pn;
            S.state[c] = COL_DONE;
          } else {
            S.state[c] = COL_ACTIVE;
          }
        }
      }
      S.fresh[c] = 0;
    }
    __syncthreads();
    if (wave == 0) {  // the anchor decision, one lane per slot
      const int st = l < PT ? S.state[l] : COL_EMPTY;
      const uint64_t m_act = __ballot(st == COL_ACTIVE), m_wait = __ballot(st == COL_WAITING);
      if (l == 0) {
        const int kn = k_it + 1;
        if ((m_act && kn - S.ctl[CTL_LAST_ANCHOR] >= anchor_every) || (m_wait && !m_act) ||
            (anchor_wait > 0 && __popcll(m_wait) >= anchor_wait))
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
bool dense_rs_fits(int mode, int n_pad, int K, int hkind, int distance) {
  return mode == 1 && K == 1 && !distance && (hk_has_l1(hkind) || hk_has_l2(hkind)) && n_pad >= 64 &&
         n_pad <= 1024;
}
int dense_rs_cols() { return kPT; }

constexpr int kRWsmall = 512 / (16 * kNW), kRWlarge = 1024 / (16 * kNW);
static int rs_rw(int n_pad) { return n_pad <= 512 ? kRWsmall : kRWlarge; }

size_t dense_rs_lds_bytes(int n_pad) {
  const int RW = rs_rw(n_pad);
  const size_t e = (size_t)kNW * RW * kCT * 64 * (RW == kRWsmall ? 16 : 8);
  const size_t b = std::max((size_t)kPT * (n_pad + 8) * 2, (size_t)kSlices * kPT * (anchor_kbq(n_pad) + 16));
  return e + b;
}

// per workgroup: the float staging of the state during anchors and value passes
// (3 x NW x RW x CT x 256 floats)
int64_t dense_rs_ws_floats(int n_pad) {
  const int RW = rs_rw(n_pad);
  return (int64_t)3 * kNW * RW * kCT * 256;
}

template <int RW, typename EV>
static hipError_t launch_rs_t(const DenseProb* d_probs, const DenseChunk* d_chunks, int nchunks, int* counter,
                              double* ws64, int64_t ws64_per_wg, float* ws, int64_t ws_per_wg, int grid, size_t lds,
                              int anchor_every, int anchor_wait, int det, hipStream_t stream) {
  auto kern = dense_rs_kernel<RW, EV>;
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
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kNW * 64), lds, stream, d_probs, d_chunks, nchunks, counter, ws64,
                     ws64_per_wg, ws, ws_per_wg, anchor_every, anchor_wait, det);
  return hipGetLastError();
}

hipError_t launch_dense_rs(int max_npad, const DenseProb* d_probs, const DenseChunk* d_chunks, int nchunks,
                           int* counter, double* ws64, int64_t ws64_per_wg, float* ws, int64_t ws_per_wg, int grid,
                           size_t lds, int anchor_every, int anchor_wait, int det, hipStream_t stream) {
  if (max_npad <= 512)
    return launch_rs_t<kRWsmall, f32x4>(d_probs, d_chunks, nchunks, counter, ws64, ws64_per_wg, ws, ws_per_wg, grid, lds,
                          anchor_every, anchor_wait, det, stream);
  if (max_npad <= 1024)
    return launch_rs_t<kRWlarge, bf16x4>(d_probs, d_chunks, nchunks, counter, ws64, ws64_per_wg, ws, ws_per_wg, grid, lds,
                          anchor_every, anchor_wait, det, stream);
  return hipErrorInvalidValue;
}

}  // namespace hopf
