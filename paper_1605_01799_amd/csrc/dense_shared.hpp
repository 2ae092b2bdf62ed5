// Pieces of the dense solver: helpers, the per-wave MFMA products, and the per-column control
// block kept in LDS.
#pragma once
#include "common.hpp"

namespace hopf {

constexpr int kMaxCols = 64;
constexpr int kNRed = 6;  // step^2, |s|^2 increment, <x',d>, (2d-v).(r-lam v), sum w|d|, |d|^2

// Per-slot state accesses (global address space; the resident slots' state is sized to stay in
// the last-level cache, so ordinary cached accesses are used).
__device__ __forceinline__ f32x4 ld_nt4(const float* p) { return *gp((const f32x4*)p); }
__device__ __forceinline__ void st_nt4(float* p, f32x4 v) { *gp((f32x4*)p) = v; }
__device__ __forceinline__ float ld_nt(const float* p) { return *gp(p); }
__device__ __forceinline__ void st_nt(float* p, float v) { *gp(p) = v; }
__device__ __forceinline__ double ld_nt(const double* p) { return *gp(p); }
__device__ __forceinline__ void st_nt(double* p, double v) { *gp(p) = v; }

// Slot-state layout (z^a, dz, e^a of a tile's PT columns, n_pad rows each): 16 x 16 blocks,
// block (row tile rt, column tile ct) at (ct RT + rt) * 256 floats (RT = n_pad / 16); inside a
// block the MFMA output lane order, lane l = column % 16 + 16 * ((row % 16) / 4) holding rows
// 4 (l / 16) .. + 3 of column l % 16 as 4 consecutive floats.  A wave's f32x4 access of a block
// is one contiguous KiB.
__device__ __forceinline__ size_t st_block(int rt, int ct, int RT) { return ((size_t)ct * RT + rt) * 256; }
__device__ __forceinline__ size_t st_index(int c, int i, int RT) {
  return st_block(i >> 4, c >> 4, RT) + 4 * ((c & 15) + 16 * ((i & 15) >> 2)) + (i & 3);
}

__device__ __forceinline__ float clampf(float z, float lo, float hi) { return fminf(fmaxf(z, lo), hi); }
// FP32 threshold of coordinate i, used for the per-iteration increments (every use of a slot's
// threshold goes through this one formula, so all of them agree bit for bit).  The product is
// rounded here and may not be contracted into a later operation: -th - ca fused into one FMA with
// the unrounded product would make the increment interval [-th - ca, th - ca] miss 0 by the
// product's rounding error, and the increments would no longer vanish at a fixed point.
__device__ __forceinline__ float theta_f(float th1f, float wf) {
#pragma clang fp contract(off)
  return th1f * wf;
}
// shrink1 of an anchor value in FP64 with the FP64 threshold: the anchor reference d^a must be
// exact, since every increment of the following iterations is measured from it.
__device__ __forceinline__ double anchor_shrink(float za, double th1, const double* w, int i) {
  const double z = (double)za, th = th1 * *gp(w + i);
  return z - fmin(fmax(z, -th), th);
}

// ---------------------------------------------------------------- GEMM pieces (one wave)
// acc[r][c] += M[16 rt_r .. , :] * B[:, 16 c ..] over the full contraction.
// All RG row tiles are always computed (a row-tile index past the end is clamped to tile 0 and
// its result discarded by the caller), so the MFMA stream has no branches.
template <int RG, int CT, int PF = 3>
__device__ __forceinline__ void gemm_bf16(const __bf16* __restrict__ M, int n_pad,
                                                 const __bf16* B, int ldb, const int* rt, int nrt,
                                                 f32x4 (&acc)[RG][CT]) {
  // A fragments (rows of M, L2-resident) stream with PF k-steps in flight; B is in LDS.  Every
  // k-step issues its prefetch (past the end it re-reads the last k-step), so the loads in flight
  // are the same on every path and each MFMA waits only for its own fragments.
  const int l = threadIdx.x & 63;
  const int lr = l & 15, lg = l >> 4;
  // M is stored in fragment order (mb_index): row tile rt, k-step kk at (rt nk + kk) 64 + l
  const int nk = n_pad >> 5;
  const HOPF_GLOBAL bf16x8* arow[RG];
#pragma unroll
  for (int r = 0; r < RG; ++r)
    arow[r] = gp((const bf16x8*)M + (size_t)(r < nrt ? rt[r] : 0) * nk * 64 + l);
  const bf16x8* bcol = (const bf16x8*)(B + lr * ldb + 8 * lg);
  const int bstride = 16 * ldb / 8;  // in bf16x8 units
  constexpr int NB = PF + 1;  // register buffers of A fragments
  bf16x8 a[NB][RG];
#pragma unroll
  for (int u = 0; u < PF; ++u) {
    const int kl = u < nk ? u : nk - 1;
#pragma unroll
    for (int r = 0; r < RG; ++r) a[u][r] = arow[r][64 * kl];
  }
  auto step = [&](int kk, int u) {  // u = kk mod NB, a compile-time constant at every call
    const int kl = kk + PF < nk ? kk + PF : nk - 1;
#pragma unroll
    for (int r = 0; r < RG; ++r) a[(u + PF) % NB][r] = arow[r][64 * kl];
    bf16x8 b[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) b[c] = bcol[c * bstride + 4 * kk];
#pragma unroll
    for (int r = 0; r < RG; ++r)
#pragma unroll
      for (int c = 0; c < CT; ++c)
        acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u][r], b[c], acc[r][c], 0, 0, 0);
  };
  // whole groups of NB k-steps without branches between them, then the tail
  const int nmain = nk - nk % NB;
  int kk = 0;
  for (; kk < nmain; kk += NB) {
#pragma unroll
    for (int u = 0; u < NB; ++u) step(kk + u, u);
  }
#pragma unroll
  for (int u = 0; u < NB - 1; ++u)
    if (kk + u < nk) step(kk + u, u);
}

// FP32: the contraction over the nks k-steps of 16 from k-step ks0 (all of them by default), B
// holding those rows from its row 0.
template <int RG, int CT, int PF = 3>
__device__ __forceinline__ void gemm_f32(const float* __restrict__ M, int n_pad, const float* B,
                                                int ldb, const int* rt, int nrt, f32x4 (&acc)[RG][CT],
                                                int ks0 = 0, int nks = -1) {
  // as gemm_bf16: PF k-steps of A fragments in flight, every k-step issuing its prefetch
  const int l = threadIdx.x & 63;
  const int lr = l & 15, lg = l >> 4;
  // M is stored in fragment order (mf_index): row tile rt, k-step ks at (rt nks_all + ks) 64 + l
  const int nks_all = n_pad >> 4;
  if (nks < 0) nks = nks_all;
  const HOPF_GLOBAL f32x4* arow[RG];
#pragma unroll
  for (int r = 0; r < RG; ++r)
    arow[r] = gp((const f32x4*)M + ((size_t)(r < nrt ? rt[r] : 0) * nks_all + ks0) * 64 + l);
  const float* bcol = B + lr * ldb + 4 * lg;
  constexpr int NB = PF + 1;
  f32x4 a[NB][RG];
#pragma unroll
  for (int u = 0; u < PF; ++u) {
    const int kl = u < nks ? u : nks - 1;
#pragma unroll
    for (int r = 0; r < RG; ++r) a[u][r] = arow[r][64 * kl];
  }
  auto step = [&](int ks, int u) {  // u = ks mod NB, a compile-time constant at every call
    const int kl = ks + PF < nks ? ks + PF : nks - 1;
#pragma unroll
    for (int r = 0; r < RG; ++r) a[(u + PF) % NB][r] = arow[r][64 * kl];
    f32x4 b[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) b[c] = *(const f32x4*)(bcol + 16 * c * ldb + 16 * ks);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < RG; ++r)
#pragma unroll
        for (int c = 0; c < CT; ++c)
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][r][q], b[c][q], acc[r][c], 0, 0, 0);
  };
  const int nmain = nks - nks % NB;
  int ks = 0;
  for (; ks < nmain; ks += NB) {
#pragma unroll
    for (int u = 0; u < NB; ++u) step(ks + u, u);
  }
#pragma unroll
  for (int u = 0; u < NB - 1; ++u)
    if (ks + u < nks) step(ks + u, u);
}

// Rows (k) of the anchor right-hand sides per LDS block of the sliced products, and the block's
// byte stride per (slice, column): the refined kernel's dynamic LDS holds kSlices PT (kbq + 16)
// bytes.
constexpr int kAnchorKB = 256;
__host__ __device__ __forceinline__ int anchor_kbq(int n_pad) {
  return pad64(n_pad) < kAnchorKB ? pad64(n_pad) : kAnchorKB;
}

// Exact anchor products in integer slices: acc[s][c] += sum over the slice pairs a + b = s (0-based)
// of Mq_a[16 rt .., k] * Bq_b[k, 16 c ..] over the nkb k-steps of 64 from k-step ks0, int8 MFMAs
// with int32 accumulation (no rounding: |acc| <= kSlices n64 64^2).  Mq in its operand order (the
// kSlices definitions); Bq the LDS block, slice b of column j at Bq + (b PT + j) ldq, k contiguous.
// A streams PF k-steps ahead; lane l takes k = 16 (l / 16) .. + 15 of a k-step in both operands.
template <int CT, int PF = 1>
__device__ __forceinline__ void gemm_slices(const int8_t* __restrict__ Mq, int RT, int nks, int rt, int ks0,
                                            int nkb, const int8_t* Bq, int ldq, i32x4 (&acc)[kSlices][CT]) {
  constexpr int PT = 16 * CT;
  const int l = threadIdx.x & 63;
  const int lr = l & 15, lg = l >> 4;
  const HOPF_GLOBAL i32x4* abase = gp((const i32x4*)Mq + ((size_t)rt * nks + ks0) * 64 + l);
  const size_t astride = (size_t)RT * nks * 64;  // units between slices
  const int8_t* bbase = Bq + lr * ldq + 16 * lg;
  constexpr int NB = PF + 1;
  i32x4 a[NB][kSlices];
  // every k-step issues its prefetch (past the end it re-reads the last k-step), so the loads in
  // flight are the same on every path (as in gemm_bf16)
#pragma unroll
  for (int u = 0; u < PF; ++u) {
    const int kl = u < nkb ? u : nkb - 1;
#pragma unroll
    for (int s = 0; s < kSlices; ++s) a[u][s] = abase[s * astride + 64 * kl];
  }
  auto step = [&](int kk, int u) {
    const int kl = kk + PF < nkb ? kk + PF : nkb - 1;
#pragma unroll
    for (int s = 0; s < kSlices; ++s) a[(u + PF) % NB][s] = abase[s * astride + 64 * kl];
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      i32x4 b[kSlices];
#pragma unroll
      for (int s = 0; s < kSlices; ++s) b[s] = *(const i32x4*)(bbase + (s * PT + 16 * c) * ldq + 64 * kk);
#pragma unroll
      for (int sa = 0; sa < kSlices; ++sa)
#pragma unroll
        for (int sb = 0; sa + sb < kSlices; ++sb)
          acc[sa + sb][c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[u][sa], b[sb], acc[sa + sb][c], 0, 0, 0);
    }
  };
  const int nmain = nkb - nkb % NB;
  int kk = 0;
  for (; kk < nmain; kk += NB) {
#pragma unroll
    for (int u = 0; u < NB; ++u) step(kk + u, u);
  }
#pragma unroll
  for (int u = 0; u < NB - 1; ++u)
    if (kk + u < nkb) step(kk + u, u);
}

// p of a value iteration written straight to the output row g (rows row0 .. row0 + 3 below n):
// a later value iteration of the same column, if the stopping test fails there, overwrites it.
__device__ __forceinline__ void store_grad(float* g, int row0, int n, f32x4 pv) {
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (row0 + q < n) st_nt(g + row0 + q, pv[q]);
}

// Value sums of a value iteration (rare: one iteration per solve).  Called by the four lanes
// l, l ^ 16, l ^ 32, l ^ 48 that hold rows of one column, all active together: their partials are
// summed in a fixed order by shuffles and the first lane group adds the result to the wave's own
// slot of the column (plain adds in the wave's program order).  No atomics: the sums, and phi,
// are the same bits on every run.
__device__ __forceinline__ void value_sums(double* slot, double v2, double v3, double v4, double v5, int l) {
  double v[4] = {v2, v3, v4, v5};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    v[q] += __shfl_xor(v[q], 16);
    v[q] += __shfl_xor(v[q], 32);
  }
  if ((l >> 4) == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) slot[q] += v[q];
  }
}

// The next chunk for a workgroup (or a wave) that schedules itself: the shared counter, or with
// det a fixed schedule in which unit u of `units` takes the chunks u, u + units, u + 2 units, ...
// (`taken` counts its chunks).  A column's passes, anchors and refills then depend only on the
// data, so every output is the same bits on every run of the same launch.
__device__ __forceinline__ int next_chunk(int* counter, int det, int unit, int units, int& taken) {
  return det ? unit + units * (taken++) : atomicAdd(counter, 1);
}

// Wave-level sum of a double across the 64 lanes (result in every lane).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Per-column (slot) scalars and the workgroup's control words, in LDS (P columns).
template <int P, int NW>
struct ColShared {
  double t[P], th1[P], th2[P], gam[P], gama[P], dgam[P];
  double ssa2[P], ssq[P], prev[P], s[P], phi[P], hp[P];
  double pn[P], best[P];
  int stall[P], col[P], j[P], k[P], state[P], phase[P], iters[P];
  int newton[P], flags[P], fresh[P], better[P];
  int rexp[P];            // column exponents of an anchor's right-hand sides
  double red[NW][P][2];  // per-wave partials of step^2 and |s|^2
  double redv[NW][P][4];  // per-wave value sums of a value iteration
  int ctl[16];
};
// Column c's value sum q over the waves, in wave order.
template <int P, int NW>
__device__ __forceinline__ double value_total(const ColShared<P, NW>& S, int c, int q) {
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) s += S.redv[w][c][q];
  return s;
}
// Clears every wave's value sums (all threads of the workgroup take part).
template <int P, int NW>
__device__ __forceinline__ void value_clear(ColShared<P, NW>& S, int tid) {
  for (int i = tid; i < NW * P * 4; i += NW * 64) (&S.redv[0][0][0])[i] = 0.0;
}
// FLAG_SOLVE_CAP: the current solve hit the iteration cap (or stalled at FP32 precision);
// FLAG_CAPPED: some solve of this slot did (reported as -2); FLAG_EXACT: the column has had an
// exact anchor product (refined wave-local kernel: only then may it stop).
// FLAG_CIN (tile kernel, sqrt(<p, D p>)): the current z lies inside the Wulff ellipsoid (d = 0);
// FLAG_INSIDE there: the anchor's za does (d^a = 0).
enum {
  FLAG_FIRST = 1, FLAG_CAPPED = 2, FLAG_INSIDE = 4, FLAG_NEWTON_CAP = 8, FLAG_SOLVE_CAP = 16, FLAG_EXACT = 32,
  FLAG_CIN = 64
};
// FP32 mode: the split-Bregman step norm is nonincreasing in exact arithmetic (the iteration
// map is firmly nonexpansive), so a step that has not reached a new minimum for this many
// iterations is rounding noise: the iterate has stalled at the working precision.
constexpr int kStallIters = 64;
enum {
  CTL_ANCHOR = 0, CTL_LAST_ANCHOR, CTL_PROB, CTL_NEXTCOL, CTL_CHUNKEND, CTL_PENDING, CTL_NOMORE,
  CTL_EXIT, CTL_BETTER, CTL_ANY, CTL_PHIPASS, CTL_WL2, CTL_TAKEN
};
enum { PH_WARMUP = 0, PH_DELTA = 1 };


}  // namespace hopf
