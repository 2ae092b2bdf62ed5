// Shared device/host definitions of the HIP library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hopf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;

// Global-memory views of generic pointers.  Pointers read out of structures in memory are
// generic ("flat") to the compiler; flat loads count against both the memory and the LDS
// wait counters, which serialises loads with LDS traffic.  Casting them to the global address
// space gives global loads, which the compiler can keep in flight.
#define HOPF_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const HOPF_GLOBAL T* gp(const T* p) { return (const HOPF_GLOBAL T*)p; }
template <typename T>
__device__ __forceinline__ HOPF_GLOBAL T* gp(T* p) { return (HOPF_GLOBAL T*)p; }
constexpr int kBlock = 256;  // 4 waves per workgroup in every kernel of the library

// Round-to-nearest-even FP32 -> BF16 (NaN stays NaN).
__device__ __forceinline__ __bf16 to_bf16(float f) { return (__bf16)f; }

// Per-column states of the dense solver.
enum ColState : int {
  COL_EMPTY = 0,    // padding column
  COL_ACTIVE = 1,   // iterating
  COL_WAITING = 2,  // converged (or capped): frozen, waits for an exact product before its value
  COL_PHI = 3,      // this iteration evaluates phi from the exact product identity
  COL_DONE = 4,     // value and gradient staged
  COL_INVALID = 5   // non-finite input or t <= 0
};

// Operand layouts of the rounded copies of M (n_pad x n_pad, rows padded with zeros): stored in
// the order the MFMA A fragments are read, so that a wave's fragment load is contiguous.
//  BF16 (16x16x32 products): fragment (row tile rt, k-step kk of 32): lane l = r + 16 g holds
//    M[16 rt + r][32 kk + 8 g .. + 7]; fragments in (rt, kk) order, 64 lanes x 8 values each.
//  FP32 (16x16x4 products, 16 columns per step): fragment (rt, ks of 16): lane l = r + 16 g holds
//    M[16 rt + r][16 ks + 4 g .. + 3].
__host__ __device__ inline size_t mb_index(int i, int j, int n_pad) {
  const int nk = n_pad >> 5;
  return (((size_t)(i >> 4) * nk + (j >> 5)) * 64 + (i & 15) + 16 * ((j >> 3) & 3)) * 8 + (j & 7);
}
__host__ __device__ inline size_t mf_index(int i, int j, int n_pad) {
  const int nks = n_pad >> 4;
  return (((size_t)(i >> 4) * nks + (j >> 4)) * 64 + (i & 15) + 16 * ((j >> 2) & 3)) * 4 + (j & 3);
}

// Hamiltonian kinds (same numbering as the public header).
// HK_WL2: sqrt(<p, diag(w) p>); HK_LINCTRL: the time-dependent H of linear controls (diagonal drift)
enum { HK_WL1 = 0, HK_L2 = 1, HK_L2_WL1 = 2, HK_WL2 = 3, HK_AL2 = 4, HK_LINF = 5, HK_LINCTRL = 6 };
// initial data: quadratic 1/2 y^T A^{-1} y, 1/2 |y|_1^2 (J* = 1/2 |p|_inf^2), 1/2 |y|_inf^2 (J* = 1/2 |p|_1^2)
enum { JK_QUAD = 0, JK_L1SQ = 1, JK_LINFSQ = 2 };
__host__ __device__ inline bool hk_has_l1(int hk) { return hk == HK_WL1 || hk == HK_L2_WL1; }
__host__ __device__ inline bool hk_has_l2(int hk) { return hk == HK_L2 || hk == HK_L2_WL1; }

// Exact products of the refined solver's anchors: M and the anchor right-hand sides are split into
// kSlices signed 7-bit integer slices under a power-of-two scale per row (per column), x =
// 2^e sum_a m_a 2^{-7a} with |m_a| <= 64, and the slice products run as int8 MFMAs with exact int32
// accumulation.  slice_exponent(max |x|) is the e of a row or column: max |x| < 2^(e - 1), so the
// scaled values lie in (-1/2, 1/2) and every rounded slice fits in [-64, 64].
constexpr int kSlices = 6;
__host__ __device__ inline int slice_exponent(double maxabs) {
  if (!(maxabs > 0.0)) return 0;
  int e = 0;
  (void)frexp(maxabs, &e);  // maxabs = f 2^e, f in [0.5, 1)
  return e + 1;
}
// Units of 16 bytes of the sliced M in the int8 MFMA operand order: slice a, row tile rt, k-step
// ks of 64 at ((a RT + rt) nks + ks) 64 + lane, lane = row % 16 + 16 ((k % 64) / 16), holding
// k % 16 = 0 .. 15 (RT = n_pad / 16, nks = n64 / 64, n64 = n_pad rounded up to 64).
__host__ __device__ inline int pad64(int n_pad) { return (n_pad + 63) & ~63; }

// Device-side view of one problem for the dense solver (one entry per problem of a launch).
struct DenseProb {
  int n, n_pad, K, level_set, hkind, max_iter;
  double lambda, tol;
  const __bf16* Mb;      // n_pad*n_pad BF16 copy of M = (A + lambda I)^{-1}
  const float* Mf;       // n_pad*n_pad FP32 copy
  const double* Md;      // n_pad*n_pad FP64
  const int8_t* Mq;      // kSlices * n_pad * pad64(n_pad) bytes: M in integer slices (refined mode)
  const int32_t* Mqe;    // n_pad row exponents of the slices
  const double* w;       // n_pad weights (0 beyond n)
  const float* wf;       // the same weights in FP32 (thresholds of the per-iteration increments)
  const double* centres; // K*n_pad (0 beyond n), or null
  // per-call arrays (already offset to this problem's first point)
  const float* x;        // npts*n
  const float* t;        // npts (eval) ; unused for distance
  int64_t npts;
  float* phi; float* grad; float* dphidt; int32_t* iters; int32_t* kstar;
  float* dist; int32_t* inside; int32_t* newton;
  double s_tol;
  int max_newton;
  // per-point best value over the K copies found so far (workspace, reset before every call)
  double* bestv; int32_t* bestk;
  // passes (products with M) summed over every column (every copy, every Newton solve) of the
  // problem's calls, or null
  unsigned long long* iter_total;
};

// A run of columns (col = point * K + k) of one problem; always whole points.
struct DenseChunk {
  int prob;
  int col0;
  int ncols;
  int pad;
};

}  // namespace hopf
