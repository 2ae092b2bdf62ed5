#pragma once
#include "common.hpp"

namespace hopf {

// mode 0: FP32 products; mode 1: BF16 increments refined by exact (integer-sliced) anchor products;
// mode 2: FP32 increments on such anchors.  The launch shape for a mode and padded size: columns
// per tile, workgroups per CU, waves per workgroup, and ks = 2 where the FP32 right-hand sides of
// the tile do not fit LDS whole (mode 2): the contraction then runs over one half of the rows at a
// time, the first half's partial products going through the staging.
// wl: the launch holds sqrt(<p, D p>) problems (their prox runs the multiplier phase; the other
// kinds are compiled without it).
struct DenseVariant {
  int pt, occ, nw, ks;
  int wl = 0;
};
DenseVariant dense_variant(int mode, int n_pad);
size_t dense_lds_bytes(int mode, int n_pad);
// Resets the chunk counter and the per-point best arrays before a launch.
hipError_t launch_reset(int* counter, double* bestv, int32_t* bestk, int64_t npts, hipStream_t stream);
hipError_t launch_dense(int mode, DenseVariant var, const DenseProb* d_probs, const DenseChunk* d_chunks,
                        int nchunks, int* counter, float* ws, double* ws64, int64_t ws_per_wg, int64_t ws64_per_wg,
                        int grid, size_t lds, int distance, int anchor_every, int anchor_wait, int det,
                        hipStream_t stream);

// Small problems (dense_small.hip): FP32 evaluation of n_pad <= 64, one wave per 16-column tile
// with the iteration in registers; refined: FP32 increments on exact FP64 anchor products.
bool dense_small_fits(int mode, int n_pad, int distance);
int dense_small_cols();       // columns per wave
int dense_small_occupancy();  // workgroups per CU
// kind: dense_small_kind(hkind) of every problem of the launch (one instance per kind of H)
int dense_small_kind(int hkind);
hipError_t launch_dense_small(int n_pad, bool refined, int kind, const DenseProb* d_probs, const DenseChunk* d_chunks,
                              int nchunks, int* counter, int grid, int anchor_every, int anchor_wait, int det,
                              hipStream_t stream);

// Refined BF16 problems of one point per column (K = 1) with 64 <= n_pad <= 1024
// (dense_rs.hip): the column state on chip, one persistent workgroup of 32 columns per CU.
bool dense_rs_fits(int mode, int n_pad, int K, int hkind, int distance);
int dense_rs_cols();                     // columns per workgroup
size_t dense_rs_lds_bytes(int n_pad);     // dynamic LDS of a launch whose largest problem has n_pad
int64_t dense_rs_ws_floats(int n_pad);    // float staging per workgroup
hipError_t launch_dense_rs(int max_npad, const DenseProb* d_probs, const DenseChunk* d_chunks, int nchunks,
                           int* counter, double* ws64, int64_t ws64_per_wg, float* ws, int64_t ws_per_wg, int grid,
                           size_t lds, int anchor_every, int anchor_wait, int det, hipStream_t stream);

}  // namespace hopf
