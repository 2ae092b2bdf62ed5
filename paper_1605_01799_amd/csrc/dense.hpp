#pragma once
#include "common.hpp"

namespace hopf {

// mode 0: FP32 products; mode 1: BF16 increments refined by FP64 anchor products.
int dense_cols_per_tile(int mode, int n_pad);
size_t dense_lds_bytes(int mode, int n_pad);
hipError_t launch_dense(int mode, int cols_per_tile, const DenseProb* d_probs, const DenseTile* d_tiles,
                        int ntiles, float* ws, int64_t ws_per_wg, int grid, size_t lds, int distance,
                        int warmup, int anchor_every, hipStream_t stream);

}  // namespace hopf
