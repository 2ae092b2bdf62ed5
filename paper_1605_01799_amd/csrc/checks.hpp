// Host-side argument checks of the C ABI.  Plain C++ (no HIP): the library calls them before
// any device work, and the CPU test suite builds this file on its own, under the address and
// undefined-behaviour sanitizers, and drives it with valid and invalid arguments.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "../../include/hopf.h"

namespace hopf {

constexpr int kMaxN = 2048;     // largest dimension
constexpr int kMaxK = 64;       // largest number of translated copies / ellipsoids
constexpr int kDiagMaxN = 32;   // per-thread path: a point's state in one thread's registers
constexpr int kRotMaxN = kMaxN;  // sqrt(<p, HA p>): HA's eigenbasis (FP64 Jacobi on the device)
constexpr int kSmallMaxN = 64;  // wave-local kernel: a point's state in one wave
// Columns of one call are (point, copy) pairs numbered point * K + copy in 32-bit integers on the
// device, so npts * K must stay below 2^31.
constexpr int64_t kMaxColumns = ((int64_t)1 << 31) - 1;

// Each check returns HOPF_OK, or a status with a message written to why (NUL-terminated, at most
// len bytes; why may be NULL).

// The problem descriptor: sizes, finiteness, symmetry, and the (H, J, precision, n) combinations
// that have a GPU path; diagonal A must be positive (HOPF_ENOTSPD otherwise).
hopf_status check_desc(const hopf_problem_desc* d, char* why, size_t len);

// A call's point count with K copies each: 0 <= npts and npts * K <= kMaxColumns.
hopf_status check_columns(int64_t npts, int32_t K, char* why, size_t len);

// A member of a ragged batch (hopf_eval_ragged runs the dense kernels only): one shared precision
// other than HOPF_F64, the quadratic J and no HOPF_H_LINF.
hopf_status check_ragged_member(int32_t q, int32_t precision, int32_t batch_precision, int32_t hkind, int32_t jkind,
                                int32_t n, char* why, size_t len);

}  // namespace hopf
