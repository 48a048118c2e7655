// Host construction of the per-kind block-Jacobi preconditioner of the final system.
#pragma once

#include <cstdint>
#include <vector>

#include "setup.hpp"

namespace aimm {

// G_self: the AIM operator on one element's own RWG functions (grid part on every
// pair plus the pre-corrected near field of lattice offset (0, 0)), column-major
// N x N (entry (row a, column b) at b * N + a).
void self_block(const Setup& st, const ArrayIn& a, std::vector<cd>& G);

// P = (D - G_self M)^-1 in FP64, column-major.  M: column-major N x N; D as
// coordinate lists.  Throws std::runtime_error if the block is singular.
void block_inverse(const std::vector<cd>& Gself, const cd* M, const int32_t* drow, const int32_t* dcol,
                   const cd* dval, int64_t dnnz, int N, std::vector<cd>& P);

}  // namespace aimm
