// XCD-aware block order for the gather kernels of libbfm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bfm {

// XCD-aware block order: workgroups are dealt round-robin to the 8 XCDs of
// an MI355X, so block b runs on XCD b % 8. Logical block xcd * per + idx
// gives each XCD a contiguous run of logical blocks, whose neighbouring data
// (shared vertices, triangles, rows) then stays in that XCD's L2.
__device__ inline int64_t xcd_block() {
    const int nblock = gridDim.x, per = nblock / 8, rem = nblock % 8;
    const int xcd = blockIdx.x % 8, idx = blockIdx.x / 8;
    return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

}  // namespace bfm
