// Direct all-pairs product on device arrays (no handle): see direct.hip.
#pragma once

#include "common.h"

namespace bfm {

struct DirectArgs {
    int64_t n = 0;                 // points (sources and candidate receivers)
    const double *xyz = nullptr;   // [n][3]
    const double *s = nullptr;     // [n] vertex weights
    const double *nrm = nullptr;   // [n][3] unit normals (needed when g != 0)
    double f = 0.0, g = 0.0;
    const double *x = nullptr;     // [n] single-layer density (f != 0)
    const double *y = nullptr;     // [n] double-layer density (g != 0)
    int64_t nr = 0;                // receivers
    const int64_t *rows = nullptr;  // [nr] receiver indices, or null for 0..nr-1
    double *out = nullptr;         // [nr]
};

// Allocates its partial-sum buffer on the stream (stream-ordered).
void direct_product(const DirectArgs &a, hipStream_t st);

// Doubles in the allocation-free entry point's device scratch array.
constexpr int64_t kDirectScratch = (int64_t)1 << 22;

// The same product with the partial sums in that array: no allocation.
void direct_product_noalloc(const DirectArgs &a, hipStream_t st);

}  // namespace bfm
