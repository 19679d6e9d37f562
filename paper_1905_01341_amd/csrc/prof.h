// Optional kernel timing: HIP events recorded on the launching stream around
// every launch of an instrumented kernel class, with the algorithmic work of
// each launch (flops or pair interactions) accumulated beside it.
#pragma once

#include <vector>

#include "common.h"

namespace bfm {

// Kernel classes. The five kernels of a fast multipole product (P2P .. L2P)
// are counted per product group: the FP64 products of GMRES at classes 0..4,
// the diagonal/right-hand-side pass at kDiagBase + 0..4 and the
// low-precision products of iterative refinement at kLoBase + 0..4.
enum KernelClass { KC_P2P = 0, KC_M2L, KC_M2M_L2L, KC_P2M, KC_L2P, KC_GMRES, KC_TREE, KC_DIAG };
constexpr int kDiagBase = 8;
constexpr int kLoBase = 13;
constexpr int kClassCount = 18;

struct Prof {
    bool on = false;
    struct Rec {
        int cls;
        hipEvent_t a, b;
        double flops;
        double bytes;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    size_t used = 0;

    hipEvent_t take() {
        if (used == pool.size()) {
            hipEvent_t e;
            BFM_HIP(hipEventCreate(&e));
            pool.push_back(e);
        }
        return pool[used++];
    }
    // begin(): returns index of the record (or -1 when off)
    int begin(int cls, hipStream_t st) {
        if (!on) return -1;
        Rec r{cls, take(), take(), 0.0, 0.0};
        BFM_HIP(hipEventRecord(r.a, st));
        recs.push_back(r);
        return (int)recs.size() - 1;
    }
    void end(int idx, hipStream_t st, double flops, double bytes) {
        if (idx < 0) return;
        BFM_HIP(hipEventRecord(recs[idx].b, st));
        recs[idx].flops = flops;
        recs[idx].bytes = bytes;
    }
    void reset() {
        recs.clear();
        used = 0;
    }
    ~Prof() {
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

}  // namespace bfm
