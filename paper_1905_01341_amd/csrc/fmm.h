// Fast multipole product for the BEM operators (Section 3.9, eq3_27):
// out_i = sum_{j != i} [ q_j / |r_i - r_j| + w_j n_j . (r_i - r_j) / |r_i - r_j|^3 ] / (4 pi)
// for nch independent channels of monopole strengths q and dipole weights w
// over the same points. Every dipole of the method points along the vertex
// normal n_j (ns1), so a channel carries only the scalar weight w. Point
// data are in the tree's sorted order.
#pragma once

#include "common.h"
#include "prof.h"
#include "tree.h"

namespace bfm {

constexpr int kDiagRec = 16;  // doubles per packed five-channel source record

struct Sources {
    int nch = 1;
    bool mono = true, dip = false;
    const double *q = nullptr;  // [nch][n] monopole strengths
    const double *w = nullptr;  // [nch][n] dipole weights (moment w_j n_j)
    // optional, five channels only: the same sources packed per point for the
    // near field, kDiagRec doubles each: x, y, z, n_x, n_y, n_z, q1, q2, q3,
    // w0, w1, w2, w3, w4 (channels 0 and 4 carry no monopole)
    const double *packed = nullptr;
};

struct FmmWork {
    int p = 0;
    // arithmetic of this group's products: BFM_PREC_FP64 (the GMRES products
    // and the diagonal pass), or BFM_PREC_FP32 / BFM_PREC_BF16X3 (the
    // low-precision products of iterative refinement, one channel)
    int prec = BFM_PREC_FP64;
    int nch_cap = 0;
    int64_t nbox_cap = 0;
    DevBuf<double> mexp, lexp;      // [nbox][nch][P]
    DevBuf<double> ops_m2m, ops_l2l, ops_m2l;  // operators, column-major per op: [op][k][row]
    DevBuf<float> mexp32, lexp32;   // low-precision expansions [nbox][P]
    DevBuf<float> part32;           // low-precision M2L results per task [ntasks][P]
    DevBuf<float> opf_m2m, opf_l2l, opf_m2l;   // FP32 operators, same layout
    // split-BF16 operators: [0] = hi, [1] = lo, [op][chunk][row][32] (K padded to 32)
    DevBuf<uint16_t> opb_m2m[2], opb_l2l[2], opb_m2l[2];
    int ops_p = 0;
    int ops_prec = -1;
    // rotation-factored M2L operators (FP64, kernel operand order, fmm_rot.hip):
    // per operator the degree blocks of A, the order blocks of T_z, those of B
    DevBuf<double> rot_a, rot_z, rot_b;
    int rot_p = 0;
    int m2l_shape = -1;    // M2L launch shape (-1: chosen by size; 3: rotation-factored, FP64)
    int m2l_orders = 0;    // 1: distant offset classes translated at reduced orders (ops.h)
    int m2l_shape_used = -1;  // shape of the last M2L launch (-1: none yet)
    // optional second stream for the near field (default priority): the
    // P2P runs there beside the far-field chain and the L2P waits for it
    hipStream_t near = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    Prof *prof = nullptr;  // optional kernel timing
    int prof_base = 0;     // class of this product group's P2P (KC_P2P .. KC_L2P follow)
};

// Build translation operators for p (host build + upload); no-op if current.
void fmm_prepare_ops(FmmWork &w, int p, hipStream_t st);

// y[c][i] (sorted order) = raw sums without the 1/(4 pi) factor.
// direct = true: all-pairs sum (no tree approximation).
void fmm_apply(FmmWork &w, const Tree &t, const Sources &src, double *y, bool direct,
               hipStream_t st);

}  // namespace bfm
