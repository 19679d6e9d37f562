// Launchers of the fast multipole product's point kernels, shared by the
// translation driver (fmm.hip) and the files that hold the kernels.
#pragma once

#include "common.h"
#include "fmm.h"
#include "tree.h"

namespace bfm {

// Harmonic recurrence tables (constant memory of the leaf kernels), once per device.
void leaf_tables_upload(int device);

// M[leaf box][c][p^2] = multipole expansion of every leaf (M must be zero),
// computed and stored in R (double, or float for low-precision products).
template <int P_, int NCH, bool MONO, bool DIP, class R = double>
void launch_p2m(const Tree &t, const Sources &src, R *M, hipStream_t st);

// y[c][i] += local expansion of point i's leaf evaluated at the point
// (expansion and arithmetic in R; y stays FP64).
template <int P_, int NCH, class R = double>
void launch_l2p(const Tree &t, const R *L, double *y, hipStream_t st);

// y[c][i] = near-field sum of receiver i (leaf and neighbour leaves).
template <int NCH, bool MONO, bool DIP>
void launch_p2p(const Tree &t, const Sources &src, double *y, hipStream_t st);

// y[i] = near-field sum of one channel in FP32 arithmetic (coordinates
// relative to the receiver's leaf centre), accumulated into FP64.
template <bool MONO, bool DIP>
void launch_p2p32(const Tree &t, const Sources &src, double *y, hipStream_t st);

// y[c][i] = near-field sum of the five packed channels (Sources::packed).
void launch_p2p_packed(const Tree &t, const double *packed, double *y, hipStream_t st);

// Rotation-factored M2L (fmm_rot.hip): operators of order p uploaded to w
// (no-op if current); the translation of operators op0 .. op0 + nops - 1 at
// order PO of expansions stored at order PS, tiles g0 .. g0 + ntiles - 1 of
// the 16-column tile prefix tile_off, added into out.
void rot_ops_upload(FmmWork &w, int p, hipStream_t st);
template <int PO, int PS>
void launch_m2l_rot(const FmmWork &w, int op0, int nops, int g0, int ntiles, const int *tile_off,
                    const TaskList &tl, int nch, const double *in, double *out, hipStream_t st);

// y[c][i] = sum over every other point (all pairs).
template <int NCH, bool MONO, bool DIP>
void launch_direct(const Tree &t, const Sources &src, double *y, hipStream_t st);

}  // namespace bfm
