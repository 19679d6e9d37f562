// Launchers of the fast multipole product's point kernels, shared by the
// translation driver (fmm.hip) and the files that hold the kernels.
#pragma once

#include "common.h"
#include "fmm.h"
#include "tree.h"

namespace bfm {

// Harmonic recurrence tables (constant memory of the leaf kernels), once per device.
void leaf_tables_upload(int device);

// M[leaf box][c][p^2] = multipole expansion of every leaf (M must be zero).
template <int P_, int NCH, bool MONO, bool DIP>
void launch_p2m(const Tree &t, const Sources &src, double *M, hipStream_t st);

// y[c][i] += local expansion of point i's leaf evaluated at the point.
template <int P_, int NCH>
void launch_l2p(const Tree &t, const double *L, double *y, hipStream_t st);

// y[c][i] = near-field sum of receiver i (leaf and neighbour leaves).
template <int NCH, bool MONO, bool DIP>
void launch_p2p(const Tree &t, const Sources &src, double *y, hipStream_t st);

// y[c][i] = near-field sum of the five packed channels (Sources::packed).
void launch_p2p_packed(const Tree &t, const double *packed, double *y, hipStream_t st);

// y[c][i] = sum over every other point (all pairs).
template <int NCH, bool MONO, bool DIP>
void launch_direct(const Tree &t, const Sources &src, double *y, hipStream_t st);

}  // namespace bfm
