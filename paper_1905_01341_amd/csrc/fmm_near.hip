// Near field of the fast multipole product (Section 3.9): direct sums of
// every leaf's receivers over the points of the leaf and its neighbours
// (P2P), and the all-pairs sum used as a check.
#include <cmath>

#include "fmm_kernels.h"

namespace bfm {

// ---------------------------------------------------------------------------
// Near field. 1/sqrt in FP64: the hardware estimate (relative error about
// 5e-8) refined by one Newton step with an FMA-formed residual.
__device__ inline double rsqrt_f64(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

// -2/sqrt(x): the same Newton step written as y (x y^2 - 3), one operation
// fewer; the factor -2 is taken out of the sums once at the end.
__device__ inline double rsqrt_m2_f64(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    return y * fma(x * y, y, -3.0);
}

constexpr int kP2PThreads = 64;
constexpr int kXcdCount = 8;  // accelerator complex dies of an MI355X

// Receivers xi..zi (R per lane) against sources [j0, j1): every lane reads
// the same source at the same time, so the loads are wave-uniform (scalar
// loads of read-only data) and no LDS staging is needed.
// SELF: the sources may include the receiver itself (r = 0, excluded);
// otherwise every pair is at a positive distance and needs no test.
template <int NCH, bool MONO, bool DIP, int R, bool SELF>
__device__ inline void p2p_pair(double sx, double sy, double sz, const double *sq, const double *sw,
                                double nx, double ny, double nz, const double *xi, const double *yi,
                                const double *zi, double (*acc)[NCH]) {
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const double dx = xi[k] - sx, dy = yi[k] - sy, dz = zi[k] - sz;
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double inv = (!SELF || r2 > 0.0) ? rsqrt_f64(r2) : 0.0;  // j == i excluded
        if (MONO) {
#pragma unroll
            for (int c = 0; c < NCH; ++c) acc[k][c] += sq[c] * inv;
        }
        if (DIP) {
            const double tt = (nx * dx + ny * dy + nz * dz) * (inv * inv * inv);
#pragma unroll
            for (int c = 0; c < NCH; ++c) acc[k][c] += sw[c] * tt;
        }
    }
}

// Receivers xi..zi (R per lane) against sources [j0, j1): every lane reads
// the same source at the same time, so the loads are wave-uniform (scalar
// loads of read-only data); sources are fetched in batches of B so one wait
// covers B sources.
template <int NCH, bool MONO, bool DIP, int R, bool SELF>
__device__ inline void p2p_range(int j0, int j1, const double *__restrict__ px,
                                 const double *__restrict__ py, const double *__restrict__ pz,
                                 const double *__restrict__ pnx, const double *__restrict__ pny,
                                 const double *__restrict__ pnz, int64_t n,
                                 const double *__restrict__ q, const double *__restrict__ w,
                                 const double *xi, const double *yi, const double *zi,
                                 double (*acc)[NCH]) {
    constexpr int B = (NCH == 1 && !DIP) ? 8 : (NCH == 1 ? 4 : 2);
    int j = j0;
    for (; j + B <= j1; j += B) {
        double bx[B], by[B], bz[B], bq[B][NCH], bw[B][NCH], bnx[B], bny[B], bnz[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            bx[u] = px[j + u];
            by[u] = py[j + u];
            bz[u] = pz[j + u];
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                bq[u][c] = MONO ? q[(int64_t)c * n + j + u] : 0.0;
                bw[u][c] = DIP ? w[(int64_t)c * n + j + u] : 0.0;
            }
            bnx[u] = DIP ? pnx[j + u] : 0.0;
            bny[u] = DIP ? pny[j + u] : 0.0;
            bnz[u] = DIP ? pnz[j + u] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < B; ++u)
            p2p_pair<NCH, MONO, DIP, R, SELF>(bx[u], by[u], bz[u], bq[u], bw[u], bnx[u], bny[u], bnz[u], xi, yi, zi,
                                        acc);
    }
    for (; j < j1; ++j) {
        double sq[NCH], sw[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            sq[c] = MONO ? q[(int64_t)c * n + j] : 0.0;
            sw[c] = DIP ? w[(int64_t)c * n + j] : 0.0;
        }
        p2p_pair<NCH, MONO, DIP, R, SELF>(px[j], py[j], pz[j], sq, sw, DIP ? pnx[j] : 0.0, DIP ? pny[j] : 0.0,
                                    DIP ? pnz[j] : 0.0, xi, yi, zi, acc);
    }
}

// Receivers rc + lane + 64 k (k < R) of the leaf whose points are [l0, r1)
// against sources s0..s1-1 of the leaf's source list (its near ranges in
// order). ATOMIC: several items share these receivers, so the sums are added
// into the (cleared) output; otherwise they are stored.
template <int NCH, bool MONO, bool DIP, int R, bool ATOMIC>
__device__ inline void p2p_pass(int rc, int l0, int r1, int s0, int s1, int nr, const int2 *__restrict__ rng,
                                const double *__restrict__ px, const double *__restrict__ py,
                                const double *__restrict__ pz, const double *__restrict__ pnx,
                                const double *__restrict__ pny, const double *__restrict__ pnz,
                                int64_t n, const double *__restrict__ q, const double *__restrict__ w,
                                double *__restrict__ y) {
    const int lane = threadIdx.x;
    double xi[R], yi[R], zi[R], acc[R][NCH];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = rc + lane + k * kP2PThreads;
        const bool ok = i < r1;
        // idle lanes sit far away: their sums are never stored
        xi[k] = ok ? px[i] : 1e100;
        yi[k] = ok ? py[i] : 0.0;
        zi[k] = ok ? pz[i] : 0.0;
#pragma unroll
        for (int c = 0; c < NCH; ++c) acc[k][c] = 0.0;
    }
    // walk the ranges, keeping the part that falls in [s0, s1); only the
    // leaf's own points [l0, r1) can coincide with a receiver, so that part
    // runs with the test and the rest without
    int cum = 0;
    for (int g = 0; g < nr && cum < s1; ++g) {
        const int2 r = rng[g];
        const int len = r.y - r.x;
        const int a = r.x + max(0, s0 - cum), b = r.x + min(len, s1 - cum);
        cum += len;
        if (a >= b) continue;
        if (a < r1 && l0 < b) {
            const int m0 = max(a, l0), m1 = min(b, r1);
            p2p_range<NCH, MONO, DIP, R, false>(a, m0, px, py, pz, pnx, pny, pnz, n, q, w, xi, yi, zi, acc);
            p2p_range<NCH, MONO, DIP, R, true>(m0, m1, px, py, pz, pnx, pny, pnz, n, q, w, xi, yi, zi, acc);
            p2p_range<NCH, MONO, DIP, R, false>(m1, b, px, py, pz, pnx, pny, pnz, n, q, w, xi, yi, zi, acc);
        } else {
            p2p_range<NCH, MONO, DIP, R, false>(a, b, px, py, pz, pnx, pny, pnz, n, q, w, xi, yi, zi, acc);
        }
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = rc + lane + k * kP2PThreads;
        if (i < r1)
            for (int c = 0; c < NCH; ++c) {
                if (ATOMIC)
                    unsafeAtomicAdd(y + (int64_t)c * n + i, acc[k][c]);
                else
                    y[(int64_t)c * n + i] = acc[k][c];
            }
    }
}

// One wave per near-field work item (a leaf chunk of up to kP2PChunk
// receivers, two per lane, and a piece of the leaf's source list). A leaf's
// sources are its merged near-field ranges (the points of up to 27
// neighbour leaves); lists longer than kP2PPiece are split into balanced
// pieces, so that no wave carries much more work than the average and there
// are more waves than slots, which lets the dispatcher balance the tail.
template <int NCH, bool MONO, bool DIP, bool ATOMIC>
__global__ void __launch_bounds__(kP2PThreads) k_p2p(const int4 *__restrict__ items,
                                                     const int *__restrict__ leaf_pt,
                                                     const int2 *__restrict__ near_rng,
                                                     const int *__restrict__ near_cnt,
                                                     const double *__restrict__ px,
                                                     const double *__restrict__ py,
                                                     const double *__restrict__ pz,
                                                     const double *__restrict__ pnx,
                                                     const double *__restrict__ pny,
                                                     const double *__restrict__ pnz, int64_t n,
                                                     const double *__restrict__ q,
                                                     const double *__restrict__ w, double *__restrict__ y) {
    constexpr int R = kP2PChunk / kP2PThreads;
    static_assert(kP2PChunk == R * kP2PThreads, "whole receivers per lane");
    // XCD-aware order: workgroups are dealt round-robin to the 8 XCDs, so XCD
    // x takes a contiguous run of items (neighbouring leaves, which share
    // their sources) and keeps those sources in its own L2
    const int nblock = gridDim.x, per = nblock / kXcdCount, rem = nblock % kXcdCount;
    const int xcd = blockIdx.x % kXcdCount, idx = blockIdx.x / kXcdCount;
    const int4 it = items[xcd * per + (xcd < rem ? xcd : rem) + idx];
    const int leaf = it.x;
    p2p_pass<NCH, MONO, DIP, R, ATOMIC>(it.y, leaf_pt[leaf], leaf_pt[leaf + 1], it.z, it.w, near_cnt[leaf],
                                        near_rng + 27 * (int64_t)leaf, px, py, pz, pnx, pny, pnz, n, q, w, y);
}

// Near field of the five-channel pass from packed source records (one
// 128-byte record per point, read at wave-uniform addresses: two scalar
// loads per source instead of one per array). Per pair:
//   t = n_j . (r_i - r_j) / r^3,  y_0 += w0 t,  y_c += q_c / r + w_c t (c = 1..3),
//   y_4 += w4 t.
template <int R, bool SELF>
__device__ inline void p2p_diag_range(int j0, int j1, const double *__restrict__ pk, const double *xi,
                                      const double *yi, const double *zi, double (*acc)[5]) {
    constexpr int B = 2;
    auto pair = [&](const double(&s)[14]) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const double dx = xi[k] - s[0], dy = yi[k] - s[1], dz = zi[k] - s[2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double inv = (!SELF || r2 > 0.0) ? rsqrt_f64(r2) : 0.0;  // j == i excluded
            const double t = (s[3] * dx + s[4] * dy + s[5] * dz) * (inv * inv * inv);
            acc[k][0] += s[9] * t;
            acc[k][1] += s[6] * inv + s[10] * t;
            acc[k][2] += s[7] * inv + s[11] * t;
            acc[k][3] += s[8] * inv + s[12] * t;
            acc[k][4] += s[13] * t;
        }
    };
    int j = j0;
    for (; j + B <= j1; j += B) {
        double rec[B][14];
#pragma unroll
        for (int u = 0; u < B; ++u)
#pragma unroll
            for (int e = 0; e < 14; ++e) rec[u][e] = pk[(int64_t)(j + u) * kDiagRec + e];
#pragma unroll
        for (int u = 0; u < B; ++u) pair(rec[u]);
    }
    for (; j < j1; ++j) {
        double rec[14];
#pragma unroll
        for (int e = 0; e < 14; ++e) rec[e] = pk[(int64_t)j * kDiagRec + e];
        pair(rec);
    }
}

// One item of the five-channel pass with R receivers per lane.
template <int R, bool ATOMIC>
__device__ inline void p2p_diag_item(int leaf, int rc, int s0, int s1, const int *__restrict__ leaf_pt,
                                     const int2 *__restrict__ near_rng, const int *__restrict__ near_cnt,
                                     const double *__restrict__ px, const double *__restrict__ py,
                                     const double *__restrict__ pz, const double *__restrict__ pk, int64_t n,
                                     double *__restrict__ y) {
    const int l0 = leaf_pt[leaf], r1 = leaf_pt[leaf + 1];
    const int nr = near_cnt[leaf];
    const int2 *rng = near_rng + 27 * (int64_t)leaf;
    const int lane = threadIdx.x;
    double xi[R], yi[R], zi[R], acc[R][5];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = rc + lane + k * kP2PThreads;
        const bool ok = i < r1;
        xi[k] = ok ? px[i] : 1e100;  // idle lanes sit far away; never stored
        yi[k] = ok ? py[i] : 0.0;
        zi[k] = ok ? pz[i] : 0.0;
#pragma unroll
        for (int c = 0; c < 5; ++c) acc[k][c] = 0.0;
    }
    int cum = 0;
    for (int g = 0; g < nr && cum < s1; ++g) {
        const int2 r = rng[g];
        const int len = r.y - r.x;
        const int a = r.x + max(0, s0 - cum), b = r.x + min(len, s1 - cum);
        cum += len;
        if (a >= b) continue;
        if (a < r1 && l0 < b) {
            const int m0 = max(a, l0), m1 = min(b, r1);
            p2p_diag_range<R, false>(a, m0, pk, xi, yi, zi, acc);
            p2p_diag_range<R, true>(m0, m1, pk, xi, yi, zi, acc);
            p2p_diag_range<R, false>(m1, b, pk, xi, yi, zi, acc);
        } else {
            p2p_diag_range<R, false>(a, b, pk, xi, yi, zi, acc);
        }
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = rc + lane + k * kP2PThreads;
        if (i < r1)
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                if (ATOMIC)
                    unsafeAtomicAdd(y + (int64_t)c * n + i, acc[k][c]);
                else
                    y[(int64_t)c * n + i] = acc[k][c];
            }
    }
}

// The five-channel counterpart of k_p2p (same items, pieces and order); a
// chunk of at most 64 receivers runs with one receiver per lane.
template <bool ATOMIC>
__global__ void __launch_bounds__(kP2PThreads) k_p2p_diag(const int4 *__restrict__ items,
                                                          const int *__restrict__ leaf_pt,
                                                          const int2 *__restrict__ near_rng,
                                                          const int *__restrict__ near_cnt,
                                                          const double *__restrict__ px,
                                                          const double *__restrict__ py,
                                                          const double *__restrict__ pz,
                                                          const double *__restrict__ pk, int64_t n,
                                                          double *__restrict__ y) {
    static_assert(kP2PChunk == 2 * kP2PThreads, "one or two receivers per lane");
    const int nblock = gridDim.x, per = nblock / kXcdCount, rem = nblock % kXcdCount;
    const int xcd = blockIdx.x % kXcdCount, idx = blockIdx.x / kXcdCount;
    const int4 it = items[xcd * per + (xcd < rem ? xcd : rem) + idx];
    const int leaf = it.x, rc = it.y;
    if (leaf_pt[leaf + 1] - rc <= kP2PThreads)
        p2p_diag_item<1, ATOMIC>(leaf, rc, it.z, it.w, leaf_pt, near_rng, near_cnt, px, py, pz, pk, n, y);
    else
        p2p_diag_item<2, ATOMIC>(leaf, rc, it.z, it.w, leaf_pt, near_rng, near_cnt, px, py, pz, pk, n, y);
}

// Symmetric near field of one channel of monopoles (the kernel 1/r is
// symmetric): every unordered pair of points is visited once and its two
// terms go to both points. Work item (leaf, r0, s0, s1): receivers [r0, r1)
// of the leaf (at most kSymChunk: one to four per lane, by the chunk's size)
// against positions s0..s1-1 of the leaf's near ranges clipped to start at
// r0. The first r1 - r0 positions are the chunk itself (pieces of the
// diagonal block, in blocks of 64 against the receiver groups: the groups
// below a block both ways, the block's own group one-sided with j == i
// excluded); the later ones (the leaf's later points and the neighbour leaves
// with higher Morton keys) are summed both ways. The lower-keyed neighbours reach these receivers from their own
// items, so each pair is summed once.
// Sources of a two-sided piece pass in blocks of 64 through LDS: at step t
// lane l takes source (l + t) mod 64, so the lanes hold 64 distinct sources
// at every step and each adds its terms for that source to the source's LDS
// slot; a block's slots then go to the output with one atomic add each.
// (The block is kept as two arrays of 16-byte (x, y) and (z, q) pairs: 64
// lanes reading consecutive 16-byte records touch every LDS bank once.)
template <int R>
__device__ inline void p2p_sym_block(const double2 *sxy, const double2 *szq, double *sacc, const double *xi,
                                     const double *yi, const double *zi, const double *qi, double (*acc)[1]) {
    const int lane = threadIdx.x;
#pragma unroll 2
    for (int t = 0; t < kP2PThreads; ++t) {
        const int s = (lane + t) & (kP2PThreads - 1);
        const double2 a = sxy[s], b = szq[s];
        double c = 0.0;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const double dx = xi[k] - a.x, dy = yi[k] - a.y, dz = zi[k] - b.x;
            const double inv = rsqrt_m2_f64(dx * dx + dy * dy + dz * dz);  // -2 / r
            acc[k][0] = fma(b.y, inv, acc[k][0]);
            c = fma(qi[k], inv, c);
        }
        atomicAdd(sacc + s, c);
    }
}

// A block of the chunk's own points as sources: source slot l is receiver
// l of group b. Group k < b is summed both ways (its pairs with group b are
// met only here), group b one-sided over every ordered pair but the
// diagonal (step 0, where each lane meets its own point), groups k > b not
// at all (their pairs with group b are met when block k is the source).
template <int R>
__device__ inline void p2p_diag_block(const double2 *sxy, const double2 *szq, double *sacc, const double *xi,
                                      const double *yi, const double *zi, const double *qi, double (*acc)[1],
                                      int b) {
    const int lane = threadIdx.x;
#pragma unroll 2
    for (int t = 0; t < kP2PThreads; ++t) {
        const int s = (lane + t) & (kP2PThreads - 1);
        const double2 a = sxy[s], w = szq[s];
        double c = 0.0;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (k > b || (k == b && t == 0)) continue;  // wave-uniform
            const double dx = xi[k] - a.x, dy = yi[k] - a.y, dz = zi[k] - w.x;
            const double inv = rsqrt_m2_f64(dx * dx + dy * dy + dz * dz);  // -2 / r
            acc[k][0] = fma(w.y, inv, acc[k][0]);
            if (k < b) c = fma(qi[k], inv, c);
        }
        if (b > 0) atomicAdd(sacc + s, c);
    }
}

// One item with R = ceil((r1 - r0) / 64) receivers per lane, so that a short
// chunk runs no all-idle receiver groups.
template <int R>
__device__ inline void p2p_sym_item(int leaf, int r0, int r1, int s0, int s1, const int2 *__restrict__ near_rng,
                                    const int *__restrict__ near_cnt, const double *__restrict__ px,
                                    const double *__restrict__ py, const double *__restrict__ pz, int64_t n,
                                    const double *__restrict__ q, double *__restrict__ y, double2 *sxy,
                                    double2 *szq, double *sacc) {
    const int lane = threadIdx.x;
    double xi[R], yi[R], zi[R], qi[R], acc[R][1];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = r0 + lane + k * kP2PThreads;
        const bool ok = i < r1;
        xi[k] = ok ? px[i] : 1e100;  // idle lanes sit far away with no weight; never stored
        yi[k] = ok ? py[i] : 0.0;
        zi[k] = ok ? pz[i] : 0.0;
        qi[k] = ok ? q[i] : 0.0;
        acc[k][0] = 0.0;
    }
    const double scale = -0.5;  // the sums hold -2 / r
    if (s1 <= r1 - r0) {
        // the chunk's own points, in blocks of 64 aligned with the receiver
        // groups (pieces of the own block start at multiples of 64)
        for (int base = s0; base < s1; base += kP2PThreads) {
            const int j = r0 + base + lane;
            const bool ok = base + lane < s1;
            sxy[lane] = ok ? make_double2(px[j], py[j]) : make_double2(-1e100, 0.0);
            szq[lane] = ok ? make_double2(pz[j], q[j]) : make_double2(0.0, 0.0);
            sacc[lane] = 0.0;
            __syncthreads();
            const int b = base / kP2PThreads;
            p2p_diag_block<R>(sxy, szq, sacc, xi, yi, zi, qi, acc, b);
            __syncthreads();
            if (ok && b > 0) unsafeAtomicAdd(y + j, -0.5 * sacc[lane]);
        }
    } else {
        const int2 *rng = near_rng + 27 * (int64_t)leaf;
        const int nr = near_cnt[leaf];
        for (int base = s0; base < s1; base += kP2PThreads) {
            // this lane's source: position base + lane of the clipped list
            const int p = base + lane;
            int j = -1, cum = 0;
            for (int g = 0; g < nr; ++g) {
                const int2 r = rng[g];
                const int a = max(r.x, r0), len = max(0, r.y - a);
                if (p >= cum && p < cum + len) j = a + (p - cum);
                cum += len;
            }
            const bool ok = p < s1 && j >= 0;
            // idle sources sit far away on the other side with no weight
            sxy[lane] = ok ? make_double2(px[j], py[j]) : make_double2(-1e100, 0.0);
            szq[lane] = ok ? make_double2(pz[j], q[j]) : make_double2(0.0, 0.0);
            sacc[lane] = 0.0;
            __syncthreads();
            p2p_sym_block<R>(sxy, szq, sacc, xi, yi, zi, qi, acc);
            __syncthreads();
            if (ok) unsafeAtomicAdd(y + j, -0.5 * sacc[lane]);
        }
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = r0 + lane + k * kP2PThreads;
        if (i < r1) unsafeAtomicAdd(y + i, scale * acc[k][0]);
    }
}

__global__ void __launch_bounds__(kP2PThreads) k_p2p_sym(const int4 *__restrict__ items,
                                                         const int *__restrict__ leaf_pt,
                                                         const int2 *__restrict__ near_rng,
                                                         const int *__restrict__ near_cnt,
                                                         const double *__restrict__ px,
                                                         const double *__restrict__ py,
                                                         const double *__restrict__ pz, int64_t n,
                                                         const double *__restrict__ q, int chunk,
                                                         double *__restrict__ y) {
    static_assert(kSymChunk == 4 * kP2PThreads, "at most four receivers per lane");
    __shared__ double2 sxy[kP2PThreads], szq[kP2PThreads];
    __shared__ double sacc[kP2PThreads];
    const int nblock = gridDim.x, per = nblock / kXcdCount, rem = nblock % kXcdCount;
    const int xcd = blockIdx.x % kXcdCount, idx = blockIdx.x / kXcdCount;
    const int4 it = items[xcd * per + (xcd < rem ? xcd : rem) + idx];
    const int leaf = it.x, r0 = it.y, s0 = it.z, s1 = it.w;
    const int r1 = min(r0 + chunk, leaf_pt[leaf + 1]);
    switch ((r1 - r0 + kP2PThreads - 1) / kP2PThreads) {
        case 1:
            p2p_sym_item<1>(leaf, r0, r1, s0, s1, near_rng, near_cnt, px, py, pz, n, q, y, sxy, szq, sacc);
            break;
        case 2:
            p2p_sym_item<2>(leaf, r0, r1, s0, s1, near_rng, near_cnt, px, py, pz, n, q, y, sxy, szq, sacc);
            break;
        case 3:
            p2p_sym_item<3>(leaf, r0, r1, s0, s1, near_rng, near_cnt, px, py, pz, n, q, y, sxy, szq, sacc);
            break;
        default:
            p2p_sym_item<4>(leaf, r0, r1, s0, s1, near_rng, near_cnt, px, py, pz, n, q, y, sxy, szq, sacc);
            break;
    }
}


// ---------------------------------------------------------------------------
// FP32 near field (low-precision products). Coordinates are taken relative to
// the receiver leaf's centre in FP64 and rounded to FP32, so that the
// rounding error of a coordinate is relative to the leaf size rather than to
// the cube; 1/r is the hardware FP32 estimate (v_rsq_f32, about one ulp).
// The sums over a block of 64 sources run in FP32 and are added into FP64
// accumulators after each block.

// Symmetric form of one channel of monopoles (k_p2p_sym's items and pair
// order): each unordered pair once, its two terms added to both points.
template <int R>
__device__ inline void p2p_sym32_block(const float4 *src, double *sacc, const float *xi, const float *yi,
                                       const float *zi, const float *qi, double *accd, int b, bool diag) {
    const int lane = threadIdx.x;
    float acc[R];
#pragma unroll
    for (int k = 0; k < R; ++k) acc[k] = 0.f;
#pragma unroll 2
    for (int t = 0; t < kP2PThreads; ++t) {
        const int s = (lane + t) & (kP2PThreads - 1);
        const float4 a = src[s];
        float c = 0.f;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            // diagonal block: groups above b skipped, group b one-sided without
            // the receiver itself (step 0), groups below both ways
            if (diag && (k > b || (k == b && t == 0))) continue;  // wave-uniform
            const float dx = xi[k] - a.x, dy = yi[k] - a.y, dz = zi[k] - a.z;
            const float inv = __builtin_amdgcn_rsqf(dx * dx + dy * dy + dz * dz);
            acc[k] = fmaf(a.w, inv, acc[k]);
            if (!diag || k < b) c = fmaf(qi[k], inv, c);
        }
        // source-side sums in FP64 slots (ds_add_f64; the FP32 LDS add
        // stalled this loop on LDS waits)
        if (!diag || b > 0) atomicAdd(sacc + s, (double)c);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) accd[k] += (double)acc[k];
}

template <int R>
__device__ inline void p2p_sym32_item(int leaf, int r0, int r1, int s0, int s1, const int2 *__restrict__ near_rng,
                                      const int *__restrict__ near_cnt, double ox, double oy, double oz,
                                      const double *__restrict__ px, const double *__restrict__ py,
                                      const double *__restrict__ pz, const double *__restrict__ q,
                                      double *__restrict__ y, float4 *src, double *sacc) {
    const int lane = threadIdx.x;
    float xi[R], yi[R], zi[R], qi[R];
    double accd[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = r0 + lane + k * kP2PThreads;
        const bool ok = i < r1;
        // idle receivers sit far away with no weight; never stored
        xi[k] = ok ? (float)(px[i] - ox) : 1e30f;
        yi[k] = ok ? (float)(py[i] - oy) : 0.f;
        zi[k] = ok ? (float)(pz[i] - oz) : 0.f;
        qi[k] = ok ? (float)q[i] : 0.f;
        accd[k] = 0.0;
    }
    if (s1 <= r1 - r0) {
        // the chunk's own points, in blocks of 64 aligned with the receiver groups
        for (int base = s0; base < s1; base += kP2PThreads) {
            const int j = r0 + base + lane;
            const bool ok = base + lane < s1;
            src[lane] = ok ? make_float4((float)(px[j] - ox), (float)(py[j] - oy), (float)(pz[j] - oz), (float)q[j])
                           : make_float4(-1e30f, 0.f, 0.f, 0.f);
            sacc[lane] = 0.0;
            __syncthreads();
            const int b = base / kP2PThreads;
            p2p_sym32_block<R>(src, sacc, xi, yi, zi, qi, accd, b, true);
            __syncthreads();
            if (ok && b > 0) unsafeAtomicAdd(y + j, sacc[lane]);
        }
    } else {
        const int2 *rng = near_rng + 27 * (int64_t)leaf;
        const int nr = near_cnt[leaf];
        for (int base = s0; base < s1; base += kP2PThreads) {
            const int p = base + lane;
            int j = -1, cum = 0;
            for (int g = 0; g < nr; ++g) {
                const int2 r = rng[g];
                const int a = max(r.x, r0), len = max(0, r.y - a);
                if (p >= cum && p < cum + len) j = a + (p - cum);
                cum += len;
            }
            const bool ok = p < s1 && j >= 0;
            src[lane] = ok ? make_float4((float)(px[j] - ox), (float)(py[j] - oy), (float)(pz[j] - oz), (float)q[j])
                           : make_float4(-1e30f, 0.f, 0.f, 0.f);
            sacc[lane] = 0.0;
            __syncthreads();
            p2p_sym32_block<R>(src, sacc, xi, yi, zi, qi, accd, 0, false);
            __syncthreads();
            if (ok) unsafeAtomicAdd(y + j, sacc[lane]);
        }
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = r0 + lane + k * kP2PThreads;
        if (i < r1) unsafeAtomicAdd(y + i, accd[k]);
    }
}

__global__ void __launch_bounds__(kP2PThreads) k_p2p_sym32(const int4 *__restrict__ items,
                                                           const int *__restrict__ leaf_pt,
                                                           const int2 *__restrict__ near_rng,
                                                           const int *__restrict__ near_cnt,
                                                           const double *__restrict__ centre, int64_t leaf0,
                                                           const double *__restrict__ px,
                                                           const double *__restrict__ py,
                                                           const double *__restrict__ pz,
                                                           const double *__restrict__ q, int chunk,
                                                           double *__restrict__ y) {
    __shared__ float4 src[kP2PThreads];
    __shared__ double sacc[kP2PThreads];
    const int nblock = gridDim.x, per = nblock / kXcdCount, rem = nblock % kXcdCount;
    const int xcd = blockIdx.x % kXcdCount, idx = blockIdx.x / kXcdCount;
    const int4 it = items[xcd * per + (xcd < rem ? xcd : rem) + idx];
    const int leaf = it.x, r0 = it.y, s0 = it.z, s1 = it.w;
    const int r1 = min(r0 + chunk, leaf_pt[leaf + 1]);
    const double *c = centre + 3 * (leaf0 + leaf);
    const double ox = c[0], oy = c[1], oz = c[2];
    switch ((r1 - r0 + kP2PThreads - 1) / kP2PThreads) {
        case 1:
            p2p_sym32_item<1>(leaf, r0, r1, s0, s1, near_rng, near_cnt, ox, oy, oz, px, py, pz, q, y, src, sacc);
            break;
        case 2:
            p2p_sym32_item<2>(leaf, r0, r1, s0, s1, near_rng, near_cnt, ox, oy, oz, px, py, pz, q, y, src, sacc);
            break;
        case 3:
            p2p_sym32_item<3>(leaf, r0, r1, s0, s1, near_rng, near_cnt, ox, oy, oz, px, py, pz, q, y, src, sacc);
            break;
        default:
            p2p_sym32_item<4>(leaf, r0, r1, s0, s1, near_rng, near_cnt, ox, oy, oz, px, py, pz, q, y, src, sacc);
            break;
    }
}

// One-sided FP32 form (any channel content; k_p2p's items and pieces):
// receivers rc + lane + 64 k of the leaf against sources s0..s1-1 of its list,
// read at wave-uniform addresses and shifted to the leaf centre per lane.
template <bool MONO, bool DIP, bool SELF>
__device__ inline void p2p32_range(int j0, int j1, double ox, double oy, double oz, const double *__restrict__ px,
                                   const double *__restrict__ py, const double *__restrict__ pz,
                                   const double *__restrict__ pnx, const double *__restrict__ pny,
                                   const double *__restrict__ pnz, const double *__restrict__ q,
                                   const double *__restrict__ w, const float *xi, const float *yi, const float *zi,
                                   double *accd) {
    constexpr int R = kP2PChunk / kP2PThreads;
    for (int b0 = j0; b0 < j1; b0 += kP2PThreads) {
        const int b1 = min(j1, b0 + kP2PThreads);
        float acc[R];
#pragma unroll
        for (int k = 0; k < R; ++k) acc[k] = 0.f;
        for (int j = b0; j < b1; ++j) {
            const float sx = (float)(px[j] - ox), sy = (float)(py[j] - oy), sz = (float)(pz[j] - oz);
            const float sq = MONO ? (float)q[j] : 0.f, sw = DIP ? (float)w[j] : 0.f;
            const float nx = DIP ? (float)pnx[j] : 0.f, ny = DIP ? (float)pny[j] : 0.f, nz = DIP ? (float)pnz[j] : 0.f;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const float dx = xi[k] - sx, dy = yi[k] - sy, dz = zi[k] - sz;
                const float r2 = dx * dx + dy * dy + dz * dz;
                const float inv = (!SELF || r2 > 0.f) ? __builtin_amdgcn_rsqf(r2) : 0.f;  // j == i excluded
                if (MONO) acc[k] = fmaf(sq, inv, acc[k]);
                if (DIP) acc[k] = fmaf(sw * (nx * dx + ny * dy + nz * dz), inv * inv * inv, acc[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < R; ++k) accd[k] += (double)acc[k];
    }
}

template <bool MONO, bool DIP, bool ATOMIC>
__global__ void __launch_bounds__(kP2PThreads) k_p2p32(const int4 *__restrict__ items,
                                                       const int *__restrict__ leaf_pt,
                                                       const int2 *__restrict__ near_rng,
                                                       const int *__restrict__ near_cnt,
                                                       const double *__restrict__ centre, int64_t leaf0,
                                                       const double *__restrict__ px, const double *__restrict__ py,
                                                       const double *__restrict__ pz, const double *__restrict__ pnx,
                                                       const double *__restrict__ pny, const double *__restrict__ pnz,
                                                       const double *__restrict__ q, const double *__restrict__ w,
                                                       double *__restrict__ y) {
    constexpr int R = kP2PChunk / kP2PThreads;
    const int nblock = gridDim.x, per = nblock / kXcdCount, rem = nblock % kXcdCount;
    const int xcd = blockIdx.x % kXcdCount, idx = blockIdx.x / kXcdCount;
    const int4 it = items[xcd * per + (xcd < rem ? xcd : rem) + idx];
    const int leaf = it.x, rc = it.y, s0 = it.z, s1 = it.w;
    const int l0 = leaf_pt[leaf], r1 = leaf_pt[leaf + 1];
    const double *c = centre + 3 * (leaf0 + leaf);
    const double ox = c[0], oy = c[1], oz = c[2];
    const int lane = threadIdx.x;
    float xi[R], yi[R], zi[R];
    double accd[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = rc + lane + k * kP2PThreads;
        const bool ok = i < r1;
        xi[k] = ok ? (float)(px[i] - ox) : 1e30f;  // idle lanes sit far away; never stored
        yi[k] = ok ? (float)(py[i] - oy) : 0.f;
        zi[k] = ok ? (float)(pz[i] - oz) : 0.f;
        accd[k] = 0.0;
    }
    const int2 *rng = near_rng + 27 * (int64_t)leaf;
    const int nr = near_cnt[leaf];
    int cum = 0;
    for (int g = 0; g < nr && cum < s1; ++g) {
        const int2 r = rng[g];
        const int len = r.y - r.x;
        const int a = r.x + max(0, s0 - cum), b = r.x + min(len, s1 - cum);
        cum += len;
        if (a >= b) continue;
        if (a < r1 && l0 < b) {
            const int m0 = max(a, l0), m1 = min(b, r1);
            p2p32_range<MONO, DIP, false>(a, m0, ox, oy, oz, px, py, pz, pnx, pny, pnz, q, w, xi, yi, zi, accd);
            p2p32_range<MONO, DIP, true>(m0, m1, ox, oy, oz, px, py, pz, pnx, pny, pnz, q, w, xi, yi, zi, accd);
            p2p32_range<MONO, DIP, false>(m1, b, ox, oy, oz, px, py, pz, pnx, pny, pnz, q, w, xi, yi, zi, accd);
        } else {
            p2p32_range<MONO, DIP, false>(a, b, ox, oy, oz, px, py, pz, pnx, pny, pnz, q, w, xi, yi, zi, accd);
        }
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = rc + lane + k * kP2PThreads;
        if (i < r1) {
            if (ATOMIC)
                unsafeAtomicAdd(y + i, accd[k]);
            else
                y[i] = accd[k];
        }
    }
}

__global__ void k_clear(double *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// All-pairs sum (checking path): 64 receivers per wave x every source.
template <int NCH, bool MONO, bool DIP>
__global__ void __launch_bounds__(kP2PThreads) k_direct(const double *__restrict__ px,
                                                        const double *__restrict__ py,
                                                        const double *__restrict__ pz,
                                                        const double *__restrict__ pnx,
                                                        const double *__restrict__ pny,
                                                        const double *__restrict__ pnz, int64_t n,
                                                        const double *__restrict__ q,
                                                        const double *__restrict__ w,
                                                        double *__restrict__ y) {
    const int64_t base = (int64_t)blockIdx.x * kP2PThreads;
    const int r1 = (int)((n - base) < kP2PThreads ? (n - base) : kP2PThreads);
    const int2 all = make_int2(0, (int)n);
    // receivers base + lane (pass of one receiver per lane), sources all points
    double xi[1], yi[1], zi[1], acc[1][NCH];
    const int i = (int)base + threadIdx.x;
    const bool ok = threadIdx.x < (unsigned)r1;
    xi[0] = ok ? px[i] : 1e100;
    yi[0] = ok ? py[i] : 0.0;
    zi[0] = ok ? pz[i] : 0.0;
    for (int c = 0; c < NCH; ++c) acc[0][c] = 0.0;
    p2p_range<NCH, MONO, DIP, 1, true>(all.x, all.y, px, py, pz, pnx, pny, pnz, n, q, w, xi, yi, zi, acc);
    if (ok)
        for (int c = 0; c < NCH; ++c) y[(int64_t)c * n + i] = acc[0][c];
}

static unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

template <int NCH, bool MONO, bool DIP>
void launch_p2p(const Tree &t, const Sources &src, double *y, hipStream_t st) {
    if (t.n_near_items <= 0) return;
    if constexpr (NCH == 1 && MONO && !DIP) {
        // one channel of monopoles: each pair once, added to both points
        BFM_CHECK(t.n_sym_items > 0, BFM_EINVAL, "symmetric near-field items missing");
        k_clear<<<1024, 256, 0, st>>>(y, t.n);
        BFM_LAUNCHED();
        k_p2p_sym<<<(unsigned)t.n_sym_items, kP2PThreads, 0, st>>>(t.sym_items.get(), t.leaf_pt.get(),
                                                                   t.near_rng.get(), t.near_cnt.get(), t.px.get(),
                                                                   t.py.get(), t.pz.get(), t.n, src.q, t.sym_chunk,
                                                                   y);
        BFM_LAUNCHED();
        return;
    }
    if (t.near_split) {
        k_clear<<<1024, 256, 0, st>>>(y, (int64_t)NCH * t.n);
        BFM_LAUNCHED();
    }
    auto kern = t.near_split ? k_p2p<NCH, MONO, DIP, true> : k_p2p<NCH, MONO, DIP, false>;
    kern<<<(unsigned)t.n_near_items, kP2PThreads, 0, st>>>(t.near_items.get(), t.leaf_pt.get(), t.near_rng.get(),
                                                           t.near_cnt.get(), t.px.get(), t.py.get(), t.pz.get(),
                                                           t.pnx.get(), t.pny.get(), t.pnz.get(), t.n, src.q, src.w,
                                                           y);
    BFM_LAUNCHED();
}

void launch_p2p_packed(const Tree &t, const double *packed, double *y, hipStream_t st) {
    if (t.n_near_items <= 0) return;
    if (t.near_split) {
        k_clear<<<1024, 256, 0, st>>>(y, (int64_t)5 * t.n);
        BFM_LAUNCHED();
    }
    auto kern = t.near_split ? k_p2p_diag<true> : k_p2p_diag<false>;
    kern<<<(unsigned)t.n_near_items, kP2PThreads, 0, st>>>(t.near_items.get(), t.leaf_pt.get(), t.near_rng.get(),
                                                           t.near_cnt.get(), t.px.get(), t.py.get(), t.pz.get(),
                                                           packed, t.n, y);
    BFM_LAUNCHED();
}

template <int NCH, bool MONO, bool DIP>
void launch_direct(const Tree &t, const Sources &src, double *y, hipStream_t st) {
    k_direct<NCH, MONO, DIP><<<nblk(t.n, kP2PThreads), kP2PThreads, 0, st>>>(
        t.px.get(), t.py.get(), t.pz.get(), t.pnx.get(), t.pny.get(), t.pnz.get(), t.n, src.q, src.w, y);
    BFM_LAUNCHED();
}


template <bool MONO, bool DIP>
void launch_p2p32(const Tree &t, const Sources &src, double *y, hipStream_t st) {
    if (t.n_near_items <= 0) return;
    const int64_t leaf0 = t.lvl_off[t.lmax];
    if constexpr (MONO && !DIP) {
        BFM_CHECK(t.n_sym_items > 0, BFM_EINVAL, "symmetric near-field items missing");
        k_clear<<<1024, 256, 0, st>>>(y, t.n);
        BFM_LAUNCHED();
        k_p2p_sym32<<<(unsigned)t.n_sym_items, kP2PThreads, 0, st>>>(
            t.sym_items.get(), t.leaf_pt.get(), t.near_rng.get(), t.near_cnt.get(), t.box_centre.get(), leaf0,
            t.px.get(), t.py.get(), t.pz.get(), src.q, t.sym_chunk, y);
        BFM_LAUNCHED();
        return;
    }
    if (t.near_split) {
        k_clear<<<1024, 256, 0, st>>>(y, t.n);
        BFM_LAUNCHED();
    }
    auto kern = t.near_split ? k_p2p32<MONO, DIP, true> : k_p2p32<MONO, DIP, false>;
    kern<<<(unsigned)t.n_near_items, kP2PThreads, 0, st>>>(t.near_items.get(), t.leaf_pt.get(), t.near_rng.get(),
                                                           t.near_cnt.get(), t.box_centre.get(), leaf0, t.px.get(),
                                                           t.py.get(), t.pz.get(), t.pnx.get(), t.pny.get(),
                                                           t.pnz.get(), src.q, src.w, y);
    BFM_LAUNCHED();
}

template void launch_p2p32<true, false>(const Tree &, const Sources &, double *, hipStream_t);
template void launch_p2p32<false, true>(const Tree &, const Sources &, double *, hipStream_t);
template void launch_p2p32<true, true>(const Tree &, const Sources &, double *, hipStream_t);

#define BFM_NEAR_INST(NCH, MONO, DIP)                                                                    \
    template void launch_p2p<NCH, MONO, DIP>(const Tree &, const Sources &, double *, hipStream_t); \
    template void launch_direct<NCH, MONO, DIP>(const Tree &, const Sources &, double *, hipStream_t);
BFM_NEAR_INST(1, true, false)
BFM_NEAR_INST(1, false, true)
BFM_NEAR_INST(1, true, true)
BFM_NEAR_INST(5, true, true)
#undef BFM_NEAR_INST

}  // namespace bfm
