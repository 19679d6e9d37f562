// Leaf expansions of the fast multipole product (Section 3.9): P2M forms
// the multipole expansion of every leaf from its points' monopoles and
// dipoles, L2P evaluates every leaf's local expansion at its points. Both
// build the regular solid harmonics of a point by the three-term recurrences
// of the box-scaled normalised basis, in registers.
//
// Both kernels run one wave per leaf work item (a leaf and up to kLeafChunk of
// its points), each lane taking kLeafChunk / 64 points, so the grid has about
// twice as many waves as the octree has leaves and every wave does the same
// amount of work.
#include <cmath>
#include <vector>

#include "fmm_kernels.h"

namespace bfm {

constexpr int kTri = kMaxP * (kMaxP + 1) / 2;  // (n, m >= 0) pairs, n < kMaxP
constexpr int kPPL = kLeafChunk / 64;            // points per lane
static_assert(kPPL * 64 == kLeafChunk, "whole points per lane");

// Recurrence of the regular harmonics for degree n > m:
//   Rt_n^m = ae(n, m) z Rt_{n-1}^m - ab(n, m) r^2 Rt_{n-2}^m,
//   ae = (2n-1)/sqrt((n-m)(n+m)), ab = sqrt((n-m-1)(n+m-1))/sqrt((n-m)(n+m)),
// and for the sectoral ones Rt_m^m = f_m (x + i y) Rt_{m-1}^{m-1},
//   f_m = sqrt((2m-1)/(2m)).
__constant__ double2 c_rec[kTri];  // (ae, ab) at tri(n, m)
__constant__ double c_sect[kMaxP];  // f_m

__host__ __device__ constexpr int tri(int n, int m) { return n * (n + 1) / 2 + m; }

void leaf_tables_upload(int device) {
    static int done_mask = 0;  // one bit per device ordinal < 32
    if (device < 32 && (done_mask >> device) & 1) return;
    std::vector<double2> rec(kTri, make_double2(0.0, 0.0));
    std::vector<double> sect(kMaxP, 0.0);
    for (int n = 0; n < kMaxP; ++n)
        for (int m = 0; m < n; ++m) {
            const double a = 1.0 / std::sqrt((double)(n - m) * (n + m));
            const double b = n >= m + 2 ? std::sqrt((double)(n - m - 1) * (n + m - 1)) : 0.0;
            rec[tri(n, m)] = make_double2((2.0 * n - 1.0) * a, b * a);
        }
    for (int m = 1; m < kMaxP; ++m) sect[m] = std::sqrt((2.0 * m - 1.0) / (2.0 * m));
    BFM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_rec), rec.data(), sizeof(double2) * kTri));
    BFM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_sect), sect.data(), sizeof(double) * kMaxP));
    if (device < 32) done_mask |= 1 << device;
}

// Pair of recurrence constants in the arithmetic type R.
template <class R>
struct Pair2 {
    R x, y;
};

// Copy the recurrence tables for order P into LDS (block-wide), rounded to R.
template <int P_, class R>
__device__ inline void stage_tables(Pair2<R> *rec, R *sect, int tid, int nthreads) {
    constexpr int NT = P_ * (P_ + 1) / 2;
    for (int t = tid; t < NT; t += nthreads) rec[t] = Pair2<R>{(R)c_rec[t].x, (R)c_rec[t].y};
    for (int t = tid; t < P_; t += nthreads) sect[t] = (R)c_sect[t];
}

// ---------------------------------------------------------------------------
// P2M. Lane l takes the item's points l, l + 64, ..., builds their regular
// harmonics order by order (loops over order m and degree k uniform across
// the wave, recurrence constants read from LDS at wave-uniform addresses)
// and sums its points' contributions for every coefficient (slot) and
// channel. The wave's 64 partial sums of each (slot, channel) column are
// buffered in LDS (one row per column) and, once COLS or more columns are
// buffered, lane t adds up row t and adds it to the leaf's expansion with an
// FP64 atomic (a leaf with more points than one item has several items).
//   Mt_n^m += q_j conj(Rt_n^m(v_j)) + (w_j / h) conj(n_j . grad_v Rt_n^m(v_j)),
// v_j = (r_j - c)/h. The directional derivative D = n_j . grad_v follows the
// same recurrence by forward differentiation:
//   D Rt_m^m = f_m [D Rt_{m-1}^{m-1} (x+iy) + Rt_{m-1}^{m-1} (n_x+i n_y)]
//   D Rt_n^m = ae (n_z Rt_{n-1} + z D Rt_{n-1}) - ab (2 v.n Rt_{n-2} + r^2 D Rt_{n-2})
// Slots run over m, then degree k >= m, then (real, imaginary) for m > 0;
// column = slot * NCH + channel.
template <int P_, int NCH, bool MONO, bool DIP, class R>
__global__ void __launch_bounds__(64) k_p2m(const int2 *__restrict__ items, int64_t leaf0,
                                            const int *__restrict__ leaf_pt, const double *__restrict__ centre,
                                            double h, const double *__restrict__ px, const double *__restrict__ py,
                                            const double *__restrict__ pz, const double *__restrict__ pnx,
                                            const double *__restrict__ pny, const double *__restrict__ pnz, int64_t n,
                                            const double *__restrict__ q, const double *__restrict__ w,
                                            R *__restrict__ mexp) {
    constexpr int PP = P_ * P_;
    constexpr int NT = P_ * (P_ + 1) / 2;
    constexpr int NCOL = PP * NCH;
    // channels with monopoles (bit c): every channel, except in the five-channel
    // set of the diagonal pass, whose channels 0 and 4 are pure dipoles
    constexpr unsigned QMASK = !MONO ? 0u : (NCH == 5 ? 0x0Eu : (1u << NCH) - 1u);
    // buffered columns at most (a power of two dividing 64); a loop trip adds
    // at most 4 NCH columns, so the buffer is flushed once it holds COLS
    constexpr int CAP = NCH == 1 ? 16 : 32;
    constexpr int COLS = CAP - 4 * NCH;
    static_assert(COLS >= 1 && 64 % CAP == 0, "flush shape");
    // a flush gives each buffered column G lanes, each summing every G-th of
    // its 64 values; rows of 64 + G doubles put those reads in distinct banks
    constexpr int G = 64 / CAP;
    __shared__ R red[CAP][64 + G];
    __shared__ Pair2<R> rec[NT];
    __shared__ R sect[P_];
    __shared__ int outi[PP];
    const int lane = threadIdx.x;
    const int2 it = items[blockIdx.x];
    const int leaf = it.x, rb = it.y;
    const int re = min(rb + kLeafChunk, leaf_pt[leaf + 1]);
    const int64_t box = leaf0 + leaf;
    stage_tables<P_, R>(rec, sect, lane, 64);
    // slot -> coefficient index in the packed expansion (n^2 + 2m - 1 + imaginary)
    for (int s = lane; s < PP; s += 64) {
        int k = s, o = s * s;
        if (s >= P_) {
            int r = s - P_, m = 1;
            while (r >= 2 * (P_ - m)) {
                r -= 2 * (P_ - m);
                ++m;
            }
            k = m + r / 2;
            o = k * k + 2 * m - 1 + (r & 1);
        }
        outi[s] = o;
    }
    const double cx = centre[3 * box], cy = centre[3 * box + 1], cz = centre[3 * box + 2];
    const double ih = 1.0 / h;
    R x[kPPL], y[kPPL], z[kPPL], r2[kPPL], sq[kPPL][NCH], sw[kPPL][NCH];
    R ux[kPPL], uy[kPPL], uz[kPPL], vu2[kPPL];
#pragma unroll
    for (int u = 0; u < kPPL; ++u) {
        const int j0 = rb + 64 * u + lane;
        const bool ok = j0 < re;
        const int j = ok ? j0 : rb;  // idle slots: the first point, zero strength
        // leaf-relative, box-scaled coordinates formed in FP64, then rounded to R
        x[u] = (R)((px[j] - cx) * ih);
        y[u] = (R)((py[j] - cy) * ih);
        z[u] = (R)((pz[j] - cz) * ih);
        r2[u] = x[u] * x[u] + y[u] * y[u] + z[u] * z[u];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            sq[u][c] = ((QMASK >> c) & 1u) ? (R)(ok ? q[(int64_t)c * n + j] : 0.0) : R(0);
            sw[u][c] = DIP ? (R)(ok ? w[(int64_t)c * n + j] * ih : 0.0) : R(0);
        }
        ux[u] = DIP ? (R)pnx[j] : R(0);
        uy[u] = DIP ? (R)pny[j] : R(0);
        uz[u] = DIP ? (R)pnz[j] : R(0);
        vu2[u] = R(2) * (x[u] * ux[u] + y[u] * uy[u] + z[u] * uz[u]);
    }
    __syncthreads();
    R *mbox = mexp + box * NCH * PP;
    int col = 0, fill = 0;  // next column, buffered columns (wave-uniform)
    // buffered column sums -> the leaf's expansion
    auto flush = [&]() {
        __syncthreads();
        const int cl = lane / G, part = lane % G;
        R s0 = 0, s1 = 0;
        if (cl < fill) {
#pragma unroll
            for (int l = 0; l < 64 / G; l += 2) {
                s0 += red[cl][l * G + part];
                s1 += red[cl][(l + 1) * G + part];
            }
        }
        R sum = s0 + s1;
#pragma unroll
        for (int o = 1; o < G; o <<= 1) sum += __shfl_xor(sum, o);
        if (cl < fill && part == 0) {
            const int cc = col - fill + cl;
            const int sl = cc / NCH, c = cc - sl * NCH;
            unsafeAtomicAdd(mbox + c * PP + outi[sl], sum);
        }
        __syncthreads();
        fill = 0;
    };
    auto put = [&](R v) {
        red[fill][lane] = v;
        ++fill;
        ++col;
    };
    R dr[kPPL], di[kPPL], Ddr[kPPL], Ddi[kPPL];  // Rt_m^m and its derivative
#pragma unroll
    for (int u = 0; u < kPPL; ++u) {
        dr[u] = 1;
        di[u] = Ddr[u] = Ddi[u] = 0;
    }
#pragma unroll 1
    for (int m = 0; m < P_; ++m) {
        if (m > 0) {
            const R f = sect[m];
#pragma unroll
            for (int u = 0; u < kPPL; ++u) {
                const R nr = (dr[u] * x[u] - di[u] * y[u]) * f, ni = (dr[u] * y[u] + di[u] * x[u]) * f;
                if (DIP) {
                    const R nDr = (Ddr[u] * x[u] - Ddi[u] * y[u] + dr[u] * ux[u] - di[u] * uy[u]) * f;
                    const R nDi = (Ddr[u] * y[u] + Ddi[u] * x[u] + dr[u] * uy[u] + di[u] * ux[u]) * f;
                    Ddr[u] = nDr;
                    Ddi[u] = nDi;
                }
                dr[u] = nr;
                di[u] = ni;
            }
        }
        // degrees k = m, m+1, ...: two register sets take turns holding the
        // current and the previous degree (the new degree overwrites the
        // previous one), two degrees per loop trip
        R Ar[kPPL], Ai[kPPL], Br[kPPL], Bi[kPPL], DAr[kPPL], DAi[kPPL], DBr[kPPL], DBi[kPPL];
#pragma unroll
        for (int u = 0; u < kPPL; ++u) {
            Ar[u] = dr[u];
            Ai[u] = di[u];
            DAr[u] = Ddr[u];
            DAi[u] = Ddi[u];
            Br[u] = Bi[u] = DBr[u] = DBi[u] = 0;
        }
        // P <- degree k from C (degree k-1) and P (degree k-2)
        auto advance = [&](int t, const R(&Cr)[kPPL], const R(&Ci)[kPPL], const R(&DCr)[kPPL],
                           const R(&DCi)[kPPL], R(&Pr)[kPPL], R(&Pi)[kPPL], R(&DPr)[kPPL],
                           R(&DPi)[kPPL]) {
            const Pair2<R> ca = rec[t];
#pragma unroll
            for (int u = 0; u < kPPL; ++u) {
                const R ez = ca.x * z[u], br = ca.y * r2[u];
                if (DIP) {
                    const R eu = ca.x * uz[u], bv = ca.y * vu2[u];
                    const R nDr = eu * Cr[u] + ez * DCr[u] - bv * Pr[u] - br * DPr[u];
                    const R nDi = eu * Ci[u] + ez * DCi[u] - bv * Pi[u] - br * DPi[u];
                    DPr[u] = nDr;
                    DPi[u] = nDi;
                }
                Pr[u] = ez * Cr[u] - br * Pr[u];
                Pi[u] = ez * Ci[u] - br * Pi[u];
            }
        };
        // the conjugated coefficient of degree k (held in C) for every channel
        auto emit = [&](const R(&Cr)[kPPL], const R(&Ci)[kPPL], const R(&DCr)[kPPL],
                        const R(&DCi)[kPPL]) {
            // a term is left out where its channel has no monopole (or no dipole)
            auto term = [&](int c, int u, R a, R da) -> R {
                const bool hq = (QMASK >> c) & 1u;
                if (hq && DIP) return sq[u][c] * a + sw[u][c] * da;
                return hq ? sq[u][c] * a : sw[u][c] * da;
            };
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                R v = term(c, 0, Cr[0], DCr[0]);
#pragma unroll
                for (int u = 1; u < kPPL; ++u) v += term(c, u, Cr[u], DCr[u]);
                put(v);
            }
            if (m > 0) {
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    R v = term(c, 0, Ci[0], DCi[0]);
#pragma unroll
                    for (int u = 1; u < kPPL; ++u) v += term(c, u, Ci[u], DCi[u]);
                    put(-v);
                }
            }
        };
        emit(Ar, Ai, DAr, DAi);
        int k = m + 1, t = tri(m + 1, m);
#pragma unroll 1
        for (; k + 1 < P_; k += 2) {
            if (fill >= COLS) flush();
            advance(t, Ar, Ai, DAr, DAi, Br, Bi, DBr, DBi);
            emit(Br, Bi, DBr, DBi);
            t += k + 1;
            advance(t, Br, Bi, DBr, DBi, Ar, Ai, DAr, DAi);
            emit(Ar, Ai, DAr, DAi);
            t += k + 2;
        }
        if (fill >= COLS) flush();
        if (k < P_) {
            advance(t, Ar, Ai, DAr, DAi, Br, Bi, DBr, DBi);
            emit(Br, Bi, DBr, DBi);
        }
    }
    flush();
}

// L2P. Lane l takes the item's points l, l + 64, ...:
//   y_i += (1/h) sum_n [Lt_n^0 Rt_n^0 + 2 sum_{m>0} Re(Lt_n^m Rt_n^m)],
// the harmonics built in registers order by order. The leaf's coefficients
// and the recurrence constants are first copied to LDS with coalesced loads;
// every step reads them at a wave-uniform LDS address.
template <int P_, int NCH, class R>
__global__ void __launch_bounds__(64) k_l2p(const int2 *__restrict__ items, int64_t leaf0,
                                            const int *__restrict__ leaf_pt, const double *__restrict__ centre,
                                            double h, const double *__restrict__ px, const double *__restrict__ py,
                                            const double *__restrict__ pz, int64_t n,
                                            const R *__restrict__ lexp, double *__restrict__ y) {
    constexpr int PP = P_ * P_;
    constexpr int NT = P_ * (P_ + 1) / 2;
    __shared__ R Ls[NCH * PP];
    __shared__ Pair2<R> rec[NT];
    __shared__ R sect[P_];
    const int lane = threadIdx.x;
    const int2 it = items[blockIdx.x];
    const int leaf = it.x, rb = it.y;
    const int re = min(rb + kLeafChunk, leaf_pt[leaf + 1]);
    const int64_t box = leaf0 + leaf;
    const R *L = lexp + box * NCH * PP;
    for (int t = lane; t < NCH * PP; t += 64) Ls[t] = L[t];
    stage_tables<P_, R>(rec, sect, lane, 64);
    const double ih = 1.0 / h;
    const double cx = centre[3 * box], cy = centre[3 * box + 1], cz = centre[3 * box + 2];
    R x[kPPL], yy[kPPL], z[kPPL], r2[kPPL], acc[kPPL][NCH];
#pragma unroll
    for (int u = 0; u < kPPL; ++u) {
        const int j0 = rb + 64 * u + lane;
        const int j = j0 < re ? j0 : rb;
        x[u] = (R)((px[j] - cx) * ih);
        yy[u] = (R)((py[j] - cy) * ih);
        z[u] = (R)((pz[j] - cz) * ih);
        r2[u] = x[u] * x[u] + yy[u] * yy[u] + z[u] * z[u];
#pragma unroll
        for (int c = 0; c < NCH; ++c) acc[u][c] = 0;
    }
    __syncthreads();
    R dr[kPPL], di[kPPL];
#pragma unroll
    for (int u = 0; u < kPPL; ++u) {
        dr[u] = 1;
        di[u] = 0;
    }
#pragma unroll 1
    for (int m = 0; m < P_; ++m) {
        if (m > 0) {
            const R f = sect[m];
#pragma unroll
            for (int u = 0; u < kPPL; ++u) {
                const R nr = (dr[u] * x[u] - di[u] * yy[u]) * f, ni = (dr[u] * yy[u] + di[u] * x[u]) * f;
                dr[u] = nr;
                di[u] = ni;
            }
        }
        R Ar[kPPL], Ai[kPPL], Br[kPPL], Bi[kPPL];  // current / previous degree, taking turns
#pragma unroll
        for (int u = 0; u < kPPL; ++u) {
            Ar[u] = dr[u];
            Ai[u] = di[u];
            Br[u] = Bi[u] = 0;
        }
        const R wgt = (m == 0) ? R(1) : R(2);
        auto advance = [&](int t, const R(&Cr)[kPPL], const R(&Ci)[kPPL], R(&Pr)[kPPL], R(&Pi)[kPPL]) {
            const Pair2<R> ca = rec[t];
#pragma unroll
            for (int u = 0; u < kPPL; ++u) {
                const R ez = ca.x * z[u], br = ca.y * r2[u];
                Pr[u] = ez * Cr[u] - br * Pr[u];
                Pi[u] = ez * Ci[u] - br * Pi[u];
            }
        };
        auto gather = [&](int li, const R(&Cr)[kPPL], const R(&Ci)[kPPL]) {
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const R lre = wgt * Ls[c * PP + li], lim = (m == 0) ? R(0) : wgt * Ls[c * PP + li + 1];
#pragma unroll
                for (int u = 0; u < kPPL; ++u) acc[u][c] += lre * Cr[u] - lim * Ci[u];
            }
        };
        int li = m * m + (m == 0 ? 0 : 2 * m - 1);  // real part of (k, m) in the packed layout
        gather(li, Ar, Ai);
        int k = m + 1, t = tri(m + 1, m);
        li += 2 * m + 1;
#pragma unroll 1
        for (; k + 1 < P_; k += 2) {
            advance(t, Ar, Ai, Br, Bi);
            gather(li, Br, Bi);
            t += k + 1;
            li += 2 * k + 1;
            advance(t, Br, Bi, Ar, Ai);
            gather(li, Ar, Ai);
            t += k + 2;
            li += 2 * k + 3;
        }
        if (k < P_) {
            advance(t, Ar, Ai, Br, Bi);
            gather(li, Br, Bi);
        }
    }
#pragma unroll
    for (int u = 0; u < kPPL; ++u) {
        const int j = rb + 64 * u + lane;
        if (j < re) {
#pragma unroll
            for (int c = 0; c < NCH; ++c) y[(int64_t)c * n + j] += (double)acc[u][c] * ih;
        }
    }
}

template <int P_, int NCH, bool MONO, bool DIP, class R>
void launch_p2m(const Tree &t, const Sources &src, R *M, hipStream_t st) {
    if (t.n_leaf_items <= 0) return;
    const int64_t leaf0 = t.lvl_off[t.lmax];
    const double hleaf = t.side / (double)(1 << t.lmax);
    k_p2m<P_, NCH, MONO, DIP, R><<<(unsigned)t.n_leaf_items, 64, 0, st>>>(
        t.leaf_items.get(), leaf0, t.leaf_pt.get(), t.box_centre.get(), hleaf, t.px.get(), t.py.get(), t.pz.get(),
        t.pnx.get(), t.pny.get(), t.pnz.get(), t.n, src.q, src.w, M);
    BFM_LAUNCHED();
}

template <int P_, int NCH, class R>
void launch_l2p(const Tree &t, const R *L, double *y, hipStream_t st) {
    if (t.n_leaf_items <= 0) return;
    const int64_t leaf0 = t.lvl_off[t.lmax];
    const double hleaf = t.side / (double)(1 << t.lmax);
    k_l2p<P_, NCH, R><<<(unsigned)t.n_leaf_items, 64, 0, st>>>(t.leaf_items.get(), leaf0, t.leaf_pt.get(),
                                                           t.box_centre.get(), hleaf, t.px.get(), t.py.get(),
                                                           t.pz.get(), t.n, L, y);
    BFM_LAUNCHED();
}

#define BFM_LEAF_INST(P)                                                                   \
    template void launch_p2m<P, 1, true, false>(const Tree &, const Sources &, double *, hipStream_t); \
    template void launch_p2m<P, 1, false, true>(const Tree &, const Sources &, double *, hipStream_t); \
    template void launch_p2m<P, 1, true, true>(const Tree &, const Sources &, double *, hipStream_t);  \
    template void launch_p2m<P, 5, true, true>(const Tree &, const Sources &, double *, hipStream_t);  \
    template void launch_l2p<P, 1>(const Tree &, const double *, double *, hipStream_t);               \
    template void launch_l2p<P, 5>(const Tree &, const double *, double *, hipStream_t);               \
    template void launch_p2m<P, 1, true, false, float>(const Tree &, const Sources &, float *, hipStream_t); \
    template void launch_p2m<P, 1, false, true, float>(const Tree &, const Sources &, float *, hipStream_t); \
    template void launch_p2m<P, 1, true, true, float>(const Tree &, const Sources &, float *, hipStream_t);  \
    template void launch_l2p<P, 1, float>(const Tree &, const float *, double *, hipStream_t);
BFM_LEAF_INST(4)
BFM_LEAF_INST(8)
BFM_LEAF_INST(12)
BFM_LEAF_INST(16)
BFM_LEAF_INST(20)
#undef BFM_LEAF_INST

}  // namespace bfm
