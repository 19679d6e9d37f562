// Fast multipole product on one GPU (Section 3.9): the far field
// (A^(dense) X) through multipole and local expansions of degrees 0..p-1,
// the near field (A^(sparse) X) by direct summation over neighbour leaves.
//
//   P2M   leaf multipoles from monopoles and dipoles            (per leaf)
//   M2M   child -> parent, level by level up to level 2         (grouped GEMM)
//   M2L   interaction lists of every level, one launch          (grouped GEMM)
//   L2L   parent -> child, level by level down to the leaves    (grouped GEMM)
//   L2P   evaluate leaf locals at the leaf's points             (per leaf)
//   P2P   leaf x (leaf + neighbours), LDS-staged source tiles   (per leaf)
//
// The three translations share one kernel: tasks grouped by operator, each
// wave multiplies one P x P operator by 16 gathered expansion columns with
// FP64 MFMA (v_mfma_f64_16x16x4f64) and adds the result into the target
// expansions with FP64 atomics.
#include <cmath>
#include <vector>

#include "common.h"
#include "fmm.h"
#include "ops.h"

namespace bfm {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int kTri = kMaxP * (kMaxP + 1) / 2;  // (n, m >= 0) pairs, n < kMaxP

__constant__ double c_rec_a[kTri];  // 1/sqrt((n-m)(n+m))
__constant__ double c_rec_b[kTri];  // sqrt((n-m-1)(n+m-1))
__constant__ double c_diag[kMaxP];  // sqrt((2m-1)/(2m))
__constant__ double c_dz[kTri];     // sqrt((n-m)(n+m))
__constant__ double c_dp[kTri];     // sqrt((n+m)(n+m-1))
__constant__ double c_dm[kTri];     // sqrt((n-m)(n-m-1))

__host__ __device__ constexpr int tri(int n, int m) { return n * (n + 1) / 2 + m; }

static void upload_tables(int device) {
    static int done_mask = 0;  // one bit per device ordinal < 32
    if (device < 32 && (done_mask >> device) & 1) return;
    std::vector<double> a(kTri, 0.0), b(kTri, 0.0), dz(kTri, 0.0), dp(kTri, 0.0), dm(kTri, 0.0);
    std::vector<double> dg(kMaxP, 0.0);
    for (int n = 0; n < kMaxP; ++n)
        for (int m = 0; m <= n; ++m) {
            const int t = tri(n, m);
            if (n > m) a[t] = 1.0 / std::sqrt((double)(n - m) * (n + m));
            if (n >= m + 2) b[t] = std::sqrt((double)(n - m - 1) * (n + m - 1));
            dz[t] = std::sqrt((double)(n - m) * (n + m));
            dp[t] = std::sqrt((double)(n + m) * (n + m - 1 > 0 ? n + m - 1 : 0));
            dm[t] = std::sqrt((double)(n - m) * (n - m - 1 > 0 ? n - m - 1 : 0));
        }
    for (int m = 1; m < kMaxP; ++m) dg[m] = std::sqrt((2.0 * m - 1.0) / (2.0 * m));
    BFM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_rec_a), a.data(), sizeof(double) * kTri));
    BFM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_rec_b), b.data(), sizeof(double) * kTri));
    BFM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_dz), dz.data(), sizeof(double) * kTri));
    BFM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_dp), dp.data(), sizeof(double) * kTri));
    BFM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_dm), dm.data(), sizeof(double) * kTri));
    BFM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_diag), dg.data(), sizeof(double) * kMaxP));
    if (device < 32) done_mask |= 1 << device;
}

// ---------------------------------------------------------------------------
// Regular harmonics of one order m (column) for n = m..p-1 at v, written to
// LDS rows re[tri(n, m)], im[tri(n, m)] (see common.h for the recurrence).
template <int P_>
__device__ inline void regular_column(int m, double x, double y, double z, double *re, double *im) {
    const double r2 = x * x + y * y + z * z;
    double dr = 1.0, di = 0.0;
    for (int k = 1; k <= m; ++k) {
        const double f = c_diag[k];
        const double nr = (dr * x - di * y) * f;
        const double ni = (dr * y + di * x) * f;
        dr = nr;
        di = ni;
    }
    double pr = 0.0, pi = 0.0;  // n - 2
    double cr = dr, ci = di;    // n - 1
    re[tri(m, m)] = cr;
    im[tri(m, m)] = ci;
    for (int n = m + 1; n < P_; ++n) {
        const int t = tri(n, m);
        const double a = c_rec_a[t], b = c_rec_b[t] * r2, c = (2.0 * n - 1.0) * z;
        const double nr = (c * cr - b * pr) * a;
        const double ni = (c * ci - b * pi) * a;
        pr = cr;
        pi = ci;
        cr = nr;
        ci = ni;
        re[t] = cr;
        im[t] = ci;
    }
}

constexpr int kChunk = 16;  // points per harmonic chunk in P2M / L2P

// P2M: Mt_n^m = sum_j q_j conj(Rt_n^m(v_j)) + (1/h) conj(mu_j . grad_v Rt_n^m(v_j)),
// v_j = (r_j - c)/h. Gradient in the normalised basis:
//   d/dz Rt_n^m = sqrt((n-m)(n+m)) Rt_{n-1}^m
//   d/dx Rt_n^m = (1/2)[sqrt((n+m)(n+m-1)) Rt_{n-1}^{m-1} - sqrt((n-m)(n-m-1)) Rt_{n-1}^{m+1}]
//   d/dy Rt_n^m = (i/2)[sqrt((n+m)(n+m-1)) Rt_{n-1}^{m-1} + sqrt((n-m)(n-m-1)) Rt_{n-1}^{m+1}]
template <int P_, int NCH, bool MONO, bool DIP>
__global__ void __launch_bounds__(256) k_p2m(int64_t leaf0, const int *leaf_pt, const double *centre,
                                             double h, const double *px, const double *py,
                                             const double *pz, int64_t n, const double *q,
                                             const double *mu, double *mexp) {
    constexpr int NT = P_ * (P_ + 1) / 2;
    constexpr int PP = P_ * P_;
    static_assert(NT <= 256 && kChunk * NCH <= 256, "phase B assumes one thread per coefficient");
    __shared__ double sre[kChunk][NT], sim[kChunk][NT];
    __shared__ double sq[NCH][kChunk], smu[NCH][3][kChunk];
    const int leaf = blockIdx.x;
    const int64_t box = leaf0 + leaf;
    const int r0 = leaf_pt[leaf], r1 = leaf_pt[leaf + 1];
    const double cx = centre[3 * box], cy = centre[3 * box + 1], cz = centre[3 * box + 2];
    const double ih = 1.0 / h;
    const int tid = threadIdx.x;
    // accumulator ownership for phase B: thread tid < NT owns (n, m)
    int own_n = 0, own_m = 0;
    if (tid < NT) {
        int t = tid;
        while (t > own_n) {
            ++own_n;
            t -= own_n;
        }
        own_m = t;
    }
    double ar[NCH], ai[NCH];
    for (int c = 0; c < NCH; ++c) ar[c] = ai[c] = 0.0;
    for (int base = r0; base < r1; base += kChunk) {
        __syncthreads();
        for (int wi = tid; wi < kChunk * P_; wi += blockDim.x) {  // 16 p > 256 when p = 20
            const int pt = wi / P_, m = wi % P_;
            const int i = base + pt;
            if (i < r1) {
                regular_column<P_>(m, (px[i] - cx) * ih, (py[i] - cy) * ih, (pz[i] - cz) * ih,
                                   &sre[pt][0], &sim[pt][0]);
            } else {
                for (int nn = m; nn < P_; ++nn) sre[pt][tri(nn, m)] = sim[pt][tri(nn, m)] = 0.0;
            }
        }
        if (tid < kChunk * NCH) {
            const int pt = tid % kChunk, c = tid / kChunk;
            const int i = base + pt;
            const bool ok = i < r1;
            sq[c][pt] = (MONO && ok) ? q[(int64_t)c * n + i] : 0.0;
            for (int d = 0; d < 3; ++d) smu[c][d][pt] = (DIP && ok) ? mu[((int64_t)c * 3 + d) * n + i] : 0.0;
        }
        __syncthreads();
        if (tid < NT) {
            const int nn = own_n, m = own_m, t = tid;
            const int cnt = (r1 - base) < kChunk ? (r1 - base) : kChunk;
            for (int pt = 0; pt < cnt; ++pt) {
                const double rr = sre[pt][t], ri = sim[pt][t];
                double gxr = 0, gxi = 0, gyr = 0, gyi = 0, gzr = 0, gzi = 0;
                if (DIP && nn > 0) {
                    // R_{n-1}^m, R_{n-1}^{m-1}, R_{n-1}^{m+1}
                    double r0r = 0, r0i = 0, rmr = 0, rmi = 0, rpr = 0, rpi = 0;
                    if (m <= nn - 1) {
                        r0r = sre[pt][tri(nn - 1, m)];
                        r0i = sim[pt][tri(nn - 1, m)];
                    }
                    if (m >= 1) {
                        rmr = sre[pt][tri(nn - 1, m - 1)];
                        rmi = sim[pt][tri(nn - 1, m - 1)];
                    } else if (nn - 1 >= 1) {  // R^{-1} = -conj(R^{1})
                        rmr = -sre[pt][tri(nn - 1, 1)];
                        rmi = sim[pt][tri(nn - 1, 1)];
                    }
                    if (m + 1 <= nn - 1) {
                        rpr = sre[pt][tri(nn - 1, m + 1)];
                        rpi = sim[pt][tri(nn - 1, m + 1)];
                    }
                    const double fz = c_dz[t], fp = 0.5 * c_dp[t], fm = 0.5 * c_dm[t];
                    gzr = fz * r0r;
                    gzi = fz * r0i;
                    gxr = fp * rmr - fm * rpr;
                    gxi = fp * rmi - fm * rpi;
                    // i * (fp * Rm + fm * Rp)
                    gyr = -(fp * rmi + fm * rpi);
                    gyi = fp * rmr + fm * rpr;
                }
                for (int c = 0; c < NCH; ++c) {
                    if (MONO) {
                        const double qq = sq[c][pt];
                        ar[c] += qq * rr;
                        ai[c] -= qq * ri;  // conj
                    }
                    if (DIP) {
                        const double mx = smu[c][0][pt], my = smu[c][1][pt], mz = smu[c][2][pt];
                        const double dr = mx * gxr + my * gyr + mz * gzr;
                        const double di = mx * gxi + my * gyi + mz * gzi;
                        ar[c] += dr * ih;
                        ai[c] -= di * ih;
                    }
                }
            }
        }
    }
    if (tid < NT) {
        for (int c = 0; c < NCH; ++c) {
            double *out = mexp + (box * NCH + c) * PP;
            if (own_m == 0) {
                out[own_n * own_n] = ar[c];
            } else {
                out[own_n * own_n + 2 * own_m - 1] = ar[c];
                out[own_n * own_n + 2 * own_m] = ai[c];
            }
        }
    }
}

// L2P: y_i += (1/h) sum_n [Lt_n^0 Rt_n^0 + 2 sum_{m>0} Re(Lt_n^m Rt_n^m)]
template <int P_, int NCH>
__global__ void __launch_bounds__(256) k_l2p(int64_t leaf0, const int *leaf_pt, const double *centre,
                                             double h, const double *px, const double *py,
                                             const double *pz, int64_t n, const double *lexp,
                                             double *y) {
    constexpr int NT = P_ * (P_ + 1) / 2;
    constexpr int PP = P_ * P_;
    constexpr int NTP = NT + 1;  // padded row
    __shared__ double sre[kChunk][NTP], sim[kChunk][NTP];
    __shared__ double sl[NCH][PP];
    const int leaf = blockIdx.x;
    const int64_t box = leaf0 + leaf;
    const int r0 = leaf_pt[leaf], r1 = leaf_pt[leaf + 1];
    const double cx = centre[3 * box], cy = centre[3 * box + 1], cz = centre[3 * box + 2];
    const double ih = 1.0 / h;
    const int tid = threadIdx.x;
    for (int k = tid; k < NCH * PP; k += blockDim.x) (&sl[0][0])[k] = lexp[box * NCH * PP + k];
    for (int base = r0; base < r1; base += kChunk) {
        __syncthreads();
        for (int wi = tid; wi < kChunk * P_; wi += blockDim.x) {
            const int pt = wi / P_, m = wi % P_;
            const int i = base + pt;
            if (i < r1)
                regular_column<P_>(m, (px[i] - cx) * ih, (py[i] - cy) * ih, (pz[i] - cz) * ih,
                                   &sre[pt][0], &sim[pt][0]);
        }
        __syncthreads();
        // 16 points x 16 partial sums per channel
        const int pt = tid >> 4, part = tid & 15;
        const int i = base + pt;
        for (int c = 0; c < NCH; ++c) {
            double acc = 0.0;
            if (i < r1) {
                for (int t = part; t < NT; t += 16) {
                    // decode (n, m) of t
                    int nn = 0, tt = t;
                    while (tt > nn) {
                        ++nn;
                        tt -= nn;
                    }
                    const int m = tt;
                    const double rr = sre[pt][t], ri = sim[pt][t];
                    if (m == 0) {
                        acc += sl[c][nn * nn] * rr;
                    } else {
                        acc += 2.0 * (sl[c][nn * nn + 2 * m - 1] * rr - sl[c][nn * nn + 2 * m] * ri);
                    }
                }
            }
            for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
            if (part == 0 && i < r1) y[(int64_t)c * n + i] += acc * ih;
        }
    }
}

// ---------------------------------------------------------------------------
// Grouped translation GEMM (FP64 MFMA). Wave g handles 16 columns of the
// column space of its operator group: column = task * nch + channel.
// KIND only separates the kernel symbols of M2L (0) and M2M/L2L (1) for
// profilers; the code is the same.
template <int PP, int KIND>
__global__ void __launch_bounds__(256) k_translate(int nops, const int *tile_off, int ntiles,
                                                   const int *op_off, const int *tsrc, const int *tdst,
                                                   int nch, int swap, const double *T,
                                                   const double *in, double *out) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = blockIdx.x * 4 + wave;
    if (g >= ntiles) return;
    int lo = 0, hi = nops;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tile_off[mid] <= g)
            lo = mid;
        else
            hi = mid;
    }
    const int op = lo;
    const int t0 = op_off[op];
    const int ncols = (op_off[op + 1] - t0) * nch;
    const int col = (g - tile_off[op]) * 16 + (lane & 15);
    const bool valid = col < ncols;
    const int task = t0 + (valid ? col / nch : 0);
    const int ch = valid ? col % nch : 0;
    const int sb = valid ? (swap ? tdst[task] : tsrc[task]) : 0;
    const int db = valid ? (swap ? tsrc[task] : tdst[task]) : 0;
    const double *bcol = in + ((int64_t)sb * nch + ch) * PP;
    const double *A = T + (int64_t)op * PP * PP + (lane & 15);
    const int kq = lane >> 4;
    dbl4 acc[PP / 16];
#pragma unroll
    for (int rb = 0; rb < PP / 16; ++rb) acc[rb] = dbl4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < PP; k0 += 4) {
        const double b = valid ? bcol[k0 + kq] : 0.0;
        const double *Ak = A + (int64_t)(k0 + kq) * PP;
#pragma unroll
        for (int rb = 0; rb < PP / 16; ++rb) {
            const double a = Ak[rb * 16];
            acc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[rb], 0, 0, 0);
        }
    }
    if (!valid) return;
    // result layout of v_mfma_f64_16x16x4f64: lane l, element r holds
    // row (l / 16) + 4 r, column l % 16 of the 16 x 16 block
    double *dcol = out + ((int64_t)db * nch + ch) * PP + kq;
#pragma unroll
    for (int rb = 0; rb < PP / 16; ++rb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) unsafeAtomicAdd(dcol + rb * 16 + 4 * r, acc[rb][r]);
    }
}

// ---------------------------------------------------------------------------
// Near field. 1/sqrt in FP64: hardware estimate refined by two Newton steps
// y <- y (3 - x y^2) / 2 (each step squares the relative error).
__device__ inline double rsqrt_f64(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = y * (1.5 - 0.5 * x * y * y);
    y = y * (1.5 - 0.5 * x * y * y);
    return y;
}

constexpr int kP2PThreads = 128;

template <int NCH, bool MONO, bool DIP>
struct SrcTile {
    double x[kP2PThreads], y[kP2PThreads], z[kP2PThreads];
    double q[MONO ? NCH : 1][kP2PThreads];
    double mx[DIP ? NCH : 1][kP2PThreads], my[DIP ? NCH : 1][kP2PThreads],
        mz[DIP ? NCH : 1][kP2PThreads];
};

template <int NCH, bool MONO, bool DIP>
__device__ inline void load_source(SrcTile<NCH, MONO, DIP> &s, int slot, int64_t j, const double *px,
                                   const double *py, const double *pz, int64_t n, const double *q,
                                   const double *mu) {
    s.x[slot] = px[j];
    s.y[slot] = py[j];
    s.z[slot] = pz[j];
    for (int c = 0; c < NCH; ++c) {
        if (MONO) s.q[c][slot] = q[(int64_t)c * n + j];
        if (DIP) {
            s.mx[c][slot] = mu[((int64_t)c * 3 + 0) * n + j];
            s.my[c][slot] = mu[((int64_t)c * 3 + 1) * n + j];
            s.mz[c][slot] = mu[((int64_t)c * 3 + 2) * n + j];
        }
    }
}

template <int NCH, bool MONO, bool DIP>
__device__ inline void interact(const SrcTile<NCH, MONO, DIP> &s, int cnt, double xi, double yi,
                                double zi, double *acc) {
    for (int jj = 0; jj < cnt; ++jj) {
        const double dx = xi - s.x[jj], dy = yi - s.y[jj], dz = zi - s.z[jj];
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double inv = (r2 > 0.0) ? rsqrt_f64(r2) : 0.0;  // j == i excluded
        const double inv3 = inv * inv * inv;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            if (MONO) acc[c] += s.q[c][jj] * inv;
            if (DIP) acc[c] += (s.mx[c][jj] * dx + s.my[c][jj] * dy + s.mz[c][jj] * dz) * inv3;
        }
    }
}

// One block per target leaf; sources = points of the (up to 27) existing
// neighbour leaves, merged into contiguous ranges and streamed through LDS.
template <int NCH, bool MONO, bool DIP>
__global__ void __launch_bounds__(kP2PThreads) k_p2p(int64_t leaf0, const int *leaf_pt, const int *nbr,
                                                     const double *px, const double *py,
                                                     const double *pz, int64_t n, const double *q,
                                                     const double *mu, double *y) {
    __shared__ SrcTile<NCH, MONO, DIP> s;
    __shared__ int rs[28], re[28], roff[29], nr;
    const int leaf = blockIdx.x;
    const int64_t box = leaf0 + leaf;
    const int tid = threadIdx.x;
    if (tid == 0) {
        // gather ranges, sort by start, merge contiguous ones
        int a[27], b[27], k = 0;
        for (int sl = 0; sl < 27; ++sl) {
            const int qb = nbr[27 * box + sl];
            if (qb < 0) continue;
            const int64_t li = qb - leaf0;
            a[k] = leaf_pt[li];
            b[k] = leaf_pt[li + 1];
            ++k;
        }
        for (int i = 1; i < k; ++i) {
            int va = a[i], vb = b[i], j = i - 1;
            while (j >= 0 && a[j] > va) {
                a[j + 1] = a[j];
                b[j + 1] = b[j];
                --j;
            }
            a[j + 1] = va;
            b[j + 1] = vb;
        }
        int m = 0;
        for (int i = 0; i < k; ++i) {
            if (m > 0 && re[m - 1] == a[i]) {
                re[m - 1] = b[i];
            } else {
                rs[m] = a[i];
                re[m] = b[i];
                ++m;
            }
        }
        roff[0] = 0;
        for (int i = 0; i < m; ++i) roff[i + 1] = roff[i] + (re[i] - rs[i]);
        nr = m;
    }
    __syncthreads();
    const int total = roff[nr];
    const int r0 = leaf_pt[leaf], r1 = leaf_pt[leaf + 1];
    for (int rc = r0; rc < r1; rc += kP2PThreads) {
        const int i = rc + tid;
        const bool ok = i < r1;
        const double xi = ok ? px[i] : 0.0, yi = ok ? py[i] : 0.0, zi = ok ? pz[i] : 0.0;
        double acc[NCH];
        for (int c = 0; c < NCH; ++c) acc[c] = 0.0;
        for (int t0 = 0; t0 < total; t0 += kP2PThreads) {
            __syncthreads();
            const int f = t0 + tid;
            if (f < total) {
                int r = 0;
                while (roff[r + 1] <= f) ++r;
                load_source(s, tid, (int64_t)rs[r] + (f - roff[r]), px, py, pz, n, q, mu);
            }
            __syncthreads();
            const int cnt = (total - t0) < kP2PThreads ? (total - t0) : kP2PThreads;
            interact(s, cnt, xi, yi, zi, acc);
        }
        if (ok)
            for (int c = 0; c < NCH; ++c) y[(int64_t)c * n + i] = acc[c];
    }
}

// All-pairs sum (checking path): block of receivers x every source.
template <int NCH, bool MONO, bool DIP>
__global__ void __launch_bounds__(kP2PThreads) k_direct(const double *px, const double *py,
                                                        const double *pz, int64_t n, const double *q,
                                                        const double *mu, double *y) {
    __shared__ SrcTile<NCH, MONO, DIP> s;
    const int tid = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * kP2PThreads + tid;
    const bool ok = i < n;
    const double xi = ok ? px[i] : 0.0, yi = ok ? py[i] : 0.0, zi = ok ? pz[i] : 0.0;
    double acc[NCH];
    for (int c = 0; c < NCH; ++c) acc[c] = 0.0;
    for (int64_t t0 = 0; t0 < n; t0 += kP2PThreads) {
        __syncthreads();
        if (t0 + tid < n) load_source(s, tid, t0 + tid, px, py, pz, n, q, mu);
        __syncthreads();
        const int cnt = (n - t0) < kP2PThreads ? (int)(n - t0) : kP2PThreads;
        interact(s, cnt, xi, yi, zi, acc);
    }
    if (ok)
        for (int c = 0; c < NCH; ++c) y[(int64_t)c * n + i] = acc[c];
}

__global__ void k_zero(double *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// ---------------------------------------------------------------------------
// Host side

void fmm_prepare_ops(FmmWork &w, int p, hipStream_t st) {
    int dev = 0;
    BFM_HIP(hipGetDevice(&dev));
    upload_tables(dev);
    if (w.ops_p == p) return;
    const int P = p * p;
    std::vector<double> rm((size_t)P * P), cm((size_t)P * P);
    auto to_cm = [&](double *dst) {
        for (int r = 0; r < P; ++r)
            for (int c = 0; c < P; ++c) dst[(size_t)c * P + r] = rm[(size_t)r * P + c];
    };
    std::vector<double> h2m((size_t)8 * P * P), h2l((size_t)8 * P * P);
    for (int o = 0; o < 8; ++o) {
        build_m2m(p, o, rm.data());
        to_cm(&h2m[(size_t)o * P * P]);
        build_l2l(p, o, rm.data());
        to_cm(&h2l[(size_t)o * P * P]);
    }
    // the 316 multipole-to-local operators are the bulk of the work: build
    // them once per process and order p
    static std::vector<double> cache_l[kMaxP + 1];
    std::vector<double> &hl = cache_l[p];
    if (hl.empty()) {
        std::vector<double> tmp((size_t)kNumM2LOps * P * P);
#pragma omp parallel for schedule(dynamic)
        for (int o = 0; o < kNumM2LOps; ++o) {
            std::vector<double> r((size_t)P * P);
            build_m2l(p, o, r.data());
            for (int a = 0; a < P; ++a)
                for (int b = 0; b < P; ++b) tmp[(size_t)o * P * P + (size_t)b * P + a] = r[(size_t)a * P + b];
        }
        hl.swap(tmp);
    }
    w.ops_m2m.ensure(h2m.size());
    w.ops_l2l.ensure(h2l.size());
    w.ops_m2l.ensure(hl.size());
    BFM_HIP(hipMemcpyAsync(w.ops_m2m.get(), h2m.data(), sizeof(double) * h2m.size(), hipMemcpyHostToDevice, st));
    BFM_HIP(hipMemcpyAsync(w.ops_l2l.get(), h2l.data(), sizeof(double) * h2l.size(), hipMemcpyHostToDevice, st));
    BFM_HIP(hipMemcpyAsync(w.ops_m2l.get(), hl.data(), sizeof(double) * hl.size(), hipMemcpyHostToDevice, st));
    BFM_HIP(hipStreamSynchronize(st));
    w.ops_p = p;
}

static unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Algorithmic flops of one source-receiver pair: shared geometry 3 (d) + 5
// (r^2) + 1 (1/r) [+ 2 for 1/r^3 with dipoles]; per channel 2 (q/r) and
// 7 (mu . d / r^3: 5 for the dot product, 2 for the scaled add).
static double p2p_flops_per_pair(int nch, bool mono, bool dip) {
    return 9.0 + (dip ? 2.0 : 0.0) + nch * ((mono ? 2.0 : 0.0) + (dip ? 7.0 : 0.0));
}

static int prof_begin(FmmWork &w, int cls, hipStream_t st) { return w.prof ? w.prof->begin(cls, st) : -1; }
static void prof_end(FmmWork &w, int idx, hipStream_t st, double flops) {
    if (w.prof) w.prof->end(idx, st, flops, 0.0);
}

template <int P_>
static void translate(FmmWork &w, int cls, TaskList &tl, int nch, bool swap, const double *T,
                      const double *in, double *out, hipStream_t st) {
    prepare_tiles(tl, nch, st);
    const int nt = tl.ntiles[nch];
    if (nt <= 0) return;
    const int pi = prof_begin(w, cls, st);
    auto kern = (cls == KC_M2L) ? k_translate<P_ * P_, 0> : k_translate<P_ * P_, 1>;
    kern<<<nblk(nt, 4), 256, 0, st>>>(tl.nops, tl.tile_off[nch].get(), nt,
                                                       tl.op_off.get(), tl.src.get(), tl.dst.get(),
                                                       nch, swap ? 1 : 0, T, in, out);
    BFM_LAUNCHED();
    const double PP = (double)P_ * P_;
    prof_end(w, pi, st, 2.0 * PP * PP * (double)tl.ntasks * nch);
}

template <int P_, int NCH, bool MONO, bool DIP>
static void run_fmm(FmmWork &w, const Tree &tc, const Sources &src, double *y, hipStream_t st) {
    Tree &t = const_cast<Tree &>(tc);
    constexpr int PP = P_ * P_;
    const int lmax = t.lmax;
    const int64_t leaf0 = t.lvl_off[lmax];
    const double hleaf = t.side / (double)(1 << lmax);
    const size_t ncoef = (size_t)t.nbox * NCH * PP;
    double *M = w.mexp.ensure(ncoef);
    double *L = w.lexp.ensure(ncoef);
    k_zero<<<1024, 256, 0, st>>>(M, (int64_t)ncoef);
    BFM_LAUNCHED();
    k_zero<<<1024, 256, 0, st>>>(L, (int64_t)ncoef);
    BFM_LAUNCHED();
    // near field first (writes y), far field adds
    int pi = prof_begin(w, KC_P2P, st);
    k_p2p<NCH, MONO, DIP><<<(unsigned)t.nleaf, kP2PThreads, 0, st>>>(
        leaf0, t.leaf_pt.get(), t.nbr.get(), t.px.get(), t.py.get(), t.pz.get(), t.n, src.q, src.mu, y);
    BFM_LAUNCHED();
    prof_end(w, pi, st, (double)(t.npairs_near - t.n) * p2p_flops_per_pair(NCH, MONO, DIP));
    pi = prof_begin(w, KC_P2M, st);
    k_p2m<P_, NCH, MONO, DIP><<<(unsigned)t.nleaf, 256, 0, st>>>(
        leaf0, t.leaf_pt.get(), t.box_centre.get(), hleaf, t.px.get(), t.py.get(), t.pz.get(), t.n,
        src.q, src.mu, M);
    BFM_LAUNCHED();
    prof_end(w, pi, st, 0.0);
    for (int l = lmax; l >= 3; --l)
        translate<P_>(w, KC_M2M_L2L, *t.m2m[l], NCH, false, w.ops_m2m.get(), M, M, st);
    translate<P_>(w, KC_M2L, t.m2l, NCH, false, w.ops_m2l.get(), M, L, st);
    for (int l = 3; l <= lmax; ++l)
        translate<P_>(w, KC_M2M_L2L, *t.m2m[l], NCH, true, w.ops_l2l.get(), L, L, st);
    pi = prof_begin(w, KC_L2P, st);
    k_l2p<P_, NCH><<<(unsigned)t.nleaf, 256, 0, st>>>(leaf0, t.leaf_pt.get(), t.box_centre.get(), hleaf,
                                                      t.px.get(), t.py.get(), t.pz.get(), t.n, L, y);
    BFM_LAUNCHED();
    prof_end(w, pi, st, 0.0);
}

template <int NCH, bool MONO, bool DIP>
static void run_direct(const Tree &t, const Sources &src, double *y, hipStream_t st) {
    k_direct<NCH, MONO, DIP><<<nblk(t.n, kP2PThreads), kP2PThreads, 0, st>>>(
        t.px.get(), t.py.get(), t.pz.get(), t.n, src.q, src.mu, y);
    BFM_LAUNCHED();
}

template <int NCH, bool MONO, bool DIP>
static void dispatch_p(FmmWork &w, const Tree &t, const Sources &src, double *y, bool direct,
                       hipStream_t st) {
    if (direct) return run_direct<NCH, MONO, DIP>(t, src, y, st);
    switch (w.p) {
        case 4: return run_fmm<4, NCH, MONO, DIP>(w, t, src, y, st);
        case 8: return run_fmm<8, NCH, MONO, DIP>(w, t, src, y, st);
        case 12: return run_fmm<12, NCH, MONO, DIP>(w, t, src, y, st);
        case 16: return run_fmm<16, NCH, MONO, DIP>(w, t, src, y, st);
        case 20: return run_fmm<20, NCH, MONO, DIP>(w, t, src, y, st);
        default: fail(BFM_EUNSUPPORTED, "expansion order p must be one of 4, 8, 12, 16, 20");
    }
}

void fmm_apply(FmmWork &w, const Tree &t, const Sources &src, double *y, bool direct, hipStream_t st) {
    BFM_CHECK(t.valid, BFM_EINVAL, "octree not built");
    if (!direct) BFM_CHECK(w.ops_p == w.p && w.p > 0, BFM_EINVAL, "translation operators not prepared");
    if (src.nch == 1 && src.mono && !src.dip) return dispatch_p<1, true, false>(w, t, src, y, direct, st);
    if (src.nch == 1 && !src.mono && src.dip) return dispatch_p<1, false, true>(w, t, src, y, direct, st);
    if (src.nch == 1 && src.mono && src.dip) return dispatch_p<1, true, true>(w, t, src, y, direct, st);
    if (src.nch == 5 && src.mono && src.dip) return dispatch_p<5, true, true>(w, t, src, y, direct, st);
    fail(BFM_EUNSUPPORTED, "unsupported source channel combination");
}

}  // namespace bfm
