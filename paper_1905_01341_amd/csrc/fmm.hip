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
// P2M. One wave per leaf; lane l takes the leaf's points l, l + 64, ... and
// evaluates the regular harmonics of its point in registers, order by order
// (the loops over order m and degree k are uniform across the wave and fully
// unrolled, so every coefficient has a fixed register slot); every kCS slots
// the wave's 64 values per slot are summed through LDS (transposed: lane t
// adds up slot t) into the leaf's running totals.
//   Mt_n^m += q_j conj(Rt_n^m(v_j)) + (w_j / h) conj(n_j . grad_v Rt_n^m(v_j)),
// v_j = (r_j - c)/h. The directional derivative D = n_j . grad_v follows the
// same recurrence by forward differentiation:
//   D Rt_m^m = [D Rt_{m-1}^{m-1} (x+iy) + Rt_{m-1}^{m-1} (n_x+i n_y)] f_m
//   D Rt_n^m = [(2n-1)(n_z Rt_{n-1} + z D Rt_{n-1}) - b (2 v.n Rt_{n-2} + r^2 D Rt_{n-2})] a
// Slots run over m, then degree k >= m, then (real, imaginary) for m > 0.
constexpr int kCS = 32;

__host__ __device__ constexpr int p2m_slot(int P, int m, int k) {
    return m == 0 ? k : P + (m - 1) * (2 * P - m) + 2 * (k - m);
}

// slot -> index in the packed expansion layout
__device__ inline int p2m_slot_out(int P, int s) {
    if (s < P) return s * s;
    s -= P;
    for (int m = 1; m < P; ++m) {
        const int cnt = 2 * (P - m);
        if (s < cnt) {
            const int k = m + s / 2;
            return k * k + 2 * m - 1 + (s & 1);
        }
        s -= cnt;
    }
    return 0;
}

template <int PP>
__device__ inline void p2m_put(int s, double v, double (&acc)[kCS], double (*red)[65], double *tot, int lane) {
    acc[s % kCS] = v;
    if (s % kCS == kCS - 1 || s == PP - 1) {
        const int base = s - s % kCS, cnt = s % kCS + 1;
#pragma unroll
        for (int t = 0; t < kCS; ++t)
            if (t < cnt) red[t][lane] = acc[t];
        __syncthreads();
        if (lane < cnt) {
            double sum = 0.0;
#pragma unroll 16
            for (int l = 0; l < 64; ++l) sum += red[lane][l];
            tot[base + lane] += sum;
        }
        __syncthreads();
    }
}

template <int P_, int NCH, bool MONO, bool DIP>
__global__ void __launch_bounds__(64) k_p2m(int64_t leaf0, const int *leaf_pt, const double *centre,
                                            double h, const double *px, const double *py,
                                            const double *pz, const double *pnx, const double *pny,
                                            const double *pnz, int64_t n, const double *q,
                                            const double *w, double *mexp) {
    constexpr int PP = P_ * P_;
    __shared__ double red[kCS][65];
    __shared__ double tot[PP];
    const int lane = threadIdx.x;
    const int leaf = blockIdx.x;
    const int64_t box = leaf0 + leaf;
    const int r0 = leaf_pt[leaf], r1 = leaf_pt[leaf + 1];
    const double cx = centre[3 * box], cy = centre[3 * box + 1], cz = centre[3 * box + 2];
    const double ih = 1.0 / h;
    for (int c = 0; c < NCH; ++c) {
        for (int t = lane; t < PP; t += 64) tot[t] = 0.0;
        for (int j0 = r0; j0 < r1; j0 += 64) {
            const int j = j0 + lane;
            const bool ok = j < r1;
            // idle lanes: a point at the centre with zero strength
            const double x = ok ? (px[j] - cx) * ih : 0.0, y = ok ? (py[j] - cy) * ih : 0.0,
                         z = ok ? (pz[j] - cz) * ih : 0.0;
            const double r2 = x * x + y * y + z * z;
            const double qq = (MONO && ok) ? q[(int64_t)c * n + j] : 0.0;
            double ux = 0.0, uy = 0.0, uz = 0.0, ww = 0.0, vu = 0.0;
            if (DIP && ok) {
                ux = pnx[j];
                uy = pny[j];
                uz = pnz[j];
                ww = w[(int64_t)c * n + j] * ih;
                vu = x * ux + y * uy + z * uz;
            }
            double acc[kCS];
            double dr = 1.0, di = 0.0, Ddr = 0.0, Ddi = 0.0;  // Rt_m^m and its derivative
#pragma unroll
            for (int m = 0; m < P_; ++m) {
                if (m > 0) {
                    const double f = c_diag[m];
                    const double nr = (dr * x - di * y) * f, ni = (dr * y + di * x) * f;
                    if (DIP) {
                        const double nDr = (Ddr * x - Ddi * y + dr * ux - di * uy) * f;
                        const double nDi = (Ddr * y + Ddi * x + dr * uy + di * ux) * f;
                        Ddr = nDr;
                        Ddi = nDi;
                    }
                    dr = nr;
                    di = ni;
                }
                double cr = dr, ci = di, Dcr = Ddr, Dci = Ddi;     // degree k
                double pr = 0.0, pi = 0.0, Dpr = 0.0, Dpi = 0.0;  // degree k - 1
#pragma unroll
                for (int k = m; k < P_; ++k) {
                    if (k > m) {
                        const int t = tri(k, m);
                        const double a = c_rec_a[t], b = c_rec_b[t], e = (2.0 * k - 1.0);
                        const double nr = (e * z * cr - b * r2 * pr) * a;
                        const double ni = (e * z * ci - b * r2 * pi) * a;
                        if (DIP) {
                            const double nDr = (e * (uz * cr + z * Dcr) - b * (2.0 * vu * pr + r2 * Dpr)) * a;
                            const double nDi = (e * (uz * ci + z * Dci) - b * (2.0 * vu * pi + r2 * Dpi)) * a;
                            Dpr = Dcr;
                            Dpi = Dci;
                            Dcr = nDr;
                            Dci = nDi;
                        }
                        pr = cr;
                        pi = ci;
                        cr = nr;
                        ci = ni;
                    }
                    const int s = p2m_slot(P_, m, k);
                    p2m_put<PP>(s, qq * cr + ww * Dcr, acc, red, tot, lane);
                    if (m > 0) p2m_put<PP>(s + 1, -(qq * ci + ww * Dci), acc, red, tot, lane);  // conjugate
                }
            }
        }
        __syncthreads();
        double *out = mexp + (box * NCH + c) * PP;
        for (int t = lane; t < PP; t += 64) out[p2m_slot_out(P_, t)] = tot[t];
        __syncthreads();
    }
}

// L2P, one thread per point: y_i += (1/h) sum_n [Lt_n^0 Rt_n^0 + 2 sum_{m>0}
// Re(Lt_n^m Rt_n^m)], the harmonics built in registers order by order (the
// order and degree are the same for every lane, so the loop is uniform).
template <int P_, int NCH>
__global__ void __launch_bounds__(256) k_l2p(int64_t leaf0, const int *pt_leaf, const double *centre,
                                             double h, const double *px, const double *py,
                                             const double *pz, int64_t n, const double *lexp,
                                             double *y) {
    constexpr int PP = P_ * P_;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t box = leaf0 + pt_leaf[i];
    const double ih = 1.0 / h;
    const double x = (px[i] - centre[3 * box]) * ih, yy = (py[i] - centre[3 * box + 1]) * ih,
                 z = (pz[i] - centre[3 * box + 2]) * ih;
    const double r2 = x * x + yy * yy + z * z;
    const double *L = lexp + box * NCH * PP;
    double acc[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) acc[c] = 0.0;
    double dr = 1.0, di = 0.0;
#pragma unroll 1
    for (int m = 0; m < P_; ++m) {
        if (m > 0) {
            const double f = c_diag[m];
            const double nr = (dr * x - di * yy) * f, ni = (dr * yy + di * x) * f;
            dr = nr;
            di = ni;
        }
        double cr = dr, ci = di, pr = 0.0, pi = 0.0;
        const double wgt = (m == 0) ? 1.0 : 2.0;
        const int im = (m == 0) ? 0 : 2 * m - 1;  // offset of the real part within degree k
#pragma unroll 2
        for (int k = m; k < P_; ++k) {
            if (k > m) {
                const int t = tri(k, m);
                const double a = c_rec_a[t], b = c_rec_b[t], e = (2.0 * k - 1.0);
                const double nr = (e * z * cr - b * r2 * pr) * a;
                const double ni = (e * z * ci - b * r2 * pi) * a;
                pr = cr;
                pi = ci;
                cr = nr;
                ci = ni;
            }
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const double *Lc = L + c * PP + k * k + im;
                const double lim = (m == 0) ? 0.0 : Lc[1];
                acc[c] += wgt * (Lc[0] * cr - lim * ci);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < NCH; ++c) y[(int64_t)c * n + i] += acc[c] * ih;
}

// ---------------------------------------------------------------------------
// Grouped translation GEMM (FP64 MFMA). A workgroup of WAVES waves owns
// WAVES x 16 columns (task x channel) of one operator's group and a slab of
// ROWS output rows; the operator slab is streamed through LDS in chunks of 16
// input coefficients and shared by all waves; each wave multiplies it by its
// 16 gathered expansion columns. The operands are passed transposed
// (D = in^T T^T), so lane l, element r of a result block holds column
// l/16 + 4r and row l%16: each quarter-wave adds 16 contiguous coefficients
// of one target expansion. Wide tiles (many waves, all rows) cut operator
// re-reads when groups are large; row slabs give parallelism when groups are
// small (coarse octree levels). KIND only separates the kernel symbols of
// M2L (0) and M2M/L2L (1) for profilers.
constexpr int kTKC = 16;
constexpr int kXcds = 8;  // accelerator complex dies of an MI355X

template <int PP, int ROWS, int WAVES, int KIND>
__global__ void __launch_bounds__(64 * WAVES) k_translate(int nops, const int *tile_off, int ntiles,
                                                          const int *op_off, const int *tsrc,
                                                          const int *tdst, int nch, int swap,
                                                          const double *T, const double *in,
                                                          double *out) {
    static_assert(PP % ROWS == 0 && ROWS % 16 == 0, "row slab");
    constexpr int NSLAB = PP / ROWS;
    __shared__ double As[2][kTKC * ROWS];  // two buffers of [k][row within slab]
    // XCD-aware order: workgroups are dealt round-robin to the 8 XCDs, so
    // XCD x takes a contiguous run of logical blocks (the tiles of a few
    // operators) and fetches each operator into its own L2 once
    const int nblock = gridDim.x, per = nblock / kXcds, rem = nblock % kXcds;
    const int xcd = blockIdx.x % kXcds, idx = blockIdx.x / kXcds;
    const int logical = xcd * per + (xcd < rem ? xcd : rem) + idx;
    const int g = logical / NSLAB, slab = logical % NSLAB;
    if (g >= ntiles) return;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
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
    const int colbase = (g - tile_off[op]) * (16 * WAVES) + wave * 16;
    const int bcolid = colbase + (lane & 15);
    const bool bok = bcolid < ncols;
    const int btask = t0 + (bok ? bcolid / nch : 0);
    const int bch = bok ? bcolid % nch : 0;
    const int sb = bok ? (swap ? tdst[btask] : tsrc[btask]) : 0;
    const double *bcol = in + ((int64_t)sb * nch + bch) * PP;
    const double *Top = T + (int64_t)op * PP * PP + slab * ROWS;
    const int kq = lane >> 4, rl = lane & 15;
    dbl4 acc[ROWS / 16];
#pragma unroll
    for (int rb = 0; rb < ROWS / 16; ++rb) acc[rb] = dbl4{0.0, 0.0, 0.0, 0.0};
    // double-buffered operator slab: the next chunk is fetched into
    // registers while the current one feeds the MFMAs from LDS
    constexpr int NT = 64 * WAVES;
    constexpr int PER = (kTKC * ROWS + NT - 1) / NT;
    double pre[PER];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + u * NT;
            if (e < kTKC * ROWS) {
                const int kk = e / ROWS, rr = e % ROWS;
                pre[u] = Top[(int64_t)(k0 + kk) * PP + rr];
            }
        }
    };
    auto stash = [&](double *dst) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + u * NT;
            if (e < kTKC * ROWS) dst[e] = pre[u];
        }
    };
    fetch(0);
    stash(As[0]);
    // the wave's input columns are prefetched one chunk ahead as well
    double bv[kTKC / 4], bn[kTKC / 4];
#pragma unroll
    for (int kk = 0; kk < kTKC / 4; ++kk) bv[kk] = bok ? bcol[4 * kk + kq] : 0.0;
    __syncthreads();
    int cur = 0;
    for (int k0 = 0; k0 < PP; k0 += kTKC) {
        const bool more = k0 + kTKC < PP;
        if (more) {
            fetch(k0 + kTKC);
#pragma unroll
            for (int kk = 0; kk < kTKC / 4; ++kk) bn[kk] = bok ? bcol[k0 + kTKC + 4 * kk + kq] : 0.0;
        }
#pragma unroll
        for (int kk = 0; kk < kTKC / 4; ++kk) {
            const double *Ak = As[cur] + (4 * kk + kq) * ROWS + rl;
#pragma unroll
            for (int rb = 0; rb < ROWS / 16; ++rb)
                acc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[kk], Ak[rb * 16], acc[rb], 0, 0, 0);
        }
        if (more) {
            stash(As[cur ^ 1]);
            __syncthreads();
            cur ^= 1;
#pragma unroll
            for (int kk = 0; kk < kTKC / 4; ++kk) bv[kk] = bn[kk];
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int col = colbase + kq + 4 * r;
        if (col >= ncols) continue;
        const int task = t0 + col / nch, ch = col % nch;
        const int db = swap ? tsrc[task] : tdst[task];
        double *dcol = out + ((int64_t)db * nch + ch) * PP + slab * ROWS + rl;
#pragma unroll
        for (int rb = 0; rb < ROWS / 16; ++rb) unsafeAtomicAdd(dcol + rb * 16, acc[rb][r]);
    }
}

// ---------------------------------------------------------------------------
// Near field. 1/sqrt in FP64: the hardware estimate (relative error about
// 5e-8) refined by one Newton step with an FMA-formed residual.
__device__ inline double rsqrt_f64(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

constexpr int kP2PThreads = 64;

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

template <int NCH, bool MONO, bool DIP, int R>
__device__ inline void p2p_pass(int rc, int l0, int r1, int nr, const int2 *__restrict__ rng,
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
    // only the leaf's own points can coincide with a receiver: the merged
    // range holding them is split so that the rest runs without the test
    for (int g = 0; g < nr; ++g) {
        const int2 r = rng[g];
        const int l1 = r1;  // the leaf's points are [l0, r1)
        if (r.x <= l0 && l1 <= r.y) {
            p2p_range<NCH, MONO, DIP, R, false>(r.x, l0, px, py, pz, pnx, pny, pnz, n, q, w, xi, yi, zi, acc);
            p2p_range<NCH, MONO, DIP, R, true>(l0, l1, px, py, pz, pnx, pny, pnz, n, q, w, xi, yi, zi, acc);
            p2p_range<NCH, MONO, DIP, R, false>(l1, r.y, px, py, pz, pnx, pny, pnz, n, q, w, xi, yi, zi, acc);
        } else {
            p2p_range<NCH, MONO, DIP, R, false>(r.x, r.y, px, py, pz, pnx, pny, pnz, n, q, w, xi, yi, zi, acc);
        }
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = rc + lane + k * kP2PThreads;
        if (i < r1)
            for (int c = 0; c < NCH; ++c) y[(int64_t)c * n + i] = acc[k][c];
    }
}

// One wave per near-field work item (a leaf and up to 64 of its receivers,
// items ordered by decreasing pair count); sources = the leaf's merged
// near-field ranges (the points of up to 27 neighbour leaves).
template <int NCH, bool MONO, bool DIP>
__global__ void __launch_bounds__(kP2PThreads) k_p2p(const int2 *__restrict__ items,
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
    const int2 it = items[blockIdx.x];
    const int leaf = it.x, rc = it.y;
    const int r1 = leaf_pt[leaf + 1];
    p2p_pass<NCH, MONO, DIP, R>(rc, leaf_pt[leaf], r1, near_cnt[leaf], near_rng + 27 * (int64_t)leaf, px, py, pz, pnx,
                                pny, pnz, n, q, w, y);
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
// (r^2) + 1 (1/r) [+ 5 for n.d and 3 for n.d / r^3 with dipoles]; per channel
// 2 (q/r) and 2 (w n.d / r^3).
static double p2p_flops_per_pair(int nch, bool mono, bool dip) {
    return 9.0 + (dip ? 8.0 : 0.0) + nch * ((mono ? 2.0 : 0.0) + (dip ? 2.0 : 0.0));
}

static int prof_begin(FmmWork &w, int cls, hipStream_t st) { return w.prof ? w.prof->begin(cls, st) : -1; }
static void prof_end(FmmWork &w, int idx, hipStream_t st, double flops) {
    if (w.prof) w.prof->end(idx, st, flops, 0.0);
}

// Middle row-slab height: a multiple of 16 dividing p^2, at most 80.
constexpr int mid_rows(int PP) { return PP == 144 ? 48 : (PP == 400 ? 80 : (PP >= 64 ? 64 : PP)); }
// Wide-tile slab: every row while the accumulators fit in registers.
constexpr int wide_rows(int PP) { return PP <= 256 ? PP : mid_rows(PP); }

template <int P_>
static void translate(FmmWork &w, int cls, TaskList &tl, int nch, bool swap, const double *T,
                      const double *in, double *out, hipStream_t st) {
    constexpr int PP = P_ * P_;
    const int64_t cols = tl.ntasks * nch;
    // Enough waves for the whole chip: all rows per wave (wide 128-column
    // tiles, fewest operator re-reads) when there are many columns, row slabs
    // (more waves, columns re-read per slab) when there are few.
    const int64_t wave_tiles = (cols + 15) / 16;
    int shape = (wave_tiles >= 8192) ? 0 : (wave_tiles * (PP / mid_rows(PP)) >= 8192 ? 1 : 2);
    if (cls == KC_M2L && w.m2l_shape >= 0) shape = w.m2l_shape;
    const int width = (shape == 0) ? 128 : 64;
    prepare_tiles(tl, nch, width, st);
    const int nt = tl.ntiles_for(nch, width);
    if (nt <= 0) return;
    const int pi = prof_begin(w, cls, st);
    const int *to = tl.tile_for(nch, width);
    const int sw = swap ? 1 : 0;
    if (shape == 0) {
        constexpr int R = wide_rows(PP);
        auto kern = (cls == KC_M2L) ? k_translate<PP, R, 8, 0> : k_translate<PP, R, 8, 1>;
        kern<<<(unsigned)(nt * (PP / R)), 512, 0, st>>>(tl.nops, to, nt, tl.op_off.get(), tl.src.get(),
                                                         tl.dst.get(), nch, sw, T, in, out);
    } else if (shape == 1) {
        constexpr int R = mid_rows(PP);
        auto kern = (cls == KC_M2L) ? k_translate<PP, R, 4, 0> : k_translate<PP, R, 4, 1>;
        kern<<<(unsigned)(nt * (PP / R)), 256, 0, st>>>(tl.nops, to, nt, tl.op_off.get(), tl.src.get(),
                                                         tl.dst.get(), nch, sw, T, in, out);
    } else {
        constexpr int R = 16;
        auto kern = (cls == KC_M2L) ? k_translate<PP, R, 4, 0> : k_translate<PP, R, 4, 1>;
        kern<<<(unsigned)(nt * (PP / R)), 256, 0, st>>>(tl.nops, to, nt, tl.op_off.get(), tl.src.get(),
                                                         tl.dst.get(), nch, sw, T, in, out);
    }
    BFM_LAUNCHED();
    prof_end(w, pi, st, 2.0 * (double)PP * PP * (double)tl.ntasks * nch);
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
    k_p2p<NCH, MONO, DIP><<<(unsigned)t.n_p2p_items, kP2PThreads, 0, st>>>(
        t.p2p_items.get(), t.leaf_pt.get(), t.near_rng.get(), t.near_cnt.get(), t.px.get(), t.py.get(), t.pz.get(),
        t.pnx.get(), t.pny.get(), t.pnz.get(), t.n, src.q, src.w, y);
    BFM_LAUNCHED();
    prof_end(w, pi, st, (double)(t.npairs_near - t.n) * p2p_flops_per_pair(NCH, MONO, DIP));
    pi = prof_begin(w, KC_P2M, st);
    k_p2m<P_, NCH, MONO, DIP><<<(unsigned)t.nleaf, 64, 0, st>>>(
        leaf0, t.leaf_pt.get(), t.box_centre.get(), hleaf, t.px.get(), t.py.get(), t.pz.get(),
        t.pnx.get(), t.pny.get(), t.pnz.get(), t.n, src.q, src.w, M);
    BFM_LAUNCHED();
    prof_end(w, pi, st, 0.0);
    for (int l = lmax; l >= 3; --l)
        translate<P_>(w, KC_M2M_L2L, *t.m2m[l], NCH, false, w.ops_m2m.get(), M, M, st);
    translate<P_>(w, KC_M2L, t.m2l, NCH, false, w.ops_m2l.get(), M, L, st);
    for (int l = 3; l <= lmax; ++l)
        translate<P_>(w, KC_M2M_L2L, *t.m2m[l], NCH, true, w.ops_l2l.get(), L, L, st);
    pi = prof_begin(w, KC_L2P, st);
    k_l2p<P_, NCH><<<nblk(t.n, 256), 256, 0, st>>>(leaf0, t.pt_leaf.get(), t.box_centre.get(), hleaf,
                                                   t.px.get(), t.py.get(), t.pz.get(), t.n, L, y);
    BFM_LAUNCHED();
    prof_end(w, pi, st, 0.0);
}

template <int NCH, bool MONO, bool DIP>
static void run_direct(const Tree &t, const Sources &src, double *y, hipStream_t st) {
    k_direct<NCH, MONO, DIP><<<nblk(t.n, kP2PThreads), kP2PThreads, 0, st>>>(
        t.px.get(), t.py.get(), t.pz.get(), t.pnx.get(), t.pny.get(), t.pnz.get(), t.n, src.q, src.w, y);
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
