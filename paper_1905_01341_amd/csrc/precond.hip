// Per-bubble spherical-harmonic preconditioner for the single-layer system.
//
// On a sphere of radius R the single-layer operator is diagonal in spherical
// harmonics with eigenvalue R/(2n+1) for degree n. Every bubble here is a
// closed surface whose vertices carry the parametrisation of a template unit
// sphere (the (theta, phi) of the initial mesh, as for the paper's shape
// filter, Section 3.7), so an approximate inverse of L restricted to bubble b
// is
//   P_b^{-1} x = (1/R_b) [ c x + G diag(2n+1 - c) G+ x ],   c = 2 (nmax + 1) + 1,
// with G the real harmonics of degree <= nmax sampled at the template
// vertices, G+ = (G^T W G)^{-1} G^T W their weighted least-squares projector
// (W = template vertex areas), and R_b = sqrt(area_b / 4 pi). Degrees above
// nmax get the first unresolved eigenvalue. Applied as a right
// preconditioner inside GMRES, so the residual GMRES monitors is the true
// one and the solution is unchanged.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include <condition_variable>
#include <exception>
#include <mutex>
#include <thread>

#include "ctx.h"

namespace bfm {

static unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Real harmonics of degree 0..nmax at unit vector d, orthonormal on the
// unit sphere and without the Condon-Shortley phase: for each degree n the
// order-0 value, then the cos(m lon) and sin(m lon) parts of orders 1..n.
// The recurrence yields sqrt((n-m)!/(n+m)!) P_n^m(cos theta) e^{i m lon};
// the factor sqrt((2n+1)/4pi) (times sqrt(2) for m > 0) normalises it.
static void sh_row(int nmax, const double d[3], double *row) {
    using cplx = std::complex<double>;
    const double x = d[0], y = d[1], z = d[2];
    const double r2 = x * x + y * y + z * z;
    std::vector<cplx> col(nmax + 1);
    cplx diag(1.0, 0.0);
    for (int m = 0; m <= nmax; ++m) {
        if (m > 0) diag *= cplx(x, y) * std::sqrt((2.0 * m - 1.0) / (2.0 * m));
        cplx pr(0.0, 0.0), cr = diag;
        for (int n = m; n <= nmax; ++n) {
            if (n > m) {
                const double a = std::sqrt((double)(n - m) * (n + m));
                const double b = (n - m - 1 > 0) ? std::sqrt((double)(n - m - 1) * (n + m - 1)) : 0.0;
                const cplx nr = ((2.0 * n - 1.0) * z * cr - r2 * b * pr) / a;
                pr = cr;
                cr = nr;
            }
            const double f = std::sqrt((2.0 * n + 1.0) / (4.0 * 3.14159265358979323846)) *
                             (m > 0 ? std::sqrt(2.0) : 1.0);
            if (m == 0) {
                row[n * n] = f * cr.real();
            } else {
                row[n * n + 2 * m - 1] = f * cr.real();
                row[n * n + 2 * m] = f * cr.imag();
            }
        }
    }
}

// In-place Cholesky solve of S X = B (S n x n SPD, row-major; B n x k).
static void cholesky_solve(int n, std::vector<double> &S, std::vector<double> &B, int k) {
    for (int j = 0; j < n; ++j) {
        double d = S[(size_t)j * n + j];
        for (int p = 0; p < j; ++p) d -= S[(size_t)j * n + p] * S[(size_t)j * n + p];
        BFM_CHECK(d > 0.0, BFM_EINVAL, "template basis: Gram matrix not positive definite");
        d = std::sqrt(d);
        S[(size_t)j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double v = S[(size_t)i * n + j];
            for (int p = 0; p < j; ++p) v -= S[(size_t)i * n + p] * S[(size_t)j * n + p];
            S[(size_t)i * n + j] = v / d;
        }
    }
    for (int c = 0; c < k; ++c) {
        for (int i = 0; i < n; ++i) {  // forward
            double v = B[(size_t)i * k + c];
            for (int p = 0; p < i; ++p) v -= S[(size_t)i * n + p] * B[(size_t)p * k + c];
            B[(size_t)i * k + c] = v / S[(size_t)i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {  // backward
            double v = B[(size_t)i * k + c];
            for (int p = i + 1; p < n; ++p) v -= S[(size_t)p * n + i] * B[(size_t)p * k + c];
            B[(size_t)i * k + c] = v / S[(size_t)i * n + i];
        }
    }
}

// Uploads G (row-major [nd][nc] on the host) and its least-squares
// projector Gp = (G^T W G)^{-1} G^T W (W = diag(wv)) in the device layouts.
static void basis_upload(int nd, int nc, const std::vector<double> &G, const std::vector<double> &wv, ShBasis &B,
                         hipStream_t st) {
    std::vector<double> S((size_t)nc * nc, 0.0), R((size_t)nc * nd, 0.0);
    for (int i = 0; i < nc; ++i)
        for (int v = 0; v < nd; ++v) R[(size_t)i * nd + v] = G[(size_t)v * nc + i] * wv[v];
    for (int i = 0; i < nc; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = 0.0;
            for (int v = 0; v < nd; ++v) s += R[(size_t)i * nd + v] * G[(size_t)v * nc + j];
            S[(size_t)i * nc + j] = S[(size_t)j * nc + i] = s;
        }
    cholesky_solve(nc, S, R, nd);
    // device layouts (column-major): G [nd x nc], Gp [nc x nd]
    std::vector<double> Gc((size_t)nd * nc), Gpc((size_t)nc * nd);
    for (int v = 0; v < nd; ++v)
        for (int i = 0; i < nc; ++i) {
            Gc[(size_t)i * nd + v] = G[(size_t)v * nc + i];
            Gpc[(size_t)v * nc + i] = R[(size_t)i * nd + v];
        }
    B.G.ensure(Gc.size());
    B.Gp.ensure(Gpc.size());
    BFM_HIP(hipMemcpyAsync(B.G.get(), Gc.data(), sizeof(double) * Gc.size(), hipMemcpyHostToDevice, st));
    BFM_HIP(hipMemcpyAsync(B.Gp.get(), Gpc.data(), sizeof(double) * Gpc.size(), hipMemcpyHostToDevice, st));
    BFM_HIP(hipStreamSynchronize(st));
    B.nc = nc;
    B.nd = nd;
}

// Real trigonometric basis of the torus angles (Section 3.7, spherical7: the
// real form of e^{i(n theta + m phi)}, |n|, |m| <= h): the products of
// {1, cos k theta, sin k theta : k = 1..h} with the same set in phi, theta
// functions slowest.
static void trig_row(int h, double th, double ph, double *row) {
    const int w = 2 * h + 1;
    std::vector<double> a(w), b(w);
    a[0] = b[0] = 1.0;
    for (int k = 1; k <= h; ++k) {
        a[2 * k - 1] = std::cos(k * th);
        a[2 * k] = std::sin(k * th);
        b[2 * k - 1] = std::cos(k * ph);
        b[2 * k] = std::sin(k * ph);
    }
    for (int i = 0; i < w; ++i)
        for (int j = 0; j < w; ++j) row[i * w + j] = a[i] * b[j];
}

void torus_basis_build(const Precond &P, int h, ShBasis &B, hipStream_t st) {
    const int nd = P.nd;
    BFM_CHECK(nd > 0 && P.genus == 1 && !P.ang_h.empty(), BFM_EINVAL, "no torus template set");
    const int nc = (2 * h + 1) * (2 * h + 1);
    BFM_CHECK(h >= 0 && nc <= nd, BFM_EINVAL, "trigonometric degree must satisfy (2 degree + 1)^2 <= vertices per bubble");
    if (B.genus == 1 && B.nmax == h && B.nd == nd && B.weighted == 0 && B.gen == P.gen) return;
    std::vector<double> G((size_t)nd * nc), wv(nd, 1.0);
    for (int v = 0; v < nd; ++v) trig_row(h, P.ang_h[2 * v], P.ang_h[2 * v + 1], &G[(size_t)v * nc]);
    basis_upload(nd, nc, G, wv, B, st);
    B.nmax = h;
    B.weighted = 0;
    B.genus = 1;
    B.gen = P.gen;
}

void sh_basis_build(const Precond &P, int nmax, ShBasis &B, hipStream_t st, bool weighted) {
    const int nd = P.nd;
    BFM_CHECK(nd > 0 && P.genus == 0 && !P.dirs_h.empty(), BFM_EINVAL, "no sphere template set");
    BFM_CHECK(nmax >= 0 && (nmax + 1) * (nmax + 1) <= nd, BFM_EINVAL,
              "harmonic degree must satisfy (degree + 1)^2 <= vertices per bubble");
    if (B.genus == 0 && B.nmax == nmax && B.nd == nd && B.weighted == (int)weighted && B.gen == P.gen) return;
    const int nc = (nmax + 1) * (nmax + 1);
    // weights: template vertex areas from the first bubble's triangles on the
    // unit directions, or all ones (plain least squares)
    std::vector<double> wv(nd, weighted ? 0.0 : 1.0);
    for (size_t k = 0; weighted && k + 2 < P.tri_h.size(); k += 3) {
        const double *a = &P.dirs_h[3 * P.tri_h[k]], *b = &P.dirs_h[3 * P.tri_h[k + 1]],
                     *d = &P.dirs_h[3 * P.tri_h[k + 2]];
        const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        const double e2[3] = {d[0] - a[0], d[1] - a[1], d[2] - a[2]};
        const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                     cz = e1[0] * e2[1] - e1[1] * e2[0];
        const double A = 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
        for (int t = 0; t < 3; ++t) wv[P.tri_h[k + t]] += A / 3.0;
    }
    std::vector<double> G((size_t)nd * nc);  // row-major [nd][nc]
    for (int v = 0; v < nd; ++v) sh_row(nmax, &P.dirs_h[3 * v], &G[(size_t)v * nc]);
    basis_upload(nd, nc, G, wv, B, st);
    B.nmax = nmax;
    B.weighted = (int)weighted;
    B.genus = 0;
    B.gen = P.gen;
}

void precond_build(bfm_ctx *c) {
    Precond &P = c->pre;
    const int nmax = c->opt.precond_degree;
    if (P.ready && P.nmax == nmax) return;
    sh_basis_build(P, nmax, P.basis, c->stream);
    const int nc = P.basis.nc;
    std::vector<double> fac(nc);
    const double cc = 2.0 * (nmax + 1) + 1.0;
    for (int n = 0; n <= nmax; ++n)
        for (int i = n * n; i < (n + 1) * (n + 1); ++i) fac[i] = (2.0 * n + 1.0) - cc;
    P.fac.ensure(nc);
    BFM_HIP(hipMemcpyAsync(P.fac.get(), fac.data(), sizeof(double) * nc, hipMemcpyHostToDevice, c->stream));
    BFM_HIP(hipStreamSynchronize(c->stream));
    P.nmax = nmax;
    P.nc = nc;
    P.cc = cc;
    P.ready = true;
}

// Per-bubble equivalent radius sqrt(area / 4 pi) from the vertex weights.
__global__ void k_bubble_radius(const double *s, int nd, double *R) {
    __shared__ double red[256];
    const int b = blockIdx.x;
    double a = 0.0;
    for (int v = threadIdx.x; v < nd; v += 256) a += s[(int64_t)b * nd + v];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) R[b] = sqrt(red[0] / (4.0 * 3.14159265358979323846));
}

// C = rowscale o (A B) + beta D, column-major FP64 on MFMA
// (v_mfma_f64_16x16x4f64). A workgroup of 4 waves owns a 64 x 64 tile of C
// (each wave a 32 x 32 quarter, 2 x 2 MFMA blocks); K advances in chunks of
// 32 staged through LDS, the next chunk's elements loaded into registers
// while the current one is multiplied. With gridDim.z = S > 1 the K range is
// split into S slices and slice z writes its raw partial product to
// W + z M N (ld M); k_gemm_sum then adds the slices in a fixed order and
// applies rowscale and beta D. rowscale and D may be null. C may alias D
// (each element is read and written by the same lane) but not A or B.
// MFMA operand layout: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]
// of a 16 x 4 by 4 x 16 product; element r of the result holds row
// l / 16 + 4 r, column l % 16.
typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int kGemmKC = 32;  // K chunk

__global__ void __launch_bounds__(256) k_gemm_nn(int M, int N, int K, int kslice, const double *A, int lda,
                                                 const double *B, int ldb, double *C, int ldc,
                                                 const double *rowscale, double beta, const double *D, int ldd,
                                                 double *W) {
    // A and B chunks ([k][row], [k][col]); after the products the same LDS
    // holds the 64 x 64 result tile ([col][row]) for coalesced stores
    __shared__ double sbuf[2 * kGemmKC * (64 + 1)];
    static_assert(2 * kGemmKC >= 64, "the result tile fits in the chunk buffers");
    double(*As)[64 + 1] = reinterpret_cast<double(*)[64 + 1]>(sbuf);
    double(*Bs)[64 + 1] = reinterpret_cast<double(*)[64 + 1]>(sbuf + kGemmKC * (64 + 1));
    double(*Cs)[64 + 1] = reinterpret_cast<double(*)[64 + 1]>(sbuf);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
    const int ka = blockIdx.z * kslice, kb = min(K, ka + kslice);
    const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
    dbl4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
    // element e = tid + 256 u of a chunk: A (64 rows x 32 k, rows fastest),
    // B (32 k x 64 columns, k fastest)
    double ra[8], rb[8];
    auto load = [&](int k0) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + 256 * u;
            const int ii = e & 63, kk = e >> 6;
            const int gi = i0 + ii, gk = k0 + kk;
            ra[u] = (gi < M && gk < kb) ? A[(int64_t)gk * lda + gi] : 0.0;
            const int kq = e & 31, jj = e >> 5;
            const int gj = j0 + jj, gk2 = k0 + kq;
            rb[u] = (gj < N && gk2 < kb) ? B[(int64_t)gj * ldb + gk2] : 0.0;
        }
    };
    if (ka < kb) load(ka);
    for (int k0 = ka; k0 < kb; k0 += kGemmKC) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + 256 * u;
            As[e >> 6][e & 63] = ra[u];
            Bs[e & 31][e >> 5] = rb[u];
        }
        __syncthreads();
        if (k0 + kGemmKC < kb) load(k0 + kGemmKC);  // in flight during the products
#pragma unroll
        for (int k4 = 0; k4 < kGemmKC / 4; ++k4) {
            const int kk = 4 * k4 + lane / 16;
            double af[2], bf[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) af[a] = As[kk][wi + 16 * a + lane % 16];
#pragma unroll
            for (int b = 0; b < 2; ++b) bf[b] = Bs[kk][wj + 16 * b + lane % 16];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
    // the tile through LDS, then each wave stores whole 64-row columns
    // (512 contiguous bytes) instead of 16 columns x 4 rows
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) Cs[wj + 16 * b + lane % 16][wi + 16 * a + lane / 16 + 4 * r] = acc[a][b][r];
    __syncthreads();
    double *Wz = W ? W + (int64_t)blockIdx.z * M * N : nullptr;
    const int gi = i0 + lane;
#pragma unroll 4
    for (int cc = wave; cc < 64; cc += 4) {
        const int gj = j0 + cc;
        if (gi < M && gj < N) {
            double val = Cs[cc][lane];
            if (Wz) {
                Wz[(int64_t)gj * M + gi] = val;
            } else {
                if (rowscale) val *= rowscale[gi];
                if (D) val += beta * D[(int64_t)gj * ldd + gi];
                C[(int64_t)gj * ldc + gi] = val;
            }
        }
    }
}

// C = rowscale o (sum over the S slices of W) + beta D
__global__ void k_gemm_sum(int M, int N, int S, const double *W, double *C, int ldc, const double *rowscale,
                           double beta, const double *D, int ldd) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t mn = (int64_t)M * N;
    if (e >= mn) return;
    const int i = (int)(e % M), j = (int)(e / M);
    double v = 0.0;
    for (int z = 0; z < S; ++z) v += W[z * mn + e];
    if (rowscale) v *= rowscale[i];
    if (D) v += beta * D[(int64_t)j * ldd + i];
    C[(int64_t)j * ldc + i] = v;
}

void gemm_f64(int M, int N, int K, const double *A, int lda, const double *B, int ldb, double *C, int ldc,
              const double *rowscale, double beta, const double *D, int ldd, DevBuf<double> *ws, hipStream_t st) {
    if (M <= 0 || N <= 0) return;
    const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
    // split K when the tiles alone leave most of the chip idle and the
    // slices stay at least two chunks deep
    int S = 1;
    if (ws && tiles < 256) S = std::max(1, std::min((512 + tiles - 1) / tiles, K / (2 * kGemmKC)));
    const int kslice = ((K + S - 1) / S + kGemmKC - 1) / kGemmKC * kGemmKC;
    S = std::max(1, (K + kslice - 1) / kslice);
    dim3 g((M + 63) / 64, (N + 63) / 64, S);
    double *W = S > 1 ? ws->ensure((size_t)S * M * N) : nullptr;
    k_gemm_nn<<<g, 256, 0, st>>>(M, N, K, kslice, A, lda, B, ldb, C, ldc, rowscale, beta, D, ldd, W);
    BFM_LAUNCHED();
    if (S > 1) {
        k_gemm_sum<<<nblk((int64_t)M * N, 256), 256, 0, st>>>(M, N, S, W, C, ldc, rowscale, beta, D, ldd);
        BFM_LAUNCHED();
    }
}

// C = A B, all column-major (the plain product of k_gemm_nn)
void gemm_nn_f64(int M, int N, int K, const double *A, int lda, const double *B, int ldb, double *C, int ldc,
                 hipStream_t st) {
    gemm_f64(M, N, K, A, lda, B, ldb, C, ldc, nullptr, 0.0, nullptr, 0, nullptr, st);
}

// out_s[i] = Y[perm[i]] / R[b] (+ cy[b]), b the bubble of perm[i]  (sorted order)
__global__ void k_precond_out(const double *Y, const int *perm, int64_t n, int nd, const double *R,
                              const double *cy, double *out) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int o = perm[i];
    const int b = o / nd;
    out[i] = Y[o] / R[b] + (cy ? cy[b] : 0.0);
}

// ---------------------------------------------------------------------------
// Coarse correction (two-level form). With Z the per-bubble indicator
// vectors and S = diag(s), the coarse matrix A_c = (S Z)^T L Z couples the
// bubbles' mean values: A_c[a][a] = sum_{i, j in a} s_i L_ij (exact, from
// the bubble's own pairs and the singular diagonal), A_c[a][b] =
// area_a area_b / (4 pi |c_a - c_b|) for a != b (each bubble seen from the
// other as a point monopole at its area centroid). After the block step
// x = P_b^{-1} v the correction adds Z A_c^{-1} (S Z)^T (v - L x), with the
// residual's bubble sums formed from the same model of L:
//   (S Z)^T L x |_a = U_a . x_a + area_a sum_{b != a} m_b / (4 pi |c_a - c_b|),
//   U_a = s_a^T L_aa (per vertex), m_b = sum_{j in b} s_j x_j.

// area and area-weighted centroid of every bubble
__global__ void k_coarse_geom(const double *xyz, const double *s, int nd, double *cen, double *area, double *usum) {
    __shared__ double red[4][256];
    const int b = blockIdx.x;
    double a[4] = {0, 0, 0, 0};
    for (int v = threadIdx.x; v < nd; v += 256) {
        const int64_t o = (int64_t)b * nd + v;
        const double w = s[o];
        a[0] += w * xyz[3 * o];
        a[1] += w * xyz[3 * o + 1];
        a[2] += w * xyz[3 * o + 2];
        a[3] += w;
    }
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = a[k];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int k = 0; k < 3; ++k) cen[3 * b + k] = red[k][0] / red[3][0];
        area[b] = red[3][0];
        usum[b] = 0.0;  // summed by k_coarse_u
    }
}

// U_j = s_j (sum_{i in a, i != j} s_i / (4 pi r_ij) + L_jj) for vertex j of
// bubble a (caller order), with the singular diagonal L_jj in its
// translation-free form summed over the own bubble only:
//   L_jj = n_j . [sum_i M_ji (r_i - r_j) - sum_i L_ji n_i],
//   M_ji = s_i n_i . (r_j - r_i) / (4 pi r^3),  L_ji = s_i / (4 pi r).
// (The other bubbles' closed surfaces contribute only their discretisation
// error to these sums; the coarse space is a preconditioner, so the own
// bubble suffices and the build does not wait for the diagonal pass.)
// One workgroup per tile (vertex block of 256, bubble; a grid-stride loop
// over tiles: a capped grid that left wave slots free for the octree build
// beside it measured slower, its kernels started later); the bubble's points
// pass through LDS in chunks. The sums run in FP32 on coordinates relative to the
// bubble's centroid (formed in FP64): the coarse space only preconditions,
// and at a mesh spacing of a tenth of the radius the relative error of r_ij
// is about 1e-6. The pair i = j (r = 0) is masked. usum[b] += the tile's
// sum of U (the coarse matrix's diagonal).
__global__ void __launch_bounds__(256) k_coarse_u(const double *xyz, const double *s, const double *nrm, int64_t nv,
                                                  int nd, int nb, const double *cen, double *U, double *usum) {
    constexpr int CH = 256;
    __shared__ float4 sp[CH];  // x, y, z, s
    __shared__ float4 sn[CH];  // n_x, n_y, n_z
    __shared__ double red[4];
    const int nvb = (nd + 255) / 256;
    for (int64_t tile = blockIdx.x; tile < (int64_t)nvb * nb; tile += gridDim.x) {
        const int b = (int)(tile / nvb);
        const int j = (int)(tile - (int64_t)b * nvb) * 256 + threadIdx.x;
        const int64_t base = (int64_t)b * nd;
        const bool ok = j < nd;
        const int64_t oj = base + (ok ? j : 0);
        const double c0x = cen[3 * b], c0y = cen[3 * b + 1], c0z = cen[3 * b + 2];
        const float xj = (float)(xyz[3 * oj] - c0x), yj = (float)(xyz[3 * oj + 1] - c0y),
                    zj = (float)(xyz[3 * oj + 2] - c0z);
        float acc = 0.f, ax = 0.f, ay = 0.f, az = 0.f;  // sum s_i / r; sum M-type vector - L-type vector
        for (int c0 = 0; c0 < nd; c0 += CH) {
            const int cn = min(CH, nd - c0);
            __syncthreads();
            for (int t = threadIdx.x; t < cn; t += 256) {
                const int64_t o = base + c0 + t;
                sp[t] = make_float4((float)(xyz[3 * o] - c0x), (float)(xyz[3 * o + 1] - c0y),
                                    (float)(xyz[3 * o + 2] - c0z), (float)s[o]);
                sn[t] = make_float4((float)nrm[o], (float)nrm[nv + o], (float)nrm[2 * nv + o], 0.f);
            }
            __syncthreads();
            const int self = j - c0;  // position of the receiver in this chunk (masked)
            for (int t = 0; t < cn; ++t) {
                const float4 q = sp[t], m = sn[t];
                const float dx = xj - q.x, dy = yj - q.y, dz = zj - q.z;  // r_j - r_i
                const float r2 = dx * dx + dy * dy + dz * dz;
                const float inv = (t == self) ? 0.f : __builtin_amdgcn_rsqf(r2);
                const float si = q.w * inv;  // s_i / r
                acc += si;
                // s_i n_i.(r_j - r_i) / r^3 (r_i - r_j) - s_i / r n_i
                const float g = (m.x * dx + m.y * dy + m.z * dz) * si * inv * inv;
                ax -= g * dx + si * m.x;
                ay -= g * dy + si * m.y;
                az -= g * dz + si * m.z;
            }
        }
        double u = 0.0;
        if (ok) {
            const double k4 = 1.0 / (4.0 * 3.14159265358979323846);
            const double ljj =
                (nrm[oj] * (double)ax + nrm[nv + oj] * (double)ay + nrm[2 * nv + oj] * (double)az) * k4;
            u = s[oj] * ((double)acc * k4 + ljj);
            U[oj] = u;
        }
        // the tile's sum of U: wave sums, then one atomic
        for (int o = 32; o > 0; o >>= 1) u += __shfl_down(u, o);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = u;
        __syncthreads();
        if (threadIdx.x == 0) atomicAdd(usum + b, red[0] + red[1] + red[2] + red[3]);
    }
}

// A (column-major nb x nb): off-diagonal point-monopole couplings; the
// diagonal from the bubble sums of U.
__global__ void k_coarse_matrix(const double *cen, const double *area, const double *usum, int nb, double *A) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)nb * nb) return;
    const int a = (int)(e % nb), b = (int)(e / nb);
    if (a == b) {
        A[e] = usum[a];
        return;
    }
    const double dx = cen[3 * a] - cen[3 * b], dy = cen[3 * a + 1] - cen[3 * b + 1], dz = cen[3 * a + 2] - cen[3 * b + 2];
    A[e] = area[a] * area[b] / (4.0 * 3.14159265358979323846 * sqrt(dx * dx + dy * dy + dz * dz));
}

// Gauss-Jordan inverse (no pivoting: the coarse matrix is symmetric positive
// definite) of the bs x bs diagonal block at (k0, k0) of A (column-major,
// leading dimension n); writes -inverse to P (column-major bs x bs).
// Thread t owns column t % 64 and rows 16 (t / 64) .. +15 in registers; each
// step publishes the pivot row and column through LDS.
constexpr int kGjBlock = 64;
constexpr int kGjThreads = 1024;
constexpr int kGjRows = kGjBlock * kGjBlock / kGjThreads;  // rows per thread
__global__ void __launch_bounds__(kGjThreads) k_gj_block(const double *A, int n, int k0, int bs, double *P) {
    // The block lives in LDS, twice: step k reads buffer k % 2 and writes the
    // other, so one barrier per step suffices. Thread (j, i0) updates column
    // j, rows i0..i0+3: sixteen waves share the step, which is bound by the
    // latency of its reads and writes rather than by their number.
    __shared__ double a[2][kGjBlock][kGjBlock + 1];  // [buffer][row][column]
    const int tid = threadIdx.x;
    const int j = tid % kGjBlock, i0 = kGjRows * (tid / kGjBlock);
    for (int e = tid; e < kGjBlock * kGjBlock; e += kGjThreads) {
        const int i = e % kGjBlock, c = e / kGjBlock;
        // identity outside the bs x bs block keeps the padded steps inert
        a[0][i][c] = (i < bs && c < bs) ? A[(int64_t)(k0 + c) * n + k0 + i] : (i == c ? 1.0 : 0.0);
    }
    __syncthreads();
    for (int k = 0; k < kGjBlock; ++k) {
        const double(*src)[kGjBlock + 1] = a[k & 1];
        double(*dst)[kGjBlock + 1] = a[(k & 1) ^ 1];
        // 1 / pivot: hardware reciprocal and two Newton steps
        const double piv = src[k][k];
        double p = __builtin_amdgcn_rcp(piv);
        p = fma(p, fma(-piv, p, 1.0), p);
        p = fma(p, fma(-piv, p, 1.0), p);
        const double rk = (j == k) ? p : src[k][j] * p;  // new row k, column j
#pragma unroll
        for (int r = 0; r < kGjRows; ++r) {
            const int i = i0 + r;
            const double f = src[i][k], old = src[i][j];
            const double upd = (j == k) ? -f * p : old - f * rk;
            dst[i][j] = (i == k) ? rk : upd;
        }
        __syncthreads();
    }
    for (int e = tid; e < kGjBlock * kGjBlock; e += kGjThreads) {
        const int i = e % kGjBlock, c = e / kGjBlock;
        if (i < bs && c < bs) P[(int64_t)c * bs + i] = -a[kGjBlock & 1][i][c];
    }
}

// row block k0..k0+bs of A := -Rn (Rn = -P^{-1} A_K,:) outside the block
// columns; column block := Cn (= -A_:,K P^{-1}) outside the block rows, and
// the diagonal block := P^{-1} = -Pn.
__global__ void k_gj_fix(double *A, int n, int k0, int bs, const double *Rn, const double *Cn, const double *Pn) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t nrow = (int64_t)bs * n;
    if (e < nrow) {  // row block, all columns j (block columns get -Pn below)
        const int r = (int)(e % bs), j = (int)(e / bs);
        if (j < k0 || j >= k0 + bs) A[(int64_t)j * n + k0 + r] = -Rn[(int64_t)j * bs + r];
        return;
    }
    e -= nrow;
    if (e >= nrow) return;
    const int i = (int)(e % n), c = (int)(e / n);  // column block, all rows i
    if (i < k0 || i >= k0 + bs)
        A[(int64_t)(k0 + c) * n + i] = Cn[(int64_t)c * n + i];
    else
        A[(int64_t)(k0 + c) * n + i] = -Pn[(int64_t)c * bs + (i - k0)];
}

// per bubble: sums[0][b] = sum s x, sums[1][b] = sum U x, sums[2][b] = sum s v,
// with x = Y / R[b] (caller order), v = X
__global__ void k_coarse_sums(const double *Y, const double *X, const double *R, const double *s,
                              const double *U, int nd, int nb, double *sums) {
    __shared__ double red[3][256];
    const int b = blockIdx.x;
    const double ir = 1.0 / R[b];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int v = threadIdx.x; v < nd; v += 256) {
        const int64_t o = (int64_t)b * nd + v;
        const double x = Y[o] * ir;
        a0 += s[o] * x;
        a1 += U[o] * x;
        a2 += s[o] * X[o];
    }
    red[0][threadIdx.x] = a0;
    red[1][threadIdx.x] = a1;
    red[2][threadIdx.x] = a2;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) sums[(int64_t)k * nb + b] = red[k][0];
}

// coarse right-hand side rc_a = sum s v - U.x - area_a sum_{b != a} m_b / (4 pi d_ab),
// written over sums[2]; one block per bubble a
__global__ void k_coarse_rhs(const double *cen, const double *area, int nb, double *sums) {
    __shared__ double red[256];
    const int a = blockIdx.x;
    const double *m = sums;
    const double ax = cen[3 * a], ay = cen[3 * a + 1], az = cen[3 * a + 2];
    double far = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) {
        if (b == a) continue;
        const double dx = ax - cen[3 * b], dy = ay - cen[3 * b + 1], dz = az - cen[3 * b + 2];
        far += m[b] / sqrt(dx * dx + dy * dy + dz * dz);
    }
    red[threadIdx.x] = far;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        sums[2 * (int64_t)nb + a] -=
            sums[(int64_t)nb + a] + area[a] * red[0] * (1.0 / (4.0 * 3.14159265358979323846));
}

// y = A x for symmetric A (nb x nb): row a read as column a; one block per row
__global__ void k_dense_mv(const double *A, const double *x, int nb, double *y) {
    __shared__ double red[256];
    const int a = blockIdx.x;
    const double *col = A + (int64_t)a * nb;
    double t = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) t += col[b] * x[b];
    red[threadIdx.x] = t;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) y[a] = red[0];
}

void precond_radii(bfm_ctx *c) {
    Precond &P = c->pre;
    P.R.ensure(c->nb);
    k_bubble_radius<<<c->nb, 256, 0, c->stream>>>(c->s.get(), P.nd, P.R.get());
    BFM_LAUNCHED();
}

void precond_apply(bfm_ctx *c, const double *in_s, double *out_s) {
    Precond &P = c->pre;
    hipStream_t st = c->stream;
    const int nd = P.nd, nc = P.nc, nb = c->nb;
    double *X = P.X.ensure((size_t)nd * nb);
    double *Cm = P.C.ensure((size_t)nc * nb);
    double *Y = P.Y.ensure((size_t)nd * nb);
    to_original(c, in_s, X);
    // C = diag(2n+1 - c) G+ X
    gemm_f64(nc, nb, nd, P.basis.Gp.get(), nc, X, nd, Cm, nc, P.fac.get(), 0.0, nullptr, 0, &P.gws, st);
    // Y = G C + c X
    gemm_f64(nd, nb, nc, P.basis.G.get(), nd, Cm, nc, Y, nd, nullptr, P.cc, X, nd, &P.gws, st);
    const double *cy = nullptr;
    if (c->opt.precond == BFM_PRECOND_SH_COARSE) {
        double *sums = P.csum.get();
        k_coarse_sums<<<nb, 256, 0, st>>>(Y, X, P.R.get(), c->s.get(), P.U.get(), nd, nb, sums);
        BFM_LAUNCHED();
        k_coarse_rhs<<<nb, 256, 0, st>>>(P.ccen.get(), P.carea.get(), nb, sums);
        BFM_LAUNCHED();
        k_dense_mv<<<nb, 256, 0, st>>>(P.Ainv.get(), sums + 2 * (int64_t)nb, nb, P.cy.get());
        BFM_LAUNCHED();
        cy = P.cy.get();
    }
    k_precond_out<<<nblk(c->nv, 256), 256, 0, st>>>(Y, c->tree.idx_a.get(), c->nv, nd, P.R.get(), cy, out_s);
    BFM_LAUNCHED();
}

// S = the bs x bs diagonal block at (k0, k0) of A (leading dimension n), packed
__global__ void k_gj_copy_block(const double *A, int n, int k0, int bs, double *S) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)bs * bs) return;
    const int i = (int)(e % bs), c = (int)(e / bs);
    S[e] = A[(int64_t)(k0 + c) * n + k0 + i];
}

__global__ void k_gj_negate(const double *S, int64_t m, double *P) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < m) P[e] = -S[e];
}

// Column blocks of the sweep: 64 (each diagonal block inverted in LDS by
// k_gj_block), or 256 on large matrices, whose diagonal blocks are inverted
// by a 64-block sweep over a packed copy. A rank-256 trailing update reads
// and writes the matrix once for 256 columns instead of 64, and the sweep
// is bound by that traffic (with 64-column blocks, 79 passes over a 200 MB
// matrix at 5000 bubbles).
constexpr int kGjOuter = 256;
constexpr int kGjOuterMin = 2048;  // matrix size from which the sweep takes 256-column blocks

// One blocked Gauss-Jordan sweep with B-column blocks (B = 64 or 256):
// per diagonal block K, P = A_KK^{-1}; A_Kj <- P A_Kj, A_ij <- A_ij - A_iK P A_Kj,
// A_iK <- -A_iK P, A_KK <- P (j, i outside K). Work: Pn (B x B), Rn (B x n),
// Cn (n x B); for B = 256 also `inner` (B^2 + 64^2 + 2 * 64 B doubles).
static void gj_sweep(double *A, int nb, int B, double *Pn, double *Rn, double *Cn, double *inner, hipStream_t st) {
    for (int k0 = 0; k0 < nb; k0 += B) {
        const int bs = std::min(B, nb - k0);
        if (B == kGjBlock) {
            k_gj_block<<<1, kGjThreads, 0, st>>>(A, nb, k0, bs, Pn);
            BFM_LAUNCHED();
        } else {
            double *S = inner, *w = inner + (size_t)B * B;
            k_gj_copy_block<<<nblk((int64_t)bs * bs, 256), 256, 0, st>>>(A, nb, k0, bs, S);
            BFM_LAUNCHED();
            gj_sweep(S, bs, kGjBlock, w, w + kGjBlock * kGjBlock, w + kGjBlock * kGjBlock + (size_t)kGjBlock * B,
                     nullptr, st);  // S = A_KK^{-1}
            k_gj_negate<<<nblk((int64_t)bs * bs, 256), 256, 0, st>>>(S, (int64_t)bs * bs, Pn);
            BFM_LAUNCHED();
        }
        // Rn = Pn A_K,:  (= -P^{-1} A_K,:), bs x nb
        gemm_nn_f64(bs, nb, bs, Pn, bs, A + k0, nb, Rn, bs, st);
        // trailing columns outside the block: A += A_:,K Rn
        if (k0 > 0)
            gemm_f64(nb, k0, bs, A + (int64_t)k0 * nb, nb, Rn, bs, A, nb, nullptr, 1.0, A, nb, nullptr, st);
        const int j1 = k0 + bs;
        if (j1 < nb)
            gemm_f64(nb, nb - j1, bs, A + (int64_t)k0 * nb, nb, Rn + (int64_t)j1 * bs, bs, A + (int64_t)j1 * nb,
                     nb, nullptr, 1.0, A + (int64_t)j1 * nb, nb, nullptr, st);
        // Cn = A_:,K Pn  (= -A_:,K P^{-1}), nb x bs
        gemm_nn_f64(nb, bs, bs, A + (int64_t)k0 * nb, nb, Pn, bs, Cn, nb, st);
        k_gj_fix<<<nblk(2 * (int64_t)bs * nb, 256), 256, 0, st>>>(A, nb, k0, bs, Rn, Cn, Pn);
        BFM_LAUNCHED();
    }
}

// In-place inverse of a symmetric positive definite n x n matrix
// (column-major) by blocked Gauss-Jordan elimination without pivoting.
void spd_inverse(double *A, int nb, DevBuf<double> &piv, DevBuf<double> &row, DevBuf<double> &col,
                 hipStream_t st) {
    const int B = nb >= kGjOuterMin ? kGjOuter : kGjBlock;
    const size_t inner = B == kGjBlock ? 0 : (size_t)B * B + kGjBlock * kGjBlock + 2 * (size_t)kGjBlock * B;
    double *Pn = piv.ensure((size_t)B * B + inner);
    double *Rn = row.ensure((size_t)B * nb);
    double *Cn = col.ensure((size_t)nb * B);
    gj_sweep(A, nb, B, Pn, Rn, Cn, inner ? Pn + (size_t)B * B : nullptr, st);
}

void coarse_build(bfm_ctx *c, hipStream_t st) {
    Precond &P = c->pre;
    const int nd = P.nd, nb = c->nb;
    P.csum.ensure(3 * (size_t)nb);  // used by precond_apply
    P.cy.ensure(nb);
    double *cen = P.ccen.ensure(3 * (size_t)nb), *area = P.carea.ensure(nb), *usum = P.cusum.ensure(nb);
    k_coarse_geom<<<nb, 256, 0, st>>>(c->xyz.get(), c->s.get(), nd, cen, area, usum);
    BFM_LAUNCHED();
    double *U = P.U.ensure((size_t)nd * nb);
    const int64_t tiles = (int64_t)nblk(nd, 256) * nb;
    k_coarse_u<<<(unsigned)tiles, 256, 0, st>>>(c->xyz.get(), c->s.get(), c->nrm.get(), c->nv, nd, nb, cen, U, usum);
    BFM_LAUNCHED();
    double *A = P.Ainv.ensure((size_t)nb * nb);
    k_coarse_matrix<<<nblk((int64_t)nb * nb, 256), 256, 0, st>>>(cen, area, usum, nb, A);
    BFM_LAUNCHED();
    spd_inverse(A, nb, P.gj_piv, P.gj_row, P.gj_col, st);
}

static void coarse_worker_wait(CoarseWorker *w);

void coarse_join(bfm_ctx *c) {
    if (!c->coarse_pending) return;
    c->coarse_pending = false;
    if (c->coarse_worker) coarse_worker_wait(c->coarse_worker);  // the build and its event are queued
    BFM_HIP(hipStreamWaitEvent(c->stream, c->ev_coarse, 0));
}

void coarse_mark(bfm_ctx *c) {
    coarse_join(c);  // an earlier build that nobody waited for (a solve that failed)
    if (!c->side) {
        BFM_HIP(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
        BFM_HIP(hipEventCreateWithFlags(&c->ev_geom, hipEventDisableTiming));
        BFM_HIP(hipEventCreateWithFlags(&c->ev_coarse, hipEventDisableTiming));
    }
    BFM_HIP(hipEventRecord(c->ev_geom, c->stream));
    c->coarse_marked = true;
}

// The coarse build is about a hundred small launches. Queued by the solving
// thread they would hold it, and so the octree build that runs beside them on
// the main stream, for a millisecond or more; a worker thread of the handle
// queues them instead. coarse_launch hands the build over and returns;
// coarse_join waits until the worker has queued the build and its completion
// event (not for the device), then orders the main stream after that event.
struct CoarseWorker {
    std::thread th;
    std::mutex mu;
    std::condition_variable cv;
    bfm_ctx *job = nullptr;  // pending build (taken by the worker)
    bool busy = false, stop = false;
    std::exception_ptr err;
};

static void coarse_worker_main(CoarseWorker *w, int device) {
    bool dev_set = false;
    for (;;) {
        bfm_ctx *c = nullptr;
        {
            std::unique_lock<std::mutex> lk(w->mu);
            w->cv.wait(lk, [&] { return w->job != nullptr || w->stop; });
            if (!w->job) return;  // stop, nothing pending
            c = w->job;
            w->job = nullptr;
        }
        try {
            if (!dev_set) {
                BFM_HIP(hipSetDevice(device));
                dev_set = true;
            }
            BFM_HIP(hipStreamWaitEvent(c->side, c->ev_geom, 0));
            coarse_build(c, c->side);
            BFM_HIP(hipEventRecord(c->ev_coarse, c->side));
        } catch (...) {
            std::lock_guard<std::mutex> lk(w->mu);
            w->err = std::current_exception();
        }
        {
            std::lock_guard<std::mutex> lk(w->mu);
            w->busy = false;
        }
        w->cv.notify_all();
    }
}

static void coarse_worker_wait(CoarseWorker *w) {
    std::unique_lock<std::mutex> lk(w->mu);
    w->cv.wait(lk, [&] { return !w->busy; });
    if (w->err) {
        std::exception_ptr e = w->err;
        w->err = nullptr;
        std::rethrow_exception(e);
    }
}

void coarse_worker_free(bfm_ctx *c) {
    CoarseWorker *w = c->coarse_worker;
    if (!w) return;
    {
        std::lock_guard<std::mutex> lk(w->mu);
        w->stop = true;
    }
    w->cv.notify_all();
    if (w->th.joinable()) w->th.join();
    delete w;
    c->coarse_worker = nullptr;
}

void coarse_launch(bfm_ctx *c) {
    if (!c->coarse_marked) coarse_mark(c);
    c->coarse_marked = false;
    if (!c->coarse_worker) {
        auto *w = new CoarseWorker();
        w->th = std::thread(coarse_worker_main, w, c->device);
        c->coarse_worker = w;
    }
    CoarseWorker *w = c->coarse_worker;
    {
        std::lock_guard<std::mutex> lk(w->mu);
        w->job = c;
        w->busy = true;
    }
    w->cv.notify_all();
    c->coarse_pending = true;
}

}  // namespace bfm
