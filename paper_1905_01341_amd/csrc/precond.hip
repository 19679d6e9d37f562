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
#include <cmath>
#include <complex>
#include <vector>

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
        BFM_CHECK(d > 0.0, BFM_EINVAL, "spherical-harmonic template: Gram matrix not positive definite");
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

void sh_basis_build(const Precond &P, int nmax, ShBasis &B, hipStream_t st) {
    const int nd = P.nd;
    BFM_CHECK(nd > 0 && !P.dirs_h.empty(), BFM_EINVAL, "no sphere template set");
    BFM_CHECK(nmax >= 1 && (nmax + 1) * (nmax + 1) <= nd, BFM_EINVAL,
              "harmonic degree must satisfy (degree + 1)^2 <= vertices per bubble");
    if (B.nmax == nmax && B.nd == nd) return;
    const int nc = (nmax + 1) * (nmax + 1);
    // template vertex areas from the first bubble's triangles on the unit directions
    std::vector<double> wv(nd, 0.0);
    for (size_t k = 0; k + 2 < P.tri_h.size(); k += 3) {
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
    // S = G^T W G ; R = G^T W  -> G+ = S^{-1} R  ([nc][nd])
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
    B.nmax = nmax;
    B.nc = nc;
    B.nd = nd;
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

// C[M x N] = A[M x K] B[K x N] (+ beta D), all column-major; 64 x 64 tiles,
// 256 threads with 4 x 4 outputs each, K staged through LDS in chunks of 16.
// rowscale (may be null) multiplies row i of A B by rowscale[i] before beta D
// is added.
__global__ void __launch_bounds__(256) k_gemm_nn(int M, int N, int K, const double *A, int lda,
                                                 const double *B, int ldb, double *C, int ldc,
                                                 const double *rowscale, double beta, const double *D,
                                                 int ldd) {
    __shared__ double As[16][64 + 1], Bs[16][64 + 1];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
    double acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += 16) {
        for (int e = threadIdx.x; e < 16 * 64; e += 256) {
            const int kk = e / 64, ii = e % 64;
            const int gi = i0 + ii, gk = k0 + kk;
            As[kk][ii] = (gi < M && gk < K) ? A[(int64_t)gk * lda + gi] : 0.0;
            const int jj = e % 64, kb = e / 64;
            const int gj = j0 + jj, gk2 = k0 + kb;
            Bs[kb][jj] = (gj < N && gk2 < K) ? B[(int64_t)gj * ldb + gk2] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = As[kk][tx + 16 * u];
                b[u] = Bs[kk][ty + 16 * u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int gi = i0 + tx + 16 * u, gj = j0 + ty + 16 * v;
            if (gi < M && gj < N) {
                double val = acc[u][v];
                if (rowscale) val *= rowscale[gi];
                if (D) val += beta * D[(int64_t)gj * ldd + gi];
                C[(int64_t)gj * ldc + gi] = val;
            }
        }
}

// C = A B, all column-major (the plain product of k_gemm_nn)
void gemm_nn_f64(int M, int N, int K, const double *A, int lda, const double *B, int ldb, double *C, int ldc,
                 hipStream_t st) {
    dim3 g((M + 63) / 64, (N + 63) / 64);
    k_gemm_nn<<<g, 256, 0, st>>>(M, N, K, A, lda, B, ldb, C, ldc, nullptr, 0.0, nullptr, 0);
    BFM_LAUNCHED();
}

// out_s[i] = Y[perm[i]] / R[bubble of perm[i]]  (sorted order)
__global__ void k_precond_out(const double *Y, const int *perm, int64_t n, int nd, const double *R,
                              double *out) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int o = perm[i];
    out[i] = Y[o] / R[o / nd];
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
    dim3 g1((nc + 63) / 64, (nb + 63) / 64), g2((nd + 63) / 64, (nb + 63) / 64);
    // C = diag(2n+1 - c) G+ X
    k_gemm_nn<<<g1, 256, 0, st>>>(nc, nb, nd, P.basis.Gp.get(), nc, X, nd, Cm, nc, P.fac.get(), 0.0, nullptr, 0);
    BFM_LAUNCHED();
    // Y = G C + c X
    k_gemm_nn<<<g2, 256, 0, st>>>(nd, nb, nc, P.basis.G.get(), nd, Cm, nc, Y, nd, nullptr, P.cc, X, nd);
    BFM_LAUNCHED();
    k_precond_out<<<nblk(c->nv, 256), 256, 0, st>>>(Y, c->tree.idx_a.get(), c->nv, nd, P.R.get(), out_s);
    BFM_LAUNCHED();
}

}  // namespace bfm
