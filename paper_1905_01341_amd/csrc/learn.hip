// Learned initial guess for GMRES (not in the paper, which warm-starts from
// the previous time step, Section 3.6): a small MLP maps each bubble's
// spherical-harmonic description to the harmonic coefficients of its q.
//
// Features of bubble b (174): the degree <= 8 coefficients (81) of the radial
// function rho_i = |r_i - c_b| / a_b, the degree <= 8 coefficients (81) of
// phi, and the offsets of the 4 nearest bubble centres divided by a_b (12),
// with c_b the vertex mean and a_b = sqrt(area_b / 4 pi). Target (81): the
// degree <= 8 coefficients of a_b q. Network: 174 -> 512 -> 512 -> 512 -> 81,
// SiLU, BF16 weights and activations with FP32 accumulation
// (v_mfma_f32_16x16x32_bf16), FP32 master weights, Adam, mean-squared loss
// on standardised features and targets. Guess: q0 = G (prediction) / a_b.
#include <hip/hip_bf16.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "learn.h"

namespace bfm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

static unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Result layout of v_mfma_f32_16x16x32_bf16: lane l, element r holds row
// kRow(l, r) and column l % 16 of the 16 x 16 block.
__device__ inline int mfma_row(int l, int r) { return 4 * (l >> 4) + r; }

// C[M x N] (FP32, row-major) (+)= A[M x K] B[K x N] + bias[N]. A is BF16 with
// K contiguous per row (A[m * lda + k]); B is BF16 with K contiguous per
// column (B[n * ldb + k]). K % 32 == 0, lda and ldb multiples of 8.
// 256 threads: 4 waves, each a 32 x 32 block (2 x 2 MFMA tiles).
__global__ void __launch_bounds__(256) k_gemm_bf16(int M, int N, int K, const __bf16 *A, int lda,
                                                   const __bf16 *B, int ldb, float *C, int ldc,
                                                   const float *bias, int accumulate) {
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int m0 = blockIdx.x * 64 + (wave >> 1) * 32, n0 = blockIdx.y * 64 + (wave & 1) * 32;
    const int kofs = 8 * (l >> 4);
    f32x4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 32) {
        bf16x8 a[2], b[2];
        for (int i = 0; i < 2; ++i) {
            const int row = m0 + 16 * i + (l & 15);
            if (row < M) {
                a[i] = *reinterpret_cast<const bf16x8 *>(A + (int64_t)row * lda + k0 + kofs);
            } else {
                for (int e = 0; e < 8; ++e) a[i][e] = (__bf16)0.0f;
            }
            const int col = n0 + 16 * i + (l & 15);
            if (col < N) {
                b[i] = *reinterpret_cast<const bf16x8 *>(B + (int64_t)col * ldb + k0 + kofs);
            } else {
                for (int e = 0; e < 8; ++e) b[i][e] = (__bf16)0.0f;
            }
        }
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + 16 * i + mfma_row(l, r), col = n0 + 16 * j + (l & 15);
                if (row < M && col < N) {
                    float v = acc[i][j][r] + (bias ? bias[col] : 0.f);
                    if (accumulate) v += C[(int64_t)row * ldc + col];
                    C[(int64_t)row * ldc + col] = v;
                }
            }
}

__device__ inline float silu_f(float z) { return z / (1.f + __expf(-z)); }
__device__ inline float silu_g(float z) {
    const float s = 1.f / (1.f + __expf(-z));
    return s * (1.f + z * (1.f - s));
}

// out[r][c] = bf16(silu(Z[r][c])) (act) or bf16(Z[r][c]); rows x cols
__global__ void k_act_bf16(const float *Z, int64_t total, int act, __bf16 *out) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < total) out[i] = (__bf16)(act ? silu_f(Z[i]) : Z[i]);
}

// out[c][r] = bf16(in[r][c]) (in FP32 or BF16), rows x cols -> cols x rows
template <class T>
__global__ void k_transpose_bf16(const T *in, int rows, int cols, __bf16 *out) {
    __shared__ float tile[32][33];
    const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
    for (int k = threadIdx.y; k < 32; k += 8) {
        const int r = r0 + k, c = c0 + threadIdx.x;
        tile[k][threadIdx.x] = (r < rows && c < cols) ? (float)in[(int64_t)r * cols + c] : 0.f;
    }
    __syncthreads();
    for (int k = threadIdx.y; k < 32; k += 8) {
        const int c = c0 + k, r = r0 + threadIdx.x;
        if (c < cols && r < rows) out[(int64_t)c * rows + r] = (__bf16)tile[threadIdx.x][k];
    }
}

// G = (Y - T) / nrows on the first `used` columns and `nrows` rows, 0 elsewhere;
// part[block] = partial sums of 0.5 (Y - T)^2 over the block.
__global__ void k_loss_grad(const float *Y, const float *T, int rows, int cols, int used, int nrows,
                            float *G, float *part) {
    __shared__ float red[256];
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    float l = 0.f;
    if (i < (int64_t)rows * cols) {
        const int r = (int)(i / cols), c = (int)(i % cols);
        float g = 0.f;
        if (r < nrows && c < used) {
            const float d = Y[i] - T[(int64_t)r * used + c];
            g = d / (float)nrows;
            l = 0.5f * d * d;
        }
        G[i] = g;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_silu_back(float *G, const float *Z, int64_t total) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < total) G[i] *= silu_g(Z[i]);
}

// db[c] = sum_r G[r][c]
__global__ void k_colsum(const float *G, int rows, int cols, float *db) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float s = 0.f;
    for (int r = 0; r < rows; ++r) s += G[(int64_t)r * cols + c];
    db[c] = s;
}

__global__ void k_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Wt[o][i] = bf16(W[i][o]) and Wn[i][o] = bf16(W[i][o]); W is in x out.
__global__ void k_refresh(const float *W, int in, int out, __bf16 *Wt, __bf16 *Wn) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)in * out) return;
    const int i = (int)(e / out), o = (int)(e % out);
    const __bf16 v = (__bf16)W[e];
    Wn[e] = v;
    Wt[(int64_t)o * in + i] = v;
}

// ---------------------------------------------------------------------------
// Features

// centre (vertex mean) and radius sqrt(area / 4 pi) of every bubble
__global__ void k_bubble_geom(const double *xyz, const double *s, int nd, double *cen, double *rad) {
    __shared__ double red[4][256];
    const int b = blockIdx.x;
    double a[4] = {0, 0, 0, 0};
    for (int v = threadIdx.x; v < nd; v += 256) {
        const int64_t o = (int64_t)b * nd + v;
        a[0] += xyz[3 * o];
        a[1] += xyz[3 * o + 1];
        a[2] += xyz[3 * o + 2];
        a[3] += s[o];
    }
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = a[k];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int k = 0; k < 3; ++k) cen[3 * b + k] = red[k][0] / nd;
        rad[b] = sqrt(red[3][0] / (4.0 * 3.14159265358979323846));
    }
}

// per vertex (caller order): rho / a_b, phi, and a_b q (any may be null)
__global__ void k_vertex_fields(const double *xyz, const double *cen, const double *rad, int nd, int64_t nv,
                                const double *phi, const double *q, double *rho_o, double *phi_o,
                                double *aq_o) {
    int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (o >= nv) return;
    const int b = (int)(o / nd);
    const double dx = xyz[3 * o] - cen[3 * b], dy = xyz[3 * o + 1] - cen[3 * b + 1],
                 dz = xyz[3 * o + 2] - cen[3 * b + 2];
    if (rho_o) rho_o[o] = sqrt(dx * dx + dy * dy + dz * dz) / rad[b];
    if (phi_o) phi_o[o] = phi[o];
    if (aq_o) aq_o[o] = q[o] * rad[b];
}

// offsets of the 4 nearest other centres / a_b (zeros when fewer exist)
__global__ void k_neighbours(const double *cen, const double *rad, int nb, float *off) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    double bd[4] = {1e300, 1e300, 1e300, 1e300};
    int bi[4] = {-1, -1, -1, -1};
    for (int o = 0; o < nb; ++o) {
        if (o == b) continue;
        const double dx = cen[3 * o] - cen[3 * b], dy = cen[3 * o + 1] - cen[3 * b + 1],
                     dz = cen[3 * o + 2] - cen[3 * b + 2];
        const double d = dx * dx + dy * dy + dz * dz;
        if (d < bd[3] || (d == bd[3] && o < bi[3])) {
            int k = 3;
            while (k > 0 && (d < bd[k - 1] || (d == bd[k - 1] && o < bi[k - 1]))) {
                bd[k] = bd[k - 1];
                bi[k] = bi[k - 1];
                --k;
            }
            bd[k] = d;
            bi[k] = o;
        }
    }
    for (int k = 0; k < 4; ++k)
        for (int d = 0; d < 3; ++d)
            off[12 * (int64_t)b + 3 * k + d] =
                bi[k] >= 0 ? (float)((cen[3 * bi[k] + d] - cen[3 * b + d]) / rad[b]) : 0.f;
}

// feature row b: [c_rho (81) | c_phi (81) | offsets (12)], coefficients
// column-major [81 x nb]
__global__ void k_assemble(const double *crho, const double *cphi, const float *off, int nb, int nc,
                           float *feat) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int w = 2 * nc + 12;
    if (e >= (int64_t)nb * w) return;
    const int b = (int)(e / w), c = (int)(e % w);
    float v;
    if (c < nc)
        v = (float)crho[(int64_t)b * nc + c];
    else if (c < 2 * nc)
        v = (float)cphi[(int64_t)b * nc + (c - nc)];
    else
        v = off[12 * (int64_t)b + (c - 2 * nc)];
    feat[e] = v;
}

// coefficients column-major [nc x nb] -> rows [nb x nc] (FP32)
__global__ void k_coef_rows(const double *coef, int nb, int nc, float *out) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < (int64_t)nb * nc) out[e] = (float)coef[e];
}

// Standardised network input: X0[r][c] = bf16((src[row][c] - mu[c]) / sd[c]) with
// row = idx ? idx[off + r] : off + r, for r < rows and c < cols; zero in the
// padding (r < R, c < ld).
__global__ void k_batch_in(const float *src, const int *idx, int64_t off, int rows, int R, int cols, int ld,
                           const float *mu, const float *sd, __bf16 *X0) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)R * ld) return;
    const int r = (int)(e / ld), c = (int)(e % ld);
    float v = 0.f;
    if (r < rows && c < cols) {
        const int64_t row = idx ? idx[off + r] : off + r;
        v = (src[row * cols + c] - mu[c]) / sd[c];
    }
    X0[e] = (__bf16)v;
}

// Standardised targets T[r][c] = (src[row][c] - mu[c]) / sd[c] (row as above)
__global__ void k_batch_targ(const float *src, const int *idx, int64_t off, int rows, int cols, const float *mu,
                             const float *sd, float *T) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)rows * cols) return;
    const int r = (int)(e / cols), c = (int)(e % cols);
    const int64_t row = idx ? idx[off + r] : off + r;
    T[e] = (src[row * cols + c] - mu[c]) / sd[c];
}

// network output rows Y [rows][ld] -> out [rows][nc] = Y * sd + mu (FP32)
__global__ void k_unstd_rows(const float *Y, int rows, int ld, int nc, const float *mu, const float *sd,
                             float *out) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)rows * nc) return;
    const int r = (int)(e / nc), c = (int)(e % nc);
    out[e] = Y[(int64_t)r * ld + c] * sd[c] + mu[c];
}

// prediction rows Y [nb][ld] -> coefficients column-major [nc x nb] in FP64
__global__ void k_unstandardise(const float *Y, int nb, int ld, int nc, const float *mu, const float *sd,
                                double *coef) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)nb * nc) return;
    const int b = (int)(e / nc), c = (int)(e % nc);
    coef[e] = (double)(Y[(int64_t)b * ld + c] * sd[c] + mu[c]);
}

// q (caller order) = synthesised values / a_b
__global__ void k_guess_out(const double *vals, const double *rad, int nd, int64_t nv, double *q) {
    int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (o < nv) q[o] = vals[o] / rad[o / nd];
}

// acc[0] += sum of part[0..n) (one block, fixed order)
__global__ void k_sum_parts(const float *part, int n, double *acc) {
    __shared__ double red[256];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) v += part[i];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) acc[0] += red[0];
}

// column mean and standard deviation of X [rows][cols] (one block per column,
// two passes in FP64); sd = 1 where the column is constant to 1e-6.
__global__ void k_colstats(const float *X, int64_t rows, int cols, float *mu, float *sd) {
    __shared__ double red[256];
    const int c = blockIdx.x;
    double s = 0.0;
    for (int64_t r = threadIdx.x; r < rows; r += 256) s += X[r * cols + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    const double m = red[0] / (double)rows;
    __syncthreads();
    double q = 0.0;
    for (int64_t r = threadIdx.x; r < rows; r += 256) {
        const double d = X[r * cols + c] - m;
        q += d * d;
    }
    red[threadIdx.x] = q;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double v = sqrt(red[0] / (double)rows);
        mu[c] = (float)m;
        sd[c] = v > 1e-6 ? (float)v : 1.f;
    }
}

// ---------------------------------------------------------------------------
// Host side

static int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

Mlp &mlp_get(bfm_ctx *c) {
    if (!c->mlp) c->mlp = new Mlp();
    return *c->mlp;
}

void mlp_free(bfm_ctx *c) {
    delete c->mlp;
    c->mlp = nullptr;
}

int64_t mlp_num_params(const Mlp &net) {
    int64_t n = 0;
    for (int k = 0; k < Mlp::kLayers; ++k) n += (int64_t)net.true_in(k) * net.true_out(k) + net.true_out(k);
    return n;
}

static void alloc_params(Mlp &net, hipStream_t st) {
    for (int k = 0; k < Mlp::kLayers; ++k) {
        const size_t nw = (size_t)net.dims[k] * net.dims[k + 1], no = net.dims[k + 1];
        for (DevBuf<float> *z : {&net.W[k], &net.mW[k], &net.vW[k], &net.dW[k]}) {
            z->ensure(nw);
            BFM_HIP(hipMemsetAsync(z->get(), 0, sizeof(float) * nw, st));
        }
        for (DevBuf<float> *z : {&net.b[k], &net.mb[k], &net.vb[k], &net.db[k]}) {
            z->ensure(no);
            BFM_HIP(hipMemsetAsync(z->get(), 0, sizeof(float) * no, st));
        }
        net.Wt[k].ensure(nw);
        net.Wn[k].ensure(nw);
    }
    net.adam_t = 0;
}

static void refresh(Mlp &net, hipStream_t st) {
    for (int k = 0; k < Mlp::kLayers; ++k) {
        const int in = net.dims[k], out = net.dims[k + 1];
        k_refresh<<<nblk((int64_t)in * out, 256), 256, 0, st>>>(net.W[k].get(), in, out, net.Wt[k].get(),
                                                                 net.Wn[k].get());
        BFM_LAUNCHED();
    }
}

static void default_norm(Mlp &net, hipStream_t st) {
    std::vector<float> h(Mlp::kNorm, 0.f);
    for (int i = 0; i < Mlp::kIn; ++i) h[Mlp::kIn + i] = 1.f;
    for (int i = 0; i < Mlp::kOut; ++i) h[2 * Mlp::kIn + Mlp::kOut + i] = 1.f;
    mlp_set_norm(net, h.data(), st);
    net.norm_set = false;
}

void mlp_init(Mlp &net, uint64_t seed, hipStream_t st) {
    alloc_params(net, st);
    std::mt19937_64 gen(seed);
    for (int k = 0; k < Mlp::kLayers; ++k) {
        const int out = net.dims[k + 1];
        const int ti = net.true_in(k), to = net.true_out(k);
        std::normal_distribution<float> nd(0.f, 1.f / std::sqrt((float)ti));
        std::vector<float> W((size_t)net.dims[k] * out, 0.f);
        for (int i = 0; i < ti; ++i)
            for (int o = 0; o < to; ++o) W[(size_t)i * out + o] = nd(gen);
        BFM_HIP(hipMemcpyAsync(net.W[k].get(), W.data(), sizeof(float) * W.size(), hipMemcpyHostToDevice, st));
    }
    refresh(net, st);
    if (!net.norm.get()) default_norm(net, st);
    BFM_HIP(hipStreamSynchronize(st));
    net.ready = true;
}

// flat host layout: for every layer W [true_in][true_out] row-major, then b [true_out]
void mlp_set_params(Mlp &net, const float *host, hipStream_t st) {
    alloc_params(net, st);
    const float *p = host;
    for (int k = 0; k < Mlp::kLayers; ++k) {
        const int out = net.dims[k + 1], ti = net.true_in(k), to = net.true_out(k);
        std::vector<float> W((size_t)net.dims[k] * out, 0.f), b(out, 0.f);
        for (int i = 0; i < ti; ++i)
            for (int o = 0; o < to; ++o) W[(size_t)i * out + o] = *p++;
        for (int o = 0; o < to; ++o) b[o] = *p++;
        BFM_HIP(hipMemcpyAsync(net.W[k].get(), W.data(), sizeof(float) * W.size(), hipMemcpyHostToDevice, st));
        BFM_HIP(hipMemcpyAsync(net.b[k].get(), b.data(), sizeof(float) * out, hipMemcpyHostToDevice, st));
        BFM_HIP(hipStreamSynchronize(st));
    }
    refresh(net, st);
    if (!net.norm.get()) default_norm(net, st);
    BFM_HIP(hipStreamSynchronize(st));
    net.ready = true;
}

void mlp_get_params(Mlp &net, float *host, bool grads, hipStream_t st) {
    BFM_CHECK(net.ready, BFM_EINVAL, "network not initialised");
    float *p = host;
    for (int k = 0; k < Mlp::kLayers; ++k) {
        const int out = net.dims[k + 1], ti = net.true_in(k), to = net.true_out(k);
        std::vector<float> W((size_t)net.dims[k] * out), b(out);
        BFM_HIP(hipMemcpyAsync(W.data(), (grads ? net.dW[k] : net.W[k]).get(), sizeof(float) * W.size(),
                               hipMemcpyDeviceToHost, st));
        BFM_HIP(hipMemcpyAsync(b.data(), (grads ? net.db[k] : net.b[k]).get(), sizeof(float) * out,
                               hipMemcpyDeviceToHost, st));
        BFM_HIP(hipStreamSynchronize(st));
        for (int i = 0; i < ti; ++i)
            for (int o = 0; o < to; ++o) *p++ = W[(size_t)i * out + o];
        for (int o = 0; o < to; ++o) *p++ = b[o];
    }
}

void mlp_set_norm(Mlp &net, const float *host, hipStream_t st) {
    for (int i = 0; i < Mlp::kIn; ++i)
        BFM_CHECK(host[Mlp::kIn + i] > 0.f, BFM_EINVAL, "standard deviations must be positive");
    for (int i = 0; i < Mlp::kOut; ++i)
        BFM_CHECK(host[2 * Mlp::kIn + Mlp::kOut + i] > 0.f, BFM_EINVAL, "standard deviations must be positive");
    net.norm.ensure(Mlp::kNorm);
    BFM_HIP(hipMemcpyAsync(net.norm.get(), host, sizeof(float) * Mlp::kNorm, hipMemcpyHostToDevice, st));
    BFM_HIP(hipStreamSynchronize(st));
    net.norm_set = true;
}

void mlp_get_norm(Mlp &net, float *host, hipStream_t st) {
    BFM_CHECK(net.norm.get(), BFM_EINVAL, "no standardisation set");
    BFM_HIP(hipMemcpyAsync(host, net.norm.get(), sizeof(float) * Mlp::kNorm, hipMemcpyDeviceToHost, st));
    BFM_HIP(hipStreamSynchronize(st));
}

static const float *mu_x(const Mlp &n) { return n.norm.get(); }
static const float *sd_x(const Mlp &n) { return n.norm.get() + Mlp::kIn; }
static const float *mu_y(const Mlp &n) { return n.norm.get() + 2 * Mlp::kIn; }
static const float *sd_y(const Mlp &n) { return n.norm.get() + 2 * Mlp::kIn + Mlp::kOut; }

static void gemm(int M, int N, int K, const __bf16 *A, int lda, const __bf16 *B, int ldb, float *C, int ldc,
                 const float *bias, hipStream_t st) {
    BFM_CHECK(K % 32 == 0 && lda % 8 == 0 && ldb % 8 == 0 && lda >= K && ldb >= K, BFM_EINVAL,
              "BF16 GEMM shape");
    dim3 g(nblk(M, 64), nblk(N, 64));
    k_gemm_bf16<<<g, 256, 0, st>>>(M, N, K, A, lda, B, ldb, C, ldc, bias, 0);
    BFM_LAUNCHED();
}

// Forward pass over R rows of X[0] (already standardised, BF16, zero padding).
static void forward(Mlp &net, int R, hipStream_t st) {
    for (int k = 0; k < Mlp::kLayers; ++k) {
        const int in = net.dims[k], out = net.dims[k + 1];
        float *Z = net.Z[k].ensure((size_t)R * out);
        gemm(R, out, in, net.X[k].get(), in, net.Wt[k].get(), in, Z, out, net.b[k].get(), st);
        if (k + 1 < Mlp::kLayers) {
            __bf16 *Xn = net.X[k + 1].ensure((size_t)R * out);
            k_act_bf16<<<nblk((int64_t)R * out, 256), 256, 0, st>>>(Z, (int64_t)R * out, 1, Xn);
            BFM_LAUNCHED();
        }
    }
}

// Backward pass for `rows` valid rows (of R) against standardised targets
// net.T [rows][kOut]; adds the summed loss to net.loss_acc[0].
static void backward(Mlp &net, int rows, int R, hipStream_t st) {
    const int L = Mlp::kLayers;
    const int outL = net.dims[L];
    float *G = net.G.ensure((size_t)R * Mlp::kHidden);
    const int nbk = (int)nblk((int64_t)R * outL, 256);
    float *part = net.part.ensure(nbk);
    k_loss_grad<<<nbk, 256, 0, st>>>(net.Z[L - 1].get(), net.T.get(), R, outL, Mlp::kOut, rows, G, part);
    BFM_LAUNCHED();
    k_sum_parts<<<1, 256, 0, st>>>(part, nbk, net.loss_acc.get());
    BFM_LAUNCHED();
    dim3 tb(32, 8);
    for (int k = L - 1; k >= 0; --k) {
        const int in = net.dims[k], out = net.dims[k + 1];
        // dW = X^T G ([in][out], K = R): both operands transposed so that K is contiguous
        __bf16 *XT = net.XT.ensure((size_t)in * R);
        __bf16 *GT = net.GT.ensure((size_t)out * R);
        k_transpose_bf16<__bf16><<<dim3(nblk(in, 32), nblk(R, 32)), tb, 0, st>>>(net.X[k].get(), R, in, XT);
        BFM_LAUNCHED();
        k_transpose_bf16<float><<<dim3(nblk(out, 32), nblk(R, 32)), tb, 0, st>>>(G, R, out, GT);
        BFM_LAUNCHED();
        gemm(in, out, R, XT, R, GT, R, net.dW[k].get(), out, nullptr, st);
        k_colsum<<<nblk(out, 256), 256, 0, st>>>(G, R, out, net.db[k].get());
        BFM_LAUNCHED();
        if (k > 0) {
            // dX = G W^T ([R][in], K = out), then through the SiLU of layer k - 1
            __bf16 *Gb = net.Gb.ensure((size_t)R * out);
            k_act_bf16<<<nblk((int64_t)R * out, 256), 256, 0, st>>>(G, (int64_t)R * out, 0, Gb);
            BFM_LAUNCHED();
            float *dX = net.dX.ensure((size_t)R * Mlp::kHidden);
            gemm(R, in, out, Gb, out, net.Wn[k].get(), out, dX, in, nullptr, st);
            k_silu_back<<<nblk((int64_t)R * in, 256), 256, 0, st>>>(dX, net.Z[k - 1].get(), (int64_t)R * in);
            BFM_LAUNCHED();
            std::swap(net.G.ptr, net.dX.ptr);
            std::swap(net.G.cap, net.dX.cap);
            G = net.G.get();
        }
    }
}

static void zero_loss(Mlp &net, hipStream_t st) {
    net.loss_acc.ensure(1);
    BFM_HIP(hipMemsetAsync(net.loss_acc.get(), 0, sizeof(double), st));
}

static double read_loss(Mlp &net, hipStream_t st) {
    double l = 0.0;
    BFM_HIP(hipMemcpyAsync(&l, net.loss_acc.get(), sizeof(double), hipMemcpyDeviceToHost, st));
    BFM_HIP(hipStreamSynchronize(st));
    return l;
}

void mlp_forward_rows(Mlp &net, int64_t rows, const float *x_dev, float *y_dev, hipStream_t st) {
    BFM_CHECK(net.ready, BFM_EINVAL, "network not initialised");
    BFM_CHECK(rows >= 1 && rows <= (1 << 24), BFM_EINVAL, "rows must be in [1, 2^24]");
    const int R = (int)round_up(rows, 64);
    __bf16 *X0 = net.X[0].ensure((size_t)R * Mlp::kInPad);
    k_batch_in<<<nblk((int64_t)R * Mlp::kInPad, 256), 256, 0, st>>>(x_dev, nullptr, 0, (int)rows, R, Mlp::kIn,
                                                                     Mlp::kInPad, mu_x(net), sd_x(net), X0);
    BFM_LAUNCHED();
    forward(net, R, st);
    k_unstd_rows<<<nblk(rows * Mlp::kOut, 256), 256, 0, st>>>(net.Z[Mlp::kLayers - 1].get(), (int)rows,
                                                               Mlp::kOutPad, Mlp::kOut, mu_y(net), sd_y(net), y_dev);
    BFM_LAUNCHED();
}

double mlp_gradient_rows(Mlp &net, int64_t rows, const float *x_dev, const float *t_dev, hipStream_t st) {
    BFM_CHECK(net.ready, BFM_EINVAL, "network not initialised");
    BFM_CHECK(rows >= 1 && rows <= (1 << 24), BFM_EINVAL, "rows must be in [1, 2^24]");
    const int R = (int)round_up(rows, 64);
    __bf16 *X0 = net.X[0].ensure((size_t)R * Mlp::kInPad);
    k_batch_in<<<nblk((int64_t)R * Mlp::kInPad, 256), 256, 0, st>>>(x_dev, nullptr, 0, (int)rows, R, Mlp::kIn,
                                                                     Mlp::kInPad, mu_x(net), sd_x(net), X0);
    BFM_LAUNCHED();
    float *T = net.T.ensure((size_t)rows * Mlp::kOut);
    k_batch_targ<<<nblk(rows * Mlp::kOut, 256), 256, 0, st>>>(t_dev, nullptr, 0, (int)rows, Mlp::kOut, mu_y(net),
                                                               sd_y(net), T);
    BFM_LAUNCHED();
    forward(net, R, st);
    zero_loss(net, st);
    backward(net, (int)rows, R, st);
    return read_loss(net, st) / (double)rows;
}

void mlp_adam(Mlp &net, float lr, hipStream_t st) {
    BFM_CHECK(net.ready, BFM_EINVAL, "network not initialised");
    net.adam_t += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float eps = 1e-8f;
    const float c1 = (float)(1.0 - std::pow(b1, net.adam_t)), c2 = (float)(1.0 - std::pow(b2, net.adam_t));
    for (int k = 0; k < Mlp::kLayers; ++k) {
        const int64_t nw = (int64_t)net.dims[k] * net.dims[k + 1];
        const int no = net.dims[k + 1];
        k_adam<<<nblk(nw, 256), 256, 0, st>>>(net.W[k].get(), net.dW[k].get(), net.mW[k].get(), net.vW[k].get(),
                                              nw, lr, (float)b1, (float)b2, eps, c1, c2);
        BFM_LAUNCHED();
        k_adam<<<nblk(no, 256), 256, 0, st>>>(net.b[k].get(), net.db[k].get(), net.mb[k].get(), net.vb[k].get(),
                                              no, lr, (float)b1, (float)b2, eps, c1, c2);
        BFM_LAUNCHED();
    }
    refresh(net, st);
}

void mlp_features(bfm_ctx *c, const double *phi_dev, const double *q_dev, float *feat, float *targ) {
    Mlp &net = mlp_get(c);
    Precond &P = c->pre;
    hipStream_t st = c->stream;
    BFM_CHECK(P.nd > 0 && P.genus == 0, BFM_EINVAL,
              "the learned guess needs a sphere template (bfm_set_sphere_template)");
    ensure_geometry(c);
    sh_basis_build(P, Mlp::kDegree, net.sh, st);
    const int nd = P.nd, nb = c->nb, nc = net.sh.nc;
    double *cen = net.cen.ensure(3 * (size_t)nb);
    double *rad = net.rad.ensure(nb);
    k_bubble_geom<<<nb, 256, 0, st>>>(c->xyz.get(), c->s.get(), nd, cen, rad);
    BFM_LAUNCHED();
    double *f1 = net.vbuf1.ensure(c->nv), *f2 = net.vbuf2.ensure(c->nv);
    k_vertex_fields<<<nblk(c->nv, 256), 256, 0, st>>>(c->xyz.get(), cen, rad, nd, c->nv, phi_dev, nullptr, f1, f2,
                                                      nullptr);
    BFM_LAUNCHED();
    double *crho = net.coef1.ensure((size_t)nc * nb), *cphi = net.coef2.ensure((size_t)nc * nb);
    gemm_nn_f64(nc, nb, nd, net.sh.Gp.get(), nc, f1, nd, crho, nc, st);
    gemm_nn_f64(nc, nb, nd, net.sh.Gp.get(), nc, f2, nd, cphi, nc, st);
    float *off = net.offs.ensure(12 * (size_t)nb);
    k_neighbours<<<nblk(nb, 128), 128, 0, st>>>(cen, rad, nb, off);
    BFM_LAUNCHED();
    k_assemble<<<nblk((int64_t)nb * Mlp::kIn, 256), 256, 0, st>>>(crho, cphi, off, nb, nc, feat);
    BFM_LAUNCHED();
    if (q_dev && targ) {
        k_vertex_fields<<<nblk(c->nv, 256), 256, 0, st>>>(c->xyz.get(), cen, rad, nd, c->nv, nullptr, q_dev,
                                                          nullptr, nullptr, f1);
        BFM_LAUNCHED();
        gemm_nn_f64(nc, nb, nd, net.sh.Gp.get(), nc, f1, nd, crho, nc, st);
        k_coef_rows<<<nblk((int64_t)nb * nc, 256), 256, 0, st>>>(crho, nb, nc, targ);
        BFM_LAUNCHED();
    }
}

void mlp_collect(bfm_ctx *c, const double *phi_dev, const double *q_dev) {
    Mlp &net = mlp_get(c);
    hipStream_t st = c->stream;
    const int nb = c->nb;
    const int64_t need = net.ds_rows + nb;
    if ((size_t)need * Mlp::kIn > net.ds_x.cap) {
        const int64_t cap = std::max<int64_t>(need, 2 * net.ds_rows);
        DevBuf<float> nx, ny;
        nx.ensure((size_t)cap * Mlp::kIn);
        ny.ensure((size_t)cap * Mlp::kOut);
        if (net.ds_rows > 0) {
            BFM_HIP(hipMemcpyAsync(nx.get(), net.ds_x.get(), sizeof(float) * net.ds_rows * Mlp::kIn,
                                   hipMemcpyDeviceToDevice, st));
            BFM_HIP(hipMemcpyAsync(ny.get(), net.ds_y.get(), sizeof(float) * net.ds_rows * Mlp::kOut,
                                   hipMemcpyDeviceToDevice, st));
        }
        BFM_HIP(hipStreamSynchronize(st));
        net.ds_x.swap(nx);
        net.ds_y.swap(ny);
    }
    mlp_features(c, phi_dev, q_dev, net.ds_x.get() + net.ds_rows * Mlp::kIn,
                 net.ds_y.get() + net.ds_rows * Mlp::kOut);
    BFM_HIP(hipStreamSynchronize(st));
    net.ds_rows = need;
}

double mlp_fit(bfm_ctx *c, int epochs, int batch, float lr, uint64_t seed) {
    Mlp &net = mlp_get(c);
    hipStream_t st = c->stream;
    const int64_t n = net.ds_rows;
    BFM_CHECK(n >= 1, BFM_EINVAL, "empty training set");
    BFM_CHECK(epochs >= 1 && batch >= 1 && batch <= 65536 && lr > 0.f, BFM_EINVAL,
              "epochs >= 1, batch in [1, 65536] and lr > 0 required");
    if (!net.ready) mlp_init(net, seed, st);
    if (!net.norm_set) {
        net.norm.ensure(Mlp::kNorm);
        float *nm = net.norm.get();
        k_colstats<<<Mlp::kIn, 256, 0, st>>>(net.ds_x.get(), n, Mlp::kIn, nm, nm + Mlp::kIn);
        BFM_LAUNCHED();
        k_colstats<<<Mlp::kOut, 256, 0, st>>>(net.ds_y.get(), n, Mlp::kOut, nm + 2 * Mlp::kIn,
                                              nm + 2 * Mlp::kIn + Mlp::kOut);
        BFM_LAUNCHED();
        net.norm_set = true;
    }
    const int B = (int)std::min<int64_t>(batch, n);
    const int R = (int)round_up(B, 64);
    net.X[0].ensure((size_t)R * Mlp::kInPad);
    net.T.ensure((size_t)B * Mlp::kOut);
    int *perm = net.perm.ensure(n);
    std::vector<int> order(n);
    std::mt19937_64 gen(seed ^ 0x9e3779b97f4a7c15ull);
    double last = 0.0;
    for (int ep = 0; ep < epochs; ++ep) {
        for (int64_t i = 0; i < n; ++i) order[i] = (int)i;
        std::shuffle(order.begin(), order.end(), gen);
        BFM_HIP(hipMemcpyAsync(perm, order.data(), sizeof(int) * n, hipMemcpyHostToDevice, st));
        zero_loss(net, st);
        for (int64_t off = 0; off + B <= n; off += B) {  // full batches only
            k_batch_in<<<nblk((int64_t)R * Mlp::kInPad, 256), 256, 0, st>>>(
                net.ds_x.get(), perm, off, B, R, Mlp::kIn, Mlp::kInPad, mu_x(net), sd_x(net), net.X[0].get());
            BFM_LAUNCHED();
            k_batch_targ<<<nblk((int64_t)B * Mlp::kOut, 256), 256, 0, st>>>(net.ds_y.get(), perm, off, B, Mlp::kOut,
                                                                            mu_y(net), sd_y(net), net.T.get());
            BFM_LAUNCHED();
            forward(net, R, st);
            backward(net, B, R, st);
            mlp_adam(net, lr, st);
        }
        last = read_loss(net, st) / (double)((n / B) * B);
    }
    return last;
}

void mlp_guess(bfm_ctx *c, const double *phi_dev, double *q_dev) {
    Mlp &net = mlp_get(c);
    hipStream_t st = c->stream;
    BFM_CHECK(net.ready && net.norm_set, BFM_EINVAL, "the learned guess needs a trained network");
    const int nb = c->nb, nd = c->pre.nd;
    const int R = (int)round_up(nb, 64);
    float *feat = net.feat.ensure((size_t)nb * Mlp::kIn);
    mlp_features(c, phi_dev, nullptr, feat, nullptr);
    __bf16 *X0 = net.X[0].ensure((size_t)R * Mlp::kInPad);
    k_batch_in<<<nblk((int64_t)R * Mlp::kInPad, 256), 256, 0, st>>>(feat, nullptr, 0, nb, R, Mlp::kIn, Mlp::kInPad,
                                                                     mu_x(net), sd_x(net), X0);
    BFM_LAUNCHED();
    forward(net, R, st);
    const int nc = Mlp::kNc;
    double *coef = net.coef2.ensure((size_t)nc * nb);
    k_unstandardise<<<nblk((int64_t)nb * nc, 256), 256, 0, st>>>(net.Z[Mlp::kLayers - 1].get(), nb, Mlp::kOutPad,
                                                                 nc, mu_y(net), sd_y(net), coef);
    BFM_LAUNCHED();
    double *vals = net.vbuf1.ensure(c->nv);
    gemm_nn_f64(nd, nb, nc, net.sh.G.get(), nd, coef, nc, vals, nd, st);
    k_guess_out<<<nblk(c->nv, 256), 256, 0, st>>>(vals, net.rad.get(), nd, c->nv, q_dev);
    BFM_LAUNCHED();
}

}  // namespace bfm
