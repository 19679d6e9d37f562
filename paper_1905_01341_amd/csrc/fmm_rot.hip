// Multipole-to-local translation by rotation (Section 3.9's M2L, factored):
// T(d) = B T_z(|d|) A, where A rotates a source box's multipole coefficients
// into a frame whose z axis points along the offset d, T_z translates along
// that axis, and B rotates the target's local coefficients back (ops.cpp).
// A and B are block diagonal by degree ((2n+1)^2 per degree) and T_z couples
// only equal orders ((p-m)^2 per order m, shared by the cosine and sine
// parts), so a translated column costs about 2 (2 sum (2n+1)^2 + sum
// (p-|m|)^2) flops instead of 2 p^4: 4p^3 against 2p^4.
//
// On the matrix cores: a workgroup of 4 waves owns 16 columns (task x
// channel) of one operator's group. Every stage is D = Op X on
// v_mfma_f64_16x16x4f64 with the operator block as the A operand and the
// columns as B, so lane l of a 16 x 16 result holds rows l/16 + 4r of column
// l%16. Stage 1 (per degree, split over the waves) reads the input columns
// from memory and writes the rotated coefficients to one LDS buffer of
// p^2 x 16 doubles; stage 2 (per order and part, split over the waves)
// translates in place in LDS; stage 3 (per degree) rotates back and adds the
// result to the target expansions atomically. The operator blocks are
// stored in the order the A operand is read: for each 16-row chunk and
// 4-wide K step of a block, 64 values in lane order, so one MFMA's operand is
// one coalesced 512-byte load.
#include <utility>
#include <vector>

#include "fmm_kernels.h"
#include "ops.h"

namespace bfm {

typedef double rot_dbl4 __attribute__((ext_vector_type(4)));

constexpr int rot_cdiv(int a, int b) { return (a + b - 1) / b; }
// MFMA operand blocks (16 rows x 4 K) of degree n's rotation block
constexpr int rot_blocks(int n) { return rot_cdiv(2 * n + 1, 16) * rot_cdiv(2 * n + 1, 4); }
// offset (doubles) of degree n's blocks in one operator's rotation array
constexpr int rot_moff(int n) {
    int o = 0;
    for (int q = 0; q < n; ++q) o += rot_blocks(q) * 64;
    return o;
}
// the same for order m of a translation along z stored at order ps
constexpr int tz_blocks(int ps, int m) { return rot_cdiv(ps - m, 16) * rot_cdiv(ps - m, 4); }
constexpr int tz_moff(int ps, int m) {
    int o = 0;
    for (int q = 0; q < m; ++q) o += tz_blocks(ps, q) * 64;
    return o;
}

template <int I>
using rot_int = std::integral_constant<int, I>;
template <int I0, int I1, class F>
__device__ inline void rot_static_for(F &&f) {
    if constexpr (I0 < I1) {
        f(rot_int<I0>{});
        rot_static_for<I0 + 1, I1>(f);
    }
}

// One degree of a rotation stage (A on the way in, B on the way out) for
// one wave: the degree's input coefficients of the 16 columns (from memory
// in stage 1, from LDS in stage 3), NC x NK MFMAs, then the result rows (to
// LDS, or added to the target expansions). Loads and LDS stores are
// unconditional (clamped addresses, selects; rows past the degree go to a
// spare row after the buffer) so that a wave's whole stage is one basic
// block the compiler can schedule: the operator and input loads of later
// degrees are issued while earlier degrees multiply.
template <int N, int PO, bool BACK>
__device__ inline void rot_degree(const double *__restrict__ op, const double *__restrict__ src, double *X, int kq,
                                  int cl, bool ok, double *outcol) {
    constexpr int S = 2 * N + 1, NC = rot_cdiv(S, 16), NK = rot_cdiv(S, 4), OFF = rot_moff(N);
    double b[NK];
#pragma unroll
    for (int kk = 0; kk < NK; ++kk) {
        const int k = 4 * kk + kq;
        const int kc = k < S ? k : S - 1;
        const double v = BACK ? X[(N * N + kc) * 16 + cl] : src[N * N + kc];
        b[kk] = (k < S && (BACK || ok)) ? v : 0.0;
    }
    double a[NC * NK];  // the degree's operator operands, all in flight before the first MFMA
#pragma unroll
    for (int e = 0; e < NC * NK; ++e) a[e] = op[OFF + e * 64];
    rot_dbl4 acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = rot_dbl4{0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < NK; ++kk)
#pragma unroll
        for (int c = 0; c < NC; ++c)
            acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c * NK + kk], b[kk], acc[c], 0, 0, 0);
    if (!BACK) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = c * 16 + kq + 4 * r;
                X[(row < S ? N * N + row : PO * PO) * 16 + cl] = acc[c][r];
            }
    } else if (ok) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = c * 16 + kq + 4 * r;
                if (row < S) unsafeAtomicAdd(outcol + N * N + row, acc[c][r]);
            }
    }
}

// One (order, part) of the translation along z, in place in LDS: item 0 is
// order 0, item 2m - 1 + part the cosine (0) or sine (1) part of order m.
template <int T, int PO, int PS>
__device__ inline void tz_item(const double *__restrict__ tz, double *X, int kq, int cl) {
    constexpr int M = (T + 1) / 2, PART = T == 0 ? 0 : (T + 1) % 2;
    constexpr int W = PO - M, NC = rot_cdiv(W, 16), NK = rot_cdiv(W, 4);
    constexpr int NKS = rot_cdiv(PS - M, 4), OFF = tz_moff(PS, M);
    auto slot = [](int n) { return M == 0 ? n * n : n * n + 2 * M - 1 + PART; };
    double b[NK];
#pragma unroll
    for (int kk = 0; kk < NK; ++kk) {
        const int k = 4 * kk + kq;
        const double v = X[slot(M + (k < W ? k : W - 1)) * 16 + cl];
        b[kk] = k < W ? v : 0.0;
    }
    double a[NC * NK];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) a[c * NK + kk] = tz[OFF + (c * NKS + kk) * 64];
    rot_dbl4 acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = rot_dbl4{0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < NK; ++kk)
#pragma unroll
        for (int c = 0; c < NC; ++c)
            acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c * NK + kk], b[kk], acc[c], 0, 0, 0);
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = c * 16 + kq + 4 * r;
            X[(row < W ? slot(M + row) : PO * PO) * 16 + cl] = acc[c][r];
        }
}

// Wave w's share of each stage: degrees w, w + 4, ... (rotations) and items
// w, w + 4, ... (translation), as straight-line code.
template <int W, int PO, bool BACK>
__device__ inline void rot_stage(const double *__restrict__ op, const double *__restrict__ src, double *X, int kq,
                                 int cl, bool ok, double *outcol) {
    rot_static_for<0, rot_cdiv(PO - W, 4)>([&](auto ic) {
        constexpr int N = W + 4 * decltype(ic)::value;
        rot_degree<N, PO, BACK>(op, src, X, kq, cl, ok, outcol);
    });
}
template <int W, int PO, int PS>
__device__ inline void tz_stage(const double *__restrict__ tz, double *X, int kq, int cl) {
    rot_static_for<0, rot_cdiv(2 * PO - 1 - W, 4)>([&](auto ic) {
        constexpr int T = W + 4 * decltype(ic)::value;
        tz_item<T, PO, PS>(tz, X, kq, cl);
    });
}

// PO: the order applied (degrees 0..PO-1, the leading blocks); PS: the
// order the operators and expansions are stored at.
// Occupancy is set by the LDS buffer (3 workgroups per CU at PO = 20, 4 at
// 16), so the register budget may follow it: the operands of a degree stay
// in flight together instead of one load per MFMA.
constexpr int rot_waves_per_eu(int po) { return po >= 20 ? 3 : (po >= 16 ? 4 : 6); }
template <int PO, int PS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, rot_waves_per_eu(PO)))) k_m2l_rot(int op0, int nops, const int *tile_off, int g0, int ntiles,
                                                 const int *op_off, const int *tsrc, const int *tdst, int nch,
                                                 const double *RA, const double *TZ, const double *RB,
                                                 const double *in, double *out) {
    static_assert(PO <= PS && PS <= kMaxP && PO >= 4, "orders");
    constexpr int LD = PS * PS;
    constexpr int RSZ = rot_moff(PS), TSZ = tz_moff(PS, PS);
    __shared__ double X[(PO * PO + 1) * 16];  // [coefficient][column], then a spare row
    // XCD-aware order: XCD x takes a contiguous run of logical tiles (the
    // tiles of a few operators), so each XCD reads an operator into its L2
    const int nblock = gridDim.x, per = nblock / 8, rem = nblock % 8;
    const int xcd = blockIdx.x % 8, idx = blockIdx.x / 8;
    const int logical = xcd * per + (xcd < rem ? xcd : rem) + idx;
    if (logical >= ntiles) return;
    const int g = g0 + logical;
    int lo = op0, hi = op0 + nops;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tile_off[mid] <= g)
            lo = mid;
        else
            hi = mid;
    }
    const int op = lo;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kq = lane >> 4, cl = lane & 15;
    const int t0 = op_off[op];
    const int ncols = (op_off[op + 1] - t0) * nch;
    const int col = (g - tile_off[op]) * 16 + cl;
    const bool ok = col < ncols;
    const int task = t0 + (ok ? col / nch : 0), ch = ok ? col % nch : 0;
    // idle columns read box 0's expansion (valid memory) and are never stored
    const double *incol = in + ((int64_t)(ok ? tsrc[task] : 0) * nch + ch) * LD;
    double *outcol = out + ((int64_t)(ok ? tdst[task] : 0) * nch + ch) * LD;
    const double *ra = RA + (int64_t)op * RSZ + lane;
    const double *rb = RB + (int64_t)op * RSZ + lane;
    const double *tz = TZ + (int64_t)op * TSZ + lane;
    // stage 1: rotate into the offset's frame (memory -> LDS)
    switch (wave) {
        case 0: rot_stage<0, PO, false>(ra, incol, X, kq, cl, ok, outcol); break;
        case 1: rot_stage<1, PO, false>(ra, incol, X, kq, cl, ok, outcol); break;
        case 2: rot_stage<2, PO, false>(ra, incol, X, kq, cl, ok, outcol); break;
        default: rot_stage<3, PO, false>(ra, incol, X, kq, cl, ok, outcol); break;
    }
    __syncthreads();
    // stage 2: translate along the axis (LDS, in place)
    switch (wave) {
        case 0: tz_stage<0, PO, PS>(tz, X, kq, cl); break;
        case 1: tz_stage<1, PO, PS>(tz, X, kq, cl); break;
        case 2: tz_stage<2, PO, PS>(tz, X, kq, cl); break;
        default: tz_stage<3, PO, PS>(tz, X, kq, cl); break;
    }
    __syncthreads();
    // stage 3: rotate back and add to the target expansions (LDS -> memory)
    switch (wave) {
        case 0: rot_stage<0, PO, true>(rb, incol, X, kq, cl, ok, outcol); break;
        case 1: rot_stage<1, PO, true>(rb, incol, X, kq, cl, ok, outcol); break;
        case 2: rot_stage<2, PO, true>(rb, incol, X, kq, cl, ok, outcol); break;
        default: rot_stage<3, PO, true>(rb, incol, X, kq, cl, ok, outcol); break;
    }
}

// Rotation-factored operators of order p in the kernel's operand order
// (built once per process and p, from build_m2l_rot).
static void host_rot_ops(int p, const std::vector<double> *&ra, const std::vector<double> *&tz,
                         const std::vector<double> *&rb) {
    static std::vector<double> cache[kMaxP + 1][3];
    std::vector<double>(&c3)[3] = cache[p];
    if (c3[0].empty()) {
        const int rsz = rot_moff(p), tsz = tz_moff(p, p);
        std::vector<double> A((size_t)kNumM2LOps * rsz, 0.0), Z((size_t)kNumM2LOps * tsz, 0.0),
            B((size_t)kNumM2LOps * rsz, 0.0);
        const int nr = m2l_rot_offset(p), nz = m2l_tz_offset(p, p);
#pragma omp parallel for schedule(dynamic)
        for (int op = 0; op < kNumM2LOps; ++op) {
            std::vector<double> a(nr), z(nz), b(nr);
            build_m2l_rot(p, op, a.data(), z.data(), b.data());
            // rotation blocks: (chunk c, K step kk, lane) -> (row c*16 + lane%16, k 4 kk + lane/16)
            for (int n = 0; n < p; ++n) {
                const int s = 2 * n + 1, nk = rot_cdiv(s, 4), ncb = rot_cdiv(s, 16);
                for (int c = 0; c < ncb; ++c)
                    for (int kk = 0; kk < nk; ++kk)
                        for (int l = 0; l < 64; ++l) {
                            const int i = c * 16 + (l & 15), k = 4 * kk + (l >> 4);
                            const size_t o = (size_t)op * rsz + rot_moff(n) + (c * nk + kk) * 64 + l;
                            if (i < s && k < s) {
                                A[o] = a[m2l_rot_offset(n) + i * s + k];
                                B[o] = b[m2l_rot_offset(n) + i * s + k];
                            }
                        }
            }
            for (int m = 0; m < p; ++m) {
                const int w = p - m, nk = rot_cdiv(w, 4), ncb = rot_cdiv(w, 16);
                for (int c = 0; c < ncb; ++c)
                    for (int kk = 0; kk < nk; ++kk)
                        for (int l = 0; l < 64; ++l) {
                            const int i = c * 16 + (l & 15), k = 4 * kk + (l >> 4);
                            if (i < w && k < w)
                                Z[(size_t)op * tsz + tz_moff(p, m) + (c * nk + kk) * 64 + l] =
                                    z[m2l_tz_offset(p, m) + i * w + k];
                        }
            }
        }
        c3[0].swap(A);
        c3[1].swap(Z);
        c3[2].swap(B);
    }
    ra = &c3[0];
    tz = &c3[1];
    rb = &c3[2];
}

void rot_ops_upload(FmmWork &w, int p, hipStream_t st) {
    if (w.rot_p == p) return;
    const std::vector<double> *ra, *tz, *rb;
    host_rot_ops(p, ra, tz, rb);
    auto up = [&](DevBuf<double> &d, const std::vector<double> &h) {
        d.ensure(h.size());
        BFM_HIP(hipMemcpyAsync(d.get(), h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, st));
    };
    up(w.rot_a, *ra);
    up(w.rot_z, *tz);
    up(w.rot_b, *rb);
    BFM_HIP(hipStreamSynchronize(st));
    w.rot_p = p;
}

template <int PO, int PS>
void launch_m2l_rot(const FmmWork &w, int op0, int nops, int g0, int ntiles, const int *tile_off,
                    const TaskList &tl, int nch, const double *in, double *out, hipStream_t st) {
    if (ntiles <= 0) return;
    BFM_CHECK(w.rot_p == PS, BFM_EINVAL, "rotation operators not prepared");
    k_m2l_rot<PO, PS><<<(unsigned)ntiles, 256, 0, st>>>(op0, nops, tile_off, g0, ntiles, tl.op_off.get(),
                                                       tl.src.get(), tl.dst.get(), nch, w.rot_a.get(),
                                                       w.rot_z.get(), w.rot_b.get(), in, out);
    BFM_LAUNCHED();
}

#define BFM_ROT(PO, PS)                                                                                              \
    template void launch_m2l_rot<PO, PS>(const FmmWork &, int, int, int, int, const int *, const TaskList &, int, \
                                         const double *, double *, hipStream_t);
BFM_ROT(4, 4)
BFM_ROT(8, 8)
BFM_ROT(12, 12)
BFM_ROT(16, 16)
BFM_ROT(12, 16)
BFM_ROT(20, 20)
BFM_ROT(16, 20)
BFM_ROT(12, 20)
BFM_ROT(4, 8)
BFM_ROT(8, 12)
BFM_ROT(8, 16)
#undef BFM_ROT

}  // namespace bfm
