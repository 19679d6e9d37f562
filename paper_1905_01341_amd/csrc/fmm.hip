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
// wave multiplies one P x P operator by 16 gathered expansion columns on the
// matrix cores and adds the result into the target expansions atomically.
// Arithmetic by product group: FP64 MFMA (v_mfma_f64_16x16x4f64) for the
// FP64 products; for the low-precision products of iterative refinement,
// FP32 expansions with FP32 MFMA (v_mfma_f32_16x16x4f32) or with split-BF16
// operands (a = hi + lo, hi = bf16(a), lo = bf16(a - hi)) on
// v_mfma_f32_16x16x32_bf16: three products hi*hi + hi*lo + lo*hi accumulated
// in FP32.
#include <hip/hip_bf16.h>

#include <cmath>
#include <type_traits>
#include <cstring>
#include <vector>

#include "fmm_kernels.h"
#include "ops.h"

namespace bfm {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// One 16 x 16 x 4 matrix-core step per operand type. Operand layout (both
// types): A[i][k] from lane 16 k + i, B[k][j] from lane 16 k + j. Result
// layout: lane l, element r holds column l % 16 and row rowof(l / 16, r).
template <class T>
struct Mma;
template <>
struct Mma<double> {
    typedef dbl4 acc_t;
    static __device__ inline acc_t step(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ inline int rowof(int q, int r) { return q + 4 * r; }
};
template <>
struct Mma<float> {
    typedef flt4 acc_t;
    static __device__ inline acc_t step(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ inline int rowof(int q, int r) { return 4 * q + r; }
};

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

// LD: stored order (expansions and operators hold LD = p^2 coefficients);
// PP <= LD: the order applied (the leading PP x PP block of each operator,
// degrees below sqrt(PP)) - smaller for distant offsets when the product
// reduces their order. The launch covers operators op0 .. op0 + nops - 1,
// whose tiles are g0 .. g0 + ntiles - 1 of the prefix tile_off.
template <int PP, int ROWS, int WAVES, int KIND, class R = double, int LD = PP>
__global__ void __launch_bounds__(64 * WAVES) k_translate(int op0, int nops, const int *tile_off, int g0,
                                                          int ntiles, const int *op_off, const int *tsrc,
                                                          const int *tdst, int nch, int swap,
                                                          const R *T, const R *in, R *out) {
    static_assert(PP % ROWS == 0 && ROWS % 16 == 0 && PP <= LD, "row slab");
    constexpr int NSLAB = PP / ROWS;
    __shared__ R As[2][kTKC * ROWS];         // two buffers of [k][row within slab]
    __shared__ R Bs[2][WAVES][kTKC / 4][64];  // two buffers of each wave's input chunk
    // XCD-aware order: workgroups are dealt round-robin to the 8 XCDs, so
    // XCD x takes a contiguous run of logical blocks (the tiles of a few
    // operators) and fetches each operator into its own L2 once
    const int nblock = gridDim.x, per = nblock / kXcds, rem = nblock % kXcds;
    const int xcd = blockIdx.x % kXcds, idx = blockIdx.x / kXcds;
    const int logical = xcd * per + (xcd < rem ? xcd : rem) + idx;
    if (logical / NSLAB >= ntiles) return;
    const int g = g0 + logical / NSLAB, slab = logical % NSLAB;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    int lo = op0, hi = op0 + nops;
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
    // idle columns read box 0's expansion (valid memory) and are never stored
    const R *bcol = in + ((int64_t)sb * nch + bch) * LD;
    const R *Top = T + (int64_t)op * LD * LD + slab * ROWS;
    const int kq = lane >> 4, rl = lane & 15;
    typename Mma<R>::acc_t acc[ROWS / 16];
#pragma unroll
    for (int rb = 0; rb < ROWS / 16; ++rb) acc[rb] = typename Mma<R>::acc_t{0, 0, 0, 0};
    // Operator slab chunks and the input columns go global -> registers ->
    // LDS (two LDS buffers); the loop is unrolled by three with no register
    // copies between the stages.
    constexpr int NT = 64 * WAVES;
    constexpr int PER = (kTKC * ROWS + NT - 1) / NT;
    constexpr bool EXACT = PER * NT == kTKC * ROWS;  // every thread moves PER elements
    static_assert(PP % kTKC == 0, "whole chunks");
    constexpr int NC = PP / kTKC;
    // three register sets take turns: while chunk c feeds the MFMAs from LDS,
    // chunk c + 1 waits in registers for its LDS buffer and chunk c + 2 is
    // being loaded, so a load has two chunks' MFMA time to arrive
    R pa[PER], pb[PER], pc[PER], ba[kTKC / 4], bb[kTKC / 4], bc[kTKC / 4];
    auto fetch = [&](int k0, R(&pre)[PER], R(&bv)[kTKC / 4]) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + u * NT;
            if (EXACT || e < kTKC * ROWS) pre[u] = Top[(int64_t)(k0 + e / ROWS) * LD + e % ROWS];
        }
#pragma unroll
        for (int kk = 0; kk < kTKC / 4; ++kk) bv[kk] = bcol[k0 + 4 * kk + kq];
    };
    // the chunk's operator slab and input columns -> LDS buffer `buf`
    auto stash = [&](int buf, const R(&pre)[PER], const R(&bv)[kTKC / 4]) {
#pragma unroll
        for (int u = 0; u < PER; ++u)
            if (EXACT || tid + u * NT < kTKC * ROWS) As[buf][tid + u * NT] = pre[u];
#pragma unroll
        for (int kk = 0; kk < kTKC / 4; ++kk) Bs[buf][wave][kk][lane] = bok ? bv[kk] : R(0);
    };
    // the MFMAs of one chunk read only LDS, so no wait on the loads in flight
    auto mult = [&](int buf) {
#pragma unroll
        for (int kk = 0; kk < kTKC / 4; ++kk) {
            const R *Ak = As[buf] + (4 * kk + kq) * ROWS + rl;
            const R b = Bs[buf][wave][kk][lane];
#pragma unroll
            for (int rb = 0; rb < ROWS / 16; ++rb) acc[rb] = Mma<R>::step(b, Ak[rb * 16], acc[rb]);
        }
    };
    fetch(0, pa, ba);
    stash(0, pa, ba);
    fetch(min(1, NC - 1) * kTKC, pb, bb);
    __syncthreads();
    // the fetches are unconditional (past the end they repeat the last
    // chunk) so that the memory-counter waits are the same on every path;
    // fully unrolled, so that the accumulators keep their registers across
    // the loop's exits (a rolled loop copies them at every pass)
#pragma unroll
    for (int c = 0; c < NC; c += 3) {
        // chunk c in LDS buffer c & 1, c + 1 in (pb, bb); load c + 2 into (pc, bc)
        fetch(min(c + 2, NC - 1) * kTKC, pc, bc);
        mult(c & 1);
        if (c + 1 >= NC) break;
        stash((c + 1) & 1, pb, bb);
        __syncthreads();
        // chunk c + 1; c + 2 in (pc, bc); load c + 3 into (pa, ba)
        fetch(min(c + 3, NC - 1) * kTKC, pa, ba);
        mult((c + 1) & 1);
        if (c + 2 >= NC) break;
        stash(c & 1, pc, bc);
        __syncthreads();
        // chunk c + 2; c + 3 in (pa, ba); load c + 4 into (pb, bb)
        fetch(min(c + 4, NC - 1) * kTKC, pb, bb);
        mult(c & 1);
        if (c + 3 >= NC) break;
        stash((c + 1) & 1, pa, ba);
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int col = colbase + Mma<R>::rowof(kq, r);
        if (col >= ncols) continue;
        const int task = t0 + col / nch, ch = col % nch;
        const int db = swap ? tsrc[task] : tdst[task];
        R *dcol = out + ((int64_t)db * nch + ch) * LD + slab * ROWS + rl;
#pragma unroll
        for (int rb = 0; rb < ROWS / 16; ++rb) unsafeAtomicAdd(dcol + rb * 16, acc[rb][r]);
    }
}

// ---------------------------------------------------------------------------
// Split-BF16 translation (low-precision products). A workgroup of four waves
// owns 128 columns (32 per wave: two blocks of 16) of one operator's group
// and a slab of ROWS output rows. K runs in chunks of 32 (the operator's K
// is zero-padded to KP, a multiple of 32). The operator's hi and lo parts
// are stored chunk-major ([op][chunk][row][32 k], BF16), so a chunk of a
// slab is one contiguous run; it passes global -> registers -> LDS (two
// buffers) and is shared by the four waves. Each wave splits its own input
// columns (FP32) into hi and lo in registers as it loads them. Per chunk,
// row block and column block: hi*hi + hi*lo + lo*hi on
// v_mfma_f32_16x16x32_bf16 (lane l: A row l % 16, B column l % 16, k =
// 8 (l / 16) + 0..7; result column l % 16, rows 4 (l / 16) + 0..3).
constexpr int kBfWaves = 4, kBfCb = 2, kBfTile = kBfWaves * kBfCb * 16;  // 128 columns
constexpr int kBfRs = 5;  // LDS row stride in 16-byte units (4 used, 1 pad: conflict-free reads)

__device__ inline void split8(const float *v, bool ok, bf16x8 &hi, bf16x8 &lo) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const float a = ok ? v[e] : 0.f;
        const __bf16 h = (__bf16)a;
        hi[e] = h;
        lo[e] = (__bf16)(a - (float)h);
    }
}

// STORE: the result of every task is stored (out = [task][LD]) for a
// reduction per target box instead of added atomically into the target.
// LD, PP, op0, g0 as for k_translate (the operators hold LD rows and
// round-up(LD, 32) / 32 chunks; K beyond PP is masked through the input).
template <int PP, int ROWS, int KIND, bool STORE, int LD = PP>
__global__ void __launch_bounds__(64 * kBfWaves) k_translate_bf3(int op0, int nops, const int *tile_off, int g0,
                                                                 int ntiles,
                                                                 const int *op_off, const int *tsrc,
                                                                 const int *tdst, int nch, int swap,
                                                                 const uint4 *Thi, const uint4 *Tlo,
                                                                 const float *in, float *out) {
    static_assert(PP % ROWS == 0 && ROWS % 16 == 0 && PP <= LD, "row slab");
    constexpr int KP = (PP + 31) / 32 * 32, NC = KP / 32, NSLAB = PP / ROWS, RB = ROWS / 16;
    constexpr int NCF = (LD + 31) / 32;  // chunks of the stored operators
    constexpr int NST = ROWS * 4;  // 16-byte units of one part (hi or lo) of a chunk's slab
    constexpr int NT = 64 * kBfWaves;
    constexpr int PER = (2 * NST + NT - 1) / NT;
    __shared__ uint4 Bh[2][ROWS * kBfRs], Bl[2][ROWS * kBfRs];
    const int nblock = gridDim.x, per = nblock / kXcds, rem = nblock % kXcds;
    const int xcd = blockIdx.x % kXcds, idx = blockIdx.x / kXcds;
    const int logical = xcd * per + (xcd < rem ? xcd : rem) + idx;
    if (logical / NSLAB >= ntiles) return;
    const int g = g0 + logical / NSLAB, slab = logical % NSLAB;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    int lo = op0, hi = op0 + nops;
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
    const int colbase = (g - tile_off[op]) * kBfTile + wave * (kBfCb * 16);
    const int kq = lane >> 4, rl = lane & 15;
    const float *acol[kBfCb];
    bool aok[kBfCb];
#pragma unroll
    for (int cb = 0; cb < kBfCb; ++cb) {
        const int col = colbase + cb * 16 + rl;
        aok[cb] = col < ncols;
        const int task = t0 + (aok[cb] ? col / nch : 0);
        const int ch = aok[cb] ? col % nch : 0;
        const int sb = aok[cb] ? (swap ? tdst[task] : tsrc[task]) : 0;
        acol[cb] = in + ((int64_t)sb * nch + ch) * LD;
    }
    // chunk c of this slab: 16-byte unit u (row u / 4, k group u % 4)
    const uint4 *sh = Thi + ((int64_t)op * NCF * LD + slab * ROWS) * 4;
    const uint4 *sl = Tlo + ((int64_t)op * NCF * LD + slab * ROWS) * 4;
    uint4 pre[PER];
    auto fetch_op = [&](int c) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + u * NT;
            if (e < 2 * NST) {
                const int part = e / NST, v = e - part * NST;
                pre[u] = (part ? sl : sh)[(int64_t)c * LD * 4 + v];
            }
        }
    };
    auto stash_op = [&](int buf) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + u * NT;
            if (e < 2 * NST) {
                const int part = e / NST, v = e - part * NST;
                (part ? Bl : Bh)[buf][(v >> 2) * kBfRs + (v & 3)] = pre[u];
            }
        }
    };
    float av[kBfCb][8];
    auto fetch_in = [&](int c) {
        const int k = c * 32 + 8 * kq;
#pragma unroll
        for (int cb = 0; cb < kBfCb; ++cb) {
            if (aok[cb] && k < PP) {
                const float4 u0 = *reinterpret_cast<const float4 *>(acol[cb] + k);
                const float4 u1 = *reinterpret_cast<const float4 *>(acol[cb] + k + 4);
                av[cb][0] = u0.x;
                av[cb][1] = u0.y;
                av[cb][2] = u0.z;
                av[cb][3] = u0.w;
                av[cb][4] = u1.x;
                av[cb][5] = u1.y;
                av[cb][6] = u1.z;
                av[cb][7] = u1.w;
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) av[cb][e] = 0.f;
            }
        }
    };
    flt4 acc[kBfCb][RB];
#pragma unroll
    for (int cb = 0; cb < kBfCb; ++cb)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) acc[cb][rb] = flt4{0.f, 0.f, 0.f, 0.f};
    fetch_op(0);
    fetch_in(0);
    stash_op(0);
    __syncthreads();
#pragma unroll 1
    for (int c = 0; c < NC; ++c) {
        const int buf = c & 1;
        bf16x8 ah[kBfCb], al[kBfCb];
#pragma unroll
        for (int cb = 0; cb < kBfCb; ++cb) split8(av[cb], true, ah[cb], al[cb]);
        if (c + 1 < NC) {  // next chunk's loads overlap this chunk's products
            fetch_op(c + 1);
            fetch_in(c + 1);
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const uint4 uh = Bh[buf][(rb * 16 + rl) * kBfRs + kq];
            const uint4 ul = Bl[buf][(rb * 16 + rl) * kBfRs + kq];
            bf16x8 bh, bl;
            memcpy(&bh, &uh, 16);
            memcpy(&bl, &ul, 16);
#pragma unroll
            for (int cb = 0; cb < kBfCb; ++cb) {
                acc[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[cb], bh, acc[cb][rb], 0, 0, 0);
                acc[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[cb], bl, acc[cb][rb], 0, 0, 0);
                acc[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[cb], bh, acc[cb][rb], 0, 0, 0);
            }
        }
        if (c + 1 < NC) {
            stash_op(buf ^ 1);
            __syncthreads();
        }
    }
#pragma unroll
    for (int cb = 0; cb < kBfCb; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int col = colbase + cb * 16 + 4 * kq + r;
            if (col >= ncols) continue;
            const int task = t0 + col / nch, ch = col % nch;
            if (STORE) {
                float *dcol = out + ((int64_t)(t0 * nch + col)) * LD + slab * ROWS + rl;
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) dcol[rb * 16] = acc[cb][rb][r];
            } else {
                const int db = swap ? tsrc[task] : tdst[task];
                float *dcol = out + ((int64_t)db * nch + ch) * LD + slab * ROWS + rl;
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) unsafeAtomicAdd(dcol + rb * 16, acc[cb][rb][r]);
            }
        }
}

// L[b] = sum of the stored M2L results of target box b's tasks, in the order
// the tasks were generated (fixed, so the sum is reproducible). One wave per
// target box: a row of LD coefficients is LD / 4 float4 groups; when that is
// under 64, the wave's lanes form G = 64 / (LD / 4) groups that take every
// G-th task (two tasks' loads in flight per lane), and the groups' sums are
// added by lane shuffles in a fixed order. Tasks at grouped positions >=
// cut1 (>= cut2) belong to the second (third) distance class and carry only
// their first pp1 (pp2) coefficients.
template <int LD>
__global__ void __launch_bounds__(64) k_m2l_reduce(const int *dst_off, const int *pos_of, int64_t box0, int cut1,
                                                   int cut2, int pp1, int pp2, const float *part, float *L) {
    static_assert(LD % 4 == 0, "whole float4 groups");
    constexpr int NV = LD / 4;
    constexpr int G = NV >= 64 ? 1 : 64 / NV;
    static_assert(G == 1 || G * NV == 64, "groups tile the wave");
    const int64_t k = blockIdx.x;
    const int a = dst_off[k], e = dst_off[k + 1];
    if (a == e) return;  // no far-field sources at this box's level (L stays zero)
    float *lb = L + (box0 + k) * LD;
    const int lane = threadIdx.x, grp = lane / (G > 1 ? NV : 64);
    auto add = [](float4 &s, const float4 v) {
        s.x += v.x;
        s.y += v.y;
        s.z += v.z;
        s.w += v.w;
    };
    for (int c0 = 0; c0 < NV; c0 += (G > 1 ? NV : 64)) {
        const int cv = c0 + (G > 1 ? lane % NV : lane);  // this lane's float4 group
        const int c = 4 * cv;
        float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
        if (cv < NV) {
            int i = a + grp;
            for (; i + G < e; i += 2 * G) {
                const int p0 = pos_of[i], p1 = pos_of[i + G];
                const int q0 = p0 >= cut2 ? pp2 : (p0 >= cut1 ? pp1 : LD);
                const int q1 = p1 >= cut2 ? pp2 : (p1 >= cut1 ? pp1 : LD);
                const float4 v0 = c < q0 ? *reinterpret_cast<const float4 *>(part + (int64_t)p0 * LD + c)
                                         : make_float4(0.f, 0.f, 0.f, 0.f);
                const float4 v1 = c < q1 ? *reinterpret_cast<const float4 *>(part + (int64_t)p1 * LD + c)
                                         : make_float4(0.f, 0.f, 0.f, 0.f);
                add(s, v0);
                add(s, v1);
            }
            if (i < e) {
                const int p0 = pos_of[i];
                const int q0 = p0 >= cut2 ? pp2 : (p0 >= cut1 ? pp1 : LD);
                if (c < q0) add(s, *reinterpret_cast<const float4 *>(part + (int64_t)p0 * LD + c));
            }
        }
        if (G > 1) {
#pragma unroll
            for (int off = 32; off >= NV; off >>= 1) {
                s.x += __shfl_down(s.x, off);
                s.y += __shfl_down(s.y, off);
                s.z += __shfl_down(s.z, off);
                s.w += __shfl_down(s.w, off);
            }
        }
        if (cv < NV && grp == 0) *reinterpret_cast<float4 *>(lb + c) = s;
    }
}

template <class R>
__global__ void k_zero(R *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = R(0);
}

// ---------------------------------------------------------------------------
// Host side

// Host FP64 operators of order p, column-major per operator ([op][k][row]):
// 8 M2M and 8 L2L built per call, the 316 M2L once per process and order.
static void host_ops(int p, std::vector<double> &h2m, std::vector<double> &h2l, const std::vector<double> *&hl_out) {
    const int P = p * p;
    std::vector<double> rm((size_t)P * P);
    auto to_cm = [&](double *dst) {
        for (int r = 0; r < P; ++r)
            for (int c = 0; c < P; ++c) dst[(size_t)c * P + r] = rm[(size_t)r * P + c];
    };
    h2m.assign((size_t)8 * P * P, 0.0);
    h2l.assign((size_t)8 * P * P, 0.0);
    for (int o = 0; o < 8; ++o) {
        build_m2m(p, o, rm.data());
        to_cm(&h2m[(size_t)o * P * P]);
        build_l2l(p, o, rm.data());
        to_cm(&h2l[(size_t)o * P * P]);
    }
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
    hl_out = &hl;
}

// BF16 round-to-nearest-even of an FP32 value (finite inputs).
static uint16_t bf16_rne(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
static double bf16_value(uint16_t h) {
    const uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return (double)f;
}

// Split-BF16 copy of nops column-major P x P operators: hi = bf16(a),
// lo = bf16(a - hi), stored [op][chunk][row][32] with K zero-padded to a
// multiple of 32.
static void split_ops(const double *cm, int nops, int P, std::vector<uint16_t> &hi, std::vector<uint16_t> &lo) {
    const int NC = (P + 31) / 32;
    hi.assign((size_t)nops * NC * P * 32, 0);
    lo.assign(hi.size(), 0);
#pragma omp parallel for schedule(static)
    for (int o = 0; o < nops; ++o)
        for (int c = 0; c < NC; ++c)
            for (int row = 0; row < P; ++row)
                for (int kk = 0; kk < 32; ++kk) {
                    const int k = c * 32 + kk;
                    if (k >= P) continue;
                    const double v = cm[((size_t)o * P + k) * P + row];
                    const uint16_t h = bf16_rne((float)v);
                    const size_t at = (((size_t)o * NC + c) * P + row) * 32 + kk;
                    hi[at] = h;
                    lo[at] = bf16_rne((float)(v - bf16_value(h)));
                }
}

template <class R>
static void upload(DevBuf<R> &d, const std::vector<R> &h, hipStream_t st) {
    d.ensure(h.size());
    BFM_HIP(hipMemcpyAsync(d.get(), h.data(), sizeof(R) * h.size(), hipMemcpyHostToDevice, st));
}

void fmm_prepare_ops(FmmWork &w, int p, hipStream_t st) {
    int dev = 0;
    BFM_HIP(hipGetDevice(&dev));
    leaf_tables_upload(dev);
    if (w.ops_p == p && w.ops_prec == w.prec) return;
    const int P = p * p;
    std::vector<double> h2m, h2l;
    const std::vector<double> *hl = nullptr;
    host_ops(p, h2m, h2l, hl);
    if (w.prec == BFM_PREC_FP64) {
        upload(w.ops_m2m, h2m, st);
        upload(w.ops_l2l, h2l, st);
        upload(w.ops_m2l, *hl, st);
        BFM_HIP(hipStreamSynchronize(st));
    } else if (w.prec == BFM_PREC_FP32) {
        std::vector<float> f2m(h2m.begin(), h2m.end()), f2l(h2l.begin(), h2l.end()), fl(hl->begin(), hl->end());
        upload(w.opf_m2m, f2m, st);
        upload(w.opf_l2l, f2l, st);
        upload(w.opf_m2l, fl, st);
        BFM_HIP(hipStreamSynchronize(st));
    } else {
        std::vector<uint16_t> hi, lo;
        split_ops(h2m.data(), 8, P, hi, lo);
        upload(w.opb_m2m[0], hi, st);
        upload(w.opb_m2m[1], lo, st);
        BFM_HIP(hipStreamSynchronize(st));
        split_ops(h2l.data(), 8, P, hi, lo);
        upload(w.opb_l2l[0], hi, st);
        upload(w.opb_l2l[1], lo, st);
        BFM_HIP(hipStreamSynchronize(st));
        split_ops(hl->data(), kNumM2LOps, P, hi, lo);
        upload(w.opb_m2l[0], hi, st);
        upload(w.opb_m2l[1], lo, st);
        BFM_HIP(hipStreamSynchronize(st));
    }
    w.ops_p = p;
    w.ops_prec = w.prec;
}

static unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Algorithmic flops of one source-receiver pair: shared geometry 3 (d) + 5
// (r^2) + 1 (1/r) [+ 5 for n.d and 3 for n.d / r^3 with dipoles]; per channel
// 2 (q/r) and 2 (w n.d / r^3).
static double p2p_flops_per_pair(int nch, bool mono, bool dip) {
    return 9.0 + (dip ? 8.0 : 0.0) + nch * ((mono ? 2.0 : 0.0) + (dip ? 2.0 : 0.0));
}

static int prof_begin(FmmWork &w, int cls, hipStream_t st) {
    return w.prof ? w.prof->begin(w.prof_base + cls, st) : -1;
}
static void prof_end(FmmWork &w, int idx, hipStream_t st, double flops) {
    if (w.prof) w.prof->end(idx, st, flops, 0.0);
}

// Middle row-slab height: a multiple of 16 dividing p^2, at most 80.
constexpr int mid_rows(int PP) { return PP == 144 ? 48 : (PP == 400 ? 80 : (PP >= 64 ? 64 : PP)); }
// Wide-tile slab: every row while 8 waves' accumulators and LDS stay small
// (p <= 12), half the rows at p = 16.
constexpr int wide_rows(int PP) { return PP <= 144 ? PP : (PP == 256 ? 128 : mid_rows(PP)); }

// Tiles of `width` columns (nch per task) before operator o of a task list.
static int tiles_before(const TaskList &tl, int nch, int width, int o) {
    int run = 0;
    for (int q = 0; q < o; ++q) run += ((tl.op_off_h[q + 1] - tl.op_off_h[q]) * nch + width - 1) / width;
    return run;
}

// One launch of k_translate over operators op0 .. op0 + nops - 1 (tiles g0 ..
// g0 + ntiles - 1) at applied order PPo, stored order LD, launch shape
// `shape` (0: 8 waves, all rows up to p = 12; 1: row slabs; 2: 16-row slabs).
template <int PPo, int LD, class R>
static void launch_translate(int shape, bool m2l, int op0, int nops, int g0, int ntiles, const int *to,
                             const TaskList &tl, int nch, int sw, const R *T, const R *in, R *out, hipStream_t st) {
    if (ntiles <= 0) return;
    if (shape == 0) {
        constexpr int RW = wide_rows(PPo);
        auto kern = m2l ? k_translate<PPo, RW, 8, 0, R, LD> : k_translate<PPo, RW, 8, 1, R, LD>;
        kern<<<(unsigned)(ntiles * (PPo / RW)), 512, 0, st>>>(op0, nops, to, g0, ntiles, tl.op_off.get(),
                                                               tl.src.get(), tl.dst.get(), nch, sw, T, in, out);
    } else if (shape == 1) {
        constexpr int RM = mid_rows(PPo);
        auto kern = m2l ? k_translate<PPo, RM, 4, 0, R, LD> : k_translate<PPo, RM, 4, 1, R, LD>;
        kern<<<(unsigned)(ntiles * (PPo / RM)), 256, 0, st>>>(op0, nops, to, g0, ntiles, tl.op_off.get(),
                                                               tl.src.get(), tl.dst.get(), nch, sw, T, in, out);
    } else {
        auto kern = m2l ? k_translate<PPo, 16, 4, 0, R, LD> : k_translate<PPo, 16, 4, 1, R, LD>;
        kern<<<(unsigned)(ntiles * (PPo / 16)), 256, 0, st>>>(op0, nops, to, g0, ntiles, tl.op_off.get(),
                                                               tl.src.get(), tl.dst.get(), nch, sw, T, in, out);
    }
    BFM_LAUNCHED();
}

// Rotation-factored M2L (fmm_rot.hip) over a whole interaction list, by
// distance class when the product reduces distant orders. Flops counted:
// 2 (2 sum_{n<q} (2n+1)^2 + sum_{|m|<q} (q-|m|)^2) per column at order q.
template <int P_>
static void translate_rot(FmmWork &w, TaskList &tl, int nch, const double *in, double *out, hipStream_t st) {
    rot_ops_upload(w, P_, st);
    prepare_tiles(tl, nch, 16, st);
    const int nt = tl.ntiles_for(nch, 16);
    if (nt <= 0) return;
    const int pi = prof_begin(w, KC_M2L, st);
    const int *to = tl.tile_for(nch, 16);
    auto col_flops = [](int q) {
        double f = 2.0 * q * (4.0 * q * q - 1.0) / 3.0;  // the two rotations
        for (int m = -(q - 1); m < q; ++m) f += (double)(q - std::abs(m)) * (q - std::abs(m));
        return 2.0 * f;
    };
    double flops = 0.0;
    if (w.m2l_orders) {
        constexpr int P1 = m2l_class_order(P_, 1), P2 = m2l_class_order(P_, 2);
        int first[kM2LClasses + 1];
        for (int c = 0; c <= kM2LClasses; ++c) first[c] = m2l_class_first_op(c);
        for (int c = 0; c < kM2LClasses; ++c) {
            const int g0 = tiles_before(tl, nch, 16, first[c]);
            const int g1 = tiles_before(tl, nch, 16, first[c + 1]);
            const int64_t nk = tl.op_off_h[first[c + 1]] - tl.op_off_h[first[c]];
            flops += col_flops(m2l_class_order(P_, c)) * (double)nk * nch;
            const int nops = first[c + 1] - first[c];
            if (c == 0)
                launch_m2l_rot<P_, P_>(w, first[c], nops, g0, g1 - g0, to, tl, nch, in, out, st);
            else if (c == 1)
                launch_m2l_rot<P1, P_>(w, first[c], nops, g0, g1 - g0, to, tl, nch, in, out, st);
            else
                launch_m2l_rot<P2, P_>(w, first[c], nops, g0, g1 - g0, to, tl, nch, in, out, st);
        }
    } else {
        flops = col_flops(P_) * (double)tl.ntasks * nch;
        launch_m2l_rot<P_, P_>(w, 0, tl.nops, 0, nt, to, tl, nch, in, out, st);
    }
    prof_end(w, pi, st, flops);
}

template <int P_, class R = double>
static void translate(FmmWork &w, int cls, TaskList &tl, int nch, bool swap, const R *T, const R *in, R *out,
                      hipStream_t st) {
    constexpr int PP = P_ * P_;
    const int64_t cols = tl.ntasks * nch;
    // Row slabs of 64 (80 at p = 20) rows unless that leaves fewer than 512
    // waves, then 16-row slabs (more waves, the input columns re-read per
    // slab); the wide 128-column tiles (shape 0, fewest operator re-reads but
    // twice the LDS per workgroup) only on request.
    const int64_t wave_tiles = (cols + 15) / 16;
    int shape = (wave_tiles * (PP / mid_rows(PP)) >= 512) ? 1 : 2;
    if (cls == KC_M2L && w.m2l_shape >= 0 && w.m2l_shape <= 2) shape = w.m2l_shape;
    if constexpr (std::is_same<R, double>::value) {
        if (cls == KC_M2L && w.m2l_shape == 3) {
            w.m2l_shape_used = 3;
            return translate_rot<P_>(w, tl, nch, in, out, st);
        }
    }
    if (cls == KC_M2L) w.m2l_shape_used = shape;
    const int width = (shape == 0) ? 128 : 64;
    prepare_tiles(tl, nch, width, st);
    const int nt = tl.ntiles_for(nch, width);
    if (nt <= 0) return;
    const int pi = prof_begin(w, cls, st);
    const int *to = tl.tile_for(nch, width);
    const int sw = swap ? 1 : 0;
    const bool m2l = cls == KC_M2L;
    double flops = 2.0 * (double)PP * PP * (double)tl.ntasks * nch;
    if (m2l && w.m2l_orders) {
        // distance classes of offsets, each at its own order (contiguous
        // operator ranges)
        constexpr int P1 = m2l_class_order(P_, 1), P2 = m2l_class_order(P_, 2);
        int first[kM2LClasses + 1];
        for (int c = 0; c <= kM2LClasses; ++c) first[c] = m2l_class_first_op(c);
        flops = 0.0;
        for (int c = 0; c < kM2LClasses; ++c) {
            const int g0 = tiles_before(tl, nch, width, first[c]);
            const int g1 = tiles_before(tl, nch, width, first[c + 1]);
            const int64_t nk = tl.op_off_h[first[c + 1]] - tl.op_off_h[first[c]];
            const int po = m2l_class_order(P_, c);
            flops += 2.0 * (double)po * po * po * po * (double)nk * nch;
            const int nops = first[c + 1] - first[c];
            if (c == 0)
                launch_translate<PP, PP, R>(shape, true, first[c], nops, g0, g1 - g0, to, tl, nch, sw, T, in, out, st);
            else if (c == 1)
                launch_translate<P1 * P1, PP, R>(shape, true, first[c], nops, g0, g1 - g0, to, tl, nch, sw, T, in, out,
                                                 st);
            else
                launch_translate<P2 * P2, PP, R>(shape, true, first[c], nops, g0, g1 - g0, to, tl, nch, sw, T, in, out,
                                                 st);
        }
    } else {
        launch_translate<PP, PP, R>(shape, m2l, 0, tl.nops, 0, nt, to, tl, nch, sw, T, in, out, st);
    }
    prof_end(w, pi, st, flops);
}

// Row slab of the split-BF16 translation: every row up to p = 12 (the input
// columns are then loaded and split once per tile), 128 rows at p = 16, 80
// at p = 20 (accumulator registers and LDS bound the slab).
constexpr int bf_rows(int PP) { return PP <= 144 ? PP : (PP == 256 ? 128 : 80); }

template <int PPo, int LD, bool STORE>
static void launch_bf3(int op0, int nops, int g0, int ntiles, const int *to, const TaskList &tl, bool swap,
                       const uint16_t *Thi, const uint16_t *Tlo, const float *in, float *out, hipStream_t st) {
    if (ntiles <= 0) return;
    constexpr int RM = bf_rows(PPo);
    k_translate_bf3<PPo, RM, STORE ? 0 : 1, STORE, LD><<<(unsigned)(ntiles * (PPo / RM)), 64 * kBfWaves, 0, st>>>(
        op0, nops, to, g0, ntiles, tl.op_off.get(), tl.src.get(), tl.dst.get(), 1, swap ? 1 : 0,
        reinterpret_cast<const uint4 *>(Thi), reinterpret_cast<const uint4 *>(Tlo), in, out);
    BFM_LAUNCHED();
}

// Split-BF16 translation of FP32 expansions (one launch shape: 128-column
// tiles, row slabs of bf_rows). M2L results are stored per task, then summed
// per target box (no atomics).
template <int P_>
static void translate_bf3(FmmWork &w, int cls, TaskList &tl, bool swap, const uint16_t *Thi, const uint16_t *Tlo,
                          const float *in, float *out, hipStream_t st) {
    constexpr int PP = P_ * P_;
    prepare_tiles(tl, 1, kBfTile, st);
    const int nt = tl.ntiles_for(1, kBfTile);
    if (cls == KC_M2L) w.m2l_shape_used = 1;
    if (nt <= 0) return;
    const int pi = prof_begin(w, cls, st);
    const int *to = tl.tile_for(1, kBfTile);
    double flops = 2.0 * (double)PP * PP * (double)tl.ntasks;
    if (cls == KC_M2L) {
        float *part = w.part32.ensure((size_t)tl.ntasks * PP);
        constexpr int P1 = m2l_class_order(P_, 1), P2 = m2l_class_order(P_, 2);
        int cut1 = (int)tl.ntasks, cut2 = (int)tl.ntasks;
        if (w.m2l_orders) {
            int first[kM2LClasses + 1];
            for (int c = 0; c <= kM2LClasses; ++c) first[c] = m2l_class_first_op(c);
            flops = 0.0;
            for (int c = 0; c < kM2LClasses; ++c) {
                const int g0 = tiles_before(tl, 1, kBfTile, first[c]);
                const int g1 = tiles_before(tl, 1, kBfTile, first[c + 1]);
                const int64_t nk = tl.op_off_h[first[c + 1]] - tl.op_off_h[first[c]];
                const int po = m2l_class_order(P_, c);
                flops += 2.0 * (double)po * po * po * po * (double)nk;
                const int nops = first[c + 1] - first[c];
                if (c == 0)
                    launch_bf3<PP, PP, true>(first[c], nops, g0, g1 - g0, to, tl, swap, Thi, Tlo, in, part, st);
                else if (c == 1)
                    launch_bf3<P1 * P1, PP, true>(first[c], nops, g0, g1 - g0, to, tl, swap, Thi, Tlo, in, part, st);
                else
                    launch_bf3<P2 * P2, PP, true>(first[c], nops, g0, g1 - g0, to, tl, swap, Thi, Tlo, in, part, st);
            }
            cut1 = tl.op_off_h[first[1]];
            cut2 = tl.op_off_h[first[2]];
        } else {
            launch_bf3<PP, PP, true>(0, tl.nops, 0, nt, to, tl, swap, Thi, Tlo, in, part, st);
        }
        if (tl.dst_nbox > 0) {
            k_m2l_reduce<PP><<<(unsigned)tl.dst_nbox, 64, 0, st>>>(tl.dst_off.get(), tl.pos_of.get(), tl.dst_box0,
                                                                  cut1, cut2, P1 * P1, P2 * P2, part, out);
            BFM_LAUNCHED();
        }
    } else {
        launch_bf3<PP, PP, false>(0, tl.nops, 0, nt, to, tl, swap, Thi, Tlo, in, out, st);
    }
    prof_end(w, pi, st, flops);
}

template <int P_, int NCH, bool MONO, bool DIP>
static void run_fmm(FmmWork &w, const Tree &tc, const Sources &src, double *y, hipStream_t st) {
    Tree &t = const_cast<Tree &>(tc);
    constexpr int PP = P_ * P_;
    const int lmax = t.lmax;
    const size_t ncoef = (size_t)t.nbox * NCH * PP;
    double *M = w.mexp.ensure(ncoef);
    double *L = w.lexp.ensure(ncoef);
    k_zero<double><<<1024, 256, 0, st>>>(M, (int64_t)ncoef);
    BFM_LAUNCHED();
    k_zero<double><<<1024, 256, 0, st>>>(L, (int64_t)ncoef);
    BFM_LAUNCHED();
    // near field (writes y) on the near-field stream when there is one,
    // beside the far-field chain; the L2P adds into y after it
    // (kernel timing runs them one after the other, so that each kernel's
    // events measure it alone)
    hipStream_t ns = (w.near && !(w.prof && w.prof->on)) ? w.near : st;
    if (ns != st) {
        BFM_HIP(hipEventRecord(w.ev_fork, st));
        BFM_HIP(hipStreamWaitEvent(ns, w.ev_fork, 0));
    }
    int pi = prof_begin(w, KC_P2P, ns);
    if (NCH == 5 && src.packed)
        launch_p2p_packed(t, src.packed, y, ns);
    else
        launch_p2p<NCH, MONO, DIP>(t, src, y, ns);
    prof_end(w, pi, ns, (double)(t.npairs_near - t.n) * p2p_flops_per_pair(NCH, MONO, DIP));
    if (ns != st) BFM_HIP(hipEventRecord(w.ev_join, ns));
    pi = prof_begin(w, KC_P2M, st);
    launch_p2m<P_, NCH, MONO, DIP>(t, src, M, st);
    prof_end(w, pi, st, 0.0);
    for (int l = lmax; l >= 3; --l)
        translate<P_>(w, KC_M2M_L2L, *t.m2m[l], NCH, false, w.ops_m2m.get(), M, M, st);
    translate<P_>(w, KC_M2L, t.m2l, NCH, false, w.ops_m2l.get(), M, L, st);
    for (int l = 3; l <= lmax; ++l)
        translate<P_>(w, KC_M2M_L2L, *t.m2m[l], NCH, true, w.ops_l2l.get(), L, L, st);
    if (ns != st) BFM_HIP(hipStreamWaitEvent(st, w.ev_join, 0));
    pi = prof_begin(w, KC_L2P, st);
    launch_l2p<P_, NCH>(t, L, y, st);
    prof_end(w, pi, st, 0.0);
}

// Low-precision product (one channel): FP32 near field, FP32 leaf expansions,
// translations on FP32 or split-BF16 matrix cores; the sums y stay FP64.
template <int P_, bool MONO, bool DIP>
static void run_fmm_lo(FmmWork &w, const Tree &tc, const Sources &src, double *y, hipStream_t st) {
    Tree &t = const_cast<Tree &>(tc);
    constexpr int PP = P_ * P_;
    const int lmax = t.lmax;
    const size_t ncoef = (size_t)t.nbox * PP;
    float *M = w.mexp32.ensure(ncoef);
    float *L = w.lexp32.ensure(ncoef);
    k_zero<float><<<1024, 256, 0, st>>>(M, (int64_t)ncoef);
    BFM_LAUNCHED();
    k_zero<float><<<1024, 256, 0, st>>>(L, (int64_t)ncoef);
    BFM_LAUNCHED();
    hipStream_t ns = (w.near && !(w.prof && w.prof->on)) ? w.near : st;
    if (ns != st) {
        BFM_HIP(hipEventRecord(w.ev_fork, st));
        BFM_HIP(hipStreamWaitEvent(ns, w.ev_fork, 0));
    }
    int pi = prof_begin(w, KC_P2P, ns);
    launch_p2p32<MONO, DIP>(t, src, y, ns);
    prof_end(w, pi, ns, (double)(t.npairs_near - t.n) * p2p_flops_per_pair(1, MONO, DIP));
    if (ns != st) BFM_HIP(hipEventRecord(w.ev_join, ns));
    pi = prof_begin(w, KC_P2M, st);
    launch_p2m<P_, 1, MONO, DIP, float>(t, src, M, st);
    prof_end(w, pi, st, 0.0);
    if (w.prec == BFM_PREC_FP32) {
        for (int l = lmax; l >= 3; --l)
            translate<P_, float>(w, KC_M2M_L2L, *t.m2m[l], 1, false, w.opf_m2m.get(), M, M, st);
        translate<P_, float>(w, KC_M2L, t.m2l, 1, false, w.opf_m2l.get(), M, L, st);
        for (int l = 3; l <= lmax; ++l)
            translate<P_, float>(w, KC_M2M_L2L, *t.m2m[l], 1, true, w.opf_l2l.get(), L, L, st);
    } else {
        for (int l = lmax; l >= 3; --l)
            translate_bf3<P_>(w, KC_M2M_L2L, *t.m2m[l], false, w.opb_m2m[0].get(), w.opb_m2m[1].get(), M, M, st);
        translate_bf3<P_>(w, KC_M2L, t.m2l, false, w.opb_m2l[0].get(), w.opb_m2l[1].get(), M, L, st);
        for (int l = 3; l <= lmax; ++l)
            translate_bf3<P_>(w, KC_M2M_L2L, *t.m2m[l], true, w.opb_l2l[0].get(), w.opb_l2l[1].get(), L, L, st);
    }
    if (ns != st) BFM_HIP(hipStreamWaitEvent(st, w.ev_join, 0));
    pi = prof_begin(w, KC_L2P, st);
    launch_l2p<P_, 1, float>(t, L, y, st);
    prof_end(w, pi, st, 0.0);
}

template <bool MONO, bool DIP>
static void dispatch_lo(FmmWork &w, const Tree &t, const Sources &src, double *y, hipStream_t st) {
    switch (w.p) {
        case 4: return run_fmm_lo<4, MONO, DIP>(w, t, src, y, st);
        case 8: return run_fmm_lo<8, MONO, DIP>(w, t, src, y, st);
        case 12: return run_fmm_lo<12, MONO, DIP>(w, t, src, y, st);
        case 16: return run_fmm_lo<16, MONO, DIP>(w, t, src, y, st);
        case 20: return run_fmm_lo<20, MONO, DIP>(w, t, src, y, st);
        default: fail(BFM_EUNSUPPORTED, "expansion order p must be one of 4, 8, 12, 16, 20");
    }
}

template <int NCH, bool MONO, bool DIP>
static void dispatch_p(FmmWork &w, const Tree &t, const Sources &src, double *y, bool direct,
                       hipStream_t st) {
    if (direct) return launch_direct<NCH, MONO, DIP>(t, src, y, st);
    if (w.prec != BFM_PREC_FP64) {
        if constexpr (NCH == 1) return dispatch_lo<MONO, DIP>(w, t, src, y, st);
        fail(BFM_EUNSUPPORTED, "low-precision products carry one channel");
    }
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
    if (!direct)
        BFM_CHECK(w.ops_p == w.p && w.p > 0 && w.ops_prec == w.prec, BFM_EINVAL, "translation operators not prepared");
    if (src.nch == 1 && src.mono && !src.dip) return dispatch_p<1, true, false>(w, t, src, y, direct, st);
    if (src.nch == 1 && !src.mono && src.dip) return dispatch_p<1, false, true>(w, t, src, y, direct, st);
    if (src.nch == 1 && src.mono && src.dip) return dispatch_p<1, true, true>(w, t, src, y, direct, st);
    if (src.nch == 5 && src.mono && src.dip) return dispatch_p<5, true, true>(w, t, src, y, direct, st);
    fail(BFM_EUNSUPPORTED, "unsupported source channel combination");
}

}  // namespace bfm
