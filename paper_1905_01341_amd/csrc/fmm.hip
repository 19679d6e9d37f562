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

#include "fmm_kernels.h"
#include "ops.h"

namespace bfm {

typedef double dbl4 __attribute__((ext_vector_type(4)));

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
    __shared__ double As[2][kTKC * ROWS];         // two buffers of [k][row within slab]
    __shared__ double Bs[2][WAVES][kTKC / 4][64];  // two buffers of each wave's input chunk
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
    // idle columns read box 0's expansion (valid memory) and are never stored
    const double *bcol = in + ((int64_t)sb * nch + bch) * PP;
    const double *Top = T + (int64_t)op * PP * PP + slab * ROWS;
    const int kq = lane >> 4, rl = lane & 15;
    dbl4 acc[ROWS / 16];
#pragma unroll
    for (int rb = 0; rb < ROWS / 16; ++rb) acc[rb] = dbl4{0.0, 0.0, 0.0, 0.0};
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
    double pa[PER], pb[PER], pc[PER], ba[kTKC / 4], bb[kTKC / 4], bc[kTKC / 4];
    auto fetch = [&](int k0, double(&pre)[PER], double(&bv)[kTKC / 4]) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + u * NT;
            if (EXACT || e < kTKC * ROWS) pre[u] = Top[(int64_t)(k0 + e / ROWS) * PP + e % ROWS];
        }
#pragma unroll
        for (int kk = 0; kk < kTKC / 4; ++kk) bv[kk] = bcol[k0 + 4 * kk + kq];
    };
    // the chunk's operator slab and input columns -> LDS buffer `buf`
    auto stash = [&](int buf, const double(&pre)[PER], const double(&bv)[kTKC / 4]) {
#pragma unroll
        for (int u = 0; u < PER; ++u)
            if (EXACT || tid + u * NT < kTKC * ROWS) As[buf][tid + u * NT] = pre[u];
#pragma unroll
        for (int kk = 0; kk < kTKC / 4; ++kk) Bs[buf][wave][kk][lane] = bok ? bv[kk] : 0.0;
    };
    // the MFMAs of one chunk read only LDS, so no wait on the loads in flight
    auto mult = [&](int buf) {
#pragma unroll
        for (int kk = 0; kk < kTKC / 4; ++kk) {
            const double *Ak = As[buf] + (4 * kk + kq) * ROWS + rl;
            const double b = Bs[buf][wave][kk][lane];
#pragma unroll
            for (int rb = 0; rb < ROWS / 16; ++rb)
                acc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(b, Ak[rb * 16], acc[rb], 0, 0, 0);
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
        const int col = colbase + kq + 4 * r;
        if (col >= ncols) continue;
        const int task = t0 + col / nch, ch = col % nch;
        const int db = swap ? tsrc[task] : tdst[task];
        double *dcol = out + ((int64_t)db * nch + ch) * PP + slab * ROWS + rl;
#pragma unroll
        for (int rb = 0; rb < ROWS / 16; ++rb) unsafeAtomicAdd(dcol + rb * 16, acc[rb][r]);
    }
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
    leaf_tables_upload(dev);
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
// Wide-tile slab: every row while 8 waves' accumulators and LDS stay small
// (p <= 12), half the rows at p = 16.
constexpr int wide_rows(int PP) { return PP <= 144 ? PP : (PP == 256 ? 128 : mid_rows(PP)); }

template <int P_>
static void translate(FmmWork &w, int cls, TaskList &tl, int nch, bool swap, const double *T,
                      const double *in, double *out, hipStream_t st) {
    constexpr int PP = P_ * P_;
    const int64_t cols = tl.ntasks * nch;
    // Row slabs of 64 (80 at p = 20) rows unless that leaves fewer than 512
    // waves, then 16-row slabs (more waves, the input columns re-read per
    // slab); the wide 128-column tiles (shape 0, fewest operator re-reads but
    // twice the LDS per workgroup) only on request.
    const int64_t wave_tiles = (cols + 15) / 16;
    int shape = (wave_tiles * (PP / mid_rows(PP)) >= 512) ? 1 : 2;
    if (cls == KC_M2L && w.m2l_shape >= 0) shape = w.m2l_shape;
    if (cls == KC_M2L) w.m2l_shape_used = shape;
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
    const size_t ncoef = (size_t)t.nbox * NCH * PP;
    double *M = w.mexp.ensure(ncoef);
    double *L = w.lexp.ensure(ncoef);
    k_zero<<<1024, 256, 0, st>>>(M, (int64_t)ncoef);
    BFM_LAUNCHED();
    k_zero<<<1024, 256, 0, st>>>(L, (int64_t)ncoef);
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

template <int NCH, bool MONO, bool DIP>
static void dispatch_p(FmmWork &w, const Tree &t, const Sources &src, double *y, bool direct,
                       hipStream_t st) {
    if (direct) return launch_direct<NCH, MONO, DIP>(t, src, y, st);
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
