// Graph capture of the GMRES product and autotuning of the fast multipole
// product (include/bfm.h: use_graph, m2l_shape, bfm_autotune).
//
// The product inside GMRES (right preconditioner, then the fast multipole
// product with the diagonal) launches a few dozen kernels whose arguments
// are fixed for one octree. It is captured once per octree into a HIP graph
// that reads a fixed input buffer and writes a fixed output buffer; each
// GMRES step copies its Krylov vector in and the product out with plain
// kernels (no memset or memcpy nodes in the graph).
#include <algorithm>
#include <cmath>
#include <vector>

#include "ctx.h"

namespace bfm {

static unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

__global__ void k_copy_vec(const double *in, int64_t n, double *out) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i];
}

static void copy_vec(const double *in, int64_t n, double *out, hipStream_t st) {
    k_copy_vec<<<nblk(n, 256), 256, 0, st>>>(in, n, out);
    BFM_LAUNCHED();
}

// An invalidated graph is kept until graph_release_stale: destroying an
// executable graph waits for the device, and the octree build, which
// invalidates it, runs beside the coarse build on a second stream.
void graph_invalidate(bfm_ctx *c) {
    if (c->mvp_graph) {
        graph_release_stale(c);
        c->mvp_graph_stale = c->mvp_graph;
        c->mvp_graph_stale_pc = c->mvp_graph_pc;
    }
    c->mvp_graph = nullptr;
    c->mvp_graph_pc = -1;
}

void graph_release_stale(bfm_ctx *c) {
    if (c->mvp_graph_stale) (void)hipGraphExecDestroy(c->mvp_graph_stale);
    c->mvp_graph_stale = nullptr;
}

// gout = A P^{-1} gin (pc) or A gin
static void mvp_body(bfm_ctx *c, bool pc) {
    if (pc) {
        double *Z = c->zbuf.ensure(c->nv);
        precond_apply(c, c->gin.get(), Z);
        matvec_sorted(c, 1.0, Z, 0.0, nullptr, c->gout.get(), true, c->opt.precision, false);
    } else {
        matvec_sorted(c, 1.0, c->gin.get(), 0.0, nullptr, c->gout.get(), true, c->opt.precision, false);
    }
}

void graph_mvp(bfm_ctx *c, const double *in_s, double *out_s, bool pc) {
    hipStream_t st = c->stream;
    const int64_t n = c->nv;
    c->gin.ensure(n);
    c->gout.ensure(n);
    copy_vec(in_s, n, c->gin.get(), st);
    if (c->mvp_graph && c->mvp_graph_pc == (int)pc) {
        BFM_HIP(hipGraphLaunch(c->mvp_graph, st));
        copy_vec(c->gout.get(), n, out_s, st);
        return;
    }
    graph_invalidate(c);
    // eager run first: every lazy preparation (tiles, buffers, operators)
    // happens here, outside the capture, and its result is this call's product.
    // The capture follows while it runs: capturing records the launches
    // without running them, so the stream need not be idle.
    mvp_body(c, pc);
    copy_vec(c->gout.get(), n, out_s, st);
    hipGraph_t g = nullptr;
    BFM_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    try {
        mvp_body(c, pc);
    } catch (...) {
        hipGraph_t junk = nullptr;
        (void)hipStreamEndCapture(st, &junk);
        if (junk) (void)hipGraphDestroy(junk);
        throw;
    }
    BFM_HIP(hipStreamEndCapture(st, &g));
    hipGraphExec_t ge = nullptr;
    // the previous octree's executable graph is updated in place when the
    // new capture has the same launches (new arguments and grid sizes),
    // which spares an instantiation and the destruction of the old one
    if (c->mvp_graph_stale && c->mvp_graph_stale_pc == (int)pc) {
        hipGraphNode_t bad = nullptr;
        hipGraphExecUpdateResult res = hipGraphExecUpdateError;
        if (hipGraphExecUpdate(c->mvp_graph_stale, g, &bad, &res) == hipSuccess && res == hipGraphExecUpdateSuccess) {
            ge = c->mvp_graph_stale;
            c->mvp_graph_stale = nullptr;
        } else {
            (void)hipGetLastError();  // a refused update leaves no error behind
        }
    }
    hipError_t e = hipSuccess;
    if (!ge) {
        graph_release_stale(c);
        e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    }
    (void)hipGraphDestroy(g);
    BFM_CHECK(e == hipSuccess, BFM_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    c->mvp_graph = ge;
    c->mvp_graph_pc = (int)pc;
}

// ---------------------------------------------------------------------------
// Autotuning

static double norm2_host(const double *d, int64_t n, hipStream_t st) {
    std::vector<double> h(n);
    BFM_HIP(hipMemcpyAsync(h.data(), d, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    BFM_HIP(hipStreamSynchronize(st));
    double s = 0.0;
    for (double v : h) s += v * v;
    return std::sqrt(s);
}

static double diff_host(const double *a, const double *b, int64_t n, hipStream_t st) {
    std::vector<double> ha(n), hb(n);
    BFM_HIP(hipMemcpyAsync(ha.data(), a, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    BFM_HIP(hipMemcpyAsync(hb.data(), b, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    BFM_HIP(hipStreamSynchronize(st));
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += (ha[i] - hb[i]) * (ha[i] - hb[i]);
    return std::sqrt(s);
}

static double maxdiff_host(const double *a, const double *b, int64_t n, hipStream_t st) {
    std::vector<double> ha(n), hb(n);
    BFM_HIP(hipMemcpyAsync(ha.data(), a, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    BFM_HIP(hipMemcpyAsync(hb.data(), b, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    BFM_HIP(hipStreamSynchronize(st));
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i) m = std::max(m, std::fabs(ha[i] - hb[i]));
    return m;
}

static double time_mvp(bfm_ctx *c, const double *x, double *y, int reps, int prec = BFM_PREC_FP64) {
    hipStream_t st = c->stream;
    matvec_sorted(c, 1.0, x, 0.0, nullptr, y, false, prec, false);  // warm-up
    hipEvent_t a, b;
    BFM_HIP(hipEventCreate(&a));
    BFM_HIP(hipEventCreate(&b));
    BFM_HIP(hipEventRecord(a, st));
    for (int r = 0; r < reps; ++r) matvec_sorted(c, 1.0, x, 0.0, nullptr, y, false, prec, false);
    BFM_HIP(hipEventRecord(b, st));
    BFM_HIP(hipEventSynchronize(b));
    float ms = 0.f;
    BFM_HIP(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms / reps;
}

void autotune(bfm_ctx *c, double mvp_tol, bfm_tune_result *out) {
    hipStream_t st = c->stream;
    const int64_t n = c->nv;
    const bfm_options saved = c->opt;
    graph_invalidate(c);
    // fixed pseudo-random input (sorted order; any vector serves)
    std::vector<double> xh(n);
    uint64_t state = 0x9e3779b97f4a7c15ull;
    for (int64_t i = 0; i < n; ++i) {
        state = state * 6364136223846793005ull + 1442695040888963407ull;
        xh[i] = (double)(state >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    }
    DevBuf<double> x, yref, y;
    x.ensure(n);
    yref.ensure(n);
    y.ensure(n);
    BFM_HIP(hipMemcpyAsync(x.get(), xh.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
    try {
        // 1. expansion order: smallest p within mvp_tol of p = 20
        c->opt.m2l_shape = -1;
        ensure_tree(c);
        const int auto_lmax = c->opt.lmax > 0 ? c->opt.lmax : c->tree.lmax;
        c->opt.p = 20;
        ensure_ops(c);
        matvec_sorted(c, 1.0, x.get(), 0.0, nullptr, yref.get(), false, BFM_PREC_FP64, false);
        const double nref = norm2_host(yref.get(), n, st);
        int best_p = 20;
        double best_err = 0.0;
        for (int p : {16, 12, 8}) {
            c->opt.p = p;
            ensure_ops(c);
            matvec_sorted(c, 1.0, x.get(), 0.0, nullptr, y.get(), false, BFM_PREC_FP64, false);
            const double err = diff_host(y.get(), yref.get(), n, st) / nref;
            if (err > mvp_tol) break;
            best_p = p;
            best_err = err;
        }
        c->opt.p = best_p;
        ensure_ops(c);
        // 1b. iterative refinement (low-precision inner products): p_lo = the
        // smallest of 8, 12, 16 whose low-precision product is within the
        // refinement step's tolerance ir_tol of the p = 20 FP64 product
        const bool ir = saved.precision != BFM_PREC_FP64;
        const double ir_tol = saved.ir_tol > 0.0 ? saved.ir_tol : 1e-4;
        int best_plo = 0;
        if (ir) {
            best_plo = 16;
            for (int plo : {8, 12, 16}) {
                c->opt.p_lo = plo;
                matvec_sorted(c, 1.0, x.get(), 0.0, nullptr, y.get(), false, saved.precision, false);
                const double err = diff_host(y.get(), yref.get(), n, st) / nref;
                if (err <= ir_tol) {
                    best_plo = plo;
                    break;
                }
            }
            c->opt.p_lo = best_plo;
        }
        // 1c. order of the diagonal/right-hand-side pass (when not set): the
        // smallest of 12, 16 (not below p) whose L_ii and M_ii are within
        // 10 mvp_tol of the pass at order 20 (L_ii: relative 2-norm; M_ii:
        // largest difference over 1/2, the size of the sums it comes from).
        // L_ii is the difference of two sums of the size of a bubble radius
        // (the translation-free form), so it needs the highest order of all
        // the pass's outputs; the tolerance is ten times the product's
        // because the solution carries about half of L_ii's relative error.
        int best_pd = saved.p_diag;
        double best_derr = 0.0;
        if (saved.p_diag <= 0) {
            best_pd = 20;
            c->opt.p_diag = 20;
            c->diag_valid = false;
            diagonal_pass(c, nullptr);
            DevBuf<double> lref, mref;
            lref.ensure(n);
            mref.ensure(n);
            BFM_HIP(hipMemcpyAsync(lref.get(), c->lii_s.get(), sizeof(double) * n, hipMemcpyDeviceToDevice, st));
            BFM_HIP(hipMemcpyAsync(mref.get(), c->mii_s.get(), sizeof(double) * n, hipMemcpyDeviceToDevice, st));
            const double lnorm = norm2_host(lref.get(), n, st);
            for (int pd : {12, 16}) {
                if (pd < c->opt.p) continue;
                c->opt.p_diag = pd;
                ensure_ops(c);
                c->diag_valid = false;
                diagonal_pass(c, nullptr);
                const double el = diff_host(c->lii_s.get(), lref.get(), n, st) / lnorm;
                const double em = maxdiff_host(c->mii_s.get(), mref.get(), n, st) / 0.5;
                const double e = std::max(el, em);
                if (e <= 10.0 * mvp_tol) {
                    best_pd = pd;
                    best_derr = e;
                    break;
                }
            }
            c->opt.p_diag = best_pd;
            ensure_ops(c);
            c->diag_valid = false;
        }
        // 2. octree depth and M2L launch shape: the depth minimises one
        // diagonal/right-hand-side pass plus the products of a typical solve
        // (ten FP64 products; with refinement two FP64 and eight
        // low-precision ones); the shape, the FP64 product at that depth
        DevBuf<double> xo;
        xo.ensure(n);
        BFM_HIP(hipMemcpyAsync(xo.get(), xh.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
        double best_cost = 1e300, best_ms = 1e300;
        int best_l = auto_lmax, best_s = -1, cand = 0;
        bool warm = false;
        for (int l = std::max(2, auto_lmax - 2); l <= std::min(15, auto_lmax + 2); ++l) {
            c->opt.lmax = l;
            c->opt.m2l_shape = -1;
            c->tree_valid = false;
            ensure_tree(c);
            ensure_ops(c);
            ensure_corr(c);  // the corrections' values follow the octree: not part of the timed pass
            if (!warm) {  // first pass uploads the diagonal pass's operators
                diagonal_pass(c, xo.get());
                warm = true;
            }
            hipEvent_t a, b;
            BFM_HIP(hipEventCreate(&a));
            BFM_HIP(hipEventCreate(&b));
            BFM_HIP(hipEventRecord(a, st));
            diagonal_pass(c, xo.get());
            BFM_HIP(hipEventRecord(b, st));
            BFM_HIP(hipEventSynchronize(b));
            float dms = 0.f;
            BFM_HIP(hipEventElapsedTime(&dms, a, b));
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
            double lvl_ms = 1e300;
            int lvl_s = -1;
            for (int shape = 0; shape <= 3; ++shape) {  // 3: the rotation-factored M2L
                c->opt.m2l_shape = shape;
                ensure_ops(c);
                const double ms = time_mvp(c, x.get(), y.get(), 5);
                ++cand;
                if (ms < lvl_ms) {
                    lvl_ms = ms;
                    lvl_s = shape;
                }
            }
            c->opt.m2l_shape = lvl_s;
            const double lo_ms = ir ? time_mvp(c, x.get(), y.get(), 5, saved.precision) : 0.0;
            const double cost = ir ? dms + 2.0 * lvl_ms + 8.0 * lo_ms : dms + 10.0 * lvl_ms;
            if (cost < best_cost) {
                best_cost = cost;
                best_ms = lvl_ms;
                best_l = l;
                best_s = lvl_s;
            }
        }
        // 3. near-field work item shape: the symmetric near field of the
        // products GMRES runs most (the low-precision ones under refinement),
        // timed alone with the library's kernel timing (which runs the near
        // field in line) at the chosen depth and M2L shape
        int best_ps = saved.p2p_shape;
        if (saved.p2p_shape < 0) {
            best_ps = 0;
            if (!c->prof.on) {
                c->opt.p = best_p;
                c->opt.lmax = best_l;
                c->opt.m2l_shape = best_s;
                const int prec = ir ? saved.precision : BFM_PREC_FP64;
                const int cls = (ir ? kLoBase : 0) + KC_P2P;
                double best_near = 1e300;
                for (int ps = 0; ps < kSymShapeCount; ++ps) {
                    c->opt.p2p_shape = ps;
                    c->tree_valid = false;
                    ensure_tree(c);
                    ensure_ops(c);
                    matvec_sorted(c, 1.0, x.get(), 0.0, nullptr, y.get(), false, prec, false);  // warm-up
                    BFM_HIP(hipStreamSynchronize(st));
                    c->prof.reset();
                    c->prof.on = true;
                    for (int r = 0; r < 3; ++r) matvec_sorted(c, 1.0, x.get(), 0.0, nullptr, y.get(), false, prec, false);
                    BFM_HIP(hipStreamSynchronize(st));
                    double ms = 0.0;
                    for (const auto &rec : c->prof.recs)
                        if (rec.cls == cls) {
                            float e = 0.f;
                            BFM_HIP(hipEventElapsedTime(&e, rec.a, rec.b));
                            ms += e;
                        }
                    c->prof.on = false;
                    c->prof.reset();
                    ++cand;
                    if (ms < best_near) {
                        best_near = ms;
                        best_ps = ps;
                    }
                }
            }
        }
        c->opt = saved;
        c->opt.p = best_p;
        c->opt.p2p_shape = best_ps;
        c->opt.p_diag = best_pd;
        c->opt.lmax = best_l;
        c->opt.m2l_shape = best_s;
        if (ir) c->opt.p_lo = best_plo;
        c->tree_valid = false;
        c->diag_valid = false;
        graph_invalidate(c);
        if (out) {
            out->p = best_p;
            out->p_lo = ir ? best_plo : 0;
            out->lmax = best_l;
            out->m2l_shape = best_s;
            out->candidates = cand;
            out->mvp_ms = best_ms;
            out->p_err = best_err;
            out->p_diag = best_pd;
            out->diag_err = best_derr;
            out->p2p_shape = best_ps;
        }
    } catch (...) {
        c->opt = saved;
        c->tree_valid = false;
        c->diag_valid = false;
        graph_invalidate(c);
        throw;
    }
}

}  // namespace bfm
