// C ABI of libbfm (declared in include/bfm.h). Every entry point catches
// internal errors and turns them into a return code plus a thread-local
// message; nothing throws across the boundary.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/bfm_debug.h"
#include "../../include/bfm_mlp.h"
#include "../../include/bfm_step.h"
#include "ctx.h"
#include "direct.h"
#include "learn.h"
#include "ops.h"

namespace bfm {

static thread_local std::string g_last_error;

[[noreturn]] void fail(int code, const std::string &msg) { throw Error{code, msg}; }

template <class F>
static int guarded(F &&f) {
    try {
        f();
        return BFM_OK;
    } catch (const Error &e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return BFM_ENOMEM;
    } catch (...) {
        g_last_error = "unexpected internal error";
        return BFM_EINVAL;
    }
}

static void check_options(const bfm_options &o) {
    BFM_CHECK(o.abi_version == BFM_ABI_VERSION, BFM_EINVAL, "abi_version mismatch");
    BFM_CHECK(o.p >= 4 && o.p <= kMaxP && o.p % 4 == 0, BFM_EINVAL,
              "p must be a multiple of 4 in [4, 20]");
    BFM_CHECK(o.p_diag == 0 || (o.p_diag >= 4 && o.p_diag <= kMaxP && o.p_diag % 4 == 0), BFM_EINVAL,
              "p_diag must be 0 or a multiple of 4 in [4, 20]");
    BFM_CHECK(o.lmax == 0 || (o.lmax >= 2 && o.lmax <= 15), BFM_EINVAL, "lmax must be 0 or in [2, 15]");
    BFM_CHECK(o.leaf_target >= 1, BFM_EINVAL, "leaf_target must be >= 1");
    BFM_CHECK(o.precision == BFM_PREC_FP64 || o.precision == BFM_PREC_FP32 || o.precision == BFM_PREC_BF16X3,
              BFM_EINVAL, "unknown precision");
    BFM_CHECK(o.p_lo == 0 || (o.p_lo >= 4 && o.p_lo <= kMaxP && o.p_lo % 4 == 0), BFM_EINVAL,
              "p_lo must be 0 or a multiple of 4 in [4, 20]");
    BFM_CHECK(o.ir_tol >= 0.0 && o.ir_tol < 1.0, BFM_EINVAL, "ir_tol must be in [0, 1)");
    BFM_CHECK(o.gmres_tol > 0.0 && o.gmres_tol < 1.0, BFM_EINVAL, "gmres_tol must be in (0, 1)");
    BFM_CHECK(o.gmres_restart >= 1 && o.gmres_restart <= 128, BFM_EINVAL,
              "gmres_restart must be in [1, 128]");
    BFM_CHECK(o.gmres_maxit >= 1, BFM_EINVAL, "gmres_maxit must be >= 1");
    BFM_CHECK(o.precond == BFM_PRECOND_NONE || o.precond == BFM_PRECOND_SH || o.precond == BFM_PRECOND_SH_COARSE,
              BFM_EINVAL, "unknown precond");
    BFM_CHECK(o.precond_degree >= 1 && o.precond_degree <= 40, BFM_EINVAL, "precond_degree must be in [1, 40]");
    BFM_CHECK(o.m2l_shape >= -1 && o.m2l_shape <= 3, BFM_EINVAL, "m2l_shape must be -1, 0, 1, 2 or 3");
    BFM_CHECK(o.m2l_orders == 0 || o.m2l_orders == 1, BFM_EINVAL, "m2l_orders must be 0 or 1");
    BFM_CHECK(o.p2p_shape >= -1 && o.p2p_shape < kSymShapeCount, BFM_EINVAL, "p2p_shape must be -1, 0, 1 or 2");
    BFM_CHECK(o.near_corr == 0 || o.near_corr == 1, BFM_EINVAL, "near_corr must be 0 or 1");
}

struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev) {
        BFM_HIP(hipGetDevice(&prev));
        if (prev != dev) BFM_HIP(hipSetDevice(dev));
    }
    ~DeviceScope() {
        int cur = -1;
        if (hipGetDevice(&cur) == hipSuccess && prev >= 0 && cur != prev) (void)hipSetDevice(prev);
    }
};

static void invalidate_positions(bfm_ctx *c) {
    c->geom_valid = false;
    c->tree_valid = false;
    c->diag_valid = false;
}

// Timing with HIP events on the handle's stream: stop() only records, ms()
// waits for the stop event, so a phase boundary does not drain the stream.
struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t st;
    explicit Timer(hipStream_t s) : st(s) {
        BFM_HIP(hipEventCreate(&a));
        BFM_HIP(hipEventCreate(&b));
        BFM_HIP(hipEventRecord(a, st));
    }
    void stop() { BFM_HIP(hipEventRecord(b, st)); }
    double ms() {
        BFM_HIP(hipEventSynchronize(b));
        float v = 0.f;
        BFM_HIP(hipEventElapsedTime(&v, a, b));
        return v;
    }
    double stop_ms() {
        stop();
        return ms();
    }
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

static void solve_rest(bfm_ctx *c, const double *phi_dev, double *q_dev, int guess, Timer &t_tree,
                       bfm_solve_info *info);

void solve_impl(bfm_ctx *c, const double *phi_dev, double *q_dev, int guess, bfm_solve_info *info) {
    BFM_CHECK(guess == BFM_GUESS_ZERO || guess == BFM_GUESS_GIVEN || guess == BFM_GUESS_LEARNED, BFM_EINVAL,
              "use_guess must be BFM_GUESS_ZERO, BFM_GUESS_GIVEN or BFM_GUESS_LEARNED");
    // phase timers only record events; their times are read once at the end
    Timer t_tree(c->stream);
    ensure_geometry(c, false);  // checked by the octree build's first wait
    // the coarse space needs only the geometry: it is built on a second stream
    // beside the octree build, whose short kernels and host round trips leave
    // most of the device free (beside the diagonal pass its serial chain of
    // small kernels would wait for every wave of the pass's large launches)
    if (c->opt.precond == BFM_PRECOND_SH_COARSE && c->pre.nd > 0 && c->pre.genus == 0) {
        coarse_mark(c);
        coarse_launch(c);
    }
    try {
        solve_rest(c, phi_dev, q_dev, guess, t_tree, info);
    } catch (...) {
        // the worker has queued the build before the call returns (no thread
        // of the handle is left running between calls)
        try {
            coarse_join(c);
        } catch (...) {
        }
        throw;
    }
}

static void solve_rest(bfm_ctx *c, const double *phi_dev, double *q_dev, int guess, Timer &t_tree,
                       bfm_solve_info *info) {
    bfm_solve_info loc{};
    const int64_t n = c->nv;
    ensure_tree(c);
    t_tree.stop();
    Timer t_guess(c->stream);
    if (guess == BFM_GUESS_LEARNED) mlp_guess(c, phi_dev, q_dev);
    t_guess.stop();
    const bool use_guess = guess != BFM_GUESS_ZERO;
    Timer t_diag(c->stream);
    diagonal_pass(c, phi_dev);
    t_diag.stop();
    Timer t_solve(c->stream);
    double *x = c->x_s.ensure(n);
    if (use_guess) to_sorted(c, q_dev, x);
    gmres_sorted(c, x, use_guess, &loc);
    to_original(c, x, q_dev);
    t_solve.stop();
    loc.t_tree_ms = t_tree.ms();
    loc.t_guess_ms = guess == BFM_GUESS_LEARNED ? t_guess.ms() : 0.0;
    loc.t_diag_ms = t_diag.ms();
    loc.t_solve_ms = t_solve.ms();
    if (info) *info = loc;
    if (!loc.converged) fail(BFM_ENOCONV, "GMRES reached gmres_maxit before the tolerance");
}

}  // namespace bfm

using namespace bfm;

extern "C" {

const char *bfm_last_error(void) { return g_last_error.c_str(); }

int bfm_default_options(bfm_options *opt) {
    if (!opt) return BFM_EINVAL;
    std::memset(opt, 0, sizeof(*opt));
    opt->abi_version = BFM_ABI_VERSION;
    opt->device = 0;
    opt->stream = nullptr;
    opt->p = 16;
    opt->p_diag = 0;
    opt->lmax = 0;
    opt->leaf_target = 64;
    opt->precision = BFM_PREC_FP64;
    opt->gmres_tol = 1e-10;
    opt->gmres_restart = 30;
    opt->gmres_maxit = 300;
    opt->precond = BFM_PRECOND_NONE;
    opt->precond_degree = 12;
    opt->use_graph = 0;
    opt->m2l_shape = -1;
    opt->p2p_shape = -1;
    opt->near_corr = 0;
    return BFM_OK;
}

int bfm_create(const bfm_options *opt, bfm_ctx **out) {
    return guarded([&] {
        BFM_CHECK(opt && out, BFM_EINVAL, "null argument");
        check_options(*opt);
        int ndev = 0;
        BFM_HIP(hipGetDeviceCount(&ndev));
        BFM_CHECK(opt->device >= 0 && opt->device < ndev, BFM_EINVAL, "device ordinal out of range");
        DeviceScope ds(opt->device);
        auto *c = new bfm_ctx();
        c->fmm.prof = &c->prof;
        c->fmm_diag.prof = &c->prof;  // the diagonal pass's kernels in their own classes
        c->fmm_diag.prof_base = kDiagBase;
        c->fmm_lo.prof = &c->prof;
        c->fmm_lo.prof_base = kLoBase;
        c->opt = *opt;
        c->device = opt->device;
        if (opt->stream) {
            c->stream = (hipStream_t)opt->stream;
        } else {
            hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
            if (e != hipSuccess) {
                delete c;
                fail(BFM_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
            }
            c->own_stream = true;
        }
        {
            hipError_t e = hipStreamCreateWithFlags(&c->near, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&c->fmm.ev_fork, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&c->fmm.ev_join, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&c->fmm_diag.ev_fork, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&c->fmm_diag.ev_join, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&c->fmm_lo.ev_fork, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&c->fmm_lo.ev_join, hipEventDisableTiming);
            if (e != hipSuccess) {
                if (c->own_stream) (void)hipStreamDestroy(c->stream);
                if (c->near) (void)hipStreamDestroy(c->near);
                delete c;
                fail(BFM_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
            }
            c->fmm.near = c->near;
            c->fmm_diag.near = c->near;
            c->fmm_lo.near = c->near;
        }
        *out = c;
    });
}

int bfm_destroy(bfm_ctx *c) {
    return guarded([&] {
        if (!c) return;
        DeviceScope ds(c->device);
        (void)hipStreamSynchronize(c->stream);
        mlp_free(c);
        step_free(c);
        graph_invalidate(c);
        graph_release_stale(c);
        try {
            coarse_join(c);  // (an error of the build is of no interest here)
        } catch (...) {
        }
        coarse_worker_free(c);
        if (c->host_small) (void)hipHostFree(c->host_small);
        if (c->host_flag) (void)hipHostFree(c->host_flag);
        if (c->side) {
            (void)hipStreamSynchronize(c->side);
            (void)hipStreamDestroy(c->side);
        }
        if (c->near) {
            (void)hipStreamSynchronize(c->near);
            (void)hipStreamDestroy(c->near);
        }
        for (bfm::FmmWork *w : {&c->fmm, &c->fmm_diag, &c->fmm_lo}) {
            if (w->ev_fork) (void)hipEventDestroy(w->ev_fork);
            if (w->ev_join) (void)hipEventDestroy(w->ev_join);
        }
        if (c->ev_geom) (void)hipEventDestroy(c->ev_geom);
        if (c->ev_coarse) (void)hipEventDestroy(c->ev_coarse);
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        delete c;
    });
}

int bfm_set_options(bfm_ctx *c, const bfm_options *opt) {
    return guarded([&] {
        BFM_CHECK(c && opt, BFM_EINVAL, "null argument");
        check_options(*opt);
        BFM_CHECK(opt->device == c->device, BFM_EINVAL, "cannot change the device of a handle");
        const bool tree_change = opt->lmax != c->opt.lmax || opt->leaf_target != c->opt.leaf_target ||
                                 opt->p2p_shape != c->opt.p2p_shape;
        const bool p_change = opt->p != c->opt.p || opt->p_diag != c->opt.p_diag ||
                              opt->m2l_orders != c->opt.m2l_orders || opt->near_corr != c->opt.near_corr;
        // (p_lo and precision take effect at the next low-precision product)
        void *keep_stream = c->opt.stream;
        c->opt = *opt;
        c->opt.stream = keep_stream;
        if (tree_change) {
            c->tree_valid = false;
            c->diag_valid = false;
        }
        if (p_change) c->diag_valid = false;
        graph_invalidate(c);
        if (opt->precond_degree != c->pre.nmax) c->pre.ready = false;
    });
}

int bfm_set_mesh(bfm_ctx *c, int64_t nv, const double *xyz, int64_t nt, const int32_t *tri, int32_t nb,
                 const int64_t *vtx_off, const int64_t *tri_off) {
    return guarded([&] {
        BFM_CHECK(c && xyz && tri, BFM_EINVAL, "null argument");
        BFM_CHECK(nv >= 4 && nt >= 4, BFM_EINVAL, "a closed surface needs >= 4 vertices and triangles");
        BFM_CHECK(nv < (int64_t)1 << 30 && nt < (int64_t)1 << 30, BFM_EINVAL, "mesh too large");
        BFM_CHECK(nb >= 0, BFM_EINVAL, "negative bubble count");
        if (c->side) {  // a coarse build in flight reads the buffers replaced below
            DeviceScope ds(c->device);
            coarse_join(c);  // the worker has queued the build
            BFM_HIP(hipStreamSynchronize(c->side));
        }
        if (nb > 1) BFM_CHECK(vtx_off && tri_off, BFM_EINVAL, "bubble ranges required when nb > 1");
        DeviceScope ds(c->device);
        std::vector<int64_t> vo, to;
        if (nb >= 1 && vtx_off && tri_off) {
            vo.assign(vtx_off, vtx_off + nb + 1);
            to.assign(tri_off, tri_off + nb + 1);
            BFM_CHECK(vo[0] == 0 && vo[nb] == nv && to[0] == 0 && to[nb] == nt, BFM_EINVAL,
                      "bubble ranges must cover all vertices and triangles");
            for (int b = 0; b < nb; ++b)
                BFM_CHECK(vo[b + 1] > vo[b] && to[b + 1] > to[b], BFM_EINVAL, "empty bubble range");
        }
        // vertex -> triangle adjacency (ascending triangle index)
        std::vector<int> cnt(nv + 1, 0);
        for (int64_t k = 0; k < 3 * nt; ++k) {
            const int v = tri[k];
            BFM_CHECK(v >= 0 && v < nv, BFM_EMESH, "triangle vertex index out of range");
            cnt[v + 1]++;
        }
        for (int64_t v = 0; v < nv; ++v) {
            BFM_CHECK(cnt[v + 1] > 0, BFM_EMESH, "vertex " + std::to_string(v) + " is in no triangle");
            cnt[v + 1] += cnt[v];
        }
        std::vector<int> adj(3 * nt), cur(cnt.begin(), cnt.end() - 1);
        for (int64_t k = 0; k < nt; ++k)
            for (int e = 0; e < 3; ++e) adj[cur[tri[3 * k + e]]++] = (int)k;
        c->nv = nv;
        c->nt = nt;
        c->nb = nb >= 1 ? nb : 1;
        if (vo.empty()) {
            vo = {0, nv};
            to = {0, nt};
        }
        c->tri_h.assign(tri, tri + 3 * nt);
        corr_invalidate(c, true);
        step_mesh_changed(c);
        c->tri0_h.clear();
        for (int64_t k = 3 * to[0]; k < 3 * to[1]; ++k) c->tri0_h.push_back(tri[k] - (int)vo[0]);
        c->pre.nd = 0;
        c->pre.genus = 0;
        c->pre.ready = false;
        c->pre.gen += 1;
        c->vtx_off = vo;
        c->tri_off = to;
        c->xyz.ensure(3 * nv);
        c->tri.ensure(3 * nt);
        c->v2t_off.ensure(nv + 1);
        c->v2t.ensure(3 * nt);
        hipStream_t st = c->stream;
        BFM_HIP(hipMemcpyAsync(c->xyz.get(), xyz, sizeof(double) * 3 * nv, hipMemcpyHostToDevice, st));
        BFM_HIP(hipMemcpyAsync(c->tri.get(), tri, sizeof(int) * 3 * nt, hipMemcpyHostToDevice, st));
        BFM_HIP(hipMemcpyAsync(c->v2t_off.get(), cnt.data(), sizeof(int) * (nv + 1), hipMemcpyHostToDevice, st));
        BFM_HIP(hipMemcpyAsync(c->v2t.get(), adj.data(), sizeof(int) * 3 * nt, hipMemcpyHostToDevice, st));
        BFM_HIP(hipStreamSynchronize(st));
        invalidate_positions(c);
    });
}

int bfm_set_sphere_template(bfm_ctx *c, int32_t nd, const double *dirs) {
    return guarded([&] {
        BFM_CHECK(c && dirs, BFM_EINVAL, "null argument");
        BFM_CHECK(c->nv > 0, BFM_EINVAL, "no mesh set");
        BFM_CHECK(nd >= 4 && (int64_t)nd * c->nb == c->nv, BFM_EINVAL,
                  "every bubble must hold nd vertices (nv = nb * nd)");
        for (int b = 0; b <= c->nb; ++b)
            BFM_CHECK(c->vtx_off[b] == (int64_t)b * nd, BFM_EINVAL, "bubble vertex ranges must be b * nd");
        for (int v : c->tri0_h) BFM_CHECK(v >= 0 && v < nd, BFM_EINVAL, "first bubble's triangles leave its range");
        for (int v = 0; v < nd; ++v) {
            const double r = std::sqrt(dirs[3 * v] * dirs[3 * v] + dirs[3 * v + 1] * dirs[3 * v + 1] +
                                       dirs[3 * v + 2] * dirs[3 * v + 2]);
            BFM_CHECK(std::fabs(r - 1.0) < 1e-6, BFM_EINVAL, "template directions must be unit vectors");
        }
        c->pre.dirs_h.assign(dirs, dirs + 3 * (size_t)nd);
        c->pre.ang_h.clear();
        c->pre.genus = 0;
        c->pre.tri_h = c->tri0_h;
        c->pre.nd = nd;
        c->pre.ready = false;
        c->pre.gen += 1;  // rebuild every harmonic basis for the new template
        step_mesh_changed(c);
    });
}

int bfm_set_torus_template(bfm_ctx *c, int32_t nd, const double *angles) {
    return guarded([&] {
        BFM_CHECK(c && angles, BFM_EINVAL, "null argument");
        BFM_CHECK(c->nv > 0, BFM_EINVAL, "no mesh set");
        BFM_CHECK(nd >= 4 && (int64_t)nd * c->nb == c->nv, BFM_EINVAL,
                  "every bubble must hold nd vertices (nv = nb * nd)");
        for (int b = 0; b <= c->nb; ++b)
            BFM_CHECK(c->vtx_off[b] == (int64_t)b * nd, BFM_EINVAL, "bubble vertex ranges must be b * nd");
        for (int v : c->tri0_h) BFM_CHECK(v >= 0 && v < nd, BFM_EINVAL, "first bubble's triangles leave its range");
        for (int v = 0; v < 2 * nd; ++v)
            BFM_CHECK(std::isfinite(angles[v]), BFM_EINVAL, "template angles must be finite");
        c->pre.ang_h.assign(angles, angles + 2 * (size_t)nd);
        c->pre.dirs_h.clear();
        c->pre.genus = 1;
        c->pre.tri_h = c->tri0_h;
        c->pre.nd = nd;
        c->pre.ready = false;
        c->pre.gen += 1;
        step_mesh_changed(c);
    });
}

int bfm_set_positions(bfm_ctx *c, const double *xyz) {
    return guarded([&] {
        BFM_CHECK(c && xyz, BFM_EINVAL, "null argument");
        BFM_CHECK(c->nv > 0, BFM_EINVAL, "no mesh set");
        DeviceScope ds(c->device);
        coarse_join(c);  // a coarse build in flight reads the positions
        BFM_HIP(hipMemcpyAsync(c->xyz.get(), xyz, sizeof(double) * 3 * c->nv, hipMemcpyHostToDevice,
                               c->stream));
        BFM_HIP(hipStreamSynchronize(c->stream));
        invalidate_positions(c);
    });
}

int bfm_set_positions_dev(bfm_ctx *c, const double *xyz) {
    return guarded([&] {
        BFM_CHECK(c && xyz, BFM_EINVAL, "null argument");
        BFM_CHECK(c->nv > 0, BFM_EINVAL, "no mesh set");
        DeviceScope ds(c->device);
        coarse_join(c);  // a coarse build in flight reads the positions
        BFM_HIP(hipMemcpyAsync(c->xyz.get(), xyz, sizeof(double) * 3 * c->nv, hipMemcpyDeviceToDevice,
                               c->stream));
        invalidate_positions(c);
    });
}

int bfm_geometry(bfm_ctx *c, double *s, double *n) {
    return guarded([&] {
        BFM_CHECK(c && s && n, BFM_EINVAL, "null argument");
        DeviceScope ds(c->device);
        ensure_geometry(c);
        std::vector<double> tmp(3 * c->nv);
        BFM_HIP(hipMemcpyAsync(s, c->s.get(), sizeof(double) * c->nv, hipMemcpyDeviceToHost, c->stream));
        BFM_HIP(hipMemcpyAsync(tmp.data(), c->nrm.get(), sizeof(double) * 3 * c->nv, hipMemcpyDeviceToHost,
                               c->stream));
        BFM_HIP(hipStreamSynchronize(c->stream));
        for (int64_t j = 0; j < c->nv; ++j)
            for (int d = 0; d < 3; ++d) n[3 * j + d] = tmp[d * c->nv + j];
    });
}

int bfm_diagonals(bfm_ctx *c, const double *phi, double *Mii, double *Lii, double *b) {
    return guarded([&] {
        BFM_CHECK(c && phi, BFM_EINVAL, "null argument");
        DeviceScope ds(c->device);
        const int64_t n = c->nv;
        BFM_CHECK(n > 0, BFM_EINVAL, "no mesh set");
        DevBuf<double> dphi, tmp;
        dphi.ensure(n);
        tmp.ensure(n);
        BFM_HIP(hipMemcpyAsync(dphi.get(), phi, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
        diagonal_pass(c, dphi.get());
        double *outs[3] = {Mii, Lii, b};
        const double *srcs[3] = {c->mii_s.get(), c->lii_s.get(), c->b_s.get()};
        for (int k = 0; k < 3; ++k) {
            if (!outs[k]) continue;
            to_original(c, srcs[k], tmp.get());
            BFM_HIP(hipMemcpyAsync(outs[k], tmp.get(), sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
            BFM_HIP(hipStreamSynchronize(c->stream));
        }
    });
}

int bfm_matvec(bfm_ctx *c, double f, const double *x, double g, const double *y, double *out,
               int add_diag, int precision, int direct) {
    return guarded([&] {
        BFM_CHECK(c && out, BFM_EINVAL, "null argument");
        BFM_CHECK(f == 0.0 || x, BFM_EINVAL, "x required when f != 0");
        BFM_CHECK(g == 0.0 || y, BFM_EINVAL, "y required when g != 0");
        DeviceScope ds(c->device);
        const int64_t n = c->nv;
        BFM_CHECK(n > 0, BFM_EINVAL, "no mesh set");
        ensure_tree(c);
        DevBuf<double> dx, dy, ds_, dout;
        hipStream_t st = c->stream;
        double *xs = nullptr, *ys = nullptr;
        if (f != 0.0) {
            dx.ensure(n);
            xs = ds_.ensure(2 * n);
            BFM_HIP(hipMemcpyAsync(dx.get(), x, sizeof(double) * n, hipMemcpyHostToDevice, st));
            to_sorted(c, dx.get(), xs);
        }
        if (g != 0.0) {
            dy.ensure(n);
            if (!ds_.get()) ds_.ensure(2 * n);
            ys = ds_.get() + n;
            BFM_HIP(hipMemcpyAsync(dy.get(), y, sizeof(double) * n, hipMemcpyHostToDevice, st));
            to_sorted(c, dy.get(), ys);
        }
        double *os = dout.ensure(2 * n);
        matvec_sorted(c, f, xs, g, ys, os, add_diag != 0, precision, direct != 0);
        to_original(c, os, os + n);
        BFM_HIP(hipMemcpyAsync(out, os + n, sizeof(double) * n, hipMemcpyDeviceToHost, st));
        BFM_HIP(hipStreamSynchronize(st));
    });
}

int bfm_solve_dev(bfm_ctx *c, const double *phi_dev, double *q_dev, int use_guess, bfm_solve_info *info) {
    return guarded([&] {
        BFM_CHECK(c && phi_dev && q_dev, BFM_EINVAL, "null argument");
        BFM_CHECK(c->nv > 0, BFM_EINVAL, "no mesh set");
        DeviceScope ds(c->device);
        solve_impl(c, phi_dev, q_dev, use_guess, info);
        BFM_HIP(hipStreamSynchronize(c->stream));
    });
}

int bfm_solve(bfm_ctx *c, const double *phi, double *q, int use_guess, bfm_solve_info *info) {
    int rc_solve = BFM_OK;
    int rc = guarded([&] {
        BFM_CHECK(c && phi && q, BFM_EINVAL, "null argument");
        BFM_CHECK(c->nv > 0, BFM_EINVAL, "no mesh set");
        DeviceScope ds(c->device);
        const int64_t n = c->nv;
        DevBuf<double> buf;
        buf.ensure(2 * n);
        hipStream_t st = c->stream;
        BFM_HIP(hipMemcpyAsync(buf.get(), phi, sizeof(double) * n, hipMemcpyHostToDevice, st));
        if (use_guess == BFM_GUESS_GIVEN)
            BFM_HIP(hipMemcpyAsync(buf.get() + n, q, sizeof(double) * n, hipMemcpyHostToDevice, st));
        try {
            solve_impl(c, buf.get(), buf.get() + n, use_guess, info);
        } catch (const Error &e) {
            if (e.code != BFM_ENOCONV) throw;
            g_last_error = e.msg;
            rc_solve = e.code;
        }
        BFM_HIP(hipMemcpyAsync(q, buf.get() + n, sizeof(double) * n, hipMemcpyDeviceToHost, st));
        BFM_HIP(hipStreamSynchronize(st));
    });
    return rc != BFM_OK ? rc : rc_solve;
}

int bfm_direct_dev(int64_t n, const double *xyz, const double *s, const double *nrm, double f, const double *x,
                   double g, const double *y, int64_t nr, const int64_t *rows, double *out, void *stream) {
    return guarded([&] {
        DirectArgs a;
        a.n = n;
        a.xyz = xyz;
        a.s = s;
        a.nrm = nrm;
        a.f = f;
        a.x = x;
        a.g = g;
        a.y = y;
        a.nr = nr;
        a.rows = rows;
        a.out = out;
        direct_product(a, (hipStream_t)stream);
    });
}

int bfm_direct_dev_noalloc(int64_t n, const double *xyz, const double *s, const double *nrm, double f,
                           const double *x, double g, const double *y, int64_t nr, const int64_t *rows, double *out,
                           void *stream) {
    return guarded([&] {
        DirectArgs a;
        a.n = n;
        a.xyz = xyz;
        a.s = s;
        a.nrm = nrm;
        a.f = f;
        a.x = x;
        a.g = g;
        a.y = y;
        a.nr = nr;
        a.rows = rows;
        a.out = out;
        direct_product_noalloc(a, (hipStream_t)stream);
    });
}

int bfm_tree_stats(bfm_ctx *c, int n, int64_t *stats) {
    return guarded([&] {
        BFM_CHECK(c && stats, BFM_EINVAL, "null argument");
        BFM_CHECK(n >= 0, BFM_EINVAL, "negative count");
        DeviceScope ds(c->device);
        ensure_tree(c);
        const Tree &t = c->tree;
        int64_t tr = 0;
        for (size_t l = 0; l < t.m2m.size(); ++l)
            if (t.m2m[l]) tr += t.m2m[l]->ntasks;
        const int64_t v[BFM_TREE_STATS] = {t.lmax, t.nleaf, t.nbox, t.npairs_near, t.m2l.ntasks, 2 * tr,
                                           t.max_leaf, c->fmm.m2l_shape_used, c->fmm_diag.m2l_shape_used};
        for (int k = 0; k < n; ++k) stats[k] = k < BFM_TREE_STATS ? v[k] : 0;
    });
}

int bfm_profile(bfm_ctx *c, int enable) {
    return guarded([&] {
        BFM_CHECK(c, BFM_EINVAL, "null argument");
        DeviceScope ds(c->device);
        BFM_HIP(hipStreamSynchronize(c->stream));
        if (enable) c->prof.reset();
        c->prof.on = enable != 0;
    });
}

int bfm_profile_read(bfm_ctx *c, int nclass, double *ms, int64_t *launches, double *flops) {
    return guarded([&] {
        BFM_CHECK(c && ms && launches && flops, BFM_EINVAL, "null argument");
        BFM_CHECK(nclass >= 0, BFM_EINVAL, "negative class count");
        DeviceScope ds(c->device);
        BFM_HIP(hipStreamSynchronize(c->stream));
        for (int k = 0; k < nclass; ++k) {
            ms[k] = 0.0;
            launches[k] = 0;
            flops[k] = 0.0;
        }
        for (const auto &r : c->prof.recs) {
            if (r.cls >= nclass) continue;
            float t = 0.f;
            BFM_HIP(hipEventElapsedTime(&t, r.a, r.b));
            ms[r.cls] += t;
            launches[r.cls] += 1;
            flops[r.cls] += r.flops;
        }
    });
}

// ---------------------------------------------------------------------------
// Learned initial guess (include/bfm_mlp.h)

int bfm_mlp_init(bfm_ctx *c, uint64_t seed) {
    return guarded([&] {
        BFM_CHECK(c, BFM_EINVAL, "null argument");
        DeviceScope ds(c->device);
        mlp_init(mlp_get(c), seed, c->stream);
    });
}

int bfm_mlp_set_params(bfm_ctx *c, const float *params) {
    return guarded([&] {
        BFM_CHECK(c && params, BFM_EINVAL, "null argument");
        DeviceScope ds(c->device);
        mlp_set_params(mlp_get(c), params, c->stream);
    });
}

int bfm_mlp_get_params(bfm_ctx *c, float *params) {
    return guarded([&] {
        BFM_CHECK(c && params, BFM_EINVAL, "null argument");
        DeviceScope ds(c->device);
        mlp_get_params(mlp_get(c), params, false, c->stream);
    });
}

int bfm_mlp_set_norm(bfm_ctx *c, const float *norm) {
    return guarded([&] {
        BFM_CHECK(c && norm, BFM_EINVAL, "null argument");
        DeviceScope ds(c->device);
        mlp_set_norm(mlp_get(c), norm, c->stream);
    });
}

int bfm_mlp_get_norm(bfm_ctx *c, float *norm) {
    return guarded([&] {
        BFM_CHECK(c && norm, BFM_EINVAL, "null argument");
        DeviceScope ds(c->device);
        mlp_get_norm(mlp_get(c), norm, c->stream);
    });
}

int bfm_mlp_forward(bfm_ctx *c, int64_t rows, const float *x, float *y) {
    return guarded([&] {
        BFM_CHECK(c && x && y, BFM_EINVAL, "null argument");
        BFM_CHECK(rows >= 1 && rows <= (1 << 24), BFM_EINVAL, "rows must be in [1, 2^24]");
        DeviceScope ds(c->device);
        hipStream_t st = c->stream;
        DevBuf<float> dx, dy;
        dx.ensure((size_t)rows * BFM_MLP_INPUTS);
        dy.ensure((size_t)rows * BFM_MLP_OUTPUTS);
        BFM_HIP(hipMemcpyAsync(dx.get(), x, sizeof(float) * rows * BFM_MLP_INPUTS, hipMemcpyHostToDevice, st));
        mlp_forward_rows(mlp_get(c), rows, dx.get(), dy.get(), st);
        BFM_HIP(hipMemcpyAsync(y, dy.get(), sizeof(float) * rows * BFM_MLP_OUTPUTS, hipMemcpyDeviceToHost, st));
        BFM_HIP(hipStreamSynchronize(st));
    });
}

int bfm_mlp_gradient(bfm_ctx *c, int64_t rows, const float *x, const float *t, float *grad, double *loss) {
    return guarded([&] {
        BFM_CHECK(c && x && t, BFM_EINVAL, "null argument");
        BFM_CHECK(rows >= 1 && rows <= (1 << 24), BFM_EINVAL, "rows must be in [1, 2^24]");
        DeviceScope ds(c->device);
        hipStream_t st = c->stream;
        DevBuf<float> dx, dt;
        dx.ensure((size_t)rows * BFM_MLP_INPUTS);
        dt.ensure((size_t)rows * BFM_MLP_OUTPUTS);
        BFM_HIP(hipMemcpyAsync(dx.get(), x, sizeof(float) * rows * BFM_MLP_INPUTS, hipMemcpyHostToDevice, st));
        BFM_HIP(hipMemcpyAsync(dt.get(), t, sizeof(float) * rows * BFM_MLP_OUTPUTS, hipMemcpyHostToDevice, st));
        Mlp &net = mlp_get(c);
        const double l = mlp_gradient_rows(net, rows, dx.get(), dt.get(), st);
        if (grad) mlp_get_params(net, grad, true, st);
        if (loss) *loss = l;
    });
}

int bfm_mlp_adam_step(bfm_ctx *c, float lr) {
    return guarded([&] {
        BFM_CHECK(c, BFM_EINVAL, "null argument");
        BFM_CHECK(lr > 0.f, BFM_EINVAL, "lr must be positive");
        DeviceScope ds(c->device);
        mlp_adam(mlp_get(c), lr, c->stream);
        BFM_HIP(hipStreamSynchronize(c->stream));
    });
}

int bfm_mlp_features(bfm_ctx *c, const double *phi, const double *q, float *feat, float *targ) {
    return guarded([&] {
        BFM_CHECK(c && phi && feat, BFM_EINVAL, "null argument");
        BFM_CHECK(c->nv > 0, BFM_EINVAL, "no mesh set");
        DeviceScope ds(c->device);
        hipStream_t st = c->stream;
        const int64_t n = c->nv, nb = c->nb;
        const bool with_t = q && targ;
        DevBuf<double> dv;
        DevBuf<float> df;
        dv.ensure(2 * n);
        df.ensure((size_t)nb * (BFM_MLP_INPUTS + BFM_MLP_OUTPUTS));
        BFM_HIP(hipMemcpyAsync(dv.get(), phi, sizeof(double) * n, hipMemcpyHostToDevice, st));
        if (with_t) BFM_HIP(hipMemcpyAsync(dv.get() + n, q, sizeof(double) * n, hipMemcpyHostToDevice, st));
        float *ft = df.get() + nb * BFM_MLP_INPUTS;
        mlp_features(c, dv.get(), with_t ? dv.get() + n : nullptr, df.get(), with_t ? ft : nullptr);
        BFM_HIP(hipMemcpyAsync(feat, df.get(), sizeof(float) * nb * BFM_MLP_INPUTS, hipMemcpyDeviceToHost, st));
        if (with_t)
            BFM_HIP(hipMemcpyAsync(targ, ft, sizeof(float) * nb * BFM_MLP_OUTPUTS, hipMemcpyDeviceToHost, st));
        BFM_HIP(hipStreamSynchronize(st));
    });
}

int bfm_mlp_collect_dev(bfm_ctx *c, const double *phi_dev, const double *q_dev) {
    return guarded([&] {
        BFM_CHECK(c && phi_dev && q_dev, BFM_EINVAL, "null argument");
        BFM_CHECK(c->nv > 0, BFM_EINVAL, "no mesh set");
        DeviceScope ds(c->device);
        mlp_collect(c, phi_dev, q_dev);
    });
}

int bfm_mlp_dataset(bfm_ctx *c, int clear, int64_t *rows) {
    return guarded([&] {
        BFM_CHECK(c, BFM_EINVAL, "null argument");
        DeviceScope ds(c->device);
        Mlp &net = mlp_get(c);
        if (clear) net.ds_rows = 0;
        if (rows) *rows = net.ds_rows;
    });
}

int bfm_mlp_fit(bfm_ctx *c, int epochs, int batch, float lr, uint64_t seed, double *loss) {
    return guarded([&] {
        BFM_CHECK(c, BFM_EINVAL, "null argument");
        DeviceScope ds(c->device);
        const double l = mlp_fit(c, epochs, batch, lr, seed);
        if (loss) *loss = l;
    });
}

int bfm_mlp_guess_dev(bfm_ctx *c, const double *phi_dev, double *q_dev) {
    return guarded([&] {
        BFM_CHECK(c && phi_dev && q_dev, BFM_EINVAL, "null argument");
        BFM_CHECK(c->nv > 0, BFM_EINVAL, "no mesh set");
        DeviceScope ds(c->device);
        mlp_guess(c, phi_dev, q_dev);
        BFM_HIP(hipStreamSynchronize(c->stream));
    });
}

int bfm_mlp_guess(bfm_ctx *c, const double *phi, double *q) {
    return guarded([&] {
        BFM_CHECK(c && phi && q, BFM_EINVAL, "null argument");
        BFM_CHECK(c->nv > 0, BFM_EINVAL, "no mesh set");
        DeviceScope ds(c->device);
        hipStream_t st = c->stream;
        const int64_t n = c->nv;
        DevBuf<double> dv;
        dv.ensure(2 * n);
        BFM_HIP(hipMemcpyAsync(dv.get(), phi, sizeof(double) * n, hipMemcpyHostToDevice, st));
        mlp_guess(c, dv.get(), dv.get() + n);
        BFM_HIP(hipMemcpyAsync(q, dv.get() + n, sizeof(double) * n, hipMemcpyDeviceToHost, st));
        BFM_HIP(hipStreamSynchronize(st));
    });
}

// ---------------------------------------------------------------------------
// Test hooks (include/bfm_debug.h)

int bfm_debug_dgemm(int device, int M, int N, int K, const double *A, const double *B, double *C) {
    return guarded([&] {
        BFM_CHECK(A && B && C, BFM_EINVAL, "null argument");
        BFM_CHECK(M >= 1 && N >= 1 && K >= 1 && (int64_t)M * N <= (1 << 26) && (int64_t)M * K <= (1 << 26) &&
                      (int64_t)K * N <= (1 << 26),
                  BFM_EINVAL, "sizes out of range");
        DeviceScope ds(device);
        DevBuf<double> a, b, c;
        a.ensure((size_t)M * K);
        b.ensure((size_t)K * N);
        c.ensure((size_t)M * N);
        BFM_HIP(hipMemcpy(a.get(), A, sizeof(double) * M * K, hipMemcpyHostToDevice));
        BFM_HIP(hipMemcpy(b.get(), B, sizeof(double) * K * N, hipMemcpyHostToDevice));
        gemm_nn_f64(M, N, K, a.get(), M, b.get(), K, c.get(), M, nullptr);
        BFM_HIP(hipDeviceSynchronize());
        BFM_HIP(hipMemcpy(C, c.get(), sizeof(double) * M * N, hipMemcpyDeviceToHost));
    });
}

int bfm_debug_spd_inverse(int device, int n, const double *A, double *Ainv) {
    return guarded([&] {
        BFM_CHECK(A && Ainv, BFM_EINVAL, "null argument");
        BFM_CHECK(n >= 1 && n <= 8192, BFM_EINVAL, "n out of range");
        DeviceScope ds(device);
        DevBuf<double> a, piv, row, col;
        a.ensure((size_t)n * n);
        BFM_HIP(hipMemcpy(a.get(), A, sizeof(double) * n * n, hipMemcpyHostToDevice));
        spd_inverse(a.get(), n, piv, row, col, nullptr);
        BFM_HIP(hipDeviceSynchronize());
        BFM_HIP(hipMemcpy(Ainv, a.get(), sizeof(double) * n * n, hipMemcpyDeviceToHost));
    });
}

int bfm_debug_probe(int device, int kind, int iters, double *ms, double *ops) {
    return guarded([&] {
        BFM_CHECK(ms && ops, BFM_EINVAL, "null argument");
        DeviceScope ds(device);
        probe_run(kind, iters, ms, ops);
    });
}

// ---------------------------------------------------------------------------
// Time-step harness (include/bfm_step.h)

int bfm_default_physics(bfm_physics *ph) {
    if (!ph) return BFM_EINVAL;
    std::memset(ph, 0, sizeof(*ph));
    ph->rho = 1.0;
    ph->p0 = 1.0;
    ph->sigma = 0.0;
    ph->kappa = 1.4;
    ph->forcing_sign = -1.0;
    ph->alpha = -1.0;
    ph->guess = BFM_GUESS_GIVEN;
    return BFM_OK;
}

int bfm_set_physics(bfm_ctx *c, const bfm_physics *ph) {
    return guarded([&] {
        BFM_CHECK(c && ph, BFM_EINVAL, "null argument");
        DeviceScope ds(c->device);
        step_set_physics(c, *ph);
    });
}

int bfm_state_set(bfm_ctx *c, const double *xyz, const double *phi, double t) {
    return guarded([&] {
        BFM_CHECK(c && xyz && phi, BFM_EINVAL, "null argument");
        DeviceScope ds(c->device);
        step_state_set(c, xyz, phi, t);
    });
}

int bfm_state_get(bfm_ctx *c, double *xyz, double *phi, double *t) {
    return guarded([&] {
        BFM_CHECK(c, BFM_EINVAL, "null argument");
        DeviceScope ds(c->device);
        step_state_get(c, xyz, phi, t);
    });
}

int bfm_step(bfm_ctx *c, double dt, bfm_step_info *info) {
    return guarded([&] {
        BFM_CHECK(c, BFM_EINVAL, "null argument");
        DeviceScope ds(c->device);
        step_advance(c, dt, info);
    });
}

int bfm_rhs(bfm_ctx *c, double t, const double *xyz, const double *phi, double *dxyz, double *dphi, double *q,
            double *H) {
    return guarded([&] {
        BFM_CHECK(c && xyz && phi, BFM_EINVAL, "null argument");
        DeviceScope ds(c->device);
        step_rhs(c, t, xyz, phi, dxyz, dphi, q, H);
    });
}

int bfm_autotune(bfm_ctx *c, double mvp_tol, bfm_tune_result *out) {
    return guarded([&] {
        BFM_CHECK(c, BFM_EINVAL, "null argument");
        BFM_CHECK(c->nv > 0, BFM_EINVAL, "no mesh set");
        BFM_CHECK(mvp_tol > 0.0, BFM_EINVAL, "mvp_tol must be positive");
        DeviceScope ds(c->device);
        bfm_tune_result r{};
        autotune(c, mvp_tol, &r);
        if (out) *out = r;
    });
}

}  // extern "C"
