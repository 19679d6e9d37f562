// Library handle and the solve pipeline.
#pragma once

#include <vector>

#include "../../include/bfm_step.h"
#include "common.h"
#include "fmm.h"
#include "prof.h"
#include "tree.h"

namespace bfm {
// Real spherical harmonics of degree <= nmax sampled at the template
// vertices (G, column-major [nd x nc]) and their weighted least-squares
// projector (Gp, column-major [nc x nd]).
struct ShBasis {
    int nmax = -1, nc = 0, nd = 0, weighted = 1;
    int genus = 0;     // 0: spherical harmonics of degree <= nmax; 1: trigonometric, degree <= nmax per angle
    uint64_t gen = 0;  // template generation the basis was built for
    DevBuf<double> G, Gp;
};
struct Precond {
    int nd = 0, nc = 0, nmax = -1;
    uint64_t gen = 1;  // bumped whenever the template changes (invalidates every ShBasis)
    double cc = 0.0;
    bool ready = false;
    int genus = 0;               // 0: sphere template (dirs_h), 1: torus template (ang_h)
    std::vector<double> dirs_h;  // template directions [nd][3]
    std::vector<double> ang_h;   // template torus angles (theta around the tube, phi around the axis) [nd][2]
    std::vector<int> tri_h;      // template triangles (first bubble, local indices)
    ShBasis basis;
    DevBuf<double> fac, R, X, C, Y;
    DevBuf<double> gws;                // split-K partial products of the GEMMs
    // coarse space of per-bubble constants (two-level form)
    DevBuf<double> U;                  // own-bubble column sums of s^T L, caller order [nv]
    DevBuf<double> ccen, carea;        // area-weighted centroids [nb][3], areas [nb]
    DevBuf<double> cusum;              // bubble sums of U [nb] (the coarse matrix's diagonal)
    DevBuf<double> Ainv, gj_row, gj_col, gj_piv;  // inverse coarse matrix [nb x nb] and Gauss-Jordan work
    DevBuf<double> csum, cy;           // per-bubble sums [3][nb], coarse correction [nb]
};
// Near-field correction matrices (corr.hip). Pattern, original order: per
// vertex i the near triangles tv[tptr[i]..tptr[i+1]) as (v0, v1, v2, the
// row slots of the three packed in bytes, 255 for i itself) and the
// columns col[rptr[i]..rptr[i+1]) (j != i ascending). Values, per octree
// in sorted order, ELL layout of width w (entry k of sorted row r at
// k * nv + r): sorted column in ecol (padding: the row itself with zero
// values)
struct NearCorr {
    DevBuf<int> tptr, tv, rptr, col;  // tv: 4 ints per entry
    DevBuf<int> ecol;
    DevBuf<double> ecl, ecm;
    int64_t nnz = 0;
    int w = 0;
    bool pattern = false;  // tptr/tv/rptr/col current for the mesh
    bool values = false;   // ecol/ecl/ecm current for the geometry and the octree's order
};
struct Mlp;      // learned initial guess (learn.hip)
struct CoarseWorker;  // host thread queueing the coarse build (precond.hip)
struct Stepper;

// time-step harness (step.hip)
}  // namespace bfm

struct bfm_ctx {
    bfm_options opt{};
    int device = 0;
    hipStream_t stream = nullptr;
    // second stream (default priority) for the coarse-space build, which runs
    // beside the diagonal pass; ev_geom orders it after the geometry,
    // ev_coarse orders GMRES after it
    hipStream_t side = nullptr;
    hipEvent_t ev_geom = nullptr, ev_coarse = nullptr;
    bool coarse_pending = false;  // a coarse build for the current geometry is in flight on `side`
    bfm::CoarseWorker *coarse_worker = nullptr;  // host thread that queues the coarse build
    bool coarse_marked = false;   // ev_geom marks the geometry a coarse build will read
    hipStream_t near = nullptr;   // near-field stream of both fast multipole products (default priority)
    bool own_stream = false;

    // mesh (original vertex order)
    int64_t nv = 0, nt = 0;
    int32_t nb = 0;
    std::vector<int64_t> vtx_off, tri_off;
    bfm::DevBuf<double> xyz;      // [nv][3]
    bfm::DevBuf<int> tri;         // [nt][3]
    bfm::DevBuf<int> v2t_off, v2t;  // vertex -> incident triangles (ascending)

    // geometry (original order): s [nv], normals SoA [3][nv]
    bfm::DevBuf<double> s, nrm;
    bfm::DevBuf<double> tri_rec;  // per triangle (half cross product x, y, z, area) [nt][4]
    bfm::DevBuf<int> flag;
    int *host_flag = nullptr;     // pinned copy of the geometry checks
    bool geom_valid = false;
    bool geom_unchecked = false;  // geometry rebuilt, its checks not yet read

    bfm::Tree tree;
    bool tree_valid = false;

    bfm::Prof prof;
    bfm::FmmWork fmm;       // FP64 products inside GMRES (order p)
    bfm::FmmWork fmm_diag;  // diagonal + right-hand-side pass (order p_diag)
    bfm::FmmWork fmm_lo;    // low-precision products (order p_lo; iterative refinement)

    // sorted-order solve data
    bfm::DevBuf<double> src_q, src_w;  // channel monopole strengths, dipole weights
    bfm::DevBuf<double> src_pk;        // packed five-channel near-field records [n][kDiagRec]
    bfm::DevBuf<double> ysum;           // channel sums
    bfm::DevBuf<double> mii_s, lii_s, b_s, phi_s;
    bool diag_valid = false;            // mii_s / lii_s current for the mesh
    bfm::NearCorr corr;                 // near-field corrections (opt.near_corr)

    bfm::Precond pre;
    std::vector<int> tri0_h;  // first bubble's triangles (local indices), kept for templates

    bfm::Mlp *mlp = nullptr;          // learned initial guess, created on first use
    bfm::Stepper *stepper = nullptr;  // time-step harness, created on first use
    std::vector<int> tri_h;           // triangles (host copy, for the harness's one-rings)

    // captured product of the GMRES iteration (use_graph): preconditioner and
    // fast multipole product from gin to gout, valid for one octree
    hipGraphExec_t mvp_graph = nullptr;
    int mvp_graph_pc = -1;                 // preconditioner the graph was captured with
    // an invalidated graph, destroyed later at a point where the stream has
    // just been waited for (its destruction waits for the device, and in the
    // octree build that wait would take in the coarse build beside it)
    hipGraphExec_t mvp_graph_stale = nullptr;
    int mvp_graph_stale_pc = -1;
    bfm::DevBuf<double> gin, gout;

    // GMRES workspace (sorted order)
    bfm::DevBuf<double> V, work, x_s, part, small, zbuf, tbuf;
    double *host_small = nullptr;       // pinned
};

namespace bfm {

void ensure_geometry(bfm_ctx *c, bool check_now = true);
// read the checks of the last geometry build; synced: the stream has been
// waited for since the build (else this waits)
void geometry_check(bfm_ctx *c, bool synced = false);
void ensure_tree(bfm_ctx *c);
void ensure_ops(bfm_ctx *c);
// operators of the low-precision product group for precision prec (FP32 or BF16X3)
void ensure_ops_lo(bfm_ctx *c, int prec);
int diag_order(const bfm_options &o);

// Five-channel pass: M_ii, L_ii (sorted) and, if phi_dev != null, b (sorted).
// phi_dev in original order.
void diagonal_pass(bfm_ctx *c, const double *phi_dev);

// out_s = f L x_s + g M y_s (+ diag) in sorted order; x_s, y_s sorted.
void matvec_sorted(bfm_ctx *c, double f, const double *x_s, double g, const double *y_s,
                   double *out_s, bool add_diag, int precision, bool direct);

// GMRES in sorted order: solves L x = b_s, x_s in/out.
void gmres_sorted(bfm_ctx *c, double *x_s, bool use_guess, bfm_solve_info *info);

// Near-field correction matrices (corr.hip); every call is a no-op unless
// opt.near_corr. corr_invalidate drops the values (and with mesh the
// pattern); ensure_corr builds what is missing; corr_apply adds
// f CL x_s + g CM y_s to out_s; corr_diagonals corrects mii_s, lii_s and,
// with phi_s non-null, b_s (all sorted)
void corr_invalidate(bfm_ctx *c, bool mesh);
void ensure_corr(bfm_ctx *c);
void corr_apply(bfm_ctx *c, double f, const double *x_s, double g, const double *y_s, double *out_s);
void corr_diagonals(bfm_ctx *c, const double *phi_s);

// Spherical-harmonic preconditioner (precond.hip)
// weighted: G+ = (G^T W G)^{-1} G^T W with W the template vertex areas; else plain least squares
void sh_basis_build(const Precond &P, int nmax, ShBasis &B, hipStream_t st, bool weighted = true);
// torus template: plain least squares onto the real trigonometric basis of
// degree <= h in each angle ((2h + 1)^2 functions)
void torus_basis_build(const Precond &P, int h, ShBasis &B, hipStream_t st);
void precond_build(bfm_ctx *c);
void precond_radii(bfm_ctx *c);
void precond_apply(bfm_ctx *c, const double *in_s, double *out_s);
// coarse correction of the two-level form on stream st (geometry of the
// current mesh only)
void coarse_build(bfm_ctx *c, hipStream_t st);
// coarse_mark records the point on the main stream after which the geometry
// is ready; coarse_launch then queues coarse_build on the side stream from
// that point (marking now if nothing is marked); GMRES waits for it
void coarse_mark(bfm_ctx *c);
void coarse_launch(bfm_ctx *c);
// order the main stream after a coarse build in flight (no-op if none)
void coarse_join(bfm_ctx *c);
// stop the handle's coarse-build thread (after the build it queued)
void coarse_worker_free(bfm_ctx *c);
// in-place inverse of an SPD n x n column-major device matrix (blocked Gauss-Jordan)
void spd_inverse(double *A, int n, DevBuf<double> &piv, DevBuf<double> &row, DevBuf<double> &col,
                 hipStream_t st);
// C = A B, column-major FP64 (precond.hip)
void gemm_nn_f64(int M, int N, int K, const double *A, int lda, const double *B, int ldb, double *C, int ldc,
                 hipStream_t st);
// C = rowscale o (A B) + beta D (rowscale, D may be null; C may alias D);
// ws non-null allows a split of K (partial products kept in ws)
void gemm_f64(int M, int N, int K, const double *A, int lda, const double *B, int ldb, double *C, int ldc,
              const double *rowscale, double beta, const double *D, int ldd, DevBuf<double> *ws, hipStream_t st);

// the solve of bfm_solve_dev: tree, diagonals and b, optional guess, GMRES
// (guess: BFM_GUESS_*); throws BFM_ENOCONV when GMRES stops at gmres_maxit
void solve_impl(bfm_ctx *c, const double *phi_dev, double *q_dev, int guess, bfm_solve_info *info);

// captured product (tune.hip)
void graph_invalidate(bfm_ctx *c);
// destroys an invalidated graph (call where the stream has just been waited for)
void graph_release_stale(bfm_ctx *c);
// out_s = A P^{-1} in_s (pc) or A in_s through the captured graph; captures on first use
void graph_mvp(bfm_ctx *c, const double *in_s, double *out_s, bool pc);
void autotune(bfm_ctx *c, double mvp_tol, bfm_tune_result *out);

// time-step harness (step.hip)
void step_free(bfm_ctx *c);

// ceiling probe (probe.hip): one timed launch of instruction mix `kind`
void probe_run(int kind, int iters, double *ms, double *ops);
void step_mesh_changed(bfm_ctx *c);
void step_set_physics(bfm_ctx *c, const bfm_physics &ph);
void step_state_set(bfm_ctx *c, const double *xyz_h, const double *phi_h, double t);
void step_state_get(bfm_ctx *c, double *xyz_h, double *phi_h, double *t);
void step_advance(bfm_ctx *c, double dt, bfm_step_info *info);
void step_rhs(bfm_ctx *c, double t, const double *xyz_h, const double *phi_h, double *dxyz, double *dphi, double *q,
              double *H);

// gather (original -> sorted) and scatter (sorted -> original)
void to_sorted(bfm_ctx *c, const double *in_orig, double *out_s);
void to_original(bfm_ctx *c, const double *in_s, double *out_orig);

}  // namespace bfm
