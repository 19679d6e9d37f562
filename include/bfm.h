/*
 * bfm.h - C ABI of the MI355X fast-multipole boundary-element library.
 *
 * The library solves the discrete boundary integral equation of a cluster
 * of gas bubbles in potential flow (Gumerov, Pityuk, Abramova, Akhatov,
 * "GPU accelerated fast multipole boundary element method for simulation
 * of 3D bubble dynamics in potential flow"): given the surface mesh and the
 * potential phi at every vertex, it returns q = dphi/dn at every vertex.
 *
 *   Problem (Section 2.2, eq2_11 - eq2_13):  L[q] - M[phi] = -phi/2 on S,
 *     G = 1/(4 pi |r - r'|),  dG/dn' = n'.(r - r')/(4 pi |r - r'|^3),
 *     n' points out of the bubble into the liquid.
 *   Discretisation (Section 3.1, eq3_1/eq3_2): vertex collocation,
 *     L q = b,  b = -phi/2 + M phi.
 *   Non-singular entries (Section 3.2, ns1): L_ij = s_j G(r_i, r_j),
 *     M_ij = s_j dG/dn_j(r_i, r_j), i != j; s_j = (1/3) sum of the areas of
 *     the triangles at j, n_j = normalised area-weighted triangle normal.
 *   Singular diagonals (Section 3.3, s3 and s5): M_ii = -1/2 - sum_{j!=i}
 *     M_ij;  L_ii = n_i . [sum_{j!=i}(M_ij r_j - L_ij n_j) + (1/2 + M_ii) r_i].
 *   Products with L and M (Section 3.9, eq3_27) use the fast multipole
 *     method over an octree (scaled to a cube, empty boxes skipped);
 *     the system is solved by restarted GMRES (Section 3.8).
 *
 * Conventions for every entry point:
 *   - Return value: BFM_OK (0) or a negative BFM_E* code; the message of
 *     the last failure on the calling thread is bfm_last_error().
 *   - Host pointers ("host" below) are read or written before the call
 *     returns and never retained. Device pointers ("_dev" entry points)
 *     must be HBM allocations on the handle's device, valid until the
 *     handle's stream has been synchronised; the _dev entry points are
 *     ordered on the handle's stream and do not synchronise it unless
 *     stated.
 *   - A handle is not thread-safe; separate handles are independent.
 *   - Arrays of vertices are indexed in the caller's vertex order.
 */
#ifndef BFM_H
#define BFM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BFM_ABI_VERSION 6

enum {
    BFM_OK = 0,
    BFM_EINVAL = -1,      /* invalid argument or option */
    BFM_ENOMEM = -2,      /* device or host allocation failed */
    BFM_EDEVICE = -3,     /* a HIP call failed */
    BFM_ENOCONV = -4,     /* GMRES hit its iteration limit; q holds the best iterate */
    BFM_EMESH = -5,       /* degenerate mesh: zero-area triangle, zero normal, index out of range */
    BFM_EUNSUPPORTED = -6 /* option combination not built */
};

/* Preconditioner of the GMRES iteration. */
enum {
    BFM_PRECOND_NONE = 0, /* unpreconditioned GMRES, as in the paper (Section 3.8) */
    BFM_PRECOND_SH = 1,   /* per-bubble spherical-harmonic approximate inverse (needs
                             bfm_set_sphere_template), applied from the right */
    BFM_PRECOND_SH_COARSE = 2 /* two-level: BFM_PRECOND_SH followed by a coarse correction in
                                 the space of per-bubble constants (one unknown per bubble,
                                 interactions between bubbles as point monopoles) */
};

/* Initial guess of bfm_solve / bfm_solve_dev (argument use_guess). */
enum {
    BFM_GUESS_ZERO = 0,    /* q = 0 */
    BFM_GUESS_GIVEN = 1,   /* q as passed in (e.g. the previous time step's, Section 3.6) */
    BFM_GUESS_LEARNED = 2  /* predicted by the trained network of bfm_mlp.h from the current
                              surface and phi; needs bfm_set_sphere_template */
};

/* Arithmetic of a fast multipole product (the paper compares single- and
 * double-precision products, Section 3.11, Table 1). The low-precision
 * modes compute the near field in FP32 with coordinates relative to the
 * receiver's leaf centre (sums added into FP64), the leaf expansions (P2M,
 * L2P) in FP32, and the translations on the matrix cores with FP32
 * expansions; the result vector stays FP64. Low-precision products carry one
 * channel (the single or the double layer). */
enum {
    BFM_PREC_FP64 = 0,  /* FP64 everywhere (FP64 VALU near field, FP64 MFMA translations) */
    BFM_PREC_FP32 = 1,  /* FP32 translations (v_mfma_f32_16x16x4f32) */
    BFM_PREC_BF16X3 = 2 /* split-BF16 translations: operator and input split as a = hi + lo
                           (hi = bf16(a), lo = bf16(a - hi), round to nearest even), three
                           products hi*hi + hi*lo + lo*hi (v_mfma_f32_16x16x32_bf16), FP32
                           accumulation */
};

typedef struct bfm_options {
    int abi_version;   /* must be BFM_ABI_VERSION */
    int device;        /* HIP device ordinal */
    void *stream;      /* hipStream_t to run on; NULL = the library creates one */
    int p;             /* expansion degrees 0..p-1 (p^2 coefficients) of the products inside
                          GMRES; multiple of 4, 4..20 */
    int p_diag;        /* expansion degrees of the once-per-solve pass for the singular
                          diagonals and b; 0 = min(20, p + 4) */
    int lmax;          /* octree depth; 0 = choose from leaf_target */
    int leaf_target;   /* mean points per non-empty leaf aimed at when lmax = 0 */
    int precision;     /* BFM_PREC_* of the products inside GMRES. FP64: plain restarted
                          GMRES. FP32 or BF16X3: mixed-precision iterative refinement -
                          each restart cycle is one refinement step: its Arnoldi process
                          uses low-precision products of order p_lo, and it ends once its
                          residual estimate has fallen by ir_tol (or at gmres_restart
                          iterations); the correction is added in FP64 and the true
                          residual b - L q is formed with an FP64 product of order p */
    int p_lo;          /* expansion order of the low-precision products (multiple of 4,
                          4..20); 0 = p */
    double ir_tol;     /* relative residual reduction that ends a refinement cycle; 0 = 1e-4 */
    double gmres_tol;  /* stop when ||b - L q||_2 <= gmres_tol ||b||_2 */
    int gmres_restart; /* Krylov dimension before restart (1..128) */
    int gmres_maxit;   /* total iteration limit */
    int precond;       /* BFM_PRECOND_* */
    int precond_degree; /* highest harmonic degree resolved by BFM_PRECOND_SH, (d+1)^2 <= nd */
    int use_graph;     /* != 0: GMRES replays each product (preconditioner + fast multipole
                          product) from one captured HIP graph per octree */
    int m2l_shape;     /* M2L launch shape: -1 = by size, 0 = wide tiles, 1 = row slabs,
                          2 = narrow slabs (dense p^2 x p^2 operators), 3 = rotation-factored
                          M2L (rotate the multipole to the offset's axis, translate along it,
                          rotate back: 4 p^3 instead of 2 p^4 flops per translation, FP64
                          products only; the diagonal/right-hand-side pass follows it); set
                          by bfm_autotune */
    int m2l_orders;    /* 0: every M2L translation at the product's order p (Section 3.9);
                          1: offsets d = (c_target - c_source)/h (box sides) translated at
                          orders falling with |d|: p for |d|^2 <= 5, 4 ceil(p/5) for 6..10,
                          4 ceil(3p/20) from 11 on (20/16/12 at p = 20, 16/16/12 at
                          p = 16) - the truncation error of a translation falls
                          geometrically with |d|, so distant offsets reach the nearest
                          ones' accuracy at lower order. Applies to every product */
    int p2p_shape;     /* work items of the symmetric one-channel near field (receivers per
                          chunk, sources per piece of the chunk's own block, per piece of the
                          rest): -1 or 0 = (256, 128, 192), 1 = (128, 128, 128), 2 = (256, 128,
                          384); set by bfm_autotune */
    int near_corr;     /* != 0: add near-field correction matrices to every product, the
                          singular diagonals and b (Section 3.9): for each collocation point
                          i the triangles touching i or its mesh neighbours are integrated
                          with a conical 8 x 8 Gauss rule (collapsed at the vertex nearest
                          r_i, exact for the weakly singular self term) and the nodal rule's
                          share of them is taken out; one sparse row per vertex (about 18
                          columns on a regular mesh), values rebuilt with the geometry,
                          pattern with the mesh. 0 = the nodal rule alone */
} bfm_options;

typedef struct bfm_solve_info {
    int iterations;      /* GMRES iterations (one product with L each) */
    int restarts;        /* completed restart cycles */
    int matvecs;         /* products with L, including explicit residuals */
    int converged;       /* 1 if the tolerance was met */
    double rel_residual; /* final ||b - L q|| / ||b|| (true residual at exit) */
    double t_tree_ms;    /* geometry + octree build */
    double t_diag_ms;    /* singular diagonals + right-hand side pass */
    double t_solve_ms;   /* GMRES */
    double t_guess_ms;   /* learned initial guess (BFM_GUESS_LEARNED), else 0 */
} bfm_solve_info;

typedef struct bfm_ctx bfm_ctx;

/* Fill *opt with defaults: p = 16, p_diag = 0, lmax = 0, leaf_target = 64,
 * FP64 (p_lo = 0, ir_tol = 0), tol 1e-10, restart 30, maxit 300, device 0,
 * stream NULL, no preconditioner (precond_degree 12), no graph, M2L shape
 * by size, every M2L at order p (m2l_orders = 0). */
int bfm_default_options(bfm_options *opt);

/* Create a handle on opt->device. The handle owns every device buffer
 * (mesh, octree, expansions, translation operators, Krylov basis). */
int bfm_create(const bfm_options *opt, bfm_ctx **out);
int bfm_destroy(bfm_ctx *ctx);

/* Replace the options of an existing handle (same device and stream).
 * Changing p rebuilds the translation operators; changing lmax or
 * leaf_target rebuilds the octree at the next call that needs it. */
int bfm_set_options(bfm_ctx *ctx, const bfm_options *opt);

/*
 * Set the surface mesh (Section 3.1): nv vertices xyz (host, [nv][3]
 * row-major, FP64), nt triangles tri (host, [nt][3] int32 vertex indices,
 * ordered r1 -> r2 -> r3 so that (r2 - r1) x (r3 - r1) points into the
 * liquid). nb bubbles own contiguous vertex ranges vtx_off[b]..vtx_off[b+1]
 * and triangle ranges tri_off[b]..tri_off[b+1] (host, int64 [nb + 1]; may
 * be NULL when nb <= 1). Copies everything; connectivity is kept until the
 * next bfm_set_mesh, positions until bfm_set_positions*.
 * Errors: BFM_EINVAL (nv < 4, nt < 4, bad ranges), BFM_EMESH (index out of
 * range, a vertex in no triangle).
 */
int bfm_set_mesh(bfm_ctx *ctx, int64_t nv, const double *xyz, int64_t nt, const int32_t *tri,
                 int32_t nb, const int64_t *vtx_off, const int64_t *tri_off);

/*
 * Spherical-harmonic template for BFM_PRECOND_SH: every bubble has nd
 * vertices numbered like a template unit sphere whose vertex directions are
 * dirs (host, [nd][3], unit vectors) - the parametrisation by the initial
 * spherical angles that the paper's shape filter uses (Section 3.7). The
 * first bubble's triangles give the template's connectivity. The
 * preconditioner scales harmonics of degree n on bubble b by (2n+1)/R_b, the
 * inverse of the single layer's eigenvalue R/(2n+1) on a sphere (R_b from
 * the bubble's area), and degrees above precond_degree by the first
 * unresolved one. Errors: BFM_EINVAL when a bubble range does not hold nd
 * vertices or the mesh has not been set.
 */
int bfm_set_sphere_template(bfm_ctx *ctx, int32_t nd, const double *dirs);

/*
 * Torus template for toroidal (genus-1) bubbles (Section 3.7: the shape
 * filter of a torus-like bubble uses the 2D Fourier basis e^{i(n theta +
 * m phi)} of the angles that place each vertex on a unit torus): every
 * bubble has nd vertices numbered like the template, whose angles are
 * angles (host, [nd][2]: theta around the tube, phi around the axis, in
 * radians). It replaces a sphere template; the time-step harness then
 * filters with the real trigonometric basis of degree <= filter_degree / 2
 * in each angle. The solve itself does not depend on the genus; the
 * harmonic preconditioners and the learned guess need a sphere template and
 * fail with BFM_EINVAL under this one. Errors: BFM_EINVAL when a bubble
 * range does not hold nd vertices, an angle is not finite or the mesh has
 * not been set.
 */
int bfm_set_torus_template(bfm_ctx *ctx, int32_t nd, const double *angles);

/* Move the vertices (same connectivity): xyz host [nv][3] or device
 * (_dev, FP64 [nv][3]). Geometry and octree are rebuilt at the next use. */
int bfm_set_positions(bfm_ctx *ctx, const double *xyz);
int bfm_set_positions_dev(bfm_ctx *ctx, const double *xyz_dev);

/* Vertex weights s_j and unit normals n_j of ns1 (Section 3.2): host
 * outputs s [nv], n [nv][3]. Errors: BFM_EMESH on a zero-area triangle or
 * a vertex whose area-weighted normal vanishes. */
int bfm_geometry(bfm_ctx *ctx, double *s, double *n);

/*
 * Singular diagonals and right-hand side (Section 3.3 s3/s5, eq3_1) by one
 * five-channel fast multipole pass at the handle's p_diag, in FP64:
 *   Mii[i] = -1/2 - sum_{j!=i} M_ij
 *   Lii[i] = n_i . [sum_{j!=i} M_ij (r_j - r_i) - sum_{j!=i} L_ij n_j]
 *   b[i]   = -phi_i/2 + Mii[i] phi_i + sum_{j!=i} M_ij phi_j
 * phi host [nv]; outputs host [nv] (any may be NULL except phi).
 */
int bfm_diagonals(bfm_ctx *ctx, const double *phi, double *Mii, double *Lii, double *b);

/*
 * Product with A = f L + g M (eq3_27) by the fast multipole method:
 *   out_i = sum_{j != i} (f L_ij x_j + g M_ij y_j) [+ f L_ii x_i + g M_ii y_i if add_diag]
 * x, y, out host [nv] (x may be NULL if f == 0, y if g == 0). precision
 * selects BFM_PREC_*; an FP64 product uses the handle's p, a low-precision
 * one its p_lo (p when 0). add_diag needs the
 * diagonals of the current mesh (computed on demand, at p_diag). direct = 1 replaces the fast multipole method by
 * the all-pairs sum on the GPU (FP64), for checking.
 */
int bfm_matvec(bfm_ctx *ctx, double f, const double *x, double g, const double *y, double *out,
               int add_diag, int precision, int direct);

/*
 * Solve L q = b for q = dphi/dn (eq3_2): geometry, octree, diagonals and
 * right-hand side, then restarted GMRES from the initial guess.
 *   phi  host [nv] (bfm_solve) or device FP64 [nv] (bfm_solve_dev)
 *   q    in: the initial guess if use_guess == BFM_GUESS_GIVEN, else ignored
 *        (BFM_GUESS_ZERO: zero; BFM_GUESS_LEARNED: the network's prediction);
 *        out: the solution. Host [nv] or device [nv] respectively.
 *   info may be NULL.
 * Returns BFM_ENOCONV (q = last iterate, info filled) when gmres_maxit is
 * reached first. bfm_solve_dev synchronises the stream before returning.
 */
int bfm_solve(bfm_ctx *ctx, const double *phi, double *q, int use_guess, bfm_solve_info *info);
int bfm_solve_dev(bfm_ctx *ctx, const double *phi_dev, double *q_dev, int use_guess,
                  bfm_solve_info *info);

/*
 * Direct (all-pairs) off-diagonal product on device arrays, without a
 * handle (Section 3.2, ns1; kernels of eq2_13):
 *   out[k] = sum_{j != i} s_j [ f x_j G(r_i, r_j) + g y_j dG/dn_j(r_i, r_j) ],
 *   G = 1/(4 pi |r_i - r_j|),  dG/dn_j = n_j . (r_i - r_j) / (4 pi |r_i - r_j|^3),
 *   i = rows[k] for k < nr (rows == NULL: i = k, nr <= n).
 * All arrays are FP64 device memory on the calling thread's current HIP
 * device, caller-owned: xyz [n][3] and nrm [n][3] row-major, s [n], x [n]
 * (read when f != 0), y and nrm (read when g != 0), rows int64 [nr], out
 * [nr]. Runs on `stream` (hipStream_t; NULL = the null stream) and returns
 * without synchronising; the pointers must stay valid until the stream has
 * passed the call. j == i is excluded by index (coincident distinct points
 * are an invalid mesh). A row index outside [0, n) gives NaN in its out
 * entry. The library allocates a partial-sum buffer of
 * (source splits x nr) doubles per call, stream-ordered.
 * Errors: BFM_EINVAL (n < 1, nr < 0, a null pointer that is needed),
 * BFM_ENOMEM, BFM_EDEVICE.
 */
int bfm_direct_dev(int64_t n, const double *xyz, const double *s, const double *nrm, double f, const double *x,
                   double g, const double *y, int64_t nr, const int64_t *rows, double *out, void *stream);

/*
 * bfm_direct_dev without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same arguments, kernels and result
 * as bfm_direct_dev, with the partial sums in a fixed device array of the
 * library (4,194,304 doubles = 32 MiB per device, held until the process
 * ends). It calls no hipMalloc, hipFree or allocating library routine.
 * Limit: (source splits x nr) <= 4,194,304, which holds for every nr up to
 * 4,063,232 receivers; a larger nr returns BFM_EINVAL before any launch.
 * Every call on one device shares that device's array: calls that overlap
 * on one device (other streams or threads) race and must be ordered by the
 * caller. Nothing in the array needs clearing (each call writes every
 * partial it reads). Errors as bfm_direct_dev.
 */
int bfm_direct_dev_noalloc(int64_t n, const double *xyz, const double *s, const double *nrm, double f,
                           const double *x, double g, const double *y, int64_t nr, const int64_t *rows, double *out,
                           void *stream);

/* Autotuning of the fast multipole product for the current mesh (not in the
 * paper, which tunes the octree depth by hand, Section 4): p = the smallest
 * of 8, 12, 16, 20 whose product with a fixed pseudo-random vector is within
 * mvp_tol (relative 2-norm) of the p = 20 product (p = 20 if none); with
 * iterative refinement (precision FP32 or BF16X3) also p_lo = the smallest
 * of 8, 12, 16 whose low-precision product is within ir_tol of that
 * reference; when p_diag is 0, p_diag = the smallest of 12, 16 (not below
 * p) whose diagonal pass is within 10 mvp_tol of the pass at order 20 (L_ii
 * in relative 2-norm, M_ii in largest difference over 1/2), else 20; then
 * the octree depth (the depth chosen from leaf_target and two levels
 * either side) that minimises one diagonal/right-hand-side pass plus the
 * products of a typical solve (ten FP64 products, or two FP64 and eight
 * low-precision ones), and the M2L launch shape (dense shapes 0..2 and the
 * rotation-factored 3) with the fastest product at that depth, and the
 * near-field work item shape (p2p_shape 0..2) with the fastest near field
 * of the products GMRES runs most (the low-precision ones under
 * refinement), timed with HIP events after a warm-up. The choice is stored
 * in the handle's options (p, p_lo, p_diag, lmax, m2l_shape, p2p_shape).
 * out may be NULL. */
typedef struct bfm_tune_result {
    int p, lmax, m2l_shape; /* chosen */
    int candidates;         /* configurations timed */
    double mvp_ms;          /* time of one FP64 product with the chosen configuration */
    double p_err;           /* relative difference of the chosen p's product from p = 20 */
    int p_lo;               /* chosen order of the low-precision products (0 without refinement) */
    int p_diag;             /* order of the diagonal/right-hand-side pass (as set, or chosen) */
    double diag_err;        /* the chosen p_diag's difference from order 20 (0 if 20 or set) */
    int p2p_shape;          /* chosen near-field work item shape (bfm_options.p2p_shape) */
} bfm_tune_result;
int bfm_autotune(bfm_ctx *ctx, double mvp_tol, bfm_tune_result *out);

/* Octree statistics of the current mesh (builds the tree if needed), the
 * first n of: stats[0] = lmax, [1] = leaves, [2] = boxes (all levels),
 * [3] = near-field pairs, [4] = M2L pairs, [5] = M2M+L2L pairs, [6] = max
 * points per leaf, [7] = launch shape (0..3 as bfm_options.m2l_shape) of
 * the last M2L launch of an FP64 GMRES product, [8] = the same for the
 * diagonal/right-hand-side pass (-1 before the first launch); entries past
 * BFM_TREE_STATS are set to 0. stats is a host array of n entries. */
#define BFM_TREE_STATS 9
int bfm_tree_stats(bfm_ctx *ctx, int n, int64_t *stats);

/*
 * Kernel timing (measurement support). The five kernels of a fast multipole
 * product are counted per product group, the group's P2P first:
 *   0..4   FP64 products of GMRES: 0 near-field P2P, 1 M2L, 2 M2M + L2L,
 *          3 P2M, 4 L2P
 *   5      GMRES vector kernels,  6 octree build (whole),
 *   7      diagonal/right-hand-side pass (whole)
 *   8..12  the diagonal/right-hand-side pass's P2P, M2L, M2M + L2L, P2M, L2P
 *   13..17 low-precision products (iterative refinement), same order
 * bfm_profile(ctx, 1) clears and starts recording HIP events around every
 * launch of these classes on the stream it is launched on; while recording,
 * the near field runs in line on the handle's stream (not beside the far
 * field) so that each kernel's events measure it alone, and GMRES does not
 * replay graphs. bfm_profile(ctx, 0) stops. bfm_profile_read synchronises
 * and returns, for the first nclass classes (host arrays of nclass entries),
 * the summed event time in ms, the number of launches and the summed
 * algorithmic work of those launches (flops for the product kernels:
 * near-field pairs x flops per pair, 2 p^4 per translated expansion column;
 * 0 for P2M, L2P and classes 5..7).
 */
#define BFM_KERNEL_CLASSES 18
int bfm_profile(bfm_ctx *ctx, int enable);
int bfm_profile_read(bfm_ctx *ctx, int nclass, double *ms, int64_t *launches, double *flops);

/* Message of the last failure on this thread ("" if none). */
const char *bfm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BFM_H */
