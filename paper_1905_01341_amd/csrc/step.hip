// Time-step harness (include/bfm_step.h): the right-hand side of eq3_14 and
// eq3_15 around the solve for q, the shape filter (Section 3.7), the
// paraboloid curvature (Section 3.5), the tangential velocity (eq3_10,
// eq3_11), and RK4 then AB6 time marching (Section 3.6).
//
// The state is stored packed, bubble by bubble: column 4b + c of an
// [nd x 4 nb] column-major matrix holds coordinate c (x, y, z) or the
// potential (c = 3) of bubble b's vertices, so that the shape filter of all
// bubbles and all four fields is two FP64 GEMMs through the template's
// harmonic basis: F S = G (G+ S).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <initializer_list>
#include <utility>
#include <vector>

#include "../../include/bfm_step.h"
#include "ctx.h"
#include "learn.h"

namespace bfm {

struct Stepper {
    bfm_physics ph{};
    bool ph_set = false;
    bool rings_ready = false;
    DevBuf<int> ring5;          // five one-ring neighbours per vertex [nv][5]
    DevBuf<int> tri_off;        // per-bubble triangle ranges [nb + 1]
    ShBasis filt;               // plain least-squares basis of the shape filter
    bool state_set = false;
    double t = 0.0;
    int steps = 0;
    DevBuf<double> S, Y, Stmp, K[3], hist[6], work, Cf;  // packed [nd][4 nb] arrays
    int hist_head = 0;
    DevBuf<double> phi_f, q, H, tri_nxv, vt, vol, V0, pg0;
    bool have_q = false;
    int solves = 0, iterations = 0;
};

static unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }
constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Kernels

// S[(4b + c) nd + v] <- xyz[3o + c] (c < 3) or phi[o] (c = 3), o = b nd + v
__global__ void k_pack(const double *xyz, const double *phi, int nd, int64_t nv, double *S) {
    int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (o >= nv) return;
    const int64_t b = o / nd, v = o % nd;
    double *col = S + 4 * b * nd + v;
    col[0] = xyz[3 * o];
    col[nd] = xyz[3 * o + 1];
    col[2 * (int64_t)nd] = xyz[3 * o + 2];
    col[3 * (int64_t)nd] = phi[o];
}

__global__ void k_unpack(const double *S, int nd, int64_t nv, double *xyz, double *phi) {
    int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (o >= nv) return;
    const int64_t b = o / nd, v = o % nd;
    const double *col = S + 4 * b * nd + v;
    if (xyz) {
        xyz[3 * o] = col[0];
        xyz[3 * o + 1] = col[nd];
        xyz[3 * o + 2] = col[2 * (int64_t)nd];
    }
    if (phi) phi[o] = col[3 * (int64_t)nd];
}

// Mean curvature by the paraboloid through five neighbours (parab1, parab2):
// local frame z = n_j, x = tangential part of the edge to the first
// neighbour; 5 x 5 system by Gaussian elimination with partial pivoting.
__global__ void k_curvature(const double *xyz, const double *nrm, const int *ring5, int64_t nv, double *H) {
    int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= nv) return;
    const double rx = xyz[3 * j], ry = xyz[3 * j + 1], rz = xyz[3 * j + 2];
    const double nx = nrm[j], ny = nrm[nv + j], nz = nrm[2 * nv + j];
    const int *nb = ring5 + 5 * j;
    double ex, ey, ez;
    {
        const int k = nb[0];
        const double dx = xyz[3 * k] - rx, dy = xyz[3 * k + 1] - ry, dz = xyz[3 * k + 2] - rz;
        const double dn = dx * nx + dy * ny + dz * nz;
        ex = dx - dn * nx;
        ey = dy - dn * ny;
        ez = dz - dn * nz;
        const double il = 1.0 / sqrt(ex * ex + ey * ey + ez * ez);
        ex *= il;
        ey *= il;
        ez *= il;
    }
    const double fx = ny * ez - nz * ey, fy = nz * ex - nx * ez, fz = nx * ey - ny * ex;  // n x e_x
    double Q[5][6];
#pragma unroll
    for (int l = 0; l < 5; ++l) {
        const int k = nb[l];
        const double dx = xyz[3 * k] - rx, dy = xyz[3 * k + 1] - ry, dz = xyz[3 * k + 2] - rz;
        const double x = dx * ex + dy * ey + dz * ez, y = dx * fx + dy * fy + dz * fz,
                     z = dx * nx + dy * ny + dz * nz;
        Q[l][0] = x;
        Q[l][1] = y;
        Q[l][2] = x * x;
        Q[l][3] = x * y;
        Q[l][4] = y * y;
        Q[l][5] = z;
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        int piv = c;
        double best = fabs(Q[c][c]);
#pragma unroll
        for (int r = c + 1; r < 5; ++r)
            if (fabs(Q[r][c]) > best) {
                best = fabs(Q[r][c]);
                piv = r;
            }
#pragma unroll
        for (int r = c + 1; r < 5; ++r)  // swap rows c and piv (register-friendly form)
            if (r == piv)
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    const double tmp = Q[c][k];
                    Q[c][k] = Q[r][k];
                    Q[r][k] = tmp;
                }
        const double inv = 1.0 / Q[c][c];
#pragma unroll
        for (int r = c + 1; r < 5; ++r) {
            const double f = Q[r][c] * inv;
#pragma unroll
            for (int k = c; k < 6; ++k) Q[r][k] -= f * Q[c][k];
        }
    }
    double B[5];
#pragma unroll
    for (int r = 4; r >= 0; --r) {
        double v = Q[r][5];
#pragma unroll
        for (int k = r + 1; k < 5; ++k) v -= Q[r][k] * B[k];
        B[r] = v / Q[r][r];
    }
    H[j] = -B[2] - B[4];
}

// (n x v)_k A_k = [(r2 - r3) phi1 + (r3 - r1) phi2 + (r1 - r2) phi3] / 2 (eq3_10 times A_k)
__global__ void k_tri_nxv(const double *xyz, const int *tri, const double *phi, int64_t nt, double *out) {
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nt) return;
    const int a = tri[3 * k], b = tri[3 * k + 1], c = tri[3 * k + 2];
    const double pa = phi[a], pb = phi[b], pc = phi[c];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double ra = xyz[3 * a + d], rb = xyz[3 * b + d], rc = xyz[3 * c + d];
        out[3 * k + d] = 0.5 * ((rb - rc) * pa + (rc - ra) * pb + (ra - rb) * pc);
    }
}

// v_t = (n x v)_j x n_j, (n x v)_j = sum_k (n x v)_k A_k / (3 s_j) (eq3_11)
__global__ void k_vertex_vt(const int *v2t_off, const int *v2t, const double *tri_nxv, const double *s,
                            const double *nrm, int64_t nv, double *vt) {
    int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= nv) return;
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int e = v2t_off[j]; e < v2t_off[j + 1]; ++e) {
        const int k = v2t[e];
        ax += tri_nxv[3 * k];
        ay += tri_nxv[3 * k + 1];
        az += tri_nxv[3 * k + 2];
    }
    const double f = 1.0 / (3.0 * s[j]);
    ax *= f;
    ay *= f;
    az *= f;
    const double nx = nrm[j], ny = nrm[nv + j], nz = nrm[2 * nv + j];
    vt[3 * j] = ay * nz - az * ny;
    vt[3 * j + 1] = az * nx - ax * nz;
    vt[3 * j + 2] = ax * ny - ay * nx;
}

// V_b = sum over the bubble's triangles of (r1 - o) . ((r2 - o) x (r3 - o)) / 6,
// o = the first vertex of the bubble's first triangle (any origin gives the
// same volume of a closed surface; a near one avoids cancellation)
__global__ void k_volume(const double *xyz, const int *tri, const int *tri_off, double *vol) {
    __shared__ double red[256];
    const int b = blockIdx.x;
    const int64_t o = tri[3 * (int64_t)tri_off[b]];
    const double ox = xyz[3 * o], oy = xyz[3 * o + 1], oz = xyz[3 * o + 2];
    double acc = 0.0;
    for (int k = tri_off[b] + threadIdx.x; k < tri_off[b + 1]; k += 256) {
        const double *p = xyz + 3 * (int64_t)tri[3 * (int64_t)k];
        const double *q = xyz + 3 * (int64_t)tri[3 * (int64_t)k + 1];
        const double *r = xyz + 3 * (int64_t)tri[3 * (int64_t)k + 2];
        const double px = p[0] - ox, py = p[1] - oy, pz = p[2] - oz;
        const double qx = q[0] - ox, qy = q[1] - oy, qz = q[2] - oz;
        const double rx = r[0] - ox, ry = r[1] - oy, rz = r[2] - oz;
        acc += px * (qy * rz - qz * ry) + py * (qz * rx - qx * rz) + pz * (qx * ry - qy * rx);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) vol[b] = red[0] / 6.0;
}

__global__ void k_gas(const double *vol, int nb, double p0, double sigma, double *V0, double *pg0) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    V0[b] = vol[b];
    const double a0 = cbrt(3.0 * vol[b] / (4.0 * kPi));
    pg0[b] = p0 + 2.0 * sigma / a0;
}

struct RhsParams {
    double inv_rho, sigma, kappa, alpha, gx, gy, gz, pinf_rho;
};

// dr/dt = u = v + alpha v_t, dphi/dt of eq3_15, written packed
__global__ void k_rhs(const double *xyz, const double *nrm, const double *q, const double *vt, const double *H,
                      const double *vol, const double *V0, const double *pg0, int nd, int64_t nv, RhsParams P,
                      double *dS) {
    int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (o >= nv) return;
    const int64_t b = o / nd, v = o % nd;
    const double qq = q[o];
    const double tx = vt[3 * o], ty = vt[3 * o + 1], tz = vt[3 * o + 2];
    const double vx = nrm[o] * qq + tx, vy = nrm[nv + o] * qq + ty, vz = nrm[2 * nv + o] * qq + tz;
    const double pg = pg0[b] * pow(V0[b] / vol[b], P.kappa);
    const double dphi = (P.alpha * tx + 0.5 * vx) * vx + (P.alpha * ty + 0.5 * vy) * vy +
                        (P.alpha * tz + 0.5 * vz) * vz - (pg - 2.0 * P.sigma * H[o]) * P.inv_rho +
                        P.gx * xyz[3 * o] + P.gy * xyz[3 * o + 1] + P.gz * xyz[3 * o + 2] + P.pinf_rho;
    double *col = dS + 4 * b * nd + v;
    col[0] = vx + P.alpha * tx;
    col[nd] = vy + P.alpha * ty;
    col[2 * (int64_t)nd] = vz + P.alpha * tz;
    col[3 * (int64_t)nd] = dphi;
}

struct Comb {
    const double *x[6];
    double w[6];
    int m;
};

// out = base + sum_k w_k x_k (out may alias base)
__global__ void k_comb(int64_t n, const double *base, Comb c, double *out) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v = base[i];
    for (int k = 0; k < c.m; ++k) v += c.w[k] * c.x[k][i];
    out[i] = v;
}

// ---------------------------------------------------------------------------
// Host side

static Stepper &stepper(bfm_ctx *c) {
    if (!c->stepper) c->stepper = new Stepper();
    return *c->stepper;
}

void step_free(bfm_ctx *c) {
    delete c->stepper;
    c->stepper = nullptr;
}

void step_mesh_changed(bfm_ctx *c) {
    if (!c->stepper) return;
    c->stepper->rings_ready = false;
    c->stepper->state_set = false;
    c->stepper->have_q = false;
}

// one-rings in counter-clockwise order from the lowest-index neighbour
static void build_rings(bfm_ctx *c, Stepper &S) {
    if (S.rings_ready) return;
    const int64_t nv = c->nv, nt = c->nt;
    BFM_CHECK((int64_t)c->tri_h.size() == 3 * nt, BFM_EINVAL, "mesh triangles not available");
    // next[j]: pairs (a -> b) of the edges opposite j, a and b consecutive counter-clockwise around j
    std::vector<int> deg(nv + 1, 0);
    for (int64_t k = 0; k < 3 * nt; ++k) deg[c->tri_h[k] + 1]++;
    for (int64_t v = 0; v < nv; ++v) deg[v + 1] += deg[v];
    std::vector<int> from(3 * nt), to(3 * nt), fill(deg.begin(), deg.end() - 1);
    for (int64_t k = 0; k < nt; ++k) {
        const int a = c->tri_h[3 * k], b = c->tri_h[3 * k + 1], d = c->tri_h[3 * k + 2];
        const int vs[3] = {a, b, d};
        for (int e = 0; e < 3; ++e) {
            const int j = vs[e], p = vs[(e + 1) % 3], r = vs[(e + 2) % 3];
            from[fill[j]] = p;
            to[fill[j]] = r;
            fill[j]++;
        }
    }
    std::vector<int> ring((size_t)5 * nv);
    for (int64_t j = 0; j < nv; ++j) {
        const int lo = deg[j], hi = deg[j + 1], valence = hi - lo;
        BFM_CHECK(valence >= 5, BFM_EMESH, "vertex " + std::to_string(j) + " has fewer than five neighbours");
        int start = from[lo];
        for (int e = lo; e < hi; ++e) start = std::min(start, from[e]);
        int cur = start;
        for (int l = 0; l < valence; ++l) {
            if (l < 5) ring[5 * j + l] = cur;
            int nxt = -1;
            for (int e = lo; e < hi; ++e)
                if (from[e] == cur) {
                    nxt = to[e];
                    break;
                }
            BFM_CHECK(nxt >= 0, BFM_EMESH, "vertex " + std::to_string(j) + " is not on a closed surface");
            cur = nxt;
        }
        BFM_CHECK(cur == start, BFM_EMESH, "one-ring of vertex " + std::to_string(j) + " is not a cycle");
    }
    S.ring5.ensure(ring.size());
    BFM_HIP(hipMemcpyAsync(S.ring5.get(), ring.data(), sizeof(int) * ring.size(), hipMemcpyHostToDevice,
                           c->stream));
    std::vector<int> to_h(c->tri_off.begin(), c->tri_off.end());
    S.tri_off.ensure(to_h.size());
    BFM_HIP(hipMemcpyAsync(S.tri_off.get(), to_h.data(), sizeof(int) * to_h.size(), hipMemcpyHostToDevice,
                           c->stream));
    BFM_HIP(hipStreamSynchronize(c->stream));
    S.rings_ready = true;
}

static void check_ready(bfm_ctx *c, Stepper &S) {
    BFM_CHECK(c->nv > 0, BFM_EINVAL, "no mesh set");
    BFM_CHECK(c->pre.nd > 0, BFM_EINVAL,
              "the time-step harness needs a template (bfm_set_sphere_template or bfm_set_torus_template)");
    BFM_CHECK(S.ph_set, BFM_EINVAL, "no physics set (bfm_set_physics)");
    const int pf = S.ph.filter_degree;
    if (c->pre.genus == 0) {
        BFM_CHECK(pf >= 0 && (int64_t)pf * pf <= c->pre.nd, BFM_EINVAL, "filter_degree^2 must not exceed nd");
    } else {
        BFM_CHECK(pf >= 0 && pf % 2 == 0 && (int64_t)(pf + 1) * (pf + 1) <= c->pre.nd, BFM_EINVAL,
                  "toroidal filter: filter_degree must be even with (filter_degree + 1)^2 <= nd");
    }
    build_rings(c, S);
    if (pf > 0) {
        // spherical: harmonics of degree 0..p_f-1; toroidal (spherical7): degree
        // 0..p_f/2 in each angle
        if (c->pre.genus == 0)
            sh_basis_build(c->pre, pf - 1, S.filt, c->stream, false);
        else
            torus_basis_build(c->pre, pf / 2, S.filt, c->stream);
    }
}

// in -> out = F in for packed arrays (out may not alias in)
static void apply_filter(bfm_ctx *c, Stepper &S, const double *in, double *out) {
    const int nd = c->pre.nd, nb = c->nb;
    const int64_t n = 4 * (int64_t)nb * nd;
    if (S.ph.filter_degree <= 0) {
        BFM_HIP(hipMemcpyAsync(out, in, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
        return;
    }
    const int nc = S.filt.nc;
    double *C = S.Cf.ensure((size_t)nc * 4 * nb);
    gemm_nn_f64(nc, 4 * nb, nd, S.filt.Gp.get(), nc, in, nd, C, nc, c->stream);
    gemm_nn_f64(nd, 4 * nb, nc, S.filt.G.get(), nd, C, nc, out, nd, c->stream);
}

static double p_inf(const bfm_physics &ph, double t) {
    if (ph.period <= 0.0 || ph.pa == 0.0) return ph.p0;
    return ph.p0 + ph.forcing_sign * ph.pa * std::sin(2.0 * kPi * t / ph.period);
}

// filtered surface of the packed state: c->xyz (solver positions) and S.phi_f
static void set_surface(bfm_ctx *c, Stepper &S, const double *Sin) {
    const int nd = c->pre.nd;
    const int64_t nv = c->nv;
    double *Sf = S.work.ensure(4 * (size_t)nv);
    apply_filter(c, S, Sin, Sf);
    double *phi = S.phi_f.ensure(nv);
    k_unpack<<<nblk(nv, 256), 256, 0, c->stream>>>(Sf, nd, nv, c->xyz.get(), phi);
    BFM_LAUNCHED();
    c->geom_valid = false;
    c->tree_valid = false;
    c->diag_valid = false;
}

// dS = F rhs(F Sin) at time t
static void rhs(bfm_ctx *c, Stepper &S, double t, const double *Sin, double *dS, int *iters) {
    hipStream_t st = c->stream;
    const int nd = c->pre.nd, nb = c->nb;
    const int64_t nv = c->nv, nt = c->nt;
    set_surface(c, S, Sin);
    ensure_geometry(c);
    double *q = S.q.ensure(nv);
    int guess = BFM_GUESS_ZERO;
    if (S.ph.guess == BFM_GUESS_GIVEN && S.have_q) guess = BFM_GUESS_GIVEN;
    if (S.ph.guess == BFM_GUESS_LEARNED) guess = BFM_GUESS_LEARNED;
    bfm_solve_info info{};
    solve_impl(c, S.phi_f.get(), q, guess, &info);
    S.have_q = true;
    S.solves += 1;
    S.iterations += info.iterations;
    if (iters) *iters += info.iterations;
    if (S.ph.collect) mlp_collect(c, S.phi_f.get(), q);
    double *H = S.H.ensure(nv);
    k_curvature<<<nblk(nv, 128), 128, 0, st>>>(c->xyz.get(), c->nrm.get(), S.ring5.get(), nv, H);
    BFM_LAUNCHED();
    double *tn = S.tri_nxv.ensure(3 * (size_t)nt);
    k_tri_nxv<<<nblk(nt, 256), 256, 0, st>>>(c->xyz.get(), c->tri.get(), S.phi_f.get(), nt, tn);
    BFM_LAUNCHED();
    double *vt = S.vt.ensure(3 * (size_t)nv);
    k_vertex_vt<<<nblk(nv, 256), 256, 0, st>>>(c->v2t_off.get(), c->v2t.get(), tn, c->s.get(), c->nrm.get(), nv,
                                               vt);
    BFM_LAUNCHED();
    double *vol = S.vol.ensure(nb);
    k_volume<<<nb, 256, 0, st>>>(c->xyz.get(), c->tri.get(), S.tri_off.get(), vol);
    BFM_LAUNCHED();
    RhsParams P{1.0 / S.ph.rho, S.ph.sigma, S.ph.kappa, S.ph.alpha, S.ph.g[0], S.ph.g[1], S.ph.g[2],
                p_inf(S.ph, t) / S.ph.rho};
    double *raw = S.Stmp.ensure(4 * (size_t)nv);
    BFM_CHECK(raw != Sin, BFM_EINVAL, "internal: rhs input aliases its work array");
    k_rhs<<<nblk(nv, 256), 256, 0, st>>>(c->xyz.get(), c->nrm.get(), q, vt, H, vol, S.V0.get(), S.pg0.get(), nd, nv,
                                         P, raw);
    BFM_LAUNCHED();
    apply_filter(c, S, raw, dS);
}

static void comb(bfm_ctx *c, int64_t n, const double *base, std::initializer_list<std::pair<double, const double *>> t,
                 double *out) {
    Comb cb{};
    cb.m = 0;
    for (const auto &p : t) {
        cb.x[cb.m] = p.second;
        cb.w[cb.m] = p.first;
        cb.m++;
    }
    k_comb<<<nblk(n, 256), 256, 0, c->stream>>>(n, base, cb, out);
    BFM_LAUNCHED();
}

// Adams-Bashforth weights of order 6, newest first (integrated Lagrange basis)
static const double kAB6[6] = {4277.0 / 1440.0, -7923.0 / 1440.0, 9982.0 / 1440.0,
                               -7298.0 / 1440.0, 2877.0 / 1440.0, -475.0 / 1440.0};

void step_set_physics(bfm_ctx *c, const bfm_physics &ph) {
    BFM_CHECK(ph.rho > 0.0 && ph.p0 >= 0.0 && ph.kappa > 0.0 && ph.sigma >= 0.0 && ph.period >= 0.0, BFM_EINVAL,
              "physics: rho > 0, p0 >= 0, kappa > 0, sigma >= 0, period >= 0 required");
    BFM_CHECK(ph.filter_degree >= 0 && ph.filter_degree <= 40, BFM_EINVAL, "filter_degree out of range");
    BFM_CHECK(ph.guess == BFM_GUESS_ZERO || ph.guess == BFM_GUESS_GIVEN || ph.guess == BFM_GUESS_LEARNED,
              BFM_EINVAL, "unknown guess");
    Stepper &S = stepper(c);
    S.ph = ph;
    S.ph_set = true;
    S.steps = 0;
    S.have_q = false;
}

void step_state_set(bfm_ctx *c, const double *xyz_h, const double *phi_h, double t) {
    Stepper &S = stepper(c);
    check_ready(c, S);
    hipStream_t st = c->stream;
    const int nd = c->pre.nd, nb = c->nb;
    const int64_t nv = c->nv;
    DevBuf<double> tmp;
    tmp.ensure(4 * (size_t)nv);
    BFM_HIP(hipMemcpyAsync(tmp.get(), xyz_h, sizeof(double) * 3 * nv, hipMemcpyHostToDevice, st));
    BFM_HIP(hipMemcpyAsync(tmp.get() + 3 * nv, phi_h, sizeof(double) * nv, hipMemcpyHostToDevice, st));
    double *Sv = S.S.ensure(4 * (size_t)nv);
    k_pack<<<nblk(nv, 256), 256, 0, st>>>(tmp.get(), tmp.get() + 3 * nv, nd, nv, Sv);
    BFM_LAUNCHED();
    // gas: volumes of the filtered initial shape
    set_surface(c, S, Sv);
    double *vol = S.vol.ensure(nb);
    k_volume<<<nb, 256, 0, st>>>(c->xyz.get(), c->tri.get(), S.tri_off.get(), vol);
    BFM_LAUNCHED();
    k_gas<<<nblk(nb, 128), 128, 0, st>>>(vol, nb, S.ph.p0, S.ph.sigma, S.V0.ensure(nb), S.pg0.ensure(nb));
    BFM_LAUNCHED();
    BFM_HIP(hipStreamSynchronize(st));
    S.t = t;
    S.steps = 0;
    S.have_q = false;
    S.state_set = true;
}

void step_state_get(bfm_ctx *c, double *xyz_h, double *phi_h, double *t) {
    Stepper &S = stepper(c);
    BFM_CHECK(S.state_set, BFM_EINVAL, "no state set (bfm_state_set)");
    const int64_t nv = c->nv;
    DevBuf<double> tmp;
    tmp.ensure(4 * (size_t)nv);
    k_unpack<<<nblk(nv, 256), 256, 0, c->stream>>>(S.S.get(), c->pre.nd, nv, tmp.get(), tmp.get() + 3 * nv);
    BFM_LAUNCHED();
    if (xyz_h)
        BFM_HIP(hipMemcpyAsync(xyz_h, tmp.get(), sizeof(double) * 3 * nv, hipMemcpyDeviceToHost, c->stream));
    if (phi_h)
        BFM_HIP(hipMemcpyAsync(phi_h, tmp.get() + 3 * nv, sizeof(double) * nv, hipMemcpyDeviceToHost, c->stream));
    BFM_HIP(hipStreamSynchronize(c->stream));
    if (t) *t = S.t;
}

void step_advance(bfm_ctx *c, double dt, bfm_step_info *info) {
    Stepper &S = stepper(c);
    BFM_CHECK(S.state_set, BFM_EINVAL, "no state set (bfm_state_set)");
    BFM_CHECK(dt > 0.0 && std::isfinite(dt), BFM_EINVAL, "dt must be positive");
    check_ready(c, S);
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = 4 * (int64_t)c->nv;
    for (auto &h : S.hist) h.ensure(n);
    double *Sv = S.S.get();
    int iters = 0, solves0 = S.solves;
    // new history slot (newest first)
    S.hist_head = (S.hist_head + 5) % 6;
    double *f0 = S.hist[S.hist_head].get();
    const bool rk = S.steps < 5;
    rhs(c, S, S.t, Sv, f0, &iters);
    if (rk) {
        double *k2 = S.K[0].ensure(n), *k3 = S.K[1].ensure(n), *k4 = S.K[2].ensure(n);
        double *y = S.Y.ensure(n);  // stage state
        comb(c, n, Sv, {{dt / 2, f0}}, y);
        rhs(c, S, S.t + dt / 2, y, k2, &iters);
        comb(c, n, Sv, {{dt / 2, k2}}, y);
        rhs(c, S, S.t + dt / 2, y, k3, &iters);
        comb(c, n, Sv, {{dt, k3}}, y);
        rhs(c, S, S.t + dt, y, k4, &iters);
        comb(c, n, Sv, {{dt / 6, f0}, {dt / 3, k2}, {dt / 3, k3}, {dt / 6, k4}}, Sv);
    } else {
        Comb cb{};
        cb.m = 6;
        for (int k = 0; k < 6; ++k) {
            cb.x[k] = S.hist[(S.hist_head + k) % 6].get();
            cb.w[k] = dt * kAB6[k];
        }
        k_comb<<<nblk(n, 256), 256, 0, c->stream>>>(n, Sv, cb, Sv);
        BFM_LAUNCHED();
    }
    BFM_HIP(hipStreamSynchronize(c->stream));
    S.t += dt;
    S.steps += 1;
    if (info) {
        info->scheme = rk ? 0 : 1;
        info->solves = S.solves - solves0;
        info->iterations = iters;
        info->t = S.t;
        info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
}

void step_rhs(bfm_ctx *c, double t, const double *xyz_h, const double *phi_h, double *dxyz, double *dphi, double *q,
              double *H) {
    Stepper &S = stepper(c);
    BFM_CHECK(S.state_set, BFM_EINVAL, "no state set (bfm_state_set): V0 and p_g0 come from it");
    check_ready(c, S);
    hipStream_t st = c->stream;
    const int nd = c->pre.nd;
    const int64_t nv = c->nv;
    DevBuf<double> tmp, Sin, dS;
    tmp.ensure(4 * (size_t)nv);
    Sin.ensure(4 * (size_t)nv);
    dS.ensure(4 * (size_t)nv);
    BFM_HIP(hipMemcpyAsync(tmp.get(), xyz_h, sizeof(double) * 3 * nv, hipMemcpyHostToDevice, st));
    BFM_HIP(hipMemcpyAsync(tmp.get() + 3 * nv, phi_h, sizeof(double) * nv, hipMemcpyHostToDevice, st));
    k_pack<<<nblk(nv, 256), 256, 0, st>>>(tmp.get(), tmp.get() + 3 * nv, nd, nv, Sin.get());
    BFM_LAUNCHED();
    rhs(c, S, t, Sin.get(), dS.get(), nullptr);
    k_unpack<<<nblk(nv, 256), 256, 0, st>>>(dS.get(), nd, nv, tmp.get(), tmp.get() + 3 * nv);
    BFM_LAUNCHED();
    if (dxyz) BFM_HIP(hipMemcpyAsync(dxyz, tmp.get(), sizeof(double) * 3 * nv, hipMemcpyDeviceToHost, st));
    if (dphi) BFM_HIP(hipMemcpyAsync(dphi, tmp.get() + 3 * nv, sizeof(double) * nv, hipMemcpyDeviceToHost, st));
    if (q) BFM_HIP(hipMemcpyAsync(q, S.q.get(), sizeof(double) * nv, hipMemcpyDeviceToHost, st));
    if (H) BFM_HIP(hipMemcpyAsync(H, S.H.get(), sizeof(double) * nv, hipMemcpyDeviceToHost, st));
    BFM_HIP(hipStreamSynchronize(st));
}

}  // namespace bfm
