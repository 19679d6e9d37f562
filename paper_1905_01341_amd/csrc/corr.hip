// Near-field correction matrices (Section 3.9: the method's nodal rule ns1
// combined with sparse corrections, the difference between the matrices of
// a high- and a low-order quadrature).
//
// With linear (hat) basis functions lambda_v on the flat triangles, the
// entries of L and M are sums over the triangles T ∋ v of integrals of G and
// dG/dn_T weighted by lambda_v; ns1 replaces each triangle's part by a third
// of its area times the kernel at the vertex. For collocation point i the
// near triangles are those with a vertex in {i} or its one-ring; on each, a
// conical Gauss product rule collapsed at the triangle's vertex nearest r_i
// (8 x 8 Gauss-Legendre nodes in s, t; y = P0 + s (P1 - P0) + s t (P2 - P1),
// dS = 2 A s ds dt) takes the integrals; when r_i is that vertex the factor s
// cancels the singularity of G and the double-layer integrand vanishes.
// C_iv (v != i) = sum over near T ∋ v of [rule - nodal share]; the diagonal
// entries and b follow from the method's identities applied to the corrected
// off-diagonal entries (s3, s5, eq3_1), so each gets a sum over its row.
//
// The pattern (near triangles and the columns of every row) depends only on
// the connectivity and is built on the host once per mesh; the values
// depend on the positions and are computed on the device, one row per
// thread, whenever the geometry or the octree (whose point order they are
// stored in) changes.
#include <algorithm>
#include <cmath>
#include <vector>

#include "ctx.h"
#include "xcd.h"

namespace bfm {

// 8-point Gauss-Legendre rule mapped to [0, 1]: nodes (1 + x_k) / 2 and
// weights w_k / 2 of the standard rule on [-1, 1] (x_k the roots of P_8).
// The quadrature loops are unrolled, so the tables fold into the code.
constexpr int kCorrG = 8;
constexpr double kCorrX[kCorrG] = {0.019855071751231912, 0.10166676129318664, 0.2372337950418355,
                                   0.4082826787521751,   0.5917173212478248,  0.7627662049581645,
                                   0.8983332387068134,   0.9801449282487681};
constexpr double kCorrW[kCorrG] = {0.050614268145188344, 0.11119051722668717, 0.15685332293894352,
                                   0.18134189168918088,  0.18134189168918088, 0.15685332293894352,
                                   0.11119051722668717,  0.050614268145188344};

static unsigned cblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Host pattern: near triangles per vertex (those of i, then the others
// touching its one-ring, each group ascending) with the row slots of their
// vertices, and the columns j != i they touch (ascending).
static void corr_pattern(bfm_ctx *c) {
    NearCorr &k = c->corr;
    const int64_t nv = c->nv, nt = c->nt;
    const std::vector<int> &tri = c->tri_h;
    std::vector<std::vector<int>> v2t(nv), ring(nv);
    for (int64_t t = 0; t < nt; ++t)
        for (int a = 0; a < 3; ++a) {
            const int v = tri[3 * t + a];
            v2t[v].push_back((int)t);
            for (int b = 0; b < 3; ++b)
                if (b != a) ring[v].push_back(tri[3 * t + b]);
        }
    std::vector<int> tptr(nv + 1, 0), rptr(nv + 1, 0), tv, col;
    std::vector<int> ts, cs;
    int w = 1;
    for (int64_t i = 0; i < nv; ++i) {
        // the triangles of i first (the self-singular ones, cheap), then the
        // rest, so that the lanes of a wave take the same branch together
        ts.clear();
        for (int j : ring[i]) ts.insert(ts.end(), v2t[j].begin(), v2t[j].end());
        std::sort(ts.begin(), ts.end());
        ts.erase(std::unique(ts.begin(), ts.end()), ts.end());
        ts.erase(std::remove_if(ts.begin(), ts.end(),
                                [&](int t) { return std::binary_search(v2t[i].begin(), v2t[i].end(), t); }),
                 ts.end());
        ts.insert(ts.begin(), v2t[i].begin(), v2t[i].end());
        cs.clear();
        for (int t : ts)
            for (int a = 0; a < 3; ++a)
                if (tri[3 * t + a] != (int)i) cs.push_back(tri[3 * t + a]);
        std::sort(cs.begin(), cs.end());
        cs.erase(std::unique(cs.begin(), cs.end()), cs.end());
        BFM_CHECK(cs.size() < 255, BFM_EINVAL, "near-field corrections: vertex with too many neighbours");
        for (int t : ts) {  // vertices of t and their row slots (255 for i itself)
            int packed = 0;
            for (int a = 0; a < 3; ++a) {
                const int v = tri[3 * t + a];
                const int k = v == (int)i ? 255 : (int)(std::lower_bound(cs.begin(), cs.end(), v) - cs.begin());
                packed |= k << (8 * a);
                tv.push_back(v);
            }
            tv.push_back(packed);
        }
        col.insert(col.end(), cs.begin(), cs.end());
        tptr[i + 1] = (int)(tv.size() / 4);
        rptr[i + 1] = (int)col.size();
        w = std::max(w, (int)cs.size());
    }
    BFM_CHECK((int64_t)w * nv < ((int64_t)1 << 31), BFM_EINVAL, "near-field corrections: mesh too large");
    hipStream_t st = c->stream;
    auto up = [&](DevBuf<int> &d, const std::vector<int> &h) {
        d.ensure(h.size());
        BFM_HIP(hipMemcpyAsync(d.get(), h.data(), sizeof(int) * h.size(), hipMemcpyHostToDevice, st));
    };
    up(k.tptr, tptr);
    up(k.tv, tv);
    up(k.rptr, rptr);
    up(k.col, col);
    k.nnz = (int64_t)col.size();
    k.w = w;
    k.ecol.ensure((size_t)w * nv);
    k.ecl.ensure((size_t)w * nv);
    k.ecm.ensure((size_t)w * nv);
    BFM_HIP(hipStreamSynchronize(st));  // the host vectors go out of scope
    k.pattern = true;
    k.values = false;
}

// 1 / sqrt(x), x > 0: the hardware estimate refined by two Newton steps
// y <- y (3 - x y^2) / 2 (each squares the relative error)
__device__ inline double inv_sqrt(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}

// One sorted row per thread: the corrections of row r (vertex i = perm[r]),
// written to the ELL slots k * nv + r in the pattern's column order. Each
// near triangle comes as (v0, v1, v2, packed slots), read one triangle
// ahead. LDS: the row's running sums sit in LDS (slot k of lane t at
// k * 64 + t, one 64-lane wave per block: no bank conflicts whatever the
// lanes' slots), written once at the end; else they are summed in place
// in the ELL arrays (rows with more than kCorrLdsSlots columns), which
// moves each line through L2 once per contribution.
//
// On a triangle not containing r_i the hat-weighted integrands are
// evaluated at y = P0 + s e1 + s t e2 as functions of t for each s:
// |r_i - y|^2 = |a|^2 - 2 t (a . s e2) + t^2 |s e2|^2 with a = r_i - P0 - s e1,
// and (r_i - y) . n_T is the same at every y of the flat triangle.
constexpr int kCorrLdsSlots = 40;  // 2 * 40 * 64 doubles = 40 KiB of LDS per block

template <bool LDS>
__global__ void __launch_bounds__(64) k_corr_values(int64_t nv, const int *__restrict__ perm,
                                                    const int *__restrict__ iperm, const double *__restrict__ xyz,
                                                    const double *__restrict__ nrm, const int *__restrict__ tptr,
                                                    const int4 *__restrict__ tv, const int *__restrict__ rptr,
                                                    const int *__restrict__ col, int w, int *__restrict__ ecol,
                                                    double *__restrict__ ecl, double *__restrict__ ecm) {
    extern __shared__ double lacc[];  // LDS: [2][w][64]
    const int lane = threadIdx.x;
    const int64_t r = xcd_block() * blockDim.x + lane;
    if (r >= nv) return;
    const int i = perm[r];
    const int r0 = rptr[i], r1 = rptr[i + 1];
    for (int e = 0; e < w; ++e) {
        ecol[e * nv + r] = e < r1 - r0 ? iperm[col[r0 + e]] : (int)r;
        if (LDS) {
            lacc[e * 64 + lane] = 0.0;
            lacc[(w + e) * 64 + lane] = 0.0;
        } else {
            ecl[e * nv + r] = 0.0;
            ecm[e * nv + r] = 0.0;
        }
    }
    const double rx = xyz[3 * (int64_t)i], ry = xyz[3 * (int64_t)i + 1], rz = xyz[3 * (int64_t)i + 2];
    const double k4 = 1.0 / (4.0 * 3.14159265358979323846);
    const int ri = i;
    const int e0 = tptr[i], e1_ = tptr[i + 1];
    int4 nxt = e0 < e1_ ? tv[e0] : make_int4(0, 0, 0, 0);
    for (int e = e0; e < e1_; ++e) {
        const int4 cur = nxt;
        if (e + 1 < e1_) nxt = tv[e + 1];
        const int v[3] = {cur.x, cur.y, cur.z};
        double P[3][3], d2[3];
        for (int q = 0; q < 3; ++q)
            for (int b = 0; b < 3; ++b) P[q][b] = xyz[3 * (int64_t)v[q] + b];
        for (int q = 0; q < 3; ++q) {
            const double dx = P[q][0] - rx, dy = P[q][1] - ry, dz = P[q][2] - rz;
            d2[q] = dx * dx + dy * dy + dz * dz;
        }
        // collapse at the vertex nearest r_i (ties within 1e-9: the first)
        const double dmin = fmin(d2[0], fmin(d2[1], d2[2]));
        const int f = d2[0] <= dmin * (1.0 + 1e-9) ? 0 : (d2[1] <= dmin * (1.0 + 1e-9) ? 1 : 2);
        const int o[3] = {f, f == 2 ? 0 : f + 1, f == 0 ? 2 : f - 1};
        double Q[3][3];
        for (int q = 0; q < 3; ++q)
            for (int b = 0; b < 3; ++b) Q[q][b] = P[o[q]][b];
        const double e1[3] = {Q[1][0] - Q[0][0], Q[1][1] - Q[0][1], Q[1][2] - Q[0][2]};
        const double e2[3] = {Q[2][0] - Q[1][0], Q[2][1] - Q[1][1], Q[2][2] - Q[1][2]};
        const double f2[3] = {Q[2][0] - Q[0][0], Q[2][1] - Q[0][1], Q[2][2] - Q[0][2]};
        double nT[3] = {e1[1] * f2[2] - e1[2] * f2[1], e1[2] * f2[0] - e1[0] * f2[2], e1[0] * f2[1] - e1[1] * f2[0]};
        const double twoA = sqrt(nT[0] * nT[0] + nT[1] * nT[1] + nT[2] * nT[2]);
        for (int b = 0; b < 3; ++b) nT[b] /= twoA;
        const double c0 = twoA * k4;
        double IL[3] = {0, 0, 0}, IM[3] = {0, 0, 0};
        if (v[o[0]] == ri) {
            // r_i is the collapse vertex: G dS = c0 ds dt / |e1 + t e2| (the
            // factor s cancels), the double layer vanishes; the s-sums of the
            // hat functions (1 - s, s (1 - t), s t) are 1/2 (1, 1 - t, t)
#pragma unroll
            for (int b = 0; b < kCorrG; ++b) {
                const double t2 = kCorrX[b];
                const double dx = e1[0] + t2 * e2[0], dy = e1[1] + t2 * e2[1], dz = e1[2] + t2 * e2[2];
                const double g = 0.5 * kCorrW[b] * c0 * inv_sqrt(dx * dx + dy * dy + dz * dz);
                IL[0] += g;
                IL[1] += g * (1.0 - t2);
                IL[2] += g * t2;
            }
        } else {
            const double qx = rx - Q[0][0], qy = ry - Q[0][1], qz = rz - Q[0][2];
            const double hT = qx * nT[0] + qy * nT[1] + qz * nT[2];
            const double ee = e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2];
#pragma unroll
            for (int a = 0; a < kCorrG; ++a) {
                const double s = kCorrX[a], cs = c0 * kCorrW[a] * s;
                const double ax = qx - s * e1[0], ay = qy - s * e1[1], az = qz - s * e1[2];
                const double aa = ax * ax + ay * ay + az * az;
                const double m2as = -2.0 * s * (ax * e2[0] + ay * e2[1] + az * e2[2]);
                const double ss = s * s * ee;
                double gl0 = 0.0, gl1 = 0.0, gm0 = 0.0, gm1 = 0.0;  // sums of w/r, w t/r, w/r^3, w t/r^3
#pragma unroll
                for (int b = 0; b < kCorrG; ++b) {
                    const double t2 = kCorrX[b], wb = kCorrW[b], wt2 = wb * t2;
                    const double ir = inv_sqrt(fma(fma(t2, ss, m2as), t2, aa));
                    const double ir3 = ir * ir * ir;
                    gl0 = fma(wb, ir, gl0);
                    gl1 = fma(wt2, ir, gl1);
                    gm0 = fma(wb, ir3, gm0);
                    gm1 = fma(wt2, ir3, gm1);
                }
                // hat functions at (s, t): 1 - s, s (1 - t), s t
                IL[0] += cs * (1.0 - s) * gl0;
                IL[1] += cs * s * (gl0 - gl1);
                IL[2] += cs * s * gl1;
                IM[0] += cs * (1.0 - s) * gm0;
                IM[1] += cs * s * (gm0 - gm1);
                IM[2] += cs * s * gm1;
            }
            for (int q = 0; q < 3; ++q) IM[q] *= hT;
        }
        const double third = twoA / 6.0;  // A / 3
        for (int q = 0; q < 3; ++q) {
            const int oq = o[q], vq = v[oq];
            if (vq == ri) continue;
            const double dx = rx - Q[q][0], dy = ry - Q[q][1], dz = rz - Q[q][2];
            const double ir = inv_sqrt(dx * dx + dy * dy + dz * dz);
            const double nl = third * k4 * ir;
            const double nm = nl * ir * ir * (dx * nrm[vq] + dy * nrm[nv + vq] + dz * nrm[2 * nv + vq]);
            const int k = (cur.w >> (8 * oq)) & 255;
            if (LDS) {
                lacc[k * 64 + lane] += IL[q] - nl;
                lacc[(w + k) * 64 + lane] += IM[q] - nm;
            } else {
                ecl[k * nv + r] += IL[q] - nl;
                ecm[k * nv + r] += IM[q] - nm;
            }
        }
    }
    if (LDS)
        for (int e = 0; e < w; ++e) {
            ecl[e * nv + r] = lacc[e * 64 + lane];
            ecm[e * nv + r] = lacc[(w + e) * 64 + lane];
        }
}

void corr_invalidate(bfm_ctx *c, bool mesh) {
    c->corr.values = false;
    if (mesh) c->corr.pattern = false;
}

void ensure_corr(bfm_ctx *c) {
    if (!c->opt.near_corr) return;
    ensure_tree(c);
    NearCorr &k = c->corr;
    if (!k.pattern) corr_pattern(c);
    if (k.values) return;
    const bool lds = k.w <= kCorrLdsSlots;
    auto kern = lds ? k_corr_values<true> : k_corr_values<false>;
    kern<<<cblk(c->nv, 64), 64, lds ? sizeof(double) * 2 * 64 * k.w : 0, c->stream>>>(
        c->nv, c->tree.idx_a.get(), c->tree.iperm.get(), c->xyz.get(), c->nrm.get(), k.tptr.get(),
        reinterpret_cast<const int4 *>(k.tv.get()), k.rptr.get(), k.col.get(), k.w, k.ecol.get(), k.ecl.get(),
        k.ecm.get());
    BFM_LAUNCHED();
    k.values = true;
}

// out_s[r] += sum_k (f CL x_s + g CM y_s)[ecol] over the row's ELL slots
template <bool X, bool Y>
__global__ void __launch_bounds__(256) k_corr_apply(int64_t nv, int w, const int *__restrict__ ecol,
                                                    const double *__restrict__ ecl, const double *__restrict__ ecm,
                                                    double f, const double *__restrict__ x, double g,
                                                    const double *__restrict__ y, double *__restrict__ out) {
    const int64_t r = xcd_block() * blockDim.x + threadIdx.x;
    if (r >= nv) return;
    double ax = 0.0, ay = 0.0;
#pragma unroll 6
    for (int e = 0; e < w; ++e) {
        const int64_t slot = e * nv + r;
        const int j = ecol[slot];
        if (X) ax += ecl[slot] * x[j];
        if (Y) ay += ecm[slot] * y[j];
    }
    out[r] += (X ? f * ax : 0.0) + (Y ? g * ay : 0.0);
}

void corr_apply(bfm_ctx *c, double f, const double *x_s, double g, const double *y_s, double *out_s) {
    if (!c->opt.near_corr) return;
    const NearCorr &k = c->corr;
    BFM_CHECK(k.pattern && k.values, BFM_EINVAL, "near-field corrections not prepared");
    const bool X = f != 0.0 && x_s, Y = g != 0.0 && y_s;
    if (!X && !Y) return;
    const unsigned nb = cblk(c->nv, 256);
    hipStream_t st = c->stream;
    if (X && Y)
        k_corr_apply<true, true><<<nb, 256, 0, st>>>(c->nv, k.w, k.ecol.get(), k.ecl.get(), k.ecm.get(), f, x_s, g,
                                                    y_s, out_s);
    else if (X)
        k_corr_apply<true, false><<<nb, 256, 0, st>>>(c->nv, k.w, k.ecol.get(), k.ecl.get(), k.ecm.get(), f, x_s,
                                                     g, nullptr, out_s);
    else
        k_corr_apply<false, true><<<nb, 256, 0, st>>>(c->nv, k.w, k.ecol.get(), k.ecl.get(), k.ecm.get(), f,
                                                     nullptr, g, y_s, out_s);
    BFM_LAUNCHED();
}

// Corrected diagonals and b (sorted): M_ii -= sum_j CM_ij;
// L_ii += n_i . [sum_j CM_ij (r_j - r_i) - sum_j CL_ij n_j];
// b_i += sum_j CM_ij (phi_j - phi_i). Padding slots (j = i, zero values)
// add nothing.
__global__ void __launch_bounds__(256) k_corr_diag(int64_t nv, int w, const int *__restrict__ ecol,
                                                   const double *__restrict__ ecl, const double *__restrict__ ecm,
                                                   const double *__restrict__ px, const double *__restrict__ py,
                                                   const double *__restrict__ pz, const double *__restrict__ pnx,
                                                   const double *__restrict__ pny, const double *__restrict__ pnz,
                                                   const double *__restrict__ phi, double *__restrict__ mii,
                                                   double *__restrict__ lii, double *__restrict__ b) {
    const int64_t r = xcd_block() * blockDim.x + threadIdx.x;
    if (r >= nv) return;
    double sm = 0.0, vx = 0.0, vy = 0.0, vz = 0.0, sb = 0.0;
    const double rx = px[r], ry = py[r], rz = pz[r];
    const double pr = phi ? phi[r] : 0.0;
#pragma unroll 6
    for (int e = 0; e < w; ++e) {
        const int64_t slot = e * nv + r;
        const int j = ecol[slot];
        const double m = ecm[slot], l = ecl[slot];
        sm += m;
        vx += m * (px[j] - rx) - l * pnx[j];
        vy += m * (py[j] - ry) - l * pny[j];
        vz += m * (pz[j] - rz) - l * pnz[j];
        if (phi) sb += m * (phi[j] - pr);
    }
    mii[r] -= sm;
    lii[r] += pnx[r] * vx + pny[r] * vy + pnz[r] * vz;
    if (phi) b[r] += sb;
}

void corr_diagonals(bfm_ctx *c, const double *phi_s) {
    if (!c->opt.near_corr) return;
    ensure_corr(c);
    const NearCorr &k = c->corr;
    const Tree &t = c->tree;
    k_corr_diag<<<cblk(c->nv, 256), 256, 0, c->stream>>>(c->nv, k.w, k.ecol.get(), k.ecl.get(), k.ecm.get(),
                                                        t.px.get(), t.py.get(), t.pz.get(), t.pnx.get(),
                                                        t.pny.get(), t.pnz.get(), phi_s, c->mii_s.get(),
                                                        c->lii_s.get(), c->b_s.get());
    BFM_LAUNCHED();
}

}  // namespace bfm
