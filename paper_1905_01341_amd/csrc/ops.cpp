// Host construction of the translation operators (multipole-to-multipole,
// multipole-to-local, local-to-local) as dense real P x P matrices in the
// normalised, box-scaled basis of common.h.
//
// Scaling. A box of side h stores Mt_n^m = M_n^m nu_n^m / h^n (multipole)
// and Lt_n^m = L_n^m h^{n+1} / nu_n^m (local), where M, L are the plain
// coefficients of phi(r) = sum M_n^m I_n^m(r - c) = sum L_n^m R_n^m(r - c).
// Then every operator depends only on the offset between box centres in
// units of the box side, so one set serves every level:
//   M2M (child side h, parent 2h, e = (c_child - c_parent)/h):
//     Mt_n^m(parent) = 2^-n nu_n^m sum_{j,k} Mt_j^k conj(Rt_{n-j}^{m-k}(e)) / (nu_j^k nu_{n-j}^{m-k})
//   M2L (both side h, d = (c_target - c_source)/h, |d|_inf in {2,3}):
//     Lt_j^k = (-1)^{j+k} sum_{n,m} Mt_n^m It_{n+j}^{m-k}(d) nu_{n+j}^{m-k} / (nu_j^k nu_n^m)
//   L2L (parent side 2h, child h, e = (c_child - c_parent)/h):
//     Lt_j^k(child) = sum_{n,m} 2^-(n+1) Lt_n^m nu_n^m Rt_{n-j}^{m-k}(e) / (nu_{n-j}^{m-k} nu_j^k)
// These follow from the addition theorem Rt-form of R_n^m(a + b) =
// sum R_j^k(a) R_{n-j}^{m-k}(b) and I_n^m(D + rho) = sum (-1)^j
// conj(R_j^k(rho)) I_{n+j}^{m+k}(D) (standard solid-harmonic translation
// theorems for the Laplace kernel; the paper uses such expansions truncated
// to degrees 0..p_fmm-1, Section 3.9).
#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <vector>

#include "common.h"
#include "ops.h"
#include "../../include/bfm_debug.h"

namespace bfm {

using cplx = std::complex<double>;

// nu_n^m = sqrt((n-|m|)! (n+|m|)!) for n < 2 kMaxP, tabulated once.
static const std::vector<double> &nu_table() {
    static const std::vector<double> tab = [] {
        const int N = 2 * kMaxP;
        std::vector<long double> f(2 * N + 1, 1.0L);
        for (int i = 2; i <= 2 * N; ++i) f[i] = f[i - 1] * (long double)i;
        std::vector<double> t((size_t)N * N, 0.0);
        for (int n = 0; n < N; ++n)
            for (int m = 0; m <= n; ++m) t[(size_t)n * N + m] = (double)sqrtl(f[n - m] * f[n + m]);
        return t;
    }();
    return tab;
}

static double nu(int n, int m) {
    if (m < 0) m = -m;
    return nu_table()[(size_t)n * (2 * kMaxP) + m];
}

static inline int tri_index(int n, int m) { return n * (n + 1) / 2 + m; }

// Regular (irregular = false) or irregular normalised harmonics of degrees
// 0..nmax-1, orders m >= 0, at (x, y, z); out indexed by tri_index.
static void harmonics(bool irregular, int nmax, double x, double y, double z, std::vector<cplx> &out) {
    out.assign((size_t)nmax * (nmax + 1) / 2, cplx(0.0, 0.0));
    const double r2 = x * x + y * y + z * z;
    const cplx xy(x, y);
    cplx diag = irregular ? cplx(1.0 / std::sqrt(r2), 0.0) : cplx(1.0, 0.0);
    for (int m = 0; m < nmax; ++m) {
        if (m > 0) {
            double f = std::sqrt((2.0 * m - 1.0) / (2.0 * m));
            diag = irregular ? diag * xy * (f / r2) : diag * xy * f;
        }
        out[tri_index(m, m)] = diag;
        for (int n = m + 1; n < nmax; ++n) {
            const double a = std::sqrt((double)(n - m) * (n + m));
            const double b = (n - m - 1 > 0) ? std::sqrt((double)(n - m - 1) * (n + m - 1)) : 0.0;
            cplx prev2 = (n - 2 >= m) ? out[tri_index(n - 2, m)] : cplx(0.0, 0.0);
            cplx v;
            if (irregular)
                v = ((2.0 * n - 1.0) * z * out[tri_index(n - 1, m)] - b * prev2) / (r2 * a);
            else
                v = ((2.0 * n - 1.0) * z * out[tri_index(n - 1, m)] - r2 * b * prev2) / a;
            out[tri_index(n, m)] = v;
        }
    }
}

// Value of order m (any sign) from the m >= 0 table.
static cplx at(const std::vector<cplx> &t, int n, int m) {
    if (m >= 0) return t[tri_index(n, m)];
    cplx v = std::conj(t[tri_index(n, -m)]);
    return ((-m) & 1) ? -v : v;
}

// Fill the real P x P matrix (row-major, T[row * P + col]) of the real-linear
// map out_j^k = sum_{n,m} G(j, k, n, m) in_n^m over the full coefficient
// set, given inputs and outputs in the packed layout of common.h.
template <class Gfn>
static void fill_real(int p, Gfn G, double *T) {
    const int P = p * p;
    for (int i = 0; i < P * P; ++i) T[i] = 0.0;
    for (int j = 0; j < p; ++j) {
        for (int k = 0; k <= j; ++k) {
            const int row_re = (k == 0) ? j * j : j * j + 2 * k - 1;
            const int row_im = j * j + 2 * k;
            for (int n = 0; n < p; ++n) {
                for (int m = 0; m <= n; ++m) {
                    if (m == 0) {
                        cplx c = G(j, k, n, 0);
                        T[row_re * P + n * n] = c.real();
                        if (k > 0) T[row_im * P + n * n] = c.imag();
                    } else {
                        const double sgn = (m & 1) ? -1.0 : 1.0;
                        cplx gp = G(j, k, n, m), gm = G(j, k, n, -m);
                        cplx cre = gp + sgn * gm;
                        cplx cim = cplx(0.0, 1.0) * (gp - sgn * gm);
                        const int col_re = n * n + 2 * m - 1, col_im = n * n + 2 * m;
                        T[row_re * P + col_re] = cre.real();
                        T[row_re * P + col_im] = cim.real();
                        if (k > 0) {
                            T[row_im * P + col_re] = cre.imag();
                            T[row_im * P + col_im] = cim.imag();
                        }
                    }
                }
            }
        }
    }
}

static void octant_offset(int octant, double e[3]) {
    e[0] = ((octant >> 2) & 1) ? 0.5 : -0.5;
    e[1] = ((octant >> 1) & 1) ? 0.5 : -0.5;
    e[2] = (octant & 1) ? 0.5 : -0.5;
}

void build_m2m(int p, int octant, double *T) {
    double e[3];
    octant_offset(octant, e);
    std::vector<cplx> R;
    harmonics(false, p, e[0], e[1], e[2], R);
    auto G = [&](int n, int m, int j, int k) -> cplx {
        // output (n, m) from input (j, k)
        const int dn = n - j, dm = m - k;
        if (dn < 0 || std::abs(dm) > dn) return cplx(0.0, 0.0);
        return std::ldexp(1.0, -n) * nu(n, m) * std::conj(at(R, dn, dm)) / (nu(j, k) * nu(dn, dm));
    };
    fill_real(p, G, T);
}

void build_l2l(int p, int octant, double *T) {
    double e[3];
    octant_offset(octant, e);
    std::vector<cplx> R;
    harmonics(false, p, e[0], e[1], e[2], R);
    auto G = [&](int j, int k, int n, int m) -> cplx {
        const int dn = n - j, dm = m - k;
        if (dn < 0 || std::abs(dm) > dn) return cplx(0.0, 0.0);
        return std::ldexp(1.0, -(n + 1)) * nu(n, m) * at(R, dn, dm) / (nu(dn, dm) * nu(j, k));
    };
    fill_real(p, G, T);
}

// Operator order: by squared offset length d^2 (nearest first), then
// lexicographic in (dx, dy, dz), so that the offsets of one distance class
// (m2l_class) are one contiguous range of operator indices.
static const std::vector<std::array<int, 3>> &m2l_offsets() {
    static const std::vector<std::array<int, 3>> list = [] {
        std::vector<std::array<int, 3>> v;
        for (int a = -3; a <= 3; ++a)
            for (int b = -3; b <= 3; ++b)
                for (int c = -3; c <= 3; ++c) {
                    if (a >= -1 && a <= 1 && b >= -1 && b <= 1 && c >= -1 && c <= 1) continue;
                    v.push_back({a, b, c});
                }
        std::stable_sort(v.begin(), v.end(), [](const std::array<int, 3> &x, const std::array<int, 3> &y) {
            return x[0] * x[0] + x[1] * x[1] + x[2] * x[2] < y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
        });
        return v;
    }();
    return list;
}

int m2l_op_index(int dx, int dy, int dz) {
    if (dx < -3 || dx > 3 || dy < -3 || dy > 3 || dz < -3 || dz > 3) return -1;
    if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1) return -1;
    const auto &v = m2l_offsets();
    for (size_t i = 0; i < v.size(); ++i)
        if (v[i][0] == dx && v[i][1] == dy && v[i][2] == dz) return (int)i;
    return -1;
}

void m2l_op_offset(int op, int d[3]) {
    const auto &v = m2l_offsets();
    if (op < 0 || op >= (int)v.size()) {
        d[0] = d[1] = d[2] = 0;
        return;
    }
    d[0] = v[op][0];
    d[1] = v[op][1];
    d[2] = v[op][2];
}

int m2l_class_first_op(int cls) {
    // classes: d^2 <= 5, 6 <= d^2 <= 10, d^2 >= 11
    const auto &v = m2l_offsets();
    const int lim[3] = {0, 6, 11};
    if (cls >= 3) return (int)v.size();
    for (size_t i = 0; i < v.size(); ++i) {
        const int d2 = v[i][0] * v[i][0] + v[i][1] * v[i][1] + v[i][2] * v[i][2];
        if (d2 >= lim[cls]) return (int)i;
    }
    return (int)v.size();
}

static_assert(m2l_class_order(20, 0) == 20 && m2l_class_order(20, 1) == 16 && m2l_class_order(20, 2) == 12,
              "class orders at p = 20");
static_assert(m2l_class_order(16, 1) == 16 && m2l_class_order(16, 2) == 12 && m2l_class_order(12, 1) == 12 &&
                  m2l_class_order(12, 2) == 8 && m2l_class_order(8, 1) == 8 && m2l_class_order(8, 2) == 8 &&
                  m2l_class_order(4, 1) == 4 && m2l_class_order(4, 2) == 4,
              "class orders");

// M2L for any real offset d (box units).
static void build_m2l_at(int p, const double d[3], double *T) {
    std::vector<cplx> I;
    harmonics(true, 2 * p - 1, d[0], d[1], d[2], I);
    auto G = [&](int j, int k, int n, int m) -> cplx {
        const int sgn = ((j + k) & 1) ? -1 : 1;
        return (double)sgn * at(I, n + j, m - k) * nu(n + j, m - k) / (nu(j, k) * nu(n, m));
    };
    fill_real(p, G, T);
}

void build_m2l(int p, int op, double *T) {
    int d[3];
    m2l_op_offset(op, d);
    const double dd[3] = {(double)d[0], (double)d[1], (double)d[2]};
    build_m2l_at(p, dd, T);
}

// ---------------------------------------------------------------------------
// Rotation-factored M2L: T(d) = B T(|d| z) A. A rotation Q with Q d = |d| z
// turns the source's multipole coefficients into those of the rotated
// configuration (A, block diagonal by degree: a rotation keeps the degree),
// the translation along z couples only equal orders (T_z, one real block
// per order m shared by the cosine and sine parts), and B takes the local
// coefficients of the rotated frame back (block diagonal by degree).
// Per degree n the blocks follow from the harmonics at points of the unit
// sphere: a multipole of a unit source at y has packed coefficients
// a(y) = (R_n^0, Re R_n^m, -Im R_n^m, ...)(y) (the conjugates of the regular
// harmonics), so A a(y) = a(Q y); a local expansion is evaluated against
// e(x) = (R_n^0, 2 Re R_n^m, -2 Im R_n^m, ...)(x), and with e(Q x) = W e(x)
// the original frame's coefficients are B L' = W^T L'. The packed parts are
// mutually orthogonal on the sphere, so with a product rule exact for
// degree 2n (Gauss-Legendre in cos(theta) x uniform in phi) each block is a
// sum over the rule's nodes divided by a diagonal Gram matrix: no linear
// solve.

static void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) {
                p1 = z;
                p0 = 1.0;
            }
            const double dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) {
                double q0 = 1.0, q1 = z;
                for (int k = 2; k <= n; ++k) {
                    const double q2 = ((2.0 * k - 1.0) * z * q1 - (k - 1.0) * q0) / k;
                    q0 = q1;
                    q1 = q2;
                }
                const double dq = n * (z * q1 - q0) / (z * z - 1.0);
                x[i] = z;
                w[i] = 2.0 / ((1.0 - z * z) * dq * dq);
                break;
            }
        }
    }
}

// A rotation (row-major 3 x 3) taking the unit vector u to +z.
static void rotation_to_z(const double u[3], double Q[9]) {
    const double c = u[2];
    const double kx = u[1], ky = -u[0];  // u x z
    const double sn = std::sqrt(kx * kx + ky * ky);
    if (sn < 1e-15) {
        const double sg = c > 0.0 ? 1.0 : -1.0;  // identity, or a half turn about x
        const double Z[9] = {1, 0, 0, 0, sg, 0, 0, 0, sg};
        for (int i = 0; i < 9; ++i) Q[i] = Z[i];
        return;
    }
    const double ax = kx / sn, ay = ky / sn;  // axis (ax, ay, 0), angle theta: cos = c, sin = sn
    const double t = 1.0 - c;
    Q[0] = c + ax * ax * t;
    Q[1] = ax * ay * t;
    Q[2] = ay * sn;
    Q[3] = ax * ay * t;
    Q[4] = c + ay * ay * t;
    Q[5] = -ax * sn;
    Q[6] = -ay * sn;
    Q[7] = ax * sn;
    Q[8] = c;
}

int m2l_rot_offset(int n) { return n * (4 * n * n - 1) / 3; }
int m2l_tz_offset(int p, int m) {
    int o = 0;
    for (int q = 0; q < m; ++q) o += (p - q) * (p - q);
    return o;
}

// Packed part c (0: order 0; 2m - 1, 2m: the two parts of order m) of the
// multipole-type (conjugate, unit weights) or local-type (weights 2, minus
// sign on the sine part) vector of degree n.
static double packed_part(const std::vector<cplx> &R, int n, int c, bool local) {
    if (c == 0) return R[tri_index(n, 0)].real();
    const int m = (c + 1) / 2;
    const cplx v = R[tri_index(n, m)];
    const double f = local ? 2.0 : 1.0;
    return (c & 1) ? f * v.real() : -f * v.imag();
}

void build_m2l_rot(int p, int op, double *A, double *Tz, double *B) {
    int di[3];
    m2l_op_offset(op, di);
    const double len = std::sqrt((double)(di[0] * di[0] + di[1] * di[1] + di[2] * di[2]));
    const double u[3] = {di[0] / len, di[1] / len, di[2] / len};
    double Q[9];
    rotation_to_z(u, Q);
    // product rule exact for degree 2 (p - 1)
    std::vector<double> gx, gw;
    gauss_legendre(p, gx, gw);
    const int nphi = 2 * p;
    const int K = p * nphi;
    std::vector<std::vector<cplx>> Hx(K), Hq(K);
    std::vector<double> wk(K);
    for (int a = 0; a < p; ++a)
        for (int b = 0; b < nphi; ++b) {
            const int k = a * nphi + b;
            const double z = gx[a], r = std::sqrt(std::max(0.0, 1.0 - z * z)), ph = 2.0 * M_PI * b / nphi;
            const double x[3] = {r * std::cos(ph), r * std::sin(ph), z};
            const double q[3] = {Q[0] * x[0] + Q[1] * x[1] + Q[2] * x[2], Q[3] * x[0] + Q[4] * x[1] + Q[5] * x[2],
                                 Q[6] * x[0] + Q[7] * x[1] + Q[8] * x[2]};
            harmonics(false, p, x[0], x[1], x[2], Hx[k]);
            harmonics(false, p, q[0], q[1], q[2], Hq[k]);
            wk[k] = gw[a] * (2.0 * M_PI / nphi);
        }
    for (int n = 0; n < p; ++n) {
        const int sz = 2 * n + 1;
        double *An = A + m2l_rot_offset(n), *Bn = B + m2l_rot_offset(n);
        std::vector<double> ga(sz, 0.0), ge(sz, 0.0);
        for (int i = 0; i < sz * sz; ++i) An[i] = Bn[i] = 0.0;
        std::vector<double> ax(sz), aq(sz), ex(sz), eq(sz);
        for (int k = 0; k < K; ++k) {
            for (int c = 0; c < sz; ++c) {
                ax[c] = packed_part(Hx[k], n, c, false);
                aq[c] = packed_part(Hq[k], n, c, false);
                ex[c] = packed_part(Hx[k], n, c, true);
                eq[c] = packed_part(Hq[k], n, c, true);
            }
            for (int c = 0; c < sz; ++c) {
                ga[c] += wk[k] * ax[c] * ax[c];
                ge[c] += wk[k] * ex[c] * ex[c];
                for (int c2 = 0; c2 < sz; ++c2) {
                    An[c * sz + c2] += wk[k] * aq[c] * ax[c2];  // sum w a(Qx) a(x)^T
                    Bn[c2 * sz + c] += wk[k] * eq[c] * ex[c2];  // (sum w e(Qx) e(x)^T)^T
                }
            }
        }
        for (int c = 0; c < sz; ++c)
            for (int c2 = 0; c2 < sz; ++c2) {
                An[c * sz + c2] /= ga[c2];
                Bn[c2 * sz + c] /= ge[c2];
            }
    }
    // translation along +z by |d|
    const int P = p * p;
    std::vector<double> Tfull((size_t)P * P);
    const double dz[3] = {0.0, 0.0, len};
    build_m2l_at(p, dz, Tfull.data());
    for (int m = 0; m < p; ++m) {
        double *Tm = Tz + m2l_tz_offset(p, m);
        const int w = p - m;
        for (int j = m; j < p; ++j)
            for (int n = m; n < p; ++n) {
                const int row = m == 0 ? j * j : j * j + 2 * m - 1, col = m == 0 ? n * n : n * n + 2 * m - 1;
                Tm[(j - m) * w + (n - m)] = Tfull[(size_t)row * P + col];
            }
    }
}

}  // namespace bfm

extern "C" int bfm_debug_operator(int p, int kind, int index, double *out, int *d_out) {
    if (!out || p < 1 || p > bfm::kMaxP) return BFM_EINVAL;
    if (kind == 0 || kind == 1) {
        if (index < 0 || index > 7) return BFM_EINVAL;
        if (kind == 0)
            bfm::build_m2m(p, index, out);
        else
            bfm::build_l2l(p, index, out);
        return BFM_OK;
    }
    if (kind == 2) {
        if (index < 0 || index >= bfm::kNumM2LOps) return BFM_EINVAL;
        bfm::build_m2l(p, index, out);
        if (d_out) bfm::m2l_op_offset(index, d_out);
        return BFM_OK;
    }
    if (kind == 3) {  // the rotation-factored M2L: A, then T_z, then B, concatenated
        if (index < 0 || index >= bfm::kNumM2LOps) return BFM_EINVAL;
        const int nr = bfm::m2l_rot_offset(p), nz = bfm::m2l_tz_offset(p, p);
        bfm::build_m2l_rot(p, index, out, out + nr, out + nr + nz);
        if (d_out) bfm::m2l_op_offset(index, d_out);
        return BFM_OK;
    }
    return BFM_EINVAL;
}
