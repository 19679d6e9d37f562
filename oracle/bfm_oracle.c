/*
 * CPU FP64 oracle for the boundary-element operators of the paper
 * "GPU accelerated fast multipole boundary element method for simulation of
 * 3D bubble dynamics in potential flow" (Gumerov, Pityuk, Abramova, Akhatov).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark use it. It shares no code with the GPU library.
 *
 * Everything here is the plain definition, written out as direct O(N^2)
 * sums in double precision, one receiver at a time, with the source loop in
 * index order (no blocking, no expansions, no reordering). OpenMP only
 * splits the receiver loop across threads; each receiver's sum is computed
 * by one thread in a fixed order, so results do not depend on the thread
 * count. Built without FMA contraction (-ffp-contract=off).
 *
 * Notation follows the paper:
 *   G(r, r')        = 1 / (4 pi |r - r'|)                      (eq2_13)
 *   dG/dn'(r, r')   = n' . (r - r') / (4 pi |r - r'|^3)        (eq2_13)
 *   L_ij = s_j G(r_i, r_j),  M_ij = s_j dG/dn_j(r_i, r_j), i != j  (ns1)
 *   s_j = (1/3) sum_{k contains j} A_k,  n_j = m_j/|m_j|,
 *   m_j = sum_{k contains j} N_k A_k                            (ns1)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define FOUR_PI 12.566370614359172953850573533118

int bfmo_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Vertex weights and normals of the nodal quadrature (ns1, Section 3.2).
 * For triangle k with vertices (r1, r2, r3):
 *   c_k = (r2 - r1) x (r3 - r1),  A_k = |c_k| / 2,  N_k = c_k / |c_k|,
 * so N_k A_k = c_k / 2. Each vertex collects A_k / 3 into s_j and N_k A_k
 * into m_j. Returns 0, or -5 when a triangle has zero area or a vertex ends
 * with |m_j| = 0, or -1 on an index out of range.
 */
int bfmo_geometry(int64_t nv, const double *xyz, int64_t nt, const int32_t *tri,
                  double *s, double *n, double *area) {
    memset(s, 0, sizeof(double) * (size_t)nv);
    memset(n, 0, sizeof(double) * 3 * (size_t)nv);
    for (int64_t k = 0; k < nt; ++k) {
        int32_t a = tri[3 * k], b = tri[3 * k + 1], c = tri[3 * k + 2];
        if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv) return -1;
        double e1[3], e2[3], ck[3];
        for (int d = 0; d < 3; ++d) {
            e1[d] = xyz[3 * b + d] - xyz[3 * a + d];
            e2[d] = xyz[3 * c + d] - xyz[3 * a + d];
        }
        ck[0] = e1[1] * e2[2] - e1[2] * e2[1];
        ck[1] = e1[2] * e2[0] - e1[0] * e2[2];
        ck[2] = e1[0] * e2[1] - e1[1] * e2[0];
        double len = sqrt(ck[0] * ck[0] + ck[1] * ck[1] + ck[2] * ck[2]);
        if (!(len > 0.0)) return -5;
        double A = 0.5 * len;
        if (area) area[k] = A;
        const int32_t v[3] = {a, b, c};
        for (int t = 0; t < 3; ++t) {
            s[v[t]] += A / 3.0;
            for (int d = 0; d < 3; ++d) n[3 * v[t] + d] += 0.5 * ck[d]; /* N_k A_k */
        }
    }
    for (int64_t j = 0; j < nv; ++j) {
        double *m = n + 3 * j;
        double len = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
        if (!(len > 0.0)) return -5;
        m[0] /= len;
        m[1] /= len;
        m[2] /= len;
    }
    return 0;
}

/*
 * Direct sums over all sources j != i for each requested receiver i
 * (Sections 3.3 and 3.1):
 *   SM[i]  = sum_{j!=i} M_ij                       (enters s3)
 *   VM[i]  = sum_{j!=i} M_ij (r_j - r_i)           (s4/s5, translation-free)
 *   PM[i]  = sum_{j!=i} M_ij r_j                   (s5 as printed)
 *   VL[i]  = sum_{j!=i} L_ij n_j                   (s4/s5)
 *   B[i]   = sum_{j!=i} M_ij (phi_j - phi_i)       (b of eq3_1 with s3)
 * rows: receiver indices (nr of them); outputs are indexed by position in rows.
 * phi may be NULL (then B is not written).
 */
void bfmo_sums(int64_t nv, const double *xyz, const double *s, const double *n,
               const double *phi, int64_t nr, const int64_t *rows,
               double *SM, double *VM, double *PM, double *VL, double *B) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nr; ++t) {
        const int64_t i = rows[t];
        const double xi = xyz[3 * i], yi = xyz[3 * i + 1], zi = xyz[3 * i + 2];
        double sm = 0.0, vm[3] = {0, 0, 0}, pm[3] = {0, 0, 0}, vl[3] = {0, 0, 0}, bb = 0.0;
        for (int64_t j = 0; j < nv; ++j) {
            if (j == i) continue;
            const double dx = xi - xyz[3 * j], dy = yi - xyz[3 * j + 1], dz = zi - xyz[3 * j + 2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double r = sqrt(r2);
            const double Lij = s[j] / (FOUR_PI * r);
            const double Mij = s[j] * (n[3 * j] * dx + n[3 * j + 1] * dy + n[3 * j + 2] * dz) /
                               (FOUR_PI * r2 * r);
            sm += Mij;
            /* r_j - r_i = -(dx, dy, dz) */
            vm[0] -= Mij * dx;
            vm[1] -= Mij * dy;
            vm[2] -= Mij * dz;
            pm[0] += Mij * xyz[3 * j];
            pm[1] += Mij * xyz[3 * j + 1];
            pm[2] += Mij * xyz[3 * j + 2];
            vl[0] += Lij * n[3 * j];
            vl[1] += Lij * n[3 * j + 1];
            vl[2] += Lij * n[3 * j + 2];
            if (phi) bb += Mij * (phi[j] - phi[i]);
        }
        if (SM) SM[t] = sm;
        for (int d = 0; d < 3; ++d) {
            if (VM) VM[3 * t + d] = vm[d];
            if (PM) PM[3 * t + d] = pm[d];
            if (VL) VL[3 * t + d] = vl[d];
        }
        if (B && phi) B[t] = bb;
    }
}

/*
 * Off-diagonal part of A = f L + g M (eq3_27) applied to (x, y):
 *   out[t] = sum_{j != i} ( f L_ij x_j + g M_ij y_j ),  i = rows[t].
 * x or y may be NULL when f or g is zero.
 */
void bfmo_offdiag_mvp(int64_t nv, const double *xyz, const double *s, const double *n,
                      double f, const double *x, double g, const double *y,
                      int64_t nr, const int64_t *rows, double *out) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nr; ++t) {
        const int64_t i = rows[t];
        const double xi = xyz[3 * i], yi = xyz[3 * i + 1], zi = xyz[3 * i + 2];
        double acc = 0.0;
        for (int64_t j = 0; j < nv; ++j) {
            if (j == i) continue;
            const double dx = xi - xyz[3 * j], dy = yi - xyz[3 * j + 1], dz = zi - xyz[3 * j + 2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double r = sqrt(r2);
            double v = 0.0;
            if (f != 0.0) v += f * (s[j] / (FOUR_PI * r)) * x[j];
            if (g != 0.0)
                v += g * (s[j] * (n[3 * j] * dx + n[3 * j + 1] * dy + n[3 * j + 2] * dz) /
                          (FOUR_PI * r2 * r)) * y[j];
            acc += v;
        }
        out[t] = acc;
    }
}

/*
 * Dense off-diagonal matrices (small meshes only): L[i*nv + j] = L_ij and
 * M[i*nv + j] = M_ij for i != j, zero on the diagonal.
 */
void bfmo_dense(int64_t nv, const double *xyz, const double *s, const double *n,
                double *L, double *M) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nv; ++i) {
        for (int64_t j = 0; j < nv; ++j) {
            if (j == i) {
                L[i * nv + j] = 0.0;
                M[i * nv + j] = 0.0;
                continue;
            }
            const double dx = xyz[3 * i] - xyz[3 * j], dy = xyz[3 * i + 1] - xyz[3 * j + 1],
                         dz = xyz[3 * i + 2] - xyz[3 * j + 2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double r = sqrt(r2);
            L[i * nv + j] = s[j] / (FOUR_PI * r);
            M[i * nv + j] = s[j] * (n[3 * j] * dx + n[3 * j + 1] * dy + n[3 * j + 2] * dz) /
                            (FOUR_PI * r2 * r);
        }
    }
}
