// Translation operators of the fast multipole method (host construction).
#pragma once

namespace bfm {

// Child octant o = 4*(ix & 1) + 2*(iy & 1) + (iz & 1) of the child's integer
// box coordinates; the child centre sits at (c_parent + (b - 1/2) h_child).
// Each builder writes a real p^2 x p^2 matrix, row-major: T[row * P + col].
void build_m2m(int p, int octant, double *T);
void build_l2l(int p, int octant, double *T);

// Multipole-to-local operators: 316 offsets d = (c_target - c_source)/h with
// components in [-3, 3] and not all in [-1, 1], numbered by |d|^2 (nearest
// first), then lexicographically.
int m2l_op_index(int dx, int dy, int dz);  // -1 when d is not a far offset
void m2l_op_offset(int op, int d[3]);
// Distance classes of the offsets (|d|^2 <= 5, 6..10, >= 11; contiguous
// operator ranges): first operator of class cls (cls = 3: 316), and the
// expansion order used for that class when a product of order p reduces the
// order of distant translations: p, then 4 ceil(p/5) and 4 ceil(3p/20)
// (about 0.8 p and 0.6 p rounded up to multiples of 4: at p = 20 the orders
// 20, 16, 12; at p = 16: 16, 16, 12; at p = 12: 12, 12, 8). A translation's
// truncation error falls like (c/|d|)^p, and the effective ratio measured
// on the nearest offsets (about 0.47 per degree at |d| = 2) puts the orders
// that match the nearest class's error at about 0.8 p for |d|^2 = 6 and
// 0.6 p for |d|^2 = 11.
int m2l_class_first_op(int cls);
constexpr int m2l_class_order(int p, int cls) {
    return cls <= 0 ? p : (cls == 1 ? 4 * ((p + 4) / 5) : 4 * ((3 * p + 19) / 20));
}
constexpr int kM2LClasses = 3;
void build_m2l(int p, int op, double *T);
// Rotation-factored M2L of operator op: T = B T_z A (see ops.cpp). A and B:
// one row-major (2n+1) x (2n+1) block per degree n < p at m2l_rot_offset(n)
// (m2l_rot_offset(p) doubles in all); T_z: one row-major (p-m) x (p-m)
// block per order m < p (rows j = m..p-1, columns n = m..p-1) at
// m2l_tz_offset(p, m) (m2l_tz_offset(p, p) in all), applied alike to the
// two parts of an order m > 0. Within a degree the packed parts are ordered
// as in the expansions: order 0, then (2m - 1, 2m) for order m.
int m2l_rot_offset(int n);
int m2l_tz_offset(int p, int m);
void build_m2l_rot(int p, int op, double *A, double *Tz, double *B);

}  // namespace bfm
