// Translation operators of the fast multipole method (host construction).
#pragma once

namespace bfm {

// Child octant o = 4*(ix & 1) + 2*(iy & 1) + (iz & 1) of the child's integer
// box coordinates; the child centre sits at (c_parent + (b - 1/2) h_child).
// Each builder writes a real p^2 x p^2 matrix, row-major: T[row * P + col].
void build_m2m(int p, int octant, double *T);
void build_l2l(int p, int octant, double *T);

// Multipole-to-local operators: 316 offsets d = (c_target - c_source)/h with
// components in [-3, 3] and not all in [-1, 1].
int m2l_op_index(int dx, int dy, int dz);  // -1 when d is not a far offset
void m2l_op_offset(int op, int d[3]);
void build_m2l(int p, int op, double *T);

}  // namespace bfm
