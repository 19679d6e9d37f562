/*
 * bfm_debug.h - introspection of libbfm for tests.
 *
 * The fast multipole translations of the paper's FMM (Section 3.9:
 * multipole and local expansions of degrees 0..p_fmm-1, translated between
 * boxes of the octree) are stored by libbfm as dense real p^2 x p^2
 * matrices in a normalised, box-scaled basis. This call exposes one of them
 * so that tests can check it against independent expansions on the CPU.
 */
#ifndef BFM_DEBUG_H
#define BFM_DEBUG_H

#ifdef __cplusplus
extern "C" {
#endif

/*
 * kind 0: multipole-to-multipole, child octant `index` (0..7) -> parent
 * kind 1: local-to-local, parent -> child octant `index` (0..7)
 * kind 2: multipole-to-local, offset operator `index` (0..315)
 * kind 3: the same operator factored by rotation, T = B T_z A: out receives
 *   A (for every degree n < p a row-major (2n+1) x (2n+1) block, blocks in
 *   order of n; p (4 p^2 - 1) / 3 doubles), then T_z (for every order
 *   m < p a row-major (p-m) x (p-m) block over degrees m..p-1, applied
 *   alike to the cosine and sine parts of the order; p (p+1)(2p+1) / 6
 *   doubles), then B (as A): A rotates the multipole coefficients to a
 *   frame whose z axis points along d, T_z translates along that axis, B
 *   rotates the local coefficients back.
 * Octant o: child box integer coordinates have low bits (o>>2 & 1, o>>1 & 1,
 * o & 1). Offset operator k: the k-th (dx, dy, dz) of [-3,3]^3 excluding
 * [-1,1]^3, ordered by dx^2 + dy^2 + dz^2 and then lexicographically,
 * meaning c_target - c_source = d * h.
 * out: host, p^2 * p^2 doubles, row-major (out[row * p^2 + col]) for
 * kinds 0..2.
 * d_out (may be NULL): for kind 2 receives the offset (dx, dy, dz).
 * Returns 0, or -1 (BFM_EINVAL) on a bad p, kind or index.
 */
int bfm_debug_operator(int p, int kind, int index, double *out, int *d_out);

/*
 * Device dense kernels on host data, for tests (need a GPU):
 * bfm_debug_dgemm: C = A B with the library's FP64 MFMA GEMM; A [M x K],
 * B [K x N], C [M x N], all column-major host arrays.
 * bfm_debug_spd_inverse: the library's in-place blocked Gauss-Jordan inverse
 * (no pivoting) of a symmetric positive definite n x n column-major matrix,
 * as used for the coarse correction of BFM_PRECOND_SH_COARSE.
 * Return BFM_OK or a BFM_E* code (message in bfm_last_error()).
 */
int bfm_debug_dgemm(int device, int M, int N, int K, const double *A, const double *B, double *C);
int bfm_debug_spd_inverse(int device, int n, const double *A, double *Ainv);

/*
 * Ceiling probe: one launch of a kernel that issues a single instruction mix
 * back to back on every CU (4096 workgroups of 256 lanes, each lane `iters`
 * rounds), timed with HIP events after a warm-up launch, so that a hot
 * kernel's throughput can be compared with what the device delivers for
 * the same mix. kind: 0 FP64 MFMA (v_mfma_f64_16x16x4f64), 1 FP64 FMA,
 * 2 FP32 FMA (not packed), 3 the FP64 near-field pair step (r^2, the 1/sqrt
 * estimate with one Newton step, two fma; 11 algorithmic flops per pair),
 * 4 the FP32 pair step (estimate only), 5 BF16 MFMA
 * (v_mfma_f32_16x16x32_bf16). ms receives the launch time, ops the flops it
 * performed (pair probes: pairs x 11). Returns BFM_OK or BFM_EINVAL (kind
 * not 0..5, iters not in [1, 2^16]) / BFM_EDEVICE.
 */
int bfm_debug_probe(int device, int kind, int iters, double *ms, double *ops);

#ifdef __cplusplus
}
#endif

#endif /* BFM_DEBUG_H */
