/*
 * Learned initial guess for the GMRES solve of bfm.h.
 *
 * Not part of the paper: the paper starts GMRES from the previous time
 * step's q (Section 3.6). This network predicts q of every bubble from its
 * shape and potential, and the solve then runs to the same tolerance, so the
 * prediction changes the iteration count only, never the solution.
 *
 * Features of bubble b (174 values, FP32): the real spherical-harmonic
 * coefficients of degree <= 8 (81 each) of |r_i - c_b| / a_b and of phi_i,
 * then the offsets of the 4 nearest other bubble centres divided by a_b (12;
 * zero where fewer exist; ties go to the lower bubble index). c_b is the
 * vertex mean, a_b = sqrt(area_b / 4 pi) with area_b the sum of the vertex
 * weights s_i (Section 3.2, ns1). Target (81): the coefficients of a_b q_i.
 * Coefficients come from the weighted least-squares projector
 * (G^T W G)^{-1} G^T W of the sphere template (bfm_set_sphere_template; W =
 * template vertex areas, one third of every incident flat triangle on the
 * unit directions), with harmonics orthonormal on the unit sphere, no
 * Condon-Shortley phase, ordered by degree n: slot n^2 for order 0, slots
 * n^2 + 2m - 1 / n^2 + 2m for the cos(m lon) / sin(m lon) parts of order m.
 * The guess is q_i = (G c)_i / a_b for predicted coefficients c.
 *
 * Network: 174 -> 512 -> 512 -> 512 -> 81, SiLU between layers, inputs and
 * targets standardised per column ((v - mu) / sd), loss 0.5 * mean over rows
 * of the squared error of the standardised outputs. Weights and layer inputs
 * are stored as BF16 for the matrix products (v_mfma_f32_16x16x32_bf16, FP32
 * accumulation), master weights and Adam moments (beta1 0.9, beta2 0.999,
 * eps 1e-8, bias-corrected) in FP32.
 *
 * Parameter layout (host FP32, BFM_MLP_NUM_PARAMS values): for each layer
 * k = 0..3 the weights W_k [in_k][out_k] row-major (y = x W_k + b_k), then
 * b_k [out_k]. Standardisation layout (BFM_MLP_NORM_SIZE values): mu_x [174],
 * sd_x [174], mu_y [81], sd_y [81]; sd > 0.
 *
 * All calls return BFM_OK or a BFM_E* code (bfm_last_error has the message).
 * Host arrays are read or written before the call returns; the handle owns
 * every device buffer. Calls on one handle must not overlap.
 */
#ifndef BFM_MLP_H
#define BFM_MLP_H

#include "bfm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define BFM_MLP_INPUTS 174
#define BFM_MLP_OUTPUTS 81
#define BFM_MLP_HIDDEN 512
#define BFM_MLP_NUM_PARAMS 656465
#define BFM_MLP_NORM_SIZE 510

/* Random initial weights (normal, sd 1 / sqrt(fan-in); biases 0), Adam state
 * cleared. Standardisation is left as set, or identity if never set. */
int bfm_mlp_init(bfm_ctx *ctx, uint64_t seed);

/* Replace (set) or read (get) all weights and biases; set clears Adam state. */
int bfm_mlp_set_params(bfm_ctx *ctx, const float *params);
int bfm_mlp_get_params(bfm_ctx *ctx, float *params);

/* Standardisation statistics. bfm_mlp_fit computes them from the training
 * set on its first call unless they were set here. */
int bfm_mlp_set_norm(bfm_ctx *ctx, const float *norm);
int bfm_mlp_get_norm(bfm_ctx *ctx, float *norm);

/* Network on host rows: x [rows][174] -> y [rows][81], standardisation
 * applied on both ends. 1 <= rows <= 2^24. */
int bfm_mlp_forward(bfm_ctx *ctx, int64_t rows, const float *x, float *y);

/* Loss and gradients over host rows x [rows][174], targets t [rows][81]
 * (unstandardised): grad [BFM_MLP_NUM_PARAMS] in the parameter layout,
 * *loss the mean loss. The gradients are kept for bfm_mlp_adam_step. */
int bfm_mlp_gradient(bfm_ctx *ctx, int64_t rows, const float *x, const float *t, float *grad, double *loss);

/* One Adam step with the last gradients (learning rate lr > 0). */
int bfm_mlp_adam_step(bfm_ctx *ctx, float lr);

/* Features [nb][174] and, if q and targ are non-NULL, targets [nb][81] of
 * the current surface and phi (host FP64 [nv]); FP32 host outputs. */
int bfm_mlp_features(bfm_ctx *ctx, const double *phi, const double *q, float *feat, float *targ);

/* Append one sample per bubble (features of the current surface and phi_dev,
 * targets from the solved q_dev; device FP64 [nv]) to the training set held
 * on the device. */
int bfm_mlp_collect_dev(bfm_ctx *ctx, const double *phi_dev, const double *q_dev);

/* Rows in the training set; clear != 0 empties it first. */
int bfm_mlp_dataset(bfm_ctx *ctx, int clear, int64_t *rows);

/* Train on the device: epochs passes over the training set in shuffled
 * (seeded) order, full batches of `batch` rows, one Adam step each at rate
 * lr. Initialises the network first if needed. *loss = mean loss of the
 * last epoch (may be NULL). */
int bfm_mlp_fit(bfm_ctx *ctx, int epochs, int batch, float lr, uint64_t seed, double *loss);

/* Predicted q for the current surface and phi (device or host FP64 [nv]). */
int bfm_mlp_guess_dev(bfm_ctx *ctx, const double *phi_dev, double *q_dev);
int bfm_mlp_guess(bfm_ctx *ctx, const double *phi, double *q);

#ifdef __cplusplus
}
#endif

#endif
