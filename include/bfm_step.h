/*
 * Time-step harness of the bubble dynamics around the solve of bfm.h.
 *
 * One right-hand side evaluation follows Sections 2.1 and 3.4-3.7:
 *   1. shape filter of bandwidth p_f on r and phi (Section 3.7, eq3_24 and
 *      spherical6): per bubble, plain least squares onto the real
 *      spherical harmonics of degree 0..p_f-1 at the template directions
 *      (bfm_set_sphere_template), F = G (G^T G)^{-1} G^T; for toroidal
 *      bubbles (bfm_set_torus_template, spherical7) onto the real
 *      trigonometric basis of degree 0..p_f/2 in each template angle
 *      (p_f even, (p_f + 1)^2 functions);
 *   2. geometry (Section 3.2), bubble volumes V_m = sum over the bubble's
 *      triangles of r1 . (r2 x r3) / 6, mean curvature H by the paraboloid
 *      through five one-ring neighbours (Section 3.5, parab1/parab2; the
 *      first five in counter-clockwise order seen from outside, starting at
 *      the neighbour with the lowest index; local x axis along the tangential
 *      projection of the edge to that neighbour);
 *   3. q = dphi/dn from the solve of bfm.h (Section 3.1), started from the
 *      previous solve's q (Section 3.6), zero, or the learned guess;
 *   4. tangential velocity (eq3_10, eq3_11), v = n q + v_t, u = v + alpha v_t
 *      (eq3_13), dr/dt = u (eq3_14) and
 *      dphi/dt = (alpha v_t + v/2) . v - (p_g - 2 sigma H)/rho + g . r + p_inf(t)/rho
 *      (eq3_15), p_g = p_g0 (V0/V)^kappa, p_g0 = p0 + 2 sigma / a0 (eq2_8);
 *      p_inf(t) = p0 + forcing_sign * P_a * sin(2 pi t / T) (eq2_6 has sign -1);
 *   5. the filter again on dr/dt and dphi/dt.
 * Steps: fourth-order Runge-Kutta for the first five, then the sixth-order
 * Adams-Bashforth method (Section 3.6). V0 and a0 = (3 V0 / 4 pi)^(1/3) come
 * from the filtered state passed to bfm_state_set.
 *
 * Requirements: a mesh whose bubbles are copies of one triangulation of a
 * sphere or a torus (bubble b holds vertices b*nd .. b*nd+nd-1 and triangles
 * in the same local order), with the template set by bfm_set_sphere_template
 * or bfm_set_torus_template; every vertex has at least five neighbours.
 *
 * State (positions and potential) lives on the device; host arrays are
 * copied in or out before the call returns. Errors: BFM_EINVAL (bad
 * argument, no mesh/template/state), BFM_EMESH (mesh unsuitable), and the
 * codes of bfm_solve; the message is in bfm_last_error().
 */
#ifndef BFM_STEP_H
#define BFM_STEP_H

#include "bfm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bfm_physics {
    double rho;          /* liquid density */
    double p0;           /* static pressure */
    double sigma;        /* surface tension */
    double kappa;        /* polytropic exponent */
    double pa;           /* acoustic amplitude P_a */
    double period;       /* acoustic period T; 0 = no forcing */
    double forcing_sign; /* sign of the sine in p_inf (the paper's eq2_6: -1) */
    double g[3];         /* gravity acceleration */
    double alpha;        /* mesh velocity factor of eq3_13 (-1: u = n q) */
    int filter_degree;   /* p_f (degrees 0..p_f-1); 0 = no filter; p_f^2 <= nd */
    int guess;           /* BFM_GUESS_ZERO, BFM_GUESS_GIVEN (previous q) or BFM_GUESS_LEARNED */
    int collect;         /* != 0: every solve appends (features, targets) to the training set
                            of bfm_mlp.h */
} bfm_physics;

typedef struct bfm_step_info {
    int scheme;          /* 0 = RK4, 1 = AB6 */
    int solves;          /* right-hand side evaluations (solves) in this step */
    int iterations;      /* GMRES iterations summed over those solves */
    double t;            /* time after the step */
    double ms;           /* wall time of the step */
} bfm_step_info;

/* rho = p0 = 1, sigma = 0, kappa = 1.4, no forcing (forcing_sign -1),
 * g = 0, alpha = -1, p_f = 0, guess = BFM_GUESS_GIVEN, collect = 0. */
int bfm_default_physics(bfm_physics *ph);

/* Set the physics; clears the integrator history. */
int bfm_set_physics(bfm_ctx *ctx, const bfm_physics *ph);

/* Set the state (host xyz [nv][3], phi [nv]) at time t; computes V0 and p_g0
 * of every bubble from the filtered state and clears the history. */
int bfm_state_set(bfm_ctx *ctx, const double *xyz, const double *phi, double t);
/* Copy the state out (host; any pointer may be NULL). */
int bfm_state_get(bfm_ctx *ctx, double *xyz, double *phi, double *t);

/* Advance the state by dt (RK4 for the first five steps after
 * bfm_state_set, then AB6 with a constant dt). info may be NULL. */
int bfm_step(bfm_ctx *ctx, double dt, bfm_step_info *info);

/* One right-hand side evaluation at time t for host arrays xyz, phi (the
 * stored state is not changed; V0 and p_g0 from bfm_state_set are used).
 * Outputs (host, any may be NULL): dxyz [nv][3], dphi [nv], and q, H [nv]
 * of the filtered surface. */
int bfm_rhs(bfm_ctx *ctx, double t, const double *xyz, const double *phi, double *dxyz, double *dphi,
            double *q, double *H);

#ifdef __cplusplus
}
#endif

#endif
