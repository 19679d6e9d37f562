// Learned initial guess: network state, training set and entry points
// (learn.hip). Everything lives on the handle's device and stream.
#pragma once

#include <hip/hip_bf16.h>

#include "ctx.h"

namespace bfm {

struct Mlp {
    static constexpr int kDegree = 8;                              // harmonic degree of features/targets
    static constexpr int kNc = (kDegree + 1) * (kDegree + 1);      // 81 coefficients
    static constexpr int kIn = 2 * kNc + 12;                       // 174 features
    static constexpr int kOut = kNc;                               // 81 outputs
    static constexpr int kHidden = 512;
    static constexpr int kLayers = 4;
    static constexpr int kInPad = 192, kOutPad = 96;               // multiples of 32 (MFMA K)
    static constexpr int kNorm = 2 * kIn + 2 * kOut;               // [mu_x | sd_x | mu_y | sd_y]
    int dims[kLayers + 1] = {kInPad, kHidden, kHidden, kHidden, kOutPad};
    int true_in(int k) const { return k == 0 ? kIn : dims[k]; }
    int true_out(int k) const { return k == kLayers - 1 ? kOut : dims[k + 1]; }

    bool ready = false;     // weights set
    bool norm_set = false;  // standardisation set
    int adam_t = 0;

    // FP32 master weights W [in][out] (zero-padded), biases, Adam moments, gradients
    DevBuf<float> W[kLayers], b[kLayers], mW[kLayers], vW[kLayers], mb[kLayers], vb[kLayers];
    DevBuf<float> dW[kLayers], db[kLayers];
    // BF16 copies: Wt [out][in] (forward operand), Wn [in][out] (backward operand)
    DevBuf<__bf16> Wt[kLayers], Wn[kLayers];
    // activations: X[k] layer inputs (BF16, [R][dims[k]]), Z[k] pre-activations (FP32)
    DevBuf<__bf16> X[kLayers], XT, GT, Gb;
    DevBuf<float> Z[kLayers], G, dX, T, part, norm;
    DevBuf<double> loss_acc;

    // features
    ShBasis sh;
    DevBuf<double> cen, rad, vbuf1, vbuf2, coef1, coef2;
    DevBuf<float> offs, feat, targ;

    // training set (rows of features and targets, FP32) and batch order
    DevBuf<float> ds_x, ds_y;
    int64_t ds_rows = 0;
    DevBuf<int> perm;
};

Mlp &mlp_get(bfm_ctx *c);
void mlp_free(bfm_ctx *c);
int64_t mlp_num_params(const Mlp &net);
void mlp_init(Mlp &net, uint64_t seed, hipStream_t st);
void mlp_set_params(Mlp &net, const float *host, hipStream_t st);
void mlp_get_params(Mlp &net, float *host, bool grads, hipStream_t st);
void mlp_set_norm(Mlp &net, const float *host, hipStream_t st);
void mlp_get_norm(Mlp &net, float *host, hipStream_t st);
// raw network on host rows (standardised by the stored statistics on both ends)
void mlp_forward_rows(Mlp &net, int64_t rows, const float *x_dev, float *y_dev, hipStream_t st);
double mlp_gradient_rows(Mlp &net, int64_t rows, const float *x_dev, const float *t_dev, hipStream_t st);
void mlp_adam(Mlp &net, float lr, hipStream_t st);
// features [nb][174] and targets [nb][81] (FP32, device) of the current mesh
void mlp_features(bfm_ctx *c, const double *phi_dev, const double *q_dev, float *feat, float *targ);
void mlp_collect(bfm_ctx *c, const double *phi_dev, const double *q_dev);
double mlp_fit(bfm_ctx *c, int epochs, int batch, float lr, uint64_t seed);
void mlp_guess(bfm_ctx *c, const double *phi_dev, double *q_dev);

}  // namespace bfm
