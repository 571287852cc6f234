// Stencil-prediction network: dimensions, parameter layout and device state.
#pragma once

#include "common.h"

namespace ls {

constexpr int MLP_I = 250;      // inputs: Re, Im of m on the 5^3 patch
constexpr int MLP_IP = 256;     // padded
constexpr int MLP_H = 256;      // hidden width
constexpr int MLP_O = 468;      // outputs: 26 off-centre 3x3 complex blocks
constexpr int MLP_OP = 480;     // padded
// flat FP32 parameters: W1 [250][256], b1, W2 [256][256], b2, W3 [256][468], b3
constexpr long MLP_OFF_W1 = 0;
constexpr long MLP_OFF_B1 = MLP_OFF_W1 + (long)MLP_I * MLP_H;
constexpr long MLP_OFF_W2 = MLP_OFF_B1 + MLP_H;
constexpr long MLP_OFF_B2 = MLP_OFF_W2 + (long)MLP_H * MLP_H;
constexpr long MLP_OFF_W3 = MLP_OFF_B2 + MLP_H;
constexpr long MLP_OFF_B3 = MLP_OFF_W3 + (long)MLP_H * MLP_O;
constexpr long MLP_NPARAM = MLP_OFF_B3 + MLP_O;
constexpr double MLP_M_SCALE = 0.3;   // input normalisation of m
constexpr double MLP_T_SCALE = 3e-3;  // target normalisation: correction = T_SCALE * output

struct MlpState {
  DevBuf w, m, v, grad;              // FP32 masters, Adam moments, gradient
  DevBuf w1b, w2b, w3b;              // BF16 copies, zero-padded
  DevBuf w1f, w2f, w3f;              // the same in MFMA fragment order, for inference
  int wver = 0, fver = -1;           // version of the BF16 copies / of the fragment-ordered ones
  int t = 0;                         // Adam step count
  bool have_grad = false;            // a backward pass has filled grad
  // activations / gradients workspace
  int ws_rows = 0;
  DevBuf z1, z2, h1b, h2b, y, dyb, dz2, dz2b, dz1, dz1b, dw, sq, part;
  // training set: features (BF16, N x 256) and targets (FP32, N x 468)
  DevBuf xs, ts;
  long nsamples = 0, cap = 0;
};

ls_status mlp_init(MlpState& st, const float* params_host, hipStream_t s);
ls_status mlp_refresh_bf16(MlpState& st, hipStream_t s);
ls_status mlp_workspace(MlpState& st, int Bm);
ls_status mlp_forward(MlpState& st, const unsigned short* xb, int Bm, hipStream_t s);
// inference only: st.y (Bm x 480) from xb, the three layers fused per tile of rows
ls_status mlp_infer(MlpState& st, const unsigned short* xb, int Bm, hipStream_t s);
ls_status mlp_backward(MlpState& st, const unsigned short* xb, const float* T, int Bm, double* loss, hipStream_t s);
ls_status mlp_bias3_grad(MlpState& st, const float* T, int Bm, float* db, hipStream_t s);
ls_status mlp_adam(MlpState& st, double lr, hipStream_t s);

}  // namespace ls
