/*
 * sg.h -- C ABI of the learned window surrogate that accompanies the lattice
 * Boltzmann library (lbm.h).  Not part of the paper: a small convolutional
 * time-stepper mapping the macroscopic fields of a lattice to the fields 16
 * lattice steps later, used with the lattice Boltzmann scheme as fallback and
 * judge.  Conventions (errors, ownership, streams) are those of lbm.h; the
 * status codes are lbm_status.
 *
 * Network: a linear U-Net without biases or activations on the first-order
 * system's variables U (inverse of Eq. sigma_num), normalised by the
 * per-sample RMS of U: 3x3 convolutions (circular padding for periodic data,
 * zero padding otherwise), two per level on four levels with 32, 64, 128, 128
 * channels, 2x2 average pooling, nearest up-sampling with additive skips;
 * every convolution output channel is scaled by a FiLM gain that is a cubic
 * Chebyshev polynomial of the material angle atan2(c_mu, c_K) (the time step
 * is taken at half the CFL-like limit, Eq. stab_cond).  Output fields:
 * U + s * y.  Convolutions run on BF16 matrix cores with FP32 accumulation;
 * split = 3 carries each FP32 operand as a hi + lo BF16 pair.
 *
 * Field arrays: input [batch][8][H][W] FP32 = (v_x, v_y, sigma_xx, sigma_yy,
 * sigma_xy, lambda, mu, rho); output and targets [batch][5][H][W] FP32 =
 * (v_x, v_y, sigma_xx, sigma_yy, sigma_xy), physical units.
 */
#ifndef SG_H
#define SG_H

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sg_net sg_net;

typedef struct {
  int32_t batch;   /* largest batch a call may use, >= 1                      */
  int32_t height;  /* H, multiple of 64                                       */
  int32_t width;   /* W, multiple of 128                                      */
  int32_t split;   /* 1: plain BF16 operands; 3: hi/lo BF16 pairs             */
  int32_t train;   /* nonzero: allocate gradient and Adam buffers             */
} sg_config;

/* Device bytes of the caller-owned workspace (0 if the config is invalid). */
size_t sg_workspace_bytes(const sg_config* cfg);

/* Number of FP32 parameters: per layer in order in, e0a, e0b, e1a, e1b, e2a,
 * e2b, e3a, e3b, d2a, d2b, d1a, d1b, d0a, d0b, out: the weights
 * [cout][cin][3][3] followed by the FiLM coefficients [cout][4]. */
int64_t sg_param_count(void);

lbm_status sg_create(const sg_config* cfg, void* d_ws, size_t ws_bytes, void* hip_stream,
                     sg_net** out);
lbm_status sg_destroy(sg_net* net);

/* Convolution kernel family: 0 (default) stages each input tile in LDS where
 * the row length at a layer is a multiple of 64 pixels or 32 or 16 pixels,
 * with the weights in LDS too for 32-channel output tiles, and uses the direct
 * kernel elsewhere; 1 uses the direct kernel (operands read from global
 * memory) for every layer; 2 is 0 with the weights always read from global
 * memory.  All compute the same products and sums (FP32 accumulation order
 * may differ); for comparisons and timing. */
lbm_status sg_set_conv_mode(sg_net* net, int32_t mode);

/* Copy the parameter vector in (resets the Adam state) or out, device to
 * device, stream-ordered. */
lbm_status sg_set_params(sg_net* net, const float* d_params);
lbm_status sg_get_params(sg_net* net, float* d_params);

/* Gradient of the last sg_train_step's loss (before its update), same layout. */
lbm_status sg_get_grads(sg_net* net, float* d_grads);

/* One surrogate call on `batch` samples: d_in [batch][8][H][W] ->
 * d_out [batch][5][H][W].  circular != 0 selects periodic padding. */
lbm_status sg_forward(sg_net* net, const float* d_in, int32_t batch, int32_t circular,
                      float* d_out);

/* Forward, loss = mean over samples, 5 components and pixels of
 * (y - (U_target - U)/s)^2, backward, and (if lr > 0) one Adam step
 * (beta1 0.9, beta2 0.999, eps 1e-8) on the FP32 master parameters.  The loss
 * before the update is written to *h_loss if non-null (synchronises). */
lbm_status sg_train_step(sg_net* net, const float* d_in, const float* d_target, int32_t batch,
                         int32_t circular, float lr, double* h_loss);

#ifdef __cplusplus
}
#endif

#endif /* SG_H */
