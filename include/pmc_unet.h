/*
 * pmc_unet.h - C ABI of the learned Monte Carlo dose denoiser (gfx950).
 *
 * The transport of pmc.h estimates dose with statistical noise that falls as
 * 1/sqrt(histories) (arXiv:1409.8336, Sec. II.B.2 and Eq. 5).  This library
 * part trains and runs a 3-D U-Net that maps a low-history dose (plus the
 * density map) to an estimate of the high-history dose, so that a plan can be
 * evaluated from far fewer histories; plain Monte Carlo remains the fallback
 * and the reference for its error (gamma index, Low et al., as used in the
 * paper's Sec. II.D).  It has no counterpart in the paper.
 *
 * Network: 4 levels (16/32/64/128 channels), one 3x3x3 convolution + leaky
 * ReLU (negative slope 0.01) per level on the way down (2x2x2 average pooling between levels) and one per
 * level on the way up (nearest 2x upsampling, concatenation with the skip),
 * then a 1x1x1 head added to the normalised input dose (residual):
 *   out = dose + scale * head(features),  scale = max(dose).
 * Input channels: dose/scale and density/2.  BF16 activations and weights on
 * the matrix cores with FP32 accumulation; FP32 master weights, Adam.
 *
 * Tensors are [n][d][h][w] float32 device arrays (w fastest); d, h and w must
 * be multiples of 8.  Every call is stream-ordered on hip_stream (NULL = the
 * null stream) and returns after enqueueing unless stated otherwise.
 * Parameter vector (pmc_unet_get_params): for each convolution in the order
 * enc1(2->16, input padded to 8 channels), enc2(16->32), enc3(32->64),
 * enc4(64->128), dec3(192->64), dec2(96->32), dec1(48->16): weights
 * [Cout][Kp] with Kp = 27*Cin rounded up to 32 (index tap*Cin + ci, tap =
 * (kz*3+ky)*3+kx, zero padding), then bias [Cout]; finally the head weights
 * [16] and bias [1].
 */
#ifndef PMC_UNET_H
#define PMC_UNET_H

#include <stdint.h>

#include "pmc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pmc_unet pmc_unet;

/* Create a network for inputs of shape [n][d][h][w] on HIP device `device`,
 * weights initialised from `seed` (He-normal convolutions, zero biases, zero
 * head: the initial network returns its input dose).  Errors: PMC_ERR_ARG (shape not multiples of 8, n < 1),
 * PMC_ERR_NOMEM, PMC_ERR_DEVICE. */
pmc_status pmc_unet_create(pmc_unet** out, int device, int n, int d, int h, int w, uint64_t seed);
pmc_status pmc_unet_destroy(pmc_unet* u);
const char* pmc_unet_last_error(const pmc_unet* u);

/* Number of float32 parameters (layout in the header comment). */
pmc_status pmc_unet_param_count(const pmc_unet* u, int64_t* count);
/* Copy the FP32 master parameters to / from host memory (count floats);
 * set_params also refreshes the BF16 weight copies.  Synchronous. */
pmc_status pmc_unet_get_params(pmc_unet* u, float* host_out);
pmc_status pmc_unet_set_params(pmc_unet* u, const float* host_in);

/* Denoise: d_out = network(d_dose, d_density). */
pmc_status pmc_unet_forward(pmc_unet* u, const float* d_dose, const float* d_density, float* d_out,
                            void* hip_stream);

/* Denoise a grid smaller than the network's shape (the network needs sides
 * divisible by 8; a treatment plan's CT need not): d_dose, d_density and
 * d_out are [n][d][h][w] (each side at most the one given to pmc_unet_create), placed
 * at the origin of the network's grid, which is zero outside them (no dose,
 * density 0).  PMC_ERR_ARG if the grid does not fit. */
pmc_status pmc_unet_forward_region(pmc_unet* u, const float* d_dose, const float* d_density, int d, int h, int w,
                                   float* d_out, void* hip_stream);

/* Forward, squared error against d_target in units of max(d_dose) summed
 * over all voxels and divided by the number of voxels of the dose region
 * (d_dose >= 1% of its maximum), and backward; gradients are added to the
 * gradient buffer, *loss_out (host, may be NULL) receives the loss.
 * Synchronous when loss_out != NULL. */
pmc_status pmc_unet_backward(pmc_unet* u, const float* d_dose, const float* d_density,
                             const float* d_target, double* loss_out, void* hip_stream);

/* Gradient buffer to host (count floats, synchronous) / reset to zero. */
pmc_status pmc_unet_get_grads(pmc_unet* u, float* host_out);
pmc_status pmc_unet_zero_grads(pmc_unet* u, void* hip_stream);

/* L2 norm of the accumulated gradient (all parameters), computed on the
 * device in FP64 and returned to *norm_out (synchronises the stream). */
pmc_status pmc_unet_grad_norm(pmc_unet* u, double* norm_out, void* hip_stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with learning rate lr on
 * grad_scale times the accumulated gradients (grad_scale in (0, 1]: the
 * caller's gradient-norm clipping, 1 = plain Adam), which it then resets to
 * zero. */
pmc_status pmc_unet_adam_step(pmc_unet* u, float lr, float grad_scale, void* hip_stream);

/* ---- single layers, for kernel tests (device pointers, BF16 as uint16) ----
 * x: [n][d][h][w][cin] channels-last; w: [cout][Kp] (see above); y:
 * [n][d][h][w][cout].  cin, cout multiples of 8, at least 8; the Kp - 27*cin
 * padding columns of w must be zero.
 * forward: y = conv(x, w) + bias (bias may be NULL), then the leaky ReLU
 * (y if y > 0 else 0.01 y) when relu != 0.
 * backward_data: dx = conv^T(dy, w) (workspace allocated internally).
 * backward_weight: dw[cout][Kp] (float32) += sum over voxels of dy (x) x. */
pmc_status pmc_nn_conv3d_forward(const uint16_t* d_x, const uint16_t* d_w, const float* d_bias,
                                 uint16_t* d_y, int n, int d, int h, int w, int cin, int cout,
                                 int relu, void* hip_stream);
pmc_status pmc_nn_conv3d_backward_data(const uint16_t* d_dy, const uint16_t* d_w, uint16_t* d_dx,
                                       int n, int d, int h, int w, int cin, int cout,
                                       void* hip_stream);
/* The data gradient of pmc_nn_conv3d_backward_data, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving and training
 * loops that forbid hipMalloc): the same kernels, with the flipped-weight
 * workspace (cin x round_up(27 cout, 32) BF16 entries) in a device-resident
 * array of 2^20 entries (2 MiB) that the library holds on every GPU it runs
 * on until the process ends.  No hipMalloc, hipFree or allocating library
 * call; stream-ordered on hip_stream, does not synchronise.  Every call on a
 * GPU shares that GPU's workspace, so calls that overlap on one GPU (other
 * streams, other threads) race: order them.  Errors: PMC_ERR_ARG (as
 * pmc_nn_conv3d_backward_data), PMC_ERR_RANGE (cin * round_up(27 cout, 32)
 * above 2^20, e.g. cin = cout = 256), PMC_ERR_DEVICE. */
pmc_status pmc_nn_conv3d_backward_data_noalloc(const uint16_t* d_dy, const uint16_t* d_w, uint16_t* d_dx,
                                               int n, int d, int h, int w, int cin, int cout,
                                               void* hip_stream);
pmc_status pmc_nn_conv3d_backward_weight(const uint16_t* d_x, const uint16_t* d_dy, float* d_dw,
                                         int n, int d, int h, int w, int cin, int cout,
                                         void* hip_stream);

/* Matrix-core throughput probe (the achievable BF16 MFMA rate the
 * convolutions are measured against): every wave of eight 256-lane
 * workgroups per CU issues iters rounds of eight independent
 * v_mfma_f32_16x16x32_bf16 on register operands; *ms_out = the best of three
 * timed launches (after one warm-up), *flop_out = the FLOP of one launch
 * (16,384 per instruction).  Allocates and frees a small output buffer.
 * Errors: PMC_ERR_ARG (iters < 1, NULL outputs), PMC_ERR_NOMEM,
 * PMC_ERR_DEVICE. */
pmc_status pmc_nn_mfma_probe(int32_t iters, void* hip_stream, double* ms_out, double* flop_out);

/* 3-D gamma index (global dose difference, distance to agreement), Low et
 * al.: for every reference voxel with ref >= cutoff_frac * max(ref),
 * gamma = min over points p of the evaluated distribution (trilinear, on a
 * cubic grid of spacing step_cm within search_cm of the voxel centre) of
 * sqrt(|p|^2/dta_cm^2 + (eval(p) - ref)^2 / (dose_frac * max(ref))^2).
 * ref and eval: [nz][ny][nx] float64 device arrays; d_gamma (float32, may be
 * NULL) receives gamma (or -1 below the cutoff).  *pass_rate (host) = the
 * fraction of evaluated voxels with gamma <= 1; *n_eval their count.
 * Synchronous.  The reduction counters (32 bytes per device) are allocated
 * on a device's first call of this function or pmc_denoise_disagreement and
 * kept; calls of the two are serialised within the process. */
pmc_status pmc_gamma_index(const double* d_ref, const double* d_eval, int nx, int ny, int nz,
                           float dx_cm, float dy_cm, float dz_cm, float dose_frac, float dta_cm,
                           float cutoff_frac, float search_cm, float step_cm, float* d_gamma,
                           double* pass_rate, int64_t* n_eval, void* hip_stream);

/* Fallback rule of the denoiser: among voxels with d_mc >= cutoff_frac *
 * max(d_mc), the fraction where |d_den - d_mc| > k_sigma * sqrt(d_var_mc),
 * i.e. where the denoised dose departs from the noisy Monte Carlo dose it
 * was computed from by more than k_sigma of that dose's own standard error
 * (Eq. 5).  A caller falls back to plain Monte Carlo when the fraction
 * exceeds its threshold.  d_den float32, d_mc and d_var_mc float64, n
 * elements each (device).  *frac_out and *n_out (host) receive the fraction
 * and the number of voxels above the cutoff.  Synchronous; shares the
 * counters of pmc_gamma_index. */
pmc_status pmc_denoise_disagreement(const float* d_den, const double* d_mc, const double* d_var_mc,
                                   int64_t n, float cutoff_frac, float k_sigma, double* frac_out,
                                   int64_t* n_out, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* PMC_UNET_H */
