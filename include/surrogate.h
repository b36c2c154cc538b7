/*
 * surrogate.h -- C ABI of the gfx950 kernels of the learned surrogate that
 * advances lattice states of the thermocapillary lattice Boltzmann scheme
 * (arXiv:2306.11320) by a fixed number of time steps.  Not part of the paper's
 * method: the lattice update of lbm.h remains the reference and the fallback.
 *
 * Network: 3x3 convolutions over frames periodic in x and zero-padded in y;
 * BF16 activations and weights, FP32 accumulation on the matrix cores
 * (v_mfma_f32_32x32x16_bf16), FP32 bias, weight gradients, master weights and
 * Adam state.
 *
 * Layouts (all device memory owned by the caller; every call is asynchronous
 * on `stream` and returns 0 or a negative error code, see sur_last_error):
 *   activations  NHWC, element (n, y, x, c) at ((n*H + y)*W + x)*C + c, with
 *                C = 32 (network input: C = 8), BF16;
 *   weights      [co = 32][tap = 9][ci], tap = 3*(dy+1) + (dx+1), BF16;
 *   W            any width >= 1 (a row is covered by 32-pixel segments; the
 *                last one is masked); pointers 16-byte aligned.
 */
#ifndef SURROGATE_H
#define SURROGATE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* out = [mask > 0] * (conv(A, w) + bias) + res, A = max(in, 0) if relu_in else
 * in, conv with dilation dil (1 <= dil <= w: taps at (dy, dx) * dil); in has
 * cin in {8, 32} channels; out has 32 channels, FP32 if out_f32 else BF16.
 * bias, res and mask may be NULL (res has out's type; mask is BF16 with 32
 * channels).  Frames of n x h x w pixels with n h ceil(w / 32) < 2^30. */
int sur_conv3x3(const void* d_in, int cin, const void* d_w, const float* d_bias, const void* d_res,
                const void* d_mask, void* d_out, int out_f32, int relu_in, int dil, int n, int h, int w,
                void* stream);

/* Weights of the adjoint (input-gradient) convolution of a layer with cin
 * input channels: wt[ci][8 - tap][co] = w[co][tap][ci], 32 x 9 x 32 BF16.
 * sur_conv3x3(dy, 32, wt, ...) with the layer's dilation then computes the
 * gradient with respect to the layer's input (periodic x, zero-padded y: the
 * exact adjoint). */
int sur_adjoint_weights(const void* d_w, int cin, void* d_wt, void* stream);

/* Weight gradient dW[co][tap][ci] = sum_p dy[p][co] A[p + dil offset(tap)][ci]
 * (A = max(in, 0) if relu_in) into d_out (32*9*cin FP32), through `groups`
 * per-workgroup partial sums in d_part (sur_wgrad_scratch_floats floats),
 * summed in a fixed order. */
int sur_weight_grad(const void* d_dy, const void* d_in, int cin, int relu_in, int dil, int n, int h, int w,
                    float* d_part, int groups, float* d_out, void* stream);
size_t sur_wgrad_scratch_floats(int cin, int groups);

/* Bias gradient db[co] = sum_p dy[p][co] (32 FP32), through 32*groups partials. */
int sur_bias_grad(const void* d_dy, int64_t npix, float* d_part, int groups, float* d_out, void* stream);

/* One Adam step (bias-corrected, step t >= 1) on n FP32 master values; writes
 * the BF16 copy d_pb. */
int sur_adam(float* d_p, const float* d_g, float* d_m1, float* d_m2, void* d_pb, int64_t n, float lr, float beta1,
             float beta2, float eps, int t, void* stream);

/* Squared error of the predicted increment delta[:, 0:nout] (FP32, 32
 * channels) against the target increment (nout FP32 channels, 1 <= nout <= 32):
 * per-workgroup partial sums into d_part[groups]; gradient
 * 2 (delta - target) * scale into d_grad (BF16, 32 channels, zero beyond nout). */
int sur_mse(const float* d_delta, const float* d_target, int64_t npix, int nout, float scale, void* d_grad,
            float* d_part, int groups, void* stream);

/* Scalings of one lattice's state.  The state is five FP32 fields of h x w
 * values (x fastest): phi, ux, uy, T and the pressure p, passed as a host
 * array of 5 device pointers in that order. */
typedef struct {
    float u;          /* velocity scale U (> 0) */
    float dT;         /* temperature scale (> 0) */
    float t_a, t_b;   /* rest temperature profile T_rest(y) = t_a + t_b y, y = row index */
    float P;          /* pressure scale (> 0) */
    float c4, c5;     /* constant conditioning inputs (channels 4 and 5) */
    float inc[5];     /* unit of the learned increment of phi, ux, uy, T, p (> 0) */
} sur_scales;

/* Network input of one frame: 8 BF16 channels (phi, ux/u, uy/u,
 * (T - T_rest(y))/dT, c4, c5, (p - P (1 - phi)/2)/P, 0) into d_x (h*w*8
 * values): the pressure less its Young-Laplace part. */
int sur_pack(const float* const* d_f, int h, int w, const sur_scales* scales, void* d_x, void* stream);
/* Target increment between states f0 and f1: (f1_c - f0_c) / inc[c] for the
 * five fields, 5 FP32 channels per pixel into d_t. */
int sur_pack_target(const float* const* d_f0, const float* const* d_f1, int64_t npix, const sur_scales* scales,
                    float* d_t, void* stream);
/* Advances the five fields in place by a predicted increment:
 * f_c += delta[:, c] inc[c], c = 0..4 (delta: FP32, 32 channels). */
int sur_advance(const float* d_delta, int64_t npix, const sur_scales* scales, float* const* d_f, void* stream);
/* The network's last layer with the state update of sur_advance fused into
 * its epilogue, on one frame of h x w pixels (h ceil(w / 32) < 2^30):
 * f_c += (conv(A, w) + bias)_c * inc[c] for c < 5, A = max(in, 0) if relu_in,
 * in BF16 NHWC with 32 channels, w and bias as for sur_conv3x3 with cin = 32,
 * dilation dil.  Bitwise equal to sur_conv3x3 into an FP32 buffer followed by
 * sur_advance, without that buffer (the 32 FP32 channels of the increment are
 * neither written nor read).  d_f: five FP32 device fields of h*w (phi, ux,
 * uy, T, p), updated in place.  Errors: NULL pointers, h or w < 1, dil out of
 * [1, w], too many segments or misaligned in / w. */
int sur_conv3x3_advance(const void* d_in, const void* d_w, const float* d_bias, int relu_in, int dil, int h, int w,
                        const sur_scales* scales, float* const* d_f, void* stream);
/* sur_conv3x3_advance (dil <= 16) that also writes the light-phase volume
 * sum (1 - phi)/2 of the updated phi, in FP64, into *d_vol (device): the
 * hybrid rollout's check of the light phase after each network block, without
 * a separate reduction over the frame.  The state is bitwise that of
 * sur_conv3x3_advance; the volume equals sur_light_volume's up to the order of
 * the FP64 sums (fixed for given h and w).  d_part: 8 * SUR_VOLUME_PARTS
 * doubles of device scratch, 8-byte aligned (per-workgroup partials, summed
 * in a fixed order by a second kernel on the same stream).  Calls that share
 * d_part must not overlap in time.  Errors: as sur_conv3x3_advance, also NULL
 * d_part or d_vol and dil > 16. */
#define SUR_VOLUME_PARTS 512
int sur_conv3x3_advance_volume(const void* d_in, const void* d_w, const float* d_bias, int relu_in, int dil, int h,
                               int w, const sur_scales* scales, float* const* d_f, double* d_part, double* d_vol,
                               void* stream);
/* Light-phase volume sum (1 - phi)/2 of a frame, in FP64, into *d_out (device),
 * through `groups` partials in d_part (8*groups doubles), summed in a fixed order. */
int sur_light_volume(const float* d_phi, int h, int w, double* d_part, int groups, double* d_out, void* stream);
/* Judge of a predicted frame a against a lattice frame b (first four fields):
 * d_out[2c] = sum (a_c - b_c)^2 and d_out[2c+1] = sum (b_c - rest_c)^2 for
 * c = phi, ux, uy, T with rest = (1, 0, 0, T_rest(y)), FP64, through `groups`
 * partials in d_part (8*groups doubles), summed in a fixed order. */
int sur_judge(const float* const* d_a, const float* const* d_b, int h, int w, const sur_scales* scales,
              double* d_part, int groups, double* d_out, void* stream);

/* sur_judge without a scratch argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same kernels and the same result as sur_judge with
 * `groups` partials.  The partials live in a library-owned static device array
 * of SUR_JUDGE_MAX_GROUPS * 8 doubles (64 KiB) on each GPU the call runs on,
 * held until the process ends; the call itself allocates nothing.  `stream`
 * must belong to the current device.  Every partial it reads is written first
 * by the same call, so nothing needs clearing, but all calls on one GPU share
 * the array: two calls that overlap in time on one GPU (different streams or
 * threads) race; calls ordered on one stream do not.
 * Errors: -1 with a message if groups is outside [1, SUR_JUDGE_MAX_GROUPS] or
 * an argument is invalid; -3 if a HIP call fails. */
#define SUR_JUDGE_MAX_GROUPS 1024
int sur_judge_noscratch(const float* const* d_a, const float* const* d_b, int h, int w, const sur_scales* scales,
                        int groups, double* d_out, void* stream);

const char* sur_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SURROGATE_H */
