/* C ABI of the warm-start surrogate network.
 *
 * A small U-Net maps force, source and relaxation-rate fields of a periodic
 * 2D lattice to an estimate of the steady velocity and scalar fields; the
 * lattice Boltzmann iteration (casclb.h) is then started from the
 * equilibrium of that estimate and run to its residual tolerance as usual,
 * so the network only changes the starting point, never the converged
 * answer.  The network is not part of the paper; the solver it warm-starts
 * is the cascaded scheme with the split force and source steps (Sec. 3-5).
 *
 * Architecture (periodic in both directions, NHWC tensors):
 *   encoder level l = 0..L-1: conv3x3 -> relu -> conv3x3 -> relu (width c_l),
 *     2x2 average pooling into level l+1;
 *   decoder level l = L-2..0: nearest 2x upsampling of level l+1's output,
 *     concatenated after level l's encoder output, conv3x3 -> relu (width c_l);
 *   output: conv3x3 (c_0 -> out_channels), no activation.
 * Convolutions use circular padding.  Parameters are one float32 vector:
 * per layer in that order, weights [Co][3][3][Ci] then biases [Co].
 *
 * Arithmetic: weights and activations in bfloat16, products accumulated in
 * float32 on the matrix cores (v_mfma_f32_16x16x32_bf16); float32 master
 * weights, gradients, Adam moments, loss gradient and network output.
 *
 * Conventions: functions return 0 (LB_OK) or a negative LB_E* code of
 * casclb.h; the message is in lb_unet_last_error.  Pointers named *_dev are
 * device memory owned by the caller; *_host are host memory owned by the
 * caller.  All device work runs on the network's stream.  A handle is not
 * thread-safe.
 */
#ifndef CASCLB_UNET_H
#define CASCLB_UNET_H

#include <stddef.h>
#include <stdint.h>

#include "casclb.h"

#ifdef __cplusplus
extern "C" {
#endif

#define LB_UNET_ABI_VERSION 1
#define LB_UNET_MAX_LEVELS 6

typedef struct lb_unet lb_unet;

typedef struct lb_unet_config {
    int32_t abi_version;                    /* LB_UNET_ABI_VERSION                      */
    int32_t levels;                         /* L, 1..LB_UNET_MAX_LEVELS                 */
    int32_t channels[LB_UNET_MAX_LEVELS];   /* c_l, multiples of 16 in [16, 256]        */
    int32_t in_channels;                    /* input channels, 1..16                    */
    int32_t out_channels;                   /* output channels, 1..16                   */
    int32_t height, width;                  /* multiples of 2^(L-1) and of 4            */
    int32_t max_batch;                      /* largest batch of forward / training calls */
    int32_t device;                         /* HIP device ordinal                       */
    void* stream;                           /* hipStream_t (NULL: the null stream)      */
} lb_unet_config;

/* Defaults: L = 4, c = {16, 32, 48, 96}, 5 inputs, 3 outputs, 256 x 256,
 * max_batch 16, device 0, null stream. */
void lb_unet_config_default(lb_unet_config* cfg);

/* Allocates parameters (zero), Adam state and the activation / gradient
 * buffers for max_batch images.  LB_EINVAL on a bad configuration,
 * LB_ENOMEM when device memory runs out. */
int lb_unet_create(lb_unet** out, const lb_unet_config* cfg);
void lb_unet_destroy(lb_unet* net);
const char* lb_unet_last_error(const lb_unet* net);

/* Number of float32 parameters (the flat vector described above). */
int64_t lb_unet_num_params(const lb_unet* net);

/* Copy the flat parameter vector in (resets the Adam state and step count)
 * or out.  Synchronises. */
int lb_unet_set_params(lb_unet* net, const float* params_host);
int lb_unet_get_params(lb_unet* net, float* params_host);

/* y = net(x) for `batch` images: x_dev float32 [batch][H][W][in_channels],
 * y_dev float32 [batch][H][W][out_channels].  Asynchronous. */
int lb_unet_forward(lb_unet* net, const float* x_dev, int32_t batch, float* y_dev);

/* Forward pass, mean squared error against target_dev (float32, shaped like
 * y), and the gradient of that loss with respect to every parameter, kept on
 * the device for lb_unet_adam; *loss (may be NULL) and grad_host (may be
 * NULL, num_params floats) receive copies.  Synchronises when either is
 * requested. */
int lb_unet_loss_grad(lb_unet* net, const float* x_dev, const float* target_dev, int32_t batch, double* loss,
                      float* grad_host);

/* Adds weight * MSE(P y, P t) to the training loss, P the mean over
 * 2^levels x 2^levels pixel blocks (levels 2x2 average poolings): the
 * largest scales of the field, which decay slowest in the solver, weigh more.
 * levels = 0 or weight = 0 turns it off (the default).  The gradient is
 * P^T (2 weight (P y - P t) / count) added to the output gradient. */
int lb_unet_set_lowpass_loss(lb_unet* net, int32_t levels, float weight);

/* One Adam step (bias-corrected, Kingma & Ba) with the gradient of the last
 * lb_unet_loss_grad call.  Asynchronous. */
int lb_unet_adam(lb_unet* net, float lr, float beta1, float beta2, float eps);

/* lb_unet_loss_grad followed by lb_unet_adam (beta1 0.9, beta2 0.999,
 * eps 1e-8); *loss may be NULL (then nothing synchronises). */
int lb_unet_train_step(lb_unet* net, const float* x_dev, const float* target_dev, int32_t batch, float lr,
                       double* loss);

/* Multiply-adds of one forward pass per image (all convolutions, at the
 * unpadded channel counts). */
double lb_unet_macs_per_image(const lb_unet* net);

#ifdef __cplusplus
}
#endif

#endif /* CASCLB_UNET_H */
