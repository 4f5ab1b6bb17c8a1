/* libvam: learned initialiser for the projection optimisation.
 *
 * The paper starts its optimisation from filtered parallel-beam projections
 * of the target (Sec. 2.3 and the Radon baseline it compares against).  This
 * small convolutional network is an addition that is not in the paper: per
 * angle it maps the target's parallel-beam projection and that filtered
 * starting point to a better starting point for the ray-traced optimisation
 * (Sec. 2.5-2.7), trained on projections the plain optimisation produced.
 *
 * Network: L convolution layers, 3x3 kernels, zero padding 1, stride 1; the
 * first takes 2 channels, the hidden layers have C channels and a ReLU, the
 * last has 1 output channel and no activation.  With x = (x0, x1) the two
 * input images of an angle and s0, s1 the input scales given at creation,
 *     a_0  = bf16(s0 x0, s1 x1)
 *     a_l  = bf16(relu(conv(a_{l-1}, bf16(W_l)) + b_l)),   l = 1 .. L-1
 *     z    = conv(a_{L-1}, bf16(W_L)) + b_L
 *     y    = x1 + z / s1          (a residual on the filtered start)
 * Convolutions accumulate in FP32; activations and gradients are stored in
 * BF16 (round to nearest even), master weights and Adam moments in FP32.
 *
 * Parameter layout (FP32, host arrays), layer after layer: W_l as
 * [c_out][3][3][c_in] followed by b_l as [c_out].
 *
 * Images are [n][H][W] FP32 device arrays, W <= 1024, H * W * n < 2^31.
 * All calls are stream-ordered; a handle is used from one stream at a time.
 * Errors are reported as for the projector calls (vam_last_error()). */
#ifndef VAM_CNN_H
#define VAM_CNN_H

#include <stdint.h>

#include "vam.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vam_cnn* vam_cnn_t;

/* Create a network of `layers` (>= 2) convolutions with `channels` (a
 * multiple of 8, <= 64) hidden channels for H x W images and batches of at
 * most `max_batch` images; allocates the workspace on the current device:
 * ~(2 (8 + (layers - 1) channels) + 4 channels + 32) bytes per pixel of a
 * batch, plus 256 x 9 x channels^2 x 4 bytes of weight-gradient partials
 * (the convolutions gather their im2col tiles on the fly, nothing of
 * 9 x channels per pixel is stored).  Parameters start at zero; set them
 * with vam_cnn_set_params. */
vam_status vam_cnn_create(int32_t layers, int32_t channels, int32_t height, int32_t width, int32_t max_batch,
                          float in_scale0, float in_scale1, vam_cnn_t* out);
vam_status vam_cnn_destroy(vam_cnn_t h);
/* Number of FP32 parameters (the layout above). */
int64_t vam_cnn_param_count(vam_cnn_t h);
/* Copy parameters in / out (host arrays of vam_cnn_param_count floats);
 * set also clears the Adam moments and step count.  Synchronous. */
vam_status vam_cnn_set_params(vam_cnn_t h, const float* params);
vam_status vam_cnn_get_params(vam_cnn_t h, float* params);
/* Training state for checkpoint and resume: state (host, 3 * param_count
 * floats) holds the parameters, then Adam's first and second moments, in
 * the layout above; adam_steps the number of Adam steps taken.  set
 * restores exactly what get returned, so training resumed from a
 * checkpoint takes the same steps as training that never stopped.
 * Synchronous. */
vam_status vam_cnn_get_state(vam_cnn_t h, float* state, int64_t* adam_steps);
vam_status vam_cnn_set_state(vam_cnn_t h, const float* state, int64_t adam_steps);
/* Inference: x [n][2][H][W] -> y [n][H][W] (device, FP32), n <= max_batch. */
vam_status vam_cnn_forward(vam_cnn_t h, const float* x, int32_t n, float* y, hipStream_t stream);
/* Loss and gradients of L = mean over the n H W pixels of (y - t)^2 s1^2
 * (the squared error in the network's scaled units) for x [n][2][H][W] and
 * targets t [n][H][W]; gradients are kept in the handle (read them with
 * vam_cnn_get_grads) for the next vam_cnn_adam_step.  loss_out (host, may
 * be NULL) synchronises the stream.  The result does not depend on
 * scheduling (fixed-order reductions). */
vam_status vam_cnn_loss_grad(vam_cnn_t h, const float* x, const float* t, int32_t n, double* loss_out,
                             hipStream_t stream);
vam_status vam_cnn_get_grads(vam_cnn_t h, float* grads);
/* One Adam step (Kingma & Ba, bias-corrected) on the last gradients. */
vam_status vam_cnn_adam_step(vam_cnn_t h, float lr, float beta1, float beta2, float eps, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* VAM_CNN_H */
