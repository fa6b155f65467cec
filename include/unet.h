/* unet.h -- C ABI of the learned-initialisation network in libimsp.so.
 *
 * The network maps the phases of a coarse multislice reconstruction (one channel
 * per slice, a centre crop of the object) to the slice potentials.  It is a U-Net
 * (Ronneberger, Fischer and Brox, 2015): `levels` levels of widths base << l, each
 * two 3x3 convolutions (zero padding 1) with ReLU; 2x2 max pooling on the way down;
 * on the way up a 2x2 stride-2 transposed convolution (no activation) whose output
 * is concatenated, in the order [upsampled, skip], with the encoder output of the
 * same level, then two 3x3 convolutions with ReLU; a final 1x1 convolution.
 * Training minimises the mean squared error after removing the mean of every
 * (sample, channel) over the pixels (a constant phase per slice is not observable),
 * with Adam (Kingma and Ba, 2015).  The paper itself does not use a network; its
 * layer-wise reconstruction (Sec. 3, Algorithm 1) is what the predicted slices
 * initialise.
 *
 * Precision: activations and their gradients are bfloat16, weights are kept in
 * FP32 (master copy) with bfloat16 copies for the matrix cores, every product
 * accumulates in FP32, the loss in FP64.
 *
 * Layout: images are NHWC (channels fastest).  The input has in_pad =
 * round_up(in_ch, 8) bfloat16 channels (pad channels must be zero); the output has
 * out_ch float channels; targets likewise out_ch floats.
 *
 * Parameters: one flat FP32 vector owned by the network (inside the caller's
 * workspace).  Layer i has a weight matrix of n_rows x kpad floats at w_offset and
 * cout floats of bias at b_offset:
 *   3x3 / 1x1 convolution:  W[co][t * cin + ci],      t = 3u + v  (1x1: t = 0)
 *   transposed convolution: W[t * cout + co][ci],     t = 2u + v, output pixel (2y + u, 2x + v)
 * with cin the padded input channel count (the concatenation's [upsampled, skip]
 * order for the first convolution of a decoder level) and zeros in every padding
 * column.  After writing parameters call un_sync_weights.
 *
 * Calls enqueue on the given stream and return without synchronising; every
 * argument is checked on the host first, and on error nothing is enqueued and a
 * negative un_status is returned with a message in un_last_error().  Calls on one
 * network must not overlap (they share its activation buffers).
 */
#ifndef UNET_H
#define UNET_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    UN_OK = 0,
    UN_ERR_INVALID_ARG = -1,
    UN_ERR_UNSUPPORTED = -2,
    UN_ERR_BUDGET = -3,
    UN_ERR_HIP = -4
} un_status;

typedef enum { UN_CONV3X3 = 0, UN_UPCONV2X2 = 1, UN_CONV1X1 = 2 } un_kind;

typedef struct {
    int32_t in_ch, out_ch;     /* 1..16 each                                                  */
    int32_t base, levels;      /* widths base << l for l < levels; base a multiple of 8;
                                  levels in [1, 5]; base << (levels - 1) <= 256               */
    int32_t height, width;     /* powers of two, each divisible by 2^(levels - 1), >= 8      */
    int32_t max_batch;         /* >= 1; the activation buffers are sized for it             */
} un_config;

typedef struct {
    int32_t kind;              /* un_kind                                                    */
    int32_t cin, cout;         /* padded input channels; output channels                     */
    int32_t taps;              /* 9, 4 or 1                                                  */
    int32_t n_rows, kpad;      /* weight matrix shape                                        */
    int64_t w_offset, b_offset;/* into the parameter vector (floats)                         */
} un_layer;

typedef struct un_net un_net;

/* Bytes of device workspace the network needs (parameters, Adam moments, bf16
 * weight copies, activations for max_batch, gradient and reduction buffers). */
un_status un_workspace_size(const un_config *cfg, size_t *ws_bytes);

/* Builds a network inside a caller-owned device workspace of at least
 * un_workspace_size bytes (256-byte aligned).  Parameters start as zeros and
 * the Adam moments are cleared by the first un_sync_weights. */
un_status un_net_create(const un_config *cfg, void *workspace, size_t ws_bytes, un_net **out);
void un_net_destroy(un_net *net);

/* Layers in parameter order: enc0.conv0, enc0.conv1, ..., enc(L-1).conv1, then for
 * l = L-2 .. 0: dec l.up, dec l.conv0, dec l.conv1, and finally the 1x1 head. */
int32_t un_layer_count(const un_net *net);
un_status un_layer_info(const un_net *net, int32_t index, un_layer *out);

/* Device pointers to the FP32 parameter vector and its gradient (same layout), and
 * the number of floats in each. */
un_status un_params(un_net *net, float **params, float **grads, int64_t *count);

/* Makes the bfloat16 copies of the parameters the kernels read, and clears the
 * Adam moments and step count.  Call after writing parameters. */
un_status un_sync_weights(un_net *net, hipStream_t stream);

/* y = network(x) for `batch` <= max_batch images. x: [batch][H][W][in_pad] bf16,
 * y: [batch][H][W][out_ch] float. */
un_status un_forward(un_net *net, hipStream_t stream, int32_t batch, const uint16_t *x, float *y);

/* Forward pass, loss and gradients: y receives the output, *loss_out (device FP64)
 * the centred mean squared error against target ([batch][H][W][out_ch] float), and
 * the gradient vector d loss / d parameters (overwritten). */
un_status un_backward(un_net *net, hipStream_t stream, int32_t batch, const uint16_t *x, const float *target,
                      float *y, double *loss_out);

/* One Adam step on the parameters with the current gradient vector, then the
 * bfloat16 copies.  The step count (for bias correction) is kept by the network. */
un_status un_adam_step(un_net *net, hipStream_t stream, float lr, float beta1, float beta2, float eps);

/* Read access to the activations of the last forward pass, for inspection:
 * index 3i+j for encoder level i (j = 0: first convolution, 1: second, 2: pooled),
 * then 3L + 3i + j for decoder level i (j = 0: upsampled, 1: first convolution,
 * 2: second).  Shape [batch][height][width][channels] bf16. */
un_status un_activation(const un_net *net, int32_t index, const uint16_t **data, int32_t *height,
                        int32_t *width, int32_t *channels);

/* Message of the last failed call on this thread. */
const char *un_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* UNET_H */
