/*
 * tsdf_nn.h -- C ABI of the learned depth prefilter in libtsdf.so.
 *
 * A small convolutional encoder-decoder that corrects a depth frame before
 * it is fused (the paper fuses raw depth, optionally bilateral-filtered,
 * Sec. 4; this learned filter is not part of the paper):
 *     input (d / 4 m, valid mask, (d - mean of the valid 3x3 neighbours) /
 *     5 cm), 3x3 convs, encoder 32 (stride 1), 64, 64,
 *     128 (stride 2 each); decoder nearest x2 upsampling + 3x3 conv to 64,
 *     64, 32 with the same-resolution encoder output added before the relu;
 *     head 3x3 conv 32 -> 1 (delta); output d + 5 cm * delta where d > 0, 0
 *     elsewhere (holes stay holes).
 * Activations are bfloat16 on the matrix cores with fp32 accumulation;
 * parameters have fp32 master copies.  Training minimises the mean |out -
 * target| over pixels valid in both, with Adam.
 *
 * Parameter vector: fp32, layers e1 e2 e3 e4 d3 d2 d1 head in this order,
 * each W[cout][3][3][cin] (row-major) followed by b[cout]; 259649 values.
 *
 * Conventions as in tsdf.h: int status (TF_OK or TF_E_*), d_* device
 * pointers owned by the caller, work enqueued on `stream` only, no device
 * allocation: the caller provides tf_nn_workspace_bytes() of device memory.
 */
#ifndef TSDF_NN_H
#define TSDF_NN_H

#include <stddef.h>
#include <stdint.h>

#include "tsdf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tf_nn tf_nn;   /* opaque, host-side */

/* tensors readable through tf_nn_tensor (ids) */
#define TF_NN_T_INPUT 0      /* x: batch x H x W x 8 bf16 (channels 3..7 zero) */
#define TF_NN_T_E1 1         /* e1..d1: post-relu activations, bf16 NHWC */
#define TF_NN_T_D1 7
#define TF_NN_T_GRAD_E1 8    /* 8..14: loss gradient at the pre-relu sums of e1..d1, bf16 NHWC */
#define TF_NN_T_OUT 15       /* output depth, fp32 metres, batch x H x W */
#define TF_NN_T_DDELTA 16    /* loss gradient at the head output, fp32 */
#define TF_NN_T_DEPTH 17     /* input depth in metres, fp32 */
#define TF_NN_T_GRADS 18     /* parameter gradients, fp32, parameter-vector layout */
#define TF_NN_T_PARAMS 19    /* fp32 master parameters */

uint32_t tf_nn_param_count(void);

/* Device bytes for batches of up to max_batch frames of height x width
 * (both multiples of 8, at most 4096); training adds the gradient, Adam and
 * backward buffers.  0 for bad arguments. */
size_t tf_nn_workspace_bytes(uint32_t max_batch, uint32_t height, uint32_t width, int training);

int tf_nn_create(uint32_t max_batch, uint32_t height, uint32_t width, int training, void *d_workspace,
                 size_t bytes, tf_nn **out);
int tf_nn_destroy(tf_nn *nn);   /* host state only */

/* Copy an fp32 parameter vector (device) in; repacks the bf16 operands and,
 * when training, clears the Adam moments and step count. */
int tf_nn_set_params(tf_nn *nn, const float *d_params, tf_stream stream);
int tf_nn_get_params(tf_nn *nn, float *d_params, tf_stream stream);

/* out = filtered depth of `batch` frames (d_depth: batch x H x W, uint16 mm
 * or fp32 metres per depth_format; d_out: batch x H x W fp32 metres).
 * Keeps the activations for tf_nn_backward. */
int tf_nn_forward(tf_nn *nn, const void *d_depth, int depth_format, uint32_t batch, float *d_out, tf_stream stream);

/* After tf_nn_forward (training instances): loss against d_target (batch x
 * H x W fp32 metres, 0 = no target) and every parameter gradient.  d_loss:
 * 2 device floats, the mean and the pixel count. */
int tf_nn_backward(tf_nn *nn, const float *d_target, float *d_loss, tf_stream stream);

/* One Adam update of the master parameters with the last gradients (step
 * count kept by the instance), then the bf16 operands are repacked. */
int tf_nn_adam_step(tf_nn *nn, float lr, float beta1, float beta2, float eps, tf_stream stream);

/* Device pointer and dims (n, h, w, c) of an internal tensor (ids above);
 * valid until the next call that writes it.  TF_E_INVAL for ids the
 * instance does not hold (gradients of an inference instance). */
int tf_nn_tensor(tf_nn *nn, int id, const void **d_ptr, int32_t dims[4]);

#ifdef __cplusplus
}
#endif

#endif /* TSDF_NN_H */
