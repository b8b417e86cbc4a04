/*
 * tsdf_filter.h -- C ABI of the bilateral depth filter of libtsdf.so (gfx950).
 *
 * The paper's view builder may apply a bilateral filter to the processed
 * depth image before tracking and fusion use it (Sec. 4, image preparation;
 * the useBilateralFilter setting of Sec. 6).  The paper gives no formula;
 * this is the standard bilateral filter restricted to valid depths:
 *
 *     out(p) = sum_q w(p, q) d(q) / sum_q w(p, q),
 *     w(p, q) = exp(-|p - q|^2 / (2 sigma_space^2)) exp(-(d(p) - d(q))^2 / (2 sigma_range^2)),
 *
 * over the (2 radius + 1)^2 window of pixels q inside the image with d(q) > 0;
 * out(p) = 0 where d(p) is not valid (holes are not filled).  Arithmetic is
 * float32: spatial weights rounded from float64, the mean accumulated as
 * d(p) + sum w (d(q) - d(p)) / sum w.
 *
 * Conventions as in tsdf.h: int status, d_* device pointers owned by the
 * caller, enqueue-only on `stream`.
 */
#ifndef TSDF_FILTER_H
#define TSDF_FILTER_H

#include "tsdf.h"

#ifdef __cplusplus
extern "C" {
#endif

#define TF_BILATERAL_MAX_RADIUS 7

typedef struct {
    int32_t radius;       /* window half-width in pixels, 1..7 */
    float sigma_space;    /* pixels, > 0 */
    float sigma_range;    /* metres, > 0 */
} tf_bilateral_params;

/* Filter the depth image d_depth (width x height; TF_DEPTH_U16_MM, converted
 * as (float)mm / 1000, or TF_DEPTH_F32_M; 0 = invalid) into d_out (width x
 * height float32 metres; must not overlap d_depth).  TF_E_INVAL for NULL
 * pointers, misaligned buffers, sides outside 1..8192 or parameters out of
 * range; TF_E_HIP if the launch fails. */
int tf_bilateral(const void *d_depth, int depth_format, int32_t width, int32_t height,
                 const tf_bilateral_params *params, float *d_out, tf_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* TSDF_FILTER_H */
