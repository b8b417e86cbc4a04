/*
 * tsdf_surfel.h -- C ABI of surfel fusion in libtsdf.so (gfx950).
 *
 * Sec. 7.3 of "InfiniTAM v3" (arXiv:1708.00783), Keller et al.'s surfel-based
 * reconstruction: a surfel has a position v, normal n, radius r, confidence c
 * and time stamp t.  Per frame every input pixel u gives a world point
 * v^g(u) and normal n^g(u); all surfels are forward-projected into the image
 * as circles, their indices written into an index map; a point's
 * corresponding surfel is the one at its pixel, updated by the weighted
 * average v <- (c v + alpha v^g) / (c + alpha), n likewise, c <- c + alpha,
 * t <- now; a point without one becomes a new surfel with c = alpha.
 *
 * Readings where the paper is silent:
 *   - input point v^c = d ((x - cx) / fx, (y - cy) / fy, 1), to the world with
 *     the inverse of pose_w2c; input normal from forward differences to the
 *     right and lower neighbours, normalised and turned to face the camera (the
 *     last row and column have none; a pixel needs a depth and a normal);
 *   - alpha = exp(-gamma^2 / (2 sigma^2)), gamma = the pixel's distance from
 *     the principal point over |(cx, cy)|;
 *   - radius r = d sqrt(2) / (2 fx) when the surfel is made, unchanged later;
 *   - index map: a surfel in front of the camera covers the pixels within
 *     rho = min(fx r / z, 8) pixels of its projection; a pixel keeps the
 *     covering surfel of least camera z, ties to the smaller index;
 *   - a pixel's surfel corresponds only if |d(u) - z| <= max_depth_diff and
 *     n^g . n >= min_normal_dot |n|;
 *   - a surfel with several corresponding points takes them all at once,
 *     (c v + sum alpha_i v_i) / (c + sum alpha_i): the paper's update applied
 *     one point after another, in any order;
 *   - new surfels are appended in pixel raster order; beyond the capacity
 *     they are dropped and TF_FLAG_SURFEL_OVERFLOW is raised;
 *   - no removal or merging (not described in the paper).
 * Decisions (coverage, depth order, gates, validity) are float32 in a fixed
 * operation order; the update sums are float32 in raster order over each
 * surfel's circle, so a frame is bit-reproducible.
 *
 * Conventions as in tsdf.h.
 */
#ifndef TSDF_SURFEL_H
#define TSDF_SURFEL_H

#include "tsdf.h"

#ifdef __cplusplus
extern "C" {
#endif

#define TF_FLAG_SURFEL_OVERFLOW 0x20u   /* new surfels beyond the capacity were dropped */

typedef struct tf_surfels tf_surfels;   /* opaque, host-side */

typedef struct {
    uint32_t capacity;        /* surfels, 1..2^26 */
    int32_t max_width;        /* largest depth image, 1..8192 */
    int32_t max_height;
    float sigma;              /* alpha falloff, > 0 (Keller et al.: 0.6) */
    float max_depth_diff;     /* metres, > 0 */
    float min_normal_dot;     /* -1..1 */
} tf_surfel_params;

/* Device bytes of a surfel map (0 if the parameters are invalid): 36 bytes per
 * surfel plus 64 bytes per pixel of per-frame buffers. */
size_t tf_surfel_workspace_bytes(const tf_surfel_params *p);

/* Create an empty map in d_workspace (256-byte aligned, caller-owned); enqueues
 * its initialisation on `stream`. */
int tf_surfel_create(const tf_surfel_params *p, void *d_workspace, size_t bytes, tf_stream stream, tf_surfels **out);
int tf_surfel_destroy(tf_surfels *m);                 /* host state only */
int tf_surfel_reset(tf_surfels *m, tf_stream stream); /* empty the map */

/* Fuse one depth frame (TF_DEPTH_U16_MM or TF_DEPTH_F32_M, at most max_width x
 * max_height) taken at pose_w2c (M_d, world->camera).  Enqueue-only. */
int tf_surfel_fuse(tf_surfels *m, const void *d_depth, int depth_format, const tf_intrinsics *intr,
                   const float pose_w2c[16], tf_stream stream);

/* Synchronising: surfel count, sticky flags and frames fused. */
int tf_surfel_stats(tf_surfels *m, uint32_t *h_count, uint32_t *h_flags, uint32_t *h_frames, tf_stream stream);

/* Copy the first n surfels (n <= count): d_pos n x 4 floats (x, y, z, radius),
 * d_nrm n x 4 floats (nx, ny, nz, confidence), d_time n int32 (frame index of
 * the last update, 0-based).  Enqueue-only. */
int tf_surfel_export(tf_surfels *m, uint32_t n, float *d_pos, float *d_nrm, int32_t *d_time, tf_stream stream);

/* The last fused frame's index map (surfel index or -1) and correspondence of
 * every pixel (surfel index, -1 for a new surfel, -2 for no input point),
 * width x height int32 each of that frame (either may be NULL).  Enqueue-only. */
int tf_surfel_export_frame(tf_surfels *m, int32_t *d_index_map, int32_t *d_corr, tf_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* TSDF_SURFEL_H */
