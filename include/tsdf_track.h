/*
 * tsdf_track.h -- C ABI of the depth tracker of libtsdf.so (gfx950).
 *
 * Sec. 4.1.1 (ITMDepthTracker) of "InfiniTAM v3" (arXiv:1708.00783): the pose
 * of a new depth image is found by aligning it with the surface point map V
 * and normal map N that the raycast (tf_raycast, Sec. 4.4) rendered from a
 * reference pose.  Each live depth point p, moved into the world by the
 * current estimate (R, t), is projected into the reference image to the pixel
 * p_bar and scored by its distance from the plane through V(p_bar) with
 * normal N(p_bar), d = (R p + t - V(p_bar))^T N(p_bar); (R, t) minimises the
 * sum of d^2 through a linear system; the two steps repeat, over a resolution
 * hierarchy of the depth image from the coarsest level to the finest.  As the
 * paper splits the work, the device computes the per-pixel terms and their
 * sums; here the 6x6 solve runs on the device as well (one thread, float64),
 * so a whole call is enqueue-only and can be captured in a HIP graph.
 *
 * Readings where the paper is silent:
 *   - the estimate is camera->world (R, t) in float64, used in float32 by the
 *     per-pixel arithmetic; poses at the boundary are world->camera (M_d);
 *   - the residual is linearised in a world-frame increment (omega, dt):
 *     q -> Exp(omega) q + dt with q = R p + t, Jacobian row (q x n, n); the
 *     normal equations (sum J^T J) xi = -(sum J^T d) are solved by Cholesky,
 *     R <- Exp(omega) R, t <- Exp(omega) t + dt (Rodrigues);
 *   - association: the nearest reference pixel floor(u + 0.5) of q projected
 *     with the reference pose and intrinsics, u = (fx c_x) / c_z + cx, needing
 *     c_z > 0, a pixel inside the reference image, V and N valid (w == 1) and
 *     |q - V| <= dist_thresh of the level;
 *   - level l + 1 halves level l (floor of the sizes); a coarse depth is the
 *     mean of the valid (> 0) depths of its 2x2 block, 0 if none; level-l
 *     intrinsics fx / 2^l, fy / 2^l, (cx + 0.5) / 2^l - 0.5, (cy + 0.5) / 2^l
 *     - 0.5; the reference maps keep their own resolution at every level;
 *   - per-pixel arithmetic is float32 in a fixed order (no contraction); the
 *     sums are float64 in a fixed order, so a call is bit-reproducible.
 *
 * Conventions as in tsdf.h: int status (TF_OK or TF_E_*), d_* device
 * pointers owned by the caller, enqueue-only on `stream`.
 */
#ifndef TSDF_TRACK_H
#define TSDF_TRACK_H

#include "tsdf.h"

#ifdef __cplusplus
extern "C" {
#endif

#define TF_TRACK_MAX_LEVELS 4

typedef struct {
    int32_t n_levels;                          /* 1..4 */
    int32_t iterations[TF_TRACK_MAX_LEVELS];   /* updates per level, index 0 = finest; 0..100 each */
    float dist_thresh[TF_TRACK_MAX_LEVELS];    /* metres, > 0: pairs with |q - V| beyond it are dropped */
    float min_update;                          /* a level stops after an update with |xi|_2 below this
                                                  (xi = (omega rad, dt m)); 0 = always run every iteration */
} tf_track_params;

/* Written to device memory at the end of tf_track (1000 bytes; 8-byte aligned). */
typedef struct {
    float pose_w2c[16];                        /* the estimate, world->camera, row-major, last row 0 0 0 1 */
    int32_t iterations[TF_TRACK_MAX_LEVELS];   /* updates applied per level */
    int32_t pairs[TF_TRACK_MAX_LEVELS];        /* pairs of the last system evaluated at the level */
    int32_t status;                            /* bit l: level l stopped on a degenerate system (fewer
                                                  than 6 pairs or a matrix not positive definite) */
    int32_t pad;
    double sums[TF_TRACK_MAX_LEVELS][28];      /* per level, the last evaluated system: sum J^T J (upper
                                                  triangle, row-major, 21), sum J^T d (6), sum d^2 */
} tf_track_result;

/* Device bytes of the tracker's workspace for a depth image of width x
 * height with n_levels levels (0 if the sizes are out of range). */
size_t tf_track_workspace_bytes(int32_t width, int32_t height, int32_t n_levels);

/* Estimate the world->camera pose of the depth image d_depth (width x height
 * of `intr`; TF_DEPTH_U16_MM or TF_DEPTH_F32_M as in tf_integrate; 0 =
 * invalid) against the reference maps d_ref_points / d_ref_normals (float4
 * world points and normals as written by tf_raycast, w == 1 valid, 16-byte
 * aligned, ref_intr->width x ref_intr->height, rendered with ref_pose_w2c),
 * starting from init_pose_w2c.  d_workspace: tf_track_workspace_bytes()
 * bytes of device memory, 256-byte aligned, used as scratch (its contents on
 * entry do not matter).  d_result: device memory for one tf_track_result.
 * Enqueue-only.  TF_E_INVAL for NULL pointers, misaligned buffers, sizes or
 * parameters out of range (image sides 1..8192, every level at least 1x1,
 * non-positive focal lengths or thresholds); TF_E_SPACE for a workspace
 * smaller than required; TF_E_HIP if a launch fails. */
int tf_track(const void *d_depth, int depth_format, const tf_intrinsics *intr, const float *d_ref_points,
             const float *d_ref_normals, const tf_intrinsics *ref_intr, const float ref_pose_w2c[16],
             const float init_pose_w2c[16], const tf_track_params *params, void *d_workspace,
             size_t workspace_bytes, tf_track_result *d_result, tf_stream stream);

/* Largest workspace tf_track_noalloc can serve (8 MiB: e.g. 1280x1024 depth
 * with four levels). */
#define TF_TRACK_NOALLOC_MAX_BYTES (8u << 20)

/* tf_track for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same computation and result, bit for bit, with the workspace taken from a
 * fixed device array of TF_TRACK_NOALLOC_MAX_BYTES that the library holds on
 * every GPU it runs on until the process ends (looked up on the first call on
 * a device).  Allocates nothing.  Every call on one GPU shares that array:
 * calls that overlap on one GPU (different streams, or threads without
 * ordering) race and must not be issued; calls in one stream order are safe
 * (each call initialises what it reads).  TF_E_SPACE when
 * tf_track_workspace_bytes(width, height, n_levels) exceeds the array; other
 * errors as tf_track. */
int tf_track_noalloc(const void *d_depth, int depth_format, const tf_intrinsics *intr, const float *d_ref_points,
                     const float *d_ref_normals, const tf_intrinsics *ref_intr, const float ref_pose_w2c[16],
                     const float init_pose_w2c[16], const tf_track_params *params, tf_track_result *d_result,
                     tf_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* TSDF_TRACK_H */
