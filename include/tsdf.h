/*
 * tsdf.h -- C ABI of libtsdf.so, a gfx950 (MI355X) implementation of the
 * per-frame hot path of voxel-hashed TSDF fusion as described in
 * "InfiniTAM v3: A Framework for Large-Scale 3D Reconstruction with Loop
 * Closure" (Prisacariu et al., arXiv:1708.00783).
 *
 * Per depth frame the caller runs
 *     tf_alloc_and_visible(depth, intrinsics, pose)   Sec. 4.2 (allocation)
 *     tf_integrate(depth, pose)                       Sec. 4.3 (integration)
 *     tf_raycast(pose, intrinsics) -> points, normals Sec. 4.4 (raycast)
 * and, with host swapping enabled, tf_swap_out after the raycast (Sec. 5).
 *
 * Conventions shared by every call
 *   - Every function returns an int status: TF_OK (0) or a negative TF_E_*.
 *   - Argument errors (NULL pointers, sizes out of range, call order) are
 *     detected on the host before anything is enqueued; nothing is launched
 *     and the volume is unchanged.
 *   - Pointers named d_* are device pointers (HBM of the current HIP device),
 *     owned by the caller and left untouched by the library beyond the call's
 *     documented outputs.  Pointers named h_* are host pointers.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is only
 *     enqueued on it; calls return without waiting, except those documented
 *     as synchronising (tf_get_stats, the tf_export_* calls, tf_swap_out,
 *     tf_save and tf_load).
 *   - pose_w2c is the paper's M_d (Sec. 4.3): the 4x4 rigid world->camera
 *     transform, 16 host floats, row-major, last row (0 0 0 1).  The library
 *     inverts it itself; its rotation block must be orthonormal.
 *   - The volume lives in a caller-provided device workspace of
 *     tf_workspace_bytes() bytes; the library never allocates device memory.
 *   - Capacity overflow during a frame does not fail the call: requests that
 *     do not fit are dropped (the paper likewise lets a later frame pick up
 *     what one frame missed, Sec. 4.2) and a sticky flag is raised, readable
 *     with tf_get_stats.
 */
#ifndef TSDF_H
#define TSDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define TF_OK 0
#define TF_E_INVAL (-1)   /* bad argument (NULL, size, alignment, range) */
#define TF_E_HIP (-2)     /* a HIP runtime call failed */
#define TF_E_ORDER (-3)   /* call order violated (e.g. integrate before alloc) */
#define TF_E_SPACE (-4)   /* workspace smaller than tf_workspace_bytes() */
#define TF_E_IO (-5)      /* file not opened, read or written, or not a volume of these parameters */

/* ---- sticky overflow flags (tf_stats.flags) ---------------------------- */
#define TF_FLAG_BLOCKS_EXHAUSTED 0x1u   /* the free-block stack ran empty (Sec. 4.2) */
#define TF_FLAG_EXCESS_EXHAUSTED 0x2u   /* the excess list ran out of slots (Sec. 3.2) */
#define TF_FLAG_REQUEST_OVERFLOW 0x4u   /* more new blocks in one frame than n_blocks */
#define TF_FLAG_TRANSFER_OVERFLOW 0x8u  /* swap candidates beyond the transfer buffer (Sec. 5, O1) */
#define TF_FLAG_BIN_OVERFLOW 0x10u      /* batched raycast: block x tile entries beyond the bin capacity */

typedef struct tf_ctx tf_ctx;    /* opaque, host-side */
typedef void *tf_stream;         /* hipStream_t */

typedef enum { TF_DEPTH_F32_M = 0, TF_DEPTH_U16_MM = 1 } tf_depth_format;

/* Pinhole intrinsics (Sec. 4.3 projParams_d = fx, fy, cx, cy) and image size. */
typedef struct {
    float fx, fy, cx, cy;
    int32_t width, height;
} tf_intrinsics;

/* Scene parameters (Sec. 3.1, 3.2, 4.3 and the swapping mode of Sec. 6). */
typedef struct {
    float voxel_size;        /* metres per voxel, > 0 */
    float mu;                /* truncation band, metres, > 0 */
    int32_t max_w;           /* weight cap maxW, 1..255 */
    uint32_t n_buckets;      /* hash buckets (ordered part), power of two, 2^4..2^26 */
    uint32_t n_excess;       /* excess-list slots (unordered part), 1..2^26 */
    uint32_t n_blocks;       /* voxel block array size, 1..2^24 */
    uint32_t max_width;      /* largest image passed to any call, 1..8192 */
    uint32_t max_height;     /* 1..8192 */
    uint32_t swap_transfer_blocks;  /* 0 = swapping disabled; else transfer buffer size */
} tf_params;

typedef struct {
    uint32_t flags;          /* TF_FLAG_* since creation/reset */
    uint32_t n_allocated;    /* blocks holding device data */
    uint32_t n_visible;      /* entries in the current visible list */
    uint32_t n_new;          /* blocks inserted by the last tf_alloc_and_visible */
    uint32_t n_free_excess;  /* unused excess slots */
    uint32_t n_swapped_in;   /* blocks fused from the host store by the last frame */
    uint32_t n_swapped_out;  /* blocks moved to the host store by the last tf_swap_out */
    uint32_t frames;         /* tf_alloc_and_visible calls since creation/reset */
    /* work totals since creation/reset (counted on the device) */
    uint64_t total_integrated_blocks;  /* visible blocks visited by tf_integrate (x512 voxels) */
    uint64_t total_written_columns;    /* 8-voxel columns (24 bytes) written back by tf_integrate */
    uint64_t total_range_records;      /* search-range records behind tf_raycast calls: one per visible
                                          block for the allocation view (an off-image block's record is
                                          empty), one per projected block for any other view */
    uint64_t total_rays_hit;           /* tf_raycast pixels with a surface hit */
    uint64_t total_requests;           /* unique insertion requests */
    uint64_t total_new_blocks;         /* blocks inserted */
    uint64_t integrate_calls;
    uint64_t raycast_calls;
} tf_stats;

/* Kernel classes timed by the optional profiler. */
enum {
    TF_K_ALLOC_RAYS = 0,   /* ray segments, probes, marks, requests (Sec. 4.2 part 1) */
    TF_K_INSERT = 1,       /* insertion and frustum re-test (Sec. 4.2 parts 2-3) */
    TF_K_VISIBLE = 2,      /* visible-list compaction (Sec. 4.2 part 3) */
    TF_K_INTEGRATE = 3,    /* integration, including any depth conversion (Sec. 4.3) */
    TF_K_RANGE_BIN = 4,    /* block projection into tile bins (Sec. 4.4) */
    TF_K_RAYCAST = 5,      /* per-tile search range and ray march (Sec. 4.4) */
    TF_K_SWAP = 6,         /* swap-in / swap-out kernels (Sec. 5) */
    TF_K_COUNT = 7
};

typedef struct {
    uint64_t launches[8];  /* timed launches per TF_K_* class */
    double ms[8];          /* summed device time (HIP events on the launch stream) */
} tf_profile;

/* Device bytes the volume needs for these parameters (0 if they are invalid). */
size_t tf_workspace_bytes(const tf_params *p);

/* Bytes of the host swap store (one 1536-byte block per hash entry, the
 * host voxel block array of Sec. 5 O2) and of the pinned host transfer buffer
 * (Sec. 5 O1); 0 when swapping is disabled. */
size_t tf_host_store_bytes(const tf_params *p);
size_t tf_host_transfer_bytes(const tf_params *p);

/* Create a volume in d_workspace (256-byte aligned, `bytes` >= tf_workspace_bytes).
 * With swapping enabled, h_store (tf_host_store_bytes, any host memory) and
 * h_transfer (tf_host_transfer_bytes, pinned: hipHostMalloc) are required;
 * both stay owned by the caller and must outlive the context.  The workspace
 * is initialised on `stream` (every entry unallocated, free lists full). */
int tf_create(const tf_params *p, void *d_workspace, size_t bytes, void *h_store,
              void *h_transfer, tf_stream stream, tf_ctx **out);
int tf_destroy(tf_ctx *ctx);
/* Return the volume to its freshly created state (enqueued on `stream`). */
int tf_reset(tf_ctx *ctx, tf_stream stream);

/* Allocation and visible list (Sec. 4.2).  d_depth: width*height values,
 * row-major, TF_DEPTH_F32_M (float metres) or TF_DEPTH_U16_MM (uint16
 * millimetres, converted as (float)mm / 1000); 0 = no measurement.
 * For every pixel with depth d > 0 the blocks along the ray segment between
 * camera depths d - mu and d + mu are looked up and missing ones inserted;
 * the visible list becomes the touched blocks plus the previous frame's
 * visible blocks that still have a corner inside the image. */
int tf_alloc_and_visible(tf_ctx *ctx, const void *d_depth, int depth_format,
                         const tf_intrinsics *intr, const float pose_w2c[16], tf_stream stream);

/* Integration (Sec. 4.3): the running-average update of every voxel of every
 * visible block from the depth map of the last tf_alloc_and_visible (same
 * size and intrinsics).  TF_E_ORDER if no allocation preceded it. */
int tf_integrate(tf_ctx *ctx, const void *d_depth, int depth_format, const float pose_w2c[16],
                 tf_stream stream);

/* Raycast (Sec. 4.4).  d_points, d_normals: width*height float4 each,
 * row-major, world frame; (x, y, z, 1) on a hit and zeros otherwise; a normal
 * is (nx, ny, nz, 1) when its SDF gradient is non-zero.  The search range is
 * the forward projection of the visible list when pose and intrinsics equal
 * those of the last tf_alloc_and_visible, else of every block with device
 * data. */
int tf_raycast(tf_ctx *ctx, const float pose_w2c[16], const tf_intrinsics *intr,
               float *d_points, float *d_normals, tf_stream stream);

/* The search range of tf_raycast on its own (Sec. 4.4): per pixel the min
 * and max camera z of the blocks whose projection covers it; +inf / -inf
 * where no block does.  d_zmin, d_zmax: width*height floats. */
int tf_range_image(tf_ctx *ctx, const float pose_w2c[16], const tf_intrinsics *intr,
                   float *d_zmin, float *d_zmax, tf_stream stream);

/* Swap out (Sec. 5): entries with device data that are not in the current
 * visible list move to the host store (lowest entry index first, at most
 * swap_transfer_blocks per call); their device blocks return to the free
 * stack and the entries are marked ptr = -1.  Synchronises `stream` (the
 * host copies the transfer buffer into the store).  TF_E_INVAL if swapping is
 * disabled. */
int tf_swap_out(tf_ctx *ctx, tf_stream stream);

/* Copies of host-store blocks (swapping only; synchronous host work): for
 * each of n entries, 512 voxels in the in-block order lx + 8 ly + 64 lz and,
 * in h_has (may be NULL), 1 if the store holds data for the entry (else the
 * default voxel is written).  TF_E_INVAL without swapping. */
int tf_export_host_voxels(tf_ctx *ctx, const int32_t *h_entries, uint32_t n, int16_t *h_sdf, uint8_t *h_w,
                          uint8_t *h_has);

/* Optional per-kernel timing: with `on` != 0 every later launch is bracketed
 * by a pair of HIP events recorded on its stream (a small host cost per
 * launch).  tf_profile_read synchronises on the outstanding events, returns
 * the totals and, if `reset` != 0, zeroes them. */
int tf_profile_enable(tf_ctx *ctx, int on);
/* Time only the kernel classes in class_mask (bit TF_K_*), and of each only
 * every `every`-th launch (every >= 1): each timed launch costs two event
 * records on the stream.  Default: all classes, every launch. */
int tf_profile_select(tf_ctx *ctx, uint32_t class_mask, uint32_t every);
int tf_profile_read(tf_ctx *ctx, tf_profile *h_out, int reset);

/* Counters and sticky flags.  Synchronises `stream`. */
int tf_get_stats(tf_ctx *ctx, tf_stats *h_out, tf_stream stream);

/* Copies of the hash table for inspection (synchronising): n_buckets +
 * n_excess entries, h_pos as 3 int16 per entry, h_offset and h_ptr one int32
 * each (Sec. 3.2 layout: offset k >= 1 -> entry n_buckets + k - 1, 0 = end of
 * chain; ptr >= 0 block, -1 swapped out, < -1 unallocated).  Any of the
 * three may be NULL. */
int tf_export_entries(tf_ctx *ctx, int16_t *h_pos, int32_t *h_offset, int32_t *h_ptr,
                      tf_stream stream);

/* The current visible list (entry indices, unordered).  Writes at most `cap`
 * indices and the full count to *h_count.  Synchronising. */
int tf_export_visible(tf_ctx *ctx, int32_t *h_list, uint32_t cap, uint32_t *h_count,
                      tf_stream stream);

/* Voxels of n entries (each should hold device data), 512 per entry in the
 * in-block order lx + 8 ly + 64 lz: short SDF (32767 == 1.0) and uchar
 * weight.  d_entries: n int32 entry indices; d_sdf: n*512 int16; d_w: n*512
 * uint8 (all device).  An entry without a device block yields the default
 * voxel (32767, 0).  Enqueued only. */
int tf_export_voxels(tf_ctx *ctx, const int32_t *d_entries, uint32_t n, int16_t *d_sdf,
                     uint8_t *d_w, tf_stream stream);

/* ==========================================================================
 * Rigid submaps, batched (Sec. 7.2)
 *
 * A batched map holds n_submaps independent volumes of identical parameters,
 * each with a fixed rigid pose P_i (world -> submap, row-major 4x4).  A depth
 * frame is fused into a caller-chosen subset of them: submap i sees the
 * camera M_d P_i^-1 (composed in double, rounded once to float).  Views are
 * raycast on the combined field of all submaps: at a world point X the
 * trilinear SDFs F_i(P_i X) averaged with their trilinear weights W_i(P_i X)
 * as weights, over the submaps with W_i > 0 (one such submap gives F_i
 * unchanged, none gives 1); a point counts as allocated when any submap has
 * a block at floor(P_i X).  The search range of a pixel is taken over the
 * blocks of every submap.  Submaps never swap.
 *
 * Memory: device workspace tf_multi_workspace_bytes() and a pinned host
 * parameter buffer of tf_multi_host_bytes() (hipHostMalloc'd), both owned by
 * the caller.  Per call the library writes the frame's parameters into the
 * pinned buffer (two alternating halves; it waits for the frame before last
 * to finish with a half before overwriting it) and copies them to the device
 * on the stream.
 * ========================================================================== */
typedef struct tf_multi tf_multi;   /* opaque, host-side */

#define TF_MULTI_MAX_SUBMAPS 64
#define TF_MULTI_MAX_SELECT 12       /* submaps one frame is fused into */
#define TF_MULTI_MAX_VIEWS 8

typedef struct {
    tf_intrinsics intr;   /* width x height at most the map's view bound */
    float pose_w2c[16];   /* world -> camera of the view */
    float *d_points;      /* height x width x 4 device floats: world hit point, w = 1 on a hit, else all 0 */
    float *d_normals;     /* height x width x 4: unit normal of the combined field, w = 1 where valid */
} tf_view;

/* launch shapes, chosen by tf_multi_autotune or set by the caller */
typedef struct {
    int32_t tile_w, tile_h;        /* raycast tile: 16x16, 32x8, 16x8 or 8x8 pixels, one workgroup each */
    int32_t integrate_threads;     /* threads per integration workgroup: 64, 128, 256 or 512 */
    int32_t integrate_groups;      /* integration workgroups per selected submap, 1..2048 */
    int32_t bin_groups;            /* workgroups per view of the binning passes, 1..65535 */
} tf_multi_config;

typedef struct {
    uint32_t flags;                     /* OR of every submap's flags and TF_FLAG_BIN_OVERFLOW */
    uint32_t n_submaps;
    uint64_t allocated_blocks;          /* sum over submaps */
    uint64_t total_integrated_blocks;   /* sum over submaps: blocks visited by integrations */
    uint64_t total_written_columns;     /* sum over submaps: 8-voxel columns written back */
    uint64_t total_bin_entries;         /* (block, tile) pairs binned by all raycasts */
    uint64_t total_block_views;         /* (block, view) pairs binned by all raycasts */
    uint64_t total_rays_hit;            /* pixels with a hit over all raycasts and views */
    uint64_t raycast_calls;
} tf_multi_stats;

/* Device workspace for n_submaps submaps of parameters p (p->max_width x
 * p->max_height bounds the depth frames; swap_transfer_blocks must be 0),
 * views up to view_w x view_h, and bin_capacity (block, tile) entries per
 * raycast call over all its views, plus 256 MiB of world-cell submap masks
 * (which submaps' blocks reach each 8-voxel world cell).  0 if an argument
 * is out of range. */
size_t tf_multi_workspace_bytes(const tf_params *p, uint32_t n_submaps, uint32_t view_w, uint32_t view_h,
                                uint32_t bin_capacity);
/* Bytes of the pinned host parameter buffer. */
size_t tf_multi_host_bytes(void);

/* poses: n_submaps x 16 host floats (P_i).  Enqueues the initialisation of
 * every submap on `stream`.  *out receives the handle.  TF_E_SPACE when
 * bytes < tf_multi_workspace_bytes(), TF_E_INVAL for other bad arguments. */
int tf_multi_create(const tf_params *p, uint32_t n_submaps, const float *poses, uint32_t view_w, uint32_t view_h,
                    uint32_t bin_capacity, void *d_workspace, size_t bytes, void *h_pinned, size_t h_bytes,
                    tf_stream stream, tf_multi **out);
int tf_multi_destroy(tf_multi *m);   /* frees host state only; waits for nothing */

/* Borrowed handle of submap i (valid until tf_multi_destroy): every
 * single-volume call applies to it (exports, statistics, its own frames in
 * its own coordinates). */
int tf_multi_submap(tf_multi *m, uint32_t i, tf_ctx **out);

int tf_multi_set_config(tf_multi *m, const tf_multi_config *c);   /* TF_E_INVAL for unsupported shapes */
int tf_multi_get_config(const tf_multi *m, tf_multi_config *c);

/* Fuse one frame (allocation, visible lists and integration of Sec. 4.2-4.3)
 * into the submaps sel[0..n_sel-1] (distinct, 1 <= n_sel <= 12), each with
 * camera pose_w2c P_i^-1.  The frame is at most p->max_width x p->max_height. */
int tf_multi_integrate(tf_multi *m, const void *d_depth, int depth_format, const tf_intrinsics *intr,
                       const float pose_w2c[16], const uint32_t *sel, uint32_t n_sel, tf_stream stream);

/* Raycast the combined field into views[0..n_views-1] (1 <= n_views <= 8). */
int tf_multi_raycast(tf_multi *m, const tf_view *views, uint32_t n_views, tf_stream stream);

/* tf_multi_integrate followed by tf_multi_raycast.  With use_graph != 0 the
 * launches are captured once into a HIP graph per (frame size, view sizes,
 * launch shapes) and replayed: a replay only rewrites the pinned parameters. */
int tf_multi_frame(tf_multi *m, const void *d_depth, int depth_format, const tf_intrinsics *intr,
                   const float pose_w2c[16], const uint32_t *sel, uint32_t n_sel, const tf_view *views,
                   uint32_t n_views, int use_graph, tf_stream stream);

/* Per-pixel search range of one view over every submap's blocks: d_zmin,
 * d_zmax (height x width device floats, camera z; +inf / -inf where no block
 * projects). */
int tf_multi_range_image(tf_multi *m, const tf_view *view, float *d_zmin, float *d_zmax, tf_stream stream);

/* Time every supported launch shape on this frame and these views (reps
 * timed repetitions each) and keep the fastest.  Integration shapes are timed
 * with a dry pass that computes every update and stores none; the frame's
 * allocation runs once, as the frame's own integration would run it, so the
 * map changes only by the blocks this frame allocates.  The views' outputs
 * are overwritten.  Synchronising.  best / best_ms (frame ms of the chosen
 * shapes) may be NULL. */
int tf_multi_autotune(tf_multi *m, const void *d_depth, int depth_format, const tf_intrinsics *intr,
                      const float pose_w2c[16], const uint32_t *sel, uint32_t n_sel, const tf_view *views,
                      uint32_t n_views, int reps, tf_multi_config *best, float *best_ms, tf_stream stream);

/* Synchronising. */
int tf_multi_get_stats(tf_multi *m, tf_multi_stats *out, tf_stream stream);

/* ==========================================================================
 * Persistence of a volume (the scene parameters and the map of Sec. 3 and
 * Sec. 6: hash table, free lists, voxel blocks, visible list and, with
 * swapping, the host store of Sec. 5)
 * ========================================================================== */

/* Write the volume to the file at `path` (created or truncated): scene
 * parameters, hash entries, both free stacks, the visible list, the
 * occupancy bits, the voxel blocks in use (runs of consecutive block
 * indices), the work counters and, with swapping, the host-store blocks the
 * store holds.  Waits for `stream` first and reads the device synchronously;
 * the volume is unchanged.  TF_E_INVAL for NULL arguments or a submap handle
 * of a batched map; TF_E_IO when the file cannot be written. */
int tf_save(tf_ctx *ctx, const char *path, tf_stream stream);

/* Replace the volume's state by the one saved at `path`.  The context must
 * have been created with parameters equal to the saved ones (every tf_params
 * field), else TF_E_IO and the volume is unchanged.  Synchronising.  After a
 * load the volume is block for block, entry for entry and counter for
 * counter the saved one (allocation continues from the same free stacks, so
 * a later frame allocates the same block indices); the next frame starts with
 * tf_alloc_and_visible (tf_integrate before it returns TF_E_ORDER).  If the
 * file ends early or holds inconsistent sizes, TF_E_IO and the volume is
 * left reset (empty). */
int tf_load(tf_ctx *ctx, const char *path, tf_stream stream);

/* ==========================================================================
 * Training targets of the learned prefilter (see tsdf_nn.h)
 * ========================================================================== */

/* Camera depth of raycast hit points: for each of width x height pixels,
 * d_depth = the camera z of the world point d_points (float4 as written by
 * tf_raycast, w = 1 on a hit) under pose_w2c, each row evaluated as
 * ((m8 x + m9 y) + m10 z) + m11; 0 where w != 1.  d_points: width*height*4
 * device floats (16-byte aligned), d_depth: width*height device floats.
 * Enqueued only. */
int tf_camera_depth(const float *d_points, int32_t width, int32_t height, const float pose_w2c[16],
                    float *d_depth, tf_stream stream);

/* Human-readable name of a status code. */
const char *tf_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif /* TSDF_H */
