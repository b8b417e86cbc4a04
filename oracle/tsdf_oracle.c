/*
 * tsdf_oracle.c -- plain, slow CPU oracle for voxel-hashed TSDF fusion.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the tests, the package's smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * What it computes (InfiniTAM v3, arXiv:1708.00783):
 *   - the voxel (short SDF, uchar weight; initial 32767 == 1.0, weight 0)   Sec. 3.1
 *   - the hash entry {pos, offset, ptr} and its ptr sentinels              Sec. 3.2
 *   - hashIndex: xor of the three coordinates times three primes, masked   Sec. 3.2
 *   - bucket of size 1 plus an unordered excess list chained by `offset`   Sec. 3.2
 *   - retrieval (bucket, then chain walk; default voxel when absent)       Sec. 3.3
 *   - insertion from prepopulated free lists                               Sec. 3.3, 4.2
 *   - allocation along the segment [d-mu, d+mu] of every pixel ray        Sec. 4.2
 *   - the visible-block list                                               Sec. 4.2
 *   - the per-voxel running-average update (computeUpdatedVoxelDepthInfo)  Sec. 4.3
 *   - the forward-projected min/max depth search range                     Sec. 4.4
 *   - the raycasting state machine with trilinear reads and refinement     Sec. 4.4
 *
 * Arithmetic is IEEE binary32 as in the paper's listing of Sec. 4.3 (float
 * pt_camera, eta, oldF, newF).  Build with -O2 -ffp-contract=off and no
 * fast-math: every float operation below is one correctly rounded IEEE
 * operation in the order written.  Where the paper leaves the order of
 * operations open, the reading used is stated at the function.
 *
 * Allocation and insertion run serially (entry order follows pixel order).
 * Integration (per block) and raycasting (per pixel) use OpenMP work sharing;
 * each item writes only its own outputs, so results do not depend on the
 * thread count.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_SDF_BLOCK 8            /* 8x8x8 voxels per block, Sec. 3.1 */
#define OR_BLOCK_VOX 512
#define OR_PTR_SWAPPED (-1)       /* ptr == -1: block lives in host memory, Sec. 3.2 */
#define OR_PTR_EMPTY (-2)         /* ptr < -1: unallocated, Sec. 3.2 */
#define OR_SDF_INIT 32767         /* short SDF initial value, == 1.0, Sec. 3.1 */
#define OR_Z_NEAR 0.05f           /* near plane of the search-range projection */
#define OR_MAX_RAY_STEPS 65536    /* hard bound on raycast iterations */
#define OR_MAX_SEGMENT_SAMPLES 64 /* samples kept per pixel segment */

#define OR_FLAG_BLOCKS_EXHAUSTED 1u
#define OR_FLAG_EXCESS_EXHAUSTED 2u
#define OR_FLAG_TRANSFER_OVERFLOW 8u

typedef struct {
    int16_t x, y, z;
    int32_t offset;   /* 0 = end of chain; k >= 1 -> entry n_buckets + k - 1 */
    int32_t ptr;      /* >= 0 block index, -1 swapped out, < -1 unallocated */
} or_entry;

typedef struct {
    float voxel_size, mu;
    int max_w;
    int n_buckets, n_excess, n_blocks;
    or_entry *e;
    int32_t *free_blocks;  int n_free_blocks;    /* stack of free block indices */
    int32_t *free_excess;  int n_free_excess;    /* stack of free excess slots */
    int16_t *sdf;          /* [block][lx + 8 ly + 64 lz] */
    uint8_t *w;
    int32_t *visible;      int n_visible;        /* ascending entry indices */
    uint8_t *mark;         /* per-entry flag used while building the visible list */
    uint32_t flags;
    /* host swapping (Sec. 5): a host voxel store with one block per hash entry */
    int swap_enabled;
    int transfer_blocks;
    int16_t *host_sdf;
    uint8_t *host_w;
    uint8_t *host_has;     /* 1 if the host store holds data for the entry */
    int n_swapped_in, n_swapped_out;
} or_volume;

/* --------------------------------------------------------------------------
 * Hash function (Sec. 3.2): coordinates are sign-extended int16 -> int,
 * reinterpreted as uint32, multiplied modulo 2^32, xor-ed and masked.
 * -------------------------------------------------------------------------- */
uint32_t or_hash(int x, int y, int z, uint32_t mask)
{
    uint32_t hx = (uint32_t)x * 73856093u;
    uint32_t hy = (uint32_t)y * 19349669u;
    uint32_t hz = (uint32_t)z * 83492791u;
    return (hx ^ hy ^ hz) & mask;
}

static int floor_div8(int a)
{
    return (a >= 0) ? a / 8 : -((-a + 7) / 8);
}

/* ------------------------------------------------------------------------ */

or_volume *or_create(float voxel_size, float mu, int max_w, int n_buckets,
                     int n_excess, int n_blocks)
{
    or_volume *v = (or_volume *)calloc(1, sizeof(or_volume));
    int n_entries = n_buckets + n_excess;
    v->voxel_size = voxel_size;
    v->mu = mu;
    v->max_w = max_w;
    v->n_buckets = n_buckets;
    v->n_excess = n_excess;
    v->n_blocks = n_blocks;
    v->e = (or_entry *)malloc(sizeof(or_entry) * (size_t)n_entries);
    v->free_blocks = (int32_t *)malloc(sizeof(int32_t) * (size_t)n_blocks);
    v->free_excess = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_excess > 0 ? n_excess : 1));
    v->sdf = (int16_t *)malloc(sizeof(int16_t) * (size_t)n_blocks * OR_BLOCK_VOX);
    v->w = (uint8_t *)malloc((size_t)n_blocks * OR_BLOCK_VOX);
    v->visible = (int32_t *)malloc(sizeof(int32_t) * (size_t)n_entries);
    v->mark = (uint8_t *)calloc((size_t)n_entries, 1);
    for (int i = 0; i < n_entries; ++i) {
        v->e[i].x = v->e[i].y = v->e[i].z = 0;
        v->e[i].offset = 0;
        v->e[i].ptr = OR_PTR_EMPTY;
    }
    /* prepopulated allocation lists (Sec. 3.3): block i and excess slot i are free */
    for (int i = 0; i < n_blocks; ++i) v->free_blocks[i] = i;
    v->n_free_blocks = n_blocks;
    for (int i = 0; i < n_excess; ++i) v->free_excess[i] = i;
    v->n_free_excess = n_excess;
    v->n_visible = 0;
    v->flags = 0;
    return v;
}

void or_destroy(or_volume *v)
{
    if (!v) return;
    free(v->e); free(v->free_blocks); free(v->free_excess); free(v->sdf); free(v->w);
    free(v->visible); free(v->mark);
    free(v->host_sdf); free(v->host_w); free(v->host_has);
    free(v);
}

int or_n_entries(const or_volume *v) { return v->n_buckets + v->n_excess; }
void or_set_threads(int n) { omp_set_num_threads(n); }
int or_get_threads(void) { return omp_get_max_threads(); }
uint32_t or_flags(const or_volume *v) { return v->flags; }
int or_n_free_blocks(const or_volume *v) { return v->n_free_blocks; }
int or_n_free_excess(const or_volume *v) { return v->n_free_excess; }
int or_n_visible(const or_volume *v) { return v->n_visible; }

/* --------------------------------------------------------------------------
 * Retrieval of an entry (Sec. 3.3): start at the bucket, compare position,
 * follow `offset` (k >= 1 -> entry n_buckets + k - 1; < 1 ends the chain, as
 * in the retrieval listing).  `min_ptr` selects the notion of a match:
 * -1 ("present": allocated or swapped out, used by allocation) or 0 ("found":
 * data on the device, used by voxel reads).
 * -------------------------------------------------------------------------- */
static int find_entry(const or_volume *v, int bx, int by, int bz, int min_ptr)
{
    int i = (int)or_hash(bx, by, bz, (uint32_t)(v->n_buckets - 1));
    for (;;) {
        const or_entry *e = &v->e[i];
        if (e->x == bx && e->y == by && e->z == bz && e->ptr >= min_ptr) return i;
        if (e->offset < 1) return -1;
        i = v->n_buckets + e->offset - 1;
    }
}

int or_lookup(const or_volume *v, int bx, int by, int bz)
{
    return find_entry(v, bx, by, bz, OR_PTR_SWAPPED);
}

static void init_block(or_volume *v, int ptr)
{
    for (int l = 0; l < OR_BLOCK_VOX; ++l) {
        v->sdf[(size_t)ptr * OR_BLOCK_VOX + l] = OR_SDF_INIT;
        v->w[(size_t)ptr * OR_BLOCK_VOX + l] = 0;
    }
}

/* --------------------------------------------------------------------------
 * Insertion (Sec. 3.3 and Sec. 4.2): reserve a block from the free-block stack
 * (the previous head goes to the entry); store the entry in its bucket if the
 * bucket is unallocated, otherwise reserve a slot of the unordered excess list
 * and link it into the bucket's chain.  The new slot is linked at the head of
 * the chain (right after the bucket entry); retrieval and insertion treat the
 * chain as a set, so this equals linking at the tail.
 * Returns the entry index, or -1 if a free list is exhausted (flag set).
 * -------------------------------------------------------------------------- */
static int insert_entry(or_volume *v, int bx, int by, int bz)
{
    int h = (int)or_hash(bx, by, bz, (uint32_t)(v->n_buckets - 1));
    int idx;
    if (v->n_free_blocks == 0) {
        v->flags |= OR_FLAG_BLOCKS_EXHAUSTED;
        return -1;
    }
    if (v->e[h].ptr < OR_PTR_SWAPPED) {
        idx = h;
    } else {
        if (v->n_free_excess == 0) {
            v->flags |= OR_FLAG_EXCESS_EXHAUSTED;
            return -1;
        }
        int slot = v->free_excess[--v->n_free_excess];
        idx = v->n_buckets + slot;
        v->e[idx].offset = v->e[h].offset;
        v->e[h].offset = slot + 1;
    }
    int ptr = v->free_blocks[--v->n_free_blocks];
    v->e[idx].x = (int16_t)bx;
    v->e[idx].y = (int16_t)by;
    v->e[idx].z = (int16_t)bz;
    v->e[idx].ptr = ptr;
    init_block(v, ptr);
    return idx;
}

int or_insert(or_volume *v, int bx, int by, int bz)
{
    int i = or_lookup(v, bx, by, bz);
    if (i >= 0) return i;
    return insert_entry(v, bx, by, bz);
}

/* --------------------------------------------------------------------------
 * Pose helpers.  M is the paper's M_d (world -> camera), 16 floats row-major
 * with rows 0..2 = [R | t].  Its inverse is [R^T | -R^T t]; each component of
 * -R^T t is evaluated in double as -((r0i t0 + r1i t1) + r2i t2) and rounded
 * once to float.
 * -------------------------------------------------------------------------- */
static void invert_pose(const float *M, float *Ri, float *ti)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Ri[3 * i + j] = M[4 * j + i];
    for (int i = 0; i < 3; ++i) {
        double s = ((double)M[i] * (double)M[3] + (double)M[4 + i] * (double)M[7]) +
                   (double)M[8 + i] * (double)M[11];
        ti[i] = (float)(-s);
    }
}

/* pt_camera = M_d * pt_model (Sec. 4.3); each row ((m0 X + m1 Y) + m2 Z) + m3 */
static void transform(const float *M, float X, float Y, float Z, float *c)
{
    for (int r = 0; r < 3; ++r)
        c[r] = ((M[4 * r] * X + M[4 * r + 1] * Y) + M[4 * r + 2] * Z) + M[4 * r + 3];
}

/* --------------------------------------------------------------------------
 * Depth ingest (Sec. 4: the view builder converts unsigned short depth to
 * float): metres = (float)mm / 1000, correctly rounded; 0 stays invalid.
 * -------------------------------------------------------------------------- */
void or_depth_from_mm(const uint16_t *mm, float *out, int n)
{
    for (int i = 0; i < n; ++i) out[i] = (float)mm[i] / 1000.0f;
}

/* --------------------------------------------------------------------------
 * The blocks a pixel's segment touches (Sec. 4.2, first part).  The segment
 * joins the back-projections of camera depths d - mu and d + mu along the
 * ray through pixel (x, y).  It is sampled at n + 1 evenly spaced points in
 * block units, n = max(1, ceil(2 L)) for segment length L (so consecutive
 * samples are at most half a block apart); the block of a sample is its
 * floor.  Writes up to `cap` block keys (consecutive duplicates kept) and
 * returns how many samples were produced.
 * -------------------------------------------------------------------------- */
typedef struct { float fx, fy, cx, cy; int W, H; } or_intr;

static int segment_blocks(float d, int x, int y, const or_intr *K, const float *Ri,
                          const float *ti, float mu, float inv_block, int *keys, int cap)
{
    float a = ((float)x - K->cx) / K->fx;
    float b = ((float)y - K->cy) / K->fy;
    float z0 = d - mu, z1 = d + mu;
    float c0[3] = {z0 * a, z0 * b, z0};
    float c1[3] = {z1 * a, z1 * b, z1};
    float q0[3], q1[3], dq[3], st[3];
    for (int r = 0; r < 3; ++r) {
        float w0 = ((Ri[3 * r] * c0[0] + Ri[3 * r + 1] * c0[1]) + Ri[3 * r + 2] * c0[2]) + ti[r];
        float w1 = ((Ri[3 * r] * c1[0] + Ri[3 * r + 1] * c1[1]) + Ri[3 * r + 2] * c1[2]) + ti[r];
        q0[r] = w0 * inv_block;
        q1[r] = w1 * inv_block;
        dq[r] = q1[r] - q0[r];
    }
    float L = sqrtf((dq[0] * dq[0] + dq[1] * dq[1]) + dq[2] * dq[2]);
    int n = (int)ceilf(2.0f * L);
    if (n < 1) n = 1;
    for (int r = 0; r < 3; ++r) st[r] = dq[r] / (float)n;
    int m = 0;
    for (int k = 0; k <= n && m < cap; ++k) {
        float qx = q0[0] + (float)k * st[0];
        float qy = q0[1] + (float)k * st[1];
        float qz = q0[2] + (float)k * st[2];
        float fx = floorf(qx), fy = floorf(qy), fz = floorf(qz);
        /* keys outside the int16 block range cannot be stored (Sec. 3.2 pos is Vector3s) */
        if (!(fx >= -32768.0f && fx <= 32767.0f && fy >= -32768.0f && fy <= 32767.0f &&
              fz >= -32768.0f && fz <= 32767.0f))
            continue;
        keys[3 * m] = (int)fx;
        keys[3 * m + 1] = (int)fy;
        keys[3 * m + 2] = (int)fz;
        ++m;
    }
    return m;
}

/* exported for the geometry pins: the block keys of one pixel */
int or_segment_blocks(float d, int x, int y, const float *intr, int W, int H,
                      const float *M, float voxel_size, float mu, int *keys, int cap)
{
    or_intr K = {intr[0], intr[1], intr[2], intr[3], W, H};
    float Ri[9], ti[3];
    invert_pose(M, Ri, ti);
    float inv_block = 1.0f / (8.0f * voxel_size);
    return segment_blocks(d, x, y, &K, Ri, ti, mu, inv_block, keys, cap);
}

/* --------------------------------------------------------------------------
 * Frustum test for carrying a block over to the next visible list (Sec. 4.2,
 * third part: live entries project inside the visible frustum): at least one
 * of its 8 corners, world (8 (b + delta)) * voxel_size, has camera z > 0 and
 * projects to 0 <= u <= W-1, 0 <= v <= H-1.
 * -------------------------------------------------------------------------- */
static int block_in_frustum(const or_volume *v, const or_entry *e, const float *M, const or_intr *K)
{
    for (int c = 0; c < 8; ++c) {
        int px = 8 * (e->x + (c & 1)), py = 8 * (e->y + ((c >> 1) & 1)), pz = 8 * (e->z + (c >> 2));
        float X = (float)px * v->voxel_size, Y = (float)py * v->voxel_size, Z = (float)pz * v->voxel_size;
        float cc[3];
        transform(M, X, Y, Z, cc);
        if (cc[2] <= 0.0f) continue;
        float rz = 1.0f / cc[2];
        float u = (K->fx * cc[0]) * rz + K->cx;
        float vv = (K->fy * cc[1]) * rz + K->cy;
        if (u >= 0.0f && u <= (float)(K->W - 1) && vv >= 0.0f && vv <= (float)(K->H - 1)) return 1;
    }
    return 0;
}

/* --------------------------------------------------------------------------
 * Host swapping helpers (Sec. 5).  The host store has one block per hash
 * entry, so only the entry index crosses the boundary.
 * -------------------------------------------------------------------------- */
int or_enable_swap(or_volume *v, int transfer_blocks)
{
    size_t n_entries = (size_t)(v->n_buckets + v->n_excess);
    v->swap_enabled = 1;
    v->transfer_blocks = transfer_blocks;
    v->host_sdf = (int16_t *)malloc(sizeof(int16_t) * n_entries * OR_BLOCK_VOX);
    v->host_w = (uint8_t *)malloc(n_entries * OR_BLOCK_VOX);
    v->host_has = (uint8_t *)calloc(n_entries, 1);
    return (v->host_sdf && v->host_w && v->host_has) ? 0 : -1;
}

/* mark bits while a frame is being allocated */
#define MK_VISIBLE 1u

static int pop_block(or_volume *v)
{
    if (v->n_free_blocks == 0) {
        v->flags |= OR_FLAG_BLOCKS_EXHAUSTED;
        return -1;
    }
    int p = v->free_blocks[--v->n_free_blocks];
    init_block(v, p);
    return p;
}

/* --------------------------------------------------------------------------
 * Secondary integration of two copies of one block (Sec. 5, O3): per voxel a
 * weighted average of the two SDF values,
 *     F = (w_a F_a + w_b F_b) / (w_a + w_b),  w = min(w_a + w_b, maxW),
 * where a copy with weight 0 carries no observation (the other copy is kept
 * unchanged).  The result goes to copy a.  The sum is commutative, so the
 * result does not depend on which copy is a.
 * -------------------------------------------------------------------------- */
static void merge_block(int16_t *sa, uint8_t *wa, const int16_t *sb, const uint8_t *wb, int max_w)
{
    for (int l = 0; l < OR_BLOCK_VOX; ++l) {
        int w_a = wa[l], w_b = wb[l];
        if (w_b == 0) continue;
        if (w_a == 0) {
            sa[l] = sb[l];
            wa[l] = wb[l];
            continue;
        }
        float fa = (float)sa[l] * (1.0f / 32767.0f);
        float fb = (float)sb[l] * (1.0f / 32767.0f);
        float avg = ((float)w_a * fa + (float)w_b * fb) / (float)(w_a + w_b);
        int w = w_a + w_b;
        if (w > max_w) w = max_w;
        sa[l] = (int16_t)(avg * 32767.0f);
        wa[l] = (uint8_t)w;
    }
}

/* --------------------------------------------------------------------------
 * Allocation and visible list for one frame (Sec. 4.2).
 *   1. every pixel with d > 0 (row-major order): the blocks its segment
 *      touches are looked up; absent ones are inserted, present ones marked;
 *      a touched entry whose block was swapped out (ptr == -1) gets a fresh
 *      device block and is queued for swap-in (Sec. 5);
 *   2. the previous visible list is re-tested: entries with a device block
 *      that still pass the frustum test stay visible;
 *   3. the visible list is every marked entry, in ascending entry order.
 * Intra-frame collisions: every distinct touched block is inserted this frame.
 * -------------------------------------------------------------------------- */
void or_alloc_and_visible(or_volume *v, const float *depth, int W, int H, const float *intr,
                          const float *M)
{
    or_intr K = {intr[0], intr[1], intr[2], intr[3], W, H};
    float Ri[9], ti[3];
    invert_pose(M, Ri, ti);
    float inv_block = 1.0f / (8.0f * v->voxel_size);
    int keys[3 * OR_MAX_SEGMENT_SAMPLES];
    v->n_swapped_in = 0;

    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            float d = depth[(size_t)y * W + x];
            if (!(d > 0.0f)) continue;
            int m = segment_blocks(d, x, y, &K, Ri, ti, v->mu, inv_block, keys, OR_MAX_SEGMENT_SAMPLES);
            for (int s = 0; s < m; ++s) {
                int bx = keys[3 * s], by = keys[3 * s + 1], bz = keys[3 * s + 2];
                int i = or_lookup(v, bx, by, bz);
                if (i < 0) {
                    i = insert_entry(v, bx, by, bz);
                    if (i < 0) continue;
                } else if (v->e[i].ptr == OR_PTR_SWAPPED) {
                    if (!v->swap_enabled) continue;   /* cannot happen without swapping */
                    int p = pop_block(v);
                    if (p < 0) continue;
                    v->e[i].ptr = p;
                }
                v->mark[i] |= MK_VISIBLE;
            }
        }
    }
    for (int k = 0; k < v->n_visible; ++k) {
        int i = v->visible[k];
        if (v->e[i].ptr >= 0 && !(v->mark[i] & MK_VISIBLE) && block_in_frustum(v, &v->e[i], M, &K))
            v->mark[i] |= MK_VISIBLE;
    }
    int n = 0, n_entries = v->n_buckets + v->n_excess;
    for (int i = 0; i < n_entries; ++i) {
        if (v->mark[i] & MK_VISIBLE) v->visible[n++] = i;
    }
    v->n_visible = n;
    /* swap-in (Sec. 5): visible entries whose host store holds data, in
     * ascending entry order and up to the transfer capacity, fuse that data
     * into their device block (the secondary integration of Sec. 5). */
    if (v->swap_enabled) {
        for (int k = 0; k < v->n_visible; ++k) {
            int i = v->visible[k];
            if (!v->host_has[i]) continue;
            if (v->n_swapped_in >= v->transfer_blocks) {
                v->flags |= OR_FLAG_TRANSFER_OVERFLOW;
                break;
            }
            merge_block(&v->sdf[(size_t)v->e[i].ptr * OR_BLOCK_VOX], &v->w[(size_t)v->e[i].ptr * OR_BLOCK_VOX],
                        &v->host_sdf[(size_t)i * OR_BLOCK_VOX], &v->host_w[(size_t)i * OR_BLOCK_VOX], v->max_w);
            v->host_has[i] = 0;
            v->n_swapped_in++;
        }
    }
    for (int i = 0; i < n_entries; ++i) v->mark[i] = 0;
}

/* --------------------------------------------------------------------------
 * Integration (Sec. 4.3): the running-average update of every voxel of every
 * visible block.  Voxel p = 8 b + (lx, ly, lz) sits at world X = p *
 * voxel_size; it is projected with the camera matrix and the pinhole model,
 * read at the nearest pixel, and its SDF becomes the weight-averaged
 * truncated distance.  Three quotients appear: the perspective division by
 * z_c, eta / mu and the new average over w + 1 observations.  The pipeline
 * evaluates them as products with reciprocals,
 *     rz  = 1 / z_c                 (one correctly rounded reciprocal)
 *     u   = (fx * x_c) * rz + cx,   v = (fy * y_c) * rz + cy
 *     f   = min(1, eta * (1/mu))
 *     avg = (w * F_old + f) * (1/(w+1))   with 1/(w+1) correctly rounded
 * and F_old = s * (1/32767).  With `divide` set, the same update takes each
 * quotient as one correctly rounded division instead (x / n for x * (1/n));
 * the two agree in real arithmetic and the tests measure how often their
 * float results differ.  The short SDF is F * 32767 truncated toward zero.
 * -------------------------------------------------------------------------- */
static void integrate_impl(or_volume *v, const float *depth, int W, int H, const float *intr, const float *M,
                           int divide)
{
    const float fx = intr[0], fy = intr[1], cx = intr[2], cy = intr[3];
    const float vs = v->voxel_size, mu = v->mu;
    const float inv_mu = 1.0f / mu;
    const float neg_mu = -mu;
    const float k_sdf = 1.0f / 32767.0f;
    const int max_w = v->max_w;
    float rcp_w[257];
    for (int k = 1; k <= 256; ++k) rcp_w[k] = 1.0f / (float)k;
    const float umax = (float)(W - 2), vmax = (float)(H - 2);

#pragma omp parallel for schedule(static)
    for (int k = 0; k < v->n_visible; ++k) {
        const or_entry *e = &v->e[v->visible[k]];
        if (e->ptr < 0) continue;
        int16_t *S = &v->sdf[(size_t)e->ptr * OR_BLOCK_VOX];
        uint8_t *Wt = &v->w[(size_t)e->ptr * OR_BLOCK_VOX];
        for (int l = 0; l < OR_BLOCK_VOX; ++l) {
            int px = 8 * e->x + (l & 7), py = 8 * e->y + ((l >> 3) & 7), pz = 8 * e->z + (l >> 6);
            float X = (float)px * vs, Y = (float)py * vs, Z = (float)pz * vs;
            float c[3];
            transform(M, X, Y, Z, c);
            if (c[2] <= 0.0f) continue;
            float u, vv;
            if (divide) {
                u = (fx * c[0]) / c[2] + cx;
                vv = (fy * c[1]) / c[2] + cy;
            } else {
                float rz = 1.0f / c[2];
                u = (fx * c[0]) * rz + cx;
                vv = (fy * c[1]) * rz + cy;
            }
            if (u < 1.0f || u > umax || vv < 1.0f || vv > vmax) continue;
            int ix = (int)(u + 0.5f), iy = (int)(vv + 0.5f);
            float d = depth[ix + iy * W];
            if (d <= 0.0f) continue;
            float eta = d - c[2];
            if (eta < neg_mu) continue;
            float f_new = divide ? eta / mu : eta * inv_mu;
            if (f_new > 1.0f) f_new = 1.0f;
            int w_old = Wt[l];
            float f_old = divide ? (float)S[l] / 32767.0f : (float)S[l] * k_sdf;
            float sum = (float)w_old * f_old + f_new;
            float avg = divide ? sum / (float)(w_old + 1) : sum * rcp_w[w_old + 1];
            int w_new = w_old + 1;
            if (w_new > max_w) w_new = max_w;
            S[l] = (int16_t)(avg * 32767.0f);
            Wt[l] = (uint8_t)w_new;
        }
    }
}

void or_integrate(or_volume *v, const float *depth, int W, int H, const float *intr, const float *M)
{
    integrate_impl(v, depth, W, H, intr, M, 0);
}

/* the same update with every quotient as a division (the statistic that
 * compares the two evaluation orders; not used by the pipeline) */
void or_integrate_divide(or_volume *v, const float *depth, int W, int H, const float *intr, const float *M)
{
    integrate_impl(v, depth, W, H, intr, M, 1);
}

/* --------------------------------------------------------------------------
 * Search range (Sec. 4.4): forward-project each block, take the 2-D bounding
 * box of its 8 projected corners (floor of the minimum, ceil of the maximum,
 * clipped to the image) and fill it with the min/max camera z of the corners.
 * A block reaching closer than the near plane is clipped there: its box is
 * that of its corners beyond the plane and of the points where its edges
 * cross the plane, and its z range starts at the plane; a block entirely
 * closer than the plane is skipped.  `blocks` lists
 * entry indices; n < 0 means "every entry with a device block".
 * Uncovered pixels keep zmin = +inf, zmax = -inf (no search interval).
 * -------------------------------------------------------------------------- */
void or_range(const or_volume *v, const int32_t *blocks, int n, int W, int H, const float *intr,
              const float *M, float *zmin, float *zmax)
{
    const float fx = intr[0], fy = intr[1], cx = intr[2], cy = intr[3];
    for (int p = 0; p < W * H; ++p) {
        zmin[p] = INFINITY;
        zmax[p] = -INFINITY;
    }
    int total = n < 0 ? v->n_buckets + v->n_excess : n;
    for (int k = 0; k < total; ++k) {
        int i = n < 0 ? k : blocks[k];
        const or_entry *e = &v->e[i];
        if (e->ptr < 0) continue;
        float zlo = INFINITY, zhi = -INFINITY;
        float cs[8][3];
        for (int c = 0; c < 8; ++c) {
            int px = 8 * (e->x + (c & 1)), py = 8 * (e->y + ((c >> 1) & 1)), pz = 8 * (e->z + (c >> 2));
            transform(M, (float)px * v->voxel_size, (float)py * v->voxel_size, (float)pz * v->voxel_size, cs[c]);
            if (cs[c][2] < zlo) zlo = cs[c][2];
            if (cs[c][2] > zhi) zhi = cs[c][2];
        }
        if (zhi < OR_Z_NEAR) continue;
        /* the part of the block in front of the near plane: its corners there
         * and the points where its edges cross the plane; the pixel box of
         * their projections */
        float umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
        for (int c = 0; c < 8; ++c) {
            if (cs[c][2] < OR_Z_NEAR) continue;
            float rz = 1.0f / cs[c][2];
            float u = (fx * cs[c][0]) * rz + cx;
            float vv = (fy * cs[c][1]) * rz + cy;
            if (u < umin) umin = u;
            if (u > umax) umax = u;
            if (vv < vmin) vmin = vv;
            if (vv > vmax) vmax = vv;
        }
        if (zlo < OR_Z_NEAR) {
            const float rzn = 1.0f / OR_Z_NEAR;
            for (int a = 0; a < 8; ++a)
                for (int bit = 1; bit < 8; bit <<= 1) {
                    if (a & bit) continue;
                    const int b = a | bit;   /* the edge from corner a to corner b */
                    if ((cs[a][2] < OR_Z_NEAR) == (cs[b][2] < OR_Z_NEAR)) continue;
                    float t = (OR_Z_NEAR - cs[a][2]) / (cs[b][2] - cs[a][2]);
                    float xe = cs[a][0] + t * (cs[b][0] - cs[a][0]);
                    float ye = cs[a][1] + t * (cs[b][1] - cs[a][1]);
                    float u = (fx * xe) * rzn + cx;
                    float vv = (fy * ye) * rzn + cy;
                    if (u < umin) umin = u;
                    if (u > umax) umax = u;
                    if (vv < vmin) vmin = vv;
                    if (vv > vmax) vmax = vv;
                }
            zlo = OR_Z_NEAR;
        }
        float fx0 = floorf(umin), fx1 = ceilf(umax), fy0 = floorf(vmin), fy1 = ceilf(vmax);
        if (fx0 < 0.0f) fx0 = 0.0f;
        if (fy0 < 0.0f) fy0 = 0.0f;
        if (fx1 > (float)(W - 1)) fx1 = (float)(W - 1);
        if (fy1 > (float)(H - 1)) fy1 = (float)(H - 1);
        if (fx0 > fx1 || fy0 > fy1) continue;
        int x0 = (int)fx0, x1 = (int)fx1, y0 = (int)fy0, y1 = (int)fy1;
        for (int yy = y0; yy <= y1; ++yy)
            for (int xx = x0; xx <= x1; ++xx) {
                int p = yy * W + xx;
                if (zlo < zmin[p]) zmin[p] = zlo;
                if (zhi > zmax[p]) zmax[p] = zhi;
            }
    }
}

/* --------------------------------------------------------------------------
 * Voxel reads for the raycast (Sec. 3.3 retrieval): the voxel at integer
 * voxel coordinates (x, y, z); an absent block reads as the default voxel
 * (F = 1, weight 0).
 * -------------------------------------------------------------------------- */
static float read_F(const or_volume *v, int x, int y, int z)
{
    int bx = floor_div8(x), by = floor_div8(y), bz = floor_div8(z);
    int i = find_entry(v, bx, by, bz, 0);
    if (i < 0) return 1.0f;
    int l = (x - 8 * bx) + 8 * (y - 8 * by) + 64 * (z - 8 * bz);
    return (float)v->sdf[(size_t)v->e[i].ptr * OR_BLOCK_VOX + l] * (1.0f / 32767.0f);
}

static int allocated_at(const or_volume *v, float X, float Y, float Z)
{
    int x = (int)floorf(X), y = (int)floorf(Y), z = (int)floorf(Z);
    return find_entry(v, floor_div8(x), floor_div8(y), floor_div8(z), 0) >= 0;
}

/* trilinear interpolation of F at voxel-unit position P: lerp a + (b - a) t
 * along x, then y, then z */
float or_trilinear(const or_volume *v, float X, float Y, float Z)
{
    float bx = floorf(X), by = floorf(Y), bz = floorf(Z);
    float tx = X - bx, ty = Y - by, tz = Z - bz;
    int ix = (int)bx, iy = (int)by, iz = (int)bz;
    float f000 = read_F(v, ix, iy, iz), f100 = read_F(v, ix + 1, iy, iz);
    float f010 = read_F(v, ix, iy + 1, iz), f110 = read_F(v, ix + 1, iy + 1, iz);
    float f001 = read_F(v, ix, iy, iz + 1), f101 = read_F(v, ix + 1, iy, iz + 1);
    float f011 = read_F(v, ix, iy + 1, iz + 1), f111 = read_F(v, ix + 1, iy + 1, iz + 1);
    float c00 = f000 + (f100 - f000) * tx;
    float c10 = f010 + (f110 - f010) * tx;
    float c01 = f001 + (f101 - f001) * tx;
    float c11 = f011 + (f111 - f011) * tx;
    float c0 = c00 + (c10 - c00) * ty;
    float c1 = c01 + (c11 - c01) * ty;
    return c0 + (c1 - c0) * tz;
}

enum { SEARCH_BLOCK_COARSE, SEARCH_BLOCK_FINE, SEARCH_SURFACE, BEHIND_SURFACE, WRONG_SIDE };

/* --------------------------------------------------------------------------
 * Raycast (Sec. 4.4).  Ray through pixel (x, y): r = ((x-cx)/fx, (y-cy)/fy,
 * 1), |r| correctly rounded, unit direction dir = R^T (r / |r|); origin o =
 * t_inv / voxel_size; position P(t) = o + t dir in voxel units.  Search
 * interval t in [zmin |r| / vs, zmax |r| / vs] from the range image.
 * State machine (step sizes in voxels, mu_v = mu / vs):
 *   COARSE      unallocated: t += 8 (one block); allocated: t -= 8, -> FINE
 *   FINE        unallocated: t += mu_v; allocated: read F,
 *               F < 0 -> WRONG_SIDE, else -> SURFACE (no step)
 *   SURFACE     unallocated: -> FINE, t += mu_v; allocated: read F,
 *               F < 0 -> BEHIND (hit), else t += max(F mu_v, 1)
 *   WRONG_SIDE  unallocated: -> FINE, t += mu_v; allocated: read F,
 *               F >= 0 -> SURFACE, else t += max(-F mu_v, 1)
 * "allocated" = the block of floor(P) has a device block.  On a hit two
 * refinement steps t += F(P(t)) mu_v follow (the first reuses the F that
 * ended the march); the point is P(t) * vs in world metres.  The normal is
 * the normalised central difference of F at P +- 1 voxel along each axis.
 * Outputs are float4: (x, y, z, 1) / (nx, ny, nz, 1), zeros on a miss (or for
 * a normal whose gradient vanishes).
 * -------------------------------------------------------------------------- */
void or_raycast(const or_volume *v, int W, int H, const float *intr, const float *M,
                const float *zmin, const float *zmax, float *points, float *normals)
{
    const float fx = intr[0], fy = intr[1], cx = intr[2], cy = intr[3];
    float Ri[9], ti[3];
    invert_pose(M, Ri, ti);
    const float vs = v->voxel_size;
    const float inv_vs = 1.0f / vs;
    const float mu_v = v->mu * inv_vs;
    const float o[3] = {ti[0] * inv_vs, ti[1] * inv_vs, ti[2] * inv_vs};

#pragma omp parallel for schedule(dynamic, 64)
    for (int p = 0; p < W * H; ++p) {
        int x = p % W, y = p / W;
        float *pt = &points[4 * (size_t)p];
        float *nm = &normals[4 * (size_t)p];
        pt[0] = pt[1] = pt[2] = pt[3] = 0.0f;
        nm[0] = nm[1] = nm[2] = nm[3] = 0.0f;
        if (!(zmin[p] <= zmax[p])) continue;
        float a = ((float)x - cx) / fx;
        float b = ((float)y - cy) / fy;
        float nr = sqrtf((a * a + b * b) + 1.0f);
        float rc[3] = {a / nr, b / nr, 1.0f / nr};
        float dir[3];
        for (int r = 0; r < 3; ++r)
            dir[r] = (Ri[3 * r] * rc[0] + Ri[3 * r + 1] * rc[1]) + Ri[3 * r + 2] * rc[2];
        float t = (zmin[p] * nr) * inv_vs;
        float t_end = (zmax[p] * nr) * inv_vs;
        int state = SEARCH_BLOCK_COARSE;
        float F = 1.0f;
        float P[3];
        int steps = 0;
        while (t < t_end && steps < OR_MAX_RAY_STEPS) {
            ++steps;
            P[0] = o[0] + t * dir[0];
            P[1] = o[1] + t * dir[1];
            P[2] = o[2] + t * dir[2];
            int alloc = allocated_at(v, P[0], P[1], P[2]);
            if (state == SEARCH_BLOCK_COARSE) {
                if (!alloc) {
                    t += 8.0f;
                } else {
                    t -= 8.0f;
                    state = SEARCH_BLOCK_FINE;
                }
            } else if (!alloc) {
                state = SEARCH_BLOCK_FINE;
                t += mu_v;
            } else {
                F = or_trilinear(v, P[0], P[1], P[2]);
                if (state == SEARCH_BLOCK_FINE) {
                    state = (F < 0.0f) ? WRONG_SIDE : SEARCH_SURFACE;
                } else if (state == SEARCH_SURFACE) {
                    if (F < 0.0f) {
                        state = BEHIND_SURFACE;
                        break;
                    }
                    float s = F * mu_v;
                    t += (s > 1.0f) ? s : 1.0f;
                } else { /* WRONG_SIDE */
                    if (F >= 0.0f) {
                        state = SEARCH_SURFACE;
                    } else {
                        float s = -F * mu_v;
                        t += (s > 1.0f) ? s : 1.0f;
                    }
                }
            }
        }
        if (state != BEHIND_SURFACE) continue;
        t += F * mu_v;
        P[0] = o[0] + t * dir[0];
        P[1] = o[1] + t * dir[1];
        P[2] = o[2] + t * dir[2];
        F = or_trilinear(v, P[0], P[1], P[2]);
        t += F * mu_v;
        P[0] = o[0] + t * dir[0];
        P[1] = o[1] + t * dir[1];
        P[2] = o[2] + t * dir[2];
        pt[0] = P[0] * vs;
        pt[1] = P[1] * vs;
        pt[2] = P[2] * vs;
        pt[3] = 1.0f;
        float gx = (or_trilinear(v, P[0] + 1.0f, P[1], P[2]) - or_trilinear(v, P[0] - 1.0f, P[1], P[2])) * 0.5f;
        float gy = (or_trilinear(v, P[0], P[1] + 1.0f, P[2]) - or_trilinear(v, P[0], P[1] - 1.0f, P[2])) * 0.5f;
        float gz = (or_trilinear(v, P[0], P[1], P[2] + 1.0f) - or_trilinear(v, P[0], P[1], P[2] - 1.0f)) * 0.5f;
        float gn = sqrtf((gx * gx + gy * gy) + gz * gz);
        if (gn > 0.0f) {
            nm[0] = gx / gn;
            nm[1] = gy / gn;
            nm[2] = gz / gn;
            nm[3] = 1.0f;
        }
    }
}

/* --------------------------------------------------------------------------
 * Swap-out (Sec. 5): entries with a device block that are not in the current
 * visible list move to the host store, lowest entry index first, up to the
 * transfer capacity; their device block returns to the free stack and the
 * entry is marked ptr = -1.
 * -------------------------------------------------------------------------- */
int or_swap_out(or_volume *v)
{
    int n_entries = v->n_buckets + v->n_excess;
    for (int k = 0; k < v->n_visible; ++k) v->mark[v->visible[k]] = 1;
    int moved = 0;
    for (int i = 0; i < n_entries && moved < v->transfer_blocks; ++i) {
        or_entry *e = &v->e[i];
        if (e->ptr < 0 || v->mark[i]) continue;
        int16_t *hs = &v->host_sdf[(size_t)i * OR_BLOCK_VOX];
        uint8_t *hw = &v->host_w[(size_t)i * OR_BLOCK_VOX];
        const int16_t *ds = &v->sdf[(size_t)e->ptr * OR_BLOCK_VOX];
        const uint8_t *dw = &v->w[(size_t)e->ptr * OR_BLOCK_VOX];
        if (v->host_has[i]) {
            /* host data that never made it back in is fused, not overwritten */
            merge_block(hs, hw, ds, dw, v->max_w);
        } else {
            memcpy(hs, ds, sizeof(int16_t) * OR_BLOCK_VOX);
            memcpy(hw, dw, OR_BLOCK_VOX);
        }
        v->host_has[i] = 1;
        v->free_blocks[v->n_free_blocks++] = e->ptr;
        e->ptr = OR_PTR_SWAPPED;
        ++moved;
    }
    for (int k = 0; k < v->n_visible; ++k) v->mark[v->visible[k]] = 0;
    v->n_swapped_out = moved;
    return moved;
}

int or_n_swapped_in(const or_volume *v) { return v->n_swapped_in; }

/* --------------------------------------------------------------------------
 * Exports for the tests
 * -------------------------------------------------------------------------- */
void or_get_entries(const or_volume *v, int16_t *pos, int32_t *offset, int32_t *ptr)
{
    int n = v->n_buckets + v->n_excess;
    for (int i = 0; i < n; ++i) {
        pos[3 * i] = v->e[i].x;
        pos[3 * i + 1] = v->e[i].y;
        pos[3 * i + 2] = v->e[i].z;
        offset[i] = v->e[i].offset;
        ptr[i] = v->e[i].ptr;
    }
}

int or_get_visible(const or_volume *v, int32_t *out)
{
    memcpy(out, v->visible, sizeof(int32_t) * (size_t)v->n_visible);
    return v->n_visible;
}

/* voxels of the given entries (each must have a device block), in the
 * in-block order l = lx + 8 ly + 64 lz */
void or_get_block_voxels(const or_volume *v, const int32_t *entries, int n, int16_t *sdf, uint8_t *w)
{
    for (int k = 0; k < n; ++k) {
        int p = v->e[entries[k]].ptr;
        memcpy(&sdf[(size_t)k * OR_BLOCK_VOX], &v->sdf[(size_t)p * OR_BLOCK_VOX], sizeof(int16_t) * OR_BLOCK_VOX);
        memcpy(&w[(size_t)k * OR_BLOCK_VOX], &v->w[(size_t)p * OR_BLOCK_VOX], OR_BLOCK_VOX);
    }
}

/* overwrite the voxels of one entry's device block (tests that assemble a
 * volume block by block); 0 if the entry has no device block */
int or_set_block_voxels(or_volume *v, int entry, const int16_t *sdf, const uint8_t *w)
{
    int p = v->e[entry].ptr;
    if (p < 0) return 0;
    memcpy(&v->sdf[(size_t)p * OR_BLOCK_VOX], sdf, sizeof(int16_t) * OR_BLOCK_VOX);
    memcpy(&v->w[(size_t)p * OR_BLOCK_VOX], w, OR_BLOCK_VOX);
    return 1;
}

/* host store contents of one entry (swap tests) */
int or_get_host_block(const or_volume *v, int entry, int16_t *sdf, uint8_t *w)
{
    if (!v->swap_enabled || !v->host_has[entry]) return 0;
    memcpy(sdf, &v->host_sdf[(size_t)entry * OR_BLOCK_VOX], sizeof(int16_t) * OR_BLOCK_VOX);
    memcpy(w, &v->host_w[(size_t)entry * OR_BLOCK_VOX], OR_BLOCK_VOX);
    return 1;
}

/* ==========================================================================
 * Submaps (Sec. 7.2).  Submap i is an ordinary volume with its own voxel
 * grid; P_i is its pose, mapping world points into the submap frame.
 * ========================================================================== */

/* rigid inverse in double: [R^T | -R^T t] */
static void invert_pose_d(const float *P, double *Q)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Q[4 * i + j] = (double)P[4 * j + i];
    for (int i = 0; i < 3; ++i)
        Q[4 * i + 3] = -(((double)P[i] * (double)P[3] + (double)P[4 + i] * (double)P[7]) + (double)P[8 + i] * (double)P[11]);
    Q[12] = Q[13] = Q[14] = 0.0;
    Q[15] = 1.0;
}

/* A * inv(P) for rigid 4x4 transforms, in double, rounded once to float:
 * the camera matrix of a submap (world->camera composed with submap->world) */
void or_compose(const float *A, const float *P, float *out)
{
    double Q[16];
    invert_pose_d(P, Q);
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            double s = (((double)A[4 * r] * Q[c] + (double)A[4 * r + 1] * Q[4 + c]) + (double)A[4 * r + 2] * Q[8 + c]) +
                       (double)A[4 * r + 3] * Q[12 + c];
            out[4 * r + c] = (float)s;
        }
}

/* search range of a view over the blocks of every submap (each projected
 * with the composed matrix V * inv(P_i)); the reading of Sec. 4.4 applied to
 * all submaps: min/max camera z over the boxes covering the pixel */
void or_multi_range(or_volume **vols, const float *poses, int n, int W, int H, const float *intr, const float *V,
                    float *zmin, float *zmax)
{
    float *zlo = (float *)malloc(sizeof(float) * (size_t)W * H);
    float *zhi = (float *)malloc(sizeof(float) * (size_t)W * H);
    for (int p = 0; p < W * H; ++p) {
        zmin[p] = INFINITY;
        zmax[p] = -INFINITY;
    }
    for (int i = 0; i < n; ++i) {
        float C[16];
        or_compose(V, &poses[16 * i], C);
        or_range(vols[i], NULL, -1, W, H, intr, C, zlo, zhi);
        for (int p = 0; p < W * H; ++p) {
            if (zlo[p] < zmin[p]) zmin[p] = zlo[p];
            if (zhi[p] > zmax[p]) zmax[p] = zhi[p];
        }
    }
    free(zlo);
    free(zhi);
}

static float read_W(const or_volume *v, int x, int y, int z)
{
    int bx = floor_div8(x), by = floor_div8(y), bz = floor_div8(z);
    int i = find_entry(v, bx, by, bz, 0);
    if (i < 0) return 0.0f;
    int l = (x - 8 * bx) + 8 * (y - 8 * by) + 64 * (z - 8 * bz);
    return (float)v->w[(size_t)v->e[i].ptr * OR_BLOCK_VOX + l];
}

/* trilinear interpolation of the weight (absent voxels weigh 0), same
 * order of operations as or_trilinear */
static float trilinear_w(const or_volume *v, float X, float Y, float Z)
{
    float bx = floorf(X), by = floorf(Y), bz = floorf(Z);
    float tx = X - bx, ty = Y - by, tz = Z - bz;
    int ix = (int)bx, iy = (int)by, iz = (int)bz;
    float f000 = read_W(v, ix, iy, iz), f100 = read_W(v, ix + 1, iy, iz);
    float f010 = read_W(v, ix, iy + 1, iz), f110 = read_W(v, ix + 1, iy + 1, iz);
    float f001 = read_W(v, ix, iy, iz + 1), f101 = read_W(v, ix + 1, iy, iz + 1);
    float f011 = read_W(v, ix, iy + 1, iz + 1), f111 = read_W(v, ix + 1, iy + 1, iz + 1);
    float c00 = f000 + (f100 - f000) * tx;
    float c10 = f010 + (f110 - f010) * tx;
    float c01 = f001 + (f101 - f001) * tx;
    float c11 = f011 + (f111 - f011) * tx;
    float c0 = c00 + (c10 - c00) * ty;
    float c1 = c01 + (c11 - c01) * ty;
    return c0 + (c1 - c0) * tz;
}

typedef struct {
    or_volume **vols;
    int n;
    float R[64][9];   /* per submap: rotation of P_i */
    float s[64][3];   /* per submap: translation of P_i in voxel units */
} or_multi_view;

/* position of world voxel-unit point P in submap i's voxel units:
 * Q = R_i P + t_i / v, each row ((r0 P0 + r1 P1) + r2 P2) + s */
static void to_submap(const or_multi_view *m, int i, const float *P, float *Q)
{
    for (int r = 0; r < 3; ++r)
        Q[r] = ((m->R[i][3 * r] * P[0] + m->R[i][3 * r + 1] * P[1]) + m->R[i][3 * r + 2] * P[2]) + m->s[i][r];
}

static int multi_allocated(const or_multi_view *m, const float *P)
{
    for (int i = 0; i < m->n; ++i) {
        float Q[3];
        to_submap(m, i, P, Q);
        if (allocated_at(m->vols[i], Q[0], Q[1], Q[2])) return 1;
    }
    return 0;
}

/* combined field F^ at world voxel-unit P: the weighted average of the
 * submaps' trilinear F, weighted by their trilinear weight, over the submaps
 * with a non-zero weight there; a single contributor gives its F unchanged;
 * none gives 1 (every corner of every submap reads the default voxel then) */
static float multi_F(const or_multi_view *m, const float *P)
{
    int cnt = 0;
    float first = 1.0f, num = 0.0f, den = 0.0f;
    for (int i = 0; i < m->n; ++i) {
        float Q[3];
        to_submap(m, i, P, Q);
        float w = trilinear_w(m->vols[i], Q[0], Q[1], Q[2]);
        if (!(w > 0.0f)) continue;
        float F = or_trilinear(m->vols[i], Q[0], Q[1], Q[2]);
        if (cnt == 0) first = F;
        num = num + w * F;
        den = den + w;
        ++cnt;
    }
    if (cnt == 0) return 1.0f;
    if (cnt == 1) return first;
    return num / den;
}

/* raycast of the combined field (Sec. 7.2: rendering the submaps together
 * as a view), with the state machine, refinement and normals of or_raycast */
void or_multi_raycast(or_volume **vols, const float *poses, int n, int W, int H, const float *intr, const float *V,
                      const float *zmin, const float *zmax, float *points, float *normals)
{
    or_multi_view m;
    m.vols = vols;
    m.n = n > 64 ? 64 : n;
    const float vs = vols[0]->voxel_size;
    const float inv_vs = 1.0f / vs;
    const float mu_v = vols[0]->mu * inv_vs;
    for (int i = 0; i < m.n; ++i) {
        const float *P = &poses[16 * i];
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 3; ++c) m.R[i][3 * r + c] = P[4 * r + c];
            m.s[i][r] = P[4 * r + 3] * inv_vs;
        }
    }
    const float fx = intr[0], fy = intr[1], cx = intr[2], cy = intr[3];
    float Ri[9], ti[3];
    invert_pose(V, Ri, ti);
    const float o[3] = {ti[0] * inv_vs, ti[1] * inv_vs, ti[2] * inv_vs};

#pragma omp parallel for schedule(dynamic, 64)
    for (int p = 0; p < W * H; ++p) {
        int x = p % W, y = p / W;
        float *pt = &points[4 * (size_t)p];
        float *nm = &normals[4 * (size_t)p];
        pt[0] = pt[1] = pt[2] = pt[3] = 0.0f;
        nm[0] = nm[1] = nm[2] = nm[3] = 0.0f;
        if (!(zmin[p] <= zmax[p])) continue;
        float a = ((float)x - cx) / fx;
        float b = ((float)y - cy) / fy;
        float nr = sqrtf((a * a + b * b) + 1.0f);
        float rc[3] = {a / nr, b / nr, 1.0f / nr};
        float dir[3];
        for (int r = 0; r < 3; ++r)
            dir[r] = (Ri[3 * r] * rc[0] + Ri[3 * r + 1] * rc[1]) + Ri[3 * r + 2] * rc[2];
        float t = (zmin[p] * nr) * inv_vs;
        float t_end = (zmax[p] * nr) * inv_vs;
        int state = SEARCH_BLOCK_COARSE;
        float F = 1.0f;
        float P[3];
        int steps = 0;
        while (t < t_end && steps < OR_MAX_RAY_STEPS) {
            ++steps;
            P[0] = o[0] + t * dir[0];
            P[1] = o[1] + t * dir[1];
            P[2] = o[2] + t * dir[2];
            int alloc = multi_allocated(&m, P);
            if (state == SEARCH_BLOCK_COARSE) {
                if (!alloc) {
                    t += 8.0f;
                } else {
                    t -= 8.0f;
                    state = SEARCH_BLOCK_FINE;
                }
            } else if (!alloc) {
                state = SEARCH_BLOCK_FINE;
                t += mu_v;
            } else {
                F = multi_F(&m, P);
                if (state == SEARCH_BLOCK_FINE) {
                    state = (F < 0.0f) ? WRONG_SIDE : SEARCH_SURFACE;
                } else if (state == SEARCH_SURFACE) {
                    if (F < 0.0f) {
                        state = BEHIND_SURFACE;
                        break;
                    }
                    float s = F * mu_v;
                    t += (s > 1.0f) ? s : 1.0f;
                } else {
                    if (F >= 0.0f) {
                        state = SEARCH_SURFACE;
                    } else {
                        float s = -F * mu_v;
                        t += (s > 1.0f) ? s : 1.0f;
                    }
                }
            }
        }
        if (state != BEHIND_SURFACE) continue;
        t += F * mu_v;
        P[0] = o[0] + t * dir[0];
        P[1] = o[1] + t * dir[1];
        P[2] = o[2] + t * dir[2];
        F = multi_F(&m, P);
        t += F * mu_v;
        P[0] = o[0] + t * dir[0];
        P[1] = o[1] + t * dir[1];
        P[2] = o[2] + t * dir[2];
        pt[0] = P[0] * vs;
        pt[1] = P[1] * vs;
        pt[2] = P[2] * vs;
        pt[3] = 1.0f;
        float q[3];
        q[0] = P[0] + 1.0f; q[1] = P[1]; q[2] = P[2];
        float fxp = multi_F(&m, q);
        q[0] = P[0] - 1.0f;
        float fxm = multi_F(&m, q);
        q[0] = P[0]; q[1] = P[1] + 1.0f;
        float fyp = multi_F(&m, q);
        q[1] = P[1] - 1.0f;
        float fym = multi_F(&m, q);
        q[1] = P[1]; q[2] = P[2] + 1.0f;
        float fzp = multi_F(&m, q);
        q[2] = P[2] - 1.0f;
        float fzm = multi_F(&m, q);
        float gx = (fxp - fxm) * 0.5f, gy = (fyp - fym) * 0.5f, gz = (fzp - fzm) * 0.5f;
        float gn = sqrtf((gx * gx + gy * gy) + gz * gz);
        if (gn > 0.0f) {
            nm[0] = gx / gn;
            nm[1] = gy / gn;
            nm[2] = gz / gn;
            nm[3] = 1.0f;
        }
    }
}
