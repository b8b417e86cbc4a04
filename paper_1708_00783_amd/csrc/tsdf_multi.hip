// tsdf_multi.hip -- gfx950 kernels of the batched rigid submaps (Sec. 7.2).
//
//   k_m_alloc / k_m_insert / k_m_visible / k_m_integrate
//       one depth frame into the submaps selected for it, blockIdx.y = slot of
//       the selection; each runs the single-volume body on its submap with the
//       camera composed with that submap's pose
//   k_m_bin<false>, k_m_scan, k_m_bin<true>
//       every allocated block of every submap against every view: count the
//       (block, tile) pairs, exclusive offsets, then fill the tile bins.  A
//       block is binned by its cube grown by kExpand voxels, so that a tile's
//       bin holds every block any trilinear read of its rays can touch
//   k_m_raycast<TW, TH>
//       one workgroup per TWxTH tile of any view: the per-pixel search range,
//       the tile's submap set and an LDS block table from the bin, then the
//       ray state machine on the combined field
//
// The combined field at a world point (voxel units) is the weighted average of
// the submaps' trilinear SDF, each weighted by its trilinear weight, over the
// submaps whose weight there is positive; one contributor gives its value
// unchanged and none gives 1.  Submaps are summed in ascending index order.
#include "tsdf_device.h"

namespace tsdf {

// ============================================================================
// integration of one frame into the selected submaps
// ============================================================================
__global__ __launch_bounds__(256) void k_m_alloc(const Vol *vols, const MFrame *f)
{
    const int y = (int)blockIdx.y;
    if (y >= f->n_sel) return;
    const Vol v = vols[f->sel[y]];
    const Cam c = f->icam[y];
    // every submap reads the one shared depth map; slot 0 writes it
    if (f->fmt == TF_DEPTH_U16_MM)
        alloc_rays_body<TF_DEPTH_U16_MM>(v, c, f->depth, y == 0);
    else
        alloc_rays_body<TF_DEPTH_F32_M>(v, c, f->depth, y == 0);
}

__global__ __launch_bounds__(256) void k_m_insert(const Vol *vols, const MFrame *f)
{
    const int y = (int)blockIdx.y;
    if (y >= f->n_sel) return;
    const Vol v = vols[f->sel[y]];
    const Cam c = f->icam[y];
    insert_body(v, c);
}

__global__ __launch_bounds__(256) void k_m_visible(const Vol *vols, const MFrame *f)
{
    const int y = (int)blockIdx.y;
    if (y >= f->n_sel) return;
    const Vol v = vols[f->sel[y]];
    visible_body(v);
}

template <int NT>
__global__ __launch_bounds__(NT) void k_m_integrate(const Vol *vols, const MFrame *f, int dry)
{
    __shared__ float rcp_w[260];
    __shared__ uint32_t wg_cols;
    const int y = (int)blockIdx.y;
    if (y >= f->n_sel) return;
    const Vol v = vols[f->sel[y]];
    const Cam c = f->icam[y];
    integrate_body<NT>(v, c, rcp_w, &wg_cols, dry != 0);
}

// ============================================================================
// tile bins of every view
// ============================================================================
// LDS of a binning workgroup: the distinct tiles of one chunk of blocks
// (open addressing on the tile index) with their entry counts, then their
// reserved positions
constexpr int kBinSlots = 1024;
constexpr int kBinProbes = 32;        // probes before a tile takes the global path
constexpr int kBinDirect = 16;        // blocks over more tiles take the global path for all of them
constexpr uint32_t kNoTile = 0xffffffffu;
constexpr int kBinBig = 128;          // blocks over many tiles whose tiles the workgroup shares
struct MBinLds {
    uint32_t tile[kBinSlots];
    uint32_t cnt[kBinSlots];
    uint32_t pos[kBinSlots];
    uint32_t first[kMaxSubmaps + 1];   // flat index of each submap's first block
    float C[kMaxSubmaps][12];          // the view's camera composed with each submap pose
    Rec big_rec[kBinBig];              // fill pass: the record of each queued block
    int4 big_box[kBinBig];             // tx0, ty0, tiles per row, tiles
    uint32_t nbig;
    uint32_t pairs;                    // count pass: (block, view) pairs of the workgroup
};

// slot of tile g in the chunk table, inserting it when `insert`; -1 when
// the first kBinProbes slots of its probe sequence hold other tiles (or,
// without insert, do not hold g).  Slots are never emptied within a chunk,
// so a tile refused once is refused for the rest of the chunk.
__device__ __forceinline__ int bin_slot(MBinLds &B, uint32_t g, bool insert)
{
    uint32_t sl = (g * 0x9e3779b1u) >> 22;   // 10 bits
    for (int k = 0; k < kBinProbes; ++k) {
        const uint32_t cur = insert ? atomicCAS(&B.tile[sl], kNoTile, g) : B.tile[sl];
        if (cur == g || (insert && cur == kNoTile)) return (int)sl;
        if (cur == kNoTile) return -1;
        sl = (sl + 1u) & (uint32_t)(kBinSlots - 1);
    }
    return -1;
}

// Every allocated block of every submap against view blockIdx.y: its cube
// grown by kExpand voxels gives the tiles whose bins take its record.  Count
// pass (FILL false): entries per tile; fill pass: the records at the tile's
// offset.  The blocks of all submaps form one flat index range (submap by
// submap); a workgroup takes 256 consecutive blocks at a time and aggregates
// their (block, tile) entries per distinct tile in LDS, so a tile costs one
// global atomic per chunk instead of one per entry (an entry whose tile the
// chunk table refuses takes a global atomic of its own).  A block over more
// than kBinDirect tiles -- near the camera it can cover thousands -- is queued
// and its tiles are shared by the workgroup's threads, one global atomic
// each.  The order of records within a bin is not fixed.
template <bool FILL>
__global__ __launch_bounds__(256) void k_m_bin(const MSub *subs, const MFrame *f, MTiles t, float voxel)
{
    __shared__ MBinLds B;
    const int vi = (int)blockIdx.y;
    if (vi >= f->n_views) return;
    const Cam vc = f->view[vi].cam;
    const int ntx = f->view[vi].ntx, base = f->view[vi].tile_base;
    const int tw = f->tw, th = f->th;
    const int n_sub = f->n_sub;
    for (int k = threadIdx.x; k < kBinSlots; k += 256) {
        B.tile[k] = kNoTile;
        B.cnt[k] = 0u;
    }
    for (int k = threadIdx.x; k < n_sub * 12; k += 256) B.C[k / 12][k % 12] = f->C[vi][k / 12][k % 12];
    if (threadIdx.x == 0) {
        B.nbig = 0u;
        B.pairs = 0u;
        uint32_t acc = 0u;
        for (int sm = 0; sm < n_sub; ++sm) {
            B.first[sm] = acc;
            acc += subs[sm].ctrl->n_alloc;
        }
        B.first[n_sub] = acc;
    }
    // Frustum pre-test: a grown cube whose bounding sphere lies wholly behind
    // the near plane, or wholly beyond one of the planes through the camera
    // centre and the image borders moved out by 2 pixels, has no point in
    // front of the near plane that projects onto the image, so cube_record
    // would reject it.  The planes in camera coordinates (x, y, z): u < -2 is
    // fx x + (cx + 2) z < 0 and u > W + 1 is fx x + (cx - W - 1) z > 0 for
    // z > 0, likewise v; their normals' lengths scale the sphere radius.  The
    // radius (half the grown cube's diagonal) is padded far beyond the
    // rounding of the centre's transform.
    const float rad = (float)(4 + kExpand) * 1.7320508f * voxel * 1.01f + 1e-4f;
    const float al_ = vc.cx + 2.0f, ar_ = vc.cx - (float)vc.W - 1.0f;
    const float at_ = vc.cy + 2.0f, ab_ = vc.cy - (float)vc.H - 1.0f;
    const float rl = rad * sqrtf(vc.fx * vc.fx + al_ * al_), rr = rad * sqrtf(vc.fx * vc.fx + ar_ * ar_);
    const float rt = rad * sqrtf(vc.fy * vc.fy + at_ * at_), rb = rad * sqrtf(vc.fy * vc.fy + ab_ * ab_);
    __syncthreads();
    const uint32_t total = B.first[n_sub];
    // whole chunks for every thread of the workgroup (barriers inside)
    for (uint32_t c0 = blockIdx.x * 256u; c0 < total; c0 += gridDim.x * 256u) {
        const uint32_t gi = c0 + threadIdx.x;
        bool hit = false;
        Rec ex, r;
        int bx = 0, by = 0, bz = 0, ptr = 0, sm = 0;
        const float *M = B.C[0];
        if (gi < total) {
            // the submap of flat index gi: the last with first[sm] <= gi
#pragma unroll
            for (int step = kMaxSubmaps / 2; step; step >>= 1)
                if (sm + step < n_sub && B.first[sm + step] <= gi) sm += step;
            M = B.C[sm];
            const int4 b = subs[sm].alist[gi - B.first[sm]];
            bx = (int16_t)(b.x & 0xffff);
            by = (int16_t)((uint32_t)b.x >> 16);
            bz = b.y;
            ptr = b.z;
            const float X = (float)(8 * bx + 4) * voxel, Y = (float)(8 * by + 4) * voxel;
            const float Z = (float)(8 * bz + 4) * voxel;
            const float xc = ((M[0] * X + M[1] * Y) + M[2] * Z) + M[3];
            const float yc = ((M[4] * X + M[5] * Y) + M[6] * Z) + M[7];
            const float zc = ((M[8] * X + M[9] * Y) + M[10] * Z) + M[11];
            const bool outside = zc + rad < kZNear || vc.fx * xc + al_ * zc < -rl || vc.fx * xc + ar_ * zc > rr ||
                                 vc.fy * yc + at_ * zc < -rt || vc.fy * yc + ab_ * zc > rb;
            hit = !outside && cube_record(M, vc, voxel, 8 * bx - kExpand, 8 * by - kExpand, 8 * bz - kExpand,
                                          8 + 2 * kExpand, ex);
        }
        if (!FILL) {
            const unsigned long long m = __ballot(hit);
            if (m && lane_id() == (uint32_t)(__ffsll((long long)m) - 1)) atomicAdd(&B.pairs, (uint32_t)__popcll(m));
        }
        const int tx0 = hit ? ex.x0 / tw : 1, tx1 = hit ? ex.x1 / tw : 0;
        const int ty0 = hit ? ex.y0 / th : 1, ty1 = hit ? ex.y1 / th : 0;
        const int nx = tx1 - tx0 + 1, ntl = nx * (ty1 - ty0 + 1);
        const bool direct = ntl > kBinDirect;
        // a block over many tiles: queued for the whole workgroup (the count
        // pass here, the fill pass with its record below), unless the queue
        // is full; its tiles then take one global atomic each from this thread
        bool queued = false;
        if (!FILL && hit && direct) {
            const uint32_t j = atomicAdd(&B.nbig, 1u);
            if (j < (uint32_t)kBinBig) {
                B.big_box[j] = make_int4(tx0, ty0, nx, ntl);
                queued = true;
            }
        }
        // entries per distinct tile of the chunk
        if (!queued)
            for (int ty = ty0; ty <= ty1; ++ty)
                for (int tx = tx0; tx <= tx1; ++tx) {
                    const uint32_t g = (uint32_t)(base + ty * ntx + tx);
                    const int sl = direct ? -1 : bin_slot(B, g, true);
                    if (sl >= 0)
                        atomicAdd(&B.cnt[sl], 1u);
                    else if (!FILL)
                        atomicAdd(&t.cnt[g], 1);
                }
        __syncthreads();
        const uint32_t nq = FILL ? 0u : (B.nbig < (uint32_t)kBinBig ? B.nbig : (uint32_t)kBinBig);
        // one global atomic per distinct tile: its count, or its range in the bin
        for (int k = threadIdx.x; k < kBinSlots; k += 256) {
            const uint32_t g = B.tile[k];
            if (g == kNoTile) continue;
            if (FILL)
                B.pos[k] = t.off[g] + (uint32_t)atomicAdd(&t.cur[g], (int)B.cnt[k]);
            else
                atomicAdd(&t.cnt[g], (int)B.cnt[k]);
        }
        __syncthreads();
        // count pass: the queued blocks' tiles, shared by every thread
        for (uint32_t j = 0; j < nq; ++j) {
            const int4 bb = B.big_box[j];
            for (int k = (int)threadIdx.x; k < bb.w; k += 256)
                atomicAdd(&t.cnt[(uint32_t)(base + (bb.y + k / bb.z) * ntx + bb.x + k % bb.z)], 1);
        }
        if (FILL && hit) {
            // the search-range box of the block itself (empty when it is
            // behind the near plane or off the image: then it only feeds
            // the table)
            if (!cube_record(M, vc, voxel, 8 * bx, 8 * by, 8 * bz, 8, r)) {
                r.x0 = 1;
                r.x1 = 0;
                r.y0 = 1;
                r.y1 = 0;
                r.zlo = __builtin_inff();
                r.zhi = -__builtin_inff();
            }
            r.bx = (int16_t)bx;
            r.by = (int16_t)by;
            r.bz = (int16_t)bz;
            r.pad = (int16_t)sm;
            r.ptr = ptr;
            r.pad2 = (int32_t)__float_as_uint(ex.zlo);   // the grown cube's least camera depth (table depth cut)
            bool fq = false;
            if (direct) {
                const uint32_t j = atomicAdd(&B.nbig, 1u);
                if (j < (uint32_t)kBinBig) {
                    B.big_rec[j] = r;
                    B.big_box[j] = make_int4(tx0, ty0, nx, ntl);
                    fq = true;
                }
            }
            if (!fq)
                for (int ty = ty0; ty <= ty1; ++ty)
                    for (int tx = tx0; tx <= tx1; ++tx) {
                        const uint32_t g = (uint32_t)(base + ty * ntx + tx);
                        const int sl = direct ? -1 : bin_slot(B, g, false);
                        const uint32_t idx =
                            sl >= 0 ? atomicAdd(&B.pos[sl], 1u) : t.off[g] + (uint32_t)atomicAdd(&t.cur[g], 1);
                        if (idx < t.cap) t.bins[idx] = r;
                    }
        }
        if (FILL) {
            __syncthreads();   // every block queued
            // fill pass: the queued blocks' records, each tile by one thread
            const uint32_t nf = B.nbig < (uint32_t)kBinBig ? B.nbig : (uint32_t)kBinBig;
            for (uint32_t j = 0; j < nf; ++j) {
                const int4 bb = B.big_box[j];
                for (int k = (int)threadIdx.x; k < bb.w; k += 256) {
                    const uint32_t g = (uint32_t)(base + (bb.y + k / bb.z) * ntx + bb.x + k % bb.z);
                    const uint32_t idx = t.off[g] + (uint32_t)atomicAdd(&t.cur[g], 1);
                    if (idx < t.cap) t.bins[idx] = B.big_rec[j];
                }
            }
            __syncthreads();   // every slot position taken and the queue read before both are cleared
        }
        for (int k = threadIdx.x; k < kBinSlots; k += 256) {
            B.tile[k] = kNoTile;
            B.cnt[k] = 0u;
        }
        if (threadIdx.x == 0) B.nbig = 0u;
        __syncthreads();
    }
    // one global atomic per workgroup for the statistics (a same-address
    // atomic from every wave and chunk serialised the count pass)
    if (!FILL && threadIdx.x == 0 && B.pairs) atomicAdd(&t.mc->tot_blkview, (unsigned long long)B.pairs);
}

// exclusive offsets of the tile counts (one workgroup); clears the counts and
// cursors for the next launch
__global__ __launch_bounds__(1024) void k_m_scan(MTiles t)
{
    __shared__ uint32_t part[1024];
    const uint32_t n = t.n_tiles;
    const uint32_t per = (n + 1023u) / 1024u;
    const uint32_t b0 = threadIdx.x * per;
    const uint32_t b1 = b0 + per < n ? b0 + per : n;
    uint32_t sum = 0;
    for (uint32_t i = b0; i < b1; ++i) sum += (uint32_t)t.cnt[i];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (uint32_t d = 1; d < 1024u; d <<= 1) {
        const uint32_t add = threadIdx.x >= d ? part[threadIdx.x - d] : 0u;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - sum;
    for (uint32_t i = b0; i < b1; ++i) {
        const uint32_t c = (uint32_t)t.cnt[i];
        t.off[i] = run;
        run += c;
        t.cnt[i] = 0;
        t.cur[i] = 0;
    }
    if (threadIdx.x == 1023) {
        const uint32_t total = part[1023];
        t.off[n] = total;
        t.mc->tot_bin += total;
        t.mc->n_raycast += 1ull;
        if (total > t.cap) t.mc->flags |= TF_FLAG_BIN_OVERFLOW;
    }
}

__global__ __launch_bounds__(256) void k_m_clear(MTiles t)
{
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < t.n_tiles; i += gridDim.x * 256u) {
        t.cnt[i] = 0;
        t.cur[i] = 0;
        t.off[i] = 0u;
        t.acc_hits[i] = 0ull;
    }
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < kWorldCells; i += gridDim.x * 256u) t.wmask[i] = 0ull;
    if (blockIdx.x == 0 && threadIdx.x == 0) t.off[t.n_tiles] = 0u;
}

// slot of world cell (cx, cy, cz) (8-voxel cells of world voxel units) in the
// submap-mask array: a 512 x 512 x 128 window, cells a window apart share a
// slot (their masks merge, which only adds submaps to visit)
__device__ __forceinline__ uint32_t wcell_index(int cx, int cy, int cz)
{
    return (((uint32_t)cx & 511u) << 16) | (((uint32_t)cy & 511u) << 7) | ((uint32_t)cz & 127u);
}

// World submap masks: every block a selected submap gained this frame (its
// allocated list past n_marked) sets the submap's bit in the 8-voxel world
// cells of its cube's world-space box, grown by two voxels.  A trilinear
// read at a point reaches voxels within one voxel per submap axis, i.e.
// within sqrt(3) voxels of the point in world space, so a submap with any
// voxel of a block under the read of point P has its bit in P's cell (the
// growth also covers the rounding of the pose transforms).  A cell's mask
// thus lists every submap that can be allocated at, or weigh in the field
// at, any point of the cell.  Blocks are never removed, so bits are never
// cleared.
__global__ __launch_bounds__(256) void k_m_mark(const Vol *vols, const MSub *subs, const MFrame *f,
                                                unsigned long long *wmask)
{
    const int y = (int)blockIdx.y;
    if (y >= f->n_sel) return;
    const int si = f->sel[y];
    const Vol v = vols[si];
    const MSub &S = subs[si];
    const uint32_t n0 = v.ctrl->n_marked;
    uint32_t n1 = v.ctrl->n_alloc;
    if (n1 > v.n_blocks) n1 = v.n_blocks;
    for (uint32_t i = n0 + blockIdx.x * 256u + threadIdx.x; i < n1; i += gridDim.x * 256u) {
        const int4 a = v.alist[i];
        const int bx = (int16_t)(a.x & 0xffff), by = (int16_t)((uint32_t)a.x >> 16), bz = a.y;
        float lo[3] = {__builtin_inff(), __builtin_inff(), __builtin_inff()};
        float hi[3] = {-__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
        for (int k = 0; k < 8; ++k) {
            // corner of the block in submap voxel units, to world: P = R^T (Q - s)
            const float q0 = (float)(8 * (bx + (k & 1))) - S.s[0];
            const float q1 = (float)(8 * (by + ((k >> 1) & 1))) - S.s[1];
            const float q2 = (float)(8 * (bz + (k >> 2))) - S.s[2];
            for (int r = 0; r < 3; ++r) {
                const float w = (S.R[r] * q0 + S.R[3 + r] * q1) + S.R[6 + r] * q2;
                lo[r] = w < lo[r] ? w : lo[r];
                hi[r] = w > hi[r] ? w : hi[r];
            }
        }
        int c0[3], c1[3];
        for (int r = 0; r < 3; ++r) {
            c0[r] = ((int)floorf(lo[r] - 2.0f)) >> 3;
            c1[r] = ((int)floorf(hi[r] + 2.0f)) >> 3;
        }
        const unsigned long long bit = 1ull << (uint32_t)si;
        for (int cx = c0[0]; cx <= c1[0]; ++cx)
            for (int cy = c0[1]; cy <= c1[1]; ++cy)
                for (int cz = c0[2]; cz <= c1[2]; ++cz) atomicOr(&wmask[wcell_index(cx, cy, cz)], bit);
    }
}

// ============================================================================
// combined-field raycast
// ============================================================================
namespace {

// Depth buckets of the table cut: 1/32 octave each from the near plane up
// (the float bits of a depth above the near plane, shifted), 256 buckets
// (about 0.05 to 12.8 m; deeper depths share the last)
constexpr uint32_t kZBuckets = 256;
constexpr uint32_t kZNearBits = 0x3d4ccccdu;   // kZNear's float bits

__device__ __forceinline__ uint32_t zbucket(uint32_t zbits)
{
    const int b = (int)(zbits >> 18) - (int)(kZNearBits >> 18);
    return b < 0 ? 0u : (b >= (int)kZBuckets ? kZBuckets - 1u : (uint32_t)b);
}

// least depth of bucket b (b >= 1)
__device__ __forceinline__ float zbucket_floor(uint32_t b)
{
    return __uint_as_float(((kZNearBits >> 18) + b) << 18);
}

// LDS of one tile: the (submap, block) -> pointer table, the tile's submaps
// in ascending order with what the field reads, and the per-pixel range
template <int NT>
struct MTileLds {
    static constexpr int TT = NT >= 128 ? 4096 : 2048;   // table slots (8 bytes each)
    unsigned long long slot[TT];                // 0 = empty, else mkey(...) | device pointer
    float Rs[kMaxSubmaps][12];                  // rotation rows, then translation (voxel units)
    const DEntry *ent[kMaxSubmaps];
    const uint32_t *occ[kMaxSubmaps];
    const uint8_t *vox[kMaxSubmaps];
    uint32_t nb[kMaxSubmaps], ne[kMaxSubmaps];
    int smid[kMaxSubmaps];
    unsigned long long mask;
    uint32_t n_tab, hits, unfit;                // unfit: a record whose key or pointer does not pack
    uint32_t cut;                               // depth buckets 0 .. cut - 1 are in the table
    float dlim;                                 // a lookup miss proves absence for reads of points shallower than this
    uint32_t zlo[NT], zhi[NT];                  // per-pixel range as float bits (all values > 0)
    uint32_t zlo_all, zhi_all;                  // from records covering the whole tile
};

template <int NT>
__device__ __forceinline__ uint32_t mslot(int sm, int bx, int by, int bz)
{
    return (hash_index(bx, by, bz, 0xffffffffu) ^ ((uint32_t)sm * 0x9e3779b1u)) & (uint32_t)(MTileLds<NT>::TT - 1);
}

// packed table slot: valid bit 63, submap (6 bits), bz, by, bx (11-bit
// two's complement each) above the 24-bit device block pointer
__device__ __forceinline__ bool mfits(int bx, int by, int bz)
{
    return bx >= -1024 && bx < 1024 && by >= -1024 && by < 1024 && bz >= -1024 && bz < 1024;
}

__device__ __forceinline__ unsigned long long mkey(int sm, int bx, int by, int bz)
{
    return (1ull << 63) | ((unsigned long long)sm << 57) | ((unsigned long long)(bz & 0x7ff) << 46) |
           ((unsigned long long)(by & 0x7ff) << 35) | ((unsigned long long)(bx & 0x7ff) << 24);
}

// Search range of the pixel and the tile's LDS state from its bin.  The range
// is a min/max over the records covering the pixel: each record updates the
// pixels of its box inside the tile with LDS atomics (positive floats order
// like their bit patterns); a record covering the whole tile updates one
// tile-wide pair instead.  Every thread of the workgroup calls it; pixel
// (px, py) is the calling thread's, the tile spans [tx0, tx0 + TW) x [ty0, ty0 + TH).
template <int NT, int TW, int TH>
__device__ __forceinline__ void m_tile_setup(const MSub *subs, const MTiles &t, uint32_t g, int tx0, int ty0,
                                             MTileLds<NT> &L)
{
    constexpr int TT = MTileLds<NT>::TT;
    for (int k = threadIdx.x; k < TT; k += NT) L.slot[k] = 0ull;
    L.zlo[threadIdx.x] = 0x7f800000u;   // +inf
    L.zhi[threadIdx.x] = 0u;            // below every positive float
    if (threadIdx.x == 0) {
        L.mask = 0ull;
        L.n_tab = 0u;
        L.hits = 0u;
        L.unfit = 0u;
        L.zlo_all = 0x7f800000u;
        L.zhi_all = 0u;
    }
    const uint32_t o0 = t.off[g];
    uint32_t o1 = t.off[g + 1];
    if (o1 > t.cap) o1 = t.cap;
    const int n = o1 > o0 ? (int)(o1 - o0) : 0;
    uint32_t cut = kZBuckets;
    if (n > TT / 2) {
        // More records than the table holds: those nearest the camera go in.
        // A histogram of the grown cubes' least depths (in the table's first
        // slots, cleared again below) gives the largest bucket prefix that
        // fits; a read at a point shallower than the first left-out bucket
        // cannot touch a left-out block (it lies in that block's grown cube).
        __syncthreads();
        uint32_t *hist = reinterpret_cast<uint32_t *>(L.slot);
        for (int j = (int)threadIdx.x; j < n; j += NT)
            atomicAdd(&hist[zbucket((uint32_t)t.bins[o0 + (uint32_t)j].pad2)], 1u);
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t acc = 0u, c = 0u;
            while (c < kZBuckets && acc + hist[c] <= (uint32_t)(TT / 2)) acc += hist[c++];
            L.cut = c;
        }
        __syncthreads();
        cut = L.cut;
        for (int k = threadIdx.x; k < kZBuckets; k += NT) hist[k] = 0u;
    }
    if (threadIdx.x == 0) L.dlim = cut >= kZBuckets ? __builtin_inff() : zbucket_floor(cut);
    __syncthreads();
    for (int j = (int)threadIdx.x; j < n; j += NT) {
        const Rec r = t.bins[o0 + (uint32_t)j];
        atomicOr(&L.mask, 1ull << (uint32_t)r.pad);
        // keys in one bin are distinct; the table is at most half full
        if (zbucket((uint32_t)r.pad2) >= cut) {
            // left out: deeper than the table's depth limit
        } else if (!mfits(r.bx, r.by, r.bz) || r.ptr >= (1 << 24)) {
            L.unfit = 1u;
        } else if (atomicAdd(&L.n_tab, 1u) < (uint32_t)(TT / 2)) {
            const unsigned long long val = mkey(r.pad, r.bx, r.by, r.bz) | (unsigned long long)r.ptr;
            uint32_t sl = mslot<NT>(r.pad, r.bx, r.by, r.bz);
            for (int k = 0; k < TT; ++k) {
                if (atomicCAS(&L.slot[sl], 0ull, val) == 0ull) break;
                sl = (sl + 1u) & (uint32_t)(TT - 1);
            }
        }
        const int x0 = r.x0 > tx0 ? r.x0 : tx0, x1 = r.x1 < tx0 + TW - 1 ? r.x1 : tx0 + TW - 1;
        const int y0 = r.y0 > ty0 ? r.y0 : ty0, y1 = r.y1 < ty0 + TH - 1 ? r.y1 : ty0 + TH - 1;
        if (x0 > x1 || y0 > y1) continue;
        const uint32_t lo = __float_as_uint(r.zlo), hi = __float_as_uint(r.zhi);
        if (x0 == tx0 && x1 == tx0 + TW - 1 && y0 == ty0 && y1 == ty0 + TH - 1) {
            atomicMin(&L.zlo_all, lo);
            atomicMax(&L.zhi_all, hi);
            continue;
        }
        for (int y = y0; y <= y1; ++y)
            for (int x = x0; x <= x1; ++x) {
                const int pi = (y - ty0) * TW + (x - tx0);
                atomicMin(&L.zlo[pi], lo);
                atomicMax(&L.zhi[pi], hi);
            }
    }
    __syncthreads();
    // the tile's submaps, ascending
    if (threadIdx.x < (unsigned)kMaxSubmaps) {
        const unsigned long long m = L.mask;
        const int sm = (int)threadIdx.x;
        if ((m >> sm) & 1ull) {
            const int k = __popcll(m & ((1ull << sm) - 1ull));
            const MSub &S = subs[sm];
            for (int q = 0; q < 9; ++q) L.Rs[k][q] = S.R[q];
            for (int q = 0; q < 3; ++q) L.Rs[k][9 + q] = S.s[q];
            L.ent[k] = S.entries;
            L.occ[k] = S.occ;
            L.vox[k] = S.voxels;
            L.nb[k] = S.n_buckets;
            L.ne[k] = S.n_excess;
            L.smid[k] = sm;
        }
    }
    __syncthreads();
}

// the calling thread's pixel range after m_tile_setup (pixel index pi in the tile)
template <int NT>
__device__ __forceinline__ void m_pixel_range(const MTileLds<NT> &L, int pi, float &zmin, float &zmax)
{
    const uint32_t lo = L.zlo[pi] < L.zlo_all ? L.zlo[pi] : L.zlo_all;
    const uint32_t hi = L.zhi[pi] > L.zhi_all ? L.zhi[pi] : L.zhi_all;
    zmin = __uint_as_float(lo);                               // +inf when nothing covers the pixel
    zmax = hi ? __uint_as_float(hi) : -__builtin_inff();
}

// device pointer of block (bx, by, bz) of the k-th submap of the tile (-1 =
// absent): the LDS table first; unless `local`, then the submap's bucket
// bitmap and hash table.  `local` holds when the table has every record of
// the tile's bin and the read belongs to a ray point at or beyond the near
// plane: every block within 3 voxels of such a point is in the bin (blocks
// are binned by their cube grown by 3 voxels), so a miss proves absence.
// A lookup in two halves, so that two submaps' lookups can be in flight
// together: begin probes the LDS table and, when the table cannot answer,
// issues the bucket's occupancy word and entry loads; end resolves them
// (walking the chain beyond the bucket when the entry is another block's).
struct MLookup {
    int ptr;        // the answer when `pending` is false
    bool pending;
    uint32_t h, ow;
    int4 w;
};

template <int NT>
__device__ __forceinline__ void m_lookup_begin(const MTileLds<NT> &L, int k, int bx, int by, int bz, bool local,
                                               MLookup &q)
{
    constexpr int TT = MTileLds<NT>::TT;
    q.pending = false;
    q.ptr = -1;
    if (!in_short_range(bx) || !in_short_range(by) || !in_short_range(bz)) return;
    const int sm = L.smid[k];
    if (mfits(bx, by, bz)) {
        const unsigned long long key = mkey(sm, bx, by, bz) >> 24;
        uint32_t sl = mslot<NT>(sm, bx, by, bz);
        for (int it = 0; it < TT; ++it) {
            const unsigned long long kk = L.slot[sl];
            if ((kk >> 24) == key) {
                q.ptr = (int)(kk & 0xffffffull);
                return;
            }
            if (kk == 0ull) break;
            sl = (sl + 1u) & (uint32_t)(TT - 1);
        }
    }
    if (local) return;
    q.pending = true;
    q.h = hash_index(bx, by, bz, L.nb[k] - 1u);
    q.ow = gload(L.occ[k] + (q.h >> 5));
    q.w = load_entry(L.ent[k], q.h);
}

template <int NT>
__device__ __forceinline__ int m_lookup_end(const MTileLds<NT> &L, int k, int bx, int by, int bz, const MLookup &q)
{
    if (!q.pending) return q.ptr;
    if (!((q.ow >> (q.h & 31u)) & 1u)) return -1;
    const uint32_t kxy = (uint32_t)(uint16_t)bx | ((uint32_t)(uint16_t)by << 16);
    const int4 w = q.w;
    if ((uint32_t)w.x == kxy && (int16_t)(w.y & 0xffff) == (int16_t)bz && w.w >= 0) return w.w;
    if (w.z < 1 || (uint32_t)(w.z - 1) >= L.ne[k]) return -1;
    int ptr = -1;
    const int e = find_entry_from(L.ent[k], L.nb[k], L.ne[k], L.nb[k] + (uint32_t)(w.z - 1), bx, by, bz, 0, &ptr);
    return e >= 0 ? ptr : -1;
}

template <int NT>
__device__ __forceinline__ int m_lookup(const MTileLds<NT> &L, int k, int bx, int by, int bz, bool local)
{
    constexpr int TT = MTileLds<NT>::TT;
    if (!in_short_range(bx) || !in_short_range(by) || !in_short_range(bz)) return -1;
    const int sm = L.smid[k];
    if (mfits(bx, by, bz)) {
        const unsigned long long key = mkey(sm, bx, by, bz) >> 24;
        uint32_t sl = mslot<NT>(sm, bx, by, bz);
        for (int it = 0; it < TT; ++it) {
            const unsigned long long kk = L.slot[sl];
            if ((kk >> 24) == key) return (int)(kk & 0xffffffull);
            if (kk == 0ull) break;
            sl = (sl + 1u) & (uint32_t)(TT - 1);
        }
    }
    if (local) return -1;
    // the bucket's occupancy bit and its entry, loaded together; the chain
    // beyond the bucket only when the entry is another block's
    const uint32_t h = hash_index(bx, by, bz, L.nb[k] - 1u);
    const uint32_t ow = gload(L.occ[k] + (h >> 5));
    const int4 w = load_entry(L.ent[k], h);
    if (!((ow >> (h & 31u)) & 1u)) return -1;
    const uint32_t kxy = (uint32_t)(uint16_t)bx | ((uint32_t)(uint16_t)by << 16);
    if ((uint32_t)w.x == kxy && (int16_t)(w.y & 0xffff) == (int16_t)bz && w.w >= 0) return w.w;
    if (w.z < 1 || (uint32_t)(w.z - 1) >= L.ne[k]) return -1;
    int ptr = -1;
    const int e = find_entry_from(L.ent[k], L.nb[k], L.ne[k], L.nb[k] + (uint32_t)(w.z - 1), bx, by, bz, 0, &ptr);
    return e >= 0 ? ptr : -1;
}

template <int NT>
__device__ __forceinline__ void to_sub(const MTileLds<NT> &L, int k, float P0, float P1, float P2, float &Q0,
                                       float &Q1, float &Q2)
{
    const float *R = L.Rs[k];
    Q0 = ((R[0] * P0 + R[1] * P1) + R[2] * P2) + R[9];
    Q1 = ((R[3] * P0 + R[4] * P1) + R[5] * P2) + R[10];
    Q2 = ((R[6] * P0 + R[7] * P1) + R[8] * P2) + R[11];
}

// position in the tile's submap list of submap sm (a bit of L.mask)
template <int NT>
__device__ __forceinline__ int tile_slot(const MTileLds<NT> &L, int sm)
{
    return __popcll(L.mask & ((1ull << (uint32_t)sm) - 1ull));
}

// the tile's submaps that can be allocated at, or weigh in the field at,
// world voxel-unit point P: the mask of P's world cell within the tile's set
template <int NT>
__device__ __forceinline__ unsigned long long m_cell_mask(const MTiles &t, const MTileLds<NT> &L, float P0, float P1,
                                                          float P2)
{
    return gload(t.wmask + wcell_index(block_of(P0), block_of(P1), block_of(P2))) & L.mask;
}

// "allocated" of the combined map: some submap has a device block at
// floor(P_i X); only the submaps of P's cell mask cm can
template <int NT>
__device__ __forceinline__ bool m_allocated(const MTileLds<NT> &L, unsigned long long cm, float P0, float P1, float P2,
                                            bool local)
{
    for (; cm; cm &= cm - 1ull) {
        const int k = tile_slot(L, __ffsll((long long)cm) - 1);
        float Q0, Q1, Q2;
        to_sub(L, k, P0, P1, P2, Q0, Q1, Q2);
        if (m_lookup(L, k, block_of(Q0), block_of(Q1), block_of(Q2), local) >= 0) return true;
    }
    return false;
}

// one submap's trilinear cell at P: the fractions, the base voxel and its
// block, the crossed faces and (once set up) the corner pointers
struct MCell {
    float tx, ty, tz;
    int ix, iy, iz;
    int p[8];
};

template <int NT>
__device__ __forceinline__ void m_cell_begin(const MTileLds<NT> &L, int k, float P0, float P1, float P2, bool local,
                                             MCell &C, MLookup &q)
{
    float Q0, Q1, Q2;
    to_sub(L, k, P0, P1, P2, Q0, Q1, Q2);
    const float fbx = floorf(Q0), fby = floorf(Q1), fbz = floorf(Q2);
    C.tx = Q0 - fbx;
    C.ty = Q1 - fby;
    C.tz = Q2 - fbz;
    C.ix = (int)fbx;
    C.iy = (int)fby;
    C.iz = (int)fbz;
    m_lookup_begin(L, k, C.ix >> 3, C.iy >> 3, C.iz >> 3, local, q);
}

// the corner pointers: the cell's own block from the pending lookup, the
// blocks across crossed faces looked up directly
template <int NT>
__device__ __forceinline__ void m_cell_end(const MTileLds<NT> &L, int k, bool local, MCell &C, const MLookup &q)
{
    const int Bx = C.ix >> 3, By = C.iy >> 3, Bz = C.iz >> 3;
    const bool sx = (C.ix & 7) == 7, sy = (C.iy & 7) == 7, sz = (C.iz & 7) == 7;
    const int p000 = m_lookup_end(L, k, Bx, By, Bz, q);
    int p100 = p000, p010 = p000, p001 = p000, p110 = p000, p101 = p000, p011 = p000, p111 = p000;
    if (sx | sy | sz) {
        if (sx) p100 = m_lookup(L, k, Bx + 1, By, Bz, local);
        if (sy) p010 = m_lookup(L, k, Bx, By + 1, Bz, local);
        if (sz) p001 = m_lookup(L, k, Bx, By, Bz + 1, local);
        p110 = (sx & sy) ? m_lookup(L, k, Bx + 1, By + 1, Bz, local) : (sx ? p100 : p010);
        p101 = (sx & sz) ? m_lookup(L, k, Bx + 1, By, Bz + 1, local) : (sx ? p100 : p001);
        p011 = (sy & sz) ? m_lookup(L, k, Bx, By + 1, Bz + 1, local) : (sy ? p010 : p001);
        p111 = (sx & sy & sz) ? m_lookup(L, k, Bx + 1, By + 1, Bz + 1, local)
                              : (sx & sy) ? p110 : (sx & sz) ? p101 : (sy & sz) ? p011 : sx ? p100 : sy ? p010 : p001;
    }
    C.p[0] = p000;
    C.p[1] = p100;
    C.p[2] = p010;
    C.p[3] = p110;
    C.p[4] = p001;
    C.p[5] = p101;
    C.p[6] = p011;
    C.p[7] = p111;
}

// the cell's SDF and weight reads (an absent corner reads block 0; its
// values are not used)
template <int NT>
__device__ __forceinline__ void m_cell_load(const MTileLds<NT> &L, int k, const MCell &C, int16_t (&s)[8],
                                            uint8_t (&w8)[8])
{
    const uint8_t *vox = L.vox[k];
    int j[8];
    cell_index(C.ix, C.iy, C.iz, (C.ix & 7) == 7, (C.iy & 7) == 7, (C.iz & 7) == 7, j);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const uint8_t *blk = vox + (size_t)(C.p[c] >= 0 ? C.p[c] : 0) * kBlockBytes;
        s[c] = gload(reinterpret_cast<const int16_t *>(blk) + j[c]);
        w8[c] = gload(blk + 1024 + j[c]);
    }
}

// one submap's term of the combined field: its trilinear weight (absent
// voxels weigh 0, same lerp order as the SDF) and, when positive, its F
__device__ __forceinline__ void m_cell_accumulate(const MCell &C, const int16_t (&s)[8], const uint8_t (&w8)[8],
                                                  int &cnt, float &first, float &num, float &den)
{
    float wf[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) wf[c] = C.p[c] >= 0 ? (float)w8[c] : 0.0f;
    const float c00 = wf[0] + (wf[1] - wf[0]) * C.tx;
    const float c10 = wf[2] + (wf[3] - wf[2]) * C.tx;
    const float c01 = wf[4] + (wf[5] - wf[4]) * C.tx;
    const float c11 = wf[6] + (wf[7] - wf[6]) * C.tx;
    const float c0 = c00 + (c10 - c00) * C.ty;
    const float c1 = c01 + (c11 - c01) * C.ty;
    const float w = c0 + (c1 - c0) * C.tz;
    if (!(w > 0.0f)) return;
    uint32_t present = 0u;
#pragma unroll
    for (int c = 0; c < 8; ++c) present |= (C.p[c] >= 0 ? 1u : 0u) << c;
    const float F = cell_lerp(present, s, C.tx, C.ty, C.tz);
    if (cnt == 0) first = F;
    num = num + w * F;
    den = den + w;
    ++cnt;
}

// combined field at world voxel-unit P over the submaps of P's cell mask cm
// (every submap with positive weight at P is one of them), in ascending
// submap order.  Submaps are taken two at a time: both cells' lookups, then
// both cells' reads are in flight together before either term is added.
template <int NT>
__device__ __forceinline__ float m_field(const MTileLds<NT> &L, unsigned long long cm, float P0, float P1, float P2,
                                         bool local)
{
    int cnt = 0;
    float first = 1.0f, num = 0.0f, den = 0.0f;
    while (cm) {
        const int ka = tile_slot(L, __ffsll((long long)cm) - 1);
        cm &= cm - 1ull;
        const bool two = cm != 0ull;
        const int kb = two ? tile_slot(L, __ffsll((long long)cm) - 1) : ka;
        if (two) cm &= cm - 1ull;
        MCell A, B;
        MLookup qa, qb;
        m_cell_begin(L, ka, P0, P1, P2, local, A, qa);
        if (two) m_cell_begin(L, kb, P0, P1, P2, local, B, qb);
        m_cell_end(L, ka, local, A, qa);
        if (two) m_cell_end(L, kb, local, B, qb);
        int16_t sa[8], sb[8];
        uint8_t wa[8], wb[8];
        m_cell_load(L, ka, A, sa, wa);
        if (two) m_cell_load(L, kb, B, sb, wb);
        m_cell_accumulate(A, sa, wa, cnt, first, num, den);
        if (two) m_cell_accumulate(B, sb, wb, cnt, first, num, den);
    }
    if (cnt == 0) return 1.0f;
    if (cnt == 1) return first;
    return num / den;
}

enum { M_COARSE, M_FINE, M_SURFACE, M_BEHIND, M_WRONG_SIDE };

// the view of flat tile index g (views are few; their tile ranges ascend)
__device__ __forceinline__ int view_of(const MFrame *f, int g)
{
    int vi = 0;
    while (vi + 1 < f->n_views && g >= f->view[vi + 1].tile_base) ++vi;
    return vi;
}

}  // namespace

// one workgroup per TW x TH tile of any view; waves cover 8x8 pixel squares
template <int TW, int TH>
__global__ __launch_bounds__(TW *TH) void k_m_raycast(const MSub *subs, const MFrame *f, MTiles t, float voxel,
                                                      float mu)
{
    constexpr int NT = TW * TH;
    __shared__ MTileLds<NT> L;
    const int g = (int)blockIdx.x;
    const int vi = view_of(f, g);
    const MView &V = f->view[vi];
    const int tile = g - V.tile_base;
    const int W = V.cam.W, H = V.cam.H;
    const int q = (int)threadIdx.x >> 6, i = (int)threadIdx.x & 63;
    const int tx0 = (tile % V.ntx) * TW, ty0 = (tile / V.ntx) * TH;
    const int lx = (q % (TW / 8)) * 8 + (i & 7), ly = (q / (TW / 8)) * 8 + (i >> 3);
    const int px = tx0 + lx, py = ty0 + ly;
    float zmin, zmax;
    m_tile_setup<NT, TW, TH>(subs, t, (uint32_t)g, tx0, ty0, L);
    m_pixel_range<NT>(L, ly * TW + lx, zmin, zmax);
    // the table holds every record of the bin shallower than its depth cut
    const bool full = L.n_tab <= (uint32_t)(MTileLds<NT>::TT / 2) && !L.unfit;
    // reads at points shallower than dcut (the cut less a voxel for the
    // normal's taps and a millimetre for rounding) can trust a table miss
    const float dcut = L.dlim - voxel - 1e-3f;
    const bool inside = px < W && py < H;
    float4 out_p = make_float4(0.f, 0.f, 0.f, 0.f), out_n = make_float4(0.f, 0.f, 0.f, 0.f);
    if (inside && zmin <= zmax) {
        const Cam &c = V.cam;
        const float inv_vs = 1.0f / voxel;
        const float mu_v = mu * inv_vs;
        const float ox = c.ti[0] * inv_vs, oy = c.ti[1] * inv_vs, oz = c.ti[2] * inv_vs;
        const float a = ((float)px - c.cx) / c.fx;
        const float b = ((float)py - c.cy) / c.fy;
        const float nr = sqrtf((a * a + b * b) + 1.0f);
        const float rcx = a / nr, rcy = b / nr, rcz = 1.0f / nr;
        const float zscale = voxel * rcz;   // camera z of ray parameter t (voxel units)
        const float dx = (c.Ri[0] * rcx + c.Ri[1] * rcy) + c.Ri[2] * rcz;
        const float dy = (c.Ri[3] * rcx + c.Ri[4] * rcy) + c.Ri[5] * rcz;
        const float dz = (c.Ri[6] * rcx + c.Ri[7] * rcy) + c.Ri[8] * rcz;
        float tt = (zmin * nr) * inv_vs;
        const float t_end = (zmax * nr) * inv_vs;
        int state = M_COARSE;
        float F = 1.0f;
        int steps = 0;
        while (tt < t_end && steps < kMaxRaySteps) {
            if (state == M_COARSE || state == M_FINE) {
                // Empty-space skip: while no block is found the march keeps
                // its fixed step; the world cells of the next kSkip positions
                // are tested together, a clear cell proves the position
                // unallocated, so the iterations skipped are those the loop
                // would run.
                const float stp = state == M_COARSE ? 8.0f : mu_v;
                constexpr int kSkip = 4;
                float tk[kSkip];
                unsigned long long wk[kSkip];
                float t2 = tt;
#pragma unroll
                for (int k = 0; k < kSkip; ++k) {
                    tk[k] = t2;
                    wk[k] = m_cell_mask<NT>(t, L, ox + t2 * dx, oy + t2 * dy, oz + t2 * dz);
                    t2 += stp;
                }
                bool stop = false;
#pragma unroll
                for (int k = 0; k < kSkip; ++k) {
                    if (stop) continue;
                    tt = tk[k];
                    if (!(tt < t_end && steps < kMaxRaySteps) || wk[k]) {
                        stop = true;
                        continue;
                    }
                    ++steps;   // an iteration on unallocated space
                }
                if (!stop) tt = t2;
                if (!(tt < t_end && steps < kMaxRaySteps)) break;
            }
            ++steps;
            const float P0 = ox + tt * dx, P1 = oy + tt * dy, P2 = oz + tt * dz;
            const bool local = full && tt * zscale >= kZNear && tt * zscale < dcut;
            // only the submaps of P's world cell can be allocated there
            const unsigned long long cm = m_cell_mask<NT>(t, L, P0, P1, P2);
            const bool alloc = cm && m_allocated(L, cm, P0, P1, P2, local);
            if (state == M_COARSE) {
                if (!alloc) {
                    tt += 8.0f;
                } else {
                    tt -= 8.0f;
                    state = M_FINE;
                }
            } else if (!alloc) {
                state = M_FINE;
                tt += mu_v;
            } else {
                F = m_field(L, cm, P0, P1, P2, local);
                if (state == M_SURFACE) {
                    if (F < 0.0f) {
                        state = M_BEHIND;
                        break;
                    }
                    const float s = F * mu_v;
                    tt += (s > 1.0f) ? s : 1.0f;
                } else if (F < 0.0f) {
                    if (state == M_FINE) {
                        state = M_WRONG_SIDE;
                    } else {
                        const float s = -F * mu_v;
                        tt += (s > 1.0f) ? s : 1.0f;
                    }
                } else {
                    // FINE or WRONG_SIDE meeting F >= 0 turns to SURFACE without
                    // a step; the SURFACE iteration that follows (if the step
                    // bound allows it) reads the same field at the same t, so
                    // its step is taken here with this F
                    state = M_SURFACE;
                    if (steps < kMaxRaySteps) {
                        ++steps;
                        const float s = F * mu_v;
                        tt += (s > 1.0f) ? s : 1.0f;
                    }
                }
            }
        }
        if (state == M_BEHIND) {
            tt += F * mu_v;
            float P0 = ox + tt * dx, P1 = oy + tt * dy, P2 = oz + tt * dz;
            F = m_field(L, m_cell_mask<NT>(t, L, P0, P1, P2), P0, P1, P2,
                        full && tt * zscale >= kZNear && tt * zscale < dcut);
            tt += F * mu_v;
            P0 = ox + tt * dx;
            P1 = oy + tt * dy;
            P2 = oz + tt * dz;
            out_p = make_float4(P0 * voxel, P1 * voxel, P2 * voxel, 1.0f);
            // the taps lie within a voxel of the hit, which the cut's margin covers
            const bool lh = full && tt * zscale >= kZNear && tt * zscale < dcut;
            // the six taps P +- e_a, one per step of a rolled loop (one copy
            // of the field code, kept by selects)
            float fp0 = 0.0f, fm0 = 0.0f, fp1 = 0.0f, fm1 = 0.0f, fp2 = 0.0f, fm2 = 0.0f;
#pragma unroll 1
            for (int tap = 0; tap < 6; ++tap) {
                const int ax = tap >> 1;
                const bool minus = (tap & 1) != 0;
                const float X = ax == 0 ? (minus ? P0 - 1.0f : P0 + 1.0f) : P0;
                const float Y = ax == 1 ? (minus ? P1 - 1.0f : P1 + 1.0f) : P1;
                const float Z = ax == 2 ? (minus ? P2 - 1.0f : P2 + 1.0f) : P2;
                const float f = m_field(L, m_cell_mask<NT>(t, L, X, Y, Z), X, Y, Z, lh);
                fp0 = tap == 0 ? f : fp0;
                fm0 = tap == 1 ? f : fm0;
                fp1 = tap == 2 ? f : fp1;
                fm1 = tap == 3 ? f : fm1;
                fp2 = tap == 4 ? f : fp2;
                fm2 = tap == 5 ? f : fm2;
            }
            const float gx = (fp0 - fm0) * 0.5f;
            const float gy = (fp1 - fm1) * 0.5f;
            const float gz = (fp2 - fm2) * 0.5f;
            const float gn = sqrtf((gx * gx + gy * gy) + gz * gz);
            if (gn > 0.0f) out_n = make_float4(gx / gn, gy / gn, gz / gn, 1.0f);
        }
    }
    if (inside) {
        const size_t p = (size_t)py * W + px;
        V.pts[p] = out_p;
        V.nrm[p] = out_n;
        if (out_p.w == 1.0f) atomicAdd(&L.hits, 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0 && L.hits) t.acc_hits[g] += L.hits;
}

// search range of one view written as an image (parity of the range)
template <int TW, int TH>
__global__ __launch_bounds__(TW *TH) void k_m_range_write(const MSub *subs, const MFrame *f, MTiles t, int vi,
                                                          float *zmin_out, float *zmax_out)
{
    constexpr int NT = TW * TH;
    __shared__ MTileLds<NT> L;
    const MView &V = f->view[vi];
    const int g = V.tile_base + (int)blockIdx.x;
    const int tile = (int)blockIdx.x;
    const int q = (int)threadIdx.x >> 6, i = (int)threadIdx.x & 63;
    const int tx0 = (tile % V.ntx) * TW, ty0 = (tile / V.ntx) * TH;
    const int lx = (q % (TW / 8)) * 8 + (i & 7), ly = (q / (TW / 8)) * 8 + (i >> 3);
    const int px = tx0 + lx, py = ty0 + ly;
    float zmin, zmax;
    m_tile_setup<NT, TW, TH>(subs, t, (uint32_t)g, tx0, ty0, L);
    m_pixel_range<NT>(L, ly * TW + lx, zmin, zmax);
    if (px >= V.cam.W || py >= V.cam.H) return;
    zmin_out[(size_t)py * V.cam.W + px] = zmin;
    zmax_out[(size_t)py * V.cam.W + px] = zmax;
}

// ============================================================================
// launchers
// ============================================================================
hipError_t launch_m_alloc(const Vol *vols, const MSub *subs, const MFrame *f, unsigned long long *wmask, int w, int h,
                          hipStream_t s)
{
    const int npix = w * h;
    hipLaunchKernelGGL(k_m_alloc, dim3((npix + 255) / 256 + kKeepGroups, kMaxSel), dim3(256), 0, s, vols, f);
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    hipLaunchKernelGGL(k_m_insert, dim3(128, kMaxSel), dim3(256), 0, s, vols, f);
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    hipLaunchKernelGGL(k_m_mark, dim3(64, kMaxSel), dim3(256), 0, s, vols, subs, f, wmask);
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    hipLaunchKernelGGL(k_m_visible, dim3(256, kMaxSel), dim3(256), 0, s, vols, f);
    return hipGetLastError();
}

hipError_t launch_m_integrate(const Vol *vols, const MFrame *f, int nt, int grid, bool dry, hipStream_t s)
{
    if (grid < 1) grid = 1;
    if (grid > kIntegrateGrid) grid = kIntegrateGrid;
    const dim3 g(grid, kMaxSel);
    switch (nt) {
    case 64: hipLaunchKernelGGL(k_m_integrate<64>, g, dim3(64), 0, s, vols, f, dry ? 1 : 0); break;
    case 128: hipLaunchKernelGGL(k_m_integrate<128>, g, dim3(128), 0, s, vols, f, dry ? 1 : 0); break;
    case 512: hipLaunchKernelGGL(k_m_integrate<512>, g, dim3(512), 0, s, vols, f, dry ? 1 : 0); break;
    default: hipLaunchKernelGGL(k_m_integrate<256>, g, dim3(256), 0, s, vols, f, dry ? 1 : 0); break;
    }
    return hipGetLastError();
}

hipError_t launch_m_bin(const MSub *subs, const MFrame *f, const MTiles &t, int n_views, int grid, float voxel,
                        hipStream_t s)
{
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_m_bin<false>, dim3(grid, n_views), dim3(256), 0, s, subs, f, t, voxel);
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    hipLaunchKernelGGL(k_m_scan, dim3(1), dim3(1024), 0, s, t);
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    hipLaunchKernelGGL(k_m_bin<true>, dim3(grid, n_views), dim3(256), 0, s, subs, f, t, voxel);
    return hipGetLastError();
}

hipError_t launch_m_raycast(const MSub *subs, const MFrame *f, const MTiles &t, float voxel, float mu, int tw, int th,
                            hipStream_t s)
{
    const dim3 g(t.n_tiles);
    if (tw == 32 && th == 8)
        hipLaunchKernelGGL((k_m_raycast<32, 8>), g, dim3(256), 0, s, subs, f, t, voxel, mu);
    else if (tw == 8 && th == 8)
        hipLaunchKernelGGL((k_m_raycast<8, 8>), g, dim3(64), 0, s, subs, f, t, voxel, mu);
    else if (tw == 16 && th == 8)
        hipLaunchKernelGGL((k_m_raycast<16, 8>), g, dim3(128), 0, s, subs, f, t, voxel, mu);
    else if (tw == 16 && th == 16)
        hipLaunchKernelGGL((k_m_raycast<16, 16>), g, dim3(256), 0, s, subs, f, t, voxel, mu);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_m_range_write(const MSub *subs, const MFrame *f, const MTiles &t, int vi, int n_tiles_view,
                                float *zmin, float *zmax, int tw, int th, hipStream_t s)
{
    const dim3 g(n_tiles_view);
    if (tw == 32 && th == 8)
        hipLaunchKernelGGL((k_m_range_write<32, 8>), g, dim3(256), 0, s, subs, f, t, vi, zmin, zmax);
    else if (tw == 8 && th == 8)
        hipLaunchKernelGGL((k_m_range_write<8, 8>), g, dim3(64), 0, s, subs, f, t, vi, zmin, zmax);
    else if (tw == 16 && th == 8)
        hipLaunchKernelGGL((k_m_range_write<16, 8>), g, dim3(128), 0, s, subs, f, t, vi, zmin, zmax);
    else if (tw == 16 && th == 16)
        hipLaunchKernelGGL((k_m_range_write<16, 16>), g, dim3(256), 0, s, subs, f, t, vi, zmin, zmax);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_m_clear(const MTiles &t, hipStream_t s)
{
    hipLaunchKernelGGL(k_m_clear, dim3(2048), dim3(256), 0, s, t);
    return hipGetLastError();
}

}  // namespace tsdf
