// tsdf_kernels.hip -- gfx950 kernels of the voxel-hashed TSDF fusion hot path.
//
// Frame pipeline (one launch each, counts stay on the device):
//   k_alloc_rays   one lane per pixel: depth ingest, segment samples, hash probes,
//                  visible marks, de-duplicated insertion requests; workgroups
//                  past the image re-test the previous visible list   (Sec. 4.2, parts 1, 3)
//   k_insert       one lane per request: free-stack pops, bucket claim or excess
//                  chain link, block init                              (Sec. 4.2, part 2)
//   k_visible      16 entries per lane: scan compaction of the marks   (Sec. 4.2, part 3)
//   k_integrate    one wave per visible block, 8 voxels per lane; for the
//                  allocation view also the block's search-range record and
//                  its 16x16-pixel tile bins                           (Sec. 4.3, 4.4)
//   k_range_bin    one lane per block: projected box -> tile bins, for any
//                  other view                                          (Sec. 4.4)
//   k_raycast      one workgroup per 16x16 tile: per-pixel search range from the
//                  tile's bin, then the ray state machine                (Sec. 4.4)
//
// Compiled with -ffp-contract=off and correctly rounded fp32 division and
// square root: every float expression below is evaluated as written, one IEEE
// operation at a time.
#include <type_traits>

#include "tsdf_device.h"

namespace tsdf {

// ============================================================================
// initialisation
// ============================================================================
__global__ __launch_bounds__(256) void k_init(Vol v)
{
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = gid; i < v.n_entries; i += stride) {
        int4 e;
        e.x = 0;
        e.y = 0;
        e.z = 0;
        e.w = kPtrEmpty;
        *reinterpret_cast<int4 *>(v.entries + i) = e;
    }
    const size_t nvis = ((size_t)v.n_entries + 15) & ~(size_t)15;
    for (size_t i = gid; i < nvis; i += stride) v.vis[i] = 0;
    for (size_t i = gid; i < v.n_blocks; i += stride) v.free_blocks[i] = (int32_t)i;
    for (size_t i = gid; i < v.n_excess; i += stride) v.free_excess[i] = (int32_t)i;
    for (size_t i = gid; i <= v.reqset_mask; i += stride) v.reqset[i] = 0ull;
    if (v.host_has)
        for (size_t i = gid; i < nvis; i += stride) v.host_has[i] = 0;
    for (size_t i = gid; i < (size_t)kIntegrateGrid; i += stride) v.acc_cols[i] = 0ull;
    for (size_t i = gid; i < (size_t)(v.n_buckets / 32u); i += stride) v.occ[i] = 0u;
    for (size_t i = gid; i < (size_t)kBrickWords; i += stride) v.brick[i] = 0u;
    if (gid == 0) {
        Ctrl c = {};
        c.free_blocks = (int32_t)v.n_blocks;
        c.free_excess = (int32_t)v.n_excess;
        *v.ctrl = c;
    }
}

// zero n counters; with ctrl, also the record count (bins abandoned unread)
__global__ __launch_bounds__(256) void k_clear_bins(int32_t *bin_count, uint32_t n, Ctrl *ctrl)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        bin_count[i] = 0;
    if (ctrl && blockIdx.x == 0 && threadIdx.x == 0) ctrl->n_rec = 0u;
}

// ============================================================================
// allocation (Sec. 4.2) and integration (Sec. 4.3), one volume per launch
// ============================================================================
template <int FMT>
__global__ __launch_bounds__(256) void k_alloc_rays(Vol v, Cam c, const void *din)
{
    alloc_rays_body<FMT>(v, c, din, true);
}

__global__ __launch_bounds__(256) void k_insert(Vol v, Cam c) { insert_body(v, c); }

__global__ __launch_bounds__(256) void k_visible(Vol v) { visible_body(v); }

__global__ __launch_bounds__(256) void k_integrate(Vol v, Cam c, int bin)
{
    __shared__ float rcp_w[260];
    __shared__ uint32_t wg_cols;
    integrate_body<256>(v, c, rcp_w, &wg_cols, false, bin != 0);
}

// ============================================================================
// depth ingest on its own (integration with a depth map other than the last
// allocation's)
// ============================================================================
template <int FMT>
__global__ __launch_bounds__(256) void k_depth_convert(float *dst, const void *src, int n)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    if (FMT == TF_DEPTH_U16_MM)
        dst[p] = (float)reinterpret_cast<const uint16_t *>(src)[p] / 1000.0f;
    else
        dst[p] = reinterpret_cast<const float *>(src)[p];
}


// ============================================================================
// search range (Sec. 4.4): project blocks, bin them by 16x16 tile
// ============================================================================
constexpr int kExpandV = 3;   // voxels added around a block when binning it

// One lane per block: its record (search-range box and z range of the block
// itself, key, device pointer) goes to every tile its cube covers -- grown by
// kExpandV voxels when every block is binned, so that a tile's bin then holds
// every block any trilinear read of the tile's rays can touch.  The (record,
// tile) writes of a wave are spread evenly over its lanes.
__global__ __launch_bounds__(256) void k_range_bin(Vol v, Cam c, int all)
{
    __shared__ Rec wrec[4][kWave];
    __shared__ uint32_t wexcl[4][kWave + 1];
    __shared__ int16_t wrect[4][kWave][3];   // tx0, ty0, nx
    const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
    const uint32_t gwave = (blockIdx.x * 256u + threadIdx.x) / kWave;
    const uint32_t nwaves = gridDim.x * (256u / kWave);
    const uint32_t n = all ? v.n_entries : v.ctrl->n_vis;
    const int ntx = (c.W + kTile - 1) / kTile;
    for (uint32_t base = gwave * kWave; base < n; base += nwaves * kWave) {
        const uint32_t i = base + lane;
        bool emit = false;
        Rec r;
        Rec ex;
        if (i < n) {
            const uint32_t e = all ? i : (uint32_t)v.vlist[i];
            const int4 w = load_entry(v.entries, e);
            if (w.w >= 0) {
                const int bx = (int16_t)(w.x & 0xffff), by = (int16_t)((uint32_t)w.x >> 16), bz = (int16_t)(w.y & 0xffff);
                // bins of every block (foreign views) grow the cubes so that a
                // complete tile table answers every lookup of the tile's rays;
                // bins of the visible list cannot, so they use the plain cube
                const int g = all ? kExpandV : 0;
                emit = cube_record(c.M, c, v.voxel, 8 * bx - g, 8 * by - g, 8 * bz - g, 8 + 2 * g, ex);
                if (emit && !block_record(v, c, bx, by, bz, r)) {
                    // only the grown cube reaches the image: a table entry with no range
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
                r.pad = 0;
                r.ptr = w.w;
                r.pad2 = 0;
            }
        }
        const unsigned long long m = __ballot(emit);
        if (!m) continue;
        const int leader = __ffsll((long long)m) - 1;
        uint32_t rb = 0;
        if ((int)lane == leader) rb = atomicAdd(&v.ctrl->n_rec, (uint32_t)__popcll(m));
        rb = __shfl(rb, leader);
        uint32_t cnt = 0;
        if (emit) {
            v.recs[rb + rank_in(m)] = r;
            const int tx0 = ex.x0 / kTile, tx1 = ex.x1 / kTile, ty0 = ex.y0 / kTile, ty1 = ex.y1 / kTile;
            cnt = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
            wrec[wv][lane] = r;
            wrect[wv][lane][0] = (int16_t)tx0;
            wrect[wv][lane][1] = (int16_t)ty0;
            wrect[wv][lane][2] = (int16_t)(tx1 - tx0 + 1);
        }
        // lanes of one wave exchange through their own LDS slice: a wave-level fence suffices
        // exclusive scan of the lanes' tile counts
        uint32_t incl = cnt;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t t = __shfl_up(incl, d);
            if ((int)lane >= d) incl += t;
        }
        wexcl[wv][lane] = incl - cnt;
        const uint32_t total = __shfl(incl, kWave - 1);
        if (lane == 0) wexcl[wv][kWave] = total;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        for (uint32_t item = lane; item < total; item += kWave) {
            // owner lane: the last j with excl[j] <= item (lanes without tiles have empty ranges)
            int j = 0;
#pragma unroll
            for (int b = 32; b; b >>= 1)
                if (wexcl[wv][j + b] <= item) j += b;
            while (wexcl[wv][j + 1] <= item) ++j;
            const uint32_t li = item - wexcl[wv][j];
            const int nx = wrect[wv][j][2];
            const int t = (wrect[wv][j][1] + (int)(li / (uint32_t)nx)) * ntx + wrect[wv][j][0] + (int)(li % (uint32_t)nx);
            const int sl = atomicAdd(&v.bin_count[t], 1);
            if (sl < kBinCap) v.bins[(size_t)t * kBinCap + sl] = wrec[wv][j];
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// LDS of a raycast tile: the (block key -> device pointer) table of the bin's
// blocks and the bin's pixel boxes and z ranges (the first 16 bytes of each
// record) for the per-pixel range
struct TileTable {
    unsigned long long key[kTileTable];   // 0 = empty slot
    int ptr[kTileTable];
    uint4 box[kBinCap];                   // x0, y0, x1, y1 (int16), zlo, zhi (float)
    uint16_t wlist[4][kBinCap];           // per wave: the staged records whose box meets its pixels
    int wcnt[4];
    int complete;                         // the table holds the whole bin
};

// slot hash of the tile's private table: products of the 16-bit coordinates
// (callers have range-checked them) with 23-bit constants, which compile to
// full-rate 24-bit multiplies, folded to the table size
__device__ __forceinline__ uint32_t table_slot(int bx, int by, int bz)
{
    const int x = (int16_t)bx, y = (int16_t)by, z = (int16_t)bz;
    const uint32_t h = (uint32_t)(x * 0x1f1f1f) ^ (uint32_t)(y * 0x3c6ef3) ^ (uint32_t)(z * 0x5a8279);
    return (h ^ (h >> 10)) & (uint32_t)(kTileTable - 1);
}

// The tile's block table and the search range of pixel (px, py) from the
// tile's bin (all records, in chunks of kBinCap and without a table, if the
// bin overflowed).  The records are staged in LDS, each also listed for the
// waves whose pixels its box meets (wave w's pixels: the 8 x 8 quadrant w of
// the tile when `quads`, else rows 4 w .. 4 w + 3); every thread then takes
// the min / max over its wave's list whose box holds its pixel: the
// per-pixel loop itself, with no atomics, over the records that can matter.
// Every thread of the workgroup calls it; zmin = +inf and zmax = -inf when
// no record covers the pixel.
__device__ __forceinline__ void tile_range(const Vol &v, int tile, int tx0, int ty0, bool quads, int px, int py,
                                           TileTable *tt, bool table, float &zmin, float &zmax)
{
    for (int k = threadIdx.x; k < kTileTable; k += 256) tt->key[k] = 0ull;
    if (threadIdx.x < 4) tt->wcnt[threadIdx.x] = 0;
    const int wave = (int)threadIdx.x >> 6;
    const int cnt = v.bin_count[tile];
    const bool fallback = cnt > kBinCap;
    const int n = fallback ? (int)v.ctrl->n_rec : cnt;
    if (threadIdx.x == 0) tt->complete = table && !fallback;
    float lo = __builtin_inff(), hi = -__builtin_inff();
    for (int base = 0; base < n; base += kBinCap) {
        const int m = n - base < kBinCap ? n - base : kBinCap;
        __syncthreads();   // the cleared table, or the previous chunk consumed
        for (int j = (int)threadIdx.x; j < m; j += 256) {
            const Rec r = fallback ? v.recs[base + j] : v.bins[(size_t)tile * kBinCap + j];
            if (table && !fallback) {
                // keys in one bin are distinct; the table is at most half full
                const unsigned long long key = pack_key(r.bx, r.by, r.bz);
                uint32_t sl = table_slot(r.bx, r.by, r.bz);
                for (int k = 0; k < kTileTable; ++k) {
                    if (atomicCAS(&tt->key[sl], 0ull, key) == 0ull) {
                        tt->ptr[sl] = r.ptr;
                        break;
                    }
                    sl = (sl + 1u) & (uint32_t)(kTileTable - 1);
                }
            }
            tt->box[j] = make_uint4((uint32_t)(uint16_t)r.x0 | ((uint32_t)(uint16_t)r.y0 << 16),
                                    (uint32_t)(uint16_t)r.x1 | ((uint32_t)(uint16_t)r.y1 << 16),
                                    __float_as_uint(r.zlo), __float_as_uint(r.zhi));
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const int wx0 = tx0 + (quads ? (w & 1) * 8 : 0), wy0 = ty0 + (quads ? (w >> 1) * 8 : 4 * w);
                const int wx1 = wx0 + (quads ? 7 : 15), wy1 = wy0 + (quads ? 7 : 3);
                if (r.x0 <= wx1 && r.x1 >= wx0 && r.y0 <= wy1 && r.y1 >= wy0)
                    tt->wlist[w][atomicAdd(&tt->wcnt[w], 1)] = (uint16_t)j;
            }
        }
        __syncthreads();
        // the order of a wave's list varies with the atomics; min and max do not
        const int nw = __builtin_amdgcn_readfirstlane(tt->wcnt[wave]);
        for (int i = 0; i < nw; ++i) {
            const uint4 b = tt->box[tt->wlist[wave][i]];
            const int x0 = (int16_t)(b.x & 0xffffu), y0 = (int16_t)(b.x >> 16);
            const int x1 = (int16_t)(b.y & 0xffffu), y1 = (int16_t)(b.y >> 16);
            if (px >= x0 && px <= x1 && py >= y0 && py <= y1) {
                const float zl = __uint_as_float(b.z), zh = __uint_as_float(b.w);
                lo = zl < lo ? zl : lo;
                hi = zh > hi ? zh : hi;
            }
        }
        // this wave's list is consumed; the next chunk's staging starts after the barrier above
        if ((threadIdx.x & 63) == 0) tt->wcnt[wave] = 0;
    }
    __syncthreads();   // the table is complete before any lookup
    zmin = lo;
    zmax = hi;
}

// End of a raycast-kind workgroup (every thread calls it, after its last
// read of the tile's bin): clear the tile's bin counter; the last workgroup
// of the launch clears the record counter.  Taken at the end of the kernel,
// the tickets of the workgroups arrive spread out in time.  No fence: every
// workgroup has read the counter before its ticket, and the next launch sees
// the stores.
__device__ __forceinline__ void finish_tile(const Vol &v, int tile, bool count_raycast)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        if (tile >= 0) v.bin_count[tile] = 0;
        const uint32_t t = atomicAdd(&v.ctrl->ray_ticket, 1u);
        if (t == gridDim.x - 1u) {
            if (count_raycast) v.ctrl->tot_rec += v.ctrl->n_rec;
            v.ctrl->n_rec = 0u;
            v.ctrl->ray_ticket = 0u;
        }
    }
}

// ============================================================================
// raycast (Sec. 4.4)
// ============================================================================
namespace {


// one-entry block cache (the paper's IndexCache, Sec. 3.3): the last block
// key looked up and its device pointer (-1 = absent or not on the device);
// `local`: lookups of this ray may trust a miss in the tile's table
struct BlockCache {
    int bx, by, bz, ptr;
    bool local;
};

// device pointer of a block (-1 = absent or not on the device): the tile's
// LDS table first; unless `local`, then the occupancy bricks and the hash table.
// `local` holds for a ray whose points all lie at or beyond the near plane in
// a tile whose table holds its whole bin: every block within kExpandV voxels
// of such a point is in the bin, so a miss proves absence.
__device__ __forceinline__ int lookup_block(const Vol &v, const TileTable *tt, int bx, int by, int bz, bool local)
{
    if (!in_short_range(bx) || !in_short_range(by) || !in_short_range(bz)) return -1;
    const unsigned long long key = pack_key(bx, by, bz);
    uint32_t sl = table_slot(bx, by, bz);
    for (int k = 0; k < kTileTable; ++k) {
        const unsigned long long kk = tt->key[sl];
        if (kk == key) return tt->ptr[sl];
        if (kk == 0ull) break;
        sl = (sl + 1u) & (uint32_t)(kTileTable - 1);
    }
    if (local) return -1;
    // the block's occupancy brick and its bucket entry, loaded together; the
    // chain beyond the bucket only when the entry is another block's
    const uint32_t h = hash_index(bx, by, bz, v.n_buckets - 1u);
    const uint32_t bw = gload(v.brick + brick_word(bx, by, bz));
    const int4 w = load_entry(v.entries, h);
    if (!(bw & brick_bit(bx, by, bz))) return -1;
    const uint32_t kxy = (uint32_t)(uint16_t)bx | ((uint32_t)(uint16_t)by << 16);
    if ((uint32_t)w.x == kxy && (int16_t)(w.y & 0xffff) == (int16_t)bz && w.w >= 0) return w.w;
    if (w.z < 1 || (uint32_t)(w.z - 1) >= v.n_excess) return -1;
    int ptr = -1;
    const int e = find_entry_from(v.entries, v.n_buckets, v.n_excess, v.n_buckets + (uint32_t)(w.z - 1), bx, by, bz, 0,
                                  &ptr);
    return e >= 0 ? ptr : -1;
}

__device__ __forceinline__ int cached_block(const Vol &v, const TileTable *tt, int bx, int by, int bz,
                                            BlockCache &cc)
{
    if (bx == cc.bx && by == cc.by && bz == cc.bz) return cc.ptr;
    cc.bx = bx;
    cc.by = by;
    cc.bz = bz;
    cc.ptr = lookup_block(v, tt, bx, by, bz, cc.local);
    return cc.ptr;
}

// A trilinear cell ready to load: the corners' SDF addresses as byte offsets
// into the voxel array (32-bit when the array spans at most 4 GiB), which
// corners have a block, and the interpolation fractions.  An absent corner
// addresses block 0; its value is not used.
template <bool kOff32>
struct RayCell {
    typename std::conditional<kOff32, uint32_t, size_t>::type o[8];
    uint32_t present;
    float tx, ty, tz;
};

// corner blocks: the cell's own block through the ray's cache; where the
// cell crosses a block face (local index 7), the neighbouring blocks by
// direct lookups
template <bool kOff32>
__device__ __forceinline__ void cell_setup(const Vol &v, const TileTable *tt, float X, float Y, float Z,
                                           BlockCache &cc, RayCell<kOff32> &C)
{
    const float bx = floorf(X), by = floorf(Y), bz = floorf(Z);
    C.tx = X - bx;
    C.ty = Y - by;
    C.tz = Z - bz;
    const int ix = (int)bx, iy = (int)by, iz = (int)bz;
    const int Bx = ix >> 3, By = iy >> 3, Bz = iz >> 3;
    const bool sx = (ix & 7) == 7, sy = (iy & 7) == 7, sz = (iz & 7) == 7;
    int p[8];
    p[0] = cached_block(v, tt, Bx, By, Bz, cc);
#pragma unroll
    for (int c = 1; c < 8; ++c) p[c] = p[0];
    if (sx | sy | sz) {
        const bool lc = cc.local;
        if (sx) p[1] = lookup_block(v, tt, Bx + 1, By, Bz, lc);
        if (sy) p[2] = lookup_block(v, tt, Bx, By + 1, Bz, lc);
        if (sz) p[4] = lookup_block(v, tt, Bx, By, Bz + 1, lc);
        p[3] = (sx & sy) ? lookup_block(v, tt, Bx + 1, By + 1, Bz, lc) : (sx ? p[1] : p[2]);
        p[5] = (sx & sz) ? lookup_block(v, tt, Bx + 1, By, Bz + 1, lc) : (sx ? p[1] : p[4]);
        p[6] = (sy & sz) ? lookup_block(v, tt, Bx, By + 1, Bz + 1, lc) : (sy ? p[2] : p[4]);
        p[7] = (sx & sy & sz) ? lookup_block(v, tt, Bx + 1, By + 1, Bz + 1, lc)
                              : (sx & sy) ? p[3] : (sx & sz) ? p[5] : (sy & sz) ? p[6] : sx ? p[1] : sy ? p[2] : p[4];
    }
    int j[8];
    cell_index(ix, iy, iz, sx, sy, sz, j);
    C.present = 0u;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        C.present |= (p[c] >= 0 ? 1u : 0u) << c;
        const uint32_t pc = p[c] >= 0 ? (uint32_t)p[c] : 0u;
        if (kOff32)
            C.o[c] = __umul24(pc, (uint32_t)kBlockBytes) + 2u * (uint32_t)j[c];
        else
            C.o[c] = (size_t)pc * kBlockBytes + 2u * (uint32_t)j[c];
    }
}

template <bool kOff32>
__device__ __forceinline__ void cell_load(const Vol &v, const RayCell<kOff32> &C, int16_t (&s)[8])
{
#pragma unroll
    for (int c = 0; c < 8; ++c) s[c] = gload(reinterpret_cast<const int16_t *>(v.voxels + C.o[c]));
}

// trilinear interpolation of F at voxel-unit P (Sec. 4.4)
template <bool kOff32>
__device__ __forceinline__ float trilinear(const Vol &v, const TileTable *tt, float X, float Y, float Z,
                                           BlockCache &cc)
{
    RayCell<kOff32> C;
    int16_t s[8];
    cell_setup(v, tt, X, Y, Z, cc, C);
    cell_load(v, C, s);
    return cell_lerp(C.present, s, C.tx, C.ty, C.tz);
}

// F(A) - F(B) with the sixteen voxel loads of both cells issued together
template <bool kOff32>
__device__ __forceinline__ float trilinear_diff(const Vol &v, const TileTable *tt, float AX, float AY, float AZ,
                                                float BX, float BY, float BZ, BlockCache &cc)
{
    RayCell<kOff32> A, B;
    int16_t sa[8], sb[8];
    cell_setup(v, tt, AX, AY, AZ, cc, A);
    cell_setup(v, tt, BX, BY, BZ, cc, B);
    cell_load(v, A, sa);
    cell_load(v, B, sb);
    return cell_lerp(A.present, sa, A.tx, A.ty, A.tz) - cell_lerp(B.present, sb, B.tx, B.ty, B.tz);
}

// The normal's central differences (Sec. 4.4): g_a = (F(P + e_a) -
// F(P - e_a)) / 2 for the three axes.  The six trilinear cells are those of
// floor(P) -+ e_a; together they read 32 distinct voxels of the 4 x 4 x 4
// around floor(P), which spans at most two blocks per axis, so the block
// pointers are looked up once and the 32 loads issued together.  Each cell
// keeps the fractions of its own point P -+ e_a, as separate trilinear reads
// would.  Returns false (nothing computed) when rounding of P -+ 1 moves a
// cell off floor(P) -+ e_a.
template <bool kOff32>
__device__ __forceinline__ bool normal_gradient(const Vol &v, const TileTable *tt, float X, float Y, float Z,
                                                BlockCache &cc, float &gx, float &gy, float &gz)
{
    const float Xp = X + 1.0f, Xm = X - 1.0f, Yp = Y + 1.0f, Ym = Y - 1.0f, Zp = Z + 1.0f, Zm = Z - 1.0f;
    const float fX = floorf(X), fY = floorf(Y), fZ = floorf(Z);
    const float fXp = floorf(Xp), fXm = floorf(Xm), fYp = floorf(Yp), fYm = floorf(Ym), fZp = floorf(Zp),
                fZm = floorf(Zm);
    if (fXp != fX + 1.0f || fXm != fX - 1.0f || fYp != fY + 1.0f || fYm != fY - 1.0f || fZp != fZ + 1.0f ||
        fZm != fZ - 1.0f)
        return false;
    const int ix = (int)fX, iy = (int)fY, iz = (int)fZ;
    const int Bx = ix >> 3, By = iy >> 3, Bz = iz >> 3;
    // the second block the range i - 1 .. i + 2 reaches on each axis (0: none)
    const int ax = (ix & 7) == 0 ? -1 : ((ix & 7) >= 6 ? 1 : 0);
    const int ay = (iy & 7) == 0 ? -1 : ((iy & 7) >= 6 ? 1 : 0);
    const int az = (iz & 7) == 0 ? -1 : ((iz & 7) >= 6 ? 1 : 0);
    int pb[8];
    pb[0] = cached_block(v, tt, Bx, By, Bz, cc);
    const bool lc = cc.local;
#pragma unroll
    for (int c = 1; c < 8; ++c) {
        const int sx = c & 1, sy = (c >> 1) & 1, sz = c >> 2;
        pb[c] = ((sx && !ax) || (sy && !ay) || (sz && !az))
                    ? -1
                    : lookup_block(v, tt, Bx + (sx ? ax : 0), By + (sy ? ay : 0), Bz + (sz ? az : 0), lc);
    }
    // voxel (ix + dx, iy + dy, iz + dz): x-cells dx -1..2, dy 0..1, dz 0..1;
    // then the y-cells' dy = -1, 2 and the z-cells' dz = -1, 2 (dx, dy 0..1)
    constexpr int kN = 32;
    int16_t sv[kN];
    uint32_t present = 0u;
#pragma unroll
    for (int i = 0; i < kN; ++i) {
        int dx, dy, dz;
        if (i < 16) {
            dx = (i & 3) - 1;
            dy = (i >> 2) & 1;
            dz = i >> 3;
        } else if (i < 24) {
            dx = i & 1;
            dy = ((i >> 1) & 1) ? 2 : -1;
            dz = (i >> 2) & 1;
        } else {
            dx = i & 1;
            dy = (i >> 1) & 1;
            dz = ((i >> 2) & 1) ? 2 : -1;
        }
        const int x = ix + dx, y = iy + dy, z = iz + dz;
        // selects, not an indexed private array (which would live in scratch)
        const bool bx = (x >> 3) != Bx, by = (y >> 3) != By, bz = (z >> 3) != Bz;
        const int pc = bz ? (by ? (bx ? pb[7] : pb[6]) : (bx ? pb[5] : pb[4]))
                          : (by ? (bx ? pb[3] : pb[2]) : (bx ? pb[1] : pb[0]));
        present |= (pc >= 0 ? 1u : 0u) << i;
        const uint32_t pu = pc >= 0 ? (uint32_t)pc : 0u;
        const uint32_t j = (uint32_t)((z & 7) + 8 * (y & 7) + 64 * (x & 7));
        if (kOff32)
            sv[i] = gload(reinterpret_cast<const int16_t *>(v.voxels + (__umul24(pu, (uint32_t)kBlockBytes) + 2u * j)));
        else
            sv[i] = gload(reinterpret_cast<const int16_t *>(v.voxels + ((size_t)pu * kBlockBytes + 2u * j)));
    }
    // a cell from 8 of the loaded voxels, corner c at (c & 1, c >> 1 & 1, c >> 2)
    auto cell = [&](const int (&idx)[8], float tx, float ty, float tz) {
        int16_t s8[8];
        uint32_t pr = 0u;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            s8[c] = sv[idx[c]];
            pr |= ((present >> idx[c]) & 1u) << c;
        }
        return cell_lerp(pr, s8, tx, ty, tz);
    };
    const float tx = X - fX, ty = Y - fY, tz = Z - fZ;
    // x-cells: index (dx + 1) + 4 dy + 8 dz
    const int xp[8] = {2, 3, 6, 7, 10, 11, 14, 15}, xm[8] = {0, 1, 4, 5, 8, 9, 12, 13};
    gx = (cell(xp, Xp - fXp, ty, tz) - cell(xm, Xm - fXm, ty, tz)) * 0.5f;
    // y-cells: dy 0 / 1 from the x-cells (dx 0 / 1: indices 1, 2 + 4 dy + 8 dz),
    // dy -1 / 2 at 16 + dx + 2 (dy == 2) + 4 dz
    const int yp[8] = {5, 6, 18, 19, 13, 14, 22, 23}, ym[8] = {16, 17, 1, 2, 20, 21, 9, 10};
    gy = (cell(yp, tx, Yp - fYp, tz) - cell(ym, tx, Ym - fYm, tz)) * 0.5f;
    // z-cells: dz 0 / 1 from the x-cells, dz -1 / 2 at 24 + dx + 2 dy + 4 (dz == 2)
    const int zp[8] = {9, 10, 13, 14, 28, 29, 30, 31}, zm[8] = {24, 25, 26, 27, 1, 2, 5, 6};
    gz = (cell(zp, tx, ty, Zp - fZp) - cell(zm, tx, ty, Zm - fZm)) * 0.5f;
    return true;
}

// "allocated" test of the march: the block of floor(P) has a device block
__device__ __forceinline__ bool allocated_at(const Vol &v, const TileTable *tt, float P0, float P1, float P2,
                                             BlockCache &cc)
{
    return cached_block(v, tt, block_of(P0), block_of(P1), block_of(P2), cc) >= 0;
}

enum { SEARCH_BLOCK_COARSE, SEARCH_BLOCK_FINE, SEARCH_SURFACE, BEHIND_SURFACE, WRONG_SIDE };

}  // namespace

// search range on its own, written as an image (tf_range_image)
__global__ __launch_bounds__(256) void k_range_write(Vol v, Cam c, float *zmin_out, float *zmax_out)
{
    __shared__ TileTable tbl;
    const int ntx = (c.W + kTile - 1) / kTile;
    const int tile = blockIdx.x;
    const int tx0 = (tile % ntx) * kTile, ty0 = (tile / ntx) * kTile;
    const int px = tx0 + (int)(threadIdx.x % kTile);
    const int py = ty0 + (int)(threadIdx.x / kTile);
    float zmin, zmax;
    tile_range(v, tile, tx0, ty0, false, px, py, &tbl, false, zmin, zmax);
    finish_tile(v, tile, false);
    if (px >= c.W || py >= c.H) return;
    zmin_out[(size_t)py * c.W + px] = zmin;
    zmax_out[(size_t)py * c.W + px] = zmax;
}

// ============================================================================
// raycast, one workgroup per 16x16 tile (Sec. 4.4): the tile's search range
// from its bin (LDS), the state machine per pixel, then the two refinement
// steps and the normal for the hits of the wave together
// ============================================================================
template <bool kOff32>
__global__ __launch_bounds__(256) void k_raycast(Vol v, Cam c, int all_blocks, float4 *pts, float4 *nrm)
{
    __shared__ TileTable tbl;
    const int ntx = (c.W + kTile - 1) / kTile, nty = (c.H + kTile - 1) / kTile;
    const int ntiles = ntx * nty;
    // workgroups go round-robin to the 8 XCDs; tiles in launch order, so that
    // the slow tiles of a region (long rays) spread over all XCDs (a band of
    // the image per XCD, for L2 locality, measured 2% slower)
    const int tile = (int)blockIdx.x;
    const bool real = tile < ntiles;
    const int q = (int)threadIdx.x >> 6, i = (int)threadIdx.x & 63;
    const int lx = (q & 1) * 8 + (i & 7), ly = (q >> 1) * 8 + (i >> 3);
    const int tx0 = real ? (tile % ntx) * kTile : 0, ty0 = real ? (tile / ntx) * kTile : 0;
    const int px = tx0 + lx, py = ty0 + ly;
    float zmin = __builtin_inff(), zmax = -__builtin_inff();
    if (real) tile_range(v, tile, tx0, ty0, true, px, py, &tbl, true, zmin, zmax);
    const bool inside = real && px < c.W && py < c.H;
    float4 out_p = make_float4(0.f, 0.f, 0.f, 0.f), out_n = make_float4(0.f, 0.f, 0.f, 0.f);
    if (inside && zmin <= zmax) {
        const float vs = v.voxel;
        const float inv_vs = 1.0f / vs;
        const float mu_v = v.mu * inv_vs;
        const float ox = c.ti[0] * inv_vs, oy = c.ti[1] * inv_vs, oz = c.ti[2] * inv_vs;
        const float a = ((float)px - c.cx) / c.fx;
        const float b = ((float)py - c.cy) / c.fy;
        const float nr = sqrtf((a * a + b * b) + 1.0f);
        const float rcx = a / nr, rcy = b / nr, rcz = 1.0f / nr;
        const float dx = (c.Ri[0] * rcx + c.Ri[1] * rcy) + c.Ri[2] * rcz;
        const float dy = (c.Ri[3] * rcx + c.Ri[4] * rcy) + c.Ri[5] * rcz;
        const float dz = (c.Ri[6] * rcx + c.Ri[7] * rcy) + c.Ri[8] * rcz;
        float t = (zmin * nr) * inv_vs;
        const float t_end = (zmax * nr) * inv_vs;
        int state = SEARCH_BLOCK_COARSE;
        float F = 1.0f;
        // with bins of every allocated block, and every point of this ray
        // (march from t - 8, two refinement steps of at most mu back) at or
        // beyond the near plane, a table miss proves absence.  Bins of the
        // visible list alone do not: trilinear reads may reach allocated
        // blocks outside it.
        const float zscale = vs * rcz;
        const bool local = all_blocks && tbl.complete && (t - 8.0f - 2.0f * mu_v) * zscale >= kZNear;
        BlockCache cc = {0x7fffffff, 0, 0, -1, local};
        int steps = 0;
        while (t < t_end && steps < kMaxRaySteps) {
            if (state == SEARCH_BLOCK_COARSE || state == SEARCH_BLOCK_FINE) {
                // Empty-space skip: the march stays in this state with a fixed
                // step while it finds no block.  Test the occupancy bricks of the next
                // kSkip positions together; a clear bit proves the block absent,
                // so those iterations are exactly the ones the loop would run.
                const float stp = state == SEARCH_BLOCK_COARSE ? 8.0f : mu_v;
                constexpr int kSkip = 4;
                float tk[kSkip];
                uint32_t hk[kSkip], wk[kSkip];
                float tt = t;
#pragma unroll
                for (int k = 0; k < kSkip; ++k) {
                    tk[k] = tt;
                    const int b0 = block_of(ox + tt * dx), b1 = block_of(oy + tt * dy), b2 = block_of(oz + tt * dz);
                    hk[k] = brick_bit(b0, b1, b2);
                    wk[k] = gload(v.brick + brick_word(b0, b1, b2));
                    tt += stp;
                }
                bool stop = false;
#pragma unroll
                for (int k = 0; k < kSkip; ++k) {
                    if (stop) continue;
                    t = tk[k];
                    if (!(t < t_end && steps < kMaxRaySteps) || (wk[k] & hk[k])) {
                        stop = true;
                        continue;
                    }
                    ++steps;                       // an iteration on unallocated space
                }
                if (!stop) t = tt;
                if (!(t < t_end && steps < kMaxRaySteps)) break;
            }
            ++steps;
            const float P0 = ox + t * dx, P1 = oy + t * dy, P2 = oz + t * dz;
            const bool alloc = allocated_at(v, &tbl, P0, P1, P2, cc);
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
                F = trilinear<kOff32>(v, &tbl, P0, P1, P2, cc);
                if (state == SEARCH_SURFACE) {
                    if (F < 0.0f) {
                        state = BEHIND_SURFACE;
                        break;
                    }
                    const float s = F * mu_v;
                    t += (s > 1.0f) ? s : 1.0f;
                } else if (F < 0.0f) {
                    if (state == SEARCH_BLOCK_FINE) {
                        state = WRONG_SIDE;
                    } else {
                        const float s = -F * mu_v;
                        t += (s > 1.0f) ? s : 1.0f;
                    }
                } else {
                    // FINE or WRONG_SIDE meeting F >= 0 turns to SURFACE without
                    // a step; the SURFACE iteration that follows (if the step
                    // bound allows it) reads the same cell at the same t, so
                    // its step is taken here with this F
                    state = SEARCH_SURFACE;
                    if (steps < kMaxRaySteps) {
                        ++steps;
                        const float s = F * mu_v;
                        t += (s > 1.0f) ? s : 1.0f;
                    }
                }
            }
        }
        if (state == BEHIND_SURFACE) {
            t += F * mu_v;
            float P0 = ox + t * dx, P1 = oy + t * dy, P2 = oz + t * dz;
            F = trilinear<kOff32>(v, &tbl, P0, P1, P2, cc);
            t += F * mu_v;
            P0 = ox + t * dx;
            P1 = oy + t * dy;
            P2 = oz + t * dz;
            out_p = make_float4(P0 * vs, P1 * vs, P2 * vs, 1.0f);
            float gx = 0.0f, gy = 0.0f, gz = 0.0f;
            // the rare rays whose shifted points round across a voxel take the
            // cells one axis per iteration
#pragma unroll 1
            for (int ax = normal_gradient<kOff32>(v, &tbl, P0, P1, P2, cc, gx, gy, gz) ? 3 : 0; ax < 3; ++ax) {
                const float d = trilinear_diff<kOff32>(v, &tbl, ax == 0 ? P0 + 1.0f : P0, ax == 1 ? P1 + 1.0f : P1,
                                                       ax == 2 ? P2 + 1.0f : P2, ax == 0 ? P0 - 1.0f : P0,
                                                       ax == 1 ? P1 - 1.0f : P1, ax == 2 ? P2 - 1.0f : P2, cc) *
                                0.5f;
                gx = ax == 0 ? d : gx;
                gy = ax == 1 ? d : gy;
                gz = ax == 2 ? d : gz;
            }
            const float gn = sqrtf((gx * gx + gy * gy) + gz * gz);
            if (gn > 0.0f) out_n = make_float4(gx / gn, gy / gn, gz / gn, 1.0f);
        }
    }
    __shared__ uint32_t wg_hits;
    if (threadIdx.x == 0) wg_hits = 0;
    __syncthreads();
    if (inside) {
        const size_t p = (size_t)py * c.W + px;
        pts[p] = out_p;
        nrm[p] = out_n;
        if (out_p.w == 1.0f) atomicAdd(&wg_hits, 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0 && wg_hits) v.acc_hits[tile] += wg_hits;
    finish_tile(v, real ? tile : -1, true);
}

// ============================================================================
// host swapping (Sec. 5)
// ============================================================================
// secondary integration of two copies of one block, per voxel: the weighted
// average (w_a F_a + w_b F_b) / (w_a + w_b), weight min(w_a + w_b, maxW); a
// copy with weight 0 carries no observation.  Result into copy a.
__device__ __forceinline__ void merge_voxel(int &sa, int &wa, int sb, int wb, int max_w)
{
    if (wb == 0) return;
    if (wa == 0) {
        sa = sb;
        wa = wb;
        return;
    }
    const float fa = (float)sa * (1.0f / 32767.0f);
    const float fb = (float)sb * (1.0f / 32767.0f);
    const float avg = ((float)wa * fa + (float)wb * fb) / (float)(wa + wb);
    int w = wa + wb;
    if (w > max_w) w = max_w;
    sa = (int16_t)(avg * 32767.0f);
    wa = w;
}

// visible entries whose host store holds data: swap-in candidates
__global__ __launch_bounds__(256) void k_swap_candidates(Vol v)
{
    const uint32_t n = v.ctrl->n_vis;
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) {
        const int e = v.vlist[i];
        if (v.host_has[e]) {
            const uint32_t k = atomicAdd(&v.ctrl->n_swap_cand, 1u);
            v.ret[k] = e;
        }
    }
}

// fuse the transferred host blocks into their device blocks; one wave per block
__global__ __launch_bounds__(256) void k_swap_merge(Vol v, uint32_t n)
{
    const uint32_t lane = lane_id();
    const uint32_t gwave = (blockIdx.x * 256u + threadIdx.x) / kWave;
    const uint32_t nwaves = gridDim.x * (256u / kWave);
    if (blockIdx.x == 0 && threadIdx.x == 0) v.ctrl->n_swapped_in = n;
    for (uint32_t k = gwave; k < n; k += nwaves) {
        const int e = v.xfer_idx[k];
        const int ptr = load_entry(v.entries, (uint32_t)e).w;
        uint8_t *dst = v.voxels + (size_t)ptr * kBlockBytes;
        const uint8_t *src = v.xfer_vox + (size_t)k * kBlockBytes;
        const int16_t *ss = reinterpret_cast<const int16_t *>(src);
        int16_t *ds = reinterpret_cast<int16_t *>(dst);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int j = (int)lane * 8 + q;
            int sa = ds[j], wa = dst[1024 + j];
            merge_voxel(sa, wa, ss[j], src[1024 + j], v.max_w);
            ds[j] = (int16_t)sa;
            dst[1024 + j] = (uint8_t)wa;
        }
        if (lane == 0) v.host_has[e] = 0;
    }
}

// Swap-out of blocks whose host copy never came back in (Sec. 5, secondary
// integration): the store copies of those entries, uploaded to xfer_host,
// are fused with the device copies the gather put into the transfer buffer
// (slot xfer_pend[k]); the result replaces the store copy.  One wave per block.
__global__ __launch_bounds__(256) void k_swap_merge_out(Vol v, uint32_t n)
{
    const uint32_t lane = lane_id();
    const uint32_t gwave = (blockIdx.x * 256u + threadIdx.x) / kWave;
    const uint32_t nwaves = gridDim.x * (256u / kWave);
    for (uint32_t k = gwave; k < n; k += nwaves) {
        uint8_t *a = v.xfer_host + (size_t)k * kBlockBytes;
        const uint8_t *b = v.xfer_vox + (size_t)v.xfer_pend[k] * kBlockBytes;
        int16_t *as = reinterpret_cast<int16_t *>(a);
        const int16_t *bs = reinterpret_cast<const int16_t *>(b);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int j = (int)lane * 8 + q;
            int sa = as[j], wa = a[1024 + j];
            merge_voxel(sa, wa, bs[j], b[1024 + j], v.max_w);
            as[j] = (int16_t)sa;
            a[1024 + j] = (uint8_t)wa;
        }
    }
}

// marks the visible entries (val = 1) or clears the marks (val = 0)
__global__ __launch_bounds__(256) void k_mark_visible(Vol v, uint8_t val)
{
    const uint32_t n = v.ctrl->n_vis;
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) v.vis[v.vlist[i]] = val;
}

// swap-out candidates: a device block and not visible.  Ordered selection of
// the lowest entry indices: per-chunk counts, a scan, then in-order writes.
// A bucket whose occupancy bit is clear never held an entry: no read.
__device__ __forceinline__ bool swap_out_candidate(const Vol &v, uint32_t e)
{
    if (e >= v.n_entries || v.vis[e] != 0) return false;
    if (e < v.n_buckets && !((v.occ[e >> 5] >> (e & 31u)) & 1u)) return false;
    return load_entry(v.entries, e).w >= 0;
}

__device__ __forceinline__ uint32_t wg_exclusive_scan(uint32_t x, uint32_t *lds, uint32_t &total)
{
    const uint32_t lane = lane_id(), w = threadIdx.x / kWave;
    uint32_t incl = x;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t t = __shfl_up(incl, d);
        if ((int)lane >= d) incl += t;
    }
    if (lane == kWave - 1) lds[w] = incl;
    __syncthreads();
    uint32_t base = 0;
    for (uint32_t k = 0; k < w; ++k) base += lds[k];
    total = lds[0] + lds[1] + lds[2] + lds[3];
    __syncthreads();
    return base + incl - x;
}

// a chunk is 16 slices of 256 consecutive entries, one entry per thread in a
// slice (coalesced reads)
__global__ __launch_bounds__(256) void k_swap_count(Vol v)
{
    __shared__ uint32_t lds[4];
    const uint32_t e0 = blockIdx.x * (uint32_t)kSwapChunk + threadIdx.x;
    uint32_t cnt = 0;
    for (int k = 0; k < 16; ++k) cnt += swap_out_candidate(v, e0 + 256u * (uint32_t)k) ? 1u : 0u;
    uint32_t total;
    wg_exclusive_scan(cnt, lds, total);
    if (threadIdx.x == 0) v.swap_chunks[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void k_swap_scan(Vol v, uint32_t nchunks)
{
    __shared__ uint32_t lds[4];
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nchunks; base += 256u) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t x = i < nchunks ? v.swap_chunks[i] : 0u;
        uint32_t total;
        const uint32_t ex = wg_exclusive_scan(x, lds, total);
        if (i < nchunks) v.swap_chunks[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) v.ctrl->n_swap_cand = carry;
}

// in entry order: slice by slice, a workgroup scan of the candidate flags
__global__ __launch_bounds__(256) void k_swap_pick(Vol v)
{
    __shared__ uint32_t lds[4];
    uint32_t base = v.swap_chunks[blockIdx.x];
    if (base >= v.transfer_blocks) return;   // uniform: every pick of this chunk is past the capacity
    const uint32_t e0 = blockIdx.x * (uint32_t)kSwapChunk + threadIdx.x;
    for (int k = 0; k < 16; ++k) {
        const uint32_t e = e0 + 256u * (uint32_t)k;
        const bool c = swap_out_candidate(v, e);
        uint32_t total;
        const uint32_t pos = base + wg_exclusive_scan(c ? 1u : 0u, lds, total);
        if (c && pos < v.transfer_blocks) v.xfer_idx[pos] = (int32_t)e;
        base += total;
    }
}

// device blocks of the selected entries into the transfer buffer; one wave per block
__global__ __launch_bounds__(256) void k_swap_gather(Vol v, uint32_t n)
{
    const uint32_t lane = lane_id();
    const uint32_t gwave = (blockIdx.x * 256u + threadIdx.x) / kWave;
    const uint32_t nwaves = gridDim.x * (256u / kWave);
    for (uint32_t k = gwave; k < n; k += nwaves) {
        const int ptr = load_entry(v.entries, (uint32_t)v.xfer_idx[k]).w;
        const uint8_t *src = v.voxels + (size_t)ptr * kBlockBytes;
        uint8_t *dst = v.xfer_vox + (size_t)k * kBlockBytes;
        reinterpret_cast<uint4 *>(dst)[lane] = reinterpret_cast<const uint4 *>(src)[lane];
        reinterpret_cast<uint2 *>(dst + 1024)[lane] = reinterpret_cast<const uint2 *>(src + 1024)[lane];
    }
}

// return the blocks to the free stack and mark the entries swapped out (one workgroup)
__global__ __launch_bounds__(256) void k_swap_release(Vol v, uint32_t n)
{
    const int32_t head = v.ctrl->free_blocks;
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < n; k += 256u) {
        const int e = v.xfer_idx[k];
        v.free_blocks[head + (int32_t)k] = v.entries[e].ptr;
        v.entries[e].ptr = kPtrSwapped;
        v.host_has[e] = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        v.ctrl->free_blocks = head + (int32_t)n;
        v.ctrl->n_swapped_out = n;
    }
}

// ============================================================================
// export of voxels in the in-block order lx + 8 ly + 64 lz
// ============================================================================
__global__ __launch_bounds__(256) void k_export_voxels(Vol v, const int32_t *ids, uint32_t n, int16_t *sdf, uint8_t *wt)
{
    const uint32_t lane = lane_id();
    const uint32_t gwave = (blockIdx.x * 256u + threadIdx.x) / kWave;
    const uint32_t nwaves = gridDim.x * (256u / kWave);
    const int lx = (int)(lane >> 3), ly = (int)(lane & 7);
    for (uint32_t k = gwave; k < n; k += nwaves) {
        const int e = ids[k];
        int ptr = -1;
        if (e >= 0 && (uint32_t)e < v.n_entries) ptr = load_entry(v.entries, (uint32_t)e).w;
        for (int lz = 0; lz < 8; ++lz) {
            int16_t s = 32767;
            uint8_t w = 0;
            if (ptr >= 0) {
                const uint8_t *blk = v.voxels + (size_t)ptr * kBlockBytes;
                s = reinterpret_cast<const int16_t *>(blk)[lane * 8 + lz];
                w = blk[1024 + lane * 8 + lz];
            }
            const size_t o = (size_t)k * kBlockVox + lx + 8 * ly + 64 * lz;
            sdf[o] = s;
            wt[o] = w;
        }
    }
}

// ============================================================================
// camera depth of raycast hits (training targets of the prefilter)
// ============================================================================
struct Row3 {
    float m8, m9, m10, m11;
};

__global__ __launch_bounds__(256) void k_camera_depth(const float4 *pts, int n, Row3 r, float *depth)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    const float4 q = pts[p];
    depth[p] = q.w == 1.0f ? ((r.m8 * q.x + r.m9 * q.y) + r.m10 * q.z) + r.m11 : 0.0f;
}

// ============================================================================
// launchers
// ============================================================================
static int cu_grid(size_t work, int per_block, int cap)
{
    size_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > (size_t)cap) g = cap;
    return (int)g;
}

hipError_t launch_init(const Vol &v, hipStream_t s)
{
    size_t work = v.n_entries;
    if (v.n_blocks > work) work = v.n_blocks;
    if ((size_t)v.reqset_mask + 1 > work) work = (size_t)v.reqset_mask + 1;
    hipLaunchKernelGGL(k_init, dim3(cu_grid(work, 256, 8192)), dim3(256), 0, s, v);
    return hipGetLastError();
}

hipError_t launch_clear_bins(int32_t *bin_count, uint32_t n, hipStream_t s, Ctrl *ctrl)
{
    hipLaunchKernelGGL(k_clear_bins, dim3(cu_grid(n, 256, 1024)), dim3(256), 0, s, bin_count, n, ctrl);
    return hipGetLastError();
}

hipError_t launch_alloc_rays(const Vol &v, const Cam &c, const void *depth, int fmt, hipStream_t s)
{
    const int npix = c.W * c.H;
    const dim3 g((npix + 255) / 256 + kKeepGroups), b(256);
    if (fmt == TF_DEPTH_U16_MM)
        hipLaunchKernelGGL(k_alloc_rays<TF_DEPTH_U16_MM>, g, b, 0, s, v, c, depth);
    else
        hipLaunchKernelGGL(k_alloc_rays<TF_DEPTH_F32_M>, g, b, 0, s, v, c, depth);
    return hipGetLastError();
}

hipError_t launch_insert(const Vol &v, const Cam &c, hipStream_t s)
{
    hipLaunchKernelGGL(k_insert, dim3(512), dim3(256), 0, s, v, c);
    return hipGetLastError();
}

hipError_t launch_visible(const Vol &v, hipStream_t s)
{
    const size_t nchunks = ((size_t)v.n_entries + 15) / 16;
    hipLaunchKernelGGL(k_visible, dim3(cu_grid(nchunks, 256, 4096)), dim3(256), 0, s, v);
    return hipGetLastError();
}

hipError_t launch_depth_convert(const Vol &v, const void *depth, int fmt, int n, hipStream_t s)
{
    const dim3 g((n + 255) / 256), b(256);
    if (fmt == TF_DEPTH_U16_MM)
        hipLaunchKernelGGL(k_depth_convert<TF_DEPTH_U16_MM>, g, b, 0, s, v.depth, depth, n);
    else
        hipLaunchKernelGGL(k_depth_convert<TF_DEPTH_F32_M>, g, b, 0, s, v.depth, depth, n);
    return hipGetLastError();
}

hipError_t launch_integrate(const Vol &v, const Cam &c, bool bin, hipStream_t s)
{
    hipLaunchKernelGGL(k_integrate, dim3(kIntegrateGrid), dim3(256), 0, s, v, c, bin ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_range_bin(const Vol &v, const Cam &c, bool all_blocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_range_bin, dim3(1024), dim3(256), 0, s, v, c, all_blocks ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_raycast(const Vol &v, const Cam &c, bool all_blocks, float4 *pts, float4 *nrm, hipStream_t s)
{
    const int grid = ((c.W + kTile - 1) / kTile) * ((c.H + kTile - 1) / kTile);   // one workgroup per tile
    if ((size_t)v.n_blocks * kBlockBytes <= 0xffffffffu)
        hipLaunchKernelGGL(k_raycast<true>, dim3(grid), dim3(256), 0, s, v, c, all_blocks ? 1 : 0, pts, nrm);
    else
        hipLaunchKernelGGL(k_raycast<false>, dim3(grid), dim3(256), 0, s, v, c, all_blocks ? 1 : 0, pts, nrm);
    return hipGetLastError();
}

hipError_t launch_range_write(const Vol &v, const Cam &c, float *zmin, float *zmax, hipStream_t s)
{
    const int ntiles = ((c.W + kTile - 1) / kTile) * ((c.H + kTile - 1) / kTile);
    hipLaunchKernelGGL(k_range_write, dim3(ntiles), dim3(256), 0, s, v, c, zmin, zmax);
    return hipGetLastError();
}

hipError_t launch_camera_depth(const float4 *pts, int n, const float *M, float *depth, hipStream_t s)
{
    const Row3 r = {M[8], M[9], M[10], M[11]};
    hipLaunchKernelGGL(k_camera_depth, dim3((n + 255) / 256), dim3(256), 0, s, pts, n, r, depth);
    return hipGetLastError();
}

hipError_t launch_export_voxels(const Vol &v, const int32_t *ids, uint32_t n, int16_t *sdf, uint8_t *w, hipStream_t s)
{
    hipLaunchKernelGGL(k_export_voxels, dim3(cu_grid((size_t)n * 64, 256, 4096)), dim3(256), 0, s, v, ids, n, sdf, w);
    return hipGetLastError();
}

}  // namespace tsdf

namespace tsdf {
hipError_t launch_swap_candidates(const Vol &v, hipStream_t s)
{
    hipLaunchKernelGGL(k_swap_candidates, dim3(256), dim3(256), 0, s, v);
    return hipGetLastError();
}

hipError_t launch_swap_merge(const Vol &v, uint32_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_swap_merge, dim3(cu_grid((size_t)n * 64, 256, 2048)), dim3(256), 0, s, v, n);
    return hipGetLastError();
}

hipError_t launch_swap_select(const Vol &v, hipStream_t s)
{
    const uint32_t nchunks = (v.n_entries + kSwapChunk - 1) / kSwapChunk;
    hipLaunchKernelGGL(k_mark_visible, dim3(256), dim3(256), 0, s, v, (uint8_t)1);
    hipLaunchKernelGGL(k_swap_count, dim3(nchunks), dim3(256), 0, s, v);
    hipLaunchKernelGGL(k_swap_scan, dim3(1), dim3(256), 0, s, v, nchunks);
    hipLaunchKernelGGL(k_swap_pick, dim3(nchunks), dim3(256), 0, s, v);
    hipLaunchKernelGGL(k_mark_visible, dim3(256), dim3(256), 0, s, v, (uint8_t)0);
    return hipGetLastError();
}

hipError_t launch_swap_gather(const Vol &v, uint32_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_swap_gather, dim3(cu_grid((size_t)n * 64, 256, 2048)), dim3(256), 0, s, v, n);
    return hipGetLastError();
}

hipError_t launch_swap_merge_out(const Vol &v, uint32_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_swap_merge_out, dim3(cu_grid((size_t)n * 64, 256, 2048)), dim3(256), 0, s, v, n);
    return hipGetLastError();
}

hipError_t launch_swap_release(const Vol &v, uint32_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_swap_release, dim3(1), dim3(256), 0, s, v, n);
    return hipGetLastError();
}
}  // namespace tsdf
