// tsdf_internal.h -- device-side data layout and kernel launchers of libtsdf.
// Internal to the library (not installed, not shared with anything else).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace tsdf {

constexpr int kBlockVox = 512;          // 8x8x8 voxels per block (Sec. 3.1)
constexpr int kBlockBytes = 1536;       // 512 x int16 SDF, then 512 x uint8 weight
constexpr int kTile = 16;               // raycast tile = the paper's 16x16 fragments (Sec. 4.4)
constexpr int kBinCap = 512;            // block records per tile before the all-records fallback
constexpr int kTileTable = 1024;        // LDS block-pointer table slots per raycast tile (> 2 kBinCap)
constexpr int32_t kPtrSwapped = -1;     // Sec. 3.2: ptr == -1 swapped out
constexpr int32_t kPtrEmpty = -2;       // Sec. 3.2: ptr < -1 unallocated
constexpr int32_t kPtrClaimed = -3;     // bucket claimed inside k_insert, block pointer pending
constexpr float kZNear = 0.05f;         // near plane of the search-range projection
constexpr int kMaxRaySteps = 65536;     // hard bound on raycast iterations
constexpr int kMaxSegmentSamples = 64;  // samples kept per pixel segment
constexpr int kIntegrateGrid = 2048;    // workgroups of the integration launch
constexpr uint32_t kBrickWords = 1u << 19;   // block-occupancy bricks: 2 MiB per volume
constexpr uint32_t kWorldCells = 1u << 25;   // submap masks of world cells (512 x 512 x 128 window): 256 MiB per batched map
constexpr int kKeepGroups = 64;         // allocation workgroups past the image: the previous list's frustum test

// vis[] byte per hash entry, reset by the visible-list compaction
constexpr uint8_t kVisTouched = 1;      // touched by a ray segment or kept in view
constexpr uint8_t kVisNew = 3;          // inserted this frame

// hash entry (Sec. 3.2), 16 bytes so that one dwordx4 load fetches it
struct alignas(16) DEntry {
    int16_t x, y, z, pad;
    int32_t offset;   // 0 ends the chain; k >= 1 -> entry n_buckets + k - 1
    int32_t ptr;      // >= 0 block, -1 swapped out, < -1 unallocated
};
static_assert(sizeof(DEntry) == 16, "entry layout");

struct alignas(16) Req {
    unsigned long long key;   // packed block position, see pack_key
    uint32_t slot;            // request-set slot to clear after insertion
    uint32_t pad;
};

// axis-aligned pixel box of a projected block, its camera-z range, and the
// block's key and device pointer (staged in LDS by the raycast)
struct alignas(16) Rec {
    int16_t x0, y0, x1, y1;
    float zlo, zhi;
    int16_t bx, by, bz, pad;
    int32_t ptr, pad2;
};
static_assert(sizeof(Rec) == 32, "record layout");

// device counters; one per volume
struct alignas(256) Ctrl {
    int32_t free_blocks;     // height of the free-block stack
    int32_t free_excess;     // height of the free excess-slot stack
    uint32_t n_req;          // unique insertion requests of the current frame
    uint32_t n_vis;          // visible-list length
    uint32_t n_ret;          // blocks to return to the free stack
    uint32_t flags;          // sticky TF_FLAG_*
    uint32_t n_rec;          // search-range records of the current raycast
    uint32_t ray_ticket;     // last-workgroup detection in the raycast kernels
    uint32_t n_new;          // blocks inserted by the last frame
    uint32_t n_swapped_in;
    uint32_t n_swapped_out;
    uint32_t frames;
    uint32_t req_overflow;   // request list overflowed this frame: sweep the request set
    uint32_t n_swap_cand;    // swap-out candidates gathered by the last swap selection
    uint32_t sweep_req;      // copy of req_overflow taken by k_insert for k_visible
    uint32_t n_alloc;        // submap volumes: length of the allocated-block list
    uint32_t n_marked;       // submap volumes: list entries already marked in the world occupancy
    // totals since creation (each written by a single thread of one kernel)
    unsigned long long tot_vis;        // blocks visited by integration
    unsigned long long tot_rec;        // projected blocks behind raycast search ranges
    unsigned long long tot_req;        // insertion requests
    unsigned long long tot_new;        // blocks inserted
    unsigned long long n_integrate;    // integration launches
    unsigned long long n_raycast;      // raycast launches
};

// device view of one volume (by value into every kernel)
struct Vol {
    DEntry *entries;
    uint8_t *vis;
    int32_t *free_blocks;
    int32_t *free_excess;
    uint8_t *voxels;                // n_blocks x kBlockBytes
    int32_t *vlist;
    unsigned long long *reqset;     // open-addressing set of requested keys
    Req *reqs;
    int32_t *ret;
    float *depth;                   // metres, last ingested frame
    Rec *recs;
    Rec *bins;                      // per tile: the records of the blocks overlapping it
    int32_t *bin_count;
    Ctrl *ctrl;
    unsigned long long *acc_cols;   // per integration workgroup: 8-voxel columns written back
    unsigned long long *acc_hits;   // per raycast tile: pixels with a hit
    uint32_t *occ;                  // bucket-occupancy bitmap: bit h set once any entry hashes to h
    uint32_t *brick;                // block-occupancy bricks (kBrickWords words), see brick_word
    uint8_t *host_has;              // swapping: 1 if the host store holds data for the entry
    int32_t *xfer_idx;              // swapping: transfer-buffer entry indices
    uint8_t *xfer_vox;              // swapping: transfer-buffer blocks
    uint8_t *xfer_host;             // swapping: host-store copies fused into swap-out blocks
    int32_t *xfer_pend;             // swapping: transfer-buffer slot of each such copy
    uint32_t *swap_chunks;          // swapping: per-chunk candidate counts, then offsets
    int4 *alist;                    // submap volumes: allocated blocks {x | y << 16, z, ptr, entry}
    uint32_t n_buckets, n_excess, n_entries, n_blocks;
    uint32_t reqset_mask, max_req;
    uint32_t transfer_blocks;
    float voxel, mu;
    int32_t max_w;
};

// camera constants of one call (by value)
struct Cam {
    float M[12];      // world -> camera rows [R | t]
    float Ri[9];      // camera -> world rotation R^T
    float ti[3];      // camera -> world translation -R^T t
    float fx, fy, cx, cy;
    int32_t W, H;
};

// workspace carving
struct Layout {
    size_t entries, vis, free_blocks, free_excess, voxels, vlist, reqset, reqs, ret, depth,
        recs, bins, bin_count, ctrl, acc_cols, acc_hits, occ, brick, host_has, xfer_idx, xfer_vox, xfer_host,
        xfer_pend, swap_chunks, total;
    uint32_t reqset_size, max_req, max_tiles;
};

// ---- kernel launchers (tsdf_kernels.hip) -----------------------------------
hipError_t launch_init(const Vol &v, hipStream_t s);
hipError_t launch_clear_bins(int32_t *bin_count, uint32_t n, hipStream_t s, Ctrl *ctrl = nullptr);
hipError_t launch_alloc_rays(const Vol &v, const Cam &c, const void *depth, int fmt, hipStream_t s);
hipError_t launch_insert(const Vol &v, const Cam &c, hipStream_t s);
hipError_t launch_visible(const Vol &v, hipStream_t s);
hipError_t launch_depth_convert(const Vol &v, const void *depth, int fmt, int n, hipStream_t s);
hipError_t launch_integrate(const Vol &v, const Cam &c, bool bin, hipStream_t s);
hipError_t launch_range_bin(const Vol &v, const Cam &c, bool all_blocks, hipStream_t s);
// all_blocks: the bins hold every allocated block (not only the visible list)
hipError_t launch_raycast(const Vol &v, const Cam &c, bool all_blocks, float4 *pts, float4 *nrm, hipStream_t s);

hipError_t launch_range_write(const Vol &v, const Cam &c, float *zmin, float *zmax, hipStream_t s);
constexpr int kSwapChunk = 4096;        // entries per workgroup of the ordered swap-out selection
hipError_t launch_swap_candidates(const Vol &v, hipStream_t s);
hipError_t launch_swap_merge(const Vol &v, uint32_t n, hipStream_t s);
hipError_t launch_swap_select(const Vol &v, hipStream_t s);
hipError_t launch_swap_gather(const Vol &v, uint32_t n, hipStream_t s);
hipError_t launch_swap_release(const Vol &v, uint32_t n, hipStream_t s);
hipError_t launch_swap_merge_out(const Vol &v, uint32_t n, hipStream_t s);
hipError_t launch_camera_depth(const float4 *pts, int n, const float *M, float *depth, hipStream_t s);
hipError_t launch_export_voxels(const Vol &v, const int32_t *ids, uint32_t n, int16_t *sdf,
                                uint8_t *w, hipStream_t s);

// ---- rigid submaps (Sec. 7.2), batched ---------------------------------------
constexpr int kMaxSubmaps = 64;         // submaps of one batched map (one bit each in a tile mask)
constexpr int kMaxSel = 12;             // submaps one frame is integrated into
constexpr int kMaxViews = 8;            // views raycast per frame
constexpr int kExpand = 3;              // voxels added around a block when binning it for the combined field

// per submap, fixed at creation: what the combined-field raycast reads
struct MSub {
    const DEntry *entries;
    const uint32_t *occ;
    const uint8_t *voxels;
    const int4 *alist;
    const Ctrl *ctrl;
    uint32_t n_buckets, n_excess;
    float R[9];       // rotation of P_i (world -> submap)
    float s[3];       // translation of P_i in voxel units
};

// one view of a frame: camera, tile grid, outputs
struct MView {
    Cam cam;
    float4 *pts, *nrm;
    int32_t ntx, nty, tile_base, pad;
};

// per-frame parameters, uploaded from pinned host memory before the launches
struct alignas(16) MFrame {
    const void *depth;
    int32_t fmt, n_sel, n_views, tw, th, n_sub;
    int32_t sel[kMaxSel];
    Cam icam[kMaxSel];                      // integration camera of each selected submap
    MView view[kMaxViews];
    float C[kMaxViews][kMaxSubmaps][12];    // view camera composed with each submap pose
};

// batched-map counters
struct alignas(256) MCtrl {
    uint32_t flags;                 // TF_FLAG_BIN_OVERFLOW
    uint32_t pad;
    unsigned long long tot_bin;     // bin entries (block x tile) of all raycasts
    unsigned long long tot_blkview; // (block, view) pairs binned by all raycasts
    unsigned long long n_raycast;   // raycast launches
};

// tile bins of one raycast launch (all views share one flat tile index)
struct MTiles {
    int32_t *cnt;         // per tile: entries (count pass), zeroed by the scan
    uint32_t *off;        // per tile + 1: exclusive offsets into bins
    int32_t *cur;         // per tile: fill cursor, zeroed by the scan
    Rec *bins;            // entries, pad = submap index
    MCtrl *mc;
    unsigned long long *acc_hits;   // per tile: pixels with a hit
    unsigned long long *wmask;   // per 8-voxel world cell (kWorldCells, see wcell_index): the submaps whose blocks may reach it
    uint32_t cap;         // capacity of bins
    uint32_t n_tiles;     // tiles over all views
};

hipError_t launch_m_alloc(const Vol *vols, const MSub *subs, const MFrame *f, unsigned long long *wmask, int max_w,
                          int max_h,
                          hipStream_t s);
hipError_t launch_m_integrate(const Vol *vols, const MFrame *f, int nt, int grid, bool dry, hipStream_t s);
hipError_t launch_m_bin(const MSub *subs, const MFrame *f, const MTiles &t, int n_views, int grid, float voxel,
                        hipStream_t s);
hipError_t launch_m_raycast(const MSub *subs, const MFrame *f, const MTiles &t, float voxel, float mu, int tw, int th,
                            hipStream_t s);
hipError_t launch_m_range_write(const MSub *subs, const MFrame *f, const MTiles &t, int view, int n_tiles_view,
                                float *zmin, float *zmax, int tw, int th, hipStream_t s);
hipError_t launch_m_clear(const MTiles &t, hipStream_t s);

}  // namespace tsdf
