// tsdf_kernels.hip -- gfx950 kernels of the voxel-hashed TSDF fusion hot path.
//
// Frame pipeline (one launch each, counts stay on the device):
//   k_alloc_rays   one lane per pixel: depth ingest, segment samples, hash probes,
//                  visible marks, de-duplicated insertion requests      (Sec. 4.2, part 1)
//   k_insert       one lane per request: free-stack pops, bucket claim or excess
//                  chain link, block init; frustum re-test of the previous visible
//                  list                                                  (Sec. 4.2, parts 2-3)
//   k_visible      16 entries per lane: wave-scan compaction of the marks (Sec. 4.2, part 3)
//   k_integrate    one wave per visible block, 8 voxels per lane         (Sec. 4.3)
//   k_range_bin    one lane per block: projected box -> 16x16-pixel tile bins (Sec. 4.4)
//   k_raycast      one workgroup per 16x16 tile: per-pixel search range from the
//                  tile's bin, then the ray state machine                (Sec. 4.4)
//
// Compiled with -ffp-contract=off and correctly rounded fp32 division and
// square root: every float expression below is evaluated as written, one IEEE
// operation at a time.
#include "tsdf_internal.h"
#include "tsdf.h"

namespace tsdf {

namespace {

constexpr int kWave = 64;

// tuning knobs of the raycast (compile-time)
#ifndef TSDF_RAY_XCD_BANDS
#define TSDF_RAY_XCD_BANDS 1    // give each XCD a contiguous band of tiles
#endif
#ifndef TSDF_RAY_BITMAP
#define TSDF_RAY_BITMAP 1       // consult the bucket-occupancy bitmap before an entry
#endif

__device__ __forceinline__ uint32_t hash_index(int x, int y, int z, uint32_t mask)
{
    // Sec. 3.2 hashIndex
    return (((uint32_t)x * 73856093u) ^ ((uint32_t)y * 19349669u) ^ ((uint32_t)z * 83492791u)) & mask;
}

__device__ __forceinline__ bool in_short_range(int a) { return a >= -32768 && a <= 32767; }

__device__ __forceinline__ unsigned long long pack_key(int x, int y, int z)
{
    return (1ull << 48) | ((unsigned long long)(uint16_t)x << 32) |
           ((unsigned long long)(uint16_t)y << 16) | (unsigned long long)(uint16_t)z;
}

__device__ __forceinline__ void unpack_key(unsigned long long k, int &x, int &y, int &z)
{
    x = (int16_t)(uint16_t)(k >> 32);
    y = (int16_t)(uint16_t)(k >> 16);
    z = (int16_t)(uint16_t)k;
}

__device__ __forceinline__ uint32_t mix_key(unsigned long long k)
{
    k ^= k >> 30;
    k *= 0xbf58476d1ce4e5b9ull;
    k ^= k >> 27;
    k *= 0x94d049bb133111ebull;
    k ^= k >> 31;
    return (uint32_t)k;
}

// loads through global-address-space pointers (the Vol pointers arrive
// inside a by-value struct, so the compiler cannot infer their space)
template <typename T>
__device__ __forceinline__ T gload(const T *p)
{
    return *(const __attribute__((address_space(1))) T *)p;
}

typedef int v4i __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int4 load_entry(const DEntry *e, uint32_t i)
{
    const v4i w = gload(reinterpret_cast<const v4i *>(e + i));
    return make_int4(w.x, w.y, w.z, w.w);
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t rank_in(unsigned long long m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Retrieval (Sec. 3.3): bucket, then the chain of `offset` links.  Matches an
// entry whose position equals the key and whose ptr >= min_ptr.  Returns the
// entry index (and its ptr) or -1.
__device__ __forceinline__ int find_entry(const Vol &v, int bx, int by, int bz, int min_ptr, int *ptr_out)
{
    if (!in_short_range(bx) || !in_short_range(by) || !in_short_range(bz)) return -1;
    uint32_t i = hash_index(bx, by, bz, v.n_buckets - 1u);
    const uint32_t kxy = (uint32_t)(uint16_t)bx | ((uint32_t)(uint16_t)by << 16);
    for (uint32_t it = 0; it <= v.n_excess; ++it) {
        int4 w = load_entry(v.entries, i);
        if ((uint32_t)w.x == kxy && (int16_t)(w.y & 0xffff) == (int16_t)bz && w.w >= min_ptr) {
            *ptr_out = w.w;
            return (int)i;
        }
        if (w.z < 1 || (uint32_t)(w.z - 1) >= v.n_excess) return -1;
        i = v.n_buckets + (uint32_t)(w.z - 1);
    }
    return -1;
}

__device__ __forceinline__ void cam_transform(const Cam &c, float X, float Y, float Z, float &x, float &y, float &z)
{
    x = ((c.M[0] * X + c.M[1] * Y) + c.M[2] * Z) + c.M[3];
    y = ((c.M[4] * X + c.M[5] * Y) + c.M[6] * Z) + c.M[7];
    z = ((c.M[8] * X + c.M[9] * Y) + c.M[10] * Z) + c.M[11];
}

// Pop up to one element per requesting lane from a stack whose height is
// *head (Sec. 4.2 "atomic subtraction on a stack of free voxel block
// indices"), with one atomic per wave; the height never goes below zero.
__device__ int32_t wave_pop(int32_t *head, const int32_t *stack, bool want)
{
    unsigned long long m = __ballot(want);
    if (m == 0) return -1;
    const int cnt = __popcll(m);
    const int leader = __ffsll((long long)m) - 1;
    int base = 0, take = 0;
    if ((int)lane_id() == leader) {
        int cur = __hip_atomic_load(head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (;;) {
            take = cur < cnt ? cur : cnt;
            if (take <= 0) {
                take = 0;
                break;
            }
            int prev = atomicCAS(head, cur, cur - take);
            if (prev == cur) {
                base = cur - take;
                break;
            }
            cur = prev;
        }
    }
    base = __shfl(base, leader);
    take = __shfl(take, leader);
    const int r = (int)rank_in(m);
    if (want && r < take) return stack[base + take - 1 - r];
    return -1;
}

// Insert a key into the per-frame request set (open addressing, linear
// probing); the lane that adds it appends it to the request list.
__device__ void request_block(const Vol &v, int bx, int by, int bz)
{
    const unsigned long long key = pack_key(bx, by, bz);
    uint32_t s = mix_key(key) & v.reqset_mask;
    for (uint32_t it = 0; it <= v.reqset_mask; ++it) {
        unsigned long long cur = __hip_atomic_load(&v.reqset[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == key) return;
        if (cur == 0ull) {
            unsigned long long prev = atomicCAS(&v.reqset[s], 0ull, key);
            if (prev == 0ull) {
                uint32_t idx = atomicAdd(&v.ctrl->n_req, 1u);
                if (idx < v.max_req) {
                    v.reqs[idx].key = key;
                    v.reqs[idx].slot = s;
                } else {
                    // more new blocks than the whole block array: the budget is exhausted too
                    atomicOr(&v.ctrl->flags, TF_FLAG_REQUEST_OVERFLOW | TF_FLAG_BLOCKS_EXHAUSTED);
                    v.ctrl->req_overflow = 1u;
                }
                return;
            }
            if (prev == key) return;
        }
        s = (s + 1u) & v.reqset_mask;
    }
    atomicOr(&v.ctrl->flags, TF_FLAG_REQUEST_OVERFLOW);
    v.ctrl->req_overflow = 1u;
}

// Frustum re-test of a block kept from the previous visible list (Sec. 4.2,
// part 3): some corner in front of the camera projects into the image.
__device__ bool block_in_frustum(const Vol &v, const Cam &c, int bx, int by, int bz)
{
    const float umax = (float)(c.W - 1), vmax = (float)(c.H - 1);
    for (int k = 0; k < 8; ++k) {
        int px = 8 * (bx + (k & 1)), py = 8 * (by + ((k >> 1) & 1)), pz = 8 * (bz + (k >> 2));
        float x, y, z;
        cam_transform(c, (float)px * v.voxel, (float)py * v.voxel, (float)pz * v.voxel, x, y, z);
        if (z <= 0.0f) continue;
        float rz = 1.0f / z;
        float u = (c.fx * x) * rz + c.cx;
        float vv = (c.fy * y) * rz + c.cy;
        if (u >= 0.0f && u <= umax && vv >= 0.0f && vv <= vmax) return true;
    }
    return false;
}

}  // namespace

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
    if (gid == 0) {
        Ctrl c = {};
        c.free_blocks = (int32_t)v.n_blocks;
        c.free_excess = (int32_t)v.n_excess;
        *v.ctrl = c;
    }
}

__global__ __launch_bounds__(256) void k_clear_bins(int32_t *bin_count, uint32_t n)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        bin_count[i] = 0;
}

// ============================================================================
// allocation, part 1: segments, probes, marks, requests
// ============================================================================
template <int FMT>
__global__ __launch_bounds__(256) void k_alloc_rays(Vol v, Cam c, const void *din)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p == 0) {
        Ctrl *C = v.ctrl;
        C->n_vis_prev = C->n_vis;
        C->sweep_req = 0u;
        C->n_vis = 0u;
        C->n_new = 0u;
        C->n_swapped_in = 0u;
    }
    const int W = c.W, H = c.H;
    if (p >= W * H) return;
    float d;
    if (FMT == TF_DEPTH_U16_MM)
        d = (float)reinterpret_cast<const uint16_t *>(din)[p] / 1000.0f;   // Sec. 4 depth ingest
    else
        d = reinterpret_cast<const float *>(din)[p];
    v.depth[p] = d;
    if (!(d > 0.0f)) return;

    // the segment between camera depths d - mu and d + mu (Sec. 4.2), in block units
    const int x = p % W, y = p / W;
    const float a = ((float)x - c.cx) / c.fx;
    const float b = ((float)y - c.cy) / c.fy;
    const float z0 = d - v.mu, z1 = d + v.mu;
    const float c0x = z0 * a, c0y = z0 * b, c0z = z0;
    const float c1x = z1 * a, c1y = z1 * b, c1z = z1;
    const float inv_block = 1.0f / (8.0f * v.voxel);
    float q0[3], dq[3];
    for (int r = 0; r < 3; ++r) {
        float w0 = ((c.Ri[3 * r] * c0x + c.Ri[3 * r + 1] * c0y) + c.Ri[3 * r + 2] * c0z) + c.ti[r];
        float w1 = ((c.Ri[3 * r] * c1x + c.Ri[3 * r + 1] * c1y) + c.Ri[3 * r + 2] * c1z) + c.ti[r];
        q0[r] = w0 * inv_block;
        float q1 = w1 * inv_block;
        dq[r] = q1 - q0[r];
    }
    const float L = sqrtf((dq[0] * dq[0] + dq[1] * dq[1]) + dq[2] * dq[2]);
    int n = (int)ceilf(2.0f * L);
    if (n < 1) n = 1;
    const float sx = dq[0] / (float)n, sy = dq[1] / (float)n, sz = dq[2] / (float)n;

    int pbx = 0, pby = 0, pbz = 0;
    bool have_prev = false;
    int m = 0;
    for (int k = 0; k <= n && m < kMaxSegmentSamples; ++k) {
        const float qx = q0[0] + (float)k * sx;
        const float qy = q0[1] + (float)k * sy;
        const float qz = q0[2] + (float)k * sz;
        const float fx = floorf(qx), fy = floorf(qy), fz = floorf(qz);
        if (!(fx >= -32768.0f && fx <= 32767.0f && fy >= -32768.0f && fy <= 32767.0f &&
              fz >= -32768.0f && fz <= 32767.0f))
            continue;
        ++m;
        const int bx = (int)fx, by = (int)fy, bz = (int)fz;
        if (have_prev && bx == pbx && by == pby && bz == pbz) continue;
        have_prev = true;
        pbx = bx;
        pby = by;
        pbz = bz;
        int ptr;
        int e = find_entry(v, bx, by, bz, kPtrSwapped, &ptr);
        if (e >= 0) {
            if (ptr >= 0) v.vis[e] = kVisTouched;
        } else {
            request_block(v, bx, by, bz);
        }
    }
}

// ============================================================================
// allocation, parts 2 and 3a: insertion and the previous list's frustum test
// ============================================================================
__global__ __launch_bounds__(256) void k_insert(Vol v, Cam c)
{
    const uint32_t lane = lane_id();
    const uint32_t gwave = (blockIdx.x * 256u + threadIdx.x) / kWave;
    const uint32_t nwaves = gridDim.x * (256u / kWave);
    uint32_t n = v.ctrl->n_req;
    if (n > v.max_req) n = v.max_req;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        v.ctrl->sweep_req = v.ctrl->req_overflow;
        v.ctrl->req_overflow = 0u;
    }

    for (uint32_t base = gwave * kWave; base < n; base += nwaves * kWave) {
        const uint32_t i = base + lane;
        const bool active = i < n;
        int bx = 0, by = 0, bz = 0;
        if (active) {
            Req r = v.reqs[i];
            v.reqset[r.slot] = 0ull;
            unpack_key(r.key, bx, by, bz);
        }
        const int32_t blk = wave_pop(&v.ctrl->free_blocks, v.free_blocks, active);
        if (active && blk < 0) atomicOr(&v.ctrl->flags, TF_FLAG_BLOCKS_EXHAUSTED);
        const uint32_t h = hash_index(bx, by, bz, v.n_buckets - 1u);
        int entry = -1;
        bool need_excess = false;
        const unsigned long long posw = (unsigned long long)(uint16_t)bx | ((unsigned long long)(uint16_t)by << 16) |
                                        ((unsigned long long)(uint16_t)bz << 32);
        if (active && blk >= 0) {
            int prev = atomicCAS(&v.entries[h].ptr, kPtrEmpty, kPtrClaimed);
            if (prev == kPtrEmpty) {
                *reinterpret_cast<unsigned long long *>(&v.entries[h]) = posw;
                v.entries[h].ptr = blk;
                entry = (int)h;
            } else {
                need_excess = true;
            }
        }
        const int32_t slot = wave_pop(&v.ctrl->free_excess, v.free_excess, need_excess);
        if (need_excess) {
            if (slot < 0) {
                atomicOr(&v.ctrl->flags, TF_FLAG_EXCESS_EXHAUSTED);
                uint32_t ri = atomicAdd(&v.ctrl->n_ret, 1u);
                v.ret[ri] = blk;
            } else {
                const uint32_t idx = v.n_buckets + (uint32_t)slot;
                *reinterpret_cast<unsigned long long *>(&v.entries[idx]) = posw;
                v.entries[idx].ptr = blk;
                int32_t old = __hip_atomic_load(&v.entries[h].offset, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                for (;;) {
                    v.entries[idx].offset = old;
                    int32_t pr = atomicCAS(&v.entries[h].offset, old, slot + 1);
                    if (pr == old) break;
                    old = pr;
                }
                entry = (int)idx;
            }
        }
        if (entry >= 0) {
            v.vis[entry] = kVisNew;
            atomicOr(&v.occ[h >> 5], 1u << (h & 31u));
        }
        // initialise each new block (Sec. 3.1: sdf 32767, weight 0) with the whole wave
        unsigned long long m = __ballot(entry >= 0);
        if (lane == 0 && m) atomicAdd(&v.ctrl->n_new, (uint32_t)__popcll(m));
        while (m) {
            const int l = __ffsll((long long)m) - 1;
            m &= m - 1;
            const int b = __shfl(blk, l);
            uint8_t *dst = v.voxels + (size_t)b * kBlockBytes;
            reinterpret_cast<uint4 *>(dst)[lane] = make_uint4(0x7fff7fffu, 0x7fff7fffu, 0x7fff7fffu, 0x7fff7fffu);
            reinterpret_cast<uint2 *>(dst + 1024)[lane] = make_uint2(0u, 0u);
        }
    }

    const uint32_t np = v.ctrl->n_vis_prev;
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < np; i += gridDim.x * 256u) {
        const int e = v.vlist[i];
        const int4 w = load_entry(v.entries, (uint32_t)e);
        if (w.w < 0 || v.vis[e] != 0) continue;
        const int bx = (int16_t)(w.x & 0xffff), by = (int16_t)((uint32_t)w.x >> 16), bz = (int16_t)(w.y & 0xffff);
        if (block_in_frustum(v, c, bx, by, bz)) v.vis[e] = kVisTouched;
    }
}

// ============================================================================
// allocation, part 3b: compaction of the marks into the visible list
// ============================================================================
__global__ __launch_bounds__(256) void k_visible(Vol v)
{
    const uint32_t lane = lane_id();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        Ctrl *C = v.ctrl;
        C->tot_req += C->n_req < v.max_req ? C->n_req : v.max_req;
        C->tot_new += C->n_new;
        C->n_req = 0u;
        C->frames += 1u;
        const uint32_t nr = C->n_ret;
        if (nr) {
            const int32_t h = C->free_blocks;
            for (uint32_t i = 0; i < nr; ++i) v.free_blocks[h + (int32_t)i] = v.ret[i];
            C->free_blocks = h + (int32_t)nr;
            C->n_ret = 0u;
        }
    }
    if (v.ctrl->sweep_req) {
        for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i <= v.reqset_mask; i += gridDim.x * 256u)
            v.reqset[i] = 0ull;
    }
    const uint32_t gwave = (blockIdx.x * 256u + threadIdx.x) / kWave;
    const uint32_t nwaves = gridDim.x * (256u / kWave);
    const uint32_t nchunks = (v.n_entries + 15u) / 16u;
    for (uint32_t cb = gwave * kWave; cb < nchunks; cb += nwaves * kWave) {
        const uint32_t ch = cb + lane;
        uint4 f = make_uint4(0u, 0u, 0u, 0u);
        if (ch < nchunks) f = reinterpret_cast<const uint4 *>(v.vis)[ch];
        const uint32_t words[4] = {f.x, f.y, f.z, f.w};
        uint32_t cnt = 0;
#pragma unroll
        for (int j = 0; j < 16; ++j) cnt += ((words[j >> 2] >> (8 * (j & 3))) & 0xffu) ? 1u : 0u;
        uint32_t incl = cnt;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            uint32_t t = __shfl_up(incl, d);
            if ((int)lane >= d) incl += t;
        }
        const uint32_t total = __shfl(incl, kWave - 1);
        if (total == 0) continue;
        uint32_t base = 0;
        if (lane == kWave - 1) base = atomicAdd(&v.ctrl->n_vis, total);
        base = __shfl(base, kWave - 1);
        uint32_t pos = base + incl - cnt;
        if (cnt) {
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if ((words[j >> 2] >> (8 * (j & 3))) & 0xffu) v.vlist[pos++] = (int32_t)(ch * 16u + (uint32_t)j);
            reinterpret_cast<uint4 *>(v.vis)[ch] = make_uint4(0u, 0u, 0u, 0u);
        }
    }
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
// integration (Sec. 4.3)
// ============================================================================
// Lane (lx, ly) = (lane >> 3, lane & 7) owns the 8 voxels lz = 0..7 of one
// column; the device in-block order lz + 8 ly + 64 lx puts them in 16
// contiguous bytes of SDF and 8 of weight, so a wave moves a block in one
// dwordx4 and one dwordx2 access per lane.
__global__ __launch_bounds__(256) void k_integrate(Vol v, Cam c)
{
    __shared__ float rcp_w[260];
    for (int k = threadIdx.x; k < 260; k += 256) rcp_w[k] = k ? 1.0f / (float)k : 0.0f;
    __syncthreads();
    const uint32_t lane = lane_id();
    const uint32_t gwave = (blockIdx.x * 256u + threadIdx.x) / kWave;
    const uint32_t nwaves = gridDim.x * (256u / kWave);
    const uint32_t nvis = v.ctrl->n_vis;
    const int lx = (int)(lane >> 3), ly = (int)(lane & 7);
    const float vs = v.voxel;
    const float inv_mu = 1.0f / v.mu;
    const float neg_mu = -v.mu;
    const float k_sdf = 1.0f / 32767.0f;
    const float umax = (float)(c.W - 2), vmax = (float)(c.H - 2);
    const int W = c.W;
    const int max_w = v.max_w;
    const float *depth = v.depth;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        v.ctrl->tot_vis += nvis;
        v.ctrl->n_integrate += 1ull;
    }
    uint32_t cols = 0;

    for (uint32_t i = gwave; i < nvis; i += nwaves) {
        const int e = v.vlist[i];
        const int4 w = load_entry(v.entries, (uint32_t)e);
        const int ptr = w.w;
        if (ptr < 0) continue;
        const int bx = (int16_t)(w.x & 0xffff), by = (int16_t)((uint32_t)w.x >> 16), bz = (int16_t)(w.y & 0xffff);
        uint8_t *blk = v.voxels + (size_t)ptr * kBlockBytes;
        uint4 s8 = reinterpret_cast<const uint4 *>(blk)[lane];
        uint2 w8 = reinterpret_cast<const uint2 *>(blk + 1024)[lane];
        uint32_t sw[4] = {s8.x, s8.y, s8.z, s8.w};
        uint32_t ww[2] = {w8.x, w8.y};
        const float X = (float)(8 * bx + lx) * vs;
        const float Y = (float)(8 * by + ly) * vs;
        const float p0 = c.M[0] * X + c.M[1] * Y;
        const float p1 = c.M[4] * X + c.M[5] * Y;
        const float p2 = c.M[8] * X + c.M[9] * Y;
        // phase 1: projection of the column's 8 voxels (no memory traffic)
        float czs[8];
        int idx[8];
        bool inimg[8];
#pragma unroll
        for (int lz = 0; lz < 8; ++lz) {
            const float Z = (float)(8 * bz + lz) * vs;
            const float cx = (p0 + c.M[2] * Z) + c.M[3];
            const float cy = (p1 + c.M[6] * Z) + c.M[7];
            const float cz = (p2 + c.M[10] * Z) + c.M[11];
            czs[lz] = cz;
            bool ok = cz > 0.0f;
            const float rz = 1.0f / (ok ? cz : 1.0f);
            const float u = (c.fx * cx) * rz + c.cx;
            const float vv = (c.fy * cy) * rz + c.cy;
            ok = ok && !(u < 1.0f || u > umax || vv < 1.0f || vv > vmax);
            const int ix = ok ? (int)(u + 0.5f) : 0, iy = ok ? (int)(vv + 0.5f) : 0;
            inimg[lz] = ok;
            idx[lz] = ix + iy * W;
        }
        // phase 2: the 8 depth reads, issued together
        float dep[8];
#pragma unroll
        for (int lz = 0; lz < 8; ++lz) dep[lz] = gload(depth + idx[lz]);
        // phase 3: the running-average update (Sec. 4.3)
        bool changed = false;
#pragma unroll
        for (int lz = 0; lz < 8; ++lz) {
            if (!inimg[lz]) continue;
            const float d = dep[lz];
            if (d <= 0.0f) continue;
            const float eta = d - czs[lz];
            if (eta < neg_mu) continue;
            float f_new = eta * inv_mu;
            if (f_new > 1.0f) f_new = 1.0f;
            const uint32_t sh = 16u * (lz & 1);
            const int s_old = (int16_t)((sw[lz >> 1] >> sh) & 0xffffu);
            const uint32_t whs = 8u * (lz & 3);
            const int w_old = (int)((ww[lz >> 2] >> whs) & 0xffu);
            const float f_old = (float)s_old * k_sdf;
            const float avg = ((float)w_old * f_old + f_new) * rcp_w[w_old + 1];
            int w_new = w_old + 1;
            if (w_new > max_w) w_new = max_w;
            const int s_new = (int16_t)(avg * 32767.0f);
            sw[lz >> 1] = (sw[lz >> 1] & ~(0xffffu << sh)) | (((uint32_t)s_new & 0xffffu) << sh);
            ww[lz >> 2] = (ww[lz >> 2] & ~(0xffu << whs)) | ((uint32_t)w_new << whs);
            changed = true;
        }
        if (changed) {
            reinterpret_cast<uint4 *>(blk)[lane] = make_uint4(sw[0], sw[1], sw[2], sw[3]);
            reinterpret_cast<uint2 *>(blk + 1024)[lane] = make_uint2(ww[0], ww[1]);
            ++cols;
        }
    }
    // per-workgroup count of written columns (no cross-workgroup atomics)
    __shared__ uint32_t wg_cols;
    if (threadIdx.x == 0) wg_cols = 0;
    __syncthreads();
    if (cols) atomicAdd(&wg_cols, cols);
    __syncthreads();
    if (threadIdx.x == 0 && wg_cols) v.acc_cols[blockIdx.x] += wg_cols;
}

// ============================================================================
// search range (Sec. 4.4): project blocks, bin their boxes by 16x16 tile
// ============================================================================
__device__ bool block_record(const Vol &v, const Cam &c, int bx, int by, int bz, Rec &r)
{
    float xs[8], ys[8], zs[8];
    float zlo = __builtin_inff(), zhi = -__builtin_inff();
    for (int k = 0; k < 8; ++k) {
        int px = 8 * (bx + (k & 1)), py = 8 * (by + ((k >> 1) & 1)), pz = 8 * (bz + (k >> 2));
        cam_transform(c, (float)px * v.voxel, (float)py * v.voxel, (float)pz * v.voxel, xs[k], ys[k], zs[k]);
        if (zs[k] < zlo) zlo = zs[k];
        if (zs[k] > zhi) zhi = zs[k];
    }
    if (zhi < kZNear) return false;
    if (zlo < kZNear) {
        r.x0 = 0;
        r.y0 = 0;
        r.x1 = (int16_t)(c.W - 1);
        r.y1 = (int16_t)(c.H - 1);
        r.zlo = kZNear;
        r.zhi = zhi;
        return true;
    }
    float umin = __builtin_inff(), umax = -__builtin_inff(), vmin = __builtin_inff(), vmax = -__builtin_inff();
    for (int k = 0; k < 8; ++k) {
        float rz = 1.0f / zs[k];
        float u = (c.fx * xs[k]) * rz + c.cx;
        float vv = (c.fy * ys[k]) * rz + c.cy;
        if (u < umin) umin = u;
        if (u > umax) umax = u;
        if (vv < vmin) vmin = vv;
        if (vv > vmax) vmax = vv;
    }
    float fx0 = floorf(umin), fx1 = ceilf(umax), fy0 = floorf(vmin), fy1 = ceilf(vmax);
    if (fx0 < 0.0f) fx0 = 0.0f;
    if (fy0 < 0.0f) fy0 = 0.0f;
    if (fx1 > (float)(c.W - 1)) fx1 = (float)(c.W - 1);
    if (fy1 > (float)(c.H - 1)) fy1 = (float)(c.H - 1);
    if (fx0 > fx1 || fy0 > fy1) return false;
    r.x0 = (int16_t)(int)fx0;
    r.x1 = (int16_t)(int)fx1;
    r.y0 = (int16_t)(int)fy0;
    r.y1 = (int16_t)(int)fy1;
    r.zlo = zlo;
    r.zhi = zhi;
    return true;
}

__global__ __launch_bounds__(256) void k_range_bin(Vol v, Cam c, int all)
{
    const uint32_t lane = lane_id();
    const uint32_t gwave = (blockIdx.x * 256u + threadIdx.x) / kWave;
    const uint32_t nwaves = gridDim.x * (256u / kWave);
    const uint32_t n = all ? v.n_entries : v.ctrl->n_vis;
    const int ntx = (c.W + kTile - 1) / kTile;
    for (uint32_t base = gwave * kWave; base < n; base += nwaves * kWave) {
        const uint32_t i = base + lane;
        bool emit = false;
        Rec r;
        if (i < n) {
            const uint32_t e = all ? i : (uint32_t)v.vlist[i];
            const int4 w = load_entry(v.entries, e);
            if (w.w >= 0) {
                const int bx = (int16_t)(w.x & 0xffff), by = (int16_t)((uint32_t)w.x >> 16), bz = (int16_t)(w.y & 0xffff);
                emit = block_record(v, c, bx, by, bz, r);
            }
        }
        const unsigned long long m = __ballot(emit);
        if (!m) continue;
        const int leader = __ffsll((long long)m) - 1;
        uint32_t rb = 0;
        if ((int)lane == leader) rb = atomicAdd(&v.ctrl->n_rec, (uint32_t)__popcll(m));
        rb = __shfl(rb, leader);
        if (emit) {
            const uint32_t idx = rb + rank_in(m);
            v.recs[idx] = r;
            const int tx0 = r.x0 / kTile, tx1 = r.x1 / kTile, ty0 = r.y0 / kTile, ty1 = r.y1 / kTile;
            for (int ty = ty0; ty <= ty1; ++ty)
                for (int tx = tx0; tx <= tx1; ++tx) {
                    const int t = ty * ntx + tx;
                    const int s = atomicAdd(&v.bin_count[t], 1);
                    if (s < kBinCap) v.bins[(size_t)t * kBinCap + s] = (int32_t)idx;
                }
        }
    }
}

// per-pixel min/max over the records of a tile's bin (all records if the
// bin overflowed); every thread of the workgroup must call it
__device__ void tile_range(const Vol &v, int tile, int px, int py, float &zmin, float &zmax, Rec *lds)
{
    zmin = __builtin_inff();
    zmax = -__builtin_inff();
    const int cnt = v.bin_count[tile];
    const bool fallback = cnt > kBinCap;
    const int n = fallback ? (int)v.ctrl->n_rec : cnt;
    for (int base = 0; base < n; base += 256) {
        const int j = base + (int)threadIdx.x;
        if (j < n) lds[threadIdx.x] = v.recs[fallback ? j : v.bins[(size_t)tile * kBinCap + j]];
        __syncthreads();
        const int m = (n - base) < 256 ? (n - base) : 256;
        for (int k = 0; k < m; ++k) {
            const Rec r = lds[k];
            if (px >= r.x0 && px <= r.x1 && py >= r.y0 && py <= r.y1) {
                if (r.zlo < zmin) zmin = r.zlo;
                if (r.zhi > zmax) zmax = r.zhi;
            }
        }
        __syncthreads();
    }
}

// last workgroup of a raycast-kind launch clears the record counter
__device__ void finish_tile(const Vol &v, int tile, bool count_raycast)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        if (tile >= 0) v.bin_count[tile] = 0;
        __threadfence();
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

__device__ __forceinline__ int block_of(float X) { return ((int)floorf(X)) >> 3; }

// one-entry block cache (the paper's IndexCache, Sec. 3.3): the last block
// key looked up and its device pointer (-1 = absent or not on the device)
struct BlockCache {
    int bx, by, bz, ptr;
};

// device pointer of a block (-1 = absent or not on the device); the bucket
// bitmap answers most probes of empty space without touching the entries
__device__ __forceinline__ int lookup_block(const Vol &v, int bx, int by, int bz)
{
    int ptr = -1, e = -1;
#if TSDF_RAY_BITMAP
    const uint32_t h = hash_index(bx, by, bz, v.n_buckets - 1u);
    if ((gload(v.occ + (h >> 5)) >> (h & 31u)) & 1u) e = find_entry(v, bx, by, bz, 0, &ptr);
#else
    e = find_entry(v, bx, by, bz, 0, &ptr);
#endif
    return e >= 0 ? ptr : -1;
}

__device__ __forceinline__ int cached_block(const Vol &v, int bx, int by, int bz, BlockCache &cc)
{
    if (bx == cc.bx && by == cc.by && bz == cc.bz) return cc.ptr;
    cc.bx = bx;
    cc.by = by;
    cc.bz = bz;
    cc.ptr = lookup_block(v, bx, by, bz);
    return cc.ptr;
}

__device__ __forceinline__ float corner_F(const Vol &v, int p, int x, int y, int z)
{
    const int j = (z & 7) + 8 * (y & 7) + 64 * (x & 7);
    const int16_t s = gload(reinterpret_cast<const int16_t *>(v.voxels + (size_t)(p >= 0 ? p : 0) * kBlockBytes) +
                            (p >= 0 ? j : 0));
    return p >= 0 ? (float)s * (1.0f / 32767.0f) : 1.0f;
}

// trilinear interpolation of F at voxel-unit P (absent voxels read 1.0):
// lerp a + (b - a) t along x, then y, then z.  The corner blocks are resolved
// first (the cell's own block through the ray's cache; blocks across a face,
// when the cell crosses one, by direct lookups), then the eight voxel loads
// are issued together.
__device__ __forceinline__ float trilinear(const Vol &v, float X, float Y, float Z, BlockCache &cc)
{
    const float bx = floorf(X), by = floorf(Y), bz = floorf(Z);
    const float tx = X - bx, ty = Y - by, tz = Z - bz;
    const int ix = (int)bx, iy = (int)by, iz = (int)bz;
    const int Bx = ix >> 3, By = iy >> 3, Bz = iz >> 3;
    const bool sx = (ix & 7) == 7, sy = (iy & 7) == 7, sz = (iz & 7) == 7;
    const int p000 = cached_block(v, Bx, By, Bz, cc);
    int p100 = p000, p010 = p000, p001 = p000, p110 = p000, p101 = p000, p011 = p000, p111 = p000;
    if (sx | sy | sz) {
        if (sx) p100 = lookup_block(v, Bx + 1, By, Bz);
        if (sy) p010 = lookup_block(v, Bx, By + 1, Bz);
        if (sz) p001 = lookup_block(v, Bx, By, Bz + 1);
        p110 = (sx & sy) ? lookup_block(v, Bx + 1, By + 1, Bz) : (sx ? p100 : p010);
        p101 = (sx & sz) ? lookup_block(v, Bx + 1, By, Bz + 1) : (sx ? p100 : p001);
        p011 = (sy & sz) ? lookup_block(v, Bx, By + 1, Bz + 1) : (sy ? p010 : p001);
        p111 = (sx & sy & sz) ? lookup_block(v, Bx + 1, By + 1, Bz + 1)
                              : (sx & sy) ? p110 : (sx & sz) ? p101 : (sy & sz) ? p011 : sx ? p100 : sy ? p010 : p001;
    }
    const float f000 = corner_F(v, p000, ix, iy, iz), f100 = corner_F(v, p100, ix + 1, iy, iz);
    const float f010 = corner_F(v, p010, ix, iy + 1, iz), f110 = corner_F(v, p110, ix + 1, iy + 1, iz);
    const float f001 = corner_F(v, p001, ix, iy, iz + 1), f101 = corner_F(v, p101, ix + 1, iy, iz + 1);
    const float f011 = corner_F(v, p011, ix, iy + 1, iz + 1), f111 = corner_F(v, p111, ix + 1, iy + 1, iz + 1);
    const float c00 = f000 + (f100 - f000) * tx;
    const float c10 = f010 + (f110 - f010) * tx;
    const float c01 = f001 + (f101 - f001) * tx;
    const float c11 = f011 + (f111 - f011) * tx;
    const float c0 = c00 + (c10 - c00) * ty;
    const float c1 = c01 + (c11 - c01) * ty;
    return c0 + (c1 - c0) * tz;
}

// "allocated" test of the march: the block of floor(P) has a device block
__device__ __forceinline__ bool allocated_at(const Vol &v, float P0, float P1, float P2, BlockCache &cc)
{
    return cached_block(v, block_of(P0), block_of(P1), block_of(P2), cc) >= 0;
}

enum { SEARCH_BLOCK_COARSE, SEARCH_BLOCK_FINE, SEARCH_SURFACE, BEHIND_SURFACE, WRONG_SIDE };

}  // namespace

// search range on its own, written as an image (tf_range_image)
__global__ __launch_bounds__(256) void k_range_write(Vol v, Cam c, float *zmin_out, float *zmax_out)
{
    __shared__ Rec lds[256];
    const int ntx = (c.W + kTile - 1) / kTile;
    const int tile = blockIdx.x;
    const int px = (tile % ntx) * kTile + (int)(threadIdx.x % kTile);
    const int py = (tile / ntx) * kTile + (int)(threadIdx.x / kTile);
    float zmin, zmax;
    tile_range(v, tile, px, py, zmin, zmax, lds);
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
__global__ __launch_bounds__(256) void k_raycast(Vol v, Cam c, float4 *pts, float4 *nrm)
{
    __shared__ Rec lds[256];
    const int ntx = (c.W + kTile - 1) / kTile, nty = (c.H + kTile - 1) / kTile;
    const int ntiles = ntx * nty;
#if TSDF_RAY_XCD_BANDS
    // workgroups go round-robin to the 8 XCDs: XCD k gets the k-th band of
    // tiles, so its L2 holds the blocks of one band of the image
    const int per = (ntiles + 7) / 8;
    const int tile = (int)(blockIdx.x % 8u) * per + (int)(blockIdx.x / 8u);
#else
    const int tile = (int)blockIdx.x;
#endif
    const bool real = tile < ntiles;
    const int q = (int)threadIdx.x >> 6, i = (int)threadIdx.x & 63;
    const int px = real ? (tile % ntx) * kTile + (q & 1) * 8 + (i & 7) : 0;
    const int py = real ? (tile / ntx) * kTile + (q >> 1) * 8 + (i >> 3) : 0;
    float zmin = __builtin_inff(), zmax = -__builtin_inff();
    if (real) tile_range(v, tile, px, py, zmin, zmax, lds);
    finish_tile(v, real ? tile : -1, true);
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
        BlockCache cc = {0x7fffffff, 0, 0, -1};
        int steps = 0;
        while (t < t_end && steps < kMaxRaySteps) {
            ++steps;
            const float P0 = ox + t * dx, P1 = oy + t * dy, P2 = oz + t * dz;
            const bool alloc = allocated_at(v, P0, P1, P2, cc);
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
                F = trilinear(v, P0, P1, P2, cc);
                if (state == SEARCH_BLOCK_FINE) {
                    state = (F < 0.0f) ? WRONG_SIDE : SEARCH_SURFACE;
                } else if (state == SEARCH_SURFACE) {
                    if (F < 0.0f) {
                        state = BEHIND_SURFACE;
                        break;
                    }
                    const float s = F * mu_v;
                    t += (s > 1.0f) ? s : 1.0f;
                } else {
                    if (F >= 0.0f) {
                        state = SEARCH_SURFACE;
                    } else {
                        const float s = -F * mu_v;
                        t += (s > 1.0f) ? s : 1.0f;
                    }
                }
            }
        }
        if (state == BEHIND_SURFACE) {
            t += F * mu_v;
            float P0 = ox + t * dx, P1 = oy + t * dy, P2 = oz + t * dz;
            F = trilinear(v, P0, P1, P2, cc);
            t += F * mu_v;
            P0 = ox + t * dx;
            P1 = oy + t * dy;
            P2 = oz + t * dz;
            out_p = make_float4(P0 * vs, P1 * vs, P2 * vs, 1.0f);
            const float gx = (trilinear(v, P0 + 1.0f, P1, P2, cc) - trilinear(v, P0 - 1.0f, P1, P2, cc)) * 0.5f;
            const float gy = (trilinear(v, P0, P1 + 1.0f, P2, cc) - trilinear(v, P0, P1 - 1.0f, P2, cc)) * 0.5f;
            const float gz = (trilinear(v, P0, P1, P2 + 1.0f, cc) - trilinear(v, P0, P1, P2 - 1.0f, cc)) * 0.5f;
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

hipError_t launch_clear_bins(int32_t *bin_count, uint32_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear_bins, dim3(cu_grid(n, 256, 1024)), dim3(256), 0, s, bin_count, n);
    return hipGetLastError();
}

hipError_t launch_alloc_rays(const Vol &v, const Cam &c, const void *depth, int fmt, hipStream_t s)
{
    const int npix = c.W * c.H;
    const dim3 g((npix + 255) / 256), b(256);
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

hipError_t launch_integrate(const Vol &v, const Cam &c, hipStream_t s)
{
    hipLaunchKernelGGL(k_integrate, dim3(kIntegrateGrid), dim3(256), 0, s, v, c);
    return hipGetLastError();
}

hipError_t launch_range_bin(const Vol &v, const Cam &c, bool all_blocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_range_bin, dim3(1024), dim3(256), 0, s, v, c, all_blocks ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_raycast(const Vol &v, const Cam &c, float4 *pts, float4 *nrm, hipStream_t s)
{
    const int ntiles = ((c.W + kTile - 1) / kTile) * ((c.H + kTile - 1) / kTile);
#if TSDF_RAY_XCD_BANDS
    const int grid = ((ntiles + 7) / 8) * 8;
#else
    const int grid = ntiles;
#endif
    hipLaunchKernelGGL(k_raycast, dim3(grid), dim3(256), 0, s, v, c, pts, nrm);
    return hipGetLastError();
}

hipError_t launch_range_write(const Vol &v, const Cam &c, float *zmin, float *zmax, hipStream_t s)
{
    const int ntiles = ((c.W + kTile - 1) / kTile) * ((c.H + kTile - 1) / kTile);
    hipLaunchKernelGGL(k_range_write, dim3(ntiles), dim3(256), 0, s, v, c, zmin, zmax);
    return hipGetLastError();
}

hipError_t launch_export_voxels(const Vol &v, const int32_t *ids, uint32_t n, int16_t *sdf, uint8_t *w, hipStream_t s)
{
    hipLaunchKernelGGL(k_export_voxels, dim3(cu_grid((size_t)n * 64, 256, 4096)), dim3(256), 0, s, v, ids, n, sdf, w);
    return hipGetLastError();
}

}  // namespace tsdf
