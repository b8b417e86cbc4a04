// tsdf_device.h -- device helpers and kernel bodies of libtsdf shared by the
// single-volume launches (tsdf_kernels.hip) and the batched-submap launches
// (tsdf_multi.hip).  Internal to the library.
//
// Compiled with -ffp-contract=off and correctly rounded fp32 division and
// square root: every float expression below is evaluated as written, one IEEE
// operation at a time.
#pragma once

#include "tsdf_internal.h"
#include "tsdf.h"

namespace tsdf {

namespace {

constexpr int kWave = 64;

__device__ __forceinline__ uint32_t hash_index(int x, int y, int z, uint32_t mask)
{
    // Sec. 3.2 hashIndex
    return (((uint32_t)x * 73856093u) ^ ((uint32_t)y * 19349669u) ^ ((uint32_t)z * 83492791u)) & mask;
}

__device__ __forceinline__ bool in_short_range(int a) { return a >= -32768 && a <= 32767; }

// Block-occupancy bricks: one bit per block position modulo a window of
// 256 blocks per axis, each 32-bit word a 4 x 4 x 2 brick of blocks, so that
// the positions of a ray share words.  Set when an entry is inserted, never
// cleared (a swapped-out entry keeps its bit): a clear bit proves the block
// absent; blocks a window apart share a bit (a false "maybe").
__device__ __forceinline__ uint32_t brick_word(int bx, int by, int bz)
{
    return (((uint32_t)(bx >> 2) & 63u) << 13) | (((uint32_t)(by >> 2) & 63u) << 7) | ((uint32_t)(bz >> 1) & 127u);
}

__device__ __forceinline__ uint32_t brick_bit(int bx, int by, int bz)
{
    return 1u << (((uint32_t)bx & 3u) | (((uint32_t)by & 3u) << 2) | (((uint32_t)bz & 1u) << 4));
}

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

// Retrieval (Sec. 3.3) from bucket i = hash_index(bx, by, bz): the bucket,
// then the chain of `offset` links.  Matches an entry whose position equals
// the key and whose ptr >= min_ptr.  Returns the entry index (and its ptr) or -1.
__device__ __forceinline__ int find_entry_from(const DEntry *entries, uint32_t n_buckets, uint32_t n_excess, uint32_t i,
                                               int bx, int by, int bz, int min_ptr, int *ptr_out)
{
    const uint32_t kxy = (uint32_t)(uint16_t)bx | ((uint32_t)(uint16_t)by << 16);
    for (uint32_t it = 0; it <= n_excess; ++it) {
        int4 w = load_entry(entries, i);
        if ((uint32_t)w.x == kxy && (int16_t)(w.y & 0xffff) == (int16_t)bz && w.w >= min_ptr) {
            *ptr_out = w.w;
            return (int)i;
        }
        if (w.z < 1 || (uint32_t)(w.z - 1) >= n_excess) return -1;
        i = n_buckets + (uint32_t)(w.z - 1);
    }
    return -1;
}

// the same from the block position alone
__device__ __forceinline__ int find_entry_in(const DEntry *entries, uint32_t n_buckets, uint32_t n_excess, int bx,
                                             int by, int bz, int min_ptr, int *ptr_out)
{
    if (!in_short_range(bx) || !in_short_range(by) || !in_short_range(bz)) return -1;
    return find_entry_from(entries, n_buckets, n_excess, hash_index(bx, by, bz, n_buckets - 1u), bx, by, bz, min_ptr,
                           ptr_out);
}

__device__ __forceinline__ int find_entry(const Vol &v, int bx, int by, int bz, int min_ptr, int *ptr_out)
{
    return find_entry_in(v.entries, v.n_buckets, v.n_excess, bx, by, bz, min_ptr, ptr_out);
}

__device__ __forceinline__ void cam_transform(const Cam &c, float X, float Y, float Z, float &x, float &y, float &z)
{
    x = ((c.M[0] * X + c.M[1] * Y) + c.M[2] * Z) + c.M[3];
    y = ((c.M[4] * X + c.M[5] * Y) + c.M[6] * Z) + c.M[7];
    z = ((c.M[8] * X + c.M[9] * Y) + c.M[10] * Z) + c.M[11];
}

// Pop up to one element per requesting lane from a stack whose height is
// *head (Sec. 4.2 "atomic subtraction on a stack of free voxel block
// indices"), with one atomic subtraction per wave.  Past exhaustion the
// height goes below zero and later pops get nothing; the visible-list kernel
// that follows every insertion clamps it back to zero before the stack takes
// any push.
__device__ __forceinline__ int32_t wave_pop(int32_t *head, const int32_t *stack, bool want)
{
    unsigned long long m = __ballot(want);
    if (m == 0) return -1;
    const int cnt = __popcll(m);
    const int leader = __ffsll((long long)m) - 1;
    int old = 0;
    if ((int)lane_id() == leader) old = atomicSub(head, cnt);
    old = __shfl(old, leader);
    const int take = old < 0 ? 0 : (old < cnt ? old : cnt);
    const int r = (int)rank_in(m);
    if (want && r < take) return stack[old - 1 - r];
    return -1;
}

// Insert a key into the per-frame request set (open addressing, linear
// probing); the lane that adds it appends it to the request list.
__device__ __forceinline__ void request_block(const Vol &v, int bx, int by, int bz)
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
__device__ __forceinline__ bool block_in_frustum(const Vol &v, const Cam &c, int bx, int by, int bz)
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

// Previous visible list entry i (Sec. 4.2, part 3): a block with a device
// block that is not marked yet stays visible while it is in view.  Rays of
// the same frame may mark it concurrently; both write kVisTouched.
__device__ __forceinline__ void keep_in_view(const Vol &v, const Cam &c, uint32_t i)
{
    const int e = v.vlist[i];
    const int4 w = load_entry(v.entries, (uint32_t)e);
    if (w.w < 0 || v.vis[e] != 0) return;
    const int bx = (int16_t)(w.x & 0xffff), by = (int16_t)((uint32_t)w.x >> 16), bz = (int16_t)(w.y & 0xffff);
    if (block_in_frustum(v, c, bx, by, bz)) v.vis[e] = kVisTouched;
}


// ============================================================================
// kernel bodies (each launch wraps one; blockIdx.x / gridDim.x index the work
// of one volume, so a batched launch may use blockIdx.y for the volume)
// ============================================================================
// ============================================================================
// allocation, part 1: segments, probes, marks, requests; the previous
// visible list's frustum re-test (part 3) in the workgroups past the image
// ============================================================================
// write_depth: keep the converted depth map (integration reads it)
template <int FMT>
__device__ __forceinline__ void alloc_rays_body(const Vol &v, const Cam &c, const void *din, bool write_depth)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p == 0) {
        Ctrl *C = v.ctrl;
        C->sweep_req = 0u;
        C->n_new = 0u;
        C->n_swapped_in = 0u;
        C->n_swap_cand = 0u;
    }
    const int W = c.W, H = c.H;
    const int pix_groups = (W * H + 255) / 256;
    if ((int)blockIdx.x >= pix_groups) {
        // the workgroups past the image re-test the previous visible list
        // (its length is still in n_vis, cleared by the insertion kernel)
        const uint32_t np = v.ctrl->n_vis;
        const uint32_t stride = (gridDim.x - (uint32_t)pix_groups) * 256u;
        for (uint32_t i = (blockIdx.x - (uint32_t)pix_groups) * 256u + threadIdx.x; i < np; i += stride)
            keep_in_view(v, c, i);
        return;
    }
    if (p >= W * H) return;
    float d;
    if (FMT == TF_DEPTH_U16_MM)
        d = (float)reinterpret_cast<const uint16_t *>(din)[p] / 1000.0f;   // Sec. 4 depth ingest
    else
        d = reinterpret_cast<const float *>(din)[p];
    if (write_depth) v.depth[p] = d;
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
            if (ptr >= 0)
                v.vis[e] = kVisTouched;
            else if (v.host_has)
                request_block(v, bx, by, bz);   // swapped out: revive with a fresh device block (Sec. 5)
        } else {
            request_block(v, bx, by, bz);
        }
    }
}

// ============================================================================
// allocation, part 2: insertion
// ============================================================================
__device__ __forceinline__ void insert_body(const Vol &v, const Cam &c)
{
    const uint32_t lane = lane_id();
    const uint32_t gwave = (blockIdx.x * 256u + threadIdx.x) / kWave;
    const uint32_t nwaves = gridDim.x * (256u / kWave);
    // the request count and this wave's first requests load together (the
    // list has max_req slots; those past the count are not used)
    uint32_t n = v.ctrl->n_req;
    const uint32_t first = gwave * kWave;
    Req rq = {};
    if (first + lane < v.max_req) rq = v.reqs[first + lane];
    if (n > v.max_req) n = v.max_req;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        v.ctrl->sweep_req = v.ctrl->req_overflow;
        v.ctrl->req_overflow = 0u;
        v.ctrl->n_vis = 0u;   // the compaction's counter (the previous list is re-tested)
    }

    for (uint32_t base = first; base < n; base += nwaves * kWave) {
        const uint32_t i = base + lane;
        const bool active = i < n;
        int bx = 0, by = 0, bz = 0;
        if (active) {
            if (base != first) rq = v.reqs[i];
            v.reqset[rq.slot] = 0ull;
            unpack_key(rq.key, bx, by, bz);
        }
        // a request for a swapped-out block revives its entry (Sec. 5)
        int revive = -1;
        if (active && v.host_has) {
            int pp;
            const int e = find_entry(v, bx, by, bz, kPtrSwapped, &pp);
            if (e >= 0 && pp == kPtrSwapped) revive = e;
        }
        // the bucket claim and the block pop go out together; a claim whose
        // pop comes back empty (blocks exhausted) is released
        const uint32_t h = hash_index(bx, by, bz, v.n_buckets - 1u);
        int prev = kPtrClaimed;
        if (active && revive < 0) prev = atomicCAS(&v.entries[h].ptr, kPtrEmpty, kPtrClaimed);
        const int32_t blk = wave_pop(&v.ctrl->free_blocks, v.free_blocks, active);
        if (active && blk < 0) atomicOr(&v.ctrl->flags, TF_FLAG_BLOCKS_EXHAUSTED);
        int entry = -1;
        bool need_excess = false;
        const unsigned long long posw = (unsigned long long)(uint16_t)bx | ((unsigned long long)(uint16_t)by << 16) |
                                        ((unsigned long long)(uint16_t)bz << 32);
        if (active && blk >= 0 && revive >= 0) {
            v.entries[revive].ptr = blk;
            entry = revive;
        } else if (active && blk >= 0) {
            if (prev == kPtrEmpty) {
                *reinterpret_cast<unsigned long long *>(&v.entries[h]) = posw;
                v.entries[h].ptr = blk;
                entry = (int)h;
            } else {
                need_excess = true;
            }
        } else if (active && revive < 0 && prev == kPtrEmpty) {
            v.entries[h].ptr = kPtrEmpty;
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
                int32_t old = 0;   // first guess: the bucket has no chain yet
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
            if (revive < 0) {
                atomicOr(&v.occ[h >> 5], 1u << (h & 31u));
                atomicOr(&v.brick[brick_word(bx, by, bz)], brick_bit(bx, by, bz));
            }
            if (revive < 0 && v.alist) {
                // submap volumes keep a list of their allocated blocks (no swapping there)
                const uint32_t ai = atomicAdd(&v.ctrl->n_alloc, 1u);
                v.alist[ai] = make_int4((int)((uint32_t)(uint16_t)bx | ((uint32_t)(uint16_t)by << 16)), bz, blk, entry);
            }
        }
        // initialise each new block (Sec. 3.1: sdf 32767, weight 0) with the whole wave
        unsigned long long m = __ballot(entry >= 0);
        const unsigned long long mi = __ballot(entry >= 0 && revive < 0);
        if (lane == 0 && mi) atomicAdd(&v.ctrl->n_new, (uint32_t)__popcll(mi));
        while (m) {
            const int l = __ffsll((long long)m) - 1;
            m &= m - 1;
            const int b = __shfl(blk, l);
            uint8_t *dst = v.voxels + (size_t)b * kBlockBytes;
            reinterpret_cast<uint4 *>(dst)[lane] = make_uint4(0x7fff7fffu, 0x7fff7fffu, 0x7fff7fffu, 0x7fff7fffu);
            reinterpret_cast<uint2 *>(dst + 1024)[lane] = make_uint2(0u, 0u);
        }
    }

}

// ============================================================================
// allocation, part 3b: compaction of the marks into the visible list
// ============================================================================
__device__ __forceinline__ void visible_body(const Vol &v)
{
    const uint32_t lane = lane_id();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        Ctrl *C = v.ctrl;
        C->tot_req += C->n_req < v.max_req ? C->n_req : v.max_req;
        C->tot_new += C->n_new;
        C->n_req = 0u;
        C->frames += 1u;
        if (v.alist) C->n_marked = C->n_alloc;   // the marking kernel has run on the new blocks
        // pops past exhaustion leave the stack heights below zero
        if (C->free_blocks < 0) C->free_blocks = 0;
        if (C->free_excess < 0) C->free_excess = 0;
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
    // a workgroup takes 256 chunks of 16 flags at a time: a scan within each
    // wave, the four wave totals combined in LDS, one counter atomic per
    // workgroup step (same-address device atomics serialise)
    __shared__ uint32_t wtot[4], wbase;
    const uint32_t wv = threadIdx.x / kWave;
    const uint32_t nchunks = (v.n_entries + 15u) / 16u;
    for (uint32_t cb = blockIdx.x * 256u; cb < nchunks; cb += gridDim.x * 256u) {
        const uint32_t ch = cb + threadIdx.x;
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
        if (lane == kWave - 1) wtot[wv] = incl;
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint32_t total = wtot[0] + wtot[1] + wtot[2] + wtot[3];
            wbase = total ? atomicAdd(&v.ctrl->n_vis, total) : 0u;
        }
        __syncthreads();
        uint32_t pos = wbase + incl - cnt;
        for (uint32_t k = 0; k < wv; ++k) pos += wtot[k];
        if (cnt) {
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if ((words[j >> 2] >> (8 * (j & 3))) & 0xffu) v.vlist[pos++] = (int32_t)(ch * 16u + (uint32_t)j);
            reinterpret_cast<uint4 *>(v.vis)[ch] = make_uint4(0u, 0u, 0u, 0u);
        }
        __syncthreads();   // wtot and wbase are rewritten by the next step
    }
}

// ============================================================================
// integration (Sec. 4.3)
// ============================================================================
// Lane (lx, ly) = (lane >> 3, lane & 7) owns the 8 voxels lz = 0..7 of one
// column; the device in-block order lz + 8 ly + 64 lx puts them in 16
// contiguous bytes of SDF and 8 of weight, so a wave moves a block in one
// dwordx4 and one dwordx2 access per lane.
// NT threads per workgroup; rcp_w (260 floats) and wg_cols are the caller's
// LDS; dry: compute every update but store nothing (timing probes).
// bin: the camera is also the next raycast's (the allocation view): each
// block's search-range record goes to slot i of the record list (an empty
// record for a block off the image) and, by the wave's lanes, to the bin of
// every 16x16 tile its box covers -- the work of k_range_bin over the visible
// list, done while the block's voxels load.
__device__ __forceinline__ bool block_record_wave(const Vol &v, const Cam &c, int bx, int by, int bz, Rec &r);

template <int NT>
__device__ __forceinline__ void integrate_body(const Vol &v, const Cam &c, float *rcp_w, uint32_t *wg_cols, bool dry,
                                               bool bin = false)
{
    for (int k = threadIdx.x; k < 260; k += NT) rcp_w[k] = k ? 1.0f / (float)k : 0.0f;
    __syncthreads();
    const uint32_t lane = lane_id();
    const uint32_t gwave = (blockIdx.x * (uint32_t)NT + threadIdx.x) / kWave;
    const uint32_t nwaves = gridDim.x * ((uint32_t)NT / kWave);
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
        if (bin) v.ctrl->n_rec = nvis;
    }
    uint32_t cols = 0;
    const int ntx = (c.W + kTile - 1) / kTile;

    for (uint32_t i = gwave; i < nvis; i += nwaves) {
        const int e = v.vlist[i];
        const int4 w = load_entry(v.entries, (uint32_t)e);
        const int ptr = w.w;
        const int bx = (int16_t)(w.x & 0xffff), by = (int16_t)((uint32_t)w.x >> 16), bz = (int16_t)(w.y & 0xffff);
        if (ptr < 0) {
            if (bin && lane == 0) {
                Rec r = {};
                r.x0 = 1;   // empty box
                v.recs[i] = r;
            }
            continue;
        }
        uint8_t *blk = v.voxels + (size_t)ptr * kBlockBytes;
        uint4 s8 = reinterpret_cast<const uint4 *>(blk)[lane];
        uint2 w8 = reinterpret_cast<const uint2 *>(blk + 1024)[lane];
        if (bin) {
            Rec r;
            const bool emit = block_record_wave(v, c, bx, by, bz, r);
            if (!emit) {
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
            r.ptr = ptr;
            r.pad2 = 0;
            if (lane == 0) v.recs[i] = r;
            if (emit) {
                const int tx0 = r.x0 / kTile, tx1 = r.x1 / kTile, ty0 = r.y0 / kTile, ty1 = r.y1 / kTile;
                const int nx = tx1 - tx0 + 1, cnt = nx * (ty1 - ty0 + 1);
                for (int k = (int)lane; k < cnt; k += kWave) {
                    const int t = (ty0 + k / nx) * ntx + tx0 + k % nx;
                    const int sl = atomicAdd(&v.bin_count[t], 1);
                    if (sl < kBinCap) v.bins[(size_t)t * kBinCap + sl] = r;
                }
            }
        }
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
        if (changed && !dry) {
            reinterpret_cast<uint4 *>(blk)[lane] = make_uint4(sw[0], sw[1], sw[2], sw[3]);
            reinterpret_cast<uint2 *>(blk + 1024)[lane] = make_uint2(ww[0], ww[1]);
            ++cols;
        }
    }
    // per-workgroup count of written columns (no cross-workgroup atomics)
    if (threadIdx.x == 0) *wg_cols = 0;
    __syncthreads();
    if (cols && !dry) atomicAdd(wg_cols, cols);
    __syncthreads();
    if (threadIdx.x == 0 && *wg_cols) v.acc_cols[blockIdx.x] += *wg_cols;
}

// ============================================================================
// search range (Sec. 4.4): the projected box and camera-z range of a block
// ============================================================================
// Box of the cube with voxel corner (x0, y0, z0) and edge `span` voxels, seen
// by camera matrix M (12 floats) with the intrinsics of c: the pixel box
// (floor/ceil, clipped to the image) of the projections of the cube's part
// beyond the near plane -- its corners there and the points where its edges
// cross the plane -- and the corners' camera-z range, starting at the plane
// for a cube that reaches closer.  False when the cube lies entirely closer
// than the plane or off the image.
__device__ __forceinline__ bool cube_record(const float *M, const Cam &c, float voxel, int x0, int y0, int z0,
                                            int span, Rec &r)
{
    float xs[8], ys[8], zs[8];
    float zlo = __builtin_inff(), zhi = -__builtin_inff();
    for (int k = 0; k < 8; ++k) {
        const int px = x0 + span * (k & 1), py = y0 + span * ((k >> 1) & 1), pz = z0 + span * (k >> 2);
        const float X = (float)px * voxel, Y = (float)py * voxel, Z = (float)pz * voxel;
        xs[k] = ((M[0] * X + M[1] * Y) + M[2] * Z) + M[3];
        ys[k] = ((M[4] * X + M[5] * Y) + M[6] * Z) + M[7];
        zs[k] = ((M[8] * X + M[9] * Y) + M[10] * Z) + M[11];
        if (zs[k] < zlo) zlo = zs[k];
        if (zs[k] > zhi) zhi = zs[k];
    }
    if (zhi < kZNear) return false;
    float umin = __builtin_inff(), umax = -__builtin_inff(), vmin = __builtin_inff(), vmax = -__builtin_inff();
    for (int k = 0; k < 8; ++k) {
        if (zs[k] < kZNear) continue;
        const float rz = 1.0f / zs[k];
        const float u = (c.fx * xs[k]) * rz + c.cx;
        const float vv = (c.fy * ys[k]) * rz + c.cy;
        umin = u < umin ? u : umin;
        umax = u > umax ? u : umax;
        vmin = vv < vmin ? vv : vmin;
        vmax = vv > vmax ? vv : vmax;
    }
    if (zlo < kZNear) {
        const float rzn = 1.0f / kZNear;
        for (int a = 0; a < 8; ++a)
            for (int bit = 1; bit < 8; bit <<= 1) {
                if (a & bit) continue;
                const int b = a | bit;   // the edge from corner a to corner b
                if ((zs[a] < kZNear) == (zs[b] < kZNear)) continue;
                const float t = (kZNear - zs[a]) / (zs[b] - zs[a]);
                const float xe = xs[a] + t * (xs[b] - xs[a]);
                const float ye = ys[a] + t * (ys[b] - ys[a]);
                const float u = (c.fx * xe) * rzn + c.cx;
                const float vv = (c.fy * ye) * rzn + c.cy;
                umin = u < umin ? u : umin;
                umax = u > umax ? u : umax;
                vmin = vv < vmin ? vv : vmin;
                vmax = vv > vmax ? vv : vmax;
            }
        zlo = kZNear;
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

__device__ __forceinline__ bool block_record(const Vol &v, const Cam &c, int bx, int by, int bz, Rec &r)
{
    return cube_record(c.M, c, v.voxel, 8 * bx, 8 * by, 8 * bz, 8, r);
}

// block_record by a whole wave (every lane active, the same block): lane l
// takes corner l & 7, and min / max go round each 8-lane group by shuffles
// (order-free, so the record is the serial one); a block reaching in front of
// the near plane takes the serial form for its edge crossings.  Every lane
// returns the same record.
__device__ __forceinline__ bool block_record_wave(const Vol &v, const Cam &c, int bx, int by, int bz, Rec &r)
{
    const int k = (int)(lane_id() & 7u);
    const int px = 8 * (bx + (k & 1)), py = 8 * (by + ((k >> 1) & 1)), pz = 8 * (bz + (k >> 2));
    const float *M = c.M;
    const float X = (float)px * v.voxel, Y = (float)py * v.voxel, Z = (float)pz * v.voxel;
    const float xs = ((M[0] * X + M[1] * Y) + M[2] * Z) + M[3];
    const float ys = ((M[4] * X + M[5] * Y) + M[6] * Z) + M[7];
    const float zs = ((M[8] * X + M[9] * Y) + M[10] * Z) + M[11];
    const bool front = !(zs < kZNear);
    const float rz = 1.0f / (front ? zs : 1.0f);
    const float u = (c.fx * xs) * rz + c.cx;
    const float vv = (c.fy * ys) * rz + c.cy;
    float zlo = zs, zhi = zs;
    float umin = front ? u : __builtin_inff(), umax = front ? u : -__builtin_inff();
    float vmin = front ? vv : __builtin_inff(), vmax = front ? vv : -__builtin_inff();
#pragma unroll
    for (int d = 1; d < 8; d <<= 1) {
        float o = __shfl_xor(zlo, d);
        zlo = o < zlo ? o : zlo;
        o = __shfl_xor(zhi, d);
        zhi = o > zhi ? o : zhi;
        o = __shfl_xor(umin, d);
        umin = o < umin ? o : umin;
        o = __shfl_xor(umax, d);
        umax = o > umax ? o : umax;
        o = __shfl_xor(vmin, d);
        vmin = o < vmin ? o : vmin;
        o = __shfl_xor(vmax, d);
        vmax = o > vmax ? o : vmax;
    }
    if (zhi < kZNear) return false;
    if (zlo < kZNear) return block_record(v, c, bx, by, bz, r);
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

// ============================================================================
// trilinear reads (Sec. 4.4)
// ============================================================================
__device__ __forceinline__ int block_of(float X) { return ((int)floorf(X)) >> 3; }

// the 2x2x2 cell of a trilinear read: corner block pointers, in-block voxel
// indices (lz + 8 ly + 64 lx) and the interpolation fractions
struct Cell {
    int p[8], j[8];
    float tx, ty, tz;
};

// in-block indices of the cell's corners: base voxel (ix, iy, iz), corner c
// at + (c & 1, c >> 1 & 1, c >> 2); a step across a block face (local index
// 7, flagged by sx, sy, sz) wraps to index 0 of the neighbouring block
__device__ __forceinline__ void cell_index(int ix, int iy, int iz, bool sx, bool sy, bool sz, int (&j)[8])
{
    j[0] = (iz & 7) + 8 * (iy & 7) + 64 * (ix & 7);
    const int dx = sx ? -448 : 64, dy = sy ? -56 : 8, dz = sz ? -7 : 1;
    j[1] = j[0] + dx;
    j[2] = j[0] + dy;
    j[3] = j[1] + dy;
    j[4] = j[0] + dz;
    j[5] = j[1] + dz;
    j[6] = j[2] + dz;
    j[7] = j[3] + dz;
}

// absent voxels read 1.0 (bit c of `present` clear: corner c has no block);
// lerp a + (b - a) t along x, then y, then z
__device__ __forceinline__ float cell_lerp(uint32_t present, const int16_t (&s)[8], float tx, float ty, float tz)
{
    float f[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) f[c] = ((present >> c) & 1u) ? (float)s[c] * (1.0f / 32767.0f) : 1.0f;
    const float c00 = f[0] + (f[1] - f[0]) * tx;
    const float c10 = f[2] + (f[3] - f[2]) * tx;
    const float c01 = f[4] + (f[5] - f[4]) * tx;
    const float c11 = f[6] + (f[7] - f[6]) * tx;
    const float c0 = c00 + (c10 - c00) * ty;
    const float c1 = c01 + (c11 - c01) * ty;
    return c0 + (c1 - c0) * tz;
}

__device__ __forceinline__ float cell_interp(const Cell &C, const int16_t (&s)[8])
{
    uint32_t present = 0u;
#pragma unroll
    for (int c = 0; c < 8; ++c) present |= (C.p[c] >= 0 ? 1u : 0u) << c;
    return cell_lerp(present, s, C.tx, C.ty, C.tz);
}

}  // namespace

}  // namespace tsdf
