// tsdf_api.hip -- host side of libtsdf: argument validation, workspace
// carving, camera constants and the C ABI declared in include/tsdf.h.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "tsdf.h"
#include "tsdf_ctx.h"
#include "tsdf_internal.h"

using namespace tsdf;

namespace tsdf {

// camera constants of a world->camera matrix M (row-major 4x4) and intrinsics
void make_cam(const float *M, const tf_intrinsics *K, Cam &c)
{
    for (int r = 0; r < 3; ++r)
        for (int j = 0; j < 4; ++j) c.M[4 * r + j] = M[4 * r + j];
    // inverse of the rigid transform: [R^T | -R^T t], -R^T t in double
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) c.Ri[3 * i + j] = M[4 * j + i];
    for (int i = 0; i < 3; ++i) {
        double s = ((double)M[i] * (double)M[3] + (double)M[4 + i] * (double)M[7]) + (double)M[8 + i] * (double)M[11];
        c.ti[i] = (float)(-s);
    }
    c.fx = K->fx;
    c.fy = K->fy;
    c.cx = K->cx;
    c.cy = K->cy;
    c.W = K->width;
    c.H = K->height;
}

}  // namespace tsdf

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool is_pow2(uint32_t x) { return x && !(x & (x - 1)); }

bool params_ok(const tf_params *p)
{
    if (!p) return false;
    if (!(p->voxel_size > 0.0f) || !(p->mu > 0.0f)) return false;
    if (p->max_w < 1 || p->max_w > 255) return false;
    if (!is_pow2(p->n_buckets) || p->n_buckets < 16u || p->n_buckets > (1u << 26)) return false;
    if (p->n_excess < 1u || p->n_excess > (1u << 26)) return false;
    if (p->n_blocks < 1u || p->n_blocks > (1u << 24)) return false;
    if (p->max_width < 1u || p->max_width > 8192u || p->max_height < 1u || p->max_height > 8192u) return false;
    if (p->swap_transfer_blocks > (1u << 20)) return false;
    return true;
}

Layout make_layout(const tf_params *p)
{
    Layout L = {};
    const size_t n_entries = (size_t)p->n_buckets + p->n_excess;
    const size_t n_vis = (n_entries + 15) & ~(size_t)15;
    L.max_req = p->n_blocks;
    uint32_t rs = 1024;
    while (rs < 2u * L.max_req) rs <<= 1;
    L.reqset_size = rs;
    L.max_tiles = ((p->max_width + kTile - 1) / kTile) * ((p->max_height + kTile - 1) / kTile);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    L.ctrl = take(sizeof(Ctrl));
    L.entries = take(n_entries * sizeof(DEntry));
    L.vis = take(n_vis);
    L.free_blocks = take((size_t)p->n_blocks * 4);
    L.free_excess = take((size_t)p->n_excess * 4);
    L.vlist = take((size_t)p->n_blocks * 4);
    L.reqset = take((size_t)rs * 8);
    L.reqs = take((size_t)L.max_req * sizeof(Req));
    L.ret = take((size_t)L.max_req * 4);
    L.depth = take((size_t)p->max_width * p->max_height * 4);
    L.recs = take((size_t)p->n_blocks * sizeof(Rec));
    L.bins = take((size_t)L.max_tiles * kBinCap * sizeof(Rec));
    L.bin_count = take((size_t)L.max_tiles * 4);
    L.acc_cols = take((size_t)kIntegrateGrid * 8);
    L.acc_hits = take((size_t)L.max_tiles * 8);
    L.occ = take((size_t)p->n_buckets / 8);
    L.brick = take((size_t)kBrickWords * 4);
    if (p->swap_transfer_blocks) {
        L.host_has = take(n_vis);
        L.xfer_idx = take((size_t)p->swap_transfer_blocks * 4);
        L.xfer_vox = take((size_t)p->swap_transfer_blocks * kBlockBytes);
        L.xfer_host = take((size_t)p->swap_transfer_blocks * kBlockBytes);
        L.xfer_pend = take((size_t)p->swap_transfer_blocks * 4);
        L.swap_chunks = take(((n_entries + kSwapChunk - 1) / kSwapChunk) * 4);
    }
    L.voxels = take((size_t)p->n_blocks * kBlockBytes);
    L.total = o;
    return L;
}

bool intr_ok(const tf_ctx *ctx, const tf_intrinsics *K)
{
    if (!K) return false;
    if (K->width < 1 || K->height < 1) return false;
    if ((uint32_t)K->width > ctx->p.max_width || (uint32_t)K->height > ctx->p.max_height) return false;
    if (!(K->fx > 0.0f) || !(K->fy > 0.0f)) return false;
    if (!(K->cx == K->cx) || !(K->cy == K->cy)) return false;
    return true;
}

bool pose_ok(const float *M)
{
    if (!M) return false;
    for (int i = 0; i < 16; ++i)
        if (!(M[i] == M[i]) || M[i] > 1e30f || M[i] < -1e30f) return false;
    return true;
}

int hip_status(hipError_t e) { return e == hipSuccess ? TF_OK : TF_E_HIP; }

hipError_t harvest(Profiler &P, int k, int slot)
{
    if (!P.pending[k][slot]) return hipSuccess;
    hipError_t e = hipEventSynchronize(P.ev[k][slot][1]);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, P.ev[k][slot][0], P.ev[k][slot][1]);
    P.pending[k][slot] = false;
    if (e != hipSuccess) return e;
    P.ms[k] += ms;
    P.launches[k] += 1;
    return hipSuccess;
}

// brackets one kernel launch with events when the profiler is on
struct Timed {
    Profiler &P;
    int k, slot;
    hipStream_t s;
    Timed(tf_ctx *ctx, int kind, hipStream_t st) : P(ctx->prof), k(kind), slot(-1), s(st)
    {
        if (!P.on || !((P.mask >> k) & 1u)) return;
        if (P.seen[k]++ % P.every) return;
        slot = P.next[k];
        if (harvest(P, k, slot) != hipSuccess) {
            slot = -1;
            return;
        }
        if (hipEventRecord(P.ev[k][slot][0], s) != hipSuccess) slot = -1;
    }
    ~Timed()
    {
        if (slot < 0) return;
        if (hipEventRecord(P.ev[k][slot][1], s) == hipSuccess) {
            P.pending[k][slot] = true;
            P.next[k] = (slot + 1) % Profiler::R;
        }
    }
};

// swap-in after the visible list (Sec. 5): the device lists the visible
// entries whose host store holds data; the host takes the lowest entry
// indices up to the transfer capacity, gathers their blocks into the pinned
// transfer buffer and sends it; one kernel fuses them into the device blocks.
hipError_t swap_in(tf_ctx *ctx, hipStream_t s)
{
    Vol &v = ctx->v;
    hipError_t e = launch_swap_candidates(v, s);
    Ctrl c;
    if (e == hipSuccess) e = hipMemcpyAsync(&c, v.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess || c.n_swap_cand == 0) return e;
    ctx->cand.resize(c.n_swap_cand);
    e = hipMemcpyAsync(ctx->cand.data(), v.ret, (size_t)c.n_swap_cand * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    std::sort(ctx->cand.begin(), ctx->cand.end());
    const uint32_t T = ctx->p.swap_transfer_blocks;
    const uint32_t m = c.n_swap_cand < T ? c.n_swap_cand : T;
    if (c.n_swap_cand > T) ctx->host_flags |= TF_FLAG_TRANSFER_OVERFLOW;
    int32_t *hidx = (int32_t *)ctx->h_transfer;
    uint8_t *hvox = (uint8_t *)ctx->h_transfer + (size_t)T * 4;
    const uint8_t *store = (const uint8_t *)ctx->h_store;
    for (uint32_t k = 0; k < m; ++k) {
        const int32_t idx = ctx->cand[k];
        hidx[k] = idx;
        memcpy(hvox + (size_t)k * kBlockBytes, store + (size_t)idx * kBlockBytes, kBlockBytes);
        ctx->host_has[idx] = 0;
    }
    e = hipMemcpyAsync(v.xfer_idx, hidx, (size_t)m * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(v.xfer_vox, hvox, (size_t)m * kBlockBytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_swap_merge(v, m, s);
    return e;
}

}  // namespace

extern "C" {

size_t tf_workspace_bytes(const tf_params *p)
{
    if (!params_ok(p)) return 0;
    return make_layout(p).total;
}

size_t tf_host_store_bytes(const tf_params *p)
{
    if (!params_ok(p) || !p->swap_transfer_blocks) return 0;
    return ((size_t)p->n_buckets + p->n_excess) * kBlockBytes;
}

size_t tf_host_transfer_bytes(const tf_params *p)
{
    if (!params_ok(p) || !p->swap_transfer_blocks) return 0;
    return (size_t)p->swap_transfer_blocks * (kBlockBytes + 4);
}

int tf_create(const tf_params *p, void *d_workspace, size_t bytes, void *h_store, void *h_transfer,
              tf_stream stream, tf_ctx **out)
{
    if (!out) return TF_E_INVAL;
    *out = nullptr;
    if (!params_ok(p) || !d_workspace) return TF_E_INVAL;
    if (((uintptr_t)d_workspace & 255u) != 0) return TF_E_INVAL;
    if (p->swap_transfer_blocks && (!h_store || !h_transfer)) return TF_E_INVAL;
    Layout L = make_layout(p);
    if (bytes < L.total) return TF_E_SPACE;
    tf_ctx *ctx = new (std::nothrow) tf_ctx();
    if (!ctx) return TF_E_INVAL;
    ctx->p = *p;
    ctx->L = L;
    ctx->ws = (uint8_t *)d_workspace;
    ctx->h_store = h_store;
    ctx->h_transfer = h_transfer;
    ctx->have_alloc = false;
    ctx->bins_pending = false;
    ctx->host_flags = 0;
    if (p->swap_transfer_blocks) ctx->host_has.assign((size_t)p->n_buckets + p->n_excess, 0);
    Vol &v = ctx->v;
    uint8_t *b = ctx->ws;
    v.entries = (DEntry *)(b + L.entries);
    v.vis = b + L.vis;
    v.free_blocks = (int32_t *)(b + L.free_blocks);
    v.free_excess = (int32_t *)(b + L.free_excess);
    v.voxels = b + L.voxels;
    v.vlist = (int32_t *)(b + L.vlist);
    v.reqset = (unsigned long long *)(b + L.reqset);
    v.reqs = (Req *)(b + L.reqs);
    v.ret = (int32_t *)(b + L.ret);
    v.depth = (float *)(b + L.depth);
    v.recs = (Rec *)(b + L.recs);
    v.bins = (Rec *)(b + L.bins);
    v.bin_count = (int32_t *)(b + L.bin_count);
    v.ctrl = (Ctrl *)(b + L.ctrl);
    v.acc_cols = (unsigned long long *)(b + L.acc_cols);
    v.acc_hits = (unsigned long long *)(b + L.acc_hits);
    v.occ = (uint32_t *)(b + L.occ);
    v.brick = (uint32_t *)(b + L.brick);
    v.host_has = p->swap_transfer_blocks ? b + L.host_has : nullptr;
    v.xfer_idx = p->swap_transfer_blocks ? (int32_t *)(b + L.xfer_idx) : nullptr;
    v.xfer_vox = p->swap_transfer_blocks ? b + L.xfer_vox : nullptr;
    v.xfer_host = p->swap_transfer_blocks ? b + L.xfer_host : nullptr;
    v.xfer_pend = p->swap_transfer_blocks ? (int32_t *)(b + L.xfer_pend) : nullptr;
    v.swap_chunks = p->swap_transfer_blocks ? (uint32_t *)(b + L.swap_chunks) : nullptr;
    v.alist = nullptr;
    v.n_buckets = p->n_buckets;
    v.n_excess = p->n_excess;
    v.n_entries = p->n_buckets + p->n_excess;
    v.n_blocks = p->n_blocks;
    v.reqset_mask = L.reqset_size - 1;
    v.max_req = L.max_req;
    v.transfer_blocks = p->swap_transfer_blocks;
    v.voxel = p->voxel_size;
    v.mu = p->mu;
    v.max_w = p->max_w;
    int st = tf_reset(ctx, stream);
    if (st != TF_OK) {
        delete ctx;
        return st;
    }
    *out = ctx;
    return TF_OK;
}

int tf_destroy(tf_ctx *ctx)
{
    if (!ctx) return TF_E_INVAL;
    if (ctx->prof.created) {
        for (int k = 0; k < TF_K_COUNT; ++k)
            for (int r = 0; r < Profiler::R; ++r) {
                if (ctx->prof.pending[k][r]) (void)hipEventSynchronize(ctx->prof.ev[k][r][1]);
                (void)hipEventDestroy(ctx->prof.ev[k][r][0]);
                (void)hipEventDestroy(ctx->prof.ev[k][r][1]);
            }
    }
    delete ctx;
    return TF_OK;
}

int tf_profile_enable(tf_ctx *ctx, int on)
{
    if (!ctx) return TF_E_INVAL;
    Profiler &P = ctx->prof;
    if (on && !P.created) {
        for (int k = 0; k < TF_K_COUNT; ++k)
            for (int r = 0; r < Profiler::R; ++r)
                for (int j = 0; j < 2; ++j)
                    if (hipEventCreate(&P.ev[k][r][j]) != hipSuccess) return TF_E_HIP;
        P.created = true;
    }
    P.on = on != 0;
    return TF_OK;
}

int tf_profile_select(tf_ctx *ctx, uint32_t class_mask, uint32_t every)
{
    if (!ctx || every < 1) return TF_E_INVAL;
    ctx->prof.mask = class_mask;
    ctx->prof.every = every;
    for (int k = 0; k < TF_K_COUNT; ++k) ctx->prof.seen[k] = 0;
    return TF_OK;
}

int tf_profile_read(tf_ctx *ctx, tf_profile *h_out, int reset)
{
    if (!ctx || !h_out) return TF_E_INVAL;
    Profiler &P = ctx->prof;
    if (P.created)
        for (int k = 0; k < TF_K_COUNT; ++k)
            for (int r = 0; r < Profiler::R; ++r)
                if (harvest(P, k, r) != hipSuccess) return TF_E_HIP;
    memset(h_out, 0, sizeof(*h_out));
    for (int k = 0; k < TF_K_COUNT; ++k) {
        h_out->launches[k] = P.launches[k];
        h_out->ms[k] = P.ms[k];
        if (reset) {
            P.launches[k] = 0;
            P.ms[k] = 0.0;
        }
    }
    return TF_OK;
}

int tf_reset(tf_ctx *ctx, tf_stream stream)
{
    if (!ctx) return TF_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_init(ctx->v, s);
    if (e == hipSuccess) e = launch_clear_bins(ctx->v.bin_count, ctx->L.max_tiles, s);
    if (e == hipSuccess) e = launch_clear_bins((int32_t *)ctx->v.acc_hits, 2 * ctx->L.max_tiles, s);
    ctx->have_alloc = false;
    ctx->bins_pending = false;
    ctx->host_flags = 0;
    std::fill(ctx->host_has.begin(), ctx->host_has.end(), (uint8_t)0);
    return hip_status(e);
}

int tf_alloc_and_visible(tf_ctx *ctx, const void *d_depth, int depth_format, const tf_intrinsics *intr,
                         const float pose_w2c[16], tf_stream stream)
{
    if (!ctx || !d_depth || !intr_ok(ctx, intr) || !pose_ok(pose_w2c)) return TF_E_INVAL;
    if (depth_format != TF_DEPTH_F32_M && depth_format != TF_DEPTH_U16_MM) return TF_E_INVAL;
    Cam c;
    make_cam(pose_w2c, intr, c);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (ctx->bins_pending) {
        // records of the previous visible list that no raycast consumed
        e = launch_clear_bins(ctx->v.bin_count, ctx->L.max_tiles, s, ctx->v.ctrl);
        if (e != hipSuccess) return TF_E_HIP;
        ctx->bins_pending = false;
    }
    {
        Timed t(ctx, TF_K_ALLOC_RAYS, s);
        e = launch_alloc_rays(ctx->v, c, d_depth, depth_format, s);
    }
    if (e == hipSuccess) {
        Timed t(ctx, TF_K_INSERT, s);
        e = launch_insert(ctx->v, c, s);
    }
    if (e == hipSuccess) {
        Timed t(ctx, TF_K_VISIBLE, s);
        e = launch_visible(ctx->v, s);
    }
    if (e == hipSuccess && ctx->p.swap_transfer_blocks) {
        Timed t(ctx, TF_K_SWAP, s);
        e = swap_in(ctx, s);
    }
    if (e != hipSuccess) return TF_E_HIP;
    ctx->have_alloc = true;
    ctx->alloc_intr = *intr;
    memcpy(ctx->alloc_pose, pose_w2c, sizeof(ctx->alloc_pose));
    ctx->alloc_depth = d_depth;
    ctx->alloc_fmt = depth_format;
    return TF_OK;
}

int tf_integrate(tf_ctx *ctx, const void *d_depth, int depth_format, const float pose_w2c[16], tf_stream stream)
{
    if (!ctx || !d_depth || !pose_ok(pose_w2c)) return TF_E_INVAL;
    if (depth_format != TF_DEPTH_F32_M && depth_format != TF_DEPTH_U16_MM) return TF_E_INVAL;
    if (!ctx->have_alloc) return TF_E_ORDER;
    hipStream_t s = (hipStream_t)stream;
    Cam c;
    make_cam(pose_w2c, &ctx->alloc_intr, c);
    Timed t(ctx, TF_K_INTEGRATE, s);
    if (d_depth != ctx->alloc_depth || depth_format != ctx->alloc_fmt) {
        hipError_t e = launch_depth_convert(ctx->v, d_depth, depth_format, c.W * c.H, s);
        if (e != hipSuccess) return TF_E_HIP;
        ctx->alloc_depth = d_depth;
        ctx->alloc_fmt = depth_format;
    }
    // the allocation's own pose: the raycast that follows will use the visible
    // list's search range, so integration bins it on the way
    const bool bin = !ctx->bins_pending && memcmp(pose_w2c, ctx->alloc_pose, sizeof(ctx->alloc_pose)) == 0;
    const hipError_t e = launch_integrate(ctx->v, c, bin, s);
    if (e != hipSuccess) return TF_E_HIP;
    if (bin) ctx->bins_pending = true;
    return TF_OK;
}

static bool same_view(const tf_ctx *ctx, const float *pose, const tf_intrinsics *K)
{
    if (!ctx->have_alloc) return false;
    if (memcmp(pose, ctx->alloc_pose, sizeof(ctx->alloc_pose)) != 0) return false;
    const tf_intrinsics &a = ctx->alloc_intr;
    return a.fx == K->fx && a.fy == K->fy && a.cx == K->cx && a.cy == K->cy && a.width == K->width &&
           a.height == K->height;
}

// The search-range bins of one raycast-kind call (consumed and cleared by it):
// those tf_integrate made for the allocation view when the call has that view,
// else k_range_bin's (after clearing unused integration bins)
static hipError_t bin_range(tf_ctx *ctx, const Cam &c, bool all, hipStream_t s)
{
    hipError_t e = hipSuccess;
    if (ctx->bins_pending) {
        ctx->bins_pending = false;
        if (!all) return hipSuccess;
        e = launch_clear_bins(ctx->v.bin_count, ctx->L.max_tiles, s, ctx->v.ctrl);
        if (e != hipSuccess) return e;
    }
    Timed t(ctx, TF_K_RANGE_BIN, s);
    return launch_range_bin(ctx->v, c, all, s);
}

int tf_raycast(tf_ctx *ctx, const float pose_w2c[16], const tf_intrinsics *intr, float *d_points,
               float *d_normals, tf_stream stream)
{
    if (!ctx || !intr_ok(ctx, intr) || !pose_ok(pose_w2c) || !d_points || !d_normals) return TF_E_INVAL;
    if ((((uintptr_t)d_points) & 15u) || (((uintptr_t)d_normals) & 15u)) return TF_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    Cam c;
    make_cam(pose_w2c, intr, c);
    const bool all = !same_view(ctx, pose_w2c, intr);
    const hipError_t e = bin_range(ctx, c, all, s);
    if (e != hipSuccess) return TF_E_HIP;
    Timed t(ctx, TF_K_RAYCAST, s);
    return hip_status(launch_raycast(ctx->v, c, all, (float4 *)d_points, (float4 *)d_normals, s));
}

int tf_range_image(tf_ctx *ctx, const float pose_w2c[16], const tf_intrinsics *intr, float *d_zmin, float *d_zmax,
                   tf_stream stream)
{
    if (!ctx || !intr_ok(ctx, intr) || !pose_ok(pose_w2c) || !d_zmin || !d_zmax) return TF_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    Cam c;
    make_cam(pose_w2c, intr, c);
    const hipError_t e = bin_range(ctx, c, !same_view(ctx, pose_w2c, intr), s);
    if (e != hipSuccess) return TF_E_HIP;
    return hip_status(launch_range_write(ctx->v, c, d_zmin, d_zmax, s));
}

int tf_swap_out(tf_ctx *ctx, tf_stream stream)
{
    if (!ctx) return TF_E_INVAL;
    if (!ctx->p.swap_transfer_blocks) return TF_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    Vol &v = ctx->v;
    Timed t(ctx, TF_K_SWAP, s);
    hipError_t e = launch_swap_select(v, s);
    Ctrl c;
    if (e == hipSuccess) e = hipMemcpyAsync(&c, v.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return TF_E_HIP;
    const uint32_t T = ctx->p.swap_transfer_blocks;
    const uint32_t m = c.n_swap_cand < T ? c.n_swap_cand : T;
    int32_t *hidx = (int32_t *)ctx->h_transfer;
    uint8_t *hvox = (uint8_t *)ctx->h_transfer + (size_t)T * 4;
    if (m) {
        e = launch_swap_gather(v, m, s);
        if (e == hipSuccess) e = hipMemcpyAsync(hidx, v.xfer_idx, (size_t)m * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(hvox, v.xfer_vox, (size_t)m * kBlockBytes, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return TF_E_HIP;
        uint8_t *store = (uint8_t *)ctx->h_store;
        // blocks whose host copy never came back in are fused with it (the
        // secondary integration, on the device, below); the others are copied
        std::vector<int32_t> &pend = ctx->cand;
        pend.clear();
        for (uint32_t k = 0; k < m; ++k) {
            const int32_t idx = hidx[k];
            if (ctx->host_has[idx])
                pend.push_back((int32_t)k);
            else
                memcpy(store + (size_t)idx * kBlockBytes, hvox + (size_t)k * kBlockBytes, kBlockBytes);
            ctx->host_has[idx] = 1;
        }
        const uint32_t np = (uint32_t)pend.size();
        if (np) {
            // the pinned buffer's blocks are consumed: stage the store copies
            // there (slot j), upload them with their transfer-buffer slots, fuse,
            // and bring the results back
            std::vector<int32_t> entry(np);
            for (uint32_t j = 0; j < np; ++j) {
                entry[j] = hidx[pend[j]];
                memcpy(hvox + (size_t)j * kBlockBytes, store + (size_t)entry[j] * kBlockBytes, kBlockBytes);
                hidx[j] = pend[j];
            }
            e = hipMemcpyAsync(v.xfer_pend, hidx, (size_t)np * 4, hipMemcpyHostToDevice, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(v.xfer_host, hvox, (size_t)np * kBlockBytes, hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = launch_swap_merge_out(v, np, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(hvox, v.xfer_host, (size_t)np * kBlockBytes, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) return TF_E_HIP;
            for (uint32_t j = 0; j < np; ++j)
                memcpy(store + (size_t)entry[j] * kBlockBytes, hvox + (size_t)j * kBlockBytes, kBlockBytes);
        }
    }
    e = launch_swap_release(v, m, s);
    return hip_status(e);
}

int tf_export_host_voxels(tf_ctx *ctx, const int32_t *h_entries, uint32_t n, int16_t *h_sdf, uint8_t *h_w,
                          uint8_t *h_has)
{
    if (!ctx || (n && (!h_entries || !h_sdf || !h_w))) return TF_E_INVAL;
    if (!ctx->p.swap_transfer_blocks) return TF_E_INVAL;
    const size_t n_entries = ctx->host_has.size();
    const uint8_t *store = (const uint8_t *)ctx->h_store;
    for (uint32_t k = 0; k < n; ++k) {
        const int32_t e = h_entries[k];
        const bool has = e >= 0 && (size_t)e < n_entries && ctx->host_has[e];
        if (h_has) h_has[k] = has ? 1 : 0;
        for (int lz = 0; lz < 8; ++lz)
            for (int ly = 0; ly < 8; ++ly)
                for (int lx = 0; lx < 8; ++lx) {
                    const int j = lz + 8 * ly + 64 * lx;            // store (device) order
                    const size_t o = (size_t)k * kBlockVox + lx + 8 * ly + 64 * lz;
                    h_sdf[o] = has ? ((const int16_t *)(store + (size_t)e * kBlockBytes))[j] : (int16_t)32767;
                    h_w[o] = has ? store[(size_t)e * kBlockBytes + 1024 + j] : (uint8_t)0;
                }
    }
    return TF_OK;
}

int tf_get_stats(tf_ctx *ctx, tf_stats *h_out, tf_stream stream)
{
    if (!ctx || !h_out) return TF_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    Ctrl c;
    hipError_t e = hipMemcpyAsync(&c, ctx->v.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return TF_E_HIP;
    h_out->flags = c.flags | ctx->host_flags;
    h_out->n_allocated = ctx->p.n_blocks - (uint32_t)c.free_blocks;
    h_out->n_visible = c.n_vis;
    h_out->n_new = c.n_new;
    h_out->n_free_excess = (uint32_t)c.free_excess;
    h_out->n_swapped_in = c.n_swapped_in;
    h_out->n_swapped_out = c.n_swapped_out;
    h_out->frames = c.frames;
    const size_t nt = ctx->L.max_tiles;
    unsigned long long *acc = (unsigned long long *)malloc((kIntegrateGrid + nt) * 8);
    if (!acc) return TF_E_INVAL;
    e = hipMemcpyAsync(acc, ctx->v.acc_cols, kIntegrateGrid * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(acc + kIntegrateGrid, ctx->v.acc_hits, nt * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        free(acc);
        return TF_E_HIP;
    }
    uint64_t cols = 0, hits = 0;
    for (int i = 0; i < kIntegrateGrid; ++i) cols += acc[i];
    for (size_t i = 0; i < nt; ++i) hits += acc[kIntegrateGrid + i];
    free(acc);
    h_out->total_integrated_blocks = c.tot_vis;
    h_out->total_written_columns = cols;
    h_out->total_range_records = c.tot_rec;
    h_out->total_rays_hit = hits;
    h_out->total_requests = c.tot_req;
    h_out->total_new_blocks = c.tot_new;
    h_out->integrate_calls = c.n_integrate;
    h_out->raycast_calls = c.n_raycast;
    return TF_OK;
}

int tf_export_entries(tf_ctx *ctx, int16_t *h_pos, int32_t *h_offset, int32_t *h_ptr, tf_stream stream)
{
    if (!ctx) return TF_E_INVAL;
    const size_t n = ctx->v.n_entries;
    DEntry *tmp = (DEntry *)malloc(n * sizeof(DEntry));
    if (!tmp) return TF_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(tmp, ctx->v.entries, n * sizeof(DEntry), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        free(tmp);
        return TF_E_HIP;
    }
    for (size_t i = 0; i < n; ++i) {
        if (h_pos) {
            h_pos[3 * i] = tmp[i].x;
            h_pos[3 * i + 1] = tmp[i].y;
            h_pos[3 * i + 2] = tmp[i].z;
        }
        if (h_offset) h_offset[i] = tmp[i].offset;
        if (h_ptr) h_ptr[i] = tmp[i].ptr;
    }
    free(tmp);
    return TF_OK;
}

int tf_export_visible(tf_ctx *ctx, int32_t *h_list, uint32_t cap, uint32_t *h_count, tf_stream stream)
{
    if (!ctx || !h_count || (cap && !h_list)) return TF_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    Ctrl c;
    hipError_t e = hipMemcpyAsync(&c, ctx->v.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return TF_E_HIP;
    *h_count = c.n_vis;
    uint32_t n = c.n_vis < cap ? c.n_vis : cap;
    if (n) {
        e = hipMemcpyAsync(h_list, ctx->v.vlist, (size_t)n * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    return hip_status(e);
}

int tf_export_voxels(tf_ctx *ctx, const int32_t *d_entries, uint32_t n, int16_t *d_sdf, uint8_t *d_w,
                     tf_stream stream)
{
    if (!ctx || (n && (!d_entries || !d_sdf || !d_w))) return TF_E_INVAL;
    if (!n) return TF_OK;
    return hip_status(launch_export_voxels(ctx->v, d_entries, n, d_sdf, d_w, (hipStream_t)stream));
}

int tf_camera_depth(const float *d_points, int32_t width, int32_t height, const float pose_w2c[16], float *d_depth,
                    tf_stream stream)
{
    if (!d_points || !d_depth || !pose_ok(pose_w2c) || width < 1 || height < 1 || width > 16384 || height > 16384)
        return TF_E_INVAL;
    if (((uintptr_t)d_points) & 15u) return TF_E_INVAL;
    return hip_status(launch_camera_depth((const float4 *)d_points, width * height, pose_w2c, d_depth,
                                          (hipStream_t)stream));
}

const char *tf_status_string(int status)
{
    switch (status) {
    case TF_OK: return "ok";
    case TF_E_INVAL: return "invalid argument";
    case TF_E_HIP: return "HIP runtime error";
    case TF_E_ORDER: return "call order violated";
    case TF_E_SPACE: return "workspace too small";
    case TF_E_IO: return "file error or not a volume of these parameters";
    default: return "unknown status";
    }
}

}  // extern "C"
