// tsdf_io.hip -- tf_save / tf_load: a volume's whole state (scene parameters,
// hash table, free lists, visible list, occupancy bits, voxel blocks, counters
// and, with swapping, the host store) to and from a file.  Host code only;
// device regions pass through a pageable bounce buffer on the caller's stream.
//
// File layout (native byte order), sections in this order:
//   FileHeader
//   Ctrl                               device counters
//   entries        n_entries x 16 B    hash table (Sec. 3.2)
//   free_blocks    n_blocks x 4 B      free-block stack (all slots)
//   free_excess    n_excess x 4 B      free excess-slot stack
//   vlist          n_vis x 4 B         visible list
//   occ, brick                         bucket- and block-occupancy bits
//   acc_cols, acc_hits                 per-workgroup work counters
//   runs           n_runs x (first block, count) uint32 pairs, then the
//                  voxel blocks of every run (1536 B each, device order)
//   [swapping]     host_has (one byte per entry, device copy), n_host, the
//                  n_host entry indices whose host-store block follows, then
//                  those blocks
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "tsdf.h"
#include "tsdf_ctx.h"
#include "tsdf_internal.h"

using namespace tsdf;

namespace {

const char kMagic[8] = {'T', 'S', 'D', 'F', 'V', 'O', 'L', '1'};
constexpr uint32_t kVersion = 1;
constexpr size_t kBounce = (size_t)64 << 20;

struct FileHeader {
    char magic[8];
    uint32_t version;
    uint32_t ctrl_bytes;
    tf_params p;
    uint32_t n_runs;
    uint32_t max_tiles;
    uint64_t reserved;
};

bool same_params(const tf_params &a, const tf_params &b)
{
    return a.voxel_size == b.voxel_size && a.mu == b.mu && a.max_w == b.max_w && a.n_buckets == b.n_buckets &&
           a.n_excess == b.n_excess && a.n_blocks == b.n_blocks && a.max_width == b.max_width &&
           a.max_height == b.max_height && a.swap_transfer_blocks == b.swap_transfer_blocks;
}

// a file and the status of the first failure (TF_E_IO or TF_E_HIP)
struct Io {
    FILE *f = nullptr;
    hipStream_t s = nullptr;
    std::vector<uint8_t> buf;
    int st = TF_OK;

    void put(const void *p, size_t n)
    {
        if (st == TF_OK && n && fwrite(p, 1, n, f) != n) st = TF_E_IO;
    }
    void get(void *p, size_t n)
    {
        if (st == TF_OK && n && fread(p, 1, n, f) != n) st = TF_E_IO;
    }
    void from_device(const void *d, size_t n)
    {
        for (size_t o = 0; st == TF_OK && o < n; o += buf.size()) {
            const size_t m = std::min(buf.size(), n - o);
            if (hipMemcpyAsync(buf.data(), (const uint8_t *)d + o, m, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                st = TF_E_HIP;
                return;
            }
            put(buf.data(), m);
        }
    }
    void to_device(void *d, size_t n)
    {
        for (size_t o = 0; st == TF_OK && o < n; o += buf.size()) {
            const size_t m = std::min(buf.size(), n - o);
            get(buf.data(), m);
            if (st != TF_OK) return;
            if (hipMemcpyAsync((uint8_t *)d + o, buf.data(), m, hipMemcpyHostToDevice, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                st = TF_E_HIP;
        }
    }
};

size_t n_vis_bytes(const tf_ctx *ctx) { return ((size_t)ctx->v.n_entries + 15) & ~(size_t)15; }

}  // namespace

extern "C" {

int tf_save(tf_ctx *ctx, const char *path, tf_stream stream)
{
    if (!ctx || !path) return TF_E_INVAL;
    if (ctx->v.alist) return TF_E_INVAL;   // a submap of a batched map
    Io io;
    io.s = (hipStream_t)stream;
    if (hipStreamSynchronize(io.s) != hipSuccess) return TF_E_HIP;
    const Vol &v = ctx->v;
    Ctrl c;
    std::vector<DEntry> ent(v.n_entries);
    if (hipMemcpyAsync(&c, v.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, io.s) != hipSuccess ||
        hipMemcpyAsync(ent.data(), v.entries, ent.size() * sizeof(DEntry), hipMemcpyDeviceToHost, io.s) !=
            hipSuccess ||
        hipStreamSynchronize(io.s) != hipSuccess)
        return TF_E_HIP;
    // the blocks in use, as runs of consecutive block indices
    std::vector<uint32_t> used;
    for (const DEntry &e : ent)
        if (e.ptr >= 0) used.push_back((uint32_t)e.ptr);
    std::sort(used.begin(), used.end());
    std::vector<uint32_t> runs;   // (first, count) pairs
    for (size_t i = 0; i < used.size();) {
        size_t j = i + 1;
        while (j < used.size() && used[j] == used[j - 1] + 1) ++j;
        runs.push_back(used[i]);
        runs.push_back((uint32_t)(j - i));
        i = j;
    }
    io.f = fopen(path, "wb");
    if (!io.f) return TF_E_IO;
    io.buf.resize(kBounce);
    FileHeader h = {};
    memcpy(h.magic, kMagic, sizeof(kMagic));
    h.version = kVersion;
    h.ctrl_bytes = (uint32_t)sizeof(Ctrl);
    h.p = ctx->p;
    h.n_runs = (uint32_t)(runs.size() / 2);
    h.max_tiles = ctx->L.max_tiles;
    io.put(&h, sizeof(h));
    io.put(&c, sizeof(c));
    io.put(ent.data(), ent.size() * sizeof(DEntry));
    io.from_device(v.free_blocks, (size_t)v.n_blocks * 4);
    io.from_device(v.free_excess, (size_t)v.n_excess * 4);
    io.from_device(v.vlist, (size_t)c.n_vis * 4);
    io.from_device(v.occ, (size_t)v.n_buckets / 8);
    io.from_device(v.brick, (size_t)kBrickWords * 4);
    io.from_device(v.acc_cols, (size_t)kIntegrateGrid * 8);
    io.from_device(v.acc_hits, (size_t)ctx->L.max_tiles * 8);
    io.put(runs.data(), runs.size() * 4);
    for (size_t r = 0; r < runs.size(); r += 2)
        io.from_device(v.voxels + (size_t)runs[r] * kBlockBytes, (size_t)runs[r + 1] * kBlockBytes);
    if (ctx->p.swap_transfer_blocks) {
        io.from_device(v.host_has, n_vis_bytes(ctx));
        std::vector<uint32_t> host;
        for (size_t i = 0; i < ctx->host_has.size(); ++i)
            if (ctx->host_has[i]) host.push_back((uint32_t)i);
        const uint32_t n_host = (uint32_t)host.size();
        io.put(&n_host, 4);
        io.put(host.data(), host.size() * 4);
        const uint8_t *store = (const uint8_t *)ctx->h_store;
        for (uint32_t e : host) io.put(store + (size_t)e * kBlockBytes, kBlockBytes);
    }
    if (fclose(io.f) != 0 && io.st == TF_OK) io.st = TF_E_IO;
    return io.st;
}

int tf_load(tf_ctx *ctx, const char *path, tf_stream stream)
{
    if (!ctx || !path) return TF_E_INVAL;
    if (ctx->v.alist) return TF_E_INVAL;
    Io io;
    io.s = (hipStream_t)stream;
    io.f = fopen(path, "rb");
    if (!io.f) return TF_E_IO;
    FileHeader h;
    io.get(&h, sizeof(h));
    if (io.st != TF_OK || memcmp(h.magic, kMagic, sizeof(kMagic)) != 0 || h.version != kVersion ||
        h.ctrl_bytes != sizeof(Ctrl) || !same_params(h.p, ctx->p) || h.max_tiles != ctx->L.max_tiles) {
        fclose(io.f);
        return TF_E_IO;
    }
    int st = tf_reset(ctx, stream);
    if (st != TF_OK) {
        fclose(io.f);
        return st;
    }
    io.buf.resize(kBounce);
    Vol &v = ctx->v;
    Ctrl c;
    io.get(&c, sizeof(c));
    // per-frame fields start clean (no pending requests, records or tickets)
    c.n_req = c.n_ret = c.n_rec = c.ray_ticket = c.req_overflow = c.sweep_req = c.n_swap_cand = 0;
    if (io.st == TF_OK && (c.n_vis > v.n_blocks || c.free_blocks < 0 || (uint32_t)c.free_blocks > v.n_blocks ||
                           c.free_excess < 0 || (uint32_t)c.free_excess > v.n_excess))
        io.st = TF_E_IO;
    if (io.st == TF_OK && (hipMemcpyAsync(v.ctrl, &c, sizeof(c), hipMemcpyHostToDevice, io.s) != hipSuccess ||
                           hipStreamSynchronize(io.s) != hipSuccess))
        io.st = TF_E_HIP;
    io.to_device(v.entries, (size_t)v.n_entries * sizeof(DEntry));
    io.to_device(v.free_blocks, (size_t)v.n_blocks * 4);
    io.to_device(v.free_excess, (size_t)v.n_excess * 4);
    io.to_device(v.vlist, (size_t)c.n_vis * 4);
    io.to_device(v.occ, (size_t)v.n_buckets / 8);
    io.to_device(v.brick, (size_t)kBrickWords * 4);
    io.to_device(v.acc_cols, (size_t)kIntegrateGrid * 8);
    io.to_device(v.acc_hits, (size_t)ctx->L.max_tiles * 8);
    std::vector<uint32_t> runs((size_t)h.n_runs * 2);
    io.get(runs.data(), runs.size() * 4);
    for (size_t r = 0; io.st == TF_OK && r < runs.size(); r += 2) {
        if ((uint64_t)runs[r] + runs[r + 1] > v.n_blocks) {
            io.st = TF_E_IO;
            break;
        }
        io.to_device(v.voxels + (size_t)runs[r] * kBlockBytes, (size_t)runs[r + 1] * kBlockBytes);
    }
    if (ctx->p.swap_transfer_blocks) {
        io.to_device(v.host_has, n_vis_bytes(ctx));
        uint32_t n_host = 0;
        io.get(&n_host, 4);
        if (io.st == TF_OK && n_host > v.n_entries) io.st = TF_E_IO;
        std::vector<uint32_t> host(io.st == TF_OK ? n_host : 0);
        io.get(host.data(), host.size() * 4);
        uint8_t *store = (uint8_t *)ctx->h_store;
        for (uint32_t e : host) {
            if (io.st != TF_OK) break;
            if (e >= v.n_entries) {
                io.st = TF_E_IO;
                break;
            }
            io.get(store + (size_t)e * kBlockBytes, kBlockBytes);
            ctx->host_has[e] = 1;
        }
    }
    fclose(io.f);
    if (io.st != TF_OK) {
        tf_reset(ctx, stream);   // a partial load leaves an empty volume, not a mixed one
        return io.st;
    }
    return TF_OK;
}

}  // extern "C"
