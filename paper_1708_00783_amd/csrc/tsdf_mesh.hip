// tsdf_mesh.hip -- marching-cubes meshing of the volume (Sec. 4, meshing
// engine) on gfx950.
//
// Three launches.  k_mesh<false> walks the hash entries in chunks of 64, one
// wave per chunk: the allocated entries are found with one ballot, and for
// each such block the wave stages the block and its +x/+y/+z
// halo (9^3 voxels, looked up in up to 7 neighbour blocks) in LDS; lane
// (x, y) classifies the 8 cells of its z column and the chunk's triangle count
// is written.  k_mesh_scan turns the counts into offsets (one workgroup, fixed
// order).  k_mesh<true> repeats the walk; a block's triangles occupy a
// contiguous range (chunk offset + earlier blocks), each lane's at a wave
// prefix over the lanes: they are built in LDS and written out with
// consecutive lanes on consecutive words.  The output order is fixed and two
// calls give the same arrays.
//
// The case table is derived at compile time from the cube's faces (constexpr),
// not tabulated: the rule of each face pairs its active edges into segments,
// the segments close into loops, each loop is oriented from the inside corners
// towards the outside ones and fanned from its smallest edge.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tsdf_ctx.h"
#include "tsdf_device.h"
#include "tsdf_mesh.h"

namespace {

using namespace tsdf;

struct McTable {
    int8_t e0[12], e1[12], axis[12];   // edge endpoints (corner indices) and axis
    int8_t ntri[256];
    int8_t tri[256][15];               // edge triples, ntri of them
};

constexpr McTable make_mc_table()
{
    McTable T{};
    int ne = 0;
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 8; ++c)
            if (!((c >> a) & 1)) {
                T.e0[ne] = (int8_t)c;
                T.e1[ne] = (int8_t)(c | (1 << a));
                T.axis[ne] = (int8_t)a;
                ++ne;
            }
    // the 6 faces: 4 corners and 4 edges each
    int fc[6][4] = {}, fe[6][4] = {};
    int f = 0;
    for (int a = 0; a < 3; ++a)
        for (int s = 0; s < 2; ++s, ++f) {
            int k = 0;
            for (int c = 0; c < 8; ++c)
                if (((c >> a) & 1) == s) fc[f][k++] = c;
            k = 0;
            for (int e = 0; e < 12; ++e)
                if (T.axis[e] != a && ((T.e0[e] >> a) & 1) == s && ((T.e1[e] >> a) & 1) == s) fe[f][k++] = e;
        }
    for (int m = 0; m < 256; ++m) {
        bool in[8] = {}, act[12] = {};
        for (int c = 0; c < 8; ++c) in[c] = (m >> c) & 1;
        for (int e = 0; e < 12; ++e) act[e] = in[T.e0[e]] != in[T.e1[e]];
        // segment graph: every active edge has exactly two neighbours
        int nb[12][2] = {}, deg[12] = {};
        for (int g = 0; g < 6; ++g) {
            int fa[4] = {}, n = 0;
            for (int k = 0; k < 4; ++k)
                if (act[fe[g][k]]) fa[n++] = fe[g][k];
            if (n == 2) {
                nb[fa[0]][deg[fa[0]]++] = fa[1];
                nb[fa[1]][deg[fa[1]]++] = fa[0];
            } else if (n == 4) {
                // ambiguous face: cut off each inside corner by its own segment
                for (int k = 0; k < 4; ++k) {
                    const int c = fc[g][k];
                    if (!in[c]) continue;
                    int inc[2] = {}, ni = 0;
                    for (int j = 0; j < 4; ++j)
                        if (T.e0[fa[j]] == c || T.e1[fa[j]] == c) inc[ni++] = fa[j];
                    nb[inc[0]][deg[inc[0]]++] = inc[1];
                    nb[inc[1]][deg[inc[1]]++] = inc[0];
                }
            }
        }
        bool seen[12] = {};
        int nt = 0;
        for (int s0 = 0; s0 < 12; ++s0) {
            if (!act[s0] || seen[s0]) continue;
            int loop[12] = {}, len = 0;
            int prev = -1, cur = s0;
            while (true) {
                loop[len++] = cur;
                seen[cur] = true;
                const int nx = nb[cur][0] != prev ? nb[cur][0] : nb[cur][1];
                prev = cur;
                cur = nx;
                if (cur == s0) break;
            }
            // orientation, in doubled integer coordinates: Newell normal of the
            // edge midpoints against the sum of inside -> outside edge directions
            int nvec[3] = {}, dvec[3] = {};
            for (int i = 0; i < len; ++i) {
                const int ea = loop[i], eb = loop[(i + 1) % len];
                int P[3] = {}, Q[3] = {};
                for (int d = 0; d < 3; ++d) {
                    P[d] = ((T.e0[ea] >> d) & 1) + ((T.e1[ea] >> d) & 1);
                    Q[d] = ((T.e0[eb] >> d) & 1) + ((T.e1[eb] >> d) & 1);
                }
                nvec[0] += P[1] * Q[2] - P[2] * Q[1];
                nvec[1] += P[2] * Q[0] - P[0] * Q[2];
                nvec[2] += P[0] * Q[1] - P[1] * Q[0];
                const int sg = in[T.e0[ea]] ? 1 : -1;      // from the inside corner to the outside one
                dvec[T.axis[ea]] += sg;
            }
            if (nvec[0] * dvec[0] + nvec[1] * dvec[1] + nvec[2] * dvec[2] < 0) {
                for (int i = 1, j = len - 1; i < j; ++i, --j) {
                    const int t = loop[i];
                    loop[i] = loop[j];
                    loop[j] = t;
                }
            }
            for (int i = 1; i + 1 < len; ++i) {
                T.tri[m][3 * nt + 0] = (int8_t)loop[0];
                T.tri[m][3 * nt + 1] = (int8_t)loop[i];
                T.tri[m][3 * nt + 2] = (int8_t)loop[i + 1];
                ++nt;
            }
        }
        T.ntri[m] = (int8_t)nt;
    }
    return T;
}

__constant__ McTable kMc = make_mc_table();

constexpr int kChunk = 64;            // hash entries per wave (one ballot)
constexpr int kCap = 256;             // triangles staged in LDS per write-out round
constexpr int kSide = 9;              // staged block + halo
constexpr int kVox = kSide * kSide * kSide;
constexpr int kUnobserved = 1 << 20;  // outside the short range: a corner with weight 0

struct MeshOut {
    float *verts;
    long long *keys;
    unsigned long long max_tri;
    unsigned long long *chunk_off;    // per chunk: triangle count, then exclusive offset
    unsigned long long *total;
};

__device__ __forceinline__ int stage_voxel(const uint8_t *blk, int idx)
{
    const int16_t s = reinterpret_cast<const int16_t *>(blk)[idx];
    return blk[1024 + idx] ? (int)s : kUnobserved;
}

// stage block (bx, by, bz) with device pointer ptr into g (index z * 81 + y * 9 + x)
__device__ __forceinline__ void stage_block(const Vol &v, int bx, int by, int bz, int ptr, int *g)
{
    const int lane = (int)__lane_id();
    // neighbour n = 1..7 at (n & 1, n >> 1 & 1, n >> 2 & 1); lane n - 1 looks it up
    int nptr = -1;
    if (lane < 7) {
        const int n = lane + 1;
        int p = -1;
        if (find_entry(v, bx + (n & 1), by + ((n >> 1) & 1), bz + ((n >> 2) & 1), 0, &p) >= 0) nptr = p;
    }
    int np[8];
    np[0] = ptr;
#pragma unroll
    for (int n = 1; n < 8; ++n) np[n] = __shfl(nptr, n - 1, 64);
    // own block: lane (x = lane >> 3, y = lane & 7) takes its z column (in-block index 64 x + 8 y + z)
    {
        const int x = lane >> 3, y = lane & 7;
        const uint8_t *blk = v.voxels + (size_t)ptr * kBlockBytes;
#pragma unroll
        for (int z = 0; z < 8; ++z) g[z * 81 + y * 9 + x] = stage_voxel(blk, 64 * x + 8 * y + z);
    }
    const int a = lane >> 3, b = lane & 7;
    // face x = 8: voxel (0, a, b) of neighbour 1
    g[b * 81 + a * 9 + 8] = np[1] >= 0 ? stage_voxel(v.voxels + (size_t)np[1] * kBlockBytes, 8 * a + b) : kUnobserved;
    // face y = 8: voxel (a, 0, b) of neighbour 2
    g[b * 81 + 8 * 9 + a] = np[2] >= 0 ? stage_voxel(v.voxels + (size_t)np[2] * kBlockBytes, 64 * a + b) : kUnobserved;
    // face z = 8: voxel (a, b, 0) of neighbour 4
    g[8 * 81 + b * 9 + a] = np[4] >= 0 ? stage_voxel(v.voxels + (size_t)np[4] * kBlockBytes, 64 * a + 8 * b) : kUnobserved;
    if (lane < 8) {
        const int k = lane;
        // edge x = 8, y = 8: voxel (0, 0, k) of neighbour 3
        g[k * 81 + 8 * 9 + 8] = np[3] >= 0 ? stage_voxel(v.voxels + (size_t)np[3] * kBlockBytes, k) : kUnobserved;
        // edge x = 8, z = 8: voxel (0, k, 0) of neighbour 5
        g[8 * 81 + k * 9 + 8] = np[5] >= 0 ? stage_voxel(v.voxels + (size_t)np[5] * kBlockBytes, 8 * k) : kUnobserved;
        // edge y = 8, z = 8: voxel (k, 0, 0) of neighbour 6
        g[8 * 81 + 8 * 9 + k] = np[6] >= 0 ? stage_voxel(v.voxels + (size_t)np[6] * kBlockBytes, 64 * k) : kUnobserved;
    }
    if (lane == 0) g[8 * 81 + 8 * 9 + 8] = np[7] >= 0 ? stage_voxel(v.voxels + (size_t)np[7] * kBlockBytes, 0) : kUnobserved;
}

// case of cell (x, y, z) of the staged grid, or 0 when a corner is unobserved
__device__ __forceinline__ int cell_case(const int *g, int x, int y, int z, int (&s)[8])
{
    int m = 0;
    bool ok = true;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        s[c] = g[(z + ((c >> 2) & 1)) * 81 + (y + ((c >> 1) & 1)) * 9 + x + (c & 1)];
        ok = ok && s[c] != kUnobserved;
        m |= (s[c] < 0 ? 1 : 0) << c;
    }
    return ok ? m : 0;
}

// the triangle's three vertices and edge keys
__device__ __forceinline__ void make_triangle(const int (&s)[8], int m, int t, int gx0, int gy0, int gz0, float voxel,
                                              float *v, long long *k)
{
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int e = kMc.tri[m][3 * t + j];
        const int c0 = kMc.e0[e], c1 = kMc.e1[e], ax = kMc.axis[e];
        int s0 = s[0], s1 = s[0];
#pragma unroll
        for (int c = 1; c < 8; ++c) {
            s0 = c == c0 ? s[c] : s0;
            s1 = c == c1 ? s[c] : s1;
        }
        const float f0 = (float)s0 * (1.0f / 32767.0f);
        const float f1 = (float)s1 * (1.0f / 32767.0f);
        const float tt = f0 / (f0 - f1);
        const int gx = gx0 + (c0 & 1), gy = gy0 + ((c0 >> 1) & 1), gz = gz0 + ((c0 >> 2) & 1);
        float px = (float)gx, py = (float)gy, pz = (float)gz;
        if (ax == 0) px = px + tt;
        else if (ax == 1) py = py + tt;
        else pz = pz + tt;
        v[3 * j + 0] = px * voxel;
        v[3 * j + 1] = py * voxel;
        v[3 * j + 2] = pz * voxel;
        k[j] = (long long)(((unsigned long long)(gx + (1 << 19)) << 42) | ((unsigned long long)(gy + (1 << 19)) << 22) |
                           ((unsigned long long)(gz + (1 << 19)) << 2) | (unsigned long long)ax);
    }
}

template <bool EMIT>
__global__ __launch_bounds__(64) void k_mesh(Vol v, MeshOut o, float voxel)
{
    __shared__ int g[kVox];
    __shared__ float sv[EMIT ? kCap * 9 : 1];
    __shared__ long long sk[EMIT ? kCap * 3 : 1];
    const int lane = (int)threadIdx.x;
    const uint32_t chunk = blockIdx.x;
    const int cx = lane & 7, cy = lane >> 3;          // the lane's cell column
    unsigned long long base = EMIT ? o.chunk_off[chunk] : 0ull;
    unsigned long long count = 0;
    const uint32_t e = chunk * kChunk + (uint32_t)lane;
    int4 w = make_int4(0, 0, 0, -2);
    if (e < v.n_entries) w = load_entry(v.entries, e);
    unsigned long long live = __ballot(w.w >= 0);
    while (live) {
        const int src = __ffsll((long long)live) - 1;
        live &= live - 1;
        const int kxy = __shfl(w.x, src, 64), kz = __shfl(w.y, src, 64), ptr = __shfl(w.w, src, 64);
        const int bx = (int16_t)(kxy & 0xffff), by = (int16_t)((uint32_t)kxy >> 16), bz = (int16_t)(kz & 0xffff);
        __syncthreads();                             // the previous block's reads are done
        stage_block(v, bx, by, bz, ptr, g);
        __syncthreads();
        int n = 0;
#pragma unroll
        for (int z = 0; z < 8; ++z) {
            int s[8];
            n += kMc.ntri[cell_case(g, cx, cy, z, s)];
        }
        if (!EMIT) {
            count += (unsigned long long)n;   // summed over lanes below
            continue;
        }
        // exclusive prefix of n over the lanes: the lane's first triangle in the block
        int pre = n;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int t = __shfl_up(pre, d, 64);
            if (lane >= d) pre += t;
        }
        const int tot = __shfl(pre, 63, 64);
        const int first = pre - n;
        const int gx0 = bx * 8 + cx, gy0 = by * 8 + cy, gz0 = bz * 8;
        // the block's triangles are contiguous in the output: build them in LDS,
        // kCap at a time, and write each round with consecutive lanes on
        // consecutive words
        for (int r0 = 0; r0 < tot; r0 += kCap) {
            if (first < r0 + kCap && first + n > r0) {
                int li = first;
                for (int z = 0; z < 8; ++z) {
                    int s[8];
                    const int m = cell_case(g, cx, cy, z, s);
                    const int nt = kMc.ntri[m];
                    for (int t = 0; t < nt; ++t, ++li)
                        if (li >= r0 && li < r0 + kCap)
                            make_triangle(s, m, t, gx0, gy0, gz0 + z, voxel, sv + (li - r0) * 9, sk + (li - r0) * 3);
                }
            }
            __syncthreads();
            const int cnt = tot - r0 < kCap ? tot - r0 : kCap;
            const unsigned long long t0 = base + (unsigned long long)r0;
            unsigned long long lim = o.max_tri > t0 ? o.max_tri - t0 : 0ull;
            const int keep = lim < (unsigned long long)cnt ? (int)lim : cnt;
            if (o.verts)
                for (int i = lane; i < keep * 9; i += 64) o.verts[t0 * 9 + (unsigned long long)i] = sv[i];
            if (o.keys)
                for (int i = lane; i < keep * 3; i += 64) o.keys[t0 * 3 + (unsigned long long)i] = sk[i];
            __syncthreads();
        }
        base += (unsigned long long)tot;
    }
    if (!EMIT) {
        // fixed-order wave sum of the lanes' counts
        for (int off = 32; off > 0; off >>= 1) count += __shfl_xor(count, off, 64);
        if (lane == 0) o.chunk_off[chunk] = count;
    }
}

// exclusive offsets of the chunk counts and the total (one workgroup of 1024)
__global__ __launch_bounds__(1024) void k_mesh_scan(unsigned long long *c, uint32_t n, unsigned long long *total)
{
    __shared__ unsigned long long part[1024];
    const uint32_t t = threadIdx.x;
    const uint32_t per = (n + 1023) / 1024;
    const uint32_t b = t * per, e = b + per < n ? b + per : n;
    unsigned long long s = 0;
    for (uint32_t i = b; i < e; ++i) s += c[i];
    part[t] = s;
    __syncthreads();
    for (uint32_t d = 1; d < 1024; d <<= 1) {
        const unsigned long long x = t >= d ? part[t - d] : 0ull;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    unsigned long long run = part[t] - s;
    for (uint32_t i = b; i < e; ++i) {
        const unsigned long long k = c[i];
        c[i] = run;
        run += k;
    }
    if (t == 1023) *total = part[1023];
}

uint32_t mesh_chunks(uint32_t n_entries) { return (n_entries + kChunk - 1) / kChunk; }

}  // namespace

extern "C" {

size_t tf_mesh_workspace_bytes(const tf_params *p)
{
    if (!p || tf_workspace_bytes(p) == 0) return 0;
    const uint32_t n_entries = p->n_buckets + p->n_excess;
    return (size_t)mesh_chunks(n_entries) * sizeof(unsigned long long);
}

int tf_mesh(tf_ctx *ctx, float *d_vertices, int64_t *d_edge_keys, uint64_t max_triangles, uint64_t *d_count,
            void *d_workspace, size_t workspace_bytes, tf_stream stream)
{
    if (!ctx || !d_count || !d_workspace) return TF_E_INVAL;
    if (((uintptr_t)d_count & 7u) || ((uintptr_t)d_workspace & 7u) || ((uintptr_t)d_vertices & 3u) ||
        ((uintptr_t)d_edge_keys & 7u))
        return TF_E_INVAL;
    const uint32_t chunks = mesh_chunks(ctx->v.n_entries);
    if (workspace_bytes < (size_t)chunks * sizeof(unsigned long long)) return TF_E_SPACE;
    MeshOut o;
    o.verts = d_vertices;
    o.keys = (long long *)d_edge_keys;
    o.max_tri = max_triangles;
    o.chunk_off = (unsigned long long *)d_workspace;
    o.total = (unsigned long long *)d_count;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_mesh<false>, dim3(chunks), dim3(64), 0, s, ctx->v, o, ctx->p.voxel_size);
    hipLaunchKernelGGL(k_mesh_scan, dim3(1), dim3(1024), 0, s, o.chunk_off, chunks, o.total);
    if (d_vertices || d_edge_keys)
        hipLaunchKernelGGL(k_mesh<true>, dim3(chunks), dim3(64), 0, s, ctx->v, o, ctx->p.voxel_size);
    return hipGetLastError() == hipSuccess ? TF_OK : TF_E_HIP;
}

}  // extern "C"
