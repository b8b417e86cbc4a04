// tsdf_surfel.hip -- surfel fusion (Sec. 7.3) on gfx950.
//
// Per frame, six launches, none waiting for the host:
//   k_sf_points  per pixel: world point, normal (forward differences), alpha,
//                validity; clears the pixel's z-buffer word
//   k_sf_splat   per surfel: project, and for every pixel of its circle an
//                atomicMin of (camera z bits << 32 | index) -- the index map is
//                the low half, independent of the order of the atomics
//   k_sf_assoc   per pixel: the index map's surfel if the depth and normal
//                gates pass, else a new surfel, else nothing
//   k_sf_update  per surfel: walks its own circle again in raster order and
//                sums the points that chose it (fixed order, no atomics), then
//                applies the weighted average
//   k_sf_count / k_sf_scan / k_sf_append / k_sf_finish: new surfels in pixel
//                raster order (per-256-pixel counts, one-workgroup scan,
//                ballot ranks), then the count
// The surfel count stays on the device; grid-stride loops read it.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "tsdf_surfel.h"

namespace {

constexpr int kPixBlock = 256;
constexpr int kSurfGrid = 2048;        // workgroups of the per-surfel launches
constexpr float kRhoMax = 8.0f;
constexpr int kFaceCorr = -2;          // corr: no input point
constexpr int kNewCorr = -1;           // corr: new surfel

struct alignas(256) SfState {
    uint32_t n;                        // surfels in the map
    uint32_t flags;
    uint32_t n_new;                    // new surfels of the current frame
    uint32_t pad;
};

struct SfMap {
    SfState *st;
    float4 *pos;                       // x, y, z, radius
    float4 *nrm;                       // nx, ny, nz, confidence
    int32_t *time;
    float4 *ipt;                       // per pixel: world point, alpha
    float4 *inr;                       // per pixel: world normal, camera depth (0: no input point)
    unsigned long long *zbuf;          // per pixel: (z bits << 32) | surfel
    int32_t *corr;                     // per pixel: surfel, kNewCorr or kFaceCorr
    uint32_t *blk;                     // per 256 pixels: new surfels, then their offset
    uint32_t cap;
};

struct SfCam {
    float M[12];                       // world -> camera rows
    float R[9], t[3];                  // camera -> world
    float fx, fy, cx, cy;
    int W, H;
};

template <int FMT>
__device__ __forceinline__ float depth_at(const void *d, int i)
{
    if (FMT == TF_DEPTH_U16_MM) return (float)((const uint16_t *)d)[i] / 1000.0f;
    return ((const float *)d)[i];
}

template <int FMT>
__global__ __launch_bounds__(256) void k_sf_points(const void *depth, SfCam c, float alpha_k, float norm_r, SfMap m)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= c.W * c.H) return;
    const int y = p / c.W, x = p - y * c.W;
    m.zbuf[p] = ~0ull;
    const float d = depth_at<FMT>(depth, p);
    float4 P = make_float4(0.f, 0.f, 0.f, 0.f), N = make_float4(0.f, 0.f, 0.f, 0.f);
    if (d > 0.0f && x + 1 < c.W && y + 1 < c.H) {
        const float dr = depth_at<FMT>(depth, p + 1), dd = depth_at<FMT>(depth, p + c.W);
        if (dr > 0.0f && dd > 0.0f) {
            const float vx = d * (((float)x - c.cx) / c.fx), vy = d * (((float)y - c.cy) / c.fy), vz = d;
            const float rx = dr * (((float)(x + 1) - c.cx) / c.fx), ry = dr * (((float)y - c.cy) / c.fy), rz = dr;
            const float bx = dd * (((float)x - c.cx) / c.fx), by = dd * (((float)(y + 1) - c.cy) / c.fy), bz = dd;
            const float ax = rx - vx, ay = ry - vy, az = rz - vz;
            const float ex = bx - vx, ey = by - vy, ez = bz - vz;
            float nx = ay * ez - az * ey, ny = az * ex - ax * ez, nz = ax * ey - ay * ex;
            const float nn = (nx * nx + ny * ny) + nz * nz;
            if (nn > 0.0f) {
                const float inv = 1.0f / sqrtf(nn);
                nx = nx * inv;
                ny = ny * inv;
                nz = nz * inv;
                if (((nx * vx + ny * vy) + nz * vz) > 0.0f) {
                    nx = -nx;
                    ny = -ny;
                    nz = -nz;
                }
                P.x = ((c.R[0] * vx + c.R[1] * vy) + c.R[2] * vz) + c.t[0];
                P.y = ((c.R[3] * vx + c.R[4] * vy) + c.R[5] * vz) + c.t[1];
                P.z = ((c.R[6] * vx + c.R[7] * vy) + c.R[8] * vz) + c.t[2];
                const float gx = (float)x - c.cx, gy = (float)y - c.cy;
                const float gam = sqrtf(gx * gx + gy * gy) / norm_r;
                P.w = expf(-(gam * gam) / alpha_k);
                N.x = (c.R[0] * nx + c.R[1] * ny) + c.R[2] * nz;
                N.y = (c.R[3] * nx + c.R[4] * ny) + c.R[5] * nz;
                N.z = (c.R[6] * nx + c.R[7] * ny) + c.R[8] * nz;
                N.w = d;
            }
        }
    }
    m.ipt[p] = P;
    m.inr[p] = N;
}

// projection of surfel position q (x, y, z, radius): false when it covers no pixel
__device__ __forceinline__ bool sf_project(const SfCam &c, float4 q, float &u, float &v, float &rho, float &Z)
{
    const float X = ((c.M[0] * q.x + c.M[1] * q.y) + c.M[2] * q.z) + c.M[3];
    const float Y = ((c.M[4] * q.x + c.M[5] * q.y) + c.M[6] * q.z) + c.M[7];
    Z = ((c.M[8] * q.x + c.M[9] * q.y) + c.M[10] * q.z) + c.M[11];
    if (!(Z > 0.0f)) return false;
    u = (c.fx * X) / Z + c.cx;
    v = (c.fy * Y) / Z + c.cy;
    rho = fminf((c.fx * q.w) / Z, kRhoMax);
    return u + rho >= 0.0f && u - rho <= (float)(c.W - 1) && v + rho >= 0.0f && v - rho <= (float)(c.H - 1);
}

__global__ __launch_bounds__(256) void k_sf_splat(SfCam c, SfMap m)
{
    const uint32_t n = m.st->n;
    for (uint32_t s = blockIdx.x * 256 + threadIdx.x; s < n; s += gridDim.x * 256) {
        float u, v, rho, Z;
        if (!sf_project(c, m.pos[s], u, v, rho, Z)) continue;
        const unsigned long long key = ((unsigned long long)__float_as_uint(Z) << 32) | s;
        // candidates from ceil(u - rho) up to one past floor(u + rho): the float32
        // circle test decides, as it may admit a pixel at distance rho + 1 ulp
        const int x0 = max(0, (int)ceilf(u - rho)), x1 = min(c.W - 1, (int)floorf(u + rho) + 1);
        const int y0 = max(0, (int)ceilf(v - rho)), y1 = min(c.H - 1, (int)floorf(v + rho) + 1);
        for (int y = y0; y <= y1; ++y) {
            const float dy = (float)y - v;
            for (int x = x0; x <= x1; ++x) {
                const float dx = (float)x - u;
                if (dx * dx + dy * dy <= rho * rho) atomicMin(&m.zbuf[y * c.W + x], key);
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_sf_assoc(SfCam c, float max_dz, float min_dot, SfMap m)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= c.W * c.H) return;
    const float4 N = m.inr[p];
    int r = kFaceCorr;
    if (N.w > 0.0f) {
        r = kNewCorr;
        const unsigned long long k = m.zbuf[p];
        if (k != ~0ull) {
            const uint32_t s = (uint32_t)(k & 0xffffffffull);
            const float Z = __uint_as_float((uint32_t)(k >> 32));
            const float4 ns = m.nrm[s];
            const float dot = (N.x * ns.x + N.y * ns.y) + N.z * ns.z;
            const float len = sqrtf((ns.x * ns.x + ns.y * ns.y) + ns.z * ns.z);
            if (fabsf(N.w - Z) <= max_dz && dot >= min_dot * len) r = (int)s;
        }
    }
    m.corr[p] = r;
}

__global__ __launch_bounds__(256) void k_sf_update(SfCam c, SfMap m, int frame)
{
    const uint32_t n = m.st->n;
    for (uint32_t s = blockIdx.x * 256 + threadIdx.x; s < n; s += gridDim.x * 256) {
        const float4 q = m.pos[s];
        float u, v, rho, Z;
        if (!sf_project(c, q, u, v, rho, Z)) continue;
        // candidates from ceil(u - rho) up to one past floor(u + rho): the float32
        // circle test decides, as it may admit a pixel at distance rho + 1 ulp
        const int x0 = max(0, (int)ceilf(u - rho)), x1 = min(c.W - 1, (int)floorf(u + rho) + 1);
        const int y0 = max(0, (int)ceilf(v - rho)), y1 = min(c.H - 1, (int)floorf(v + rho) + 1);
        float sa = 0.f, svx = 0.f, svy = 0.f, svz = 0.f, snx = 0.f, sny = 0.f, snz = 0.f;
        for (int y = y0; y <= y1; ++y) {
            const float dy = (float)y - v;
            for (int x = x0; x <= x1; ++x) {
                const float dx = (float)x - u;
                if (!(dx * dx + dy * dy <= rho * rho)) continue;
                const int p = y * c.W + x;
                if (m.corr[p] != (int)s) continue;
                const float4 P = m.ipt[p];
                const float4 N = m.inr[p];
                sa += P.w;
                svx += P.w * P.x;
                svy += P.w * P.y;
                svz += P.w * P.z;
                snx += P.w * N.x;
                sny += P.w * N.y;
                snz += P.w * N.z;
            }
        }
        if (sa > 0.0f) {
            float4 nr = m.nrm[s];
            const float cc = nr.w, den = cc + sa;
            float4 np = q;
            np.x = (cc * q.x + svx) / den;
            np.y = (cc * q.y + svy) / den;
            np.z = (cc * q.z + svz) / den;
            nr.x = (cc * nr.x + snx) / den;
            nr.y = (cc * nr.y + sny) / den;
            nr.z = (cc * nr.z + snz) / den;
            nr.w = den;
            m.pos[s] = np;
            m.nrm[s] = nr;
            m.time[s] = frame;
        }
    }
}

__global__ __launch_bounds__(256) void k_sf_count(int npix, SfMap m)
{
    __shared__ uint32_t wc[4];
    const int p = blockIdx.x * 256 + threadIdx.x;
    const bool nw = p < npix && m.corr[p] == kNewCorr;
    const unsigned long long b = __ballot(nw);
    if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = (uint32_t)__popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) m.blk[blockIdx.x] = ((wc[0] + wc[1]) + wc[2]) + wc[3];
}

// exclusive offsets of the per-block counts, the frame's total in st->n_new
__global__ __launch_bounds__(1024) void k_sf_scan(int nblk, SfMap m)
{
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int per = (nblk + 1023) / 1024;
    const int b = t * per, e = min(b + per, nblk);
    uint32_t s = 0;
    for (int i = b; i < e; ++i) s += m.blk[i];
    part[t] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const uint32_t x = t >= d ? part[t - d] : 0u;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    uint32_t run = part[t] - s;
    for (int i = b; i < e; ++i) {
        const uint32_t k = m.blk[i];
        m.blk[i] = run;
        run += k;
    }
    if (t == 1023) m.st->n_new = part[1023];
}

__global__ __launch_bounds__(256) void k_sf_append(SfCam c, SfMap m, int frame)
{
    __shared__ uint32_t wc[4];
    const int p = blockIdx.x * 256 + threadIdx.x;
    const int npix = c.W * c.H;
    const bool nw = p < npix && m.corr[p] == kNewCorr;
    const unsigned long long b = __ballot(nw);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) wc[wave] = (uint32_t)__popcll(b);
    __syncthreads();
    if (!nw) return;
    uint32_t off = m.blk[blockIdx.x];
    for (int w = 0; w < wave; ++w) off += wc[w];
    off += (uint32_t)__popcll(b & ((1ull << lane) - 1ull));
    const uint32_t idx = m.st->n + off;
    if (idx >= m.cap) {
        atomicOr(&m.st->flags, (uint32_t)TF_FLAG_SURFEL_OVERFLOW);
        return;
    }
    const float4 P = m.ipt[p];
    const float4 N = m.inr[p];
    m.pos[idx] = make_float4(P.x, P.y, P.z, (N.w * 0.70710677f) / c.fx);
    m.nrm[idx] = make_float4(N.x, N.y, N.z, P.w);
    m.time[idx] = frame;
}

__global__ void k_sf_finish(SfMap m)
{
    const uint32_t n = m.st->n + m.st->n_new;
    m.st->n = n < m.cap ? n : m.cap;
}

__global__ __launch_bounds__(256) void k_sf_init(SfMap m)
{
    if (threadIdx.x == 0) {
        m.st->n = 0;
        m.st->flags = 0;
        m.st->n_new = 0;
        m.st->pad = 0;
    }
}

__global__ __launch_bounds__(256) void k_sf_frame_out(int npix, const unsigned long long *zbuf, const int32_t *corr,
                                                      int32_t *imap, int32_t *cout)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= npix) return;
    if (imap) imap[p] = zbuf[p] == ~0ull ? -1 : (int32_t)(zbuf[p] & 0xffffffffull);
    if (cout) cout[p] = corr[p];
}

struct SfLayout {
    size_t st, pos, nrm, time, ipt, inr, zbuf, corr, blk, total;
};

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

bool sf_layout(const tf_surfel_params *p, SfLayout *L)
{
    if (!p || p->capacity < 1 || p->capacity > (1u << 26) || p->max_width < 1 || p->max_height < 1 ||
        p->max_width > 8192 || p->max_height > 8192)
        return false;
    if (!(p->sigma > 0.0f) || !(p->sigma < 1e30f) || !(p->max_depth_diff > 0.0f) || !(p->max_depth_diff < 1e30f) ||
        !(p->min_normal_dot >= -1.0f) || !(p->min_normal_dot <= 1.0f))
        return false;
    const size_t cap = p->capacity, npix = (size_t)p->max_width * p->max_height;
    const size_t nblk = (npix + kPixBlock - 1) / kPixBlock;
    size_t o = 0;
    L->st = o;
    o += 256;
    L->pos = o;
    o += up256(cap * 16);
    L->nrm = o;
    o += up256(cap * 16);
    L->time = o;
    o += up256(cap * 4);
    L->ipt = o;
    o += up256(npix * 16);
    L->inr = o;
    o += up256(npix * 16);
    L->zbuf = o;
    o += up256(npix * 8);
    L->corr = o;
    o += up256(npix * 4);
    L->blk = o;
    o += up256(nblk * 4);
    L->total = o;
    return true;
}

}  // namespace

struct tf_surfels {
    tf_surfel_params p;
    SfMap m;
    uint32_t frames;
    int last_w, last_h;
};

extern "C" {

size_t tf_surfel_workspace_bytes(const tf_surfel_params *p)
{
    SfLayout L;
    return sf_layout(p, &L) ? L.total : 0;
}

int tf_surfel_create(const tf_surfel_params *p, void *d_workspace, size_t bytes, tf_stream stream, tf_surfels **out)
{
    SfLayout L;
    if (!out || !d_workspace || !sf_layout(p, &L) || ((uintptr_t)d_workspace & 255u)) return TF_E_INVAL;
    if (bytes < L.total) return TF_E_SPACE;
    tf_surfels *s = new tf_surfels();
    s->p = *p;
    char *w = (char *)d_workspace;
    s->m.st = (SfState *)(w + L.st);
    s->m.pos = (float4 *)(w + L.pos);
    s->m.nrm = (float4 *)(w + L.nrm);
    s->m.time = (int32_t *)(w + L.time);
    s->m.ipt = (float4 *)(w + L.ipt);
    s->m.inr = (float4 *)(w + L.inr);
    s->m.zbuf = (unsigned long long *)(w + L.zbuf);
    s->m.corr = (int32_t *)(w + L.corr);
    s->m.blk = (uint32_t *)(w + L.blk);
    s->m.cap = p->capacity;
    s->frames = 0;
    s->last_w = s->last_h = 0;
    hipLaunchKernelGGL(k_sf_init, dim3(1), dim3(256), 0, (hipStream_t)stream, s->m);
    if (hipGetLastError() != hipSuccess) {
        delete s;
        return TF_E_HIP;
    }
    *out = s;
    return TF_OK;
}

int tf_surfel_destroy(tf_surfels *m)
{
    if (!m) return TF_E_INVAL;
    delete m;
    return TF_OK;
}

int tf_surfel_reset(tf_surfels *m, tf_stream stream)
{
    if (!m) return TF_E_INVAL;
    m->frames = 0;
    m->last_w = m->last_h = 0;
    hipLaunchKernelGGL(k_sf_init, dim3(1), dim3(256), 0, (hipStream_t)stream, m->m);
    return hipGetLastError() == hipSuccess ? TF_OK : TF_E_HIP;
}

int tf_surfel_fuse(tf_surfels *m, const void *d_depth, int depth_format, const tf_intrinsics *K,
                   const float pose_w2c[16], tf_stream stream)
{
    if (!m || !d_depth || !K || !pose_w2c) return TF_E_INVAL;
    if (depth_format != TF_DEPTH_F32_M && depth_format != TF_DEPTH_U16_MM) return TF_E_INVAL;
    if (K->width < 1 || K->height < 1 || K->width > m->p.max_width || K->height > m->p.max_height) return TF_E_INVAL;
    if (!(K->fx > 0.0f) || !(K->fy > 0.0f) || !(K->cx == K->cx) || !(K->cy == K->cy)) return TF_E_INVAL;
    if ((uintptr_t)d_depth & (depth_format == TF_DEPTH_F32_M ? 3u : 1u)) return TF_E_INVAL;
    for (int i = 0; i < 16; ++i)
        if (!(pose_w2c[i] == pose_w2c[i]) || pose_w2c[i] > 1e30f || pose_w2c[i] < -1e30f) return TF_E_INVAL;
    SfCam c;
    for (int i = 0; i < 12; ++i) c.M[i] = pose_w2c[i];
    // camera -> world in float64, rounded once
    double R[9], t[3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) R[3 * i + j] = (double)pose_w2c[4 * j + i];
    for (int i = 0; i < 3; ++i)
        t[i] = -((R[3 * i] * (double)pose_w2c[3] + R[3 * i + 1] * (double)pose_w2c[7]) +
                 R[3 * i + 2] * (double)pose_w2c[11]);
    for (int i = 0; i < 9; ++i) c.R[i] = (float)R[i];
    for (int i = 0; i < 3; ++i) c.t[i] = (float)t[i];
    c.fx = K->fx;
    c.fy = K->fy;
    c.cx = K->cx;
    c.cy = K->cy;
    c.W = K->width;
    c.H = K->height;
    const float alpha_k = (float)(2.0 * (double)m->p.sigma * (double)m->p.sigma);
    const float norm_r = sqrtf(K->cx * K->cx + K->cy * K->cy);
    const int npix = c.W * c.H, nblk = (npix + kPixBlock - 1) / kPixBlock;
    const int frame = (int)m->frames;
    hipStream_t s = (hipStream_t)stream;
    if (depth_format == TF_DEPTH_U16_MM)
        hipLaunchKernelGGL(k_sf_points<TF_DEPTH_U16_MM>, dim3(nblk), dim3(256), 0, s, d_depth, c, alpha_k, norm_r, m->m);
    else
        hipLaunchKernelGGL(k_sf_points<TF_DEPTH_F32_M>, dim3(nblk), dim3(256), 0, s, d_depth, c, alpha_k, norm_r, m->m);
    hipLaunchKernelGGL(k_sf_splat, dim3(kSurfGrid), dim3(256), 0, s, c, m->m);
    hipLaunchKernelGGL(k_sf_assoc, dim3(nblk), dim3(256), 0, s, c, m->p.max_depth_diff, m->p.min_normal_dot, m->m);
    hipLaunchKernelGGL(k_sf_update, dim3(kSurfGrid), dim3(256), 0, s, c, m->m, frame);
    hipLaunchKernelGGL(k_sf_count, dim3(nblk), dim3(256), 0, s, npix, m->m);
    hipLaunchKernelGGL(k_sf_scan, dim3(1), dim3(1024), 0, s, nblk, m->m);
    hipLaunchKernelGGL(k_sf_append, dim3(nblk), dim3(256), 0, s, c, m->m, frame);
    hipLaunchKernelGGL(k_sf_finish, dim3(1), dim3(1), 0, s, m->m);
    if (hipGetLastError() != hipSuccess) return TF_E_HIP;
    m->frames += 1;
    m->last_w = c.W;
    m->last_h = c.H;
    return TF_OK;
}

int tf_surfel_stats(tf_surfels *m, uint32_t *h_count, uint32_t *h_flags, uint32_t *h_frames, tf_stream stream)
{
    if (!m) return TF_E_INVAL;
    SfState st;
    if (hipMemcpyAsync(&st, m->m.st, sizeof(st), hipMemcpyDeviceToHost, (hipStream_t)stream) != hipSuccess ||
        hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
        return TF_E_HIP;
    if (h_count) *h_count = st.n;
    if (h_flags) *h_flags = st.flags;
    if (h_frames) *h_frames = m->frames;
    return TF_OK;
}

int tf_surfel_export(tf_surfels *m, uint32_t n, float *d_pos, float *d_nrm, int32_t *d_time, tf_stream stream)
{
    if (!m || n > m->p.capacity) return TF_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    if (n && d_pos && hipMemcpyAsync(d_pos, m->m.pos, (size_t)n * 16, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return TF_E_HIP;
    if (n && d_nrm && hipMemcpyAsync(d_nrm, m->m.nrm, (size_t)n * 16, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return TF_E_HIP;
    if (n && d_time && hipMemcpyAsync(d_time, m->m.time, (size_t)n * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return TF_E_HIP;
    return TF_OK;
}

int tf_surfel_export_frame(tf_surfels *m, int32_t *d_index_map, int32_t *d_corr, tf_stream stream)
{
    if (!m) return TF_E_INVAL;
    const int npix = m->last_w * m->last_h;
    if (npix == 0 || (!d_index_map && !d_corr)) return TF_OK;
    hipLaunchKernelGGL(k_sf_frame_out, dim3((npix + 255) / 256), dim3(256), 0, (hipStream_t)stream, npix,
                       (const unsigned long long *)m->m.zbuf, (const int32_t *)m->m.corr, d_index_map, d_corr);
    return hipGetLastError() == hipSuccess ? TF_OK : TF_E_HIP;
}

}  // extern "C"
