// tsdf_track.hip -- the depth tracker (Sec. 4.1.1, ITMDepthTracker) on gfx950.
//
// Per iteration two launches: in k_trk_sums every thread scores the live depth
// pixels of a fixed grid-stride slice against the reference point and normal
// maps (float32 pair terms, float64 sums), the wave and then the workgroup
// reduce them in a fixed order into one partial per workgroup; k_trk_solve (one
// workgroup) reduces the partials in a fixed order, solves the 6x6 normal
// equations by Cholesky in float64 and updates the pose on the device.  The
// kernel boundary orders the partials before their reduction, so no workgroup
// needs a device-scope fence.  The pyramid levels are built by 2x2 valid-mean
// kernels first.  Nothing waits for the host, so a call can be captured in a
// HIP graph.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>

#include "tsdf_track.h"

namespace {

constexpr int kThreads = 256;
constexpr int kMaxGroups = 512;      // workgroups of a sums launch (fixed per level size)
constexpr int kTerms = 29;           // 21 (J^T J) + 6 (J^T d) + sum d^2 + pair count
constexpr int kPartStride = 32;      // doubles per workgroup partial
constexpr int kSlices = 8;           // parallel slices of the final reduction
constexpr size_t kStateBytes = 2048;

struct alignas(256) TrkState {
    double R[9], t[3];               // camera->world estimate
    float Rf[9], tf[3];              // its float32 rounding, read by the pair terms
    int32_t done[TF_TRACK_MAX_LEVELS];
    int32_t iterations[TF_TRACK_MAX_LEVELS];
    int32_t pairs[TF_TRACK_MAX_LEVELS];
    int32_t status;
    uint32_t pad;
    double sums[TF_TRACK_MAX_LEVELS][28];
};
static_assert(sizeof(TrkState) <= kStateBytes, "tracker state");
static_assert(sizeof(tf_track_result) == 1000, "result layout");

struct TrkInit {
    double R[9], t[3];
};

struct TrkLevel {
    const float *depth;
    int W, H;
    float fx, fy, cx, cy;
};

struct TrkRef {
    const float4 *V, *N;
    int W, H;
    float fx, fy, cx, cy;
    float m[12];                     // rows 0-2 of the reference world->camera matrix
};

__global__ __launch_bounds__(128) void k_trk_init(TrkState *st, TrkInit ini)
{
    const int i = threadIdx.x;
    if (i < 9) {
        st->R[i] = ini.R[i];
        st->Rf[i] = (float)ini.R[i];
    }
    if (i < 3) {
        st->t[i] = ini.t[i];
        st->tf[i] = (float)ini.t[i];
    }
    if (i < TF_TRACK_MAX_LEVELS) {
        st->done[i] = 0;
        st->iterations[i] = 0;
        st->pairs[i] = 0;
    }
    if (i == 0) {
        st->status = 0;
        st->pad = 0;
    }
    for (int k = i; k < TF_TRACK_MAX_LEVELS * 28; k += blockDim.x) (&st->sums[0][0])[k] = 0.0;
}

// a0: millimetres to metres, correctly rounded (the fusion's ingest)
__global__ __launch_bounds__(256) void k_trk_mm(const uint16_t *mm, int n, float *out)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = (float)mm[i] / 1000.0f;
}

// next pyramid level: mean of the valid depths of each 2x2 block, raster order
__global__ __launch_bounds__(256) void k_trk_down(const float *src, int Ws, float *dst, int Wd, int Hd)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= Wd * Hd) return;
    const int y = i / Wd, x = i - y * Wd;
    const float *s = src + (size_t)(2 * y) * Ws + 2 * x;
    const float v[4] = {s[0], s[1], s[Ws], s[Ws + 1]};
    float tot = 0.0f, cnt = 0.0f;
    for (int k = 0; k < 4; ++k)
        if (v[k] > 0.0f) {
            tot = tot + v[k];
            cnt = cnt + 1.0f;
        }
    dst[i] = cnt > 0.0f ? tot / cnt : 0.0f;
}

__device__ inline double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// the 6x6 solve and the pose update (one thread)
__device__ void solve_and_update(TrkState *st, const double *tot, int level, double min_update)
{
    const int n = (int)tot[28];
    st->pairs[level] = n;
    for (int k = 0; k < 28; ++k) st->sums[level][k] = tot[k];
    double A[6][6];
    int m = 0;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i; j < 6; ++j) {
            A[i][j] = tot[m];
            A[j][i] = tot[m];
            ++m;
        }
    // Cholesky A = L L^T (fully unrolled, so that everything stays in registers)
    double L[6][6];
    bool ok = n >= 6;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double s = A[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
        if (!(s > 0.0)) {
            ok = false;
            s = 1.0;
        }
        L[j][j] = sqrt(s);
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            double v = A[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
            L[i][j] = v / L[j][j];
        }
    }
    if (!ok) {
        st->done[level] = 1;
        st->status |= 1 << level;
        return;
    }
    double y[6], xi[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double v = -tot[21 + i];
#pragma unroll
        for (int k = 0; k < i; ++k) v -= L[i][k] * y[k];
        y[i] = v / L[i][i];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        double v = y[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) v -= L[k][i] * xi[k];
        xi[i] = v / L[i][i];
    }
    // dR = Exp(omega) by Rodrigues' formula
    const double wx = xi[0], wy = xi[1], wz = xi[2];
    const double th = sqrt(wx * wx + wy * wy + wz * wz);
    const double K[9] = {0.0, -wz, wy, wz, 0.0, -wx, -wy, wx, 0.0};
    double K2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            K2[3 * i + j] = K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j] + K[3 * i + 2] * K[6 + j];
    double a = 1.0, b = 0.0;
    if (th >= 1e-12) {
        a = sin(th) / th;
        b = (1.0 - cos(th)) / (th * th);
    }
    double dR[9];
    for (int k = 0; k < 9; ++k) dR[k] = (k % 4 == 0 ? 1.0 : 0.0) + a * K[k] + b * K2[k];
    double R[9], t[3];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
            R[3 * i + j] = dR[3 * i] * st->R[j] + dR[3 * i + 1] * st->R[3 + j] + dR[3 * i + 2] * st->R[6 + j];
        t[i] = dR[3 * i] * st->t[0] + dR[3 * i + 1] * st->t[1] + dR[3 * i + 2] * st->t[2] + xi[3 + i];
    }
    for (int k = 0; k < 9; ++k) {
        st->R[k] = R[k];
        st->Rf[k] = (float)R[k];
    }
    for (int k = 0; k < 3; ++k) {
        st->t[k] = t[k];
        st->tf[k] = (float)t[k];
    }
    st->iterations[level] += 1;
    double nx = 0.0;
    for (int k = 0; k < 6; ++k) nx += xi[k] * xi[k];
    if (sqrt(nx) < min_update) st->done[level] = 1;
}

// One iteration at one level, part 1: pair terms and per-workgroup sums.
__global__ __launch_bounds__(kThreads) void k_trk_sums(TrkLevel L, TrkRef r, float tau2, const TrkState *st,
                                                       double *part, int level)
{
    if (st->done[level]) return;     // the same for every workgroup of the launch
    const float R0 = st->Rf[0], R1 = st->Rf[1], R2 = st->Rf[2];
    const float R3 = st->Rf[3], R4 = st->Rf[4], R5 = st->Rf[5];
    const float R6 = st->Rf[6], R7 = st->Rf[7], R8 = st->Rf[8];
    const float t0 = st->tf[0], t1 = st->tf[1], t2 = st->tf[2];
    double acc[kTerms];
    for (int k = 0; k < kTerms; ++k) acc[k] = 0.0;
    const int n = L.W * L.H;
    for (int p = blockIdx.x * kThreads + threadIdx.x; p < n; p += gridDim.x * kThreads) {
        const float d = L.depth[p];
        if (!(d > 0.0f)) continue;
        const int y = p / L.W;
        const int x = p - y * L.W;
        const float px = d * (((float)x - L.cx) / L.fx);
        const float py = d * (((float)y - L.cy) / L.fy);
        const float pz = d;
        const float qx = ((R0 * px + R1 * py) + R2 * pz) + t0;
        const float qy = ((R3 * px + R4 * py) + R5 * pz) + t1;
        const float qz = ((R6 * px + R7 * py) + R8 * pz) + t2;
        const float cxr = ((r.m[0] * qx + r.m[1] * qy) + r.m[2] * qz) + r.m[3];
        const float cyr = ((r.m[4] * qx + r.m[5] * qy) + r.m[6] * qz) + r.m[7];
        const float czr = ((r.m[8] * qx + r.m[9] * qy) + r.m[10] * qz) + r.m[11];
        if (!(czr > 0.0f)) continue;
        const float u = (r.fx * cxr) / czr + r.cx;
        const float v = (r.fy * cyr) / czr + r.cy;
        const float ui = floorf(u + 0.5f);
        const float vi = floorf(v + 0.5f);
        if (!(ui >= 0.0f && ui <= (float)(r.W - 1) && vi >= 0.0f && vi <= (float)(r.H - 1))) continue;
        const size_t k = (size_t)(int)vi * (size_t)r.W + (size_t)(int)ui;
        const float4 V = r.V[k];
        const float4 N = r.N[k];
        if (V.w != 1.0f || N.w != 1.0f) continue;
        const float dx = qx - V.x, dy = qy - V.y, dz = qz - V.z;
        if (!((dx * dx + dy * dy) + dz * dz <= tau2)) continue;
        const float res = (dx * N.x + dy * N.y) + dz * N.z;
        const double J[6] = {(double)(qy * N.z - qz * N.y), (double)(qz * N.x - qx * N.z),
                             (double)(qx * N.y - qy * N.x), (double)N.x, (double)N.y, (double)N.z};
        int m = 0;
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = i; j < 6; ++j) acc[m++] += J[i] * J[j];
#pragma unroll
        for (int i = 0; i < 6; ++i) acc[21 + i] += J[i] * (double)res;
        acc[27] += (double)res * (double)res;
        acc[28] += 1.0;
    }
    __shared__ double wsum[kThreads / 64][kTerms];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kTerms; ++k) {
        const double s = wave_sum(acc[k]);
        if (lane == 0) wsum[wave][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < kTerms) {
        const int k = threadIdx.x;
        part[(size_t)blockIdx.x * kPartStride + k] = ((wsum[0][k] + wsum[1][k]) + wsum[2][k]) + wsum[3][k];
    }
}

// Part 2 (one workgroup): the partials of `groups` workgroups in a fixed
// order, then the solve and the pose update.
__global__ __launch_bounds__(kThreads) void k_trk_solve(TrkState *st, const double *part, int groups, int level,
                                                        double min_update)
{
    if (st->done[level]) return;
    __shared__ double red[kSlices][kTerms];
    __shared__ double tot[kTerms];
    if (threadIdx.x < kSlices * kTerms) {
        const int k = threadIdx.x / kSlices, s = threadIdx.x % kSlices;
        double v = 0.0;
        // 8 loads in flight per step, added in the same (ascending) order
        for (int g0 = s; g0 < groups; g0 += 8 * kSlices) {
            double x[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int g = g0 + j * kSlices;
                x[j] = g < groups ? part[(size_t)g * kPartStride + k] : 0.0;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (g0 + j * kSlices < groups) v += x[j];
        }
        red[s][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < kTerms) {
        double v = 0.0;
        for (int s = 0; s < kSlices; ++s) v += red[s][threadIdx.x];
        tot[threadIdx.x] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) solve_and_update(st, tot, level, min_update);
}

__global__ __launch_bounds__(128) void k_trk_finish(const TrkState *st, tf_track_result *out)
{
    const int i = threadIdx.x;
    if (i < 3) {
        // world->camera = (R^T, -R^T t)
        for (int j = 0; j < 3; ++j) out->pose_w2c[4 * i + j] = (float)st->R[3 * j + i];
        const double tw = -((st->R[i] * st->t[0] + st->R[3 + i] * st->t[1]) + st->R[6 + i] * st->t[2]);
        out->pose_w2c[4 * i + 3] = (float)tw;
    }
    if (i == 3) {
        out->pose_w2c[12] = 0.0f;
        out->pose_w2c[13] = 0.0f;
        out->pose_w2c[14] = 0.0f;
        out->pose_w2c[15] = 1.0f;
        out->status = st->status;
        out->pad = 0;
    }
    if (i < TF_TRACK_MAX_LEVELS) {
        out->iterations[i] = st->iterations[i];
        out->pairs[i] = st->pairs[i];
    }
    for (int k = i; k < TF_TRACK_MAX_LEVELS * 28; k += blockDim.x) (&out->sums[0][0])[k] = (&st->sums[0][0])[k];
}

struct TrkLayout {
    size_t state, part, level[TF_TRACK_MAX_LEVELS], total;
    int W[TF_TRACK_MAX_LEVELS], H[TF_TRACK_MAX_LEVELS];
};

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

bool track_layout(int32_t W, int32_t H, int32_t levels, TrkLayout *o)
{
    if (W < 1 || H < 1 || W > 8192 || H > 8192 || levels < 1 || levels > TF_TRACK_MAX_LEVELS) return false;
    size_t off = 0;
    o->state = off;
    off += kStateBytes;
    o->part = off;
    off += up256((size_t)kMaxGroups * kPartStride * sizeof(double));
    for (int l = 0; l < levels; ++l) {
        o->W[l] = W >> l;
        o->H[l] = H >> l;
        if (o->W[l] < 1 || o->H[l] < 1) return false;
        o->level[l] = off;
        off += up256((size_t)o->W[l] * o->H[l] * sizeof(float));
    }
    o->total = off;
    return true;
}

bool finite(float v) { return v == v && v < 1e30f && v > -1e30f; }

bool pose_ok(const float *M)
{
    if (!M) return false;
    for (int i = 0; i < 16; ++i)
        if (!finite(M[i])) return false;
    return true;
}

bool intr_ok(const tf_intrinsics *K)
{
    return K && K->width >= 1 && K->height >= 1 && K->width <= 8192 && K->height <= 8192 && K->fx > 0.0f &&
           K->fy > 0.0f && finite(K->fx) && finite(K->fy) && finite(K->cx) && finite(K->cy);
}

}  // namespace

// Shared by tf_track and the entry point that brings no workspace of its own.
int tsdf_track_impl(const void *d_depth, int depth_format, const tf_intrinsics *intr, const float *d_ref_points,
                    const float *d_ref_normals, const tf_intrinsics *ref_intr, const float ref_pose_w2c[16],
                    const float init_pose_w2c[16], const tf_track_params *tp, void *d_workspace,
                    size_t workspace_bytes, tf_track_result *d_result, tf_stream stream)
{
    if (!d_depth || !d_ref_points || !d_ref_normals || !d_workspace || !d_result || !tp) return TF_E_INVAL;
    if (depth_format != TF_DEPTH_F32_M && depth_format != TF_DEPTH_U16_MM) return TF_E_INVAL;
    if (!intr_ok(intr) || !intr_ok(ref_intr) || !pose_ok(ref_pose_w2c) || !pose_ok(init_pose_w2c)) return TF_E_INVAL;
    if (((uintptr_t)d_ref_points & 15u) || ((uintptr_t)d_ref_normals & 15u) || ((uintptr_t)d_workspace & 255u) ||
        ((uintptr_t)d_result & 7u))
        return TF_E_INVAL;
    if ((uintptr_t)d_depth & (depth_format == TF_DEPTH_F32_M ? 3u : 1u)) return TF_E_INVAL;
    const int levels = tp->n_levels;
    TrkLayout Lay;
    if (!track_layout(intr->width, intr->height, levels, &Lay)) return TF_E_INVAL;
    for (int l = 0; l < levels; ++l) {
        if (tp->iterations[l] < 0 || tp->iterations[l] > 100) return TF_E_INVAL;
        if (!(tp->dist_thresh[l] > 0.0f) || !finite(tp->dist_thresh[l])) return TF_E_INVAL;
    }
    if (!(tp->min_update >= 0.0f) || !finite(tp->min_update)) return TF_E_INVAL;
    if (workspace_bytes < Lay.total) return TF_E_SPACE;

    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)d_workspace;
    TrkState *st = (TrkState *)(ws + Lay.state);
    double *part = (double *)(ws + Lay.part);
    // the inverse of the initial world->camera matrix, in float64
    TrkInit ini;
    const float *M = init_pose_w2c;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) ini.R[3 * i + j] = (double)M[4 * j + i];
    for (int i = 0; i < 3; ++i)
        ini.t[i] = -((ini.R[3 * i] * (double)M[3] + ini.R[3 * i + 1] * (double)M[7]) + ini.R[3 * i + 2] * (double)M[11]);
    hipLaunchKernelGGL(k_trk_init, dim3(1), dim3(128), 0, s, st, ini);

    const float *lvl[TF_TRACK_MAX_LEVELS];
    if (depth_format == TF_DEPTH_U16_MM) {
        const int n = Lay.W[0] * Lay.H[0];
        float *d0 = (float *)(ws + Lay.level[0]);
        hipLaunchKernelGGL(k_trk_mm, dim3((n + 255) / 256), dim3(256), 0, s, (const uint16_t *)d_depth, n, d0);
        lvl[0] = d0;
    } else {
        lvl[0] = (const float *)d_depth;
    }
    for (int l = 1; l < levels; ++l) {
        float *dl = (float *)(ws + Lay.level[l]);
        const int n = Lay.W[l] * Lay.H[l];
        hipLaunchKernelGGL(k_trk_down, dim3((n + 255) / 256), dim3(256), 0, s, lvl[l - 1], Lay.W[l - 1], dl, Lay.W[l],
                           Lay.H[l]);
        lvl[l] = dl;
    }
    TrkRef ref;
    ref.V = (const float4 *)d_ref_points;
    ref.N = (const float4 *)d_ref_normals;
    ref.W = ref_intr->width;
    ref.H = ref_intr->height;
    ref.fx = ref_intr->fx;
    ref.fy = ref_intr->fy;
    ref.cx = ref_intr->cx;
    ref.cy = ref_intr->cy;
    for (int k = 0; k < 12; ++k) ref.m[k] = ref_pose_w2c[k];
    for (int l = levels - 1; l >= 0; --l) {
        // level intrinsics in float64, rounded once
        const double sc = (double)(1 << l);
        TrkLevel L;
        L.depth = lvl[l];
        L.W = Lay.W[l];
        L.H = Lay.H[l];
        L.fx = (float)((double)intr->fx / sc);
        L.fy = (float)((double)intr->fy / sc);
        L.cx = (float)(((double)intr->cx + 0.5) / sc - 0.5);
        L.cy = (float)(((double)intr->cy + 0.5) / sc - 0.5);
        const float tau = tp->dist_thresh[l];
        const float tau2 = tau * tau;
        const size_t npix = (size_t)L.W * L.H;
        int groups = (int)((npix + kThreads - 1) / kThreads);
        if (groups > kMaxGroups) groups = kMaxGroups;
        for (int it = 0; it < tp->iterations[l]; ++it) {
            hipLaunchKernelGGL(k_trk_sums, dim3(groups), dim3(kThreads), 0, s, L, ref, tau2, (const TrkState *)st,
                               part, l);
            hipLaunchKernelGGL(k_trk_solve, dim3(1), dim3(kThreads), 0, s, st, (const double *)part, groups, l,
                               (double)tp->min_update);
        }
    }
    hipLaunchKernelGGL(k_trk_finish, dim3(1), dim3(128), 0, s, (const TrkState *)st, d_result);
    return hipGetLastError() == hipSuccess ? TF_OK : TF_E_HIP;
}

// The workspace of tf_track_noalloc: a fixed device array, one copy per GPU,
// held until the process ends.  Host code never passes `scratch` itself to a
// kernel (in host code the name is not a device address); it passes the
// address hipGetSymbolAddress returns for the current device.
namespace {
constexpr size_t kScratchBytes = (size_t)TF_TRACK_NOALLOC_MAX_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices];

// the current device's copy of `scratch`, looked up once per device
int scratch_address(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return TF_E_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return TF_E_HIP;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return TF_OK;
}
}  // namespace

extern "C" {

int tf_track_noalloc(const void *d_depth, int depth_format, const tf_intrinsics *intr, const float *d_ref_points,
                     const float *d_ref_normals, const tf_intrinsics *ref_intr, const float ref_pose_w2c[16],
                     const float init_pose_w2c[16], const tf_track_params *params, tf_track_result *d_result,
                     tf_stream stream)
{
    if (!intr || !params) return TF_E_INVAL;
    const size_t need = tf_track_workspace_bytes(intr->width, intr->height, params->n_levels);
    if (need == 0) return TF_E_INVAL;
    if (need > kScratchBytes) return TF_E_SPACE;
    void *ws = nullptr;
    const int st = scratch_address(&ws);
    if (st != TF_OK) return st;
    return tsdf_track_impl(d_depth, depth_format, intr, d_ref_points, d_ref_normals, ref_intr, ref_pose_w2c,
                           init_pose_w2c, params, ws, kScratchBytes, d_result, stream);
}

size_t tf_track_workspace_bytes(int32_t width, int32_t height, int32_t n_levels)
{
    TrkLayout L;
    return track_layout(width, height, n_levels, &L) ? L.total : 0;
}

int tf_track(const void *d_depth, int depth_format, const tf_intrinsics *intr, const float *d_ref_points,
             const float *d_ref_normals, const tf_intrinsics *ref_intr, const float ref_pose_w2c[16],
             const float init_pose_w2c[16], const tf_track_params *params, void *d_workspace,
             size_t workspace_bytes, tf_track_result *d_result, tf_stream stream)
{
    return tsdf_track_impl(d_depth, depth_format, intr, d_ref_points, d_ref_normals, ref_intr, ref_pose_w2c,
                           init_pose_w2c, params, d_workspace, workspace_bytes, d_result, stream);
}

}  // extern "C"
