// tsdf_filter.hip -- the bilateral depth filter of the image preparation
// stage (Sec. 4; Sec. 6 useBilateralFilter) on gfx950.
//
// One workgroup per 16x16 output tile: the tile and its halo of `radius`
// pixels are staged in LDS once (u16 millimetres converted on the way), the
// spatial weights too, and each thread forms one output pixel's weighted
// mean from LDS.  The work is a small stencil: HBM traffic is one read and
// one write of the image.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "tsdf_filter.h"

namespace {

constexpr int kTile = 16;
constexpr int kMaxSide = kTile + 2 * TF_BILATERAL_MAX_RADIUS;
constexpr int kMaxTaps = (2 * TF_BILATERAL_MAX_RADIUS + 1) * (2 * TF_BILATERAL_MAX_RADIUS + 1);

struct BilArgs {
    int r;
    float inv2sr2;                 // 1 / (2 sigma_range^2)
    float ws[kMaxTaps];            // spatial weights, row-major over (dy, dx)
};

template <int FMT>
__device__ __forceinline__ float load_depth(const void *src, size_t i)
{
    if (FMT == TF_DEPTH_U16_MM) return (float)((const uint16_t *)src)[i] / 1000.0f;
    return ((const float *)src)[i];
}

template <int FMT>
__global__ __launch_bounds__(256) void k_bilateral(const void *src, int W, int H, BilArgs a, float *out)
{
    __shared__ float tile[kMaxSide * kMaxSide];
    __shared__ float ws[kMaxTaps];
    const int r = a.r, side = kTile + 2 * r, taps = (2 * r + 1) * (2 * r + 1);
    const int x0 = (int)blockIdx.x * kTile - r, y0 = (int)blockIdx.y * kTile - r;
    for (int i = threadIdx.x; i < side * side; i += 256) {
        const int ty = i / side, tx = i - ty * side;
        const int gx = x0 + tx, gy = y0 + ty;
        // outside the image reads as invalid, which the window skips
        tile[i] = (gx >= 0 && gx < W && gy >= 0 && gy < H) ? load_depth<FMT>(src, (size_t)gy * W + gx) : 0.0f;
    }
    for (int i = threadIdx.x; i < taps; i += 256) ws[i] = a.ws[i];
    __syncthreads();
    const int lx = threadIdx.x & 15, ly = threadIdx.x >> 4;
    const int x = (int)blockIdx.x * kTile + lx, y = (int)blockIdx.y * kTile + ly;
    if (x >= W || y >= H) return;
    const float *c = tile + (ly + r) * side + (lx + r);
    const float dp = c[0];
    float res = 0.0f;
    if (dp > 0.0f) {
        float sw = 0.0f, swd = 0.0f;
        int k = 0;
        for (int dy = -r; dy <= r; ++dy) {
            const float *row = c + dy * side;
            for (int dx = -r; dx <= r; ++dx, ++k) {
                const float dq = row[dx];
                if (dq > 0.0f) {
                    const float e = dq - dp;
                    const float w = ws[k] * expf(-(e * e) * a.inv2sr2);
                    sw += w;
                    swd += w * e;
                }
            }
        }
        res = dp + swd / sw;       // sw >= 1: the centre's own weight
    }
    out[(size_t)y * W + x] = res;
}

}  // namespace

extern "C" int tf_bilateral(const void *d_depth, int depth_format, int32_t width, int32_t height,
                            const tf_bilateral_params *p, float *d_out, tf_stream stream)
{
    if (!d_depth || !d_out || !p) return TF_E_INVAL;
    if (depth_format != TF_DEPTH_F32_M && depth_format != TF_DEPTH_U16_MM) return TF_E_INVAL;
    if (width < 1 || height < 1 || width > 8192 || height > 8192) return TF_E_INVAL;
    if (p->radius < 1 || p->radius > TF_BILATERAL_MAX_RADIUS) return TF_E_INVAL;
    if (!(p->sigma_space > 0.0f) || !(p->sigma_range > 0.0f) || !(p->sigma_space < 1e30f) ||
        !(p->sigma_range < 1e30f))
        return TF_E_INVAL;
    if (((uintptr_t)d_out & 3u) || ((uintptr_t)d_depth & (depth_format == TF_DEPTH_F32_M ? 3u : 1u)))
        return TF_E_INVAL;
    const size_t in_bytes = (size_t)width * height * (depth_format == TF_DEPTH_F32_M ? 4 : 2);
    const uintptr_t a0 = (uintptr_t)d_depth, a1 = a0 + in_bytes;
    const uintptr_t b0 = (uintptr_t)d_out, b1 = b0 + (size_t)width * height * 4;
    if (a0 < b1 && b0 < a1) return TF_E_INVAL;
    BilArgs a;
    a.r = p->radius;
    const double ss = p->sigma_space, sr = p->sigma_range;
    a.inv2sr2 = (float)(1.0 / (2.0 * sr * sr));
    int k = 0;
    for (int dy = -a.r; dy <= a.r; ++dy)
        for (int dx = -a.r; dx <= a.r; ++dx) a.ws[k++] = (float)exp(-(double)(dx * dx + dy * dy) / (2.0 * ss * ss));
    const dim3 grid((width + kTile - 1) / kTile, (height + kTile - 1) / kTile), block(256);
    hipStream_t s = (hipStream_t)stream;
    if (depth_format == TF_DEPTH_U16_MM)
        hipLaunchKernelGGL(k_bilateral<TF_DEPTH_U16_MM>, grid, block, 0, s, d_depth, width, height, a, d_out);
    else
        hipLaunchKernelGGL(k_bilateral<TF_DEPTH_F32_M>, grid, block, 0, s, d_depth, width, height, a, d_out);
    return hipGetLastError() == hipSuccess ? TF_OK : TF_E_HIP;
}
