// nn_kernels.hip -- gfx950 kernels of the learned depth prefilter.
//
// The 3x3 convolutions are implicit GEMMs on the bf16 matrix cores
// (v_mfma_f32_16x16x32_bf16, fp32 accumulation):
//   k_conv_fwd          encoder: M = output pixels, N = cout, K = (tap, ci);
//                       the workgroup's input tile is staged in LDS, the
//                       operand reads from it apply the stride
//   k_conv_fwd_up       decoder (nearest 2x upsampling, then 3x3): per output
//                       parity a 2x2 convolution of the source (a tile staged
//                       in LDS) on folded weights split into bf16 high and
//                       low halves, K = (source offset, half, ci)
//   k_conv_bwd_data_s2  stride-2 layers: M = input pixels, N = cin, K = the
//                       taps that reach the input pixel's parity x co
//   k_conv_bwd_data_up  decoder: the adjoint of the folded forward, K = (16
//                       parity x offset, half, co)
//   k_conv_wgrad        M = cout, N = cin of one tap, K = pixels of one chunk:
//                       both operands are staged transposed in LDS; per-chunk
//                       partial sums are reduced in a fixed order
// Bias, skip add / skip gradient and relu (mask) are fused into every
// epilogue, which is staged in LDS and written as 16-byte pixel vectors.
// The 32->1 head, the loss, input packing and Adam are plain VALU kernels.
//
// MFMA 16x16x32 operand layout (per lane l of the wave): A row l%16, k
// (l/16)*8 .. +7; B column l%16, same k; D column l%16, rows (l/16)*4 .. +3.
#include "nn_internal.h"
#include "tsdf.h"

namespace tsdf {
namespace nn {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;   // NaN
    u += 0x7fffu + ((u >> 16) & 1u);                      // round to nearest even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ u32x4 ld16(const uint16_t *p)
{
    return *(const __attribute__((address_space(1))) u32x4 *)p;
}

__device__ __forceinline__ bf16x8 as_bf(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

}  // namespace

// ============================================================================
// input packing: depth -> metres and (d / 4, valid, hp, 0 x 5) bf16, where
// hp = (d - mean of the valid 3x3 neighbours) / 5 cm on valid pixels
// ============================================================================
template <int FMT>
__device__ __forceinline__ float depth_at(const void *depth, size_t i)
{
    float d;
    if (FMT == TF_DEPTH_U16_MM)
        d = (float)reinterpret_cast<const uint16_t *>(depth)[i] / 1000.0f;
    else
        d = reinterpret_cast<const float *>(depth)[i];
    return d > 0.0f ? d : 0.0f;
}

// One workgroup per 16x16 tile of one image: the tile's depths in metres with
// a one-pixel border (-1 outside the image) are converted once into LDS, then
// each pixel sums its valid 3x3 neighbours from there in row-major order.
template <int FMT>
__global__ __launch_bounds__(256) void k_make_input(const void *depth, int N, int H, int W, uint16_t *x, float *dm)
{
    __shared__ float t[18][18];
    const int tx = (int)blockIdx.x * 16, ty = (int)blockIdx.y * 16, n = (int)blockIdx.z;
    for (int k = (int)threadIdx.x; k < 18 * 18; k += 256) {
        const int iy = ty - 1 + k / 18, ix = tx - 1 + k % 18;
        float v = -1.0f;
        if (iy >= 0 && iy < H && ix >= 0 && ix < W) v = depth_at<FMT>(depth, ((size_t)n * H + iy) * W + ix);
        t[k / 18][k % 18] = v;
    }
    __syncthreads();
    const int lx = (int)threadIdx.x & 15, ly = (int)threadIdx.x >> 4;
    const int xx = tx + lx, y = ty + ly;
    if (xx >= W || y >= H) return;
    const size_t p = ((size_t)n * H + y) * W + xx;
    const float d = t[ly + 1][lx + 1];
    float s = 0.0f, c = 0.0f;
    for (int ky = 0; ky < 3; ++ky)
        for (int kx = 0; kx < 3; ++kx) {
            const float v = t[ly + ky][lx + kx];
            if (v > 0.0f) {
                s += v;
                c += 1.0f;
            }
        }
    const float hp = d > 0.0f ? (d - s / c) / kCorrScale : 0.0f;
    dm[p] = d;
    u32x4 v = {(uint32_t)f2bf(d * 0.25f) | ((uint32_t)(d > 0.0f ? f2bf(1.0f) : 0u) << 16), (uint32_t)f2bf(hp), 0u,
               0u};
    *reinterpret_cast<u32x4 *>(x + p * 8) = v;
}

// ============================================================================
// epilogue of the implicit-GEMM convolutions.  In the MFMA result a lane holds
// 4 pixels of one channel per 16x16 tile, so the per-element bias / skip /
// activation reads and the output writes would be 2-byte accesses.  A wave
// stages each 16-pixel row tile in its own LDS tile instead; every lane then
// handles whole 16-byte vectors (one pixel, 8 channels).  The tile is the
// wave's own, so a wave-scope fence and barrier order the staging writes
// before the other lanes' reads (a wave's LDS instructions execute in order).
// ============================================================================
template <int NT>
struct alignas(16) EpiTile {
    float v[16][NT * 16 + 4];   // +4: the staging writes of one instruction hit distinct banks
};

template <int NT, typename F>
__device__ __forceinline__ void epilogue_tile(EpiTile<NT> &st, const f32x4 (&a)[NT], int lane, F &&emit)
{
    const int r = lane & 15, gq = lane >> 4;
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) st.v[gq * 4 + i][j * 16 + r] = a[j][i];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int u = 0; u < (32 * NT + 63) / 64; ++u) {
        const int v = lane + 64 * u;   // 16 pixels x 2 NT vectors of 8 channels
        if (v < 32 * NT) {
            const int pix = v / (2 * NT), c8 = (v - pix * 2 * NT) * 8;
            const f32x4 lo = *reinterpret_cast<const f32x4 *>(&st.v[pix][c8]);
            const f32x4 hi = *reinterpret_cast<const f32x4 *>(&st.v[pix][c8 + 4]);
            emit(pix, c8, lo, hi);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// two floats to packed bf16 (low half = a) by v_cvt_pk_bf16_f32: round to
// nearest even, the same bits as f2bf for every finite value
__device__ __forceinline__ uint32_t bf2(float a, float b)
{
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    bf16x2 v;
    v[0] = (__bf16)a;
    v[1] = (__bf16)b;
    return __builtin_bit_cast(uint32_t, v);
}

// forward: o[e] = bf16(relu(x[e] + bias[e] (+ skip[e]))), e = 0..7
template <bool SKIP>
__device__ __forceinline__ void fwd_store8(uint16_t *o, f32x4 lo, f32x4 hi, const float *bias, const uint16_t *skip)
{
    const float x[8] = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    u32x4 sk = {0u, 0u, 0u, 0u};
    if (SKIP) sk = ld16(skip);
    u32x4 ov;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        float v0 = x[2 * e] + bias[2 * e], v1 = x[2 * e + 1] + bias[2 * e + 1];
        if (SKIP) {
            v0 += bf2f((uint16_t)(sk[e] & 0xffffu));
            v1 += bf2f((uint16_t)(sk[e] >> 16));
        }
        ov[e] = bf2(v0 > 0.0f ? v0 : 0.0f, v1 > 0.0f ? v1 : 0.0f);
    }
    *reinterpret_cast<u32x4 *>(o) = ov;
}

// backward data: o[e] = bf16(x[e] (+ skipg[e])), zero where act[e] <= 0
template <bool SKIP>
__device__ __forceinline__ void bwd_store8(uint16_t *o, f32x4 lo, f32x4 hi, const uint16_t *skipg, const uint16_t *act)
{
    const float x[8] = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    u32x4 sk = {0u, 0u, 0u, 0u};
    if (SKIP) sk = ld16(skipg);
    const u32x4 av = ld16(act);
    u32x4 ov;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        float v0 = x[2 * e], v1 = x[2 * e + 1];
        if (SKIP) {
            v0 += bf2f((uint16_t)(sk[e] & 0xffffu));
            v1 += bf2f((uint16_t)(sk[e] >> 16));
        }
        if (!(bf2f((uint16_t)(av[e] & 0xffffu)) > 0.0f)) v0 = 0.0f;
        if (!(bf2f((uint16_t)(av[e] >> 16)) > 0.0f)) v1 = 0.0f;
        ov[e] = bf2(v0, v1);
    }
    *reinterpret_cast<u32x4 *>(o) = ov;
}

// ============================================================================
// fp32 master weights -> bf16 GEMM operands of every conv layer
// ============================================================================
// Forward operands are stored in MFMA fragment order: element
// ((step * cout / 16 + tile) * 64 + lane) * 8 + e holds the B value of lane
// lane = gq * 16 + r at K step `step`, i.e. output channel tile * 16 + r and
// k = step * 32 + gq * 8 + e.  The 64 lanes' 16-byte fragments of one (step,
// tile) are contiguous, so a fragment load reads whole cache lines.
__device__ __forceinline__ void frag_coords(int j, int cout, int &co, int &k)
{
    const int e = j & 7, lane = (j >> 3) & 63, st = (j >> 9) / (cout / 16), tile = (j >> 9) - st * (cout / 16);
    co = tile * 16 + (lane & 15);
    k = st * 32 + (lane >> 4) * 8 + e;
}

__device__ __forceinline__ void pack_g(const float *w, int cin, int cinp, int cout, int i, uint16_t *g)
{
    int co, k;
    frag_coords(i, cout, co, k);
    const int tap = k / cinp, ci = k % cinp;
    g[i] = (tap < 9 && ci < cin) ? f2bf(w[(co * 9 + tap) * cin + ci]) : (uint16_t)0;
}

__device__ __forceinline__ void pack_t(const float *w, int cin, int cout, int i, uint16_t *t)
{
    const int ci = i / (9 * cout), k = i % (9 * cout), tap = k / cout, co = k % cout;
    t[i] = ci < cin ? f2bf(w[(co * 9 + tap) * cin + ci]) : (uint16_t)0;
}

// Nearest 2x upsampling followed by a 3x3 convolution, folded by output
// parity: output pixel (2m + py, 2n + px) reads only the 2x2 source pixels
// (m + py - 1 + a, n + px - 1 + b), a, b in {0, 1}.  Tap ky lands on source
// row offset a = ((py + ky - 1) >> 1) + 1 - py (likewise kx -> b): per axis
// one offset receives one tap and the other two, so per parity the four
// offsets receive 1, 2, 2 and 4 of the 9 taps.  The folded weight of an
// offset is s = the fp32 sum of the bf16 taps landing there (ascending ky,
// kx); it is carried as two bf16 numbers, hi = bf16(s) and lo = bf16(s - hi),
// so that a product with a bf16 activation sums the taps' products: hi + lo
// equals s exactly where at most two taps land (the rounding error of a
// two-term sum is representable in the same precision) and within 2^-17 of
// s at the four-tap offset.  The one-tap offset (a, b) = (py, px) has lo = 0.
// Zero padding agrees: a source row is outside the image exactly when every
// tap landing on it is.
__device__ __forceinline__ uint16_t folded_weight(const float *w, int cin, int par, int co, int q, int ci, int lo)
{
    const int py = par >> 1, px = par & 1, a = q >> 1, b = q & 1;
    float s = 0.0f;
    if (ci < cin)
        for (int ky = 0; ky < 3; ++ky) {
            if (((py + ky - 1) >> 1) + 1 - py != a) continue;
            for (int kx = 0; kx < 3; ++kx) {
                if (((px + kx - 1) >> 1) + 1 - px != b) continue;
                s += bf2f(f2bf(w[(co * 9 + ky * 3 + kx) * cin + ci]));
            }
        }
    const uint16_t hi = f2bf(s);
    return lo ? f2bf(s - bf2f(hi)) : hi;
}

// forward operand gu[lo][par][cout x 4 cinp matrix in fragment order], the
// matrix's K index k = q * cinp + ci, q = a * 2 + b
__device__ __forceinline__ void pack_up(const float *w, int cin, int cinp, int cout, int i, uint16_t *gu)
{
    const int k4 = 4 * cinp;
    const int half = 4 * cout * k4;
    const int lo = i / half, j = i - lo * half;
    const int par = j / (cout * k4), rem = j - par * cout * k4;
    int co, k;
    frag_coords(rem, cout, co, k);
    const int q = k / cinp, ci = k - (k / cinp) * cinp;
    gu[i] = folded_weight(w, cin, par, co, q, ci, lo);
}

// backward-data operand of the same folded weights: tu[lo][ci][(par * 4 + q) * cout + co]
__device__ __forceinline__ void pack_tu(const float *w, int cin, int cinp, int cout, int i, uint16_t *tu)
{
    const int half = cinp * 16 * cout;
    const int lo = i / half, j = i - lo * half;
    const int ci = j / (16 * cout), rem = j - ci * 16 * cout, pq = rem / cout, co = rem - (rem / cout) * cout;
    tu[i] = folded_weight(w, cin, pq >> 2, co, pq & 3, ci, lo);
}

// every conv layer's packed weights in one launch: thread i belongs to the
// layer whose [start, next start) range holds it
__global__ __launch_bounds__(256) void k_pack(PackJobs J)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    int l = 0;
    while (l < kLayers - 1 && i >= J.start[l + 1]) ++l;
    if (l >= kLayers - 1) return;
    const PackJob &p = J.job[l];
    const int li = i - J.start[l];
    if (li < p.n_g) {
        if (p.up)
            pack_up(p.w, p.cin, p.cinp, p.cout, li, p.g);
        else
            pack_g(p.w, p.cin, p.cinp, p.cout, li, p.g);
    }
    if (p.t && li < p.n_t) {
        if (p.up)
            pack_tu(p.w, p.cin, p.cinp, p.cout, li, p.t);
        else
            pack_t(p.w, p.cin, p.cout, li, p.t);
    }
}

// ============================================================================
// Workgroups of the staged forward kernels go round-robin to the 8 XCDs;
// remapped so that XCD x takes the x-th contiguous band of tiles, the
// neighbouring tiles that share input rows share that XCD's L2.  The grid is
// rounded up to a multiple of 8; tiles past the end stage zeros and store
// nothing.
// ============================================================================
__device__ __forceinline__ long xcd_band_tile(long ntiles)
{
    const long per = (ntiles + 7) / 8;
    return (long)(blockIdx.x % 8u) * per + blockIdx.x / 8u;
}

// stage rows iy0 .. iy0 + IR - 1, columns ix0 .. ix0 + IC - 1 of one image's
// NHWC bf16 tensor (CINP channels) in LDS, RS bytes per pixel, zeros outside
template <int CINP, int IR, int IC, int RS>
__device__ __forceinline__ void stage_tile(unsigned char *tile, const uint16_t *in, int nimg, int Hs, int Ws,
                                           int iy0, int ix0, bool live)
{
    constexpr int CH = CINP / 8;
    for (int i = (int)threadIdx.x; i < IR * IC * CH; i += 256) {
        const int ch = i % CH, pc = i / CH, c = pc % IC, rr = pc / IC;
        const int sy = iy0 + rr, sx = ix0 + c;
        u32x4 v = {0u, 0u, 0u, 0u};
        if (live && sy >= 0 && sy < Hs && sx >= 0 && sx < Ws)
            v = ld16(in + (((size_t)nimg * Hs + sy) * Ws + sx) * CINP + ch * 8);
        *reinterpret_cast<u32x4 *>(tile + (rr * IC + c) * RS + ch * 16) = v;
    }
    __syncthreads();
}

// ============================================================================
// forward 3x3 convolution (no skip input): a workgroup takes ROWS = 4 / NS
// output rows x 16 T columns; it stages the input rows and columns those
// reach (with the stride) in LDS with coalesced 16-byte loads, then each
// wave computes 16 T pixels of one row x COUT / NS channels, A fragments
// from LDS, B fragments (fragment order) from global memory
// ============================================================================
template <int CINP, int COUT, int STRIDE, int T, int NS>
__global__ __launch_bounds__(256) void k_conv_fwd(const uint16_t *in, int Hs, int Ws, const uint16_t *g,
                                                  const float *bias, uint16_t *out, int N, int Ho, int Wo)
{
    static_assert(NS == 1 || NS == 2 || NS == 4, "channel split must divide the 4 waves of a workgroup");
    constexpr int KP = ((9 * CINP + 31) / 32) * 32;
    constexpr int NT = COUT / 16 / NS;
    constexpr int ROWS = 4 / NS;
    constexpr int IR = STRIDE * (ROWS - 1) + 3, IC = STRIDE * (16 * T - 1) + 3;
    constexpr int RS = CINP * 2 + 16;   // +16 bytes: neighbouring pixels' fragments start on different banks
    __shared__ __attribute__((aligned(16))) unsigned char tile[IR * IC * RS];
    const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6, r = lane & 15, gq = lane >> 4;
    const int tx = (Wo + 16 * T - 1) / (16 * T), ty = (Ho + ROWS - 1) / ROWS;
    const long ntiles = (long)N * ty * tx;
    const long wt = xcd_band_tile(ntiles);
    const bool live = wt < ntiles;
    const long gt = live ? wt : 0;
    const int xt = (int)(gt % tx);
    const long nyt = gt / tx;
    const int nimg = (int)(nyt / ty), y0 = (int)(nyt - (long)nimg * ty) * ROWS, x0 = xt * 16 * T;
    stage_tile<CINP, IR, IC, RS>(tile, in, nimg, Hs, Ws, STRIDE * y0 - 1, STRIDE * x0 - 1, live);
    const int yy = w / NS, cbase = (w % NS) * (COUT / NS);
    f32x4 acc[T][NT];
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[t][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int k0 = 0; k0 < KP; k0 += 32) {
        const int k = k0 + gq * 8;
        const int tap = k / CINP, ci = k - (k / CINP) * CINP;
        const int ky = tap / 3, kx = tap - (tap / 3) * 3;
        bf16x8 a[T];
#pragma unroll
        for (int t = 0; t < T; ++t) {
            u32x4 v = {0u, 0u, 0u, 0u};
            if (tap < 9)   // K padding past the 9 taps multiplies zeros
                v = *reinterpret_cast<const u32x4 *>(tile + ((STRIDE * yy + ky) * IC + STRIDE * (t * 16 + r) + kx) * RS +
                                                     ci * 2);
            a[t] = as_bf(v);
        }
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const bf16x8 b = as_bf(ld16(g + ((size_t)((k0 / 32) * (COUT / 16) + cbase / 16 + j) * 64 + lane) * 8));
#pragma unroll
            for (int t = 0; t < T; ++t) acc[t][j] = mfma(a[t], b, acc[t][j]);
        }
    }
    __shared__ EpiTile<NT> st[4];
    const int oy = y0 + yy;
#pragma unroll
    for (int t = 0; t < T; ++t)
        epilogue_tile(st[w], acc[t], lane, [&](int pix, int c8, f32x4 lo, f32x4 hi) {
            const int ox = x0 + t * 16 + pix;
            if (!live || oy >= Ho || ox >= Wo) return;
            const size_t p = ((size_t)nimg * Ho + oy) * Wo + ox;
            const int co = cbase + c8;
            fwd_store8<false>(out + p * COUT + co, lo, hi, bias + co, nullptr);
        });
}

// Forward of an upsampled layer on the parity-folded weights (split into
// high and low halves; the one-tap offset has no low half: 7 cinp
// multiply-adds per output instead of 9 cinp).  A workgroup = the 4 output
// parities (one per wave) of one (image, source row m, run of 16 T source
// columns) and one of NS shares of the output channels; it stages source
// rows m - 1 .. m + 1 and columns c0 - 1 .. c0 + 16 T, which every parity's
// 2x2 offsets read, in LDS.
template <int CINP, int COUT, bool SKIP, int T, int NS>
__global__ __launch_bounds__(256) void k_conv_fwd_up(const uint16_t *in, int Hs, int Ws, const uint16_t *gu,
                                                     const float *bias, const uint16_t *skip, uint16_t *out, int N)
{
    constexpr int K4 = 4 * CINP;
    constexpr int NT = COUT / 16 / NS;
    constexpr int TC = 16 * T + 2;
    constexpr int RS = CINP * 2 + 16;
    static_assert(CINP % 32 == 0, "a K step stays inside one source offset");
    __shared__ __attribute__((aligned(16))) unsigned char tile[3 * TC * RS];
    const int lane = (int)threadIdx.x & 63, r = lane & 15, gq = lane >> 4;
    const int runs = (Ws + 16 * T - 1) / (16 * T);
    const long ntiles = (long)N * Hs * runs * NS;
    const long wt = xcd_band_tile(ntiles);
    const bool live = wt < ntiles;
    const int cbase = (int)(wt % NS) * (COUT / NS);
    const long gt = live ? wt / NS : 0;
    const int run = (int)(gt % runs);
    const long nm = gt / runs;
    const int nimg = (int)(nm / Hs), m = (int)(nm - (long)nimg * Hs);
    const int c0 = run * 16 * T;
    stage_tile<CINP, 3, TC, RS>(tile, in, nimg, Hs, Ws, m - 1, c0 - 1, live);
    const int par = (int)threadIdx.x >> 6;
    const int py = par >> 1, px = par & 1;
    const int Ho = 2 * Hs, Wo = 2 * Ws;
    f32x4 acc[T][NT];
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[t][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const uint16_t *gp = gu + (size_t)par * COUT * K4;
    const uint16_t *gl = gp + (size_t)4 * COUT * K4;   // low halves
#pragma unroll 2
    for (int k0 = 0; k0 < K4; k0 += 32) {
        const int k = k0 + gq * 8;
        const int q = k / CINP, ci = k - (k / CINP) * CINP;
        const bool split = q != par;   // wave-uniform: one source offset per K step
        const int row = py + (q >> 1);
        bf16x8 av[T];
#pragma unroll
        for (int t = 0; t < T; ++t)
            av[t] = as_bf(*reinterpret_cast<const u32x4 *>(tile + (row * TC + t * 16 + r + px + (q & 1)) * RS + ci * 2));
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const size_t wo = ((size_t)((k0 / 32) * (COUT / 16) + cbase / 16 + j) * 64 + lane) * 8;
            const bf16x8 b = as_bf(ld16(gp + wo));
#pragma unroll
            for (int t = 0; t < T; ++t) acc[t][j] = mfma(av[t], b, acc[t][j]);
            if (split) {
                const bf16x8 bl = as_bf(ld16(gl + wo));
#pragma unroll
                for (int t = 0; t < T; ++t) acc[t][j] = mfma(av[t], bl, acc[t][j]);
            }
        }
    }
    const size_t orow = ((size_t)nimg * Ho + 2 * m + py) * Wo;
    __shared__ EpiTile<NT> st[4];
#pragma unroll
    for (int t = 0; t < T; ++t)
        epilogue_tile(st[par], acc[t], lane, [&](int pix, int c8, f32x4 lo, f32x4 hi) {
            const int nn = c0 + t * 16 + pix;
            if (!live || nn >= Ws) return;
            const size_t p = orow + 2 * nn + px;
            const int co = cbase + c8;
            fwd_store8<SKIP>(out + p * COUT + co, lo, hi, bias + co, SKIP ? skip + p * COUT + co : nullptr);
        });
}

// ============================================================================
// backward data: gradient at the conv input (the source, for an upsampled
// input), then + skip gradient, then the source's relu mask
// ============================================================================
// backward data of an upsampled layer: the adjoint of the parity-folded
// forward.  Source pixel (m, n) collects, for each output parity (py, px)
// and source offset (a, b), the output pixel (2 m' + py, 2 n' + px) with
// m' = m + 1 - py - a, n' = n + 1 - px - b, on the same split folded
// weights as the forward (high and low halves; 28 COUT multiply-adds per
// source channel instead of 36 COUT).  Then the source's relu mask.  A wave
// takes 32 source pixels and CIN / NS channels.
template <int CIN, int COUT, int NS>
__global__ __launch_bounds__(256) void k_conv_bwd_data_up(const uint16_t *gpre, const uint16_t *tu,
                                                          const uint16_t *act, uint16_t *gout, int N, int Hs, int Ws)
{
    static_assert(NS == 1 || NS == 2 || NS == 4, "channel split must divide the 4 waves of a workgroup");
    static_assert(COUT % 32 == 0, "a K step is 32 output channels of one (parity, offset)");
    constexpr int K16 = 16 * COUT;
    constexpr int NT = CIN / 16 / NS;
    const int lane = (int)threadIdx.x & 63, r = lane & 15, gq = lane >> 4;
    const long P = (long)N * Hs * Ws;
    const int Ho = 2 * Hs, Wo = 2 * Ws;
    const int wid = (int)blockIdx.x * 4 + ((int)threadIdx.x >> 6);
    const int cbase = (wid % NS) * (CIN / NS);
    const long p0 = (long)(wid / NS) * 32;   // waves past P load nothing and store nothing
    int pn[2], pm[2], pnn[2];
    bool pv[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        long p = p0 + t * 16 + r;
        pv[t] = p < P;
        if (!pv[t]) p = 0;
        pn[t] = (int)(p / ((long)Hs * Ws));
        const int rem = (int)(p - (long)pn[t] * Hs * Ws);
        pm[t] = rem / Ws;
        pnn[t] = rem - pm[t] * Ws;
    }
    f32x4 acc[2][NT];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[t][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const uint16_t *tl = tu + (size_t)CIN * K16;   // low halves
    for (int pq = 0; pq < 16; ++pq) {
        const int py = pq >> 3, px = (pq >> 2) & 1, a = (pq >> 1) & 1, b = pq & 1;
        const bool split = (pq & 3) != (pq >> 2);   // offset (a, b) != (py, px): two or four taps
#pragma unroll 2
        for (int co0 = 0; co0 < COUT; co0 += 32) {
            const int co = co0 + gq * 8;
            bf16x8 av[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int mo = pm[t] + 1 - py - a, no = pnn[t] + 1 - px - b;
                u32x4 v = {0u, 0u, 0u, 0u};
                if (pv[t] && mo >= 0 && mo < Hs && no >= 0 && no < Ws)
                    v = ld16(gpre + (((size_t)pn[t] * Ho + 2 * mo + py) * Wo + 2 * no + px) * COUT + co);
                av[t] = as_bf(v);
            }
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const size_t wo = (size_t)(cbase + j * 16 + r) * K16 + pq * COUT + co;
                const bf16x8 bv = as_bf(ld16(tu + wo));
                acc[0][j] = mfma(av[0], bv, acc[0][j]);
                acc[1][j] = mfma(av[1], bv, acc[1][j]);
                if (split) {
                    const bf16x8 bl = as_bf(ld16(tl + wo));
                    acc[0][j] = mfma(av[0], bl, acc[0][j]);
                    acc[1][j] = mfma(av[1], bl, acc[1][j]);
                }
            }
        }
    }
    __shared__ EpiTile<NT> st[4];
#pragma unroll
    for (int t = 0; t < 2; ++t)
        epilogue_tile(st[threadIdx.x >> 6], acc[t], lane, [&](int pix, int c8, f32x4 lo, f32x4 hi) {
            const long p = p0 + t * 16 + pix;
            if (p >= P) return;
            const size_t o = (size_t)p * CIN + cbase + c8;
            bwd_store8<false>(gout + o, lo, hi, nullptr, act + o);
        });
}

// backward data of a stride-2 layer by input parity: input pixel
// (2m + py, 2n + px) receives gradient only through the taps ky = 1 (py = 0)
// or ky in {0, 2} (py = 1), likewise kx, from output pixel
// ((iy + 1 - ky) / 2, (ix + 1 - kx) / 2) -- 1, 2 or 4 of the 9 taps.  A wave
// takes 32 same-parity columns of one input row and CIN / NS channels; the
// skip gradient and the relu mask are fused as in k_conv_bwd_data.
template <int CIN, int COUT, bool SKIP, int NS>
__global__ __launch_bounds__(256) void k_conv_bwd_data_s2(const uint16_t *gpre, int Ho, int Wo, const uint16_t *tw,
                                                          const uint16_t *skipg, const uint16_t *act, uint16_t *gout,
                                                          int N, int Hq, int Wq)
{
    static_assert(NS == 1 || NS == 2 || NS == 4, "channel split must divide the 4 waves of a workgroup");
    static_assert(COUT % 32 == 0, "a K step is 32 output channels of one tap");
    constexpr int K9 = 9 * COUT;
    constexpr int NT = CIN / 16 / NS;
    const int lane = (int)threadIdx.x & 63, r = lane & 15, gq = lane >> 4;
    const int Wh = (Wq + 1) >> 1, runs = (Wh + 31) >> 5;
    const long wid = (long)blockIdx.x * 4 + ((int)threadIdx.x >> 6);
    const bool live = wid / NS < (long)N * Hq * 2 * runs;   // dead waves still join the epilogue barriers
    const long grp = live ? wid / NS : 0;
    const int cbase = (int)(wid % NS) * (CIN / NS);
    const int run = (int)(grp % runs);
    const long rp = grp / runs;
    const int px = (int)(rp & 1);
    const long ni = rp >> 1;   // image * Hq + input row
    const int nimg = (int)(ni / Hq), iy = (int)(ni - (long)nimg * Hq);
    const int py = iy & 1;
    f32x4 acc[2][NT];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[t][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int nty = py ? 2 : 1, ntx = px ? 2 : 1;
    for (int a = 0; a < nty; ++a) {
        const int ky = py ? 2 * a : 1;
        const int oy = (iy + 1 - ky) >> 1;
        const bool rowok = oy >= 0 && oy < Ho;
        for (int b = 0; b < ntx; ++b) {
            const int kx = px ? 2 * b : 1;
            const int tap = ky * 3 + kx;
            for (int co0 = 0; co0 < COUT; co0 += 32) {
                const int co = co0 + gq * 8;
                bf16x8 av[2];
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const int ix = 2 * (run * 32 + t * 16 + r) + px;
                    const int ox = (ix + 1 - kx) >> 1;
                    u32x4 v = {0u, 0u, 0u, 0u};
                    if (rowok && ix < Wq && ox >= 0 && ox < Wo)
                        v = ld16(gpre + (((size_t)nimg * Ho + oy) * Wo + ox) * COUT + co);
                    av[t] = as_bf(v);
                }
#pragma unroll
                for (int j = 0; j < NT; ++j) {
                    const bf16x8 bv = as_bf(ld16(tw + (size_t)(cbase + j * 16 + r) * K9 + tap * COUT + co));
                    acc[0][j] = mfma(av[0], bv, acc[0][j]);
                    acc[1][j] = mfma(av[1], bv, acc[1][j]);
                }
            }
        }
    }
    const size_t prow = ((size_t)nimg * Hq + iy) * Wq;
    __shared__ EpiTile<NT> st[4];
#pragma unroll
    for (int t = 0; t < 2; ++t)
        epilogue_tile(st[threadIdx.x >> 6], acc[t], lane, [&](int pix, int c8, f32x4 lo, f32x4 hi) {
            const int ix = 2 * (run * 32 + t * 16 + pix) + px;
            if (!live || ix >= Wq) return;
            const size_t o = (prow + ix) * CIN + cbase + c8;
            bwd_store8<SKIP>(gout + o, lo, hi, SKIP ? skipg + o : nullptr, act + o);
        });
}

// ============================================================================
// weight gradient of one tap over one pixel chunk:
// partial[chunk][co][tap][ci] = sum_p gpre[p][co] * in_tap(p)[ci]; the bias
// gradient partial[chunk][co] comes from the tap-0 workgroups
// ============================================================================
template <int CINP, int COUT, int STRIDE, bool UP, bool FOLD>
__global__ __launch_bounds__(256) void k_conv_wgrad(const uint16_t *gpre, const uint16_t *in, int Hs, int Ws, int N,
                                                    int Ho, int Wo, float *partial, float *partial_b, int chunk_pix,
                                                    int nchunk)
{
    static_assert(!FOLD || (UP && STRIDE == 1), "the parity fold is for upsampled stride-1 layers");
    constexpr int CT = CINP < 16 ? 16 : CINP;
    constexpr int NTAP = FOLD ? 16 : 9;   // taps, or (output parity, source offset) pairs
    constexpr int MT = COUT / 16, NTT = CT / 16, TILES = MT * NTT, TPW = (TILES + 3) / 4;
    constexpr int KS = kWgradStep;   // pixels staged per round (4 MFMA k-steps)
    constexpr int LD = KS + 8;       // LDS row pitch in bf16 elements (16-byte aligned rows)
    constexpr int GV = KS * (COUT / 8), IV = KS * (CT / 8);   // 16-byte vectors staged per round
    static_assert(KS % 64 == 0, "the column swizzle below permutes within 64-pixel spans");
    // the pixel column of LDS row `row` is XORed with 8 ((row / 8) % 8): the
    // transposed 16-bit writes of one instruction (8 rows apart per lane
    // group) then spread over the banks, and 8 consecutive pixels stay one
    // aligned 16-byte operand read
    auto swz = [](int row) { return ((row >> 3) & 7) << 3; };
    __shared__ uint16_t gT[COUT][LD];
    __shared__ uint16_t iT[CT][LD];
    // workgroups are dealt to the 8 XCDs round-robin by their linear index:
    // the NTAP taps of a chunk get indices of one residue mod 8, so they run
    // on one XCD and read the chunk's gradient and input through the same L2
    const int id = (int)blockIdx.x, slot = id >> 3;
    const int chunk = (id & 7) + 8 * (slot / NTAP), tap = slot - (slot / NTAP) * NTAP;
    if (chunk >= nchunk) return;
    const int ky = tap / 3, kx = tap - (tap / 3) * 3;
    // FOLD: tap = (py * 2 + px) * 4 + a * 2 + b; the pixels are the source
    // grid (m, n), read at output (2m + py, 2n + px) and source
    // (m + py - 1 + a, n + px - 1 + b)
    const int fpy = tap >> 3, fpx = (tap >> 2) & 1, fa = (tap >> 1) & 1, fb = tap & 1;
    const long P = FOLD ? (long)N * Hs * Ws : (long)N * Ho * Wo;
    const long c0 = (long)chunk * chunk_pix;
    const long c1 = c0 + chunk_pix < P ? c0 + chunk_pix : P;
    const int w = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63, r = lane & 15, gq = lane >> 4;
    const int Hc = UP ? 2 * Hs : Hs, Wc = UP ? 2 * Ws : Ws;
    f32x4 acc[TPW];
#pragma unroll
    for (int j = 0; j < TPW; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bpart = 0.0f;   // bias gradient: thread threadIdx.x < COUT owns channel threadIdx.x
    for (long pb = c0; pb < c1; pb += KS) {
        u32x4 gv[(GV + 255) / 256], iv[(IV + 255) / 256];
#pragma unroll
        for (int q = 0; q < (GV + 255) / 256; ++q) {
            const int v = (int)threadIdx.x + 256 * q;
            const int pi = v / (COUT / 8), cv = (v - pi * (COUT / 8)) * 8;
            const long p = pb + pi;
            gv[q] = u32x4{0u, 0u, 0u, 0u};
            if (v < GV && p < c1) {
                size_t po = (size_t)p;
                if (FOLD) {
                    const int n = (int)(p / ((long)Hs * Ws));
                    const int rem = (int)(p - (long)n * Hs * Ws);
                    const int m = rem / Ws, nn = rem - (rem / Ws) * Ws;
                    po = ((size_t)n * Ho + 2 * m + fpy) * Wo + 2 * nn + fpx;
                }
                gv[q] = ld16(gpre + po * COUT + cv);
            }
        }
#pragma unroll
        for (int q = 0; q < (IV + 255) / 256; ++q) {
            const int v = (int)threadIdx.x + 256 * q;
            const int pi = v / (CT / 8), cv = (v - pi * (CT / 8)) * 8;
            const long p = pb + pi;
            iv[q] = u32x4{0u, 0u, 0u, 0u};
            if (FOLD && v < IV && p < c1 && cv < CINP) {
                const int n = (int)(p / ((long)Hs * Ws));
                const int rem = (int)(p - (long)n * Hs * Ws);
                const int m = rem / Ws, nn = rem - (rem / Ws) * Ws;
                const int sy = m + fpy - 1 + fa, sx = nn + fpx - 1 + fb;
                if (sy >= 0 && sy < Hs && sx >= 0 && sx < Ws)
                    iv[q] = ld16(in + (((size_t)n * Hs + sy) * Ws + sx) * CINP + cv);
            } else if (!FOLD && v < IV && p < c1 && cv < CINP) {
                const int n = (int)(p / ((long)Ho * Wo));
                const int rem = (int)(p - (long)n * Ho * Wo);
                const int oy = rem / Wo, ox = rem - (rem / Wo) * Wo;
                const int iy = STRIDE * oy + ky - 1, ix = STRIDE * ox + kx - 1;
                if (iy >= 0 && iy < Hc && ix >= 0 && ix < Wc) {
                    const int sy = UP ? (iy >> 1) : iy, sx = UP ? (ix >> 1) : ix;
                    iv[q] = ld16(in + (((size_t)n * Hs + sy) * Ws + sx) * CINP + cv);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < (GV + 255) / 256; ++q) {
            const int v = (int)threadIdx.x + 256 * q;
            const int pi = v / (COUT / 8), cv = (v - pi * (COUT / 8)) * 8;
            if (v < GV)
#pragma unroll
                for (int e = 0; e < 8; ++e) gT[cv + e][pi ^ swz(cv + e)] = (uint16_t)(gv[q][e >> 1] >> (16 * (e & 1)));
        }
#pragma unroll
        for (int q = 0; q < (IV + 255) / 256; ++q) {
            const int v = (int)threadIdx.x + 256 * q;
            const int pi = v / (CT / 8), cv = (v - pi * (CT / 8)) * 8;
            if (v < IV)
#pragma unroll
                for (int e = 0; e < 8; ++e) iT[cv + e][pi ^ swz(cv + e)] = (uint16_t)(iv[q][e >> 1] >> (16 * (e & 1)));
        }
        __syncthreads();
        if ((FOLD ? (tap & 3) : tap) == 0 && (int)threadIdx.x < COUT)
            for (int k = 0; k < KS; ++k) bpart += bf2f(gT[threadIdx.x][k ^ swz((int)threadIdx.x)]);
#pragma unroll
        for (int kk = 0; kk < KS; kk += 32)
#pragma unroll
            for (int j = 0; j < TPW; ++j) {
                const int tile = w * TPW + j;
                if (tile < TILES) {
                    const int mt = tile / NTT, nt = tile - (tile / NTT) * NTT;
                    const bf16x8 a = as_bf(*reinterpret_cast<const u32x4 *>(&gT[mt * 16 + r][(kk + gq * 8) ^ swz(mt * 16 + r)]));
                    const bf16x8 b = as_bf(*reinterpret_cast<const u32x4 *>(&iT[nt * 16 + r][(kk + gq * 8) ^ swz(nt * 16 + r)]));
                    acc[j] = mfma(a, b, acc[j]);
                }
            }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
        const int tile = w * TPW + j;
        if (tile >= TILES) continue;
        const int mt = tile / NTT, nt = tile - (tile / NTT) * NTT;
        const int ci = nt * 16 + r;
        if (ci >= CINP) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int co = mt * 16 + gq * 4 + i;
            partial[(((size_t)chunk * COUT + co) * NTAP + tap) * CINP + ci] = acc[j][i];
        }
    }
    // bias partials: one per chunk, or one per chunk and output parity (FOLD)
    if (FOLD && (tap & 3) == 0 && (int)threadIdx.x < COUT)
        partial_b[((size_t)chunk * 4 + (tap >> 2)) * COUT + threadIdx.x] = bpart;
    if (!FOLD && tap == 0 && (int)threadIdx.x < COUT) partial_b[(size_t)chunk * COUT + threadIdx.x] = bpart;
}

// weight gradient of the first layer (8 padded input channels, stride 1):
// all 9 taps in one workgroup as the N rows tap * 8 + ci (72 rows, padded to
// 80 with zeros), so the gradient operand is staged once per chunk instead of
// once per tap; same partial layout as k_conv_wgrad ([chunk][co][tap][ci])
template <int COUT>
__global__ __launch_bounds__(256) void k_conv_wgrad_c8(const uint16_t *gpre, const uint16_t *in, int H, int W, int N,
                                                       float *partial, float *partial_b, int chunk_pix, int nchunk)
{
    constexpr int KS = kWgradStep;
    constexpr int LD = KS + 8;
    constexpr int NR = 80;   // 72 (tap, ci) rows + 8 zero rows
    constexpr int MT = COUT / 16, NTT = NR / 16, TILES = MT * NTT, TPW = (TILES + 3) / 4;
    constexpr int GV = KS * (COUT / 8), IV = KS * 9;   // 16-byte vectors staged per round
    static_assert(KS == 64, "one staging vector per (tap, pixel): pixel = v % 64");
    auto swz = [](int row) { return ((row >> 3) & 7) << 3; };
    __shared__ uint16_t gT[COUT][LD];
    __shared__ uint16_t iT[NR][LD];
    const int chunk = (int)blockIdx.x;
    if (chunk >= nchunk) return;
    const long P = (long)N * H * W;
    const long c0 = (long)chunk * chunk_pix;
    const long c1 = c0 + chunk_pix < P ? c0 + chunk_pix : P;
    const int w = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63, r = lane & 15, gq = lane >> 4;
    for (int i = (int)threadIdx.x; i < 8 * LD; i += 256) iT[72 + i / LD][i % LD] = 0;
    f32x4 acc[TPW];
#pragma unroll
    for (int j = 0; j < TPW; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bpart = 0.0f;
    for (long pb = c0; pb < c1; pb += KS) {
        u32x4 gv[(GV + 255) / 256], iv[(IV + 255) / 256];
#pragma unroll
        for (int q = 0; q < (GV + 255) / 256; ++q) {
            const int v = (int)threadIdx.x + 256 * q;
            const int pi = v / (COUT / 8), cv = (v - pi * (COUT / 8)) * 8;
            const long p = pb + pi;
            gv[q] = u32x4{0u, 0u, 0u, 0u};
            if (v < GV && p < c1) gv[q] = ld16(gpre + (size_t)p * COUT + cv);
        }
#pragma unroll
        for (int q = 0; q < (IV + 255) / 256; ++q) {
            const int v = (int)threadIdx.x + 256 * q;
            const int tap = v / KS, pi = v - (v / KS) * KS;
            const long p = pb + pi;
            iv[q] = u32x4{0u, 0u, 0u, 0u};
            if (v < IV && p < c1) {
                const int n = (int)(p / ((long)H * W));
                const int rem = (int)(p - (long)n * H * W);
                const int y = rem / W, x = rem - (rem / W) * W;
                const int iy = y + tap / 3 - 1, ix = x + tap % 3 - 1;
                if (iy >= 0 && iy < H && ix >= 0 && ix < W) iv[q] = ld16(in + (((size_t)n * H + iy) * W + ix) * 8);
            }
        }
#pragma unroll
        for (int q = 0; q < (GV + 255) / 256; ++q) {
            const int v = (int)threadIdx.x + 256 * q;
            const int pi = v / (COUT / 8), cv = (v - pi * (COUT / 8)) * 8;
            if (v < GV)
#pragma unroll
                for (int e = 0; e < 8; ++e) gT[cv + e][pi ^ swz(cv + e)] = (uint16_t)(gv[q][e >> 1] >> (16 * (e & 1)));
        }
#pragma unroll
        for (int q = 0; q < (IV + 255) / 256; ++q) {
            const int v = (int)threadIdx.x + 256 * q;
            const int tap = v / KS, pi = v - (v / KS) * KS;
            if (v < IV)
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    iT[tap * 8 + e][pi ^ swz(tap * 8 + e)] = (uint16_t)(iv[q][e >> 1] >> (16 * (e & 1)));
        }
        __syncthreads();
        if ((int)threadIdx.x < COUT)
            for (int k = 0; k < KS; ++k) bpart += bf2f(gT[threadIdx.x][k ^ swz((int)threadIdx.x)]);
#pragma unroll
        for (int kk = 0; kk < KS; kk += 32)
#pragma unroll
            for (int j = 0; j < TPW; ++j) {
                const int tile = w * TPW + j;
                if (tile < TILES) {
                    const int mt = tile / NTT, nt = tile - (tile / NTT) * NTT;
                    const bf16x8 a = as_bf(*reinterpret_cast<const u32x4 *>(&gT[mt * 16 + r][(kk + gq * 8) ^ swz(mt * 16 + r)]));
                    const bf16x8 b = as_bf(*reinterpret_cast<const u32x4 *>(&iT[nt * 16 + r][(kk + gq * 8) ^ swz(nt * 16 + r)]));
                    acc[j] = mfma(a, b, acc[j]);
                }
            }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
        const int tile = w * TPW + j;
        if (tile >= TILES) continue;
        const int mt = tile / NTT, nt = tile - (tile / NTT) * NTT;
        const int row = nt * 16 + r;   // tap * 8 + ci
        if (row >= 72) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int co = mt * 16 + gq * 4 + i;
            partial[((size_t)chunk * COUT + co) * 72 + row] = acc[j][i];
        }
    }
    if ((int)threadIdx.x < COUT) partial_b[(size_t)chunk * COUT + threadIdx.x] = bpart;
}

// fixed-order sum of the chunk partials into the fp32 gradient vector: a
// workgroup takes 64 consecutive partial entries j (weights with the padded
// input channels, then the biases); wave sl sums chunks sl, sl + 4, ... with
// eight loads in flight per lane, and the four wave sums are added in LDS
template <bool FOLD>
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float *partial, const float *partial_b, int chunks,
                                                      int cout, int cin, int cinp, float *dw, float *db)
{
    __shared__ float red[4][64];
    const int nw = cout * 9 * cinp;
    const int j = (int)blockIdx.x * 64 + ((int)threadIdx.x & 63), sl = (int)threadIdx.x >> 6;
    const bool isw = j < nw, valid = j < nw + cout;
    float s = 0.0f;
    if (valid && !FOLD) {
        const float *src = isw ? partial + j : partial_b + (j - nw);
        const size_t stride = isw ? (size_t)nw : (size_t)cout;
        float a[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] = 0.0f;
        int c = sl;
        for (; c + 28 < chunks; c += 32)
#pragma unroll
            for (int k = 0; k < 8; ++k) a[k] += src[(size_t)(c + 4 * k) * stride];
        for (; c < chunks; c += 4) a[0] += src[(size_t)c * stride];
        s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    } else if (valid) {
        // FOLD: partial[chunk][co][16][cinp] over (output parity, source
        // offset); tap (ky, kx) of parity (py, px) sits at offset
        // a = floor((py + ky - 1) / 2) + 1 - py, likewise b; bias partials
        // [chunk][4 parities][cout]
        int off[4];
        size_t stride;
        const float *src;
        if (isw) {
            const int co = j / (9 * cinp), rem = j - co * 9 * cinp, tap = rem / cinp, ci = rem - (rem / cinp) * cinp;
            const int ky = tap / 3, kx = tap - (tap / 3) * 3;
#pragma unroll
            for (int par = 0; par < 4; ++par) {
                const int py = par >> 1, px = par & 1;
                const int fa = ((py + ky - 1) >> 1) + 1 - py, fb = ((px + kx - 1) >> 1) + 1 - px;
                off[par] = ((co * 16 + par * 4 + fa * 2 + fb) * cinp) + ci;
            }
            src = partial;
            stride = (size_t)cout * 16 * cinp;
        } else {
#pragma unroll
            for (int par = 0; par < 4; ++par) off[par] = par * cout + (j - nw);
            src = partial_b;
            stride = (size_t)4 * cout;
        }
        float a[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        int c = sl;
        for (; c + 12 < chunks; c += 16)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float *q = src + (size_t)(c + 4 * k) * stride;
                a[k] += (q[off[0]] + q[off[1]]) + (q[off[2]] + q[off[3]]);
            }
        for (; c < chunks; c += 4) {
            const float *q = src + (size_t)c * stride;
            a[0] += (q[off[0]] + q[off[1]]) + (q[off[2]] + q[off[3]]);
        }
        s = (a[0] + a[1]) + (a[2] + a[3]);
    }
    red[sl][threadIdx.x & 63] = s;
    __syncthreads();
    if (sl != 0 || !valid) return;
    const int l = (int)threadIdx.x;
    const float t = (red[0][l] + red[1][l]) + (red[2][l] + red[3][l]);
    if (isw) {
        const int co = j / (9 * cinp), rem = j - co * 9 * cinp, tap = rem / cinp, ci = rem - (rem / cinp) * cinp;
        if (ci < cin) dw[(co * 9 + tap) * cin + ci] = t;
    } else {
        db[j - nw] = t;
    }
}

// ============================================================================
// head: delta = conv(d1, 32 -> 1); out = d + 5 cm delta on valid pixels
// ============================================================================
// One workgroup per 16x16 output tile of one image: the tile's d1 with a
// one-pixel halo (zeros outside the image) is staged in LDS once, and the 288
// weights, the same for every lane, are read through the scalar cache.  The
// sum runs tap by tap, channel by channel, from the bias, one fused
// multiply-add (a single rounding) per term.
__global__ __launch_bounds__(256) void k_head_fwd(const uint16_t *d1, const float *__restrict__ w,
                                                  const float *__restrict__ b, const float *dm, float *out, int N,
                                                  int H, int W)
{
    __shared__ u32x4 tile[18 * 18 * 4];
    const int tx = (int)blockIdx.x * 16, ty = (int)blockIdx.y * 16, n = (int)blockIdx.z;
    for (int k = threadIdx.x; k < 18 * 18 * 4; k += 256) {
        const int pix = k >> 2, q = k & 3;
        const int iy = ty - 1 + pix / 18, ix = tx - 1 + pix % 18;
        u32x4 v = {0u, 0u, 0u, 0u};
        if (iy >= 0 && iy < H && ix >= 0 && ix < W) v = ld16(d1 + (((size_t)n * H + iy) * W + ix) * 32 + 8 * q);
        tile[k] = v;
    }
    __syncthreads();
    const int lx = (int)threadIdx.x & 15, ly = (int)threadIdx.x >> 4;
    const int x = tx + lx, y = ty + ly;
    if (x >= W || y >= H) return;
    float s = b[0];
    for (int tap = 0; tap < 9; ++tap) {
        const int iy = y + tap / 3 - 1, ix = x + tap % 3 - 1;
        if (iy < 0 || iy >= H || ix < 0 || ix >= W) continue;
        const u32x4 *src = tile + ((ly + tap / 3) * 18 + lx + tap % 3) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const u32x4 v = src[q];
#pragma unroll
            for (int e = 0; e < 8; ++e) s = fmaf(w[tap * 32 + 8 * q + e], bf2f((uint16_t)(v[e >> 1] >> (16 * (e & 1)))), s);
        }
    }
    const size_t p = ((size_t)n * H + y) * W + x;
    const float d = dm[p];
    out[p] = d > 0.0f ? d + kCorrScale * s : 0.0f;
}

// masked L1 in four fixed-order steps (no atomics; the same sums every run):
// per-workgroup valid counts, their total, per-workgroup |out - target| sums
// with the gradient, then the mean
__global__ __launch_bounds__(256) void k_loss_count(const float *dm, const float *target, int n, unsigned *part)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    const int c = __syncthreads_count(p < n && dm[p] > 0.0f && target[p] > 0.0f);
    if (threadIdx.x == 0) part[blockIdx.x] = (unsigned)c;
}

__global__ __launch_bounds__(256) void k_loss_total(const unsigned *part, int nwg, unsigned *cnt)
{
    __shared__ unsigned red[256];
    unsigned c = 0u;
    for (int i = (int)threadIdx.x; i < nwg; i += 256) c += part[i];
    red[threadIdx.x] = c;
    __syncthreads();
    for (int m = 128; m > 0; m >>= 1) {
        if ((int)threadIdx.x < m) red[threadIdx.x] += red[threadIdx.x + m];
        __syncthreads();
    }
    if (threadIdx.x == 0) cnt[0] = red[0];
}

__global__ __launch_bounds__(256) void k_loss_grad(const float *out, const float *dm, const float *target, int n,
                                                   const unsigned *cnt, float *ddelta, float *part)
{
    __shared__ float red[4];
    const int p = blockIdx.x * 256 + threadIdx.x;
    const float inv_n = *cnt ? 1.0f / (float)*cnt : 0.0f;
    float a = 0.0f;
    if (p < n) {
        float g = 0.0f;
        if (dm[p] > 0.0f && target[p] > 0.0f) {
            const float diff = out[p] - target[p];
            g = diff > 0.0f ? inv_n : (diff < 0.0f ? -inv_n : 0.0f);
            a = diff < 0.0f ? -diff : diff;
        }
        ddelta[p] = kCorrScale * g;
    }
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) a += __shfl_xor(a, m);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_loss_final(const float *part, int nwg, const unsigned *cnt, float *loss)
{
    __shared__ float red[256];
    float s = 0.0f;
    for (int i = (int)threadIdx.x; i < nwg; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int m = 128; m > 0; m >>= 1) {
        if ((int)threadIdx.x < m) red[threadIdx.x] += red[threadIdx.x + m];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        loss[0] = *cnt ? red[0] / (float)*cnt : 0.0f;
        loss[1] = (float)*cnt;
    }
}

// gradient at d1 through the head: g[p][c] = sum_tap ddelta[p - tap + 1] w[tap][c], relu mask of d1
__global__ __launch_bounds__(256) void k_head_bwd(const float *ddelta, const float *w, const uint16_t *d1,
                                                  uint16_t *g_d1, int N, int H, int W)
{
    __shared__ float ws[288];
    for (int k = threadIdx.x; k < 288; k += 256) ws[k] = w[k];
    __syncthreads();
    const long P = (long)N * H * W;
    const long p = (long)blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    const int n = (int)(p / ((long)H * W));
    const int rem = (int)(p - (long)n * H * W);
    const int y = rem / W, x = rem - (rem / W) * W;
    float g[32];
#pragma unroll
    for (int c = 0; c < 32; ++c) g[c] = 0.0f;
    for (int tap = 0; tap < 9; ++tap) {
        const int oy = y - tap / 3 + 1, ox = x - tap % 3 + 1;
        if (oy < 0 || oy >= H || ox < 0 || ox >= W) continue;
        const float dd = ddelta[((size_t)n * H + oy) * W + ox];
        if (dd == 0.0f) continue;
#pragma unroll
        for (int c = 0; c < 32; ++c) g[c] += dd * ws[tap * 32 + c];
    }
    const uint16_t *a = d1 + (size_t)p * 32;
    uint16_t *o = g_d1 + (size_t)p * 32;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const u32x4 av = ld16(a + 8 * q);
        u32x4 ov;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint16_t a0 = (uint16_t)(av[e] & 0xffffu), a1 = (uint16_t)(av[e] >> 16);
            const uint16_t v0 = bf2f(a0) > 0.0f ? f2bf(g[8 * q + 2 * e]) : (uint16_t)0;
            const uint16_t v1 = bf2f(a1) > 0.0f ? f2bf(g[8 * q + 2 * e + 1]) : (uint16_t)0;
            ov[e] = (uint32_t)v0 | ((uint32_t)v1 << 16);
        }
        *reinterpret_cast<u32x4 *>(o + 8 * q) = ov;
    }
}

// head weight gradient of one pixel chunk, gathered from the input side:
// dw[tap][c] = sum_p ddelta[p] d1[p + off(tap)][c] = sum_q d1[q][c] ddelta[q - off(tap)],
// so every d1 pixel is read once.  Thread t takes pixel t / 4 of each
// 64-pixel pass and channels 8 (t % 4) .. +7; the 16 lanes of a wave with the
// same channel octet are summed by a fixed butterfly, the 4 waves in LDS.
// partial[j * nchunk + chunk]: j = tap * 32 + c, j = 288 the bias (the sum of
// ddelta, from the octet-0 lanes)
__global__ __launch_bounds__(256) void k_head_wgrad(const float *ddelta, const uint16_t *d1, int N, int H, int W,
                                                    float *partial, int chunk_pix)
{
    __shared__ float red[4][4][73];
    const long P = (long)N * H * W;
    const long c0 = (long)blockIdx.x * chunk_pix;
    const long c1 = c0 + chunk_pix < P ? c0 + chunk_pix : P;
    const int oct = (int)threadIdx.x & 3, lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
    float acc[9][8], bsum = 0.0f;
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
        for (int e = 0; e < 8; ++e) acc[k][e] = 0.0f;
    for (long q = c0 + ((int)threadIdx.x >> 2); q < c1; q += 64) {
        const int n = (int)(q / ((long)H * W));
        const int rem = (int)(q - (long)n * H * W);
        const int y = rem / W, x = rem - (rem / W) * W;
        const u32x4 v = ld16(d1 + (size_t)q * 32 + 8 * oct);
        float a[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) a[e] = bf2f((uint16_t)(v[e >> 1] >> (16 * (e & 1))));
        const float *drow = ddelta + (size_t)n * H * W;
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int py = y - tap / 3 + 1, px = x - tap % 3 + 1;
            if (py < 0 || py >= H || px < 0 || px >= W) continue;
            const float dd = drow[(size_t)py * W + px];
#pragma unroll
            for (int e = 0; e < 8; ++e) acc[tap][e] += dd * a[e];
            if (tap == 4 && oct == 0) bsum += dd;
        }
    }
#pragma unroll
    for (int m = 4; m < 64; m <<= 1) {
#pragma unroll
        for (int k = 0; k < 9; ++k)
#pragma unroll
            for (int e = 0; e < 8; ++e) acc[k][e] += __shfl_xor(acc[k][e], m);
        bsum += __shfl_xor(bsum, m);
    }
    if (lane < 4) {
#pragma unroll
        for (int k = 0; k < 9; ++k)
#pragma unroll
            for (int e = 0; e < 8; ++e) red[wv][oct][k * 8 + e] = acc[k][e];
        red[wv][oct][72] = bsum;
    }
    __syncthreads();
    const int nchunk = (int)gridDim.x;
    for (int j = (int)threadIdx.x; j < 289; j += 256) {
        // j = tap * 32 + c (c = 8 oct + e); the bias sits at octet 0, slot 72
        const int tap = j >> 5, c = j & 31;
        const int o = j < 288 ? c >> 3 : 0, k = j < 288 ? tap * 8 + (c & 7) : 72;
        const float s = (red[0][o][k] + red[1][o][k]) + (red[2][o][k] + red[3][o][k]);
        partial[(size_t)j * nchunk + blockIdx.x] = s;
    }
}

// fixed-order sum of the head partials: workgroup j sums row j of partial
__global__ __launch_bounds__(256) void k_head_reduce(const float *partial, int chunks, float *dw, float *db)
{
    __shared__ float red[256];
    const int j = (int)blockIdx.x;
    float s = 0.0f;
    for (int c = (int)threadIdx.x; c < chunks; c += 256) s += partial[(size_t)j * chunks + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int m = 128; m > 0; m >>= 1) {
        if ((int)threadIdx.x < m) red[threadIdx.x] += red[threadIdx.x + m];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (j < 288)
            dw[j] = red[0];
        else
            db[0] = red[0];
    }
}

// Adam (Kingma & Ba, Algorithm 1); c1 = 1 - beta1^t, c2 = 1 - beta2^t
__global__ __launch_bounds__(256) void k_adam(float *p, const float *g, float *m, float *v, int n, float lr,
                                              float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    p[i] = p[i] - lr * mh / (sqrtf(vh) + eps);
}

// ============================================================================
// launchers
// ============================================================================
static dim3 grid1(long n, int per) { return dim3((unsigned)((n + per - 1) / per)); }

hipError_t launch_make_input(const void *depth, int fmt, int N, int H, int W, uint16_t *x, float *dm, hipStream_t s)
{
    const dim3 g((unsigned)((W + 15) / 16), (unsigned)((H + 15) / 16), (unsigned)N);
    if (fmt == TF_DEPTH_U16_MM)
        hipLaunchKernelGGL(k_make_input<TF_DEPTH_U16_MM>, g, dim3(256), 0, s, depth, N, H, W, x, dm);
    else
        hipLaunchKernelGGL(k_make_input<TF_DEPTH_F32_M>, g, dim3(256), 0, s, depth, N, H, W, x, dm);
    return hipGetLastError();
}

hipError_t launch_pack(const Net &net, const float *params, uint16_t *g, uint16_t *t, hipStream_t s)
{
    PackJobs J = {};
    int at = 0;
    for (int l = 0; l < kLayers - 1; ++l) {
        const LayerDesc &L = net.L[l];
        PackJob &p = J.job[l];
        p.w = params + L.w_off;
        p.g = g + L.g_off;
        p.t = L.t_off >= 0 ? t + L.t_off : nullptr;
        p.cin = L.cin;
        p.cinp = L.cinp;
        p.cout = L.cout;
        p.kp = L.kp;
        p.up = L.up;
        p.n_g = L.up ? 2 * 16 * L.cout * L.cinp : L.cout * L.kp;   // up layers: high and low halves
        p.n_t = p.t ? L.cinp * (L.up ? 2 * 16 : 9) * L.cout : 0;
        J.start[l] = at;
        at += p.n_g > p.n_t ? p.n_g : p.n_t;
    }
    J.start[kLayers - 1] = at;
    hipLaunchKernelGGL(k_pack, grid1(at, 256), dim3(256), 0, s, J);
    return hipGetLastError();
}


hipError_t launch_conv_fwd(int layer, const uint16_t *in, int Hs, int Ws, const uint16_t *g, const float *bias,
                           const uint16_t *skip, uint16_t *out, int N, int Ho, int Wo, hipStream_t s)
{
    // encoder tiles: 4 / NS output rows x 16 T columns per workgroup, the
    // stride-2 layers splitting their output channels over the 4 waves (one
    // output row per workgroup); decoder tiles: one source row x 16 T
    // columns, the smaller layers' channels split over NS workgroups (shapes
    // measured at 640x480)
    const dim3 b(256);
    auto enc_grid = [&](int T, int NS) {
        const long nt = (long)N * ((Ho + 4 / NS - 1) / (4 / NS)) * ((Wo + 16 * T - 1) / (16 * T));
        return dim3((unsigned)((nt + 7) / 8 * 8));
    };
    auto up_grid = [&](int T, int NS) {
        const long nt = (long)N * Hs * ((Ws + 16 * T - 1) / (16 * T)) * NS;
        return dim3((unsigned)((nt + 7) / 8 * 8));
    };
    if (layer < 4 && skip) return hipErrorInvalidValue;
    if (layer >= 4 && (Ho != 2 * Hs || Wo != 2 * Ws)) return hipErrorInvalidValue;
    switch (layer) {
    case 0: hipLaunchKernelGGL((k_conv_fwd<8, 32, 1, 2, 1>), enc_grid(2, 1), b, 0, s, in, Hs, Ws, g, bias, out, N, Ho, Wo); break;
    case 1: hipLaunchKernelGGL((k_conv_fwd<32, 64, 2, 2, 4>), enc_grid(2, 4), b, 0, s, in, Hs, Ws, g, bias, out, N, Ho, Wo); break;
    case 2: hipLaunchKernelGGL((k_conv_fwd<64, 64, 2, 1, 4>), enc_grid(1, 4), b, 0, s, in, Hs, Ws, g, bias, out, N, Ho, Wo); break;
    case 3: hipLaunchKernelGGL((k_conv_fwd<64, 128, 2, 1, 4>), enc_grid(1, 4), b, 0, s, in, Hs, Ws, g, bias, out, N, Ho, Wo); break;
    case 4: hipLaunchKernelGGL((k_conv_fwd_up<128, 64, true, 1, 4>), up_grid(1, 4), b, 0, s, in, Hs, Ws, g, bias, skip, out, N); break;
    case 5: hipLaunchKernelGGL((k_conv_fwd_up<64, 64, true, 2, 2>), up_grid(2, 2), b, 0, s, in, Hs, Ws, g, bias, skip, out, N); break;
    case 6: hipLaunchKernelGGL((k_conv_fwd_up<64, 32, true, 2, 1>), up_grid(2, 1), b, 0, s, in, Hs, Ws, g, bias, skip, out, N); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_head_fwd(const uint16_t *d1, const float *w, const float *b, const float *dm, float *out, int N,
                           int H, int W, hipStream_t s)
{
    hipLaunchKernelGGL(k_head_fwd, dim3((W + 15) / 16, (H + 15) / 16, N), dim3(256), 0, s, d1, w, b, dm, out, N, H, W);
    return hipGetLastError();
}

// scratch: [0] the valid count (uint32), then loss_scratch_words(n_pix) - 4
// words of per-workgroup counts and sums; loss: [0] mean, [1] count
hipError_t launch_loss(const float *out, const float *dm, const float *target, int n_pix, float *ddelta,
                       float *scratch, float *loss, hipStream_t s)
{
    const int nwg = (n_pix + 255) / 256;
    unsigned *cnt = reinterpret_cast<unsigned *>(scratch);
    unsigned *pc = cnt + 4;
    float *ps = scratch + 4 + nwg;
    hipLaunchKernelGGL(k_loss_count, dim3(nwg), dim3(256), 0, s, dm, target, n_pix, pc);
    hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(256), 0, s, pc, nwg, cnt);
    hipLaunchKernelGGL(k_loss_grad, dim3(nwg), dim3(256), 0, s, out, dm, target, n_pix, cnt, ddelta, ps);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, ps, nwg, cnt, loss);
    return hipGetLastError();
}

hipError_t launch_head_bwd(const float *ddelta, const float *w, const uint16_t *d1, uint16_t *g_d1, int N, int H,
                           int W, hipStream_t s)
{
    hipLaunchKernelGGL(k_head_bwd, grid1((long)N * H * W, 256), dim3(256), 0, s, ddelta, w, d1, g_d1, N, H, W);
    return hipGetLastError();
}

hipError_t launch_head_wgrad(const float *ddelta, const uint16_t *d1, int N, int H, int W, float *partial,
                             int chunks, float *dw, float *db, hipStream_t s)
{
    const long P = (long)N * H * W;
    const int per = (int)((P + chunks - 1) / chunks);
    const int nc = (int)((P + per - 1) / per);
    hipLaunchKernelGGL(k_head_wgrad, dim3(nc), dim3(256), 0, s, ddelta, d1, N, H, W, partial, per);
    hipLaunchKernelGGL(k_head_reduce, dim3(289), dim3(256), 0, s, partial, nc, dw, db);
    return hipGetLastError();
}

// workgroups of k_conv_bwd_data_s2: N Hq input rows x 2 column parities x runs of 32 x NS waves
static dim3 s2_grid(int N, int Hq, int Wq, int NS)
{
    const long waves = (long)N * Hq * 2 * ((((Wq + 1) >> 1) + 31) >> 5) * NS;
    return dim3((unsigned)((waves + 3) / 4));
}

hipError_t launch_conv_bwd_data(int layer, const uint16_t *gpre, int Ho, int Wo, const uint16_t *t,
                                const uint16_t *skipg, const uint16_t *act, uint16_t *gout, int N, int Hq, int Wq,
                                hipStream_t s)
{
    const long P = (long)N * Hq * Wq;
    const dim3 g1 = grid1(P, 128), g4 = grid1(P, 32), b(256);
    if (layer >= 4 && (Ho != 2 * Hq || Wo != 2 * Wq)) return hipErrorInvalidValue;
    switch (layer) {
    // stride-2 layers: only the taps of each input parity
    case 1: hipLaunchKernelGGL((k_conv_bwd_data_s2<32, 64, true, 1>), s2_grid(N, Hq, Wq, 1), b, 0, s, gpre, Ho, Wo, t, skipg, act, gout, N, Hq, Wq); break;
    case 2: hipLaunchKernelGGL((k_conv_bwd_data_s2<64, 64, true, 1>), s2_grid(N, Hq, Wq, 1), b, 0, s, gpre, Ho, Wo, t, skipg, act, gout, N, Hq, Wq); break;
    case 3: hipLaunchKernelGGL((k_conv_bwd_data_s2<64, 128, true, 2>), s2_grid(N, Hq, Wq, 2), b, 0, s, gpre, Ho, Wo, t, skipg, act, gout, N, Hq, Wq); break;
    // upsampled layers: the adjoint of the parity-folded forward (t holds the folded weights)
    case 4: hipLaunchKernelGGL((k_conv_bwd_data_up<128, 64, 4>), g4, b, 0, s, gpre, t, act, gout, N, Hq, Wq); break;
    case 5: hipLaunchKernelGGL((k_conv_bwd_data_up<64, 64, 1>), g1, b, 0, s, gpre, t, act, gout, N, Hq, Wq); break;
    case 6: hipLaunchKernelGGL((k_conv_bwd_data_up<64, 32, 1>), g1, b, 0, s, gpre, t, act, gout, N, Hq, Wq); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_conv_wgrad(int layer, const uint16_t *gpre, const uint16_t *in, int Hs, int Ws, int N, int Ho,
                             int Wo, float *partial, int chunks, float *dw, float *db, hipStream_t s)
{
    // the decoder layers (4-6) run folded: 16 (parity, offset) taps over the source grid
    const bool fold = layer >= 4;
    const int ntap = fold ? 16 : 9;
    const long P = fold ? (long)N * Hs * Ws : (long)N * Ho * Wo;
    if (fold && (Ho != 2 * Hs || Wo != 2 * Ws)) return hipErrorInvalidValue;
    int per = (int)((P + chunks - 1) / chunks);
    per = ((per + kWgradStep - 1) / kWgradStep) * kWgradStep;
    const int nc = (int)((P + per - 1) / per);
    float *pb = partial;   // bias partials after the weight partials
    const dim3 gr(ntap * ((nc + 7) / 8) * 8), b(256);   // (tap, chunk) pairs, chunks padded to a multiple of 8
    int cout = 0, cin = 0, cinp = 0;
    switch (layer) {
    case 0: cout = 32; cin = 3; cinp = 8; pb += (size_t)nc * 32 * 9 * 8;   // all taps per workgroup
        hipLaunchKernelGGL((k_conv_wgrad_c8<32>), dim3(nc), b, 0, s, gpre, in, Ho, Wo, N, partial, pb, per, nc); break;
    case 1: cout = 64; cin = cinp = 32; pb += (size_t)nc * 64 * 9 * 32;
        hipLaunchKernelGGL((k_conv_wgrad<32, 64, 2, false, false>), gr, b, 0, s, gpre, in, Hs, Ws, N, Ho, Wo, partial, pb, per, nc); break;
    case 2: cout = 64; cin = cinp = 64; pb += (size_t)nc * 64 * 9 * 64;
        hipLaunchKernelGGL((k_conv_wgrad<64, 64, 2, false, false>), gr, b, 0, s, gpre, in, Hs, Ws, N, Ho, Wo, partial, pb, per, nc); break;
    case 3: cout = 128; cin = cinp = 64; pb += (size_t)nc * 128 * 9 * 64;
        hipLaunchKernelGGL((k_conv_wgrad<64, 128, 2, false, false>), gr, b, 0, s, gpre, in, Hs, Ws, N, Ho, Wo, partial, pb, per, nc); break;
    case 4: cout = 64; cin = cinp = 128; pb += (size_t)nc * 64 * 16 * 128;
        hipLaunchKernelGGL((k_conv_wgrad<128, 64, 1, true, true>), gr, b, 0, s, gpre, in, Hs, Ws, N, Ho, Wo, partial, pb, per, nc); break;
    case 5: cout = 64; cin = cinp = 64; pb += (size_t)nc * 64 * 16 * 64;
        hipLaunchKernelGGL((k_conv_wgrad<64, 64, 1, true, true>), gr, b, 0, s, gpre, in, Hs, Ws, N, Ho, Wo, partial, pb, per, nc); break;
    case 6: cout = 32; cin = cinp = 64; pb += (size_t)nc * 32 * 16 * 64;
        hipLaunchKernelGGL((k_conv_wgrad<64, 32, 1, true, true>), gr, b, 0, s, gpre, in, Hs, Ws, N, Ho, Wo, partial, pb, per, nc); break;
    default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (fold)
        hipLaunchKernelGGL(k_wgrad_reduce<true>, grid1((long)cout * 9 * cinp + cout, 64), dim3(256), 0, s, partial, pb,
                           nc, cout, cin, cinp, dw, db);
    else
        hipLaunchKernelGGL(k_wgrad_reduce<false>, grid1((long)cout * 9 * cinp + cout, 64), dim3(256), 0, s, partial, pb,
                           nc, cout, cin, cinp, dw, db);
    return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, int n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s)
{
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, grid1(n, 256), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace nn
}  // namespace tsdf
