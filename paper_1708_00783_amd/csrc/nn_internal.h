// nn_internal.h -- layer table, tensor layout and launchers of the learned
// depth prefilter (a small 3x3 convolutional encoder-decoder in front of
// integration).  Internal to libtsdf.
//
// Tensors are NHWC bfloat16 (stored as uint16 bit patterns); the network
// input has its 3 channels (depth / 4 m, valid mask, deviation from the 3x3
// valid mean in 5 cm units) padded to 8.  Conv
// weights are kept as fp32 master copies in the parameter vector (per layer
// W[cout][3][3][cin] then b[cout], layers in forward order) and packed to
// bf16 GEMM operands: G, the cout x KP matrix with k = tap * CINP + ci (KP =
// 9 CINP rounded up to 32) for the forward pass, stored in MFMA fragment
// order (the 64 lanes' 16-byte B fragments of one K step and 16-channel tile
// contiguous), and T[cin][9 cout] with k = tap * cout + co for the
// backward-data pass.  A layer that reads the 2x upsampled source instead
// packs its taps folded by output parity (the sum of the taps that land on
// each 2x2 source offset), each folded weight split into a bf16 high half and
// the bf16 remainder: G[2 halves][4 parities][cout x 4 CINP, fragment order]
// and T[2 halves][cin][16 cout].
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace tsdf {
namespace nn {

constexpr int kLayers = 8;              // e1 e2 e3 e4 d3 d2 d1 head
constexpr float kDepthScale = 4.0f;     // metres: input normalisation (d / 4 m)
constexpr float kCorrScale = 0.05f;     // metres: unit of the head's depth correction
constexpr int kWgradStep = 64;          // pixels per LDS staging round of the conv weight gradient
constexpr int kWgradChunkPix = 512;     // target pixels per chunk of a conv weight-gradient reduction

constexpr int kWgradFoldChunkPix = 2048; // the same for the folded decoder layers (16 taps per chunk)

// pixel chunks of a conv weight-gradient reduction over P pixels
inline int wgrad_chunks(long P, int pix_per_chunk = kWgradChunkPix)
{
    const long c = P / pix_per_chunk;
    return (int)(c < 64 ? 64 : (c > 512 ? 512 : c));
}

constexpr int kHeadChunks = 1024;       // pixel chunks of the head's weight-gradient reduction

struct LayerDesc {
    int cin, cinp, cout, stride, up;    // up: the conv reads up2(source)
    int src;                            // activation index of the source (-1 = network input)
    int skip;                           // activation index added before the relu (-1 none)
    int w_off, b_off;                   // fp32 parameter offsets
    int kp;                             // forward GEMM K (padded)
    int g_off, t_off;                   // bf16 packed-weight offsets (elements); an up layer's are
                                        // parity-folded and split: [2 halves][4 parities][cout][4 offsets
                                        // x cinp] and [2 halves][cinp][4 parities x 4 offsets x cout]
    int scale;                          // output resolution divisor (1, 2, 4, 8)
};

// activation indices: 0 = x (input), 1..7 = e1 e2 e3 e4 d3 d2 d1
constexpr int kActs = 8;

struct Net {
    LayerDesc L[kLayers];
    int n_params;
    int g_elems, t_elems;
};

// layer table (host and device agree; computed once on the host)
Net make_net();

// activation buffer of a (N, H, W) problem: channels and scale per index
inline int act_channels(int a) { static const int c[kActs] = {8, 32, 64, 64, 128, 64, 64, 32}; return c[a]; }
inline int act_scale(int a) { static const int s[kActs] = {1, 1, 2, 4, 8, 4, 2, 1}; return s[a]; }

hipError_t launch_make_input(const void *depth, int fmt, int N, int H, int W, uint16_t *x, float *dm, hipStream_t s);
// one layer's share of the weight packing (forward g, backward-data t)
struct PackJob {
    const float *w;
    uint16_t *g, *t;
    int cin, cinp, cout, kp, up, n_g, n_t;
};
struct PackJobs {
    PackJob job[kLayers - 1];
    int start[kLayers];   // first thread of each layer; start[kLayers - 1] = total
};

hipError_t launch_pack(const Net &net, const float *params, uint16_t *g, uint16_t *t, hipStream_t s);
hipError_t launch_conv_fwd(int layer, const uint16_t *in, int Hs, int Ws, const uint16_t *g, const float *bias,
                           const uint16_t *skip, uint16_t *out, int N, int Ho, int Wo, hipStream_t s);
hipError_t launch_head_fwd(const uint16_t *d1, const float *w, const float *b, const float *dm, float *out, int N,
                           int H, int W, hipStream_t s);
// 32-bit words of loss scratch for n_pix pixels: the count, padding, and a
// count and a sum per 256-pixel workgroup
inline size_t loss_scratch_words(long n_pix) { return 4 + 2 * (size_t)((n_pix + 255) / 256); }
hipError_t launch_loss(const float *out, const float *dm, const float *target, int n_pix, float *ddelta,
                       float *scratch, float *loss, hipStream_t s);
hipError_t launch_head_bwd(const float *ddelta, const float *w, const uint16_t *d1, uint16_t *g_d1, int N, int H,
                           int W, hipStream_t s);
hipError_t launch_head_wgrad(const float *ddelta, const uint16_t *d1, int N, int H, int W, float *partial,
                             int chunks, float *dw, float *db, hipStream_t s);
hipError_t launch_conv_bwd_data(int layer, const uint16_t *gpre, int Ho, int Wo, const uint16_t *t,
                                const uint16_t *skipg, const uint16_t *act, uint16_t *gout, int N, int Hq, int Wq,
                                hipStream_t s);
hipError_t launch_conv_wgrad(int layer, const uint16_t *gpre, const uint16_t *in, int Hs, int Ws, int N, int Ho,
                             int Wo, float *partial, int chunks, float *dw, float *db, hipStream_t s);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, int n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s);

}  // namespace nn
}  // namespace tsdf
