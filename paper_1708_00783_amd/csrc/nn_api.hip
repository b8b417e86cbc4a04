// nn_api.hip -- host side of the learned depth prefilter: layer table,
// workspace carving, forward / backward orchestration, Adam, the C ABI of
// include/tsdf_nn.h.
#include <string.h>

#include <new>

#include "nn_internal.h"
#include "tsdf.h"
#include "tsdf_nn.h"

using namespace tsdf::nn;

namespace tsdf {
namespace nn {

Net make_net()
{
    // cin, cinp, cout, stride, up, src act, skip act
    static const int T[kLayers][7] = {
        {3, 8, 32, 1, 0, 0, -1},    {32, 32, 64, 2, 0, 1, -1},  {64, 64, 64, 2, 0, 2, -1},
        {64, 64, 128, 2, 0, 3, -1}, {128, 128, 64, 1, 1, 4, 3}, {64, 64, 64, 1, 1, 5, 2},
        {64, 64, 32, 1, 1, 6, 1},   {32, 32, 1, 1, 0, 7, -1},
    };
    static const int S[kLayers] = {1, 2, 4, 8, 4, 2, 1, 1};
    Net n = {};
    int off = 0, go = 0, to = 0;
    for (int l = 0; l < kLayers; ++l) {
        LayerDesc &L = n.L[l];
        L.cin = T[l][0];
        L.cinp = T[l][1];
        L.cout = T[l][2];
        L.stride = T[l][3];
        L.up = T[l][4];
        L.src = T[l][5];
        L.skip = T[l][6];
        L.scale = S[l];
        L.w_off = off;
        off += L.cout * 9 * L.cin;
        L.b_off = off;
        off += L.cout;
        L.kp = ((9 * L.cinp + 31) / 32) * 32;
        if (l < kLayers - 1) {
            L.g_off = go;
            // upsampled layers: the forward reads parity-folded 2x2 weights,
            // split into bf16 high and low halves
            go += L.up ? 2 * 4 * L.cout * 4 * L.cinp : L.cout * L.kp;
            L.t_off = l > 0 ? to : -1;
            if (l > 0) to += L.cinp * (L.up ? 2 * 16 : 9) * L.cout;   // up layers: [half][ci][par][a][b][co]
        } else {
            L.g_off = L.t_off = -1;
        }
    }
    n.n_params = off;
    n.g_elems = go;
    n.t_elems = to;
    return n;
}

}  // namespace nn
}  // namespace tsdf

namespace {

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct NLayout {
    size_t act[kActs], grad[kActs], dm, out, ddelta, params, grads, m, v, g, t, partial, hpartial, scratch, loss, total;
};

bool nlayout(const Net &net, uint32_t B, uint32_t H, uint32_t W, int training, NLayout &L)
{
    if (B < 1 || B > 1024 || H < 8 || W < 8 || H > 4096 || W > 4096 || (H & 7) || (W & 7)) return false;
    L = {};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = a256(o + bytes);
        return at;
    };
    const size_t px = (size_t)B * H * W;
    for (int a = 0; a < kActs; ++a) {
        const size_t s = act_scale(a);
        L.act[a] = take(2 * (size_t)B * (H / s) * (W / s) * act_channels(a));
        L.grad[a] = (training && a > 0) ? take(2 * (size_t)B * (H / s) * (W / s) * act_channels(a)) : 0;
    }
    L.dm = take(4 * px);
    L.out = take(4 * px);
    L.params = take(4 * (size_t)net.n_params);
    L.g = take(2 * (size_t)net.g_elems);
    L.t = take(2 * (size_t)net.t_elems);
    if (training) {
        L.ddelta = take(4 * px);
        L.grads = take(4 * (size_t)net.n_params);
        L.m = take(4 * (size_t)net.n_params);
        L.v = take(4 * (size_t)net.n_params);
        size_t mx = 0;
        for (int l = 0; l < kLayers - 1; ++l) {
            // the decoder layers reduce 16 (parity, offset) taps over the source grid, 4 bias partials
            const LayerDesc &Ll = net.L[l];
            const size_t P = Ll.up ? (size_t)B * (H / (2 * Ll.scale)) * (W / (2 * Ll.scale))
                                   : (size_t)B * (H / Ll.scale) * (W / Ll.scale);
            const size_t e = (size_t)wgrad_chunks((long)P, Ll.up ? kWgradFoldChunkPix : kWgradChunkPix) *
                             ((size_t)Ll.cout * (Ll.up ? 16 : 9) * Ll.cinp + (Ll.up ? 4 : 1) * Ll.cout);
            if (e > mx) mx = e;
        }
        L.partial = take(4 * mx);
        L.hpartial = take(4 * (size_t)kHeadChunks * 289);
        L.scratch = take(4 * loss_scratch_words((long)px));
        L.loss = take(16);
    }
    L.total = o;
    return true;
}

}  // namespace

struct tf_nn {
    Net net;
    NLayout L;
    uint32_t B, H, W;
    int training;
    uint8_t *ws;
    uint32_t batch;        // batch of the last forward
    int have_forward;
    int have_params;
    int step;              // Adam steps taken
    uint16_t *act[kActs];
    uint16_t *grad[kActs];
    float *dm, *out, *ddelta, *params, *grads, *m, *v, *partial, *hpartial, *scratch;
    uint16_t *g, *t;
};

namespace {

int hs(hipError_t e) { return e == hipSuccess ? TF_OK : TF_E_HIP; }

int dims_of(const tf_nn *nn, int a, int32_t d[4])
{
    const int s = act_scale(a);
    d[0] = (int32_t)nn->batch;
    d[1] = (int32_t)(nn->H / s);
    d[2] = (int32_t)(nn->W / s);
    d[3] = act_channels(a);
    return TF_OK;
}

}  // namespace

extern "C" {

uint32_t tf_nn_param_count(void) { return (uint32_t)make_net().n_params; }

size_t tf_nn_workspace_bytes(uint32_t B, uint32_t H, uint32_t W, int training)
{
    NLayout L;
    if (!nlayout(make_net(), B, H, W, training != 0, L)) return 0;
    return L.total;
}

int tf_nn_create(uint32_t B, uint32_t H, uint32_t W, int training, void *d_ws, size_t bytes, tf_nn **out)
{
    if (!out || !d_ws) return TF_E_INVAL;
    *out = nullptr;
    const Net net = make_net();
    NLayout L;
    if (!nlayout(net, B, H, W, training != 0, L)) return TF_E_INVAL;
    if ((uintptr_t)d_ws & 255u) return TF_E_INVAL;
    if (bytes < L.total) return TF_E_SPACE;
    tf_nn *nn = new (std::nothrow) tf_nn();
    if (!nn) return TF_E_INVAL;
    nn->net = net;
    nn->L = L;
    nn->B = B;
    nn->H = H;
    nn->W = W;
    nn->training = training != 0;
    nn->ws = (uint8_t *)d_ws;
    uint8_t *b = nn->ws;
    for (int a = 0; a < kActs; ++a) {
        nn->act[a] = (uint16_t *)(b + L.act[a]);
        nn->grad[a] = (nn->training && a > 0) ? (uint16_t *)(b + L.grad[a]) : nullptr;
    }
    nn->dm = (float *)(b + L.dm);
    nn->out = (float *)(b + L.out);
    nn->params = (float *)(b + L.params);
    nn->g = (uint16_t *)(b + L.g);
    nn->t = (uint16_t *)(b + L.t);
    if (nn->training) {
        nn->ddelta = (float *)(b + L.ddelta);
        nn->grads = (float *)(b + L.grads);
        nn->m = (float *)(b + L.m);
        nn->v = (float *)(b + L.v);
        nn->partial = (float *)(b + L.partial);
        nn->hpartial = (float *)(b + L.hpartial);
        nn->scratch = (float *)(b + L.scratch);
    }
    *out = nn;
    return TF_OK;
}

int tf_nn_destroy(tf_nn *nn)
{
    if (!nn) return TF_E_INVAL;
    delete nn;
    return TF_OK;
}

int tf_nn_set_params(tf_nn *nn, const float *d_params, tf_stream stream)
{
    if (!nn || !d_params) return TF_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    const size_t n = (size_t)nn->net.n_params;
    hipError_t e = hipMemcpyAsync(nn->params, d_params, 4 * n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && nn->training) {
        // fresh optimiser state (not a graph-captured call)
        e = hipMemsetAsync(nn->m, 0, 4 * n, s);
        if (e == hipSuccess) e = hipMemsetAsync(nn->v, 0, 4 * n, s);
        nn->step = 0;
    }
    if (e == hipSuccess) e = launch_pack(nn->net, nn->params, nn->g, nn->t, s);
    nn->have_params = e == hipSuccess;
    return hs(e);
}

int tf_nn_get_params(tf_nn *nn, float *d_params, tf_stream stream)
{
    if (!nn || !d_params) return TF_E_INVAL;
    return hs(hipMemcpyAsync(d_params, nn->params, 4 * (size_t)nn->net.n_params, hipMemcpyDeviceToDevice,
                             (hipStream_t)stream));
}

int tf_nn_forward(tf_nn *nn, const void *d_depth, int fmt, uint32_t batch, float *d_out, tf_stream stream)
{
    if (!nn || !d_depth || !d_out || batch < 1 || batch > nn->B) return TF_E_INVAL;
    if (fmt != TF_DEPTH_F32_M && fmt != TF_DEPTH_U16_MM) return TF_E_INVAL;
    if (!nn->have_params) return TF_E_ORDER;
    hipStream_t s = (hipStream_t)stream;
    const int N = (int)batch, H = (int)nn->H, W = (int)nn->W;
    hipError_t e = launch_make_input(d_depth, fmt, N, H, W, nn->act[0], nn->dm, s);
    for (int l = 0; l < kLayers - 1 && e == hipSuccess; ++l) {
        const LayerDesc &L = nn->net.L[l];
        const int ss = act_scale(L.src);
        const int Hs = H / ss, Ws = W / ss;
        const int Ho = H / L.scale, Wo = W / L.scale;
        e = launch_conv_fwd(l, nn->act[L.src], Hs, Ws, nn->g + L.g_off, nn->params + L.b_off,
                            L.skip >= 0 ? nn->act[L.skip] : nullptr, nn->act[l + 1], N, Ho, Wo, s);
    }
    const LayerDesc &Hd = nn->net.L[kLayers - 1];
    if (e == hipSuccess)
        e = launch_head_fwd(nn->act[7], nn->params + Hd.w_off, nn->params + Hd.b_off, nn->dm, nn->out, N, H, W, s);
    if (e == hipSuccess && d_out != nn->out)
        e = hipMemcpyAsync(d_out, nn->out, 4 * (size_t)N * H * W, hipMemcpyDeviceToDevice, s);
    nn->batch = batch;
    nn->have_forward = e == hipSuccess;
    return hs(e);
}

int tf_nn_backward(tf_nn *nn, const float *d_target, float *d_loss, tf_stream stream)
{
    if (!nn || !d_target || !d_loss || !nn->training) return TF_E_INVAL;
    if (!nn->have_forward) return TF_E_ORDER;
    hipStream_t s = (hipStream_t)stream;
    const int N = (int)nn->batch, H = (int)nn->H, W = (int)nn->W;
    const Net &net = nn->net;
    const LayerDesc &Hd = net.L[kLayers - 1];
    hipError_t e = launch_loss(nn->out, nn->dm, d_target, N * H * W, nn->ddelta, nn->scratch, d_loss, s);
    if (e == hipSuccess) e = launch_head_bwd(nn->ddelta, nn->params + Hd.w_off, nn->act[7], nn->grad[7], N, H, W, s);
    if (e == hipSuccess)
        e = launch_head_wgrad(nn->ddelta, nn->act[7], N, H, W, nn->hpartial, kHeadChunks, nn->grads + Hd.w_off,
                              nn->grads + Hd.b_off, s);
    // conv layers from the last to the first: weight gradient, then the
    // gradient at the source (skip gradient and relu mask fused)
    static const int skipg_of[kLayers] = {-1, 7, 6, 5, -1, -1, -1, -1};   // gradient added at the source
    for (int l = kLayers - 2; l >= 0 && e == hipSuccess; --l) {
        const LayerDesc &L = net.L[l];
        const int ss = act_scale(L.src);
        const int Hs = H / ss, Ws = W / ss, Ho = H / L.scale, Wo = W / L.scale;
        uint16_t *gpre = nn->grad[l + 1];
        e = launch_conv_wgrad(l, gpre, nn->act[L.src], Hs, Ws, N, Ho, Wo, nn->partial,
                              L.up ? wgrad_chunks((long)N * Hs * Ws, kWgradFoldChunkPix) : wgrad_chunks((long)N * Ho * Wo),
                              nn->grads + L.w_off, nn->grads + L.b_off, s);
        if (e == hipSuccess && l > 0)
            e = launch_conv_bwd_data(l, gpre, Ho, Wo, nn->t + L.t_off,
                                     skipg_of[l] >= 0 ? nn->grad[skipg_of[l]] : nullptr, nn->act[L.src],
                                     nn->grad[L.src], N, Hs, Ws, s);
    }
    return hs(e);
}

int tf_nn_adam_step(tf_nn *nn, float lr, float b1, float b2, float eps, tf_stream stream)
{
    if (!nn || !nn->training || !(lr >= 0.0f) || !(b1 >= 0.0f && b1 < 1.0f) || !(b2 >= 0.0f && b2 < 1.0f) ||
        !(eps > 0.0f))
        return TF_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    nn->step += 1;
    hipError_t e = launch_adam(nn->params, nn->grads, nn->m, nn->v, nn->net.n_params, lr, b1, b2, eps, nn->step, s);
    if (e == hipSuccess) e = launch_pack(nn->net, nn->params, nn->g, nn->t, s);
    return hs(e);
}

int tf_nn_tensor(tf_nn *nn, int id, const void **d_ptr, int32_t dims[4])
{
    if (!nn || !d_ptr || !dims) return TF_E_INVAL;
    if (id >= TF_NN_T_INPUT && id <= TF_NN_T_D1) {
        *d_ptr = nn->act[id];
        return dims_of(nn, id, dims);
    }
    if (id >= TF_NN_T_GRAD_E1 && id < TF_NN_T_GRAD_E1 + 7) {
        if (!nn->training) return TF_E_INVAL;
        const int a = id - TF_NN_T_GRAD_E1 + 1;
        *d_ptr = nn->grad[a];
        return dims_of(nn, a, dims);
    }
    int32_t d[4] = {(int32_t)nn->batch, (int32_t)nn->H, (int32_t)nn->W, 1};
    switch (id) {
    case TF_NN_T_OUT: *d_ptr = nn->out; break;
    case TF_NN_T_DEPTH: *d_ptr = nn->dm; break;
    case TF_NN_T_DDELTA:
        if (!nn->training) return TF_E_INVAL;
        *d_ptr = nn->ddelta;
        break;
    case TF_NN_T_GRADS:
        if (!nn->training) return TF_E_INVAL;
        *d_ptr = nn->grads;
        d[0] = nn->net.n_params;
        d[1] = d[2] = d[3] = 1;
        break;
    case TF_NN_T_PARAMS:
        *d_ptr = nn->params;
        d[0] = nn->net.n_params;
        d[1] = d[2] = d[3] = 1;
        break;
    default: return TF_E_INVAL;
    }
    memcpy(dims, d, sizeof(d));
    return TF_OK;
}

}  // extern "C"
