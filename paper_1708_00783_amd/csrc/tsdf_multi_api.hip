// tsdf_multi_api.hip -- host side of the batched rigid submaps (Sec. 7.2):
// workspace carving, composed cameras, the per-frame parameter upload, HIP
// graph capture and replay, and the launch-shape autotuner.
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "tsdf.h"
#include "tsdf_ctx.h"
#include "tsdf_internal.h"

using namespace tsdf;

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct MLayout {
    size_t sub_bytes, subs, vols, msubs, frames, alists, depth, cnt, cur, off, hits, mc, wmask, bins, total;
    uint32_t max_tiles;
};

// smallest tile is 8x8 pixels
uint32_t tiles_of(uint32_t w, uint32_t h, uint32_t tw, uint32_t th) { return ((w + tw - 1) / tw) * ((h + th - 1) / th); }

bool mlayout(const tf_params *p, uint32_t n, uint32_t vw, uint32_t vh, uint32_t cap, MLayout &L)
{
    if (!p || n < 1 || n > (uint32_t)kMaxSubmaps || vw < 1 || vh < 1 || vw > 8192 || vh > 8192) return false;
    if (cap < 1 || cap > (1u << 30) || p->swap_transfer_blocks) return false;
    const size_t sb = tf_workspace_bytes(p);
    if (!sb) return false;
    L = {};
    L.sub_bytes = align256(sb);
    L.max_tiles = (uint32_t)kMaxViews * tiles_of(vw, vh, 8, 8);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    L.subs = take(L.sub_bytes * n);
    L.vols = take(sizeof(Vol) * n);
    L.msubs = take(sizeof(MSub) * n);
    L.frames = take(sizeof(MFrame) * 2);
    L.alists = take((size_t)16 * p->n_blocks * n);
    L.depth = take((size_t)4 * p->max_width * p->max_height);
    L.cnt = take((size_t)4 * L.max_tiles);
    L.cur = take((size_t)4 * L.max_tiles);
    L.off = take((size_t)4 * (L.max_tiles + 1));
    L.hits = take((size_t)8 * L.max_tiles);
    L.mc = take(sizeof(MCtrl));
    L.wmask = take((size_t)8 * kWorldCells);
    L.bins = take((size_t)sizeof(Rec) * cap);
    L.total = o;
    return true;
}

bool shape_ok(const tf_multi_config *c)
{
    if (!c) return false;
    const bool tile = (c->tile_w == 16 && c->tile_h == 16) || (c->tile_w == 32 && c->tile_h == 8) ||
                      (c->tile_w == 16 && c->tile_h == 8) || (c->tile_w == 8 && c->tile_h == 8);
    const int nt = c->integrate_threads;
    return tile && (nt == 64 || nt == 128 || nt == 256 || nt == 512) && c->integrate_groups >= 1 &&
           c->integrate_groups <= kIntegrateGrid && c->bin_groups >= 1 && c->bin_groups <= 65535;
}

// A * inv(P) for rigid transforms, in double, rounded once to float
void compose(const float *A, const float *P, float *out)
{
    double Q[16];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Q[4 * i + j] = (double)P[4 * j + i];
    for (int i = 0; i < 3; ++i)
        Q[4 * i + 3] = -(((double)P[i] * (double)P[3] + (double)P[4 + i] * (double)P[7]) + (double)P[8 + i] * (double)P[11]);
    Q[12] = Q[13] = Q[14] = 0.0;
    Q[15] = 1.0;
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            const double s = (((double)A[4 * r] * Q[c] + (double)A[4 * r + 1] * Q[4 + c]) + (double)A[4 * r + 2] * Q[8 + c]) +
                             (double)A[4 * r + 3] * Q[12 + c];
            out[4 * r + c] = (float)s;
        }
}

bool pose_ok(const float *M)
{
    if (!M) return false;
    for (int i = 0; i < 16; ++i)
        if (!(M[i] == M[i]) || M[i] > 1e30f || M[i] < -1e30f) return false;
    return true;
}

bool intr_ok(const tf_intrinsics *K, uint32_t wmax, uint32_t hmax)
{
    if (!K || K->width < 1 || K->height < 1) return false;
    if ((uint32_t)K->width > wmax || (uint32_t)K->height > hmax) return false;
    if (!(K->fx > 0.0f) || !(K->fy > 0.0f) || !(K->cx == K->cx) || !(K->cy == K->cy)) return false;
    return true;
}

}  // namespace

// what a captured graph depends on besides the pinned parameters
struct GraphKey {
    int valid;
    int do_int, do_ray, fw, fh, n_views, tiles;
    tf_multi_config cfg;
};

struct tf_multi {
    tf_params p;
    uint32_t n;
    uint32_t vw, vh, cap;
    MLayout L;
    uint8_t *ws;
    std::vector<tf_ctx *> subs;
    std::vector<float> poses;        // n x 16
    Vol *d_vols;
    MSub *d_msubs;
    MFrame *d_frame[2];
    MFrame *h_frame[2];
    float *d_depth;
    MTiles t;
    tf_multi_config cfg;
    int half;                        // pinned half of the next call
    hipEvent_t done[2];
    bool done_pending[2];
    hipStream_t cap_stream;
    hipGraphExec_t gexec[2];
    GraphKey gkey[2];
};

namespace {

int hip_status(hipError_t e) { return e == hipSuccess ? TF_OK : TF_E_HIP; }

// frame parameters into the pinned half h (waits for that half's last use)
hipError_t begin_half(tf_multi *m, int h)
{
    if (m->done_pending[h]) {
        hipError_t e = hipEventSynchronize(m->done[h]);
        if (e != hipSuccess) return e;
        m->done_pending[h] = false;
    }
    return hipSuccess;
}

int fill_integrate(tf_multi *m, MFrame &F, const void *d_depth, int fmt, const tf_intrinsics *K, const float *pose,
                   const uint32_t *sel, uint32_t n_sel)
{
    if (!d_depth || (fmt != TF_DEPTH_F32_M && fmt != TF_DEPTH_U16_MM)) return TF_E_INVAL;
    if (!intr_ok(K, m->p.max_width, m->p.max_height) || !pose_ok(pose)) return TF_E_INVAL;
    if (!sel || n_sel < 1 || n_sel > (uint32_t)kMaxSel) return TF_E_INVAL;
    for (uint32_t a = 0; a < n_sel; ++a) {
        if (sel[a] >= m->n) return TF_E_INVAL;
        for (uint32_t b = 0; b < a; ++b)
            if (sel[a] == sel[b]) return TF_E_INVAL;
    }
    F.depth = d_depth;
    F.fmt = fmt;
    F.n_sel = (int32_t)n_sel;
    for (uint32_t a = 0; a < n_sel; ++a) {
        float Mi[16];
        compose(pose, &m->poses[16 * (size_t)sel[a]], Mi);
        F.sel[a] = (int32_t)sel[a];
        make_cam(Mi, K, F.icam[a]);
    }
    return TF_OK;
}

int fill_views(tf_multi *m, MFrame &F, const tf_view *views, uint32_t n_views, int &tiles)
{
    if (!views || n_views < 1 || n_views > (uint32_t)kMaxViews) return TF_E_INVAL;
    const int tw = m->cfg.tile_w, th = m->cfg.tile_h;
    int base = 0;
    for (uint32_t k = 0; k < n_views; ++k) {
        const tf_view &V = views[k];
        if (!intr_ok(&V.intr, m->vw, m->vh) || !pose_ok(V.pose_w2c) || !V.d_points || !V.d_normals) return TF_E_INVAL;
        MView &mv = F.view[k];
        make_cam(V.pose_w2c, &V.intr, mv.cam);
        mv.pts = (float4 *)V.d_points;
        mv.nrm = (float4 *)V.d_normals;
        mv.ntx = (V.intr.width + tw - 1) / tw;
        mv.nty = (V.intr.height + th - 1) / th;
        mv.tile_base = base;
        mv.pad = 0;
        base += mv.ntx * mv.nty;
        for (uint32_t i = 0; i < m->n; ++i) {
            float C[16];
            compose(V.pose_w2c, &m->poses[16 * (size_t)i], C);
            memcpy(F.C[k][i], C, 12 * sizeof(float));
        }
    }
    if ((uint32_t)base > m->L.max_tiles) return TF_E_INVAL;
    F.n_views = (int32_t)n_views;
    tiles = base;
    return TF_OK;
}

// the launches of one call, reading the device parameters of half h
hipError_t enqueue(tf_multi *m, int h, bool do_int, bool do_ray, int fw, int fh, int n_views, int tiles, bool dry,
                   hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(m->d_frame[h], m->h_frame[h], sizeof(MFrame), hipMemcpyHostToDevice, s);
    const MFrame *f = m->d_frame[h];
    if (e == hipSuccess && do_int) {
        e = launch_m_alloc(m->d_vols, m->d_msubs, f, m->t.wmask, fw, fh, s);
        if (e == hipSuccess)
            e = launch_m_integrate(m->d_vols, f, m->cfg.integrate_threads, m->cfg.integrate_groups, dry, s);
    }
    if (e == hipSuccess && do_ray) {
        MTiles t = m->t;
        t.n_tiles = (uint32_t)tiles;
        e = launch_m_bin(m->d_msubs, f, t, n_views, m->cfg.bin_groups, m->p.voxel_size, s);
        if (e == hipSuccess)
            e = launch_m_raycast(m->d_msubs, f, t, m->p.voxel_size, m->p.mu, m->cfg.tile_w, m->cfg.tile_h, s);
    }
    return e;
}

// one call: parameters into a pinned half, then the launches (direct or as a
// graph replay), then the half's completion event
int run(tf_multi *m, const void *d_depth, int fmt, const tf_intrinsics *K, const float *pose, const uint32_t *sel,
        uint32_t n_sel, const tf_view *views, uint32_t n_views, bool use_graph, bool dry, hipStream_t s)
{
    const bool do_int = d_depth != nullptr, do_ray = views != nullptr;
    const int h = m->half;
    hipError_t e = begin_half(m, h);
    if (e != hipSuccess) return TF_E_HIP;
    MFrame &F = *m->h_frame[h];
    F.tw = m->cfg.tile_w;
    F.th = m->cfg.tile_h;
    F.n_sub = (int32_t)m->n;
    F.n_sel = 0;
    F.n_views = 0;
    int st = TF_OK, tiles = 0, fw = 0, fh = 0;
    if (do_int) {
        st = fill_integrate(m, F, d_depth, fmt, K, pose, sel, n_sel);
        fw = K ? K->width : 0;
        fh = K ? K->height : 0;
    }
    if (st == TF_OK && do_ray) st = fill_views(m, F, views, n_views, tiles);
    if (st != TF_OK) return st;
    if (!use_graph) {
        e = enqueue(m, h, do_int, do_ray, fw, fh, (int)n_views, tiles, dry, s);
    } else {
        GraphKey k = {1, do_int, do_ray, fw, fh, do_ray ? (int)n_views : 0, tiles, m->cfg};
        if (!m->gkey[h].valid || memcmp(&k, &m->gkey[h], sizeof(GraphKey)) != 0) {
            if (m->gexec[h]) {
                (void)hipGraphExecDestroy(m->gexec[h]);
                m->gexec[h] = nullptr;
            }
            m->gkey[h].valid = 0;
            hipGraph_t g = nullptr;
            e = hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                hipError_t e2 = enqueue(m, h, do_int, do_ray, fw, fh, (int)n_views, tiles, false, m->cap_stream);
                e = hipStreamEndCapture(m->cap_stream, &g);
                if (e == hipSuccess) e = e2;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&m->gexec[h], g, nullptr, nullptr, 0);
            if (g) (void)hipGraphDestroy(g);
            if (e == hipSuccess) m->gkey[h] = k;
        }
        if (e == hipSuccess) e = hipGraphLaunch(m->gexec[h], s);
    }
    if (e == hipSuccess) e = hipEventRecord(m->done[h], s);
    if (e == hipSuccess) m->done_pending[h] = true;
    m->half = 1 - h;
    return hip_status(e);
}

}  // namespace

extern "C" {

size_t tf_multi_workspace_bytes(const tf_params *p, uint32_t n, uint32_t vw, uint32_t vh, uint32_t cap)
{
    MLayout L;
    if (!mlayout(p, n, vw, vh, cap, L)) return 0;
    return L.total;
}

size_t tf_multi_host_bytes(void) { return 2 * ((sizeof(MFrame) + 255) & ~(size_t)255); }

int tf_multi_create(const tf_params *p, uint32_t n, const float *poses, uint32_t vw, uint32_t vh, uint32_t cap,
                    void *d_ws, size_t bytes, void *h_pinned, size_t h_bytes, tf_stream stream, tf_multi **out)
{
    if (!out || !poses || !d_ws || !h_pinned) return TF_E_INVAL;
    *out = nullptr;
    MLayout L;
    if (!mlayout(p, n, vw, vh, cap, L)) return TF_E_INVAL;
    if (((uintptr_t)d_ws & 255u) || ((uintptr_t)h_pinned & 15u)) return TF_E_INVAL;
    if (bytes < L.total) return TF_E_SPACE;
    if (h_bytes < tf_multi_host_bytes()) return TF_E_SPACE;
    for (uint32_t i = 0; i < n; ++i)
        if (!pose_ok(poses + 16 * (size_t)i)) return TF_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    tf_multi *m = new (std::nothrow) tf_multi();
    if (!m) return TF_E_INVAL;
    m->p = *p;
    m->n = n;
    m->vw = vw;
    m->vh = vh;
    m->cap = cap;
    m->L = L;
    m->ws = (uint8_t *)d_ws;
    m->poses.assign(poses, poses + 16 * (size_t)n);
    m->cfg = {16, 16, 256, 256, 256};
    m->half = 0;
    uint8_t *b = m->ws;
    m->d_vols = (Vol *)(b + L.vols);
    m->d_msubs = (MSub *)(b + L.msubs);
    m->d_frame[0] = (MFrame *)(b + L.frames);
    m->d_frame[1] = m->d_frame[0] + 1;
    const size_t hh = (sizeof(MFrame) + 255) & ~(size_t)255;
    m->h_frame[0] = (MFrame *)h_pinned;
    m->h_frame[1] = (MFrame *)((uint8_t *)h_pinned + hh);
    memset(h_pinned, 0, tf_multi_host_bytes());
    m->d_depth = (float *)(b + L.depth);
    m->t.cnt = (int32_t *)(b + L.cnt);
    m->t.cur = (int32_t *)(b + L.cur);
    m->t.off = (uint32_t *)(b + L.off);
    m->t.acc_hits = (unsigned long long *)(b + L.hits);
    m->t.mc = (MCtrl *)(b + L.mc);
    m->t.wmask = (unsigned long long *)(b + L.wmask);
    m->t.bins = (Rec *)(b + L.bins);
    m->t.cap = cap;
    m->t.n_tiles = L.max_tiles;
    int st = TF_OK;
    std::vector<Vol> hv(n);
    std::vector<MSub> hs(n);
    const float inv_vs = 1.0f / p->voxel_size;
    for (uint32_t i = 0; i < n && st == TF_OK; ++i) {
        tf_ctx *c = nullptr;
        st = tf_create(p, b + L.subs + L.sub_bytes * i, L.sub_bytes, nullptr, nullptr, stream, &c);
        if (st != TF_OK) break;
        m->subs.push_back(c);
        c->v.alist = (int4 *)(b + L.alists + (size_t)16 * p->n_blocks * i);
        hv[i] = c->v;
        hv[i].depth = m->d_depth;   // batched launches share one depth map
        MSub &S = hs[i];
        S.entries = c->v.entries;
        S.occ = c->v.occ;
        S.voxels = c->v.voxels;
        S.alist = c->v.alist;
        S.ctrl = c->v.ctrl;
        S.n_buckets = c->v.n_buckets;
        S.n_excess = c->v.n_excess;
        const float *P = poses + 16 * (size_t)i;
        for (int r = 0; r < 3; ++r) {
            for (int q = 0; q < 3; ++q) S.R[3 * r + q] = P[4 * r + q];
            S.s[r] = P[4 * r + 3] * inv_vs;
        }
    }
    hipError_t e = hipSuccess;
    if (st == TF_OK) e = hipMemcpyAsync(m->d_vols, hv.data(), sizeof(Vol) * n, hipMemcpyHostToDevice, s);
    if (st == TF_OK && e == hipSuccess)
        e = hipMemcpyAsync(m->d_msubs, hs.data(), sizeof(MSub) * n, hipMemcpyHostToDevice, s);
    if (st == TF_OK && e == hipSuccess) {
        MCtrl mc = {};
        e = hipMemcpyAsync(m->t.mc, &mc, sizeof(MCtrl), hipMemcpyHostToDevice, s);
    }
    if (st == TF_OK && e == hipSuccess) e = launch_m_clear(m->t, s);
    // the host copies above come from this frame's stack: wait for them
    if (st == TF_OK && e == hipSuccess) e = hipStreamSynchronize(s);
    if (st == TF_OK && e == hipSuccess) e = hipEventCreateWithFlags(&m->done[0], hipEventDisableTiming);
    if (st == TF_OK && e == hipSuccess) e = hipEventCreateWithFlags(&m->done[1], hipEventDisableTiming);
    if (st == TF_OK && e == hipSuccess) e = hipStreamCreateWithFlags(&m->cap_stream, hipStreamNonBlocking);
    if (st == TF_OK && e != hipSuccess) st = TF_E_HIP;
    if (st != TF_OK) {
        tf_multi_destroy(m);
        return st;
    }
    *out = m;
    return TF_OK;
}

int tf_multi_destroy(tf_multi *m)
{
    if (!m) return TF_E_INVAL;
    for (int h = 0; h < 2; ++h) {
        if (m->gexec[h]) (void)hipGraphExecDestroy(m->gexec[h]);
        if (m->done[h]) (void)hipEventDestroy(m->done[h]);
    }
    if (m->cap_stream) (void)hipStreamDestroy(m->cap_stream);
    for (tf_ctx *c : m->subs) tf_destroy(c);
    delete m;
    return TF_OK;
}

int tf_multi_submap(tf_multi *m, uint32_t i, tf_ctx **out)
{
    if (!m || !out || i >= m->n) return TF_E_INVAL;
    *out = m->subs[i];
    return TF_OK;
}

int tf_multi_set_config(tf_multi *m, const tf_multi_config *c)
{
    if (!m || !shape_ok(c)) return TF_E_INVAL;
    m->cfg = *c;
    return TF_OK;
}

int tf_multi_get_config(const tf_multi *m, tf_multi_config *c)
{
    if (!m || !c) return TF_E_INVAL;
    *c = m->cfg;
    return TF_OK;
}

int tf_multi_integrate(tf_multi *m, const void *d_depth, int fmt, const tf_intrinsics *K, const float pose[16],
                       const uint32_t *sel, uint32_t n_sel, tf_stream stream)
{
    if (!m || !d_depth) return TF_E_INVAL;
    return run(m, d_depth, fmt, K, pose, sel, n_sel, nullptr, 0, false, false, (hipStream_t)stream);
}

int tf_multi_raycast(tf_multi *m, const tf_view *views, uint32_t n_views, tf_stream stream)
{
    if (!m || !views) return TF_E_INVAL;
    return run(m, nullptr, 0, nullptr, nullptr, nullptr, 0, views, n_views, false, false, (hipStream_t)stream);
}

int tf_multi_frame(tf_multi *m, const void *d_depth, int fmt, const tf_intrinsics *K, const float pose[16],
                   const uint32_t *sel, uint32_t n_sel, const tf_view *views, uint32_t n_views, int use_graph,
                   tf_stream stream)
{
    if (!m || !d_depth || !views) return TF_E_INVAL;
    return run(m, d_depth, fmt, K, pose, sel, n_sel, views, n_views, use_graph != 0, false, (hipStream_t)stream);
}

int tf_multi_range_image(tf_multi *m, const tf_view *view, float *d_zmin, float *d_zmax, tf_stream stream)
{
    if (!m || !view || !d_zmin || !d_zmax) return TF_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    const int h = m->half;
    if (begin_half(m, h) != hipSuccess) return TF_E_HIP;
    MFrame &F = *m->h_frame[h];
    F.tw = m->cfg.tile_w;
    F.th = m->cfg.tile_h;
    F.n_sub = (int32_t)m->n;
    F.n_sel = 0;
    int tiles = 0;
    int st = fill_views(m, F, view, 1, tiles);
    if (st != TF_OK) return st;
    hipError_t e = hipMemcpyAsync(m->d_frame[h], m->h_frame[h], sizeof(MFrame), hipMemcpyHostToDevice, s);
    MTiles t = m->t;
    t.n_tiles = (uint32_t)tiles;
    if (e == hipSuccess) e = launch_m_bin(m->d_msubs, m->d_frame[h], t, 1, m->cfg.bin_groups, m->p.voxel_size, s);
    if (e == hipSuccess)
        e = launch_m_range_write(m->d_msubs, m->d_frame[h], t, 0, tiles, d_zmin, d_zmax, m->cfg.tile_w, m->cfg.tile_h,
                                 s);
    if (e == hipSuccess) e = hipEventRecord(m->done[h], s);
    if (e == hipSuccess) m->done_pending[h] = true;
    m->half = 1 - h;
    return hip_status(e);
}

int tf_multi_autotune(tf_multi *m, const void *d_depth, int fmt, const tf_intrinsics *K, const float pose[16],
                      const uint32_t *sel, uint32_t n_sel, const tf_view *views, uint32_t n_views, int reps,
                      tf_multi_config *best, float *best_ms, tf_stream stream)
{
    if (!m || !d_depth || !views || reps < 1 || reps > 100) return TF_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    const tf_multi_config keep = m->cfg;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return TF_E_HIP;
    int st = TF_OK;
    // one candidate: an untimed warm-up, then `reps` runs each timed on its
    // own; the median of those times (robust to a stray slow run)
    auto timed = [&](const tf_multi_config &c, bool integ, float &ms) -> int {
        m->cfg = c;
        std::vector<float> t;
        for (int r = -1; r < reps; ++r) {
            if (r >= 0 && hipEventRecord(e0, s) != hipSuccess) return TF_E_HIP;
            const int rs = integ ? run(m, d_depth, fmt, K, pose, sel, n_sel, nullptr, 0, false, true, s)
                                 : run(m, nullptr, 0, nullptr, nullptr, nullptr, 0, views, n_views, false, false, s);
            if (rs != TF_OK) return rs;
            if (r >= 0) {
                float x = 0.0f;
                if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&x, e0, e1) != hipSuccess)
                    return TF_E_HIP;
                t.push_back(x);
            }
        }
        std::sort(t.begin(), t.end());
        ms = t[t.size() / 2];
        return TF_OK;
    };
    // Each stage's candidates are timed in two interleaved passes (so that a
    // drift of the clock or of the cache state between candidates averages
    // out), each keeping its better median; a later candidate replaces the
    // best only when it is faster by more than 2%, so near-ties keep the
    // earlier (default-first) order and repeated runs pick the same shape.
    auto pick = [&](const std::vector<tf_multi_config> &cand, bool integ, tf_multi_config &bc, float &bt) -> int {
        std::vector<float> best(cand.size(), 3.4e38f);
        for (int pass = 0; pass < 2; ++pass)
            for (size_t i = 0; i < cand.size(); ++i) {
                float ms = 0.0f;
                const int r = timed(cand[i], integ, ms);
                if (r != TF_OK) return r;
                if (ms < best[i]) best[i] = ms;
            }
        size_t bi = 0;
        for (size_t i = 1; i < cand.size(); ++i)
            if (best[i] < 0.98f * best[bi]) bi = i;
        bc = cand[bi];
        bt = best[bi];
        return TF_OK;
    };
    // the frame's allocation (dry integration passes re-run it: idempotent
    // for one frame, since every touched block exists after the first)
    tf_multi_config cur = keep;
    float ms_int = 0.0f, ms_ray = 0.0f;
    static const int nts[4] = {64, 128, 256, 512};
    static const int grps[4] = {64, 128, 256, 512};
    std::vector<tf_multi_config> ci;
    for (int a = 0; a < 4; ++a)
        for (int g = 0; g < 4; ++g) {
            tf_multi_config c = cur;
            c.integrate_threads = nts[a];
            c.integrate_groups = grps[g];
            ci.push_back(c);
        }
    tf_multi_config bcfg = cur;
    st = pick(ci, true, bcfg, ms_int);
    cur = bcfg;
    static const int tws[4][2] = {{16, 16}, {32, 8}, {16, 8}, {8, 8}};
    static const int bgs[3] = {64, 256, 1024};
    std::vector<tf_multi_config> cr;
    for (int a = 0; a < 4; ++a)
        for (int g = 0; g < 3; ++g) {
            tf_multi_config c = cur;
            c.tile_w = tws[a][0];
            c.tile_h = tws[a][1];
            c.bin_groups = bgs[g];
            cr.push_back(c);
        }
    if (st == TF_OK) st = pick(cr, false, bcfg, ms_ray);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != TF_OK) {
        m->cfg = keep;
        return st;
    }
    m->cfg = bcfg;
    if (best) *best = bcfg;
    if (best_ms) *best_ms = ms_int + ms_ray;
    return TF_OK;
}

int tf_multi_get_stats(tf_multi *m, tf_multi_stats *out, tf_stream stream)
{
    if (!m || !out) return TF_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    memset(out, 0, sizeof(*out));
    out->n_submaps = m->n;
    for (tf_ctx *c : m->subs) {
        tf_stats st;
        int r = tf_get_stats(c, &st, stream);
        if (r != TF_OK) return r;
        out->flags |= st.flags;
        out->allocated_blocks += st.n_allocated;
        out->total_integrated_blocks += st.total_integrated_blocks;
        out->total_written_columns += st.total_written_columns;
    }
    MCtrl mc;
    std::vector<unsigned long long> hits(m->L.max_tiles);
    hipError_t e = hipMemcpyAsync(&mc, m->t.mc, sizeof(MCtrl), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hits.data(), m->t.acc_hits, 8 * (size_t)m->L.max_tiles, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return TF_E_HIP;
    out->flags |= mc.flags;
    out->total_bin_entries = mc.tot_bin;
    out->total_block_views = mc.tot_blkview;
    out->raycast_calls = mc.n_raycast;
    for (unsigned long long h : hits) out->total_rays_hit += h;
    return TF_OK;
}

}  // extern "C"
