// tsdf_ctx.h -- host-side state of a libtsdf volume, shared by the single-volume
// API (tsdf_api.hip) and the batched submaps (tsdf_multi_api.hip).  Internal.
#pragma once

#include <vector>

#include "tsdf.h"
#include "tsdf_internal.h"

// ring of HIP event pairs per kernel class; a slot is harvested before reuse
struct Profiler {
    static const int R = 128;
    bool on = false;
    bool created = false;
    hipEvent_t ev[TF_K_COUNT][R][2];
    bool pending[TF_K_COUNT][R] = {};
    int next[TF_K_COUNT] = {};
    uint64_t launches[TF_K_COUNT] = {};
    double ms[TF_K_COUNT] = {};
    uint32_t mask = ~0u;              // kernel classes timed
    uint32_t every = 1;               // time every n-th launch of a class
    uint64_t seen[TF_K_COUNT] = {};   // launches of each class while on
};

struct tf_ctx {
    tf_params p;
    Profiler prof;
    tsdf::Layout L;
    tsdf::Vol v;
    uint8_t *ws;
    void *h_store;
    void *h_transfer;
    bool have_alloc;
    bool bins_pending;                // tf_integrate binned the allocation view's search-range records
    tf_intrinsics alloc_intr;
    float alloc_pose[16];
    const void *alloc_depth;
    int alloc_fmt;
    uint32_t host_flags;              // flags raised on the host (transfer overflow)
    std::vector<uint8_t> host_has;    // host mirror: the store holds data for the entry
    std::vector<int32_t> cand;        // swap-in candidates of the current frame
};

namespace tsdf {
void make_cam(const float *M, const tf_intrinsics *K, Cam &c);
}  // namespace tsdf
