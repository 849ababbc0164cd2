// Host-side internals shared by the C ABI (ca_api.cpp) and the serving
// loop (ca_server.cpp): plans, the context, and the enqueue of one batch.
// Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <map>
#include <vector>

#include "ca_cnn.h"

namespace cahost {

using ca::FrameDev;
using ca::Record;

struct Shape {
    int32_t W, H;
};

struct Plan {
    // cache key
    std::vector<ca_frame_desc> dims;
    int32_t n_h = 0, n_v = 0, attempts = 0;
    double alpha = 0, t_g = 0, t_theta = 0, t_iota = 0;
    // device buffers (one allocation)
    void *mem = nullptr;
    size_t bytes = 0;
    FrameDev *fd = nullptr;
    int32_t *strips = nullptr;
    float *lut = nullptr;
    ca_point *cand = nullptr;
    Record *rec = nullptr;
    uint32_t *ctl = nullptr;    // fused-kernel control words (zero between calls)
    ca_result *res2 = nullptr;  // handcrafted results of a learned call with fallback
    int32_t *flist = nullptr;   // frame indices grouped by frame shape
    struct ShapeClass {
        int32_t W, H, first, count;
    };
    std::vector<ShapeClass> classes;
    std::vector<Shape> shapes;  // distinct frame shapes; shape k's strips at table k * S
    bool dynamic = false;       // a serving plan: descriptors rewritten per batch, not cached
    int32_t tuned_schedule = -1; // faster schedule of this batch (ca_autotune), -1 untuned
    int32_t tuned_pipeline = 1;  // sub-batches of its split calls (ca_autotune)
    // launch facts
    int32_t n_frames = 0, P = 0, groups = 0, sg_len = 0, line_pitch = 0;
    int32_t rec_groups = 0;     // attempt-group records per frame the block holds (16 lanes)
    bool rows_aligned = false;  // every row offset a multiple of 16
    size_t lds = 0;
    size_t fused_lds = 0;
    int32_t fused_grid = 0;     // resident workgroups of the fused kernel
    int32_t pins = 0;           // graphs that replay this plan (never evicted while > 0)
    uint64_t last_use = 0;
};

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess)
            return;
        ok = prev == dev || hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (ok && prev >= 0)
            (void)hipSetDevice(prev);
    }
};

}  // namespace cahost

struct ca_ctx {
    int device = 0;
    size_t budget = 0;
    size_t used = 0;
    size_t max_lds = 0;
    uint64_t tick = 0;
    std::vector<cahost::Plan *> plans;
    // kernel timing: 4 events per timed call (before strips, between kernels, after select)
    std::vector<hipEvent_t> prof_events;
    int32_t prof_capacity = 0;
    int32_t prof_used = 0;
    // schedule options (ca_set_option)
    int64_t schedule = CA_SCHEDULE_AUTO;
    int64_t lag = 4;
    int64_t queues = 0;         // 0: 8 when the batch has >= 16 frames, else 1
    int64_t grid = 0;           // 0: resident workgroups from the occupancy query
    int64_t spin_limit = 1 << 20;
    int64_t pipeline = 0;       // sub-batches of a split-schedule call (1: no side streams;
                                // 0: the batch's autotuned count under CA_SCHEDULE_AUTO, else 1)
    int32_t last_schedule = -1, last_pipeline = 0;  // what the last ca_autotune chose
    int n_cu = 0;
    // side streams of the pipelined split schedule, with their fork/join events
    hipStream_t side[2] = {nullptr, nullptr};
    hipEvent_t fork = nullptr;
    hipEvent_t join[2] = {nullptr, nullptr};
    uint8_t *model = nullptr;   // learned scorer, device block (ca_set_model)
    float *train = nullptr;     // master weights [kCnnParams], then momentum [kCnnParams]
    float *partial = nullptr;   // gradient partials [grad_grid][kCnnGradStride]
    int grad_grid = 0;
    uint8_t *model2d = nullptr;   // the paper's 2-D scorer, device block (ca_set_model_2d)
    float *train2d = nullptr;     // its master weights [kC2Params], then momentum
    float *partial2d = nullptr;   // its gradient partials [grad2d_grid][kC2GradStride]
    int grad2d_grid = 0;
    int64_t strips_per_group = 0;   // 0: tuned per frame shape
    int64_t ransac_lanes = 0;       // 0: chosen per batch from its attempt workgroups
    int cnn_groups_per_xcd = 0;     // resident learned-strip workgroups per XCD (0: not queried)
    std::map<std::array<int32_t, 4>, int32_t> tuned;   // (W, H, n_h, n_v) -> strip items per group
    // score tables of the last (t_g, t_theta, t_iota): SG[lut_sg_len] | ST | SI
    bool lut_valid = false;
    double lut_key[3] = {0, 0, 0};
    int32_t lut_sg_len = 0;
    float lut_cache[CA_SG_CAPACITY + ca::kQtBins + ca::kLumaLevels];
    float lut_st[ca::kQtBins];
    float lut_si[ca::kLumaLevels];
};


namespace cahost {

int validate(const ca_frame_desc *dims, int32_t n, const ca_params &p);
// Eq. 1 positions of n strips across an extent (floor, clamped to [1, extent - 2]).
int strip_positions(int32_t extent, int32_t n, double alpha, int32_t *pos);

// Byte layout of a plan's device block.  Its first image_bytes bytes
// (frame descriptors, strip tables, score tables, frame list grouped by
// shape, zeroed control words) are built on the host and uploaded with one
// copy; candidates, attempt-group records and fallback results follow and
// are written by the kernels only.
struct PlanLayout {
    size_t o_fd = 0, o_strips = 0, o_lut = 0, o_flist = 0, o_ctl = 0, image_bytes = 0;
    size_t o_cand = 0, o_rec = 0, o_res2 = 0, total = 0;
    int32_t n_shapes = 0;
};
// The context's score tables for p (computed once per (t_g, t_theta, t_iota)).
const float *cached_tables(ca_ctx *ctx, const ca_params &p, int32_t *sg_len);
// Launch facts of pl (P, groups, sg_len, line pitch, LDS sizes, row
// alignment; not the fused grid) and the layout L; the distinct shapes go to
// shapes[0 .. max_shapes).  With `image`, also writes the host image
// (image_cap >= L->image_bytes).  CA_E_NOMEM for more than max_shapes
// shapes or a short image, CA_E_UNSUPPORTED when a strip tile exceeds LDS.
int plan_layout(const ca_ctx *ctx, const ca_frame_desc *dims, int32_t n, const ca_params &p,
                const float *lut, int32_t sg_len, Shape *shapes, int32_t max_shapes, Plan *pl,
                PlanLayout *L, uint8_t *image, size_t image_cap);
// Points pl's buffers into the device block at base.
void plan_pointers(Plan *pl, void *base, const PlanLayout &L);
// Resident workgroups of the fused kernel for this LDS size.
int fused_grid(const ca_ctx *ctx, size_t fused_lds);
// Once per device with the device current: locate the no-allocation entry
// point's scratch (ca_noalloc.hip).
int scratch_setup(int device);
int build_plan(ca_ctx *ctx, const ca_frame_desc *dims, int32_t n, const ca_params &p, Plan **out);
void free_plan(ca_ctx *ctx, Plan *pl);
// Enqueue the whole path for frames [0, n) of a plan on stream s.
int enqueue(ca_ctx *ctx, Plan *pl, const uint8_t *frames, int32_t n, const ca_params &p,
            ca_point *points_out, ca_attempt *attempts_out, ca_result *out, hipStream_t s,
            bool timed);

}  // namespace cahost
