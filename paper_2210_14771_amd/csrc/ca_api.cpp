// Host core of the content-area estimator: the C ABI declared in
// include/contentarea.h.  Validates arguments, builds and caches per-batch
// plans (strip positions of Eq. 1, the score tables of Eq. 2, scratch
// buffers) in device memory, and enqueues the three kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "ca_host.h"

namespace cahost {

constexpr double kPi = 3.14159265358979323846;

// ------------------------------------------------------------- tables -----

int strip_positions(int32_t extent, int32_t n, double alpha, int32_t *pos)
{
    // Eq. 1: h_i = extent / (1 + exp(-(alpha / N)(i - (N - 1) / 2)))
    if (extent < 3 || n < 0)
        return CA_E_INVAL;
    for (int32_t i = 0; i < n; ++i) {
        const double t = (alpha / (double)n) * ((double)i - (double)(n - 1) / 2.0);
        const double h = (double)extent / (1.0 + std::exp(-t));
        int32_t p = (int32_t)std::floor(h);
        p = p < 1 ? 1 : p;
        p = p > extent - 2 ? extent - 2 : p;
        pos[i] = p;
    }
    return CA_OK;
}

int score_tables(const ca_params &p, float *sg, int32_t *sg_len, float *st, float *si)
{
    // s_g = tanh(|g| / t_g) at |g| = q / 8; the table ends at its first 1.0f
    int32_t n = 0;
    for (int32_t q = 0; q < CA_SG_CAPACITY; ++q) {
        const float v = (float)std::tanh((double)q / (8.0 * p.t_g));
        sg[q] = v;
        n = q + 1;
        if (v == 1.0f)
            break;
    }
    *sg_len = n;
    // s_theta = 1 - tanh(theta_q / t_theta): theta_q is the lower edge of
    // pseudo-angle bin q (u = q / 1024 = |c x g| / (|c x g| + c.g) below 90 deg)
    for (int32_t q = 0; q < ca::kQtBins; ++q) {
        const double u = (double)q / 1024.0;
        const double th = u <= 1.0 ? std::atan2(u, 1.0 - u) : kPi - std::atan2(2.0 - u, u - 1.0);
        st[q] = (float)(1.0 - std::tanh(th * (180.0 / kPi) / p.t_theta_deg));
    }
    // s_iota = 1 - tanh(iota / t_iota)
    for (int32_t i = 0; i < ca::kLumaLevels; ++i)
        si[i] = (float)(1.0 - std::tanh((double)i / p.t_iota));
    return CA_OK;
}

// --------------------------------------------------------------- plans ----

bool same_key(const Plan &pl, const ca_frame_desc *dims, int32_t n, const ca_params &p)
{
    return pl.n_frames == n && pl.n_h == p.n_hstrips && pl.n_v == p.n_vstrips
           && pl.attempts == p.ransac_attempts && pl.alpha == p.alpha && pl.t_g == p.t_g
           && pl.t_theta == p.t_theta_deg && pl.t_iota == p.t_iota
           && std::memcmp(pl.dims.data(), dims, sizeof(ca_frame_desc) * (size_t)n) == 0;
}

}  // namespace cahost

using namespace cahost;

namespace cahost {

void free_plan(ca_ctx *ctx, Plan *pl)
{
    if (pl->mem) {
        (void)hipDeviceSynchronize();  // the plan may still be in use by queued work
        (void)hipFree(pl->mem);
        ctx->used -= pl->bytes;
    }
    delete pl;
}

int validate(const ca_frame_desc *dims, int32_t n, const ca_params &p)
{
    if (p.n_hstrips < 0 || p.n_vstrips < 0 || p.n_hstrips > CA_MAX_STRIPS
        || p.n_vstrips > CA_MAX_STRIPS || p.n_hstrips + p.n_vstrips < 1)
        return CA_E_INVAL;
    if (p.ransac_attempts < 1 || p.ransac_attempts > CA_MAX_ATTEMPTS)
        return CA_E_INVAL;
    if (p.refine_iters < 0 || p.refine_iters > 64 || (p.sampler != 0 && p.sampler != 1))
        return CA_E_INVAL;
    if (p.scorer != CA_SCORER_HANDCRAFTED && p.scorer != CA_SCORER_LEARNED
        && p.scorer != CA_SCORER_LEARNED_2D)
        return CA_E_INVAL;
    if (!(p.fallback_inlier_frac >= 0.0f && p.fallback_inlier_frac <= 1.0f))
        return CA_E_INVAL;
    if (!(p.t_g > 0) || !(p.t_theta_deg > 0) || !(p.t_iota > 0) || !(p.t_ri >= 0)
        || !std::isfinite(p.alpha) || !std::isfinite(p.t_ps) || !std::isfinite(p.t_cs)
        || !std::isfinite(p.r_min) || !std::isfinite(p.r_max) || !std::isfinite(p.d_max)
        || !std::isfinite(p.t_ri) || p.t_px < 0)
        return CA_E_INVAL;
    for (int32_t i = 0; i < n; ++i) {
        const ca_frame_desc &d = dims[i];
        if (d.width < 16 || d.height < 16 || d.width > CA_MAX_EXTENT || d.height > CA_MAX_EXTENT)
            return CA_E_INVAL;
        if (d.byte_offset < 0 || (int64_t)d.row_stride < 3 * (int64_t)d.width)
            return CA_E_INVAL;
        if (d.pixel_stride != 3)
            return CA_E_UNSUPPORTED;
    }
    return CA_OK;
}

const float *cached_tables(ca_ctx *ctx, const ca_params &p, int32_t *sg_len)
{
    // the score tables of the last (t_g, t_theta, t_iota) are kept in the
    // context: SG[sg_len] | ST[2049] | SI[256]
    if (!ctx->lut_valid || ctx->lut_key[0] != p.t_g || ctx->lut_key[1] != p.t_theta_deg
        || ctx->lut_key[2] != p.t_iota) {
        float *sg = ctx->lut_cache;
        int32_t n = 0;
        score_tables(p, sg, &n, ctx->lut_st, ctx->lut_si);
        std::memmove(sg + n, ctx->lut_st, sizeof(float) * ca::kQtBins);
        std::memmove(sg + n + ca::kQtBins, ctx->lut_si, sizeof(float) * ca::kLumaLevels);
        ctx->lut_sg_len = n;
        ctx->lut_key[0] = p.t_g;
        ctx->lut_key[1] = p.t_theta_deg;
        ctx->lut_key[2] = p.t_iota;
        ctx->lut_valid = true;
    }
    *sg_len = ctx->lut_sg_len;
    return ctx->lut_cache;
}

int plan_layout(const ca_ctx *ctx, const ca_frame_desc *dims, int32_t n, const ca_params &p,
                const float *lut, int32_t sg_len, Shape *shapes, int32_t max_shapes, Plan *pl,
                PlanLayout *L, uint8_t *image, size_t image_cap)
{
    const int32_t S = p.n_hstrips + p.n_vstrips;
    pl->n_frames = n;
    pl->n_h = p.n_hstrips;
    pl->n_v = p.n_vstrips;
    pl->attempts = p.ransac_attempts;
    pl->alpha = p.alpha;
    pl->t_g = p.t_g;
    pl->t_theta = p.t_theta_deg;
    pl->t_iota = p.t_iota;
    pl->P = 2 * S;
    pl->groups = ca::attempt_groups(p.ransac_attempts, ca::kLanesPerAttempt);
    pl->rec_groups = ca::attempt_groups(p.ransac_attempts, ca::kMaxLanesPerAttempt);
    pl->sg_len = sg_len;
    // distinct frame shapes in order of first appearance
    int32_t n_shapes = 0, longest = 0;
    pl->rows_aligned = true;
    for (int32_t i = 0; i < n; ++i) {
        const ca_frame_desc &d = dims[i];
        int32_t k = 0;
        while (k < n_shapes && !(shapes[k].W == d.width && shapes[k].H == d.height))
            ++k;
        if (k == n_shapes) {
            if (n_shapes == max_shapes)
                return CA_E_NOMEM;
            shapes[n_shapes++] = {d.width, d.height};
        }
        longest = std::max(longest, std::max(d.width, d.height));
        if ((d.byte_offset % 16) != 0 || (d.row_stride % 16) != 0)
            pl->rows_aligned = false;
    }
    pl->line_pitch = (int32_t)align_up((size_t)longest, 16);
    pl->lds = ca::strip_lds_bytes(sg_len, pl->line_pitch);
    pl->fused_lds = ca::fused_lds_bytes(sg_len, pl->line_pitch);
    if (pl->lds > ctx->max_lds || pl->fused_lds > ctx->max_lds)
        return CA_E_UNSUPPORTED;
    const size_t lut_len = (size_t)sg_len + ca::kQtBins + ca::kLumaLevels;
    L->n_shapes = n_shapes;
    L->o_fd = 0;
    L->o_strips = align_up(sizeof(FrameDev) * (size_t)n, 256);
    L->o_lut = align_up(L->o_strips + sizeof(int32_t) * (size_t)n_shapes * (size_t)S, 256);
    L->o_flist = align_up(L->o_lut + sizeof(float) * lut_len, 256);
    L->o_ctl = align_up(L->o_flist + sizeof(int32_t) * (size_t)n, 256);
    L->image_bytes = L->o_ctl + sizeof(uint32_t) * ca::ctl_words(n);
    L->o_cand = align_up(L->image_bytes, 256);
    L->o_rec = align_up(L->o_cand + sizeof(ca_point) * (size_t)n * (size_t)pl->P, 256);
    L->o_res2 = align_up(L->o_rec + sizeof(Record) * (size_t)n * (size_t)pl->rec_groups, 256);
    L->total = align_up(L->o_res2 + sizeof(ca_result) * (size_t)n, 256);
    if (!image)
        return CA_OK;
    if (image_cap < L->image_bytes)
        return CA_E_NOMEM;
    std::memset(image, 0, L->image_bytes);
    FrameDev *fd = reinterpret_cast<FrameDev *>(image + L->o_fd);
    int32_t *strips = reinterpret_cast<int32_t *>(image + L->o_strips);
    int32_t *flist = reinterpret_cast<int32_t *>(image + L->o_flist);
    for (int32_t k = 0; k < n_shapes; ++k) {
        strip_positions(shapes[k].H, p.n_hstrips, p.alpha, strips + (size_t)k * S);
        strip_positions(shapes[k].W, p.n_vstrips, p.alpha, strips + (size_t)k * S + p.n_hstrips);
    }
    std::memcpy(image + L->o_lut, lut, sizeof(float) * lut_len);
    // frame indices grouped by shape: the strip kernel may be launched per shape
    int32_t at = 0;
    for (int32_t k = 0; k < n_shapes; ++k)
        for (int32_t i = 0; i < n; ++i)
            if (dims[i].width == shapes[k].W && dims[i].height == shapes[k].H) {
                flist[at++] = i;
                const ca_frame_desc &d = dims[i];
                fd[i] = FrameDev{d.byte_offset, d.width, d.height, d.row_stride, k * S, d.frame_uid};
            }
    return CA_OK;
}

void plan_pointers(Plan *pl, void *base_mem, const PlanLayout &L)
{
    uint8_t *base = static_cast<uint8_t *>(base_mem);
    pl->fd = reinterpret_cast<FrameDev *>(base + L.o_fd);
    pl->strips = reinterpret_cast<int32_t *>(base + L.o_strips);
    pl->lut = reinterpret_cast<float *>(base + L.o_lut);
    pl->flist = reinterpret_cast<int32_t *>(base + L.o_flist);
    pl->ctl = reinterpret_cast<uint32_t *>(base + L.o_ctl);
    pl->cand = reinterpret_cast<ca_point *>(base + L.o_cand);
    pl->rec = reinterpret_cast<Record *>(base + L.o_rec);
    pl->res2 = reinterpret_cast<ca_result *>(base + L.o_res2);
}

int fused_grid(const ca_ctx *ctx, size_t fused_lds)
{
    int per_cu = 0;
    if (ca::fused_occupancy(fused_lds, &per_cu) != hipSuccess || per_cu < 1) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    return per_cu * ctx->n_cu;
}

int build_plan(ca_ctx *ctx, const ca_frame_desc *dims, int32_t n, const ca_params &p, Plan **out)
{
    Plan *pl = new (std::nothrow) Plan();
    if (!pl)
        return CA_E_NOMEM;
    pl->dims.assign(dims, dims + n);
    int32_t sg_len = 0;
    const float *lut = cached_tables(ctx, p, &sg_len);
    std::vector<Shape> shapes((size_t)n);
    PlanLayout L;
    int rc = plan_layout(ctx, dims, n, p, lut, sg_len, shapes.data(), n, pl, &L, nullptr, 0);
    std::vector<uint8_t> image;
    if (rc == CA_OK) {
        image.resize(L.image_bytes);
        rc = plan_layout(ctx, dims, n, p, lut, sg_len, shapes.data(), n, pl, &L, image.data(),
                         image.size());
    }
    if (rc != CA_OK) {
        delete pl;
        return rc;
    }
    shapes.resize((size_t)L.n_shapes);
    int32_t first = 0;
    for (const Shape &sh : shapes) {
        int32_t count = 0;
        for (int32_t i = 0; i < n; ++i)
            count += dims[i].width == sh.W && dims[i].height == sh.H;
        pl->classes.push_back({sh.W, sh.H, first, count});
        first += count;
    }
    pl->shapes = shapes;
    pl->fused_grid = fused_grid(ctx, pl->fused_lds);

    // evict least recently used unpinned plans until this one fits the budget
    while (ctx->used + L.total > ctx->budget) {
        long lru = -1;
        for (size_t k = 0; k < ctx->plans.size(); ++k)
            if (ctx->plans[k]->pins == 0
                && (lru < 0 || ctx->plans[k]->last_use < ctx->plans[(size_t)lru]->last_use))
                lru = (long)k;
        if (lru < 0)
            break;
        free_plan(ctx, ctx->plans[(size_t)lru]);
        ctx->plans.erase(ctx->plans.begin() + lru);
    }
    if (ctx->used + L.total > ctx->budget) {
        delete pl;
        return CA_E_NOMEM;
    }
    if (hipMalloc(&pl->mem, L.total) != hipSuccess) {
        (void)hipGetLastError();
        delete pl;
        return CA_E_NOMEM;
    }
    pl->bytes = L.total;
    ctx->used += L.total;
    plan_pointers(pl, pl->mem, L);
    // plans are built once per batch shape; a blocking upload keeps them simple
    if (hipMemcpy(pl->mem, image.data(), image.size(), hipMemcpyHostToDevice) != hipSuccess
        || hipDeviceSynchronize() != hipSuccess) {
        (void)hipGetLastError();
        free_plan(ctx, pl);
        return CA_E_DEVICE;
    }
    ctx->plans.push_back(pl);
    *out = pl;
    return CA_OK;
}

// Validated parameters and the (cached or new) plan of a batch.  The caller
// holds a DeviceGuard.
int get_plan(ca_ctx *ctx, const ca_frame_desc *dims, int32_t n, const ca_params &p, Plan **out)
{
    int rc = validate(dims, n, p);
    if (rc != CA_OK)
        return rc;
    Plan *pl = nullptr;
    for (Plan *c : ctx->plans)
        if (!c->dynamic && same_key(*c, dims, n, p)) {
            pl = c;
            break;
        }
    if (!pl) {
        rc = build_plan(ctx, dims, n, p, &pl);
        if (rc != CA_OK)
            return rc;
    }
    pl->last_use = ++ctx->tick;
    *out = pl;
    return CA_OK;
}

// Enqueue the whole path for one batch on stream `s`.
int32_t strips_per_group(const ca_ctx *ctx, int32_t W, int32_t H, const ca_params &p)
{
    if (ctx->strips_per_group > 0)
        return (int32_t)ctx->strips_per_group;
    const auto it = ctx->tuned.find({W, H, p.n_hstrips, p.n_vstrips});
    return it == ctx->tuned.end() ? 1 : it->second;
}

// Strip launches of one shape class with T items per workgroup.
hipError_t launch_class_strips(const ca::StripArgs &base, const Plan *pl,
                               const Plan::ShapeClass &c, int32_t T, int32_t S, hipStream_t st)
{
    ca::StripArgs a = base;
    a.frame0 = 0;
    a.frame_list = pl->flist + c.first;
    a.n_items = c.count * S;
    a.items_per_group = T;
    const int32_t groups = (a.n_items + T - 1) / T;
    a.per_xcd = (groups + 7) / 8;
    return ca::launch_strips(a, pl->lds, st);
}

// Lanes per RANSAC attempt of an n-frame split call: the fewest that give
// at least one attempt workgroup per compute unit (a small batch otherwise
// leaves most of the device idle), at most 8 (measured on 8 x 640x480 with
// 256 attempts: 16.5, 14.4, 13.5 and 15.4 us per launch at 2, 4, 8 and 16
// lanes; beyond 8 the per-attempt solves repeated on every lane cost more
// than the shorter point loops save).
int32_t ransac_lanes(const ca_ctx *ctx, int32_t n, int32_t attempts)
{
    if (ctx->ransac_lanes > 0)
        return (int32_t)ctx->ransac_lanes;
    constexpr int32_t kAutoMaxLanes = 8;
    int32_t lanes = ca::kLanesPerAttempt;
    while (lanes < kAutoMaxLanes
           && (int64_t)n * ca::attempt_groups(attempts, lanes) < (int64_t)ctx->n_cu)
        lanes *= 2;
    return lanes;
}

// keep: the learned results when this is the handcrafted pass of the
// fallback (frames whose learned result stands are skipped; that pass takes
// the split schedule, whose kernels implement the skip), else null.
int enqueue_one(ca_ctx *ctx, Plan *pl, const uint8_t *frames, int32_t n, const ca_params &p,
                ca_point *points_out, ca_attempt *attempts_out, ca_result *out, hipStream_t s,
                bool timed, const ca_result *keep = nullptr, float keep_frac = 0.0f)
{
    const bool fused = ctx->schedule == CA_SCHEDULE_FUSED
                       || (ctx->schedule == CA_SCHEDULE_AUTO
                           && pl->tuned_schedule == CA_SCHEDULE_FUSED);
    const bool fused_path = fused && p.scorer == CA_SCORER_HANDCRAFTED && !keep;
    // the persistent kernel takes attempt groups of two lanes per attempt
    const int32_t lanes =
        fused_path ? ca::kLanesPerAttempt : ransac_lanes(ctx, n, p.ransac_attempts);
    const int32_t groups = ca::attempt_groups(p.ransac_attempts, lanes);

    ca::StripArgs sa;
    sa.frames = frames;
    sa.fd = pl->fd;
    sa.strips = pl->strips;
    sa.lut = pl->lut;
    sa.cand = points_out ? points_out : pl->cand;
    sa.sg_len = pl->sg_len;
    sa.n_h = p.n_hstrips;
    sa.n_v = p.n_vstrips;
    sa.n_items = n * (p.n_hstrips + p.n_vstrips);
    sa.per_xcd = (sa.n_items + 7) / 8;
    sa.line_pitch = pl->line_pitch;
    sa.aligned = (pl->rows_aligned && (reinterpret_cast<uintptr_t>(frames) % 16) == 0) ? 1 : 0;
    sa.frame0 = 0;
    sa.frame_list = nullptr;
    sa.items_per_group = 1;
    sa.keep = keep;
    sa.keep_frac = keep_frac;

    ca::RansacArgs ra;
    ra.fd = pl->fd;
    ra.cand = sa.cand;
    ra.rec = pl->rec;
    ra.dbg = attempts_out;
    ra.seed = p.seed;
    ra.t_ri = p.t_ri;
    ra.r_min = p.r_min;
    ra.r_max = p.r_max;
    ra.d_max = p.d_max;
    ra.t_ps = (float)p.t_ps;
    ra.t_px = p.scorer != CA_SCORER_HANDCRAFTED ? 0 : p.t_px;  // Table A1: t_px is handcrafted only
    ra.P = pl->P;
    ra.attempts = p.ransac_attempts;
    ra.refine = p.refine_iters;
    ra.sampler = p.sampler;
    ra.groups = groups;
    ra.lanes = lanes;
    ra.frame0 = 0;
    ra.groups_done = pl->ctl + ca::kCtlFrames + n;
    ra.keep = keep;
    ra.keep_frac = keep_frac;

    ca::SelectArgs se;
    se.rec = pl->rec;
    se.out = out;
    se.threshold = p.t_cs * 16777216.0 * (double)pl->P;
    se.P = pl->P;
    se.groups = groups;
    se.n_frames = n;

    hipEvent_t *ev = nullptr;
    if (timed && ctx->prof_used < ctx->prof_capacity)
        ev = &ctx->prof_events[4 * (size_t)ctx->prof_used++];
    if (fused_path) {
        ca::FusedArgs fa;
        fa.s = sa;
        fa.r = ra;
        fa.se = se;
        fa.ctl = pl->ctl;
        fa.nq = ctx->queues > 0 ? (int32_t)ctx->queues : (n >= 16 ? ca::kMaxQueues : 1);
        fa.lag = (int32_t)ctx->lag;
        fa.spin_limit = (uint32_t)ctx->spin_limit;
        int grid = ctx->grid > 0 ? (int)ctx->grid : pl->fused_grid;
        grid = (grid + fa.nq - 1) / fa.nq * fa.nq;  // equal workgroups per queue
        // the whole call is one kernel: it is timed as the strip-scoring slot
        if (ca::launch_fused(fa, grid, pl->fused_lds, s, ev ? ev[0] : nullptr, ev ? ev[1] : nullptr)
                != hipSuccess
            || (ev && (hipEventRecord(ev[2], s) != hipSuccess || hipEventRecord(ev[3], s) != hipSuccess)))
            return CA_E_DEVICE;
        return CA_OK;
    }
    // strips then RANSAC for frames [f0, f1) on stream st
    const int S = p.n_hstrips + p.n_vstrips;
    const bool learned = p.scorer == CA_SCORER_LEARNED;
    const bool learned2d = p.scorer == CA_SCORER_LEARNED_2D;
    // tev (timed calls): the strip kernel between tev[0] and tev[1], RANSAC
    // between tev[2] and tev[3], each pair taken by the dispatch itself (the
    // per-shape strip launches of a mixed batch between two marker events)
    auto launch_range = [&](int32_t f0, int32_t f1, hipStream_t st, hipEvent_t *tev) {
        hipEvent_t s0 = tev ? tev[0] : nullptr, s1 = tev ? tev[1] : nullptr;
        hipEvent_t r0 = tev ? tev[2] : nullptr, r1 = tev ? tev[3] : nullptr;
        ca::StripArgs a2 = sa;
        a2.frame0 = f0;
        a2.n_items = (f1 - f0) * S;
        a2.per_xcd = (a2.n_items + 7) / 8;
        ca::RansacArgs r2 = ra;
        r2.frame0 = f0;
        bool ok;
        if (learned2d) {
            ca::Cnn2dStripArgs c;
            c.frames = frames;
            c.fd = pl->fd;
            c.strips = pl->strips;
            c.model = ctx->model2d;
            c.cand = sa.cand;
            c.n_h = p.n_hstrips;
            c.n_v = p.n_vstrips;
            c.n_items = a2.n_items;
            c.per_xcd = a2.per_xcd;
            c.frame0 = f0;
            ok = ca::launch_cnn2d_strips(c, st, s0, s1) == hipSuccess;
        } else if (learned) {
            ca::CnnStripArgs c;
            c.frames = frames;
            c.fd = pl->fd;
            c.strips = pl->strips;
            c.model = ctx->model;
            c.cand = sa.cand;
            c.n_h = p.n_hstrips;
            c.n_v = p.n_vstrips;
            c.n_items = a2.n_items;
            c.per_xcd = a2.per_xcd;
            c.frame0 = f0;
            if (ctx->cnn_groups_per_xcd == 0)
                ctx->cnn_groups_per_xcd =
                    std::max(1, (ctx->n_cu > 0 ? ctx->n_cu : 256) / 8 * ca::cnn_strips_blocks_per_cu());
            ok = ca::launch_cnn_strips(c, std::min(c.per_xcd, ctx->cnn_groups_per_xcd), st, s0, s1)
                 == hipSuccess;
        } else if (f0 == 0 && f1 == n && !pl->dynamic
                   && (pl->classes.size() > 1
                       || strips_per_group(ctx, pl->classes[0].W, pl->classes[0].H, p) != 1)) {
            // the whole batch: one launch per frame shape, each with its tile
            ok = !s0 || hipEventRecord(s0, st) == hipSuccess;
            for (const Plan::ShapeClass &c : pl->classes)
                ok = ok
                     && launch_class_strips(sa, pl, c, strips_per_group(ctx, c.W, c.H, p), S, st)
                            == hipSuccess;
            ok = ok && (!s1 || hipEventRecord(s1, st) == hipSuccess);
        } else {
            ok = ca::launch_strips(a2, pl->lds, st, s0, s1) == hipSuccess;
        }
        return ok && ca::launch_ransac(r2, se, f1 - f0, st, r0, r1) == hipSuccess;
    };
    const int64_t want = ctx->pipeline > 0 ? ctx->pipeline
                         : (ctx->schedule == CA_SCHEDULE_AUTO ? pl->tuned_pipeline : 1);
    const int32_t nsub = want > 1 ? (int32_t)std::min<int64_t>(want, n) : 1;
    if (nsub == 1) {
        return launch_range(0, n, s, ev) ? CA_OK : CA_E_DEVICE;
    }
    // sub-batches alternate over two side streams, forked from and joined
    // back into the caller's stream: one sub-batch's RANSAC (ALU bound)
    // overlaps the next one's strip loads (HBM bound); the whole call is
    // timed in slot 0
    const int used = nsub < 2 ? nsub : 2;
    if ((ev && hipEventRecord(ev[0], s) != hipSuccess) || hipEventRecord(ctx->fork, s) != hipSuccess)
        return CA_E_DEVICE;
    for (int k = 0; k < used; ++k)
        if (hipStreamWaitEvent(ctx->side[k], ctx->fork, 0) != hipSuccess)
            return CA_E_DEVICE;
    for (int32_t j = 0; j < nsub; ++j) {
        const int32_t f0 = (int32_t)((int64_t)j * n / nsub);
        const int32_t f1 = (int32_t)((int64_t)(j + 1) * n / nsub);
        if (f1 > f0 && !launch_range(f0, f1, ctx->side[j & 1], nullptr))
            return CA_E_DEVICE;
    }
    for (int k = 0; k < used; ++k)
        if (hipEventRecord(ctx->join[k], ctx->side[k]) != hipSuccess
            || hipStreamWaitEvent(s, ctx->join[k], 0) != hipSuccess)
            return CA_E_DEVICE;
    if (ev && (hipEventRecord(ev[1], s) != hipSuccess || hipEventRecord(ev[2], s) != hipSuccess
               || hipEventRecord(ev[3], s) != hipSuccess))
        return CA_E_DEVICE;
    return CA_OK;
}

// One call: the learned scorer's pipeline, then, with a fallback fraction,
// the handcrafted pipeline into the plan's second result array and a
// per-frame choice between the two.  The handcrafted kernels skip the frames
// whose learned result stands (the same rule as the choice), so that pass
// costs in proportion to the frames that fall back.
int enqueue(ca_ctx *ctx, Plan *pl, const uint8_t *frames, int32_t n, const ca_params &p,
            ca_point *points_out, ca_attempt *attempts_out, ca_result *out, hipStream_t s,
            bool timed)
{
    int rc = enqueue_one(ctx, pl, frames, n, p, points_out, attempts_out, out, s, timed);
    if (rc != CA_OK || p.scorer == CA_SCORER_HANDCRAFTED || !(p.fallback_inlier_frac > 0.0f))
        return rc;
    ca_params h = p;
    h.scorer = CA_SCORER_HANDCRAFTED;
    h.fallback_inlier_frac = 0.0f;
    rc = enqueue_one(ctx, pl, frames, n, h, nullptr, nullptr, pl->res2, s, false, out,
                     p.fallback_inlier_frac);
    if (rc != CA_OK)
        return rc;
    return ca::launch_fallback(out, pl->res2, n, p.fallback_inlier_frac, s) == hipSuccess
               ? CA_OK
               : CA_E_DEVICE;
}

int run(ca_ctx *ctx, const uint8_t *frames, const ca_frame_desc *dims, int32_t n,
        const ca_params *params, ca_point *points_out, ca_attempt *attempts_out, ca_result *out,
        void *stream)
{
    if (!ctx || n < 0)
        return CA_E_INVAL;
    if (n == 0)
        return CA_OK;
    if (!frames || !dims || !out)
        return CA_E_INVAL;
    ca_params p;
    if (params)
        p = *params;
    else
        ca_default_params(&p);
    int rc = validate(dims, n, p);
    if (rc != CA_OK)
        return rc;
    if ((p.scorer == CA_SCORER_LEARNED && !ctx->model)
        || (p.scorer == CA_SCORER_LEARNED_2D && !ctx->model2d))
        return CA_E_INVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return CA_E_DEVICE;
    Plan *pl = nullptr;
    rc = get_plan(ctx, dims, n, p, &pl);
    if (rc != CA_OK)
        return rc;
    return enqueue(ctx, pl, frames, n, p, points_out, attempts_out, out,
                   static_cast<hipStream_t>(stream), true);
}

}  // namespace cahost

struct ca_graph {
    ca_ctx *ctx = nullptr;
    Plan *plan = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

void ca_default_params(ca_params *p)
{
    if (!p)
        return;
    std::memset(p, 0, sizeof(*p));
    // Appendix A, Table A1; three refinements (Section 2.2.5)
    p->n_hstrips = 16;
    p->n_vstrips = 16;
    p->alpha = 8.0;
    p->t_g = 20.0;
    p->t_theta_deg = 30.0;
    p->t_iota = 25.0;
    p->t_ps = 0.03;
    p->t_cs = 0.06;
    p->t_px = 3;
    p->refine_iters = 3;
    p->t_ri = 3.0;
    p->r_min = 0.1;
    p->r_max = 0.8;
    p->d_max = 0.2;
    p->ransac_attempts = 256;
    p->sampler = 0;
    p->seed = 0;
    p->scorer = CA_SCORER_HANDCRAFTED;
}

int ca_create(ca_ctx **out, int device, size_t budget)
{
    if (!out)
        return CA_E_INVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) {
        (void)hipGetLastError();
        return CA_E_DEVICE;
    }
    if (device < 0 || device >= count)
        return CA_E_INVAL;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device)
        != hipSuccess)
        return CA_E_DEVICE;
    ca_ctx *c = new (std::nothrow) ca_ctx();
    if (!c)
        return CA_E_NOMEM;
    int n_cu = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess
        || n_cu < 1) {
        delete c;
        return CA_E_DEVICE;
    }
    c->device = device;
    c->budget = budget ? budget : ((size_t)1 << 30);
    c->max_lds = (size_t)lds;
    c->n_cu = n_cu;
    {
        DeviceGuard guard(device);
        bool ok = guard.ok;
        for (int k = 0; k < 2 && ok; ++k)
            ok = hipStreamCreateWithFlags(&c->side[k], hipStreamNonBlocking) == hipSuccess
                 && hipEventCreateWithFlags(&c->join[k], hipEventDisableTiming) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) == hipSuccess;
        // the device address of the no-allocation entry point's scratch on
        // this device (a failure only disables that entry point)
        (void)scratch_setup(device);
        if (!ok) {
            (void)hipGetLastError();
            ca_destroy(c);
            return CA_E_DEVICE;
        }
    }
    *out = c;
    return CA_OK;
}

static void release_profile(ca_ctx *ctx)
{
    for (hipEvent_t e : ctx->prof_events)
        (void)hipEventDestroy(e);
    ctx->prof_events.clear();
    ctx->prof_capacity = 0;
    ctx->prof_used = 0;
}

void ca_destroy(ca_ctx *ctx)
{
    if (!ctx)
        return;
    {
        DeviceGuard guard(ctx->device);
        (void)hipDeviceSynchronize();
        release_profile(ctx);
        for (Plan *p : ctx->plans)
            free_plan(ctx, p);
        for (int k = 0; k < 2; ++k) {
            if (ctx->side[k])
                (void)hipStreamDestroy(ctx->side[k]);
            if (ctx->join[k])
                (void)hipEventDestroy(ctx->join[k]);
        }
        if (ctx->fork)
            (void)hipEventDestroy(ctx->fork);
        if (ctx->model)
            (void)hipFree(ctx->model);
        if (ctx->train)
            (void)hipFree(ctx->train);
        if (ctx->partial)
            (void)hipFree(ctx->partial);
        (void)hipFree(ctx->model2d);
        (void)hipFree(ctx->train2d);
        (void)hipFree(ctx->partial2d);
    }
    delete ctx;
}

int ca_profile_begin(ca_ctx *ctx, int32_t max_calls)
{
    if (!ctx || max_calls < 1)
        return CA_E_INVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return CA_E_DEVICE;
    (void)hipDeviceSynchronize();
    release_profile(ctx);
    try {
        ctx->prof_events.assign(4 * (size_t)max_calls, nullptr);
    } catch (...) {
        return CA_E_NOMEM;
    }
    for (hipEvent_t &e : ctx->prof_events)
        if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
            release_profile(ctx);
            return CA_E_DEVICE;
        }
    ctx->prof_capacity = max_calls;
    ctx->prof_used = 0;
    return CA_OK;
}

int ca_profile_end(ca_ctx *ctx, ca_kernel_times *out)
{
    if (!ctx || !out)
        return CA_E_INVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return CA_E_DEVICE;
    std::memset(out, 0, sizeof(*out));
    int rc = CA_OK;
    for (int32_t c = 0; c < ctx->prof_used; ++c) {
        hipEvent_t *ev = &ctx->prof_events[4 * (size_t)c];
        if (hipEventSynchronize(ev[3]) != hipSuccess) {
            rc = CA_E_DEVICE;
            break;
        }
        // slots: strip kernel(s) ev0 -> ev1, RANSAC ev2 -> ev3, and the gap
        // between them ev1 -> ev2
        const int from[3] = {0, 2, 1}, to[3] = {1, 3, 2};
        for (int k = 0; k < 3; ++k) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, ev[from[k]], ev[to[k]]) != hipSuccess) {
                rc = CA_E_DEVICE;
                break;
            }
            out->total_ms[k] += ms;
            out->launches[k] += 1;
        }
    }
    release_profile(ctx);
    return rc;
}

int ca_estimate_area(ca_ctx *ctx, const uint8_t *frames, const ca_frame_desc *dims, int32_t n,
                     const ca_params *params, ca_result *out, void *stream)
{
    try {
        return run(ctx, frames, dims, n, params, nullptr, nullptr, out, stream);
    } catch (...) {
        return CA_E_NOMEM;
    }
}

int ca_debug_candidates(ca_ctx *ctx, const uint8_t *frames, const ca_frame_desc *dims, int32_t n,
                        const ca_params *params, ca_point *points, ca_result *out, void *stream)
{
    if (n > 0 && !points)
        return CA_E_INVAL;
    try {
        return run(ctx, frames, dims, n, params, points, nullptr, out, stream);
    } catch (...) {
        return CA_E_NOMEM;
    }
}

int ca_debug_attempts(ca_ctx *ctx, const uint8_t *frames, const ca_frame_desc *dims, int32_t n,
                      const ca_params *params, ca_attempt *attempts, ca_result *out, void *stream)
{
    if (n > 0 && !attempts)
        return CA_E_INVAL;
    try {
        return run(ctx, frames, dims, n, params, nullptr, attempts, out, stream);
    } catch (...) {
        return CA_E_NOMEM;
    }
}

int ca_graph_create(ca_ctx *ctx, const uint8_t *frames, const ca_frame_desc *dims, int32_t n,
                    const ca_params *params, ca_result *out, int32_t calls, ca_graph **graph)
{
    if (!graph)
        return CA_E_INVAL;
    *graph = nullptr;
    if (!ctx || n < 1 || !frames || !dims || !out || calls < 1 || calls > 4096)
        return CA_E_INVAL;
    ca_params p;
    if (params)
        p = *params;
    else
        ca_default_params(&p);
    if ((p.scorer == CA_SCORER_LEARNED && !ctx->model)
        || (p.scorer == CA_SCORER_LEARNED_2D && !ctx->model2d))
        return CA_E_INVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return CA_E_DEVICE;
    Plan *pl = nullptr;
    int rc = get_plan(ctx, dims, n, p, &pl);
    if (rc != CA_OK)
        return rc;
    ca_graph *g = new (std::nothrow) ca_graph();
    if (!g)
        return CA_E_NOMEM;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        delete g;
        return CA_E_DEVICE;
    }
    rc = CA_OK;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        rc = CA_E_DEVICE;
    } else {
        for (int32_t i = 0; i < calls && rc == CA_OK; ++i)
            rc = enqueue(ctx, pl, frames, n, p, nullptr, nullptr, out, s, false);
        hipGraph_t gr = nullptr;
        if (hipStreamEndCapture(s, &gr) != hipSuccess || !gr) {
            rc = CA_E_DEVICE;
        } else {
            g->graph = gr;
            if (rc == CA_OK && hipGraphInstantiate(&g->exec, gr, nullptr, nullptr, 0) != hipSuccess)
                rc = CA_E_DEVICE;
        }
    }
    (void)hipStreamDestroy(s);
    if (rc != CA_OK) {
        (void)hipGetLastError();
        if (g->exec)
            (void)hipGraphExecDestroy(g->exec);
        if (g->graph)
            (void)hipGraphDestroy(g->graph);
        delete g;
        return rc;
    }
    g->ctx = ctx;
    g->plan = pl;
    ++pl->pins;
    *graph = g;
    return CA_OK;
}

int ca_graph_launch(ca_graph *g, void *stream)
{
    if (!g)
        return CA_E_INVAL;
    DeviceGuard guard(g->ctx->device);
    if (!guard.ok)
        return CA_E_DEVICE;
    return hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)) == hipSuccess ? CA_OK
                                                                                    : CA_E_DEVICE;
}

void ca_graph_destroy(ca_graph *g)
{
    if (!g)
        return;
    {
        DeviceGuard guard(g->ctx->device);
        (void)hipDeviceSynchronize();
        (void)hipGraphExecDestroy(g->exec);
        (void)hipGraphDestroy(g->graph);
    }
    --g->plan->pins;
    delete g;
}

namespace {

constexpr size_t kTrainFloats = 2 * (size_t)CA_CNN_PARAMS;

bool finite_all(const float *v, int32_t n)
{
    for (int32_t i = 0; i < n; ++i)
        if (!std::isfinite(v[i]))
            return false;
    return true;
}

}  // namespace

int ca_set_model(ca_ctx *ctx, const float *prm, int32_t n)
{
    if (!ctx || !prm || n != CA_CNN_PARAMS || !finite_all(prm, n))
        return CA_E_INVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return CA_E_DEVICE;
    if (!ctx->model) {
        if (hipMalloc(&ctx->model, ca::kCnnModelBytes) != hipSuccess) {
            (void)hipGetLastError();
            ctx->model = nullptr;
            return CA_E_NOMEM;
        }
    }
    if (!ctx->train) {
        if (hipMalloc(&ctx->train, kTrainFloats * sizeof(float)) != hipSuccess) {
            (void)hipGetLastError();
            ctx->train = nullptr;
            return CA_E_NOMEM;
        }
    }
    if (hipDeviceSynchronize() != hipSuccess
        || hipMemcpy(ctx->train, prm, (size_t)n * sizeof(float), hipMemcpyHostToDevice)
               != hipSuccess
        || hipMemset(ctx->train + CA_CNN_PARAMS, 0, (size_t)n * sizeof(float)) != hipSuccess
        || ca::launch_cnn_pack(ctx->train, ctx->model, nullptr) != hipSuccess
        || hipDeviceSynchronize() != hipSuccess)
        return CA_E_DEVICE;
    return CA_OK;
}

int ca_get_model(ca_ctx *ctx, float *prm, float *mom, int32_t n)
{
    if (!ctx || !prm || n != CA_CNN_PARAMS || !ctx->train)
        return CA_E_INVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return CA_E_DEVICE;
    if (hipDeviceSynchronize() != hipSuccess
        || hipMemcpy(prm, ctx->train, (size_t)n * sizeof(float), hipMemcpyDeviceToHost)
               != hipSuccess)
        return CA_E_DEVICE;
    if (mom && hipMemcpy(mom, ctx->train + CA_CNN_PARAMS, (size_t)n * sizeof(float),
                         hipMemcpyDeviceToHost) != hipSuccess)
        return CA_E_DEVICE;
    return CA_OK;
}

int ca_set_momentum(ca_ctx *ctx, const float *mom, int32_t n)
{
    if (!ctx || !mom || n != CA_CNN_PARAMS || !ctx->train || !finite_all(mom, n))
        return CA_E_INVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return CA_E_DEVICE;
    if (hipDeviceSynchronize() != hipSuccess
        || hipMemcpy(ctx->train + CA_CNN_PARAMS, mom, (size_t)n * sizeof(float),
                     hipMemcpyHostToDevice) != hipSuccess)
        return CA_E_DEVICE;
    return CA_OK;
}

int ca_cnn_gradients(ca_ctx *ctx, const uint8_t *win, const int32_t *range, const float *target,
                     const float *weight, int32_t n, float scale, float *grad, float *loss,
                     void *stream)
{
    if (!ctx || n < 0 || !grad || !loss || !std::isfinite(scale)
        || (n > 0 && (!win || !range || !target || !weight)))
        return CA_E_INVAL;
    if (!ctx->model)
        return CA_E_INVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return CA_E_DEVICE;
    if (!ctx->partial) {
        // two resident workgroups per compute unit (LDS and registers allow two)
        const int grid = 2 * (ctx->n_cu > 0 ? ctx->n_cu : 256);
        if (hipMalloc(&ctx->partial, (size_t)grid * ca::kCnnGradStride * sizeof(float))
            != hipSuccess) {
            (void)hipGetLastError();
            ctx->partial = nullptr;
            return CA_E_NOMEM;
        }
        ctx->grad_grid = grid;
    }
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const int grid = n < ctx->grad_grid ? (n > 0 ? n : 1) : ctx->grad_grid;
    ca::CnnTrainArgs a;
    a.model = ctx->model;
    a.win = win;
    a.range = range;
    a.target = target;
    a.weight = weight;
    a.partial = ctx->partial;
    a.scale = scale;
    a.n = n;
    if (ca::launch_cnn_grad(a, grid, st) != hipSuccess
        || ca::launch_cnn_reduce(ctx->partial, grid, grad, loss, st) != hipSuccess)
        return CA_E_DEVICE;
    return CA_OK;
}

int ca_cnn_sgd_step(ca_ctx *ctx, const float *grad, float lr, float mu, void *stream)
{
    if (!ctx || !grad || !std::isfinite(lr) || !std::isfinite(mu))
        return CA_E_INVAL;
    if (!ctx->train)
        return CA_E_INVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return CA_E_DEVICE;
    return ca::launch_cnn_update(ctx->train, ctx->train + CA_CNN_PARAMS, grad, lr, mu, ctx->model,
                                 static_cast<hipStream_t>(stream)) == hipSuccess
               ? CA_OK
               : CA_E_DEVICE;
}

int ca_cnn_window_logits(ca_ctx *ctx, const uint8_t *win, const int32_t *range, int32_t n,
                         float *z, void *stream)
{
    if (!ctx || n < 0 || (n > 0 && (!win || !range || !z)))
        return CA_E_INVAL;
    if (!ctx->model)
        return CA_E_INVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return CA_E_DEVICE;
    return ca::launch_cnn_windows(ctx->model, win, range, z, n, static_cast<hipStream_t>(stream))
                   == hipSuccess
               ? CA_OK
               : CA_E_DEVICE;
}

// ---------------------------------------- the paper's 2-D scorer (2.2.4) --

int ca_set_model_2d(ca_ctx *ctx, const float *prm, int32_t n)
{
    if (!ctx || !prm || n != CA_CNN2D_PARAMS || !finite_all(prm, n))
        return CA_E_INVAL;
    for (int c = 0; c < 3; ++c)
        if (!(prm[3 + c] > 0.0f))
            return CA_E_INVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return CA_E_DEVICE;
    if (!ctx->model2d && hipMalloc(&ctx->model2d, ca::kC2ModelBytes) != hipSuccess) {
        (void)hipGetLastError();
        ctx->model2d = nullptr;
        return CA_E_NOMEM;
    }
    if (!ctx->train2d && hipMalloc(&ctx->train2d, 2 * sizeof(float) * ca::kC2Params) != hipSuccess) {
        (void)hipGetLastError();
        ctx->train2d = nullptr;
        return CA_E_NOMEM;
    }
    if (hipDeviceSynchronize() != hipSuccess
        || hipMemcpy(ctx->train2d, prm, (size_t)n * sizeof(float), hipMemcpyHostToDevice)
               != hipSuccess
        || hipMemset(ctx->train2d + ca::kC2Params, 0, (size_t)n * sizeof(float)) != hipSuccess
        || ca::launch_cnn2d_pack(ctx->train2d, ctx->model2d, nullptr) != hipSuccess
        || hipDeviceSynchronize() != hipSuccess)
        return CA_E_DEVICE;
    return CA_OK;
}

int ca_get_model_2d(ca_ctx *ctx, float *prm, float *mom, int32_t n)
{
    if (!ctx || !prm || n != CA_CNN2D_PARAMS || !ctx->train2d)
        return CA_E_INVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return CA_E_DEVICE;
    if (hipDeviceSynchronize() != hipSuccess
        || hipMemcpy(prm, ctx->train2d, (size_t)n * sizeof(float), hipMemcpyDeviceToHost)
               != hipSuccess)
        return CA_E_DEVICE;
    if (mom && hipMemcpy(mom, ctx->train2d + ca::kC2Params, (size_t)n * sizeof(float),
                         hipMemcpyDeviceToHost) != hipSuccess)
        return CA_E_DEVICE;
    return CA_OK;
}

int ca_set_momentum_2d(ca_ctx *ctx, const float *mom, int32_t n)
{
    if (!ctx || !mom || n != CA_CNN2D_PARAMS || !ctx->train2d || !finite_all(mom, n))
        return CA_E_INVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return CA_E_DEVICE;
    if (hipDeviceSynchronize() != hipSuccess
        || hipMemcpy(ctx->train2d + ca::kC2Params, mom, (size_t)n * sizeof(float),
                     hipMemcpyHostToDevice) != hipSuccess)
        return CA_E_DEVICE;
    return CA_OK;
}

int ca_cnn2d_window_logits(ca_ctx *ctx, const uint8_t *win, const int32_t *geom,
                           const int32_t *range, int32_t n, float *z, void *stream)
{
    if (!ctx || n < 0 || (n > 0 && (!win || !geom || !range || !z)))
        return CA_E_INVAL;
    if (!ctx->model2d)
        return CA_E_INVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return CA_E_DEVICE;
    return ca::launch_cnn2d_windows(ctx->model2d, win, geom, range, z, n,
                                    static_cast<hipStream_t>(stream)) == hipSuccess
               ? CA_OK
               : CA_E_DEVICE;
}

int ca_cnn2d_gradients(ca_ctx *ctx, const uint8_t *win, const int32_t *geom, const int32_t *range,
                       const float *target, const float *weight, int32_t n, float scale,
                       float *grad, float *loss, void *stream)
{
    if (!ctx || n < 0 || !grad || !loss || !std::isfinite(scale)
        || (n > 0 && (!win || !geom || !range || !target || !weight)))
        return CA_E_INVAL;
    if (!ctx->model2d)
        return CA_E_INVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return CA_E_DEVICE;
    if (!ctx->partial2d) {
        const int grid = ca::cnn2d_grad_blocks_per_cu() * (ctx->n_cu > 0 ? ctx->n_cu : 256);
        if (hipMalloc(&ctx->partial2d, (size_t)grid * ca::kC2GradStride * sizeof(float))
            != hipSuccess) {
            (void)hipGetLastError();
            ctx->partial2d = nullptr;
            return CA_E_NOMEM;
        }
        ctx->grad2d_grid = grid;
    }
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const int grid = n < ctx->grad2d_grid ? (n > 0 ? n : 1) : ctx->grad2d_grid;
    ca::Cnn2dTrainArgs a;
    a.model = ctx->model2d;
    a.win = win;
    a.geom = geom;
    a.range = range;
    a.target = target;
    a.weight = weight;
    a.partial = ctx->partial2d;
    a.scale = scale;
    a.n = n;
    if (ca::launch_cnn2d_grad(a, grid, st) != hipSuccess
        || ca::launch_cnn2d_reduce(ctx->partial2d, grid, grad, loss, st) != hipSuccess)
        return CA_E_DEVICE;
    return CA_OK;
}

int ca_cnn2d_sgd_step(ca_ctx *ctx, const float *grad, float lr, float mu, void *stream)
{
    if (!ctx || !grad || !std::isfinite(lr) || !std::isfinite(mu))
        return CA_E_INVAL;
    if (!ctx->train2d)
        return CA_E_INVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return CA_E_DEVICE;
    return ca::launch_cnn2d_update(ctx->train2d, ctx->train2d + ca::kC2Params, grad, lr, mu,
                                   ctx->model2d, static_cast<hipStream_t>(stream)) == hipSuccess
               ? CA_OK
               : CA_E_DEVICE;
}

int ca_selftest_mfma(ca_ctx *ctx, float *out, void *stream)
{
    if (!ctx || !out)
        return CA_E_INVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return CA_E_DEVICE;
    return ca::launch_mfma_probe(out, static_cast<hipStream_t>(stream)) == hipSuccess ? CA_OK
                                                                                       : CA_E_DEVICE;
}

int ca_autotune(ca_ctx *ctx, const uint8_t *frames, const ca_frame_desc *dims, int32_t n,
                const ca_params *params, int32_t reps, void *stream, int32_t *schedule_out)
{
    if (!ctx || n < 0 || reps < 1 || reps > 1000)
        return CA_E_INVAL;
    if (n == 0)
        return CA_OK;
    if (!frames || !dims)
        return CA_E_INVAL;
    ca_params p;
    if (params)
        p = *params;
    else
        ca_default_params(&p);
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return CA_E_DEVICE;
    Plan *pl = nullptr;
    int rc = get_plan(ctx, dims, n, p, &pl);
    if (rc != CA_OK)
        return rc;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    ca::StripArgs sa;
    sa.frames = frames;
    sa.fd = pl->fd;
    sa.strips = pl->strips;
    sa.lut = pl->lut;
    sa.cand = pl->cand;
    sa.sg_len = pl->sg_len;
    sa.n_h = p.n_hstrips;
    sa.n_v = p.n_vstrips;
    sa.line_pitch = pl->line_pitch;
    sa.aligned = (pl->rows_aligned && (reinterpret_cast<uintptr_t>(frames) % 16) == 0) ? 1 : 0;
    sa.frame0 = 0;
    sa.frame_list = nullptr;
    sa.items_per_group = 1;
    sa.n_items = 0;
    sa.per_xcd = 0;
    const int32_t S = p.n_hstrips + p.n_vstrips;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0)
            (void)hipEventDestroy(e0);
        return CA_E_DEVICE;
    }
    rc = CA_OK;
    for (const Plan::ShapeClass &c : pl->classes) {
        int32_t best_t = 1;
        float best_ms = 0.0f;
        for (int32_t T : {1, 2, 4, 8}) {
            bool ok = launch_class_strips(sa, pl, c, T, S, st) == hipSuccess   // warm-up
                      && hipEventRecord(e0, st) == hipSuccess;
            for (int32_t r = 0; ok && r < reps; ++r)
                ok = launch_class_strips(sa, pl, c, T, S, st) == hipSuccess;
            float ms = 0.0f;
            ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess
                 && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
            if (!ok) {
                rc = CA_E_DEVICE;
                break;
            }
            if (T == 1 || ms < best_ms) {
                best_ms = ms;
                best_t = T;
            }
        }
        if (rc != CA_OK)
            break;
        ctx->tuned[{c.W, c.H, p.n_hstrips, p.n_vstrips}] = best_t;
    }
    // whole calls of this batch: the split schedule (with the tiles just
    // chosen) in one call or cut into 2 or 4 pipelined sub-batches, against
    // the persistent one; the fastest serves CA_SCHEDULE_AUTO (with the
    // pipeline option at 0).  Each is timed eagerly and replayed from a
    // captured one-call graph, and counts by the slower of the two (the
    // side streams of the pipelined calls overlap differently in the two
    // forms), so the choice holds for eager callers and graph users alike.
    auto time_graph = [&](float *ms) {
        hipStream_t cs = nullptr;
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
            return false;
        hipGraph_t gr = nullptr;
        hipGraphExec_t ex = nullptr;
        bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            const bool enq =
                enqueue(ctx, pl, frames, n, p, nullptr, nullptr, pl->res2, cs, false) == CA_OK;
            ok = hipStreamEndCapture(cs, &gr) == hipSuccess && gr && enq
                 && hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0) == hipSuccess;
        }
        ok = ok && hipGraphLaunch(ex, st) == hipSuccess && hipEventRecord(e0, st) == hipSuccess;
        for (int32_t r = 0; ok && r < reps; ++r)
            ok = hipGraphLaunch(ex, st) == hipSuccess;
        ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess
             && hipEventElapsedTime(ms, e0, e1) == hipSuccess;
        if (ex)
            (void)hipGraphExecDestroy(ex);
        if (gr)
            (void)hipGraphDestroy(gr);
        (void)hipStreamDestroy(cs);
        return ok;
    };
    if (rc == CA_OK && p.scorer == CA_SCORER_HANDCRAFTED) {
        const int64_t saved_schedule = ctx->schedule, saved_pipeline = ctx->pipeline;
        struct Trial {
            int64_t schedule, pipeline;
        };
        const Trial trials[4] = {{CA_SCHEDULE_SPLIT, 1}, {CA_SCHEDULE_SPLIT, 2},
                                 {CA_SCHEDULE_SPLIT, 4}, {CA_SCHEDULE_FUSED, 1}};
        int best = 0;
        float best_ms = 0.0f;
        for (int k = 0; k < 4 && rc == CA_OK; ++k) {
            if (trials[k].pipeline > n)
                continue;
            ctx->schedule = trials[k].schedule;
            ctx->pipeline = trials[k].pipeline;
            bool ok = enqueue(ctx, pl, frames, n, p, nullptr, nullptr, pl->res2, st, false) == CA_OK
                      && hipEventRecord(e0, st) == hipSuccess;
            for (int32_t r = 0; ok && r < reps; ++r)
                ok = enqueue(ctx, pl, frames, n, p, nullptr, nullptr, pl->res2, st, false) == CA_OK;
            float ms = 0.0f, ms_graph = 0.0f;
            ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess
                 && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && time_graph(&ms_graph);
            ms = ms > ms_graph ? ms : ms_graph;
            if (!ok)
                rc = CA_E_DEVICE;
            else if (k == 0 || ms < best_ms) {
                best = k;
                best_ms = ms;
            }
        }
        ctx->schedule = saved_schedule;
        ctx->pipeline = saved_pipeline;
        if (rc == CA_OK) {
            pl->tuned_schedule = (int32_t)trials[best].schedule;
            pl->tuned_pipeline = (int32_t)trials[best].pipeline;
            ctx->last_schedule = pl->tuned_schedule;
            ctx->last_pipeline = pl->tuned_pipeline;
        }
    }
    if (rc == CA_OK && schedule_out)
        *schedule_out = pl->tuned_schedule;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int ca_get_last_autotune(ca_ctx *ctx, int32_t *schedule, int32_t *pipeline)
{
    if (!ctx || !schedule || !pipeline)
        return CA_E_INVAL;
    *schedule = ctx->last_schedule;
    *pipeline = ctx->last_pipeline;
    return CA_OK;
}

int ca_get_tuning(ca_ctx *ctx, int32_t W, int32_t H, int32_t n_h, int32_t n_v, int32_t *out)
{
    if (!ctx || !out)
        return CA_E_INVAL;
    const auto it = ctx->tuned.find({W, H, n_h, n_v});
    *out = it == ctx->tuned.end() ? 0 : it->second;
    return CA_OK;
}

int ca_set_option(ca_ctx *ctx, int32_t option, int64_t value)
{
    if (!ctx)
        return CA_E_INVAL;
    switch (option) {
    case CA_OPT_SCHEDULE:
        if (value != CA_SCHEDULE_SPLIT && value != CA_SCHEDULE_FUSED
            && value != CA_SCHEDULE_AUTO)
            return CA_E_INVAL;
        ctx->schedule = value;
        return CA_OK;
    case CA_OPT_LAG:
        if (value < 0 || value > (1 << 20))
            return CA_E_INVAL;
        ctx->lag = value;
        return CA_OK;
    case CA_OPT_QUEUES:
        if (value < 0 || value > ca::kMaxQueues)
            return CA_E_INVAL;
        ctx->queues = value;
        return CA_OK;
    case CA_OPT_GRID:
        if (value < 0 || value > (1 << 20))
            return CA_E_INVAL;
        ctx->grid = value;
        return CA_OK;
    case CA_OPT_SPIN_LIMIT:
        if (value < 1 || value > 0xFFFFFFFFll)
            return CA_E_INVAL;
        ctx->spin_limit = value;
        return CA_OK;
    case CA_OPT_PIPELINE:
        if (value < 0 || value > 1024)
            return CA_E_INVAL;
        ctx->pipeline = value;
        return CA_OK;
    case CA_OPT_STRIPS_PER_GROUP:
        if (value < 0 || value > 16)
            return CA_E_INVAL;
        ctx->strips_per_group = value;
        return CA_OK;
    case CA_OPT_RANSAC_LANES:
        if (value != 0 && value != 2 && value != 4 && value != 8 && value != 16)
            return CA_E_INVAL;
        ctx->ransac_lanes = value;
        return CA_OK;
    default:
        return CA_E_INVAL;
    }
}

int ca_get_option(ca_ctx *ctx, int32_t option, int64_t *value)
{
    if (!ctx || !value)
        return CA_E_INVAL;
    switch (option) {
    case CA_OPT_SCHEDULE:
        *value = ctx->schedule;
        return CA_OK;
    case CA_OPT_LAG:
        *value = ctx->lag;
        return CA_OK;
    case CA_OPT_QUEUES:
        *value = ctx->queues;
        return CA_OK;
    case CA_OPT_GRID:
        *value = ctx->grid;
        return CA_OK;
    case CA_OPT_SPIN_LIMIT:
        *value = ctx->spin_limit;
        return CA_OK;
    case CA_OPT_PIPELINE:
        *value = ctx->pipeline;
        return CA_OK;
    case CA_OPT_STRIPS_PER_GROUP:
        *value = ctx->strips_per_group;
        return CA_OK;
    case CA_OPT_RANSAC_LANES:
        *value = ctx->ransac_lanes;
        return CA_OK;
    default:
        return CA_E_INVAL;
    }
}

int ca_device_status(ca_ctx *ctx)
{
    if (!ctx)
        return CA_E_INVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok || hipDeviceSynchronize() != hipSuccess)
        return CA_E_DEVICE;
    int rc = CA_OK;
    for (Plan *pl : ctx->plans) {
        uint32_t err = 0;
        if (hipMemcpy(&err, pl->ctl + ca::kCtlError, sizeof(err), hipMemcpyDeviceToHost)
            != hipSuccess)
            return CA_E_DEVICE;
        if (err) {
            rc = CA_E_DEVICE;
            const uint32_t zero = 0;
            if (hipMemcpy(pl->ctl + ca::kCtlError, &zero, sizeof(zero), hipMemcpyHostToDevice)
                != hipSuccess)
                return CA_E_DEVICE;
        }
    }
    return rc;
}

int ca_check_args(const ca_frame_desc *dims, int32_t n, const ca_params *params)
{
    if (n < 0 || (n > 0 && !dims))
        return CA_E_INVAL;
    ca_params p;
    if (params)
        p = *params;
    else
        ca_default_params(&p);
    return validate(dims, n, p);
}

int ca_strip_positions(int32_t extent, int32_t n, double alpha, int32_t *pos)
{
    if (!pos && n > 0)
        return CA_E_INVAL;
    return strip_positions(extent, n, alpha, pos);
}

int ca_score_tables(const ca_params *p, float *sg, int32_t *sg_len, float *st, float *si)
{
    if (!sg || !sg_len || !st || !si)
        return CA_E_INVAL;
    ca_params q;
    if (p)
        q = *p;
    else
        ca_default_params(&q);
    if (!(q.t_g > 0) || !(q.t_theta_deg > 0) || !(q.t_iota > 0))
        return CA_E_INVAL;
    return score_tables(q, sg, sg_len, st, si);
}

const char *ca_error_string(int code)
{
    switch (code) {
    case CA_OK:
        return "ok";
    case CA_E_INVAL:
        return "invalid argument";
    case CA_E_UNSUPPORTED:
        return "unsupported frame layout or parameter combination";
    case CA_E_NOMEM:
        return "workspace budget exceeded or out of memory";
    case CA_E_DEVICE:
        return "HIP runtime error";
    case CA_E_SCRATCH:
        return "batch exceeds the fixed scratch of ca_estimate_area_noalloc (frames, frame "
               "shapes or bytes)";
    default:
        return "unknown error";
    }
}

const char *ca_version(void) { return "contentarea-gfx950 0.1.0"; }

}  // extern "C"
