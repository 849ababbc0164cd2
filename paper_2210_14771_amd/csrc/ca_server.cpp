// Serving loop: continuous batching of many video streams on one GPU.
//
// Host side: per-stream FIFOs of submitted frames, admission of streams by
// the HBM budget of their frame rings (first fit over one device arena),
// copies into ring slots, and batches launched whenever fewer than
// max_inflight are on the GPU.  Everything runs on one HIP stream of the
// server, in order: a frame's copy precedes the batch that reads it, and no
// work waits on another stream.  Device side: the
// estimator's kernels on each batch, then one kernel that folds the batch's
// results into the per-stream filtered circles, in sequence order.
//
// Every buffer is allocated, and every table computed, in ca_server_create
// (per in-flight slot: one block of max_batch frames' descriptors, strip
// tables, score tables, candidates and records, plus pinned staging) and in
// ca_server_open (the stream's strip positions).  ca_server_step only
// queries events and enqueues asynchronous work: event queries, copies into
// ring slots, one copy of the batch's descriptors and strip tables from
// pinned staging, the kernels, copies of the results into pinned memory, an
// event record.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <unordered_map>
#include <vector>

#include "ca_host.h"

namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

constexpr size_t kSlotAlign = 256;

// First-fit allocator over [0, size) with coalescing free list.
struct Arena {
    std::map<size_t, size_t> free_list;   // offset -> bytes
    size_t size = 0, used = 0;

    void reset(size_t bytes)
    {
        size = bytes;
        used = 0;
        free_list.clear();
        if (bytes)
            free_list[0] = bytes;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        for (auto it = free_list.begin(); it != free_list.end(); ++it)
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_list.erase(it);
                if (rest)
                    free_list[at] = rest;
                used += bytes;
                return true;
            }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        used -= bytes;
        auto it = free_list.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_list.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_list.erase(next);
        }
        if (it != free_list.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_list.erase(it);
            }
        }
    }
};

struct Pending {
    uint64_t seq;
    const uint8_t *src;
    int64_t stride;
    int32_t is_dev;     // 0 host, 1 device (copied), 2 device lent until served
    int64_t t_submit;
};

struct Stream {
    int32_t id = 0, W = 0, H = 0;
    bool admitted = false, closing = false;
    int32_t state = -1;                  // index of its device state
    size_t ring_off = 0, slot_bytes = 0; // ring in the arena
    std::vector<int32_t> free_slots;
    std::deque<Pending> queue;           // submitted, not yet copied
    int64_t outstanding = 0;             // copied or in flight, not yet served
    uint64_t last_seq = 0;
    bool any_seq = false;
    std::vector<int32_t> table;          // strip positions: n_h rows then n_v columns
};

struct Entry {                          // one frame from copy to retirement
    Stream *st;
    uint64_t seq;
    int32_t slot;                       // ring slot, or -1: read in place
    int64_t t_submit;
    const uint8_t *src = nullptr;       // a lent frame (slot -1) and its row stride
    int64_t stride = 0;
};

struct Batch {                          // one in-flight slot
    cahost::Plan plan;                  // buffers for max_batch frames, one device block
    ca_result *res_dev = nullptr;       // [max_batch]
    float4 *filt_dev = nullptr;         // [max_batch]
    int4 *runs_dev = nullptr;           // [max_batch]
    uint8_t *stage = nullptr;           // pinned: descriptors, then strip tables
    int4 *runs_host = nullptr;
    ca_result *res_host = nullptr;
    float4 *filt_host = nullptr;
    hipEvent_t done = nullptr;
    std::vector<Entry> entries;
    int64_t t_launch = 0;
    bool busy = false;
};

}  // namespace

struct ca_server {
    ca_ctx *ctx = nullptr;
    ca_server_config cfg{};
    hipStream_t compute = nullptr;
    uint8_t *arena_mem = nullptr;
    Arena arena;
    float4 *state_dev = nullptr;        // [max_streams]
    std::vector<int32_t> free_states;
    std::unordered_map<int32_t, Stream *> streams;
    std::vector<Stream *> order;        // admitted and waiting streams, by open time
    std::deque<Stream *> waiting;       // not yet admitted, first come first served
    std::deque<Entry> ready;            // copied, waiting for a batch
    std::vector<Batch> batches;
    std::deque<size_t> inflight;        // batch slots in launch order
    std::deque<ca_served> done;         // served, not yet returned
    cahost::PlanLayout layout;          // of every slot's block (max_batch frames)
    std::map<int32_t, int32_t> fused_grid;  // per LDS line pitch (fused schedule only)
    int64_t n_submitted = 0, n_served = 0, n_batches = 0;
};

namespace {

size_t frame_bytes(int32_t W, int32_t H)
{
    return ((size_t)3 * W * H + kSlotAlign - 1) / kSlotAlign * kSlotAlign;
}

void free_batch(Batch &b)
{
    if (b.done)
        (void)hipEventDestroy(b.done);
    (void)hipFree(b.plan.mem);
    (void)hipFree(b.res_dev);
    (void)hipFree(b.filt_dev);
    (void)hipFree(b.runs_dev);
    (void)hipHostFree(b.stage);
    (void)hipHostFree(b.runs_host);
    (void)hipHostFree(b.res_host);
    (void)hipHostFree(b.filt_host);
}

// The launch facts of a batch: its frames' descriptors and the strip tables
// of its distinct shapes into the slot's pinned staging (laid out as the
// head of the device block), the LDS line pitch of its longest extent.
// Returns the bytes to upload.
size_t stage_batch(ca_server *s, Batch &b, size_t n)
{
    const int32_t S = s->cfg.params.n_hstrips + s->cfg.params.n_vstrips;
    ca::FrameDev *fd = reinterpret_cast<ca::FrameDev *>(b.stage + s->layout.o_fd);
    int32_t *tables = reinterpret_cast<int32_t *>(b.stage + s->layout.o_strips);
    std::vector<const Stream *> shapes;  // one strip table per distinct shape
    int32_t longest = 0;
    bool aligned = true;
    for (size_t i = 0; i < n; ++i) {
        const Entry &e = b.entries[i];
        size_t k = 0;
        while (k < shapes.size() && !(shapes[k]->W == e.st->W && shapes[k]->H == e.st->H))
            ++k;
        if (k == shapes.size()) {
            shapes.push_back(e.st);
            std::memcpy(tables + k * (size_t)S, e.st->table.data(), sizeof(int32_t) * (size_t)S);
        }
        ca::FrameDev &d = fd[i];
        if (e.slot >= 0) {
            d.offset = (int64_t)(e.st->ring_off + (size_t)e.slot * e.st->slot_bytes);
        } else {
            // a lent frame: its address relative to the arena the kernels
            // take as the frames' base (flat device addresses)
            d.offset = (int64_t)(reinterpret_cast<uintptr_t>(e.src)
                                 - reinterpret_cast<uintptr_t>(s->arena_mem));
            aligned = aligned && (d.offset % 16) == 0;
        }
        d.W = e.st->W;
        d.H = e.st->H;
        d.rs = e.slot >= 0 ? 3 * e.st->W : (int32_t)e.stride;
        d.table = (int32_t)k * S;
        d.uid = ((uint64_t)(uint32_t)e.st->id << 32) | (e.seq & 0xFFFFFFFFull);
        longest = std::max(longest, std::max(e.st->W, e.st->H));
        aligned = aligned && (d.rs % 16) == 0;     // ring slots start 256-byte aligned
    }
    cahost::Plan &pl = b.plan;
    pl.n_frames = (int32_t)n;
    pl.line_pitch = (int32_t)cahost::align_up((size_t)longest, 16);
    pl.lds = ca::strip_lds_bytes(pl.sg_len, pl.line_pitch);
    pl.fused_lds = ca::fused_lds_bytes(pl.sg_len, pl.line_pitch);
    pl.rows_aligned = aligned;
    if (s->ctx->schedule == CA_SCHEDULE_FUSED) {
        auto it = s->fused_grid.find(pl.line_pitch);
        if (it == s->fused_grid.end())
            it = s->fused_grid.emplace(pl.line_pitch, cahost::fused_grid(s->ctx, pl.fused_lds))
                     .first;
        pl.fused_grid = it->second;
    }
    return s->layout.o_strips + sizeof(int32_t) * shapes.size() * (size_t)S;
}

bool try_admit(ca_server *s, Stream *st)
{
    if (s->free_states.empty())
        return false;
    const size_t bytes = st->slot_bytes * (size_t)s->cfg.ring_slots;
    size_t off = 0;
    if (!s->arena.alloc(bytes, &off))
        return false;
    st->ring_off = off;
    st->state = s->free_states.back();
    s->free_states.pop_back();
    st->free_slots.clear();
    for (int32_t k = s->cfg.ring_slots - 1; k >= 0; --k)
        st->free_slots.push_back(k);
    st->admitted = true;
    // a fresh filtered circle, ordered before any batch of this stream
    (void)hipMemsetAsync(s->state_dev + st->state, 0, sizeof(float4), s->compute);
    return true;
}

void release_stream(ca_server *s, Stream *st)
{
    if (st->admitted) {
        s->arena.release(st->ring_off, st->slot_bytes * (size_t)s->cfg.ring_slots);
        s->free_states.push_back(st->state);
    }
    s->streams.erase(st->id);
    s->order.erase(std::find(s->order.begin(), s->order.end(), st));
    delete st;
}

int retire(ca_server *s)
{
    while (!s->inflight.empty()) {
        Batch &b = s->batches[s->inflight.front()];
        const hipError_t q = hipEventQuery(b.done);
        if (q == hipErrorNotReady)
            return CA_OK;
        if (q != hipSuccess)
            return CA_E_DEVICE;
        const int64_t t = now_ns();
        for (size_t i = 0; i < b.entries.size(); ++i) {
            const Entry &e = b.entries[i];
            ca_served out;
            std::memset(&out, 0, sizeof(out));
            out.stream_id = e.st->id;
            out.seq = e.seq;
            out.result = b.res_host[i];
            out.fcx = b.filt_host[i].x;
            out.fcy = b.filt_host[i].y;
            out.fr = b.filt_host[i].z;
            out.fweight = b.filt_host[i].w;
            out.filtered_valid = b.filt_host[i].w > 0.0f ? 1 : 0;
            out.t_submit_ns = e.t_submit;
            out.t_launch_ns = b.t_launch;
            out.t_done_ns = t;
            out.batch_size = (int32_t)b.entries.size();
            s->done.push_back(out);
            if (e.slot >= 0)
                e.st->free_slots.push_back(e.slot);
            --e.st->outstanding;
            ++s->n_served;
        }
        // closed streams whose last frame was in this batch (entries are
        // grouped by stream, so each appears in one run)
        std::vector<Stream *> finished;
        for (size_t i = 0; i < b.entries.size(); ++i) {
            Stream *st = b.entries[i].st;
            if ((i == 0 || b.entries[i - 1].st != st) && st->closing && st->outstanding == 0
                && st->queue.empty())
                finished.push_back(st);
        }
        b.entries.clear();
        for (Stream *st : finished)
            release_stream(s, st);
        b.busy = false;
        s->inflight.pop_front();
    }
    return CA_OK;
}

void admit(ca_server *s)
{
    while (!s->waiting.empty() && try_admit(s, s->waiting.front()))
        s->waiting.pop_front();
}

// Copies of submitted frames into free ring slots: frames in device memory
// go into one batched copy launch per kMaxIngest frames (k_ingest; a lone
// frame takes the runtime's 2-D copy, measured quicker for one frame),
// frames in host memory into one 2-D copy each.  Lent frames are ready at
// once, read in place; a stream's frames stay in submission order (a lent
// frame waits behind a copied one that waits for a slot).
int ingest(ca_server *s)
{
    ca::IngestArgs batch;
    batch.n = 0;
    auto flush = [&]() {
        if (batch.n == 0)
            return true;
        bool ok;
        if (batch.n == 1) {
            const ca::IngestCopy &c = batch.c[0];
            ok = hipMemcpy2DAsync(c.dst, (size_t)c.width, c.src, (size_t)c.spitch, (size_t)c.width,
                                  (size_t)c.rows, hipMemcpyDeviceToDevice, s->compute)
                 == hipSuccess;
        } else {
            ok = ca::launch_ingest(batch, s->compute) == hipSuccess;
        }
        batch.n = 0;
        return ok;
    };
    for (Stream *st : s->order) {
        if (!st->admitted)
            continue;
        while (!st->queue.empty()) {
            const Pending p = st->queue.front();
            if (p.is_dev == 2) {
                // lent: read in place by its batch, no slot and no copy
                st->queue.pop_front();
                s->ready.push_back({st, p.seq, -1, p.t_submit, p.src, p.stride});
                ++st->outstanding;
                continue;
            }
            if (st->free_slots.empty())
                break;
            st->queue.pop_front();
            const int32_t slot = st->free_slots.back();
            st->free_slots.pop_back();
            uint8_t *dst = s->arena_mem + st->ring_off + (size_t)slot * st->slot_bytes;
            if (p.is_dev) {
                ca::IngestCopy &c = batch.c[batch.n++];
                c.src = p.src;
                c.dst = dst;
                c.spitch = p.stride;
                c.width = 3 * st->W;
                c.rows = st->H;
                if (batch.n == ca::kMaxIngest && !flush())
                    return CA_E_DEVICE;
            } else if (hipMemcpy2DAsync(dst, (size_t)3 * st->W, p.src, (size_t)p.stride,
                                        (size_t)3 * st->W, (size_t)st->H, hipMemcpyHostToDevice,
                                        s->compute) != hipSuccess) {
                return CA_E_DEVICE;
            }
            s->ready.push_back({st, p.seq, slot, p.t_submit, nullptr, 0});
            ++st->outstanding;
        }
    }
    return flush() ? CA_OK : CA_E_DEVICE;
}

int launch(ca_server *s)
{
    while (!s->ready.empty() && (int32_t)s->inflight.size() < s->cfg.max_inflight) {
        size_t slot = 0;
        while (slot < s->batches.size() && s->batches[slot].busy)
            ++slot;
        if (slot == s->batches.size())
            return CA_OK;
        Batch &b = s->batches[slot];
        const size_t n = std::min<size_t>(s->ready.size(), (size_t)s->cfg.max_batch);
        b.entries.assign(s->ready.begin(), s->ready.begin() + (ptrdiff_t)n);
        s->ready.erase(s->ready.begin(), s->ready.begin() + (ptrdiff_t)n);
        // frames of one stream contiguous and in sequence order
        std::stable_sort(b.entries.begin(), b.entries.end(), [](const Entry &x, const Entry &y) {
            return x.st->state != y.st->state ? x.st->state < y.st->state : x.seq < y.seq;
        });
        int32_t n_runs = 0;
        for (size_t i = 0; i < n; ++i) {
            const Entry &e = b.entries[i];
            if (i == 0 || b.entries[i - 1].st != e.st)
                b.runs_host[n_runs++] = make_int4(e.st->state, (int)i, (int)i + 1, 0);
            else
                b.runs_host[n_runs - 1].z = (int)i + 1;
        }
        const size_t upload = stage_batch(s, b, n);
        // the batch's frames were copied earlier on the same stream
        const hipStream_t cs = s->compute;
        if (hipMemcpyAsync(b.plan.mem, b.stage, upload, hipMemcpyHostToDevice, cs) != hipSuccess
            || hipMemcpyAsync(b.runs_dev, b.runs_host, (size_t)n_runs * sizeof(int4),
                              hipMemcpyHostToDevice, cs) != hipSuccess)
            return CA_E_DEVICE;
        int rc = cahost::enqueue(s->ctx, &b.plan, s->arena_mem, (int32_t)n, s->cfg.params, nullptr,
                                 nullptr, b.res_dev, cs, false);
        if (rc != CA_OK)
            return rc;
        if (ca::launch_stream_update(b.res_dev, b.runs_dev, n_runs, s->state_dev, b.filt_dev,
                                     s->cfg.smooth, cs) != hipSuccess
            || hipMemcpyAsync(b.res_host, b.res_dev, n * sizeof(ca_result), hipMemcpyDeviceToHost,
                              cs) != hipSuccess
            || hipMemcpyAsync(b.filt_host, b.filt_dev, n * sizeof(float4), hipMemcpyDeviceToHost,
                              cs) != hipSuccess
            || hipEventRecord(b.done, cs) != hipSuccess)
            return CA_E_DEVICE;
        b.t_launch = now_ns();
        b.busy = true;
        s->inflight.push_back(slot);
        ++s->n_batches;
    }
    return CA_OK;
}

bool valid_config(const ca_server_config &c)
{
    return c.max_streams >= 1 && c.max_streams <= 65536 && c.ring_slots >= 1
           && c.ring_slots <= 64 && c.max_batch >= 1 && c.max_batch <= 4096
           && c.max_inflight >= 1 && c.max_inflight <= 8 && c.hbm_budget > 0
           && c.smooth >= 0.0f && c.smooth < 1.0f;
}

}  // namespace

int ca_server_create(ca_ctx *ctx, const ca_server_config *cfg, ca_server **out)
{
    if (!ctx || !cfg || !out || !valid_config(*cfg))
        return CA_E_INVAL;
    *out = nullptr;
    ca_frame_desc probe;
    std::memset(&probe, 0, sizeof(probe));
    probe.width = probe.height = 16;
    probe.row_stride = 48;
    probe.pixel_stride = 3;
    if (cahost::validate(&probe, 1, cfg->params) != CA_OK)
        return CA_E_INVAL;
    if ((cfg->params.scorer == CA_SCORER_LEARNED && !ctx->model)
        || (cfg->params.scorer == CA_SCORER_LEARNED_2D && !ctx->model2d))
        return CA_E_INVAL;
    cahost::DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return CA_E_DEVICE;
    ca_server *s = new (std::nothrow) ca_server();
    if (!s)
        return CA_E_NOMEM;
    s->ctx = ctx;
    s->cfg = *cfg;
    const size_t B = (size_t)cfg->max_batch;
    bool ok = hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking) == hipSuccess
              && hipMalloc(&s->arena_mem, cfg->hbm_budget) == hipSuccess
              && hipMalloc(&s->state_dev, sizeof(float4) * (size_t)cfg->max_streams) == hipSuccess
              && hipMemset(s->state_dev, 0, sizeof(float4) * (size_t)cfg->max_streams)
                     == hipSuccess;
    // the layout of a slot's block: max_batch frames, each of its own shape
    // (so the strip tables of any batch fit), score tables uploaded once
    int32_t sg_len = 0;
    const float *lut = ok ? cahost::cached_tables(ctx, cfg->params, &sg_len) : nullptr;
    std::vector<ca_frame_desc> dims(B);
    for (size_t i = 0; i < B; ++i) {
        ca_frame_desc &d = dims[i];
        std::memset(&d, 0, sizeof(d));
        d.width = 16 + (int32_t)i;
        d.height = 16;
        d.row_stride = 3 * d.width;
        d.pixel_stride = 3;
    }
    std::vector<cahost::Shape> shapes(B);
    std::vector<uint8_t> image;
    cahost::Plan proto;
    if (ok) {
        int rc = cahost::plan_layout(ctx, dims.data(), (int32_t)B, cfg->params, lut, sg_len,
                                     shapes.data(), (int32_t)B, &proto, &s->layout, nullptr, 0);
        if (rc == CA_OK) {
            image.resize(s->layout.image_bytes);
            rc = cahost::plan_layout(ctx, dims.data(), (int32_t)B, cfg->params, lut, sg_len,
                                     shapes.data(), (int32_t)B, &proto, &s->layout, image.data(),
                                     image.size());
        }
        if (rc != CA_OK) {
            ca_server_destroy(s);
            return rc;
        }
    }
    s->batches.resize(ok ? (size_t)cfg->max_inflight : 0);
    const size_t stage_bytes = s->layout.image_bytes;
    for (Batch &b : s->batches) {
        b.plan.P = proto.P;
        b.plan.groups = proto.groups;
        b.plan.sg_len = proto.sg_len;
        b.plan.dynamic = true;
        ok = ok && hipMalloc(&b.plan.mem, s->layout.total) == hipSuccess
             && hipMemcpy(b.plan.mem, image.data(), image.size(), hipMemcpyHostToDevice)
                    == hipSuccess
             && hipMalloc(&b.res_dev, B * sizeof(ca_result)) == hipSuccess
             && hipMalloc(&b.filt_dev, B * sizeof(float4)) == hipSuccess
             && hipMalloc(&b.runs_dev, B * sizeof(int4)) == hipSuccess
             && hipHostMalloc(&b.stage, stage_bytes) == hipSuccess
             && hipHostMalloc(&b.runs_host, B * sizeof(int4)) == hipSuccess
             && hipHostMalloc(&b.res_host, B * sizeof(ca_result)) == hipSuccess
             && hipHostMalloc(&b.filt_host, B * sizeof(float4)) == hipSuccess
             && hipEventCreateWithFlags(&b.done, hipEventDisableTiming) == hipSuccess;
        if (ok)
            cahost::plan_pointers(&b.plan, b.plan.mem, s->layout);
    }
    ok = ok && hipDeviceSynchronize() == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        ca_server_destroy(s);
        return CA_E_NOMEM;
    }
    s->arena.reset(cfg->hbm_budget);
    for (int32_t k = cfg->max_streams - 1; k >= 0; --k)
        s->free_states.push_back(k);
    *out = s;
    return CA_OK;
}

void ca_server_destroy(ca_server *s)
{
    if (!s)
        return;
    cahost::DeviceGuard guard(s->ctx->device);
    if (s->compute)
        (void)hipStreamSynchronize(s->compute);
    for (Batch &b : s->batches)
        free_batch(b);
    for (auto &kv : s->streams)
        delete kv.second;
    (void)hipFree(s->arena_mem);
    (void)hipFree(s->state_dev);
    if (s->compute)
        (void)hipStreamDestroy(s->compute);
    delete s;
}

int ca_server_open(ca_server *s, int32_t id, int32_t W, int32_t H, int32_t *admitted)
{
    if (!s || !admitted || id < 0 || s->streams.count(id) || W < 16 || H < 16
        || W > CA_MAX_EXTENT || H > CA_MAX_EXTENT)
        return CA_E_INVAL;
    const size_t slot = frame_bytes(W, H);
    if (slot * (size_t)s->cfg.ring_slots > s->cfg.hbm_budget)
        return CA_E_INVAL;
    // the strip kernels stage a line of the frame's longest extent in LDS
    const size_t pitch = cahost::align_up((size_t)std::max(W, H), 16);
    const int32_t sg_len = s->batches.empty() ? 0 : s->batches[0].plan.sg_len;
    if (ca::strip_lds_bytes(sg_len, (int)pitch) > s->ctx->max_lds
        || ca::fused_lds_bytes(sg_len, (int)pitch) > s->ctx->max_lds)
        return CA_E_UNSUPPORTED;
    Stream *st = new (std::nothrow) Stream();
    if (!st)
        return CA_E_NOMEM;
    st->id = id;
    st->W = W;
    st->H = H;
    st->slot_bytes = slot;
    // the stream's strip positions (Eq. 1), computed once here
    const ca_params &p = s->cfg.params;
    try {
        st->table.assign((size_t)(p.n_hstrips + p.n_vstrips), 0);
    } catch (...) {
        delete st;
        return CA_E_NOMEM;
    }
    cahost::strip_positions(H, p.n_hstrips, p.alpha, st->table.data());
    cahost::strip_positions(W, p.n_vstrips, p.alpha, st->table.data() + p.n_hstrips);
    s->streams[id] = st;
    s->order.push_back(st);
    cahost::DeviceGuard guard(s->ctx->device);
    if (!guard.ok)
        return CA_E_DEVICE;
    if (s->waiting.empty() && try_admit(s, st)) {
        *admitted = 1;
    } else {
        s->waiting.push_back(st);
        *admitted = 0;
    }
    return CA_OK;
}

int ca_server_close(ca_server *s, int32_t id)
{
    if (!s)
        return CA_E_INVAL;
    auto it = s->streams.find(id);
    if (it == s->streams.end() || it->second->closing)
        return CA_E_INVAL;
    Stream *st = it->second;
    st->closing = true;
    if (!st->admitted) {
        if (!st->queue.empty())
            return CA_OK;    // admitted later, served, then released
        s->waiting.erase(std::find(s->waiting.begin(), s->waiting.end(), st));
        release_stream(s, st);
        return CA_OK;
    }
    if (st->outstanding == 0 && st->queue.empty())
        release_stream(s, st);
    return CA_OK;
}

int ca_server_submit(ca_server *s, int32_t id, uint64_t seq, const uint8_t *src, int64_t stride,
                     int32_t src_is_device)
{
    if (!s || !src)
        return CA_E_INVAL;
    auto it = s->streams.find(id);
    if (it == s->streams.end() || it->second->closing)
        return CA_E_INVAL;
    Stream *st = it->second;
    if (stride < 3 * (int64_t)st->W || (st->any_seq && seq <= st->last_seq)
        || src_is_device < 0 || src_is_device > 2 || (src_is_device == 2 && stride > INT32_MAX))
        return CA_E_INVAL;
    st->any_seq = true;
    st->last_seq = seq;
    st->queue.push_back({seq, src, stride, src_is_device, now_ns()});
    ++s->n_submitted;
    return CA_OK;
}

int ca_server_step(ca_server *s, ca_served *out, int32_t max_out, int32_t *n_out)
{
    if (!s || !n_out || max_out < 0 || (max_out > 0 && !out))
        return CA_E_INVAL;
    *n_out = 0;
    cahost::DeviceGuard guard(s->ctx->device);
    if (!guard.ok)
        return CA_E_DEVICE;
    int rc = retire(s);
    if (rc != CA_OK)
        return rc;
    admit(s);
    rc = ingest(s);
    if (rc != CA_OK)
        return rc;
    rc = launch(s);
    if (rc != CA_OK)
        return rc;
    int32_t k = 0;
    while (k < max_out && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    *n_out = k;
    return CA_OK;
}

int ca_server_stats(ca_server *s, int64_t out[8])
{
    if (!s || !out)
        return CA_E_INVAL;
    int64_t queued = 0, admitted = 0;
    for (Stream *st : s->order) {
        queued += (int64_t)st->queue.size();
        admitted += st->admitted ? 1 : 0;
    }
    int64_t inflight = 0;
    for (size_t k : s->inflight)
        inflight += (int64_t)s->batches[k].entries.size();
    out[0] = s->n_submitted;
    out[1] = s->n_served;
    out[2] = queued;
    out[3] = inflight + (int64_t)s->ready.size();
    out[4] = admitted;
    out[5] = (int64_t)s->waiting.size();
    out[6] = s->n_batches;
    out[7] = (int64_t)s->arena.used;
    return CA_OK;
}
