// Host-core harness: the library's host code (ca_api.cpp, ca_server.cpp),
// compiled with g++ against a stand-in HIP runtime (hip_stub/) under
// AddressSanitizer and UndefinedBehaviorSanitizer, driven without a GPU.
//
// The stand-in models device memory as host memory (large blocks as
// inaccessible reservations that only bounds checks touch), asynchronous
// work as done some event polls after it is enqueued, and the kernels as
// functions that check their arguments (every frame, strip table and
// output index inside its allocation) and write zero results.  While a
// scenario steps a server, any synchronous runtime call (allocation, free,
// blocking copy or memset, any synchronize) aborts the run: ca_server_step
// must only enqueue work and poll events.
//
// Scenarios (argv[1]): serve_sequence, few_slots, memory_wait, batch_api.
// Test infrastructure only.
#include <hip/hip_runtime.h>

#include <sys/mman.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "ca_host.h"

// ------------------------------------------------------------ runtime ----

namespace {

bool g_forbid_sync = false;      // set around ca_server_step
const char *g_forbid_where = "";
int g_event_lag = 2;             // polls before a recorded event completes
long g_async_ops = 0;

struct Alloc {
    size_t bytes;
    bool accessible;             // host-backed (else an inaccessible reservation)
    bool pinned;
};
std::map<uintptr_t, Alloc> g_allocs;

[[noreturn]] void fail(const char *fmt, const char *what)
{
    std::fprintf(stderr, fmt, what);
    std::fprintf(stderr, "\n");
    std::abort();
}

void sync_call(const char *name)
{
    if (g_forbid_sync) {
        std::fprintf(stderr, "synchronous runtime call %s inside %s\n", name, g_forbid_where);
        std::abort();
    }
}

// The allocation holding [p, p + n), or null for memory the runtime did
// not hand out (the caller's own host memory).
const Alloc *find(const void *p, size_t n)
{
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    auto it = g_allocs.upper_bound(a);
    if (it == g_allocs.begin())
        return nullptr;
    --it;
    if (a >= it->first + it->second.bytes)
        return nullptr;
    if (a + n > it->first + it->second.bytes)
        fail("access beyond the end of a runtime allocation (%s)", "bounds");
    return &it->second;
}

void check_device(const void *p, size_t n, const char *what)
{
    if (n == 0)
        return;
    const Alloc *al = find(p, n);
    if (!al || al->pinned)
        fail("device access outside device memory: %s", what);
}

void copy(void *dst, const void *src, size_t n, hipMemcpyKind kind)
{
    if (n == 0)
        return;
    const Alloc *d = find(dst, n), *s = find(src, n);
    if (kind == hipMemcpyHostToDevice || kind == hipMemcpyDeviceToDevice)
        check_device(dst, n, "copy destination");
    if (kind == hipMemcpyDeviceToHost || kind == hipMemcpyDeviceToDevice)
        check_device(src, n, "copy source");
    if ((d && !d->accessible) || (s && !s->accessible))
        return;                  // a reservation: checked, not copied
    std::memmove(dst, src, n);
}

}  // namespace

struct ihipStream_t {
    int id;
};
struct ihipEvent_t {
    bool recorded = false;
    int polls_left = 0;
};
struct ihipGraph_t {
    int unused;
};
struct ihipGraphExec_t {
    int unused;
};

hipError_t hipGetDeviceCount(int *count)
{
    *count = 1;
    return hipSuccess;
}
hipError_t hipGetDevice(int *dev)
{
    *dev = 0;
    return hipSuccess;
}
hipError_t hipSetDevice(int dev) { return dev == 0 ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipDeviceGetAttribute(int *value, hipDeviceAttribute_t attr, int)
{
    *value = attr == hipDeviceAttributeMaxSharedMemoryPerBlock ? 160 * 1024 : 256;
    return hipSuccess;
}
hipError_t hipDeviceSynchronize(void)
{
    sync_call("hipDeviceSynchronize");
    return hipSuccess;
}
hipError_t hipGetLastError(void) { return hipSuccess; }

hipError_t hipMalloc(void **ptr, size_t bytes)
{
    sync_call("hipMalloc");
    if (bytes == 0)
        bytes = 1;
    void *p;
    bool accessible = bytes <= ((size_t)256 << 20);
    if (accessible) {
        p = std::calloc(1, bytes);
    } else {
        p = mmap(nullptr, bytes, PROT_NONE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
        if (p == MAP_FAILED)
            p = nullptr;
    }
    if (!p)
        return hipErrorOutOfMemory;
    g_allocs[reinterpret_cast<uintptr_t>(p)] = {bytes, accessible, false};
    *ptr = p;
    return hipSuccess;
}
hipError_t hipFree(void *ptr)
{
    sync_call("hipFree");
    if (!ptr)
        return hipSuccess;
    auto it = g_allocs.find(reinterpret_cast<uintptr_t>(ptr));
    if (it == g_allocs.end() || it->second.pinned)
        fail("hipFree of %s", "memory hipMalloc did not return");
    if (it->second.accessible)
        std::free(ptr);
    else
        munmap(ptr, it->second.bytes);
    g_allocs.erase(it);
    return hipSuccess;
}
hipError_t hipHostMalloc(void **ptr, size_t bytes, unsigned)
{
    sync_call("hipHostMalloc");
    void *p = std::calloc(1, bytes ? bytes : 1);
    if (!p)
        return hipErrorOutOfMemory;
    g_allocs[reinterpret_cast<uintptr_t>(p)] = {bytes ? bytes : 1, true, true};
    *ptr = p;
    return hipSuccess;
}
hipError_t hipHostFree(void *ptr)
{
    sync_call("hipHostFree");
    if (!ptr)
        return hipSuccess;
    auto it = g_allocs.find(reinterpret_cast<uintptr_t>(ptr));
    if (it == g_allocs.end() || !it->second.pinned)
        fail("hipHostFree of %s", "memory hipHostMalloc did not return");
    std::free(ptr);
    g_allocs.erase(it);
    return hipSuccess;
}

hipError_t hipMemcpy(void *dst, const void *src, size_t bytes, hipMemcpyKind kind)
{
    sync_call("hipMemcpy");
    copy(dst, src, bytes, kind);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind kind,
                          hipStream_t)
{
    ++g_async_ops;
    if (kind == hipMemcpyHostToDevice) {
        const Alloc *s = find(src, bytes);
        if (g_forbid_sync && (!s || !s->pinned))
            fail("asynchronous copy from unpinned host memory inside %s", g_forbid_where);
    }
    copy(dst, src, bytes, kind);
    return hipSuccess;
}
hipError_t hipMemcpy2DAsync(void *dst, size_t dpitch, const void *src, size_t spitch,
                            size_t width, size_t height, hipMemcpyKind kind, hipStream_t)
{
    ++g_async_ops;
    if (height == 0 || width == 0)
        return hipSuccess;
    if (width > dpitch || width > spitch)
        fail("2-D copy %s", "row wider than its pitch");
    const size_t dn = dpitch * (height - 1) + width, sn = spitch * (height - 1) + width;
    if (kind == hipMemcpyHostToDevice || kind == hipMemcpyDeviceToDevice)
        check_device(dst, dn, "2-D copy destination");
    if (kind == hipMemcpyDeviceToDevice)
        check_device(src, sn, "2-D copy source");
    return hipSuccess;   // frame bytes are not needed by the stand-in kernels
}
hipError_t hipMemset(void *dst, int value, size_t bytes)
{
    sync_call("hipMemset");
    check_device(dst, bytes, "memset");
    const Alloc *al = find(dst, bytes);
    if (al && al->accessible)
        std::memset(dst, value, bytes);
    return hipSuccess;
}
hipError_t hipMemsetAsync(void *dst, int value, size_t bytes, hipStream_t)
{
    ++g_async_ops;
    check_device(dst, bytes, "memset");
    const Alloc *al = find(dst, bytes);
    if (al && al->accessible)
        std::memset(dst, value, bytes);
    return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned)
{
    sync_call("hipStreamCreateWithFlags");
    static int next = 1;
    *s = new ihipStream_t{next++};
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s)
{
    sync_call("hipStreamDestroy");
    delete s;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t)
{
    sync_call("hipStreamSynchronize");
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned)
{
    ++g_async_ops;
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode)
{
    sync_call("hipStreamBeginCapture");
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *graph)
{
    sync_call("hipStreamEndCapture");
    *graph = new ihipGraph_t{0};
    return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t *e)
{
    sync_call("hipEventCreate");
    *e = new ihipEvent_t();
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e)
{
    sync_call("hipEventDestroy");
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t)
{
    ++g_async_ops;
    e->recorded = true;
    e->polls_left = g_event_lag;
    return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e)
{
    if (e->recorded && e->polls_left > 0) {
        --e->polls_left;
        return hipErrorNotReady;
    }
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e)
{
    sync_call("hipEventSynchronize");
    e->polls_left = 0;
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t)
{
    *ms = 0.01f;
    return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t *exec, hipGraph_t, hipGraphNode_t *, char *, size_t)
{
    sync_call("hipGraphInstantiate");
    *exec = new ihipGraphExec_t{0};
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t)
{
    ++g_async_ops;
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t exec)
{
    sync_call("hipGraphExecDestroy");
    delete exec;
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t graph)
{
    sync_call("hipGraphDestroy");
    delete graph;
    return hipSuccess;
}

// ------------------------------------------------------ kernel stand-ins --

namespace {

long g_frames_checked = 0;

// One frame of a launch: its descriptor, every byte its strips can read,
// and its strip table.
void check_frame(const uint8_t *frames, const ca::FrameDev *fd, const int32_t *strips, int32_t f,
                 int32_t n_h, int32_t n_v, int32_t line_pitch)
{
    check_device(fd + f, sizeof(ca::FrameDev), "frame descriptor");
    const ca::FrameDev &d = fd[f];
    const int32_t S = n_h + n_v;
    if (d.W < 16 || d.H < 16 || d.rs < 3 * d.W || d.offset < 0)
        fail("frame descriptor %s", "out of range");
    if (line_pitch < std::max(d.W, d.H))
        fail("LDS line pitch %s", "shorter than the frame's longest extent");
    if (d.table < 0 || d.table % S != 0)
        fail("strip table index %s", "not a table start");
    check_device(frames + d.offset, (size_t)d.rs * (size_t)(d.H - 1) + 3 * (size_t)d.W, "frame bytes");
    check_device(strips + d.table, sizeof(int32_t) * (size_t)S, "strip table");
    for (int32_t i = 0; i < S; ++i) {
        const int32_t v = strips[d.table + i], ext = i < n_h ? d.H : d.W;
        if (v < 1 || v > ext - 2)
            fail("strip position %s", "outside the frame");
    }
    ++g_frames_checked;
}

void write_results(ca_result *out, int32_t first, int32_t n)
{
    check_device(out + first, sizeof(ca_result) * (size_t)n, "results");
    std::memset(out + first, 0, sizeof(ca_result) * (size_t)n);
}

}  // namespace

namespace ca {

size_t strip_lds_bytes(int sg_len, int line_pitch)
{
    return (size_t)(sg_len + kQtBins + kLumaLevels) * sizeof(float) + 16 + 3 * (size_t)line_pitch;
}
size_t fused_lds_bytes(int sg_len, int line_pitch) { return strip_lds_bytes(sg_len, line_pitch) + 4096; }

hipError_t launch_strips(const StripArgs &a, size_t lds_bytes, hipStream_t, hipEvent_t, hipEvent_t)
{
    ++g_async_ops;
    const int32_t S = a.n_h + a.n_v;
    if (lds_bytes < strip_lds_bytes(a.sg_len, a.line_pitch))
        fail("strip launch %s", "with too little LDS");
    for (int32_t k = 0; k < a.n_items / S; ++k) {
        const int32_t f = a.frame_list ? a.frame_list[k] : a.frame0 + k;
        check_frame(a.frames, a.fd, a.strips, f, a.n_h, a.n_v, a.line_pitch);
        if (a.keep)
            check_device(a.keep + f, sizeof(ca_result), "learned results to keep");
    }
    return hipSuccess;
}
hipError_t launch_ransac(const RansacArgs &a, const SelectArgs &sel, int n_frames, hipStream_t,
                         hipEvent_t, hipEvent_t)
{
    ++g_async_ops;
    check_device(a.cand + (size_t)a.frame0 * a.P, sizeof(ca_point) * (size_t)n_frames * a.P,
                 "candidates");
    check_device(a.rec + (size_t)a.frame0 * a.groups, sizeof(Record) * (size_t)n_frames * a.groups,
                 "records");
    if (a.groups_done)
        check_device(a.groups_done + a.frame0, sizeof(uint32_t) * (size_t)n_frames, "counters");
    if (a.keep)
        check_device(a.keep + a.frame0, sizeof(ca_result) * (size_t)n_frames,
                     "learned results to keep");
    write_results(sel.out, a.frame0, n_frames);
    return hipSuccess;
}
hipError_t launch_fused(const FusedArgs &a, int grid, size_t lds_bytes, hipStream_t, hipEvent_t,
                        hipEvent_t)
{
    ++g_async_ops;
    if (grid < 1 || lds_bytes < fused_lds_bytes(a.s.sg_len, a.s.line_pitch))
        fail("fused launch %s", "with a bad grid or too little LDS");
    const int32_t S = a.s.n_h + a.s.n_v;
    for (int32_t f = 0; f < a.s.n_items / S; ++f)
        check_frame(a.s.frames, a.s.fd, a.s.strips, f, a.s.n_h, a.s.n_v, a.s.line_pitch);
    check_device(a.ctl, sizeof(uint32_t) * ctl_words(a.se.n_frames), "control words");
    write_results(a.se.out, 0, a.se.n_frames);
    return hipSuccess;
}
hipError_t launch_stream_update(const ca_result *res, const int4 *runs, int n_runs, float4 *state,
                                float4 *filt, float, hipStream_t)
{
    ++g_async_ops;
    int expect = 0;
    for (int r = 0; r < n_runs; ++r) {
        check_device(runs + r, sizeof(int4), "run");
        const int4 run = runs[r];
        if (run.y != expect || run.z <= run.y)
            fail("stream runs %s", "not contiguous");
        expect = run.z;
        check_device(state + run.x, sizeof(float4), "stream state");
        check_device(res + run.y, sizeof(ca_result) * (size_t)(run.z - run.y), "run results");
        for (int i = run.y; i < run.z; ++i)
            filt[i] = state[run.x];
    }
    return hipSuccess;
}
hipError_t launch_ingest(const IngestArgs &a, hipStream_t)
{
    ++g_async_ops;
    if (a.n < 1 || a.n > kMaxIngest)
        fail("ingest launch %s", "with a bad copy count");
    for (int i = 0; i < a.n; ++i) {
        const IngestCopy &c = a.c[i];
        if (c.width < 1 || c.rows < 1 || c.spitch < c.width)
            fail("ingest copy %s", "with a bad shape");
        check_device(c.dst, (size_t)c.width * (size_t)c.rows, "ingest destination");
        check_device(c.src, (size_t)c.spitch * (size_t)(c.rows - 1) + (size_t)c.width,
                     "ingest source");
    }
    return hipSuccess;
}
hipError_t launch_fallback(ca_result *out, const ca_result *fallback, int n, float, hipStream_t)
{
    ++g_async_ops;
    check_device(out, sizeof(ca_result) * (size_t)n, "results");
    check_device(fallback, sizeof(ca_result) * (size_t)n, "fallback results");
    return hipSuccess;
}
hipError_t fused_occupancy(size_t, int *blocks_per_cu)
{
    *blocks_per_cu = 2;
    return hipSuccess;
}
hipError_t launch_cnn_strips(const CnnStripArgs &a, int groups_per_xcd, hipStream_t, hipEvent_t,
                             hipEvent_t)
{
    ++g_async_ops;
    if (groups_per_xcd < 1)
        fail("learned strip launch %s", "without workgroups");
    const int32_t S = a.n_h + a.n_v;
    for (int32_t k = 0; k < a.n_items / S; ++k)
        check_frame(a.frames, a.fd, a.strips, a.frame0 + k, a.n_h, a.n_v, 16384);
    return hipSuccess;
}
int cnn_strips_blocks_per_cu() { return 2; }
hipError_t launch_cnn_grad(const CnnTrainArgs &, int, hipStream_t) { return hipSuccess; }
hipError_t launch_cnn_reduce(const float *, int, float *, float *, hipStream_t) { return hipSuccess; }
hipError_t launch_cnn_update(float *, float *, const float *, float, float, uint8_t *, hipStream_t)
{
    return hipSuccess;
}
hipError_t launch_cnn_pack(const float *, uint8_t *, hipStream_t) { return hipSuccess; }
hipError_t launch_mfma_probe(float *, hipStream_t) { return hipSuccess; }
hipError_t launch_cnn2d_strips(const Cnn2dStripArgs &a, hipStream_t, hipEvent_t, hipEvent_t)
{
    ++g_async_ops;
    const int32_t S = a.n_h + a.n_v;
    for (int32_t k = 0; k < a.n_items / S; ++k)
        check_frame(a.frames, a.fd, a.strips, a.frame0 + k, a.n_h, a.n_v, 16384);
    return hipSuccess;
}
hipError_t launch_cnn2d_windows(const uint8_t *, const uint8_t *, const int32_t *,
                                const int32_t *, float *, int, hipStream_t)
{
    return hipSuccess;
}
hipError_t launch_cnn2d_grad(const Cnn2dTrainArgs &, int, hipStream_t) { return hipSuccess; }
hipError_t launch_cnn2d_reduce(const float *, int, float *, float *, hipStream_t)
{
    return hipSuccess;
}
hipError_t launch_cnn2d_update(float *, float *, const float *, float, float, uint8_t *,
                               hipStream_t)
{
    return hipSuccess;
}
hipError_t launch_cnn2d_pack(const float *, uint8_t *, hipStream_t) { return hipSuccess; }
int cnn2d_grad_blocks_per_cu() { return 1; }
hipError_t launch_cnn_windows(const uint8_t *, const uint8_t *, const int32_t *, float *, int,
                              hipStream_t)
{
    return hipSuccess;
}

}  // namespace ca

namespace cahost {
int scratch_setup(int) { return CA_OK; }
}  // namespace cahost

// ------------------------------------------------------------- scenarios --

namespace {

struct Frame {
    int32_t stream;
    uint64_t seq;
    double t;
};

struct Sim {
    std::vector<std::pair<int32_t, int32_t>> shapes;   // per stream
    std::vector<Frame> arrivals;                       // by time
};

// serve_bench's workload: streams of 720p, 1080p and 4K in turn, Poisson
// arrivals at 30-60 frames/s each over `seconds`.
Sim make_sim(int n_streams, double seconds, unsigned seed)
{
    static const int32_t kShapes[3][2] = {{1280, 720}, {1920, 1080}, {3840, 2160}};
    std::mt19937_64 rng(seed);
    Sim sim;
    for (int s = 0; s < n_streams; ++s) {
        sim.shapes.push_back({kShapes[s % 3][0], kShapes[s % 3][1]});
        const double fps = std::uniform_real_distribution<double>(30.0, 60.0)(rng);
        std::exponential_distribution<double> gap(fps);
        double t = 0.0;
        for (uint64_t k = 0;; ++k) {
            t += gap(rng);
            if (t >= seconds)
                break;
            sim.arrivals.push_back({s, k, t});
        }
    }
    std::stable_sort(sim.arrivals.begin(), sim.arrivals.end(),
                     [](const Frame &a, const Frame &b) { return a.t < b.t; });
    return sim;
}

#define CHECK(cond)                                                                         \
    do {                                                                                    \
        if (!(cond)) {                                                                      \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond);         \
            std::abort();                                                                   \
        }                                                                                   \
    } while (0)

int step(ca_server *srv, std::vector<ca_served> &got)
{
    ca_served buf[256];
    int32_t n = 0;
    g_forbid_sync = true;
    g_forbid_where = "ca_server_step";
    const int rc = ca_server_step(srv, buf, 256, &n);
    g_forbid_sync = false;
    CHECK(rc == CA_OK);
    got.insert(got.end(), buf, buf + n);
    return n;
}

ca_server_config config(int max_batch, int max_inflight, size_t budget, int scorer)
{
    ca_server_config c;
    std::memset(&c, 0, sizeof(c));
    c.max_streams = 64;
    c.ring_slots = 2;
    c.max_batch = max_batch;
    c.max_inflight = max_inflight;
    c.hbm_budget = budget;
    c.smooth = 0.8f;
    ca_default_params(&c.params);
    c.params.n_hstrips = 32;
    c.params.n_vstrips = 32;
    c.params.ransac_attempts = 1024;
    if (scorer) {
        c.params.scorer = CA_SCORER_LEARNED;
        c.params.fallback_inlier_frac = 0.5f;
    }
    return c;
}

// Serve every arrival; realtime: a simulated clock advancing dt per loop,
// frames submitted once their arrival time has passed; else all at once.
// Every frame must come back once, per stream in sequence order, within a
// bounded number of steps.
void serve(ca_ctx *ctx, const Sim &sim, const ca_server_config &cfg, bool realtime,
           const std::vector<uint8_t *> &src, const char *name)
{
    ca_server *srv = nullptr;
    CHECK(ca_server_create(ctx, &cfg, &srv) == CA_OK);
    std::set<int32_t> ids;
    for (const Frame &f : sim.arrivals)
        ids.insert(f.stream);
    for (int32_t id : ids) {
        int32_t adm = 0;
        CHECK(ca_server_open(srv, id, sim.shapes[(size_t)id].first, sim.shapes[(size_t)id].second,
                             &adm) == CA_OK);
    }
    std::vector<ca_served> got;
    size_t next = 0;
    double now = 0.0;
    long loops = 0;
    const double dt = 20e-6;
    const double t_end = sim.arrivals.empty() ? 0.0 : sim.arrivals.back().t;
    const long limit = (realtime ? (long)(t_end / dt) : 0) + 20 * (long)sim.arrivals.size() + 10000;
    while (got.size() < sim.arrivals.size()) {
        while (next < sim.arrivals.size() && (!realtime || sim.arrivals[next].t <= now)) {
            const Frame &f = sim.arrivals[next++];
            const int32_t W = sim.shapes[(size_t)f.stream].first;
            const uint8_t *p = src[(size_t)(f.stream % 3)];
            // every other frame of a stream lent (read in place), the rest copied
            CHECK(ca_server_submit(srv, f.stream, f.seq, p, 3 * (int64_t)W, f.seq % 2 ? 1 : 2)
                  == CA_OK);
        }
        step(srv, got);
        now += dt;
        if (++loops > limit) {
            int64_t st[8];
            ca_server_stats(srv, st);
            std::fprintf(stderr,
                         "%s: no progress after %ld steps: submitted %lld served %lld queued %lld "
                         "in flight %lld batches %lld\n",
                         name, loops, (long long)st[0], (long long)st[1], (long long)st[2],
                         (long long)st[3], (long long)st[6]);
            std::abort();
        }
    }
    std::map<int32_t, uint64_t> last;
    std::set<std::pair<int32_t, uint64_t>> seen;
    for (const ca_served &r : got) {
        CHECK(seen.insert({r.stream_id, r.seq}).second);
        auto it = last.find(r.stream_id);
        CHECK(it == last.end() || r.seq > it->second);
        last[r.stream_id] = r.seq;
        CHECK(r.t_submit_ns <= r.t_launch_ns && r.t_launch_ns <= r.t_done_ns);
    }
    for (int32_t id : ids)
        CHECK(ca_server_close(srv, id) == CA_OK);
    step(srv, got);
    int64_t st[8];
    CHECK(ca_server_stats(srv, st) == CA_OK);
    CHECK(st[0] == (int64_t)sim.arrivals.size() && st[1] == st[0] && st[7] == 0);
    std::printf("ok %s frames=%zu batches=%lld steps=%ld\n", name, got.size(), (long long)st[6],
                loops);
    ca_server_destroy(srv);
}

std::vector<uint8_t *> sources()
{
    static const int32_t kShapes[3][2] = {{1280, 720}, {1920, 1080}, {3840, 2160}};
    std::vector<uint8_t *> out;
    for (const auto &s : kShapes) {
        void *p = nullptr;
        CHECK(hipMalloc(&p, (size_t)3 * s[0] * s[1]) == hipSuccess);
        out.push_back(static_cast<uint8_t *>(p));
    }
    return out;
}

void release(std::vector<uint8_t *> &v)
{
    for (uint8_t *p : v)
        CHECK(hipFree(p) == hipSuccess);
    v.clear();
}

void set_model(ca_ctx *ctx)
{
    std::vector<float> prm(CA_CNN_PARAMS, 0.01f);
    CHECK(ca_set_model(ctx, prm.data(), CA_CNN_PARAMS) == CA_OK);
}

// serve_bench's sequence: per scorer, a warm-up server fed every frame at
// once, then a second server of the same context in real time.
void scenario_serve_sequence(double seconds)
{
    ca_ctx *ctx = nullptr;
    CHECK(ca_create(&ctx, 0, 0) == CA_OK);
    set_model(ctx);
    auto src = sources();
    const Sim sim = make_sim(48, seconds, 2210);
    for (int scorer = 0; scorer < 2; ++scorer) {
        const ca_server_config cfg = config(64, 2, (size_t)4 << 30, scorer);
        serve(ctx, sim, cfg, false, src, scorer ? "learned warm-up" : "plain warm-up");
        serve(ctx, sim, cfg, true, src, scorer ? "learned realtime" : "plain realtime");
    }
    release(src);
    ca_destroy(ctx);
}

// More distinct stream shapes than frames per batch, and every schedule
// option: each batch carries its own strip tables.
void scenario_few_slots()
{
    ca_ctx *ctx = nullptr;
    CHECK(ca_create(&ctx, 0, 0) == CA_OK);
    auto src = sources();
    const Sim sim = make_sim(6, 0.2, 7);
    for (int64_t sched : {CA_SCHEDULE_SPLIT, CA_SCHEDULE_FUSED}) {
        CHECK(ca_set_option(ctx, CA_OPT_SCHEDULE, sched) == CA_OK);
        serve(ctx, sim, config(1, 1, (size_t)1 << 30, 0), true, src, "one frame per batch");
        serve(ctx, sim, config(2, 3, (size_t)1 << 30, 0), false, src, "two frames per batch");
    }
    CHECK(ca_set_option(ctx, CA_OPT_SCHEDULE, CA_SCHEDULE_SPLIT) == CA_OK);
    CHECK(ca_set_option(ctx, CA_OPT_PIPELINE, 2) == CA_OK);
    serve(ctx, sim, config(4, 2, (size_t)1 << 30, 0), false, src, "pipelined sub-batches");
    release(src);
    ca_destroy(ctx);
}

// Streams wait for memory and are admitted as others close.
void scenario_memory_wait()
{
    ca_ctx *ctx = nullptr;
    CHECK(ca_create(&ctx, 0, 0) == CA_OK);
    auto src = sources();
    const size_t ring = 2 * (((size_t)3 * 1920 * 1080 + 255) / 256 * 256);
    ca_server_config cfg = config(8, 2, 2 * ring, 0);
    ca_server *srv = nullptr;
    CHECK(ca_server_create(ctx, &cfg, &srv) == CA_OK);
    const int32_t ids[4] = {1, 4, 7, 10};
    int32_t adm[4];
    for (int k = 0; k < 4; ++k)
        CHECK(ca_server_open(srv, ids[k], 1920, 1080, &adm[k]) == CA_OK);
    CHECK(adm[0] && adm[1] && !adm[2] && !adm[3]);
    // submission modes other than host (0), device (1) and lent (2), and a
    // lent frame's stride beyond 32 bits, are rejected before any state changes
    CHECK(ca_server_submit(srv, ids[0], 0, src[1], 3 * 1920, 3) == CA_E_INVAL);
    CHECK(ca_server_submit(srv, ids[0], 0, src[1], 3 * 1920, -1) == CA_E_INVAL);
    CHECK(ca_server_submit(srv, ids[0], 0, src[1], (int64_t)1 << 32, 2) == CA_E_INVAL);
    for (int k = 0; k < 4; ++k)
        for (uint64_t q = 0; q < 3; ++q)
            CHECK(ca_server_submit(srv, ids[k], q, src[1], 3 * 1920, 1) == CA_OK);
    std::vector<ca_served> got;
    for (int i = 0; i < 1000 && got.size() < 6; ++i)
        step(srv, got);
    CHECK(got.size() == 6);
    for (const ca_served &r : got)
        CHECK(r.stream_id == 1 || r.stream_id == 4);
    CHECK(ca_server_close(srv, 1) == CA_OK && ca_server_close(srv, 4) == CA_OK);
    for (int i = 0; i < 1000 && got.size() < 12; ++i)
        step(srv, got);
    CHECK(got.size() == 12);
    int64_t st[8];
    CHECK(ca_server_stats(srv, st) == CA_OK);
    CHECK(st[4] == 2 && st[5] == 0);
    ca_server_destroy(srv);
    release(src);
    ca_destroy(ctx);
    std::printf("ok memory wait\n");
}

// The batch API: mixed shapes, plan caching and eviction under a small
// budget, candidates and attempts, pipelined and fused schedules, graphs.
void scenario_batch_api()
{
    ca_ctx *ctx = nullptr;
    CHECK(ca_create(&ctx, 0, (size_t)4 << 20) == CA_OK);
    const int32_t shapes[4][2] = {{720, 576}, {1280, 720}, {1920, 1080}, {3840, 2160}};
    size_t total = 0;
    std::vector<ca_frame_desc> dims;
    for (int i = 0; i < 10; ++i) {
        ca_frame_desc d;
        std::memset(&d, 0, sizeof(d));
        d.width = shapes[i % 4][0];
        d.height = shapes[i % 4][1];
        d.row_stride = 3 * d.width;
        d.pixel_stride = 3;
        d.byte_offset = (int64_t)total;
        d.frame_uid = (uint64_t)i;
        total += (size_t)3 * d.width * d.height;
        dims.push_back(d);
    }
    void *frames = nullptr, *out = nullptr, *pts = nullptr, *att = nullptr;
    CHECK(hipMalloc(&frames, total) == hipSuccess);
    CHECK(hipMalloc(&out, sizeof(ca_result) * 10) == hipSuccess);
    CHECK(hipMalloc(&pts, sizeof(ca_point) * 10 * 128) == hipSuccess);
    CHECK(hipMalloc(&att, sizeof(ca_attempt) * 10 * 256) == hipSuccess);
    ca_params p;
    ca_default_params(&p);
    p.n_hstrips = 32;
    p.n_vstrips = 32;
    const uint8_t *f = static_cast<const uint8_t *>(frames);
    ca_result *o = static_cast<ca_result *>(out);
    for (int64_t sched : {CA_SCHEDULE_SPLIT, CA_SCHEDULE_FUSED, CA_SCHEDULE_AUTO}) {
        CHECK(ca_set_option(ctx, CA_OPT_SCHEDULE, sched) == CA_OK);
        for (int64_t pipe : {1, 2, 4}) {
            CHECK(ca_set_option(ctx, CA_OPT_PIPELINE, pipe) == CA_OK);
            for (int n = 1; n <= 10; n += 3)   // batches of several sizes: plans evicted
                CHECK(ca_estimate_area(ctx, f, dims.data(), n, &p, o, nullptr) == CA_OK);
        }
    }
    CHECK(ca_debug_candidates(ctx, f, dims.data(), 10, &p, static_cast<ca_point *>(pts), o,
                              nullptr) == CA_OK);
    CHECK(ca_debug_attempts(ctx, f, dims.data(), 10, &p, static_cast<ca_attempt *>(att), o,
                            nullptr) == CA_OK);
    ca_graph *g = nullptr;
    CHECK(ca_graph_create(ctx, f, dims.data(), 10, &p, o, 3, &g) == CA_OK);
    CHECK(ca_graph_launch(g, nullptr) == CA_OK);
    ca_graph_destroy(g);
    // argument errors are caught before anything is enqueued
    ca_frame_desc bad = dims[0];
    bad.width = 8;
    CHECK(ca_estimate_area(ctx, f, &bad, 1, &p, o, nullptr) == CA_E_INVAL);
    bad = dims[0];
    bad.pixel_stride = 4;
    CHECK(ca_estimate_area(ctx, f, &bad, 1, &p, o, nullptr) == CA_E_UNSUPPORTED);
    CHECK(hipFree(frames) == hipSuccess && hipFree(out) == hipSuccess);
    CHECK(hipFree(pts) == hipSuccess && hipFree(att) == hipSuccess);
    ca_destroy(ctx);
    std::printf("ok batch api frames_checked=%ld\n", g_frames_checked);
}

}  // namespace

int main(int argc, char **argv)
{
    const std::string what = argc > 1 ? argv[1] : "";
    if (what == "serve_sequence")
        scenario_serve_sequence(argc > 2 ? std::atof(argv[2]) : 2.0);
    else if (what == "few_slots")
        scenario_few_slots();
    else if (what == "memory_wait")
        scenario_memory_wait();
    else if (what == "batch_api")
        scenario_batch_api();
    else {
        std::fprintf(stderr, "unknown scenario\n");
        return 2;
    }
    if (!g_allocs.empty()) {
        std::fprintf(stderr, "%zu runtime allocations not freed\n", g_allocs.size());
        return 1;
    }
    std::printf("async operations %ld\n", g_async_ops);
    return 0;
}
