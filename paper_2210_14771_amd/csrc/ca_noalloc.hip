// ca_estimate_area_noalloc: the whole estimate of ca_estimate_area without
// any device allocation, for callers that cannot allocate.  Instead of a
// cached plan (one hipMalloc per batch shape) the call lays its descriptors,
// strip tables, score tables, control words, candidates and attempt-group
// records out in one fixed array in device memory, `scratch`, and runs the
// same kernels over it.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "ca_host.h"

namespace {

constexpr size_t up256(size_t v) { return (v + 255) / 256 * 256; }

// The uploaded part of a call (descriptors, strip tables of at most
// CA_NOALLOC_MAX_SHAPES shapes, score tables, frame list, control words) at
// its largest, in the layout cahost::plan_layout gives it.
constexpr size_t kImageBytes =
    up256(sizeof(ca::FrameDev) * CA_NOALLOC_MAX_FRAMES)
    + up256(sizeof(int32_t) * CA_NOALLOC_MAX_SHAPES * 2 * CA_MAX_STRIPS)
    + up256(sizeof(float) * (CA_SG_CAPACITY + ca::kQtBins + ca::kLumaLevels))
    + up256(sizeof(int32_t) * CA_NOALLOC_MAX_FRAMES)
    + sizeof(uint32_t) * (ca::kCtlFrames + 2 * (size_t)CA_NOALLOC_MAX_FRAMES);
static_assert(kImageBytes < CA_NOALLOC_SCRATCH_BYTES, "scratch smaller than its upload");

constexpr int kMaxDevices = 16;

// One call's device workspace.  Every device the library runs on holds its
// own copy until the process ends; all calls on one device share it.
static __device__ __align__(256) uint8_t scratch[CA_NOALLOC_SCRATCH_BYTES];

struct DeviceSlot {
    std::mutex mu;               // one call at a time builds and uploads the image
    void *ptr = nullptr;         // device address of this device's `scratch`
    hipEvent_t uploaded = nullptr;  // the last upload from `image` has been read
    bool recorded = false;
    cahost::Shape shapes[CA_NOALLOC_MAX_SHAPES];
    alignas(256) uint8_t image[kImageBytes];
};

DeviceSlot g_slots[kMaxDevices];
std::mutex g_setup_mu;

}  // namespace

namespace cahost {

// Once per device, with that device current (called by ca_create): the
// device address of `scratch` (the name itself is only a host-side stand-in)
// and the event that orders reuse of the host image.
int scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return CA_E_DEVICE;
    std::lock_guard<std::mutex> lock(g_setup_mu);
    DeviceSlot &d = g_slots[device];
    if (d.ptr)
        return CA_OK;
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return CA_E_DEVICE;
    }
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return CA_E_DEVICE;
    }
    d.uploaded = ev;
    d.ptr = ptr;
    return CA_OK;
}

}  // namespace cahost

extern "C" int ca_estimate_area_noalloc(ca_ctx *ctx, const uint8_t *frames,
                                        const ca_frame_desc *dims, int32_t n,
                                        const ca_params *params, ca_result *out, void *stream)
{
    using namespace cahost;
    try {
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
        if (n > CA_NOALLOC_MAX_FRAMES)
            return CA_E_SCRATCH;
        if (ctx->device < 0 || ctx->device >= kMaxDevices)
            return CA_E_DEVICE;
        DeviceSlot &d = g_slots[ctx->device];
        if (!d.ptr)
            return CA_E_DEVICE;
        DeviceGuard guard(ctx->device);
        if (!guard.ok)
            return CA_E_DEVICE;
        std::lock_guard<std::mutex> lock(d.mu);
        // the previous call's upload must have read the host image before it
        // is rewritten
        if (d.recorded && hipEventSynchronize(d.uploaded) != hipSuccess)
            return CA_E_DEVICE;
        Plan pl;
        pl.dynamic = true;          // one strip launch over all shapes, nothing cached
        int32_t sg_len = 0;
        const float *lut = cached_tables(ctx, p, &sg_len);
        PlanLayout L;
        rc = plan_layout(ctx, dims, n, p, lut, sg_len, d.shapes, CA_NOALLOC_MAX_SHAPES, &pl, &L,
                         d.image, sizeof(d.image));
        if (rc == CA_E_NOMEM)
            return CA_E_SCRATCH;    // more frame shapes than the scratch holds tables for
        if (rc != CA_OK)
            return rc;
        if (L.total > CA_NOALLOC_SCRATCH_BYTES)
            return CA_E_SCRATCH;
        pl.fused_grid = fused_grid(ctx, pl.fused_lds);
        plan_pointers(&pl, d.ptr, L);
        const hipStream_t s = static_cast<hipStream_t>(stream);
        // descriptors, tables and zeroed control words: one copy ordered
        // before the kernels on the caller's stream
        if (hipMemcpyAsync(d.ptr, d.image, L.image_bytes, hipMemcpyHostToDevice, s) != hipSuccess
            || hipEventRecord(d.uploaded, s) != hipSuccess) {
            (void)hipGetLastError();
            return CA_E_DEVICE;
        }
        d.recorded = true;
        return enqueue(ctx, &pl, frames, n, p, nullptr, nullptr, out, s, false);
    } catch (...) {
        return CA_E_NOMEM;
    }
}
