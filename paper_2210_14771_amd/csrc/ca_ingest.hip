// Frame copies of the serving loop: every frame one step of the server
// moves into its stream's ring slot, in one launch.  Each frame is copied by
// its own row of workgroups (blockIdx.y); where source rows are contiguous
// and both ends are 16-byte aligned the frame is copied as a flat run of
// 16-byte words, two per thread and pass, else byte by byte.
#include <algorithm>

#include "ca_internal.h"

namespace ca {
namespace {

constexpr int kIngestUnroll = 2;   // 16-byte words per thread and pass

__global__ __launch_bounds__(kBlock) void k_ingest(IngestArgs a)
{
    const int f = blockIdx.y;
    if (f >= a.n)
        return;
    const IngestCopy c = a.c[f];
    const int64_t total = (int64_t)c.rows * c.width;
    const bool flat = c.spitch == c.width && (reinterpret_cast<uintptr_t>(c.src) & 15) == 0
                      && (reinterpret_cast<uintptr_t>(c.dst) & 15) == 0 && (total & 15) == 0;
    const int64_t step = (int64_t)gridDim.x * kBlock;
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (flat) {
        const uint4 *src = reinterpret_cast<const uint4 *>(c.src);
        uint4 *dst = reinterpret_cast<uint4 *>(c.dst);
        const int64_t n16 = total >> 4;
        for (int64_t i = t; i < n16; i += kIngestUnroll * step) {
            uint4 v[kIngestUnroll];
#pragma unroll
            for (int u = 0; u < kIngestUnroll; ++u) {
                const int64_t k = i + u * step;
                v[u] = src[k < n16 ? k : i];
            }
#pragma unroll
            for (int u = 0; u < kIngestUnroll; ++u) {
                const int64_t k = i + u * step;
                if (k < n16)
                    dst[k] = v[u];
            }
        }
    } else {
        for (int64_t i = t; i < total; i += step) {
            const int64_t row = i / c.width;
            const int64_t col = i - row * c.width;
            c.dst[i] = c.src[row * c.spitch + col];
        }
    }
}

}  // namespace

hipError_t launch_ingest(const IngestArgs &a, hipStream_t s)
{
    if (a.n <= 0)
        return hipSuccess;
    if (a.n > kMaxIngest)
        return hipErrorInvalidValue;
    // workgroups per frame: one pass over the largest frame, at most 2048
    // (a single frame of a real-time step then still fills the device)
    int64_t largest = 0;
    for (int i = 0; i < a.n; ++i)
        largest = std::max(largest, (int64_t)a.c[i].rows * a.c[i].width);
    const int64_t per_pass = (int64_t)kBlock * 16 * kIngestUnroll;
    const int64_t want = (largest + per_pass - 1) / per_pass;
    const int gx = (int)std::min<int64_t>(std::max<int64_t>(want, 1), 2048);
    hipLaunchKernelGGL(k_ingest, dim3(gx, a.n), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace ca
