// Internal interface between the host core (ca_api.cpp) and the gfx950
// kernels (ca_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "contentarea.h"

namespace ca {

constexpr int kBlock = 256;      // threads per workgroup (k_strips_pair: two strips, 2 kBlock)
constexpr size_t kPairLdsMax = 65536;  // LDS bytes the paired strip kernel may take
constexpr int kHalfThreads = 128; // threads per half strip
constexpr int kLanesPerAttempt = 2;   // lanes sharing one RANSAC attempt (fused schedule, and
                                      // the split schedule when a batch fills the device)
constexpr int kMaxLanesPerAttempt = 16;  // small batches spread attempts over more workgroups
// Attempt groups (workgroups) per frame with `lanes` lanes per attempt.
inline int attempt_groups(int attempts, int lanes) { return (attempts * lanes + kBlock - 1) / kBlock; }
constexpr int kChunk = 8;        // most pixels one thread scores per pass (a 1920-pixel line in one pass)
constexpr int kQtBins = 2049;    // pseudo-angle bins, 0 .. 2048
constexpr int kLumaLevels = 256;

// One frame as the kernels see it (32 bytes).
struct FrameDev {
    int64_t offset;   // first byte relative to the frames base
    int32_t W, H;
    int32_t rs;       // row stride in bytes
    int32_t table;    // index of the frame's first strip position in the strip table
    uint64_t uid;     // RNG counter word
};

// Best attempt of one (frame, attempt group).
struct Record {
    uint64_t key;     // (qsum << 16) | (0xFFFF - attempt); 0 = nothing kept
    double cx, cy, r2;
    int32_t inliers;
    int32_t n_points;
    int32_t pad[2];
};

struct StripArgs {
    const uint8_t *frames;
    const FrameDev *fd;
    const int32_t *strips;  // per distinct frame shape: n_h rows then n_v columns
    const float *lut;       // SG[sg_len] | ST[2049] | SI[256]
    ca_point *cand;         // [n_frames][P]
    int32_t sg_len;
    int32_t n_h, n_v;
    int32_t n_items;        // n_frames * (n_h + n_v)
    int32_t per_xcd;        // items per XCD slice (grid = 8 * per_xcd)
    int32_t line_pitch;     // bytes per LDS tile row (>= longest line, multiple of 16)
    int32_t aligned;        // every frame row starts 16-byte aligned
    int32_t frame0;         // first frame of this launch (items cover frames frame0 ..)
    const int32_t *frame_list;  // or the frames of this launch (null: frame0, frame0 + 1, ..)
    int32_t items_per_group;    // strip items one workgroup takes in turn (tables loaded once)
    // With keep set (the handcrafted pass of the learned scorer's fallback),
    // frames whose learned result keep[f] stands under the fallback rule at
    // keep_frac are skipped: their handcrafted result is never used.
    const ca_result *keep = nullptr;
    float keep_frac = 0.0f;
};

struct RansacArgs {
    const FrameDev *fd;
    const ca_point *cand;
    Record *rec;            // [n_frames][groups]
    ca_attempt *dbg;        // optional per-attempt records
    uint64_t seed;
    double t_ri, r_min, r_max, d_max;
    float t_ps;
    int32_t t_px;
    int32_t P;
    int32_t attempts;
    int32_t refine;
    int32_t sampler;
    int32_t groups;         // attempt groups (workgroups of kBlock / lanes attempts) per frame
    int32_t lanes;          // lanes per attempt: 2, 4, 8 or 16
    int32_t frame0;         // first frame of this launch (blockIdx.y counts from it)
    uint32_t *groups_done;  // per frame: groups finished (the last one selects), or null
    const ca_result *keep = nullptr;   // as in StripArgs: frames to skip
    float keep_frac = 0.0f;
};

struct SelectArgs {
    const Record *rec;
    ca_result *out;
    double threshold;       // t_cs * 2^24 * P
    int32_t P;
    int32_t groups;
    int32_t n_frames;
};

// Control words of the fused kernel (zero between calls; the kernel restores
// them before it ends).  Each queue ticket sits on its own 128-byte line.
constexpr int kMaxQueues = 8;
constexpr int kCtlLine = 32;                       // uint32 words per 128 bytes
constexpr int kCtlRetired = kMaxQueues * kCtlLine; // workgroups that have left the loop
constexpr int kCtlError = kCtlRetired + kCtlLine;  // nonzero: a wait hit its spin limit
constexpr int kCtlFrames = kCtlError + kCtlLine;   // strips_done[B] then groups_done[B]

inline size_t ctl_words(int n_frames) { return (size_t)kCtlFrames + 2 * (size_t)n_frames; }

struct FusedArgs {
    StripArgs s;
    RansacArgs r;
    SelectArgs se;
    uint32_t *ctl;
    int32_t nq;             // work queues (frames f with f % nq == q go to queue q)
    int32_t lag;            // frames between a frame's strip items and its RANSAC items
    uint32_t spin_limit;    // polls before a wait gives up and flags an error
};

size_t strip_lds_bytes(int sg_len, int line_pitch);
size_t fused_lds_bytes(int sg_len, int line_pitch);
// start/stop (optional): events the dispatch itself records around the kernel
hipError_t launch_strips(const StripArgs &a, size_t lds_bytes, hipStream_t s,
                         hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
hipError_t launch_ransac(const RansacArgs &a, const SelectArgs &sel, int n_frames, hipStream_t s,
                         hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
hipError_t launch_fused(const FusedArgs &a, int grid, size_t lds_bytes, hipStream_t s,
                        hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
// Serving: fold each run of a batch's results (one stream's frames, in
// sequence order: run = (state index, first, end)) into the stream's
// filtered circle (cx, cy, r, weight); filt[i] = the state after frame i.
hipError_t launch_stream_update(const ca_result *res, const int4 *runs, int n_runs, float4 *state,
                                float4 *filt, float decay, hipStream_t s);
// out[f] = fallback[f] (reason + CA_REASON_FALLBACK) where out[f] has fewer
// than 3 points or inliers < frac * n_points.
hipError_t launch_fallback(ca_result *out, const ca_result *fallback, int n, float frac,
                           hipStream_t s);
hipError_t fused_occupancy(size_t lds_bytes, int *blocks_per_cu);

// Serving: the frame copies of one step into ring slots, in one launch.
// Frame i: `rows` rows of `width` bytes from src (rows `spitch` apart) to
// dst (rows contiguous).  Passed by value (kernel arguments), so the host
// array may be reused as soon as the launch returns.
struct IngestCopy {
    const uint8_t *src;
    uint8_t *dst;
    int64_t spitch;
    int32_t width, rows;
};
constexpr int kMaxIngest = 64;   // copies per launch
struct IngestArgs {
    IngestCopy c[kMaxIngest];
    int32_t n;
};
hipError_t launch_ingest(const IngestArgs &a, hipStream_t s);

}  // namespace ca
