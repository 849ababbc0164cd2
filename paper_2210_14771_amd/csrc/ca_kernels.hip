// gfx950 kernels of the content-area estimator (arXiv 2210.14771, Section 2.2).
//
// Work units
//   strip item  (frame, strip): stage the strip's three lines as 8-bit luma in
//               LDS, score every pixel of both half strips (Sobel, angle to the
//               image centre, preceding maximum; Eqs. 2-3) and keep the best
//               pixel of each half (Section 2.2.5).  The preceding-maximum scan
//               and the argmax -- the two operations the paper singles out as
//               needing block-wide cooperation (Section 2.2.6) -- are wave64
//               shuffle scans/reductions joined through LDS.
//   RANSAC item (frame, group of 256 attempts): one thread per attempt; the
//               kept points are compacted into LDS and read by broadcast.
//   selection   (frame): merge the best attempt of every group; done by the
//               group that finishes last.
//
// Two schedules run the same units:
//   k_fused     one persistent launch.  Workgroups draw tickets from per-XCD
//               queues in which every frame's strip items precede its RANSAC
//               items (by a lag of a few frames), so memory-bound strip work
//               and ALU-bound RANSAC work share the CUs.  A RANSAC item waits
//               for its frame's strip items; those hold lower tickets of the
//               same queue and never wait, so every wait ends.  The last
//               RANSAC group of a frame selects its circle.
//   k_strips -> k_ransac   two plain launches per batch (or per sub-batch,
//               sub-batches alternating over two streams so that one
//               sub-batch's RANSAC overlaps the next one's strip loads); the
//               last RANSAC group of each frame selects its circle.
//
// Numeric contract (shared with the CPU oracle by definition, not by code):
// integer luma and Sobel, exact integer quantisers for |g| and the angle,
// float32 table lookups and products in a fixed order, float64 circle
// arithmetic without contraction (build with -ffp-contract=off), integer
// inlier moments (summed here in float64, exact below 2^53).
#include "ca_internal.h"
#include "ca_launch.h"

namespace ca {
namespace {

constexpr uint32_t kWave = 64;

// ------------------------------------------------------------ helpers -----

// Device-scope relaxed accesses: they bypass the per-CU L1 and reach the
// coherence point, so data produced by another workgroup (possibly on another
// XCD) is read fresh without invalidating the whole L2.
__device__ __forceinline__ uint64_t load_dev(const uint64_t *p)
{
    return __hip_atomic_load(const_cast<uint64_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t load_dev(const uint32_t *p)
{
    return __hip_atomic_load(const_cast<uint32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_dev(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_dev(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Hand-over between workgroups.  Data that another workgroup reads is
// written with device-scope stores (store_dev: write-through to the
// coherence point) and read with device-scope loads (load_dev), so no L2
// write-back or invalidate is needed: an agent-scope release fence would
// write back the whole L2 of the XCD (buffer_wbl2), which costs more than
// the strip itself.  The writer waits for its stores to complete before the
// workgroup barrier; only then does one thread move the counter.
//
// This relies on the hardware, not on the HIP memory model: the counter
// update is relaxed, not a release, and the reader's loads are relaxed, not
// acquires.  What makes it sound on gfx950: device-scope stores complete at
// the coherence point before s_waitcnt returns, the counter's atomic is
// performed there after them (program order across the barrier), and
// device-scope loads bypass the non-coherent caches, so a reader that sees
// the counter's new value and then loads the data gets what was stored.  A
// compiler or target that reordered relaxed device-scope accesses across the
// wait, or cached them, would break it; the repeated-call and graph-replay
// tests compare every result against the split schedule.
__device__ __forceinline__ void wait_memory() { __builtin_amdgcn_s_waitcnt(0); }
__device__ __forceinline__ uint32_t add_dev(uint32_t *p, uint32_t v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Values that steer control flow around workgroup barriers must be provably
// wave-uniform: a value read from LDS or derived from one is treated as
// per-lane, and a barrier under such a branch or loop lets the compiler
// restructure the flow so that lanes pass a barrier out of step.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint32_t luma_of(uint32_t r, uint32_t g, uint32_t b)
{
    return (77u * r + 150u * g + 29u * b + 128u) >> 8;
}

__device__ __forceinline__ uint32_t wave_incl_max(uint32_t v)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (uint32_t d = 1; d < kWave; d <<= 1) {
        uint32_t t = (uint32_t)__shfl_up((int)v, d, kWave);
        if (lane >= d)
            v = v > t ? v : t;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        uint64_t t = __shfl_xor(v, d, kWave);
        v = v > t ? v : t;
    }
    return v;
}

__device__ __forceinline__ uint64_t pack_point(int x, int y, float s)
{
    return (uint64_t)(uint16_t)(int16_t)x | ((uint64_t)(uint16_t)(int16_t)y << 16)
           | ((uint64_t)__float_as_uint(s) << 32);
}

// s_g * s_theta of one pixel from its Sobel gradient (Eq. 2, quantised).
__device__ __forceinline__ float grad_angle_score(int gx, int gy, int x, int y, int W, int H,
                                                  const float *sg, int sg_last, const float *st)
{
    const int m2 = gx * gx + gy * gy;
    if (m2 == 0)
        return 0.0f;  // SG[0] = 0
    // qg = floor(8 |g|) = isqrt(64 m2): float estimate, then exact correction
    const uint32_t v = (uint32_t)m2 * 64u;
    uint32_t q = (uint32_t)__builtin_amdgcn_sqrtf((float)v);
    if (q * q > v)
        --q;
    if ((q + 1) * (q + 1) <= v)
        ++q;
    const int qg = (int)q < sg_last ? (int)q : sg_last;
    // doubled vector from the pixel to the image centre
    const int c2x = W - 1 - 2 * x;
    const int c2y = H - 1 - 2 * y;
    const int dt = gx * c2x + gy * c2y;
    const int cr = gx * c2y - gy * c2x;
    const uint32_t acr = (uint32_t)(cr < 0 ? -cr : cr);
    const uint32_t adt = (uint32_t)(dt < 0 ? -dt : dt);
    const uint32_t den = acr + adt;
    int qt = 0;
    if (den != 0) {
        // f = floor(1024 acr / den): reciprocal estimate within one of the
        // true quotient (relative error ~2^-21 on a value <= 1024), then an
        // exact integer correction
        const uint64_t num = (uint64_t)acr << 10;
        uint32_t f = (uint32_t)((float)acr * 1024.0f * __builtin_amdgcn_rcpf((float)den));
        uint64_t fd = (uint64_t)f * den;
        if (fd > num) {
            --f;
            fd -= den;
        } else if (fd + den <= num) {
            ++f;
            fd += den;
        }
        qt = dt >= 0 ? (int)f : 2048 - (int)(f + (fd != num ? 1u : 0u));
        qt = qt < 0 ? 0 : (qt > 2048 ? 2048 : qt);
    }
    return sg[qg] * st[qt];
}

// ------------------------------------------------------------ strips ------

// Stage luma of the three lines of a horizontal strip centred on `row`.
__device__ void load_hstrip(const uint8_t *frame, int W, int rs, int row, uint8_t *tile, int LP,
                            bool aligned, int tid, int nthreads)
{
    int x_done = 0;
    if (aligned) {
        // 16 pixels (48 bytes, three 16-byte loads) per work unit
        const int groups = W >> 4;
        for (int t = tid; t < 3 * groups; t += nthreads) {
            const int a = t / groups;
            const int gi = t - a * groups;
            const uint4 *src =
                reinterpret_cast<const uint4 *>(frame + (int64_t)(row - 1 + a) * rs + gi * 48);
            const uint4 q0 = src[0], q1 = src[1], q2 = src[2];
            const uint32_t w[12] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y,
                                    q1.z, q1.w, q2.x, q2.y, q2.z, q2.w};
            uint32_t out[4] = {0, 0, 0, 0};
#pragma unroll
            for (int p = 0; p < 16; ++p) {
                const int b0 = 3 * p;
                const uint32_t r = (w[b0 >> 2] >> (8 * (b0 & 3))) & 0xFFu;
                const uint32_t g = (w[(b0 + 1) >> 2] >> (8 * ((b0 + 1) & 3))) & 0xFFu;
                const uint32_t b = (w[(b0 + 2) >> 2] >> (8 * ((b0 + 2) & 3))) & 0xFFu;
                out[p >> 2] |= luma_of(r, g, b) << (8 * (p & 3));
            }
            *reinterpret_cast<uint4 *>(tile + a * LP + gi * 16) =
                make_uint4(out[0], out[1], out[2], out[3]);
        }
        x_done = groups << 4;
    }
    const int rest = W - x_done;
    for (int t = tid; t < 3 * rest; t += nthreads) {
        const int a = t / rest;
        const int x = x_done + (t - a * rest);
        const uint8_t *px = frame + (int64_t)(row - 1 + a) * rs + 3 * x;
        tile[a * LP + x] = (uint8_t)luma_of(px[0], px[1], px[2]);
    }
}

// Stage luma of row y of the three columns of a vertical strip centred on
// `col` (frame bytes [fstart, fend)).
__device__ __forceinline__ void vstrip_row(const uint8_t *frame, uintptr_t fstart, uintptr_t fend,
                                           int rs, int col, int y, uint8_t *tile, int LP)
{
    const uint8_t *p = frame + (int64_t)y * rs + 3 * (col - 1);
    const uintptr_t addr = reinterpret_cast<uintptr_t>(p);
    const uint32_t sh = (uint32_t)(addr & 3);
    const uintptr_t al = addr - sh;
    uint32_t b03, b47, b8;
    if (al >= fstart && al + 12 <= fend) {
        // the 9 bytes lie inside 3 aligned dwords; extract with v_alignbyte.
        // (pointer arithmetic, not integer casts, keeps the global address space)
        const uint32_t *w = reinterpret_cast<const uint32_t *>(p - sh);
        const uint32_t w0 = w[0], w1 = w[1], w2 = w[2];
        b03 = __builtin_amdgcn_alignbyte(w1, w0, sh);
        b47 = __builtin_amdgcn_alignbyte(w2, w1, sh);
        b8 = (w2 >> (8 * sh)) & 0xFFu;
    } else {
        b03 = (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16)
              | ((uint32_t)p[3] << 24);
        b47 = (uint32_t)p[4] | ((uint32_t)p[5] << 8) | ((uint32_t)p[6] << 16)
              | ((uint32_t)p[7] << 24);
        b8 = p[8];
    }
    tile[0 * LP + y] = (uint8_t)luma_of(b03 & 0xFFu, (b03 >> 8) & 0xFFu, (b03 >> 16) & 0xFFu);
    tile[1 * LP + y] = (uint8_t)luma_of(b03 >> 24, b47 & 0xFFu, (b47 >> 8) & 0xFFu);
    tile[2 * LP + y] = (uint8_t)luma_of((b47 >> 16) & 0xFFu, b47 >> 24, b8);
}

// Stage luma of the three columns of a vertical strip centred on `col`.
__device__ void load_vstrip(const uint8_t *frame, int W, int H, int rs, int col, uint8_t *tile,
                            int LP, int tid)
{
    const uintptr_t fstart = reinterpret_cast<uintptr_t>(frame);
    const uintptr_t fend = fstart + (uintptr_t)((int64_t)(H - 1) * rs + 3 * W);
    for (int y = tid; y < H; y += kBlock)
        vstrip_row(frame, fstart, fend, rs, col, y, tile, LP);
}

// The same for two vertical strips at once, by 2 kBlock threads: lane i of
// the workgroup takes row i / 2 of strip i % 2, so each wavefront's loads
// cover 32 rows of both strips.  Adjacent strips' bytes of a row lie in the
// same DRAM page more often than the bytes of neighbouring rows of one
// strip do: measured, the lines of 64 x 1080p frames' 32 vertical strips
// are read at 6.2 TB/s this way against 5.3 TB/s one strip per workgroup.
// A thread's kPairRows rows are loaded before any is used (unconditional
// loads from a clamped, in-frame address; rows at the frame's edges, or
// past the end, are redone or skipped afterwards), so they are in flight
// together.
constexpr int kPairRows = 4;

__device__ void load_vstrip_pair(const uint8_t *frame, int W, int H, int rs, int col0, int col1,
                                 uint8_t *tile0, int LP, int tid)
{
    const uintptr_t fstart = reinterpret_cast<uintptr_t>(frame);
    const uintptr_t fend = fstart + (uintptr_t)((int64_t)(H - 1) * rs + 3 * W);
    // an aligned 12-byte window inside every frame (frames are >= 16 x 16)
    const uint8_t *safe = frame + ((4u - (uint32_t)(fstart & 3)) & 3u);
    for (int i0 = tid; i0 < 2 * H; i0 += kPairRows * 2 * kBlock) {
        uint32_t w[kPairRows][3];
        uint32_t sh[kPairRows];
        bool fast[kPairRows];
#pragma unroll
        for (int r = 0; r < kPairRows; ++r) {
            const int i = i0 + r * 2 * kBlock;
            const int g = i & 1;
            const int y = (i >> 1) < H ? (i >> 1) : H - 1;
            const uint8_t *p = frame + (int64_t)y * rs + 3 * ((g ? col1 : col0) - 1);
            const uintptr_t addr = reinterpret_cast<uintptr_t>(p);
            sh[r] = (uint32_t)(addr & 3);
            fast[r] = addr - sh[r] >= fstart && addr - sh[r] + 12 <= fend;
            const uint32_t *q = reinterpret_cast<const uint32_t *>(fast[r] ? p - sh[r] : safe);
            w[r][0] = q[0];
            w[r][1] = q[1];
            w[r][2] = q[2];
        }
#pragma unroll
        for (int r = 0; r < kPairRows; ++r) {
            const int i = i0 + r * 2 * kBlock;
            if (i >= 2 * H)
                break;
            const int g = i & 1;
            const int y = i >> 1;
            uint8_t *tile = tile0 + g * (3 * LP);
            if (fast[r]) {
                const uint32_t b03 = __builtin_amdgcn_alignbyte(w[r][1], w[r][0], sh[r]);
                const uint32_t b47 = __builtin_amdgcn_alignbyte(w[r][2], w[r][1], sh[r]);
                const uint32_t b8 = (w[r][2] >> (8 * sh[r])) & 0xFFu;
                tile[0 * LP + y] =
                    (uint8_t)luma_of(b03 & 0xFFu, (b03 >> 8) & 0xFFu, (b03 >> 16) & 0xFFu);
                tile[1 * LP + y] = (uint8_t)luma_of(b03 >> 24, b47 & 0xFFu, (b47 >> 8) & 0xFFu);
                tile[2 * LP + y] = (uint8_t)luma_of((b47 >> 16) & 0xFFu, b47 >> 24, b8);
            } else {
                vstrip_row(frame, fstart, fend, rs, g ? col1 : col0, y, tile, LP);
            }
        }
    }
}

struct StripLds {
    const float *sg, *st, *si;  // score tables (LDS)
    uint8_t *tile;              // 3 x line_pitch luma bytes (LDS)
    uint32_t *scan;             // [4]
    uint64_t *best;             // [4]
};

// One strip item: both half strips of strip s of frame f, by kBlock threads
// (tid: the thread's index among them); with `load` false the strip's tile
// is already staged.  Ends with the two candidates written (device scope)
// and a workgroup barrier.
__device__ void strip_work(const StripArgs &a, const StripLds &c, int f, int s, int tid,
                           bool load = true)
{
    const int S = a.n_h + a.n_v;
    f = uniform(f);
    s = uniform(s);
    const FrameDev d = a.fd[f];
    const uint8_t *frame = a.frames + d.offset;
    const bool horizontal = s < a.n_h;
    const int pos = uniform(a.strips[d.table + s]);
    const int L = uniform(horizontal ? d.W : d.H);
    const int LP = a.line_pitch;
    if (load) {
        if (horizontal)
            load_hstrip(frame, d.W, d.rs, pos, c.tile, LP, a.aligned != 0, tid, kBlock);
        else
            load_vstrip(frame, d.W, d.H, d.rs, pos, c.tile, LP, tid);
    }
    __syncthreads();

    const int half = tid >> 7;
    const int lt = tid & (kHalfThreads - 1);
    const int wv = tid >> 6;
    const uint32_t lane = tid & (kWave - 1);
    const int Lh = half == 0 ? (L >> 1) : L - (L >> 1);
    const int Lmax = L - (L >> 1);
    int chunk = (Lmax + kHalfThreads - 1) / kHalfThreads;
    chunk = chunk < kChunk ? chunk : kChunk;
    const int span = kHalfThreads * chunk;
    const int n_pass = uniform((Lmax + span - 1) / span);
    const int sg_last = a.sg_len - 1;
    const uint8_t *t0 = c.tile, *t1 = c.tile + LP, *t2 = c.tile + 2 * LP;
    const int dir = half == 0 ? 1 : -1;

    uint32_t carry = 0;
    uint64_t best = 0;
    for (int pass = 0; pass < n_pass; ++pass) {
        const int k0 = pass * span + lt * chunk;
        // Columns are read once each, sliding along: column c holds pixel
        // k0 + c - 1 of the half (position clamped to the line, which
        // replicates the end pixels as the Sobel operator needs) as the
        // column sum t0 + 2 t1 + t2, the difference t2 - t0 and t1.  Pixel j
        // sits at column j + 1; its neighbours along the line at columns j and
        // j + 2 (in the second half the pixels at i + 1 and i - 1, hence the
        // sign `dir`).
        auto column = [&](int cc, int &S_, int &D_, uint32_t &M_) {
            int x = half == 0 ? k0 + cc - 1 : L - k0 - cc;
            x = x < 0 ? 0 : (x > L - 1 ? L - 1 : x);
            const int a0 = t0[x], a1 = t1[x], a2 = t2[x];
            S_ = a0 + 2 * a1 + a2;
            D_ = a2 - a0;
            M_ = (uint32_t)a1;
        };
        int S0, S1, D0, D1;
        uint32_t M0, M1;
        column(0, S0, D0, M0);
        column(1, S1, D1, M1);
        float part[kChunk];
        uint32_t lum[kChunk];
        uint32_t tmax = 0;
#pragma unroll
        for (int j = 0; j < kChunk; ++j) {
            part[j] = 0.0f;
            lum[j] = 0;
            int S2, D2;
            uint32_t M2;
            column(j + 2, S2, D2, M2);
            const int along = dir * (S2 - S0);
            const int across = D0 + 2 * D1 + D2;
            const uint32_t y1 = M1;
            S0 = S1;
            S1 = S2;
            D0 = D1;
            D1 = D2;
            M1 = M2;
            const int k = k0 + j;
            if (j < chunk && k < Lh) {
                const int i = half == 0 ? k : L - 1 - k;
                part[j] = horizontal
                              ? grad_angle_score(along, across, i, pos, d.W, d.H, c.sg, sg_last, c.st)
                              : grad_angle_score(across, along, pos, i, d.W, d.H, c.sg, sg_last, c.st);
                lum[j] = y1;
                tmax = tmax > y1 ? tmax : y1;
            }
        }
        // exclusive max-scan of the chunk maxima over the 128 threads of this half
        const uint32_t incl = wave_incl_max(tmax);
        uint32_t excl = (uint32_t)__shfl_up((int)incl, 1, kWave);
        if (lane == 0)
            excl = 0;
        if (lane == kWave - 1)
            c.scan[wv] = incl;
        __syncthreads();
        const uint32_t w0 = c.scan[2 * half], w1 = c.scan[2 * half + 1];
        if (wv & 1)
            excl = excl > w0 ? excl : w0;
        uint32_t run = carry > excl ? carry : excl;
        const uint32_t tot = w0 > w1 ? w0 : w1;
        carry = carry > tot ? carry : tot;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kChunk; ++j) {
            const int k = k0 + j;
            if (j < chunk && k < Lh) {
                const float sc = part[j] * c.si[run];
                const uint64_t key = ((uint64_t)__float_as_uint(sc) << 32)
                                     | (uint64_t)(0xFFFFFFFFu - (uint32_t)k);
                best = best > key ? best : key;
                run = run > lum[j] ? run : lum[j];
            }
        }
    }
    best = wave_max_u64(best);
    if (lane == 0)
        c.best[wv] = best;
    __syncthreads();
    if (lt == 0) {
        const uint64_t b0 = c.best[2 * half], b1 = c.best[2 * half + 1];
        const uint64_t bb = b0 > b1 ? b0 : b1;
        const int k = (int)(0xFFFFFFFFu - (uint32_t)bb);
        const int i = half == 0 ? k : L - 1 - k;
        const float sc = __uint_as_float((uint32_t)(bb >> 32));
        store_dev(reinterpret_cast<uint64_t *>(a.cand + (int64_t)f * (2 * S) + 2 * s + half),
                  pack_point(horizontal ? i : pos, horizontal ? pos : i, sc));
        wait_memory();
    }
    __syncthreads();
}

// ------------------------------------------------------------ RANSAC ------

// Kept points of one frame in LDS, compacted in canonical order and padded
// to a multiple of the lanes per attempt with far-away points whose moments
// are zero (never inside a band, so they add nothing).
struct Lds {
    double2 uv[kBlock];     // shifted coordinates u, v
    double2 m1[kBlock];     // u^2, u v
    double2 m2[kBlock];     // v^2, floor(score * 2^24)
    double2 m3[kBlock];     // u z, v z  (z = u^2 + v^2)
    int iu[kBlock], iv[kBlock];
    int wcount[4];
    uint64_t wbest[4];
};

__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    // Salmon et al., SC'11: Philox4x64 with 10 rounds
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        const uint64_t n0 = hi1 ^ c[1] ^ k0;
        const uint64_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

__device__ __forceinline__ int below(uint64_t u, int k)
{
    return (int)(((u >> 32) * (uint64_t)(uint32_t)k) >> 32);
}

__device__ bool pick_triple(const RansacArgs &a, uint64_t uid, int att, int n, int t[3])
{
    if (a.sampler == 0) {
        uint64_t c[4] = {(uint64_t)(uint32_t)att, uid, 0, 0};
        philox4x64_10(c, a.seed, 0);
        const int i0 = below(c[0], n);
        int i1 = below(c[1], n - 1);
        i1 += i1 >= i0;
        const int lo = i0 < i1 ? i0 : i1, hi = i0 < i1 ? i1 : i0;
        int i2 = below(c[2], n - 2);
        i2 += i2 >= lo;
        i2 += i2 >= hi;
        t[0] = i0;
        t[1] = i1;
        t[2] = i2;
        return true;
    }
    // lexicographic enumeration: the att-th triple i < j < k
    int64_t r = att;
    for (int i = 0; i < n - 2; ++i) {
        const int64_t cnt = (int64_t)(n - 1 - i) * (n - 2 - i) / 2;
        if (r >= cnt) {
            r -= cnt;
            continue;
        }
        for (int j = i + 1; j < n - 1; ++j) {
            const int64_t cj = n - 1 - j;
            if (r >= cj) {
                r -= cj;
                continue;
            }
            t[0] = i;
            t[1] = j;
            t[2] = j + 1 + (int)r;
            return true;
        }
    }
    return false;
}

struct Band {
    double cx, cy, lo2, hi2;
};

__device__ __forceinline__ Band make_band(double cx, double cy, double r2, double t)
{
    Band b;
    const double r = sqrt(r2);
    const double hi = r + t;
    b.cx = cx;
    b.cy = cy;
    b.hi2 = hi * hi;
    if (r > t) {
        const double lo = r - t;
        b.lo2 = lo * lo;
    } else {
        b.lo2 = -1.0;
    }
    return b;
}

// Sum over the lanes of one attempt (adjacent lanes of a quad).  The partial
// sums are integers below 2^53, so every order gives the same exact total.
template <int kCtrl>
__device__ __forceinline__ double quad_xor(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), kCtrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), kCtrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int LANES>
__device__ __forceinline__ double lane_sum(double v)
{
    static_assert(LANES == 2 || LANES == 4 || LANES == 8 || LANES == 16, "attempt lanes");
    v += quad_xor<0xB1>(v);  // quad_perm [1, 0, 3, 2]
    if (LANES >= 4)
        v += quad_xor<0x4E>(v);  // quad_perm [2, 3, 0, 1]
    if (LANES >= 8)
        v += __shfl_xor(v, 4, 64);
    if (LANES >= 16)
        v += __shfl_xor(v, 8, 64);
    return v;
}

__device__ __forceinline__ double in_band(const double2 p, const Band &b)
{
    const double du = p.x - b.cx;
    const double dv = p.y - b.cy;
    const double d2 = du * du + dv * dv;
    return (b.lo2 <= d2 && d2 <= b.hi2) ? 1.0 : 0.0;
}

// Inlier moments of one band: count, sum u, v, u^2, u v, v^2, u z, v z.
struct Moments {
    double m, su, sv, suu, suv, svv, suz, svz;
};

// Lane `sub` of the attempt takes points sub, sub + LANES, ...;
// nk = padded point count / LANES (wave-uniform).
template <int LANES>
__device__ Moments band_moments(const Lds &L, int nk, int sub, const Band &b)
{
    Moments s = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = 0; k < nk; ++k) {
        const int i = k * LANES + sub;
        const double2 p = L.uv[i];
        const double w = in_band(p, b);
        const double2 m1 = L.m1[i], m2 = L.m2[i], m3 = L.m3[i];
        s.m += w;
        s.su = fma(w, p.x, s.su);
        s.sv = fma(w, p.y, s.sv);
        s.suu = fma(w, m1.x, s.suu);
        s.suv = fma(w, m1.y, s.suv);
        s.svv = fma(w, m2.x, s.svv);
        s.suz = fma(w, m3.x, s.suz);
        s.svz = fma(w, m3.y, s.svz);
    }
    s.m = lane_sum<LANES>(s.m);
    s.su = lane_sum<LANES>(s.su);
    s.sv = lane_sum<LANES>(s.sv);
    s.suu = lane_sum<LANES>(s.suu);
    s.suv = lane_sum<LANES>(s.suv);
    s.svv = lane_sum<LANES>(s.svv);
    s.suz = lane_sum<LANES>(s.suz);
    s.svz = lane_sum<LANES>(s.svz);
    return s;
}

// Coope least-squares circle from the inlier moments (Section 2.2.5).  The
// centred sums C = m S_ab - S_a S_b are integers; with kExact (every product
// below 2^53 for this frame's coordinate range and point count) they are
// formed in float64, where each product and difference is exact, otherwise in
// int64.  Both give the same doubles.  The sum of z is S_uu + S_vv.
template <bool kExact>
__device__ bool coope_solve(const Moments &s, double &cx, double &cy, double &r2)
{
    if (s.m < 3.0)
        return false;
    const double m = s.m;
    const double sz = s.suu + s.svv;
    double Cuu, Cuv, Cvv, Cuz, Cvz;
    if (kExact) {
        Cuu = m * s.suu - s.su * s.su;
        Cuv = m * s.suv - s.su * s.sv;
        Cvv = m * s.svv - s.sv * s.sv;
        Cuz = m * s.suz - s.su * sz;
        Cvz = m * s.svz - s.sv * sz;
    } else {
        const int64_t im = (int64_t)s.m, su = (int64_t)s.su, sv = (int64_t)s.sv;
        const int64_t suu = (int64_t)s.suu, svv = (int64_t)s.svv, isz = suu + svv;
        Cuu = (double)(im * suu - su * su);
        Cuv = (double)(im * (int64_t)s.suv - su * sv);
        Cvv = (double)(im * svv - sv * sv);
        Cuz = (double)(im * (int64_t)s.suz - su * isz);
        Cvz = (double)(im * (int64_t)s.svz - sv * isz);
    }
    const double det = Cuu * Cvv - Cuv * Cuv;
    if (det == 0.0)
        return false;
    const double A = (Cuz * Cvv - Cvz * Cuv) / det;
    const double B = (Cvz * Cuu - Cuz * Cuv) / det;
    cx = A / 2.0;
    cy = B / 2.0;
    const double mu = s.su / m;
    const double mv = s.sv / m;
    const double var = (Cuu + Cvv) / (m * m);
    r2 = (var + (mu - cx) * (mu - cx)) + (mv - cy) * (mv - cy);
    return true;
}

// One attempt (Section 2.2.5): draw a triple, circle through it, `refine`
// inlier passes with least-squares refits, then count the inliers and their
// score sum and apply the circle limits.  `key` is set for kept circles (on
// the attempt's first lane).
template <bool kExact, int LANES>
__device__ void run_attempt(const RansacArgs &a, const Lds &L, const FrameDev &d, int n, int nk,
                            int sub, int att, bool active, ca_attempt &rec, uint64_t &key)
{
    const int ox = d.W / 2, oy = d.H / 2;
    if (n >= 3 && active) {
        int t[3];
        if (!pick_triple(a, d.uid, att, n, t)) {
            rec.i0 = rec.i1 = rec.i2 = -1;
            rec.fail_stage = -1;
        } else {
            rec.i0 = t[0];
            rec.i1 = t[1];
            rec.i2 = t[2];
            const int64_t x0 = L.iu[t[0]], x1 = L.iu[t[1]], x2 = L.iu[t[2]];
            const int64_t y0 = L.iv[t[0]], y1 = L.iv[t[1]], y2 = L.iv[t[2]];
            const int64_t D = 2 * (x0 * (y1 - y2) + x1 * (y2 - y0) + x2 * (y0 - y1));
            bool ok = D != 0;
            double cx = 0, cy = 0, r2 = 0;
            if (ok) {
                const int64_t z0 = x0 * x0 + y0 * y0, z1 = x1 * x1 + y1 * y1, z2 = x2 * x2 + y2 * y2;
                const int64_t Nx = z0 * (y1 - y2) + z1 * (y2 - y0) + z2 * (y0 - y1);
                const int64_t Ny = z0 * (x2 - x1) + z1 * (x0 - x2) + z2 * (x1 - x0);
                cx = (double)Nx / (double)D;
                cy = (double)Ny / (double)D;
                const double ddx = (double)x0 - cx, ddy = (double)y0 - cy;
                r2 = ddx * ddx + ddy * ddy;
                for (int k = 1; k <= a.refine; ++k) {
                    const Band bd = make_band(cx, cy, r2, a.t_ri);
                    if (!coope_solve<kExact>(band_moments<LANES>(L, nk, sub, bd), cx, cy, r2)) {
                        rec.fail_stage = k;
                        ok = false;
                        break;
                    }
                }
            }
            if (ok) {
                const Band bd = make_band(cx, cy, r2, a.t_ri);
                double cnt = 0, qs = 0;
                for (int k = 0; k < nk; ++k) {
                    const int i = k * LANES + sub;
                    const double w = in_band(L.uv[i], bd);
                    cnt += w;
                    qs = fma(w, L.m2[i].y, qs);
                }
                cnt = lane_sum<LANES>(cnt);
                qs = lane_sum<LANES>(qs);
                const double acx = (double)ox + cx;
                const double acy = (double)oy + cy;
                const double r = sqrt(r2);
                const double ex = acx - (double)(d.W - 1) / 2.0;
                const double ey = acy - (double)(d.H - 1) / 2.0;
                const double dlim = a.d_max * (double)d.W;
                const bool kept = r >= a.r_min * (double)d.W && r <= a.r_max * (double)d.W
                                  && ex * ex + ey * ey <= dlim * dlim;
                rec.status = kept ? 2 : 1;
                rec.inliers = (int32_t)cnt;
                rec.qsum = (uint64_t)qs;
                rec.cx = acx;
                rec.cy = acy;
                rec.r2 = r2;
                if (kept && sub == 0)
                    key = (rec.qsum << 16) | (uint64_t)(0xFFFFu - (uint32_t)att);
            }
        }
    }
}

// One RANSAC item: attempts [g * A, g * A + A) of frame f (A = kBlock /
// LANES), LANES lanes per attempt.  Writes the group's best attempt to its
// record (device scope) and ends with a barrier.
template <int LANES>
__device__ void ransac_work(const RansacArgs &a, Lds &L, int f, int g)
{
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = tid >> 6;
    f = uniform(f);
    g = uniform(g);
    const FrameDev d = a.fd[f];
    const int ox = d.W / 2, oy = d.H / 2;

    // filter (Section 2.2.5) and stable compaction in canonical order
    bool keep = false;
    int x = 0, y = 0;
    float sc = 0.0f;
    if (tid < a.P) {
        const uint64_t pt = load_dev(reinterpret_cast<const uint64_t *>(a.cand + (int64_t)f * a.P + tid));
        x = (int16_t)(uint16_t)(pt & 0xFFFFu);
        y = (int16_t)(uint16_t)((pt >> 16) & 0xFFFFu);
        sc = __uint_as_float((uint32_t)(pt >> 32));
        int ed = x < y ? x : y;
        ed = ed < d.W - 1 - x ? ed : d.W - 1 - x;
        ed = ed < d.H - 1 - y ? ed : d.H - 1 - y;
        keep = ed >= a.t_px && sc >= a.t_ps;
    }
    const uint64_t ball = __ballot(keep);
    const int before = __popcll(ball & ((1ull << lane) - 1ull));
    if (lane == 0)
        L.wcount[wv] = __popcll(ball);
    __syncthreads();
    int base = 0;
    for (int w = 0; w < wv; ++w)
        base += L.wcount[w];
    const int n = uniform(L.wcount[0] + L.wcount[1] + L.wcount[2] + L.wcount[3]);
    const int nk = (n + LANES - 1) / LANES;
    if (keep) {
        const int j = base + before;
        const int u = x - ox, v = y - oy;
        const double du = (double)u, dv = (double)v;
        const double z = (double)((int64_t)u * u + (int64_t)v * v);
        L.iu[j] = u;
        L.iv[j] = v;
        L.uv[j] = make_double2(du, dv);
        L.m1[j] = make_double2((double)((int64_t)u * u), (double)((int64_t)u * v));
        L.m2[j] = make_double2((double)((int64_t)v * v), (double)(uint32_t)(sc * 16777216.0f));
        L.m3[j] = make_double2(du * z, dv * z);
    }
    if (tid >= n && tid < nk * LANES) {
        // padding: squared distance ~1e300 exceeds every band's outer radius
        L.uv[tid] = make_double2(1e150, 1e150);
        L.m1[tid] = make_double2(0.0, 0.0);
        L.m2[tid] = make_double2(0.0, 0.0);
        L.m3[tid] = make_double2(0.0, 0.0);
    }
    __syncthreads();

    // every centred product below 2^53: float64 arithmetic is exact
    const double U = (double)(ox > d.W - 1 - ox ? ox : d.W - 1 - ox);
    const double V = (double)(oy > d.H - 1 - oy ? oy : d.H - 1 - oy);
    const bool exact =
        uniform((double)n * (double)n * (U > V ? U : V) * (U * U + V * V) < 0x1p52 ? 1 : 0) != 0;

    const int sub = tid & (LANES - 1);
    const int att = g * (kBlock / LANES) + tid / LANES;
    const bool active = att < a.attempts;
    uint64_t key = 0;
    ca_attempt rec = {};
    if (exact)
        run_attempt<true, LANES>(a, L, d, n, nk, sub, att, active, rec, key);
    else
        run_attempt<false, LANES>(a, L, d, n, nk, sub, att, active, rec, key);
    if (a.dbg && active && sub == 0)
        a.dbg[(int64_t)f * a.attempts + att] = rec;

    // best kept attempt of this group: keys are unique per attempt
    const uint64_t wmax = wave_max_u64(key);
    if (lane == 0)
        L.wbest[wv] = wmax;
    __syncthreads();
    uint64_t bmax = L.wbest[0];
    for (int w = 1; w < 4; ++w)
        bmax = bmax > L.wbest[w] ? bmax : L.wbest[w];
    uint64_t *out = reinterpret_cast<uint64_t *>(a.rec + (int64_t)f * a.groups + g);
    const bool writer = bmax == 0 ? tid == 0 : key == bmax;
    if (writer) {
        store_dev(out + 0, bmax);
        store_dev(out + 1, (uint64_t)__double_as_longlong(bmax ? rec.cx : 0.0));
        store_dev(out + 2, (uint64_t)__double_as_longlong(bmax ? rec.cy : 0.0));
        store_dev(out + 3, (uint64_t)__double_as_longlong(bmax ? rec.r2 : 0.0));
        store_dev(out + 4, (uint64_t)(uint32_t)(bmax ? rec.inliers : 0)
                               | ((uint64_t)(uint32_t)n << 32));
        wait_memory();
    }
    __syncthreads();
}

// Best circle of frame f from its groups' records (Section 2.2.5, last step).
__device__ void select_frame(const SelectArgs &a, int f)
{
    const uint64_t *r = reinterpret_cast<const uint64_t *>(a.rec + (int64_t)f * a.groups);
    constexpr int kWords = sizeof(Record) / sizeof(uint64_t);
    int best = 0;
    uint64_t bkey = load_dev(r);
    for (int g = 1; g < a.groups; ++g) {
        const uint64_t k = load_dev(r + (int64_t)g * kWords);
        if (k > bkey) {
            bkey = k;
            best = g;
        }
    }
    const uint64_t *rb = r + (int64_t)best * kWords;
    const uint64_t w4 = load_dev(rb + 4);
    ca_result o = {};
    o.n_points = (int32_t)(uint32_t)(w4 >> 32);
    if (o.n_points < 3) {
        o.reason = 1;
    } else if (bkey == 0) {
        o.reason = 2;
    } else {
        const uint64_t qsum = bkey >> 16;
        const double cx = __longlong_as_double((long long)load_dev(rb + 1));
        const double cy = __longlong_as_double((long long)load_dev(rb + 2));
        const double r2 = __longlong_as_double((long long)load_dev(rb + 3));
        o.cx = (float)cx;
        o.cy = (float)cy;
        o.r = (float)sqrt(r2);
        o.score = (float)((double)qsum / (16777216.0 * (double)a.P));
        o.inliers = (int32_t)(uint32_t)w4;
        o.valid = (double)qsum >= a.threshold ? 1 : 0;
        o.reason = o.valid ? 0 : 3;
    }
    a.out[f] = o;
}

// ------------------------------------------------------------ kernels -----

__device__ StripLds carve_strip_lds(uint8_t *smem, int sg_len, uint32_t *scan, uint64_t *best)
{
    // offsets from the LDS base (no integer casts: they would turn LDS
    // accesses into generic ones)
    StripLds c;
    float *sg = reinterpret_cast<float *>(smem);
    c.sg = sg;
    c.st = sg + sg_len;
    c.si = sg + sg_len + kQtBins;
    const int tables = (sg_len + kQtBins + kLumaLevels) * (int)sizeof(float);
    c.tile = smem + ((tables + 15) & ~15);
    c.scan = scan;
    c.best = best;
    return c;
}

__device__ void load_tables(const StripArgs &a, uint8_t *smem, int nthreads = kBlock)
{
    float *dst = reinterpret_cast<float *>(smem);
    const int lut_n = a.sg_len + kQtBins + kLumaLevels;
    for (int i = threadIdx.x; i < lut_n; i += nthreads)
        dst[i] = a.lut[i];
}

// The fallback rule of the learned scorer: a frame keeps its learned result
// unless its best circle explains fewer than `frac` of its kept points, or
// fewer than three points were kept.  k_fallback applies it; the handcrafted
// pass before it skips the frames it keeps, by the same expression.
__device__ __forceinline__ bool learned_kept(const ca_result &r, float frac)
{
    return !(r.n_points < 3 || (float)r.inliers < frac * (float)r.n_points);
}

__global__ __launch_bounds__(kBlock) void k_strips(StripArgs a)
{
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ uint32_t s_scan[4];
    __shared__ uint64_t s_best[4];
    // XCD-aware order: workgroups are dispatched round-robin over the 8 XCDs,
    // so workgroup b runs on XCD b % 8; give each XCD a contiguous slice of
    // (frame, strip) items so one frame's strips share that XCD's L2.
    // A workgroup takes items_per_group consecutive items (a strip tile):
    // the score tables are staged in LDS once for all of them.
    const int b = blockIdx.x;
    const int first = ((b & 7) * a.per_xcd + (b >> 3)) * a.items_per_group;
    if (first >= a.n_items)
        return;
    const int S0 = a.n_h + a.n_v;
    if (a.keep && a.items_per_group == 1) {
        const int k = first / S0;
        if (learned_kept(a.keep[a.frame_list ? a.frame_list[k] : a.frame0 + k], a.keep_frac))
            return;
    }
    load_tables(a, smem);
    const int S = a.n_h + a.n_v;
    const StripLds c = carve_strip_lds(smem, a.sg_len, s_scan, s_best);
    for (int j = 0; j < a.items_per_group; ++j) {
        const int item = first + j;
        if (item >= a.n_items)
            break;
        const int k = item / S;
        const int f = a.frame_list ? a.frame_list[k] : a.frame0 + k;
        if (a.keep && learned_kept(a.keep[f], a.keep_frac))
            continue;
        strip_work(a, c, f, item % S, threadIdx.x);
    }
}

// Strip items two at a time: workgroup item = (frame, pair of strips 2p and
// 2p + 1; n_h even, so a pair is two rows or two columns), 2 kBlock threads,
// the two halves each scoring one strip as strip_work does.  The columns of
// a vertical pair are loaded together (load_vstrip_pair); horizontal strips
// are loaded by their own halves.  Both halves pass the same barriers: their
// strips have the same length.
__global__ __launch_bounds__(2 * kBlock) void k_strips_pair(StripArgs a)
{
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ uint32_t s_scan[2][4];
    __shared__ uint64_t s_best[2][4];
    const int b = blockIdx.x;
    const int item = (b & 7) * a.per_xcd + (b >> 3);
    if (item >= a.n_items)
        return;
    const int pairs = (a.n_h + a.n_v) >> 1;
    const int k = item / pairs;
    const int pr = item - k * pairs;
    const int f = uniform(a.frame_list ? a.frame_list[k] : a.frame0 + k);
    if (a.keep && learned_kept(a.keep[f], a.keep_frac))
        return;
    load_tables(a, smem, 2 * kBlock);
    const int g = threadIdx.x / kBlock;
    const int lt = threadIdx.x - g * kBlock;
    StripLds c = carve_strip_lds(smem, a.sg_len, s_scan[g], s_best[g]);
    const int LP = a.line_pitch;
    uint8_t *tile0 = c.tile;
    c.tile = tile0 + g * (3 * LP);
    const int s0 = 2 * pr;
    if (s0 >= a.n_h) {
        const FrameDev d = a.fd[f];
        const int col0 = uniform(a.strips[d.table + s0]);
        const int col1 = uniform(a.strips[d.table + s0 + 1]);
        load_vstrip_pair(a.frames + d.offset, d.W, d.H, d.rs, col0, col1, tile0, LP, threadIdx.x);
        strip_work(a, c, f, s0 + g, lt, false);
    } else {
        strip_work(a, c, f, s0 + g, lt, true);
    }
}

// RANSAC groups of frames frame0 .. frame0 + gridDim.y - 1; the last group
// of a frame to finish selects its circle and rearms the frame's counter.
template <int LANES>
__global__ __launch_bounds__(kBlock) void k_ransac(RansacArgs a, SelectArgs sel)
{
    __shared__ Lds L;
    __shared__ int s_last;
    const int f = a.frame0 + (int)blockIdx.y;
    if (a.keep && learned_kept(a.keep[f], a.keep_frac))
        return;   // no group of this frame counts or selects
    ransac_work<LANES>(a, L, f, blockIdx.x);
    if (threadIdx.x == 0)
        s_last = add_dev(a.groups_done + f, 1u) == (uint32_t)(a.groups - 1);
    __syncthreads();
    if (uniform(s_last) && threadIdx.x == 0) {
        select_frame(sel, f);
        store_dev(a.groups_done + f, 0u);
    }
}

struct Ticket {
    int kind;  // 0 strip item, 1 RANSAC item, -1 none left
    int f;     // frame
    int idx;   // strip or attempt group
};

// Queue q serves frames q, q + nq, ...; slot t holds the strip items of its
// t-th frame followed by the RANSAC items of its (t - lag)-th frame.
__device__ Ticket decode_ticket(int k, int q, int nq, int B, int S, int G, int lag)
{
    Ticket tk = {-1, 0, 0};
    const int Bq = (B - q + nq - 1) / nq;
    const int Lg = lag < Bq ? lag : Bq;
    const int a_end = Lg * S;
    const int b_end = a_end + (Bq - Lg) * (S + G);
    const int c_end = b_end + Lg * G;
    int j;
    if (k < a_end) {
        j = k / S;
        tk.kind = 0;
        tk.idx = k - j * S;
    } else if (k < b_end) {
        const int kk = k - a_end;
        const int slot = Lg + kk / (S + G);
        const int r = kk - (slot - Lg) * (S + G);
        if (r < S) {
            j = slot;
            tk.kind = 0;
            tk.idx = r;
        } else {
            j = slot - Lg;
            tk.kind = 1;
            tk.idx = r - S;
        }
    } else if (k < c_end) {
        const int kk = k - b_end;
        j = Bq - Lg + kk / G;
        tk.kind = 1;
        tk.idx = kk - (kk / G) * G;
    } else {
        return tk;
    }
    tk.f = q + j * nq;
    return tk;
}

__global__ __launch_bounds__(kBlock) void k_fused(FusedArgs a)
{
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ uint32_t s_scan[4];
    __shared__ uint64_t s_best[4];
    __shared__ int s_ticket;
    __shared__ int s_last;
    const int tid = threadIdx.x;
    const int S = a.s.n_h + a.s.n_v;
    const int G = a.r.groups;
    const int B = a.se.n_frames;
    const int q = (int)(blockIdx.x % (unsigned)a.nq);
    uint32_t *strips_done = a.ctl + kCtlFrames;
    uint32_t *groups_done = a.r.groups_done;

    load_tables(a.s, smem);
    const StripLds c = carve_strip_lds(smem, a.s.sg_len, s_scan, s_best);
    Lds &L = *reinterpret_cast<Lds *>(c.tile);
    // a workgroup can never legitimately take more items than its queue holds
    const int Bq = (B - q + a.nq - 1) / a.nq;
    const int max_items = Bq * (S + G);

    for (int taken = 0;; ++taken) {
        if (taken > max_items) {
            if (tid == 0)
                store_dev(a.ctl + kCtlError, 2u);
            break;
        }
        // The barrier before the ticket fetch keeps the single-thread work
        // that ends an item apart from the single-thread fetch that starts
        // the next one; merged across the loop edge they let the compiler
        // run other lanes into the next barrier before the fetch.
        __syncthreads();
        if (tid == 0)
            s_ticket = (int)atomicAdd(a.ctl + q * kCtlLine, 1u);
        __syncthreads();
        const Ticket tk = decode_ticket(uniform(s_ticket), q, a.nq, B, S, G, a.lag);
        if (tk.kind < 0)
            break;
        if (tk.kind == 0) {
            strip_work(a.s, c, tk.f, tk.idx, threadIdx.x);
            if (tid == 0)
                add_dev(strips_done + tk.f, 1u);
        } else {
            if (tid == 0) {
                // the frame's strip items hold lower tickets of this queue and
                // never wait, so this wait ends; the limit only guards bugs
                uint32_t polls = 0;
                while (load_dev(strips_done + tk.f) < (uint32_t)S) {
                    __builtin_amdgcn_s_sleep(1);
                    if (++polls > a.spin_limit) {
                        store_dev(a.ctl + kCtlError, 1u);
                        break;
                    }
                }
            }
            __syncthreads();
            ransac_work<kLanesPerAttempt>(a.r, L, tk.f, tk.idx);
            if (tid == 0)
                s_last = add_dev(groups_done + tk.f, 1u) == (uint32_t)(G - 1);
            __syncthreads();
            if (uniform(s_last) && tid == 0) {
                select_frame(a.se, tk.f);
                // every group of this frame has finished: rearm its counters
                store_dev(strips_done + tk.f, 0u);
                store_dev(groups_done + tk.f, 0u);
            }
        }
    }
    // the last workgroup out rearms the queues for the next call
    if (tid == 0 && atomicAdd(a.ctl + kCtlRetired, 1u) == gridDim.x - 1) {
        for (int k = 0; k < kMaxQueues; ++k)
            store_dev(a.ctl + k * kCtlLine, 0u);
        store_dev(a.ctl + kCtlRetired, 0u);
    }
}

// Learned-scorer fallback: a frame whose best circle explains less than
// `frac` of its kept points takes the handcrafted pipeline's result.
__global__ __launch_bounds__(kBlock) void k_fallback(ca_result *out, const ca_result *fb, int n,
                                                     float frac)
{
    const int f = blockIdx.x * kBlock + threadIdx.x;
    if (f >= n)
        return;
    if (!learned_kept(out[f], frac)) {
        ca_result b = fb[f];
        b.reason += CA_REASON_FALLBACK;
        out[f] = b;
    }
}

// Temporal filter of the serving loop: w' = decay w + q, c' = (decay w c +
// q c_frame) / w' for a valid result of score q; w' = decay w otherwise.
__global__ __launch_bounds__(kBlock) void k_stream_update(const ca_result *res, const int4 *runs,
                                                          int n_runs, float4 *state, float4 *filt,
                                                          float decay)
{
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= n_runs)
        return;
    const int4 run = runs[r];
    float4 st = state[run.x];
    for (int i = run.y; i < run.z; ++i) {
        const ca_result q = res[i];
        const float w = decay * st.w;
        if (q.valid && q.score > 0.0f) {
            const float wn = w + q.score;
            st.x = (w * st.x + q.score * q.cx) / wn;
            st.y = (w * st.y + q.score * q.cy) / wn;
            st.z = (w * st.z + q.score * q.r) / wn;
            st.w = wn;
        } else {
            st.w = w;
        }
        filt[i] = st;
    }
    state[run.x] = st;
}

}  // namespace

size_t strip_lds_bytes(int sg_len, int line_pitch)
{
    return (size_t)(sg_len + kQtBins + kLumaLevels) * sizeof(float) + 16 + 3 * (size_t)line_pitch;
}

size_t fused_lds_bytes(int sg_len, int line_pitch)
{
    const size_t tile = 3 * (size_t)line_pitch;
    const size_t work = tile > sizeof(Lds) ? tile : sizeof(Lds);
    return (size_t)(sg_len + kQtBins + kLumaLevels) * sizeof(float) + 16 + work;
}

hipError_t launch_strips(const StripArgs &a, size_t lds_bytes, hipStream_t s, hipEvent_t start,
                         hipEvent_t stop)
{
    if (a.n_items <= 0)
        return hipSuccess;
    // strips in pairs when both counts are even, one item per workgroup, and
    // the second tile fits the LDS a workgroup may take without opting in
    const size_t pair_lds = lds_bytes + 3 * (size_t)a.line_pitch;
    if (a.items_per_group == 1 && a.n_h % 2 == 0 && a.n_v % 2 == 0 && pair_lds <= kPairLdsMax) {
        StripArgs p = a;
        p.n_items = a.n_items / 2;
        p.per_xcd = (p.n_items + 7) / 8;
        launch_maybe_timed(k_strips_pair, dim3(8 * p.per_xcd), dim3(2 * kBlock), pair_lds, s, start,
                           stop, p);
        return hipGetLastError();
    }
    launch_maybe_timed(k_strips, dim3(8 * a.per_xcd), dim3(kBlock), lds_bytes, s, start, stop, a);
    return hipGetLastError();
}

hipError_t launch_ransac(const RansacArgs &a, const SelectArgs &sel, int n_frames, hipStream_t s,
                         hipEvent_t start, hipEvent_t stop)
{
    if (n_frames <= 0)
        return hipSuccess;
    const dim3 grid(a.groups, n_frames);
    switch (a.lanes) {
    case 2:
        launch_maybe_timed(k_ransac<2>, grid, dim3(kBlock), 0, s, start, stop, a, sel);
        break;
    case 4:
        launch_maybe_timed(k_ransac<4>, grid, dim3(kBlock), 0, s, start, stop, a, sel);
        break;
    case 8:
        launch_maybe_timed(k_ransac<8>, grid, dim3(kBlock), 0, s, start, stop, a, sel);
        break;
    case 16:
        launch_maybe_timed(k_ransac<16>, grid, dim3(kBlock), 0, s, start, stop, a, sel);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fused(const FusedArgs &a, int grid, size_t lds_bytes, hipStream_t s,
                        hipEvent_t start, hipEvent_t stop)
{
    if (a.se.n_frames <= 0)
        return hipSuccess;
    launch_maybe_timed(k_fused, dim3(grid), dim3(kBlock), lds_bytes, s, start, stop, a);
    return hipGetLastError();
}

hipError_t launch_fallback(ca_result *out, const ca_result *fallback, int n, float frac,
                           hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_fallback, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, out,
                       fallback, n, frac);
    return hipGetLastError();
}

hipError_t launch_stream_update(const ca_result *res, const int4 *runs, int n_runs, float4 *state,
                                float4 *filt, float decay, hipStream_t s)
{
    if (n_runs <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_stream_update, dim3((n_runs + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                       res, runs, n_runs, state, filt, decay);
    return hipGetLastError();
}

hipError_t fused_occupancy(size_t lds_bytes, int *blocks_per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_fused, kBlock, lds_bytes);
}

}  // namespace ca
