// Device renderer of the synthetic endoscopic image model: the training set
// of the learned scorer (hundreds of thousands of frames) and the hard
// evaluation frames.  An input generator only, built as its own library: it
// holds none of the estimator's arithmetic and shares no code with it.
//
// Image model (the CPU renderer of the package states the same one): a smooth
// tissue-like colour field inside a circle, a dark grey noisy border, the
// transition an analytically Gaussian-blurred step whose 50 % level lies on
// the circle.  Hard frames add a dark rim that leaves only a small luma step
// at the edge, specular blobs and white dot-matrix text in the border.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11),
// counter (x, y, 0, 0) under the frame's 64-bit key, turned into four
// normals by the Box-Muller transform; a pixel's value depends only on its
// frame and coordinates, so windows cut from a rendered frame equal windows
// rendered directly.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "synth_gpu.h"

namespace {

constexpr int kBlock = 256;
constexpr int kKindNoBorder = 2;
constexpr int kGlyphW = 5, kGlyphH = 7;
constexpr int kWin = 128, kHalo = 8, kOut = 112, kLines = 8;

struct U4 {
    uint32_t v[4];
};

__device__ __forceinline__ void mulhilo(uint32_t a, uint32_t b, uint32_t &hi, uint32_t &lo)
{
    const uint64_t p = (uint64_t)a * b;
    hi = (uint32_t)(p >> 32);
    lo = (uint32_t)p;
}

// Philox4x32 with 10 rounds: multipliers 0xD2511F53, 0xCD9E8D57; key
// increments (Weyl constants) 0x9E3779B9, 0xBB67AE85.
__device__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1)
{
    for (int round = 0; round < 10; ++round) {
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo(0xD2511F53u, c.v[0], hi0, lo0);
        mulhilo(0xCD9E8D57u, c.v[2], hi1, lo1);
        U4 n;
        n.v[0] = hi1 ^ c.v[1] ^ k0;
        n.v[1] = lo1;
        n.v[2] = hi0 ^ c.v[3] ^ k1;
        n.v[3] = lo0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ float unit_open(uint32_t u)
{
    return ((float)(u >> 8) + 0.5f) * (1.0f / 16777216.0f);   // (0, 1)
}

// Four standard normals of pixel (x, y) of a frame.
__device__ void normals(const SynthFrame &f, int x, int y, float n[4])
{
    U4 c;
    c.v[0] = (uint32_t)x;
    c.v[1] = (uint32_t)y;
    c.v[2] = 0;
    c.v[3] = 0;
    const U4 r = philox4x32_10(c, f.key0, f.key1);
    for (int i = 0; i < 2; ++i) {
        const float rad = sqrtf(-2.0f * logf(unit_open(r.v[2 * i])));
        float s, co;
        sincosf(6.283185307179586f * unit_open(r.v[2 * i + 1]), &s, &co);
        n[2 * i] = rad * co;
        n[2 * i + 1] = rad * s;
    }
}

// Linear interpolation of an n_in-point control line onto n_out samples
// placed at i (n_in - 1) / (n_out - 1).
__device__ __forceinline__ void lerp_index(int i, int n_out, int n_in, int &i0, float &t)
{
    const float pos = n_out > 1 ? (float)i * (float)(n_in - 1) / (float)(n_out - 1) : 0.0f;
    int k = (int)floorf(pos);
    k = k < 0 ? 0 : (k > n_in - 2 ? n_in - 2 : k);
    i0 = k;
    t = pos - (float)k;
}

__device__ __forceinline__ float bilerp(const float *g, int gh, int gw, int H, int W, int x, int y)
{
    int iy, ix;
    float ty, tx;
    lerp_index(y, H, gh, iy, ty);
    lerp_index(x, W, gw, ix, tx);
    const float a = g[iy * gw + ix] * (1.0f - tx) + g[iy * gw + ix + 1] * tx;
    const float b = g[(iy + 1) * gw + ix] * (1.0f - tx) + g[(iy + 1) * gw + ix + 1] * tx;
    return a * (1.0f - ty) + b * ty;
}

__device__ bool text_pixel(const SynthFrame &f, const uint64_t *glyphs, int x, int y)
{
    if (f.text_scale <= 0)
        return false;
    const float fx = ((float)x - f.text_x) / (float)f.text_scale;
    const float fy = ((float)y - f.text_y) / (float)f.text_scale;
    if (fx < 0.0f || fy < 0.0f)
        return false;
    const int cx = (int)fx, cy = (int)fy;
    const int ch = cx / (kGlyphW + 1), col = cx % (kGlyphW + 1);
    const int ln = cy / (kGlyphH + 2), row = cy % (kGlyphH + 2);
    if (ch >= f.text_chars || ln >= f.text_lines || col >= kGlyphW || row >= kGlyphH)
        return false;
    const uint64_t bits = glyphs[f.glyph_off + ln * f.text_chars + ch];
    return (bits >> (row * kGlyphW + col)) & 1u;
}

__device__ void render_pixel(const SynthFrame &f, const float *grids, const uint64_t *glyphs, int x,
                             int y, uint8_t out[3])
{
    const float *g = grids + f.grid_off;
    const int n0 = f.gh0 * f.gw0, n1 = f.gh1 * f.gw1;
    const float base = bilerp(g, f.gh0, f.gw0, f.height, f.width, x, y);
    const float fine = bilerp(g + n0, f.gh1, f.gw1, f.height, f.width, x, y);
    float lum = f.mean_luma * (1.0f + 0.18f * base + 0.06f * fine);
    const bool bordered = f.kind != kKindNoBorder;
    const float dx = (float)x - f.cx, dy = (float)y - f.cy;
    const float rho = sqrtf(dx * dx + dy * dy);
    float fall = 1.0f;
    if (bordered && f.edge_step > 0.0f) {
        // dark rim: content luma falls to 6 + edge_step at the circle
        const float rim = (6.0f + f.edge_step) / f.mean_luma;
        float u = (f.r - rho) / (0.3f * f.r);
        u = u < 0.0f ? 0.0f : (u > 1.0f ? 1.0f : u);
        fall = rim + (1.0f - rim) * u * u * (3.0f - 2.0f * u);
    } else if (f.vignette > 0.0f) {
        float q;
        if (bordered) {
            q = rho / f.r;
        } else {
            const float ex = (float)x - 0.5f * (float)(f.width - 1);
            const float ey = (float)y - 0.5f * (float)(f.height - 1);
            q = sqrtf(ex * ex + ey * ey)
                / (0.5f * sqrtf((float)f.width * f.width + (float)f.height * f.height));
        }
        q = q < 1.0f ? q : 1.0f;
        fall = 1.0f - f.vignette * q * q;
    }
    float nz[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (!(f.flags & SYNTH_NO_NOISE))
        normals(f, x, y, nz);
    float c[3];
    for (int k = 0; k < 3; ++k) {
        const float chroma = bilerp(g + n0 + n1 + k * n0, f.gh0, f.gw0, f.height, f.width, x, y);
        c[k] = lum * f.tint[k] * (1.0f + 0.08f * chroma) * fall + 2.0f * nz[k];
    }
    if (bordered) {
        const float alpha = normcdff((f.r - rho) / f.blur);
        float b = 6.0f + f.border_sigma * nz[3];
        for (int i = 0; i < f.n_blobs; ++i) {
            const float bx = (float)x - f.blob[i][0], by = (float)y - f.blob[i][1];
            const float rr = f.blob[i][2];
            b += f.blob[i][3] * expf(-(bx * bx + by * by) / (2.0f * rr * rr));
        }
        for (int k = 0; k < 3; ++k)
            c[k] = alpha * c[k] + (1.0f - alpha) * b;
        if (text_pixel(f, glyphs, x, y))
            c[0] = c[1] = c[2] = 240.0f;
    }
    for (int k = 0; k < 3; ++k) {
        float v = rintf(c[k]);
        v = v < 0.0f ? 0.0f : (v > 255.0f ? 255.0f : v);
        out[k] = (uint8_t)v;
    }
}

// grid.y = frame; each thread renders 4 consecutive pixels of a row-major frame.
__global__ __launch_bounds__(kBlock) void k_render_frames(const SynthFrame *frames,
                                                          const float *grids,
                                                          const uint64_t *glyphs, uint8_t *out)
{
    const SynthFrame f = frames[blockIdx.y];
    const int64_t n = (int64_t)f.width * f.height;
    uint8_t *dst = out + f.out_offset;
    for (int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * 4; i < n;
         i += (int64_t)gridDim.x * kBlock * 4) {
        for (int j = 0; j < 4 && i + j < n; ++j) {
            const int y = (int)((i + j) / f.width), x = (int)((i + j) % f.width);
            uint8_t px[3];
            render_pixel(f, grids, glyphs, x, y, px);
            dst[3 * (i + j)] = px[0];
            dst[3 * (i + j) + 1] = px[1];
            dst[3 * (i + j) + 2] = px[2];
        }
    }
}

// One block per training window: desc = (frame, horizontal, line, start);
// window element n is strip position start + n.  Writes the window [8][128][3]
// (lines line-3 .. line+4, clamped), its in-strip range, and for the central
// positions the soft edge label exp(-(rho - r)^2 / 18) (Gaussian, sigma 3 px,
// of the distance of the strip pixel to the circle; 0 without a border) and
// the loss weight (1 + edge_boost * label inside the strip, else 0).
__global__ __launch_bounds__(kBlock) void k_render_windows(const SynthFrame *frames,
                                                           const int32_t *desc, const float *grids,
                                                           const uint64_t *glyphs, float edge_boost,
                                                           uint8_t *win, int32_t *range,
                                                           float *target, float *weight)
{
    const int w = blockIdx.x;
    const SynthFrame f = frames[desc[4 * w]];
    const bool horizontal = desc[4 * w + 1] != 0;
    const int line = desc[4 * w + 2];
    const int start = desc[4 * w + 3];
    const int L = horizontal ? f.width : f.height;
    const int extent = horizontal ? f.height : f.width;
    uint8_t *dst = win + (int64_t)w * (kLines * kWin * 3);
    for (int i = threadIdx.x; i < kLines * kWin; i += kBlock) {
        const int j = i / kWin, n = i % kWin;
        const int p = start + n;
        uint8_t px[3] = {0, 0, 0};
        if (p >= 0 && p < L) {
            int across = line + j - 3;
            across = across < 0 ? 0 : (across > extent - 1 ? extent - 1 : across);
            render_pixel(f, grids, glyphs, horizontal ? p : across, horizontal ? across : p, px);
        }
        uint8_t *o = dst + (j * kWin + n) * 3;
        o[0] = px[0];
        o[1] = px[1];
        o[2] = px[2];
    }
    if (threadIdx.x == 0) {
        const int lo = start < 0 ? -start : 0;
        const int hi = L - start < kWin ? L - start : kWin;
        range[2 * w] = lo;
        range[2 * w + 1] = hi > lo ? hi : lo;
    }
    if (threadIdx.x < kOut) {
        const int p = start + kHalo + threadIdx.x;
        float t = 0.0f, wt = 0.0f;
        if (p >= 0 && p < L) {
            if (f.kind != kKindNoBorder) {
                const float x = (float)(horizontal ? p : line), y = (float)(horizontal ? line : p);
                const float d = sqrtf((x - f.cx) * (x - f.cx) + (y - f.cy) * (y - f.cy)) - f.r;
                t = expf(-d * d / 18.0f);
            }
            wt = 1.0f + edge_boost * t;
        }
        target[(int64_t)w * kOut + threadIdx.x] = t;
        weight[(int64_t)w * kOut + threadIdx.x] = wt;
    }
}

}  // namespace

extern "C" {

int synth_render_frames(const SynthFrame *frames, int32_t n, int32_t max_pixels,
                        const float *grids, const uint64_t *glyphs, uint8_t *out, void *stream)
{
    if (n < 0 || max_pixels < 0 || (n > 0 && (!frames || !grids || !glyphs || !out)))
        return -1;
    if (n == 0 || max_pixels == 0)
        return 0;
    int64_t blocks = ((int64_t)max_pixels + 4 * kBlock - 1) / (4 * kBlock);
    blocks = blocks < 4096 ? blocks : 4096;
    hipLaunchKernelGGL(k_render_frames, dim3((unsigned)blocks, (unsigned)n), dim3(kBlock), 0,
                       static_cast<hipStream_t>(stream), frames, grids, glyphs, out);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

int synth_render_windows(const SynthFrame *frames, const int32_t *desc, int32_t n,
                         const float *grids, const uint64_t *glyphs, float edge_boost,
                         uint8_t *win, int32_t *range, float *target, float *weight, void *stream)
{
    if (n < 0 || (n > 0 && (!frames || !desc || !grids || !glyphs || !win || !range || !target
                            || !weight)))
        return -1;
    if (n == 0)
        return 0;
    hipLaunchKernelGGL(k_render_windows, dim3((unsigned)n), dim3(kBlock), 0,
                       static_cast<hipStream_t>(stream), frames, desc, grids, glyphs, edge_boost,
                       win, range, target, weight);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // extern "C"
