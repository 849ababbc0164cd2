// gfx950 kernels of the paper's own learned edge scorer (arXiv 2210.14771,
// Section 2.2.4): three 3x3 convolutions with 8, 16 and 32 output features,
// each followed by a ReLU, a 1x1 convolution to one logit and a sigmoid, on
// RGBXY input (colours normalised by the training data's per-channel mean
// and standard deviation, pixel coordinates normalised to [-0.5, 0.5] about
// the image centre), applied to strips seven lines thick (the network's
// receptive field), so a strip's scores are the whole-image network's output
// on the strip's centre line.
//
// A strip is processed in windows of 128 positions: band lines 0..6 (the
// strip line -3 .. +3) of the input, lines 1..5 of layer 1, 2..4 of layer 2
// and line 3 of layer 3.  Each layer is one GEMM per output line on
// v_mfma_f32_16x16x32_bf16: activations are stored position-major
// ([line][position][channel], channels contiguous, one zero guard position
// at each end), so the 8 channels of one tap at one position are one
// 16-byte LDS load, and K = (3 da + dl) C_pad + c walks the 3x3 taps.  For a
// vertical strip the band's lines are frame columns: the weights' two
// spatial axes swap roles, so the model block holds both orientations.
// Every layer's input is zero outside the frame and beyond the strip ends
// ("same" zero padding of the whole-image network).  Weights and hidden
// activations are bfloat16, sums are float32 MFMA accumulators.
#include "ca_cnn.h"
#include "ca_launch.h"

namespace ca {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kPos = kC2Win + 2;   // positions of a buffer line, guards included
constexpr int kC2Halo = 3;         // the network's receptive-field radius
constexpr int kC2Stride = kC2Win - 2 * kC2Halo;   // exact logits per strip window
constexpr int kTrainHalo = 8;      // training windows carry logits 8 .. 119
constexpr int kTrainOut = kC2Win - 2 * kTrainHalo;
constexpr int kC2Floats = 96;      // floats of the model's float block
constexpr int kWaves = kBlock / 64;

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ __bf16 to_bf16(float v) { return (__bf16)v; }

// LDS of the forward pass: input (7 lines, 8 channels: RGBXY and 3 zeros),
// layer 1 (5 lines x 8), layer 2 (3 x 16), layer 3 (1 x 32), logits.
struct alignas(16) FwdLds {
    __bf16 x0[kC2Band * kPos * 8];
    __bf16 h1[5 * kPos * 8];
    __bf16 h2[3 * kPos * 16];
    __bf16 h3[kPos * 32];
    float z[kC2Win];
    float fb[kC2Floats];   // the model's float block (biases, w4, b4, colour statistics)
};

// The backward pass adds the signals at the pre-activations (ReLU and masks
// applied) of layers 3, 2 and 1, the logit gradients and a zero line.
struct alignas(16) GradLds {
    FwdLds f;
    __bf16 dp3[kPos * 32];
    __bf16 dp2[3 * kPos * 16];
    __bf16 dp1[5 * kPos * 8];
    __bf16 zero[kPos * 32];
    __bf16 ones[4];
    float dz[kC2Win];
    float loss[kBlock / 64];
};

// Clear a buffer (both guards included); a workgroup-wide loop.
__device__ void clear(__bf16 *p, int n)
{
    for (int i = threadIdx.x; i < n; i += kBlock)
        p[i] = to_bf16(0.0f);
}

// The A operand of a layer's GEMMs (weights [M][KP], M = 16 MT output
// channels) as this lane's MFMA fragments: loaded once, kept in registers
// for every tile of every window the workgroup computes.
template <int KP, int MT>
struct Frag {
    bf16x8 a[MT][KP / 32];
};

template <int KP, int MT>
__device__ __forceinline__ Frag<KP, MT> load_frag(const __bf16 *A)
{
    const int lane = threadIdx.x & 63;
    Frag<KP, MT> f;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int ks = 0; ks < KP / 32; ++ks)
            f.a[mt][ks] = *reinterpret_cast<const bf16x8 *>(A + (mt * 16 + (lane & 15)) * KP
                                                            + 32 * ks + 8 * (lane >> 4));
    return f;
}

// One 3x3 convolution layer over a window as GEMMs, one per output line i:
// acc[m][n] = sum_k A[m][k] B_i[k][n] with B_i[(3 da + dl) CP + c][n] =
// X[line i + da][n + dl - 1][c] (lines outside [x_lo, x_hi) read the zero
// line).  A wave takes position tiles (16 positions of one output line) and
// computes all MT channel tiles of each from one read of its B fragments;
// epi(i, m0, n, acc) receives rows m0 .. m0 + 3 of column n.
template <int CP, int KP, int MT, int OUT_LINES, class Epi>
__device__ __forceinline__ void gemm3x3(const Frag<KP, MT> &F, const __bf16 *X, int x_lo,
                                        int x_hi, const __bf16 *zero, Epi epi)
{
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    constexpr int NT = kC2Win / 16;
    constexpr int CB = CP / 8;
    constexpr int G = 9 * CB;   // real 8-wide K groups; the rest have zero weights
    static_assert((OUT_LINES * NT) % kWaves == 0, "tiles must split evenly over the waves");
    const int kq = lane >> 4;
#pragma unroll
    for (int t = 0; t < OUT_LINES * NT / kWaves; ++t) {
        const int tile = wv + kWaves * t;
        const int nt = tile % NT;
        const int i = tile / NT;
        const int n = nt * 16 + (lane & 15);
        f32x4 acc[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
            acc[mt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < KP / 32; ++ks) {
            int g = 4 * ks + kq;
            g = g < G ? g : 0;
            const int tap = g / CB, cb = g - CB * (g / CB);
            const int da = tap / 3, dl = tap - 3 * (tap / 3);
            const int line = i + da;
            const __bf16 *src = (line >= x_lo && line < x_hi) ? X + (line - x_lo) * kPos * CP : zero;
            const bf16x8 b = *reinterpret_cast<const bf16x8 *>(src + (n + dl) * CP + 8 * cb);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.a[mt][ks], b, acc[mt], 0, 0, 0);
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
            epi(i, mt * 16 + 4 * kq, n, acc[mt]);
    }
}

// The forward weights of one orientation in registers: the three layers' A
// fragments and this lane's biases (rows m0 .. m0 + 3 of its accumulators).
struct FwdW {
    Frag<96, 1> w1;
    Frag<96, 1> w2;
    Frag<160, 2> w3;
    float b1[4], b2[4], b3[2][4];
};

// fb: the model's float block (in LDS).  With `paired`, layer 1's weights
// are those of output-line pairs (rows 8..15 the second line's channels).
__device__ __forceinline__ void load_fwd_weights(FwdW &W, const uint8_t *model, bool hz,
                                                 const float *fb, bool paired = false)
{
    const __bf16 *A = reinterpret_cast<const __bf16 *>(model) + (hz ? 0 : kC2Orient);
    W.w1 = load_frag<96, 1>(A + (paired ? kC2P1 : kC2A[0]));
    W.w2 = load_frag<96, 1>(A + kC2A[1]);
    W.w3 = load_frag<160, 2>(A + kC2A[2]);
    const int m0 = 4 * ((threadIdx.x & 63) >> 4);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        W.b1[j] = paired ? fb[kC2FB[0] + (m0 & 7) + j] : (m0 < 8 ? fb[kC2FB[0] + m0 + j] : 0.0f);
        W.b2[j] = fb[kC2FB[1] + m0 + j];
        W.b3[0][j] = fb[kC2FB[2] + m0 + j];
        W.b3[1][j] = fb[kC2FB[2] + 16 + m0 + j];
    }
}

// The model's float block into L.fb (a workgroup-wide copy; the caller
// synchronises before reading it).
__device__ void stage_floats(FwdLds &L, const uint8_t *model)
{
    const float *src = reinterpret_cast<const float *>(model + kC2FloatsOff);
    for (int i = threadIdx.x; i < kC2Floats; i += kBlock)
        L.fb[i] = src[i];
}

// Input encoding of one band position: colours normalised, coordinates in
// [-0.5, 0.5] as (2 x - (W - 1)) / (2 (W - 1)), taken as a product with the
// reciprocal rw = 1 / (2 (W - 1)) (and rh for y); channels 5..7 are zero.
// (x, y) is the pixel, (W, H) the frame.
__device__ __forceinline__ void encode(__bf16 *dst, uint32_t r, uint32_t g, uint32_t b, int x,
                                       int y, int W, int H, float rw, float rh, const float *fb)
{
    bf16x8 v;
    v[0] = to_bf16(((float)r - fb[kC2FMean + 0]) * fb[kC2FInv + 0]);
    v[1] = to_bf16(((float)g - fb[kC2FMean + 1]) * fb[kC2FInv + 1]);
    v[2] = to_bf16(((float)b - fb[kC2FMean + 2]) * fb[kC2FInv + 2]);
    v[3] = to_bf16((float)(2 * x - (W - 1)) * rw);
    v[4] = to_bf16((float)(2 * y - (H - 1)) * rh);
    v[5] = v[6] = v[7] = to_bf16(0.0f);
    *reinterpret_cast<bf16x8 *>(dst) = v;
}
__device__ __forceinline__ float coord_scale(int extent) { return 1.0f / (float)(2 * (extent - 1)); }

__device__ __forceinline__ bool line_in(uint32_t line_ok, int j) { return (line_ok >> j) & 1u; }

// Forward pass of the window whose input is in L.x0: logits of all 128
// positions into L.z (exact where the whole receptive field is inside the
// window).  line_ok bit j: band line j lies in the frame; positions outside
// [lo, hi) are beyond the strip.
__device__ void forward(FwdLds &L, const FwdW &W, uint32_t line_ok, int lo, int hi)
{
    gemm3x3<8, 96, 1, 5>(W.w1, L.x0, 0, kC2Band, nullptr,
                         [&](int i, int m0, int n, const f32x4 &acc) {
                             if (m0 >= 8)
                                 return;
                             const bool keep = line_in(line_ok, i + 1) && n >= lo && n < hi;
                             bf16x4 o;
#pragma unroll
                             for (int j = 0; j < 4; ++j) {
                                 const float v = fmaxf(acc[j] + W.b1[j], 0.0f);
                                 o[j] = to_bf16(keep ? v : 0.0f);
                             }
                             *reinterpret_cast<bf16x4 *>(L.h1 + (i * kPos + n + 1) * 8 + m0) = o;
                         });
    __syncthreads();
    gemm3x3<8, 96, 1, 3>(W.w2, L.h1, 0, 5, nullptr,
                         [&](int i, int m0, int n, const f32x4 &acc) {
                             const bool keep = line_in(line_ok, i + 2) && n >= lo && n < hi;
                             bf16x4 o;
#pragma unroll
                             for (int j = 0; j < 4; ++j) {
                                 const float v = fmaxf(acc[j] + W.b2[j], 0.0f);
                                 o[j] = to_bf16(keep ? v : 0.0f);
                             }
                             *reinterpret_cast<bf16x4 *>(L.h2 + (i * kPos + n + 1) * 16 + m0) = o;
                         });
    __syncthreads();
    gemm3x3<16, 160, 2, 1>(W.w3, L.h2, 0, 3, nullptr,
                           [&](int, int m0, int n, const f32x4 &acc) {
                               const bool keep = line_in(line_ok, 3) && n >= lo && n < hi;
                               bf16x4 o;
#pragma unroll
                               for (int j = 0; j < 4; ++j) {
                                   const float v = fmaxf(acc[j] + W.b3[m0 >> 4][j], 0.0f);
                                   o[j] = to_bf16(keep ? v : 0.0f);
                               }
                               *reinterpret_cast<bf16x4 *>(L.h3 + (n + 1) * 32 + m0) = o;
                           });
    __syncthreads();
    const int n = threadIdx.x;
    if (n < kC2Win) {
        const __bf16 *h = L.h3 + (n + 1) * 32;
        float z = L.fb[kC2FB4];
#pragma unroll
        for (int o = 0; o < 32; ++o)
            z = fmaf(L.fb[kC2FW4 + o], (float)h[o], z);
        L.z[n] = z;
    }
    __syncthreads();
}

// The input of a rendered window [8][128][3] (lines line-3 .. line+4,
// clamped to the frame): band lines 0..6, zero outside the frame or strip.
__device__ void load_window(FwdLds &L, const uint8_t *src, const int32_t *g, const float *fb,
                            uint32_t line_ok, int lo, int hi)
{
    const bool hz = g[0] != 0;
    const int line = g[1], start = g[2], W = g[3], H = g[4];
    for (int i = threadIdx.x; i < kC2Band * kC2Win; i += kBlock) {
        const int j = i / kC2Win, n = i - kC2Win * (i / kC2Win);
        __bf16 *dst = L.x0 + (j * kPos + n + 1) * 8;
        if (!line_in(line_ok, j) || n < lo || n >= hi) {
            *reinterpret_cast<bf16x8 *>(dst) = bf16x8{};
            continue;
        }
        const uint8_t *px = src + (j * kC2Win + n) * 3;
        const int across = line - 3 + j, along = start + n;
        encode(dst, px[0], px[1], px[2], hz ? along : across, hz ? across : along, W, H,
               coord_scale(W), coord_scale(H), fb);
    }
}

__device__ __forceinline__ uint32_t band_lines(int line, int extent)
{
    uint32_t ok = 0;
    for (int j = 0; j < kC2Band; ++j) {
        const int r = line - 3 + j;
        ok |= (r >= 0 && r < extent) ? (1u << j) : 0u;
    }
    return ok;
}

__device__ __forceinline__ float sigmoid(float z) { return 1.0f / (1.0f + __expf(-z)); }

// ----------------------------------------------------------- inference --

// Learned candidates, wave level.  A workgroup takes one (frame, strip) item
// (XCD-aware: workgroup b takes item (b % 8) per_xcd + b / 8); each of its
// four waves scores windows of 64 positions of the strip on its own --
// window w by wave w mod 4 -- with private LDS buffers and the layers'
// weights in its registers, so no workgroup barrier separates the layers and
// the waves of a compute unit overlap one another's memory and LDS latency.
// The pixels of a wave's next window are loaded into registers while its
// current window's layers run.  The workgroup joins its waves' best pixels
// per half strip (ties: outermost).

constexpr int kWWin = 64;                        // positions of a wave window
constexpr int kWPos = kWWin + 2;                 // with a guard position at each end
constexpr int kWStride = kWWin - 2 * kC2Halo;    // exact logits per wave window
// A wave's two buffers: P holds the input (7 lines x 8 channels) and later
// layer 2 (3 x 16), Q layer 1 (5 x 8) and later layer 3 (1 x 32).  Guard
// positions and rows of one layout read under another hold stale finite
// values (the buffers are zeroed once); they only feed the 3 halo positions
// at each window end, whose outputs are discarded.
constexpr int kWP = kC2Band * kWPos * 8 > 3 * kWPos * 16 ? kC2Band * kWPos * 8 : 3 * kWPos * 16;
constexpr int kWQ = 5 * kWPos * 8 > kWPos * 32 ? 5 * kWPos * 8 : kWPos * 32;
struct alignas(16) WaveBufs {
    __bf16 p[kWP];
    __bf16 q[kWQ];
};

// LDS written by some lanes of a wave and read by others next: keep the
// compiler from moving memory operations across (the hardware keeps a
// wave's LDS operations in order).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// One 3x3 layer over a wave window, all tiles by this wave: for output line
// i, acc[m][n] = bias[m] + sum_k A[m][k] X[line i + da][n + dl - 1][c] with
// k = (3 da + dl) CP + c.  The lane's B offsets (its K group of each k-step)
// are computed once; tiles then differ by constant offsets.  epi(i, nt, mt,
// acc) receives rows 16 mt + 4 (lane / 16) .. + 3 of column 16 nt + lane % 16.
// NLO input lines per output index (3; 4 for layer 1 by output-line pairs,
// whose output index i covers lines 2 i and 2 i + 1: LSTEP = 2).
template <int CP, int KP, int MT, int OUT_LINES, int NLO = 3, int LSTEP = 1, class Epi>
__device__ __forceinline__ void wave_gemm3x3(const Frag<KP, MT> &F, const float (&bias)[MT][4],
                                             const __bf16 *X, Epi epi)
{
    const int lane = threadIdx.x & 63;
    constexpr int NT = kWWin / 16;
    constexpr int CB = CP / 8;
    constexpr int G = 3 * NLO * CB;   // real 8-wide K groups; the rest have zero weights
    constexpr int KS = KP / 32;
    int boff[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        int g = 4 * ks + (lane >> 4);
        g = g < G ? g : 0;
        const int tap = g / CB, cb = g - CB * (g / CB);
        const int da = tap / 3, dl = tap - 3 * (tap / 3);
        boff[ks] = ((da * kWPos + dl + (lane & 15)) * CP + 8 * cb);
    }
    // one output line at a time, its NT position tiles together: their
    // accumulator chains are independent, so their MFMAs interleave
#pragma unroll
    for (int i = 0; i < OUT_LINES; ++i) {
        const __bf16 *b0 = X + LSTEP * i * kWPos * CP;
        f32x4 acc[NT][MT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                acc[nt][mt] = f32x4{bias[mt][0], bias[mt][1], bias[mt][2], bias[mt][3]};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            bf16x8 b[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                b[nt] = *reinterpret_cast<const bf16x8 *>(b0 + nt * 16 * CP + boff[ks]);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[nt][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.a[mt][ks], b[nt],
                                                                          acc[nt][mt], 0, 0, 0);
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                epi(i, nt, mt, acc[nt][mt]);
    }
}

// ReLU and the frame / strip mask in one median: clamp to [0, +inf) where
// the activation exists, to [0, 0] elsewhere; stored as bfloat16.
__device__ __forceinline__ bf16x4 relu_bf16(const f32x4 &acc, float top)
{
    bf16x4 o;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        o[j] = to_bf16(__builtin_amdgcn_fmed3f(acc[j], 0.0f, top));
    return o;
}

// The 1x1 layer's weights this lane needs (its 8 of layer 3's 32 channels).
struct OutW {
    float w4[2][4];
    float b4;
};

// Logit of position `lane` of the wave window whose input is in B.p.  The
// 1x1 layer is folded into layer 3's epilogue: each lane dots its 8
// channels, the four lane groups holding a position's 32 channels add up by
// shuffles, and lane group q keeps position tile q.
__device__ __forceinline__ float wave_forward2d(WaveBufs &B, const FwdW &W, const OutW &O,
                                                uint32_t line_ok, int lo, int hi)
{
    const int lane = threadIdx.x & 63;
    const int col = lane & 15, m0 = 4 * (lane >> 4);
    // tops[nt]: the mask of this lane's column in position tile nt
    float tops[kWWin / 16];
#pragma unroll
    for (int nt = 0; nt < kWWin / 16; ++nt) {
        const int n = nt * 16 + col;
        tops[nt] = (n >= lo && n < hi) ? __builtin_inff() : 0.0f;
    }
    const float b1[1][4] = {{W.b1[0], W.b1[1], W.b1[2], W.b1[3]}};
    const float b2[1][4] = {{W.b2[0], W.b2[1], W.b2[2], W.b2[3]}};
    // layer 1 by output-line pairs (1, 2), (3, 4), (5, -): lane groups 0-1
    // hold the pair's first line, 2-3 its second
    wave_gemm3x3<8, 96, 1, 3, 4, 2>(W.w1, b1, B.p, [&](int i, int nt, int, const f32x4 &acc) {
        const int line = 2 * i + (m0 >> 3);
        if (line >= 5)
            return;
        const float top = line_in(line_ok, line + 1) ? tops[nt] : 0.0f;
        *reinterpret_cast<bf16x4 *>(B.q + (line * kWPos + nt * 16 + col + 1) * 8 + (m0 & 7)) =
            relu_bf16(acc, top);
    });
    wave_sync();
    wave_gemm3x3<8, 96, 1, 3>(W.w2, b2, B.q, [&](int i, int nt, int, const f32x4 &acc) {
        const float top = line_in(line_ok, i + 2) ? tops[nt] : 0.0f;
        *reinterpret_cast<bf16x4 *>(B.p + (i * kWPos + nt * 16 + col + 1) * 16 + m0) =
            relu_bf16(acc, top);
    });
    wave_sync();
    float part[kWWin / 16];
#pragma unroll
    for (int nt = 0; nt < kWWin / 16; ++nt)
        part[nt] = 0.0f;
    const bool mid = line_in(line_ok, 3);
    wave_gemm3x3<16, 160, 2, 1>(W.w3, W.b3, B.p, [&](int, int nt, int mt, const f32x4 &acc) {
        const bf16x4 h = relu_bf16(acc, mid ? tops[nt] : 0.0f);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            part[nt] = fmaf(O.w4[mt][j], (float)h[j], part[nt]);
    });
    float mine = 0.0f;
#pragma unroll
    for (int nt = 0; nt < kWWin / 16; ++nt) {
        float v = part[nt];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        mine = (lane >> 4) == nt ? v : mine;
    }
    return O.b4 + mine;
}

__global__ __launch_bounds__(kBlock) void k_cnn2d_strips(Cnn2dStripArgs a)
{
    __shared__ WaveBufs wb[kWaves];
    __shared__ float s_fb[kC2Floats];
    __shared__ uint64_t s_best[kWaves][2];
    const int item = (int)(blockIdx.x & 7) * a.per_xcd + (int)(blockIdx.x >> 3);
    if (item >= a.n_items || (int)(blockIdx.x >> 3) >= a.per_xcd)
        return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int S = a.n_h + a.n_v;
    const int f = uniform_int(a.frame0 + item / S);
    const int st = uniform_int(item % S);
    const FrameDev d = a.fd[f];
    const uint8_t *frame = a.frames + d.offset;
    const bool hz = st < a.n_h;
    const int pos = uniform_int(a.strips[d.table + st]);
    const int L_ = hz ? d.W : d.H;
    const int extent = hz ? d.H : d.W;
    const uint32_t line_ok = band_lines(pos, extent);
    WaveBufs &B = wb[wv];
    {
        const float *src = reinterpret_cast<const float *>(a.model + kC2FloatsOff);
        for (int i = threadIdx.x; i < kC2Floats; i += kBlock)
            s_fb[i] = src[i];
        uint4 *z = reinterpret_cast<uint4 *>(&B);
        for (int i = lane; i < (int)(sizeof(WaveBufs) / 16); i += 64)
            z[i] = make_uint4(0u, 0u, 0u, 0u);
    }
    __syncthreads();
    FwdW W;
    load_fwd_weights(W, a.model, hz, s_fb, true);
    OutW O;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            O.w4[mt][j] = s_fb[kC2FW4 + 16 * mt + 4 * (lane >> 4) + j];
    O.b4 = s_fb[kC2FB4];
    uint64_t best[2] = {0, 0};
    const int n_win = (L_ + kWStride - 1) / kWStride;
    const float rw = coord_scale(d.W), rh = coord_scale(d.H);

    // This wave's next window's pixels, fetched one window ahead: band
    // position i = lane + 64 k in slot k (horizontal strips: positions
    // fastest; vertical strips: lines fastest -- adjacent pixels of a row).
    constexpr int kSlots = kC2Band * kWWin / 64;
    // raw bytes: R | G << 8 and B of each slot, split only when encoded, so
    // nothing waits for the loads before the next window's turn; slots
    // outside the frame or the strip load pixel (0, 0) and are dropped
    uint32_t prg[kSlots], pb[kSlots];
    uint32_t have = 0;
    auto window = [&](int w, int &start, int &lo, int &hi) {
        start = w * kWStride - kC2Halo;
        lo = start >= 0 ? 0 : -start;
        hi = L_ - start < kWWin ? L_ - start : kWWin;
    };
    auto slot_pos = [&](int k, int &j, int &n) {
        const int i = lane + 64 * k;
        j = hz ? i / kWWin : i % kC2Band;
        n = hz ? i % kWWin : i / kC2Band;
    };
    auto fetch = [&](int w) {
        int start, lo, hi;
        window(w, start, lo, hi);
        have = 0;
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
            int j, n;
            slot_pos(k, j, n);
            const bool ok = line_in(line_ok, j) && n >= lo && n < hi;
            const int across = pos - 3 + j, along = start + n;
            const int x = ok ? (hz ? along : across) : 0, y = ok ? (hz ? across : along) : 0;
            const uint8_t *px = frame + (int64_t)y * d.rs + 3 * x;
            uint16_t rg;
            __builtin_memcpy(&rg, px, 2);
            prg[k] = rg;
            pb[k] = px[2];
            have |= ok ? 1u << k : 0u;
        }
    };
    if (wv < n_win)
        fetch(wv);
    for (int w = wv; w < n_win; w += kWaves) {
        int start, lo, hi;
        window(w, start, lo, hi);
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
            int j, n;
            slot_pos(k, j, n);
            __bf16 *dst = B.p + (j * kWPos + n + 1) * 8;
            if (!((have >> k) & 1u)) {
                *reinterpret_cast<bf16x8 *>(dst) = bf16x8{};
                continue;
            }
            const int across = pos - 3 + j, along = start + n;
            encode(dst, prg[k] & 0xFFu, prg[k] >> 8, pb[k], hz ? along : across,
                   hz ? across : along, d.W, d.H, rw, rh, s_fb);
        }
        wave_sync();
        if (w + kWaves < n_win)
            fetch(w + kWaves);
        const float z = wave_forward2d(B, W, O, line_ok, lo, hi);
        const int p = start + lane;
        if (lane >= kC2Halo && lane < kWWin - kC2Halo && p < L_) {
            const float sc = sigmoid(z);
            const int half = p < (L_ >> 1) ? 0 : 1;
            const int k = half == 0 ? p : L_ - 1 - p;
            const uint64_t key = ((uint64_t)__float_as_uint(sc) << 32)
                                 | (uint64_t)(0xFFFFFFFFu - (uint32_t)k);
            best[half] = best[half] > key ? best[half] : key;
        }
        // the next window's input overwrites P, which layer 3 has read
        wave_sync();
    }
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        uint64_t v = best[half];
#pragma unroll
        for (int dd = 32; dd >= 1; dd >>= 1) {
            const uint64_t t = __shfl_xor(v, dd, 64);
            v = v > t ? v : t;
        }
        if (lane == 0)
            s_best[wv][half] = v;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const int half = threadIdx.x;
        uint64_t bb = s_best[0][half];
        for (int w2 = 1; w2 < kWaves; ++w2)
            bb = bb > s_best[w2][half] ? bb : s_best[w2][half];
        const int k = (int)(0xFFFFFFFFu - (uint32_t)bb);
        const int i = half == 0 ? k : L_ - 1 - k;
        ca_point pt;
        pt.x = (int16_t)(hz ? i : pos);
        pt.y = (int16_t)(hz ? pos : i);
        pt.score = __uint_as_float((uint32_t)(bb >> 32));
        a.cand[(int64_t)f * (2 * S) + 2 * st + half] = pt;
    }
}

// Logits of positions 8 .. 119 of rendered windows (one workgroup per window,
// grid-stride).
__global__ __launch_bounds__(kBlock) void k_cnn2d_windows(const uint8_t *model,
                                                          const uint8_t *win,
                                                          const int32_t *geom,
                                                          const int32_t *range, float *z_out,
                                                          int n_windows)
{
    __shared__ FwdLds L;
    clear(L.x0, kC2Band * kPos * 8);
    clear(L.h1, 5 * kPos * 8);
    clear(L.h2, 3 * kPos * 16);
    stage_floats(L, model);
    __syncthreads();
    FwdW W;
    for (int wi = blockIdx.x; wi < n_windows; wi += gridDim.x) {
        const int32_t *g = geom + 8 * wi;
        const bool hz = g[0] != 0;
        const int lo = uniform_int(range[2 * wi]), hi = uniform_int(range[2 * wi + 1]);
        const uint32_t line_ok = band_lines(g[1], hz ? g[4] : g[3]);
        __syncthreads();
        load_window(L, win + (int64_t)wi * (8 * kC2Win * 3), g, L.fb, line_ok, lo, hi);
        load_fwd_weights(W, model, hz, L.fb);
        __syncthreads();
        forward(L, W, line_ok, lo, hi);
        const int n = threadIdx.x;
        if (n >= kTrainHalo && n < kC2Win - kTrainHalo)
            z_out[(int64_t)wi * kTrainOut + n - kTrainHalo] = L.z[n];
    }
}

// ------------------------------------------------------------- training --
//
// Per window: the forward pass; dz = scale w (sigmoid(z) - t) on the
// central positions inside the strip; the signals at the pre-activations
// dP3 = [h3 > 0] w4 dz, dP2 = [h2 > 0] (flipped-W3 convolution of dP3),
// dP1 = [h1 > 0] (flipped-W2 convolution of dP2), each stored in bfloat16
// (the input-gradient convolutions are forward-shaped GEMMs on MFMA); then
// the weight and bias gradients as sums over the window's positions, in
// float32 registers that every thread keeps across the windows of its
// workgroup.  Work units of 4 output channels x 4 inputs (one 3x3 tap of a
// layer, frame orientation, one output line): thread t holds units t, t+256,
// t+512 in the order
//   [0, 288)    layer 3: o4 (8), tap (9), c4 (4)
//   [288, 504)  layer 2: o4 (4), tap (9), c4 (2), line (3)
//   [504, 684)  layer 1: o4 (2), tap (9), c4 (2), line (5)
//   [684, 714)  biases: layer 3 o4 (8); layer 2 o4 (4) x line (3); layer 1
//               o4 (2) x line (5)
//   [714, 723)  w4 o4 (8), b4.
// Each workgroup writes its unit sums; k_cnn2d_reduce adds them up in a
// fixed order (deterministic) and maps them to model-file order.

struct Unit {
    int kind;         // 0 product, 1 bias, 2 w4 / b4 (from the logit gradients)
    int p_off, p_step;   // dP (or h3): 4 channels at p_off + n p_step
    int q_off, q_step;   // input: 4 channels at q_off + n q_step (ones for a bias)
    bool is_b4;
};

__device__ Unit unit_of(int u, bool hz, const GradLds &G)
{
    // offsets are in bfloat16 elements from the start of GradLds
    const __bf16 *base = reinterpret_cast<const __bf16 *>(&G);
    auto off = [&](const __bf16 *p) { return (int)(p - base); };
    Unit U{0, 0, 0, 0, 0, false};
    auto taps = [&](int tap, int &da, int &dl) {
        const int dy = tap / 3, dx = tap - 3 * (tap / 3);
        da = hz ? dy : dx;
        dl = hz ? dx : dy;
    };
    int da = 0, dl = 0;
    if (u < 288) {
        const int o4 = u % 8, tap = (u / 8) % 9, c4 = u / 72;
        taps(tap, da, dl);
        U.p_off = off(G.dp3 + 32 + 4 * o4);
        U.p_step = 32;
        U.q_off = off(G.f.h2 + (da * kPos + dl) * 16 + 4 * c4);
        U.q_step = 16;
    } else if (u < 504) {
        const int v = u - 288;
        const int o4 = v % 4, tap = (v / 4) % 9, c4 = (v / 36) % 2, r = v / 72;
        taps(tap, da, dl);
        U.p_off = off(G.dp2 + (r * kPos + 1) * 16 + 4 * o4);
        U.p_step = 16;
        U.q_off = off(G.f.h1 + ((r + da) * kPos + dl) * 8 + 4 * c4);
        U.q_step = 8;
    } else if (u < 684) {
        const int v = u - 504;
        const int o4 = v % 2, tap = (v / 2) % 9, c4 = (v / 18) % 2, r = v / 36;
        taps(tap, da, dl);
        U.p_off = off(G.dp1 + (r * kPos + 1) * 8 + 4 * o4);
        U.p_step = 8;
        U.q_off = off(G.f.x0 + ((r + da) * kPos + dl) * 8 + 4 * c4);
        U.q_step = 8;
    } else if (u < 714) {
        U.kind = 1;
        U.q_off = off(G.ones);
        U.q_step = 0;
        if (u < 692) {
            U.p_off = off(G.dp3 + 32 + 4 * (u - 684));
            U.p_step = 32;
        } else if (u < 704) {
            const int v = u - 692;
            U.p_off = off(G.dp2 + ((v / 4) * kPos + 1) * 16 + 4 * (v % 4));
            U.p_step = 16;
        } else {
            const int v = u - 704;
            U.p_off = off(G.dp1 + ((v / 2) * kPos + 1) * 8 + 4 * (v % 2));
            U.p_step = 8;
        }
    } else {
        U.kind = 2;
        U.is_b4 = u == 722;
        U.p_off = off(G.f.h3 + 32 + 4 * (u - 714));
        U.p_step = 32;
    }
    return U;
}

__global__ __launch_bounds__(kBlock) void k_cnn2d_grad(Cnn2dTrainArgs a)
{
    extern __shared__ __align__(16) uint8_t c2_smem[];
    GradLds &G = *reinterpret_cast<GradLds *>(c2_smem);
    FwdLds &L = G.f;
    const __bf16 *lds = reinterpret_cast<const __bf16 *>(&G);
    const float *fb = L.fb;
    stage_floats(L, a.model);
    clear(L.x0, kC2Band * kPos * 8);
    clear(L.h1, 5 * kPos * 8);
    clear(L.h2, 3 * kPos * 16);
    clear(L.h3, kPos * 32);
    clear(G.dp3, kPos * 32);
    clear(G.dp2, 3 * kPos * 16);
    clear(G.dp1, 5 * kPos * 8);
    clear(G.zero, kPos * 32);
    if (threadIdx.x < 4)
        G.ones[threadIdx.x] = to_bf16(1.0f);
    float acc[3][16];
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int e = 0; e < 16; ++e)
            acc[s][e] = 0.0f;
    float loss = 0.0f;
    const int t = threadIdx.x;
    for (int wi = blockIdx.x; wi < a.n; wi += gridDim.x) {
        const int32_t *g = a.geom + 8 * wi;
        const bool hz = g[0] != 0;
        const int lo = uniform_int(a.range[2 * wi]), hi = uniform_int(a.range[2 * wi + 1]);
        const uint32_t line_ok = band_lines(g[1], hz ? g[4] : g[3]);
        const __bf16 *A = reinterpret_cast<const __bf16 *>(a.model) + (hz ? 0 : kC2Orient);
        __syncthreads();
        load_window(L, a.win + (int64_t)wi * (8 * kC2Win * 3), g, fb, line_ok, lo, hi);
        FwdW W;
        load_fwd_weights(W, a.model, hz, fb);
        __syncthreads();
        forward(L, W, line_ok, lo, hi);
        // logit gradients and the loss (soft binary cross entropy)
        if (t < kC2Win) {
            float dz = 0.0f;
            if (t >= kTrainHalo && t < kC2Win - kTrainHalo && t >= lo && t < hi) {
                const int q = t - kTrainHalo;
                const float tg = a.target[(int64_t)wi * kTrainOut + q];
                const float wt = a.weight[(int64_t)wi * kTrainOut + q];
                const float z = L.z[t];
                const float s = sigmoid(z);
                // -(t log s + (1 - t) log(1 - s)) = max(z, 0) - z t + log(1 + e^-|z|)
                loss += a.scale * wt * (fmaxf(z, 0.0f) - z * tg + log1pf(__expf(-fabsf(z))));
                dz = a.scale * wt * (s - tg);
            }
            G.dz[t] = dz;
        }
        __syncthreads();
        // w4 and b4 (before h3 is overwritten)
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int u = t + kBlock * s;
            if (u < 714 || u >= kC2Units)
                continue;
            const Unit U = unit_of(u, hz, G);
            for (int n = 0; n < kC2Win; ++n) {
                const float dz = G.dz[n];
                if (U.is_b4) {
                    acc[s][0] += dz;
                } else {
                    const bf16x4 h = *reinterpret_cast<const bf16x4 *>(lds + U.p_off + n * U.p_step);
#pragma unroll
                    for (int o = 0; o < 4; ++o)
                        acc[s][4 * o] += (float)h[o] * dz;
                }
            }
        }
        // dP3 = [h3 > 0] w4 dz
        for (int i = t; i < kC2Win * 32; i += kBlock) {
            const int n = i >> 5, o = i & 31;
            const float h = (float)L.h3[(n + 1) * 32 + o];
            G.dp3[(n + 1) * 32 + o] = to_bf16(h > 0.0f ? fb[kC2FW4 + o] * G.dz[n] : 0.0f);
        }
        __syncthreads();
        // dP2 = [h2 > 0] (flipped W3 * dP3): output lines 0..2 of layer 2;
        // the dP3 line sits at band line 3, i.e. input line 2 of the GEMM
        gemm3x3<32, 288, 1, 3>(load_frag<288, 1>(A + kC2F3), G.dp3, 2, 3, G.zero,
                               [&](int i, int m0, int n, const f32x4 &v) {
                                   const __bf16 *h = L.h2 + (i * kPos + n + 1) * 16 + m0;
                                   bf16x4 o;
#pragma unroll
                                   for (int j = 0; j < 4; ++j)
                                       o[j] = to_bf16((float)h[j] > 0.0f ? v[j] : 0.0f);
                                   *reinterpret_cast<bf16x4 *>(G.dp2 + (i * kPos + n + 1) * 16 + m0) = o;
                               });
        __syncthreads();
        // dP1 = [h1 > 0] (flipped W2 * dP2): lines 0..4 of layer 1; dP2 lines
        // are GEMM input lines 2..4
        gemm3x3<16, 160, 1, 5>(load_frag<160, 1>(A + kC2F2), G.dp2, 2, 5, G.zero,
                               [&](int i, int m0, int n, const f32x4 &v) {
                                   if (m0 >= 8)
                                       return;
                                   const __bf16 *h = L.h1 + (i * kPos + n + 1) * 8 + m0;
                                   bf16x4 o;
#pragma unroll
                                   for (int j = 0; j < 4; ++j)
                                       o[j] = to_bf16((float)h[j] > 0.0f ? v[j] : 0.0f);
                                   *reinterpret_cast<bf16x4 *>(G.dp1 + (i * kPos + n + 1) * 8 + m0) = o;
                               });
        __syncthreads();
        // weight and bias gradients
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int u = t + kBlock * s;
            if (u >= 714)
                continue;
            const Unit U = unit_of(u, hz, G);
            for (int n = 0; n < kC2Win; ++n) {
                const bf16x4 p = *reinterpret_cast<const bf16x4 *>(lds + U.p_off + n * U.p_step);
                const bf16x4 q = *reinterpret_cast<const bf16x4 *>(lds + U.q_off + n * U.q_step);
#pragma unroll
                for (int o = 0; o < 4; ++o)
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        acc[s][4 * o + c] += (float)p[o] * (float)q[c];
            }
        }
    }
    // loss: wave sums, then the workgroup's
#pragma unroll
    for (int dd = 32; dd >= 1; dd >>= 1)
        loss += __shfl_xor(loss, dd, 64);
    __syncthreads();
    if ((t & 63) == 0)
        G.loss[t >> 6] = loss;
    __syncthreads();
    float *out = a.partial + (int64_t)blockIdx.x * kC2GradStride;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const int u = t + kBlock * s;
        if (u < kC2Units)
#pragma unroll
            for (int e = 0; e < 16; ++e)
                out[16 * u + e] = acc[s][e];
    }
    if (t == 0) {
        float l = 0.0f;
        for (int w2 = 0; w2 < kBlock / 64; ++w2)
            l += G.loss[w2];
        out[16 * kC2Units] = l;
    }
}

// Gradient in model-file order from the workgroups' unit sums (fixed order:
// workgroups, then a layer's output lines); the normaliser gets zero.
__global__ __launch_bounds__(kBlock) void k_cnn2d_reduce(const float *partial, int grid,
                                                         float *grad, float *loss)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i > kC2Params)
        return;
    // the (unit, entry) pairs summed for parameter i
    int u0 = -1, e0 = 0, step = 0, count = 0;
    if (i == kC2Params) {
        u0 = kC2Units;
        count = 1;
    } else if (i >= kC2FileW[0] && i < kC2FileB4) {
        int l = 2;
        while (l > 0 && i < kC2FileW[l])
            --l;
        constexpr int cin[3] = {5, 8, 16}, cout[3] = {8, 16, 32};
        const int wn = cout[l] * cin[l] * 9;
        if (i >= kC2FileW4) {
            const int o = i - kC2FileW4;
            u0 = 714 + o / 4;
            e0 = 4 * (o % 4);
            count = 1;
        } else if (i < kC2FileW[l] + wn) {
            const int r = i - kC2FileW[l];
            const int o = r / (cin[l] * 9), c = (r / 9) % cin[l], tap = r % 9;
            e0 = 4 * (o % 4) + c % 4;
            if (l == 2) {
                u0 = o / 4 + 8 * (tap + 9 * (c / 4));
                count = 1;
            } else if (l == 1) {
                u0 = 288 + o / 4 + 4 * (tap + 9 * (c / 4));
                step = 72;
                count = 3;
            } else {
                u0 = 504 + o / 4 + 2 * (tap + 9 * (c / 4));
                step = 36;
                count = 5;
            }
        } else {
            const int o = i - (kC2FileW[l] + wn);
            e0 = 4 * (o % 4);
            if (l == 2) {
                u0 = 684 + o / 4;
                count = 1;
            } else if (l == 1) {
                u0 = 692 + o / 4;
                step = 4;
                count = 3;
            } else {
                u0 = 704 + o / 4;
                step = 2;
                count = 5;
            }
        }
    } else if (i == kC2FileB4) {
        u0 = 722;
        count = 1;
    }
    float v = 0.0f;
    for (int g = 0; g < grid; ++g)
        for (int k = 0; k < count; ++k)
            v += partial[(int64_t)g * kC2GradStride + 16 * (u0 + k * step) + e0];
    if (i == kC2Params)
        *loss = v;
    else
        grad[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_cnn2d_sgd(float *master, float *mom, const float *grad,
                                                      float lr, float mu)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= kC2Params)
        return;
    const float m = mu * mom[i] + grad[i];
    mom[i] = m;
    master[i] -= lr * m;
}

// Device model block from the float32 master weights (file order); every
// slot, padding included, is written.
__global__ __launch_bounds__(kBlock) void k_cnn2d_pack(const float *master, uint8_t *model)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    constexpr int cin[3] = {5, 8, 16}, cout[3] = {8, 16, 32}, cp[3] = {8, 8, 16};
    if (i < 2 * kC2Orient) {
        const int orient = i / kC2Orient, e = i - kC2Orient * (i / kC2Orient);
        float v = 0.0f;
        int l, o, c, da, dl;
        bool real = false;
        if (e >= kC2P1) {
            // layer 1 for two output lines at once: row m = 8 s + o is output
            // channel o of the pair's line s; K = (3 lo + dl) 8 + c over the
            // pair's four input lines lo = 0 .. 3 (tap da = lo - s)
            const int r = e - kC2P1;
            const int m = r / 96, k = r % 96;
            const int g = k / 8, sl = m / 8;
            l = 0;
            o = m % 8;
            c = k % 8;
            da = g / 3 - sl;
            dl = g % 3;
            real = c < cin[0] && da >= 0 && da < 3;
        } else if (e < kC2F2) {
            l = e < kC2A[1] ? 0 : e < kC2A[2] ? 1 : 2;
            const int r = e - kC2A[l];
            const int m = r / kC2KP[l], k = r % kC2KP[l];
            const int tap = k / cp[l];
            c = k % cp[l];
            o = m;
            da = tap / 3;
            dl = tap % 3;
            real = m < cout[l] && tap < 9 && c < cin[l];
        } else {
            l = e < kC2F3 ? 1 : 2;
            const int r = e - (l == 1 ? kC2F2 : kC2F3);
            const int kp = l == 1 ? 160 : 288;
            const int m = r / kp, k = r % kp;
            const int tap = k / cout[l];
            o = k % cout[l];
            c = m;
            da = 2 - tap / 3;
            dl = 2 - tap % 3;
            real = m < cin[l] && tap < 9;
        }
        if (real) {
            const int dy = orient == 0 ? da : dl, dx = orient == 0 ? dl : da;
            v = master[kC2FileW[l] + ((o * cin[l] + c) * 3 + dy) * 3 + dx];
        }
        reinterpret_cast<__bf16 *>(model)[i] = to_bf16(v);
        return;
    }
    const int f = i - 2 * kC2Orient;
    if (f >= 96)
        return;
    float *fb = reinterpret_cast<float *>(model + kC2FloatsOff);
    float v = 0.0f;
    if (f < 8)
        v = master[kC2FileB[0] + f];
    else if (f < 24)
        v = master[kC2FileB[1] + f - 8];
    else if (f < 56)
        v = master[kC2FileB[2] + f - 24];
    else if (f < 88)
        v = (float)to_bf16(master[kC2FileW4 + f - 56]);
    else if (f == 88)
        v = master[kC2FileB4];
    else if (f < 95)
        v = master[f - 89];     // mean[3], inv_std[3]
    fb[f] = v;
}

}  // namespace

hipError_t launch_cnn2d_strips(const Cnn2dStripArgs &a, hipStream_t s, hipEvent_t start,
                               hipEvent_t stop)
{
    if (a.n_items <= 0)
        return hipSuccess;
    launch_maybe_timed(k_cnn2d_strips, dim3(8 * a.per_xcd), dim3(kBlock), 0, s, start, stop, a);
    return hipGetLastError();
}

hipError_t launch_cnn2d_windows(const uint8_t *model, const uint8_t *win, const int32_t *geom,
                                const int32_t *range, float *z, int n, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    const int grid = n < 2048 ? n : 2048;
    hipLaunchKernelGGL(k_cnn2d_windows, dim3(grid), dim3(kBlock), 0, s, model, win, geom, range,
                       z, n);
    return hipGetLastError();
}

int cnn2d_grad_blocks_per_cu()
{
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_cnn2d_grad, kBlock, sizeof(GradLds))
            != hipSuccess
        || b < 1) {
        (void)hipGetLastError();
        b = 1;
    }
    return b;
}

hipError_t launch_cnn2d_grad(const Cnn2dTrainArgs &a, int grid, hipStream_t s)
{
    if (grid <= 0)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cnn2d_grad, dim3(grid), dim3(kBlock), sizeof(GradLds), s, a);
    return hipGetLastError();
}

hipError_t launch_cnn2d_reduce(const float *partial, int grid, float *grad_out, float *loss_out,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_cnn2d_reduce, dim3((kC2Params + 1 + kBlock - 1) / kBlock), dim3(kBlock),
                       0, s, partial, grid, grad_out, loss_out);
    return hipGetLastError();
}

hipError_t launch_cnn2d_update(float *master, float *momentum, const float *grad, float lr,
                               float mom, uint8_t *model, hipStream_t s)
{
    hipLaunchKernelGGL(k_cnn2d_sgd, dim3((kC2Params + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                       master, momentum, grad, lr, mom);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    return launch_cnn2d_pack(master, model, s);
}

hipError_t launch_cnn2d_pack(const float *master, uint8_t *model, hipStream_t s)
{
    constexpr int slots = 2 * kC2Orient + 96;
    hipLaunchKernelGGL(k_cnn2d_pack, dim3((slots + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                       master, model);
    return hipGetLastError();
}

}  // namespace ca
