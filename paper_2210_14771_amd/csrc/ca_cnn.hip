// gfx950 kernels of the learned strip scorer: a 1-D CNN along each strip
// whose output probability replaces the handcrafted edge score (arXiv
// 2210.14771, Section 2.2.4).  Input at each strip position: the 3 colours
// of 8 lines (24 channels, (v - 128) / 64, exact in bfloat16); four width-5
// convolutions 24 -> 16 -> 32 -> 32 -> 16 with ReLU, a 1x1 convolution to a
// logit, a sigmoid.  Weights and hidden activations are bfloat16, sums are
// float32 (MFMA accumulators).
//
// A strip is processed in windows of 128 positions advancing by 112: the
// 8 positions at each end of a window are the receptive-field halo, so the
// 112 central logits of every window are exact and the windows tile the
// strip.  Positions beyond the strip ends are zero in every layer's input.
//
// Each convolution is one GEMM per window: with activations stored
// position-major (channels contiguous), the 5 taps x C_in inputs of output
// position n are the contiguous run X[(n - 2) C_in .. (n + 3) C_in), so the
// im2col matrix is the activation buffer itself.  Tiles are
// v_mfma_f32_16x16x32_bf16: A = weights [C_out][5 C_in] (padded to a
// multiple of 32 with zeros), B = activations, 16 output channels x 16
// positions per tile.
#include "ca_cnn.h"
#include "ca_launch.h"

namespace ca {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

// One 16x16 tile of D = A (16 x 32k) * B (32k x 16) with A rows and B columns
// read as 8 consecutive bf16 per lane.  Lane l holds A[l % 16][8 (l / 16) ..]
// and B[8 (l / 16) ..][l % 16]; the result D[4 (l / 16) + j][l % 16], j < 4.
template <int KSTEPS>
__device__ __forceinline__ f32x4 mfma_tile(const __bf16 *a_row, const __bf16 *b_col)
{
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < KSTEPS; ++ks) {
        const bf16x8 a = *reinterpret_cast<const bf16x8 *>(a_row + 32 * ks);
        const bf16x8 b = *reinterpret_cast<const bf16x8 *>(b_col + 32 * ks);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
    return acc;
}

__device__ __forceinline__ __bf16 to_bf16(float v) { return (__bf16)v; }

// Forward convolution layer over a window: Y[n][m] = relu(b[m] + sum_k
// W[m][k] X[(n + G - 2) CIN + k]) for the 128 window positions, zero for
// positions outside [lo, hi).
template <int CIN, int COUT, int KP>
__device__ void conv_forward(const __bf16 *W, const float *bias, const __bf16 *X, __bf16 *Y, int lo,
                             int hi)
{
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    constexpr int MT = COUT / 16;
    constexpr int NT = kCnnWin / 16;
    const int kq = 8 * (lane >> 4);
    for (int tile = wv; tile < MT * NT; tile += 4) {
        const int mt = tile % MT;
        const int nt = tile / MT;
        const int m = mt * 16 + (lane & 15);
        const int n = nt * 16 + (lane & 15);
        const f32x4 acc = mfma_tile<KP / 32>(W + m * KP + kq, X + (n + kCnnGuard - 2) * CIN + kq);
        const int mo = mt * 16 + 4 * (lane >> 4);
        const bool inside = n >= lo && n < hi;
        __bf16 o[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float v = acc[j] + bias[mo + j];
            v = v > 0.0f ? v : 0.0f;
            o[j] = inside ? to_bf16(v) : to_bf16(0.0f);
        }
        __bf16 *dst = Y + (n + kCnnGuard) * COUT + mo;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            dst[j] = o[j];
    }
}

// Logits of all 128 window positions into z (valid for the central 112).
// Weights w (GEMM layout) may live in LDS or in global memory.
__device__ void window_forward(const __bf16 *w, const float *fb, const __bf16 *x0, __bf16 *h1,
                               __bf16 *h2, __bf16 *h3, __bf16 *h4, float *zo, int lo, int hi)
{
    conv_forward<24, 16, 128>(w + kCnnWOff[0], fb + kCnnBOff[0], x0, h1, lo, hi);
    __syncthreads();
    conv_forward<16, 32, 96>(w + kCnnWOff[1], fb + kCnnBOff[1], h1, h2, lo, hi);
    __syncthreads();
    conv_forward<32, 32, 160>(w + kCnnWOff[2], fb + kCnnBOff[2], h2, h3, lo, hi);
    __syncthreads();
    conv_forward<32, 16, 160>(w + kCnnWOff[3], fb + kCnnBOff[3], h3, h4, lo, hi);
    __syncthreads();
    const int n = threadIdx.x;
    if (n < kCnnWin) {
        const __bf16 *h = h4 + (n + kCnnGuard) * 16;
        float z = fb[kCnnW5Off + 16];
#pragma unroll
        for (int c = 0; c < 16; ++c)
            z = fmaf(fb[kCnnW5Off + c], (float)h[c], z);
        zo[n] = z;
    }
    __syncthreads();
}

// One uint8 window [8][128][3] into the position-major input buffer,
// zero outside [lo, hi).
__device__ void load_window(__bf16 *x0, const uint8_t *src, int lo, int hi)
{
    for (int i = threadIdx.x; i < kCnnLines * kCnnWin * 3; i += kBlock) {
        const int line = i / (kCnnWin * 3);
        const int rem = i - line * (kCnnWin * 3);
        const int n = rem / 3, ch = rem - 3 * (rem / 3);
        const float v = (n >= lo && n < hi) ? ((float)src[i] - 128.0f) * (1.0f / 64.0f) : 0.0f;
        x0[(n + kCnnGuard) * 24 + 3 * line + ch] = to_bf16(v);
    }
}

__device__ __forceinline__ float sigmoid(float z) { return 1.0f / (1.0f + __expf(-z)); }

// Clear the guard rows 0..G-1 and W+G..W+2G-1 of a position-major buffer.
__device__ void zero_guards(__bf16 *buf, int chans)
{
    for (int i = threadIdx.x; i < 2 * kCnnGuard * chans; i += kBlock) {
        const int row = i / chans;
        const int r = row < kCnnGuard ? row : kCnnWin + row;
        buf[r * chans + i % chans] = to_bf16(0.0f);
    }
}

// --------------------------------------------------- wave-level forward --
//
// Inference: one wavefront computes one whole window, with every weight
// fragment of the four convolutions resident in its registers (the A
// operands: 25 x 16 bytes per lane) and its own activation buffers in LDS, so
// the layers need no workgroup barrier.  Each B fragment (activations) is read
// once per k-step and used for every output-channel tile of the layer; the 1x1
// layer is folded into the last convolution's epilogue (a sum over the four
// lane groups holding a position's 16 channels).

// Two activation buffers per wave, 32 channels wide, used in turn: A holds
// the input (24 channels) and later the second layer's output, B the first
// and the third layer's.  Rows of one layout read under another (guard rows,
// the tail of a narrower layout) hold stale finite values; they only ever
// feed halo positions, whose outputs are discarded.
constexpr int kWaveBuf = kCnnRows * 32;                   // bf16 elements per buffer
constexpr int kWaveBytes = 2 * kWaveBuf * 2;              // A and B of one wave

struct WaveFrag {
    bf16x8 w1[1][4];
    bf16x8 w2[2][3];
    bf16x8 w3[2][5];
    bf16x8 w4[1][5];
    float b1[1][4], b2[2][4], b3[2][4], b4[1][4];
    float w5[4];
    float b5;
};

template <int MT, int KS>
__device__ __forceinline__ void load_frag(bf16x8 (&f)[MT][KS], float (&b)[MT][4], const __bf16 *W,
                                          const float *bias, int lane)
{
    constexpr int KP = KS * 32;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
            f[mt][ks] = *reinterpret_cast<const bf16x8 *>(W + (mt * 16 + (lane & 15)) * KP
                                                          + 32 * ks + 8 * (lane >> 4));
#pragma unroll
        for (int j = 0; j < 4; ++j)
            b[mt][j] = bias[mt * 16 + 4 * (lane >> 4) + j];
    }
}

__device__ void load_wave_frag(WaveFrag &fr, const uint8_t *model, int lane)
{
    const __bf16 *W = reinterpret_cast<const __bf16 *>(model);
    const float *fb = reinterpret_cast<const float *>(model + kCnnFloatsOff);
    load_frag<1, 4>(fr.w1, fr.b1, W + kCnnWOff[0], fb + kCnnBOff[0], lane);
    load_frag<2, 3>(fr.w2, fr.b2, W + kCnnWOff[1], fb + kCnnBOff[1], lane);
    load_frag<2, 5>(fr.w3, fr.b3, W + kCnnWOff[2], fb + kCnnBOff[2], lane);
    load_frag<1, 5>(fr.w4, fr.b4, W + kCnnWOff[3], fb + kCnnBOff[3], lane);
#pragma unroll
    for (int j = 0; j < 4; ++j)
        fr.w5[j] = fb[kCnnW5Off + 4 * (lane >> 4) + j];
    fr.b5 = fb[kCnnW5Off + 16];
}

// LDS written by some lanes of the wave and read by others next: keep the
// compiler from moving memory operations across (the hardware keeps a wave's
// LDS operations in order).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// One convolution layer over the window: groups of kNB position tiles with
// independent accumulators (their MFMA chains interleave), every output-
// channel tile per B fragment.
constexpr int kNB = 4;

// Element offset of channels c .. c + 7 (c a multiple of 4) of row `row` in
// a wave's position-major buffer of C channels.  With 32 or 16 channels the
// 16-byte chunks of a row are permuted by row (XOR with bits of the row
// index) so that the 16 lanes of one LDS pass, which read or write 16
// consecutive rows at the same channel, hit 16 distinct groups of 4 banks
// instead of 4 (32 channels) or 8 (16 channels); 24-channel rows already do.
// The permutation depends only on row / 4 mod 4 (row / 8 mod 2), so shifting
// by whole 16-row tiles keeps it.
template <int C>
__device__ __forceinline__ int act_off(int row, int c)
{
    static_assert(C == 16 || C == 24 || C == 32, "buffer width");
    if (C == 32)
        return row * 32 + ((((c >> 3) ^ (row >> 2)) & 3) << 3) + (c & 7);
    if (C == 16)
        return row * 16 + ((((c >> 3) ^ (row >> 3)) & 1) << 3) + (c & 7);
    return row * 24 + c;
}

template <int CIN, int COUT, int MT, int KS>
__device__ __forceinline__ void wave_conv(const bf16x8 (&A)[MT][KS], const float (&bias)[MT][4],
                                          const __bf16 *X, __bf16 *Y, int lo, int hi, int lane)
{
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    const int kq = 8 * (lane >> 4);
    // this lane's B-fragment offsets (K index 32 ks + kq = tap * CIN + c) and
    // output offsets, for position lane % 16; tiles 16 rows on add t 16 CIN
    int boff[KS], yoff[MT];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int k = 32 * ks + kq;
        boff[ks] = act_off<CIN>((lane & 15) + kCnnGuard - 2 + k / CIN, k % CIN);
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
        yoff[mt] = act_off<COUT>((lane & 15) + kCnnGuard, mt * 16 + 4 * (lane >> 4));
#pragma unroll 1
    for (int g = 0; g < kCnnWin / 16 / kNB; ++g) {
        const int n0 = g * kNB * 16 + (lane & 15);
        const __bf16 *b0 = X + g * kNB * 16 * CIN;
        // accumulators start at the bias
        f32x4 acc[kNB][MT];
#pragma unroll
        for (int t = 0; t < kNB; ++t)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                acc[t][mt] = f32x4{bias[mt][0], bias[mt][1], bias[mt][2], bias[mt][3]};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            bf16x8 bv[kNB];
#pragma unroll
            for (int t = 0; t < kNB; ++t)
                bv[t] = *reinterpret_cast<const bf16x8 *>(b0 + t * 16 * CIN + boff[ks]);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int t = 0; t < kNB; ++t)
                    acc[t][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt][ks], bv[t],
                                                                          acc[t][mt], 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < kNB; ++t) {
            const int n = n0 + 16 * t;
            // ReLU and the strip mask in one median: clamp to [0, +inf)
            // inside the strip, to [0, 0] outside
            const float top = (n >= lo && n < hi) ? __builtin_inff() : 0.0f;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                bf16x4 o;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    o[j] = to_bf16(__builtin_amdgcn_fmed3f(acc[t][mt][j], 0.0f, top));
                *reinterpret_cast<bf16x4 *>(Y + (n - (lane & 15)) * COUT + yoff[mt]) = o;
            }
        }
    }
}

// Last convolution (32 -> 16) with the 1x1 layer folded in: z[n] for the
// wave's 128 positions, handed out in two calls of `emit(n, z)` in which
// every lane holds one position (lane group q takes position tile q of the
// group), so the sigmoid and the argmax that follow run on full waves.
template <typename Emit>
__device__ __forceinline__ void wave_conv_out(const WaveFrag &fr, const __bf16 *X, int lo, int hi,
                                              int lane, Emit emit)
{
    const int kq = 8 * (lane >> 4);
    int boff[5];
#pragma unroll
    for (int ks = 0; ks < 5; ++ks)
        boff[ks] = act_off<32>((lane & 15) + kCnnGuard - 2 + ks, kq);
#pragma unroll 1
    for (int g = 0; g < kCnnWin / 16 / kNB; ++g) {
        const int n0 = g * kNB * 16 + (lane & 15);
        const __bf16 *b0 = X + g * kNB * 16 * 32;
        f32x4 acc[kNB];
#pragma unroll
        for (int t = 0; t < kNB; ++t)
            acc[t] = f32x4{fr.b4[0][0], fr.b4[0][1], fr.b4[0][2], fr.b4[0][3]};
#pragma unroll
        for (int ks = 0; ks < 5; ++ks) {
            bf16x8 bv[kNB];
#pragma unroll
            for (int t = 0; t < kNB; ++t)
                bv[t] = *reinterpret_cast<const bf16x8 *>(b0 + t * 16 * 32 + boff[ks]);
#pragma unroll
            for (int t = 0; t < kNB; ++t)
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fr.w4[0][ks], bv[t], acc[t], 0, 0,
                                                                 0);
        }
        static_assert(kNB == 4, "one position tile per lane group");
        float mine = 0.0f;
#pragma unroll
        for (int t = 0; t < kNB; ++t) {
            const int n = n0 + 16 * t;
            const float top = (n >= lo && n < hi) ? __builtin_inff() : 0.0f;
            float part = 0.0f;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float h = (float)to_bf16(__builtin_amdgcn_fmed3f(acc[t][j], 0.0f, top));
                part = fmaf(fr.w5[j], h, part);
            }
            part += __shfl_xor(part, 16, 64);
            part += __shfl_xor(part, 32, 64);
            mine = (lane >> 4) == t ? part : mine;
        }
        emit(n0 + 16 * (lane >> 4), fr.b5 + mine);
    }
}

// Logits of one window whose input rows are in w.x0: all 128 positions, in
// 2 calls of emit, one position per lane (positions outside the strip carry
// unspecified values).
template <typename Emit>
__device__ __forceinline__ void wave_forward(const WaveFrag &fr, __bf16 *A, __bf16 *B, int lo,
                                             int hi, int lane, Emit emit)
{
    wave_sync();
    wave_conv<24, 16, 1, 4>(fr.w1, fr.b1, A, B, lo, hi, lane);
    wave_sync();
    wave_conv<16, 32, 2, 3>(fr.w2, fr.b2, B, A, lo, hi, lane);
    wave_sync();
    wave_conv<32, 32, 2, 5>(fr.w3, fr.b3, A, B, lo, hi, lane);
    wave_sync();
    wave_conv_out(fr, B, lo, hi, lane, emit);
    wave_sync();
}

// Zero one wave's buffers once: afterwards every row holds a finite value.
// Guard rows and halo positions only ever feed halo outputs (the receptive
// field of a central position stays inside the window), so later windows
// may leave stale finite values there.
__device__ void wave_clear(__bf16 *x0, int lane)
{
    uint4 *p = reinterpret_cast<uint4 *>(x0);
    for (int i = lane; i < kWaveBytes / 16; i += 64)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// Gather one window of a strip into a wave's x0: lane l fills positions 2l and
// 2l + 1 (24 channels each: 8 lines x RGB, (v - 128) / 64); positions outside
// the strip are zero.  Where the pair lies inside the strip and every dword
// touched lies inside the frame (decided once per lane), bytes come from
// aligned dword loads split with v_alignbyte (a horizontal strip: 6 bytes of
// each of 8 rows; a vertical one: 24 bytes of each of 2 rows); elsewhere
// (strip ends, clamped lines, frame edges) from byte loads.
__device__ __forceinline__ void store_row24(__bf16 *row, const uint32_t (&u)[6])
{
    typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));
    bf16x8v *dst = reinterpret_cast<bf16x8v *>(row);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        bf16x8v o;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = 8 * c + e;
            const float b = (float)((u[k >> 2] >> (8 * (k & 3))) & 0xFFu);
            o[e] = to_bf16(fmaf(b, 1.0f / 64.0f, -2.0f));   // exact: (b - 128) / 64
        }
        dst[c] = o;
    }
}

__device__ __forceinline__ void wave_gather(__bf16 *x0, const uint8_t *frame, int W, int H, int rs,
                                            bool horizontal, int pos, int L, int start, int lane)
{
    const int p = start + 2 * lane;
    const int extent = horizontal ? H : W;
    // every dword window below stays inside the frame: horizontal, 3p - 3 >= 0
    // and 3p + 12 <= 3W; vertical, 3(pos - 3) - 3 >= 0 and 3(pos - 3) + 28 <= 3W
    const bool fast = p >= 0 && p + 1 < L
                      && (horizontal ? (p >= 1 && p <= W - 4) : (pos >= 4 && pos <= W - 7));
    uint32_t u[2][6];
    if (fast) {
        if (horizontal) {
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int i = 0; i < 6; ++i)
                    u[k][i] = 0;
#pragma unroll
            for (int j = 0; j < kCnnLines; ++j) {
                int row = pos + j - 3;
                row = row < 0 ? 0 : (row > extent - 1 ? extent - 1 : row);
                const uint8_t *q = frame + (int64_t)row * rs + 3 * p;
                const uint32_t sh = (uint32_t)(reinterpret_cast<uintptr_t>(q) & 3);
                const uint32_t *w = reinterpret_cast<const uint32_t *>(q - sh);
                const uint32_t w0 = w[0], w1 = w[1], w2 = w[2];
                const uint32_t b03 = __builtin_amdgcn_alignbyte(w1, w0, sh);
                const uint32_t b47 = __builtin_amdgcn_alignbyte(w2, w1, sh);
                // bytes 3j .. 3j + 2 of each position's 24
                const uint32_t p0 = b03 & 0xFFFFFFu;
                const uint32_t p1 = (b03 >> 24) | ((b47 & 0xFFFFu) << 8);
                const int k = 3 * j;
                u[0][k >> 2] |= p0 << (8 * (k & 3));
                if ((k & 3) > 1)
                    u[0][(k >> 2) + 1] |= p0 >> (32 - 8 * (k & 3));
                u[1][k >> 2] |= p1 << (8 * (k & 3));
                if ((k & 3) > 1)
                    u[1][(k >> 2) + 1] |= p1 >> (32 - 8 * (k & 3));
            }
        } else {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const uint8_t *q = frame + (int64_t)(p + k) * rs + 3 * (pos - 3);
                const uint32_t sh = (uint32_t)(reinterpret_cast<uintptr_t>(q) & 3);
                const uint32_t *w = reinterpret_cast<const uint32_t *>(q - sh);
                uint32_t wd[7];
#pragma unroll
                for (int i = 0; i < 7; ++i)
                    wd[i] = w[i];
#pragma unroll
                for (int i = 0; i < 6; ++i)
                    u[k][i] = __builtin_amdgcn_alignbyte(wd[i + 1], wd[i], sh);
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int pk = p + k;
#pragma unroll
            for (int i = 0; i < 6; ++i)
                u[k][i] = 0x80808080u;   // (128 - 128) / 64 = 0
            if (pk >= 0 && pk < L) {
#pragma unroll
                for (int j = 0; j < kCnnLines; ++j) {
                    int across = pos + j - 3;
                    across = across < 0 ? 0 : (across > extent - 1 ? extent - 1 : across);
                    const uint8_t *px = horizontal ? frame + (int64_t)across * rs + 3 * pk
                                                   : frame + (int64_t)pk * rs + 3 * across;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const int b = 3 * j + c;
                        u[k][b >> 2] = (u[k][b >> 2] & ~(0xFFu << (8 * (b & 3))))
                                       | ((uint32_t)px[c] << (8 * (b & 3)));
                    }
                }
            }
        }
    }
    store_row24(x0 + (2 * lane + kCnnGuard) * 24, u[0]);
    store_row24(x0 + (2 * lane + 1 + kCnnGuard) * 24, u[1]);
}

// --------------------------------------------------------------- kernels --

__global__ __launch_bounds__(kBlock) void k_mfma_probe(float *out)
{
    // A[m][k] = (m * 7 + k * 3) % 11 - 5, B[k][n] = (k * 5 + n * 2) % 13 - 6,
    // small integers: every product and sum is exact in float32.
    const int lane = threadIdx.x;
    if (lane >= 64)
        return;
    __bf16 a[8], b[8];
    for (int i = 0; i < 8; ++i) {
        const int k = 8 * (lane >> 4) + i;
        a[i] = to_bf16((float)(((lane & 15) * 7 + k * 3) % 11 - 5));
        b[i] = to_bf16((float)((k * 5 + (lane & 15) * 2) % 13 - 6));
    }
    const bf16x8 av = {a[0], a[1], a[2], a[3], a[4], a[5], a[6], a[7]};
    const bf16x8 bv = {b[0], b[1], b[2], b[3], b[4], b[5], b[6], b[7]};
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
    for (int j = 0; j < 4; ++j)
        out[(4 * (lane >> 4) + j) * 16 + (lane & 15)] = acc[j];
}

// Logits of the central positions of uint8 windows [n][8][128][3]: one
// wavefront per window.
__global__ __launch_bounds__(kCnnWaveBlock) void k_cnn_windows(const uint8_t *model,
                                                               const uint8_t *win,
                                                               const int32_t *range, float *z_out,
                                                               int n_windows)
{
    extern __shared__ __align__(16) uint8_t cnn_smem[];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    __bf16 *x0 = reinterpret_cast<__bf16 *>(cnn_smem + wv * kWaveBytes);
    __bf16 *hb = x0 + kWaveBuf;
    WaveFrag fr;
    load_wave_frag(fr, model, lane);
    wave_clear(x0, lane);
    const int waves = gridDim.x * (kCnnWaveBlock / 64);
    for (int wi = blockIdx.x * (kCnnWaveBlock / 64) + wv; wi < n_windows; wi += waves) {
        const int lo = uniform_int(range[2 * wi]);
        const int hi = uniform_int(range[2 * wi + 1]);
        const uint8_t *src = win + (int64_t)wi * (kCnnLines * kCnnWin * 3);
        wave_sync();
        for (int i = lane; i < kCnnLines * kCnnWin * 3; i += 64) {
            const int line = i / (kCnnWin * 3);
            const int rem = i - line * (kCnnWin * 3);
            const int n = rem / 3, ch = rem - 3 * (rem / 3);
            const float v = (n >= lo && n < hi) ? ((float)src[i] - 128.0f) * (1.0f / 64.0f) : 0.0f;
            x0[(n + kCnnGuard) * 24 + 3 * line + ch] = to_bf16(v);
        }
        wave_forward(fr, x0, hb, lo, hi, lane, [&](int n, float z) {
            if (n >= kCnnHalo && n < kCnnWin - kCnnHalo)
                z_out[(int64_t)wi * kCnnOut + n - kCnnHalo] = z;
        });
    }
}

// Learned candidates: both half strips of each (frame, strip) item, scored
// by the network, best pixel of each half (ties: outermost).  A workgroup of
// kCnnWaveBlock / 64 waves takes items in turn (XCD-aware slices); its waves
// share an item's windows.
__global__ __launch_bounds__(kCnnWaveBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_cnn_strips(CnnStripArgs a)
{
    extern __shared__ __align__(16) uint8_t cnn_smem[];
    __shared__ uint64_t s_best[kCnnWaveBlock / 64][2];
    constexpr int kWaves = kCnnWaveBlock / 64;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    __bf16 *x0 = reinterpret_cast<__bf16 *>(cnn_smem + wv * kWaveBytes);
    __bf16 *hb = x0 + kWaveBuf;
    const int xcd = blockIdx.x & 7;
    const int per_xcd_groups = gridDim.x >> 3;
    const int first = xcd * a.per_xcd;
    const int last = min(first + a.per_xcd, a.n_items);
    if (first + (int)(blockIdx.x >> 3) >= last)
        return;
    WaveFrag fr;
    load_wave_frag(fr, a.model, lane);
    wave_clear(x0, lane);
    const int S = a.n_h + a.n_v;
    for (int item = first + (int)(blockIdx.x >> 3); item < last; item += per_xcd_groups) {
        const int f = uniform_int(a.frame0 + item / S);
        const int st = uniform_int(item % S);
        const FrameDev d = a.fd[f];
        const uint8_t *frame = a.frames + d.offset;
        const bool horizontal = st < a.n_h;
        const int pos = uniform_int(a.strips[d.table + st]);
        const int L = uniform_int(horizontal ? d.W : d.H);
        const int n_win = (L + kCnnOut - 1) / kCnnOut;
        uint64_t best[2] = {0, 0};
        for (int w = wv; w < n_win; w += kWaves) {
            const int p0 = w * kCnnOut;
            const int start = p0 - kCnnHalo;
            const int lo = start >= 0 ? 0 : -start;
            const int hi = L - start < kCnnWin ? L - start : kCnnWin;
            wave_sync();
            wave_gather(x0, frame, d.W, d.H, d.rs, horizontal, pos, L, start, lane);
            wave_forward(fr, x0, hb, lo, hi, lane, [&](int n, float z) {
                const int p = start + n;
                if (n >= kCnnHalo && n < kCnnWin - kCnnHalo && p < L) {
                    const float sc = sigmoid(z);
                    const int half = p < (L >> 1) ? 0 : 1;
                    const int k = half == 0 ? p : L - 1 - p;
                    const uint64_t key = ((uint64_t)__float_as_uint(sc) << 32)
                                         | (uint64_t)(0xFFFFFFFFu - (uint32_t)k);
                    best[half] = best[half] > key ? best[half] : key;
                }
            });
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
            const int i = half == 0 ? k : L - 1 - k;
            ca_point pt;
            pt.x = (int16_t)(horizontal ? i : pos);
            pt.y = (int16_t)(horizontal ? pos : i);
            pt.score = __uint_as_float((uint32_t)(bb >> 32));
            a.cand[(int64_t)f * (2 * S) + 2 * st + half] = pt;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------- training --
//
// Backward pass of one window, given the forward activations (bfloat16) of
// the same window.  Backward signals dP_l (the gradient at layer l's
// pre-activation, ReLU mask applied) are stored in bfloat16, sums are float32
// MFMA accumulators.  Only the central 112 logits carry a loss; every
// activation they depend on is exact within the window, so the window's
// gradients equal those of the whole strip restricted to those positions.
//
//   input gradients   dX_{l-1} = flipped-weight convolution of dP_l (a
//                     forward-shaped GEMM), masked by h_{l-1} > 0;
//   weight gradients  dW_l[o][t C_in + c] = sum_n dP_l[n][o] X[n + t - 2][c],
//                     an MFMA GEMM whose reduction runs over the 128
//                     positions; the tiles stay in registers across all the
//                     windows of a workgroup;
//   bias gradients    per-thread sums of dP_l, reduced at the end.

struct __attribute__((aligned(16))) CnnGradLds {
    float fb[128];
    __bf16 x0[kCnnRows * 24];
    __bf16 h1[kCnnRows * 16];
    __bf16 h2[kCnnRows * 32];
    __bf16 h3[kCnnRows * 32];   // later dP2, position-major
    __bf16 h4[kCnnRows * 16];   // later dP4, position-major
    __bf16 d32[kCnnRows * 32];  // dP3, position-major
    __bf16 t[2][32 * kCnnWin];  // channel-major dP of two consecutive layers
    float z[kCnnWin];           // logits, then dL/dz
};

// Input gradient of one layer: Dout/Tout[n][c] = [h(n, c) > 0] * sum_k'
// Wf[c][k'] D[(n + G - 2) CI + k'], zero outside [lo, hi).  CI = channels of
// dP (the layer's outputs), CO = the layer's inputs.
template <int CI, int CO, int KP>
__device__ void input_grad(const __bf16 *Wf, const __bf16 *D, const __bf16 *Hmask, __bf16 *Dout,
                           __bf16 *Tout, int lo, int hi)
{
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    constexpr int MT = CO / 16;
    constexpr int NT = kCnnWin / 16;
    const int kq = 8 * (lane >> 4);
    for (int tile = wv; tile < MT * NT; tile += 4) {
        const int mt = tile % MT;
        const int nt = tile / MT;
        const int m = mt * 16 + (lane & 15);
        const int n = nt * 16 + (lane & 15);
        const f32x4 acc = mfma_tile<KP / 32>(Wf + m * KP + kq, D + (n + kCnnGuard - 2) * CI + kq);
        const int mo = mt * 16 + 4 * (lane >> 4);
        const bool inside = n >= lo && n < hi;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bool open = inside && (float)Hmask[(n + kCnnGuard) * CO + mo + j] > 0.0f;
            const __bf16 o = to_bf16(open ? acc[j] : 0.0f);
            if (Dout)
                Dout[(n + kCnnGuard) * CO + mo + j] = o;
            Tout[(mo + j) * kCnnWin + n] = o;
        }
    }
}

// Weight-gradient tiles of one layer, accumulated in registers: tile i of
// wave wv is tile wv + 4 i of the layer's (COUT / 16) x (KP / 16) tiles.
template <int CIN, int COUT, int KP, int NPW>
__device__ __forceinline__ void weight_grad(f32x4 (&acc)[NPW], const __bf16 *T, const __bf16 *X)
{
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    constexpr int MT = COUT / 16;
    constexpr int TILES = MT * (KP / 16);
    const int kq = 8 * (lane >> 4);
#pragma unroll
    for (int i = 0; i < NPW; ++i) {
        const int tile = wv + 4 * i;
        if (tile < TILES) {
            const int mt = tile % MT;
            const int nt = tile / MT;
            const __bf16 *a_row = T + (mt * 16 + (lane & 15)) * kCnnWin + kq;
            const __bf16 *b_col = X + (kq + kCnnGuard - 2) * CIN + nt * 16 + (lane & 15);
            f32x4 c = acc[i];
#pragma unroll
            for (int ks = 0; ks < kCnnWin / 32; ++ks) {
                const bf16x8 av = *reinterpret_cast<const bf16x8 *>(a_row + 32 * ks);
                bf16x8 bv;
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    bv[e] = b_col[(32 * ks + e) * CIN];
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
            }
            acc[i] = c;
        }
    }
}

template <int COUT, int KP, int NPW>
__device__ __forceinline__ void store_weight_grad(const f32x4 (&acc)[NPW], float *out)
{
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    constexpr int MT = COUT / 16;
    constexpr int TILES = MT * (KP / 16);
#pragma unroll
    for (int i = 0; i < NPW; ++i) {
        const int tile = wv + 4 * i;
        if (tile < TILES) {
            const int o = (tile % MT) * 16 + 4 * (lane >> 4);
            const int k = (tile / MT) * 16 + (lane & 15);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                out[(o + j) * KP + k] = acc[i][j];
        }
    }
}

// Sum of a channel-major dP over this thread's share of positions: 16
// channels -> 16 threads x 8 positions per channel, 32 -> 8 x 16.
template <int C>
__device__ __forceinline__ float bias_share(const __bf16 *T)
{
    constexpr int per = kCnnWin * C / kBlock;
    const int c = threadIdx.x / (kBlock / C);
    const int n0 = (threadIdx.x % (kBlock / C)) * per;
    float v = 0.0f;
#pragma unroll
    for (int i = 0; i < per; ++i)
        v += (float)T[c * kCnnWin + n0 + i];
    return v;
}

__global__ __launch_bounds__(kBlock) void k_cnn_grad(CnnTrainArgs a)
{
    __shared__ CnnGradLds s;
    const int tid = threadIdx.x;
    const __bf16 *W = reinterpret_cast<const __bf16 *>(a.model);
    const __bf16 *Wf = reinterpret_cast<const __bf16 *>(a.model + kCnnFlipOff);
    const float *mf = reinterpret_cast<const float *>(a.model + kCnnFloatsOff);
    for (int i = tid; i < 128; i += kBlock)
        s.fb[i] = i < kCnnFloats ? mf[i] : 0.0f;
    zero_guards(s.x0, 24);
    zero_guards(s.h1, 16);
    zero_guards(s.h2, 32);
    zero_guards(s.h3, 32);
    zero_guards(s.h4, 16);
    zero_guards(s.d32, 32);

    const f32x4 zero4 = {0.0f, 0.0f, 0.0f, 0.0f};
    f32x4 g1[2], g2[3], g3[5], g4[3];
#pragma unroll
    for (int i = 0; i < 2; ++i)
        g1[i] = zero4;
#pragma unroll
    for (int i = 0; i < 3; ++i)
        g2[i] = g4[i] = zero4;
#pragma unroll
    for (int i = 0; i < 5; ++i)
        g3[i] = zero4;
    float pb1 = 0.0f, pb2 = 0.0f, pb3 = 0.0f, pb4 = 0.0f, pw5 = 0.0f, pb5 = 0.0f, ploss = 0.0f;

    for (int wi = blockIdx.x; wi < a.n; wi += gridDim.x) {
        const int lo = uniform_int(a.range[2 * wi]);
        const int hi = uniform_int(a.range[2 * wi + 1]);
        load_window(s.x0, a.win + (int64_t)wi * (kCnnLines * kCnnWin * 3), lo, hi);
        __syncthreads();
        window_forward(W, s.fb, s.x0, s.h1, s.h2, s.h3, s.h4, s.z, lo, hi);

        // loss and dL/dz at the central positions inside the strip
        if (tid < kCnnWin) {
            const int n = tid;
            float dz = 0.0f;
            if (n >= kCnnHalo && n < kCnnWin - kCnnHalo && n >= lo && n < hi) {
                const int64_t j = (int64_t)wi * kCnnOut + (n - kCnnHalo);
                const float wt = a.weight[j] * a.scale;
                const float t = a.target[j];
                const float z = s.z[n];
                dz = wt * (sigmoid(z) - t);
                // soft binary cross entropy in its logit form
                ploss += wt * (fmaxf(z, 0.0f) - z * t + log1pf(expf(-fabsf(z))));
            }
            pb5 += dz;
            s.z[n] = dz;
        }
        __syncthreads();
        // layer 5 (1x1): dW5, and dP4 = [h4 > 0] w5 dz, in place of h4
        {
            const int c = tid & 15;
            const float w5 = s.fb[kCnnW5Off + c];
#pragma unroll
            for (int i = 0; i < kCnnWin * 16 / kBlock; ++i) {
                const int n = (tid >> 4) + 16 * i;
                const float h = (float)s.h4[(n + kCnnGuard) * 16 + c];
                const float dz = s.z[n];
                pw5 = fmaf(dz, h, pw5);
                const __bf16 v = to_bf16(h > 0.0f ? w5 * dz : 0.0f);
                s.h4[(n + kCnnGuard) * 16 + c] = v;
                s.t[0][c * kCnnWin + n] = v;
            }
        }
        __syncthreads();
        // layer 4: 32 -> 16
        weight_grad<32, 16, 160, 3>(g4, s.t[0], s.h3);
        input_grad<16, 32, 96>(Wf + kCnnFOff[2], s.h4, s.h3, s.d32, s.t[1], lo, hi);
        pb4 += bias_share<16>(s.t[0]);
        __syncthreads();
        // layer 3: 32 -> 32
        weight_grad<32, 32, 160, 5>(g3, s.t[1], s.h2);
        input_grad<32, 32, 160>(Wf + kCnnFOff[1], s.d32, s.h2, s.h3, s.t[0], lo, hi);
        pb3 += bias_share<32>(s.t[1]);
        __syncthreads();
        // layer 2: 16 -> 32
        weight_grad<16, 32, 96, 3>(g2, s.t[0], s.h1);
        input_grad<32, 16, 160>(Wf + kCnnFOff[0], s.h3, s.h1, nullptr, s.t[1], lo, hi);
        pb2 += bias_share<32>(s.t[0]);
        __syncthreads();
        // layer 1: 24 -> 16
        weight_grad<24, 16, 128, 2>(g1, s.t[1], s.x0);
        pb1 += bias_share<16>(s.t[1]);
        __syncthreads();
    }

    float *out = a.partial + (int64_t)blockIdx.x * kCnnGradStride;
    store_weight_grad<16, 128, 2>(g1, out + kCnnWOff[0]);
    store_weight_grad<32, 96, 3>(g2, out + kCnnWOff[1]);
    store_weight_grad<32, 160, 5>(g3, out + kCnnWOff[2]);
    store_weight_grad<16, 160, 3>(g4, out + kCnnWOff[3]);

    float *red = reinterpret_cast<float *>(&s.t[0][0]);   // 7 x 256 floats
    red[0 * kBlock + tid] = pb1;
    red[1 * kBlock + tid] = pb2;
    red[2 * kBlock + tid] = pb3;
    red[3 * kBlock + tid] = pb4;
    red[4 * kBlock + tid] = pw5;
    red[5 * kBlock + tid] = pb5;
    red[6 * kBlock + tid] = ploss;
    __syncthreads();
    if (tid < 128) {
        const int r = tid;
        float v = 0.0f;
        if (r < 16) {                       // b1: threads 16 r .. 16 r + 15
            for (int i = 0; i < 16; ++i)
                v += red[0 * kBlock + 16 * r + i];
        } else if (r < 48) {                // b2: threads 8 o .. 8 o + 7
            for (int i = 0; i < 8; ++i)
                v += red[1 * kBlock + 8 * (r - 16) + i];
        } else if (r < 80) {                // b3
            for (int i = 0; i < 8; ++i)
                v += red[2 * kBlock + 8 * (r - 48) + i];
        } else if (r < 96) {                // b4
            for (int i = 0; i < 16; ++i)
                v += red[3 * kBlock + 16 * (r - 80) + i];
        } else if (r < 112) {               // w5[c]: threads c + 16 i
            for (int i = 0; i < 16; ++i)
                v += red[4 * kBlock + (r - 96) + 16 * i];
        } else if (r == 112 || r == 113) {  // b5, loss
            for (int i = 0; i < kBlock; ++i)
                v += red[(r == 112 ? 5 : 6) * kBlock + i];
        }
        out[kCnnWElems + r] = v;
    }
}

// Parameter layout of the model file (float32): per layer W[o][c][t], b[o].
struct FileLayer {
    int cin, cout, kp, woff, fw, fb;
};
__device__ __forceinline__ FileLayer file_layer(int l)
{
    switch (l) {
    case 0: return {24, 16, 128, kCnnWOff[0], 0, 1920};
    case 1: return {16, 32, 96, kCnnWOff[1], 1936, 4496};
    case 2: return {32, 32, 160, kCnnWOff[2], 4528, 9648};
    default: return {32, 16, 160, kCnnWOff[3], 9680, 12240};
    }
}
constexpr int kFileW5 = 12256;
constexpr int kFileB5 = 12272;

// Sum the workgroup partials; scatter to the model-file order.
__global__ __launch_bounds__(kBlock) void k_cnn_reduce(const float *partial, int grid,
                                                       float *grad, float *loss)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= kCnnGradStride)
        return;
    float v = 0.0f;
    for (int g = 0; g < grid; ++g)
        v += partial[(int64_t)g * kCnnGradStride + i];
    if (i < kCnnWElems) {
        const int l = i < kCnnWOff[1] ? 0 : i < kCnnWOff[2] ? 1 : i < kCnnWOff[3] ? 2 : 3;
        const FileLayer L = file_layer(l);
        const int o = (i - L.woff) / L.kp;
        const int k = (i - L.woff) - o * L.kp;
        if (k >= 5 * L.cin)
            return;
        const int t = k / L.cin, c = k - t * L.cin;
        grad[L.fw + (o * L.cin + c) * 5 + t] = v;
        return;
    }
    const int r = i - kCnnWElems;
    if (r < 96) {
        const int l = r < kCnnBOff[1] ? 0 : r < kCnnBOff[2] ? 1 : r < kCnnBOff[3] ? 2 : 3;
        grad[file_layer(l).fb + r - kCnnBOff[l]] = v;
    } else if (r < 112) {
        grad[kFileW5 + r - 96] = v;
    } else if (r == 112) {
        grad[kFileB5] = v;
    } else if (r == 113) {
        loss[0] = v;
    }
}

// SGD with momentum: m = mu m + g, p -= lr m.
__global__ __launch_bounds__(kBlock) void k_cnn_sgd(float *master, float *mom, const float *grad,
                                                    float lr, float mu)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= kCnnParams)
        return;
    const float m = mu * mom[i] + grad[i];
    mom[i] = m;
    master[i] -= lr * m;
}

// Device model block from float32 master weights: every slot (padding
// included) is written.
__global__ __launch_bounds__(kBlock) void k_cnn_pack(const float *master, uint8_t *model)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    __bf16 *w = reinterpret_cast<__bf16 *>(model);
    float *fb = reinterpret_cast<float *>(model + kCnnFloatsOff);
    __bf16 *wf = reinterpret_cast<__bf16 *>(model + kCnnFlipOff);
    if (i < kCnnWElems) {
        const int l = i < kCnnWOff[1] ? 0 : i < kCnnWOff[2] ? 1 : i < kCnnWOff[3] ? 2 : 3;
        const FileLayer L = file_layer(l);
        const int o = (i - L.woff) / L.kp;
        const int k = (i - L.woff) - o * L.kp;
        float v = 0.0f;
        if (k < 5 * L.cin) {
            const int t = k / L.cin, c = k - t * L.cin;
            v = master[L.fw + (o * L.cin + c) * 5 + t];
        }
        w[i] = to_bf16(v);
        return;
    }
    int r = i - kCnnWElems;
    if (r < 128) {
        float v = 0.0f;
        if (r < 96) {
            const int l = r < kCnnBOff[1] ? 0 : r < kCnnBOff[2] ? 1 : r < kCnnBOff[3] ? 2 : 3;
            v = master[file_layer(l).fb + r - kCnnBOff[l]];
        } else if (r < 112) {
            v = (float)to_bf16(master[kFileW5 + r - 96]);
        } else if (r == 112) {
            v = master[kFileB5];
        }
        fb[r] = v;
        return;
    }
    r -= 128;
    if (r < kCnnFElems) {
        // Wf_l[c][t' C_out + o] = W_l[o][c][4 - t'] for layers 2, 3, 4
        const int q = r < kCnnFOff[1] ? 0 : r < kCnnFOff[2] ? 1 : 2;
        const FileLayer L = file_layer(q + 1);
        const int kpf = q == 2 ? 96 : 160;
        const int c = (r - kCnnFOff[q]) / kpf;
        const int k = (r - kCnnFOff[q]) - c * kpf;
        float v = 0.0f;
        if (k < 5 * L.cout) {
            const int tp = k / L.cout, o = k - tp * L.cout;
            v = master[L.fw + (o * L.cin + c) * 5 + (4 - tp)];
        }
        wf[r] = to_bf16(v);
    }
}

}  // namespace

hipError_t launch_mfma_probe(float *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_mfma_probe, dim3(1), dim3(kBlock), 0, s, out);
    return hipGetLastError();
}

constexpr size_t kCnnWaveLds = (size_t)(kCnnWaveBlock / 64) * kWaveBytes;

hipError_t launch_cnn_windows(const uint8_t *model, const uint8_t *win, const int32_t *range,
                              float *z, int n, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    const int waves = kCnnWaveBlock / 64;
    int grid = (n + waves - 1) / waves;
    grid = grid < 1024 ? grid : 1024;
    hipLaunchKernelGGL(k_cnn_windows, dim3(grid), dim3(kCnnWaveBlock), kCnnWaveLds, s, model, win,
                       range, z, n);
    return hipGetLastError();
}

int cnn_strips_blocks_per_cu()
{
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_cnn_strips, kCnnWaveBlock, kCnnWaveLds)
            != hipSuccess
        || b < 1) {
        (void)hipGetLastError();
        b = 1;
    }
    return b;
}

hipError_t launch_cnn_strips(const CnnStripArgs &a, int groups_per_xcd, hipStream_t s,
                             hipEvent_t start, hipEvent_t stop)
{
    if (a.n_items <= 0)
        return hipSuccess;
    launch_maybe_timed(k_cnn_strips, dim3(8 * groups_per_xcd), dim3(kCnnWaveBlock), kCnnWaveLds, s,
                       start, stop, a);
    return hipGetLastError();
}

}  // namespace ca

namespace ca {

hipError_t launch_cnn_grad(const CnnTrainArgs &a, int grid, hipStream_t s)
{
    if (grid <= 0)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cnn_grad, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cnn_reduce(const float *partial, int grid, float *grad_out, float *loss_out,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_cnn_reduce, dim3((kCnnGradStride + kBlock - 1) / kBlock), dim3(kBlock), 0,
                       s, partial, grid, grad_out, loss_out);
    return hipGetLastError();
}

hipError_t launch_cnn_update(float *master, float *momentum, const float *grad, float lr,
                             float mom, uint8_t *model, hipStream_t s)
{
    hipLaunchKernelGGL(k_cnn_sgd, dim3((kCnnParams + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                       master, momentum, grad, lr, mom);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    return launch_cnn_pack(master, model, s);
}

hipError_t launch_cnn_pack(const float *master, uint8_t *model, hipStream_t s)
{
    constexpr int slots = kCnnWElems + 128 + kCnnFElems;
    hipLaunchKernelGGL(k_cnn_pack, dim3((slots + kBlock - 1) / kBlock), dim3(kBlock), 0, s, master,
                       model);
    return hipGetLastError();
}

}  // namespace ca
