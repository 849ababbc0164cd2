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
__device__ void window_forward(CnnLds &s, int lo, int hi)
{
    const __bf16 *w = s.w;
    conv_forward<24, 16, 128>(w + kCnnWOff[0], s.fb + kCnnBOff[0], s.x0, s.h1, lo, hi);
    __syncthreads();
    conv_forward<16, 32, 96>(w + kCnnWOff[1], s.fb + kCnnBOff[1], s.h1, s.h2, lo, hi);
    __syncthreads();
    conv_forward<32, 32, 160>(w + kCnnWOff[2], s.fb + kCnnBOff[2], s.h2, s.h3, lo, hi);
    __syncthreads();
    conv_forward<32, 16, 160>(w + kCnnWOff[3], s.fb + kCnnBOff[3], s.h3, s.h4, lo, hi);
    __syncthreads();
    const int n = threadIdx.x;
    if (n < kCnnWin) {
        const __bf16 *h = s.h4 + (n + kCnnGuard) * 16;
        float z = s.fb[kCnnW5Off + 16];
#pragma unroll
        for (int c = 0; c < 16; ++c)
            z = fmaf(s.fb[kCnnW5Off + c], (float)h[c], z);
        s.z[n] = z;
    }
    __syncthreads();
}

// Copy the model into LDS and clear the guard rows of the activation buffers.
__device__ void load_model(CnnLds &s, const uint8_t *model)
{
    const uint4 *src = reinterpret_cast<const uint4 *>(model);
    uint4 *dst = reinterpret_cast<uint4 *>(s.w);
    constexpr int n16 = (kCnnWElems * 2) / 16;
    for (int i = threadIdx.x; i < n16; i += kBlock)
        dst[i] = src[i];
    const float *fsrc = reinterpret_cast<const float *>(model + kCnnWElems * 2);
    for (int i = threadIdx.x; i < kCnnFloats; i += kBlock)
        s.fb[i] = fsrc[i];
    __bf16 *bufs[5] = {s.x0, s.h1, s.h2, s.h3, s.h4};
    const int chans[5] = {24, 16, 32, 32, 16};
    for (int b = 0; b < 5; ++b)
        for (int i = threadIdx.x; i < 2 * kCnnGuard * chans[b]; i += kBlock) {
            const int row = i / chans[b];
            const int r = row < kCnnGuard ? row : kCnnWin + row;  // rows 0..G-1 and W+G..W+2G-1
            bufs[b][r * chans[b] + i % chans[b]] = to_bf16(0.0f);
        }
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

// Logits of the central positions of uint8 windows [n][8][128][3].
__global__ __launch_bounds__(kBlock) void k_cnn_windows(const uint8_t *model, const uint8_t *win,
                                                        const int32_t *range, float *z_out,
                                                        int n_windows)
{
    __shared__ CnnLds s;
    load_model(s, model);
    for (int wi = blockIdx.x; wi < n_windows; wi += gridDim.x) {
        const int lo = uniform_int(range[2 * wi]);
        const int hi = uniform_int(range[2 * wi + 1]);
        const uint8_t *src = win + (int64_t)wi * (kCnnLines * kCnnWin * 3);
        for (int i = threadIdx.x; i < kCnnLines * kCnnWin * 3; i += kBlock) {
            const int line = i / (kCnnWin * 3);
            const int rem = i - line * (kCnnWin * 3);
            const int n = rem / 3, ch = rem - 3 * (rem / 3);
            const float v = (n >= lo && n < hi) ? ((float)src[i] - 128.0f) * (1.0f / 64.0f) : 0.0f;
            s.x0[(n + kCnnGuard) * 24 + 3 * line + ch] = to_bf16(v);
        }
        __syncthreads();
        window_forward(s, lo, hi);
        const int t = threadIdx.x;
        if (t < kCnnOut)
            z_out[(int64_t)wi * kCnnOut + t] = s.z[t + kCnnHalo];
        __syncthreads();
    }
}

// Learned candidates: both half strips of each (frame, strip) item, scored
// by the network, best pixel of each half (ties: outermost).
__global__ __launch_bounds__(kBlock) void k_cnn_strips(CnnStripArgs a)
{
    __shared__ CnnLds s;
    __shared__ uint64_t s_best[4];
    const int b = blockIdx.x;
    const int item = (b & 7) * a.per_xcd + (b >> 3);
    if (item >= a.n_items)
        return;
    load_model(s, a.model);
    const int S = a.n_h + a.n_v;
    const int f = uniform_int(a.frame0 + item / S);
    const int st = uniform_int(item % S);
    const FrameDev d = a.fd[f];
    const uint8_t *frame = a.frames + d.offset;
    const bool horizontal = st < a.n_h;
    const int pos = uniform_int(a.strips[d.table + st]);
    const int L = uniform_int(horizontal ? d.W : d.H);
    const int extent = horizontal ? d.H : d.W;
    const int tid = threadIdx.x;
    uint64_t best[2] = {0, 0};
    for (int p0 = 0; p0 < L; p0 += kCnnOut) {
        const int lo = p0 >= kCnnHalo ? 0 : kCnnHalo - p0;
        const int hi = L - p0 + kCnnHalo < kCnnWin ? L - p0 + kCnnHalo : kCnnWin;
        // gather: 8 lines x 128 positions x 3 colours
        for (int i = tid; i < kCnnLines * kCnnWin; i += kBlock) {
            int line, n;
            if (horizontal) {
                line = i / kCnnWin;
                n = i - line * kCnnWin;
            } else {
                n = i / kCnnLines;
                line = i - n * kCnnLines;
            }
            const int p = p0 - kCnnHalo + n;
            __bf16 *dst = s.x0 + (n + kCnnGuard) * 24 + 3 * line;
            if (p < 0 || p >= L) {
                dst[0] = dst[1] = dst[2] = to_bf16(0.0f);
                continue;
            }
            int across = pos + line - 3;
            across = across < 0 ? 0 : (across > extent - 1 ? extent - 1 : across);
            const uint8_t *px = horizontal ? frame + (int64_t)across * d.rs + 3 * p
                                           : frame + (int64_t)p * d.rs + 3 * across;
            dst[0] = to_bf16(((float)px[0] - 128.0f) * (1.0f / 64.0f));
            dst[1] = to_bf16(((float)px[1] - 128.0f) * (1.0f / 64.0f));
            dst[2] = to_bf16(((float)px[2] - 128.0f) * (1.0f / 64.0f));
        }
        __syncthreads();
        window_forward(s, lo, hi);
        if (tid < kCnnOut) {
            const int p = p0 + tid;
            if (p < L) {
                const float sc = 1.0f / (1.0f + __expf(-s.z[tid + kCnnHalo]));
                const int half = p < (L >> 1) ? 0 : 1;
                const int k = half == 0 ? p : L - 1 - p;
                const uint64_t key = ((uint64_t)__float_as_uint(sc) << 32)
                                     | (uint64_t)(0xFFFFFFFFu - (uint32_t)k);
                best[half] = best[half] > key ? best[half] : key;
            }
        }
        __syncthreads();
    }
    // reduce the two keys over the workgroup
    const int lane = tid & 63, wv = tid >> 6;
    for (int half = 0; half < 2; ++half) {
        uint64_t v = best[half];
#pragma unroll
        for (int dd = 32; dd >= 1; dd >>= 1) {
            const uint64_t t = __shfl_xor(v, dd, 64);
            v = v > t ? v : t;
        }
        if (lane == 0)
            s_best[wv] = v;
        __syncthreads();
        if (tid == 0) {
            uint64_t bb = s_best[0];
            for (int w2 = 1; w2 < 4; ++w2)
                bb = bb > s_best[w2] ? bb : s_best[w2];
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

}  // namespace

hipError_t launch_mfma_probe(float *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_mfma_probe, dim3(1), dim3(kBlock), 0, s, out);
    return hipGetLastError();
}

hipError_t launch_cnn_windows(const uint8_t *model, const uint8_t *win, const int32_t *range,
                              float *z, int n, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    const int grid = n < 1024 ? n : 1024;
    hipLaunchKernelGGL(k_cnn_windows, dim3(grid), dim3(kBlock), 0, s, model, win, range, z, n);
    return hipGetLastError();
}

hipError_t launch_cnn_strips(const CnnStripArgs &a, hipStream_t s)
{
    if (a.n_items <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_cnn_strips, dim3(8 * a.per_xcd), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace ca
