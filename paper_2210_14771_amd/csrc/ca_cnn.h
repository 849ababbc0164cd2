// Internal interface of the learned strip scorer (host core <-> kernels).
#pragma once

#include "ca_internal.h"

namespace ca {

// Geometry of a window: 128 positions, an 8-position halo at each end (the
// network's receptive-field radius), 112 exact logits in the middle.
constexpr int kCnnWin = 128;
constexpr int kCnnHalo = 8;
constexpr int kCnnOut = kCnnWin - 2 * kCnnHalo;
constexpr int kCnnGuard = 4;   // zero rows around each activation buffer
constexpr int kCnnRows = kCnnWin + 2 * kCnnGuard;
constexpr int kCnnLines = 8;   // lines across a learned strip: pos-3 .. pos+4
constexpr int kCnnWaveBlock = 128;   // inference workgroup: 2 waves, one window each

// Device model block: bfloat16 GEMM weights W_l[C_out][K_pad] with
// k = tap * C_in + c (zero padding to K_pad), then float32 biases of layers
// 1-4, the 16 weights (bfloat16 values) and the bias of the 1x1 layer.
constexpr int kCnnWOff[4] = {0, 16 * 128, 16 * 128 + 32 * 96, 16 * 128 + 32 * 96 + 32 * 160};
constexpr int kCnnWElems = 16 * 128 + 32 * 96 + 32 * 160 + 16 * 160;   // 12800
constexpr int kCnnBOff[4] = {0, 16, 48, 80};
constexpr int kCnnW5Off = 96;                                           // w5[16], then b5
constexpr int kCnnFloats = 96 + 16 + 1;
// Flipped weights for the input gradients of layers 2-4:
// Wf_l[c][t' C_out + o] = W_l[o][(4 - t') C_in + c], K' padded to 32.
constexpr int kCnnFOff[3] = {0, 16 * 160, 16 * 160 + 32 * 160};       // layers 2, 3, 4
constexpr int kCnnFElems = 16 * 160 + 32 * 160 + 32 * 96;              // 10752
constexpr size_t kCnnFloatsOff = (size_t)kCnnWElems * 2;               // byte offset
constexpr size_t kCnnFlipOff = kCnnFloatsOff + 128 * sizeof(float);    // byte offset
constexpr size_t kCnnModelBytes = kCnnFlipOff + (size_t)kCnnFElems * 2;
constexpr int kCnnParams = 12273;   // float32 parameters of the model file
// Gradient accumulators in GEMM layout: W1..W4 as kCnnWElems floats, then
// biases of layers 1-4 (96), w5 (16), b5, the loss: kCnnGradStride floats.
constexpr int kCnnGradStride = kCnnWElems + 128;

struct CnnStripArgs {
    const uint8_t *frames;
    const FrameDev *fd;
    const int32_t *strips;
    const uint8_t *model;
    ca_point *cand;
    int32_t n_h, n_v;
    int32_t n_items;
    int32_t per_xcd;
    int32_t frame0;
};

struct CnnTrainArgs {
    const uint8_t *model;     // device model block (weights read from global memory)
    const uint8_t *win;       // [n][8][128][3]
    const int32_t *range;     // [n][2]
    const float *target;      // [n][112]
    const float *weight;      // [n][112] loss weight per output position
    float *partial;           // [grid][kCnnGradStride]
    float scale;              // multiplies every position's loss term
    int32_t n;
};

hipError_t launch_cnn_grad(const CnnTrainArgs &a, int grid, hipStream_t s);
// Sum `grid` partials, then (file order) grad_out[i] and loss_out[0].
hipError_t launch_cnn_reduce(const float *partial, int grid, float *grad_out, float *loss_out,
                             hipStream_t s);
// SGD with momentum on the float32 master weights (file order), then repack
// the device model block.
hipError_t launch_cnn_update(float *master, float *momentum, const float *grad, float lr,
                             float mom, uint8_t *model, hipStream_t s);
// Repack the device model block from master weights.
hipError_t launch_cnn_pack(const float *master, uint8_t *model, hipStream_t s);

hipError_t launch_mfma_probe(float *out, hipStream_t s);
hipError_t launch_cnn_windows(const uint8_t *model, const uint8_t *win, const int32_t *range,
                              float *z, int n, hipStream_t s);
// Learned candidates; a.per_xcd = items per XCD slice, groups_per_xcd =
// workgroups per XCD (each takes the slice's items in turn).
hipError_t launch_cnn_strips(const CnnStripArgs &a, int groups_per_xcd, hipStream_t s,
                             hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
// Resident workgroups of k_cnn_strips per compute unit.
int cnn_strips_blocks_per_cu();

// ------------------------------------------------ 2-D scorer (paper) --
//
// The paper's own network: three 3x3 convolutions 5 -> 8 -> 16 -> 32 with
// ReLU, a 1x1 convolution to one logit, a sigmoid, on RGBXY bands of seven
// lines.  Model-file order (float32): mean[3], inv_std[3], W1[8][5][3][3],
// b1, W2[16][8][3][3], b2, W3[32][16][3][3], b3, w4[32], b4.
constexpr int kC2Params = 6215;
constexpr int kC2FileW[3] = {6, 374, 1542};     // file offsets of W1, W2, W3
constexpr int kC2FileB[3] = {366, 1526, 6150};  // and of b1, b2, b3
constexpr int kC2FileW4 = 6182;
constexpr int kC2FileB4 = 6214;
constexpr int kC2Win = 128;    // positions of a window
constexpr int kC2Band = 7;     // lines of a band
// Device model block, per band orientation (0: horizontal strips, weights
// [dy][dx]; 1: vertical strips, [dx][dy]): bfloat16 GEMM weights A[m][k]
// with k = (3 da + dl) C_pad + c for the forward convolutions, and flipped
// weights F[c][(3 da' + dl') C_out + o] = W[o][c][2 - da'][2 - dl'] for the
// input gradients of layers 2 and 3, and layer 1 again for two output lines
// at once (P[8 s + o][(3 lo + dl) 8 + c] = W1[o][c][lo - s][dl] over the
// pair's four input lines lo, zero where lo - s is not a tap); then float32
// b1, b2, b3, w4 (values of bfloat16), b4, mean, inv_std.
constexpr int kC2KP[3] = {96, 96, 160};          // padded K of the forward GEMMs
constexpr int kC2A[3] = {0, 16 * 96, 2 * 16 * 96};  // offsets within an orientation
constexpr int kC2F2 = 2 * 16 * 96 + 32 * 160;    // flipped layer 2: [16][160]
constexpr int kC2F3 = kC2F2 + 16 * 160;          // flipped layer 3: [16][288]
constexpr int kC2P1 = kC2F3 + 16 * 288;          // layer 1 by output-line pairs: [16][96]
constexpr int kC2Orient = kC2P1 + 16 * 96;       // bfloat16 elements per orientation
constexpr size_t kC2FloatsOff = (size_t)2 * kC2Orient * 2;
constexpr int kC2FB[3] = {0, 8, 24};             // float offsets of b1, b2, b3
constexpr int kC2FW4 = 56, kC2FB4 = 88, kC2FMean = 89, kC2FInv = 92;
constexpr size_t kC2ModelBytes = kC2FloatsOff + 96 * sizeof(float);
// Gradient partials: 723 units of 16 float32 sums (4 output channels x 4
// inputs), then the loss.
constexpr int kC2Units = 723;
constexpr int kC2GradStride = kC2Units * 16 + 16;

struct Cnn2dStripArgs {
    const uint8_t *frames;
    const FrameDev *fd;
    const int32_t *strips;
    const uint8_t *model;
    ca_point *cand;
    int32_t n_h, n_v;
    int32_t n_items;
    int32_t per_xcd;
    int32_t frame0;
};

struct Cnn2dTrainArgs {
    const uint8_t *model;
    const uint8_t *win;       // [n][8][128][3]: lines line-3 .. line+4
    const int32_t *geom;      // [n][8]: horizontal, line, start, width, height
    const int32_t *range;     // [n][2]
    const float *target;      // [n][112]
    const float *weight;      // [n][112]
    float *partial;           // [grid][kC2GradStride]
    float scale;
    int32_t n;
};

hipError_t launch_cnn2d_strips(const Cnn2dStripArgs &a, hipStream_t s, hipEvent_t start = nullptr,
                               hipEvent_t stop = nullptr);
hipError_t launch_cnn2d_windows(const uint8_t *model, const uint8_t *win, const int32_t *geom,
                                const int32_t *range, float *z, int n, hipStream_t s);
hipError_t launch_cnn2d_grad(const Cnn2dTrainArgs &a, int grid, hipStream_t s);
hipError_t launch_cnn2d_reduce(const float *partial, int grid, float *grad_out, float *loss_out,
                               hipStream_t s);
hipError_t launch_cnn2d_update(float *master, float *momentum, const float *grad, float lr,
                               float mom, uint8_t *model, hipStream_t s);
hipError_t launch_cnn2d_pack(const float *master, uint8_t *model, hipStream_t s);
int cnn2d_grad_blocks_per_cu();

}  // namespace ca
