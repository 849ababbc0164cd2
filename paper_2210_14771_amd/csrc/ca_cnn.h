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

// Device model block: bfloat16 GEMM weights W_l[C_out][K_pad] with
// k = tap * C_in + c (zero padding to K_pad), then float32 biases of layers
// 1-4, the 16 weights (bfloat16 values) and the bias of the 1x1 layer.
constexpr int kCnnWOff[4] = {0, 16 * 128, 16 * 128 + 32 * 96, 16 * 128 + 32 * 96 + 32 * 160};
constexpr int kCnnWElems = 16 * 128 + 32 * 96 + 32 * 160 + 16 * 160;   // 12800
constexpr int kCnnBOff[4] = {0, 16, 48, 80};
constexpr int kCnnW5Off = 96;                                           // w5[16], then b5
constexpr int kCnnFloats = 96 + 16 + 1;
constexpr size_t kCnnModelBytes = (size_t)kCnnWElems * 2 + 128 * sizeof(float);
constexpr int kCnnParams = 12273;   // float32 parameters of the model file

struct __attribute__((aligned(16))) CnnLds {
    __bf16 w[kCnnWElems];
    float fb[128];
    __bf16 x0[kCnnRows * 24];
    __bf16 h1[kCnnRows * 16];
    __bf16 h2[kCnnRows * 32];
    __bf16 h3[kCnnRows * 32];
    __bf16 h4[kCnnRows * 16];
    float z[kCnnWin];
};

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

hipError_t launch_mfma_probe(float *out, hipStream_t s);
hipError_t launch_cnn_windows(const uint8_t *model, const uint8_t *win, const int32_t *range,
                              float *z, int n, hipStream_t s);
hipError_t launch_cnn_strips(const CnnStripArgs &a, hipStream_t s);

}  // namespace ca
