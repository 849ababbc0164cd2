/* Device renderer of synthetic endoscopic frames (input generator of the
 * learned scorer's training set and of hard evaluation frames).  Not part of
 * the estimator: libcasynth.so is a separate library.
 *
 * The caller validates every recipe (the library reads what it is given):
 * grid_off .. grid_off + 5 control grids inside `grids`, glyph_off ..
 * glyph_off + text_lines * text_chars inside `glyphs` when text_scale > 0,
 * n_blobs <= 4, width/height >= 2, out_offset + 3 width height inside `out`,
 * window frame indices < the number of recipes.  Return 0, -1 for a bad
 * argument, -4 for a HIP launch error.  Asynchronous on `stream`. */
#pragma once
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t width, height, kind, n_blobs;
    float cx, cy, r, blur;
    float border_sigma, vignette, mean_luma, edge_step;  /* edge_step > 0: hard rim */
    float tint[3];
    int32_t grid_off;      /* control grids: base [gh0][gw0], fine [gh1][gw1], 3 chroma [gh0][gw0] */
    int32_t gh0, gw0, gh1, gw1;
    uint32_t key0, key1;   /* Philox key of the frame's noise */
    int32_t glyph_off, text_scale;
    float text_x, text_y;
    int32_t text_lines, text_chars;
    float blob[4][4];      /* x, y, radius, amplitude */
    int64_t out_offset;    /* byte offset of the frame in `out` (rows of 3 width bytes) */
    int32_t flags;         /* SYNTH_NO_NOISE: zero pixel and border noise */
    int32_t pad;
} SynthFrame;              /* 192 bytes */

#define SYNTH_NO_NOISE 1

/* Render n frames (uint8 RGB, row-major) into `out`; max_pixels = the largest
 * width * height among them. */
int synth_render_frames(const SynthFrame *frames_dev, int32_t n, int32_t max_pixels,
                        const float *grids_dev, const uint64_t *glyphs_dev, uint8_t *out_dev,
                        void *stream);

/* Render n training windows.  desc_dev: int32 [n][4] = (frame, horizontal,
 * line, start); window element k is strip position start + k.  Outputs:
 * win [n][8][128][3] uint8 (lines line-3 .. line+4, clamped to the frame),
 * range [n][2] (in-strip window positions), target [n][112] and weight
 * [n][112] of the central positions 8 .. 119. */
int synth_render_windows(const SynthFrame *frames_dev, const int32_t *desc_dev, int32_t n,
                         const float *grids_dev, const uint64_t *glyphs_dev, float edge_boost,
                         uint8_t *win_dev, int32_t *range_dev, float *target_dev,
                         float *weight_dev, void *stream);

#ifdef __cplusplus
}
#endif
