/*
 * contentarea.h -- C ABI of the MI355X (gfx950) endoscopic content-area
 * estimator.
 *
 * The method is the "lean GPU-based pipeline" of Budd et al., arXiv
 * 2210.14771, Section 2.2: sample horizontal (and here also vertical) strips
 * of each RGB frame (Section 2.2.2, Eq. 1), score every pixel of each half
 * strip from its Sobel gradient magnitude, the angle between the gradient
 * and the direction to the image centre and the maximum intensity preceding
 * it (Section 2.2.3, Eqs. 2-3), keep the best pixel of each half strip,
 * filter, and fit a circle by RANSAC over point triples with least-squares
 * refits (Section 2.2.5).  The result per frame is a circle, or "no circle":
 * the content area is then the whole frame (Section 2.2.1).
 *
 * Conventions
 *   - Frames are 8-bit RGB, channel-interleaved (R, G, B per pixel), rows
 *     `row_stride` bytes apart.  Coordinates are pixel indices: pixel
 *     (x, y) has its centre at (x, y); +x right, +y down.
 *   - Device pointers are HIP device memory of the context's device.  The
 *     library only reads `frames_dev` and only writes the output array.
 *   - `stream` is a hipStream_t (NULL: the legacy default stream).  Every
 *     call only enqueues work: results are ready when the stream has
 *     completed it.  The caller keeps the frames and outputs alive until then.
 *   - Every entry point returns CA_OK (0) or a negative CA_E_* code and never
 *     throws.  Argument errors are detected before anything is enqueued.
 *     Device faults surface at the caller's next stream synchronisation.
 *   - A context is not thread-safe: use one context per host thread.
 *     Calls on one context may target different streams; the context
 *     serialises its own scratch use by enqueuing on the given stream, so
 *     calls on two different streams of one context must not overlap.
 *   - Contexts are independent (each owns its buffers): calls of several
 *     contexts on one device may overlap on different streams.  Keeping a
 *     few batches in flight that way lets one batch's RANSAC (FP64 ALU) run
 *     beside other batches' strip loads (HBM).
 */
#ifndef CONTENTAREA_H
#define CONTENTAREA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CA_OK 0
#define CA_E_INVAL (-1)        /* null pointer or argument out of range */
#define CA_E_UNSUPPORTED (-2)  /* layout the library does not handle (pixel_stride != 3) */
#define CA_E_NOMEM (-3)        /* workspace budget of the context exceeded */
#define CA_E_DEVICE (-4)       /* a HIP runtime call failed */
#define CA_E_SCRATCH (-5)      /* batch larger than ca_estimate_area_noalloc's fixed scratch */

#define CA_MAX_STRIPS 64       /* per direction */
#define CA_MAX_ATTEMPTS 4096
#define CA_MAX_EXTENT 16384    /* largest width or height */

/* Opaque context: device, cached strip tables and score tables, workspace. */
typedef struct ca_ctx ca_ctx;

/* One frame of a batch (32 bytes). */
typedef struct {
    int32_t width, height;   /* pixels, each in [16, CA_MAX_EXTENT] */
    int32_t row_stride;      /* bytes between the starts of two rows, >= 3 * width */
    int32_t pixel_stride;    /* bytes between pixels; must be 3 (packed RGB; planar or padded
                                pixels, and a separate stride between channels, are not
                                supported: other values return CA_E_UNSUPPORTED) */
    int64_t byte_offset;     /* first byte of the frame relative to `frames_dev`, >= 0;
                                bytes [byte_offset, byte_offset + (height - 1) * row_stride
                                + 3 * width) must lie in the caller's allocation (the
                                library cannot see device extents and reads only these) */
    uint64_t frame_uid;      /* identifies the frame to the RANSAC sampler: the
                                triples depend on (seed, frame_uid, attempt) only,
                                never on the frame's position in the batch */
} ca_frame_desc;

/* Parameters: Appendix A, Table A1, plus the vertical strips, the RANSAC
 * attempt count and the sampler.  Get the paper's values from
 * ca_default_params() and override fields. */
typedef struct {
    int32_t n_hstrips;       /* N horizontal strips, Eq. 1 (16) */
    int32_t n_vstrips;       /* vertical strips along the width (16; 0 = paper-literal) */
    double alpha;            /* strip weighting toward the frame edges, Eq. 1 (8) */
    double t_g;              /* gradient magnitude soft threshold, Eq. 2 (20) */
    double t_theta_deg;      /* gradient direction soft threshold in degrees, Eq. 2 (30) */
    double t_iota;           /* preceding maximum intensity soft threshold, Eq. 2 (25) */
    double t_ps;             /* point score threshold (0.03), compared in float32 */
    double t_cs;             /* circle score threshold (0.06) on sum(inlier scores) / P */
    int32_t t_px;            /* candidates closer than this to the frame edge are dropped (3) */
    int32_t refine_iters;    /* least-squares refits per attempt (3) */
    double t_ri;             /* inlier distance in pixels (3) */
    double r_min, r_max;     /* radius limits, multiples of the width (0.1, 0.8) */
    double d_max;            /* centre offset limit, multiple of the width (0.2) */
    int32_t ransac_attempts; /* attempts per frame, [1, CA_MAX_ATTEMPTS] (256) */
    int32_t sampler;         /* 0 random triples; 1 the a-th triple in lexicographic order */
    uint64_t seed;           /* key of the counter-based sampler */
    int32_t scorer;          /* CA_SCORER_HANDCRAFTED (Section 2.2.3) or CA_SCORER_LEARNED
                                (Section 2.2.4; needs ca_set_model; t_px is not applied) */
    float fallback_inlier_frac; /* learned scorer only: a frame whose best circle has
                                   inliers < fallback_inlier_frac * n_points (or fewer than
                                   3 kept points) takes the handcrafted pipeline's result
                                   instead; 0 (default) = no fallback; [0, 1] */
} ca_params;

#define CA_SCORER_HANDCRAFTED 0
#define CA_SCORER_LEARNED 1
#define CA_SCORER_LEARNED_2D 2  /* the paper's own network (ca_set_model_2d) */
#define CA_REASON_FALLBACK 256

/* Result per frame (32 bytes). */
typedef struct {
    float cx, cy, r;         /* best circle, pixel-index coordinates (0 if none) */
    float score;             /* sum of the circle's inlier scores / P, P = 2 (n_hstrips + n_vstrips) */
    int32_t inliers;         /* inliers of the best circle */
    int32_t n_points;        /* candidate points kept after filtering */
    int32_t valid;           /* 1: content area = disc within the frame; 0: whole frame */
    int32_t reason;          /* 0 valid, 1 fewer than 3 points, 2 no attempt within the
                                radius and centre limits, 3 best score below t_cs;
                                + CA_REASON_FALLBACK when the learned scorer's result
                                was replaced by the handcrafted one */
} ca_result;

/* Best pixel of one half strip (8 bytes).  Frame f's P candidates are
 * stored at [f * P, (f + 1) * P) in canonical order: horizontal strip i
 * gives 2i (left half) and 2i+1 (right half); vertical strip j gives
 * 2 n_hstrips + 2j (top) and 2 n_hstrips + 2j + 1 (bottom). */
typedef struct {
    int16_t x, y;
    float score;             /* s = s_g s_theta s_iota, Eq. 3 */
} ca_point;

/* One RANSAC attempt (56 bytes), for tests. */
typedef struct {
    int32_t status;          /* 0 degenerate, 1 outside the radius/centre limits, 2 kept */
    int32_t fail_stage;      /* status 0: 0 collinear triple, k refit k had < 3 inliers
                                or a singular system, -1 no triple (enumeration exhausted) */
    int32_t i0, i1, i2;      /* triple, indices into the kept points (canonical order) */
    int32_t inliers;         /* inliers of the final circle */
    uint64_t qsum;           /* sum over those inliers of floor(score * 2^24) */
    double cx, cy, r2;       /* final circle: centre and squared radius */
} ca_attempt;

/* Fill `p` with the paper's defaults (Table A1); 16 + 16 strips, 256 random
 * attempts, seed 0. */
void ca_default_params(ca_params *p);

/* Create a context on HIP device `device`.  `workspace_budget_bytes` caps the
 * device memory the context may hold for tables and scratch (0 = 1 GiB).
 * Returns CA_E_INVAL for a null `ctx` or a bad device, CA_E_DEVICE if HIP
 * fails. */
int ca_create(ca_ctx **ctx, int device, size_t workspace_budget_bytes);

/* Release everything the context holds.  Synchronises the device first.
 * Null is ignored. */
void ca_destroy(ca_ctx *ctx);

/* Estimate the content area of `n_frames` frames (Section 2.2).
 *   frames_dev  device base address of the frames (read only)
 *   dims_host   host array of n_frames descriptors (copied during the call)
 *   params      host pointer (copied during the call); NULL = defaults
 *   out_dev     device array of n_frames results (written by the stream)
 * n_frames = 0 is a no-op.  Errors: CA_E_INVAL (null pointer, size or
 * parameter out of range), CA_E_UNSUPPORTED (pixel_stride != 3), CA_E_NOMEM
 * (budget too small for this batch; the context stays usable), CA_E_DEVICE. */
int ca_estimate_area(ca_ctx *ctx, const uint8_t *frames_dev, const ca_frame_desc *dims_host,
                     int32_t n_frames, const ca_params *params, ca_result *out_dev,
                     void *stream);

/* ca_estimate_area without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results and errors as
 * ca_estimate_area, computed by the same kernels.  Instead of the
 * context's cached per-batch buffers, the call uses one fixed array in
 * device memory of CA_NOALLOC_SCRATCH_BYTES per GPU, which the library
 * holds until the process ends and which every call on that GPU shares
 * (it keeps the last call's contents; each call rewrites what it reads).
 * Calls that overlap on one GPU -- on two streams, or from two contexts --
 * therefore race: serialise them (one stream per GPU).  The call uploads
 * its descriptors and tables from host memory the library holds with one
 * copy on `stream`, and waits on the host for the previous call's upload
 * to have been read.  Limits: at most CA_NOALLOC_MAX_FRAMES frames of at
 * most CA_NOALLOC_MAX_SHAPES distinct shapes, and the layout must fit the
 * scratch (about 3.6 KB per frame at 64 + 64 strips and 4096 attempts);
 * beyond them CA_E_SCRATCH, with nothing enqueued. */
#define CA_NOALLOC_SCRATCH_BYTES (4u << 20)
#define CA_NOALLOC_MAX_FRAMES 1024
#define CA_NOALLOC_MAX_SHAPES 64
int ca_estimate_area_noalloc(ca_ctx *ctx, const uint8_t *frames_dev,
                             const ca_frame_desc *dims_host, int32_t n_frames,
                             const ca_params *params, ca_result *out_dev, void *stream);

/* The same pipeline, additionally writing every frame's P candidates
 * (Section 2.2.5, first sentence) to `points_dev` (n_frames * P entries). */
int ca_debug_candidates(ca_ctx *ctx, const uint8_t *frames_dev, const ca_frame_desc *dims_host,
                        int32_t n_frames, const ca_params *params, ca_point *points_dev,
                        ca_result *out_dev, void *stream);

/* The same pipeline, additionally writing every RANSAC attempt
 * (n_frames * ransac_attempts records, frame-major) to `attempts_dev`.
 * Frames with fewer than 3 kept points get all-zero records. */
int ca_debug_attempts(ca_ctx *ctx, const uint8_t *frames_dev, const ca_frame_desc *dims_host,
                      int32_t n_frames, const ca_params *params, ca_attempt *attempts_dev,
                      ca_result *out_dev, void *stream);

/* Learned strip scorer (Section 2.2.4): a 1-D CNN along each strip.  Input
 * at each strip position: the R, G, B values v of 8 lines (pos-3 .. pos+4,
 * clamped) as (v - 128) / 64, 24 channels; four width-5 convolutions
 * 24 -> 16 -> 32 -> 32 -> 16 with ReLU and zero padding beyond the strip ends,
 * a 1x1 convolution to one logit, score = sigmoid(logit).  Weights and
 * hidden activations are bfloat16, sums float32.
 *
 * Model file: CA_CNN_PARAMS float32 values in the order W1[16][24][5], b1[16],
 * W2[32][16][5], b2[32], W3[32][32][5], b3[32], W4[16][32][5], b4[16],
 * W5[1][16][1], b5[1] (W[out][in][tap]); weights are rounded to bfloat16
 * when loaded. */
#define CA_CNN_PARAMS 12273
#define CA_CNN_WINDOW 128      /* positions per window */
#define CA_CNN_OUTPUTS 112     /* exact logits per window: positions 8 .. 119 */

/* Load (host pointer) the model used by scorer CA_SCORER_LEARNED.  The values
 * become the context's float32 master weights (training starts from them
 * with zero momentum); the device model holds their bfloat16 roundings.
 * Blocking.  CA_E_INVAL for a wrong count or a non-finite value. */
int ca_set_model(ca_ctx *ctx, const float *params_host, int32_t n_params);

/* Copy the master weights and, when `momentum_host` is not NULL, the SGD
 * momentum (CA_CNN_PARAMS floats each, model-file order) to the host.
 * Blocking.  CA_E_INVAL without a model. */
int ca_get_model(ca_ctx *ctx, float *params_host, float *momentum_host, int32_t n_params);

/* Replace the SGD momentum (host array, model-file order), e.g. to resume
 * training from a checkpoint taken with ca_get_model.  Blocking. */
int ca_set_momentum(ca_ctx *ctx, const float *momentum_host, int32_t n_params);

/* The paper's own learned scorer (Section 2.2.4), scorer
 * CA_SCORER_LEARNED_2D: three 3x3 convolutions with 8, 16 and 32 output
 * features, each followed by a ReLU, a 1x1 convolution to one logit, score =
 * sigmoid(logit), on five input channels per pixel, RGBXY: each colour v as
 * bf16((v - mean_c) * inv_std_c) in float32 arithmetic (the training data's
 * per-channel statistics, part of the model), the pixel coordinates as
 * bf16((2x - (W - 1)) / (2 (W - 1))) and likewise for y, in [-0.5, 0.5] with
 * 0 at the image centre.  Every layer's input is zero outside the frame
 * ("same" zero padding).  Applied to strips seven lines thick, the
 * receptive field, so a strip's scores are the whole-image network's output
 * on the strip's line.  Weights and hidden activations are bfloat16, sums
 * float32.
 *
 * Model file: CA_CNN2D_PARAMS float32 values in the order mean[3],
 * inv_std[3], W1[8][5][3][3], b1[8], W2[16][8][3][3], b2[16],
 * W3[32][16][3][3], b3[32], w4[32], b4[1] (W[out][in][dy][dx], channels
 * R, G, B, X, Y); weights are rounded to bfloat16 when loaded.  The
 * normaliser (the first 6 values) is not trained: its gradient is zero. */
#define CA_CNN2D_PARAMS 6215

/* Load (host pointer) the model used by CA_SCORER_LEARNED_2D; as
 * ca_set_model (master weights, zero momentum).  Blocking.  CA_E_INVAL for a
 * wrong count, a non-finite value or a non-positive inv_std. */
int ca_set_model_2d(ca_ctx *ctx, const float *params_host, int32_t n_params);

/* As ca_get_model and ca_set_momentum, for the 2-D model.  Blocking. */
int ca_get_model_2d(ca_ctx *ctx, float *params_host, float *momentum_host, int32_t n_params);
int ca_set_momentum_2d(ca_ctx *ctx, const float *momentum_host, int32_t n_params);

/* Logits of the CA_CNN_OUTPUTS central positions (8 .. 119) of n rendered
 * windows under the 2-D model.
 *   windows_dev  uint8 [n][8][CA_CNN_WINDOW][3]: lines line-3 .. line+4 of
 *                a strip (clamped to the frame; the network uses the first 7)
 *   geom_dev     int32 [n][8]: horizontal (1: the strip is a row), line,
 *                start (frame position of window position 0), frame width,
 *                frame height, 0, 0, 0
 *   range_dev    int32 [n][2]: window positions [lo, hi) inside the strip
 *   logits_dev   float [n][CA_CNN_OUTPUTS]
 * Enqueued on `stream`.  Needs ca_set_model_2d. */
int ca_cnn2d_window_logits(ca_ctx *ctx, const uint8_t *windows_dev, const int32_t *geom_dev,
                           const int32_t *range_dev, int32_t n_windows, float *logits_dev,
                           void *stream);

/* Gradients of the 2-D model, as ca_cnn_gradients (the same loss over the
 * central positions of windows, the same argument meanings, plus geom_dev as
 * for ca_cnn2d_window_logits); grad_dev holds CA_CNN2D_PARAMS floats in
 * model-file order.  The backward pass stores its signals in bfloat16 and
 * sums in float32.  The calls of one context share a gradient workspace:
 * calls that overlap on different streams race. */
int ca_cnn2d_gradients(ca_ctx *ctx, const uint8_t *windows_dev, const int32_t *geom_dev,
                       const int32_t *range_dev, const float *target_dev,
                       const float *weight_dev, int32_t n_windows, float scale, float *grad_dev,
                       float *loss_dev, void *stream);

/* One SGD step with momentum on the 2-D model's master weights (as
 * ca_cnn_sgd_step), then the device model is rebuilt from them. */
int ca_cnn2d_sgd_step(ca_ctx *ctx, const float *grad_dev, float lr, float momentum,
                      void *stream);

/* Training (Section 2.2.4: soft binary cross entropy against blurred edge
 * labels, SGD).  Gradients, with respect to the master weights, of
 *   L = scale * sum_i sum_j weight[i][j] * BCE(sigmoid(z_ij), target[i][j])
 * over n windows of the current model, z_ij the logit of central position
 * 8 + j of window i (the forward pass of ca_cnn_window_logits).  The
 * backward pass stores its signals in bfloat16 and sums in float32; each
 * hidden unit's ReLU passes the gradient where its stored activation is > 0.
 *   windows_dev  uint8 [n][8][CA_CNN_WINDOW][3], as for ca_cnn_window_logits
 *   range_dev    int32 [n][2], as for ca_cnn_window_logits; central
 *                positions outside [lo, hi) carry no loss
 *   target_dev   float [n][CA_CNN_OUTPUTS], soft labels in [0, 1]
 *   weight_dev   float [n][CA_CNN_OUTPUTS], >= 0
 *   grad_dev     float [CA_CNN_PARAMS], written in model-file order
 *   loss_dev     float [1], the value of L
 * Enqueued on `stream` (device pointers, asynchronous).  The context's
 * gradient workspace is shared by its calls: calls that overlap on
 * different streams race.  n = 0 writes zeros.  Needs ca_set_model. */
int ca_cnn_gradients(ca_ctx *ctx, const uint8_t *windows_dev, const int32_t *range_dev,
                     const float *target_dev, const float *weight_dev, int32_t n_windows,
                     float scale, float *grad_dev, float *loss_dev, void *stream);

/* One SGD step with momentum on the master weights, m = mu m + g,
 * p = p - lr m (g: device array of CA_CNN_PARAMS floats in model-file
 * order), then the device model is rebuilt from p.  Enqueued on `stream`. */
int ca_cnn_sgd_step(ca_ctx *ctx, const float *grad_dev, float lr, float momentum,
                    void *stream);

/* Logits of windows (for tests and training data checks): `windows_dev` is
 * uint8 [n][8][CA_CNN_WINDOW][3] (line, position, colour); `range_dev` is
 * int32 [n][2]: positions lo .. hi-1 of each window lie inside its strip (the
 * others are zero in every layer's input).  Writes float32
 * [n][CA_CNN_OUTPUTS] logits of positions 8 .. 119 (values at positions
 * outside the strip are unspecified).  Needs ca_set_model. */
int ca_cnn_window_logits(ca_ctx *ctx, const uint8_t *windows_dev, const int32_t *range_dev,
                         int32_t n_windows, float *logits_dev, void *stream);

/* Diagnostic: one v_mfma_f32_16x16x32_bf16 on fixed integer inputs
 * A[m][k] = (7m + 3k) mod 11 - 5, B[k][n] = (5k + 2n) mod 13 - 6; writes the
 * 16 x 16 product row-major to `out_dev` (256 floats). */
int ca_selftest_mfma(ca_ctx *ctx, float *out_dev, void *stream);

/* Host-side helpers (no device work). */

/* The argument checks ca_estimate_area applies before enqueuing anything:
 * CA_OK, CA_E_INVAL or CA_E_UNSUPPORTED.  `params` NULL = defaults. */
int ca_check_args(const ca_frame_desc *dims_host, int32_t n_frames, const ca_params *params);

/* Eq. 1 positions of n strips along an axis of `extent` pixels: floor, then
 * clamped to [1, extent - 2].  Returns CA_E_INVAL for extent < 3 or n < 0. */
int ca_strip_positions(int32_t extent, int32_t n, double alpha, int32_t *pos);

/* Score tables of Eq. 2 as the kernels use them: sg[q] = tanh(q / (8 t_g))
 * for q < *sg_len (the table stops at the first entry equal to 1.0f; larger
 * indices read the last entry), st[q] = 1 - tanh(theta_q / t_theta) for the
 * 2049 pseudo-angle bins, si[i] = 1 - tanh(i / t_iota) for 256 levels.
 * `sg` must hold CA_SG_CAPACITY floats; `sg_len` receives the used length. */
#define CA_SG_CAPACITY 11541
int ca_score_tables(const ca_params *p, float *sg, int32_t *sg_len, float *st, float *si);

/* A captured HIP graph replaying `calls` estimate calls on fixed buffers:
 * for callers that run the same batch layout repeatedly (a serving loop, a
 * benchmark) and want one launch instead of one per kernel. */
typedef struct ca_graph ca_graph;

/* Capture `calls` back-to-back calls of ca_estimate_area with these
 * arguments into a graph (the plan is built first, outside the capture).
 * The graph keeps the device pointers: the frames and `out_dev` must stay
 * allocated, and the context alive, until ca_graph_destroy.  The context's
 * plan for this batch is never evicted while a graph uses it.  Each launch
 * recomputes every result from the current contents of the frames.
 * Errors as ca_estimate_area; `calls` in [1, 4096]. */
int ca_graph_create(ca_ctx *ctx, const uint8_t *frames_dev, const ca_frame_desc *dims_host,
                    int32_t n_frames, const ca_params *params, ca_result *out_dev,
                    int32_t calls, ca_graph **graph);

/* Enqueue one replay on `stream` (a hipStream_t; NULL: default stream). */
int ca_graph_launch(ca_graph *graph, void *stream);

/* Synchronise the device and release the graph.  Null is ignored. */
void ca_graph_destroy(ca_graph *graph);

/* Schedule options of a context (ca_set_option / ca_get_option). */
#define CA_OPT_SCHEDULE 1      /* CA_SCHEDULE_AUTO (default), CA_SCHEDULE_SPLIT or
                                  CA_SCHEDULE_FUSED */
#define CA_OPT_LAG 2           /* fused: frames between a frame's strip and RANSAC work (4) */
#define CA_OPT_QUEUES 3        /* fused: work queues 1..8; 0 = 8 for >= 16 frames, else 1 */
#define CA_OPT_GRID 4          /* fused: workgroups; 0 = as many as fit on the device */
#define CA_OPT_SPIN_LIMIT 5    /* fused: polls before a wait gives up (a guard, 2^20) */
#define CA_OPT_PIPELINE 6      /* split: sub-batches per call, alternating over two
                                  internal streams forked from and joined into the
                                  caller's stream (1 = everything on the caller's
                                  stream); 0 (default) = under CA_SCHEDULE_AUTO the
                                  count ca_autotune measured fastest for the batch
                                  (1, 2 or 4), else 1 */
#define CA_OPT_STRIPS_PER_GROUP 7  /* split: strip items per workgroup tile, 1..16, for
                                      every frame shape; 0 (default) = the autotuned value
                                      of each shape (ca_autotune), else 1 */
#define CA_OPT_RANSAC_LANES 8  /* split: lanes per RANSAC attempt, 2, 4, 8 or 16 (a
                                  workgroup takes 256 / lanes attempts); 0 (default) = the
                                  fewest lanes that give the batch at least one attempt
                                  workgroup per compute unit, at most 8.  Results do
                                  not depend on it. */
#define CA_SCHEDULE_SPLIT 0    /* per (sub-)batch two launches: strip scoring, then RANSAC
                                  whose last group per frame selects the circle */
#define CA_SCHEDULE_FUSED 1    /* one persistent launch drawing both kinds of work from
                                  per-XCD queues; same results */
#define CA_SCHEDULE_AUTO 2     /* per batch the schedule ca_autotune measured fastest
                                  (split in one call when the batch was not tuned) */

/* Autotuner of the split schedule's strip tiles.  A workgroup of the strip
 * kernel stages the score tables in LDS once and then scores T strip items
 * in turn (T = 1, 2, 4, 8); frames of each distinct shape in a batch are
 * launched together with their own T.  For each frame shape of the batch
 * (enqueued on `stream`, frames as for ca_estimate_area), times `reps`
 * launches of the strip kernel per candidate T with HIP events and keeps
 * the fastest for (width, height, n_hstrips, n_vstrips) in the context.
 * Then (handcrafted scorer) it times `reps` whole calls of the batch under
 * the split schedule with those tiles, in one call and in 2 and 4 pipelined
 * sub-batches (CA_OPT_PIPELINE), and under the persistent fused schedule,
 * each both eagerly and as a replayed one-call graph (a candidate counts by
 * the slower of the two), and keeps the fastest for this batch (used with
 * CA_SCHEDULE_AUTO and the
 * pipeline option at 0); *schedule_out (may be NULL) receives its schedule,
 * ca_get_last_autotune the schedule and sub-batch count.  Later calls (and
 * graphs captured later) use the results.  Blocking.  Results never depend
 * on T, on the sub-batches or on the schedule. */
int ca_autotune(ca_ctx *ctx, const uint8_t *frames_dev, const ca_frame_desc *dims_host,
                int32_t n_frames, const ca_params *params, int32_t reps, void *stream,
                int32_t *schedule_out);

/* What the last ca_autotune of this context chose for its batch: the
 * schedule (CA_SCHEDULE_SPLIT or CA_SCHEDULE_FUSED; -1 before any) and the
 * sub-batches of its split calls (0 before any).  Host pointers. */
int ca_get_last_autotune(ca_ctx *ctx, int32_t *schedule, int32_t *pipeline);

/* The tuned T of a frame shape and strip counts (0 if not tuned). */
int ca_get_tuning(ca_ctx *ctx, int32_t width, int32_t height, int32_t n_hstrips,
                  int32_t n_vstrips, int32_t *strips_per_group);

/* Set or read an option.  CA_E_INVAL for an unknown option or value. */
int ca_set_option(ca_ctx *ctx, int32_t option, int64_t value);
int ca_get_option(ca_ctx *ctx, int32_t option, int64_t *value);

/* Synchronise the device and report whether every fused call so far ended
 * its waits normally (CA_OK), or whether one gave up at the spin limit
 * (CA_E_DEVICE: the results of that call are not to be trusted).  Clears
 * the flag. */
int ca_device_status(ca_ctx *ctx);

/* Kernel timing (HIP events taken by each kernel's own dispatch, so each
 * duration is the kernel's execution alone).  Index 0: strip scoring, 1:
 * RANSAC with selection, 2: the gap between them.  When a call is one fused
 * kernel it is reported at index 0; a pipelined set of sub-batches, or the
 * per-shape strip launches of a mixed batch, between marker events recorded
 * on the caller's stream. */
typedef struct {
    double total_ms[3];      /* summed kernel durations */
    int64_t launches[3];     /* number of timed launches */
} ca_kernel_times;

/* Start timing the next `max_calls` estimate calls of this context (events
 * are created here, none during the calls).  CA_E_INVAL for max_calls < 1. */
int ca_profile_begin(ca_ctx *ctx, int32_t max_calls);

/* Wait for the timed calls, write their totals and release the events. */
int ca_profile_end(ca_ctx *ctx, ca_kernel_times *out);

/* ---------------------------------------------------------------- serving --
 * Continuous batching of many video streams (the per-frame method of
 * Section 2.2 applied to live footage; temporal filtering with the circle
 * score as confidence is the extension named in Section 4).
 *
 * A stream is opened with its frame shape and is admitted when its frame
 * ring (ring_slots frames of 3 width height bytes) fits in the server's HBM
 * budget and fewer than max_streams streams are admitted; otherwise it waits
 * (first come, first served) until closed streams free memory.  Frames are
 * submitted per stream in sequence order; each takes a free slot of its
 * stream's ring (frames wait on the host while the ring is full), is copied
 * into it on the server's HIP stream, and joins the next batch.  ca_server_step
 * makes progress without blocking: it retires finished batches, admits
 * streams, starts copies and, while fewer than max_inflight batches are on
 * the GPU, launches the frames that are ready as one batch.  Frames that
 * arrive while other batches run are admitted as slots free up, so work of
 * different arrivals overlaps on the device.
 *
 * Per-stream state stays on the device: after each batch a kernel folds every
 * frame's result, in sequence order, into its stream's filtered circle:
 * with score q of a valid result and decay lambda = `smooth`,
 *   w' = lambda w + q,  c' = (lambda w c + q c_frame) / w'  (centre and radius),
 * and w' = lambda w for an invalid one.  A frame's own result depends only on
 * its bytes, the parameters and its RNG uid (stream_id << 32 | seq mod 2^32);
 * the filtered circle only on its stream's earlier frames: both are the same
 * whatever else is being served. */
typedef struct ca_server ca_server;

typedef struct {
    int32_t max_streams;     /* streams admitted at once, 1 .. 65536 */
    int32_t ring_slots;      /* frame slots per admitted stream, 1 .. 64 */
    int32_t max_batch;       /* frames per launched batch, 1 .. 4096 */
    int32_t max_inflight;    /* batches on the GPU at once, 1 .. 8 */
    uint64_t hbm_budget;     /* bytes for all admitted streams' frame rings */
    float smooth;            /* temporal filter decay lambda, [0, 1) */
    int32_t reserved;
    ca_params params;        /* per-frame parameters (scorer, fallback, ...) */
} ca_server_config;

/* One served frame (96 bytes). */
typedef struct {
    int32_t stream_id;
    int32_t filtered_valid;  /* the stream's filtered circle exists (w > 0) */
    uint64_t seq;
    ca_result result;        /* this frame's own estimate */
    float fcx, fcy, fr;      /* the stream's filtered circle after this frame */
    float fweight;           /* its accumulated confidence w */
    int64_t t_submit_ns;     /* steady-clock times: submission, */
    int64_t t_launch_ns;     /*   launch of the frame's batch, */
    int64_t t_done_ns;       /*   and when ca_server_step saw the batch finished */
    int32_t batch_size;      /* frames in the frame's batch */
    int32_t pad;
} ca_served;

/* Create a server on a context with a learned model if params.scorer asks
 * for it (ca_set_model first).  Allocates (blocking) everything the server
 * will use: the budget, per in-flight batch one device block sized for
 * max_batch frames (descriptors, one strip table per frame, score tables,
 * candidates, attempt records) with its pinned staging, and one HIP stream
 * (default priority) on which all of its work runs in order.
 * CA_E_INVAL for a bad config, CA_E_NOMEM. */
int ca_server_create(ca_ctx *ctx, const ca_server_config *cfg, ca_server **server);

/* Finish all work (blocking) and release everything.  Null is ignored. */
void ca_server_destroy(ca_server *server);

/* Open stream `stream_id` (>= 0, not open) with frames of width x height
 * (16 .. CA_MAX_EXTENT each).  *admitted = 1 if its ring was reserved now,
 * 0 if it waits for memory.  The stream's strip positions (Eq. 1) are
 * computed here; each batch then carries the tables of its own shapes, so
 * any number of distinct shapes may be open.  CA_E_INVAL for a bad shape, a
 * negative or duplicate id, or a ring larger than the whole budget. */
int ca_server_open(ca_server *server, int32_t stream_id, int32_t width, int32_t height,
                   int32_t *admitted);

/* Close a stream: its queued and in-flight frames are still served; its
 * ring is released after the last one. */
int ca_server_close(ca_server *server, int32_t stream_id);

/* Submit the next frame of an open stream: `src` holds height rows of
 * 3 width bytes, `row_stride` bytes apart, in device memory
 * (src_is_device = 1) or pinned host memory (0), copied into a slot of the
 * stream's ring when one is free; or in device memory lent to the server
 * (2): the frame's batch reads it in place, with no ring slot and no copy
 * (row_stride at most INT32_MAX), and it must stay allocated until the
 * frame is served.  In every mode `src` must stay unchanged until the frame
 * is served.  `seq` must increase per stream; a stream's frames are served
 * in submission order whatever their modes.  CA_E_INVAL for another
 * src_is_device, a short stride, a closed or unknown stream. */
int ca_server_submit(ca_server *server, int32_t stream_id, uint64_t seq, const uint8_t *src,
                     int64_t row_stride, int32_t src_is_device);

/* Make progress; write up to max_out served frames to `out` (host) in
 * completion order, their count to *n_out.  Served frames beyond max_out are
 * kept for the next call.  Never blocks on the GPU: the call only polls
 * events and enqueues asynchronous copies (into ring slots, and from and to
 * pinned staging) and kernels on the server's stream; it allocates,
 * frees and synchronises nothing. */
int ca_server_step(ca_server *server, ca_served *out, int32_t max_out, int32_t *n_out);

/* Counts: [0] frames submitted, [1] served, [2] queued on the host,
 * [3] in flight, [4] streams admitted, [5] streams waiting, [6] batches
 * launched, [7] budget bytes in use. */
int ca_server_stats(ca_server *server, int64_t out[8]);

/* Static description of a return code. */
const char *ca_error_string(int code);

/* Library version string. */
const char *ca_version(void);

#ifdef __cplusplus
}
#endif
#endif
