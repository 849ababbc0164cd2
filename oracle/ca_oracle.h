/*
 * ca_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, sequential CPU reference ("oracle") for the endoscopic content
 * area estimator of Budd et al., "Rapid and robust endoscopic content area
 * estimation" (arXiv 2210.14771), Section 2.2.  It exists to check the HIP
 * library against; it is not part of the product path.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no source, header, table or constant generator with the library.
 *
 * Every function works on one frame (or one small table) at a time with
 * plain loops, in the order the paper gives the steps.  Floating point is
 * IEEE double except where the numeric contract fixes float32 (the score
 * tables and the score product).  Build with -O2 -ffp-contract=off.
 */
#ifndef CA_ORACLE_H
#define CA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Parameters, Appendix A (Table A1) plus the readings listed in the source. */
typedef struct {
    int32_t n_hstrips;      /* N for horizontal strips (paper: 16) */
    int32_t n_vstrips;      /* N for vertical strips (0 = horizontal only, as in the paper) */
    double alpha;           /* strip weighting, Eq. 1 (8) */
    double t_g;             /* gradient-magnitude soft threshold, Eq. 2 (20) */
    double t_theta_deg;     /* gradient-direction soft threshold in degrees, Eq. 2 (30) */
    double t_iota;          /* preceding-maximum soft threshold, Eq. 2 (25) */
    double t_ps;            /* point score threshold (0.03), compared in float32 */
    double t_cs;            /* circle score threshold (0.06), applied to sum / P */
    int32_t t_px;           /* edge margin in pixels (3) */
    int32_t refine_iters;   /* least-squares refinements per attempt (3) */
    double t_ri;            /* RANSAC inlier distance in pixels (3) */
    double r_min, r_max;    /* radius bounds as multiples of the width (0.1, 0.8) */
    double d_max;           /* centre offset bound as a multiple of the width (0.2) */
    int32_t attempts;       /* RANSAC attempts */
    int32_t sampler;        /* 0 = random triples, 1 = lexicographic enumeration */
    uint64_t seed;          /* RNG key */
} or_params;

typedef struct {
    int32_t x, y;           /* pixel index of the best pixel of the half strip */
    float score;            /* its score s, Eq. 3 */
    int32_t keep;           /* 1 if it survives the edge-margin and score filters */
} or_point;

typedef struct {
    int32_t status;         /* 0 degenerate, 1 rejected by radius/centre limits, 2 kept */
    int32_t fail_stage;     /* for status 0: 0 = collinear triple, k = refinement k failed */
    int32_t i0, i1, i2;     /* triple (indices into the kept points) */
    int32_t inliers;        /* inlier count of the final circle */
    uint64_t qsum;          /* sum of 2^24-scaled inlier scores of the final circle */
    double cx, cy, r2;      /* final circle, pixel-index coordinates, squared radius */
} or_attempt;

typedef struct {
    float cx, cy, r;        /* circle (pixel-index coordinates) */
    float score;            /* best circle score / P */
    int32_t inliers;        /* inlier count of the best circle */
    int32_t n_points;       /* kept candidate points */
    int32_t valid;          /* 1 = circle; 0 = content fills the rectangle */
    int32_t reason;         /* 0 ok, 1 fewer than 3 points, 2 no kept attempt, 3 below t_cs */
    int32_t best_attempt;   /* index of the winning attempt or -1 */
    int32_t pad;
    uint64_t qsum;          /* winning circle's integer score sum */
    double cxd, cyd, r2d;   /* winning circle before rounding to float */
} or_result;

void or_default_params(or_params *p);

/* Eq. 1: strip positions along an axis of `extent` pixels. Writes n ints. */
int or_strip_positions(int32_t extent, int32_t n, double alpha, int32_t *pos);

/* Score tables (Eq. 2 with quantised arguments). Sizes: sg[or_sg_size()],
 * st[2049], si[256]. */
int32_t or_sg_size(void);
void or_build_tables(const or_params *p, float *sg, float *st, float *si);

/* Integer BT.601 luma of one RGB pixel. */
int32_t or_luma(int32_t r, int32_t g, int32_t b);

/* Per-pixel quantities of one scored pixel (x, y) of a frame, for tests. */
typedef struct {
    int32_t luma, gx, gy, qg, qt, iota_unused;
    int64_t dt, cr;
} or_pixel;
int or_pixel_features(const uint8_t *frame, int32_t w, int32_t h, int32_t row_stride,
                      int32_t x, int32_t y, or_pixel *out);

/* Quantisers on their own. */
int32_t or_qgrad(int64_t m2);
int32_t or_qtheta(int64_t dt, int64_t cr);

/* Candidates of one frame: P = 2 (n_hstrips + n_vstrips) points, canonical order.
 * `ideal` = 0 uses the quantised, tabulated score of the numeric contract;
 * `ideal` = 1 scores with unquantised double tanh/atan2 (a measuring aid,
 * never a parity target). Returns P or a negative error. */
int or_candidates(const uint8_t *frame, int32_t w, int32_t h, int32_t row_stride,
                  const or_params *p, int ideal, or_point *out);

/* Score of every pixel of one half strip, in scan order (k = 0 is the outer
 * edge). Writes the half-strip length of floats into `scores` and the pixel
 * coordinates into xs/ys. `strip` indexes H strips then V strips; `half` 0/1. */
int or_half_strip_scores(const uint8_t *frame, int32_t w, int32_t h, int32_t row_stride,
                         const or_params *p, int32_t strip, int32_t half, int ideal,
                         float *scores, int32_t *xs, int32_t *ys);

/* Philox4x64-10 block function (Salmon et al., SC'11). */
void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Triple of attempt `a` among n points (n >= 3) for the random sampler. */
void or_draw_triple(uint64_t seed, uint64_t frame_uid, int32_t a, int32_t n, int32_t t[3]);

/* Closed-form circle through three integer points; 0 if collinear. */
int or_circle3(const int64_t xs[3], const int64_t ys[3], double *cx, double *cy, double *r2);

/* Least-squares (Coope) circle through integer points; 0 if degenerate. */
int or_lsq_circle(const int64_t *xs, const int64_t *ys, int32_t m, double *cx, double *cy,
                  double *r2);

/* Run every RANSAC attempt on a kept point list (coordinates relative to the
 * frame, canonical order). Writes `attempts` records. */
int or_ransac_attempts(const int32_t *xs, const int32_t *ys, const uint32_t *sq, int32_t n,
                       int32_t w, int32_t h, uint64_t frame_uid, const or_params *p,
                       or_attempt *out);

/* Whole pipeline on one frame. `attempts_out` may be NULL. */
int or_estimate(const uint8_t *frame, int32_t w, int32_t h, int32_t row_stride,
                uint64_t frame_uid, const or_params *p, or_point *points_out,
                or_attempt *attempts_out, or_result *res);

/* The same estimate with every triple of the kept points tried once (all
 * C(n,3) attempts, lexicographic); used to check the samplers. */
int or_estimate_bruteforce(const uint8_t *frame, int32_t w, int32_t h, int32_t row_stride,
                           uint64_t frame_uid, const or_params *p, or_result *res);

#ifdef __cplusplus
}
#endif
#endif
