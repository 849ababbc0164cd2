/*
 * ca_oracle.c -- TEST INFRASTRUCTURE ONLY (see ca_oracle.h).
 *
 * A plain, sequential CPU statement of the content-area estimator of
 * arXiv 2210.14771, Section 2.2, used to check the HIP library.  It is
 * deliberately slow and obvious: one frame at a time, one pixel at a time,
 * one attempt at a time, no blocking, fusion or reordering.
 *
 * Pipeline (Section 2.2.1): choose strips (Eq. 1), score every pixel of each
 * half strip (Section 2.2.3, Eqs. 2-3), take the best pixel of each half
 * strip, filter, then RANSAC with least-squares refits (Section 2.2.5).
 *
 * Readings where the paper leaves a choice open (all listed in the design
 * notes of the repository):
 *   - strip rows/columns: floor of Eq. 1, clamped to [1, extent-2];
 *     a strip is the scored line plus its two neighbours (the Sobel support);
 *     vertical strips repeat Eq. 1 along the width.
 *   - intensity: integer BT.601 luma Y = (77R + 150G + 29B + 128) >> 8.
 *   - Sobel with replicated borders; +x right, +y down.
 *   - the centre vector points from the pixel to the image centre
 *     ((W-1)/2, (H-1)/2); it is doubled to stay integral.
 *   - gradient magnitude quantised to 1/8 (qg = floor(8 |g|)); the angle
 *     between g and c quantised to a monotone pseudo-angle in [0, 2048];
 *     tanh of each quantised value is tabulated in float32 and the score is
 *     the float32 product (SG * ST) * SI.
 *   - iota: maximum luma of the pixels of the scored line strictly between
 *     the outer image edge and the pixel, 0 for the outermost pixel.
 *   - argmax ties go to the outermost pixel; filtering happens after the
 *     argmax; a kept point has edge distance >= t_px and score >= t_ps.
 *   - RANSAC triples from Philox4x64-10 keyed by the seed, counter
 *     (attempt, frame uid); coordinates are shifted by (W/2, H/2) (integer
 *     division) before fitting; K least-squares refits; the circle is scored
 *     by the inliers of its final circle; scores are summed as integers
 *     floor(s * 2^24); the circle score threshold applies to that sum / P.
 */
#include "ca_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846
#define OR_QT_MAX 2048
#define OR_SG_SIZE 11541 /* floor(8 * sqrt(2 * 1020^2)) + 1 */
#define OR_Q24 16777216.0f

void or_default_params(or_params *p)
{
    /* Appendix A, Table A1, and Section 2.2.5. */
    p->n_hstrips = 16;
    p->n_vstrips = 16;
    p->alpha = 8.0;
    p->t_g = 20.0;
    p->t_theta_deg = 30.0;
    p->t_iota = 25.0;
    p->t_ps = 0.03;
    p->t_cs = 0.06;
    p->t_px = 3;
    p->refine_iters = 3;
    p->t_ri = 3.0;
    p->r_min = 0.1;
    p->r_max = 0.8;
    p->d_max = 0.2;
    p->attempts = 256;
    p->sampler = 0;
    p->seed = 0;
}

/* ---------------------------------------------------------------- Eq. 1 -- */

int or_strip_positions(int32_t extent, int32_t n, double alpha, int32_t *pos)
{
    if (extent < 3 || n < 0)
        return -1;
    for (int32_t i = 0; i < n; ++i) {
        double t = (alpha / (double)n) * ((double)i - (double)(n - 1) / 2.0);
        double hpos = (double)extent / (1.0 + exp(-t));
        int32_t row = (int32_t)floor(hpos);
        if (row < 1)
            row = 1;
        if (row > extent - 2)
            row = extent - 2;
        pos[i] = row;
    }
    return 0;
}

/* --------------------------------------------------------- Eq. 2 tables -- */

int32_t or_sg_size(void) { return OR_SG_SIZE; }

/* Angle in degrees at the lower edge of pseudo-angle bin q (u = q / 1024):
 * the pseudo-angle is |c x g| / (|c x g| + c.g) for c.g >= 0, which equals
 * tan(t) / (1 + tan(t)), hence t = atan2(u, 1 - u); mirrored past 90 deg. */
static double or_bin_angle_deg(int32_t q)
{
    double u = (double)q / 1024.0;
    double t;
    if (u <= 1.0)
        t = atan2(u, 1.0 - u);
    else
        t = OR_PI - atan2(2.0 - u, u - 1.0);
    return t * (180.0 / OR_PI);
}

void or_build_tables(const or_params *p, float *sg, float *st, float *si)
{
    /* s_g = tanh(|g| / t_g) at |g| = q / 8 */
    for (int32_t q = 0; q < OR_SG_SIZE; ++q)
        sg[q] = (float)tanh((double)q / (8.0 * p->t_g));
    /* s_theta = 1 - tanh(theta / t_theta) */
    for (int32_t q = 0; q <= OR_QT_MAX; ++q)
        st[q] = (float)(1.0 - tanh(or_bin_angle_deg(q) / p->t_theta_deg));
    /* s_iota = 1 - tanh(iota / t_iota) */
    for (int32_t i = 0; i < 256; ++i)
        si[i] = (float)(1.0 - tanh((double)i / p->t_iota));
}

/* ------------------------------------------------ per-pixel features ----- */

int32_t or_luma(int32_t r, int32_t g, int32_t b)
{
    return (77 * r + 150 * g + 29 * b + 128) >> 8;
}

static int32_t or_Y(const uint8_t *f, int32_t w, int32_t h, int32_t rs, int32_t x, int32_t y)
{
    if (x < 0)
        x = 0;
    if (x > w - 1)
        x = w - 1;
    if (y < 0)
        y = 0;
    if (y > h - 1)
        y = h - 1;
    const uint8_t *px = f + (int64_t)y * rs + (int64_t)x * 3;
    return or_luma(px[0], px[1], px[2]);
}

static int64_t or_isqrt(int64_t v)
{
    int64_t r = (int64_t)sqrt((double)v);
    while (r * r > v)
        --r;
    while ((r + 1) * (r + 1) <= v)
        ++r;
    return r;
}

int32_t or_qgrad(int64_t m2)
{
    return (int32_t)or_isqrt(64 * m2); /* floor(8 * sqrt(m2)) */
}

int32_t or_qtheta(int64_t dt, int64_t cr)
{
    int64_t acr = cr < 0 ? -cr : cr;
    int64_t adt = dt < 0 ? -dt : dt;
    int64_t den = acr + adt;
    if (den == 0)
        return 0;
    if (dt >= 0)
        return (int32_t)((1024 * acr) / den);
    return (int32_t)(OR_QT_MAX - (1024 * acr + den - 1) / den);
}

int or_pixel_features(const uint8_t *f, int32_t w, int32_t h, int32_t rs, int32_t x, int32_t y,
                      or_pixel *o)
{
    if (!f || !o || x < 0 || y < 0 || x >= w || y >= h)
        return -1;
    /* 3x3 Sobel (Section 2.2.3) */
    int32_t gx = (or_Y(f, w, h, rs, x + 1, y - 1) + 2 * or_Y(f, w, h, rs, x + 1, y)
                  + or_Y(f, w, h, rs, x + 1, y + 1))
                 - (or_Y(f, w, h, rs, x - 1, y - 1) + 2 * or_Y(f, w, h, rs, x - 1, y)
                    + or_Y(f, w, h, rs, x - 1, y + 1));
    int32_t gy = (or_Y(f, w, h, rs, x - 1, y + 1) + 2 * or_Y(f, w, h, rs, x, y + 1)
                  + or_Y(f, w, h, rs, x + 1, y + 1))
                 - (or_Y(f, w, h, rs, x - 1, y - 1) + 2 * or_Y(f, w, h, rs, x, y - 1)
                    + or_Y(f, w, h, rs, x + 1, y - 1));
    /* doubled vector from the pixel to the image centre */
    int64_t c2x = (int64_t)(w - 1) - 2 * (int64_t)x;
    int64_t c2y = (int64_t)(h - 1) - 2 * (int64_t)y;
    o->luma = or_Y(f, w, h, rs, x, y);
    o->gx = gx;
    o->gy = gy;
    o->dt = (int64_t)gx * c2x + (int64_t)gy * c2y;
    o->cr = (int64_t)gx * c2y - (int64_t)gy * c2x;
    o->qg = or_qgrad((int64_t)gx * gx + (int64_t)gy * gy);
    o->qt = or_qtheta(o->dt, o->cr);
    o->iota_unused = 0;
    return 0;
}

/* ------------------------------------------------------ half strips ------ */

typedef struct {
    int32_t n_h, n_v;
    int32_t *rows, *cols;
    float *sg, *st, *si;
} or_plan;

static int or_plan_make(or_plan *pl, int32_t w, int32_t h, const or_params *p)
{
    memset(pl, 0, sizeof(*pl));
    pl->n_h = p->n_hstrips;
    pl->n_v = p->n_vstrips;
    pl->rows = (int32_t *)malloc(sizeof(int32_t) * (size_t)(pl->n_h + 1));
    pl->cols = (int32_t *)malloc(sizeof(int32_t) * (size_t)(pl->n_v + 1));
    pl->sg = (float *)malloc(sizeof(float) * OR_SG_SIZE);
    pl->st = (float *)malloc(sizeof(float) * (OR_QT_MAX + 1));
    pl->si = (float *)malloc(sizeof(float) * 256);
    if (!pl->rows || !pl->cols || !pl->sg || !pl->st || !pl->si)
        return -1;
    or_strip_positions(h, pl->n_h, p->alpha, pl->rows);
    or_strip_positions(w, pl->n_v, p->alpha, pl->cols);
    or_build_tables(p, pl->sg, pl->st, pl->si);
    return 0;
}

static void or_plan_free(or_plan *pl)
{
    free(pl->rows);
    free(pl->cols);
    free(pl->sg);
    free(pl->st);
    free(pl->si);
}

/* Coordinates of pixel k (k = 0 at the outer image edge) of a half strip. */
static void or_half_pixel(const or_plan *pl, int32_t w, int32_t h, int32_t strip, int32_t half,
                          int32_t k, int32_t *x, int32_t *y)
{
    if (strip < pl->n_h) {
        *y = pl->rows[strip];
        *x = half == 0 ? k : w - 1 - k;
    } else {
        *x = pl->cols[strip - pl->n_h];
        *y = half == 0 ? k : h - 1 - k;
    }
}

static int32_t or_half_len(const or_plan *pl, int32_t w, int32_t h, int32_t strip, int32_t half)
{
    int32_t extent = strip < pl->n_h ? w : h;
    return half == 0 ? extent / 2 : extent - extent / 2;
}

/* Score of one pixel given its features and the preceding maximum (Eq. 2-3). */
static float or_score_q(const or_plan *pl, const or_pixel *px, int32_t iota)
{
    return (pl->sg[px->qg] * pl->st[px->qt]) * pl->si[iota];
}

static double or_score_ideal(const or_params *p, const or_pixel *px, int32_t iota)
{
    double gnorm = sqrt((double)px->gx * px->gx + (double)px->gy * px->gy);
    if (gnorm == 0.0)
        return 0.0;
    double theta = atan2(fabs((double)px->cr), (double)px->dt) * (180.0 / OR_PI);
    return tanh(gnorm / p->t_g) * (1.0 - tanh(theta / p->t_theta_deg))
           * (1.0 - tanh((double)iota / p->t_iota));
}

static int or_scan_half(const uint8_t *f, int32_t w, int32_t h, int32_t rs, const or_params *p,
                        const or_plan *pl, int32_t strip, int32_t half, int ideal, float *scores,
                        int32_t *xs, int32_t *ys, or_point *best)
{
    int32_t len = or_half_len(pl, w, h, strip, half);
    int32_t iota = 0;          /* max luma strictly before pixel k */
    double best_s = -1.0;
    int32_t best_k = -1;
    float best_f = 0.0f;
    for (int32_t k = 0; k < len; ++k) {
        int32_t x, y;
        or_half_pixel(pl, w, h, strip, half, k, &x, &y);
        or_pixel px;
        or_pixel_features(f, w, h, rs, x, y, &px);
        double s;
        float sf;
        if (ideal) {
            s = or_score_ideal(p, &px, iota);
            sf = (float)s;
        } else {
            sf = or_score_q(pl, &px, iota);
            s = (double)sf;
        }
        if (scores)
            scores[k] = sf;
        if (xs)
            xs[k] = x;
        if (ys)
            ys[k] = y;
        if (s > best_s) { /* strict: ties keep the outermost pixel */
            best_s = s;
            best_k = k;
            best_f = sf;
        }
        if (px.luma > iota)
            iota = px.luma;
    }
    if (best) {
        int32_t x, y;
        or_half_pixel(pl, w, h, strip, half, best_k, &x, &y);
        best->x = x;
        best->y = y;
        best->score = best_f;
        int32_t ed = x;
        if (y < ed)
            ed = y;
        if (w - 1 - x < ed)
            ed = w - 1 - x;
        if (h - 1 - y < ed)
            ed = h - 1 - y;
        best->keep = (ed >= p->t_px && best_f >= (float)p->t_ps) ? 1 : 0;
    }
    return len;
}

static int or_check(int32_t w, int32_t h, int32_t rs, const or_params *p)
{
    if (w < 16 || h < 16 || rs < 3 * w)
        return -1;
    if (p->n_hstrips < 0 || p->n_vstrips < 0 || p->n_hstrips > 64 || p->n_vstrips > 64
        || p->n_hstrips + p->n_vstrips < 1)
        return -1;
    if (p->attempts < 1 || p->refine_iters < 0)
        return -1;
    return 0;
}

int or_half_strip_scores(const uint8_t *f, int32_t w, int32_t h, int32_t rs, const or_params *p,
                         int32_t strip, int32_t half, int ideal, float *scores, int32_t *xs,
                         int32_t *ys)
{
    if (!f || or_check(w, h, rs, p) < 0)
        return -1;
    if (strip < 0 || strip >= p->n_hstrips + p->n_vstrips || half < 0 || half > 1)
        return -1;
    or_plan pl;
    if (or_plan_make(&pl, w, h, p) < 0) {
        or_plan_free(&pl);
        return -2;
    }
    int len = or_scan_half(f, w, h, rs, p, &pl, strip, half, ideal, scores, xs, ys, NULL);
    or_plan_free(&pl);
    return len;
}

int or_candidates(const uint8_t *f, int32_t w, int32_t h, int32_t rs, const or_params *p,
                  int ideal, or_point *out)
{
    if (!f || !out || or_check(w, h, rs, p) < 0)
        return -1;
    or_plan pl;
    if (or_plan_make(&pl, w, h, p) < 0) {
        or_plan_free(&pl);
        return -2;
    }
    int32_t ns = pl.n_h + pl.n_v;
    for (int32_t s = 0; s < ns; ++s)
        for (int32_t half = 0; half < 2; ++half)
            or_scan_half(f, w, h, rs, p, &pl, s, half, ideal, NULL, NULL, NULL,
                         &out[2 * s + half]);
    or_plan_free(&pl);
    return 2 * ns;
}

/* ----------------------------------------------------------- Philox ------ */

static void or_mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 prod = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(prod >> 64);
    *lo = (uint64_t)prod;
}

void or_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    /* Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as easy as
     * 1, 2, 3", SC'11 -- Philox4x64 with 10 rounds. */
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        or_mulhilo64(M0, c0, &hi0, &lo0);
        or_mulhilo64(M1, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

static int32_t or_below(uint64_t u, int32_t k)
{
    /* map the top 32 random bits onto [0, k) */
    return (int32_t)(((u >> 32) * (uint64_t)k) >> 32);
}

void or_draw_triple(uint64_t seed, uint64_t uid, int32_t a, int32_t n, int32_t t[3])
{
    /* uniform sampling of three distinct points (Section 2.2.5) */
    uint64_t ctr[4] = {(uint64_t)(uint32_t)a, uid, 0, 0};
    uint64_t key[2] = {seed, 0};
    uint64_t u[4];
    or_philox4x64_10(ctr, key, u);
    int32_t i0 = or_below(u[0], n);
    int32_t i1 = or_below(u[1], n - 1);
    if (i1 >= i0)
        ++i1;
    int32_t lo = i0 < i1 ? i0 : i1;
    int32_t hi = i0 < i1 ? i1 : i0;
    int32_t i2 = or_below(u[2], n - 2);
    if (i2 >= lo)
        ++i2;
    if (i2 >= hi)
        ++i2;
    t[0] = i0;
    t[1] = i1;
    t[2] = i2;
}

/* a-th triple (i < j < k) of n items in lexicographic order; 0 if a >= C(n,3). */
static int or_unrank_triple(int64_t a, int32_t n, int32_t t[3])
{
    for (int32_t i = 0; i < n - 2; ++i) {
        int64_t rest = (int64_t)(n - 1 - i) * (n - 2 - i) / 2; /* C(n-1-i, 2) */
        if (a >= rest) {
            a -= rest;
            continue;
        }
        for (int32_t j = i + 1; j < n - 1; ++j) {
            int64_t cnt = n - 1 - j;
            if (a >= cnt) {
                a -= cnt;
                continue;
            }
            t[0] = i;
            t[1] = j;
            t[2] = j + 1 + (int32_t)a;
            return 1;
        }
    }
    return 0;
}

/* --------------------------------------------------------- circles ------- */

int or_circle3(const int64_t x[3], const int64_t y[3], double *cx, double *cy, double *r2)
{
    /* circumcentre of three points (closed form) */
    int64_t D = 2 * (x[0] * (y[1] - y[2]) + x[1] * (y[2] - y[0]) + x[2] * (y[0] - y[1]));
    if (D == 0)
        return 0;
    int64_t z0 = x[0] * x[0] + y[0] * y[0];
    int64_t z1 = x[1] * x[1] + y[1] * y[1];
    int64_t z2 = x[2] * x[2] + y[2] * y[2];
    int64_t Nx = z0 * (y[1] - y[2]) + z1 * (y[2] - y[0]) + z2 * (y[0] - y[1]);
    int64_t Ny = z0 * (x[2] - x[1]) + z1 * (x[0] - x[2]) + z2 * (x[1] - x[0]);
    *cx = (double)Nx / (double)D;
    *cy = (double)Ny / (double)D;
    double dx = (double)x[0] - *cx;
    double dy = (double)y[0] - *cy;
    *r2 = dx * dx + dy * dy;
    return 1;
}

int or_lsq_circle(const int64_t *x, const int64_t *y, int32_t m, double *cx, double *cy,
                  double *r2)
{
    /* Coope (1993): the circle x^2 + y^2 = 2a x + 2b y + c is linear in
     * (a, b, c); its least-squares solution in centred moments. */
    if (m < 3)
        return 0;
    int64_t Su = 0, Sv = 0, Suu = 0, Suv = 0, Svv = 0, Suz = 0, Svz = 0, Sz = 0;
    for (int32_t i = 0; i < m; ++i) {
        int64_t z = x[i] * x[i] + y[i] * y[i];
        Su += x[i];
        Sv += y[i];
        Suu += x[i] * x[i];
        Suv += x[i] * y[i];
        Svv += y[i] * y[i];
        Suz += x[i] * z;
        Svz += y[i] * z;
        Sz += z;
    }
    int64_t M = m;
    int64_t Cuu = M * Suu - Su * Su;
    int64_t Cuv = M * Suv - Su * Sv;
    int64_t Cvv = M * Svv - Sv * Sv;
    int64_t Cuz = M * Suz - Su * Sz;
    int64_t Cvz = M * Svz - Sv * Sz;
    double det = (double)Cuu * (double)Cvv - (double)Cuv * (double)Cuv;
    if (det == 0.0)
        return 0;
    double A = ((double)Cuz * (double)Cvv - (double)Cvz * (double)Cuv) / det;
    double B = ((double)Cvz * (double)Cuu - (double)Cuz * (double)Cuv) / det;
    *cx = A / 2.0;
    *cy = B / 2.0;
    double mu = (double)Su / (double)M;
    double mv = (double)Sv / (double)M;
    double var = (double)(Cuu + Cvv) / ((double)M * (double)M);
    *r2 = (var + (mu - *cx) * (mu - *cx)) + (mv - *cy) * (mv - *cy);
    return 1;
}

/* inlier band |d - r| <= t, tested on squared distances */
typedef struct {
    double cx, cy, lo2, hi2;
} or_band;

static or_band or_make_band(double cx, double cy, double r2, double t)
{
    or_band b;
    double r = sqrt(r2);
    double hi = r + t;
    b.cx = cx;
    b.cy = cy;
    b.hi2 = hi * hi;
    if (r > t) {
        double lo = r - t;
        b.lo2 = lo * lo;
    } else {
        b.lo2 = -1.0; /* no inner bound */
    }
    return b;
}

static int or_is_inlier(const or_band *b, int64_t u, int64_t v)
{
    double du = (double)u - b->cx;
    double dv = (double)v - b->cy;
    double d2 = du * du + dv * dv;
    return b->lo2 <= d2 && d2 <= b->hi2;
}

/* One RANSAC attempt from a given triple (Section 2.2.5). Coordinates u, v
 * are the shifted ones. */
static void or_attempt_from_triple(const int64_t *u, const int64_t *v, const uint32_t *sq,
                                   int32_t n, const int32_t t[3], int32_t w, int32_t h,
                                   const or_params *p, int64_t *scr_u, int64_t *scr_v,
                                   or_attempt *o)
{
    int64_t ox = w / 2, oy = h / 2;
    o->i0 = t[0];
    o->i1 = t[1];
    o->i2 = t[2];
    o->inliers = 0;
    o->qsum = 0;
    o->cx = o->cy = o->r2 = 0.0;
    o->status = 0;
    o->fail_stage = 0;
    int64_t tx[3] = {u[t[0]], u[t[1]], u[t[2]]};
    int64_t ty[3] = {v[t[0]], v[t[1]], v[t[2]]};
    double cx, cy, r2;
    if (!or_circle3(tx, ty, &cx, &cy, &r2))
        return; /* collinear triple */
    for (int32_t k = 1; k <= p->refine_iters; ++k) {
        or_band b = or_make_band(cx, cy, r2, p->t_ri);
        int32_t m = 0;
        for (int32_t i = 0; i < n; ++i)
            if (or_is_inlier(&b, u[i], v[i])) {
                scr_u[m] = u[i];
                scr_v[m] = v[i];
                ++m;
            }
        if (!or_lsq_circle(scr_u, scr_v, m, &cx, &cy, &r2)) {
            o->fail_stage = k;
            return;
        }
    }
    /* score the final circle by its own inliers */
    or_band b = or_make_band(cx, cy, r2, p->t_ri);
    int32_t m = 0;
    uint64_t q = 0;
    for (int32_t i = 0; i < n; ++i)
        if (or_is_inlier(&b, u[i], v[i])) {
            ++m;
            q += sq[i];
        }
    double acx = (double)ox + cx;
    double acy = (double)oy + cy;
    o->inliers = m;
    o->qsum = q;
    o->cx = acx;
    o->cy = acy;
    o->r2 = r2;
    /* limits on the circle, as multiples of the width */
    double r = sqrt(r2);
    double dx = acx - (double)(w - 1) / 2.0;
    double dy = acy - (double)(h - 1) / 2.0;
    double dlim = p->d_max * (double)w;
    int ok = r >= p->r_min * (double)w && r <= p->r_max * (double)w
             && dx * dx + dy * dy <= dlim * dlim;
    o->status = ok ? 2 : 1;
}

static int or_ransac_impl(const int32_t *xs, const int32_t *ys, const uint32_t *sq, int32_t n,
                          int32_t w, int32_t h, uint64_t uid, const or_params *p,
                          int64_t n_attempts, int sampler, or_attempt *out, int64_t *best_a,
                          or_attempt *best)
{
    int64_t *u = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1) * 4);
    if (!u)
        return -2;
    int64_t *v = u + (n > 0 ? n : 1);
    int64_t *su = v + (n > 0 ? n : 1);
    int64_t *sv = su + (n > 0 ? n : 1);
    for (int32_t i = 0; i < n; ++i) {
        u[i] = (int64_t)xs[i] - w / 2;
        v[i] = (int64_t)ys[i] - h / 2;
    }
    *best_a = -1;
    for (int64_t a = 0; a < n_attempts; ++a) {
        or_attempt o;
        int32_t t[3];
        int have;
        if (sampler == 0) {
            or_draw_triple(p->seed, uid, (int32_t)a, n, t);
            have = 1;
        } else {
            have = or_unrank_triple(a, n, t);
        }
        if (have) {
            or_attempt_from_triple(u, v, sq, n, t, w, h, p, su, sv, &o);
        } else {
            memset(&o, 0, sizeof(o));
            o.i0 = o.i1 = o.i2 = -1;
            o.fail_stage = -1; /* enumeration exhausted */
        }
        if (out)
            out[a] = o;
        if (o.status == 2 && (*best_a < 0 || o.qsum > best->qsum)) {
            *best_a = a;
            *best = o;
        }
    }
    free(u);
    return 0;
}

int or_ransac_attempts(const int32_t *xs, const int32_t *ys, const uint32_t *sq, int32_t n,
                       int32_t w, int32_t h, uint64_t uid, const or_params *p, or_attempt *out)
{
    if (!xs || !ys || !sq || !out || n < 3 || p->attempts < 1)
        return -1;
    int64_t best_a;
    or_attempt best;
    return or_ransac_impl(xs, ys, sq, n, w, h, uid, p, p->attempts, p->sampler, out, &best_a,
                          &best);
}

static int or_estimate_impl(const uint8_t *f, int32_t w, int32_t h, int32_t rs, uint64_t uid,
                            const or_params *p, int brute, or_point *pts_out,
                            or_attempt *att_out, or_result *res)
{
    if (!f || !res || or_check(w, h, rs, p) < 0)
        return -1;
    int32_t P = 2 * (p->n_hstrips + p->n_vstrips);
    or_point *pts = (or_point *)malloc(sizeof(or_point) * (size_t)P);
    int32_t *xs = (int32_t *)malloc(sizeof(int32_t) * (size_t)P);
    int32_t *ys = (int32_t *)malloc(sizeof(int32_t) * (size_t)P);
    uint32_t *sq = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)P);
    if (!pts || !xs || !ys || !sq) {
        free(pts);
        free(xs);
        free(ys);
        free(sq);
        return -2;
    }
    or_candidates(f, w, h, rs, p, 0, pts);
    if (pts_out)
        memcpy(pts_out, pts, sizeof(or_point) * (size_t)P);
    /* kept points in canonical order */
    int32_t n = 0;
    for (int32_t i = 0; i < P; ++i)
        if (pts[i].keep) {
            xs[n] = pts[i].x;
            ys[n] = pts[i].y;
            sq[n] = (uint32_t)(pts[i].score * OR_Q24);
            ++n;
        }
    memset(res, 0, sizeof(*res));
    res->n_points = n;
    res->best_attempt = -1;
    if (n < 3) {
        res->reason = 1;
        if (att_out)
            memset(att_out, 0, sizeof(or_attempt) * (size_t)p->attempts);
        goto done;
    }
    {
        int64_t best_a;
        or_attempt best;
        int64_t na = p->attempts;
        int sampler = p->sampler;
        if (brute) {
            na = (int64_t)n * (n - 1) * (n - 2) / 6;
            sampler = 1;
        }
        if (or_ransac_impl(xs, ys, sq, n, w, h, uid, p, na, sampler, brute ? NULL : att_out,
                           &best_a, &best) < 0) {
            free(pts);
            free(xs);
            free(ys);
            free(sq);
            return -2;
        }
        if (best_a < 0) {
            res->reason = 2;
            goto done;
        }
        res->best_attempt = (int32_t)best_a;
        res->qsum = best.qsum;
        res->inliers = best.inliers;
        res->cxd = best.cx;
        res->cyd = best.cy;
        res->r2d = best.r2;
        res->cx = (float)best.cx;
        res->cy = (float)best.cy;
        res->r = (float)sqrt(best.r2);
        res->score = (float)((double)best.qsum / (16777216.0 * (double)P));
        double thr = p->t_cs * 16777216.0 * (double)P;
        if ((double)best.qsum >= thr) {
            res->valid = 1;
            res->reason = 0;
        } else {
            res->reason = 3;
        }
    }
done:
    free(pts);
    free(xs);
    free(ys);
    free(sq);
    return 0;
}

int or_estimate(const uint8_t *f, int32_t w, int32_t h, int32_t rs, uint64_t uid,
                const or_params *p, or_point *pts_out, or_attempt *att_out, or_result *res)
{
    return or_estimate_impl(f, w, h, rs, uid, p, 0, pts_out, att_out, res);
}

int or_estimate_bruteforce(const uint8_t *f, int32_t w, int32_t h, int32_t rs, uint64_t uid,
                           const or_params *p, or_result *res)
{
    return or_estimate_impl(f, w, h, rs, uid, p, 1, NULL, NULL, res);
}
