/* Test driver: runs the C oracle on raw RGB frames read from files, so that a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer (host code only)
 * checks the oracle's memory accesses and arithmetic.  Usage:
 *   driver W H ATTEMPTS NH NV frame.rgb [frame.rgb ...]
 * Prints one line per frame: valid inliers n_points. */
#include <stdio.h>
#include <stdlib.h>

#include "ca_oracle.h"

int main(int argc, char **argv)
{
    if (argc < 7)
        return 2;
    const int w = atoi(argv[1]), h = atoi(argv[2]);
    or_params p;
    or_default_params(&p);
    p.attempts = atoi(argv[3]);
    p.n_hstrips = atoi(argv[4]);
    p.n_vstrips = atoi(argv[5]);
    const size_t bytes = (size_t)w * (size_t)h * 3;
    uint8_t *frame = (uint8_t *)malloc(bytes);
    or_point *pts = (or_point *)malloc(sizeof(or_point) * 2 * (size_t)(p.n_hstrips + p.n_vstrips));
    or_attempt *att = (or_attempt *)malloc(sizeof(or_attempt) * (size_t)p.attempts);
    if (!frame || !pts || !att)
        return 3;
    for (int i = 6; i < argc; ++i) {
        FILE *f = fopen(argv[i], "rb");
        if (!f || fread(frame, 1, bytes, f) != bytes)
            return 4;
        fclose(f);
        or_result r;
        if (or_estimate(frame, w, h, 3 * w, (uint64_t)i, &p, pts, att, &r) != 0)
            return 5;
        printf("%d %d %d\n", r.valid, r.inliers, r.n_points);
    }
    free(att);
    free(pts);
    free(frame);
    return 0;
}
