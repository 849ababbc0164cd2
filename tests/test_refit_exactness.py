"""The refit's centred sums C = m S_ab - S_a S_b are integers.  The GPU forms
them in float64 when n^2 max(U, V) Z < 2^52 for the frame (U, V the largest
|u|, |v|; Z = U^2 + V^2; n kept points), and in int64 otherwise.  This checks
on the CPU, with exact Python integers as the reference, that under that
bound every float64 product and difference in the formulas is exact, at the
extremes the API allows (frames up to 16384 pixels a side, 256 points),
including points placed at the corners where the sums are largest."""
import numpy as np
import pytest

BOUND = 2.0 ** 52


def exact_path_applies(n, W, H):
    ox, oy = W // 2, H // 2
    U = max(ox, W - 1 - ox)
    V = max(oy, H - 1 - oy)
    return float(n) * float(n) * float(max(U, V)) * float(U * U + V * V) < BOUND


def centred_sums_float64(m, su, sv, suu, suv, svv, suz, svz):
    f = np.float64
    m, su, sv, suu, suv, svv, suz, svz = map(f, (m, su, sv, suu, suv, svv, suz, svz))
    sz = suu + svv
    return (m * suu - su * su, m * suv - su * sv, m * svv - sv * sv,
            m * suz - su * sz, m * svz - sv * sz)


def centred_sums_exact(m, su, sv, suu, suv, svv, suz, svz):
    sz = suu + svv
    return (m * suu - su * su, m * suv - su * sv, m * svv - sv * sv,
            m * suz - su * sz, m * svz - sv * sz)


def moments(us, vs):
    us = [int(u) for u in us]
    vs = [int(v) for v in vs]
    z = [u * u + v * v for u, v in zip(us, vs)]
    return (len(us), sum(us), sum(vs), sum(u * u for u in us), sum(u * v for u, v in zip(us, vs)),
            sum(v * v for v in vs), sum(u * zz for u, zz in zip(us, z)),
            sum(v * zz for v, zz in zip(vs, z)))


def check(us, vs):
    S = moments(us, vs)
    got = centred_sums_float64(*S)
    want = centred_sums_exact(*S)
    for g, w in zip(got, want):
        assert float(g) == float(w) and int(g) == w


@pytest.mark.parametrize("W,H", [(640, 480), (1920, 1080), (3840, 2160), (7680, 4320),
                                 (16384, 64), (64, 16384), (4096, 4096)])
def test_float64_centred_sums_are_exact_under_the_bound(W, H):
    rng = np.random.default_rng(W * 7 + H)
    ox, oy = W // 2, H // 2
    for n in (3, 8, 64, 128, 256):
        if not exact_path_applies(n, W, H):
            continue
        for _ in range(20):
            x = rng.integers(0, W, n)
            y = rng.integers(0, H, n)
            check(x - ox, y - oy)
        # the largest sums: every point at the same far corner, and split
        # between opposite corners
        check(np.full(n, -ox), np.full(n, -oy))
        check(np.full(n, W - 1 - ox), np.full(n, H - 1 - oy))
        half = n // 2
        check(np.r_[np.full(half, -ox), np.full(n - half, W - 1 - ox)],
              np.r_[np.full(half, H - 1 - oy), np.full(n - half, -oy)])


def test_bound_values():
    # the bound sends the largest extents with many points to the int64 form
    assert not exact_path_applies(256, 16384, 16384)
    assert not exact_path_applies(256, 16384, 512)
    assert exact_path_applies(8, 8192, 2048)
    assert exact_path_applies(128, 1920, 1080)
    assert exact_path_applies(256, 3840, 2160)


def test_float64_can_fail_beyond_the_bound():
    # clusters at two opposite corners of a 16384 x 16384 frame: some point
    # sets lose bits in float64, so the bound is not vacuous (all of them lie
    # outside it)
    W = H = 16384
    ox, oy = W // 2, H // 2
    rng = np.random.default_rng(0)
    failed = 0
    for _ in range(200):
        n = int(rng.integers(150, 257))
        a, b = rng.integers(0, 40, n), rng.integers(0, 40, n)
        side = rng.integers(0, 2, n)
        us = np.where(side == 0, a, W - 1 - a) - ox
        vs = np.where(side == 0, b, H - 1 - b) - oy
        S = moments(us, vs)
        got = centred_sums_float64(*S)
        want = centred_sums_exact(*S)
        if any(int(g) != w for g, w in zip(got, want)):
            assert not exact_path_applies(n, W, H)
            failed += 1
    assert failed > 0
