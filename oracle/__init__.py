"""TEST INFRASTRUCTURE ONLY: ctypes wrapper of the plain C oracle.

The oracle (``ca_oracle.c``) is a slow, sequential CPU statement of the
content-area estimator of arXiv 2210.14771, Section 2.2, used to check the
HIP library.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import this package; the library never does, and this package
imports nothing from the library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ca_oracle.c")
LIB_PATH = os.path.join(HERE, "_build", "libcaoracle.so")
CFLAGS = ["-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no contraction, no fast math)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    os.makedirs(os.path.dirname(LIB_PATH), exist_ok=True)
    tmp = LIB_PATH + ".tmp"
    subprocess.run(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Params(C.Structure):
    _fields_ = [("n_hstrips", C.c_int32), ("n_vstrips", C.c_int32), ("alpha", C.c_double),
                ("t_g", C.c_double), ("t_theta_deg", C.c_double), ("t_iota", C.c_double),
                ("t_ps", C.c_double), ("t_cs", C.c_double), ("t_px", C.c_int32),
                ("refine_iters", C.c_int32), ("t_ri", C.c_double), ("r_min", C.c_double),
                ("r_max", C.c_double), ("d_max", C.c_double), ("attempts", C.c_int32),
                ("sampler", C.c_int32), ("seed", C.c_uint64)]


class Point(C.Structure):
    _fields_ = [("x", C.c_int32), ("y", C.c_int32), ("score", C.c_float), ("keep", C.c_int32)]


class Attempt(C.Structure):
    _fields_ = [("status", C.c_int32), ("fail_stage", C.c_int32), ("i0", C.c_int32),
                ("i1", C.c_int32), ("i2", C.c_int32), ("inliers", C.c_int32),
                ("qsum", C.c_uint64), ("cx", C.c_double), ("cy", C.c_double), ("r2", C.c_double)]


class Result(C.Structure):
    _fields_ = [("cx", C.c_float), ("cy", C.c_float), ("r", C.c_float), ("score", C.c_float),
                ("inliers", C.c_int32), ("n_points", C.c_int32), ("valid", C.c_int32),
                ("reason", C.c_int32), ("best_attempt", C.c_int32), ("pad", C.c_int32),
                ("qsum", C.c_uint64), ("cxd", C.c_double), ("cyd", C.c_double),
                ("r2d", C.c_double)]


class Pixel(C.Structure):
    _fields_ = [("luma", C.c_int32), ("gx", C.c_int32), ("gy", C.c_int32), ("qg", C.c_int32),
                ("qt", C.c_int32), ("iota_unused", C.c_int32), ("dt", C.c_int64),
                ("cr", C.c_int64)]


POINT_DTYPE = np.dtype([("x", "<i4"), ("y", "<i4"), ("score", "<f4"), ("keep", "<i4")])
ATTEMPT_DTYPE = np.dtype([("status", "<i4"), ("fail_stage", "<i4"), ("i0", "<i4"),
                          ("i1", "<i4"), ("i2", "<i4"), ("inliers", "<i4"), ("qsum", "<u8"),
                          ("cx", "<f8"), ("cy", "<f8"), ("r2", "<f8")])
RESULT_DTYPE = np.dtype([("cx", "<f4"), ("cy", "<f4"), ("r", "<f4"), ("score", "<f4"),
                         ("inliers", "<i4"), ("n_points", "<i4"), ("valid", "<i4"),
                         ("reason", "<i4"), ("best_attempt", "<i4"), ("pad", "<i4"),
                         ("qsum", "<u8"), ("cxd", "<f8"), ("cyd", "<f8"), ("r2d", "<f8")])
assert POINT_DTYPE.itemsize == C.sizeof(Point)
assert ATTEMPT_DTYPE.itemsize == C.sizeof(Attempt)
assert RESULT_DTYPE.itemsize == C.sizeof(Result)

_lib = None
_P = C.POINTER


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        u8p, i32p, f32p = _P(C.c_uint8), _P(C.c_int32), _P(C.c_float)
        L.or_default_params.argtypes = [_P(Params)]
        L.or_strip_positions.argtypes = [C.c_int32, C.c_int32, C.c_double, i32p]
        L.or_sg_size.restype = C.c_int32
        L.or_build_tables.argtypes = [_P(Params), f32p, f32p, f32p]
        L.or_luma.argtypes = [C.c_int32] * 3
        L.or_luma.restype = C.c_int32
        L.or_pixel_features.argtypes = [u8p, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                        C.c_int32, _P(Pixel)]
        L.or_qgrad.argtypes = [C.c_int64]
        L.or_qgrad.restype = C.c_int32
        L.or_qtheta.argtypes = [C.c_int64, C.c_int64]
        L.or_qtheta.restype = C.c_int32
        L.or_candidates.argtypes = [u8p, C.c_int32, C.c_int32, C.c_int32, _P(Params), C.c_int,
                                    C.c_void_p]
        L.or_half_strip_scores.argtypes = [u8p, C.c_int32, C.c_int32, C.c_int32, _P(Params),
                                           C.c_int32, C.c_int32, C.c_int, f32p, i32p, i32p]
        L.or_philox4x64_10.argtypes = [_P(C.c_uint64), _P(C.c_uint64), _P(C.c_uint64)]
        L.or_draw_triple.argtypes = [C.c_uint64, C.c_uint64, C.c_int32, C.c_int32, i32p]
        L.or_circle3.argtypes = [_P(C.c_int64), _P(C.c_int64), _P(C.c_double),
                                 _P(C.c_double), _P(C.c_double)]
        L.or_lsq_circle.argtypes = [_P(C.c_int64), _P(C.c_int64), C.c_int32, _P(C.c_double),
                                    _P(C.c_double), _P(C.c_double)]
        L.or_ransac_attempts.argtypes = [i32p, i32p, _P(C.c_uint32), C.c_int32, C.c_int32,
                                         C.c_int32, C.c_uint64, _P(Params), C.c_void_p]
        L.or_estimate.argtypes = [u8p, C.c_int32, C.c_int32, C.c_int32, C.c_uint64, _P(Params),
                                  C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_estimate_bruteforce.argtypes = [u8p, C.c_int32, C.c_int32, C.c_int32, C.c_uint64,
                                             _P(Params), C.c_void_p]
        _lib = L
    return _lib


def params(**kw) -> Params:
    """Paper defaults (Table A1) with keyword overrides."""
    p = Params()
    lib().or_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _frame(frame: np.ndarray):
    f = np.ascontiguousarray(frame, dtype=np.uint8)
    if f.ndim != 3 or f.shape[2] != 3:
        raise ValueError("frame must be uint8 [H, W, 3]")
    return f, f.shape[1], f.shape[0], f.strides[0]


def _u8(a):
    return a.ctypes.data_as(_P(C.c_uint8))


def strip_positions(extent: int, n: int, alpha: float = 8.0) -> np.ndarray:
    out = np.zeros(max(n, 1), dtype=np.int32)
    rc = lib().or_strip_positions(extent, n, alpha, out.ctypes.data_as(_P(C.c_int32)))
    if rc != 0:
        raise ValueError("bad strip arguments")
    return out[:n]


def tables(p: Params | None = None):
    """(SG, ST, SI) float32 score tables."""
    p = p or params()
    sg = np.zeros(lib().or_sg_size(), dtype=np.float32)
    st = np.zeros(2049, dtype=np.float32)
    si = np.zeros(256, dtype=np.float32)
    f = lambda a: a.ctypes.data_as(_P(C.c_float))  # noqa: E731
    lib().or_build_tables(C.byref(p), f(sg), f(st), f(si))
    return sg, st, si


def luma(r: int, g: int, b: int) -> int:
    return lib().or_luma(r, g, b)


def qgrad(m2: int) -> int:
    return lib().or_qgrad(m2)


def qtheta(dt: int, cr: int) -> int:
    return lib().or_qtheta(dt, cr)


def pixel_features(frame: np.ndarray, x: int, y: int) -> dict:
    f, w, h, rs = _frame(frame)
    o = Pixel()
    if lib().or_pixel_features(_u8(f), w, h, rs, x, y, C.byref(o)) != 0:
        raise ValueError("pixel out of range")
    return {k: getattr(o, k) for k, _ in Pixel._fields_ if k != "iota_unused"}


def candidates(frame: np.ndarray, p: Params | None = None, ideal: bool = False) -> np.ndarray:
    p = p or params()
    f, w, h, rs = _frame(frame)
    P = 2 * (p.n_hstrips + p.n_vstrips)
    out = np.zeros(P, dtype=POINT_DTYPE)
    rc = lib().or_candidates(_u8(f), w, h, rs, C.byref(p), int(ideal), out.ctypes.data)
    if rc < 0:
        raise ValueError(f"or_candidates failed: {rc}")
    return out


def half_strip_scores(frame: np.ndarray, strip: int, half: int, p: Params | None = None,
                      ideal: bool = False):
    p = p or params()
    f, w, h, rs = _frame(frame)
    n = max(w, h)
    sc = np.zeros(n, dtype=np.float32)
    xs = np.zeros(n, dtype=np.int32)
    ys = np.zeros(n, dtype=np.int32)
    L = lib().or_half_strip_scores(_u8(f), w, h, rs, C.byref(p), strip, half, int(ideal),
                                   sc.ctypes.data_as(_P(C.c_float)),
                                   xs.ctypes.data_as(_P(C.c_int32)),
                                   ys.ctypes.data_as(_P(C.c_int32)))
    if L < 0:
        raise ValueError("bad half strip")
    return sc[:L], xs[:L], ys[:L]


def philox4x64_10(ctr, key) -> list[int]:
    c = (C.c_uint64 * 4)(*ctr)
    k = (C.c_uint64 * 2)(*key)
    o = (C.c_uint64 * 4)()
    lib().or_philox4x64_10(c, k, o)
    return list(o)


def draw_triple(seed: int, uid: int, a: int, n: int) -> tuple[int, int, int]:
    t = (C.c_int32 * 3)()
    lib().or_draw_triple(seed, uid, a, n, t)
    return tuple(t)


def circle3(xs, ys):
    x = (C.c_int64 * 3)(*[int(v) for v in xs])
    y = (C.c_int64 * 3)(*[int(v) for v in ys])
    cx, cy, r2 = C.c_double(), C.c_double(), C.c_double()
    ok = lib().or_circle3(x, y, C.byref(cx), C.byref(cy), C.byref(r2))
    return (cx.value, cy.value, r2.value) if ok else None


def lsq_circle(xs, ys):
    m = len(xs)
    x = (C.c_int64 * max(m, 1))(*[int(v) for v in xs])
    y = (C.c_int64 * max(m, 1))(*[int(v) for v in ys])
    cx, cy, r2 = C.c_double(), C.c_double(), C.c_double()
    ok = lib().or_lsq_circle(x, y, m, C.byref(cx), C.byref(cy), C.byref(r2))
    return (cx.value, cy.value, r2.value) if ok else None


def ransac_attempts(xs, ys, sq, w: int, h: int, uid: int, p: Params) -> np.ndarray:
    xs = np.ascontiguousarray(xs, dtype=np.int32)
    ys = np.ascontiguousarray(ys, dtype=np.int32)
    sq = np.ascontiguousarray(sq, dtype=np.uint32)
    out = np.zeros(p.attempts, dtype=ATTEMPT_DTYPE)
    rc = lib().or_ransac_attempts(xs.ctypes.data_as(_P(C.c_int32)),
                                  ys.ctypes.data_as(_P(C.c_int32)),
                                  sq.ctypes.data_as(_P(C.c_uint32)), len(xs), w, h, uid,
                                  C.byref(p), out.ctypes.data)
    if rc < 0:
        raise ValueError(f"or_ransac_attempts failed: {rc}")
    return out


def estimate(frame: np.ndarray, p: Params | None = None, uid: int = 0,
             with_points: bool = False, with_attempts: bool = False):
    """Whole pipeline on one frame -> RESULT_DTYPE record (and optional detail)."""
    p = p or params()
    f, w, h, rs = _frame(frame)
    P = 2 * (p.n_hstrips + p.n_vstrips)
    res = np.zeros(1, dtype=RESULT_DTYPE)
    pts = np.zeros(P, dtype=POINT_DTYPE) if with_points else None
    att = np.zeros(p.attempts, dtype=ATTEMPT_DTYPE) if with_attempts else None
    rc = lib().or_estimate(_u8(f), w, h, rs, uid, C.byref(p),
                           pts.ctypes.data if pts is not None else None,
                           att.ctypes.data if att is not None else None, res.ctypes.data)
    if rc < 0:
        raise ValueError(f"or_estimate failed: {rc}")
    out = [res[0]]
    if with_points:
        out.append(pts)
    if with_attempts:
        out.append(att)
    return out[0] if len(out) == 1 else tuple(out)


def estimate_bruteforce(frame: np.ndarray, p: Params | None = None, uid: int = 0):
    p = p or params()
    f, w, h, rs = _frame(frame)
    res = np.zeros(1, dtype=RESULT_DTYPE)
    rc = lib().or_estimate_bruteforce(_u8(f), w, h, rs, uid, C.byref(p), res.ctypes.data)
    if rc < 0:
        raise ValueError(f"or_estimate_bruteforce failed: {rc}")
    return res[0]


def estimate_batch(frames: np.ndarray, p: Params | None = None, uids=None,
                   threads: int = 1) -> np.ndarray:
    """Oracle on every frame of a [B, H, W, 3] batch; ``threads`` > 1 runs
    frames concurrently (ctypes releases the GIL during each call)."""
    p = p or params()
    B = frames.shape[0]
    uids = list(range(B)) if uids is None else [int(u) for u in uids]
    out = np.zeros(B, dtype=RESULT_DTYPE)

    def one(i):
        out[i] = estimate(frames[i], p, uids[i])

    if threads <= 1:
        for i in range(B):
            one(i)
    else:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(one, range(B)))
    return out
