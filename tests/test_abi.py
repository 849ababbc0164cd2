"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
and its host-side helpers (argument checks, Eq. 1 positions, Eq. 2 tables)
agree with the oracle.  No device work runs here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_2210_14771_amd import _native as N
from paper_2210_14771_amd import api
from paper_2210_14771_amd.build import LIB_PATH

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "contentarea.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ca_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB_PATH), "build the library first"
    L = C.CDLL(LIB_PATH)
    names = _declared()
    assert "ca_estimate_area" in names and len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert set(N.EXPORTS) == set(names)


def test_struct_sizes_match_header():
    text = open(os.path.join(ROOT, "include", "contentarea.h")).read()
    assert "(32 bytes)" in text and "(8 bytes)" in text and "(56 bytes)" in text
    assert C.sizeof(N.FrameDesc) == 32 and C.sizeof(N.ResultRec) == 32
    assert C.sizeof(N.PointRec) == 8 and C.sizeof(N.AttemptRec) == 56


def test_defaults_equal_oracle_defaults():
    p, q = api.default_params(), oracle.params()
    for f in ("n_hstrips", "n_vstrips", "alpha", "t_g", "t_theta_deg", "t_iota", "t_ps", "t_cs",
              "t_px", "refine_iters", "t_ri", "r_min", "r_max", "d_max", "sampler", "seed"):
        assert getattr(p, f) == getattr(q, f), f
    assert p.ransac_attempts == q.attempts


@pytest.mark.parametrize("extent,n", [(480, 16), (640, 16), (1080, 32), (1920, 32), (2160, 64),
                                      (3840, 64), (17, 5), (16, 1)])
def test_strip_positions_equal_oracle(extent, n):
    np.testing.assert_array_equal(api.strip_positions(extent, n), oracle.strip_positions(extent, n))


@pytest.mark.parametrize("kw", [{}, {"t_g": 7.5, "t_theta_deg": 12.0, "t_iota": 60.0},
                                {"t_g": 55.0}])
def test_score_tables_bytewise_equal_oracle(kw):
    sg, st, si = api.score_tables(api.default_params(**kw))
    osg, ost, osi = oracle.tables(oracle.params(**kw))
    assert sg.tobytes() == osg[:len(sg)].tobytes()
    # beyond its end the library's gradient table is saturated: every oracle entry is 1.0f
    assert sg[-1] == 1.0 and np.all(osg[len(sg):] == 1.0)
    assert st.tobytes() == ost.tobytes() and si.tobytes() == osi.tobytes()


def _descs(n, w=640, h=480, **kw):
    a = (N.FrameDesc * n)()
    for i in range(n):
        a[i].width, a[i].height, a[i].row_stride, a[i].pixel_stride = w, h, 3 * w, 3
        a[i].byte_offset = i * 3 * w * h
        a[i].frame_uid = i
        for k, v in kw.items():
            setattr(a[i], k, v)
    return a


def _check(descs, n, **pkw):
    p = api.default_params(**pkw)
    return N.lib().ca_check_args(descs, n, C.byref(p))


def test_argument_checks():
    L = N.lib()
    assert _check(_descs(4), 4) == N.CA_OK
    assert L.ca_check_args(None, 0, None) == N.CA_OK
    assert L.ca_check_args(None, 3, None) == N.CA_E_INVAL
    assert L.ca_check_args(None, -1, None) == N.CA_E_INVAL
    assert _check(_descs(1, w=15), 1) == N.CA_E_INVAL
    assert _check(_descs(1, h=10), 1) == N.CA_E_INVAL
    assert _check(_descs(1, w=N.CA_MAX_EXTENT + 1), 1) == N.CA_E_INVAL
    assert _check(_descs(1, row_stride=100), 1) == N.CA_E_INVAL
    assert _check(_descs(1, byte_offset=-16), 1) == N.CA_E_INVAL
    assert _check(_descs(1, pixel_stride=4), 1) == N.CA_E_UNSUPPORTED
    assert _check(_descs(1), 1, n_hstrips=65) == N.CA_E_INVAL
    assert _check(_descs(1), 1, n_hstrips=0, n_vstrips=0) == N.CA_E_INVAL
    assert _check(_descs(1), 1, n_hstrips=0, n_vstrips=4) == N.CA_OK
    assert _check(_descs(1), 1, n_hstrips=64, n_vstrips=64) == N.CA_OK
    assert _check(_descs(1), 1, ransac_attempts=0) == N.CA_E_INVAL
    assert _check(_descs(1), 1, ransac_attempts=N.CA_MAX_ATTEMPTS + 1) == N.CA_E_INVAL
    assert _check(_descs(1), 1, ransac_attempts=N.CA_MAX_ATTEMPTS) == N.CA_OK
    assert _check(_descs(1), 1, sampler=2) == N.CA_E_INVAL
    assert _check(_descs(1), 1, t_g=0.0) == N.CA_E_INVAL
    assert _check(_descs(1), 1, t_cs=float("nan")) == N.CA_E_INVAL
    assert _check(_descs(1), 1, t_px=-1) == N.CA_E_INVAL


def test_null_context_is_rejected_without_device_work():
    L = N.lib()
    d = _descs(1)
    assert L.ca_estimate_area(None, None, d, 1, None, None, None) == N.CA_E_INVAL
    assert L.ca_debug_candidates(None, None, d, 1, None, None, None, None) == N.CA_E_INVAL
    assert L.ca_debug_attempts(None, None, d, 1, None, None, None, None) == N.CA_E_INVAL
    assert L.ca_create(None, 0, 0) == N.CA_E_INVAL
    L.ca_destroy(None)


def test_error_strings():
    L = N.lib()
    for code in (0, -1, -2, -3, -4, 7):
        assert isinstance(L.ca_error_string(code), bytes)
    assert L.ca_error_string(-3) != L.ca_error_string(-4)
    assert L.ca_version().startswith(b"contentarea")
