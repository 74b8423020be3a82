"""The C-ABI libraries load and export every declared symbol; argument checks that need no GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    src = open(header).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tto?_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def ttlib():
    from paper_2007_08576_amd import tt
    if not os.path.exists(tt.LIB_PATH):
        from paper_2007_08576_amd import build
        build.build()
    return tt


def test_gpu_library_exports_every_declared_symbol(ttlib):
    L = ttlib.lib()
    names = _declared(os.path.join(ROOT, "include", "tt.h"))
    assert "tt_track_frame" in names and "tt_create_stream" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_oracle_library_exports_every_declared_symbol(O):
    L = O.lib()
    names = _declared(os.path.join(ROOT, "oracle", "tt_oracle.h"))
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_default_params_and_strerror(ttlib):
    p = ttlib.default_params()
    assert (p.w_orb, p.w_angle, p.w_rotation) == (10.0, 20.0, 100.0)
    assert (p.ransac_refs, p.ransac_iters, p.knn) == (30, 10, 4)
    for code in (0, -1, -2, -3, -4, -5):
        assert ttlib.strerror(code)


def test_create_stream_rejects_bad_arguments_before_touching_the_device(ttlib):
    L = ttlib.lib()
    K = ttlib.intrinsics(64, 48, 50, 50, 32, 24)
    h = C.c_void_p()
    for kw in (dict(knn=3), dict(num_control_points=0), dict(H=0.0), dict(precision=7), dict(ransac_refs=0)):
        p = ttlib.default_params(**kw)
        assert L.tt_create_stream(C.byref(p), C.byref(K), None, C.byref(h)) == ttlib.TT_EINVAL
    p = ttlib.default_params()
    bad = ttlib.intrinsics(2, 48, 50, 50, 32, 24)
    assert L.tt_create_stream(C.byref(p), C.byref(bad), None, C.byref(h)) == ttlib.TT_EINVAL
    assert L.tt_create_stream(None, C.byref(K), None, C.byref(h)) == ttlib.TT_EINVAL
    assert L.tt_set_template(None, None, 0, None, None, 0) == ttlib.TT_EINVAL
    assert L.tt_track_frame(None, None, None, None, 0, None, None, None) == ttlib.TT_EINVAL
    assert L.tt_destroy(None) == ttlib.TT_EINVAL


def test_product_does_not_reference_the_oracle():
    """The product package neither imports nor loads anything from oracle/."""
    pkg = os.path.join(ROOT, "paper_2007_08576_amd")
    pat = re.compile(r"^\s*(from|import)\s+oracle\b|tt_oracle|libtt_oracle|tto_", re.M)
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                assert not pat.search(open(os.path.join(dirpath, f)).read()), f
