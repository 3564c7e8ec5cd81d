"""CPU checks of the C ABI library: it loads and exports every symbol that
include/wmb.h declares; parameter validation that needs no GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1701_07452_amd import build, wmb
    if build.is_stale():
        build.build_library()
    return wmb.load_library()


def header_functions():
    src = open(os.path.join(ROOT, "include", "wmb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wmb_[a-z_]+)\s*\(", src)))


def test_header_declares_the_binding_exports():
    from paper_1701_07452_amd import wmb
    assert header_functions() == sorted(wmb.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in header_functions():
        assert hasattr(lib, name), name


def test_create_validates_params(lib):
    from paper_1701_07452_amd import wmb
    h = C.c_void_p()
    good = wmb.make_params()
    assert lib.wmb_create(C.byref(good), C.byref(h)) == 0
    assert lib.wmb_destroy(h) == 0
    for field, val in [("gamma", 1.0), ("cfl", 0.0), ("ghost", 3), ("precision", 7), ("limiter_beta", 2.5),
                       ("p_floor", 0.0), ("rho_protect", -1.0), ("dt_lag", 2)]:
        p = wmb.make_params()
        setattr(p, field, val)
        h = C.c_void_p()
        assert lib.wmb_create(C.byref(p), C.byref(h)) == wmb.WMB_EINVAL, field
    assert lib.wmb_strerror(wmb.WMB_ECFL).decode().startswith("dt above")
    # the last field of the struct is read (a layout mismatch would misplace it)
    p = wmb.make_params(dt_lag=1)
    h = C.c_void_p()
    assert lib.wmb_create(C.byref(p), C.byref(h)) == 0
    assert lib.wmb_destroy(h) == 0


def test_pool_bytes(lib):
    from paper_1701_07452_amd import inputs as I
    from paper_1701_07452_amd import wmb
    G = I.uniform_grid(64, 32)
    p32 = wmb.make_params(precision=wmb.WMB_FP32)
    p64 = wmb.make_params(precision=wmb.WMB_FP64)
    b32, b64 = wmb.pool_bytes(p32, G.descs), wmb.pool_bytes(p64, G.descs)
    vol = 42 ** 3
    assert b32 >= 8 * 73 * vol * 4 and b64 >= 8 * 73 * vol * 8
    assert b64 == 2 * b32
