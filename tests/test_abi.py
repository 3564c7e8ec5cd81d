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
    assert abs(b64 - 2 * b32) <= 256 * len(G.descs)  # regions are 256-byte aligned


def test_pool_bytes_with_scratch_groups(lib):
    """With scratch groups the patches keep 22 words of state a ghosted zone
    and share the 51 words of step intermediates group by group (whole
    x-rows dealt in turn): 2 x 2 x 2 patches of 32^3 have 4 x-rows, so 4
    groups hold one row (2 patches) each and the pool is 8 states and 2
    scratch slots; 2 groups hold 2 rows each (4 slots)."""
    from paper_1701_07452_amd import inputs as I
    from paper_1701_07452_amd import wmb

    G = I.uniform_grid(64, 32)
    g = 4
    vol = (32 + 2 * g) ** 3
    for prec, es in ((wmb.WMB_FP32, 4), (wmb.WMB_FP64, 8)):
        def align(b):
            return (b + 255) // 256 * 256
        st, sc = align(22 * vol * es), align(51 * vol * es)
        sizes = {k: wmb.pool_bytes(wmb.make_params(precision=prec, ghost=g, scratch_groups=k), G.descs)
                 for k in (0, 1, 2, 4, 8)}
        assert sizes[0] == sizes[1] == 8 * (st + sc)
        assert sizes[2] == 8 * st + 4 * sc
        assert sizes[4] == 8 * st + 2 * sc
        assert sizes[8] == 8 * st + 2 * sc  # only 4 rows: groups beyond them stay empty
    p = wmb.make_params(scratch_groups=65)
    h = C.c_void_p()
    assert lib.wmb_create(C.byref(p), C.byref(h)) == wmb.WMB_EINVAL


C_PROGRAM = r"""
#include <stdio.h>
#include <string.h>
#include "wmb.h"

int main(void) {
    wmb_params p;
    memset(&p, 0, sizeof p);
    p.gamma = 5.0 / 3.0;
    p.cfl = 0.4;
    for (int k = 0; k < 7; k++) p.eps[k] = (k % 2 == 0) ? 0.1 : 0.0;
    p.limiter_beta = 1.0;
    p.rho_floor = 1e-10;
    p.p_floor = 1e-10;
    for (int a = 0; a < 3; a++) p.dx[a] = 1.0 / 32;
    p.degen_tol = 1e-12;
    p.ghost = 4;
    p.precision = WMB_FP32;
    wmb_ctx *c = NULL;
    int rc = wmb_create(&p, &c);
    int rc_bad;
    p.dt_lag = 3;
    {
        wmb_ctx *d = NULL;
        rc_bad = wmb_create(&p, &d);
    }
    printf("%zu %zu %d %d %s\n", sizeof(wmb_params), sizeof(wmb_patch_desc), rc, rc_bad, wmb_strerror(WMB_ESIZE));
    return wmb_destroy(c);
}
"""


def test_header_is_c_and_links(lib, tmp_path):
    """The header compiles as C99 with gcc (-Wall -Werror); a C program links
    against libwmb.so, creates and destroys a context and reads an error
    string (no GPU needed); its struct sizes equal the ctypes binding's."""
    import shutil
    import subprocess

    from paper_1701_07452_amd import build, wmb
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    src = tmp_path / "abi.c"
    src.write_text(C_PROGRAM)
    exe = tmp_path / "abi"
    libdir = os.path.dirname(build.LIB)
    cmd = ["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe),
           "-L", libdir, "-l:libwmb.so", "-Wl,-rpath," + libdir, "-Wl,-rpath,/opt/rocm/lib"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    sp, sd, rc, rc_bad, msg = out.stdout.split(" ", 4)
    assert int(sp) == C.sizeof(wmb.Params) and int(sd) == C.sizeof(wmb.PatchDesc)
    assert int(rc) == 0 and int(rc_bad) == wmb.WMB_EINVAL
    assert msg.strip() == lib.wmb_strerror(wmb.WMB_ESIZE).decode()


def test_patch_table_checks_reject_malformed_tables(lib):
    """wmb_init_patches validates the neighbour table before it touches the
    device: random corruptions of a valid 3 x 2 x 2 table (ids out of range,
    wrong self entry, asymmetric or inconsistent edges, bad extents, huge
    edges) are all rejected with WMB_EINVAL, without a crash.  A table whose
    corrupted entry points outside the patch list is checked before any chain
    through it is followed.  (The valid table itself passes the check; on a
    machine without a GPU the call then fails later, in HIP.)"""
    import numpy as np

    from paper_1701_07452_amd import inputs as I
    from paper_1701_07452_amd import wmb

    G = I.patch_grid([8, 8, 8], [8, 8], [8, 8], periodic=(True, False, True))
    good = wmb.descs_to_c(G.descs, G.origin)
    n = len(G.descs)
    rng = np.random.default_rng(7)
    cases = 0
    for trial in range(400):
        d = (wmb.PatchDesc * n)()
        C.memmove(d, good, C.sizeof(d))
        i = int(rng.integers(n))
        kind = trial % 5
        if kind == 0:  # id out of range (either side), on a face entry
            d[i].nbr[int(rng.choice([4, 10, 12, 14, 16, 22]))] = int(rng.choice([-2, n, n + 1000, 2 ** 30]))
        elif kind == 1:  # self entry
            d[i].nbr[13] = (i + 1) % n
        elif kind == 2:  # some other entry moved to another patch
            t = int(rng.choice([t for t in range(27) if t != 13]))
            d[i].nbr[t] = (d[i].nbr[t] + 1 + int(rng.integers(n - 1))) % n if d[i].nbr[t] >= 0 else int(rng.integers(n))
        elif kind == 3:  # an extent that breaks the face-sharing rule, or below the ghost width
            d[i].n[int(rng.integers(3))] = int(rng.choice([3, 9, 12]))
        else:  # an absurd edge
            d[i].n[int(rng.integers(3))] = int(rng.choice([70000, 2 ** 31 - 1]))
        h = C.c_void_p()
        p = wmb.make_params(ghost=4)
        assert lib.wmb_create(C.byref(p), C.byref(h)) == 0
        rc = lib.wmb_init_patches(h, n, d, C.c_void_p(1), C.c_uint64(1 << 40), None)
        assert rc == wmb.WMB_EINVAL, (trial, kind, rc)
        assert lib.wmb_destroy(h) == 0
        cases += 1
    assert cases == 400


@pytest.mark.parametrize("prec,edge,ok", [(1, 511, True), (1, 512, False), (0, 504, True), (0, 505, False)])
def test_edge_limits_of_the_kernels(lib, prec, edge, ok):
    """Interior edges beyond what the kernels take are rejected up front
    (WMB_EINVAL from wmb_pool_bytes and wmb_init_patches), before any device
    work: at most 511 zones along any axis (the sweeps' packed pencil
    rectangles), and at most 504 in FP64 (a Step-1 sweep block holds a whole
    pencil of n + 8 zones with 16 doubles of LDS a zone).  Thin patches keep
    the region far below its 4 GiB limit, so this check is the binding one."""
    from paper_1701_07452_amd import inputs as I
    from paper_1701_07452_amd import wmb

    for axis in range(3):
        n = [8, 8, 8]
        n[axis] = edge
        G = I.uniform_grid(tuple(n), tuple(n))
        p = wmb.make_params(ghost=4, precision=prec)
        d = wmb.descs_to_c(G.descs, G.origin)
        out = C.c_uint64(0)
        rc = lib.wmb_pool_bytes(C.byref(p), 1, d, C.byref(out))
        assert (rc == 0) == ok, (axis, rc)
        h = C.c_void_p()
        assert lib.wmb_create(C.byref(p), C.byref(h)) == 0
        rc = lib.wmb_init_patches(h, 1, d, C.c_void_p(1), C.c_uint64(1 << 40), None)
        if ok:
            assert rc != wmb.WMB_EINVAL  # passes the checks (then needs a GPU)
        else:
            assert rc == wmb.WMB_EINVAL
            assert b"above" in lib.wmb_last_error(h)
        assert lib.wmb_destroy(h) == 0
