"""Thin ctypes binding of ``libwmb.so`` (the C ABI declared in include/wmb.h).

Argument marshalling only: every step of the update runs in the HIP kernels.
Torch provides the device pool (one uint8 tensor) and the stream.  There is no
fallback: if the library is missing or no GPU is present, this module raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwmb.so")

WMB_OK, WMB_EINVAL, WMB_ENOMEM, WMB_EHIP, WMB_ESTATE, WMB_ECFL, WMB_ESIZE, WMB_EORDER = 0, -1, -2, -3, -4, -5, -6, -7
WMB_FP64, WMB_FP32 = 0, 1

EXPORTS = [
    "wmb_create", "wmb_pool_bytes", "wmb_init_patches", "wmb_set_state", "wmb_get_state", "wmb_get_stored",
    "wmb_fill_ghosts", "wmb_compute_dt", "wmb_advance", "wmb_run_steps", "wmb_diagnostics",
    "wmb_diagnostics_noalloc", "wmb_debug_stage",
    "wmb_autotune", "wmb_set_tuning", "wmb_set_schedule", "wmb_keep_stages", "wmb_set_active", "wmb_set_present",
    "wmb_profile_step", "wmb_destroy",
    "wmb_strerror", "wmb_last_error",
]
KERNEL_CLASSES = ["fill", "dt", "sweep1_x", "sweep1_y", "sweep1_z", "ct_half",
                  "sweep2_x", "sweep2_y", "sweep2_z", "update"]


class WmbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("wmb error %d: %s" % (code, msg))
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("gamma", C.c_double),
        ("cfl", C.c_double),
        ("eps", C.c_double * 7),
        ("limiter_beta", C.c_double),
        ("rho_floor", C.c_double),
        ("p_floor", C.c_double),
        ("dx", C.c_double * 3),
        ("degen_tol", C.c_double),
        ("ghost", C.c_int32),
        ("precision", C.c_int32),
        ("rho_protect", C.c_double),
        ("p_protect", C.c_double),
        ("dt_lag", C.c_int32),
        ("scratch_groups", C.c_int32),
    ]


class PatchDesc(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("nbr", C.c_int32 * 27), ("origin", C.c_int64 * 3)]


def make_params(dx=(1.0, 1.0, 1.0), gamma=5.0 / 3.0, cfl=0.4, ghost=5, precision=WMB_FP64,
                eps=(0.1, 0.0, 0.1, 0.0, 0.1, 0.0, 0.1), limiter_beta=1.0, rho_floor=1e-10, p_floor=1e-10,
                degen_tol=1e-12, rho_protect=0.0, p_protect=0.0, dt_lag=0, scratch_groups=0) -> Params:
    p = Params()
    p.gamma = gamma
    p.cfl = cfl
    for k in range(7):
        p.eps[k] = eps[k]
    p.limiter_beta = limiter_beta
    p.rho_floor = rho_floor
    p.p_floor = p_floor
    for a in range(3):
        p.dx[a] = dx[a]
    p.degen_tol = degen_tol
    p.ghost = ghost
    p.precision = precision
    p.rho_protect = rho_protect
    p.p_protect = p_protect
    p.dt_lag = dt_lag
    p.scratch_groups = scratch_groups
    return p


_lib = None


def load_library():
    """Load libwmb.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libwmb.so not built: run __graft_entry__.build() (or python -m paper_1701_07452_amd.build)")
    lib = C.CDLL(LIB_PATH)
    dp, vp = C.POINTER(C.c_double), C.c_void_p
    lib.wmb_create.argtypes = [C.POINTER(Params), C.POINTER(vp)]
    lib.wmb_pool_bytes.argtypes = [C.POINTER(Params), C.c_int32, C.POINTER(PatchDesc), C.POINTER(C.c_uint64)]
    lib.wmb_init_patches.argtypes = [vp, C.c_int32, C.POINTER(PatchDesc), vp, C.c_uint64, vp]
    lib.wmb_set_state.argtypes = [vp, C.c_int32, dp, dp]
    lib.wmb_get_state.argtypes = [vp, C.c_int32, dp, dp]
    lib.wmb_get_stored.argtypes = [vp, C.c_int32, dp, dp]
    lib.wmb_fill_ghosts.argtypes = [vp]
    lib.wmb_compute_dt.argtypes = [vp, dp]
    lib.wmb_advance.argtypes = [vp, C.c_double]
    lib.wmb_run_steps.argtypes = [vp, C.c_int32]
    lib.wmb_diagnostics.argtypes = [vp, dp, dp, dp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    lib.wmb_diagnostics_noalloc.argtypes = [vp, vp]
    lib.wmb_debug_stage.argtypes = [vp, C.c_int32, C.c_int32, dp]
    lib.wmb_profile_step.argtypes = [vp, dp, C.c_int32]
    lib.wmb_autotune.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.c_int32]
    lib.wmb_set_tuning.argtypes = [vp, C.POINTER(C.c_int32), C.c_int32]
    lib.wmb_set_schedule.argtypes = [vp, C.c_int32]
    lib.wmb_keep_stages.argtypes = [vp, C.c_int32]
    lib.wmb_set_active.argtypes = [vp, C.c_int32, C.c_int32]
    lib.wmb_set_present.argtypes = [vp, C.c_int32, C.c_int32]
    lib.wmb_destroy.argtypes = [vp]
    lib.wmb_strerror.argtypes = [C.c_int]
    lib.wmb_strerror.restype = C.c_char_p
    lib.wmb_last_error.argtypes = [vp]
    lib.wmb_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("wmb_strerror", "wmb_last_error"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def descs_to_c(descs, origins=None):
    arr = (PatchDesc * len(descs))()
    for i, (n, nbr) in enumerate(descs):
        for a in range(3):
            arr[i].n[a] = int(n[a])
            arr[i].origin[a] = int(origins[i][a]) if origins is not None else 0
        for t in range(27):
            arr[i].nbr[t] = int(nbr[t])
    return arr


def pool_bytes(params: Params, descs) -> int:
    lib = load_library()
    arr = descs_to_c(descs)
    out = C.c_uint64(0)
    rc = lib.wmb_pool_bytes(C.byref(params), len(descs), arr, C.byref(out))
    if rc != WMB_OK:
        raise WmbError(rc, lib.wmb_strerror(rc).decode())
    return int(out.value)


class Sim:
    """One context over a batch of patches on one GPU."""

    def __init__(self, params: Params, descs, origins=None, device="cuda:0", stream=None, pool=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the patch update runs only on the HIP library")
        self.lib = load_library()
        self.params = params
        self.n = [tuple(int(x) for x in n) for n, _ in descs]
        self.g = int(params.ghost)
        self.npatch = len(descs)
        self.h = C.c_void_p()
        self._check(self.lib.wmb_create(C.byref(params), C.byref(self.h)), ctx=False)
        self._descs = descs_to_c(descs, origins)
        nbytes = pool_bytes(params, descs)
        self.device = torch.device(device)
        self.pool = pool if pool is not None else torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._check(self.lib.wmb_init_patches(self.h, self.npatch, self._descs, C.c_void_p(self.pool.data_ptr()),
                                              C.c_uint64(self.pool.numel()), C.c_void_p(self.stream.cuda_stream)))

    # ------------------------------------------------------------------
    def _check(self, rc, ctx=True):
        if rc != WMB_OK:
            msg = self.lib.wmb_strerror(rc).decode()
            if ctx and self.h:
                msg += ": " + self.lib.wmb_last_error(self.h).decode()
            raise WmbError(rc, msg)

    def close(self):
        """Destroy the context and drop the pool tensor (its memory returns to
        torch's caching allocator once no other reference holds it)."""
        if getattr(self, "h", None) and self.h.value:
            self.lib.wmb_destroy(self.h)
            self.h = C.c_void_p()
        self.pool = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stored_shape(self, ip):
        nx, ny, nz = self.n[ip]
        g = self.g
        return (nz + 2 * g, ny + 2 * g, nx + 2 * g)

    # ------------------------------------------------------------------
    def set_state(self, ip, q, b):
        nx, ny, nz = self.n[ip]
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(8, nz, ny, nx)
        b = np.ascontiguousarray(b, dtype=np.float64).reshape(3, nz, ny, nx)
        self._check(self.lib.wmb_set_state(self.h, ip, _dp(q), _dp(b)))

    def get_state(self, ip):
        nx, ny, nz = self.n[ip]
        q = np.zeros((8, nz, ny, nx))
        b = np.zeros((3, nz, ny, nx))
        self._check(self.lib.wmb_get_state(self.h, ip, _dp(q), _dp(b)))
        return q, b

    def get_stored(self, ip):
        sh = self.stored_shape(ip)
        q = np.zeros((8,) + sh)
        b = np.zeros((3,) + sh)
        self._check(self.lib.wmb_get_stored(self.h, ip, _dp(q), _dp(b)))
        return q, b

    def fill_ghosts(self):
        self._check(self.lib.wmb_fill_ghosts(self.h))

    def compute_dt(self, fetch=True) -> Optional[float]:
        if fetch:
            out = np.zeros(1)
            self._check(self.lib.wmb_compute_dt(self.h, _dp(out)))
            return float(out[0])
        self._check(self.lib.wmb_compute_dt(self.h, None))
        return None

    def advance(self, dt: float = 0.0):
        self._check(self.lib.wmb_advance(self.h, float(dt)))

    def run_steps(self, nsteps: int):
        self._check(self.lib.wmb_run_steps(self.h, int(nsteps)))

    def diagnostics(self):
        tot = np.zeros(8)
        dn = np.zeros(1)
        dr = np.zeros(1)
        nf = C.c_int64(0)
        self._check(self.lib.wmb_diagnostics(self.h, _dp(tot), _dp(dn), _dp(dr), C.byref(nf), None))
        return tot, float(dn[0]), float(dr[0]), int(nf.value)

    def diagnostics_noalloc(self, out):
        """Enqueue the allocation-free diagnostics into `out`, a float64 device
        tensor of 12 (totals[8], div b normalised, raw, floors, protected)."""
        import torch

        if out.dtype != torch.float64 or out.numel() < 12 or not out.is_cuda or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 device tensor of 12 elements")
        self._check(self.lib.wmb_diagnostics_noalloc(self.h, C.c_void_p(out.data_ptr())))
        return out

    def protected_faces(self):
        """Faces that took the HLL flux (protection floors) since creation."""
        npr = C.c_int64(0)
        self._check(self.lib.wmb_diagnostics(self.h, None, None, None, None, C.byref(npr)))
        return int(npr.value)

    def debug_stage(self, ip, stage):
        sh = self.stored_shape(ip)
        nw = {1: 24, 3: 3, 5: 24, 6: 3}.get(stage, 3)
        out = np.zeros((nw,) + sh)
        self._check(self.lib.wmb_debug_stage(self.h, ip, stage, _dp(out)))
        return out.reshape((3, 8) + sh) if nw == 24 else out

    def autotune(self, reps=3):
        """Pick the sweep block shapes, the fused corrector's band rows and the Steps 3-4 / 8-11
        tiles by timing (or from the per-process cache; reps < 0 forces timing); returns
        {(stage, axis, edge): shape}, with (3, 0, 0) the Steps 3-4 tile width, (4, 0, 0) the
        Steps 8-11 tile zones, (5, 0, 0) their launch form and (6, 0, 0) the fused corrector's
        band rows (0: three separate corrector sweeps)."""
        buf = (C.c_int32 * 256)()
        self._check(self.lib.wmb_autotune(self.h, int(reps), buf, 256))
        out, k = {}, 0
        while k + 4 <= 256 and buf[k] != 0:
            out[(buf[k], buf[k + 1], buf[k + 2])] = buf[k + 3]
            k += 4
        return out

    def set_tuning(self, tuning):
        """Apply {(stage, axis, edge): shape} (as autotune returns it) without timing."""
        flat = [v for (st, ax, e), W in sorted(tuning.items()) for v in (st, ax, e, W)]
        buf = (C.c_int32 * max(len(flat), 1))(*flat)
        self._check(self.lib.wmb_set_tuning(self.h, buf, len(flat)))

    def set_schedule(self, groups):
        """Captured-step schedule: 1 (concurrent sweep branches) or 2..4 patch groups."""
        self._check(self.lib.wmb_set_schedule(self.h, int(groups)))

    def set_active(self, ip, on=True):
        """Freeze (on=False) or thaw a patch; the captured graphs stay valid."""
        self._check(self.lib.wmb_set_active(self.h, int(ip), 1 if on else 0))

    def set_present(self, ip, on=True):
        """Remove (on=False) or add back a patch slot of the init table; the captured graphs stay valid."""
        self._check(self.lib.wmb_set_present(self.h, int(ip), 1 if on else 0))

    def keep_stages(self, on=True):
        """Let later steps store the Step-9 edges for debug_stage(6)."""
        self._check(self.lib.wmb_keep_stages(self.h, 1 if on else 0))

    def profile_step(self):
        """Per-kernel-class durations (ms) of one eager step; advances the state."""
        out = np.zeros(len(KERNEL_CLASSES))
        self._check(self.lib.wmb_profile_step(self.h, _dp(out), len(KERNEL_CLASSES)))
        return dict(zip(KERNEL_CLASSES, out.tolist()))

    def synchronize(self):
        self.stream.synchronize()


def tuning_to_str(tuning):
    """{(1, 0, 32): 16, ...} -> '1x32=16,...' (stage, axis letter, edge)."""
    return ",".join("%d%s%d=%d" % (st, "xyz"[ax], e, W) for (st, ax, e), W in sorted(tuning.items()))


def tuning_from_str(s):
    out = {}
    for item in filter(None, s.split(",")):
        key, W = item.split("=")
        st, ax, e = int(key[0]), "xyz".index(key[1]), int(key[2:])
        out[(st, ax, e)] = int(W)
    return out


def sim_from_grid(G, q=None, b=None, **params_kw):
    """Convenience: Sim over a PatchGrid, optionally uploading global arrays."""
    from . import inputs as I

    prm = make_params(**params_kw)
    sim = Sim(prm, G.descs, origins=G.origin)
    if q is not None:
        for ip, (qp, bp) in enumerate(I.iter_split(G, q, b)):
            sim.set_state(ip, qp, bp)
    return sim
