"""ctypes wrapper of ``wmb_oracle.c`` (the FP64 reference; test infrastructure).

Verbs mirror the GPU library: create with patch descriptors, set/get interior
state, fill ghosts, compute dt, advance, run steps, diagnostics.  All arrays are
host numpy float64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wmb_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build_oracle(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no contraction, OpenMP over patches)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class OracleParams(C.Structure):
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
        ("pad_", C.c_int32),
        ("rho_protect", C.c_double),
        ("p_protect", C.c_double),
    ]


class _PatchDesc(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("nbr", C.c_int32 * 27)]


def default_params(dx=(1.0, 1.0, 1.0), gamma=5.0 / 3.0, cfl=0.4, ghost=5,
                   eps=(0.1, 0.0, 0.1, 0.0, 0.1, 0.0, 0.1), limiter_beta=1.0,
                   rho_floor=1e-10, p_floor=1e-10, degen_tol=1e-12, rho_protect=0.0,
                   p_protect=0.0) -> OracleParams:
    p = OracleParams()
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
    p.rho_protect = rho_protect
    p.p_protect = p_protect
    return p


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_oracle(force=True)
        lib = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        lib.orc_create.restype = C.c_void_p
        lib.orc_create.argtypes = [C.POINTER(OracleParams), C.c_int, C.POINTER(_PatchDesc)]
        lib.orc_destroy.argtypes = [C.c_void_p]
        lib.orc_keep_stages.argtypes = [C.c_void_p, C.c_int]
        lib.orc_set_state.argtypes = [C.c_void_p, C.c_int, dp, dp]
        lib.orc_get_state.argtypes = [C.c_void_p, C.c_int, dp, dp]
        lib.orc_get_stored.argtypes = [C.c_void_p, C.c_int, dp, dp]
        lib.orc_set_stored.argtypes = [C.c_void_p, C.c_int, dp, dp]
        lib.orc_fill_ghosts.argtypes = [C.c_void_p]
        lib.orc_compute_dt.restype = C.c_double
        lib.orc_compute_dt.argtypes = [C.c_void_p]
        lib.orc_advance.argtypes = [C.c_void_p, C.c_double]
        lib.orc_run_steps.restype = C.c_double
        lib.orc_run_steps.argtypes = [C.c_void_p, C.c_int]
        lib.orc_stage.restype = C.c_int
        lib.orc_stage.argtypes = [C.c_void_p, C.c_int, C.c_int, dp]
        lib.orc_diagnostics.argtypes = [C.c_void_p, dp, dp, dp, C.POINTER(C.c_int64)]
        lib.orc_phys_flux.argtypes = [dp, C.c_double, dp]
        lib.orc_eigensystem.argtypes = [dp, dp, C.POINTER(OracleParams), dp, dp, dp]
        lib.orc_line_fluxes.argtypes = [C.POINTER(OracleParams), C.c_int, dp, dp, C.c_double, dp]
        lib.orc_hll_flux.argtypes = [dp, dp, C.POINTER(OracleParams), dp]
        lib.orc_floor_state.restype = C.c_int
        lib.orc_floor_state.argtypes = [C.POINTER(OracleParams), dp]
        lib.orc_floor_added.argtypes = [C.c_void_p, dp]
        lib.orc_num_threads.restype = C.c_int
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def phys_flux(u, gamma):
    """Physical flux of the 1D system for a frame-ordered 8-state."""
    lib = _load()
    u = np.ascontiguousarray(u, dtype=np.float64)
    f = np.zeros(8)
    lib.orc_phys_flux(_p(u), gamma, _p(f))
    return f


def eigensystem(uL, uR, params: OracleParams):
    """Roe eigenvalues (7), right eigenvectors R[c, k] and left L[k, c] (7x7)."""
    lib = _load()
    uL = np.ascontiguousarray(uL, dtype=np.float64)
    uR = np.ascontiguousarray(uR, dtype=np.float64)
    lam = np.zeros(7)
    R = np.zeros(49)
    L = np.zeros(49)
    lib.orc_eigensystem(_p(uL), _p(uR), C.byref(params), _p(lam), _p(R), _p(L))
    return lam, R.reshape(7, 7), L.reshape(7, 7)


def hll_flux(uL, uR, params: OracleParams):
    """HLL flux of the protection path for two frame-ordered 8-states."""
    lib = _load()
    uL = np.ascontiguousarray(uL, dtype=np.float64)
    uR = np.ascontiguousarray(uR, dtype=np.float64)
    out = np.zeros(8)
    lib.orc_hll_flux(_p(uL), _p(uR), C.byref(params), _p(out))
    return out


def floor_state(params: OracleParams, u):
    """The floor rule applied to one lab-ordered 8-state; returns (fired, new state)."""
    lib = _load()
    u = np.array(u, dtype=np.float64)
    hit = lib.orc_floor_state(C.byref(params), _p(u))
    return bool(hit), u


def line_fluxes(params: OracleParams, q8: np.ndarray, bf: np.ndarray, lam: float) -> np.ndarray:
    """MHDTVD fluxes on a line: q8 (m, 8) frame states, bf (m,) left-face B_par.
    Returns (m, 8) fluxes at faces 2..m-2 (NaN elsewhere)."""
    lib = _load()
    q8 = np.ascontiguousarray(q8, dtype=np.float64)
    bf = np.ascontiguousarray(bf, dtype=np.float64)
    m = q8.shape[0]
    out = np.zeros((m, 8))
    lib.orc_line_fluxes(C.byref(params), m, _p(q8), _p(bf), lam, _p(out))
    return out


class OracleSim:
    """Host FP64 simulation over patches (same verbs as the GPU library)."""

    def __init__(self, params: OracleParams, descs):
        """descs: list of (n(3,), nbr(27,)) with n = (nx, ny, nz)."""
        self.lib = _load()
        self.params = params
        arr = (_PatchDesc * len(descs))()
        self.n = []
        for i, (n, nbr) in enumerate(descs):
            for a in range(3):
                arr[i].n[a] = int(n[a])
            for t in range(27):
                arr[i].nbr[t] = int(nbr[t])
            self.n.append(tuple(int(x) for x in n))
        self.npatch = len(descs)
        self.h = self.lib.orc_create(C.byref(params), len(descs), arr)
        self.g = params.ghost

    def close(self):
        if self.h:
            self.lib.orc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stored_shape(self, ip):
        nx, ny, nz = self.n[ip]
        g = self.g
        return (nz + 2 * g, ny + 2 * g, nx + 2 * g)

    def keep_stages(self, on=True):
        self.lib.orc_keep_stages(self.h, 1 if on else 0)

    def set_state(self, ip, q, b):
        nx, ny, nz = self.n[ip]
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(8, nz, ny, nx)
        b = np.ascontiguousarray(b, dtype=np.float64).reshape(3, nz, ny, nx)
        self.lib.orc_set_state(self.h, ip, _p(q), _p(b))

    def get_state(self, ip):
        nx, ny, nz = self.n[ip]
        q = np.zeros((8, nz, ny, nx))
        b = np.zeros((3, nz, ny, nx))
        self.lib.orc_get_state(self.h, ip, _p(q), _p(b))
        return q, b

    def get_stored(self, ip):
        sh = self.stored_shape(ip)
        q = np.zeros((8,) + sh)
        b = np.zeros((3,) + sh)
        self.lib.orc_get_stored(self.h, ip, _p(q), _p(b))
        return q, b

    def set_stored(self, ip, q, b):
        sh = self.stored_shape(ip)
        q = np.ascontiguousarray(q, dtype=np.float64).reshape((8,) + sh)
        b = np.ascontiguousarray(b, dtype=np.float64).reshape((3,) + sh)
        self.lib.orc_set_stored(self.h, ip, _p(q), _p(b))

    def fill_ghosts(self):
        self.lib.orc_fill_ghosts(self.h)

    def compute_dt(self) -> float:
        return float(self.lib.orc_compute_dt(self.h))

    def advance(self, dt: float):
        self.lib.orc_advance(self.h, float(dt))

    def run_steps(self, nsteps: int) -> float:
        return float(self.lib.orc_run_steps(self.h, int(nsteps)))

    def stage(self, ip, stage):
        sh = self.stored_shape(ip)
        nw = {1: 24, 2: 3, 3: 3, 4: 24, 5: 24, 6: 3}[stage]
        out = np.zeros((nw,) + sh)
        rc = self.lib.orc_stage(self.h, ip, stage, _p(out))
        if rc != 0:
            raise RuntimeError("stage %d not kept (rc=%d)" % (stage, rc))
        if nw == 24:
            return out.reshape((3, 8) + sh)
        return out

    def diagnostics(self):
        tot = np.zeros(8)
        dn = np.zeros(1)
        dr = np.zeros(1)
        nf = C.c_int64(0)
        self.lib.orc_diagnostics(self.h, _p(tot), _p(dn), _p(dr), C.byref(nf))
        return tot, float(dn[0]), float(dr[0]), int(nf.value)

    def floor_added(self):
        """(mass, total energy) the final-update floors added since creation, times dV."""
        out = np.zeros(2)
        self.lib.orc_floor_added(self.h, _p(out))
        return float(out[0]), float(out[1])

    def num_threads(self) -> int:
        return int(self.lib.orc_num_threads())
