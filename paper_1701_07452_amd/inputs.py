"""Seeded synthetic inputs for the patch MHD update.

This module is the only code that both the GPU path's callers (tests, bench)
and the FP64 oracle's callers use.  It holds none of the method's arithmetic:
it builds patch tilings and neighbour tables, initial states (primitive fields
converted to the conserved state of the 1D system's definition), face fields
from edge-centred vector potentials (so the discrete div b is zero), and the
closed-form solutions used as convergence targets.  Everything is numpy FP64
and seeded.

Workloads (shapes and distributions after the paper's test problems):
  * linear fast magnetosonic wave along the cube diagonal (Sect. 6.1 setup:
    rho = 1, P = 3/5, gamma = 5/3, B = (1, sqrt2, 1/2) in the wave frame);
  * Gaussian random velocity with a k^-5/3 energy spectrum (turbulence-like);
  * uneven tensor-product tilings with edge sizes from {16, 24, 32, 48, 64};
  * Orszag-Tang vortex extended in z (Sect. 6.5 setup);
  * lognormal-density Mach-5 turbulence at plasma beta 1;
  * circularly polarised Alfven wave (Sect. 6.9 setup) oblique to the grid.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = 5.0 / 3.0


# --------------------------------------------------------------------------
# patch tilings
# --------------------------------------------------------------------------

@dataclass
class PatchGrid:
    """Tensor-product tiling of a box into patches.

    sizes[a] lists the interior edge length of each slab along axis a (x, y, z).
    Patch id = (kz * py + jy) * px + ix.  nbr[27] follows the offset order
    9 (dz+1) + 3 (dy+1) + (dx+1); periodic axes wrap, along the others an
    offset that leaves the box is -1 (a domain boundary, outflow).
    """
    sizes: tuple
    descs: list = field(default_factory=list)
    origin: list = field(default_factory=list)

    @property
    def nblocks(self):
        return tuple(len(s) for s in self.sizes)

    @property
    def shape(self):
        """global interior shape (Nz, Ny, Nx)"""
        return (sum(self.sizes[2]), sum(self.sizes[1]), sum(self.sizes[0]))

    @property
    def npatch(self):
        px, py, pz = self.nblocks
        return px * py * pz

    def zones(self) -> int:
        return int(np.prod(self.shape))


def patch_grid(sizes_x, sizes_y, sizes_z, periodic=(True, True, True)) -> PatchGrid:
    sizes = (tuple(int(s) for s in sizes_x), tuple(int(s) for s in sizes_y), tuple(int(s) for s in sizes_z))
    G = PatchGrid(sizes)
    px, py, pz = G.nblocks
    offs = [np.concatenate([[0], np.cumsum(s)[:-1]]).astype(int) for s in sizes]
    for kz in range(pz):
        for jy in range(py):
            for ix in range(px):
                n = (sizes[0][ix], sizes[1][jy], sizes[2][kz])
                nbr = []
                for dz in (-1, 0, 1):
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            c = [ix + dx, jy + dy, kz + dz]
                            inside = all(periodic[a] or 0 <= c[a] < (px, py, pz)[a] for a in range(3))
                            nbr.append((((kz + dz) % pz) * py + (jy + dy) % py) * px + (ix + dx) % px if inside else -1)
                G.descs.append((n, nbr))
                G.origin.append((int(offs[0][ix]), int(offs[1][jy]), int(offs[2][kz])))
    return G


def uniform_grid(N, n, periodic=(True, True, True)) -> PatchGrid:
    """N^3 box (N may be a 3-tuple x,y,z) cut into patches of edge n (tuple ok)."""
    Nt = (N, N, N) if np.isscalar(N) else tuple(N)
    nt = (n, n, n) if np.isscalar(n) else tuple(n)
    for a in range(3):
        if Nt[a] % nt[a]:
            raise ValueError("box not divisible by patch size")
    return patch_grid([nt[0]] * (Nt[0] // nt[0]), [nt[1]] * (Nt[1] // nt[1]), [nt[2]] * (Nt[2] // nt[2]), periodic)


def uneven_grid(nb=(8, 10, 5), choices=(16, 24, 32, 48, 64), seed=170107453) -> PatchGrid:
    """Uneven batch: per-slab edge sizes drawn with a seed, separately per axis."""
    rng = np.random.default_rng(seed)
    sx = rng.choice(choices, size=nb[0])
    sy = rng.choice(choices, size=nb[1])
    sz = rng.choice(choices, size=nb[2])
    return patch_grid(sx, sy, sz)


def split(G: PatchGrid, q, b):
    """Global interior arrays (8|3, Nz, Ny, Nx) -> per-patch (q, b) lists."""
    out = []
    for (n, _), (ox, oy, oz) in zip(G.descs, G.origin):
        sl = (slice(None), slice(oz, oz + n[2]), slice(oy, oy + n[1]), slice(ox, ox + n[0]))
        out.append((np.ascontiguousarray(q[sl]), np.ascontiguousarray(b[sl])))
    return out


def iter_split(G: PatchGrid, q, b):
    """Like split, one patch at a time (no second copy of the whole box)."""
    for (n, _), (ox, oy, oz) in zip(G.descs, G.origin):
        sl = (slice(None), slice(oz, oz + n[2]), slice(oy, oy + n[1]), slice(ox, ox + n[0]))
        yield np.ascontiguousarray(q[sl]), np.ascontiguousarray(b[sl])


def gather(G: PatchGrid, parts):
    """Per-patch (q, b) -> global (8, Nz, Ny, Nx), (3, Nz, Ny, Nx)."""
    q = np.zeros((8,) + G.shape)
    b = np.zeros((3,) + G.shape)
    for (n, _), (ox, oy, oz), (qp, bp) in zip(G.descs, G.origin, parts):
        sl = (slice(None), slice(oz, oz + n[2]), slice(oy, oy + n[1]), slice(ox, ox + n[0]))
        q[sl] = qp
        b[sl] = bp
    return q, b


# --------------------------------------------------------------------------
# field construction helpers
# --------------------------------------------------------------------------

def coords(shape, dx, origin=(0.0, 0.0, 0.0)):
    """Zone-centre coordinates x, y, z (each (Nz, Ny, Nx)) and left-face coordinates."""
    Nz, Ny, Nx = shape
    xc = origin[0] + (np.arange(Nx) + 0.5) * dx[0]
    yc = origin[1] + (np.arange(Ny) + 0.5) * dx[1]
    zc = origin[2] + (np.arange(Nz) + 0.5) * dx[2]
    xf = origin[0] + np.arange(Nx) * dx[0]
    yf = origin[1] + np.arange(Ny) * dx[1]
    zf = origin[2] + np.arange(Nz) * dx[2]
    return (xc, yc, zc), (xf, yf, zf)


def curl_of_edge_potential(Ax, Ay, Az, dx):
    """Face field b = curl A on a periodic grid.

    Ax[k,j,i] sits on the x-edge (x_i centre, y_{j-1/2}, z_{k-1/2}), Ay on
    (x_{i-1/2}, y_j, z_{k-1/2}), Az on (x_{i-1/2}, y_{j-1/2}, z_k).  b_x[k,j,i]
    is on the face x_{i-1/2}; likewise b_y, b_z.  The discrete divergence of the
    result is zero to rounding.
    """
    def up(a, axis):  # value at index + 1 along a (z=0, y=1, x=2) axis, periodic
        return np.roll(a, -1, axis=axis)

    bx = (up(Az, 1) - Az) / dx[1] - (up(Ay, 0) - Ay) / dx[2]
    by = (up(Ax, 0) - Ax) / dx[2] - (up(Az, 2) - Az) / dx[0]
    bz = (up(Ay, 2) - Ay) / dx[0] - (up(Ax, 1) - Ax) / dx[1]
    return np.stack([bx, by, bz])


def face_average(b):
    """Zone-centred field as the mean of the two faces along each axis (periodic)."""
    return np.stack([0.5 * (b[0] + np.roll(b[0], -1, axis=2)),
                     0.5 * (b[1] + np.roll(b[1], -1, axis=1)),
                     0.5 * (b[2] + np.roll(b[2], -1, axis=0))])


def conserved(rho, v, Bcc, P, gamma=GAMMA):
    """Conserved state (rho, rho v, B, E) with E = P/(gamma-1) + rho v^2/2 + B^2/2."""
    rho = np.asarray(rho, dtype=np.float64)
    shape = np.broadcast_shapes(rho.shape, v[0].shape, Bcc[0].shape, np.shape(P))
    q = np.zeros((8,) + shape)
    q[0] = rho
    for a in range(3):
        q[1 + a] = rho * v[a]
        q[4 + a] = Bcc[a]
    q[7] = P / (gamma - 1.0) + 0.5 * rho * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2) + 0.5 * (Bcc[0] ** 2 + Bcc[1] ** 2 + Bcc[2] ** 2)
    return q


def uniform_faces(shape, B0):
    return np.stack([np.full(shape, float(B0[a])) for a in range(3)])


# --------------------------------------------------------------------------
# linear fast wave along the diagonal (C1 workload; convergence target)
# --------------------------------------------------------------------------

def _primitive_matrix(rho, vx, bx, by, bz, p, gamma):
    """Quasi-linear matrix of the 1D primitive MHD system, W = (rho, vx, vy, vz, By, Bz, P),
    with Bx a parameter (textbook form, written out independently of any solver)."""
    A = np.zeros((7, 7))
    A[0, 0] = vx; A[0, 1] = rho
    A[1, 1] = vx; A[1, 4] = by / rho; A[1, 5] = bz / rho; A[1, 6] = 1.0 / rho
    A[2, 2] = vx; A[2, 4] = -bx / rho
    A[3, 3] = vx; A[3, 5] = -bx / rho
    A[4, 1] = by; A[4, 2] = -bx; A[4, 4] = vx
    A[5, 1] = bz; A[5, 3] = -bx; A[5, 5] = vx
    A[6, 1] = gamma * p; A[6, 6] = vx
    return A


@dataclass
class LinearWave:
    """Plane wave q = qbar + amp * dq * cos(k.x - omega t) on a periodic box."""
    kvec: np.ndarray
    omega: float
    qbar: np.ndarray   # (8,)
    dq: np.ndarray     # (8,) conserved eigenvector (lab frame)
    dB: np.ndarray     # (3,) field part of dq
    B0: np.ndarray
    amp: float
    speed: float       # phase speed along k
    period: float

    def exact(self, shape, dx, t):
        (xc, yc, zc), (xf, yf, zf) = coords(shape, dx)
        Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
        ph = self.kvec[0] * X + self.kvec[1] * Y + self.kvec[2] * Z - self.omega * t
        return self.qbar[:, None, None, None] + self.amp * self.dq[:, None, None, None] * np.cos(ph)[None]


def frame_basis(khat):
    """Right-handed basis (khat, e1, e2) with e1 perpendicular to khat."""
    khat = np.asarray(khat, float) / np.linalg.norm(khat)
    trial = np.array([0.0, 0.0, 1.0]) if abs(khat[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    e1 = np.cross(trial, khat)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(khat, e1)
    return khat, e1, e2


def fast_wave_diagonal(N, amp=1e-6, gamma=GAMMA, wave="fast"):
    """Linear MHD wave along (1,1,1) on the unit periodic cube with N^3 zones.

    Background rho = 1, P = 3/5, v = 0, wave-frame field (B_par, B_t1, B_t2) =
    (1, sqrt2, 1/2) with e1 = (-1,1,0)/sqrt2, e2 = khat x e1.  Then a = 1,
    c_a = 1, and the fast / slow speeds are 2 and 1/2.  The eigenvector is
    taken from numpy.linalg.eig of the primitive quasi-linear matrix and
    normalised to d(rho) = 1.  Returns (q, b, wave) with q zone-centred point
    values (zone field = face average) and b = B0 + curl of the edge potential.
    """
    khat = np.array([1.0, 1.0, 1.0]) / math.sqrt(3.0)
    e1 = np.array([-1.0, 1.0, 0.0]) / math.sqrt(2.0)
    e2 = np.cross(khat, e1)
    rho0, p0 = 1.0, 0.6
    bpar, bt1, bt2 = 1.0, math.sqrt(2.0), 0.5
    B0 = bpar * khat + bt1 * e1 + bt2 * e2
    A = _primitive_matrix(rho0, 0.0, bpar, bt1, bt2, p0, gamma)
    w, V = np.linalg.eig(A)
    w = w.real
    V = V.real
    order = np.argsort(w)
    pick = {"fast": order[6], "alfven": order[5], "slow": order[4], "entropy": None}[wave]
    if pick is None:  # entropy mode: pure density
        vec = np.array([1.0, 0, 0, 0, 0, 0, 0])
        speed = 0.0
    else:
        vec = V[:, pick]
        speed = w[pick]
        if wave == "alfven":
            vec = vec / np.linalg.norm(vec[2:4])
        else:
            vec = vec / vec[0]
    drho, dv_f, dB_f, dp = vec[0], vec[1:4], vec[4:6], vec[6]
    dv = dv_f[0] * khat + dv_f[1] * e1 + dv_f[2] * e2
    dB = dB_f[0] * e1 + dB_f[1] * e2
    qbar = np.zeros(8)
    qbar[0] = rho0
    qbar[4:7] = B0
    qbar[7] = p0 / (gamma - 1.0) + 0.5 * float(B0 @ B0)
    dq = np.zeros(8)
    dq[0] = drho
    dq[1:4] = rho0 * dv
    dq[4:7] = dB
    dq[7] = dp / (gamma - 1.0) + float(B0 @ dB)
    k = 2.0 * math.pi * np.array([1.0, 1.0, 1.0])
    kmag = float(np.linalg.norm(k))
    omega = kmag * speed
    period = (2.0 * math.pi / abs(omega)) if speed != 0.0 else float("inf")
    wv = LinearWave(kvec=k, omega=omega, qbar=qbar, dq=dq, dB=dB, B0=B0, amp=amp, speed=speed, period=period)

    shape = (N, N, N)
    dx = (1.0 / N,) * 3
    (xc, yc, zc), (xf, yf, zf) = coords(shape, dx)
    # edge potential of the perturbation: A = amp (dB x k)/|k|^2 sin(k.x)
    avec = amp * np.cross(dB, k) / kmag ** 2
    Zf, Yf, Xc = np.meshgrid(zf, yf, xc, indexing="ij")
    Ax = avec[0] * np.sin(k[0] * Xc + k[1] * Yf + k[2] * Zf)
    Zf, Yc, Xf = np.meshgrid(zf, yc, xf, indexing="ij")
    Ay = avec[1] * np.sin(k[0] * Xf + k[1] * Yc + k[2] * Zf)
    Zc, Yf, Xf = np.meshgrid(zc, yf, xf, indexing="ij")
    Az = avec[2] * np.sin(k[0] * Xf + k[1] * Yf + k[2] * Zc)
    b = curl_of_edge_potential(Ax, Ay, Az, dx) + uniform_faces(shape, B0)
    Bcc = face_average(b)
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    c = amp * np.cos(k[0] * X + k[1] * Y + k[2] * Z)
    rho = rho0 + drho * c
    v = [dv[a] * c for a in range(3)]
    p = p0 + dp * c
    q = conserved(rho, v, Bcc, p, gamma)
    return q, b, wv


# --------------------------------------------------------------------------
# circularly polarised Alfven wave (exact nonlinear solution)
# --------------------------------------------------------------------------

def cp_alfven(N, khat=(1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0), box=(3.0, 1.5, 1.5), gamma=GAMMA, amp=0.1):
    """Circularly polarised Alfven wave on a (2N, N, N) grid over box (3, 3/2, 3/2),
    wavelength 1 along khat = (1/3, 2/3, 2/3): rho = 1, P = 0.1, B_par = 1,
    v_par = 0, B_t1 = amp sin(2 pi x_par), B_t2 = amp cos(2 pi x_par), v_t = B_t.
    The wave moves toward -khat at speed 1 (period 1).  Returns (q, b, exact_fn, dx)."""
    shape = (N, N, 2 * N)
    dx = (box[0] / (2 * N), box[1] / N, box[2] / N)
    kh, e1, e2 = frame_basis(khat)
    (xc, yc, zc), (xf, yf, zf) = coords(shape, dx)
    twopi = 2.0 * math.pi

    def phase(X, Y, Z, t=0.0):
        return twopi * (kh[0] * X + kh[1] * Y + kh[2] * Z + t)

    # potential of the transverse part: A = amp/(2 pi) (sin phi e1 + cos phi e2)
    def Avec(X, Y, Z):
        ph = phase(X, Y, Z)
        return amp / twopi * (np.sin(ph)[None] * e1[:, None, None, None] + np.cos(ph)[None] * e2[:, None, None, None])

    Zf, Yf, Xc = np.meshgrid(zf, yf, xc, indexing="ij")
    Ax = Avec(Xc, Yf, Zf)[0]
    Zf, Yc, Xf = np.meshgrid(zf, yc, xf, indexing="ij")
    Ay = Avec(Xf, Yc, Zf)[1]
    Zc, Yf, Xf = np.meshgrid(zc, yf, xf, indexing="ij")
    Az = Avec(Xf, Yf, Zc)[2]
    b = curl_of_edge_potential(Ax, Ay, Az, dx) + uniform_faces(shape, kh * 1.0)
    Bcc = face_average(b)

    def state(t):
        Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
        ph = phase(X, Y, Z, t)
        bt = amp * (np.sin(ph)[None] * e1[:, None, None, None] + np.cos(ph)[None] * e2[:, None, None, None])
        return bt

    bt0 = state(0.0)
    v = [bt0[a] for a in range(3)]
    q = conserved(np.ones(shape), v, Bcc, 0.1, gamma)

    def exact(t):
        bt = state(t)
        Bex = np.stack([kh[a] + bt[a] for a in range(3)])
        return conserved(np.ones(shape), [bt[a] for a in range(3)], Bex, 0.1, gamma)

    return q, b, exact, dx


# --------------------------------------------------------------------------
# spectral random fields
# --------------------------------------------------------------------------

def gaussian_field(shape, seed, ncomp=3, slope=-11.0 / 6.0, box=None, solenoidal=False, rng=None, workers=None):
    """Gaussian random field with |k|^slope amplitude for 1 <= |k| <= N/2 (k in
    units of 2 pi / L per axis), zero mean.  Returns (ncomp,) + shape.
    workers: threads for the FFTs (scipy.fft), for the largest boxes; None
    keeps numpy's FFT."""
    rng = np.random.default_rng(seed) if rng is None else rng
    Nz, Ny, Nx = shape
    box = box or (1.0, 1.0, 1.0)
    noise = rng.standard_normal((ncomp,) + shape)
    if workers is None:
        rfftn, irfftn = np.fft.rfftn, np.fft.irfftn
    else:
        import scipy.fft as sf

        rfftn = lambda a, axes: sf.rfftn(a, axes=axes, workers=workers)  # noqa: E731
        irfftn = lambda a, s, axes: sf.irfftn(a, s=s, axes=axes, workers=workers)  # noqa: E731
    fk = rfftn(noise, axes=(1, 2, 3))
    del noise
    kz = np.fft.fftfreq(Nz, d=1.0 / Nz)
    ky = np.fft.fftfreq(Ny, d=1.0 / Ny)
    kx = np.fft.rfftfreq(Nx, d=1.0 / Nx)
    # physical wavenumber in units of 2 pi / (unit length): integer index / L
    KZ, KY, KX = np.meshgrid(kz / box[2], ky / box[1], kx / box[0], indexing="ij")
    kmag = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    kmax = min(Nx / box[0], Ny / box[1], Nz / box[2]) / 2.0
    kmin = 1.0 / max(box)
    filt = np.where((kmag >= kmin) & (kmag <= kmax), np.power(np.maximum(kmag, 1e-30), slope), 0.0)
    fk *= filt[None]
    if solenoidal and ncomp == 3:
        k2 = np.maximum(kmag ** 2, 1e-30)
        kdot = KX * fk[0] + KY * fk[1] + KZ * fk[2]
        fk[0] -= KX * kdot / k2
        fk[1] -= KY * kdot / k2
        fk[2] -= KZ * kdot / k2
    f = irfftn(fk, s=shape, axes=(1, 2, 3))
    f -= f.mean(axis=(1, 2, 3), keepdims=True)
    return f


def turbulence(N, seed=170107452, mach=1.0, rho0=1.0, p0=1.0, B0=(0.1, 0.0, 0.0), gamma=GAMMA, shape=None, box=None):
    """Turbulence-like state: uniform rho, P, B; Gaussian random velocity with a
    k^-5/3 energy spectrum scaled to rms Mach `mach` (not projected)."""
    shape = shape or (N, N, N)
    v = gaussian_field(shape, seed, 3, box=box)
    cs = math.sqrt(gamma * p0 / rho0)
    vrms = math.sqrt(float(np.mean(np.sum(v ** 2, axis=0))))
    v *= mach * cs / vrms
    b = uniform_faces(shape, B0)
    q = conserved(np.full(shape, rho0), [v[0], v[1], v[2]], face_average(b), p0, gamma)
    return q, b


def high_contrast_turbulence(N, seed_rho=170107455, seed_v=170107456, sigma_ln=1.5, mach=5.0, gamma=GAMMA,
                             workers=None, log=None):
    """Lognormal density (sigma_ln), P = 1, B = (sqrt2, 0, 0) (beta 1), solenoidal
    velocity at rms Mach `mach` of the c_s = sqrt(gamma).  workers: FFT threads
    (see gaussian_field); log: optional callable told when each field is done."""
    shape = (N, N, N)
    lr = gaussian_field(shape, seed_rho, 1, workers=workers)[0]
    if log:
        log("log density field done")
    lr *= sigma_ln / lr.std()
    rho = np.exp(lr)
    rho /= rho.mean()
    v = gaussian_field(shape, seed_v, 3, solenoidal=True, workers=workers)
    if log:
        log("velocity field done")
    cs = math.sqrt(gamma)
    v *= mach * cs / math.sqrt(float(np.mean(np.sum(v ** 2, axis=0))))
    b = uniform_faces(shape, (math.sqrt(2.0), 0.0, 0.0))
    q = conserved(rho, [v[0], v[1], v[2]], face_average(b), 1.0, gamma)
    return q, b


def orszag_tang_3d(N, gamma=GAMMA):
    """Orszag-Tang vortex extended in z on the unit cube: v = (-sin 2pi y,
    sin 2pi x, 0.1 sin 2pi z), rho = 25/(36 pi), P = 5/(12 pi), field from the
    edge potential A_z = (4 pi)^-1/2 [cos(2 pi y)/(2 pi) + cos(4 pi x)/(4 pi)]."""
    shape = (N, N, N)
    dx = (1.0 / N,) * 3
    (xc, yc, zc), (xf, yf, zf) = coords(shape, dx)
    B0 = 1.0 / math.sqrt(4.0 * math.pi)
    Zc, Yf, Xf = np.meshgrid(zc, yf, xf, indexing="ij")
    Az = B0 * (np.cos(2 * math.pi * Yf) / (2 * math.pi) + np.cos(4 * math.pi * Xf) / (4 * math.pi))
    zero = np.zeros(shape)
    b = curl_of_edge_potential(zero, zero, Az, dx)
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    v = [-np.sin(2 * math.pi * Y), np.sin(2 * math.pi * X), 0.1 * np.sin(2 * math.pi * Z)]
    q = conserved(np.full(shape, 25.0 / (36.0 * math.pi)), v, face_average(b), 5.0 / (12.0 * math.pi), gamma)
    return q, b


def orszag_tang_2d(N, nz=5, gamma=GAMMA):
    """The planar Orszag-Tang vortex (Sect. 6) on the unit square, as a box
    N x N x nz with zones of 1/N (periodic; every z-plane the same):
    v = (-sin 2pi y, sin 2pi x, 0), rho = 25/(36 pi), P = 5/(12 pi), field
    from the edge potential A_z = (4 pi)^-1/2 [cos(2 pi y)/(2 pi) + cos(4 pi x)/(4 pi)]."""
    shape = (nz, N, N)
    dx = (1.0 / N,) * 3
    (xc, yc, zc), (xf, yf, zf) = coords(shape, dx)
    B0 = 1.0 / math.sqrt(4.0 * math.pi)
    Zc, Yf, Xf = np.meshgrid(zc, yf, xf, indexing="ij")
    Az = B0 * (np.cos(2 * math.pi * Yf) / (2 * math.pi) + np.cos(4 * math.pi * Xf) / (4 * math.pi))
    zero = np.zeros(shape)
    b = curl_of_edge_potential(zero, zero, Az, dx)
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    v = [-np.sin(2 * math.pi * Y), np.sin(2 * math.pi * X), zero]
    q = conserved(np.full(shape, 25.0 / (36.0 * math.pi)), v, face_average(b), 5.0 / (12.0 * math.pi), gamma)
    return q, b


def random_smooth(shape, seed, dx=None, amp=0.1, nmodes=3, gamma=GAMMA, B0=(0.7, -0.4, 0.5)):
    """Smooth random state on a periodic box: a few low Fourier modes of random
    amplitude in rho, v, P and in an edge vector potential (so div b = 0)."""
    rng = np.random.default_rng(seed)
    Nz, Ny, Nx = shape
    dx = dx or (1.0 / Nx, 1.0 / Ny, 1.0 / Nz)
    L = (Nx * dx[0], Ny * dx[1], Nz * dx[2])
    (xc, yc, zc), (xf, yf, zf) = coords(shape, dx)

    def field(Xs, Ys, Zs):
        out = np.zeros(np.broadcast_shapes(Xs.shape, Ys.shape, Zs.shape))
        for _ in range(nmodes):
            kk = rng.integers(-2, 3, size=3)
            ph = rng.uniform(0, 2 * math.pi)
            a = rng.uniform(-1, 1)
            out = out + a * np.cos(2 * math.pi * (kk[0] * Xs / L[0] + kk[1] * Ys / L[1] + kk[2] * Zs / L[2]) + ph)
        return out

    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    rho = 1.0 + 0.5 * amp * field(X, Y, Z)
    p = 1.0 + 0.5 * amp * field(X, Y, Z)
    v = [amp * field(X, Y, Z) for _ in range(3)]
    Zf, Yf, Xc = np.meshgrid(zf, yf, xc, indexing="ij")
    Ax = amp * 0.05 * field(Xc, Yf, Zf)
    Zf, Yc, Xf = np.meshgrid(zf, yc, xf, indexing="ij")
    Ay = amp * 0.05 * field(Xf, Yc, Zf)
    Zc, Yf, Xf = np.meshgrid(zc, yf, xf, indexing="ij")
    Az = amp * 0.05 * field(Xf, Yf, Zc)
    b = curl_of_edge_potential(Ax, Ay, Az, dx) + uniform_faces(shape, B0)
    q = conserved(rho, v, face_average(b), p, gamma)
    return q, b


def shock_tube_x(shape, gamma=2.0, left=(1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 1.0),
                 right=(0.125, 0.0, 0.0, 0.0, -1.0, 0.0, 0.1), bx=0.75):
    """Periodic double shock tube varying only along x: (rho, vx, vy, vz, By, Bz, P)
    = left on the middle half, right elsewhere; uniform B_x (Brio-Wu states)."""
    Nz, Ny, Nx = shape
    i = np.arange(Nx)
    mid = (i >= Nx // 4) & (i < 3 * Nx // 4)
    prim = np.where(mid[None, :], np.array(left)[:, None], np.array(right)[:, None])
    full = np.broadcast_to(prim[:, None, None, :], (7,) + shape)
    b = np.stack([np.full(shape, bx), np.array(full[4]), np.array(full[5])])
    Bcc = face_average(b)
    q = conserved(full[0], [full[1], full[2], full[3]], Bcc, full[6], gamma)
    return q, np.ascontiguousarray(b)


def field_loop(shape, dx, v=(2.0, 1.0, 1.0), amp=1e-3, R0=0.3, gamma=GAMMA):
    """Weak field loop (A_z = amp max(R0 - r, 0) about the box centre in x-y),
    rho = 1, P = 1, uniform velocity v (v_z != 0 exercises the source term)."""
    Nz, Ny, Nx = shape
    L = (Nx * dx[0], Ny * dx[1], Nz * dx[2])
    (xc, yc, zc), (xf, yf, zf) = coords(shape, dx, origin=(-L[0] / 2, -L[1] / 2, -L[2] / 2))
    Zc, Yf, Xf = np.meshgrid(zc, yf, xf, indexing="ij")
    Az = amp * np.maximum(R0 - np.sqrt(Xf ** 2 + Yf ** 2), 0.0)
    zero = np.zeros(shape)
    b = curl_of_edge_potential(zero, zero, Az, dx)
    vv = [np.full(shape, float(v[a])) for a in range(3)]
    q = conserved(np.ones(shape), vv, face_average(b), 1.0, gamma)
    return q, b
