"""The paper's validation problems (Sect. 6: RJ95 2a and 4a, Brio & Wu, the
3D magnetised blast) run by the oracle as regression tests.  The paper shows
figures only, so the checks are properties any correct solution has:
positivity, the untouched states beyond the fastest waves, exact
conservation (through the boundary fluxes where the domain has outflow
ends), div b at round-off.  Symmetry is pinned on smooth states: the update
commutes with a cyclic relabelling of the axes and with point inversion to
round-off.  (On the centred blast itself the mirror images drift apart by
far more than round-off: where the exact solution has a zero, such as the
mass flux through the centre faces, rounding picks the branch of the
upwind and limiter decisions.)
"""
import math

import numpy as np
import pytest

from oracle import phys_flux
from paper_1701_07452_amd import inputs as I
from tests._helpers import oracle_gather, oracle_sim


def _tube(left, right, bx, gamma, N, t_end, L=2.0, n_t=5, cfl=0.4):
    """Planar tube along x on [0, L] (discontinuity at L/2), N zones in 8
    patches, outflow at the x ends, periodic across; run to t_end (last step
    shortened).  L = 2 keeps every wave of the paper's setups (run on the unit
    interval there) away from the ends."""
    G = I.patch_grid([N // 8] * 8, [n_t], [n_t], periodic=(False, True, True))
    Nz, Ny, Nx = G.shape
    i = np.arange(Nx)
    lo = i < Nx // 2
    prim = np.where(lo[None, :], np.array(left)[:, None], np.array(right)[:, None])
    full = np.broadcast_to(prim[:, None, None, :], (7,) + G.shape)
    b = np.stack([np.full(G.shape, bx), np.array(full[4]), np.array(full[5])])
    q = I.conserved(full[0], [full[1], full[2], full[3]], I.face_average(b), full[6], gamma)
    dx = (L / Nx,) * 3
    sim = oracle_sim(G, q, b, dx=dx, gamma=gamma, cfl=cfl)
    tot0, _, _, _ = sim.diagnostics()
    t = 0.0
    while t < t_end - 1e-14:
        sim.fill_ghosts()
        dt = min(sim.compute_dt(), t_end - t)
        sim.advance(dt)
        t += dt
    tot1, dn, _, nfl = sim.diagnostics()
    qn, bn = oracle_gather(G, sim)
    sim.close()
    return q, qn, tot0, tot1, dn, nfl, dx


def _frame8(rho, v, by, bz, p, bx, gamma):
    return np.array([rho, rho * v[0], rho * v[1], rho * v[2], bx, by, bz,
                     p / (gamma - 1) + 0.5 * rho * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2) + 0.5 * (bx * bx + by * by + bz * bz)])


S4PI = math.sqrt(4 * math.pi)
TUBES = {
    # (left, right) as (rho, vx, vy, vz, By, Bz, P), B_x, gamma, t (Sect. 6)
    "RJ95_2a": ((1.08, 1.2, 0.01, 0.5, 3.6 / S4PI, 2 / S4PI, 0.95), (1.0, 0, 0, 0, 4 / S4PI, 2 / S4PI, 1.0),
                2 / S4PI, 5.0 / 3.0, 0.2),
    "RJ95_4a": ((1.0, 0, 0, 0, 1.0, 0, 1.0), (0.2, 0, 0, 0, 0, 0, 0.1), 1.0, 5.0 / 3.0, 0.15),
    "BrioWu": ((1.0, 0, 0, 0, 1.0, 0, 1.0), (0.125, 0, 0, 0, -1.0, 0, 0.1), 0.75, 2.0, 0.08),
}


@pytest.mark.parametrize("name", sorted(TUBES))
def test_shock_tube(name):
    left, right, bx, gamma, t_end = TUBES[name]
    N = 128
    q0, qn, tot0, tot1, dn, nfl, dx = _tube(left, right, bx, gamma, N, t_end)
    # positivity, no floor needed
    rho = qn[0]
    p = (gamma - 1) * (qn[7] - 0.5 * (qn[1] ** 2 + qn[2] ** 2 + qn[3] ** 2) / rho - 0.5 * (qn[4:7] ** 2).sum(0))
    assert rho.min() > 0 and p.min() > 0 and nfl == 0
    # the end states beyond the fast waves (|x - L/2| > 0.7) are untouched but
    # for the scheme's precursor, which decays by orders of magnitude a zone
    edge = np.r_[0:N // 8, N - N // 8:N]
    assert np.abs(qn[..., edge] - q0[..., edge]).max() <= 1e-6
    ends = np.r_[0:4, N - 4:N]
    assert np.abs(qn[..., ends] - q0[..., ends]).max() <= 1e-20
    # the totals change by exactly the boundary fluxes of the constant end states
    fl = phys_flux(_frame8(left[0], left[1:4], left[4], left[5], left[6], bx, gamma), gamma)
    fr = phys_flux(_frame8(right[0], right[1:4], right[4], right[5], right[6], bx, gamma), gamma)
    area = qn.shape[1] * qn.shape[2] * dx[1] * dx[2]
    # frame rows (rho, m_x, m_y, m_z, B_x, B_y, B_z, E) are the lab rows along x
    for c in range(8):
        expect = tot0[c] + (fl[c] - fr[c]) * t_end * area
        assert abs(tot1[c] - expect) <= 1e-12 * max(1.0, abs(tot0[c])), (name, c)
    # planar: every transverse line is the same
    assert np.array_equal(qn, np.broadcast_to(qn[:, :1, :1, :], qn.shape))
    assert dn < 1e-12


BLAST_GRID = ([7, 7, 7], [10, 11, 10], [7, 7, 7])  # 21 x 31 x 21 zones, 27 patches


def _blast(shape=(21, 31, 21)):
    """3D magnetised blast (Sect. 6): box (1, 3/2, 1), rho = 1,
    B = (10/sqrt2, 10/sqrt2, 0), P = 100 within r < 0.125 of the centre, 1
    elsewhere, periodic, gamma 5/3; coarse grid.  Odd zone counts put the
    centre on a zone centre, so that no face lies on a plane of symmetry
    (there the mass flux cancels to round-off and the corner-EMF upwinding
    would follow the rounding)."""
    Nz, Ny, Nx = shape
    dx = (1.0 / Nx, 1.5 / Ny, 1.0 / Nz)
    (xc, yc, zc), _ = I.coords(shape, dx, origin=(-0.5, -0.75, -0.5))
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    p = np.where(np.sqrt(X ** 2 + Y ** 2 + Z ** 2) < 0.125, 100.0, 1.0)
    b = I.uniform_faces(shape, (10 / math.sqrt(2), 10 / math.sqrt(2), 0.0))
    q = I.conserved(np.ones(shape), [np.zeros(shape)] * 3, I.face_average(b), p)
    return q, b, dx


def test_blast_conservation():
    q, b, dx = _blast()
    G = I.patch_grid(*BLAST_GRID)
    sim = oracle_sim(G, q, b, dx=dx)
    tot0, _, _, nf0 = sim.diagnostics()
    t = 0.0
    clean = 0
    while t < 0.02 - 1e-14:
        sim.fill_ghosts()
        dt = min(sim.compute_dt(), 0.02 - t)
        sim.advance(dt)
        t += dt
        tot1, dn, _, nfl = sim.diagnostics()
        # mass, momentum and field totals are exact in every step; total
        # energy is exact in every step in which no pressure floor fired
        for c in range(7):
            assert abs(tot1[c] - tot0[c]) <= 1e-12 * max(1.0, abs(tot0[c]))
        if nfl == nf0:
            assert abs(tot1[7] - tot0[7]) <= 1e-12 * abs(tot0[7])
            clean += 1
        tot0, nf0 = tot1, nfl
        assert dn < 1e-11
    qn, bn = oracle_gather(G, sim)
    sim.close()
    # at plasma beta 0.02 the 100:1 jump drives the floor in a few zones (14
    # of 13671 here, in two of the 20 steps)
    assert clean >= 15 and nfl <= 0.01 * 21 * 31 * 21
    # the blast expanded: the centre pressure dropped, the density has a shell
    assert qn[0].max() > 1.2 and qn[0].min() < 0.9
    assert (qn[0] > 0).all()


def _rotate(q, b):
    """Relabel the axes cyclically (new x = old y, new y = old z, new z = old x)."""
    T = lambda a: np.transpose(a, (2, 0, 1))
    return np.stack([T(q[i]) for i in (0, 2, 3, 1, 5, 6, 4, 7)]), np.stack([T(b[i]) for i in (1, 2, 0)])


def _invert(q, b):
    """Point inversion r -> -r of a periodic state: v odd, B (axial) even; the
    left face of a zone is the image of the right face of its mirror zone."""
    R = lambda a: a[::-1, ::-1, ::-1]
    q2 = np.stack([R(q[0])] + [-R(q[c]) for c in (1, 2, 3)] + [R(q[c]) for c in (4, 5, 6, 7)])
    b2 = np.stack([np.roll(R(b[a]), 1, axis=2 - a) for a in range(3)])
    return q2, b2


@pytest.mark.parametrize("sym", ["rotate", "invert"])
@pytest.mark.parametrize("B0", [(0.7, -0.4, 0.5), (0.0, 0.0, 0.0)])
def test_update_commutes_with_symmetry(sym, B0):
    """Three steps of a smooth random state (16^3 as 8 patches, fixed dt)
    commute with the symmetry to round-off: a dropped or mis-signed
    transverse term, or an axis-specific index slip, breaks this."""
    N = 16
    op = _rotate if sym == "rotate" else _invert
    q, b = I.random_smooth((N, N, N), 5, amp=0.5, B0=B0)
    G = I.uniform_grid(N, 8)

    def run(q, b):
        sim = oracle_sim(G, q, b, dx=(1.0 / N,) * 3)
        for _ in range(3):
            sim.fill_ghosts()
            sim.advance(0.005)
        out = oracle_gather(G, sim)
        sim.close()
        return out

    qa, ba = op(*run(q, b))
    qb, bb = run(*op(q, b))
    assert np.abs(qa - qb).max() <= 1e-14
    assert np.abs(ba - bb).max() <= 1e-14


def test_orszag_tang_2d_planar():
    """The planar Orszag-Tang vortex (Sect. 6) as a 64 x 64 x 5 box (16
    patches of 16 x 16 x 5, periodic), 10 steps: every z-plane stays the same
    bitwise (the 3D update of a z-invariant state is the 2D update); totals
    exact; div b at round-off; the same run as one 64 x 64 x 5 patch,
    bitwise.  v_z and B_z do not stay 0: where the transverse field of a face
    vanishes (B_y changes sign across the x-faces at x = 1/4, 3/4) the
    eigenvectors take the degenerate basis (1, 1)/sqrt2 in the transverse
    plane; the slow and Alfven families then carry the transverse jump with
    different entropy fixes and limiters, which moves some v_y into v_z (B_z
    reaches 1.2% of |B| after these 10 steps, linearly growing).  The planar
    (2.5D) form of the scheme does the same."""
    q, b = I.orszag_tang_2d(64)
    dx = (1.0 / 64,) * 3
    out = []
    for G in (I.patch_grid([16] * 4, [16] * 4, [5]), I.patch_grid([64], [64], [5])):
        sim = oracle_sim(G, q, b, dx=dx)
        tot0, _, _, _ = sim.diagnostics()
        for _ in range(10):
            sim.fill_ghosts()
            sim.advance(sim.compute_dt())
        tot1, dn, _, nfl = sim.diagnostics()
        out.append(oracle_gather(G, sim))
        sim.close()
        for c in range(8):
            assert abs(tot1[c] - tot0[c]) <= 1e-12 * max(1.0, abs(tot0[c]))
        assert dn < 1e-12 and nfl == 0
    (qa, ba), (qb, bb) = out
    assert np.array_equal(qa, qb) and np.array_equal(ba, bb)
    assert np.array_equal(qa, np.broadcast_to(qa[:, :1], qa.shape))
    assert np.array_equal(ba, np.broadcast_to(ba[:, :1], ba.shape))
    assert np.abs(qa[3]).max() <= 0.02 * np.abs(qa[1:3]).max()
    assert np.abs(qa[6]).max() <= 0.02 * np.abs(qa[4:6]).max()
    # the vortex evolved
    assert np.abs(qa[0] - q[0]).max() > 1e-3
