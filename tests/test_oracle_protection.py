"""Pins of the oracle's protection path (Appendix A, last paragraph): the HLL
flux that replaces the MHDTVD flux at faces where a protection floor is
exceeded, and the trigger.

H1 HLL consistency u(q, q) = F(q); H2 supersonic upwinding (all waves one way:
the HLL flux is the upwind physical flux); H3 the strong-rarefaction line on
which the plain Roe-type update produces a negative pressure, stays positive
with protection floors, and uses the protection only where it is needed; H4
with the floors off the line fluxes are bitwise those of the plain scheme;
H5 a 3D periodic run with protection conserves the totals exactly and keeps
div b at round-off.
"""
import numpy as np
import pytest

from oracle import OracleSim, default_params, hll_flux, line_fluxes, phys_flux
from paper_1701_07452_amd import inputs as I


def state(rho, v, b, p, gam):
    v = np.asarray(v, float)
    b = np.asarray(b, float)
    return np.array([rho, rho * v[0], rho * v[1], rho * v[2], b[0], b[1], b[2],
                     p / (gam - 1) + 0.5 * rho * v @ v + 0.5 * b @ b])


def test_H1_hll_consistency():
    rng = np.random.default_rng(5)
    for _ in range(20):
        gam = 5.0 / 3.0
        u = state(rng.uniform(0.2, 3), rng.normal(size=3), rng.normal(size=3), rng.uniform(0.1, 2), gam)
        P = default_params(gamma=gam)
        f = hll_flux(u, u, P)
        ref = phys_flux(u, gam)
        assert np.abs(f - ref).max() <= 1e-14 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_H2_supersonic_upwind(sign):
    """Both states move faster than their fast speed in the same direction:
    b- = 0 (or b+ = 0) and the HLL flux is F of the upwind state exactly."""
    gam = 5.0 / 3.0
    P = default_params(gamma=gam)
    uL = state(1.0, [sign * 6.0, 0.3, -0.2], [0.5, 0.4, 0.1], 0.6, gam)
    uR = state(0.8, [sign * 5.5, -0.1, 0.2], [0.5, 0.2, -0.3], 0.5, gam)
    f = hll_flux(uL, uR, P)
    up = uL if sign > 0 else uR
    ref = phys_flux(up, gam)
    assert np.abs(f - ref).max() <= 1e-13 * np.abs(ref).max()


def _rarefaction_update(prot, vel=3.0, m=40, steps=3, bx=0.1):
    """Einfeldt-type 1-2-0-3 line (rho = 1, P = 0.4, v = -/+vel, gamma = 1.4)
    advanced with the line fluxes at CFL 0.4 (dx = 1, no floors); returns the
    minimum density and pressure over the updated zones after each step."""
    gam = 1.4
    P = default_params(gamma=gam, rho_floor=1e-12, p_floor=1e-12, rho_protect=prot, p_protect=prot)
    q = np.array([state(1.0, [-vel if s < m // 2 else vel, 0, 0], [bx, 0, 0], 0.4, gam) for s in range(m)])
    bf = np.full(m, bx)
    out = []
    for _ in range(steps):
        rho = q[:, 0]
        v = q[:, 1] / rho
        b2 = (q[:, 4:7] ** 2).sum(1)
        p = (gam - 1) * (q[:, 7] - 0.5 * rho * v * v - 0.5 * b2)
        if not np.all(p > 0):
            out.append((np.nan, np.nan))
            break
        dt = 0.4 / np.max(np.abs(v) + np.sqrt((gam * p + b2) / rho))
        F = line_fluxes(P, q, bf, dt)
        qn = q.copy()
        qn[2:m - 2] = q[2:m - 2] - dt * (F[3:m - 1] - F[2:m - 2])
        q = qn
        r = q[2:m - 2, 0]
        vv = q[2:m - 2, 1] / r
        pp = (gam - 1) * (q[2:m - 2, 7] - 0.5 * r * vv * vv - 0.5 * (q[2:m - 2, 4:7] ** 2).sum(1))
        out.append((r.min(), pp.min()))
    return out, q


def test_H3_strong_rarefaction_positivity():
    plain, _ = _rarefaction_update(0.0, steps=1)
    assert plain[0][1] < 0.0, "the plain update must fail here for the pin to mean anything"
    prot, _ = _rarefaction_update(1e-3, steps=3)
    for r, p in prot:
        assert r > 0.0 and p > 0.0
    # far from the rarefaction the protected and plain lines agree bitwise
    _, qa = _rarefaction_update(0.0, steps=1)
    _, qb = _rarefaction_update(1e-3, steps=1)
    assert np.array_equal(qa[:10], qb[:10]) and np.array_equal(qa[-10:], qb[-10:])
    assert not np.array_equal(qa, qb)


def test_H4_floors_off_is_plain():
    rng = np.random.default_rng(9)
    gam = 5.0 / 3.0
    m = 24
    q = np.array([state(rng.uniform(0.5, 2), rng.normal(size=3) * 0.5, rng.normal(size=3), rng.uniform(0.3, 2), gam)
                  for _ in range(m)])
    bf = q[:, 4].copy()
    a = line_fluxes(default_params(gamma=gam), q, bf, 0.05)
    b = line_fluxes(default_params(gamma=gam, rho_protect=0.0, p_protect=0.0), q, bf, 0.05)
    assert np.array_equal(np.nan_to_num(a, nan=7.0), np.nan_to_num(b, nan=7.0))
    # on smooth data (small jumps) floors well below every state change nothing
    x = np.arange(m) / m
    qs = np.array([state(1 + 0.1 * np.sin(2 * np.pi * t), [0.1 * np.cos(2 * np.pi * t), 0.05, 0], [0.7, 0.4, -0.2],
                         1.0 + 0.05 * np.sin(4 * np.pi * t), gam) for t in x])
    bs = qs[:, 4].copy()
    a = line_fluxes(default_params(gamma=gam), qs, bs, 0.05)
    c = line_fluxes(default_params(gamma=gam, rho_protect=1e-3, p_protect=1e-3), qs, bs, 0.05)
    assert np.array_equal(np.nan_to_num(a, nan=7.0), np.nan_to_num(c, nan=7.0))


def test_H5_protected_3d_conservation_and_divb():
    q, b = I.high_contrast_turbulence(16)
    G = I.uniform_grid(16, 8)
    P = default_params(dx=(1 / 16,) * 3, rho_floor=1e-8, p_floor=1e-8, rho_protect=0.05, p_protect=0.05)
    sim = OracleSim(P, G.descs)
    for ip, (qp, bp) in enumerate(I.split(G, q, b)):
        sim.set_state(ip, qp, bp)
    t0, _, _, _ = sim.diagnostics()
    sim.run_steps(3)
    t1, dn, _, nfl = sim.diagnostics()
    for c in (0, 1, 2, 3, 4, 5, 6):
        assert abs(t1[c] - t0[c]) <= 1e-12 * max(1.0, abs(t0[c]))
    assert dn < 1e-11
    # the protection acted: the plain run differs
    plain = OracleSim(default_params(dx=(1 / 16,) * 3, rho_floor=1e-8, p_floor=1e-8), G.descs)
    for ip, (qp, bp) in enumerate(I.split(G, q, b)):
        plain.set_state(ip, qp, bp)
    plain.run_steps(3)
    assert not np.array_equal(sim.get_state(0)[0], plain.get_state(0)[0])
    sim.close()
    plain.close()
