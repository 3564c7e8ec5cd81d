"""Pins of the oracle's floor arithmetic (Appendix A, final paragraph: density
and pressure floors applied when crossed).  Reading: a density below rho_floor
is raised to it with the momentum kept; then a pressure below p_floor (from
the equation of state of Sect. 5 with the raised density) is raised to it by
adding thermal energy.  Nothing else changes.

F1 checks the rule on single states through the equation of state; F2 checks
it inside a step on the periodic Einfeldt-type line (a strong rarefaction
where the plain update needs the floors, and a shock), where the floors fire
in a well-defined set of zones each step: the floored zones end exactly at
the floor, mass (with pressure floors only), momentum and the zone field are
conserved to round-off, and the totals change by exactly what the floors
report having added.
"""
import numpy as np
import pytest

from oracle import default_params, floor_state
from paper_1701_07452_amd import inputs as I
from tests._helpers import oracle_gather, oracle_sim


def pressure(u, gam):
    """Pressure of lab-ordered 8-states (component axis first), Sect. 5."""
    return (gam - 1) * (u[7] - 0.5 * (u[1] ** 2 + u[2] ** 2 + u[3] ** 2) / u[0] - 0.5 * (u[4] ** 2 + u[5] ** 2 + u[6] ** 2))


def test_F1_floor_rule_single_states():
    gam = 5 / 3
    rf, pf = 0.1, 0.05
    P = default_params(gamma=gam, rho_floor=rf, p_floor=pf)
    rng = np.random.default_rng(21)
    seen = {"rho": 0, "p": 0, "none": 0}
    for _ in range(400):
        rho = rng.choice([rng.uniform(0.01, 0.1), rng.uniform(0.1, 2.0)])
        v = rng.normal(size=3)
        B = rng.normal(size=3)
        p = rng.uniform(-0.2, 0.3)
        u = np.array([rho, *(rho * v), *B, p / (gam - 1) + 0.5 * rho * v @ v + 0.5 * B @ B])
        hit, w = floor_state(P, u)
        # momentum and zone field untouched, bitwise
        assert np.array_equal(w[1:7], u[1:7])
        assert w[0] == max(u[0], rf)
        u1 = u.copy()
        u1[0] = w[0]
        p1 = pressure(u1, gam)  # pressure after the density floor, energy unchanged
        scale = (gam - 1) * (abs(u[7]) + 0.5 * (u[1:4] @ u[1:4]) / w[0] + 0.5 * B @ B)
        if p1 < pf:
            assert abs(pressure(w, gam) - pf) <= 1e-14 * scale
            assert w[7] > u[7]
            seen["p"] += 1
        else:
            assert w[7] == u[7]
        assert hit == (u[0] < rf or p1 < pf)
        if u[0] < rf:
            seen["rho"] += 1
        if not hit:
            seen["none"] += 1
    assert min(seen.values()) > 30, seen


def _einfeldt(rho_floor, p_floor):
    G = I.patch_grid([32, 32], [8], [8])
    q, b = I.shock_tube_x(G.shape, gamma=1.4, left=(1.0, -3.0, 0.0, 0.0, 0.0, 0.0, 0.4),
                          right=(1.0, 3.0, 0.0, 0.0, 0.0, 0.0, 0.4), bx=0.1)
    return G, oracle_sim(G, q, b, dx=(1 / 64,) * 3, gamma=1.4, rho_floor=rho_floor, p_floor=p_floor)


@pytest.mark.parametrize("rho_floor", [1e-12, 0.3])
def test_F2_floors_in_the_step(rho_floor):
    gam, pf = 1.4, 1e-3
    G, sim = _einfeldt(rho_floor, pf)
    dV = (1 / 64) ** 3
    fired_rho = 0
    for step in range(5):
        tot0, _, _, n0 = sim.diagnostics()
        m0, e0 = sim.floor_added()
        qa, _ = oracle_gather(G, sim)
        sim.fill_ghosts()
        sim.advance(sim.compute_dt())
        tot, dn, _, n1 = sim.diagnostics()
        m1, e1 = sim.floor_added()
        q, _ = oracle_gather(G, sim)
        nfl = n1 - n0
        assert nfl > 0, step
        p = pressure(q, gam)
        scale = (gam - 1) * (np.abs(q[7]) + 0.5 * (q[1:4] ** 2).sum(0) / q[0] + 0.5 * (q[4:7] ** 2).sum(0))
        at_p = np.abs(p - pf) <= 1e-14 * scale
        at_rho = q[0] == rho_floor
        # no zone below a floor; the zones at a floor are the floored ones
        assert q[0].min() >= rho_floor and np.all(p >= pf - 1e-14 * scale)
        assert int((at_p | at_rho).sum()) == nfl, (step, int(at_p.sum()), int(at_rho.sum()), nfl)
        fired_rho += int(at_rho.sum())
        # momentum and zone field: flux form and untouched by floors
        big = np.abs(qa).sum(axis=(1, 2, 3)) * dV
        assert np.all(np.abs(tot[1:7] - tot0[1:7]) <= 1e-14 * big[1:7])
        # mass and energy change by exactly what the floors added
        assert abs((tot[0] - tot0[0]) - (m1 - m0)) <= 1e-14 * big[0]
        assert abs((tot[7] - tot0[7]) - (e1 - e0)) <= 1e-14 * big[7]
        assert e1 - e0 > 0
        assert dn < 1e-13
    if rho_floor > 1e-6:
        assert fired_rho > 0 and m1 > 0
    else:
        assert m1 == 0.0
    sim.close()
