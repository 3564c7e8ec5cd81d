"""Pins of the oracle's 1D building blocks: flux, Roe eigensystem, MHDTVD flux.

P1 Roe property, P2 eigen-relation with a finite-difference Jacobian of the
flux printed in Sect. 5, P3 consistency, P4 Lax-Wendroff closed form in smooth
single-wave data, P12 closed-form speeds of the paper's printed setups.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import default_params, eigensystem, line_fluxes, phys_flux

C7 = [0, 1, 2, 3, 5, 6, 7]
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_setups.json")))


def flux_from_paper(u, gam):
    """Flux vector of the 1D conservative form as printed in Sect. 5 (retyped here
    independently of the oracle; used only to build a finite-difference Jacobian)."""
    rho, mx, my, mz, bx, by, bz, e = u
    vx, vy, vz = mx / rho, my / rho, mz / rho
    b2 = bx * bx + by * by + bz * bz
    p = (gam - 1) * (e - 0.5 * rho * (vx * vx + vy * vy + vz * vz) - 0.5 * b2)
    ps = p + 0.5 * b2
    return np.array([rho * vx, rho * vx * vx + ps - bx * bx, rho * vx * vy - bx * by, rho * vx * vz - bx * bz,
                     0.0, by * vx - bx * vy, bz * vx - bx * vz, (e + ps) * vx - bx * (bx * vx + by * vy + bz * vz)])


def state(rho, v, b, p, gam):
    v = np.asarray(v, float)
    b = np.asarray(b, float)
    return np.array([rho, rho * v[0], rho * v[1], rho * v[2], b[0], b[1], b[2],
                     p / (gam - 1) + 0.5 * rho * v @ v + 0.5 * b @ b])


def random_pair(rng, gam, kind="generic"):
    bx = rng.normal()
    def one():
        rho = rng.uniform(0.2, 3.0)
        v = rng.normal(size=3)
        bt = rng.normal(size=2)
        if kind == "bt0":
            bt = bt * 1e-9
        if kind == "bx0":
            pass
        return rho, v, bt, rng.uniform(0.05, 3.0)
    if kind == "bx0":
        bx = 0.0
    L, R = one(), one()
    uL = state(L[0], L[1], [bx, *L[2]], L[3], gam)
    uR = state(R[0], R[1], [bx, *R[2]], R[3], gam)
    return uL, uR


@pytest.mark.parametrize("kind", ["generic", "bt0", "bx0"])
def test_P1_roe_property(kind):
    """sum_k a_k alpha_k R_k = F(uR) - F(uL) for random pairs, incl. near-degenerate."""
    P = default_params()
    rng = np.random.default_rng(11)
    worst = 0.0
    for _ in range(300):
        uL, uR = random_pair(rng, P.gamma, kind)
        lam, R, L = eigensystem(uL, uR, P)
        alpha = L @ (uR - uL)[C7]
        dF = (phys_flux(uR, P.gamma) - phys_flux(uL, P.gamma))[C7]
        err = np.abs(R @ (lam * alpha) - dF).max() / max(np.abs(dF).max(), 1e-300)
        worst = max(worst, err)
    assert worst < 1e-12, worst


def test_P1_flux_matches_printed_vector():
    rng = np.random.default_rng(3)
    for _ in range(50):
        u = state(rng.uniform(0.3, 2), rng.normal(size=3), rng.normal(size=3), rng.uniform(0.1, 2), 5 / 3)
        assert np.allclose(phys_flux(u, 5 / 3), flux_from_paper(u, 5 / 3), rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("kind", ["generic", "bt0", "bx0"])
def test_P2_left_right_inverse_and_jacobian(kind):
    """L R = I; at uL = uR the eigenpairs satisfy A R_k = a_k R_k with A the
    finite-difference Jacobian of the printed flux; speeds match Sect. 5."""
    P = default_params()
    gam = P.gamma
    rng = np.random.default_rng(5)
    for _ in range(40):
        uL, _ = random_pair(rng, gam, kind)
        lam, R, L = eigensystem(uL, uL, P)
        assert np.abs(L @ R - np.eye(7)).max() < 1e-12
        # Jacobian over the 7 components (B_par fixed), central differences
        A = np.zeros((7, 7))
        for c in range(7):
            h = 1e-6 * max(1.0, abs(uL[C7[c]]))
            up = uL.copy(); up[C7[c]] += h
            um = uL.copy(); um[C7[c]] -= h
            A[:, c] = (flux_from_paper(up, gam) - flux_from_paper(um, gam))[C7] / (2 * h)
        scale = np.abs(A).max()
        for k in range(7):
            res = A @ R[:, k] - lam[k] * R[:, k]
            assert np.abs(res).max() < 1e-7 * scale * max(1.0, np.abs(R[:, k]).max()), (k, res)
        # eigenvalues against the printed speed formulas
        rho = uL[0]; vx = uL[1] / rho
        b2 = uL[4] ** 2 + uL[5] ** 2 + uL[6] ** 2
        p = (gam - 1) * (uL[7] - 0.5 * (uL[1] ** 2 + uL[2] ** 2 + uL[3] ** 2) / rho - 0.5 * b2)
        a2 = gam * p / rho
        disc = math.sqrt(max((a2 + b2 / rho) ** 2 - 4 * a2 * uL[4] ** 2 / rho, 0.0))
        cf = math.sqrt(0.5 * (a2 + b2 / rho + disc))
        cs = math.sqrt(max(0.5 * (a2 + b2 / rho - disc), 0.0))
        ca = abs(uL[4]) / math.sqrt(rho)
        want = [vx - cf, vx - ca, vx - cs, vx, vx + cs, vx + ca, vx + cf]
        assert np.allclose(lam, want, rtol=1e-10, atol=1e-7 * cf)


def test_P3_consistency_exact():
    """MHDTVD flux of a constant line equals the physical flux, bitwise."""
    P = default_params()
    rng = np.random.default_rng(7)
    for _ in range(20):
        u = state(rng.uniform(0.3, 2), rng.normal(size=3), rng.normal(size=3), rng.uniform(0.1, 2), P.gamma)
        q8 = np.tile(u, (12, 1))
        bf = np.full(12, u[4])
        F = line_fluxes(P, q8, bf, 0.3)
        # the flux uses the state rebuilt from its primitives; compare with the
        # flux of that rebuilt state
        rho, v = u[0], u[1:4] / u[0]
        p = (P.gamma - 1) * (u[7] - 0.5 * rho * v @ v - 0.5 * u[4:7] @ u[4:7])
        ref = phys_flux(state(rho, v, u[4:7], p, P.gamma), P.gamma)
        for s in range(2, 11):
            assert np.array_equal(F[s], ref)
        assert np.isnan(F[0]).all() and np.isnan(F[1]).all() and np.isnan(F[11]).all()


@pytest.mark.parametrize("eps", [0.0, 0.1, 0.45])
def test_P4_lax_wendroff_single_wave(eps):
    """Entropy wave with B = 0 and density linear in x: only the entropy wave is
    excited with a uniform alpha, the limiter is inactive, and the modified flux
    equals 1/2 (F_L + F_R) - (lam a^2 / 2) dq with a = v_x (textbook LW)."""
    gam = 5 / 3
    P = default_params(eps=(eps,) * 7)
    m = 16
    v0, p0, lam = 0.7, 1.0, 0.45
    q8 = np.array([state(1.0 + 0.01 * s, [v0, 0, 0], [0, 0, 0], p0, gam) for s in range(m)])
    F = line_fluxes(P, q8, np.zeros(m), lam)
    for s in range(2, m - 1):
        uL, uR = q8[s - 1], q8[s]
        lw = 0.5 * (phys_flux(uL, gam) + phys_flux(uR, gam)) - 0.5 * lam * v0 ** 2 * (uR - uL)
        lw[4] = 0.0
        assert np.allclose(F[s], lw, rtol=1e-13, atol=1e-15), (s, F[s] - lw)


def test_first_order_upwind_when_limited():
    """With the limiter switched off by a sign change at every face (alternating
    g-tilde), g = 0 and the flux is the Roe upwind flux 1/2(F_L+F_R) - 1/2 |A| dq."""
    gam = 5 / 3
    P = default_params(eps=(0.0,) * 7)
    m = 16
    v0, lam = 0.7, 0.45
    q8 = np.array([state(1.0 + (0.1 if s % 2 else 0.0), [v0, 0, 0], [0, 0, 0], 1.0, gam) for s in range(m)])
    F = line_fluxes(P, q8, np.zeros(m), lam)
    for s in range(2, m - 1):
        uL, uR = q8[s - 1], q8[s]
        up = 0.5 * (phys_flux(uL, gam) + phys_flux(uR, gam)) - 0.5 * abs(v0) * (uR - uL)
        up[4] = 0.0
        assert np.allclose(F[s], up, rtol=1e-13, atol=1e-15)


def test_P12_printed_setup_speeds():
    """Sect. 6.1 MHD background: c_f = 2, c_a = 1, c_s = 1/2 exactly (a = 1)."""
    g = GOLD["linear_wave_mhd_background"]
    P = default_params(gamma=g["gamma"])
    u = state(g["rho"], [0, 0, 0], g["B"], g["P"], g["gamma"])
    lam, _, _ = eigensystem(u, u, P)
    d = g["derived_from_printed_speed_formulas"]
    want = [-d["c_f"], -d["c_a"], -d["c_s"], 0.0, d["c_s"], d["c_a"], d["c_f"]]
    assert np.allclose(lam, want, rtol=0, atol=1e-14)
    ot = GOLD["orszag_tang"]
    P2 = default_params(gamma=ot["gamma"])
    u = state(ot["rho"], [0, 0, 0], [0, 0, 0], ot["P"], ot["gamma"])
    lam, _, _ = eigensystem(u, u, P2)
    assert abs(lam[6] - ot["sound_speed"]) < 1e-14


def test_brio_wu_line_is_finite_and_conservative():
    """A single steep jump (Sect. 6.4 states) gives finite fluxes; a periodic 1D
    update with them conserves the line totals to roundoff."""
    gd = GOLD["brio_wu"]
    gam = gd["gamma"]
    P = default_params(gamma=gam)
    N, g = 64, 5
    q = np.array([state(*(lambda w: (w[0], w[1:4], [gd["Bx"], w[4], w[5]], w[6]))(gd["left"] if N // 4 <= i < 3 * N // 4 else gd["right"]), gam) for i in range(N)])
    tot0 = q.sum(0)
    dx = 1.0 / N
    for _ in range(30):
        qq = np.concatenate([q[-g:], q, q[:g]])
        F = line_fluxes(P, qq, np.full(N + 2 * g, gd["Bx"]), 0.2)
        assert np.isfinite(F[g:g + N + 1]).all()
        q = q - 0.2 * (F[g + 1:g + N + 1] - F[g:g + N])
    assert np.allclose(q.sum(0), tot0, rtol=1e-13, atol=1e-12)


def _entropy_line(rho, v0, gam, p0=1.0):
    """Frame 8-states of a line carrying only an entropy wave: density varies,
    velocity (v0 along the line), pressure and B = 0 are uniform."""
    return np.array([state(r, [v0, 0, 0], [0, 0, 0], p0, gam) for r in rho])


@pytest.mark.parametrize("eps,v0,lam", [(0.3, 0.7, 0.45), (0.3, -0.7, 0.45), (0.45, 0.5, 0.6),
                                        (0.2, 0.0, 0.5), (0.1, 0.7, 0.45), (0.3, 0.6, 1.0)])
def test_P4b_entropy_fix_first_order(eps, v0, lam):
    """Entropy-fix branch of Q (Appendix A, the numerical-viscosity coefficient
    with epsilon_k).  An alternating density line makes g-tilde change sign at
    every face, so every limiter value g is 0 and the scheme reduces to the
    first-order flux 1/2 (F_L + F_R) - Q(nu) dq / (2 lam), nu = lam v0, with
    Q(chi) = chi^2/(4 eps) + eps for |chi| < 2 eps (here |nu| < 2 eps except
    for the (0.1, 0.7, 0.45) case, which takes |chi|, and the (0.3, 0.6, 1.0)
    case, which sits exactly on the branch point |nu| = 2 eps, where both
    expressions give 2 eps).  Only the entropy wave is excited (B = 0,
    uniform v and P), so dq is a multiple of its eigenvector."""
    gam = 5 / 3
    P = default_params(eps=(eps,) * 7)
    m = 16
    rho = [1.0 + (0.1 if s % 2 else 0.0) for s in range(m)]
    q8 = _entropy_line(rho, v0, gam)
    F = line_fluxes(P, q8, np.zeros(m), lam)
    nu = lam * v0
    Q = nu * nu / (4 * eps) + eps if abs(nu) < 2 * eps else abs(nu)
    if abs(nu) == 2 * eps:
        assert abs(Q - 2 * eps) < 1e-15
    for s in range(2, m - 1):
        uL, uR = q8[s - 1], q8[s]
        ref = 0.5 * (phys_flux(uL, gam) + phys_flux(uR, gam)) - Q * (uR - uL) / (2 * lam)
        ref[4] = 0.0
        assert np.allclose(F[s], ref, rtol=1e-13, atol=1e-15), (s, F[s] - ref)


def sweby_phi(theta, beta):
    """Sweby's limiter family in flux-limiter form (Sweby 1984; LeVeque,
    Numerical Methods for Conservation Laws, Sect. 16.2): beta = 1 minmod,
    beta = 2 superbee."""
    return max(0.0, min(beta * theta, 1.0), min(theta, beta))


@pytest.mark.parametrize("beta", [1.0, 1.25, 1.5, 2.0])
@pytest.mark.parametrize("v0", [0.7, -0.55])
def test_P4c_sweby_family_flux_limiter_form(beta, v0):
    """The limiter (Appendix A, SWEBY with parameter beta) against the
    textbook flux-limiter scheme.  For linear advection at speed a with
    Courant number nu = lam a, eps = 0 and a Sweby limiter phi, Harten's
    modified flux reduces to the upwind flux plus the limited anti-diffusion
        F_{i+1/2} = F(u_up) + 1/2 |a| (1 - |nu|) phi(theta) (u_{i+1} - u_i),
    theta = (u_up - u_up-1) / (u_{i+1} - u_i) the upwind slope ratio.  A
    line carrying only an entropy wave (B = 0, uniform v and P) is such an
    advection for every component, so each face of a random density line
    must match it; beta > 1 (beyond minmod) is exercised wherever the slope
    ratio is away from 1."""
    gam = 5 / 3
    P = default_params(eps=(0.0,) * 7, limiter_beta=beta)
    rng = np.random.default_rng(int(beta * 100) + (1 if v0 > 0 else 2))
    m, lam = 40, 0.45
    rho = 1.0 + 0.4 * rng.random(m)
    q8 = _entropy_line(rho, v0, gam)
    F = line_fluxes(P, q8, np.zeros(m), lam)
    nu = abs(lam * v0)
    checked = 0
    for s in range(3, m - 2):  # face s between zones s-1 and s
        up = s - 1 if v0 > 0 else s
        d = rho[s] - rho[s - 1]
        dup = rho[up] - rho[up - 1] if v0 > 0 else rho[up + 1] - rho[up]
        theta = dup / d
        ref = phys_flux(q8[up], gam) + 0.5 * abs(v0) * (1 - nu) * sweby_phi(theta, beta) * (q8[s] - q8[s - 1])
        ref[4] = 0.0
        assert np.allclose(F[s], ref, rtol=1e-12, atol=1e-14), (s, theta, F[s] - ref)
        checked += 1
    assert checked == m - 5
