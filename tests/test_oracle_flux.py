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
