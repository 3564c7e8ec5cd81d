"""Pins of the oracle's domain boundaries (outflow: zero-gradient extension
along an axis whose neighbour entry is -1).

O1 a uniform state is a fixed point with outflow on every axis; O2 Brio-Wu
data along one axis with outflow on that axis: the 3D step equals the plain
1D conservative update with the line extended by copies of its end zones,
bitwise; O3 a blast that has not reached the boundary: outflow and periodic
boundaries give bitwise the same state, and the totals are conserved; O4 the
ghosts of an outflow side hold copies of the boundary zone (and of the
boundary face for the normal field).
"""
import numpy as np
import pytest

from oracle import line_fluxes
from paper_1701_07452_amd import inputs as I
from tests._helpers import oracle_gather, oracle_sim


def test_O1_uniform_fixed_point_all_outflow():
    shape = (12, 10, 16)
    q = np.zeros((8,) + shape)
    q[0] = 1.3
    q[1], q[2], q[3] = 0.2, -0.1, 0.05
    B = (0.4, -0.3, 0.2)
    b = I.uniform_faces(shape, B)
    q[4:7] = np.array(B)[:, None, None, None]
    q[7] = 1.0 / (2.0 / 3.0) + 0.5 * (0.2 ** 2 + 0.1 ** 2 + 0.05 ** 2) / 1.3 + 0.5 * sum(x * x for x in B)
    G = I.patch_grid([8, 8], [10], [6, 6], periodic=(False, False, False))
    sim = oracle_sim(G, q, b, dx=(0.1, 0.1, 0.1))
    for _ in range(3):
        sim.fill_ghosts()
        sim.advance(sim.compute_dt())
    qn, bn = oracle_gather(G, sim)
    assert np.array_equal(qn, q) and np.array_equal(bn, b)
    sim.close()


@pytest.mark.parametrize("axis", [0, 2])
def test_O2_outflow_line_reduction(axis):
    N, g = 32, 5
    shape = [8, 8, 8]
    shape[2 - axis] = N
    shape = tuple(shape)
    q0, b0 = I.shock_tube_x((8, 8, N), gamma=2.0)
    cm = [(0 + axis) % 3, (1 + axis) % 3, (2 + axis) % 3]
    lineq, lineb = q0[:, 0, 0, :], b0[:, 0, 0, :]

    def place(v):
        s = [1, 1, 1]
        s[2 - axis] = N
        return np.broadcast_to(v.reshape(s), shape)

    q = np.zeros((8,) + shape)
    b = np.zeros((3,) + shape)
    q[0], q[7] = place(lineq[0]), place(lineq[7])
    for c in range(3):
        q[1 + cm[c]] = place(lineq[1 + c])
        q[4 + cm[c]] = place(lineq[4 + c])
        b[cm[c]] = place(lineb[c])
    dx = (1.0 / N,) * 3
    periodic = [True, True, True]
    periodic[axis] = False
    n = (shape[2], shape[1], shape[0])
    half = list(n)
    half[axis] = N // 2
    G = I.uniform_grid(n, tuple(half), periodic=tuple(periodic))  # two patches along the axis
    sim = oracle_sim(G, q, b, dx=dx, gamma=2.0)
    P = sim.params

    def line(a):
        sl = [0, 0, 0]
        sl[2 - axis] = slice(None)
        return a[(slice(None),) + tuple(sl)]

    fr = np.stack([lineq[0], lineq[1], lineq[2], lineq[3], lineq[4], lineq[5], lineq[6], lineq[7]], -1)
    bpar = lineb[0]
    for _ in range(8):
        sim.fill_ghosts()
        dt = sim.compute_dt()
        sim.advance(dt)
        qq = np.concatenate([np.repeat(fr[:1], g, 0), fr, np.repeat(fr[-1:], g, 0)])
        bf = np.concatenate([np.repeat(bpar[:1], g), bpar, np.repeat(bpar[-1:], g)])
        F = line_fluxes(P, qq, bf, dt / dx[0])
        fr = fr - dt / dx[0] * (F[g + 1:g + N + 1] - F[g:g + N])
    qn, bn = oracle_gather(G, sim)
    got = line(qn)
    ref = np.stack([fr[:, 0], fr[:, 1], fr[:, 2], fr[:, 3], fr[:, 4], fr[:, 5], fr[:, 6], fr[:, 7]])
    frame = np.stack([got[0], got[1 + cm[0]], got[1 + cm[1]], got[1 + cm[2]], got[4 + cm[0]], got[4 + cm[1]],
                      got[4 + cm[2]], got[7]])
    assert np.array_equal(frame, ref)
    sim.close()


def _blast(N=24):
    shape = (N, N, N)
    dx = (1.0 / N,) * 3
    (xc, yc, zc), _ = I.coords(shape, dx, origin=(-0.5, -0.5, -0.5))
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    p = np.where(r < 0.1, 10.0, 0.1)
    B0 = (0.5, 0.3, 0.0)
    b = I.uniform_faces(shape, B0)
    q = I.conserved(np.ones(shape), [np.zeros(shape)] * 3, I.face_average(b), p)
    return q, b, dx


def test_O3_contained_blast_outflow_equals_periodic():
    q, b, dx = _blast(24)
    res = []
    for per in ((True, True, True), (False, False, False)):
        G = I.uniform_grid(24, 12, periodic=per)
        sim = oracle_sim(G, q, b, dx=dx)
        t0, _, _, _ = sim.diagnostics()
        for _ in range(3):
            sim.fill_ghosts()
            sim.advance(sim.compute_dt())
        t1, dn, _, _ = sim.diagnostics()
        res.append(oracle_gather(G, sim))
        for c in range(8):
            assert abs(t1[c] - t0[c]) <= 1e-13 * max(1.0, abs(t0[c]))
        assert dn < 1e-12
        sim.close()
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])


def test_O4_outflow_ghost_values():
    q, b = I.random_smooth((8, 10, 12), 21)
    G = I.patch_grid([12], [10], [8], periodic=(False, True, False))
    sim = oracle_sim(G, q, b, dx=(0.1, 0.1, 0.1))
    sim.fill_ghosts()
    qs, bs = sim.get_stored(0)
    g = 5
    n = (12, 10, 8)
    # x-ghosts of interior rows: copies of the boundary zone; b_x: the boundary face
    for i in range(g):
        assert np.array_equal(qs[:, g:g + 8, g:g + 10, i], qs[:, g:g + 8, g:g + 10, g])
        assert np.array_equal(qs[:, g:g + 8, g:g + 10, g + n[0] + i], qs[:, g:g + 8, g:g + 10, g + n[0] - 1])
        assert np.array_equal(bs[0, g:g + 8, g:g + 10, i], bs[0, g:g + 8, g:g + 10, g])
        assert np.array_equal(bs[1:, g:g + 8, g:g + 10, i], bs[1:, g:g + 8, g:g + 10, g])
    for i in range(1, g):
        assert np.array_equal(bs[0, g:g + 8, g:g + 10, g + n[0] + i], bs[0, g:g + 8, g:g + 10, g + n[0]])
    # a corner ghost (x < 0, z >= n_z) is the boundary zone (0, y, n_z - 1)
    assert np.array_equal(qs[:, g + 8 + 2, g + 3, 1], qs[:, g + 7, g + 3, g])
    sim.close()
