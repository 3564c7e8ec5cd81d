"""Unit tests of the seeded input generators (no GPU, no oracle)."""
import math

import numpy as np

from paper_1701_07452_amd import inputs as I


def divb(b, dx):
    return ((np.roll(b[0], -1, 2) - b[0]) / dx[0] + (np.roll(b[1], -1, 1) - b[1]) / dx[1]
            + (np.roll(b[2], -1, 0) - b[2]) / dx[2])


def test_vector_potential_fields_are_divergence_free():
    for q, b, dx in [
        I.fast_wave_diagonal(16)[:2] + ((1 / 16,) * 3,),
        I.orszag_tang_3d(16) + ((1 / 16,) * 3,),
        I.random_smooth((12, 10, 8), 3) + ((1 / 8, 1 / 10, 1 / 12),),
    ]:
        assert np.abs(divb(b, dx)).max() * min(dx) < 1e-13
    q, b, ex, dx = I.cp_alfven(8)
    assert np.abs(divb(b, dx)).max() * min(dx) < 1e-13


def test_turbulence_statistics_and_seed():
    q, b = I.turbulence(32)
    v = q[1:4] / q[0]
    cs = math.sqrt(5 / 3)
    assert abs(math.sqrt(np.mean(np.sum(v ** 2, 0))) / cs - 1.0) < 1e-12
    assert np.abs(v.mean(axis=(1, 2, 3))).max() < 1e-12
    q2, _ = I.turbulence(32)
    assert np.array_equal(q, q2)
    q3, _ = I.turbulence(32, seed=5)
    assert not np.array_equal(q, q3)
    # spectrum: shell-averaged energy falls roughly as k^-5/3
    vk = np.fft.fftn(v, axes=(1, 2, 3))
    k = np.fft.fftfreq(32, 1 / 32)
    K = np.sqrt(k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2)
    E = np.sum(np.abs(vk) ** 2, 0)
    ks = np.arange(2, 12)
    Ek = np.array([E[(K >= kk - 0.5) & (K < kk + 0.5)].sum() for kk in ks])
    slope = np.polyfit(np.log(ks), np.log(Ek), 1)[0]
    assert -2.2 < slope < -1.2, slope


def test_high_contrast_statistics():
    q, b = I.high_contrast_turbulence(32)
    rho = q[0]
    assert abs(rho.mean() - 1.0) < 1e-12
    assert abs(np.log(rho).std() - 1.5) < 0.05
    v = q[1:4] / rho
    assert abs(math.sqrt(np.mean(np.sum(v ** 2, 0))) - 5 * math.sqrt(5 / 3)) < 1e-9


def test_uneven_grid_tiling_and_neighbours():
    G = I.uneven_grid()
    assert G.npatch == 400
    Nz, Ny, Nx = G.shape
    assert G.zones() == Nx * Ny * Nz
    # every face neighbour shares the face extent (tensor-product tiling)
    for (n, nbr), o in zip(G.descs, G.origin):
        assert nbr[13] == G.descs.index((n, nbr))
        for ax, (lo, hi) in enumerate(((12, 14), (10, 16), (4, 22))):
            for t in (lo, hi):
                m = G.descs[nbr[t]][0]
                for a in range(3):
                    if a != ax:
                        assert m[a] == n[a]


def test_split_gather_roundtrip():
    G = I.patch_grid([8, 16], [8, 8], [16])
    q = np.random.default_rng(0).normal(size=(8,) + G.shape)
    b = np.random.default_rng(1).normal(size=(3,) + G.shape)
    q2, b2 = I.gather(G, I.split(G, q, b))
    assert np.array_equal(q, q2) and np.array_equal(b, b2)


def test_fast_wave_eigenvector_is_the_fast_mode():
    q, b, wv = I.fast_wave_diagonal(8)
    assert abs(wv.speed - 2.0) < 1e-12
    assert abs(wv.period - 1 / (2 * math.sqrt(3))) < 1e-12
