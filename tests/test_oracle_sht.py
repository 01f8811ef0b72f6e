"""Pins of the oracle's spherical harmonic transforms: literal O(n^2) ring
sums against the library FFT, adjointness <Y a, m> = <a, Y^T m>, the exact
Gauss-Legendre round trip A Y = 1, pixel-by-pixel evaluation of the explicit
Goldberg harmonics, and the closed-form maps of pure E and pure B modes."""

import numpy as np
import pytest

from oracle.geometry import healpix_grid, gl_grid, pixel_angles, pixel_weights
from oracle.harmonics import goldberg_sylm
from oracle.sht import (SHT, alm_dot, alm_index, lm_arrays, nalm, ring_analysis,
                        ring_synthesis, to_full, to_packed)


def rand_alm(lmax, rng):
    n = nalm(lmax)
    ls, ms = lm_arrays(lmax)
    a = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    a[:, ms == 0] = a[:, ms == 0].real
    a[1:, ls < 2] = 0
    return a


def test_healpix_geometry_counts():
    for nside in (1, 2, 4, 16, 64):
        g = healpix_grid(nside)
        assert len(g["theta"]) == 4 * nside - 1
        assert g["nphi"].sum() == 12 * nside * nside
        assert np.allclose(g["theta"] + g["theta"][::-1], np.pi)      # N/S mirror
        assert np.all(g["nphi"] == g["nphi"][::-1])
        assert np.isclose(pixel_weights(g).sum(), 4 * np.pi)


def test_gl_geometry():
    g = gl_grid(9, 17)
    assert np.isclose(pixel_weights(g).sum(), 4 * np.pi)
    assert np.allclose(g["theta"] + g["theta"][::-1], np.pi)


@pytest.mark.parametrize("n,lmax", [(4, 6), (12, 6), (16, 7), (20, 30), (33, 16), (64, 32)])
def test_ring_sums_direct_vs_fft(n, lmax):
    rng = np.random.default_rng(n)
    F = rng.standard_normal(2 * lmax + 1) + 1j * rng.standard_normal(2 * lmax + 1)
    p0 = 0.37
    a = ring_synthesis(F, n, p0, lmax, direct=True)
    b = ring_synthesis(F, n, p0, lmax, direct=False)
    assert np.allclose(a, b, atol=1e-12)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    a = ring_analysis(x, n, p0, lmax, direct=True)
    b = ring_analysis(x, n, p0, lmax, direct=False)
    assert np.allclose(a, b, atol=1e-12)


def test_packing_roundtrip():
    rng = np.random.default_rng(0)
    lmax = 9
    a = rand_alm(lmax, rng)[0]
    full = to_full(a, lmax)
    assert np.allclose(to_packed(full, lmax), a)
    # reality: a_{l,-m} = (-1)^m conj(a_lm)
    for l in range(lmax + 1):
        for m in range(1, l + 1):
            assert np.isclose(full[l, lmax - m], (-1) ** m * np.conj(full[l, lmax + m]))


@pytest.mark.parametrize("grid,lmax", [(healpix_grid(8), 16), (healpix_grid(4), 13),
                                       (gl_grid(11, 21), 10)])
def test_adjointness(grid, lmax):
    rng = np.random.default_rng(1)
    sht = SHT(grid, lmax)
    a = rand_alm(lmax, rng)
    m = rng.standard_normal((3, grid["npix"]))
    lhs = float(np.sum(sht.synthesis(a) * m))
    yt = sht.adjoint(m)
    rhs = sum(alm_dot(a[f], yt[f], lmax) for f in range(3))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs) * 10


def test_gl_round_trip_exact():
    rng = np.random.default_rng(2)
    lmax = 16
    sht = SHT(gl_grid(lmax + 1, 2 * lmax + 1), lmax)
    a = rand_alm(lmax, rng)
    assert np.abs(sht.analysis(sht.synthesis(a)) - a).max() < 1e-13


def test_dense_goldberg_evaluation_matches_separable():
    """Synthesis at every pixel by explicitly evaluating Goldberg's spin
    harmonics and summing over l and m = -l..l (no ring FFT, no recurrence)."""
    rng = np.random.default_rng(3)
    g = healpix_grid(2)
    lmax = 4
    sht = SHT(g, lmax)
    a = rand_alm(lmax, rng)
    th, ph = pixel_angles(g)
    AT, AE, AB = (to_full(a[f], lmax) for f in range(3))
    I = np.zeros(th.size, dtype=complex)
    P = np.zeros(th.size, dtype=complex)
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            I += AT[l, lmax + m] * goldberg_sylm(0, l, m, th, ph)
            if l >= 2:
                P += -(AE[l, lmax + m] + 1j * AB[l, lmax + m]) * goldberg_sylm(2, l, m, th, ph)
    maps = sht.synthesis(a)
    assert np.allclose(maps[0], I.real, atol=1e-12)
    assert np.allclose(maps[1], P.real, atol=1e-12)
    assert np.allclose(maps[2], P.imag, atol=1e-12)
    assert np.abs(I.imag).max() < 1e-12


def test_pure_e_and_b_maps():
    """a^E_20 = 1 gives Q = -sqrt(15/32pi) sin^2 theta, U = 0; a^B_20 = 1
    gives Q = 0, U = -sqrt(15/32pi) sin^2 theta (Zaldarriaga-Seljak)."""
    g = healpix_grid(4)
    lmax = 4
    sht = SHT(g, lmax)
    th, _ = pixel_angles(g)
    amp = -np.sqrt(15 / (32 * np.pi)) * np.sin(th) ** 2
    a = np.zeros((3, nalm(lmax)), dtype=complex)
    a[1, alm_index(2, 0, lmax)] = 1
    m = sht.synthesis(a)
    assert np.allclose(m[1], amp, atol=1e-15) and np.abs(m[2]).max() < 1e-15
    a[:] = 0
    a[2, alm_index(2, 0, lmax)] = 1
    m = sht.synthesis(a)
    assert np.allclose(m[2], amp, atol=1e-15) and np.abs(m[1]).max() < 1e-15
    # a T monopole is the constant 1/sqrt(4 pi)
    a[:] = 0
    a[0, 0] = 1
    assert np.allclose(sht.synthesis(a)[0], 1 / np.sqrt(4 * np.pi))


def test_sampled_evaluations_match_full():
    rng = np.random.default_rng(4)
    g = healpix_grid(16)
    lmax = 32
    sht = SHT(g, lmax)
    a = rand_alm(lmax, rng)
    full = sht.synthesis(a)
    rings = [0, 5, 31, 62]
    for r, blk in zip(rings, sht.synthesis(a, rings=rings)):
        o, n = g["offset"][r], g["nphi"][r]
        assert np.array_equal(blk, full[:, o:o + n])
    m = rng.standard_normal((3, g["npix"]))
    yt = sht.adjoint(m)
    modes = [(5, 3), (32, 32), (2, 0), (17, 1), (0, 0)]
    sm = sht.adjoint_modes(m, modes)
    for k, (l, mm) in enumerate(modes):
        assert np.allclose(sm[:, k], yt[:, alm_index(l, mm, lmax)], atol=1e-12)


def test_unchunked_equals_chunked():
    rng = np.random.default_rng(5)
    g = healpix_grid(8)
    lmax = 16
    a = rand_alm(lmax, rng)
    s1 = SHT(g, lmax)
    s2 = SHT(g, lmax, cache_bytes=0, chunk_bytes=1)
    assert np.allclose(s1.synthesis(a), s2.synthesis(a), atol=1e-14)
    m = rng.standard_normal((3, g["npix"]))
    assert np.allclose(s1.adjoint(m), s2.adjoint(m), atol=1e-13)


def test_adjoint_over_ring_subsets_sums_to_the_whole():
    """The sampled adjoint (a partial sum over the given rings) over a
    partition of the rings adds up to the full adjoint."""
    lmax = 8
    g = healpix_grid(4)
    sht = SHT(g, lmax)
    rng = np.random.default_rng(3)
    maps = rng.standard_normal((3, g["npix"]))
    nr = len(g["theta"])
    parts = [np.arange(0, nr, 3), np.arange(1, nr, 3), np.arange(2, nr, 3)]
    total = sum(sht.adjoint(maps, rings=r) for r in parts)
    full = sht.adjoint(maps)
    assert np.abs(total - full).max() <= 1e-13 * np.abs(full).max()
