"""Pins of the oracle parts that its other tests take for granted: the
HEALPix ring geometry and the residual of Appendix C away from the solution.

HEALPix (Gorski et al. 2005) fixes, independently of the ring formulas:

* the 12 base pixels (Nside 1): centres at z = 2/3 and -2/3 with
  phi = pi/4 + k pi/2, and at z = 0 with phi = k pi/2;
* equal area: the spherical cap above the centre of north ring i holds the
  pixels of the rings before it plus half of ring i, each of area
  4 pi / N_pix (this fixes every ring's z, in the caps and the belt);
* the hierarchy: every base pixel is cut into Nside x Nside pixels, so its
  centre is a pixel centre at odd Nside and the midpoint of two
  neighbouring pixel centres of the same ring at even Nside (this fixes the
  first-pixel longitude phi0 and its alternation in the belt).

Appendix C writes the Wiener filter equation as A x = y with
A = 1 + S^1/2 N^-1 S^1/2, x = S^-1/2 s, y = S^1/2 N^-1 d; on the sphere
N^-1 becomes Y^T N^-1 Y and N^-1 d becomes Y^T N^-1 d.  The residual
||A x - y|| / ||y|| of an arbitrary iterate is compared with that
definition in dense matrices (S^1/2 from the eigendecomposition of the whole
prior matrix, Y^T as the transpose of the dense synthesis matrix).

Each pin is also shown to catch a planted mistake: a flipped belt phi0
parity, a mis-typed cap z, and S^1/2 and S^+1/2 in each other's place.
"""

import numpy as np
import pytest

from oracle import dense, dm
from oracle.geometry import gl_grid, healpix_grid, pixel_angles
from oracle.sht import SHT, lm_arrays, nalm
from paper_1801_05358_amd import inputs


# ----------------------------------------------------------------------------
# HEALPix geometry
# ----------------------------------------------------------------------------
def base_pixel_centres():
    """(z, phi) of the 12 base pixels, Gorski et al. 2005 (Fig. 3 / Sec. 4)."""
    out = []
    for z, first in ((2.0 / 3.0, np.pi / 4), (0.0, 0.0), (-2.0 / 3.0, np.pi / 4)):
        out += [(z, first + k * np.pi / 2) for k in range(4)]
    return out


def check_base_pixels(grid_fn):
    g = grid_fn(1)
    th, ph = pixel_angles(g)
    got = sorted(zip(np.round(np.cos(th), 14), np.round(np.mod(ph, 2 * np.pi), 14)))
    want = sorted((round(z, 14), round(p, 14)) for z, p in base_pixel_centres())
    return len(got) == 12 and np.allclose(np.array(got), np.array(want), rtol=0, atol=1e-13)


def check_equal_area(grid_fn, nsides=(1, 2, 3, 4, 7, 16, 64)):
    for nside in nsides:
        g = grid_fn(nside)
        npix = g["npix"]
        before = 0
        for k in range(2 * nside):              # north rings and the equator
            n = int(g["nphi"][k])
            cap = 2.0 * np.pi * (1.0 - np.cos(g["theta"][k]))
            if abs(cap - (before + 0.5 * n) * 4.0 * np.pi / npix) > 1e-12:
                return False
            before += n
    return True


def check_hierarchy(grid_fn, nsides=range(1, 10)):
    for nside in nsides:
        g = grid_fn(nside)
        z = np.cos(g["theta"])
        for zc, pc in base_pixel_centres():
            k = int(np.argmin(np.abs(z - zc)))
            if abs(z[k] - zc) > 1e-12:
                return False
            n, p0 = int(g["nphi"][k]), g["phi0"][k]
            # position of the base centre in units of the ring's pixel spacing
            j = (pc - p0) * n / (2.0 * np.pi)
            frac = j - np.floor(j)
            want = 0.0 if nside % 2 == 1 else 0.5
            if min(abs(frac - want), abs(frac - want - 1.0), abs(frac - want + 1.0)) > 1e-9:
                return False
    return True


def flipped_belt_parity(nside):
    """Planted mistake: phi0 = pi/(4 nside) on the belt rings with
    (i - nside) odd instead of even."""
    g = healpix_grid(nside)
    for k in range(len(g["theta"])):
        i = k + 1
        if nside <= i <= 3 * nside:
            g["phi0"][k] = 0.0 if (i - nside) % 2 == 0 else np.pi / (4.0 * nside)
    return g


def mistyped_cap_z(nside):
    """Planted mistake: z = 1 - i^2 / (3 nside) in the polar caps."""
    g = healpix_grid(nside)
    nr = len(g["theta"])
    for k in range(nr):
        i = k + 1
        j = min(i, 4 * nside - i)
        if j < nside:
            z = 1.0 - j * j / (3.0 * nside)
            g["theta"][k] = np.arccos(np.clip(z if i < 2 * nside else -z, -1, 1))
    return g


def test_base_pixel_centres():
    assert check_base_pixels(healpix_grid)


def test_equal_area_rings():
    assert check_equal_area(healpix_grid)


def test_base_pixels_subdivide():
    assert check_hierarchy(healpix_grid)


def test_geometry_pins_catch_planted_mistakes():
    # a flipped belt parity keeps the equal-area rings but moves the pixels
    assert check_equal_area(flipped_belt_parity)
    assert not check_base_pixels(flipped_belt_parity)
    assert not check_hierarchy(flipped_belt_parity)
    # a mis-typed cap z keeps the longitudes but breaks equal area
    assert not check_equal_area(mistyped_cap_z)


# ----------------------------------------------------------------------------
# Appendix C residual away from the solution
# ----------------------------------------------------------------------------
def dense_sqrt(S):
    """S^1/2 and S^+1/2 of a symmetric positive semi-definite matrix from its
    eigendecomposition (eigenvalues below 1e-12 of the largest count as 0)."""
    w, V = np.linalg.eigh(S)
    pos = w > 1e-12 * w.max()
    h = np.where(pos, np.sqrt(np.where(pos, w, 0.0)), 0.0)
    ih = np.where(pos, 1.0 / np.sqrt(np.where(pos, w, 1.0)), 0.0)
    return (V * h) @ V.T, (V * ih) @ V.T


def appendix_c(sht, u, d, ncov, obs, cl, swap=False):
    """||A x - y|| / ||y||, A = 1 + S^1/2 Y^T N^-1 Y S^1/2, x = S^+1/2 u,
    y = S^1/2 Y^T N^-1 d, in dense matrices (swap: the planted mistake of
    S^1/2 and S^+1/2 in each other's place)."""
    lmax = sht.lmax
    Y = dense.synthesis_matrix(sht)
    st = dm.setup(sht.grid, ncov, obs, d)
    NI = dense.pixel_matrix(st["ninv"])
    half, ihalf = dense_sqrt(dense.prior_matrix(cl, lmax))
    if swap:
        half, ihalf = ihalf, half
    x = ihalf @ dense.alm_to_x(u, lmax)
    A = np.eye(len(x)) + half @ Y.T @ NI @ Y @ half
    y = half @ Y.T @ NI @ st["d0"].reshape(-1)
    return float(np.linalg.norm(A @ x - y) / np.linalg.norm(y))


def random_iterate(cl, lmax, rng):
    """An iterate in the range of S (every solve ends in it: at mu = 0 the
    filter of eq 8 vanishes where S does), otherwise arbitrary."""
    ls, ms = lm_arrays(lmax)
    u = rng.standard_normal((3, nalm(lmax))) + 1j * rng.standard_normal((3, nalm(lmax)))
    u[:, ms == 0] = u[:, ms == 0].real
    u *= np.sqrt(cl[[0, 1, 2]][:, ls])          # TT, EE, BB scale; zero where the spectrum is
    return u


@pytest.mark.parametrize("grid", ["gl", "healpix"])
def test_residual_matches_appendix_c_away_from_the_solution(grid):
    lmax = 4
    g = gl_grid(lmax + 1, 2 * lmax + 1) if grid == "gl" else healpix_grid(2)
    sht = SHT(g, lmax)
    rng = np.random.default_rng(7)
    p = inputs.make_problem(1, nside=2, lmax=lmax) if grid == "healpix" else None
    cl = inputs.spectra(lmax)
    npix = g["npix"]
    ncov = np.stack([np.exp(rng.standard_normal(npix) * 0.5)] * 1 + [2 * np.exp(rng.standard_normal(npix) * 0.5)] * 2)
    obs = rng.random(npix) >= 0.2 if p is None else p["obs"]
    d = sht.synthesis(inputs.draw_signal(cl, lmax, rng)) + np.sqrt(ncov) * rng.standard_normal((3, npix))
    for _ in range(3):
        u = random_iterate(cl, lmax, rng)
        want = appendix_c(sht, u, d, ncov, obs, cl)
        got = dm.residual(sht, u, d, ncov, obs, cl)
        assert 1e-3 < want and abs(got - want) < 1e-12 * want, (got, want)
        # the planted mistake moves the value far outside that tolerance
        assert abs(appendix_c(sht, u, d, ncov, obs, cl, swap=True) - want) > 1e-3 * want


def test_residual_pin_catches_planted_mistake(monkeypatch):
    """The oracle's residual with S^1/2 and S^+1/2 in each other's place no
    longer matches the dense definition."""
    lmax = 4
    g = gl_grid(lmax + 1, 2 * lmax + 1)
    sht = SHT(g, lmax)
    rng = np.random.default_rng(8)
    cl = inputs.spectra(lmax)
    npix = g["npix"]
    ncov = np.ones((3, npix)) * 0.5
    obs = rng.random(npix) >= 0.2
    d = sht.synthesis(inputs.draw_signal(cl, lmax, rng)) + rng.standard_normal((3, npix))
    u = random_iterate(cl, lmax, rng)
    want = appendix_c(sht, u, d, ncov, obs, cl)
    real_mf = dm.matrix_function
    calls = []

    def swapped(cl_, fn):
        # residual() asks first for S^1/2, then for S^+1/2: hand them out swapped
        calls.append(fn)
        if len(calls) == 1:
            return real_mf(cl_, lambda s: np.where(s > 0, 1.0 / np.sqrt(np.where(s > 0, s, 1.0)), 0.0))
        if len(calls) == 2:
            return real_mf(cl_, lambda s: np.sqrt(np.maximum(s, 0.0)))
        return real_mf(cl_, fn)

    monkeypatch.setattr(dm, "matrix_function", swapped)
    got = dm.residual(sht, u, d, ncov, obs, cl)
    assert abs(got - want) > 1e-3 * want
