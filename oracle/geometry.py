"""Ring grids on the sphere (oracle; test infrastructure only).

The paper's basis change is a flat-sky FFT (Sec. 2.1, eqs 12-16); moving the
method to the sphere replaces it with a spherical harmonic transform on an
iso-latitude ring grid.  Two grids are used:

* HEALPix RING (Gorski et al. 2005): equal-area pixels, weight 4 pi / N_pix.
* Gauss-Legendre: exact quadrature for band-limited products, used for the
  exact Wiener-filter pins.

A grid is a dict with per-ring arrays ``theta`` (colatitude), ``nphi``,
``phi0`` (longitude of the first pixel), ``wring`` (per-pixel quadrature
weight on that ring) and ``offset`` (index of the ring's first pixel).
"""

import numpy as np


def healpix_grid(nside):
    """HEALPix RING geometry for ``nside``: 4 nside - 1 rings from north."""
    nside = int(nside)
    nrings = 4 * nside - 1
    theta = np.empty(nrings)
    nphi = np.empty(nrings, dtype=np.int64)
    phi0 = np.empty(nrings)
    for k in range(nrings):
        i = k + 1
        if i < nside:                       # north polar cap
            z = 1.0 - i * i / (3.0 * nside * nside)
            n = 4 * i
            p0 = np.pi / (4.0 * i)
        elif i <= 3 * nside:                # equatorial belt
            z = 4.0 / 3.0 - 2.0 * i / (3.0 * nside)
            n = 4 * nside
            p0 = np.pi / (4.0 * nside) if (i - nside) % 2 == 0 else 0.0
        else:                               # south cap mirrors ring 4 nside - i
            j = 4 * nside - i
            z = -(1.0 - j * j / (3.0 * nside * nside))
            n = 4 * j
            p0 = np.pi / (4.0 * j)
        theta[k] = np.arccos(z)
        nphi[k] = n
        phi0[k] = p0
    npix = 12 * nside * nside
    offset = np.concatenate([[0], np.cumsum(nphi)[:-1]])
    assert offset[-1] + nphi[-1] == npix
    wring = np.full(nrings, 4.0 * np.pi / npix)
    return dict(kind="healpix", nside=nside, theta=theta, nphi=nphi,
                phi0=phi0, wring=wring, offset=offset, npix=npix)


def gl_grid(ntheta, nphi):
    """Gauss-Legendre grid: ``ntheta`` rings at the Gauss nodes, ``nphi``
    equally spaced pixels per ring starting at phi = 0."""
    x, g = np.polynomial.legendre.leggauss(int(ntheta))
    order = np.argsort(-x)                  # north (z = +1) first
    x, g = x[order], g[order]
    theta = np.arccos(x)
    nphi_arr = np.full(ntheta, int(nphi), dtype=np.int64)
    phi0 = np.zeros(ntheta)
    wring = 2.0 * np.pi * g / nphi
    offset = np.arange(ntheta, dtype=np.int64) * nphi
    return dict(kind="gl", theta=theta, nphi=nphi_arr, phi0=phi0,
                wring=wring, offset=offset, npix=int(ntheta) * int(nphi))


def pixel_weights(grid):
    """Per-pixel quadrature weight w_p."""
    return np.repeat(grid["wring"], grid["nphi"])


def pixel_angles(grid):
    """(theta_p, phi_p) of every pixel centre, ring order."""
    th = np.repeat(grid["theta"], grid["nphi"])
    ph = np.concatenate([grid["phi0"][k] + 2.0 * np.pi * np.arange(n) / n
                         for k, n in enumerate(grid["nphi"])])
    return th, ph
