"""Seeded synthetic inputs for the dual messenger workloads.

This module holds input recipes only -- spectra, Gaussian draws, masks and
noise patterns -- and none of the method's arithmetic (no transform, no
filter, no iteration).  Both the GPU library's callers and the CPU checker
consume what it produces.

Recipes (all random numbers from NumPy's PCG64 with explicit seeds
``1000 * cfg + 10 * role + k``):

* spectra, l >= 2 (zero below): C^TT = 1e3 / (l (l+1)), C^EE = 0.05 C^TT,
  C^TE = 0.3 sqrt(C^TT C^EE), C^BB = 0.01 C^EE;
* signal harmonic coefficients: per l, the Cholesky factor of the TE block
  times unit normals (the paper simulates its maps the same way, Sec. 3.1);
  m = 0 real with variance C, m > 0 with real and imaginary parts of
  variance C / 2 each;
* masks: a Galactic-like band |latitude| < b plus circular holes with
  centres uniform on the sphere;
* noise variance per pixel for T, with Q = U = 2x that of T:
  (a) log-normal  exp(0.5 g) (1 + cos^2 theta),  g ~ N(0, 1);
  (b) scan-like  sigma0^2 * R^(1 - h),  h = (1 + cos gamma) / 2, gamma the
      angle to a tilted scan pole at (theta, phi) = (60 deg, 45 deg); the
      range is exactly R : 1;
* noise realizations n_p = sqrt(N_p) g on observed pixels;
* correlated pixel noise (3x3 per pixel): off-diagonal terms as fixed
  fractions of the geometric means of the variances (correlation matrix
  [[1, .3, -.15], [.3, 1, .2], [-.15, .2, 1]]), and distinct temperature
  and polarization masks (the polarization band 3 deg narrower, the two
  with independent holes, at least 1.5 pixel sides in radius, and the
  temperature mask with twice as many, so
  that some pixels observe T only and some Q, U only); realizations
  L_p g with L_p the Cholesky factor of N_p, zero on unobserved
  components.
"""

import numpy as np

(ROLE_SIGNAL, ROLE_NOISE, ROLE_HOLES, ROLE_PATTERN, ROLE_CR_SIGNAL, ROLE_CR_NOISE, ROLE_HOLES_P,
 ROLE_NOISE6) = range(8)


def seed_for(cfg, role, k=0):
    return 1000 * int(cfg) + 10 * int(role) + int(k)


def rng_for(cfg, role, k=0):
    return np.random.Generator(np.random.PCG64(seed_for(cfg, role, k)))


# ----------------------------------------------------------------------------
# spectra and signal draws
# ----------------------------------------------------------------------------
def spectra(lmax):
    """[4, lmax+1] in the order TT, EE, BB, TE."""
    l = np.arange(lmax + 1, dtype=np.float64)
    TT = np.zeros(lmax + 1)
    TT[2:] = 1e3 / (l[2:] * (l[2:] + 1))
    EE = 0.05 * TT
    TE = 0.3 * np.sqrt(TT * EE)
    BB = 0.01 * EE
    return np.stack([TT, EE, BB, TE])


def nalm(lmax):
    return (lmax + 1) * (lmax + 2) // 2


def lm_of_index(lmax):
    """(l, m) of every packed index, packed m-major: idx = m(2lmax+1-m)/2 + l."""
    ms = np.repeat(np.arange(lmax + 1), lmax + 1 - np.arange(lmax + 1))
    start = ms * (2 * lmax + 1 - ms) // 2
    ls = np.arange(nalm(lmax)) - start
    return ls, ms


def draw_signal(cl, lmax, rng):
    """Gaussian harmonic coefficients [3, nalm] (T, E, B) with prior cl."""
    TT, EE, BB, TE = cl
    ls, ms = lm_of_index(lmax)
    n = ls.size
    g = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    g[:, ms == 0] = (g[:, ms == 0].real * np.sqrt(2.0)).astype(np.complex128)
    g /= np.sqrt(2.0)
    # Cholesky of [[TT, TE], [TE, EE]] per l (lower triangular)
    l11 = np.sqrt(TT)
    with np.errstate(divide="ignore", invalid="ignore"):
        l21 = np.where(l11 > 0, TE / np.where(l11 > 0, l11, 1.0), 0.0)
    l22 = np.sqrt(np.maximum(EE - l21 ** 2, 0.0))
    a = np.empty((3, n), dtype=np.complex128)
    a[0] = l11[ls] * g[0]
    a[1] = l21[ls] * g[0] + l22[ls] * g[1]
    a[2] = np.sqrt(BB)[ls] * g[2]
    return a


# ----------------------------------------------------------------------------
# pixel centres (for masks and noise patterns only)
# ----------------------------------------------------------------------------
def healpix_centres(nside):
    """(theta, phi) of HEALPix RING pixel centres."""
    th, ph = [], []
    for i in range(1, 4 * nside):
        if i < nside:
            z, n, p0 = 1 - i * i / (3.0 * nside * nside), 4 * i, np.pi / (4 * i)
        elif i <= 3 * nside:
            z = 4.0 / 3.0 - 2.0 * i / (3.0 * nside)
            n = 4 * nside
            p0 = np.pi / (4 * nside) if (i - nside) % 2 == 0 else 0.0
        else:
            j = 4 * nside - i
            z, n, p0 = -(1 - j * j / (3.0 * nside * nside)), 4 * j, np.pi / (4 * j)
        th.append(np.full(n, np.arccos(z)))
        ph.append(p0 + 2 * np.pi * np.arange(n) / n)
    return np.concatenate(th), np.concatenate(ph)


def gl_centres(ntheta, nphi):
    x, _ = np.polynomial.legendre.leggauss(ntheta)
    x = np.sort(x)[::-1]
    th = np.repeat(np.arccos(x), nphi)
    ph = np.tile(2 * np.pi * np.arange(nphi) / nphi, ntheta)
    return th, ph


# ----------------------------------------------------------------------------
# masks and noise
# ----------------------------------------------------------------------------
def band_mask(theta, bdeg):
    """True = observed; masks |latitude| < bdeg."""
    lat = 0.5 * np.pi - theta
    return np.abs(lat) >= np.deg2rad(bdeg)


def hole_mask(theta, phi, nholes, radius_deg, rng):
    """True = observed; masks pixels whose centre is within radius of any of
    ``nholes`` centres drawn uniformly on the sphere."""
    obs = np.ones(theta.size, dtype=bool)
    if nholes == 0:
        return obs
    zc = rng.uniform(-1, 1, nholes)
    pc = rng.uniform(0, 2 * np.pi, nholes)
    sc = np.sqrt(1 - zc * zc)
    rad = np.deg2rad(radius_deg)
    cosr = np.cos(rad)
    # pixels come in rings of non-decreasing colatitude: only the slice
    # |theta - theta_c| <= radius can fall inside a hole
    assert np.all(np.diff(theta) >= 0)
    for k in range(nholes):
        tc = np.arccos(zc[k])
        lo, hi = np.searchsorted(theta, [tc - rad - 1e-12, tc + rad + 1e-12])
        t, p = theta[lo:hi], phi[lo:hi]
        dot = np.sin(t) * sc[k] * np.cos(p - pc[k]) + np.cos(t) * zc[k]
        obs[lo:hi] &= dot < cosr
    return obs


def noise_lognormal(theta, rng, sigma_ln=0.5):
    """T variance exp(sigma_ln g) (1 + cos^2 theta); Q = U = 2 T."""
    vt = np.exp(sigma_ln * rng.standard_normal(theta.size)) * (1 + np.cos(theta) ** 2)
    return np.stack([vt, 2 * vt, 2 * vt])


def noise_scan(theta, phi, dyn, sigma0sq=1.0, pole=(60.0, 45.0)):
    """T variance sigma0^2 dyn^(1 - h), h = (1 + cos gamma) / 2; Q = U = 2 T."""
    tp, pp = np.deg2rad(pole[0]), np.deg2rad(pole[1])
    cosg = (np.sin(theta) * np.sin(tp) * np.cos(phi - pp) + np.cos(theta) * np.cos(tp))
    h = 0.5 * (1 + cosg)
    vt = sigma0sq * dyn ** (1 - h)
    return np.stack([vt, 2 * vt, 2 * vt])


def draw_noise(ncov, obs, rng):
    n = np.sqrt(ncov) * rng.standard_normal(ncov.shape)
    return np.where(obs[None, :], n, 0.0)


# correlated pixel noise: the layout (II, IQ, IU, QQ, QU, UU) of a symmetric
# 3x3 per-pixel covariance
SYM6 = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))


def correlate_noise(ncov, rho_tp=0.3, rho_qu=0.2):
    """A correlated per-pixel covariance built from diagonal variances
    (II, QQ, UU): N_IQ = rho_tp sqrt(II QQ), N_IU = -rho_tp/2 sqrt(II UU),
    N_QU = rho_qu sqrt(QQ UU) (positive definite for these small rho).
    Returns [6, npix] in the SYM6 layout."""
    II, QQ, UU = ncov
    return np.stack([II, rho_tp * np.sqrt(II * QQ), -0.5 * rho_tp * np.sqrt(II * UU), QQ,
                     rho_qu * np.sqrt(QQ * UU), UU])


def draw_noise6(ncov6, obs3, rng):
    """n_p = L_p g with L_p L_p^T = N_p (per pixel), zero on unobserved
    components.  obs3: [3, npix] bool."""
    N = np.zeros((ncov6.shape[1], 3, 3))
    for k, (i, j) in enumerate(SYM6):
        N[:, i, j] = ncov6[k]
        N[:, j, i] = ncov6[k]
    L = np.linalg.cholesky(N)
    n = np.einsum("pij,jp->ip", L, rng.standard_normal((3, ncov6.shape[1])))
    return np.where(obs3, n, 0.0)


# ----------------------------------------------------------------------------
# workload configurations
# ----------------------------------------------------------------------------
CONFIGS = {
    # cfg: nside, lmax, mask band (deg), holes, noise kind, dyn, steps, iters/step, nrhs
    1: dict(nside=16, lmax=32, band=20.0, holes=0, noise="lognormal", dyn=None, nsteps=20, iters=10, nrhs=1),
    2: dict(nside=256, lmax=512, band=15.0, holes=200, noise="scan", dyn=100.0, nsteps=20, iters=10, nrhs=1),
    3: dict(nside=1024, lmax=2048, band=15.0, holes=1000, noise="scan", dyn=100.0, nsteps=20, iters=10, nrhs=1),
    4: dict(nside=512, lmax=1024, band=15.0, holes=200, noise="scan", dyn=100.0, nsteps=20, iters=10, nrhs=64),
    5: dict(nside=2048, lmax=4096, band=float(np.rad2deg(np.arcsin(0.30))), holes=5000, noise="scan",
            dyn=1000.0, nsteps=30, iters=10, nrhs=8),
}
LAMBDA0 = 1e3
HOLE_RADIUS_DEG = 0.5


def make_problem(cfg, nside=None, lmax=None, holes=None, grid="healpix", ntheta=None, nphi=None):
    """Mask, noise covariance and spectra of configuration ``cfg`` (1..5),
    optionally at another resolution (same recipe).  Returns a dict with
    cl [4, lmax+1], ncov [3, npix], obs [npix] bool, theta, phi."""
    c = dict(CONFIGS[cfg])
    if nside is not None:
        c["nside"] = nside
    if lmax is not None:
        c["lmax"] = lmax
    if holes is not None:
        c["holes"] = holes
    if grid == "healpix":
        th, ph = healpix_centres(c["nside"])
    else:
        th, ph = gl_centres(ntheta, nphi)
    obs = band_mask(th, c["band"]) & hole_mask(th, ph, c["holes"], HOLE_RADIUS_DEG, rng_for(cfg, ROLE_HOLES))
    if c["noise"] == "lognormal":
        ncov = noise_lognormal(th, rng_for(cfg, ROLE_PATTERN))
    else:
        ncov = noise_scan(th, ph, c["dyn"])
    c.update(cl=spectra(c["lmax"]), ncov=ncov, obs=obs, theta=th, phi=ph, lambda0=LAMBDA0)
    return c


def signal_alm(cfg, lmax, k=0, role=ROLE_SIGNAL):
    return draw_signal(spectra(lmax), lmax, rng_for(cfg, role, k))


def noise_map(cfg, ncov, obs, k=0, role=ROLE_NOISE):
    return draw_noise(ncov, obs, rng_for(cfg, role, k))


def correlated_problem(cfg, **kw):
    """make_problem plus correlated noise and distinct T / P masks: adds
    ncov6 [6, npix] (SYM6 layout), obs_t and obs_p [npix] bool and obs3
    [3, npix] (I observed where obs_t, Q and U where obs_p)."""
    p = make_problem(cfg, **kw)
    th, ph = p["theta"], p["phi"]
    holes = max(2 * p["holes"], 4)
    # holes at least 1.5 pixel sides across, so that they remove pixels on
    # coarse grids too
    rad = max(HOLE_RADIUS_DEG, 1.5 * float(np.rad2deg(np.sqrt(4 * np.pi / th.size))))
    obs_t = band_mask(th, p["band"]) & hole_mask(th, ph, holes, rad, rng_for(cfg, ROLE_HOLES))
    obs_p = band_mask(th, p["band"] - 3.0) & hole_mask(th, ph, holes // 2, rad, rng_for(cfg, ROLE_HOLES_P))
    p.update(ncov6=correlate_noise(p["ncov"]), obs_t=obs_t, obs_p=obs_p, obs3=np.stack([obs_t, obs_p, obs_p]))
    return p


def noise_map6(cfg, ncov6, obs3, k=0, role=ROLE_NOISE6):
    return draw_noise6(ncov6, obs3, rng_for(cfg, role, k))
