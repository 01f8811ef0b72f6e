"""Pins of the oracle's adaptive working resolution (the hierarchical
framework of the text after eq 9 and the working-resolution proposal of
Sec. 4): at truncation mu the prior clamped at mu is mu 1 above ell_iter(mu),
so the transforms of that cooling step run with a band limit a little above
ell_iter.

* ell_iter against the closed form for the workloads' spectra: the largest
  eigenvalue of the TE block is c C^TT with c fixed by the ratios EE/TT and
  TE / sqrt(TT EE), so ell_iter solves l (l + 1) <= c 1e3 / mu;
* above ell_iter the filter of eq 8 is the constant mu / (mu + tau) in T, E
  and B with no TE coupling (nothing left to resolve);
* a band limit at or above lmax reproduces solve() to the last bit;
* a truncated step equals the same step computed by transforms built for
  the smaller band limit (an independent route through the packed layouts);
* the band limits rise with the cooling and end at lmax (mu = 0).
"""

import numpy as np

from oracle import dm
from oracle.geometry import healpix_grid
from oracle.sht import SHT, alm_index, lm_arrays, nalm
from paper_1801_05358_amd import inputs


def test_ell_iter_closed_form():
    lmax = 4096
    cl = inputs.spectra(lmax)
    r, rho = 0.05, 0.3                      # EE / TT and TE / sqrt(TT EE) of the recipe
    c = (1 + r) / 2 + np.sqrt(((1 - r) / 2) ** 2 + rho * rho * r)
    for mu in (1e-1, 3e-3, 1e-3, 2.7e-4, 1e-5, 1e-6):
        x = c * 1e3 / mu
        want = int(np.floor((-1 + np.sqrt(1 + 4 * x)) / 2))
        # rounding of the root: check the defining inequality on both sides
        while want * (want + 1) > x:
            want -= 1
        while (want + 1) * (want + 2) <= x:
            want += 1
        want = min(want, lmax) if want >= 2 else -1
        assert dm.ell_iter(cl, mu) == want, (mu, dm.ell_iter(cl, mu), want)
    assert dm.ell_iter(cl, 0.0) == lmax
    assert dm.ell_iter(cl, 1e9) == -1


def test_filter_is_constant_above_ell_iter():
    lmax = 600
    cl = inputs.spectra(lmax)
    tau, mu = 1e-6, 5e-3
    li = dm.ell_iter(cl, mu)
    assert 2 < li < lmax
    FTT, FTE, FEE, FBB = dm.messenger_filter(cl, mu, tau)
    k = mu / (mu + tau)
    for F in (FTT, FEE, FBB):
        assert np.allclose(F[li + 1:], k, rtol=1e-14, atol=0)
    assert np.all(np.abs(FTE[li + 1:]) < 1e-14)
    assert abs(FTT[li] - k) > 1e-9 * k        # at ell_iter the prior still resolves T


def problem(nside, lmax):
    p = inputs.make_problem(1, nside=nside, lmax=lmax)
    sht = SHT(healpix_grid(nside), lmax)
    d = sht.synthesis(inputs.signal_alm(1, lmax, 0)) + inputs.noise_map(1, p["ncov"], p["obs"], 0)
    return p, sht, d


def test_full_band_reproduces_solve():
    p, sht, d = problem(4, 8)
    a = dm.solve(sht, d, p["ncov"], p["obs"], p["cl"], 1e3, 3, 4)
    b = dm.solve(sht, d, p["ncov"], p["obs"], p["cl"], 1e3, 3, 4, adaptive=1e9)
    assert b["lcuts"] == [8, 8, 8]
    assert np.array_equal(a["u"], b["u"])


def test_truncated_step_equals_smaller_transforms():
    nside, lmax, L = 8, 16, 9
    p, sht, d = problem(nside, lmax)
    st = dm.setup(sht.grid, p["ncov"], p["obs"], d)
    lam = 300.0
    mu = (lam - 1.0) * st["tau"]
    t = st["d0"]
    # the oracle's route: full-band transforms, band-limited filter
    u = dm.messenger_run_counts(sht, t, st["K"], st["b"], st["tau"], p["cl"], [lam], [1], lcuts=[L])[0]
    ux = sht.synthesis(u)
    # independent route: transforms built for band limit L
    small = SHT(sht.grid, L)
    F = dm.messenger_filter(p["cl"][:, :L + 1], mu, st["tau"])
    uL = dm.apply_blocks(F, small.analysis(t), L)
    uxL = small.synthesis(uL)
    ls, ms = lm_arrays(lmax)
    emb = np.zeros((3, nalm(lmax)), dtype=complex)
    lsL, msL = lm_arrays(L)
    emb[:, [alm_index(l, m, lmax) for l, m in zip(lsL, msL)]] = uL
    assert np.all(u[:, ls > L] == 0)
    assert np.abs(u - emb).max() <= 1e-13 * np.abs(emb).max()
    assert np.abs(ux - uxL).max() <= 1e-13 * np.abs(uxL).max()


def test_band_limits_follow_the_cooling():
    nside, lmax = 16, 32
    p, sht, d = problem(nside, lmax)
    # at Nside 16 tau is large (4 pi / 3072 pixels), so the cooling starts
    # higher than the workloads' 1e3 for the truncation to show
    r = dm.solve(sht, d, p["ncov"], p["obs"], p["cl"], 1e5, 6, 2, adaptive=1.25)
    lc = r["lcuts"]
    assert all(a <= b for a, b in zip(lc, lc[1:])) and lc[-1] == lmax and lc[0] < lmax, lc
    st = dm.setup(sht.grid, p["ncov"], p["obs"], d)
    lams = dm.schedule(1e5, 6)
    assert lc == [dm.working_lmax(p["cl"], (x - 1) * st["tau"], lmax, 1.25) for x in lams]
    ls, _ = lm_arrays(lmax)
    assert np.any(r["u"][:, ls > lc[0]] != 0)        # the last steps run the full band
