"""Pins of the oracle's refinement by the modified Jacobi relaxation
(Appendix A), on the CPU.

* The Wiener filter residual vanishes at the exact Wiener filter from dense
  linear algebra (eq 2), and not at a perturbed solution.
* The messenger run driven by weighted data g = P d is solve() itself.
* On a Gauss-Legendre grid (exact quadrature) the corrections reach the
  dense Wiener filter to rounding; on HEALPix, where the messenger's own
  fixed point is off by 1e-2 (quadrature error), they converge
  geometrically to the dense Wiener filter as well; with correlated 3x3
  noise and distinct temperature and polarization masks on the exact
  quadrature grid.
"""

import numpy as np

from oracle import dense, dm
from oracle.geometry import gl_grid, healpix_grid, pixel_weights
from oracle.sht import SHT, alm_dot
from paper_1801_05358_amd import inputs


def small_problem(grid, lmax, seed, maskfrac=0.1, dyn=3.0, sscale=1e-2):
    rng = np.random.default_rng(seed)
    sht = SHT(grid, lmax)
    cl = inputs.spectra(lmax) * sscale
    w = pixel_weights(grid)
    nt = (1 + (dyn - 1) * rng.random(grid["npix"])) * w.mean() / w
    ncov = np.stack([nt, 2 * nt, 2 * nt])
    obs = rng.random(grid["npix"]) >= maskfrac
    s = inputs.draw_signal(cl, lmax, rng)
    d = sht.synthesis(s) + np.sqrt(ncov) * rng.standard_normal((3, grid["npix"]))
    return sht, cl, ncov, obs, d


def rel(a, b, lmax):
    num = sum(alm_dot(a[f] - b[f], a[f] - b[f], lmax) for f in range(3))
    den = sum(alm_dot(b[f], b[f], lmax) for f in range(3))
    return float(np.sqrt(num / den))


def norm(a, lmax):
    return float(np.sqrt(sum(alm_dot(a[f], a[f], lmax) for f in range(3))))


def test_residual_vanishes_at_dense_wiener_filter():
    lmax = 8
    sht, cl, ncov, obs, d = small_problem(healpix_grid(4), lmax, seed=41)
    wf = dense.wiener_filter(sht, d, ncov, obs, cl)
    st = dm.setup(sht.grid, ncov, obs, d)
    r = dm.wf_residual(sht, wf, st, cl)
    y = dm.wf_residual(sht, np.zeros_like(wf), st, cl)
    assert norm(y, lmax) > 0
    assert norm(r, lmax) < 1e-12 * norm(y, lmax)
    # a perturbation of one coefficient shows up in the residual
    bad = wf.copy()
    bad[0, 10] *= 1.01
    assert norm(dm.wf_residual(sht, bad, st, cl), lmax) > 1e-6 * norm(y, lmax)


def test_weighted_run_with_pd_is_solve():
    lmax = 8
    sht, cl, ncov, obs, d = small_problem(healpix_grid(4), lmax, seed=42)
    st = dm.setup(sht.grid, ncov, obs, d)
    g = dm.pix_apply(st["ninv"], st["d0"])
    tp = st["tau"] / pixel_weights(sht.grid)
    u = dm.messenger_run(sht, st["d0"], st["K"], tp * g, st["tau"], cl, 1e3, 3, 4)[0]
    assert rel(u, dm.solve(sht, d, ncov, obs, cl, 1e3, 3, 4)["u"], lmax) < 1e-13


def test_gauss_legendre_reaches_dense_wiener_filter():
    lmax = 6
    sht, cl, ncov, obs, d = small_problem(gl_grid(lmax + 1, 2 * lmax + 1), lmax, seed=43)
    wf = dense.wiener_filter(sht, d, ncov, obs, cl)
    s0 = dm.solve(sht, d, ncov, obs, cl, 1e3, 5, 20)["u"]
    r = dm.refine(sht, d, ncov, obs, cl, 1e3, 5, 20, 5)
    assert rel(s0, wf, lmax) > 1e-6
    assert rel(r["u"], wf, lmax) < 1e-12
    h = r["history"]
    assert all(h[k + 1] < 1e-2 * h[k] for k in range(3)), h


def test_healpix_converges_to_dense_wiener_filter():
    """The plain messenger's HEALPix fixed point is not the Wiener filter;
    the corrections converge to it, by a factor below 0.5 each."""
    lmax = 8
    sht, cl, ncov, obs, d = small_problem(healpix_grid(4), lmax, seed=44)
    wf = dense.wiener_filter(sht, d, ncov, obs, cl)
    s0 = dm.solve(sht, d, ncov, obs, cl, 1e3, 3, 4)["u"]
    r = dm.refine(sht, d, ncov, obs, cl, 1e3, 3, 4, 14)
    assert rel(s0, wf, lmax) > 1e-2
    assert rel(r["u"], wf, lmax) < 1e-6
    h = r["history"]
    assert all(h[k + 1] < 0.5 * h[k] for k in range(len(h) - 1)), h


def test_correlated_noise_and_distinct_masks():
    """On the exact-quadrature grid, where the messenger run converges for
    correlated noise too (on HEALPix a long run can grow along directions
    with K_p near 1, since Y^T W Y exceeds 1 there)."""
    lmax = 8
    grid = gl_grid(lmax + 1, 2 * lmax + 1)
    rng = np.random.default_rng(45)
    sht = SHT(grid, lmax)
    cl = inputs.spectra(lmax) * 1e-2
    w = pixel_weights(grid)
    L = rng.standard_normal((grid["npix"], 3, 3)) * 0.3 + np.eye(3) * np.array([1.0, 1.4, 1.4])
    N = np.einsum("pij,pkj->pik", L, L) * (w.mean() / w)[:, None, None]
    ncov6 = np.stack([N[:, i, j] for i, j in dm.SYM6])
    obs = (rng.random(grid["npix"]) >= 0.1, rng.random(grid["npix"]) >= 0.25)
    d = sht.synthesis(inputs.draw_signal(cl, lmax, rng)) + rng.standard_normal((3, grid["npix"]))
    wf = dense.wiener_filter(sht, d, ncov6, obs, cl)
    s0 = dm.solve(sht, d, ncov6, obs, cl, 1e3, 5, 20)["u"]
    r = dm.refine(sht, d, ncov6, obs, cl, 1e3, 5, 20, 6)
    assert rel(s0, wf, lmax) > 1e-3
    assert rel(r["u"], wf, lmax) < 1e-8
    h = r["history"]
    assert all(h[k + 1] < 0.2 * h[k] for k in range(len(h) - 1)), h


def test_divergent_corrections_last_and_best_iterate():
    """With 100:1 scan noise and holes on HEALPix at lmax = 2 Nside the
    short messenger run is too rough an inverse and the corrections stall,
    then grow.  Appendix A's relaxation returns the last iterate, whose
    residual is the last entry of the history; select="best" returns the
    iterate of smallest residual, whose residual is that minimum (both
    recomputed here)."""
    nside, lmax = 16, 32
    p = inputs.make_problem(2, nside=nside, lmax=lmax, holes=20)
    sht = SHT(healpix_grid(nside), lmax)
    d = sht.synthesis(inputs.signal_alm(2, lmax, 0)) + inputs.noise_map(2, p["ncov"], p["obs"], 0)
    st = dm.setup(sht.grid, p["ncov"], p["obs"], d)
    y = dm.wf_residual(sht, np.zeros((3, (lmax + 1) * (lmax + 2) // 2), dtype=complex), st, p["cl"])
    last = dm.refine(sht, d, p["ncov"], p["obs"], p["cl"], 1e3, 5, 10, 8)
    h = last["history"]
    assert h[-1] > min(h) and 0 < last["best"] < len(h) - 1, h
    assert last["chosen"] == len(h) - 1
    got = norm(dm.wf_residual(sht, last["u"], st, p["cl"]), lmax) / norm(y, lmax)
    assert abs(got - h[-1]) < 1e-12 * h[-1]
    best = dm.refine(sht, d, p["ncov"], p["obs"], p["cl"], 1e3, 5, 10, 8, select="best")
    assert best["history"] == h and best["chosen"] == best["best"] == last["best"]
    got = norm(dm.wf_residual(sht, best["u"], st, p["cl"]), lmax) / norm(y, lmax)
    assert abs(got - min(h)) < 1e-12 * min(h)


def test_eps_rule_refinement_reaches_dense_wiener_filter():
    """Appendix A's own prescription: the first solve under the Cauchy rule
    records its iterations per cooling step, and the corrections run those
    counts; on the exact-quadrature grid they reach the dense Wiener filter."""
    lmax = 6
    sht, cl, ncov, obs, d = small_problem(gl_grid(lmax + 1, 2 * lmax + 1), lmax, seed=46)
    wf = dense.wiener_filter(sht, d, ncov, obs, cl)
    plain = dm.solve_eps(sht, d, ncov, obs, cl, 1e3, 0.5, 1e-2, 1e-3, 1.1, 2000)
    r = dm.refine_eps(sht, d, ncov, obs, cl, 1e3, 0.5, 1e-2, 1e-3, 1.1, 2000, 4)
    assert sum(r["counts"]) == plain["iterations"] and min(r["counts"]) >= 1
    assert rel(plain["u"], wf, lmax) > 1e-5
    assert rel(r["u"], wf, lmax) < 1e-10
    h = r["history"]
    assert all(h[k + 1] < 0.1 * h[k] for k in range(3)), h
