"""Pins of the oracle's dual messenger solver against closed forms and dense
linear algebra:

* closed form: on HEALPix with unmasked homogeneous noise of equal T/Q/U
  variance n, K = 0 and b = d, so after any schedule ending at mu = 0 the
  result is exactly S (S + n Omega)^-1 A d (eq 8 at mu = 0, eq 9 with
  N_bar = 0 -- the corner case of Sec. 2.1);
* Gauss-Legendre grid: the iteration converges to the exact Wiener filter
  of eq 2, solved densely;
* HEALPix: it converges to the dense messenger fixed point (A Y != 1 there);
* chi^2 at the Wiener filter equals d^T (Y S Y^T + N)^-1 d on the observed
  pixels (eq 3 at its minimum);
* eq 18: the fluctuation maps of eq 19 have covariance (S^-1 + N^-1)^-1;
* a mask written as N^-1 = 0 agrees with a mask written as noise 1e10
  (Sec. 2.1 vs Appendix B).
"""

import numpy as np
import pytest

from oracle import dense, dm
from oracle.geometry import gl_grid, healpix_grid, pixel_weights
from oracle.sht import SHT, alm_dot, lm_arrays
from paper_1801_05358_amd import inputs


def rel(a, b, lmax):
    num = sum(alm_dot(a[f] - b[f], a[f] - b[f], lmax) for f in range(3))
    den = sum(alm_dot(b[f], b[f], lmax) for f in range(3))
    return np.sqrt(num / den)


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


def test_schedule_endpoints():
    lam = dm.schedule(1e3, 20)
    assert lam[0] == 1e3 and lam[-1] == 1.0
    assert np.allclose(lam[1:] / lam[:-1], 1e3 ** (-1 / 19))
    assert np.all(dm.schedule(1e3, 1) == 1.0)


def test_filter_eigen_truncation():
    """F = max(S_j, mu) / (max(S_j, mu) + tau) in the eigenbasis of S_l:
    at mu = 0 it is S (S + tau)^-1; at mu above every eigenvalue it is
    mu / (mu + tau) times the identity."""
    lmax = 12
    cl = inputs.spectra(lmax)
    TT, EE, BB, TE = cl
    tau = 0.7
    F = dm.messenger_filter(cl, 0.0, tau)
    for l in range(lmax + 1):
        S = np.array([[TT[l], TE[l]], [TE[l], EE[l]]])
        M = S @ np.linalg.inv(S + tau * np.eye(2))
        assert np.allclose([F[0][l], F[1][l], F[2][l]], [M[0, 0], M[0, 1], M[1, 1]], atol=1e-15)
        assert np.isclose(F[3][l], BB[l] / (BB[l] + tau))
    mu = 10 * cl.max()
    F = dm.messenger_filter(cl, mu, tau)
    assert np.allclose(F[0], mu / (mu + tau)) and np.allclose(F[1], 0, atol=1e-15)


def test_closed_form_homogeneous_noise_healpix():
    rng = np.random.default_rng(11)
    g = healpix_grid(8)
    lmax = 16
    sht = SHT(g, lmax)
    cl = inputs.spectra(lmax)
    n = 0.3
    d = sht.synthesis(inputs.draw_signal(cl, lmax, rng)) + np.sqrt(n) * rng.standard_normal((3, g["npix"]))
    ncov = np.full((3, g["npix"]), n)
    r = dm.solve(sht, d, ncov, None, cl, 1e3, 5, 3)
    Ad = sht.analysis(d)
    tau = n * 4 * np.pi / g["npix"]
    TT, EE, BB, TE = cl
    ls, _ = lm_arrays(lmax)
    want = np.zeros_like(Ad)
    for l in range(lmax + 1):
        S = np.array([[TT[l], TE[l]], [TE[l], EE[l]]])
        M = S @ np.linalg.inv(S + tau * np.eye(2))
        k = ls == l
        want[0, k] = M[0, 0] * Ad[0, k] + M[0, 1] * Ad[1, k]
        want[1, k] = M[1, 0] * Ad[0, k] + M[1, 1] * Ad[1, k]
        want[2, k] = BB[l] / (BB[l] + tau) * Ad[2, k]
    assert rel(r["u"], want, lmax) < 1e-14
    # and the messenger t stays equal to d: u_x after the final step is Y u
    assert np.allclose(r["ux"], sht.synthesis(r["u"]), atol=1e-13)


def test_closed_form_area_homogeneous_noise_gl():
    """On a GL grid, N_p = nu / w_p gives tau = nu and Y^T N^-1 Y = 1/nu, so
    the output is both S (S + nu)^-1 A d and the exact dense WF."""
    rng = np.random.default_rng(12)
    lmax = 8
    g = gl_grid(lmax + 1, 2 * lmax + 1)
    sht = SHT(g, lmax)
    cl = inputs.spectra(lmax)
    nu = 0.05
    ncov = np.tile(nu / pixel_weights(g), (3, 1))
    d = sht.synthesis(inputs.draw_signal(cl, lmax, rng)) + np.sqrt(ncov) * rng.standard_normal((3, g["npix"]))
    r = dm.solve(sht, d, ncov, None, cl, 1e3, 4, 2)
    assert np.isclose(r["tau"], nu)
    wf = dense.wiener_filter(sht, d, ncov, None, cl)
    assert rel(r["u"], wf, lmax) < 1e-13


def test_gl_fixed_point_is_exact_wiener_filter():
    lmax = 6
    sht, cl, ncov, obs, d = small_problem(gl_grid(lmax + 1, 2 * lmax + 1), lmax, seed=7)
    wf = dense.wiener_filter(sht, d, ncov, obs, cl)
    r = dm.solve(sht, d, ncov, obs, cl, 1e3, 5, 120)
    assert r["cauchy"] < 1e-13
    assert rel(r["u"], wf, lmax) < 1e-10
    assert dm.residual(sht, r["u"], d, ncov, obs, cl) < 1e-10


def test_healpix_fixed_point_is_dense_messenger_system():
    lmax = 8
    sht, cl, ncov, obs, d = small_problem(healpix_grid(4), lmax, seed=8)
    fp = dense.messenger_fixed_point(sht, d, ncov, obs, cl)
    r = dm.solve(sht, d, ncov, obs, cl, 1e3, 5, 120)
    assert rel(r["u"], fp, lmax) < 1e-10
    # HEALPix quadrature is not exact, so the fixed point is biased
    wf = dense.wiener_filter(sht, d, ncov, obs, cl)
    assert 1e-3 < rel(fp, wf, lmax) < 0.2


def test_chi2_identity_at_wiener_filter():
    lmax = 6
    sht, cl, ncov, obs, d = small_problem(gl_grid(lmax + 1, 2 * lmax + 1), lmax, seed=9)
    wf = dense.wiener_filter(sht, d, ncov, obs, cl)
    Y = dense.synthesis_matrix(sht)
    S = dense.prior_matrix(cl, lmax)
    o = np.tile(obs, 3)
    C = (Y @ S @ Y.T)[np.ix_(o, o)] + np.diag(ncov.reshape(-1)[o])
    dv = d.reshape(-1)[o]
    want = dv @ np.linalg.solve(C, dv)
    assert np.isclose(dm.chi2(sht, wf, d, ncov, obs, cl), want, rtol=1e-10)


@pytest.mark.slow
def test_fluctuation_covariance_eq18():
    """Sample covariance of f = s_hat - W d_hat over many draws approaches
    (S^-1 + Y^T N^-1 Y)^-1 (statistical, 40000 draws); the prior S itself is far off."""
    lmax = 3
    g = gl_grid(lmax + 1, 2 * lmax + 1)
    sht, cl, ncov, obs, _ = small_problem(g, lmax, seed=10, sscale=1.0)
    Y = dense.synthesis_matrix(sht)
    post = dense.posterior_covariance(sht, ncov, obs, cl, Y=Y)
    S = dense.prior_matrix(cl, lmax)
    st = dm.setup(g, ncov, obs, np.zeros((3, g["npix"])))
    ninv = st["ninv"].reshape(-1)
    W = np.linalg.solve(np.eye(S.shape[0]) + S @ ((Y.T * ninv) @ Y), S @ (Y.T * ninv))
    rng = np.random.default_rng(0)
    n = 40000
    L = np.linalg.cholesky(S + 1e-300 * np.eye(S.shape[0]) + np.diag((np.diag(S) == 0) * 1.0))
    L[np.diag(S) == 0, :] = 0
    shat = L @ rng.standard_normal((S.shape[0], n))
    nhat = np.sqrt(ncov.reshape(-1))[:, None] * rng.standard_normal((Y.shape[0], n))
    f = shat - W @ (Y @ shat + nhat)
    cov = f @ f.T / n
    err = np.linalg.norm(cov - post) / np.linalg.norm(post)
    assert err < 0.04
    assert np.linalg.norm(cov - S) / np.linalg.norm(post) > 0.5


def test_mask_as_large_noise_agrees():
    lmax = 8
    sht, cl, ncov, obs, d = small_problem(healpix_grid(4), lmax, seed=13, maskfrac=0.2)
    r1 = dm.solve(sht, d, ncov, obs, cl, 1e3, 3, 4)
    big = np.where(obs[None, :], ncov, 1e10)
    d2 = np.where(obs[None, :], d, 0.0)
    r2 = dm.solve(sht, d2, big, None, cl, 1e3, 3, 4)
    assert rel(r2["u"], r1["u"], lmax) < 1e-8


def test_linearity_for_constrained_realizations():
    """eq 19: W(d - d_hat) + s_hat = W d + (s_hat - W d_hat)."""
    lmax = 8
    sht, cl, ncov, obs, d = small_problem(healpix_grid(4), lmax, seed=14)
    rng = np.random.default_rng(3)
    shat = inputs.draw_signal(cl, lmax, rng)
    dhat = sht.synthesis(shat) + np.where(obs, np.sqrt(ncov) * rng.standard_normal(ncov.shape), 0)
    scr = dm.constrained_realization(sht, d, dhat, shat, ncov, obs, cl, 1e3, 3, 5)
    wd = dm.solve(sht, d, ncov, obs, cl, 1e3, 3, 5)["u"]
    wdh = dm.solve(sht, dhat, ncov, obs, cl, 1e3, 3, 5)["u"]
    assert rel(scr, wd + (shat - wdh), lmax) < 1e-12


# ----------------------------------------------------------------------------
# the epsilon-driven schedule (Algorithm 1's stopping rule, Sec. 3.2)
# ----------------------------------------------------------------------------
def test_eps_schedule_is_geometric_down_to_one():
    lam = dm.eps_schedule(1e3, 0.75)
    assert lam[0] == 1e3 and lam[-1] == 1.0
    assert np.all(lam[:-1] > 1.0)
    assert np.allclose(lam[1:-1] / lam[:-2], 0.75, rtol=1e-15, atol=0)
    # the last geometric value is the first one not above 1 times 1/beta
    assert lam[-2] * 0.75 <= 1.0
    assert np.array_equal(dm.eps_schedule(1.0, 0.5), [1.0])
    assert np.array_equal(dm.eps_schedule(16.0, 0.5), [16.0, 8.0, 4.0, 2.0, 1.0])


def test_eps_thresholds_cool_by_eta_with_floor():
    eps = dm.eps_thresholds(30, 1e-4, 1e-6, 1.1)
    assert eps[0] == 1e-4 and eps[-1] == 1e-6
    assert np.all(np.diff(eps) <= 0)
    assert np.isclose(eps[1], 1e-4 / 1.1, rtol=1e-15)
    # the floor: 1e-4 / 1.1^j reaches 1e-6 at j = 49 (beyond 30 steps, so
    # only the last entry is at the floor here)
    assert np.all(eps[:-1] > 1e-6)
    long = dm.eps_thresholds(60, 1e-4, 1e-6, 1.1)
    assert np.all(long[49:] == 1e-6) and long[48] > 1e-6


def test_eps_mode_with_loose_threshold_is_one_iteration_per_step():
    """With thresholds above any Cauchy ratio every step stops after one
    iteration, which is the fixed schedule with one iteration per step over
    the same lambdas (16 -> 1 by halving = 16^(1 - k/4))."""
    lmax = 6
    sht, cl, ncov, obs, d = small_problem(gl_grid(lmax + 1, 2 * lmax + 1), lmax, seed=21)
    r = dm.solve_eps(sht, d, ncov, obs, cl, 16.0, 0.5, 10.0, 10.0, 1.0, 1000)
    ref = dm.solve(sht, d, ncov, obs, cl, 16.0, 5, 1)
    assert r["iterations"] == 5 and r["steps"] == [0, 1, 2, 3, 4]
    assert r["trace"][0] == 1.0                         # u_0 = 0
    assert rel(r["u"], ref["u"], lmax) < 1e-13


def test_eps_mode_iteration_cap():
    """A threshold of zero never stops a step: the cap ends the solve, and
    at lambda = 1 that is the fixed schedule with the cap's iteration count."""
    lmax = 6
    sht, cl, ncov, obs, d = small_problem(gl_grid(lmax + 1, 2 * lmax + 1), lmax, seed=22)
    r = dm.solve_eps(sht, d, ncov, obs, cl, 1.0, 0.5, 0.0, 0.0, 1.0, 7)
    ref = dm.solve(sht, d, ncov, obs, cl, 1.0, 1, 7)
    assert r["iterations"] == 7 and set(r["steps"]) == {0}
    assert rel(r["u"], ref["u"], lmax) < 1e-13


def test_eps_mode_converges_to_exact_wiener_filter_on_gl():
    """On an exact-quadrature grid the stopping rule with a tight final
    threshold ends at the exact WF (eq 2); every step ends below its
    threshold, and the Cauchy ratio of each step's first iteration after
    cooling is larger than the last one of the step before (the peaks of
    Fig. 4)."""
    lmax = 6
    sht, cl, ncov, obs, d = small_problem(gl_grid(lmax + 1, 2 * lmax + 1), lmax, seed=23)
    r = dm.solve_eps(sht, d, ncov, obs, cl, 1e3, 0.75, 1e-4, 1e-12, 1.1, 100000)
    wf = dense.wiener_filter(sht, d, ncov, obs, cl)
    assert r["iterations"] < 100000
    assert r["trace"][-1] < 1e-12
    assert rel(r["u"], wf, lmax) < 1e-9
    tr, st = np.array(r["trace"]), np.array(r["steps"])
    for j in range(len(r["lambdas"])):
        assert tr[st == j][-1] < r["eps"][j]
    firsts = [np.flatnonzero(st == j)[0] for j in range(1, len(r["lambdas"]))]
    assert all(tr[i] > tr[i - 1] for i in firsts)


def test_diagnostics_record_the_iterates():
    """The per-iteration record (Fig. 4) holds chi^2 and the residual of the
    iterate after iterations 2, 4, 6 of a 2 x 3 schedule (every 2nd and the
    last), each equal to the diagnostics of that iterate recomputed from a
    run stopped there."""
    from oracle.geometry import healpix_grid
    from oracle.sht import SHT
    from paper_1801_05358_amd import inputs
    nside, lmax = 4, 8
    p = inputs.make_problem(1, nside=nside, lmax=lmax)
    sht = SHT(healpix_grid(nside), lmax)
    d = sht.synthesis(inputs.signal_alm(1, lmax, 0)) + inputs.noise_map(1, p["ncov"], p["obs"], 0)
    r = dm.solve(sht, d, p["ncov"], p["obs"], p["cl"], 1e3, 2, 3, diagnostics_every=2)
    g = r["diagnostics"]
    assert g["iteration"] == [2, 4, 6]
    st = dm.setup(sht.grid, p["ncov"], p["obs"], d)
    lam = dm.schedule(1e3, 2)
    for i, c2, rs in zip(g["iteration"], g["chi2"], g["residual"]):
        counts = [min(i, 3), max(i - 3, 0)]
        u = dm.messenger_run_counts(sht, st["d0"], st["K"], st["b"], st["tau"], p["cl"], lam, counts)[0]
        assert abs(c2 - dm.chi2(sht, u, d, p["ncov"], p["obs"], p["cl"])) <= 1e-12 * c2
        assert abs(rs - dm.residual(sht, u, d, p["ncov"], p["obs"], p["cl"])) <= 1e-12 * rs
    assert np.array_equal(r["u"], dm.solve(sht, d, p["ncov"], p["obs"], p["cl"], 1e3, 2, 3)["u"])
    e = dm.solve_eps(sht, d, p["ncov"], p["obs"], p["cl"], 1e3, 0.5, 1e-2, 1e-3, 1.1, 7, diagnostics_every=3)
    assert e["diagnostics"]["iteration"] == [3, 6, 7]
