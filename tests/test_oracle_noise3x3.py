"""Pins of the oracle's correlated 3x3 pixel noise (eq 11) and distinct
temperature and polarization masks (Appendix B):

* with zero correlations the 3x3 path reduces exactly to the diagonal one;
* the inverse noise covariance with Sigma^-1 = 0 on unobserved components
  is the limit of N^-1 as those noise amplitudes go to infinity at fixed
  correlation matrix C (brute force with amplitudes 1e6 and 1e8 times
  larger: the observed block converges, the rest vanishes as 1 / s);
* the messenger update t = K u_x + b equals Appendix B's messenger equation
  written out with N_bar^-1 = Sigma^-1 P^T (Delta - alpha P Sigma^-2 P^T)^-1
  P Sigma^-1 from the eigendecomposition C = P^T Delta P;
* the messenger variance is tight: every K_p has eigenvalues in [0, 1] and
  one pixel reaches 0 (alpha is the smallest admissible eigenvalue);
* Gauss-Legendre grid: the iteration converges to the exact Wiener filter
  with the block-diagonal N^-1 (dense solve); HEALPix: to the dense
  messenger fixed point;
* chi^2 at the Wiener filter equals d^T (1 + N^-1 Y S Y^T)^-1 N^-1 d, its
  closed-form minimum, and has no linear term around it;
* the input recipe's correlated draws have covariance N_p.
"""

import numpy as np

from oracle import dense, dm
from oracle.geometry import gl_grid, healpix_grid, pixel_weights
from oracle.sht import SHT, alm_dot
from paper_1801_05358_amd import inputs


def rel(a, b, lmax):
    num = sum(alm_dot(a[f] - b[f], a[f] - b[f], lmax) for f in range(3))
    den = sum(alm_dot(b[f], b[f], lmax) for f in range(3))
    return np.sqrt(num / den)


def corr_problem(grid, lmax, seed, sscale=1e-2, mask_t=0.15, mask_p=0.1):
    rng = np.random.default_rng(seed)
    sht = SHT(grid, lmax)
    cl = inputs.spectra(lmax) * sscale
    w = pixel_weights(grid)
    nt = (1 + 2 * rng.random(grid["npix"])) * w.mean() / w
    ncov6 = inputs.correlate_noise(np.stack([nt, 2 * nt, 2 * nt]))
    obs_t = rng.random(grid["npix"]) >= mask_t
    obs_p = rng.random(grid["npix"]) >= mask_p
    obs3 = np.stack([obs_t, obs_p, obs_p])
    d = sht.synthesis(inputs.draw_signal(cl, lmax, rng)) + inputs.draw_noise6(ncov6, obs3, rng)
    return sht, cl, ncov6, (obs_t, obs_p), d


def test_zero_correlation_reduces_to_diagonal():
    lmax = 8
    g = healpix_grid(4)
    sht, cl, ncov6, obs, d = corr_problem(g, lmax, seed=1)
    diag = ncov6[[0, 3, 5]]
    ncov6z = np.zeros_like(ncov6)
    ncov6z[[0, 3, 5]] = diag
    a = dm.setup(g, diag, obs, d)
    b = dm.setup(g, ncov6z, obs, d)
    assert np.isclose(a["tau"], b["tau"], rtol=1e-15)
    for f in range(3):
        assert np.allclose(b["K"][f, f], a["K"][f], rtol=1e-14, atol=1e-15)
        assert np.allclose(b["ninv"][f, f], a["ninv"][f], rtol=1e-14, atol=0)
        for g2 in range(3):
            if g2 != f:
                assert np.all(b["K"][f, g2] == 0) and np.all(b["ninv"][f, g2] == 0)
    assert np.allclose(b["b"], a["b"], rtol=1e-13, atol=1e-15 * np.abs(a["b"]).max())
    ua = dm.solve(sht, d, diag, obs, cl, 1e3, 3, 4)["u"]
    ub = dm.solve(sht, d, ncov6z, obs, cl, 1e3, 3, 4)["u"]
    assert rel(ub, ua, lmax) < 1e-12


def test_masked_precision_is_infinite_variance_limit():
    """Appendix B: Sigma^-1 = 0 on masked components; the same as letting
    their noise amplitude go to infinity with the correlation matrix
    fixed.  Checked against the inverse of N with those amplitudes scaled
    by s = 1e6 and 1e8, and alpha_p against the smallest eigenvalue of N
    at s = 1e7."""
    g = healpix_grid(4)
    _, _, ncov6, obs, d = corr_problem(g, 4, seed=2, mask_t=0.3, mask_p=0.3)
    st = dm.setup(g, ncov6, obs, d)
    o = st["obs"]
    N = dm.noise_blocks(ncov6)
    sig = np.sqrt(np.einsum("pii->pi", N))
    C = N / (sig[:, :, None] * sig[:, None, :])
    seen = o.any(axis=0)
    partial = seen & ~o.all(axis=0)
    assert partial.sum() > 10
    P = np.moveaxis(st["ninv"], -1, 0)
    assert np.all(P[~seen] == 0)

    def scaled(s):
        big = np.where(o.T, sig, s * sig)
        return C * big[:, :, None] * big[:, None, :]

    # the observed block converges as 1 / s^2, the rest vanishes as 1 / s
    for s in (1e6, 1e8):
        Ns = scaled(s)
        for q in np.flatnonzero(seen):
            lim = np.linalg.inv(Ns[q])
            oo = np.outer(o[:, q], o[:, q])
            scale = np.abs(P[q]).max()
            assert np.allclose(P[q][oo], lim[oo], rtol=0, atol=1e-9 * scale), q
            assert np.abs(P[q] - lim).max() < 10 / s * scale, q
    Ns = scaled(1e7)
    w = pixel_weights(g)
    alpha = np.array([np.linalg.eigvalsh(Ns[q])[0] for q in np.flatnonzero(seen)])
    assert np.isclose(st["tau"], np.min(alpha * w[seen]), rtol=1e-9)


def test_update_is_appendix_b_messenger_equation():
    """t = (N_bar^-1 + T^-1)^-1 (T^-1 u_x + N_bar^-1 d) per pixel, N_bar^-1
    from the eigendecomposition of the correlation matrix with Sigma^-1 = 0
    on unobserved components, against t = K u_x + b."""
    g = healpix_grid(4)
    _, _, ncov6, obs, d = corr_problem(g, 4, seed=3, mask_t=0.3, mask_p=0.3)
    st = dm.setup(g, ncov6, obs, d)
    rng = np.random.default_rng(5)
    ux = rng.standard_normal(d.shape)
    t = dm.pix_apply(st["K"], ux) + st["b"]
    N = dm.noise_blocks(ncov6)
    Tp = st["tau"] / pixel_weights(g)
    checked = 0
    for q in range(g["npix"]):
        o = st["obs"][:, q]
        if not o.any():
            continue
        sig = np.sqrt(np.diag(N[q]))
        C = N[q] / np.outer(sig, sig)
        delta, V = np.linalg.eigh(C)              # C = P^T Delta P with P = V^T
        Pm = V.T
        sinv = np.where(o, 1.0 / sig, 0.0)        # Sigma^-1, zero on masked components
        inner = np.diag(delta) - Tp[q] * Pm @ np.diag(sinv ** 2) @ Pm.T
        if np.linalg.cond(inner) > 1e8:           # the pixel(s) where alpha is attained
            continue
        nbar_inv = np.diag(sinv) @ Pm.T @ np.linalg.inv(inner) @ Pm @ np.diag(sinv)
        lhs = np.linalg.inv(nbar_inv + np.eye(3) / Tp[q])
        want = lhs @ (ux[:, q] / Tp[q] + nbar_inv @ d[:, q])
        assert np.allclose(t[:, q], want, rtol=1e-9, atol=1e-9 * np.abs(want).max()), q
        checked += 1
    assert checked > 0.9 * g["npix"] * 0.5


def test_messenger_variance_is_tight():
    g = healpix_grid(4)
    _, _, ncov6, obs, d = corr_problem(g, 4, seed=4)
    st = dm.setup(g, ncov6, obs, d)
    K = np.moveaxis(st["K"], -1, 0)
    ev = np.linalg.eigvalsh(K)
    assert ev.min() > -1e-13 and ev.max() <= 1 + 1e-13
    assert abs(ev.min()) < 1e-12


def test_gl_fixed_point_is_exact_wiener_filter_correlated():
    lmax = 6
    sht, cl, ncov6, obs, d = corr_problem(gl_grid(lmax + 1, 2 * lmax + 1), lmax, seed=7)
    wf = dense.wiener_filter(sht, d, ncov6, obs, cl)
    r = dm.solve(sht, d, ncov6, obs, cl, 1e3, 5, 150)
    assert r["cauchy"] < 1e-13
    assert rel(r["u"], wf, lmax) < 1e-10
    assert dm.residual(sht, r["u"], d, ncov6, obs, cl) < 1e-10


def test_healpix_fixed_point_correlated():
    lmax = 8
    sht, cl, ncov6, obs, d = corr_problem(healpix_grid(4), lmax, seed=8)
    fp = dense.messenger_fixed_point(sht, d, ncov6, obs, cl)
    r = dm.solve(sht, d, ncov6, obs, cl, 1e3, 5, 150)
    assert rel(r["u"], fp, lmax) < 1e-10


def test_chi2_minimum_closed_form_correlated():
    lmax = 6
    sht, cl, ncov6, obs, d = corr_problem(gl_grid(lmax + 1, 2 * lmax + 1), lmax, seed=9)
    wf = dense.wiener_filter(sht, d, ncov6, obs, cl)
    st = dm.setup(sht.grid, ncov6, obs, d)
    Y = dense.synthesis_matrix(sht)
    S = dense.prior_matrix(cl, lmax)
    P = dense.pixel_matrix(st["ninv"])
    dv = st["d0"].reshape(-1)
    want = dv @ np.linalg.solve(np.eye(P.shape[0]) + P @ Y @ S @ Y.T, P @ dv)
    c0 = dm.chi2(sht, wf, d, ncov6, obs, cl)
    assert np.isclose(c0, want, rtol=1e-10)
    # no linear term: chi^2(u + e v) = chi^2(u - e v) > chi^2(u)
    rng = np.random.default_rng(1)
    v = inputs.draw_signal(cl, lmax, rng)
    cp = dm.chi2(sht, wf + 1e-2 * v, d, ncov6, obs, cl)
    cm = dm.chi2(sht, wf - 1e-2 * v, d, ncov6, obs, cl)
    assert cp > c0 and cm > c0
    assert abs(cp - cm) < 1e-8 * (cp - c0)


def test_correlated_draws_have_covariance_n():
    n = 40000
    N = np.array([[2.0, 0.3, -0.2], [0.3, 1.5, 0.25], [-0.2, 0.25, 1.0]])
    ncov6 = np.array([N[i, j] for i, j in dm.SYM6])[:, None] * np.ones(n)
    x = inputs.draw_noise6(ncov6, np.ones((3, n), dtype=bool), np.random.default_rng(0))
    cov = x @ x.T / n
    assert np.abs(cov - N).max() < 0.05
    o = np.ones((3, n), dtype=bool)
    o[1:, ::2] = False
    y = inputs.draw_noise6(ncov6, o, np.random.default_rng(0))
    assert np.all(y[1:, ::2] == 0) and np.all(y[0] != 0)


def test_correlated_problem_recipe():
    p = inputs.correlated_problem(1)
    ot, op = p["obs_t"], p["obs_p"]
    assert (ot & ~op).sum() > 0 and (~ot & op).sum() > 0
    assert op.mean() > ot.mean()
    N = dm.noise_blocks(p["ncov6"])
    assert np.linalg.eigvalsh(N).min() > 0
