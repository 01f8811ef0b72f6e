"""Dual messenger Wiener filter for (I, Q, U) -> (T, E, B) on the sphere
(oracle; test infrastructure only).

Follows the paper step by step (Kodi Ramanah, Lavaux & Wandelt 2018):

* eq 4 / Algorithm 1: the messenger covariance T = alpha 1 with alpha the
  smallest noise eigenvalue; the pixel noise is diagonal or the full 3x3
  block of eq 11, with a common mask or distinct T and P masks
  (Appendix B).  On a grid with quadrature weights w_p the
  harmonic-space messenger variance is tau = min_p (alpha_p w_p) and the
  pixel-space one T_p = tau / w_p (for HEALPix, w = 4 pi / N_pix and
  tau = alpha w is the sphere's counterpart of sigma^-1 alpha);
* eq 8 with the Heaviside truncation of the signal covariance (text after
  eq 9): per ell, in the eigenbasis of the 3x3 block S_l (eq 10),
      u = (S_bar + U)(S_bar + xi)^-1 t_hat,  S_bar + U = max(S_j, mu),
      xi = mu + tau,
  i.e. the filter max(S_j, mu) / (max(S_j, mu) + tau);
* eq 9, rewritten without N_bar^-1 (which also covers the N_bar = 0 corner
  case of Sec. 2.1):  t = u_x + T N^-1 (d - u_x) = K u_x + b,
  K = 1 - T N^-1, b = T N^-1 d, with N^-1 = 0 in masked pixels;
* Algorithm 1's loop: t_0 = d; each iteration is  t_hat = A t,
  u = F^mu t_hat, u_x = Y u, t = K u_x + b;  xi is cooled geometrically
  until mu = 0.  The cooling uses lambda_k = xi_k / tau, geometric from
  lambda_0 down to exactly 1 over the given number of steps, with a fixed
  number of iterations per step;
* the paper's own stopping rule (Algorithm 1, Sec. 3.2): per cooling step
  iterate until the Cauchy ratio drops below a threshold that is itself
  cooled by a factor eta per step, xi <- beta xi until mu = 0;
* diagnostics: the Cauchy ratio of Algorithm 1's stopping rule, the residual
  ||A x - y|| / ||y|| with A = 1 + S^1/2 N^-1 S^1/2 (Appendix C; here
  x = S^-1/2 u, y = S^1/2 Y^T N^-1 d) and the chi^2 of eq 3;
* constrained realizations, eq 19: s_CR = W(d - d_hat) + s_hat;
* Appendix A's refinement (modified Jacobi relaxation), in the form that
  carries over to the sphere: corrections s += W~(W Y r) with r the
  residual of the Wiener filter equation on the range of S (refine());
* the hierarchical framework's adaptive working resolution (text after
  eq 9, Sec. 4): at truncation mu only the scales up to ell_iter(mu) carry
  signal information, and the transforms of that cooling step run with a
  band limit a little above it (adaptive= in solve() and solve_eps()).
"""

import numpy as np

from .geometry import pixel_weights
from .sht import alm_dot, lm_arrays


# ----------------------------------------------------------------------------
# setup (eq 4, Algorithm 1 initialisation)
# ----------------------------------------------------------------------------
def observed(obs, npix):
    """Per-component observation indicator [3, npix] bool.  obs: None (all
    observed), a common mask [npix], a pair (obs_t, obs_p) of a temperature
    and a polarization mask (Q and U share obs_p), or [3, npix]."""
    if obs is None:
        return np.ones((3, npix), dtype=bool)
    if isinstance(obs, (tuple, list)):
        ot, op = (np.asarray(x, dtype=bool).reshape(npix) for x in obs)
        return np.stack([ot, op, op])
    o = np.asarray(obs, dtype=bool)
    return np.broadcast_to(o.reshape(-1, npix), (3, npix)).copy()


SYM6 = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))


def noise_blocks(ncov6):
    """[6, npix] in the order (II, IQ, IU, QQ, QU, UU) -> N [npix, 3, 3]."""
    N = np.zeros((ncov6.shape[1], 3, 3))
    for k, (i, j) in enumerate(SYM6):
        N[:, i, j] = ncov6[k]
        N[:, j, i] = ncov6[k]
    return N


def pix_apply(M, x):
    """Per-pixel operator on maps [..., 3, npix]: M is diagonal [3, npix]
    or a 3x3 block per pixel [3, 3, npix]."""
    if M.ndim == 2:
        return M * x
    return np.einsum("fgp,...gp->...fp", M, x)


def setup(grid, ncov, obs, d):
    """ncov: per-pixel noise covariance, diagonal [3, npix] (II, QQ, UU) or
    the symmetric 3x3 block of eq 11 [6, npix] (II, IQ, IU, QQ, QU, UU);
    obs: see observed(); d [..., 3, npix].

    Masks follow Appendix B: with N_p = Sigma C Sigma and Sigma^-1 = 0 on
    the unobserved components, the inverse noise covariance P_p is the
    block of N_p^-1 on the observed components, zero elsewhere (for a
    diagonal N_p simply 1 / N_pf on observed components).  The messenger
    variance uses alpha_p = 1 / lambda_max(P_p): the smallest eigenvalue of
    N_p when all components are observed, and its limit as the unobserved
    variances go to infinity at fixed correlations otherwise.  Appendix B's
    messenger equation t = (N_bar^-1 + T^-1)^-1 (T^-1 u_x + N_bar^-1 d)
    with N_bar = N - T reduces to t = K u_x + b, K = 1 - T_p P_p,
    b = T_p P_p d0.

    Returns dict(tau, K, b, ninv = P, tn = T_p P, d0 = d zeroed on
    unobserved components, obs = [3, npix] indicator); K, ninv and tn are
    [3, npix] for diagonal noise and [3, 3, npix] otherwise."""
    npix = grid["npix"]
    w = pixel_weights(grid)
    o = observed(obs, npix)
    seen = o.any(axis=0)
    if ncov.shape[0] == 3:
        ninv = np.where(o, 1.0 / np.where(o, ncov, 1.0), 0.0)
        alpha_p = np.min(np.where(o, ncov, np.inf), axis=0)   # smallest eigenvalue of N_p
    else:
        N = noise_blocks(ncov)
        P = np.zeros_like(N)
        P[seen] = np.linalg.inv(N[seen])
        P *= o.T[:, :, None] & o.T[:, None, :]
        alpha_p = np.full(npix, np.inf)
        alpha_p[seen] = 1.0 / np.linalg.eigvalsh(P[seen])[:, -1]
        ninv = np.moveaxis(P, 0, -1)
    tau = float(np.min(alpha_p[seen] * w[seen]))
    Tp = tau / w
    tn = Tp * ninv
    K = (1.0 - tn) if ninv.ndim == 2 else (np.eye(3)[:, :, None] - tn)
    d0 = np.where(o, d, 0.0)
    b = pix_apply(tn, d0)
    return dict(tau=tau, K=K, b=b, ninv=ninv, tn=tn, d0=d0, obs=o)


# ----------------------------------------------------------------------------
# per-ell filters (eq 8 with the Heaviside truncation)
# ----------------------------------------------------------------------------
def signal_blocks(cl):
    """cl [4, lmax+1] in the order TT, EE, BB, TE -> (S2 [l, 2, 2], BB [l])."""
    TT, EE, BB, TE = cl
    S2 = np.stack([np.stack([TT, TE], -1), np.stack([TE, EE], -1)], -2)
    return S2, BB


def matrix_function(cl, fn):
    """Apply a scalar function to the eigenvalues of each S_l (eq 10):
    returns (FTT, FTE, FEE, FBB)."""
    S2, BB = signal_blocks(cl)
    vals, vecs = np.linalg.eigh(S2)
    fv = fn(vals)
    M = np.einsum("lij,lj,lkj->lik", vecs, fv, vecs)
    return M[:, 0, 0], M[:, 0, 1], M[:, 1, 1], fn(BB)


def messenger_filter(cl, mu, tau):
    """F_l = R^T diag(max(S_j, mu) / (max(S_j, mu) + tau)) R."""
    return matrix_function(cl, lambda s: np.maximum(s, mu) / (np.maximum(s, mu) + tau))


def apply_blocks(F, a, lmax):
    """u = F a per (l, m) with the 3x3 (TE block + B) matrix of each l."""
    FTT, FTE, FEE, FBB = F
    ls, _ = lm_arrays(lmax)
    u = np.empty_like(a)
    u[0] = FTT[ls] * a[0] + FTE[ls] * a[1]
    u[1] = FTE[ls] * a[0] + FEE[ls] * a[1]
    u[2] = FBB[ls] * a[2]
    return u


# ----------------------------------------------------------------------------
# adaptive working resolution (text after eq 9; Sec. 4)
# ----------------------------------------------------------------------------
def prior_top_eigenvalue(cl):
    """Largest eigenvalue of each S_l (the TE block and BB), [lmax+1]."""
    S2, BB = signal_blocks(cl)
    return np.maximum(np.linalg.eigvalsh(S2)[:, -1], BB)


def ell_iter(cl, mu):
    """The largest l whose prior S_l has an eigenvalue >= mu: above it the
    prior clamped at mu (the truncation of the text after eq 9) is mu 1 in
    every field, so the filter is the constant mu / (mu + tau) and carries no
    signal information; -1 if there is no such l."""
    top = prior_top_eigenvalue(cl)
    idx = np.nonzero(top >= mu)[0]
    return int(idx[-1]) if idx.size else -1


def working_lmax(cl, mu, lmax, factor):
    """Band limit of the transforms at truncation mu: slightly above
    ell_iter (Sec. 4: the working resolution follows ell_iter with its
    Nyquist frequency a little higher), L = min(lmax, max(2, ceil(factor
    ell_iter))) for factor >= 1."""
    li = ell_iter(cl, mu)
    return int(min(lmax, max(2, int(np.ceil(factor * li - 1e-9)))))


def schedule(lambda0, nsteps):
    """lambda_k = lambda0^(1 - k/(K-1)), k = 0..K-1; the last one is 1."""
    if nsteps <= 1:
        return np.ones(max(nsteps, 1))
    k = np.arange(nsteps)
    lam = float(lambda0) ** (1.0 - k / (nsteps - 1))
    lam[-1] = 1.0
    return lam


# ----------------------------------------------------------------------------
# the iteration (Algorithm 1)
# ----------------------------------------------------------------------------
def diagnostics_recorder(sht, d, ncov, obs, cl, every):
    """Per-iteration record of the diagnostics (Fig. 4): after iteration i
    (counted from 1) whenever i is a multiple of ``every`` and after the
    last one, the chi^2 of eq 3 and the Appendix C residual of the iterate
    u_i.  Returns (record(u, i, last), the dict of lists it fills)."""
    out = dict(iteration=[], chi2=[], residual=[])

    def record(u, i, last):
        if every <= 0 or not (i % every == 0 or last):
            return
        out["iteration"].append(i)
        out["chi2"].append(chi2(sht, u, d, ncov, obs, cl))
        out["residual"].append(residual(sht, u, d, ncov, obs, cl))
    return record, out


def adaptive_lcuts(cl, lambdas, tau, lmax, factor):
    """Per cooling step the working band limit (working_lmax at mu_k =
    (lambda_k - 1) tau); factor 0 = the full band throughout."""
    if not factor:
        return None
    return [working_lmax(cl, (lam - 1.0) * tau, lmax, factor) for lam in lambdas]


def solve(sht, d, ncov, obs, cl, lambda0, nsteps, iters_per_step, trace=False, diagnostics_every=0,
          adaptive=0.0):
    """Run the dual messenger loop.  Returns dict(u [3, nalm], ux = Y u
    [3, npix], tau, cauchy (last), trace (list of per-iteration cauchy),
    diagnostics (with diagnostics_every > 0: iteration, chi2, residual
    lists, see diagnostics_recorder), lcuts (with adaptive = factor >= 1:
    the working band limit of each cooling step, adaptive_lcuts))."""
    st = setup(sht.grid, ncov, obs, d)
    record, diag = diagnostics_recorder(sht, d, ncov, obs, cl, diagnostics_every)
    lams = schedule(lambda0, nsteps)
    lcuts = adaptive_lcuts(cl, lams, st["tau"], sht.lmax, adaptive)
    u, ux, cauchy = messenger_run_counts(sht, st["d0"], st["K"], st["b"], st["tau"], cl, lams,
                                         [iters_per_step] * len(lams), record=record, lcuts=lcuts)
    return dict(u=u, ux=ux, tau=st["tau"], cauchy=cauchy[-1] if cauchy else float("nan"),
                trace=cauchy if trace else None, setup=st, diagnostics=diag if diagnostics_every > 0 else None,
                lcuts=lcuts)


def messenger_run(sht, t, K, b, tau, cl, lambda0, nsteps, iters_per_step):
    """Algorithm 1's loop under the fixed schedule from the messenger t,
    with the pixel update t = K u_x + b.  Returns (u, u_x = Y u, the
    per-iteration Cauchy ratios)."""
    lams = schedule(lambda0, nsteps)
    return messenger_run_counts(sht, t, K, b, tau, cl, lams, [iters_per_step] * len(lams))


def band_limited(F, L):
    """The filter F with its rows above l = L set to zero: u = P_L F t_hat,
    the harmonic update restricted to the working band limit L."""
    out = tuple(np.array(f, dtype=float) for f in F)
    for f in out:
        f[L + 1:] = 0.0
    return out


def messenger_run_counts(sht, t, K, b, tau, cl, lambdas, counts, record=None, lcuts=None):
    """The same loop with counts[k] iterations at cooling step k (lambda =
    lambdas[k]); record (optional) is called as record(u_i, i, last) after
    each iteration's harmonic update; lcuts (optional) gives each step's
    working band limit L_k (band_limited; None or L_k >= lmax: the full
    band)."""
    lmax = sht.lmax
    u_prev = None
    cauchy = []
    u = ux = None
    total, i = sum(counts), 0
    for k, (lam, count) in enumerate(zip(lambdas, counts)):
        mu = (lam - 1.0) * tau
        F = messenger_filter(cl, mu, tau)
        if lcuts is not None and lcuts[k] < lmax:
            F = band_limited(F, lcuts[k])
        for _ in range(count):
            t_hat = sht.analysis(t)
            u = apply_blocks(F, t_hat, lmax)
            i += 1
            if record is not None:
                record(u, i, i == total)
            ux = sht.synthesis(u)
            t = pix_apply(K, ux) + b
            if u_prev is not None:
                cauchy.append(cauchy_ratio(u, u_prev, lmax))
            u_prev = u
    return u, ux, cauchy


def eps_schedule(lambda0, beta):
    """The cooling of Algorithm 1 driven to its end: xi <- beta xi, i.e.
    lambda_j = lambda0 beta^j while it is above 1, then a last step at
    lambda = 1 (mu = 0)."""
    lam = []
    v = float(lambda0)
    while v > 1.0:
        lam.append(v)
        v *= beta
    lam.append(1.0)
    return np.array(lam)


def eps_thresholds(nsteps, eps_start, eps_end, eta):
    """The cooled Cauchy threshold of Sec. 3.2: relaxed by eta per cooling
    step, eps_j = max(eps_end, eps_start eta^-j), and eps_end at the last
    step (lambda = 1)."""
    eps = np.maximum(eps_end, eps_start * float(eta) ** -np.arange(nsteps, dtype=float))
    eps[-1] = eps_end
    return eps


def solve_eps(sht, d, ncov, obs, cl, lambda0, beta, eps_start, eps_end, eta, max_iters, diagnostics_every=0,
              adaptive=0.0):
    """Algorithm 1 with its stopping rule: at each cooling step repeat the
    iteration until ||u_i - u_{i-1}|| / ||u_i|| < eps_j (u_0 = 0, so every
    step runs at least one iteration), then cool; stop early once max_iters
    iterations have run in total.  Returns dict(u, ux, tau, iterations,
    trace = per-iteration Cauchy ratios, steps = cooling step of each
    iteration, diagnostics as in solve())."""
    lmax = sht.lmax
    record, diag = diagnostics_recorder(sht, d, ncov, obs, cl, diagnostics_every)
    st = setup(sht.grid, ncov, obs, d)
    tau, K, b = st["tau"], st["K"], st["b"]
    t = st["d0"].copy()
    u_prev = np.zeros((3, lm_arrays(lmax)[0].size), dtype=complex)
    lams = eps_schedule(lambda0, beta)
    eps = eps_thresholds(len(lams), eps_start, eps_end, eta)
    lcuts = adaptive_lcuts(cl, lams, tau, lmax, adaptive)
    trace, steps = [], []
    u = ux = None
    for j, lam in enumerate(lams):
        F = messenger_filter(cl, (lam - 1.0) * tau, tau)
        if lcuts is not None and lcuts[j] < lmax:
            F = band_limited(F, lcuts[j])
        while len(trace) < max_iters:
            t_hat = sht.analysis(t)
            u = apply_blocks(F, t_hat, lmax)
            ux = sht.synthesis(u)
            t = pix_apply(K, ux) + b
            c = cauchy_ratio(u, u_prev, lmax)
            trace.append(c)
            steps.append(j)
            u_prev = u
            last = (c < eps[j] and j == len(lams) - 1) or len(trace) >= max_iters
            record(u, len(trace), last)
            if c < eps[j]:
                break
        if len(trace) >= max_iters:
            break
    return dict(u=u, ux=ux, tau=tau, iterations=len(trace), trace=trace, steps=steps, lambdas=lams, eps=eps,
                diagnostics=diag if diagnostics_every > 0 else None, lcuts=lcuts)


# ----------------------------------------------------------------------------
# diagnostics (Appendix C residual, eq 3 chi^2)
# ----------------------------------------------------------------------------
def residual(sht, u, d, ncov, obs, cl, ux=None):
    """||A x - y|| / ||y||, A = 1 + S^1/2 Y^T N^-1 Y S^1/2, x = S^+1/2 u,
    y = S^1/2 Y^T N^-1 d (pseudo-inverse on the zero modes of S)."""
    lmax = sht.lmax
    st = setup(sht.grid, ncov, obs, d)
    ninv, d0 = st["ninv"], st["d0"]
    if ux is None:
        ux = sht.synthesis(u)
    half = matrix_function(cl, lambda s: np.sqrt(np.maximum(s, 0.0)))
    ihalf = matrix_function(cl, lambda s: np.where(s > 0, 1.0 / np.sqrt(np.where(s > 0, s, 1.0)), 0.0))
    r = apply_blocks(ihalf, u, lmax) + apply_blocks(half, sht.adjoint(pix_apply(ninv, ux - d0)), lmax)
    y = apply_blocks(half, sht.adjoint(pix_apply(ninv, d0)), lmax)
    nr = sum(alm_dot(r[f], r[f], lmax) for f in range(3))
    ny = sum(alm_dot(y[f], y[f], lmax) for f in range(3))
    return float(np.sqrt(nr / ny))


def chi2(sht, u, d, ncov, obs, cl, ux=None):
    """(d - Y u)^T N^-1 (d - Y u) + u^dagger S^+ u."""
    lmax = sht.lmax
    st = setup(sht.grid, ncov, obs, d)
    if ux is None:
        ux = sht.synthesis(u)
    res = st["d0"] - ux
    sinv = matrix_function(cl, lambda s: np.where(s > 0, 1.0 / np.where(s > 0, s, 1.0), 0.0))
    su = apply_blocks(sinv, u, lmax)
    return float(np.sum(res * pix_apply(st["ninv"], res)) + sum(alm_dot(u[f], su[f], lmax) for f in range(3)))


def cauchy_ratio(u, u_prev, lmax):
    """||u_i - u_{i-1}|| / ||u_i||, harmonic L2 over T, E, B (Algorithm 1's
    stopping rule, applied to the iterate u)."""
    num = sum(alm_dot(u[f] - u_prev[f], u[f] - u_prev[f], lmax) for f in range(3))
    den = sum(alm_dot(u[f], u[f], lmax) for f in range(3))
    return float(np.sqrt(num / den)) if den > 0 else 0.0


# ----------------------------------------------------------------------------
# refinement by the modified Jacobi relaxation (Appendix A)
# ----------------------------------------------------------------------------
def prior_pinv(cl):
    """S^+ per l: the pseudo-inverse of the TE block and of BB (zero where
    the spectrum is zero)."""
    return matrix_function(cl, lambda s: np.where(s > 0, 1.0 / np.where(s > 0, s, 1.0), 0.0))


def prior_range(cl):
    """Pi per l: the orthogonal projector onto the range of S_l."""
    return matrix_function(cl, lambda s: (s > 0).astype(float))


def wf_residual(sht, s, st, cl):
    """r = Pi Y^T P (d0 - Y s) - S^+ s, the residual of the Wiener filter
    equation (S^+ + Pi Y^T P Y) s = Pi Y^T P d on the range of S (eq 2 in
    the form (1 + S Y^T P Y) s = S Y^T P d, multiplied by S^+)."""
    lmax = sht.lmax
    e = sht.adjoint(pix_apply(st["ninv"], st["d0"] - sht.synthesis(s)))
    return apply_blocks(prior_range(cl), e, lmax) - apply_blocks(prior_pinv(cl), s, lmax)


def refine(sht, d, ncov, obs, cl, lambda0, nsteps, iters, ncorr, select="last"):
    """Appendix A's relaxation on the sphere: s_0 = W~ d (the fixed-schedule
    messenger run of solve()), then ncorr corrections
        s_{n+1} = s_n + W~(g_n),  g_n = W Y r_n,  r_n = wf_residual(s_n),
    where W~(g) is the same messenger run (schedule and counts) driven by
    weighted data g in place of P d, b = T_p g, from t_0 = 0: one linear
    operator for every correction.  (Started from P^+ g, the pseudo-inverse
    image that t_0 = d0 is for g = P d, a short run's transient overshoots
    where N_p has large eigenvalues, and the corrections diverge with
    correlated noise.)
    W Y is a right inverse of the adjoint Y^T where the quadrature is exact,
    so g_n stands for the data whose Wiener filter is A^-1 r_n; the paper's
    flat-sky form (data minus W^+ s_n) needs a square, unitary basis change.
    The fixed point has r = 0 whenever Y^T W Y is invertible, whatever the
    grid and W~.  The corrections converge only where W~ is close enough to
    the inverse.  Appendix A's relaxation returns its last iterate
    (select="last"); select="best" returns instead the iterate with the
    smallest residual norm (the first of equal ones), never worse than s_0
    where the corrections diverge.  Returns dict(u, history = ||r_n|| /
    ||Pi Y^T P d0|| before each correction and after the last, best = the
    index of the smallest entry of that history, chosen = the index of u)."""
    st = setup(sht.grid, ncov, obs, d)
    lams = schedule(lambda0, nsteps)
    counts = [iters] * len(lams)
    s0 = messenger_run_counts(sht, st["d0"], st["K"], st["b"], st["tau"], cl, lams, counts)[0]
    return corrections(sht, st, cl, s0, lams, counts, ncorr, select)


def refine_eps(sht, d, ncov, obs, cl, lambda0, beta, eps_start, eps_end, eta, max_iters, ncorr, select="last"):
    """Appendix A's prescription under Algorithm 1's stopping rule: the first
    solve runs with the Cauchy rule (solve_eps), the iterations it spent at
    each cooling step are recorded, and every correction runs those counts
    (so that W~ is one fixed operator).  Returns refine()'s dict plus
    counts."""
    r0 = solve_eps(sht, d, ncov, obs, cl, lambda0, beta, eps_start, eps_end, eta, max_iters)
    lams = r0["lambdas"]
    counts = [r0["steps"].count(k) for k in range(len(lams))]
    st = setup(sht.grid, ncov, obs, d)
    out = corrections(sht, st, cl, r0["u"], lams, counts, ncorr, select)
    out["counts"] = counts
    return out


def corrections(sht, st, cl, s, lambdas, counts, ncorr, select="last"):
    """The corrections of refine() from s_0 = s, W~ = the messenger run with
    counts[k] iterations at lambdas[k]."""
    lmax = sht.lmax
    tau, K = st["tau"], st["K"]
    w = pixel_weights(sht.grid)
    Tp = tau / w
    y = apply_blocks(prior_range(cl), sht.adjoint(pix_apply(st["ninv"], st["d0"])), lmax)
    ny = np.sqrt(sum(alm_dot(y[f], y[f], lmax) for f in range(3)))

    def rel_norm(r):
        return float(np.sqrt(sum(alm_dot(r[f], r[f], lmax) for f in range(3))) / ny)

    hist, iterates = [], []
    for _ in range(ncorr):
        r = wf_residual(sht, s, st, cl)
        hist.append(rel_norm(r))
        iterates.append(s)
        g = w * sht.synthesis(r)
        delta = messenger_run_counts(sht, np.zeros_like(g), K, Tp * g, tau, cl, lambdas, counts)[0]
        s = s + delta
    hist.append(rel_norm(wf_residual(sht, s, st, cl)))
    iterates.append(s)
    best = int(np.argmin(hist))
    if select not in ("last", "best"):
        raise ValueError(f"select must be 'last' or 'best', not {select!r}")
    chosen = best if select == "best" else len(iterates) - 1
    return dict(u=iterates[chosen], history=hist, best=best, chosen=chosen)


# ----------------------------------------------------------------------------
# constrained realizations (eq 19)
# ----------------------------------------------------------------------------
def constrained_realization(sht, d, dhat, shat, ncov, obs, cl, lambda0, nsteps, iters):
    """s_CR = W(d - d_hat) + s_hat, one messenger run on d - d_hat."""
    r = solve(sht, d - dhat, ncov, obs, cl, lambda0, nsteps, iters)
    return r["u"] + shat
