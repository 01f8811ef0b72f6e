"""Dense linear algebra for tiny maps (oracle; test infrastructure only).

A real field's harmonic coefficients are mapped to real coordinates x in
which the prior is diagonal per coordinate block: for each (l, m = 0) one
coordinate Re a_l0, for each (l, m > 0) two coordinates sqrt(2) Re a_lm and
sqrt(2) Im a_lm, so that |x|^2 = sum over l and m = -l..l of |a_lm|^2.  In
these coordinates:

* the dense synthesis matrix Y has one column per coordinate (the map of the
  corresponding unit coefficient vector);
* the exact Wiener filter (eq 2, written as (1 + S Y^T N^-1 Y) x = S Y^T N^-1 d
  so that a singular S is allowed) is a direct linear solve;
* the messenger fixed point at mu = 0 (eqs 8-9 at convergence) solves
  (1 - F A Y + F A T N^-1 Y) u = F A T N^-1 d  with A = Y^T W.
"""

import numpy as np

from .geometry import pixel_weights
from .sht import lm_arrays, nalm
from .dm import setup, messenger_filter


def pixel_matrix(M):
    """Dense [3 npix, 3 npix] of a per-pixel operator (diagonal [3, npix]
    or 3x3 blocks [3, 3, npix]) in the map ordering (component-major)."""
    if M.ndim == 2:
        return np.diag(M.reshape(-1))
    npix = M.shape[-1]
    D = np.zeros((3 * npix, 3 * npix))
    p = np.arange(npix)
    for f in range(3):
        for g in range(3):
            D[f * npix + p, g * npix + p] = M[f, g]
    return D


def coords(lmax):
    """List of (field, l, m, part) for every real coordinate; part 0 = Re,
    1 = Im.  E and B start at l = 2."""
    out = []
    ls, ms = lm_arrays(lmax)
    for f in range(3):
        for l, m in zip(ls, ms):
            if f > 0 and l < 2:
                continue
            out.append((f, l, m, 0))
            if m > 0:
                out.append((f, l, m, 1))
    return out


def x_to_alm(x, lmax):
    cs = coords(lmax)
    a = np.zeros((3, nalm(lmax)), dtype=np.complex128)
    ls, ms = lm_arrays(lmax)
    idx = {(l, m): k for k, (l, m) in enumerate(zip(ls, ms))}
    for v, (f, l, m, p) in zip(x, cs):
        k = idx[(l, m)]
        if m == 0:
            a[f, k] += v
        elif p == 0:
            a[f, k] += v / np.sqrt(2.0)
        else:
            a[f, k] += 1j * v / np.sqrt(2.0)
    return a


def alm_to_x(a, lmax):
    cs = coords(lmax)
    ls, ms = lm_arrays(lmax)
    idx = {(l, m): k for k, (l, m) in enumerate(zip(ls, ms))}
    x = np.empty(len(cs))
    for j, (f, l, m, p) in enumerate(cs):
        v = a[f, idx[(l, m)]]
        if m == 0:
            x[j] = v.real
        elif p == 0:
            x[j] = np.sqrt(2.0) * v.real
        else:
            x[j] = np.sqrt(2.0) * v.imag
    return x


def synthesis_matrix(sht):
    """Dense Y [3 npix, ncoord]: column j = Y applied to unit coordinate j."""
    lmax = sht.lmax
    cs = coords(lmax)
    cols = []
    for j in range(len(cs)):
        e = np.zeros(len(cs))
        e[j] = 1.0
        cols.append(sht.synthesis(x_to_alm(e, lmax)).reshape(-1))
    return np.stack(cols, axis=1)


def prior_matrix(cl, lmax):
    """Dense S in x coordinates: C^{XY}_l between the T/E coordinates of the
    same (l, m, part), C^BB_l on B."""
    TT, EE, BB, TE = cl
    cs = coords(lmax)
    pos = {c: j for j, c in enumerate(cs)}
    S = np.zeros((len(cs), len(cs)))
    for j, (f, l, m, p) in enumerate(cs):
        if f == 0:
            S[j, j] = TT[l]
            if (1, l, m, p) in pos:
                S[j, pos[(1, l, m, p)]] = TE[l]
        elif f == 1:
            S[j, j] = EE[l]
            S[j, pos[(0, l, m, p)]] = TE[l]
        else:
            S[j, j] = BB[l]
    return S


def filter_matrix(F, lmax):
    FTT, FTE, FEE, FBB = F
    cs = coords(lmax)
    pos = {c: j for j, c in enumerate(cs)}
    M = np.zeros((len(cs), len(cs)))
    for j, (f, l, m, p) in enumerate(cs):
        if f == 0:
            M[j, j] = FTT[l]
            if (1, l, m, p) in pos:
                M[j, pos[(1, l, m, p)]] = FTE[l]
        elif f == 1:
            M[j, j] = FEE[l]
            M[j, pos[(0, l, m, p)]] = FTE[l]
        else:
            M[j, j] = FBB[l]
    return M


def wiener_filter(sht, d, ncov, obs, cl, Y=None):
    """Exact WF (eq 2) of the pixelised problem; returns packed alm."""
    lmax = sht.lmax
    Y = synthesis_matrix(sht) if Y is None else Y
    st = setup(sht.grid, ncov, obs, d)
    NI = pixel_matrix(st["ninv"])
    S = prior_matrix(cl, lmax)
    YtN = Y.T @ NI
    lhs = np.eye(S.shape[0]) + S @ (YtN @ Y)
    rhs = S @ (YtN @ st["d0"].reshape(-1))
    return x_to_alm(np.linalg.solve(lhs, rhs), lmax)


def messenger_fixed_point(sht, d, ncov, obs, cl, Y=None):
    """Fixed point of the messenger iteration at mu = 0 (the limit the
    method reaches on a grid where A Y != 1); returns packed alm."""
    lmax = sht.lmax
    Y = synthesis_matrix(sht) if Y is None else Y
    st = setup(sht.grid, ncov, obs, d)
    w = np.tile(pixel_weights(sht.grid), 3)
    A = Y.T * w[None, :]
    F = filter_matrix(messenger_filter(cl, 0.0, st["tau"]), lmax)
    TN = pixel_matrix(st["tn"])
    FA = F @ A
    lhs = np.eye(F.shape[0]) - FA @ Y + FA @ (TN @ Y)
    rhs = FA @ (TN @ st["d0"].reshape(-1))
    return x_to_alm(np.linalg.solve(lhs, rhs), lmax)


def posterior_covariance(sht, ncov, obs, cl, Y=None):
    """(S^-1 + Y^T N^-1 Y)^-1 on the range of S (eq 18), written as
    (1 + S Y^T N^-1 Y)^-1 S."""
    lmax = sht.lmax
    Y = synthesis_matrix(sht) if Y is None else Y
    st = setup(sht.grid, ncov, obs, np.zeros((3, sht.grid["npix"])))
    S = prior_matrix(cl, lmax)
    lhs = np.eye(S.shape[0]) + S @ ((Y.T @ pixel_matrix(st["ninv"])) @ Y)
    return np.linalg.solve(lhs, S)
