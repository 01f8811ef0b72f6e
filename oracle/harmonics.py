"""Wigner-d functions and spin-weighted Legendre functions (oracle).

Test infrastructure only.  Textbook definitions:

* Wigner d^l_{m m'}(theta) via the three-term recurrence in l at fixed
  (m, m'), started from the closed-form edge values at l0 = max(|m|, |m'|):

    l sqrt(((l+1)^2 - m^2)((l+1)^2 - m'^2)) d^{l+1}
        = (2l+1)(l(l+1) cos(theta) - m m') d^l
          - (l+1) sqrt((l^2 - m^2)(l^2 - m'^2)) d^{l-1}

  with  d^j_{m', j} = sqrt((2j)! / ((j+m')! (j-m')!)) c^{j+m'} s^{j-m'},
  c = cos(theta/2), s = sin(theta/2), and the symmetries
  d^j_{a,b} = d^j_{-b,-a},  d^j_{j,m'} = (-1)^{j-m'} d^j_{m',j}.

* Spin-weighted harmonics (Goldberg et al. 1967 convention):
    sY_lm(theta, phi) = (-1)^s sqrt((2l+1)/(4 pi)) d^l_{m,-s}(theta) e^{i m phi}
  so the real "spin Legendre function" is
    slam_lm(theta) = (-1)^s sqrt((2l+1)/(4 pi)) d^l_{m,-s}(theta).
  For s = 0 this is the orthonormal Y_lm with the Condon-Shortley phase.

Edge values of high order underflow double precision near the poles
(sin^m theta), so the recurrence carries each value as a mantissa times
2**e with an integer exponent per entry, and converts back with ldexp at
the end (true underflow then gives 0).  No entry is ever skipped.
"""

import numpy as np
from math import lgamma

_RESCALE_BITS = 256
_BIG = 2.0 ** _RESCALE_BITS


def _edge_log(j, a):
    """log sqrt((2j)! / ((j+a)! (j-a)!)), the edge-value prefactor."""
    return 0.5 * (lgamma(2 * j + 1) - lgamma(j + a + 1) - lgamma(j - a + 1))


def wigner_d(lmax, mp, theta, ms):
    """d^l_{m, mp}(theta) for l = 0..lmax and every m in ``ms``.

    Returns an array of shape (len(theta), lmax + 1, len(ms)); entries with
    l < max(|m|, |mp|) are zero.
    """
    theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    ms = np.atleast_1d(np.asarray(ms, dtype=np.int64))
    nt, nm = theta.size, ms.size
    out = np.zeros((nt, lmax + 1, nm))
    lc = np.log(np.cos(0.5 * theta))[:, None]      # log cos(theta/2)
    ls = np.log(np.sin(0.5 * theta))[:, None]      # log sin(theta/2)
    cost = np.cos(theta)[:, None]

    l0 = np.maximum(np.abs(ms), abs(mp))           # first nonzero l per m
    # edge value at l0 in log form: log|d| = L + pc*log c + ps*log s, sign
    logmag = np.empty((nt, nm))
    sign = np.empty(nm)
    for k, m in enumerate(ms):
        j = int(l0[k])
        if abs(m) >= abs(mp):
            if m >= 0:    # d^j_{j, mp} = (-1)^{j-mp} d^j_{mp, j}
                pref, pc, ps, sg = _edge_log(j, mp), j + mp, j - mp, (-1) ** ((j - mp) % 2)
            else:         # d^j_{-j, mp} = d^j_{-mp, j}
                pref, pc, ps, sg = _edge_log(j, -mp), j - mp, j + mp, 1
        else:
            if mp >= 0:   # d^j_{m, j}
                pref, pc, ps, sg = _edge_log(j, m), j + m, j - m, 1
            else:         # d^j_{m, -j} = (-1)^{j+m} d^j_{-m, j}
                pref, pc, ps, sg = _edge_log(j, -m), j - m, j + m, (-1) ** ((j + m) % 2)
        lm = pref + pc * lc[:, 0] + ps * ls[:, 0]
        logmag[:, k] = lm
        sign[k] = sg
    # mantissa / exponent representation of the edge value
    e_seed = np.floor(logmag / np.log(2.0)).astype(np.int64)
    m_seed = sign[None, :] * np.exp(logmag - e_seed * np.log(2.0))

    prev = np.zeros((nt, nm))      # d^{l-1} mantissa
    cur = np.zeros((nt, nm))       # d^{l} mantissa
    expo = np.zeros((nt, nm), dtype=np.int64)
    mm = ms.astype(np.float64)[None, :]
    mpf = float(mp)
    for l in range(lmax + 1):
        start = (l0 == l)[None, :]
        if l >= 1:
            lp = float(l - 1)               # step l-1 -> l
            active = (l0 <= l - 1)[None, :]
            if l - 1 == 0:
                # only m = mp = 0 reaches here: d^1_{00} = cos(theta)
                nxt = cost * np.ones((1, nm))
            else:
                den = lp * np.sqrt(np.maximum(((lp + 1) ** 2 - mm ** 2) * ((lp + 1) ** 2 - mpf ** 2), 0.0))
                a = (2 * lp + 1) * (lp * (lp + 1) * cost - mm * mpf)
                b = (lp + 1) * np.sqrt(np.maximum((lp ** 2 - mm ** 2) * (lp ** 2 - mpf ** 2), 0.0))
                with np.errstate(divide="ignore", invalid="ignore"):
                    nxt = (a * cur - b * prev) / den
            nxt = np.where(active, nxt, 0.0)
            prev = np.where(active, cur, prev)
            cur = nxt
            # keep mantissas bounded: values only grow out of an underflow
            big = np.abs(cur) > _BIG
            if big.any():
                cur = np.where(big, cur / _BIG, cur)
                prev = np.where(big, prev / _BIG, prev)
                expo = expo + big * _RESCALE_BITS
        cur = np.where(start, m_seed, cur)
        prev = np.where(start, 0.0, prev)
        expo = np.where(start, e_seed, expo)
        val = np.ldexp(cur, np.clip(expo, -100000, 100000).astype(np.int32))
        out[:, l, :] = np.where((l0 <= l)[None, :], val, 0.0)
    return out


def spin_lambda(lmax, s, theta, ms):
    """Real spin-s Legendre functions slam_lm(theta), shape (nθ, lmax+1, nm):
    sY_lm(theta, phi) = slam_lm(theta) e^{i m phi}  (Goldberg convention)."""
    d = wigner_d(lmax, -s, theta, ms)
    ell = np.arange(lmax + 1, dtype=np.float64)
    norm = ((-1.0) ** s) * np.sqrt((2 * ell + 1) / (4 * np.pi))
    out = d * norm[None, :, None]
    if s != 0:
        out[:, :abs(s), :] = 0.0        # spin-s harmonics vanish for l < |s|
    return out


def goldberg_sylm(s, l, m, theta, phi):
    """Explicit finite-sum spin harmonic sY_lm(theta, phi) of Goldberg et al.
    (1967) -- an independent route used to pin ``spin_lambda``:

    sY_lm = (-1)^m sqrt((l+m)!(l-m)!(2l+1) / (4 pi (l+s)!(l-s)!))
            sin^{2l}(theta/2) sum_r C(l-s, r) C(l+s, r+s-m) (-1)^{l-r-s}
            e^{i m phi} cot^{2r+s-m}(theta/2)
    """
    from math import comb, factorial
    theta = np.asarray(theta, dtype=np.float64)
    pref = ((-1.0) ** m) * np.sqrt(factorial(l + m) * factorial(l - m) * (2 * l + 1)
                                   / (4 * np.pi * factorial(l + s) * factorial(l - s)))
    cot = 1.0 / np.tan(0.5 * theta)
    tot = np.zeros_like(theta)
    for r in range(0, l - s + 1):
        k2 = r + s - m
        if k2 < 0 or k2 > l + s:
            continue
        tot = tot + comb(l - s, r) * comb(l + s, k2) * ((-1.0) ** (l - r - s)) * cot ** (2 * r + s - m)
    return pref * np.sin(0.5 * theta) ** (2 * l) * tot * np.exp(1j * m * np.asarray(phi))
