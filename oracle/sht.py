"""Spin-0 + spin-2 spherical harmonic transforms on a ring grid (oracle).

Test infrastructure only.  The paper's basis change is the flat-sky Fourier
transform with the E/B rotation (Sec. 2.1, eqs 12-16, with F F^dagger =
sigma 1).  On the sphere the same role is played by:

* synthesis Y : (a^T, a^E, a^B)_lm -> (I, Q, U) maps, with
      I   = sum_lm a^T_lm  Y_lm
      Q+iU = sum_lm  2a_lm  2Y_lm,   Q-iU = sum_lm -2a_lm -2Y_lm,
      +-2a_lm = -(a^E_lm +- i a^B_lm)          (Zaldarriaga & Seljak 1997)
* adjoint Y^T (plain adjoint, no quadrature weights), for the inner product
  <a, b> = sum_{l, m=-l..l} conj(a_lm) b_lm on harmonic coefficients and the
  real dot product on maps;
* analysis A = Y^T W, W = diag(pixel quadrature weights).

Everything is done with the full m range -lmax..lmax in complex arithmetic,
with a direct per-ring Fourier sum, and with no north/south symmetry.  A real
field stores only m >= 0 ("packed"): idx(l, m) = m (2 lmax + 1 - m) / 2 + l,
and a_{l,-m} = (-1)^m conj(a_lm).
"""

import numpy as np

from .harmonics import spin_lambda


# ----------------------------------------------------------------------------
# packed <-> full harmonic coefficient layouts
# ----------------------------------------------------------------------------
def nalm(lmax):
    return (lmax + 1) * (lmax + 2) // 2


def alm_index(l, m, lmax):
    return m * (2 * lmax + 1 - m) // 2 + l


def lm_arrays(lmax):
    """(l, m) of every packed index, m-major."""
    ls, ms = [], []
    for m in range(lmax + 1):
        for l in range(m, lmax + 1):
            ls.append(l)
            ms.append(m)
    return np.array(ls), np.array(ms)


def to_full(a, lmax):
    """Packed m>=0 coefficients of a real field -> array [l, m + lmax]."""
    ls, ms = lm_arrays(lmax)
    full = np.zeros((lmax + 1, 2 * lmax + 1), dtype=np.complex128)
    full[ls, lmax + ms] = a
    full[ls, lmax - ms] = ((-1.0) ** ms) * np.conj(a)
    return full


def to_packed(full, lmax):
    ls, ms = lm_arrays(lmax)
    return full[ls, lmax + ms].copy()


def alm_dot(a, b, lmax):
    """<a, b> = sum over l and m = -l..l of conj(a) b for real fields given
    in packed form (m > 0 counted twice)."""
    ls, ms = lm_arrays(lmax)
    wt = np.where(ms == 0, 1.0, 2.0)
    return float(np.sum(wt * np.real(np.conj(a) * b)))


# ----------------------------------------------------------------------------
# per-ring Fourier sums
# ----------------------------------------------------------------------------
def ring_synthesis(F, n, phi0, lmax, direct=None):
    """x_j = sum_{m=-lmax..lmax} F_m exp(i m (phi0 + 2 pi j / n)), j < n.

    ``direct=True`` evaluates the sum literally; otherwise the m terms are
    folded modulo n and an inverse FFT (library primitive) is used."""
    ms = np.arange(-lmax, lmax + 1)
    if direct is None:
        direct = n * ms.size <= 65536
    if direct:
        phi = phi0 + 2.0 * np.pi * np.arange(n) / n
        return np.exp(1j * np.outer(phi, ms)) @ F
    c = np.zeros(n, dtype=np.complex128)
    np.add.at(c, np.mod(ms, n), F * np.exp(1j * ms * phi0))
    return np.fft.ifft(c) * n


def ring_analysis(x, n, phi0, lmax, direct=None):
    """G_m = sum_j x_j exp(-i m (phi0 + 2 pi j / n)) for m = -lmax..lmax."""
    ms = np.arange(-lmax, lmax + 1)
    if direct is None:
        direct = n * ms.size <= 65536
    if direct:
        phi = phi0 + 2.0 * np.pi * np.arange(n) / n
        return np.exp(-1j * np.outer(ms, phi)) @ x
    X = np.fft.fft(x)
    return X[np.mod(ms, n)] * np.exp(-1j * ms * phi0)


# ----------------------------------------------------------------------------
# the transform object
# ----------------------------------------------------------------------------
class SHT:
    """Y, Y^T and A = Y^T W on ``grid`` up to ``lmax``.

    The spin Legendre tables of a ring depend only on its colatitude, so they
    are cached when they fit in ``cache_bytes``; otherwise they are recomputed
    per chunk of rings.
    """

    def __init__(self, grid, lmax, cache_bytes=2 << 30, chunk_bytes=256 << 20):
        self.grid = grid
        self.lmax = int(lmax)
        self.ms = np.arange(-self.lmax, self.lmax + 1)
        per_ring = (self.lmax + 1) * self.ms.size * 8 * 3
        nr = len(grid["theta"])
        self.chunk = max(1, min(nr, chunk_bytes // per_ring))
        self._cache = None
        if per_ring * nr <= cache_bytes:
            self._cache = self._tables(np.arange(nr))

    def _tables(self, rings):
        th = self.grid["theta"][rings]
        return (spin_lambda(self.lmax, 0, th, self.ms),
                spin_lambda(self.lmax, 2, th, self.ms),
                spin_lambda(self.lmax, -2, th, self.ms))

    def _chunks(self, rings):
        rings = np.asarray(rings)
        for s in range(0, rings.size, self.chunk):
            rr = rings[s:s + self.chunk]
            if self._cache is not None:
                yield rr, tuple(t[rr] for t in self._cache)
            else:
                yield rr, self._tables(rr)

    # -- synthesis ----------------------------------------------------------
    def synthesis(self, alm, rings=None):
        """alm [3, nalm] (T, E, B) -> maps [3, npix] (I, Q, U).

        With ``rings`` given, returns a list of [3, nphi] arrays for those
        rings only (sampled evaluation)."""
        lmax, g = self.lmax, self.grid
        AT = to_full(alm[0], lmax)
        AE = to_full(alm[1], lmax)
        AB = to_full(alm[2], lmax)
        A2p = -(AE + 1j * AB)
        A2m = -(AE - 1j * AB)
        sampled = rings is not None
        rings = np.arange(len(g["theta"])) if rings is None else np.asarray(rings)
        out = [] if sampled else np.zeros((3, g["npix"]))
        for rr, (l0, l2p, l2m) in self._chunks(rings):
            FT = np.einsum("rlm,lm->rm", l0, AT)
            FP = np.einsum("rlm,lm->rm", l2p, A2p)
            FM = np.einsum("rlm,lm->rm", l2m, A2m)
            for k, r in enumerate(rr):
                n, p0 = int(g["nphi"][r]), g["phi0"][r]
                t = ring_synthesis(FT[k], n, p0, lmax)
                P = ring_synthesis(FP[k], n, p0, lmax)      # Q + iU
                M = ring_synthesis(FM[k], n, p0, lmax)      # Q - iU
                block = np.stack([t.real, (0.5 * (P + M)).real, (0.5 * (P - M) / 1j).real])
                if sampled:
                    out.append(block)
                else:
                    o = int(g["offset"][r])
                    out[:, o:o + n] = block
        return out

    # -- adjoint -----------------------------------------------------------
    def adjoint(self, maps, rings=None):
        """Y^T: maps [3, npix] (I, Q, U) -> alm [3, nalm] (T, E, B).  With
        ``rings`` given, only those rings' terms of the sum (a partial sum,
        for sampled evaluation)."""
        lmax, g = self.lmax, self.grid
        aT = np.zeros((lmax + 1, self.ms.size), dtype=np.complex128)
        a2p = np.zeros_like(aT)
        a2m = np.zeros_like(aT)
        rings = np.arange(len(g["theta"])) if rings is None else np.asarray(rings)
        for rr, (l0, l2p, l2m) in self._chunks(rings):
            GT = np.empty((rr.size, self.ms.size), dtype=np.complex128)
            GP = np.empty_like(GT)
            GM = np.empty_like(GT)
            for k, r in enumerate(rr):
                n, p0, o = int(g["nphi"][r]), g["phi0"][r], int(g["offset"][r])
                I, Q, U = maps[0, o:o + n], maps[1, o:o + n], maps[2, o:o + n]
                GT[k] = ring_analysis(I.astype(np.complex128), n, p0, lmax)
                GP[k] = ring_analysis(Q + 1j * U, n, p0, lmax)
                GM[k] = ring_analysis(Q - 1j * U, n, p0, lmax)
            aT += np.einsum("rlm,rm->lm", l0, GT)
            a2p += np.einsum("rlm,rm->lm", l2p, GP)
            a2m += np.einsum("rlm,rm->lm", l2m, GM)
        aE = -0.5 * (a2p + a2m)
        aB = 0.5j * (a2p - a2m)
        return np.stack([to_packed(aT, lmax), to_packed(aE, lmax), to_packed(aB, lmax)])

    def analysis(self, maps):
        """A = Y^T W: quadrature-weighted adjoint."""
        from .geometry import pixel_weights
        return self.adjoint(maps * pixel_weights(self.grid)[None, :])

    # -- sampled adjoint: only some (l, m) --------------------------------
    def adjoint_modes(self, maps, modes):
        """Y^T evaluated only at the listed (l, m), m >= 0; returns [3, K]."""
        lmax, g = self.lmax, self.grid
        modes = [(int(l), int(m)) for l, m in modes]
        ms_u = sorted(set(m for _, m in modes))
        lhi = max(l for l, _ in modes)
        nr = len(g["theta"])
        GT = np.empty((nr, len(ms_u)), dtype=np.complex128)
        GP = np.empty_like(GT)
        GM = np.empty_like(GT)
        for r in range(nr):
            n, p0, o = int(g["nphi"][r]), g["phi0"][r], int(g["offset"][r])
            I, Q, U = maps[0, o:o + n], maps[1, o:o + n], maps[2, o:o + n]
            phi = p0 + 2.0 * np.pi * np.arange(n) / n
            E = np.exp(-1j * np.outer(ms_u, phi))
            GT[r] = E @ I
            GP[r] = E @ (Q + 1j * U)
            GM[r] = E @ (Q - 1j * U)
        th = g["theta"]
        l0 = spin_lambda(lhi, 0, th, ms_u)
        l2p = spin_lambda(lhi, 2, th, ms_u)
        l2m = spin_lambda(lhi, -2, th, ms_u)
        out = np.zeros((3, len(modes)), dtype=np.complex128)
        for k, (l, m) in enumerate(modes):
            j = ms_u.index(m)
            aT = np.sum(l0[:, l, j] * GT[:, j])
            ap = np.sum(l2p[:, l, j] * GP[:, j])
            am = np.sum(l2m[:, l, j] * GM[:, j])
            out[:, k] = [aT, -0.5 * (ap + am), 0.5j * (ap - am)]
        return out
