"""GPU parity of the split ring transforms on small grids.

A ring of length n = 4 i whose Bluestein buffer would exceed the plan's
limit is transformed as four length-i transforms joined by a radix-4 step
(needed at Nside 2048).  DMWF_FFT_MAX_ELEMS, read when a plan is made,
lowers the limit so that small grids take that path for most of their
rings: transforms and messenger iterations must then match the oracle to
FP64 rounding (1e-12), on the FP64 vector path, the batched FP64
matrix-core path (9 RHS: a full column tile and a ragged one) and, within
1e-6, the mixed path.
"""

import numpy as np
import pytest

from oracle import dm
from oracle.geometry import gl_grid, healpix_grid
from oracle.sht import SHT, alm_dot, lm_arrays, nalm
from paper_1801_05358_amd import inputs

pytestmark = pytest.mark.gpu

SPECS = [("hp", 8, 16, 32), ("hp", 40, 60, 32), ("hp", 40, 60, 256), ("gl", (17, 36), 16, 32)]
IDS = [f"{k}{g}-l{l}-max{e}" for k, g, l, e in SPECS]


@pytest.fixture(scope="module")
def dmwf():
    from paper_1801_05358_amd import dmwf as mod
    assert mod.device_count() > 0, "no GPU visible"
    return mod


def rand_alm(lmax, rng, nrhs):
    n = nalm(lmax)
    ls, ms = lm_arrays(lmax)
    a = rng.standard_normal((nrhs, 3, n)) + 1j * rng.standard_normal((nrhs, 3, n))
    a[..., ms == 0] = a[..., ms == 0].real
    a[..., 1:, ls < 2] = 0
    return a


def rel_alm(a, b, lmax):
    num = sum(alm_dot(a[f] - b[f], a[f] - b[f], lmax) for f in range(3))
    den = sum(alm_dot(b[f], b[f], lmax) for f in range(3))
    return float(np.sqrt(num / den))


def rel_map(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def make(spec, dmwf, monkeypatch, max_rhs, precision):
    kind, g, lmax, max_elems = spec
    monkeypatch.setenv("DMWF_FFT_MAX_ELEMS", str(max_elems))
    if kind == "hp":
        grid = healpix_grid(g)
        plan = dmwf.Plan(lmax=lmax, nside=g, max_rhs=max_rhs, precision=precision)
    else:
        grid = gl_grid(*g)
        plan = dmwf.Plan(lmax=lmax, ntheta=g[0], nphi=g[1], max_rhs=max_rhs, precision=precision)
    monkeypatch.delenv("DMWF_FFT_MAX_ELEMS")
    return grid, plan, lmax


def split_rings(grid, max_elems):
    """Rings whose Bluestein buffer (power of two >= 2 n - 1) exceeds the
    limit and whose length is a multiple of 4: the split ones."""
    n = np.asarray(grid["nphi"])
    M = 2 ** np.ceil(np.log2(2 * n - 1)).astype(int)
    pow2 = (n & (n - 1)) == 0
    return int(np.sum(~pow2 & (M > max_elems) & (n % 4 == 0)))


@pytest.mark.parametrize("precision,nrhs", [("fp64", 1), ("fp64", 9), ("mixed", 9)])
@pytest.mark.parametrize("spec", SPECS, ids=IDS)
def test_split_transforms(spec, precision, nrhs, dmwf, monkeypatch):
    prec = dmwf.FP64 if precision == "fp64" else dmwf.MIXED
    grid, plan, lmax = make(spec, dmwf, monkeypatch, nrhs, prec)
    assert split_rings(grid, spec[3]) > 0
    print(f"split transforms {spec} {precision} nrhs={nrhs}", flush=True)
    rng = np.random.default_rng(31 + lmax)
    sht = SHT(grid, lmax)
    a = rand_alm(lmax, rng, nrhs)
    m = rng.standard_normal((nrhs, 3, grid["npix"]))
    maps, alm, adj = plan.alm2map(a), plan.map2alm(m), plan.adjoint(m)
    tol = 1e-12 if precision == "fp64" else 1e-6
    for k in sorted({0, nrhs - 1}):
        assert rel_map(maps[k], sht.synthesis(a[k])) < tol, k
        assert rel_alm(alm[k], sht.analysis(m[k]), lmax) < tol, k
        assert rel_alm(adj[k], sht.adjoint(m[k]), lmax) < tol, k
    plan.close()


@pytest.mark.parametrize("nrhs", [1, 9])
@pytest.mark.parametrize("spec", [s for s in SPECS if s[0] == "hp"], ids=[i for i, s in zip(IDS, SPECS) if s[0] == "hp"])
def test_split_iterations(spec, nrhs, dmwf, monkeypatch):
    """Three messenger iterations (the fused inverse transform, pixel
    update and forward transform of each split ring) against the oracle."""
    kind, nside, lmax, _ = spec
    p = inputs.make_problem(2, nside=nside, lmax=lmax, holes=10)
    grid, plan, _ = make(spec, dmwf, monkeypatch, nrhs, dmwf.FP64)
    print(f"split iterations {spec} nrhs={nrhs}", flush=True)
    plan.set_spectra(p["cl"])
    plan.set_noise(p["ncov"], p["obs"])
    sht = SHT(grid, lmax)
    rng = np.random.default_rng(5)
    D = np.stack([sht.synthesis(inputs.signal_alm(2, lmax, k)) + inputs.noise_map(2, p["ncov"], p["obs"], k)
                  for k in range(nrhs)])
    T = D + 0.1 * rng.standard_normal(D.shape)
    lam = 11.0
    alm, tout = plan.iterate(D, T, lam, 3)
    for k in sorted({0, nrhs - 1}):
        st = dm.setup(grid, p["ncov"], p["obs"], D[k])
        F = dm.messenger_filter(p["cl"], (lam - 1) * st["tau"], st["tau"])
        t = T[k]
        for _ in range(3):
            u = dm.apply_blocks(F, sht.analysis(t), lmax)
            t = dm.pix_apply(st["K"], sht.synthesis(u)) + st["b"]
        assert rel_alm(alm[k], u, lmax) < 1e-12, k
        assert rel_map(tout[k], t) < 1e-12, k
    plan.close()
