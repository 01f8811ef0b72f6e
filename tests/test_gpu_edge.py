"""Degenerate and boundary cases of the solve on the GPU, against the oracle
or against what the method fixes exactly.

* Zero data give the zero solution, exactly, on every path; a zero RHS in
  a batch leaves the other RHS unchanged.
* Full sky (no mask), a single observed pixel, and a zero B-mode spectrum
  (B stays exactly zero) match the oracle to 1e-10.
* The smallest HEALPix grids (Nside 1, lmax 2; Nside 2, lmax 5) match the
  oracle, on the FP64 and the batched paths.
"""

import numpy as np
import pytest

from oracle import dm
from oracle.geometry import healpix_grid
from oracle.sht import SHT, alm_dot
from paper_1801_05358_amd import inputs

pytestmark = pytest.mark.gpu

SCHED = (1e3, 3, 4)


@pytest.fixture(scope="module")
def dmwf():
    from paper_1801_05358_amd import dmwf as mod
    assert mod.device_count() > 0, "no GPU visible"
    return mod


def rel(a, b, lmax):
    num = sum(alm_dot(a[f] - b[f], a[f] - b[f], lmax) for f in range(3))
    den = sum(alm_dot(b[f], b[f], lmax) for f in range(3))
    return float(np.sqrt(num / den))


def problem(nside=None, lmax=None, nrhs=1):
    p = inputs.make_problem(1, nside=nside, lmax=lmax)
    sht = SHT(healpix_grid(p["nside"]), p["lmax"])
    D = np.stack([sht.synthesis(inputs.signal_alm(1, p["lmax"], k)) + inputs.noise_map(1, p["ncov"], p["obs"], k)
                  for k in range(nrhs)])
    return p, sht, D


def plan_for(dmwf, p, max_rhs=1, precision=None, obs="default", cl=None):
    kw = {} if precision is None else dict(precision=precision)
    plan = dmwf.Plan(lmax=p["lmax"], nside=p["nside"], max_rhs=max_rhs, **kw)
    plan.set_spectra(p["cl"] if cl is None else cl)
    plan.set_noise(p["ncov"], p["obs"] if isinstance(obs, str) else obs)
    plan.set_schedule(*SCHED)
    return plan


@pytest.mark.parametrize("precision,nrhs", [("fp64", 1), ("fp64", 9), ("mixed", 2)])
def test_zero_data_gives_zero(dmwf, precision, nrhs):
    p, sht, D = problem(nrhs=nrhs)
    print(f"zero data {precision} nrhs={nrhs}", flush=True)
    prec = dmwf.FP64 if precision == "fp64" else dmwf.MIXED
    plan = plan_for(dmwf, p, nrhs, prec)
    out = plan.wiener_filter(np.zeros_like(D), want_map=True)
    assert not np.any(out["alm"]) and not np.any(out["map"])
    if nrhs > 1:
        # a zero RHS among others: the others are what they are alone
        Dz = D.copy()
        Dz[1] = 0.0
        a = plan.wiener_filter(D)["alm"]
        b = plan.wiener_filter(Dz)["alm"]
        assert not np.any(b[1])
        keep = [k for k in range(nrhs) if k != 1]
        assert np.array_equal(a[keep], b[keep])


def test_full_sky(dmwf):
    p, sht, D = problem()
    plan = plan_for(dmwf, p, obs=None)
    u = plan.wiener_filter(D[0])["alm"][0]
    ref = dm.solve(sht, D[0], p["ncov"], None, p["cl"], *SCHED)["u"]
    assert rel(u, ref, p["lmax"]) < 1e-10


def test_single_observed_pixel(dmwf):
    p, sht, D = problem()
    obs = np.zeros(sht.grid["npix"], dtype=bool)
    obs[1234] = True
    plan = plan_for(dmwf, p, obs=obs)
    u = plan.wiener_filter(D[0])["alm"][0]
    ref = dm.solve(sht, D[0], p["ncov"], obs, p["cl"], *SCHED)["u"]
    assert np.abs(ref).max() > 0
    assert rel(u, ref, p["lmax"]) < 1e-10


@pytest.mark.parametrize("precision,nrhs", [("fp64", 1), ("mixed", 2)])
def test_zero_b_spectrum(dmwf, precision, nrhs):
    p, sht, D = problem(nrhs=nrhs)
    cl = p["cl"].copy()
    cl[2] = 0.0                                    # BB
    prec = dmwf.FP64 if precision == "fp64" else dmwf.MIXED
    plan = plan_for(dmwf, p, nrhs, prec, cl=cl)
    out = plan.wiener_filter(D)["alm"]
    for k in range(nrhs):
        assert not np.any(out[k][2]), k
        ref = dm.solve(sht, D[k], p["ncov"], p["obs"], cl, *SCHED)["u"]
        num = sum(alm_dot(out[k][f] - ref[f], out[k][f] - ref[f], p["lmax"]) for f in (0, 1))
        den = sum(alm_dot(ref[f], ref[f], p["lmax"]) for f in (0, 1))
        assert np.sqrt(num / den) < (1e-10 if precision == "fp64" else 1e-5)


@pytest.mark.parametrize("nside,lmax", [(1, 2), (2, 5)])
@pytest.mark.parametrize("precision,nrhs", [("fp64", 1), ("fp64", 8), ("mixed", 2)])
def test_smallest_grids(dmwf, nside, lmax, precision, nrhs):
    p, sht, D = problem(nside, lmax, nrhs)
    print(f"smallest grid nside={nside} lmax={lmax} {precision} nrhs={nrhs}", flush=True)
    prec = dmwf.FP64 if precision == "fp64" else dmwf.MIXED
    plan = plan_for(dmwf, p, nrhs, prec)
    out = plan.wiener_filter(D)["alm"]
    tol = 1e-10 if precision == "fp64" else 1e-5
    for k in range(nrhs):
        ref = dm.solve(sht, D[k], p["ncov"], p["obs"], p["cl"], *SCHED)["u"]
        assert rel(out[k], ref, lmax) < tol, k
