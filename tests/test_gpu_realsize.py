"""Solve parity at full workload sizes.

* Configuration 2 (HEALPix Nside 256, lmax 512, |b| < 15 deg + 200 holes,
  100:1 scan noise): the first cooling step of the fixed schedule
  (10 iterations at lambda = 1e3) against the CPU oracle's iterate stored by
  tests/golden/make_config2_golden.py.  FP64 single RHS within 1e-10 per
  field; the batched mixed path with 2 and with 8 RHS (RHS 0 the stored
  problem, the others the same signal with independent noise) within 1e-5
  per field, 64-wide l-bin errors printed.
* Configuration 3 (Nside 1024, lmax 2048, |b| < 15 deg + 1000 holes, the
  benchmark's mask and noise), 8 RHS in one launch as the benchmark runs
  them: one messenger iteration u = F^lambda A t on sampled (l, m) for three
  of the RHS, FP64 within 1e-11 of the sampled scale, mixed within 1e-5
  relative per field.
"""

import importlib.util
import os

import numpy as np
import pytest

from oracle import dm
from oracle.geometry import healpix_grid, pixel_weights
from oracle.sht import SHT, alm_dot, alm_index, lm_arrays
from paper_1801_05358_amd import inputs

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
_spec = importlib.util.spec_from_file_location("make_config2_golden",
                                               os.path.join(HERE, "golden", "make_config2_golden.py"))
golden2 = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(golden2)


@pytest.fixture(scope="module")
def dmwf():
    from paper_1801_05358_amd import dmwf as mod
    assert mod.device_count() > 0, "no GPU visible"
    return mod


def rel_field(a, b, lmax, f):
    return float(np.sqrt(alm_dot(a[f] - b[f], a[f] - b[f], lmax) / alm_dot(b[f], b[f], lmax)))


def bin_errors(a, b, lmax, width=64):
    """Per field, the relative L2 error in l-bins of the given width (m > 0
    counted twice)."""
    ls, ms = lm_arrays(lmax)
    w = np.where(ms > 0, 2.0, 1.0)
    out = []
    for f in range(3):
        d2 = np.bincount(ls // width, w * np.abs(a[f] - b[f]) ** 2)
        r2 = np.bincount(ls // width, w * np.abs(b[f]) ** 2)
        out.append(np.sqrt(np.where(r2 > 0, d2 / np.where(r2 > 0, r2, 1), 0)))
    return out


@pytest.fixture(scope="module")
def cfg2():
    g = np.load(golden2.OUT)
    print("config 2 inputs", flush=True)
    p, grid, d = golden2.problem(0)
    chk = np.array([d.sum(), np.abs(d).sum(), (d * d).sum()])
    assert np.allclose(chk, g["d_checksum"], rtol=1e-12, atol=1e-9), "the input recipe changed"
    assert int(g["nside"]) == p["nside"] and int(g["lmax"]) == p["lmax"]
    return dict(p=p, grid=grid, d=d, u=g["u"])


def plan2(dmwf, c, nrhs, precision):
    p = c["p"]
    plan = dmwf.Plan(lmax=p["lmax"], nside=p["nside"], max_rhs=nrhs, precision=precision)
    plan.set_spectra(p["cl"])
    plan.set_noise(p["ncov"], p["obs"])
    # the workloads' schedule, stopped after its first cooling step
    plan.set_schedule(golden2.LAMBDA0, golden2.NSTEPS, golden2.ITERS, max_iters=golden2.ITERS)
    return plan


def test_config2_first_cooling_step_fp64(dmwf, cfg2):
    print("config 2 first cooling step, FP64, 1 RHS", flush=True)
    lmax = cfg2["p"]["lmax"]
    plan = plan2(dmwf, cfg2, 1, dmwf.FP64)
    out = plan.wiener_filter(cfg2["d"], want_stats=True)
    u = out["alm"][0]
    assert out["stats"][0]["iterations"] == golden2.ITERS
    errs = [rel_field(u, cfg2["u"], lmax, f) for f in range(3)]
    print("FP64 per field", errs, flush=True)
    assert max(errs) < 1e-10, errs
    plan.close()


@pytest.mark.parametrize("nrhs", [2, 8])
def test_config2_first_cooling_step_mixed(dmwf, cfg2, nrhs):
    print(f"config 2 first cooling step, mixed, {nrhs} RHS", flush=True)
    p, lmax = cfg2["p"], cfg2["p"]["lmax"]
    signal = cfg2["d"] - inputs.noise_map(golden2.CFG, p["ncov"], p["obs"], 0)
    D = np.stack([cfg2["d"]] + [signal + inputs.noise_map(golden2.CFG, p["ncov"], p["obs"], k)
                                for k in range(1, nrhs)])
    plan = plan2(dmwf, cfg2, nrhs, dmwf.MIXED)
    u = plan.wiener_filter(D)["alm"][0]
    errs = [rel_field(u, cfg2["u"], lmax, f) for f in range(3)]
    bins = bin_errors(u, cfg2["u"], lmax)
    print(f"mixed {nrhs} RHS per field", errs, "worst 64-wide l-bin", [float(b.max()) for b in bins], flush=True)
    assert max(errs) < 1e-5, errs
    plan.close()


# ----------------------------------------------------------------------------
# configuration 3, one iteration of 8 RHS
# ----------------------------------------------------------------------------
CFG3 = 3
NRHS3 = 8
SAMPLE3 = (0, 5, 7)


@pytest.fixture(scope="module")
def cfg3():
    p = inputs.make_problem(CFG3)
    nside, lmax = p["nside"], p["lmax"]
    grid = healpix_grid(nside)
    sht = SHT(grid, lmax, cache_bytes=0)
    print(f"config 3 inputs nside={nside} lmax={lmax} nrhs={NRHS3}", flush=True)
    t = np.stack([inputs.noise_map(CFG3, p["ncov"], p["obs"], k) for k in range(NRHS3)])
    rng = np.random.default_rng(2048)
    modes = [(0, 0), (2, 0), (3, 1), (17, 5), (300, 3), (lmax // 2, lmax // 2 - 1), (lmax, lmax), (lmax, 11),
             (lmax - 1, lmax // 3), (1500, 1499)]
    for _ in range(4):
        l = int(rng.integers(2, lmax + 1))
        modes.append((l, int(rng.integers(0, l + 1))))
    w = pixel_weights(grid)[0]
    ref = {k: sht.adjoint_modes(t[k], modes) * w for k in SAMPLE3}
    print("config 3 oracle samples done", flush=True)
    return dict(p=p, grid=grid, t=t, modes=modes, ref=ref)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_config3_one_iteration(dmwf, cfg3, precision):
    """dm_iterate on 8 RHS: u = F^lambda A t for the given messenger t."""
    p = cfg3["p"]
    lmax = p["lmax"]
    print(f"config 3 one iteration, {precision}, {NRHS3} RHS", flush=True)
    prec = dmwf.FP64 if precision == "fp64" else dmwf.MIXED
    plan = dmwf.Plan(lmax=lmax, nside=p["nside"], max_rhs=NRHS3, precision=prec)
    plan.set_spectra(p["cl"])
    plan.set_noise(p["ncov"], p["obs"])
    lam = 211.0
    t = cfg3["t"]
    u, _ = plan.iterate(t[::-1].copy(), t, lam, 1)
    plan.close()
    st = dm.setup(cfg3["grid"], p["ncov"], p["obs"], t[0])
    FTT, FTE, FEE, FBB = dm.messenger_filter(p["cl"], (lam - 1) * st["tau"], st["tau"])
    ls = np.array([l for l, _ in cfg3["modes"]])
    idx = [alm_index(l, m, lmax) for l, m in cfg3["modes"]]
    for k in SAMPLE3:
        a = cfg3["ref"][k]
        want = np.stack([FTT[ls] * a[0] + FTE[ls] * a[1], FTE[ls] * a[0] + FEE[ls] * a[1], FBB[ls] * a[2]])
        got = u[k][:, idx]
        for f in range(3):
            err = got[f] - want[f]
            if precision == "fp64":
                tol = 1e-11 * np.abs(want[f]).max()
                assert np.abs(err).max() <= tol, (k, f, np.abs(err).max(), tol)
            else:
                rel = np.linalg.norm(err) / np.linalg.norm(want[f])
                assert rel < 1e-5, (k, f, rel)
