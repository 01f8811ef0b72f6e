"""Per-iteration diagnostics (Fig. 4): the chi^2 of eq 3 and the Appendix C
residual of the iterate, recorded by the library during a solve, against
the oracle's record of the same schedule.

* Fixed cooling on configuration 1 (FP64, one RHS): the records after
  every 5th iteration and the last match the oracle's to 1e-10 (chi^2) and
  1e-8 (residual); tracing leaves the iterate bitwise unchanged; the mixed
  batched path's records match to 1e-5.
* Algorithm 1's own stopping rule with the settings of Sec. 3.2 (beta = 3/4,
  threshold 1e-4 -> 1e-6 cooled by eta = 1.1) on configuration 1 over the
  full sky, against the oracle's stored record
  (tests/golden/make_trace_golden.py): the library takes the same decision
  at every one of its ~1200 iterations through the 26 cooling steps, with
  the same Cauchy ratios, chi^2 and residuals.
"""

import importlib.util
import os

import numpy as np
import pytest

from oracle import dm
from oracle.geometry import healpix_grid
from oracle.sht import SHT, alm_dot
from paper_1801_05358_amd import inputs

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
_spec = importlib.util.spec_from_file_location("make_trace_golden",
                                               os.path.join(HERE, "golden", "make_trace_golden.py"))
tgold = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(tgold)


@pytest.fixture(scope="module")
def dmwf():
    from paper_1801_05358_amd import dmwf as mod
    assert mod.device_count() > 0, "no GPU visible"
    return mod


def cfg1(nrhs):
    p = inputs.make_problem(1)
    sht = SHT(healpix_grid(p["nside"]), p["lmax"])
    D = np.stack([sht.synthesis(inputs.signal_alm(1, p["lmax"], k)) + inputs.noise_map(1, p["ncov"], p["obs"], k)
                  for k in range(nrhs)])
    return p, sht, D


def make_plan(dmwf, p, nrhs=1, precision=None):
    kw = {} if precision is None else dict(precision=precision)
    plan = dmwf.Plan(lmax=p["lmax"], nside=p["nside"], max_rhs=nrhs, **kw)
    plan.set_spectra(p["cl"])
    plan.set_noise(p["ncov"], p["obs"])
    return plan


def test_fixed_schedule_trace_matches_oracle(dmwf):
    p, sht, D = cfg1(1)
    print("diagnostics trace, fixed schedule, FP64", flush=True)
    plan = make_plan(dmwf, p)
    plan.set_schedule(1e3, 3, 4)
    plain = plan.wiener_filter(D[0])["alm"][0]
    it0, _, _ = plan.diagnostics_trace()
    assert it0.size == 0
    plan.set_diagnostics(5)
    traced = plan.wiener_filter(D[0], want_stats=True)
    assert np.array_equal(traced["alm"][0], plain)
    it, c2, rs = plan.diagnostics_trace()
    ref = dm.solve(sht, D[0], p["ncov"], p["obs"], p["cl"], 1e3, 3, 4, diagnostics_every=5)["diagnostics"]
    assert list(it) == ref["iteration"] == [5, 10, 12]
    assert np.allclose(c2[:, 0], ref["chi2"], rtol=1e-10, atol=0), (c2[:, 0], ref["chi2"])
    assert np.allclose(rs[:, 0], ref["residual"], rtol=1e-8, atol=0), (rs[:, 0], ref["residual"])
    # the last record is the solve's own final diagnostics
    st = traced["stats"][0]
    assert abs(c2[-1, 0] - st["chi2"]) <= 1e-12 * st["chi2"]
    assert abs(rs[-1, 0] - st["residual"]) <= 1e-10 * st["residual"]
    assert dmwf.lib().dm_set_diagnostics(plan._h, -1) == dmwf.DM_EINVAL
    plan.set_diagnostics(0)
    plan.wiener_filter(D[0])
    assert plan.diagnostics_trace()[0].size == 0
    plan.close()


def test_mixed_batched_trace(dmwf):
    p, sht, D = cfg1(2)
    print("diagnostics trace, fixed schedule, mixed 2 RHS", flush=True)
    plan = make_plan(dmwf, p, nrhs=2, precision=dmwf.MIXED)
    plan.set_schedule(1e3, 3, 4)
    plan.set_diagnostics(4)
    plan.wiener_filter(D)
    it, c2, rs = plan.diagnostics_trace()
    assert list(it) == [4, 8, 12] and c2.shape == (3, 2)
    for k in range(2):
        ref = dm.solve(sht, D[k], p["ncov"], p["obs"], p["cl"], 1e3, 3, 4, diagnostics_every=4)["diagnostics"]
        assert np.allclose(c2[:, k], ref["chi2"], rtol=1e-5, atol=0), (k, c2[:, k], ref["chi2"])
        assert np.allclose(rs[:, k], ref["residual"], rtol=1e-5, atol=0), (k, rs[:, k], ref["residual"])
    plan.close()


def test_paper_stopping_rule_matches_stored_record(dmwf):
    g = tgold.read()
    p, sht, d = tgold.problem()
    print(f"Sec. 3.2 stopping rule, {g['steps'].size} iterations", flush=True)
    plan = make_plan(dmwf, p)
    plan.set_schedule_eps(tgold.LAMBDA0, tgold.BETA, tgold.EPS_START, tgold.EPS_END, tgold.ETA, tgold.MAX_ITERS)
    plan.set_diagnostics(tgold.EVERY)
    out = plan.wiener_filter(d, want_stats=True)
    cauchy, steps = plan.schedule_trace()
    it, c2, rs = plan.diagnostics_trace()
    # the same decision at every iteration (the stored margin says no ratio
    # was within rounding of its threshold)
    assert g["margin"] > 1e-5
    assert np.array_equal(steps, g["steps"]), (steps.size, g["steps"].size)
    assert out["stats"][0]["iterations"] == g["steps"].size
    # late ratios are differences of nearly equal iterates: agreement to 1e-6
    assert np.allclose(cauchy, g["cauchy"], rtol=1e-6, atol=0)
    assert np.array_equal(it, g["diag_iter"])
    assert np.allclose(c2[:, 0], g["chi2"], rtol=1e-10, atol=0)
    assert np.allclose(rs[:, 0], g["residual"], rtol=1e-8, atol=0)
    plan.close()
