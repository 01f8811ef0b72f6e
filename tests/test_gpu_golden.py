"""The library on the stored tiny problem of tests/golden/dm_nside2_lmax4.txt
(HEALPix Nside 2, lmax 4; the oracle's results written by
tests/golden/make_golden.py): analysis to 1e-12, the plain and the refined
solve (last and best iterate) to 1e-10 on the FP64 path, the plain solve within 1e-5 per field on
the batched mixed path."""

import importlib.util
import os

import numpy as np
import pytest

from oracle.sht import alm_dot

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
_spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "golden", "make_golden.py"))
golden = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(golden)


@pytest.fixture(scope="module")
def dmwf():
    from paper_1801_05358_amd import dmwf as mod
    assert mod.device_count() > 0, "no GPU visible"
    return mod


def rel_field(a, b, f):
    lmax = golden.LMAX
    return float(np.sqrt(alm_dot(a[f] - b[f], a[f] - b[f], lmax) / alm_dot(b[f], b[f], lmax)))


def make(dmwf, g, nrhs, precision):
    plan = dmwf.Plan(lmax=golden.LMAX, nside=golden.NSIDE, max_rhs=nrhs, precision=precision)
    plan.set_spectra(g["cl"])
    plan.set_noise(g["ncov"], g["obs"].astype(bool))
    plan.set_schedule(*golden.SCHED)
    return plan


def test_fp64_matches_stored_oracle_results(dmwf):
    g = golden.read()
    print("golden tiny problem, FP64", flush=True)
    plan = make(dmwf, g, 1, dmwf.FP64)
    a = plan.map2alm(g["d"])
    assert np.abs(a - g["analysis"]).max() <= 1e-12 * np.abs(g["analysis"]).max()
    u = plan.wiener_filter(g["d"])["alm"][0]
    for f in range(3):
        assert rel_field(u, g["u_plain"], f) < 1e-10, f
    plan.set_refinement(golden.NCORR)
    u = plan.wiener_filter(g["d"])["alm"][0]
    for f in range(3):
        assert rel_field(u, g["u_refined"], f) < 1e-10, f
    plan.set_refinement_select(True)
    u = plan.wiener_filter(g["d"])["alm"][0]
    for f in range(3):
        assert rel_field(u, g["u_refined_best"], f) < 1e-10, f


def test_mixed_matches_stored_oracle_results(dmwf):
    g = golden.read()
    print("golden tiny problem, mixed 2 RHS", flush=True)
    plan = make(dmwf, g, 2, dmwf.MIXED)
    out = plan.wiener_filter(np.stack([g["d"], g["d"]]))["alm"]
    for k in range(2):
        for f in range(3):
            assert rel_field(out[k], g["u_plain"], f) < 1e-5, (k, f)
