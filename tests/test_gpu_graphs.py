"""Fixed-schedule cooling steps run as HIP graphs (recorded once per step,
launched on the solve's stream).  Every solve, repeated with other work and
synchronisations in between, must equal the directly launched solve bit
for bit: the graph holds the same kernels in the same order."""

import os

import numpy as np
import pytest

from oracle.geometry import healpix_grid
from oracle.sht import SHT
from paper_1801_05358_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dmwf():
    from paper_1801_05358_amd import dmwf as mod
    assert mod.device_count() > 0, "no GPU visible"
    return mod


def make_plan(dmwf, p, max_rhs, precision, graphs):
    old = os.environ.get("DMWF_GRAPHS")
    os.environ["DMWF_GRAPHS"] = "1" if graphs else "0"
    try:
        plan = dmwf.Plan(lmax=p["lmax"], nside=p["nside"], max_rhs=max_rhs, precision=precision)
    finally:
        if old is None:
            del os.environ["DMWF_GRAPHS"]
        else:
            os.environ["DMWF_GRAPHS"] = old
    plan.set_spectra(p["cl"])
    plan.set_noise(p["ncov"], p["obs"])
    plan.set_schedule(1e3, 4, 5)
    return plan


@pytest.mark.parametrize("precision,nrhs", [("fp64", 1), ("mixed", 2)])
def test_graph_solves_equal_direct_solves(dmwf, precision, nrhs):
    p = inputs.make_problem(1)
    sht = SHT(healpix_grid(p["nside"]), p["lmax"])
    D = np.stack([sht.synthesis(inputs.signal_alm(1, p["lmax"], k)) + inputs.noise_map(1, p["ncov"], p["obs"], k)
                  for k in range(nrhs)])
    prec = dmwf.FP64 if precision == "fp64" else dmwf.MIXED
    direct = make_plan(dmwf, p, nrhs, prec, graphs=False)
    want = direct.wiener_filter(D, want_map=True, want_stats=True)
    graph = make_plan(dmwf, p, nrhs, prec, graphs=True)
    rng = np.random.default_rng(3)
    for rep in range(3):
        got = graph.wiener_filter(D, want_map=True, want_stats=True)
        assert np.array_equal(got["alm"], want["alm"]), rep
        assert np.array_equal(got["map"], want["map"]), rep
        for a, b in zip(got["stats"], want["stats"]):
            assert (a["residual"], a["chi2"], a["cauchy"]) == (b["residual"], b["chi2"], b["cauchy"]), rep
        # other work on the plan between the replays
        graph.alm2map(rng.standard_normal((nrhs, 3, graph.nalm)) + 0j)
    # with per-kernel timing on, the solve runs its launches directly
    graph.profile(True)
    got = graph.wiener_filter(D)
    graph.profile(False)
    assert np.array_equal(got["alm"], want["alm"])
