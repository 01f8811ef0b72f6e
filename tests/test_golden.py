"""The stored tiny problem of tests/golden/dm_nside2_lmax4.txt (written by
tests/golden/make_golden.py from the oracle): the seeded input recipe still
gives its inputs, and the oracle still gives its results from them (a guard
against silent changes of the oracle's arithmetic)."""

import importlib.util
import os

import numpy as np

from oracle import dm
from oracle.geometry import healpix_grid
from oracle.sht import SHT

HERE = os.path.dirname(os.path.abspath(__file__))
_spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "golden", "make_golden.py"))
golden = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(golden)


def test_inputs_recipe_unchanged():
    g = golden.read()
    p, sht, d = golden.problem()
    assert np.array_equal(g["cl"], p["cl"])
    assert np.array_equal(g["ncov"], p["ncov"])
    assert np.array_equal(g["obs"].astype(bool), p["obs"])
    assert np.allclose(g["d"], d, rtol=0, atol=1e-15 * np.abs(d).max())


def test_oracle_reproduces_stored_results():
    g = golden.read()
    sht = SHT(healpix_grid(golden.NSIDE), golden.LMAX)
    obs = g["obs"].astype(bool)
    got = {
        "analysis": sht.analysis(g["d"]),
        "u_plain": dm.solve(sht, g["d"], g["ncov"], obs, g["cl"], *golden.SCHED)["u"],
        "u_refined": dm.refine(sht, g["d"], g["ncov"], obs, g["cl"], *golden.SCHED, golden.NCORR)["u"],
        "u_refined_best": dm.refine(sht, g["d"], g["ncov"], obs, g["cl"], *golden.SCHED, golden.NCORR,
                                    select="best")["u"],
    }
    for k, v in got.items():
        assert np.abs(v - g[k]).max() <= 1e-12 * np.abs(g[k]).max(), k
