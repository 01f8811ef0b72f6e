"""The autotuner of the launch shapes: it picks the batched Legendre
kernels' m-chunks and synthesis waves among its candidates, leaving results
unchanged to the last bit (they only move work between waves, workgroups
and XCDs), and the ring step's workgroup widths of its two size classes
(results within FP64 rounding); it reuses choices from its cache file."""

import numpy as np
import pytest

from oracle.geometry import healpix_grid
from oracle.sht import SHT
from paper_1801_05358_amd import inputs

pytestmark = pytest.mark.gpu

CAND = {0, 1, 2, 4, 8}


@pytest.fixture(scope="module")
def dmwf():
    from paper_1801_05358_amd import dmwf as mod
    assert mod.device_count() > 0, "no GPU visible"
    return mod


def test_autotune(dmwf, tmp_path, monkeypatch):
    monkeypatch.delenv("DMWF_TUNE_CACHE", raising=False)
    p = inputs.make_problem(2, nside=64, lmax=128, holes=20)
    sht = SHT(healpix_grid(p["nside"]), p["lmax"])
    D = np.stack([sht.synthesis(inputs.signal_alm(2, p["lmax"], k)) + inputs.noise_map(2, p["ncov"], p["obs"], k)
                  for k in range(2)])

    def plan():
        q = dmwf.Plan(lmax=p["lmax"], nside=p["nside"], max_rhs=2, precision=dmwf.MIXED)
        q.set_spectra(p["cl"])
        q.set_noise(p["ncov"], p["obs"])
        q.set_schedule(1e3, 3, 3)
        return q

    a = plan()
    before = a.wiener_filter(D)["alm"]
    r = a.autotune(2)
    print("autotune", r, flush=True)
    assert r["syn_mchunk"] in CAND and r["ana_mchunk"] in CAND and r["syn_waves"] in (1, 2, 4, 8)
    assert r["syn_ms"] > 0 and r["ana_ms"] > 0 and r["ring_ms"] == 0      # 2 RHS: one ring launch
    assert np.array_equal(a.wiener_filter(D)["alm"], before)
    # every synthesis width gives the same bits
    for w in (1, 2, 8):
        monkeypatch.setenv("DMWF_SYN_WAVES", str(w))
        q = plan()
        assert np.array_equal(q.wiener_filter(D)["alm"], before), w
        q.close()
    monkeypatch.delenv("DMWF_SYN_WAVES")
    # cache: the first plan measures and appends, the next one reads
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("DMWF_TUNE_CACHE", str(cache))
    b = plan()
    rb = b.autotune(2)
    assert cache.exists() and rb["syn_ms"] > 0
    c = plan()
    rc = c.autotune(2)
    assert all(rc[k] == rb[k] for k in ("syn_mchunk", "ana_mchunk", "syn_waves"))
    assert rc["syn_ms"] == 0 and rc["ana_ms"] == 0
    assert np.array_equal(c.wiener_filter(D)["alm"], before)
    # a single RHS on an FP64 plan does not use the batched kernels
    f = dmwf.Plan(lmax=p["lmax"], nside=p["nside"], max_rhs=1)
    rf = f.autotune(1)
    assert rf["syn_ms"] == 0 and rf["ana_ms"] == 0


def test_autotune_ring_widths(dmwf, monkeypatch):
    """With 4 RHS and two ring size classes (the size bound lowered so that a
    small grid has both), the ring widths are tuned too; the solve after
    tuning matches the one before within FP64 rounding."""
    monkeypatch.delenv("DMWF_TUNE_CACHE", raising=False)
    monkeypatch.setenv("DMWF_RING_SMALL_M", "128")
    p = inputs.make_problem(2, nside=64, lmax=128, holes=20)
    sht = SHT(healpix_grid(p["nside"]), p["lmax"])
    D = np.stack([sht.synthesis(inputs.signal_alm(2, p["lmax"], k)) + inputs.noise_map(2, p["ncov"], p["obs"], k)
                  for k in range(4)])
    q = dmwf.Plan(lmax=p["lmax"], nside=p["nside"], max_rhs=4, precision=dmwf.FP64)
    q.set_spectra(p["cl"])
    q.set_noise(p["ncov"], p["obs"])
    q.set_schedule(1e3, 2, 3)
    before = q.wiener_filter(D)["alm"]
    r = q.autotune(4)
    print("autotune ring", r, flush=True)
    assert r["ring_ms"] > 0 and r["ring_big_threads"] in (512, 1024) and r["ring_small_threads"] in (256, 512, 1024)
    after = q.wiener_filter(D)["alm"]
    assert np.abs(after - before).max() <= 1e-12 * np.abs(before).max()
