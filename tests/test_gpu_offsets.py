"""Column tiles far from the first RHS, and band limits at which the lanes'
byte offsets pass 2^32.  The batched matrix-core transforms address each
column tile of 8 RHS from a uniform base plus one byte offset per lane,
32-bit while a tile's span of 8 RHS x 3 fields of nalm complex FP64 values
stays below 2^32 bytes, 64-bit beyond.

A property that holds at any size stands in for the oracle, which cannot
run these sizes: with RHS k equal to 2^(k // g - 4) times RHS k % g, both
transforms' outputs scale the same way, and a power-of-two scale commutes
with every rounding step, so each RHS must reproduce its group-mate's
result times the scale to rounding.  A lane that reads or writes through a
wrapped offset breaks this by O(1).
"""

import pytest

pytestmark = pytest.mark.gpu

CASES = [
    # 8 column tiles at the benchmark's size: the last tiles start
    # 56 x 3 x nalm complex values past the first RHS
    ("mixed", 1024, 2048, 64, 8),
    # lmax 5000: one tile's span is 5.8 GB, past 2^32 bytes
    ("fp64", 1667, 5000, 8, 1),
    ("mixed", 1667, 5000, 8, 1),
]


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1801_05358_amd import dmwf
    assert dmwf.device_count() > 0, "no GPU visible"
    return torch, dmwf


def scales(torch, nrhs, g):
    return torch.tensor([2.0 ** (k // g - 4) for k in range(nrhs)], dtype=torch.float64, device="cuda")


def check_scaled(torch, out, nrhs, g, tol, what):
    s = scales(torch, nrhs, g)
    for k in range(g, nrhs):
        want = out[k % g] * s[k] / s[k % g]
        err = float((out[k] - want).abs().max() / want.abs().max())
        assert err <= tol, f"{what}: RHS {k} off its scaled copy of RHS {k % g} by {err:.3e}"


@pytest.mark.parametrize("precision,nside,lmax,nrhs,g", CASES,
                         ids=[f"{p}-n{n}-l{l}-b{b}" for p, n, l, b, _ in CASES])
def test_scaled_copies_stay_scaled(env, precision, nside, lmax, nrhs, g):
    torch, dmwf = env
    print(f"offsets {precision} nside {nside} lmax {lmax} nrhs {nrhs}", flush=True)
    prec = dmwf.MIXED if precision == "mixed" else dmwf.FP64
    tol = 1e-6 if precision == "mixed" else 1e-12
    with dmwf.Plan(lmax=lmax, nside=nside, max_rhs=nrhs, precision=prec) as plan:
        gen = torch.Generator(device="cuda").manual_seed(5000 + lmax)
        s = scales(torch, nrhs, g).view(nrhs, 1, 1)
        npix = plan.npix
        a0 = torch.randn((g, 3, 2 * plan.nalm), generator=gen, dtype=torch.float64, device="cuda")
        alm = (a0.repeat(nrhs // g, 1, 1) * s).contiguous()
        maps = torch.empty((nrhs, 3, npix), dtype=torch.float64, device="cuda")
        plan.alm2map_device(alm, maps)
        torch.cuda.synchronize()
        assert torch.isfinite(maps).all()
        check_scaled(torch, maps, nrhs, g, tol, "synthesis")
        del alm

        m0 = torch.randn((g, 3, npix), generator=gen, dtype=torch.float64, device="cuda")
        m = (m0.repeat(nrhs // g, 1, 1) * s).contiguous()
        out = torch.empty((nrhs, 3, 2 * plan.nalm), dtype=torch.float64, device="cuda")
        plan.map2alm_device(m, out)
        torch.cuda.synchronize()
        assert torch.isfinite(out).all()
        check_scaled(torch, out, nrhs, g, tol, "analysis")
