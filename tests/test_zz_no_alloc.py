"""The allocation-free analysis dm_map2alm_device_noalloc against
dm_map2alm_device through the C ABI: the same values to the last bit (the
same kernels in the same order, only their work memory differs), on two
calls in a row, the second with a smaller input, on the FP64 single-RHS
kernels and on the mixed batched (FP32 matrix-core) kernels; work memory
beyond its fixed array is refused with a message.  Runs alone or after the
other GPU tests."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1801_05358_amd import dmwf
    assert dmwf.device_count() > 0, "no GPU visible"
    assert torch.cuda.is_available()
    return dmwf, torch


def maps(torch, plan, nrhs, seed):
    rng = np.random.default_rng(seed)
    m = rng.standard_normal((nrhs, 3, plan.npix))
    return torch.from_numpy(m).to("cuda:0")


def compare(dmwf, torch, plan, nrhs, seed):
    stream = torch.cuda.current_stream()
    m = maps(torch, plan, nrhs, seed)
    want = torch.full((nrhs, 3, plan.nalm * 2), np.nan, dtype=torch.float64, device="cuda:0")
    got = torch.full_like(want, np.nan)
    plan.map2alm_device(m, want, stream=stream)
    plan.map2alm_device_noalloc(m, got, stream=stream)
    torch.cuda.synchronize()
    w, g = want.cpu().numpy(), got.cpu().numpy()
    assert np.all(np.isfinite(w)) and np.all(np.isfinite(g))
    assert np.array_equal(w, g), float(np.abs(w - g).max())
    return np.abs(w).max()


@pytest.mark.parametrize("precision,nrhs", [("fp64", (3, 1)), ("mixed", (4, 2))])
def test_noalloc_matches_map2alm_device(env, precision, nrhs):
    dmwf, torch = env
    prec = dmwf.FP64 if precision == "fp64" else dmwf.MIXED
    print(f"no-alloc analysis, {precision}, nrhs {nrhs}", flush=True)
    plan = dmwf.Plan(lmax=32, nside=16, max_rhs=max(nrhs), precision=prec)
    # two calls in a row, the second with fewer right-hand sides
    assert compare(dmwf, torch, plan, nrhs[0], 1) > 0
    assert compare(dmwf, torch, plan, nrhs[1], 2) > 0
    plan.close()
    # then a smaller grid on a plan of its own (the array keeps the last
    # call's contents; nothing may depend on them)
    small = dmwf.Plan(lmax=16, nside=8, max_rhs=1)
    assert compare(dmwf, torch, small, 1, 3) > 0
    small.close()


def test_noalloc_refuses_work_beyond_its_array(env):
    dmwf, torch = env
    print("no-alloc analysis, size refusal", flush=True)
    plan = dmwf.Plan(lmax=128, nside=64, max_rhs=64)
    m = torch.zeros((64, 3, plan.npix), dtype=torch.float64, device="cuda:0")
    a = torch.zeros((64, 3, plan.nalm * 2), dtype=torch.float64, device="cuda:0")
    with pytest.raises(dmwf.DmwfError) as e:
        plan.map2alm_device_noalloc(m, a)
    assert e.value.status == dmwf.DM_EINVAL and "bytes of work memory" in str(e.value)
    # a smaller batch on the same plan fits
    plan.map2alm_device_noalloc(m[:2].contiguous(), a[:2].contiguous())
    torch.cuda.synchronize()
    plan.close()
