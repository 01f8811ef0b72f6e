"""Benchmark: dual messenger Wiener-filter iterations per second on one GPU.

Workload (the configuration the headline metric is quoted on): HEALPix
Nside 1024, lmax 2048, mask |b| < 15 deg plus 1000 holes of radius 0.5 deg,
scan-like noise with a 100:1 range (Q = U = 2x T), TT/EE/BB/TE spectra
C^TT = 1e3/(l(l+1)), synthetic seeded data d = Y s + n.  One step is one full
messenger iteration of Algorithm 1 for every right-hand side in the batch:
ring FFT analysis -> Legendre analysis + filter -> Legendre synthesis ->
ring FFT synthesis + pixel update.  The timed region runs K iterations as a
cooling schedule (10 iterations per step, lambda 1e3 -> 1) on inputs already
resident in GPU memory.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DM iterations/s at Nside=1024,lmax=2048: mixed/batched vs FP64 at ≤1e-5 rel"
PEAK_FP64_VALU = 256 * 64 * 2 * 2.4e9 / 1e12     # TFLOP/s: CUs x lanes x FMA x clock
HBM_PEAK = 8000.0                                 # GB/s


def legendre_flops(npairs, nalm, nrhs):
    """Algorithmic FLOPs of one Legendre launch (analysis or synthesis): per
    (l, m, ring pair) point 16 for the three recursions (spin 0: 4, spin +-2:
    2 x 5 + 2) and 20 per right-hand side for the contraction (spin 0: one
    complex x real multiply-add, spin 2: four)."""
    return float(npairs) * float(nalm) * (16.0 + 20.0 * nrhs)


def ring_bytes(npix, nrings, mmax, nrhs, p=8):
    """Algorithmic bytes of one ring FFT + pixel-update launch: ring Fourier
    data read and written (3 fields, (mmax+1) complex per ring, both
    directions) plus K (shared) and b (per RHS) per pixel."""
    return float(nrhs) * 3 * nrings * (mmax + 1) * 2 * p * 2 + 3.0 * npix * p * (1 + nrhs)


def cpu_baseline(lmax, nside, alm):
    """Time the CPU FP64 oracle on a bounded sample of the same transform:
    synthesis of a few rings spread over the sphere, scaled to all rings and
    doubled for the analysis of one iteration."""
    from threadpoolctl import threadpool_limits
    from oracle.geometry import healpix_grid
    from oracle.sht import SHT
    grid = healpix_grid(nside)
    nr = len(grid["theta"])
    sample = [0, nside // 2, nside, 2 * nside - 1, 3 * nside, nr - 1]
    with threadpool_limits(limits=1):
        sht = SHT(grid, lmax, cache_bytes=0)
        t0 = time.perf_counter()
        sht.synthesis(alm, rings=sample)
        dt = time.perf_counter() - t0
    per_iter = 2.0 * dt * nr / len(sample)
    return {"value": 1.0 / per_iter, "unit": "iterations/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle synthesis of {len(sample)} of {nr} rings at Nside {nside}, lmax {lmax} "
                      f"({dt:.1f} s), scaled by {nr}/{len(sample)} rings and x2 for the analysis; "
                      f"NumPy FP64, BLAS limited to 1 thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--nside", type=int, default=1024)
    ap.add_argument("--lmax", type=int, default=2048)
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU sharding "
              f"is described in DESIGN.md, not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1801_05358_amd import dmwf, inputs

    nside, lmax, B = args.nside, args.lmax, args.nrhs
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    log(f"[bench] workload nside={nside} lmax={lmax} nrhs={B}")
    prob = inputs.make_problem(3, nside=nside, lmax=lmax)
    prec = dmwf.MIXED if args.precision == "mixed" else dmwf.FP64
    plan = dmwf.Plan(lmax=lmax, nside=nside, max_rhs=B, device=0, precision=prec)
    plan.set_spectra(prob["cl"])
    plan.set_noise(prob["ncov"], prob["obs"])
    dev = torch.device("cuda:0")
    # synthetic data d = Y s + n, made with the library's own synthesis
    s = np.stack([inputs.signal_alm(3, lmax, k) for k in range(B)])
    alm_t = torch.from_numpy(s.view(np.float64).reshape(B, 3, -1)).to(dev)
    d_t = torch.empty((B, 3, plan.npix), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    plan.alm2map_device(alm_t, d_t, stream=stream)
    noise = np.stack([inputs.noise_map(3, prob["ncov"], prob["obs"], k) for k in range(B)])
    d_t += torch.from_numpy(noise).to(dev)
    out_t = torch.empty((B, 3, plan.nalm * 2), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    log("[bench] inputs resident")

    def schedule(k):
        if k % 10 == 0:
            plan.set_schedule(1e3, k // 10, 10)
        else:
            plan.set_schedule(1e3, 1, k)

    # warmup
    if args.warmup > 0:
        schedule(args.warmup)
        plan.wiener_filter_device(d_t, out_t, stream=stream)
        torch.cuda.synchronize()
    log("[bench] warmup done")

    schedule(args.steps)
    plan.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.wiener_filter_device(d_t, out_t, stream=stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = plan.kernel_times()
    plan.profile(False)
    log(f"[bench] timed {args.steps} iterations in {dt:.3f} s; kernels {kt}")
    its = args.steps / dt

    # dominant kernel: the Legendre launches
    ana_ms, ana_n = kt["legendre_analysis"]
    syn_ms, syn_n = kt["legendre_synthesis"]
    dom = "legendre_synthesis" if syn_ms >= ana_ms else "legendre_analysis"
    ms, n = kt[dom]
    flops = legendre_flops(plan.nrings // 2 + 1, plan.nalm, B)
    achieved = flops / (ms / n * 1e-3) / 1e12
    ring_ms, ring_n = kt["ring_fft_pointwise"]
    rb = ring_bytes(plan.npix, plan.nrings, lmax, B)

    rec = {
        "metric": METRIC, "value": round(its, 4), "unit": "iterations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * dt / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"HEALPix Nside {nside}, lmax {lmax}, mask |b|<15 deg + 1000 holes, scan noise "
                               f"100:1, cooling lambda 1e3->1 in steps of 10 iterations, {B} right-hand side(s), "
                               f"FP64 path",
                   "nside": nside, "lmax": lmax, "nrhs": B, "precision": "fp64"},
        "roofline": {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3),
                     "peak": PEAK_FP64_VALU, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_VALU, 4),
                     "traffic": None},
        "kernels_ms_avg": {k: round(v[0] / max(v[1], 1), 4) for k, v in kt.items()},
        "ring_fft_hbm": {"achieved": round(rb / (ring_ms / max(ring_n, 1) * 1e-3) / 1e9, 1), "peak": HBM_PEAK,
                         "unit": "GB/s"},
    }
    if not args.no_cpu:
        log("[bench] timing the CPU oracle sample")
        rec["cpu_baseline"] = cpu_baseline(lmax, nside, s[0])
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
