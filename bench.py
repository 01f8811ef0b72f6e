"""Benchmark: dual messenger Wiener-filter iterations per second on one GPU.

Workload: HEALPix Nside 1024, lmax 2048, mask |b| < 15 deg plus 1000 holes
of radius 0.5 deg, scan-like noise with a 100:1 range (Q = U = 2x T),
TT/EE/BB/TE spectra C^TT = 1e3/(l(l+1)), synthetic seeded data d = Y s + n.
One step is one full messenger iteration of Algorithm 1 for every
right-hand side (RHS) of the batch: ring FFT analysis -> Legendre analysis
+ harmonic filter -> Legendre synthesis -> ring FFT synthesis + pixel
update.  The timed region runs K iterations as a cooling schedule (10
iterations per step, lambda 1e3 -> 1) on inputs already resident in GPU
memory.

The headline is the mixed-precision batched path (FP32 matrix-core
contraction, FP64 recursion, FFT and iterate; B = 8 RHS): value = RHS
iterations per second.  Beside it: the plain FP64 path at B = 1 on the same
data, the mixed result's relative error per field against the FP64 GPU
path after the same schedule (gate 1e-5), the roofline of the dominant
kernel and the CPU oracle timed on a bounded sample.

Prints one JSON line.  Usage:
  python bench.py [--gpus 1] [--steps K] [--warmup W] [--nrhs B] [--precision mixed|fp64]
  python bench.py --traffic FETCH_CSV WRITE_CSV   (no GPU: turn two rocprofv3 --pmc
      counter files into the per-launch HBM traffic summary under profiles/)
"""

import argparse
import gc
import csv
import re
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DM iterations/s at Nside=1024,lmax=2048: mixed/batched vs FP64 at ≤1e-5 rel"
CLOCK_GHZ = 2.4
PEAK = {   # dense vendor peaks, TFLOP/s
    "fp64_valu": 256 * 4 * 16 * 2 * CLOCK_GHZ / 1e3,    # CUs x SIMDs x lanes x FMA x clock = 78.6
    "fp32_mfma": 157.3,
    "fp64_mfma": 78.6,
}
HBM_PEAK = 8000.0                                         # GB/s
ACC_GATE = 1e-5
COPY_BYTES = 1 << 30                                      # calibration copy for the traffic counters
# kernel class -> (name key, dispatches per step): the ring step of the
# 8-RHS workload at Nside 1024 runs as two launches of the same kernel (the
# large and the small transforms), summed per step
TRAFFIC_KERNELS = {"legendre_analysis": ("bana_kernel", 1), "legendre_synthesis": ("bsyn_kernel", 1),
                   "ring_fft_pointwise": ("ring_kernel<3", 2)}
KERNEL_SOURCES = {"legendre_analysis": "legendre_mfma.hip", "legendre_synthesis": "legendre_mfma.hip",
                  "ring_fft_pointwise": "ringfft.hip"}


def legendre_flops(npairs, nalm, nrhs):
    """Algorithmic FLOPs of one Legendre launch (analysis or synthesis): per
    (l, m, ring pair) point 16 for the recursions shared by all RHS (spin 0:
    4, spin +-2: 2 x 5 + 2) and 20 per RHS for the contraction (spin 0: one
    complex x real multiply-add, spin 2: four)."""
    return float(npairs) * float(nalm) * (16.0 + 20.0 * nrhs)


def ring_bytes(npix, nrings, mmax, nrhs, p_ring=8, p_map=8):
    """Algorithmic bytes of one ring FFT + pixel-update launch (synthesis,
    update and analysis of every ring): ring Fourier data read and written
    (3 fields, (mmax+1) complex per ring, p_ring bytes per real: 4 where the
    mixed batched path stores them in FP32) plus K (shared) and b (per RHS),
    p_map bytes per real."""
    return float(nrhs) * 3 * nrings * (mmax + 1) * 2 * p_ring * 2 + 3.0 * npix * p_map * (1 + nrhs)


def _pow2(n):
    return n & (n - 1) == 0


def ring_lds_bytes(nside, mmax, nrhs, max_elems=8192):
    """LDS bytes (read, written) of one ring step (synthesis, pixel update
    and analysis of every HEALPix ring pair), in the kernel's own terms:
    16-byte elements (FP64 complex); a transform of size M = 2^a or 3 2^a
    runs ceil(a / 3) radix-8 passes (plus one radix-3 pass), each reading
    and writing the buffer once; the fold writes the buffer, the pixel
    update reads and writes the ring, the unfold reads two values per m.  A
    Bluestein length (size rules of the plan's FFT tables: the smaller of
    2^k and 3 2^k holding 2n - 1 points) takes two transforms and the kernel
    product per direction, and zero padding after the fold and the update.
    None when some length would be split (its launch has another layout)."""
    def r3(n):
        return n >= 24 and n % 3 == 0 and _pow2(n // 3)

    def blue(n):
        m2 = 1
        while m2 < 2 * n - 1:
            m2 *= 2
        m3 = 24
        while m3 < 2 * n - 1:
            m3 *= 2
        return min(m2, m3)

    def passes(M):
        P = M // 3 if M % 3 == 0 else M
        return (P.bit_length() - 1 + 2) // 3 + (1 if M % 3 == 0 else 0)

    rd = wr = 0
    for i in range(1, 2 * nside + 1):
        n = 4 * i if i < nside else 4 * nside
        direct = _pow2(n) or r3(n)
        M = n if direct else blue(n)
        if not direct and M > max_elems:
            return None
        pp = passes(M)
        if direct:
            r = 2 * pp * M + n + 2 * (mmax + 1)
            w = n + 2 * pp * M + n
        else:
            r = 2 * (2 * pp * M + M) + n + 2 * (mmax + 1)
            w = M + 2 * (2 * pp * M + M) + n + (M - n)
        rd += r
        wr += w
    f = 16.0 * 3 * nrhs
    return rd * f, wr * f


def lds_rates():
    """Measured chip-wide LDS read and write rates (bytes/s) of the ring
    kernel's access pattern, from the committed probe summary."""
    rec = {}
    with open(os.path.join(ROOT, "profiles", "lds_bandwidth_mi355x.txt")) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    return float(rec["read_TBps"]) * 1e12, float(rec["write_TBps"]) * 1e12


def source_sha(kernel):
    with open(os.path.join(ROOT, "paper_1801_05358_amd", "csrc", KERNEL_SOURCES[kernel]), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_file(kernel, prec, nrhs):
    return os.path.join(ROOT, "profiles", f"traffic_{kernel}_nside1024_lmax2048_{prec}_b{nrhs}.txt")


def read_traffic(kernel, prec, nrhs):
    """HBM bytes per launch of ``kernel`` from its committed counter summary,
    or None when there is none or the kernel source changed since."""
    path = traffic_file(kernel, prec, nrhs)
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    if rec.get("source_sha256_16") != source_sha(kernel):
        return None
    return float(rec["bytes_per_launch"])


def traffic_from_csv(fetch_csv, write_csv, prec, nrhs, command, last):
    """Per-launch HBM bytes of the Legendre kernels from two rocprofv3 --pmc
    runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by what the
    same counter reads for the calibration copy of COPY_BYTES.  Only each
    kernel's last ``last`` dispatches count: the autotuner's candidate
    launches come first and run other workgroup placements."""
    def per_kernel(path, counter):
        acc = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            acc.setdefault(r["Kernel_Name"], {}).setdefault(r["Dispatch_Id"], 0.0)
            acc[r["Kernel_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"]) * 1024.0
        return acc
    fetch, write = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")

    def find(acc, key, per):
        # the ring step runs once per iteration but the last: a solve of k
        # iterations has k - 1 of them, so the ring keeps 2/3 as many steps
        # as the Legendre kernels keep launches (two 3-iteration solves)
        steps = last if per == 1 else max(1, last * 2 // 3)
        for name, d in acc.items():
            if key in name:
                v = [x for _, x in sorted(d.items(), key=lambda kv: int(kv[0]))][-steps * per:]
                return [sum(v[i:i + per]) for i in range(0, len(v) - per + 1, per)]
        return []

    def copy_factor(path, counter):
        # the calibration copy is the run's last buffer-copy dispatch
        last, val = -1, 0.0
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter and "copyBuffer" in r["Kernel_Name"] and int(r["Dispatch_Id"]) > last:
                last, val = int(r["Dispatch_Id"]), 0.0
            if r["Counter_Name"] == counter and int(r["Dispatch_Id"]) == last:
                val += float(r["Counter_Value"]) * 1024.0
        return COPY_BYTES / val if val > 0 else None

    ff, fw = copy_factor(fetch_csv, "FETCH_SIZE"), copy_factor(write_csv, "WRITE_SIZE")
    for kernel, (key, per) in TRAFFIC_KERNELS.items():
        f, w = find(fetch, key, per), find(write, key, per)
        if not f or not w or ff is None or fw is None:
            print(f"no counters for {kernel}", file=sys.stderr)
            continue
        fb = sum(f) / len(f) * ff
        wb = sum(w) / len(w) * fw
        with open(traffic_file(kernel, prec, nrhs), "w") as out:
            out.write(f"# HBM traffic per launch of {kernel} ({key}, {per} dispatch(es) per step summed), "
                      f"Nside 1024, lmax 2048, {prec}, B = {nrhs}\n")
            out.write(f"# from rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE runs of:\n#   {command}\n")
            out.write(f"# counters scaled by a {COPY_BYTES} B device copy: fetch x{ff:.4f}, write x{fw:.4f}\n")
            out.write(f"source_sha256_16: {source_sha(kernel)}\n")
            out.write(f"dispatches: {len(f)}\n")
            out.write(f"fetch_bytes_per_launch: {fb:.6e}\n")
            out.write(f"write_bytes_per_launch: {wb:.6e}\n")
            out.write(f"bytes_per_launch: {fb + wb:.6e}\n")
        print(f"{kernel}: fetch {fb / 1e9:.3f} GB, write {wb / 1e9:.3f} GB per launch")


COUNTER_KERNELS = ("bana_kernel", "bsyn_kernel", "ring_kernel", "combine_kernel", "leg_analysis_kernel",
                   "leg_synth_kernel")


def counter_summary(csv_paths, out, command, title, last):
    """Per-kernel counter summary from rocprofv3 --pmc runs (one CSV per
    pass): each counter's value per dispatch (summed over the rows of that
    dispatch), averaged over each kernel's last ``last`` dispatches, for the
    transform kernels; then derived figures where their counters are there:
    MFMA FLOP (the MOPS counters count 512 FLOP each), the MFMA pipe's busy
    fraction (busy cycles per SIMD over the GPU-active cycles times the 1024
    SIMDs), VALU and LDS instructions per MFMA instruction."""
    def short(n):
        n = re.sub(r"dmwf::\(anonymous namespace\)::", "", n)
        return re.sub(r"\(.*$", "", n)[:60]
    vals = {}
    for path in csv_paths:
        for r in csv.DictReader(open(path)):
            k = short(r["Kernel_Name"])
            if not any(c in k for c in COUNTER_KERNELS):
                continue
            d = vals.setdefault(k, {}).setdefault(r["Counter_Name"], {})
            d[int(r["Dispatch_Id"])] = d.get(int(r["Dispatch_Id"]), 0.0) + float(r["Counter_Value"])
            # the dispatch's duration (ns) from its timestamps, once per dispatch and pass
            t = vals[k].setdefault("duration_ns", {})
            key = (path, int(r["Dispatch_Id"]))
            if key not in t:
                t[key] = float(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    lines = [f"# {title}", f"# command (one run per pass): {command}",
             f"# per kernel: counter averages over its last {last} dispatches"]
    for k in sorted(vals):
        avg = {}
        for c, d in sorted(vals[k].items()):
            v = [x for _, x in sorted(d.items())][-last:]
            avg[c] = sum(v) / len(v)
        lines.append("")
        lines.append(f"[{k}]")
        for c, v in avg.items():
            lines.append(f"{c}: {v:.6e}")
        if "SQ_INSTS_VALU_MFMA_MOPS_F32" in avg or "SQ_INSTS_VALU_MFMA_MOPS_F64" in avg:
            fl = 512.0 * (avg.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0) + avg.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0))
            lines.append(f"derived_mfma_flop: {fl:.6e}")
        if "SQ_VALU_MFMA_BUSY_CYCLES" in avg and avg.get("duration_ns"):
            # busy cycles summed over the 1024 SIMDs, over the dispatch's cycles at the peak clock
            lines.append(f"derived_mfma_busy_frac: "
                         f"{avg['SQ_VALU_MFMA_BUSY_CYCLES'] / (1024 * avg['duration_ns'] * CLOCK_GHZ):.4f}")
        mf = avg.get("SQ_INSTS_MFMA") or (avg.get("SQ_INSTS_VALU_MFMA_F32", 0.0) + avg.get("SQ_INSTS_VALU_MFMA_F64", 0.0))
        if mf:
            if "SQ_INSTS_VALU" in avg:
                lines.append(f"derived_valu_per_mfma: {(avg['SQ_INSTS_VALU'] - mf) / mf:.3f}")
            if "SQ_INSTS_LDS" in avg:
                lines.append(f"derived_lds_per_mfma: {avg['SQ_INSTS_LDS'] / mf:.3f}")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def kernel_summary(stats_csv, trace_csv, out, command, title, last):
    """Kernel-time summary of a rocprofv3 --kernel-trace --stats run: the
    profiler's own statistics over every dispatch (the autotuner's candidate
    launches included), then, from the trace, each kernel's average over its
    last ``last`` dispatches (the run whose HIP-event times the bench reports)."""
    def short(n):
        n = re.sub(r"dmwf::\(anonymous namespace\)::", "", n)
        return re.sub(r"\(.*$", "", n)[:60]
    lines = [f"# {title}", f"# command: {command}", "# rocprofv3 kernel statistics over all dispatches (microseconds)",
             f"{'kernel':60s} {'calls':>6s} {'avg_us':>12s} {'min_us':>12s} {'max_us':>12s} {'pct':>7s}"]
    for r in csv.DictReader(open(stats_csv)):
        if float(r["Percentage"]) < 0.01:
            continue
        lines.append(f"{short(r['Name']):60s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:12.1f} "
                     f"{float(r['MinNs']) / 1e3:12.1f} {float(r['MaxNs']) / 1e3:12.1f} {float(r['Percentage']):7.2f}")
    per = {}
    for r in csv.DictReader(open(trace_csv)):
        per.setdefault(short(r["Kernel_Name"]), []).append(
            (int(r["Dispatch_Id"]), (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3))
    lines += ["", f"# from the kernel trace: average over each kernel's last {last} dispatches (microseconds)",
              f"{'kernel':60s} {'n':>6s} {'avg_us':>12s}"]
    rows = []
    for k, v in per.items():
        d = [t for _, t in sorted(v)][-last:]
        rows.append((sum(d) / len(d), k, len(d)))
    for avg, k, n in sorted(rows, reverse=True):
        if avg >= 50.0:
            lines.append(f"{k:60s} {n:6d} {avg:12.1f}")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


_CPU_WORK = {}      # the CPU baseline's inputs, inherited by forked workers


def _oracle_rings(rings):
    """One worker's share of the CPU baseline: the oracle's synthesis of alm
    on the given rings and its adjoint (the analysis without weights, whose
    cost is the same) summed over the same rings, with one BLAS thread.
    Returns the seconds taken."""
    lmax, nside, alm, maps = (_CPU_WORK[k] for k in ("lmax", "nside", "alm", "maps"))
    from threadpoolctl import threadpool_limits
    from oracle.geometry import healpix_grid
    from oracle.sht import SHT
    with threadpool_limits(limits=1):
        sht = SHT(healpix_grid(nside), lmax, cache_bytes=0)
        t0 = time.perf_counter()
        sht.synthesis(alm, rings=rings)
        sht.adjoint(maps, rings=rings)
        return time.perf_counter() - t0


def cpu_baseline(lmax, nside, alm, maps, cl, K, b, tau, per_core=6, max_workers=16):
    """The CPU FP64 oracle on a bounded sample of one iteration of the same
    workload (one RHS): the transforms (synthesis and adjoint) on a sample
    of rings spread from pole to pole, scaled to all rings, plus the
    harmonic update and the pixel update over the whole map, timed once.
    Single core: per_core rings in one process.  All cores: a pool of
    min(max_workers, cpu count) processes, each with one BLAS thread, on
    per_core rings each (the oracle's transforms are sums over rings, so
    the rings split over processes); the iteration estimate is the pool's
    wall time scaled by all rings over the rings it did."""
    import multiprocessing as mp
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import dm
    from oracle.geometry import healpix_grid
    nr = 4 * nside - 1
    nw = max(1, min(max_workers, os.cpu_count() or 1))

    def spread(count, offset=0.0):
        return sorted(set(int(round((i + offset) * (nr - 1) / max(count - 1, 1))) for i in range(count)))

    one = spread(per_core)
    # the pointwise parts of an iteration (eq 8's filter, eq 9's update) over everything
    with threadpool_limits(limits=1):
        grid = healpix_grid(nside)
        F = dm.messenger_filter(cl, 10.0 * tau, tau)
        t0 = time.perf_counter()
        dm.apply_blocks(F, alm, lmax)
        dm.pix_apply(K, maps) + b
        t_point = time.perf_counter() - t0
    _CPU_WORK.update(lmax=lmax, nside=nside, alm=alm, maps=maps)
    t1 = _oracle_rings(one)
    single = t1 * nr / len(one) + t_point
    # all cores: every worker a sample of its own
    samples = [spread(per_core, (w + 0.5) / nw) for w in range(nw)]
    samples = [[min(r, nr - 1) for r in sm] for sm in samples]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(nw) as pool:
        pool.map(_oracle_rings, samples, chunksize=1)
    wall = time.perf_counter() - t0
    done = sum(len(sm) for sm in samples)
    multi = wall * nr / done + t_point
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": 1.0 / multi, "unit": "RHS-iterations/s", "cores": nw, "kind": "oracle",
            "single_core_value": 1.0 / single, "nproc": os.cpu_count(), "cpu_model": model,
            "sample": f"one oracle iteration at Nside {nside}, lmax {lmax} (one RHS): synthesis and adjoint "
                      f"transforms timed on {len(one)} rings spread pole to pole ({t1:.1f} s on one core) and, "
                      f"with {nw} processes of one BLAS thread each, on {done} rings ({wall:.1f} s wall), "
                      f"scaled to all {nr} rings, plus the filter and pixel update over the whole map "
                      f"({t_point:.1f} s); NumPy FP64, full m range, no symmetry"}


def field_errors(x, ref, nalm, lmax):
    """Relative L2 error per field (T, E, B) of alm x against ref (complex
    [B, 3, nalm]), with m > 0 counted twice; max over RHS.  Also the worst
    bin of width 64 in l per field and the first degree of that bin."""
    import numpy as np
    ms = np.repeat(np.arange(lmax + 1), np.arange(lmax + 1, 0, -1))
    ls = np.concatenate([np.arange(m, lmax + 1) for m in range(lmax + 1)])
    w = np.where(ms > 0, 2.0, 1.0)
    d2 = np.abs(x - ref) ** 2 * w
    r2 = np.abs(ref) ** 2 * w
    tot = np.sqrt(d2.sum(-1) / r2.sum(-1))                       # [B, 3]
    bins = ls // 64
    nb = bins.max() + 1
    worst, where = [], []
    for f in range(3):
        db = np.zeros((x.shape[0], nb))
        rb = np.zeros((x.shape[0], nb))
        for b in range(x.shape[0]):
            db[b] = np.bincount(bins, d2[b, f], nb)
            rb[b] = np.bincount(bins, r2[b, f], nb)
        ok = rb > 0
        e = np.sqrt(np.where(ok, db / np.where(ok, rb, 1), 0)).max(0)      # worst RHS per bin
        worst.append(float(e.max()))
        where.append(int(64 * e.argmax()))
    return tot.max(0).tolist(), worst, where


def eps_table(args, plan, prob, d_t, dev, stream, log):
    """Algorithm 1 with its own stopping rule (beta = 3/4, threshold cooled
    by eta = 1.1 from 1e-4 to the final value, lambda from 1e3) on RHS 0,
    one run per final threshold, each capped at --eps-cap iterations, with
    chi^2 and the Appendix C residual of the iterate every 100 iterations and
    at the end; prints one JSON line."""
    import numpy as np
    import torch
    rows = []
    out = torch.empty((1, 3, plan.nalm * 2), dtype=torch.float64, device=dev)
    d1 = d_t[:1].contiguous()
    plan.set_diagnostics(100)
    for eps in (1e-4, 1e-5, 1e-6):
        plan.set_schedule_eps(1e3, 0.75, 1e-4, eps, 1.1, args.eps_cap)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = plan.wiener_filter_device(d1, out, stream=stream, want_stats=True)[0]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        cauchy, steps = plan.schedule_trace()
        it, c2, rs = plan.diagnostics_trace()
        nsteps = int(np.ceil(np.log(1e3) / -np.log(0.75))) + 1
        rows.append({"eps": eps, "iterations": int(st["iterations"]), "seconds": round(dt, 3),
                     "capped": bool(st["iterations"] >= args.eps_cap),
                     "cooling_step_reached": int(steps[-1]) if steps.size else 0, "cooling_steps": nsteps,
                     "last_cauchy": float(f"{cauchy[-1]:.4e}") if cauchy.size else None,
                     "chi2": float(f"{st['chi2']:.6e}"), "residual": float(f"{st['residual']:.4e}"),
                     "trace_every_100": {"iteration": it.tolist(),
                                         "chi2": [float(f"{v:.6e}") for v in c2[:, 0]],
                                         "residual": [float(f"{v:.4e}") for v in rs[:, 0]]}})
        log(f"[bench] eps {eps:g}: {rows[-1]['iterations']} iterations, {dt:.1f} s, step "
            f"{rows[-1]['cooling_step_reached']}/{nsteps}, chi2 {st['chi2']:.4e}, residual {st['residual']:.3e}")
    plan.set_diagnostics(0)
    nside, lmax = prob["nside"], prob["lmax"]
    print(json.dumps({"kind": "eps_table", "workload": f"HEALPix Nside {nside}, lmax {lmax}, configuration "
                      f"{args.cfg} mask and noise, one RHS, FP64", "schedule": "lambda 1e3, beta 3/4, threshold "
                      "1e-4 cooled by eta 1.1 to eps, cap " + str(args.eps_cap), "chi2_dof_expected":
                      "3 N_obs +- sqrt(6 N_obs)", "n_obs_pixels": int(prob["obs"].sum()), "rows": rows}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cfg", type=int, default=3, choices=[2, 3, 4, 5],
                    help="workload recipe (mask, noise, sizes) of configuration 2..5; 3 is the metric's")
    ap.add_argument("--nside", type=int, default=None, help="override the configuration's Nside")
    ap.add_argument("--lmax", type=int, default=None, help="override the configuration's lmax")
    ap.add_argument("--nrhs", type=int, default=8)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="mixed")
    ap.add_argument("--noise", choices=["diag", "corr"], default="diag",
                    help="diag: diagonal noise, one mask; corr: correlated 3x3 noise with distinct T and P masks")
    ap.add_argument("--refine", type=int, default=0,
                    help="also run one solve with this many Appendix A corrections and report its residuals")
    ap.add_argument("--adaptive", type=float, default=0.0,
                    help="adaptive working resolution factor (>= 1; 0 = off) for the timed and reference solves")
    ap.add_argument("--eps-table", action="store_true",
                    help="instead of the headline: Algorithm 1 under its stopping rule (Sec. 3.2 settings) for "
                         "final thresholds 1e-4, 1e-5, 1e-6 on one RHS (FP64), iterations, time, chi2 and residual "
                         "per run (the layout of the paper's Table 1)")
    ap.add_argument("--eps-cap", type=int, default=2000, help="iteration cap of each --eps-table run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle sample")
    ap.add_argument("--no-check", action="store_true", help="skip the FP64 reference solve and baseline")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with one device copy of 1 GiB (scale for the traffic counters)")
    ap.add_argument("--traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"))
    ap.add_argument("--traffic-command", default="")
    ap.add_argument("--traffic-last", type=int, default=6,
                    help="dispatches per kernel that count (the timed and the profiled run of --steps 3)")
    ap.add_argument("--kernel-summary", nargs=3, metavar=("STATS_CSV", "TRACE_CSV", "OUT"),
                    help="write a kernel-time summary from a rocprofv3 --kernel-trace --stats run")
    ap.add_argument("--counter-summary", nargs="+", metavar="CSV_OR_OUT",
                    help="write a per-kernel counter summary: the --pmc CSV files of the passes, then OUT")
    ap.add_argument("--summary-title", default="")
    ap.add_argument("--summary-last", type=int, default=20,
                    help="dispatches per kernel averaged from the trace (the profiled run of --steps 20)")
    args = ap.parse_args()
    if args.traffic:
        traffic_from_csv(args.traffic[0], args.traffic[1], args.precision, args.nrhs, args.traffic_command,
                         args.traffic_last)
        return
    if args.kernel_summary:
        kernel_summary(*args.kernel_summary, args.traffic_command, args.summary_title, args.summary_last)
        return
    if args.counter_summary:
        counter_summary(args.counter_summary[:-1], args.counter_summary[-1], args.traffic_command,
                        args.summary_title, args.summary_last)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the library has no multi-GPU "
              f"path; batched right-hand sides would shard across GPUs without communication.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1801_05358_amd import dmwf, inputs

    cfg = args.cfg
    B = args.nrhs
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    corr = args.noise == "corr"
    if corr:
        prob = inputs.correlated_problem(cfg, nside=args.nside, lmax=args.lmax)
        ncov, obs = prob["ncov6"], (prob["obs_t"], prob["obs_p"])
    else:
        prob = inputs.make_problem(cfg, nside=args.nside, lmax=args.lmax)
        ncov, obs = prob["ncov"], prob["obs"]
    nside, lmax = prob["nside"], prob["lmax"]
    log(f"[bench] workload cfg={cfg} nside={nside} lmax={lmax} nrhs={B} precision={args.precision}")
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()

    def make_plan(prec, nrhs):
        plan = dmwf.Plan(lmax=lmax, nside=nside, max_rhs=nrhs, device=0, precision=prec)
        plan.set_spectra(prob["cl"])
        plan.set_noise(ncov, obs)
        if args.adaptive:
            plan.set_adaptive_resolution(args.adaptive)
        return plan

    def set_iters(plan, k):
        if k % 10 == 0:
            plan.set_schedule(1e3, k // 10, 10)
        else:
            plan.set_schedule(1e3, 1, k)

    prec = dmwf.MIXED if args.precision == "mixed" else dmwf.FP64
    # precompute, reported apart from the iterations: the plan (grid, FFT and
    # recursion tables, buffers), the spectra and the noise setup (a0)
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    plan = make_plan(prec, B)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    # synthetic data d = Y s + n, made with the library's own synthesis
    s = np.stack([inputs.signal_alm(cfg, lmax, k) for k in range(B)])
    alm_t = torch.from_numpy(s.view(np.float64).reshape(B, 3, -1)).to(dev)
    d_t = torch.empty((B, 3, plan.npix), dtype=torch.float64, device=dev)
    plan.alm2map_device(alm_t, d_t, stream=stream)
    noise = np.stack([inputs.noise_map6(cfg, ncov, prob["obs3"], k) if corr else inputs.noise_map(cfg, ncov, obs, k)
                      for k in range(B)])
    d_t += torch.from_numpy(noise).to(dev)
    del noise
    out_t = torch.empty((B, 3, plan.nalm * 2), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    log("[bench] inputs resident")

    if args.eps_table:
        eps_table(args, plan, prob, d_t, dev, stream, log)
        return

    tune = plan.autotune(B)
    log(f"[bench] autotune {tune}")
    if args.warmup > 0:
        set_iters(plan, args.warmup)
        plan.wiener_filter_device(d_t, out_t, stream=stream)
        torch.cuda.synchronize()
    log("[bench] warmup done")

    set_iters(plan, args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.wiener_filter_device(d_t, out_t, stream=stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"[bench] timed {args.steps} iterations in {dt:.3f} s")
    # per-kernel times (HIP events on the launch stream) from a separate run,
    # so that the events do not perturb the timed one
    # the band limits of the timed schedule (adaptive working resolution)
    band = plan.step_band_limits().tolist()
    # (with adaptive resolution the profiled run repeats the timed schedule,
    # so that its kernel times average over the same band limits)
    prof_it = args.steps if args.adaptive else min(args.steps, 20)
    set_iters(plan, prof_it)
    prof_t = torch.empty_like(out_t)
    plan.profile(True)
    plan.wiener_filter_device(d_t, prof_t, stream=stream)
    torch.cuda.synchronize()
    kt = plan.kernel_times()
    plan.profile(False)
    del prof_t
    log(f"[bench] kernels over {prof_it} profiled iterations: {kt}")
    its = args.steps / dt

    # dominant kernel
    dom = max(("legendre_analysis", "legendre_synthesis"), key=lambda k: kt[k][0])
    ms, n = kt[dom]
    flops = legendre_flops(plan.nrings // 2 + 1, plan.nalm, B)
    if args.adaptive and band:
        # per launch, averaged over the schedule: the points up to each step's band limit
        flops = sum(legendre_flops(plan.nrings // 2 + 1, (L + 1) * (L + 2) // 2, B) for L in band) / len(band)
    achieved = flops / (ms / n * 1e-3) / 1e12
    batched = B >= 8 or args.precision == "mixed"
    if args.precision == "mixed":
        bound, peak = "mfma", PEAK["fp32_mfma"]
    elif batched:
        bound, peak = "mfma", PEAK["fp64_mfma"]
    else:
        bound, peak = "alu", PEAK["fp64_valu"]
    traffic = read_traffic(dom, args.precision, B) if (cfg, nside, lmax, corr) == (3, 1024, 2048, False) else None
    wk = plan.transform_work()
    ring_ms, ring_n = kt["ring_fft_pointwise"]
    ring_traffic = (read_traffic("ring_fft_pointwise", args.precision, B)
                    if (cfg, nside, lmax, corr) == (3, 1024, 2048, False) else None)
    # the mixed path keeps the ring Fourier data in FP32 when the batched
    # matrix-core kernels run (from 2 RHS on); K and b stay FP64
    rb = ring_bytes(plan.npix, plan.nrings, lmax, B, p_ring=4 if (args.precision == "mixed" and B >= 2) else 8)
    band, holes, dyn = prob["band"], prob["holes"], prob["dyn"]
    prec_text = ("mixed: FP32 matrix-core contraction, FP64 recursion, FFT and iterate"
                 if args.precision == "mixed" else "FP64 throughout")
    rec = {
        "metric": METRIC, "value": round(B * its, 3), "unit": "RHS-iterations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * dt / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"HEALPix Nside {nside}, lmax {lmax}, " + (
                               f"T mask |b|<{band:.4g} deg + {2 * holes} holes, P mask |b|<{band - 3:.4g} deg + "
                               f"{holes} other holes, correlated 3x3 scan noise {dyn:g}:1 (Q = U = 2 T, "
                               f"correlations .3/-.15/.2), "
                               if corr else
                               f"mask |b|<{band:.4g} deg + {holes} holes of 0.5 deg, scan noise {dyn:g}:1 "
                               f"(Q = U = 2 T), ") +
                               f"cooling lambda 1e3 -> 1 in steps of 10 "
                               f"iterations, {B} right-hand sides per launch ({prec_text})" +
                               (f", adaptive working resolution factor {args.adaptive:g}" if args.adaptive else ""),
                   "recipe": f"configuration {cfg}", "nside": nside, "lmax": lmax, "nrhs": B,
                   "precision": args.precision, "noise": args.noise},
        "setup_s": round(setup_s, 3),
        "solve_iterations_per_s": round(its, 4),
        "rhs_iterations_per_s": round(B * its, 3),
        "roofline": {"bound": bound, "kernel": dom, "achieved": round(achieved, 3), "peak": peak,
                     "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                     "traffic": traffic,
                     # the points at or above their start degrees, where the
                     # kernels run the recursion and contraction
                     "executed_points_ratio": round(wk[1] / wk[0], 4),
                     "executed_frac": round(achieved * wk[1] / wk[0] / peak, 4)},
        "kernels_ms_avg": {k: round(v[0] / max(v[1], 1), 4) for k, v in kt.items()},
        "autotune": {k: tune[k] for k in ("syn_mchunk", "ana_mchunk", "syn_waves", "ring_big_threads",
                                          "ring_small_threads")},
        "ring_fft_hbm": {"achieved": round(rb / (ring_ms / max(ring_n, 1) * 1e-3) / 1e9, 1), "peak": HBM_PEAK,
                         "unit": "GB/s", "frac": round(rb / (ring_ms / max(ring_n, 1) * 1e-3) / 1e9 / HBM_PEAK, 4),
                         "algorithmic_bytes": rb, "traffic": ring_traffic},
    }
    # the ring step's LDS roofline: its LDS bytes at the measured read and
    # write rates, against the measured step time
    lds = ring_lds_bytes(nside, lmax, B)
    if lds is not None:
        rr, wr = lds_rates()
        floor_ms = 1e3 * (lds[0] / rr + lds[1] / wr)
        step_ms = ring_ms / max(ring_n, 1)
        rec["ring_fft_lds"] = {"bound": "lds", "read_bytes": lds[0], "write_bytes": lds[1],
                               "floor_ms": round(floor_ms, 4), "measured_ms": round(step_ms, 4),
                               "frac": round(floor_ms / step_ms, 4),
                               "peak": "measured read/write rates, profiles/lds_bandwidth_mi355x.txt"}

    if args.adaptive:
        rec["adaptive_resolution"] = {"factor": args.adaptive,
                                      "band_limits_per_cooling_step": band,
                                      "note": "roofline flops averaged over the cooling steps' band limits"}

    if args.refine > 0:
        # Appendix A's corrections on the same batch and schedule (reported
        # beside the line; `value` is the plain solve's rate)
        log(f"[bench] refined solve, {args.refine} corrections")
        set_iters(plan, args.steps)
        plan.set_refinement(args.refine)
        ref_out = torch.empty_like(out_t)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plan.wiener_filter_device(d_t, ref_out, stream=stream)
        torch.cuda.synchronize()
        tr = time.perf_counter() - t1
        h = plan.refinement_trace()
        rec["refinement"] = {"corrections": args.refine, "iterations_per_run": args.steps, "seconds": round(tr, 3),
                             "wf_residual_max_over_rhs": [float(f"{v:.3e}") for v in h.max(axis=1)],
                             "note": "relative Wiener filter residual before each correction and after the last"}
        plan.set_refinement(0)
        del ref_out

    # the timed plan's device memory goes back before the reference plans
    # are made (at Nside 2048 two 8-RHS plans do not fit together)
    nalm = plan.nalm
    del plan
    gc.collect()
    torch.cuda.synchronize()
    if not args.no_check:
        # the same RHS through the plain FP64 path, same schedule
        if args.precision == "mixed":
            log("[bench] FP64 reference solve")
            ref_plan = make_plan(dmwf.FP64, B)
            ref_t = torch.empty_like(out_t)
            set_iters(ref_plan, args.steps)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ref_plan.wiener_filter_device(d_t, ref_t, stream=stream)
            torch.cuda.synchronize()
            tr = time.perf_counter() - t1
            x = out_t.cpu().numpy().view(np.complex128).reshape(B, 3, -1)
            r = ref_t.cpu().numpy().view(np.complex128).reshape(B, 3, -1)
            tot, worst, where = field_errors(x, r, nalm, lmax)
            rec["accuracy"] = {"reference": f"FP64 GPU path, same {B} RHS and schedule",
                               "rel_l2_T_E_B": [float(f"{v:.3e}") for v in tot],
                               "worst_l_bin_T_E_B": [float(f"{v:.3e}") for v in worst],
                               "worst_l_bin_start_T_E_B": where,
                               "max": float(f"{max(tot):.3e}"), "gate": ACC_GATE,
                               "gate_on": "relative L2 per field over all (l, m)",
                               "pass": max(tot) <= ACC_GATE,
                               "bins_pass": max(worst) <= ACC_GATE}
            rec["fp64_same_batch_rhs_iterations_per_s"] = round(B * args.steps / tr, 3)
            del ref_plan, ref_t
        log("[bench] FP64 single-RHS baseline")
        base = make_plan(dmwf.FP64, 1)
        bout = torch.empty((1, 3, base.nalm * 2), dtype=torch.float64, device=dev)
        set_iters(base, args.warmup if args.warmup > 0 else 10)
        base.wiener_filter_device(d_t[:1].contiguous(), bout, stream=stream)
        set_iters(base, args.steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        base.wiener_filter_device(d_t[:1].contiguous(), bout, stream=stream)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t1
        rec["fp64_b1_iterations_per_s"] = round(args.steps / tb, 4)
        rec["speedup_vs_fp64_b1"] = round(B * its / (args.steps / tb), 3)
        del base, bout
    if args.calibrate_copy:
        src = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_cpu:
        log("[bench] timing the CPU oracle sample")
        from oracle import dm
        from oracle.geometry import healpix_grid
        st = dm.setup(healpix_grid(nside), ncov, obs, inputs.noise_map(cfg, ncov, obs, 0))
        rec["cpu_baseline"] = cpu_baseline(lmax, nside, s[0], st["d0"], prob["cl"], st["K"], st["b"], st["tau"])
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
