"""CPU checks of bench.py's host logic (no GPU): it refuses more than one
GPU with a message, a committed traffic summary counts only while the
kernel source it was measured on is unchanged, and the kernel-time summary keeps each
kernel's last dispatches (the run whose HIP-event times the bench
reports), leaving out the autotuner's earlier candidate launches."""

import csv
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
bench = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(bench)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_committed_traffic_summaries_follow_their_sources():
    """A traffic summary counts only while the kernel source it was measured
    on is unchanged: read_traffic gives its bytes then, and None after a
    change (the bench line then reports traffic null)."""
    for kernel in ("legendre_analysis", "legendre_synthesis"):
        path = bench.traffic_file(kernel, "mixed", 8)
        assert os.path.exists(path), path
        sha = [l.split(":", 1)[1].strip() for l in open(path) if l.startswith("source_sha256_16")][0]
        rec = bench.read_traffic(kernel, "mixed", 8)
        if sha == bench.source_sha(kernel):
            assert rec is not None and rec > 0, kernel
        else:
            assert rec is None, kernel


def test_kernel_summary_keeps_the_last_dispatches(tmp_path):
    stats = tmp_path / "stats.csv"
    trace = tmp_path / "trace.csv"
    with open(stats, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs"])
        w.writerow(["void bana_kernel<float, 8, float>(x)", 4, 0, 2500, 90.0, 1000, 4000])
        w.writerow(["tiny_kernel", 1, 0, 10, 0.001, 10, 10])
    with open(trace, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kind", "Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        # two candidate launches first (400 us), then two tuned ones (100 us, 300 us)
        for did, dur in ((1, 400000), (2, 400000), (3, 100000), (4, 300000)):
            w.writerow(["KERNEL_DISPATCH", did, "void bana_kernel<float, 8, float>(x)", 100, 100 + dur])
    out = tmp_path / "summary.txt"
    bench.kernel_summary(str(stats), str(trace), str(out), "cmd", "title", 2)
    text = out.read_text()
    assert "# command: cmd" in text and "tiny_kernel" not in text
    last = [l for l in text.splitlines() if l.startswith("void bana_kernel") and l.split()[-2] == "2"]
    assert last and float(last[0].split()[-1]) == 200.0


def test_ring_lds_model_counts_passes():
    """The LDS model of the ring step, by hand at Nside 1 (two ring pairs of
    4 pixels, one radix-4 pass per transform): per field and pair the fold
    writes 4 elements, the two transforms read and write 4 each, the update
    reads and writes 4, the unfold reads 2 (mmax + 1) = 6, at 16 bytes per
    element, 3 fields.  A split length (a Bluestein size above the LDS
    buffer, Nside 2048) has no model."""
    r, w = bench.ring_lds_bytes(1, 2, 1)
    assert r == 2 * (2 * 4 + 4 + 6) * 16 * 3 and w == 2 * (4 + 2 * 4 + 4) * 16 * 3
    r, w = bench.ring_lds_bytes(1024, 2048, 8)
    assert abs(r / 1e9 - 58.39) < 0.01 and abs(w / 1e9 - 59.72) < 0.01
    assert bench.ring_lds_bytes(2048, 4096, 8) is None
    rr, wr = bench.lds_rates()
    assert 1e13 < wr < rr < 2e14


def test_field_errors_find_the_worst_bin():
    """The accuracy record: a relative perturbation of 1e-3 on degrees >= 128
    of one RHS's B field is the worst 64-wide bin (starting at 128) with error
    1e-3; the other fields are exact."""
    import numpy as np
    lmax = 130
    nalm = (lmax + 1) * (lmax + 2) // 2
    rng = np.random.default_rng(0)
    ref = rng.standard_normal((2, 3, nalm)) + 1j * rng.standard_normal((2, 3, nalm))
    x = ref.copy()
    ls = np.concatenate([np.arange(m, lmax + 1) for m in range(lmax + 1)])
    x[1, 2, ls >= 128] *= 1 + 1e-3
    tot, worst, where = bench.field_errors(x, ref, nalm, lmax)
    assert tot[:2] == [0.0, 0.0] and 0 < tot[2] < 1e-3
    assert worst[:2] == [0.0, 0.0] and abs(worst[2] - 1e-3) < 1e-12
    assert where[2] == 128
