"""Writes tests/golden/dm_nside2_lmax4.txt: a tiny seeded dual messenger
problem (HEALPix Nside 2, lmax 4; configuration 1's recipe) with the CPU
oracle's results.  Calls only oracle/ and the seeded input generators.

Stored: the spectra, the noise variances, the mask and the data (inputs),
then the oracle's analysis A d, its plain solve (Algorithm 1 under the
fixed cooling, 3 steps x 4 iterations from lambda 1e3) and the solve with
two corrections of Appendix A's relaxation (its last iterate, and the
iterate of smallest residual).  Usage:
    python tests/golden/make_golden.py
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import dm  # noqa: E402
from oracle.geometry import healpix_grid  # noqa: E402
from oracle.sht import SHT  # noqa: E402
from paper_1801_05358_amd import inputs  # noqa: E402

NSIDE, LMAX = 2, 4
SCHED = (1e3, 3, 4)
NCORR = 2
OUT = os.path.join(HERE, "dm_nside2_lmax4.txt")


def problem():
    p = inputs.make_problem(1, nside=NSIDE, lmax=LMAX)
    sht = SHT(healpix_grid(NSIDE), LMAX)
    d = sht.synthesis(inputs.signal_alm(1, LMAX, 0)) + inputs.noise_map(1, p["ncov"], p["obs"], 0)
    return p, sht, d


def results(p, sht, d):
    return {
        "analysis": sht.analysis(d),
        "u_plain": dm.solve(sht, d, p["ncov"], p["obs"], p["cl"], *SCHED)["u"],
        "u_refined": dm.refine(sht, d, p["ncov"], p["obs"], p["cl"], *SCHED, NCORR)["u"],
        "u_refined_best": dm.refine(sht, d, p["ncov"], p["obs"], p["cl"], *SCHED, NCORR, select="best")["u"],
    }


def write():
    p, sht, d = problem()
    res = results(p, sht, d)
    lines = [
        "# Tiny dual messenger problem, HEALPix Nside 2 (48 pixels), lmax 4, and the CPU oracle's results.",
        "# Written by tests/golden/make_golden.py (oracle/ and the seeded inputs only).",
        f"# schedule: lambda0 {SCHED[0]:g}, {SCHED[1]} cooling steps x {SCHED[2]} iterations (Algorithm 1,",
        "# fixed cooling); refined: the same plus "
        f"{NCORR} corrections of Appendix A's relaxation, returning the last iterate",
        "# (u_refined) or the iterate of smallest Wiener filter residual (u_refined_best).",
        "# alm: fields T, E, B; m-major triangular, index m (2 lmax + 1 - m) / 2 + l; 're im' per value.",
        "# Sections: name, shape, then one value (or one 're im' pair) per line.",
    ]

    def real(name, a):
        a = np.asarray(a, dtype=float)
        lines.append(f"[{name}] {' '.join(str(x) for x in a.shape)}")
        lines.extend(repr(float(v)) for v in a.reshape(-1))

    def cplx(name, a):
        lines.append(f"[{name}] {' '.join(str(x) for x in a.shape)} complex")
        lines.extend(f"{float(v.real)!r} {float(v.imag)!r}" for v in a.reshape(-1))

    real("cl", p["cl"])
    real("ncov", p["ncov"])
    real("obs", p["obs"].astype(float))
    real("d", d)
    for k, v in res.items():
        cplx(k, v)
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


def read(path=OUT):
    """{name: array} from the fixture."""
    out, name, shape, is_c, vals = {}, None, None, False, []

    def close():
        if name is not None:
            a = np.array(vals)
            if is_c:
                a = a[:, 0] + 1j * a[:, 1]
            out[name] = a.reshape(shape)

    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("["):
            close()
            head, rest = line[1:].split("]")
            parts = rest.split()
            is_c = parts[-1] == "complex"
            shape = tuple(int(x) for x in (parts[:-1] if is_c else parts))
            name, vals = head, []
        else:
            vals.append([float(x) for x in line.split()] if is_c else float(line))
    close()
    return out


if __name__ == "__main__":
    write()
    print(OUT)
