"""Write the oracle's P_l(k) for the 512^3, l <= 4 survey workload to tests/golden/.

Runs only the FP64 oracle (oracle/) on the seeded synthetic catalog of synth.config_c2
(1e6 lognormal galaxies, 2e7 randoms, L = 2500 Mpc/h), with TSC painting, interlacing and
compensation, observer at (0, 0, -1500) Mpc/h and 64 k bins of width 0.01 h/Mpc.  Takes about
10 minutes and ~25 GB of memory on 8 cores.

    python tests/golden/make_workload_golden.py [--workers 8]
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.estimator import default_params, multipoles  # noqa: E402
from synth import catalog_digest, config_c2  # noqa: E402

NMESH, BOX, ELL_MAX = 512, 2500.0, 4
OBSERVER = (0.0, 0.0, -1500.0)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "workload_512_l4_poles.txt")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=8)
    args = ap.parse_args()
    t0 = time.perf_counter()
    data, rand, info = config_c2()
    kn = math.pi * NMESH / BOX
    edges = np.arange(int(math.floor(kn / 0.01)) + 1, dtype=np.float64) * 0.01
    p = default_params(NMESH, BOX, observer=OBSERVER, window=3, interlaced=True, compensated=True)
    res = multipoles(data, rand, p, ELL_MAX, edges, workers=args.workers)
    with open(OUT, "w") as f:
        f.write("# FP64 oracle P_l(k) of the 512^3, l <= 4 survey workload (Sec. 2.1, eqs. for P_l and A_l;\n")
        f.write("# FKP field and normalisation of Sec. 2; TSC + interlacing + compensation of Sec. 2.3).\n")
        f.write("# Written by tests/golden/make_workload_golden.py from oracle/ only.\n")
        f.write(f"# catalog: synth.config_c2(), n_data {info['n_data']}, n_rand {info['n_rand']}, "
                f"digest {catalog_digest(data, rand)}\n")
        f.write(f"# nmesh {NMESH} box_len {BOX} observer {OBSERVER} window 3 interlaced 1 compensated 1\n")
        f.write(f"# alpha {res['alpha']!r}\n# norm_I {res['norm_I']!r}\n# shot_noise {res['shot_noise']!r}\n")
        f.write("# columns: k_lo k_hi n_modes k_mean P0 P2 P4\n")
        for b in range(len(edges) - 1):
            row = [edges[b], edges[b + 1], res["n_modes"][b], res["k_mean"][b]] + [res["poles"][i][b] for i in range(3)]
            f.write(" ".join(repr(float(v)) if i != 2 else str(int(v)) for i, v in enumerate(row)) + "\n")
    print(f"wrote {OUT} in {time.perf_counter() - t0:.0f} s")


if __name__ == "__main__":
    main()
