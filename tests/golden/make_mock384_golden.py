"""Write the oracle's P_l(k) for one 384^3 covariance mock to tests/golden/.

Runs only the FP64 oracle (oracle/) on synth.batch_mock(2): the third mock of the uneven-size
batch (Nmesh 384, L = 2000 Mpc/h, seeded lognormal survey, 10x randoms), painted with TSC,
interlacing and compensation, observer at (0, 0, -1500) Mpc/h, even l <= 4, k edges 0.01 h/Mpc
up to the Nyquist frequency.  Takes a few minutes and ~10 GB of memory on 8 cores.

    python tests/golden/make_mock384_golden.py [--workers 8]
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
from synth import batch_mock, catalog_digest  # noqa: E402

MOCK, BOX, ELL_MAX = 2, 2000.0, 4
OBSERVER = (0.0, 0.0, -1500.0)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mock384_l4_poles.txt")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=8)
    args = ap.parse_args()
    t0 = time.perf_counter()
    data, rand, info, n = batch_mock(MOCK)
    assert n == 384
    kn = math.pi * n / BOX
    edges = np.arange(int(math.floor(kn / 0.01)) + 1, dtype=np.float64) * 0.01
    p = default_params(n, BOX, observer=OBSERVER, window=3, interlaced=True, compensated=True)
    res = multipoles(data, rand, p, ELL_MAX, edges, workers=args.workers)
    with open(OUT, "w") as f:
        f.write("# FP64 oracle P_l(k) of one 384^3 covariance mock (Sec. 2.1, eqs. for P_l and A_l; FKP field\n")
        f.write("# and normalisation of Sec. 2; TSC + interlacing + compensation of Sec. 2.3).\n")
        f.write("# Written by tests/golden/make_mock384_golden.py from oracle/ only.\n")
        f.write(f"# catalog: synth.batch_mock({MOCK}), n_data {info['n_data']}, n_rand {info['n_rand']}, "
                f"digest {catalog_digest(data, rand)}\n")
        f.write(f"# nmesh {n} box_len {BOX} observer {OBSERVER} window 3 interlaced 1 compensated 1\n")
        f.write(f"# alpha {res['alpha']!r}\n# norm_I {res['norm_I']!r}\n# shot_noise {res['shot_noise']!r}\n")
        f.write("# columns: k_lo k_hi n_modes k_mean P0 P2 P4\n")
        for b in range(len(edges) - 1):
            row = [edges[b], edges[b + 1], res["n_modes"][b], res["k_mean"][b]] + [res["poles"][i][b] for i in range(3)]
            f.write(" ".join(repr(float(v)) if i != 2 else str(int(v)) for i, v in enumerate(row)) + "\n")
    print(f"wrote {OUT} in {time.perf_counter() - t0:.0f} s")


if __name__ == "__main__":
    main()
