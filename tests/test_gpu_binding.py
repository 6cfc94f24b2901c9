"""GPU tests of the Python binding's process set-up: a plan created before the caller has
touched torch (the binding loads torch's HIP runtime before the library, and initialises
torch's device state before routing allocations through its caching allocator)."""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("first", ["plan", "wedges"])
def test_plan_before_torch_import(gpu, first):
    # a fresh interpreter: nothing but the package is imported before the first call
    code = ("import sys, numpy as np\n"
            "from paper_1704_02357_amd import Plan, wedges\n"
            "if sys.argv[1] == 'wedges':\n"
            "    wedges(np.ones((3, 4)), 4, np.linspace(0.0, 1.0, 3))\n"
            "rng = np.random.default_rng(1)\n"
            "pos = rng.uniform(-50.0, 50.0, (2000, 3))\n"
            "nb = np.full(2000, 2000 / 100.0 ** 3)\n"
            "with Plan(32, 100.0, observer=(0.0, 0.0, -300.0)) as p:\n"
            "    p.paint((pos, None, nb), None)\n"
            "    r = p.compute_multipoles(2, np.arange(0.0, 0.9, 0.1))\n"
            "assert np.isfinite(r['poles'][0][1:]).all()\n"
            "print('binding ok', flush=True)\n")
    r = subprocess.run([sys.executable, "-c", code, first], cwd=ROOT, capture_output=True, text=True, timeout=300)
    print(r.stdout[-500:], r.stderr[-2000:])
    assert r.returncode == 0 and "binding ok" in r.stdout
