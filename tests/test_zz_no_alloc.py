"""GPU test of pkm_kmu_global_noalloc, the (k, mu) binning for callers that cannot allocate
device memory, called through the C ABI and checked against pkm_kmu_global on the same
painted plan: mode counts exactly, P(k, mu) to FP64 rounding (the two accumulate their sums
over different block counts).  Two calls in a row, the second with fewer cells, so that
what the first left in the shared scratch array cannot leak into the second."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest

from tests.parity_util import small_catalogs

pytestmark = pytest.mark.gpu

L = 300.0
OBS = (30.0, -40.0, -700.0)


def _call(fn, plan, ke, me):
    ke = np.ascontiguousarray(ke, dtype=np.float64)
    me = np.ascontiguousarray(me, dtype=np.float64)
    pk = np.full((ke.size - 1, me.size - 1), -7.0)
    nm = np.full((ke.size - 1, me.size - 1), -7, dtype=np.int64)
    st = fn(plan.h, ke.ctypes.data_as(C.c_void_p), ke.size, me.ctypes.data_as(C.c_void_p), me.size,
            pk.ctypes.data_as(C.c_void_p), nm.ctypes.data_as(C.c_void_p))
    return st, pk, nm


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_kmu_matches_allocating_entry_point(gpu, prec):
    from paper_1704_02357_amd import Plan
    from paper_1704_02357_amd.pkm import load_library
    lib = load_library()
    n = 48
    d, r = small_catalogs(4000, 30000, L, seed=61)
    plan = Plan(n, L, observer=OBS, window=3, interlaced=True, compensated=True, precision=prec,
                los=(1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0))
    plan.paint(d, r)
    kf = 2 * np.pi / L
    cases = [(np.arange(0.5, 24.0, 0.5) * kf, np.linspace(0.0, 1.0, 21)),   # 47 x 20 cells
             (np.array([1.0, 3.0, 6.0, 9.0]) * kf, np.array([0.0, 0.3, 0.8, 1.0]))]  # 3 x 3 cells
    for i, (ke, me) in enumerate(cases):
        print(f"[case] noalloc kmu prec={prec} call {i}: {ke.size - 1} x {me.size - 1} cells", flush=True)
        st_a, pk_a, nm_a = _call(lib.pkm_kmu_global, plan, ke, me)
        st_b, pk_b, nm_b = _call(lib.pkm_kmu_global_noalloc, plan, ke, me)
        assert st_a == 0 and st_b == 0, (st_a, st_b, lib.pkm_plan_last_error(plan.h))
        assert np.array_equal(nm_a, nm_b)
        assert nm_a.sum() > 0
        full = nm_a > 0
        assert np.array_equal(np.isnan(pk_a), ~full) and np.array_equal(np.isnan(pk_b), ~full)
        raw = np.abs(pk_a[full]) + plan_shot(plan, d, r)
        err = float(np.max(np.abs(pk_b[full] - pk_a[full]) / raw))
        print(f"[noalloc] prec={prec} call {i} max scaled diff {err:.2e}", flush=True)
        assert err <= 1e-12
    # beyond the scratch array's 3072 cells: refused, outputs untouched
    st, pk, nm = _call(lib.pkm_kmu_global_noalloc, plan, np.linspace(0.0, 0.6, 102), np.linspace(0.0, 1.0, 32))
    assert st == 1 and np.all(pk == -7.0) and np.all(nm == -7)
    assert b"3072" in lib.pkm_plan_last_error(plan.h)
    plan.close()


def plan_shot(plan, d, r):
    """Shot-noise level of the painted catalogs (scale of the raw power), from a multipole call."""
    res = plan.compute_multipoles(0, np.array([0.0, 0.05]))
    return res["shot_noise"]
