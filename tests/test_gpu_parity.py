"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same
seeded inputs.  Sizes span several tiles and ragged tails; the full-size workload case
lives in test_gpu_workloads.py."""
import math

import numpy as np
import pytest

from tests.parity_util import TOL, assert_pole_parity, oracle_params, small_catalogs

pytestmark = pytest.mark.gpu


def _plan(n, L, prec, observer, window=3, interlaced=True, compensated=True, **kw):
    from paper_1704_02357_amd import Plan
    return Plan(n, L, observer=observer, window=window, interlaced=interlaced, compensated=compensated,
                precision=prec, **kw)


OBS = (30.0, -40.0, -700.0)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n", [16, 32, 48, 64, 96, 128, 256])
def test_fft3d_forward_inverse(gpu, prec, n):
    import torch
    print(f"[case] fft3d n={n} prec={prec}", flush=True)
    rdt = torch.float64 if prec else torch.float32
    cdt = torch.complex128 if prec else torch.complex64
    rng = np.random.default_rng(n)
    x = rng.normal(size=(n, n, n))
    plan = _plan(n, 100.0, prec, OBS)
    xin = torch.tensor(x, dtype=rdt, device="cuda")
    out = torch.empty((n, n, n // 2), dtype=cdt, device="cuda")
    plan.fft3d_forward(xin, out)
    ref = np.fft.rfftn(x)[:, :, : n // 2]
    got = out.cpu().numpy()
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    tol = 1e-13 if prec else 2e-6
    assert err < tol, err
    # inverse of the half spectrum (kz = N/2 plane taken as zero)
    full = np.fft.rfftn(x)
    full[:, :, n // 2] = 0.0
    xref = np.fft.irfftn(full, s=(n, n, n))
    xo = torch.empty((n, n, n), dtype=rdt, device="cuda")
    plan.fft3d_inverse(out, xo)
    err = np.max(np.abs(xo.cpu().numpy() - xref)) / np.max(np.abs(xref))
    assert err < tol, err
    plan.close()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("window,interlaced,compensated", [(1, False, False), (2, False, True), (3, True, True),
                                                           (2, True, False)])
def test_paint_and_combined_field(gpu, prec, window, interlaced, compensated):
    from oracle.catalog import catalog_scalars
    from oracle.estimator import density_fields
    print(f"[case] paint prec={prec} window={window} il={interlaced} comp={compensated}", flush=True)
    n, L = 32, 200.0
    d, r = small_catalogs(3000, 20000, L, seed=10 + window)
    plan = _plan(n, L, prec, OBS, window, interlaced, compensated)
    plan.paint(d, r)
    p = oracle_params(n, L, OBS, window, interlaced, compensated)
    sc, c_full, dc = density_fields(d, r, p)
    from oracle.mesh import fkp_meshes
    d1, d2 = fkp_meshes(d, r, sc["alpha"], n, L, p["box_origin"], window, interlaced)
    tol_mesh = 1e-13 if prec else 2e-6
    g1 = plan.read_buffer(0)
    assert np.max(np.abs(g1 - d1)) <= tol_mesh * np.max(np.abs(d1))
    if interlaced:
        g2 = plan.read_buffer(1)
        assert np.max(np.abs(g2 - d2)) <= tol_mesh * np.max(np.abs(d2))
    c = plan.read_buffer(2)
    cref = c_full[:, :, : n // 2]
    tol = 1e-12 if prec else 5e-6
    assert np.max(np.abs(c - cref)) <= tol * np.max(np.abs(cref))
    gdc = plan.read_buffer(3)
    assert np.max(np.abs(gdc - dc)) <= tol * np.max(np.abs(dc))
    plan.close()


CASES = [
    # (n, window, interlaced, compensated, ell_max, with_randoms)
    (32, 3, True, True, 4, True),
    (32, 2, False, True, 4, True),
    (32, 1, False, False, 6, True),
    (48, 3, True, True, 4, True),
    (32, 3, True, True, 16, True),
    (32, 2, False, True, 2, False),
    (16, 3, True, False, 8, True),
]


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("case", CASES, ids=[f"n{c[0]}w{c[1]}i{int(c[2])}c{int(c[3])}l{c[4]}r{int(c[5])}" for c in CASES])
def test_multipoles_small(gpu, prec, case):
    from oracle.estimator import multipoles
    n, window, interlaced, compensated, lmax, with_r = case
    print(f"[case] multipoles prec={prec} {case}", flush=True)
    L = 300.0
    d, r = small_catalogs(4000, 30000 if with_r else 0, L, seed=n + lmax + window)
    edges = np.arange(0.0, math.pi * n / L + 1e-9, 0.03)
    edges = np.append(edges, math.pi * n / L * 1.2)  # a ragged last bin reaching beyond Nyquist
    plan = _plan(n, L, prec, OBS, window, interlaced, compensated, ell_max_hint=lmax)
    plan.paint(d, r)
    got = plan.compute_multipoles(lmax, edges)
    ref = multipoles(d, r, oracle_params(n, L, OBS, window, interlaced, compensated), lmax, edges)
    assert got["n_transforms"] == ref["n_transforms"]
    assert_pole_parity(got, ref, prec, f"n={n} w={window} il={interlaced} c={compensated} l={lmax}")
    plan.close()


@pytest.mark.parametrize("prec", [1, 0])
def test_groups_split_equals_single_group(gpu, prec):
    """Forcing many small field groups (several HBM-resident groups per l) changes nothing
    beyond rounding."""
    n, L = 32, 300.0
    d, r = small_catalogs(3000, 20000, L, seed=5)
    edges = np.linspace(0.02, 0.3, 9)
    a = _plan(n, L, prec, OBS, ell_max_hint=8)
    a.paint(d, r)
    ra = a.compute_multipoles(8, edges)
    b = _plan(n, L, prec, OBS, ell_max_hint=8, max_group=3)
    b.paint(d, r)
    rb = b.compute_multipoles(8, edges)
    assert b.stats()["n_groups"] > a.stats()["n_groups"]
    scale = np.maximum(np.abs(ra["poles"]), np.abs(ra["poles"][0] + ra["shot_noise"]))
    assert np.max(np.abs(ra["poles"] - rb["poles"]) / scale) < (1e-13 if prec else 1e-6)
    assert np.array_equal(ra["n_modes"], rb["n_modes"])


@pytest.mark.parametrize("prec", [1, 0])
def test_repeat_compute_and_repaint(gpu, prec):
    """Several computes after one paint agree; a second paint replaces the first."""
    from oracle.estimator import multipoles
    n, L = 32, 300.0
    d, r = small_catalogs(3000, 20000, L, seed=8)
    d2, r2 = small_catalogs(2000, 15000, L, seed=9)
    edges = np.linspace(0.02, 0.3, 9)
    plan = _plan(n, L, prec, OBS)
    plan.paint(d, r)
    x = plan.compute_multipoles(4, edges)
    y = plan.compute_multipoles(2, edges)
    assert np.allclose(x["poles"][:2], y["poles"], rtol=0, atol=1e-9 * np.max(np.abs(x["poles"])))
    plan.paint(d2, r2)
    z = plan.compute_multipoles(4, edges)
    ref = multipoles(d2, r2, oracle_params(n, L, OBS, 3, True, True), 4, edges)
    assert_pole_parity(z, ref, prec, "repaint")


def test_device_resident_catalog(gpu):
    import torch
    from oracle.estimator import multipoles
    n, L = 32, 300.0
    d, r = small_catalogs(3000, 20000, L, seed=12)
    edges = np.linspace(0.02, 0.3, 9)
    plan = _plan(n, L, 1, OBS)
    T = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    plan.paint((T(d.pos), T(d.w), T(d.nbar)), (T(r.pos), T(r.w), T(r.nbar)))
    got = plan.compute_multipoles(4, edges)
    ref = multipoles(d, r, oracle_params(n, L, OBS, 3, True, True), 4, edges)
    assert_pole_parity(got, ref, 1, "device catalog")


@pytest.mark.parametrize("prec", [1, 0])
def test_kmu_global(gpu, prec):
    from oracle.global_los import pkmu
    n, L = 32, 300.0
    d, r = small_catalogs(3000, 20000, L, seed=14)
    kedges = np.linspace(0.02, 0.3, 8)
    muedges = np.array([0.0, 0.05, 0.25, 0.5, 0.75, 1.0])
    los = (0.0, 0.0, 1.0)
    plan = _plan(n, L, prec, OBS, los=los)
    plan.paint(d, r)
    pk, nm = plan.kmu_global(kedges, muedges)
    pref, nref = pkmu(d, r, oracle_params(n, L, OBS, 3, True, True), kedges, muedges, los)
    assert np.array_equal(nm, nref)
    ok = nref > 0
    raw = np.abs(pref) + 1.0 / (3000 / L ** 3)
    assert np.max(np.abs(pk[ok] - pref[ok]) / raw[ok]) < TOL[prec]


def test_error_paths(gpu):
    from paper_1704_02357_amd import PkmError
    n, L = 16, 100.0
    plan = _plan(n, L, 1, OBS)
    with pytest.raises(PkmError) as e:
        plan.compute_multipoles(4, [0.0, 0.1, 0.2])
    assert e.value.status == 2  # compute before paint
    d, r = small_catalogs(100, 1000, L, seed=1)
    with pytest.raises(PkmError) as e:
        plan.paint(d, (r.pos, r.w, None))   # randoms without nbar
    assert e.value.status == 1
    plan.paint(d, r)
    for bad in ([0.1, 0.1, 0.2], [0.2, 0.1], [-0.1, 0.1], [0.1]):
        with pytest.raises(PkmError) as e:
            plan.compute_multipoles(4, bad)
        assert e.value.status == 1
    with pytest.raises(PkmError):
        plan.compute_multipoles(3, [0.0, 0.1])
    with pytest.raises(PkmError):
        plan.compute_multipoles(18, [0.0, 0.1])
    with pytest.raises(PkmError) as e:
        plan.kmu_global([0.0, 0.1], [0.0, 1.0])   # plan has no global line of sight
    assert e.value.status == 1
    # the plan still works after rejected calls
    assert np.isfinite(plan.compute_multipoles(2, [0.07, 0.2, 0.3])["poles"]).any()


@pytest.mark.parametrize("prec", [1, 0])
def test_edge_cases(gpu, prec):
    """Particles outside the box wrap; a single galaxy in a periodic box; empty bins -> NaN."""
    from oracle.estimator import multipoles
    n, L = 16, 100.0
    rng = np.random.default_rng(4)
    from synth import Catalog
    pos = rng.uniform(-90, 90, (500, 3))          # reaches far outside [-50, 50)
    d = Catalog(pos, None, None)
    edges = np.array([0.0, 0.01, 0.07, 0.2, 0.5, 2.0])   # first bin empty, last beyond Nyquist
    p = oracle_params(n, L, OBS, 3, True, True)
    plan = _plan(n, L, prec, OBS)
    plan.paint(d, None)
    got = plan.compute_multipoles(4, edges)
    ref = multipoles(d, None, p, 4, edges)
    assert got["n_modes"][0] == 0 and np.all(np.isnan(got["poles"][:, 0])) and np.isnan(got["k_mean"][0])
    assert_pole_parity(got, ref, prec, "edge")
    one = Catalog(np.array([[1.0, 2.0, 3.0]]), None, None)
    plan.paint(one, None)
    got = plan.compute_multipoles(2, edges)
    ref = multipoles(one, None, p, 2, edges)
    assert_pole_parity(got, ref, prec, "one galaxy")


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("observer", [(0.0, 0.0, 0.0), (-103.125, 37.5, -65.625), (-1000.0, -1000.0, -1000.0)],
                         ids=["centre-node", "interior-node", "along-111"])
def test_observer_positions(gpu, prec, observer):
    """Observers at the box centre and at an interior mesh node (a node with no direction:
    its weighted values are zero for l > 0), and one whose line of sight already lies along
    (1,1,1): the harmonic frame is then the identity.  l <= 8 against the oracle."""
    from oracle.estimator import multipoles
    n, L = 32, 300.0
    d, r = small_catalogs(4000, 30000, L, seed=77)
    edges = np.arange(0.0, math.pi * n / L + 1e-9, 0.03)
    print(f"[case] observer={observer} prec={prec}", flush=True)
    plan = _plan(n, L, prec, observer, ell_max_hint=8)
    plan.paint(d, r)
    got = plan.compute_multipoles(8, edges)
    plan.close()
    ref = multipoles(d, r, oracle_params(n, L, observer, 3, True, True), 8, edges)
    assert_pole_parity(got, ref, prec, f"observer {observer}")


@pytest.mark.parametrize("prec", [0, 1])
def test_paint_weights_over_three_decades(gpu, prec):
    """Painted meshes (both, interlaced TSC) for weights log-uniform in [0.01, 10] on data and
    randoms: the FP32 form accumulates in fixed point with a per-tile scale set by the
    largest |w|, the FP64 form in FP64."""
    from oracle.catalog import catalog_scalars
    from oracle.mesh import fkp_meshes
    from synth import Catalog
    n, L = 32, 200.0
    rng = np.random.default_rng(303)
    o = -0.5 * L
    nd, nr = 4000, 30000
    d = Catalog(o + rng.random((nd, 3)) * L, 10.0 ** rng.uniform(-2, 1, nd), np.full(nd, nd / L ** 3))
    r = Catalog(o + rng.random((nr, 3)) * L, 10.0 ** rng.uniform(-2, 1, nr), np.full(nr, nd / L ** 3))
    print(f"[case] paint three-decade weights prec={prec}", flush=True)
    plan = _plan(n, L, prec, OBS, 3, True, True)
    plan.paint(d, r)
    sc = catalog_scalars(d, r, L)
    p = oracle_params(n, L, OBS, 3, True, True)
    d1, d2 = fkp_meshes(d, r, sc["alpha"], n, L, p["box_origin"], 3, True)
    tol = 1e-13 if prec else 2e-6
    for which, ref in ((0, d1), (1, d2)):
        got = plan.read_buffer(which)
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        print(f"[paint] mesh {which} prec={prec} max_err/max={err:.2e}", flush=True)
        assert err <= tol
    plan.close()
