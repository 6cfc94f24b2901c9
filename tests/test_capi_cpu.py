"""C ABI checks that need no GPU: the library loads, exports every declared symbol, and its
host-only entry points agree with the oracle; parameter validation rejects bad input
before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pkm.h")


def _lib():
    from paper_1704_02357_amd.pkm import load_library, lib_path
    if not os.path.exists(lib_path()):
        pytest.skip("libpkm.so not built")
    return load_library()


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pkm_[a-z0-9_]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    lib = _lib()
    syms = declared_symbols()
    assert len(syms) >= 14
    for s in syms:
        assert hasattr(lib, s), s
    from paper_1704_02357_amd import ABI_VERSION
    assert lib.pkm_abi_version() == ABI_VERSION
    assert lib.pkm_status_str(0) == b"ok"
    assert lib.pkm_status_str(2) == b"compute before paint"


def test_wedges_match_oracle():
    from paper_1704_02357_amd import wedges
    from oracle.wedges import wedges as owedges
    rng = np.random.default_rng(3)
    poles = rng.normal(size=(9, 7))
    for edges in (np.linspace(0, 1, 11), np.array([0, 0.05, 0.3, 0.31, 0.9, 1.0])):
        got = wedges(poles, 16, edges)
        ref = owedges(poles, list(range(0, 17, 2)), edges)
        assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


def test_nonuniform_edges_match_oracle():
    from paper_1704_02357_amd import nonuniform_mu_edges
    from oracle.systematics import nonuniform_mu_edges as oedges
    # the oracle polishes roots of a degree-(lmax+1) polynomial in the monomial basis, whose
    # coefficients reach ~1e4 at lmax = 16: its edges carry ~1e-12 absolute error there
    for lmax in (2, 4, 8, 16):
        assert np.max(np.abs(nonuniform_mu_edges(lmax) - oedges(lmax))) < 1e-10


@pytest.mark.parametrize("lmax", [0, 4, 8, 16])
def test_kaiser_gamma_matches_oracle(lmax):
    from paper_1704_02357_amd import kaiser_wedge_gamma, nonuniform_mu_edges
    from oracle.covariance import kaiser_gamma
    for edges in (np.linspace(0, 1, 10), nonuniform_mu_edges(max(lmax, 2)), np.array([0.0, 0.2, 0.9, 1.0])):
        for beta in (0.0, 0.35, 1.2):
            got = kaiser_wedge_gamma(lmax, edges, beta)
            ref = kaiser_gamma(lmax, edges, beta)
            assert np.max(np.abs(got - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_kaiser_gamma_validation():
    from paper_1704_02357_amd import PkmError, kaiser_wedge_gamma
    for args in ((3, [0, 1], 0.3), (4, [0.5, 0.2], 0.3), (4, [0, 1.5], 0.3), (4, [0, 1], float("nan")),
                 (66, [0, 1], 0.3)):
        with pytest.raises(PkmError):
            kaiser_wedge_gamma(*args)


def test_wedges_validation():
    lib = _lib()
    poles = np.zeros((3, 4))
    out = np.zeros((4, 2))
    P = lambda a: a.ctypes.data_as(C.c_void_p)
    bad = np.array([0.0, 0.7, 0.5])  # not increasing
    assert lib.pkm_wedges(P(poles), 4, 4, P(bad), 3, P(out)) == 1
    assert lib.pkm_wedges(P(poles), 3, 4, P(np.array([0, 0.5, 1.0])), 3, P(out)) == 1  # odd ell_max
    assert lib.pkm_wedges(P(poles), 4, 4, P(np.array([0, 0.5, 1.5])), 3, P(out)) == 1  # outside [0, 1]
    assert lib.pkm_nonuniform_mu_edges(3, P(np.zeros(4))) == 1


@pytest.mark.parametrize("field,value", [("nmesh", 100), ("nmesh", 2048), ("nmesh", 54), ("box_len", -1.0),
                                         ("window", 4), ("precision", 2), ("ell_max_hint", 5), ("ell_max_hint", 18),
                                         ("deterministic", 2)])
def test_plan_create_rejects_bad_params(field, value):
    lib = _lib()
    from paper_1704_02357_amd.pkm import Params
    p = Params()
    p.nmesh, p.box_len, p.window, p.interlaced, p.compensated, p.precision = 64, 100.0, 3, 1, 1, 0
    setattr(p, field, value)
    h = C.c_void_p()
    assert lib.pkm_plan_create(C.byref(p), None, C.byref(h)) == 1
    assert not h.value


def test_shape_validation_rejects_before_device():
    """Launch shapes that break a kernel limit are refused with PKM_EINVAL before any device
    work (so this runs without a GPU)."""
    lib = _lib()
    from paper_1704_02357_amd.pkm import Device, Shape, make_params
    p = make_params(64, 300.0, observer=(0.0, 0.0, -500.0))
    d = Device()
    bad = [dict(tile=3), dict(e_col=5), dict(e_col=12), dict(paint_tile=32), dict(post_axis=3),
           dict(e_z=8, zlines=128), dict(e_post=4, tile_post=32), dict(zlines=3)]
    for b in bad:
        sh = Shape()
        for k, v in b.items():
            setattr(sh, k, v)
        h = C.c_void_p()
        st = lib.pkm_plan_create_shaped(C.byref(p), C.byref(d), C.byref(sh), C.byref(h))
        assert st == 1, (b, st)


def test_particle_limit_rejected_on_host():
    """More than PKM_MAX_PARTICLES data + random objects (the painting sort's 32-bit counts
    and offsets) is refused on the host before any array is read."""
    lib = _lib()
    from paper_1704_02357_amd.pkm import Catalog, MAX_PARTICLES
    hdr = open(HEADER).read()
    assert f"#define PKM_MAX_PARTICLES ((int64_t){MAX_PARTICLES})" in hdr
    fake = C.c_void_p(0x1000)  # never dereferenced: the check reads only the structs
    def cat(n, on_dev=1):
        return Catalog(fake, None, fake, n, on_dev)
    ok_d, ok_r = cat(1000), cat(20000)
    assert lib.pkm_check_catalogs(C.byref(ok_d), C.byref(ok_r)) == 0
    assert lib.pkm_check_catalogs(C.byref(ok_d), None) == 0
    for d, r in ((cat(MAX_PARTICLES - 10), cat(11)), (cat(MAX_PARTICLES + 1), None), (cat(2 ** 31), cat(5)),
                 (cat(0), ok_r), (ok_d, cat(0)), (cat(-1), None)):
        assert lib.pkm_check_catalogs(C.byref(d), None if r is None else C.byref(r)) == 1
    assert lib.pkm_check_catalogs(C.byref(cat(MAX_PARTICLES - 10)), C.byref(cat(10))) == 0
    nonbar = Catalog(fake, None, None, 10, 1)
    assert lib.pkm_check_catalogs(C.byref(ok_d), C.byref(nonbar)) == 1


def test_server_config_validation_on_host():
    """Bad server configurations are refused before any device call."""
    lib = _lib()
    from paper_1704_02357_amd.pkm import ALLOC_FN, ServerConfig
    for field, value in (("max_inflight", 0), ("max_inflight", 33), ("field_group", -1), ("field_group", 257)):
        cfg = ServerConfig()
        cfg.device_id, cfg.max_inflight = 0, 2
        setattr(cfg, field, value)
        h = C.c_void_p()
        assert lib.pkm_server_create(C.byref(cfg), C.byref(h)) == 1, field
        assert not h.value
    cfg = ServerConfig()
    cfg.max_inflight = 2
    cfg.alloc = ALLOC_FN(lambda size, stream, ctx: None)  # an allocator without a free
    h = C.c_void_p()
    assert lib.pkm_server_create(C.byref(cfg), C.byref(h)) == 1


def test_plan_footprint_on_host():
    """pkm_plan_footprint: host arithmetic only; grows with l_max and particles, caps at
    max_group fields, adds the 64-bit paint accumulators in deterministic mode, and rejects
    invalid parameters with -1."""
    from paper_1704_02357_amd import plan_footprint
    from paper_1704_02357_amd.pkm import PkmError
    kw = dict(window=3, interlaced=True, compensated=True, precision=0)
    a = plan_footprint(128, 500.0, 4, 40, 10_000, **kw)
    b = plan_footprint(128, 500.0, 8, 40, 10_000, **kw)
    c = plan_footprint(128, 500.0, 8, 40, 1_000_000, **kw)
    g = plan_footprint(128, 500.0, 16, 40, 10_000, max_group=4, **kw)
    d = plan_footprint(128, 500.0, 4, 40, 10_000, deterministic=True, **kw)
    mesh = 4 * 128 ** 3
    assert a < b < c and c - b == 80 * 990_000
    assert g < plan_footprint(128, 500.0, 4, 40, 10_000, max_group=8, **kw)
    assert d - a == 2 * 8 * 128 ** 3
    assert b - a >= (45 - 15) * mesh  # 30 more weighted fields
    for bad in (dict(nmesh=100), dict(ell_max=18), dict(n_edges=1)):
        args = dict(nmesh=128, box_len=500.0, ell_max=4, n_edges=40, n_particles=10)
        args.update(bad)
        with pytest.raises(PkmError):
            plan_footprint(args.pop("nmesh"), args.pop("box_len"), args.pop("ell_max"), args.pop("n_edges"),
                           args.pop("n_particles"), **kw)
