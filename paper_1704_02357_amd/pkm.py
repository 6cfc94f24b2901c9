"""ctypes binding of libpkm (include/pkm.h): argument marshalling only.

Every step of the estimator runs in the HIP library.  PyTorch supplies device memory (its
caching allocator is passed to the library as the plan's allocator) and the HIP stream.
If the library is missing the import of a Plan raises: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ABI_VERSION = 4
MAX_PARTICLES = 2 ** 31 - 2 ** 16   # PKM_MAX_PARTICLES: data + random objects per estimate
NGP, CIC, TSC = 1, 2, 3
FP32, FP64 = 0, 1
SPHERICAL, CARTESIAN = 0, 1   # decompositions of L_l(khat . xhat) (Sec. 2.1)
LOS_LOCAL, LOS_GLOBAL = 0, 1
STATUS = {0: "PKM_OK", 1: "PKM_EINVAL", 2: "PKM_EORDER", 3: "PKM_ENOMEM", 4: "PKM_EDEVICE", 5: "PKM_EBUSY",
          6: "PKM_ECANCELLED"}


class PkmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("nmesh", C.c_int32), ("box_len", C.c_double), ("box_origin", C.c_double * 3),
                ("observer", C.c_double * 3), ("los_mode", C.c_int32), ("los", C.c_double * 3),
                ("window", C.c_int32), ("interlaced", C.c_int32), ("compensated", C.c_int32),
                ("precision", C.c_int32), ("ell_max_hint", C.c_int32), ("max_group", C.c_int32),
                ("deterministic", C.c_int32)]


class Catalog(C.Structure):
    _fields_ = [("pos", C.c_void_p), ("w", C.c_void_p), ("nbar", C.c_void_p), ("n", C.c_int64),
                ("on_device", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("poles", C.c_void_p), ("k_mean", C.c_void_p), ("n_modes", C.c_void_p), ("alpha", C.c_double),
                ("norm_I", C.c_double), ("shot_noise", C.c_double), ("n_transforms", C.c_int32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Device(C.Structure):
    _fields_ = [("device_id", C.c_int32), ("hip_stream", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("alloc_ctx", C.c_void_p)]


class Shape(C.Structure):
    _fields_ = [(f, C.c_int32) for f in ("e_col", "tile", "e_z", "zlines", "e_post", "tile_post", "paint_tile",
                                          "post_axis")]


def _shape(d):
    sh = Shape()
    for f, _ in Shape._fields_:
        setattr(sh, f, int((d or {}).get(f, 0)))
    return sh


class ServerConfig(C.Structure):
    _fields_ = [("device_id", C.c_int32), ("hbm_budget_bytes", C.c_int64), ("max_inflight", C.c_int32),
                ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_ctx", C.c_void_p), ("field_group", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("params", Params), ("ell_max", C.c_int32), ("k_edges", C.c_void_p), ("n_edges", C.c_int32),
                ("data", Catalog), ("randoms", Catalog), ("has_randoms", C.c_int32), ("catalog_id", C.c_uint64)]


class ServerStats(C.Structure):
    _fields_ = [("completed", C.c_int64), ("failed", C.c_int64), ("queued", C.c_int64), ("inflight", C.c_int64),
                ("resident_plans", C.c_int64), ("resident_bytes", C.c_int64), ("peak_bytes", C.c_int64),
                ("max_concurrent", C.c_int32), ("latency_p50_ms", C.c_double), ("latency_p99_ms", C.c_double),
                ("latency_mean_ms", C.c_double), ("throughput_per_s", C.c_double),
                ("completed_fp32", C.c_int64), ("completed_fp64", C.c_int64),
                ("latency_p50_ms_fp32", C.c_double), ("latency_p99_ms_fp32", C.c_double),
                ("latency_p50_ms_fp64", C.c_double), ("latency_p99_ms_fp64", C.c_double),
                ("mesh_reuses", C.c_int64), ("registered_catalogs", C.c_int64), ("registered_bytes", C.c_int64)]


STAGES = ["sums", "fill", "paint", "zfwd", "ycol", "xcombine", "iycol", "zpre", "xpost", "reduce"]


class Stats(C.Structure):
    _fields_ = [("device_bytes", C.c_int64), ("n_transforms", C.c_int32), ("n_groups", C.c_int32),
                ("ms_paint", C.c_double), ("ms_compute", C.c_double), ("model_bytes_paint", C.c_double),
                ("model_bytes_compute", C.c_double), ("stage_ms", C.c_double * 10),
                ("stage_launches", C.c_int64 * 10)]


_LIB = None


def lib_path() -> str:
    return os.environ.get("PKM_LIBRARY", os.path.join(HERE, "libpkm.so"))


def load_library():
    """Load libpkm.so (raises OSError if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = lib_path()
    if not os.path.exists(path):
        raise OSError(f"{path} not found: build it with paper_1704_02357_amd/build.py")
    # torch's ROCm build carries its own HIP runtime under the same soname as the system one
    # the library links.  Loading torch first makes the library bind to that copy, so the
    # process holds one HIP runtime whichever of the two the caller touches first (loading the
    # library first and torch later would leave two, and the second finds no device).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    P = C.c_void_p
    sig = {
        "pkm_abi_version": (C.c_int, []),
        "pkm_status_str": (C.c_char_p, [C.c_int]),
        "pkm_check_catalogs": (C.c_int, [C.POINTER(Catalog), C.POINTER(Catalog)]),
        "pkm_plan_create": (C.c_int, [C.POINTER(Params), C.POINTER(Device), C.POINTER(P)]),
        "pkm_paint": (C.c_int, [P, C.POINTER(Catalog), C.POINTER(Catalog)]),
        "pkm_compute_multipoles": (C.c_int, [P, C.c_int32, P, C.c_int32, C.POINTER(Result)]),
        "pkm_compute_multipoles_basis": (C.c_int, [P, C.c_int32, P, C.c_int32, C.c_int32, C.POINTER(Result)]),
        "pkm_compute_multipoles_all": (C.c_int, [P, C.c_int32, P, C.c_int32, C.POINTER(Result)]),
        "pkm_kmu_global": (C.c_int, [P, P, C.c_int32, P, C.c_int32, P, P]),
        "pkm_kmu_global_noalloc": (C.c_int, [P, P, C.c_int32, P, C.c_int32, P, P]),
        "pkm_wedges": (C.c_int, [P, C.c_int32, C.c_int32, P, C.c_int32, P]),
        "pkm_kaiser_wedge_gamma": (C.c_int, [C.c_int32, P, C.c_int32, C.c_double, P]),
        "pkm_nonuniform_mu_edges": (C.c_int, [C.c_int32, P]),
        "pkm_stats": (C.c_int, [P, C.POINTER(Stats)]),
        "pkm_set_stage_timing": (C.c_int, [P, C.c_int32]),
        "pkm_reset_stats": (C.c_int, [P]),
        "pkm_plan_last_error": (C.c_char_p, [P]),
        "pkm_plan_destroy": (None, [P]),
        "pkm_fft3d_forward": (C.c_int, [P, P, P]),
        "pkm_fft3d_inverse": (C.c_int, [P, P, P]),
        "pkm_plan_read_buffer": (C.c_int, [P, C.c_int32, P, C.c_size_t]),
        "pkm_prepare": (C.c_int, [P, C.c_int32, P, C.c_int32, C.c_int64]),
        "pkm_plan_create_shaped": (C.c_int, [C.POINTER(Params), C.POINTER(Device), C.POINTER(Shape), C.POINTER(P)]),
        "pkm_plan_shape": (C.c_int, [P, C.POINTER(Shape)]),
        "pkm_autotune": (C.c_int, [C.POINTER(Params), C.POINTER(Device), C.c_int32, C.c_int64, C.c_int32,
                                   C.POINTER(Shape), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "pkm_enqueue": (C.c_int, [P, C.POINTER(Catalog), C.POINTER(Catalog)]),
        "pkm_query": (C.c_int, [P]),
        "pkm_finish": (C.c_int, [P, C.POINTER(Result)]),
        "pkm_batch_create": (C.c_int, [C.c_int32, C.POINTER(P)]),
        "pkm_batch_add": (C.c_int, [P, P, C.POINTER(Catalog), C.POINTER(Catalog), C.POINTER(C.c_int32)]),
        "pkm_batch_run": (C.c_int, [P, C.c_int32, C.POINTER(C.c_double)]),
        "pkm_batch_result": (C.c_int, [P, C.c_int32, C.POINTER(Result)]),
        "pkm_batch_size": (C.c_int32, [P]),
        "pkm_batch_last_error": (C.c_char_p, [P]),
        "pkm_batch_destroy": (None, [P]),
        "pkm_server_create": (C.c_int, [C.POINTER(ServerConfig), C.POINTER(P)]),
        "pkm_plan_footprint": (C.c_int64, [C.POINTER(Params), C.c_int32, C.c_int32, C.c_int64]),
        "pkm_server_register_catalog": (C.c_int, [P, C.POINTER(Catalog), C.POINTER(Catalog),
                                                  C.POINTER(C.c_uint64)]),
        "pkm_server_unregister_catalog": (C.c_int, [P, C.c_uint64]),
        "pkm_server_submit": (C.c_int, [P, C.POINTER(Request), C.POINTER(C.c_int64)]),
        "pkm_server_poll": (C.c_int, [P, C.c_int64, C.POINTER(Result)]),
        "pkm_server_wait": (C.c_int, [P, C.c_int64, C.POINTER(Result)]),
        "pkm_server_stats": (C.c_int, [P, C.POINTER(ServerStats)]),
        "pkm_server_reset_stats": (C.c_int, [P]),
        "pkm_server_last_error": (C.c_char_p, [P]),
        "pkm_server_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def wedges(poles: np.ndarray, ell_max: int, mu_edges) -> np.ndarray:
    """eq. wedge-est on the host (FP64): returns (n_k, n_mu)."""
    lib = load_library()
    poles = np.ascontiguousarray(poles, dtype=np.float64)
    mu = np.ascontiguousarray(mu_edges, dtype=np.float64)
    nk = poles.shape[1]
    out = np.empty((nk, mu.size - 1))
    st = lib.pkm_wedges(_ptr(poles), ell_max, nk, _ptr(mu), mu.size, _ptr(out))
    if st:
        raise PkmError(st, "pkm_wedges rejected its arguments")
    return out


def kaiser_wedge_gamma(ell_max: int, mu_edges, beta: float) -> np.ndarray:
    """Sec. 4.1 eq. gamma (host, FP64): (n_mu, n_mu) angular covariance of Kaiser wedges."""
    lib = load_library()
    mu = np.ascontiguousarray(mu_edges, dtype=np.float64)
    out = np.empty((mu.size - 1, mu.size - 1))
    st = lib.pkm_kaiser_wedge_gamma(int(ell_max), _ptr(mu), mu.size, float(beta), _ptr(out))
    if st:
        raise PkmError(st, "pkm_kaiser_wedge_gamma rejected its arguments")
    return out


def plan_footprint(nmesh, box_len, ell_max, n_edges, n_particles, **params) -> int:
    """Device bytes a plan would hold for one estimate (the serving loop's admission figure);
    keyword arguments as for Plan."""
    p = make_params(nmesh, box_len, **params)
    b = load_library().pkm_plan_footprint(C.byref(p), int(ell_max), int(n_edges), int(n_particles))
    if b < 0:
        raise PkmError(1, "pkm_plan_footprint rejected its arguments")
    return int(b)


def nonuniform_mu_edges(ell_max: int) -> np.ndarray:
    lib = load_library()
    out = np.empty(ell_max // 2 + 2)
    st = lib.pkm_nonuniform_mu_edges(ell_max, _ptr(out))
    if st:
        raise PkmError(st, "pkm_nonuniform_mu_edges rejected its arguments")
    return out


class _TorchAllocator:
    """Routes the library's device allocations through torch's caching allocator."""

    def __init__(self, device: int):
        import torch
        # raw allocations need torch's device state, which torch sets up lazily on first use
        torch.cuda.init()
        self.torch = torch
        self.device = device
        self.error = None  # the last failed allocation's exception (callbacks cannot raise)
        self.c_alloc = ALLOC_FN(self._alloc)
        self.c_free = FREE_FN(self._free)

    def _alloc(self, size, stream, ctx):
        try:
            return int(self.torch.cuda.caching_allocator_alloc(int(size), self.device, stream or 0))
        except Exception as e:
            self.error = f"{type(e).__name__}: {e}"
            return None

    def _free(self, ptr, stream, ctx):
        try:
            self.torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:
            pass


def make_params(nmesh, box_len, *, box_origin=None, observer=(0.0, 0.0, 0.0), window=TSC, interlaced=True,
                compensated=True, precision=FP32, ell_max_hint=4, max_group=0, los=None,
                deterministic=False) -> Params:
    p = Params()
    p.nmesh = int(nmesh)
    p.box_len = float(box_len)
    o = (-0.5 * box_len,) * 3 if box_origin is None else box_origin
    for a in range(3):
        p.box_origin[a] = float(o[a])
        p.observer[a] = float(observer[a])
    if los is not None:
        p.los_mode = LOS_GLOBAL
        for a in range(3):
            p.los[a] = float(los[a])
    p.window, p.interlaced, p.compensated = int(window), int(bool(interlaced)), int(bool(compensated))
    p.precision, p.ell_max_hint, p.max_group = int(precision), int(ell_max_hint), int(max_group)
    p.deterministic = int(bool(deterministic))
    return p


def _result_arrays(ell_max: int, nb: int, all_ell: bool = False):
    poles = np.empty((ell_max + 1 if all_ell else ell_max // 2 + 1, nb))
    kmean = np.empty(nb)
    nmodes = np.empty(nb, dtype=np.int64)
    r = Result()
    r.poles, r.k_mean, r.n_modes = poles.ctypes.data, kmean.ctypes.data, nmodes.ctypes.data
    return r, poles, kmean, nmodes


def _result_dict(r, poles, kmean, nmodes, ell_max, all_ell: bool = False):
    return dict(poles=poles, k_mean=kmean, n_modes=nmodes, alpha=r.alpha, norm_I=r.norm_I, shot_noise=r.shot_noise,
                n_transforms=r.n_transforms, ells=list(range(0, ell_max + 1, 1 if all_ell else 2)))


def _marshal_catalog(cat, keep):
    """A pkm_catalog over (pos, w, nbar) of host arrays or CUDA tensors; the converted arrays
    are appended to `keep`, which must outlive the call they are passed to."""
    if cat is None:
        return None
    pos, w, nbar = cat if isinstance(cat, tuple) else (cat.pos, cat.w, getattr(cat, "nbar", None))
    c = Catalog()
    on_dev = hasattr(pos, "is_cuda") and pos.is_cuda
    if on_dev:
        import torch
        arrs = [None if a is None else a.to(torch.float64).contiguous() for a in (pos, w, nbar)]
        c.pos, c.w, c.nbar = [None if a is None else a.data_ptr() for a in arrs]
    else:
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in (pos, w, nbar)]
        c.pos, c.w, c.nbar = [None if a is None else a.ctypes.data for a in arrs]
    c.n = int(arrs[0].shape[0])
    c.on_device = int(on_dev)
    keep.append(arrs)
    return c


class Plan:
    """One mesh configuration.  Inputs may be numpy arrays (host) or torch CUDA tensors."""

    def __init__(self, nmesh: int, box_len: float, *, box_origin=None, observer=(0.0, 0.0, 0.0), window=TSC,
                 interlaced=True, compensated=True, precision=FP32, ell_max_hint=4, max_group=0, los=None,
                 device: int = 0, stream=None, torch_allocator: bool = True, shape=None, deterministic=False):
        self.lib = load_library()
        p = make_params(nmesh, box_len, box_origin=box_origin, observer=observer, window=window,
                        interlaced=interlaced, compensated=compensated, precision=precision,
                        ell_max_hint=ell_max_hint, max_group=max_group, los=los, deterministic=deterministic)
        self.params = p
        self.nmesh = p.nmesh
        self.precision = p.precision
        d = Device()
        d.device_id = device
        self._stream_obj = stream
        if stream is not None:
            d.hip_stream = C.c_void_p(int(getattr(stream, "cuda_stream", stream)))
        self._alloc = None
        if torch_allocator:
            self._alloc = _TorchAllocator(device)
            d.alloc = self._alloc.c_alloc
            d.free = self._alloc.c_free
        self.dev = d
        h = C.c_void_p()
        sh = _shape(shape) if shape else None
        st = self.lib.pkm_plan_create_shaped(C.byref(p), C.byref(d), C.byref(sh) if sh is not None else None,
                                             C.byref(h))
        if st:
            msg = self.lib.pkm_plan_last_error(None)
            why = msg.decode() if msg else ""
            if self._alloc is not None and self._alloc.error:
                why += f" (torch allocator: {self._alloc.error})"
            raise PkmError(st, "pkm_plan_create failed" + (" (shape rejected)" if shape and st == 1 else "")
                           + (f": {why}" if why else ""))
        self.h = h
        self._keep = []

    # -- helpers ------------------------------------------------------------------------
    def _check(self, st, what):
        if st:
            msg = self.lib.pkm_plan_last_error(self.h)
            raise PkmError(st, f"{what}: {msg.decode() if msg else ''}")

    def _catalog(self, cat):
        return _marshal_catalog(cat, self._keep)

    # -- API ----------------------------------------------------------------------------
    def paint(self, data, randoms=None):
        self._keep = []
        d = self._catalog(data)
        r = self._catalog(randoms)
        st = self.lib.pkm_paint(self.h, C.byref(d), C.byref(r) if r is not None else None)
        self._keep = []
        self._check(st, "pkm_paint")

    def compute_multipoles(self, ell_max: int, k_edges, basis: int = SPHERICAL) -> dict:
        """basis SPHERICAL (2l+1 transforms per l) or CARTESIAN (the monomial decomposition)."""
        e = np.ascontiguousarray(k_edges, dtype=np.float64)
        r, poles, kmean, nmodes = _result_arrays(ell_max, e.size - 1)
        st = self.lib.pkm_compute_multipoles_basis(self.h, int(ell_max), _ptr(e), e.size, int(basis), C.byref(r))
        self._check(st, "pkm_compute_multipoles_basis")
        return _result_dict(r, poles, kmean, nmodes, ell_max)

    def compute_multipoles_all(self, ell_max: int, k_edges) -> dict:
        """Every l <= ell_max, odd included: even rows P_l, odd rows R_l = Im P_l (eq. Pell-ours)."""
        e = np.ascontiguousarray(k_edges, dtype=np.float64)
        r, poles, kmean, nmodes = _result_arrays(ell_max, e.size - 1, all_ell=True)
        st = self.lib.pkm_compute_multipoles_all(self.h, int(ell_max), _ptr(e), e.size, C.byref(r))
        self._check(st, "pkm_compute_multipoles_all")
        return _result_dict(r, poles, kmean, nmodes, ell_max, all_ell=True)

    # -- asynchronous estimate -------------------------------------------------------------
    def prepare(self, ell_max: int, k_edges, max_particles: int):
        """Host tables and buffers for estimates of up to max_particles objects."""
        e = np.ascontiguousarray(k_edges, dtype=np.float64)
        self._check(self.lib.pkm_prepare(self.h, int(ell_max), _ptr(e), e.size, int(max_particles)), "pkm_prepare")
        self._prep = (int(ell_max), e.size - 1)

    def enqueue(self, data, randoms=None):
        """Enqueue paint + multipoles of device-resident catalogs; returns at once."""
        self._akeep = [self._catalog(data), self._catalog(randoms)]
        d, r = self._akeep
        self._check(self.lib.pkm_enqueue(self.h, C.byref(d), C.byref(r) if r is not None else None), "pkm_enqueue")

    def query(self) -> bool:
        st = self.lib.pkm_query(self.h)
        if st == 5:
            return False
        self._check(st, "pkm_query")
        return True

    def finish(self) -> dict:
        ell_max, nb = self._prep
        r, poles, kmean, nmodes = _result_arrays(ell_max, nb)
        self._check(self.lib.pkm_finish(self.h, C.byref(r)), "pkm_finish")
        self._akeep = []
        return _result_dict(r, poles, kmean, nmodes, ell_max)

    def kmu_global(self, k_edges, mu_edges):
        ke = np.ascontiguousarray(k_edges, dtype=np.float64)
        me = np.ascontiguousarray(mu_edges, dtype=np.float64)
        pk = np.empty((ke.size - 1, me.size - 1))
        nm = np.empty((ke.size - 1, me.size - 1), dtype=np.int64)
        st = self.lib.pkm_kmu_global(self.h, _ptr(ke), ke.size, _ptr(me), me.size, _ptr(pk), _ptr(nm))
        self._check(st, "pkm_kmu_global")
        return pk, nm

    def stats(self) -> dict:
        s = Stats()
        self._check(self.lib.pkm_stats(self.h, C.byref(s)), "pkm_stats")
        out = {f: getattr(s, f) for f, _ in Stats._fields_ if not f.startswith("stage_")}
        out["stage_ms"] = {STAGES[i]: s.stage_ms[i] for i in range(10)}
        out["stage_launches"] = {STAGES[i]: int(s.stage_launches[i]) for i in range(10)}
        return out

    def shape(self) -> dict:
        sh = Shape()
        self._check(self.lib.pkm_plan_shape(self.h, C.byref(sh)), "pkm_plan_shape")
        return {f: getattr(sh, f) for f, _ in Shape._fields_}

    def set_stage_timing(self, on: bool):
        self._check(self.lib.pkm_set_stage_timing(self.h, int(bool(on))), "pkm_set_stage_timing")

    def reset_stats(self):
        self._check(self.lib.pkm_reset_stats(self.h), "pkm_reset_stats")

    def read_buffer(self, which: int) -> np.ndarray:
        n = self.nmesh
        rdt = np.float64 if self.precision == FP64 else np.float32
        cdt = np.complex128 if self.precision == FP64 else np.complex64
        if which == 2:
            out = np.empty((n, n, n // 2), dtype=cdt)
        else:
            out = np.empty((n, n, n), dtype=rdt)
        st = self.lib.pkm_plan_read_buffer(self.h, int(which), out.ctypes.data, out.nbytes)
        self._check(st, "pkm_plan_read_buffer")
        return out

    def fft3d_forward(self, real_dev, out_dev):
        self._check(self.lib.pkm_fft3d_forward(self.h, real_dev.data_ptr(), out_dev.data_ptr()), "pkm_fft3d_forward")

    def fft3d_inverse(self, half_dev, out_dev):
        self._check(self.lib.pkm_fft3d_inverse(self.h, half_dev.data_ptr(), out_dev.data_ptr()), "pkm_fft3d_inverse")

    def close(self):
        if getattr(self, "h", None):
            self.lib.pkm_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Batch:
    """Many estimates issued as one unit (optionally one HIP graph launch)."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        h = C.c_void_p()
        st = self.lib.pkm_batch_create(int(device), C.byref(h))
        if st:
            raise PkmError(st, "pkm_batch_create failed")
        self.h = h
        self._items = []

    def _check(self, st, what):
        if st:
            msg = self.lib.pkm_batch_last_error(self.h)
            raise PkmError(st, f"{what}: {msg.decode() if msg else ''}")

    def add(self, plan: "Plan", data, randoms=None) -> int:
        d, r = plan._catalog(data), plan._catalog(randoms)
        idx = C.c_int32()
        self._check(self.lib.pkm_batch_add(self.h, plan.h, C.byref(d), C.byref(r) if r is not None else None,
                                           C.byref(idx)), "pkm_batch_add")
        self._items.append((plan, plan._prep, (data, randoms)))
        return idx.value

    def run(self, use_graph: bool = True) -> float:
        ms = C.c_double()
        self._check(self.lib.pkm_batch_run(self.h, int(bool(use_graph)), C.byref(ms)), "pkm_batch_run")
        return ms.value

    def result(self, index: int) -> dict:
        ell_max, nb = self._items[index][1]
        r, poles, kmean, nmodes = _result_arrays(ell_max, nb)
        self._check(self.lib.pkm_batch_result(self.h, int(index), C.byref(r)), "pkm_batch_result")
        return _result_dict(r, poles, kmean, nmodes, ell_max)

    def __len__(self):
        return int(self.lib.pkm_batch_size(self.h))

    def close(self):
        if getattr(self, "h", None):
            self.lib.pkm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Request loop on one device: admission by HBM footprint, overlapping estimates."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0, max_inflight: int = 4, allocator=None,
                 field_group: int = 0):
        """allocator: None (the device's stream-ordered pool) or an object with ctypes
        callbacks c_alloc / c_free of pkm_device's allocator signature.  field_group > 0: plans
        keep that many weighted fields and serve every l_max (pkm_server_config.field_group)."""
        self.lib = load_library()
        cfg = ServerConfig()
        cfg.device_id, cfg.hbm_budget_bytes, cfg.max_inflight = int(device), int(hbm_budget_bytes), int(max_inflight)
        cfg.field_group = int(field_group)
        self._allocator = allocator
        if allocator is not None:
            cfg.alloc, cfg.free = allocator.c_alloc, allocator.c_free
        h = C.c_void_p()
        st = self.lib.pkm_server_create(C.byref(cfg), C.byref(h))
        if st:
            raise PkmError(st, "pkm_server_create failed")
        self.h = h
        self._shape = {}

    def _check(self, st, what):
        if st:
            msg = self.lib.pkm_server_last_error(self.h)
            raise PkmError(st, f"{what}: {msg.decode() if msg else ''}")

    def register_catalog(self, data, randoms=None) -> int:
        """Copy a catalog (and randoms) to the device once; requests name it by the id."""
        keep = []
        d = _marshal_catalog(data, keep)
        r = _marshal_catalog(randoms, keep)
        cid = C.c_uint64()
        self._check(self.lib.pkm_server_register_catalog(self.h, C.byref(d), C.byref(r) if r is not None else None,
                                                         C.byref(cid)), "pkm_server_register_catalog")
        return cid.value

    def unregister_catalog(self, catalog_id: int):
        self._check(self.lib.pkm_server_unregister_catalog(self.h, int(catalog_id)), "pkm_server_unregister_catalog")

    def submit(self, nmesh, box_len, ell_max, k_edges, data=None, randoms=None, *, catalog_id: int = 0,
               **params) -> int:
        """Queue one estimate of host catalogs, or of a registered catalog (catalog_id);
        keyword arguments as for Plan."""
        rq = Request()
        rq.params = make_params(nmesh, box_len, **params)
        e = np.ascontiguousarray(k_edges, dtype=np.float64)
        rq.ell_max, rq.k_edges, rq.n_edges = int(ell_max), e.ctypes.data, e.size
        rq.catalog_id = int(catalog_id)
        keep = [e]
        if not catalog_id:
            if data is None:
                raise ValueError("submit needs host catalogs or a registered catalog_id")
            for field, cat in (("data", data), ("randoms", randoms)):
                if cat is None:
                    continue
                arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64)
                        for a in (cat.pos, cat.w, getattr(cat, "nbar", None))]
                keep.append(arrs)
                c = getattr(rq, field)
                c.pos, c.w, c.nbar = [None if a is None else a.ctypes.data for a in arrs]
                c.n, c.on_device = int(arrs[0].shape[0]), 0
            rq.has_randoms = int(randoms is not None)
        t = C.c_int64()
        self._check(self.lib.pkm_server_submit(self.h, C.byref(rq), C.byref(t)), "pkm_server_submit")
        self._shape[t.value] = (int(ell_max), e.size - 1)
        return t.value

    def _collect(self, fn, ticket):
        ell_max, nb = self._shape[ticket]
        r, poles, kmean, nmodes = _result_arrays(ell_max, nb)
        st = fn(self.h, int(ticket), C.byref(r))
        if st == 5:
            return None
        self._shape.pop(ticket, None)
        self._check(st, "server result")
        return _result_dict(r, poles, kmean, nmodes, ell_max)

    def poll(self, ticket: int):
        return self._collect(self.lib.pkm_server_poll, ticket)

    def wait(self, ticket: int) -> dict:
        return self._collect(self.lib.pkm_server_wait, ticket)

    def stats(self) -> dict:
        s = ServerStats()
        self._check(self.lib.pkm_server_stats(self.h, C.byref(s)), "pkm_server_stats")
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def reset_stats(self):
        self._check(self.lib.pkm_server_reset_stats(self.h), "pkm_server_reset_stats")

    def close(self):
        if getattr(self, "h", None):
            self.lib.pkm_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(nmesh, box_len, *, ell_max=4, n_particles=None, reps=2, device=0, cache=None, **params) -> dict:
    """Pick launch shapes by timing (pkm_autotune); keyword arguments as for Plan.  With
    `cache` (a JSON file path) results are stored per device and configuration and reused."""
    import json
    key = None
    if cache:
        import torch
        cfg = dict(params, nmesh=int(nmesh), box_len=float(box_len), ell_max=int(ell_max))
        key = json.dumps({"device": torch.cuda.get_device_name(device), **{k: cfg[k] for k in sorted(cfg)}},
                         default=str)
        try:
            with open(cache) as f:
                db = json.load(f)
        except (OSError, ValueError):
            db = {}
        if key in db:
            return db[key]
    lib = load_library()
    p = make_params(nmesh, box_len, ell_max_hint=max(ell_max, params.pop("ell_max_hint", 0)), **params)
    d = Device()
    d.device_id = device
    n_particles = int(n_particles or min(2_000_000, 8 * int(nmesh) ** 3 // 64))
    best, bms, dms = Shape(), C.c_double(), C.c_double()
    st = lib.pkm_autotune(C.byref(p), C.byref(d), int(ell_max), n_particles, int(reps), C.byref(best), C.byref(bms),
                          C.byref(dms))
    if st:
        raise PkmError(st, "pkm_autotune failed")
    out = {f: getattr(best, f) for f, _ in Shape._fields_}
    out.update(ms=bms.value, default_ms=dms.value)
    if cache:
        db[key] = out
        with open(cache, "w") as f:
            json.dump(db, f, indent=1)
    return out
