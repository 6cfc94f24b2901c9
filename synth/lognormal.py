"""Seeded lognormal mock catalogs with a survey cut and radial redshift-space distortions.

The paper measures on BOSS DR12 CMASS cutsky mocks, QPM boxes and cubic N-body boxes
(Sec. 3.2 and Sec. 4.1); none are available here, so these seeded synthetic catalogs stand
in for them with the same box scales and a BOSS-like number density.

Recipe (all randomness from ``numpy.random.default_rng(seed)``, PCG64):

1. Gaussian field delta_G on an ng^3 grid over the box, with spectrum
   P_G(k) = 2e4 (k/0.02) / (1 + (k/0.02)^2.6) (Mpc/h)^3; the k = 0 mode is zero.
2. Lognormal density delta_LN = exp(delta_G - sigma^2/2) - 1.
3. Zel'dovich displacement psi with psi_k = i k delta_k / k^2.
4. Survey S = box  AND  rmin < |x - obs| < rmax  AND  angle(x - obs, +z) <= half-angle.
5. Each cell receives Poisson(nbar V_cell (1 + delta_LN)) objects placed uniformly in it,
   nbar = n_gal / V_S.
6. Radial RSD: s = x + f (psi . rhat) rhat; an object is kept iff s lies in S.
7. Randoms are uniform in S (separate stream, seed + 1), random_factor times n_gal.
8. w = 1 (or U(0.5, 1.5) when ``weights='random'``) and nbar = n_gal / V_S per object.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.fft as sfft


@dataclasses.dataclass
class Catalog:
    pos: np.ndarray            # (n, 3) float64, absolute Cartesian coordinates [Mpc/h]
    w: np.ndarray | None       # (n,) float64 or None (unit weights)
    nbar: np.ndarray | None    # (n,) float64 or None

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


@dataclasses.dataclass
class SurveyGeometry:
    box_len: float
    observer: tuple = (0.0, 0.0, -1500.0)
    rmin: float = 1000.0
    rmax: float = 2000.0
    half_angle_deg: float = 30.0

    @property
    def box_origin(self):
        h = -0.5 * self.box_len
        return (h, h, h)

    def inside(self, x: np.ndarray) -> np.ndarray:
        o = np.asarray(self.box_origin)
        inb = np.all((x >= o) & (x < o + self.box_len), axis=1)
        d = x - np.asarray(self.observer)
        r = np.sqrt(np.sum(d * d, axis=1))
        cosang = np.where(r > 0, d[:, 2] / np.where(r > 0, r, 1.0), -1.0)
        return inb & (r > self.rmin) & (r < self.rmax) & (cosang >= math.cos(math.radians(self.half_angle_deg)))

    def cone_shell_volume(self) -> float:
        ca = math.cos(math.radians(self.half_angle_deg))
        return 2.0 * math.pi / 3.0 * (1.0 - ca) * (self.rmax ** 3 - self.rmin ** 3)

    def sample_cone_shell(self, rng: np.random.Generator, n: int) -> np.ndarray:
        """Uniform points in the (unclipped) cone-shell around the observer."""
        r3 = rng.uniform(self.rmin ** 3, self.rmax ** 3, n)
        r = np.cbrt(r3)
        ca = math.cos(math.radians(self.half_angle_deg))
        mu = rng.uniform(ca, 1.0, n)
        phi = rng.uniform(0.0, 2.0 * math.pi, n)
        st = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
        out = np.empty((n, 3))
        out[:, 0] = r * st * np.cos(phi)
        out[:, 1] = r * st * np.sin(phi)
        out[:, 2] = r * mu
        return out + np.asarray(self.observer)

    def volume(self, seed: int = 0, n_mc: int = 10_000_000) -> float:
        """V_S: analytic when the cone-shell fits in the box, else seeded Monte Carlo."""
        o = np.asarray(self.box_origin)
        # corners of the cone-shell bounding box
        ca = math.cos(math.radians(self.half_angle_deg))
        sa = math.sin(math.radians(self.half_angle_deg))
        obs = np.asarray(self.observer)
        lo = obs + np.array([-self.rmax * sa, -self.rmax * sa, self.rmin * ca])
        hi = obs + np.array([self.rmax * sa, self.rmax * sa, self.rmax])
        if np.all(lo >= o) and np.all(hi < o + self.box_len):
            return self.cone_shell_volume()
        rng = np.random.default_rng(seed)
        inside = 0
        done = 0
        chunk = 1_000_000
        while done < n_mc:
            m = min(chunk, n_mc - done)
            inside += int(np.count_nonzero(self.inside(self.sample_cone_shell(rng, m))))
            done += m
        return self.cone_shell_volume() * inside / n_mc


def _model_pk(k: np.ndarray) -> np.ndarray:
    x = k / 0.02
    return 2.0e4 * x / (1.0 + x ** 2.6)


def _gaussian_fields(rng: np.random.Generator, ng: int, box_len: float, workers: int):
    """delta_G and the Zel'dovich displacement on an ng^3 grid (float64)."""
    white = rng.standard_normal((ng, ng, ng))
    wk = sfft.rfftn(white, workers=workers)
    del white
    kf = 2.0 * math.pi / box_len
    kx = sfft.fftfreq(ng, d=1.0 / ng) * kf
    kz = sfft.rfftfreq(ng, d=1.0 / ng) * kf
    vcell = (box_len / ng) ** 3
    k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
    k2[0, 0, 0] = 1.0
    amp = np.sqrt(_model_pk(np.sqrt(k2)) / vcell)
    amp[0, 0, 0] = 0.0
    dk = wk * amp
    del wk, amp
    delta = sfft.irfftn(dk, s=(ng, ng, ng), workers=workers)
    psi = []
    for axis in range(3):
        if axis == 0:
            ka = kx[:, None, None]
        elif axis == 1:
            ka = kx[None, :, None]
        else:
            ka = kz[None, None, :]
        psi.append(sfft.irfftn(1j * ka / k2 * dk, s=(ng, ng, ng), workers=workers).astype(np.float32))
    return delta, psi


def uniform_survey_randoms(geom: SurveyGeometry, n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    out = []
    got = 0
    while got < n:
        m = max(1024, int((n - got) * 1.3) + 1024)
        pts = geom.sample_cone_shell(rng, m)
        pts = pts[geom.inside(pts)]
        out.append(pts)
        got += pts.shape[0]
    return np.concatenate(out)[:n]


def lognormal_survey(geom: SurveyGeometry, n_gal: int, seed: int, ng: int = 256,
                     f: float = 0.75, random_factor: float = 10.0, weights: str = "unit",
                     workers: int | None = None):
    """Return (data, randoms, info) for one seeded lognormal survey mock."""
    import os
    workers = workers or max(1, min(16, os.cpu_count() or 1))
    rng = np.random.default_rng(seed)
    vs = geom.volume(seed=seed + 7)
    nbar = n_gal / vs
    delta, psi = _gaussian_fields(rng, ng, geom.box_len, workers)
    sig2 = float(np.var(delta))
    # lognormal density, evaluated cell by cell
    dln = np.exp(delta - 0.5 * sig2)
    del delta
    h = geom.box_len / ng
    lam = (nbar * h ** 3) * dln.ravel()
    del dln
    counts = rng.poisson(lam)
    del lam
    cells = np.repeat(np.arange(counts.size, dtype=np.int64), counts)
    del counts
    ix = cells // (ng * ng)
    iy = (cells // ng) % ng
    iz = cells % ng
    o = np.asarray(geom.box_origin)
    x = np.empty((cells.size, 3))
    u = rng.random((cells.size, 3))
    x[:, 0] = o[0] + (ix + u[:, 0]) * h
    x[:, 1] = o[1] + (iy + u[:, 1]) * h
    x[:, 2] = o[2] + (iz + u[:, 2]) * h
    # radial RSD from the displacement at the cell
    d = x - np.asarray(geom.observer)
    r = np.sqrt(np.sum(d * d, axis=1))
    rhat = d / r[:, None]
    pr = (psi[0].ravel()[cells] * rhat[:, 0] + psi[1].ravel()[cells] * rhat[:, 1]
          + psi[2].ravel()[cells] * rhat[:, 2]).astype(np.float64)
    s = x + (f * pr)[:, None] * rhat
    keep = geom.inside(s)
    pos = np.ascontiguousarray(s[keep])
    rpos = uniform_survey_randoms(geom, int(round(random_factor * n_gal)), seed + 1)
    wrng = np.random.default_rng(seed + 2)
    if weights == "random":
        wd = wrng.uniform(0.5, 1.5, pos.shape[0])
        wr = wrng.uniform(0.5, 1.5, rpos.shape[0])
    else:
        wd = np.ones(pos.shape[0])
        wr = np.ones(rpos.shape[0])
    data = Catalog(pos, wd, np.full(pos.shape[0], nbar))
    rand = Catalog(rpos, wr, np.full(rpos.shape[0], nbar))
    info = dict(seed=seed, volume=vs, nbar=nbar, n_data=pos.shape[0], n_rand=rpos.shape[0],
                sigma2_G=sig2, ng=ng)
    return data, rand, info


def uniform_box(box_len: float, n: int, seed: int, origin=None) -> Catalog:
    """Unclustered (Poisson) catalog filling a periodic box [o, o+L)^3."""
    rng = np.random.default_rng(seed)
    o = np.full(3, -0.5 * box_len) if origin is None else np.asarray(origin, dtype=np.float64)
    pos = o + rng.random((n, 3)) * box_len
    return Catalog(pos, np.ones(n), None)


def modulated_box(box_len: float, n: int, seed: int, j: int, amp: float, origin=None) -> Catalog:
    """Poisson catalog in a periodic box whose mean density is modulated in the (x, y) plane,
    n(x) proportional to 1 + amp [cos(2 pi j x'/L) + cos(2 pi j y'/L)] / 2 with x' = x - o,
    the transverse systematic of the cubic-box test in Sec. 3.2 (drawn by rejection; the
    modulation puts its power on the four modes j k_f along x and y, all at mu = 0 for a line of
    sight along z).  0 <= amp <= 1."""
    if not 0.0 <= amp <= 1.0:
        raise ValueError("amp must be in [0, 1]")
    rng = np.random.default_rng(seed)
    o = np.full(3, -0.5 * box_len) if origin is None else np.asarray(origin, dtype=np.float64)
    out = []
    have = 0
    while have < n:
        u = rng.random((max(2 * (n - have), 1024), 3))
        p = (1.0 + 0.5 * amp * (np.cos(2 * np.pi * j * u[:, 0]) + np.cos(2 * np.pi * j * u[:, 1]))) / (1.0 + amp)
        keep = u[rng.random(u.shape[0]) < p]
        out.append(keep[: n - have])
        have += out[-1].shape[0]
    pos = o + np.concatenate(out) * box_len
    return Catalog(pos, np.ones(n), None)


# Named workloads -------------------------------------------------------------------------

def config_c1(seed: int = 1704, n_gal: int = 30_000):
    """L=1000 Mpc/h box, 64^3 mesh, 3e4 galaxies, 10x randoms (the small plain-FP64 case)."""
    geom = SurveyGeometry(box_len=1000.0)
    return lognormal_survey(geom, n_gal, seed, ng=64)


def config_c2(seed: int = 1705, n_gal: int = 1_000_000, ng: int = 512, random_factor: float = 20.0):
    """L=2500 Mpc/h box, 512^3 mesh, 1e6 galaxies, 2e7 randoms (the headline case)."""
    geom = SurveyGeometry(box_len=2500.0)
    return lognormal_survey(geom, n_gal, seed, ng=ng, random_factor=random_factor)


def config_c3(seed: int = 1706, n_gal: int = 4_000_000, ng: int = 512, random_factor: float = 10.0):
    """L=3000 Mpc/h box, 1024^3 mesh, 4e6 galaxies, 4e7 randoms (the fine-wedge case)."""
    geom = SurveyGeometry(box_len=3000.0)
    return lognormal_survey(geom, n_gal, seed, ng=ng, random_factor=random_factor)


def batch_mock(i: int, box_len: float = 2000.0):
    """The i-th mock of the uneven-size covariance batch: (data, randoms, info, nmesh)."""
    nmesh = (128, 256, 384)[i % 3]
    rng = np.random.default_rng(2000 + i)
    n_gal = int(round(math.exp(rng.uniform(math.log(5e4), math.log(8e5)))))
    geom = SurveyGeometry(box_len=box_len)
    d, r, info = lognormal_survey(geom, n_gal, 2000 + i, ng=min(nmesh, 256))
    return d, r, info, nmesh
