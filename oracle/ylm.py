"""Real spherical harmonics exactly as printed in eq. real-Ylm (Sec. 2.1), FP64.

Y_lm = sqrt((2l+1)/(2 pi) (l-m)!/(l+m)!) P_l^m(cos theta) cos(m phi)      m > 0
     = sqrt((2l+1)/(4 pi)) P_l(cos theta)                                 m = 0
     = sqrt((2l+1)/(2 pi) (l-|m|)!/(l+|m|)!) P_l^|m|(cos theta) sin(|m| phi)  m < 0

P_l^m is the associated Legendre function WITHOUT the Condon-Shortley phase (the printed
formula carries none).  The values come from scipy's complex harmonic ``sph_harm_y``
(which includes the (-1)^m phase):  Y_lm(real) = sqrt(2) (-1)^m Re Y_l^m for m > 0,
sqrt(2) (-1)^|m| Im Y_l^|m| for m < 0 and Re Y_l^0 for m = 0.  The polar angle is taken as
theta = arctan2(sqrt(x^2 + y^2), z), which stays accurate next to the poles (arccos of
z/r does not).  A zero vector gets Y_lm = 0 for l > 0 (and the constant for l = 0).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import sph_harm_y


def angles(xyz: np.ndarray):
    xyz = np.asarray(xyz, dtype=np.float64)
    rho = np.hypot(xyz[..., 0], xyz[..., 1])
    theta = np.arctan2(rho, xyz[..., 2])
    phi = np.arctan2(xyz[..., 1], xyz[..., 0])
    r = np.hypot(rho, xyz[..., 2])
    return r, theta, phi


def real_ylm(ell: int, m: int, xyz: np.ndarray) -> np.ndarray:
    """Real Y_lm of the direction of each vector in ``xyz`` (shape (..., 3))."""
    if abs(m) > ell:
        raise ValueError("|m| must be <= ell")
    r, theta, phi = angles(xyz)
    am = abs(m)
    y = sph_harm_y(ell, am, theta, phi)
    if m == 0:
        out = np.real(y)
    elif m > 0:
        out = math.sqrt(2.0) * (-1.0) ** am * np.real(y)
    else:
        out = math.sqrt(2.0) * (-1.0) ** am * np.imag(y)
    out = np.asarray(out, dtype=np.float64)
    if ell > 0:
        out = np.where(r > 0, out, 0.0)
    return out
