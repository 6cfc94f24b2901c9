"""Gaussian mocks with linear Kaiser distortions for the wedge-covariance study of Sec. 4.1.

Each mock is a Gaussian random field on an n^3 grid whose spectrum is
(1 + beta mu^2)^2 P(k) with mu = k_z/|k| (line of sight along z, eq. kaiser), delivered as
weights w = 1 + delta of one object sitting exactly on every mesh node.  Painted with NGP and
neither interlacing nor compensation, the mesh is then w itself, so an estimate sees the
field's modes with no shot noise and no window: the setting of the linear-theory covariance.

Only input generation happens here (white noise shaped in Fourier space); it holds none of
the estimator's arithmetic.  torch is used so that thousands of mocks can be drawn on the
device that consumes them; the same call runs on the CPU.
"""
from __future__ import annotations

import math

import numpy as np


def model_pk(k):
    """The shape used by the lognormal mocks, (Mpc/h)^3."""
    x = k / 0.02
    return 2.0e4 * x / (1.0 + x ** 2.6)


def node_positions(n: int, box_len: float, device="cpu", origin=None):
    """(n^3, 3) float64 positions o + c L/n of the mesh nodes, x slowest (the mesh order)."""
    import torch
    o = torch.full((3,), -0.5 * box_len, dtype=torch.float64) if origin is None else \
        torch.as_tensor(origin, dtype=torch.float64)
    c = torch.arange(n, dtype=torch.float64) * (box_len / n)
    gx, gy, gz = torch.meshgrid(c, c, c, indexing="ij")
    pos = torch.stack([gx.reshape(-1), gy.reshape(-1), gz.reshape(-1)], dim=1) + o[None, :]
    return pos.to(device)


class KaiserBox:
    """Draws mocks of one (n, L, beta) setting; the spectral filter is built once."""

    def __init__(self, n: int, box_len: float, beta: float, bias: float = 1.0, sigma_cell: float = 0.05,
                 device="cpu"):
        import torch
        self.n, self.box_len, self.device = n, box_len, device
        kf = 2.0 * math.pi / box_len
        f = np.fft.fftfreq(n, 1.0 / n) * kf
        fz = np.fft.rfftfreq(n, 1.0 / n) * kf
        k2 = f[:, None, None] ** 2 + f[None, :, None] ** 2 + fz[None, None, :] ** 2
        k2[0, 0, 0] = 1.0
        mu2 = fz[None, None, :] ** 2 / k2
        amp = bias * (1.0 + beta * mu2) * np.sqrt(model_pk(np.sqrt(k2)))
        amp[0, 0, 0] = 0.0
        # normalise the per-cell rms of delta to sigma_cell (weights stay near 1)
        var = (2.0 * np.sum(amp[:, :, 1:] ** 2) + np.sum(amp[:, :, :1] ** 2)) / float(n) ** 3
        amp *= sigma_cell / math.sqrt(var)
        self.filter = torch.tensor(amp, dtype=torch.float64, device=device)

    def weights(self, seed: int, out=None):
        """w = 1 + delta (float64, n^3, mesh order) of mock `seed`."""
        import torch
        n = self.n
        g = torch.Generator(device=self.device)
        g.manual_seed(int(seed))
        white = torch.randn((n, n, n), generator=g, dtype=torch.float64, device=self.device)
        delta = torch.fft.irfftn(torch.fft.rfftn(white) * self.filter, s=(n, n, n))
        w = delta.reshape(-1) + 1.0
        if out is None:
            return w
        out.copy_(w)
        return out
