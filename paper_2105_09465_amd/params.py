"""Parameter containers of one lensed-source reconstruction and their C structs.

Names follow the paper: SPLE lens (theta_E, q, phi, slope, centre x0, y0) with
external shear (gamma1, gamma2) (Sec. 2.2); RBF kernel lengthscale and
amplitude (Sec. 3.1); noise sigma; a Sersic mean function; a Gaussian PSF.
"""
from __future__ import annotations

import dataclasses
import math

from . import _lib


@dataclasses.dataclass(frozen=True)
class Grid:
    n: int
    ss: int
    pix_scale: float
    cx: float = 0.0
    cy: float = 0.0

    @property
    def M(self):
        return self.n * self.ss

    @property
    def N(self):
        return self.M * self.M

    @property
    def n_pix(self):
        return self.n * self.n

    def c(self):
        return _lib.gpl_grid(self.n, self.ss, self.pix_scale, self.cx, self.cy)


@dataclasses.dataclass(frozen=True)
class Lens:
    theta_E: float
    q: float
    phi: float
    slope: float
    x0: float
    y0: float
    gamma1: float
    gamma2: float

    NAMES = ("theta_E", "q", "phi", "slope", "x0", "y0", "gamma1", "gamma2")

    def c(self):
        return _lib.gpl_lens(*(float(getattr(self, k)) for k in self.NAMES))

    def as_tuple(self):
        return tuple(float(getattr(self, k)) for k in self.NAMES)


@dataclasses.dataclass(frozen=True)
class Sersic:
    """Circular Sersic profile given by its central brightness `peak`."""

    peak: float
    R_e: float
    n_sersic: float
    xs: float
    ys: float

    def c(self):
        bn = _lib.lib.gpl_sersic_bn(self.n_sersic)
        return _lib.gpl_source(self.peak * math.exp(-bn), self.R_e, self.n_sersic, bn, self.xs, self.ys)


@dataclasses.dataclass(frozen=True)
class Kernel:
    lengthscale: float
    amplitude: float
    kind: int = 0  # 0: RBF (eq. "grbf"); 1: pixel-shape windowed kernel (eq. "covariance")

    def c(self):
        return _lib.gpl_kernel(self.kind, self.lengthscale, self.amplitude)


@dataclasses.dataclass(frozen=True)
class PSF:
    fwhm: float
    radius: int = 0

    def c(self):
        return _lib.gpl_psf(self.fwhm, self.radius)


@dataclasses.dataclass(frozen=True)
class Problem:
    grid: Grid
    lens: Lens
    source: Sersic
    kernel: Kernel
    psf: PSF
    noise_sigma: float

    def replace(self, **kw):
        return dataclasses.replace(self, **kw)
