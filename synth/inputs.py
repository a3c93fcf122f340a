"""Workload definitions and seeded random draws (no method arithmetic here).

Workloads follow the paper's mock-data setting: a lensed image of a few
arcseconds, supersampled pixels that are locally averaged (Sec. 4.1), an SPLE
lens with external shear whose parameters come from uniform priors
(Sec. 4.1, Table "lens-params"), a single-layer RBF GP source (Sec. 3.1) plus
a smooth Sersic mean function (footnote on the mean function in Sec. 3.1), and
i.i.d. Gaussian noise set so the brightest pixel has SNR ~ 30 (Sec. 4.1).

Every stream of random numbers is drawn from numpy's PCG64 seeded through a
SeedSequence of (base seed, workload index, stream tag), so the GPU path and
the oracle consume identical arrays.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BASE_SEED = 2105_09465

# stream tags, one per kind of draw
_TAG_LENS, _TAG_PROBE, _TAG_GP, _TAG_NOISE, _TAG_RFF, _TAG_TRACE = 1, 2, 3, 4, 5, 6


@dataclasses.dataclass(frozen=True)
class Lens:
    """SPLE + external shear parameters (Sec. 2.2): angles in arcsec, phi in rad."""

    theta_E: float
    q: float
    phi: float
    slope: float
    x0: float
    y0: float
    gamma1: float
    gamma2: float

    def as_tuple(self):
        return (self.theta_E, self.q, self.phi, self.slope, self.x0, self.y0, self.gamma1, self.gamma2)


LENS_PARAM_NAMES = ("theta_E", "q", "phi", "slope", "x0", "y0", "gamma1", "gamma2")


@dataclasses.dataclass(frozen=True)
class Source:
    """Circular Sersic mean function: peak brightness, effective radius, index, centre."""

    peak: float
    R_e: float
    n_sersic: float
    xs: float
    ys: float


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: int  # image side in pixels
    ss: int  # supersampling factor per axis
    pix_scale: float  # arcsec per image pixel
    lens: Lens
    source: Source
    ell: float  # GP lengthscale (arcsec)
    amp: float  # GP root variance alpha
    noise_sigma: float
    psf_fwhm: float  # arcsec; 0 disables the PSF
    n_probes: int
    cg_tol: float
    max_iter: int
    n_lanczos: int
    fixed_iters: int = 0  # >0: run exactly this many CG iterations

    @property
    def M(self) -> int:
        return self.n * self.ss

    @property
    def N(self) -> int:
        return self.M * self.M

    @property
    def n_pix(self) -> int:
        return self.n * self.n

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def _rng(index: int, tag: int, sub: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([BASE_SEED, index, tag, sub])))


# Shared hyperparameters: lengthscale 0.04", amplitude 0.3, noise 0.02, PSF FWHM 0.1"
ELL, AMP, SIGMA, FWHM = 0.04, 0.3, 0.02, 0.1
PIX = 0.05
SERSIC_N, SERSIC_RE = 1.5, 0.1


def draw_lens(index: int, sub: int = 0) -> Lens:
    """Lens drawn from the priors: slope U(1.8,2.2), theta_E U(0.8,1.4)", q U(0.6,0.95),
    centre U(-0.2,0.2)", position angle U(0,2pi), shear magnitude U(0,0.08) with a
    uniform orientation psi in U(0,pi): (gamma1, gamma2) = |g| (cos 2psi, sin 2psi)."""
    r = _rng(index, _TAG_LENS, sub)
    slope = r.uniform(1.8, 2.2)
    theta_E = r.uniform(0.8, 1.4)
    q = r.uniform(0.6, 0.95)
    x0, y0 = r.uniform(-0.2, 0.2, size=2)
    phi = r.uniform(0.0, 2 * math.pi)
    g = r.uniform(0.0, 0.08)
    psi = r.uniform(0.0, math.pi)
    return Lens(theta_E, q, phi, slope, float(x0), float(y0), g * math.cos(2 * psi), g * math.sin(2 * psi))


def draw_source_offset(index: int, sub: int = 0):
    r = _rng(index, _TAG_LENS, 1000 + sub)
    xs, ys = r.uniform(-0.1, 0.1, size=2)
    return float(xs), float(ys)


def workload(index: int, sub: int = 0) -> Workload:
    """The five workloads (index 0..4); `sub` selects another prior draw."""
    src = Source(peak=30 * SIGMA, R_e=SERSIC_RE, n_sersic=SERSIC_N, xs=0.0, ys=0.0)
    if index == 0:
        lens = Lens(0.6, 0.8, math.radians(30.0), 2.0, 0.0, 0.0, 0.03, 0.0)
        return Workload("plain-fp64-24px", 24, 1, PIX, lens, src, ELL, AMP, SIGMA, FWHM,
                        n_probes=16, cg_tol=0.0, max_iter=50, n_lanczos=30, fixed_iters=50)
    xs, ys = draw_source_offset(index, sub)
    src = dataclasses.replace(src, xs=xs, ys=ys)
    lens = draw_lens(index, sub)
    if index == 1:
        return Workload("fp32-100px-ss2", 100, 2, PIX, lens, src, ELL, AMP, SIGMA, FWHM,
                        n_probes=16, cg_tol=1e-6, max_iter=1000, n_lanczos=30)
    if index == 2:
        return Workload("mixed-200px-ss2", 200, 2, PIX, lens, src, ELL, AMP, SIGMA, FWHM,
                        n_probes=63, cg_tol=1e-6, max_iter=1000, n_lanczos=30)
    if index == 3:
        return Workload("grad-100px-ss2", 100, 2, PIX, lens, src, ELL, AMP, SIGMA, FWHM,
                        n_probes=16, cg_tol=1e-6, max_iter=1000, n_lanczos=30)
    if index == 4:
        return Workload("serve", 64, 1, PIX, lens, src, ELL, AMP, SIGMA, FWHM,
                        n_probes=16, cg_tol=1e-6, max_iter=1000, n_lanczos=30)
    raise ValueError(index)


def rademacher(n: int, m: int, index: int, sub: int = 0) -> np.ndarray:
    """(n, m) float64 array of independent +-1 entries (Hutchinson probes)."""
    r = _rng(index, _TAG_PROBE, sub)
    return (r.integers(0, 2, size=(n, m), dtype=np.int8) * 2 - 1).astype(np.float64)


_TAG_PC_PROBE = 7
_TAG_VIGP = 8


def preconditioned_probe_normals(n: int, k: int, m: int, index: int, sub: int = 0):
    """Standard normals for m probes of a rank-k preconditioner on n pixels:
    g (m, k) and h (m, n), both float64."""
    r = _rng(index, _TAG_PC_PROBE, sub)
    return r.standard_normal((m, k)), r.standard_normal((m, n))


def vigp_normals(n32: int, step: int, index: int = 1):
    """Standard normals of one reparametrised sample of the variational step:
    the 7 lens-parameter normals (float64) and n32 source-parameter normals."""
    r = _rng(index, _TAG_VIGP, step)
    return r.standard_normal(7), r.standard_normal(n32)


def gp_normals(N: int, index: int, sub: int = 0) -> np.ndarray:
    """Standard normals for an exact (factorised) GP draw over N points."""
    return _rng(index, _TAG_GP, sub).standard_normal(N)


def rff_draws(M: int, index: int, sub: int = 0):
    """Random Fourier feature draws: (omega (M,2) standard normals, phase U(0,2pi), weights N(0,1))."""
    r = _rng(index, _TAG_RFF, sub)
    omega = r.standard_normal((M, 2))
    phase = r.uniform(0.0, 2 * math.pi, size=M)
    w = r.standard_normal(M)
    return omega, phase, w


def noise_normals(n_pix: int, index: int, sub: int = 0) -> np.ndarray:
    return _rng(index, _TAG_NOISE, sub).standard_normal(n_pix)


def source_grid(n: int = 40, spacing: float = 0.03, cx: float = 0.0, cy: float = 0.0):
    """Regular n x n grid of source-plane points (row-major, y increasing with
    the row), `spacing` arcsec apart and centred on (cx, cy): the paper's
    source-plane grid is 40 x 40 at 30 mas (Sec. 4.1). Returns (gx, gy) float64."""
    o = (np.arange(n) - (n - 1) / 2.0) * spacing
    gy, gx = np.meshgrid(o + cy, o + cx, indexing="ij")
    return gx.ravel(), gy.ravel()


SERVE_SIDES = (48, 64, 96, 128, 160)


def serving_trace(n_requests: int, rate_hz: float, index: int = 4, sub: int = 0):
    """Poisson arrival trace: list of (arrival_s, side, ss, request_sub_seed)."""
    r = _rng(index, _TAG_TRACE, sub)
    gaps = r.exponential(1.0 / rate_hz, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    sides = r.choice(np.array(SERVE_SIDES), size=n_requests)
    sss = r.choice(np.array([1, 2]), size=n_requests)
    return [(float(t[i]), int(sides[i]), int(sss[i]), 1000 + i) for i in range(n_requests)]


def serving_request(side: int, ss: int, req_seed: int) -> Workload:
    """A serving request: lens and source offset from the priors, given size."""
    base = workload(4, req_seed)
    return base.replace(name=f"serve-{side}px-ss{ss}", n=side, ss=ss)
