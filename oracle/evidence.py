"""Exact GP evidence, posterior mean and variational objective (oracle, FP64).

Sec. 3.1, eq. "gp-mll" prints 2 ln p(d|theta) = d^T (K+S)^{-1} d + ln|2 pi (K+S)|
with the minus signs lost. Reading: -2 ln p = r^T A^{-1} r + ln|2 pi A| with
r = d - B mu (mean function, Sec. 3.1 footnote) and A = B K B^T + S, S = sigma^2 I
(the observation operator B of `psf` maps source-plane fluxes to image pixels).

Sec. 3.7, eq. "gp-exact-mean": posterior mean of the fluxes K (K+S)^{-1} d; with
the observation operator and the mean function, f_hat = mu + K B^T A^{-1} r.

App. D.1, eq. "hyper-loss": after optimising the diagonal variational posterior,
the loss is d^T (K+S)^{-1} d + sum_k N ln(alpha_k^2 + sigma^2); single layer here
("paper limit form": N is the number of source points).

Everything is dense: A is formed explicitly, factorised by LAPACK Cholesky, and
the log-determinant is twice the sum of the log-diagonal of the factor.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from . import grid, kernel, lens as lensmod, psf, source


class Problem:
    """Plain container for one reconstruction: grid, lens, source, kernel, noise, PSF."""

    def __init__(self, n, ss, pix_scale, lens, src, ell, amp, sigma, fwhm, cx=0.0, cy=0.0):
        self.n, self.ss, self.pix_scale = int(n), int(ss), float(pix_scale)
        self.cx, self.cy = float(cx), float(cy)  # image centre (crops)
        self.lens = tuple(float(v) for v in lens)
        self.src = tuple(float(v) for v in src)  # (peak, R_e, n_sersic, xs, ys)
        self.ell, self.amp, self.sigma, self.fwhm = float(ell), float(amp), float(sigma), float(fwhm)

    @property
    def N(self):
        return (self.n * self.ss) ** 2

    @property
    def n_pix(self):
        return self.n * self.n

    @property
    def h(self):
        return self.pix_scale / self.ss

    def taps(self):
        return psf.psf_taps(self.fwhm, self.h)

    def points(self):
        return lensmod.raytrace(*self.coords(), self.lens)

    def coords(self):
        return grid.fine_coords(self.n, self.ss, self.pix_scale, self.cx, self.cy)

    def mean(self, px, py):
        return source.sersic(px, py, *self.src)

    def B(self, f):
        return psf.apply_B(f, self.n, self.ss, self.taps())

    def BT(self, x):
        return psf.apply_BT(x, self.n, self.ss, self.taps())


def assemble_A(prob: Problem, px, py, block: int = 512) -> np.ndarray:
    """A = B K B^T + sigma^2 I, built one block of K's rows at a time."""
    N, n_pix = px.size, prob.n_pix
    C = np.empty((N, n_pix))  # K B^T
    for s in range(0, N, block):
        Kb = kernel.rbf_matrix(px[s:s + block], py[s:s + block], prob.ell, prob.amp, px, py)
        C[s:s + block] = prob.B(Kb.T).T
    A = np.empty((n_pix, n_pix))
    for s in range(0, n_pix, block):
        A[:, s:s + block] = prob.B(C[:, s:s + block])
    del C
    A = 0.5 * (A + A.T)
    A[np.diag_indices(n_pix)] += prob.sigma ** 2
    return A


def exact_evidence(A: np.ndarray, r: np.ndarray):
    """Cholesky evidence terms: dict(quad, logdet, lnp, u) for residual r."""
    L = sla.cholesky(A, lower=True, check_finite=False)
    u = sla.cho_solve((L, True), r, check_finite=False)
    quad = float(r @ u)
    logdet = 2.0 * float(np.sum(np.log(np.diag(L))))
    lnp = -0.5 * (quad + logdet + r.size * math.log(2.0 * math.pi))
    return dict(quad=quad, logdet=logdet, lnp=lnp, u=u, L=L)


def diag_variance_limit(amps, sigma):
    """App. D, eq. "paramvariance-layer": optimal diagonal variational variance of
    the source parameters of each layer, alpha_k^2 sigma^2 / (alpha_k^2 + sigma^2)."""
    a2 = np.asarray(amps, dtype=np.float64) ** 2
    return a2 * sigma * sigma / (a2 + sigma * sigma)


def vi_objective(quad: float, N: int, amp: float, sigma: float) -> float:
    """App. D.1 loss, single layer: quad + N ln(alpha^2 + sigma^2)."""
    return quad + N * math.log(amp * amp + sigma * sigma)


def vi_objective_full(quad: float, N: int, amp: float, sigma: float) -> float:
    """App. D.1 loss before simplification (eq. "hyper-loss", first line):
    quad + ln|Omega^2| - ln|Sigma_y| with Sigma_y at the variance limit, plus the
    constant N ln sigma^2 that the simplified form absorbs."""
    s2 = float(diag_variance_limit([amp], sigma)[0])
    return quad + N * math.log(amp * amp) - N * math.log(s2) + N * math.log(sigma * sigma)


def solve_problem(prob: Problem, d: np.ndarray, want_mean: bool = True):
    """Full exact reconstruction: points, residual, evidence, posterior mean."""
    px, py = prob.points()
    mu = prob.mean(px, py)
    r = d - prob.B(mu)
    A = assemble_A(prob, px, py)
    ev = exact_evidence(A, r)
    out = dict(px=px, py=py, mu=mu, r=r, A=A, **ev)
    out["vi"] = vi_objective(ev["quad"], px.size, prob.amp, prob.sigma)
    if want_mean:
        w = prob.BT(ev["u"])
        fhat = mu + kernel.kernel_mvm(px, py, w, prob.ell, prob.amp)
        out["w"] = w
        out["fhat"] = fhat
        out["image"] = prob.B(fhat)
    return out
