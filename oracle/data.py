"""Synthetic observations from the generative model (oracle, FP64).

Sec. 3.3, eq. "gp-gen1": d ~ N(f, S), f ~ N(mu, K) (with the mean function of
Sec. 3.1); observed through B (PSF + local averaging, see `psf`):
d = B (mu + g) + sigma * eps, g ~ GP(0, k_RBF) at the ray-traced points.

The paper's mocks lens HST galaxy images (Sec. 4.1); those images are not used
here. The GP draw g is exact for small N (Cholesky of K + tiny jitter, standard
normals supplied by the caller) and, for large N, uses random Fourier features
(Rahimi & Recht 2007): g(p) = alpha sqrt(2/M) sum_m w_m cos(omega_m . p / ell + b_m)
with omega ~ N(0, I), b ~ U(0, 2 pi), w ~ N(0, 1), whose covariance is exactly
the RBF kernel in expectation.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import evidence, kernel


def gp_draw_exact(px, py, ell, amp, normals, jitter=1e-10):
    K = kernel.rbf_matrix(px, py, ell, amp)
    K[np.diag_indices(px.size)] += jitter * amp * amp
    L = sla.cholesky(K, lower=True, check_finite=False)
    return L @ normals


def gp_draw_rff(px, py, ell, amp, omega, phase, w, block=4096):
    M = w.size
    out = np.empty(px.size)
    for s in range(0, px.size, block):
        arg = (np.outer(px[s:s + block], omega[:, 0]) + np.outer(py[s:s + block], omega[:, 1])) / ell + phase
        out[s:s + block] = amp * np.sqrt(2.0 / M) * (np.cos(arg) @ w)
    return out


def simulate(prob: evidence.Problem, noise, gp_normals=None, rff=None):
    """Observed image d (length n_pix) and the noiseless fine-grid truth."""
    px, py = prob.points()
    mu = prob.mean(px, py)
    if gp_normals is not None:
        g = gp_draw_exact(px, py, prob.ell, prob.amp, gp_normals)
    elif rff is not None:
        g = gp_draw_rff(px, py, prob.ell, prob.amp, *rff)
    else:
        g = np.zeros_like(mu)
    truth = mu + g
    d = prob.B(truth) + prob.sigma * np.asarray(noise)
    return d, truth
