"""Sersic mean function (oracle, FP64).

Sec. 3.1 (footnote on the mean function): a prior dependence of the source on
position enters the marginal likelihood through d -> d - mu(p). The paper names
a Sersic profile (Sec. 1) without defining it; reading: circular Sersic
mu(p) = I_e exp(-b_n [(|p - p_s| / R_e)^(1/n) - 1]) with b_n the half-light
constant, i.e. the root of P(2n, b_n) = 1/2 (regularised lower incomplete
gamma), and I_e = peak * exp(-b_n) so that `peak` is the central brightness.
"""
from __future__ import annotations

import numpy as np
from scipy import special


def sersic_bn(n: float) -> float:
    """Half-light constant: P(2n, b_n) = 1/2."""
    return float(special.gammaincinv(2.0 * n, 0.5))


def sersic(px, py, peak, R_e, n, xs, ys):
    """Sersic brightness at source-plane points."""
    bn = sersic_bn(n)
    I_e = peak * np.exp(-bn)
    r = np.hypot(np.asarray(px) - xs, np.asarray(py) - ys)
    return I_e * np.exp(-bn * ((r / R_e) ** (1.0 / n) - 1.0))


def sersic_grad(px, py, peak, R_e, n, xs, ys):
    """d mu / d p (shape (N, 2)); d mu / d p_s is its negative. Analytic in r."""
    bn = sersic_bn(n)
    mu = sersic(px, py, peak, R_e, n, xs, ys)
    dx, dy = np.asarray(px) - xs, np.asarray(py) - ys
    r = np.hypot(dx, dy)
    with np.errstate(divide="ignore", invalid="ignore"):
        # d mu / d r = -mu * b_n / n * r^(1/n - 1) / R_e^(1/n)
        dmu_dr = -mu * bn / n * (r ** (1.0 / n - 1.0)) / (R_e ** (1.0 / n))
        gx = np.where(r > 0, dmu_dr * dx / r, 0.0)
        gy = np.where(r > 0, dmu_dr * dy / r, 0.0)
    return np.stack([gx, gy], axis=-1)
