"""Ray tracing through an SPLE lens with external shear (oracle, FP64).

Sec. 2.1, lens equation: x = xi - alpha(xi).
Sec. 2.2: elliptical coordinates (R_x, R_y) = diag(sqrt q, 1/sqrt q) rot(phi) (xi - xi_0),
tan(varphi) = R_y / R_x; SPLE deflection (eq. "dispsple", complex notation)

    alpha = theta_E * 2 sqrt(q)/(1+q) * (theta_E/R)^(slope-2)
            * 2F1(1, (slope-1)/2; (5-slope)/2; -(1-q)/(1+q) e^{2 i varphi}) * e^{i varphi}

and the external-shear deflection [[g1, g2], [g2, -g1]] xi.

Readings (the paper is silent on them):
  * the complex SPLE deflection lives in the lens-aligned, unscaled frame and is
    rotated back by -phi into the sky frame;
  * the shear acts about the optical axis (it multiplies xi, as printed);
  * R is floored at 1e-9 arcsec so the lens centre itself stays finite.

2F1 with first parameter 1 is summed from its defining power series,
sum_k (b)_k/(c)_k z^k, which converges for |z| = (1-q)/(1+q) < 1.
"""
from __future__ import annotations

import numpy as np

R_FLOOR = 1e-9


def hyp2f1_one(b: float, c: float, z: np.ndarray, rtol: float = 1e-17, kmax: int = 100000) -> np.ndarray:
    """2F1(1, b; c; z) by its power series (complex z, |z| < 1), term ratio (b+k)/(c+k) z."""
    z = np.asarray(z, dtype=np.complex128)
    term = np.ones_like(z)
    total = np.ones_like(z)
    for k in range(kmax):
        term = term * ((b + k) / (c + k)) * z
        total = total + term
        if np.all(np.abs(term) <= rtol * np.abs(total)):
            break
    else:  # pragma: no cover
        raise RuntimeError("2F1 series did not converge")
    return total


def elliptical_coords(xi_x, xi_y, q, phi, x0, y0):
    """(R_x, R_y) of Sec. 2.2 for image-plane points."""
    dx, dy = np.asarray(xi_x) - x0, np.asarray(xi_y) - y0
    c, s = np.cos(phi), np.sin(phi)
    xp = c * dx + s * dy
    yp = -s * dx + c * dy
    return np.sqrt(q) * xp, yp / np.sqrt(q)


def sple_deflection(xi_x, xi_y, theta_E, q, phi, slope, x0, y0):
    """SPLE deflection (alpha_x, alpha_y) in the sky frame, eq. "dispsple"."""
    Rx, Ry = elliptical_coords(xi_x, xi_y, q, phi, x0, y0)
    R = np.maximum(np.hypot(Rx, Ry), R_FLOOR)
    varphi = np.arctan2(Ry, Rx)
    z = -(1.0 - q) / (1.0 + q) * np.exp(2j * varphi)
    F = hyp2f1_one((slope - 1.0) / 2.0, (5.0 - slope) / 2.0, z)
    a = theta_E * 2.0 * np.sqrt(q) / (1.0 + q) * (theta_E / R) ** (slope - 2.0) * F * np.exp(1j * varphi)
    ax_l, ay_l = a.real, a.imag  # lens-aligned frame
    c, s = np.cos(phi), np.sin(phi)
    return c * ax_l - s * ay_l, s * ax_l + c * ay_l


def shear_deflection(xi_x, xi_y, gamma1, gamma2):
    """External shear deflection [[g1, g2], [g2, -g1]] xi (Sec. 2.2)."""
    xi_x, xi_y = np.asarray(xi_x), np.asarray(xi_y)
    return gamma1 * xi_x + gamma2 * xi_y, gamma2 * xi_x - gamma1 * xi_y


def raytrace(xi_x, xi_y, lens):
    """Source-plane positions p = xi - alpha_SPLE(xi) - alpha_shear(xi) (eq. "lens").

    `lens` is a sequence (theta_E, q, phi, slope, x0, y0, gamma1, gamma2)."""
    theta_E, q, phi, slope, x0, y0, g1, g2 = lens
    ax, ay = sple_deflection(xi_x, xi_y, theta_E, q, phi, slope, x0, y0)
    sx, sy = shear_deflection(xi_x, xi_y, g1, g2)
    return np.asarray(xi_x) - ax - sx, np.asarray(xi_y) - ay - sy


def convergence(xi_x, xi_y, theta_E, q, phi, slope, x0, y0):
    """SPLE convergence kappa = (3-slope)/2 (theta_E/R)^(slope-1) (Sec. 2.2)."""
    Rx, Ry = elliptical_coords(xi_x, xi_y, q, phi, x0, y0)
    R = np.hypot(Rx, Ry)
    return (3.0 - slope) / 2.0 * (theta_E / R) ** (slope - 1.0)


def raytrace_jacobian(xi_x, xi_y, lens, rel_step: float = 1e-3):
    """dp/dtheta for the 8 lens parameters, shape (N, 2, 8).

    Five-point central differences in FP64 (truncation O(h^4)); parameter order
    (theta_E, q, phi, slope, x0, y0, gamma1, gamma2). Angles use an absolute step."""
    lens = np.asarray(lens, dtype=np.float64)
    scale = np.array([lens[0], lens[1], 1.0, 1.0, lens[0], lens[0], 1.0, 1.0])
    N = np.size(xi_x)
    J = np.empty((N, 2, 8))
    for k in range(8):
        h = rel_step * scale[k]
        if k == 1:  # keep q inside (0, 1]
            h = min(h, 0.25 * (1.0 - lens[1])) if lens[1] < 1.0 else h
        vals = []
        for m in (-2, -1, 1, 2):
            t = lens.copy()
            t[k] += m * h
            vals.append(np.stack(raytrace(xi_x, xi_y, t), axis=-1))
        J[:, :, k] = (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h)
    return J
