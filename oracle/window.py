"""Pixel-shape (windowed) covariance, transmission factorisation and source
reconstruction (oracle, FP64).

Sec. 3.2: each observed pixel integrates the source brightness over its
projected area, approximated by a Gaussian indicator w_i(x) = N(x - p_i, Z_i)
(eq. "window-function") whose covariance comes from the pixel axes a_i, b_i
(eq. "window-kernel"): Z_i = (a a^T + b b^T) / (4 pi); App. C shows this
satisfies int w_i^2 = 1/A_i with A_i = |a_i x b_i|. The axes are half the
distance between the projected centres of the two neighbouring pixels along
each grid axis (footnote to eq. "window-kernel"). With the RBF covariance of
eq. "grbf" (Sigma = l^2 I), eq. "covariance" gives
    K_ij = alpha^2 sqrt|2 pi Sigma| N(p_i - p_j, Z_i + Sigma + Z_j),
which reduces to the RBF kernel as Z -> 0.

Sec. 3.4, eq. "transmission": K ~ alpha^2 T T^T with
    T_ik = A_k N(p_i - q_k, Z_i + Sigma/2),  A_k = |2 pi Sigma|^{1/4} / sqrt(rho(q_k)),
rho the density of the inducing points q, estimated (footnote there) from the
area of the circle reaching the k-th closest inducing point, k = 20.
Sec. 3.5, eq. "gp-reconstruction": beta(x) = sum_k A_k N(x - q_k, Sigma/2) y_k.

Readings (the paper is silent): at a grid edge the single neighbour's centre
is used, a = p_next - p (or p - p_prev), the same scale as half the two-sided
difference; the k-th closest point to an inducing point q is counted among the
other inducing points (q itself excluded).
"""
from __future__ import annotations

import math

import numpy as np


def pixel_axes(px, py, M: int):
    """(a, b) per point of an M x M grid in row-major order, each (N, 2): half
    the difference of the projected neighbours along the grid's x (a) and y (b)
    axes; one-sided at the edges."""
    P = np.stack([np.asarray(px, dtype=np.float64).reshape(M, M), np.asarray(py, dtype=np.float64).reshape(M, M)],
                 axis=-1)

    def axis_diff(Q, ax):
        D = np.empty_like(Q)
        if Q.shape[ax] == 1:
            return np.zeros_like(Q)
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        mid = [slice(None)] * 3
        lo[ax], hi[ax] = slice(0, -2), slice(2, None)
        mid[ax] = slice(1, -1)
        D[tuple(mid)] = 0.5 * (Q[tuple(hi)] - Q[tuple(lo)])
        first = [slice(None)] * 3
        second = [slice(None)] * 3
        first[ax], second[ax] = 0, 1
        D[tuple(first)] = Q[tuple(second)] - Q[tuple(first)]
        last = [slice(None)] * 3
        prev = [slice(None)] * 3
        last[ax], prev[ax] = -1, -2
        D[tuple(last)] = Q[tuple(last)] - Q[tuple(prev)]
        return D

    a = axis_diff(P, 1).reshape(-1, 2)  # along x (columns)
    b = axis_diff(P, 0).reshape(-1, 2)  # along y (rows)
    return a, b


def shape_cov(a, b):
    """Z = (a a^T + b b^T) / (4 pi) as (zxx, zxy, zyy), eq. "window-kernel"."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    f = 1.0 / (4.0 * math.pi)
    return np.stack([f * (a[:, 0] ** 2 + b[:, 0] ** 2), f * (a[:, 0] * a[:, 1] + b[:, 0] * b[:, 1]),
                     f * (a[:, 1] ** 2 + b[:, 1] ** 2)], axis=-1)


def gauss2(dx, dy, cxx, cxy, cyy):
    """Bivariate normal density N(d, C) = exp(-d^T C^{-1} d / 2) / (2 pi sqrt|C|)."""
    det = cxx * cyy - cxy * cxy
    q = (cyy * dx * dx - 2.0 * cxy * dx * dy + cxx * dy * dy) / det
    return np.exp(-0.5 * q) / (2.0 * math.pi * np.sqrt(det))


def windowed_kernel_matrix(px, py, Z, ell, amp, qx=None, qy=None, Zq=None):
    """K_ij = alpha^2 sqrt|2 pi Sigma| N(p_i - q_j, Z_i + Sigma + Zq_j), Sigma = l^2 I
    (eq. "covariance"); q, Zq default to p, Z. Z as (N, 3) = (zxx, zxy, zyy)."""
    px = np.asarray(px, dtype=np.float64)
    py = np.asarray(py, dtype=np.float64)
    Z = np.zeros((px.size, 3)) if Z is None else np.asarray(Z, dtype=np.float64)
    if qx is None:
        qx, qy, Zq = px, py, Z
    qx = np.asarray(qx, dtype=np.float64)
    qy = np.asarray(qy, dtype=np.float64)
    Zq = np.zeros((qx.size, 3)) if Zq is None else np.asarray(Zq, dtype=np.float64)
    s2 = ell * ell
    cxx = Z[:, 0][:, None] + Zq[:, 0][None, :] + s2
    cxy = Z[:, 1][:, None] + Zq[:, 1][None, :]
    cyy = Z[:, 2][:, None] + Zq[:, 2][None, :] + s2
    dx = px[:, None] - qx[None, :]
    dy = py[:, None] - qy[None, :]
    return amp * amp * (2.0 * math.pi * s2) * gauss2(dx, dy, cxx, cxy, cyy)


def windowed_kernel_mvm(px, py, Z, V, ell, amp, block: int = 2048):
    """Y = K V for the windowed K, one block of rows at a time."""
    px = np.asarray(px, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    Y = np.empty((px.size,) + V.shape[1:])
    Z = np.asarray(Z, dtype=np.float64)
    for s in range(0, px.size, block):
        Kb = windowed_kernel_matrix(px[s:s + block], np.asarray(py)[s:s + block], Z[s:s + block], ell, amp, px, py, Z)
        Y[s:s + block] = Kb @ V
    return Y


def knn_density(qx, qy, k: int = 20):
    """rho(q) = k / (pi r_k^2), r_k the distance from q to its k-th closest other
    inducing point (footnote to eq. "transmission"), by brute force."""
    qx = np.asarray(qx, dtype=np.float64)
    qy = np.asarray(qy, dtype=np.float64)
    rho = np.empty(qx.size)
    for s in range(0, qx.size, 1024):
        d2 = (qx[s:s + 1024, None] - qx[None, :]) ** 2 + (qy[s:s + 1024, None] - qy[None, :]) ** 2
        d2[np.arange(d2.shape[0]), np.arange(s, s + d2.shape[0])] = np.inf  # exclude q itself
        rk2 = np.partition(d2, k - 1, axis=1)[:, k - 1]
        rho[s:s + 1024] = k / (math.pi * rk2)
    return rho


def knn_radius(qx, qy, k: int = 20, rows=None):
    """(r_k, nn): distance from each point (or each point of `rows`) to its
    k-th closest other point and that neighbour's index (brute force; the
    density of `knn_density` is k / (pi r_k^2))."""
    qx = np.asarray(qx, dtype=np.float64)
    qy = np.asarray(qy, dtype=np.float64)
    rows = np.arange(qx.size) if rows is None else np.asarray(rows)
    r = np.empty(rows.size)
    nn = np.empty(rows.size, dtype=np.int64)
    for s in range(0, rows.size, 1024):
        rr = rows[s:s + 1024]
        d2 = (qx[rr, None] - qx[None, :]) ** 2 + (qy[rr, None] - qy[None, :]) ** 2
        d2[np.arange(rr.size), rr] = np.inf
        idx = np.argsort(d2, axis=1, kind="stable")[:, k - 1]
        nn[s:s + 1024] = idx
        r[s:s + 1024] = np.sqrt(d2[np.arange(rr.size), idx])
    return r, nn


def transmission_weights(rho, ell):
    """A_k = |2 pi Sigma|^{1/4} / sqrt(rho_k) with Sigma = l^2 I (2-D)."""
    return math.sqrt(2.0 * math.pi * ell * ell) / np.sqrt(np.asarray(rho, dtype=np.float64))


def transmission_matrix(px, py, Z, qx, qy, ell, A):
    """T_ik = A_k N(p_i - q_k, Z_i + Sigma/2) (eq. "transmission"); Z None for no
    pixel shapes."""
    px = np.asarray(px, dtype=np.float64)
    py = np.asarray(py, dtype=np.float64)
    Z = np.zeros((px.size, 3)) if Z is None else np.asarray(Z, dtype=np.float64)
    h = 0.5 * ell * ell
    dx = px[:, None] - np.asarray(qx, dtype=np.float64)[None, :]
    dy = py[:, None] - np.asarray(qy, dtype=np.float64)[None, :]
    return np.asarray(A)[None, :] * gauss2(dx, dy, Z[:, 0][:, None] + h, Z[:, 1][:, None], Z[:, 2][:, None] + h)


def reconstruct_brightness(x, y, qx, qy, yk, ell, A):
    """beta(x) = sum_k A_k N(x - q_k, Sigma/2) y_k (eq. "gp-reconstruction")."""
    return transmission_matrix(x, y, None, qx, qy, ell, A) @ np.asarray(yk, dtype=np.float64)
