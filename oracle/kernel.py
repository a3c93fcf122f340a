"""Gaussian RBF covariance over source-plane points (oracle, FP64).

Sec. 3.1, eq. "grbf": k(x1, x2) = alpha^2 exp(-(x1-x2)^T Sigma^{-1} (x1-x2) / 2),
with the isotropic kernel Sigma = ell^2 I (eq. "grbf-layers" and the text after
it). The matrix K_ij = k(p_i, p_j) is formed explicitly here (dense, or one
row block at a time for the matrix-free product).
"""
from __future__ import annotations

import numpy as np


def sqdist(ax, ay, bx, by):
    """Squared distances |a_i - b_j|^2 as an (len(a), len(b)) array."""
    dx = np.asarray(ax)[:, None] - np.asarray(bx)[None, :]
    dy = np.asarray(ay)[:, None] - np.asarray(by)[None, :]
    return dx * dx + dy * dy


def rbf_matrix(px, py, ell, amp, qx=None, qy=None):
    """Dense K with K_ij = amp^2 exp(-|p_i - q_j|^2 / (2 ell^2)); q defaults to p."""
    if qx is None:
        qx, qy = px, py
    return amp * amp * np.exp(-sqdist(px, py, qx, qy) / (2.0 * ell * ell))


def kernel_mvm(px, py, V, ell, amp, block: int = 2048):
    """Y = K V without storing K: one block of rows of K at a time."""
    px = np.asarray(px, dtype=np.float64)
    py = np.asarray(py, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    Y = np.empty((px.size,) + V.shape[1:])
    for s in range(0, px.size, block):
        Kb = rbf_matrix(px[s:s + block], py[s:s + block], ell, amp, px, py)
        Y[s:s + block] = Kb @ V
    return Y


def kernel_mvm_rows(px, py, rows, V, ell, amp):
    """Selected rows of K V (for spot checks of large products)."""
    Kr = rbf_matrix(np.asarray(px)[rows], np.asarray(py)[rows], ell, amp, px, py)
    return Kr @ V


def kernel_abs_mvm_rows(px, py, rows, V, ell, amp):
    """Selected rows of |K| |V| (entrywise absolute values): the scale of each
    output entry, used to state per-entry error bounds of a product."""
    Kr = rbf_matrix(np.asarray(px)[rows], np.asarray(py)[rows], ell, amp, px, py)
    return Kr @ np.abs(V)
