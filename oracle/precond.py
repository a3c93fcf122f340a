"""Low-rank preconditioned CG and stochastic log-determinant (oracle, FP64).

Sec. 3.3 discusses evaluating eq. "gp-mll" the way GPyTorch does: conjugate
gradients for the solves and a stochastic Lanczos estimate of the
log-determinant, and it names the noise of that estimate (1-2%) as the reason
the paper avoids it. GPyTorch (Gardner et al. 2018, the reference Sec. 3.3
cites) lowers that noise with a preconditioner P = L L^T + sigma^2 I built from
a partial pivoted Cholesky factor L of the kernel part of the matrix; log|P|
is exact by the matrix determinant lemma and only log|P^{-1/2} A P^{-1/2}|, a
matrix close to the identity, is estimated. Written out here:

* partial pivoted Cholesky of a PSD matrix M (greedy: each step takes the
  largest remaining diagonal entry; Harbrecht, Peters & Schneider 2012);
* log|L L^T + s I_n| = (n - k) ln s + ln|s I_k + L^T L|;
* P^{-1} v = (v - L (s I_k + L^T L)^{-1} L^T v) / s (Woodbury);
* preconditioned CG (column-independent, x_0 = 0), whose alpha/beta give the
  Lanczos tridiagonal of P^{-1/2} A P^{-1/2} started at P^{-1/2} b, with the
  same formulas as plain CG; the quadrature weight is b^T P^{-1} b;
* probes z ~ N(0, P) as z = L g + sqrt(s) h with g, h standard normals, so that
  P^{-1/2} z ~ N(0, I): ln|A| = ln|P| + E[z^T P^{-1} z e_1^T ln(T) e_1].
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from . import krylov


def pivoted_cholesky(M: np.ndarray, k: int, pivots=None):
    """Rank-k partial pivoted Cholesky of the PSD matrix M: L (n x k) and the
    pivot order, with M ~ L L^T exact on the pivot rows and columns. The pivot
    of step j is the largest diagonal entry of M - L L^T (or pivots[j] if an
    order is given)."""
    n = M.shape[0]
    k = min(k, n)
    d = np.diag(M).astype(np.float64).copy()
    L = np.zeros((n, k))
    piv = []
    for j in range(k):
        p = int(np.argmax(d)) if pivots is None else int(pivots[j])
        piv.append(p)
        col = M[:, p] - L[:, :j] @ L[p, :j]
        L[:, j] = col / math.sqrt(col[p])
        d -= L[:, j] ** 2
        d[p] = 0.0
    return L, np.array(piv)


def logdet_lowrank_plus_shift(L: np.ndarray, s: float) -> float:
    """ln|L L^T + s I_n| by the matrix determinant lemma."""
    n, k = L.shape
    G = s * np.eye(k) + L.T @ L
    R = sla.cholesky(G, lower=True)
    return (n - k) * math.log(s) + 2.0 * float(np.sum(np.log(np.diag(R))))


def woodbury_solver(L: np.ndarray, s: float):
    """v -> (L L^T + s I)^{-1} v for blocks v (n x m)."""
    k = L.shape[1]
    R = sla.cholesky(s * np.eye(k) + L.T @ L, lower=True)

    def solve(V):
        V = np.asarray(V, dtype=np.float64)
        W = sla.cho_solve((R, True), L.T @ V)
        return (V - L @ W) / s
    return solve


def pcg(Amul, Minv, Bm, tol=1e-6, max_iter=1000, n_lanczos=30, fixed_iters=0):
    """Preconditioned CG on A X = B, one recurrence per column (x_0 = 0):
    z = M^{-1} r, alpha = r.z / p.Ap, beta = r'.z' / r.z, p = z' + beta p; a
    column stops once |r|/|b| <= tol. Returns X, iters, relres, the alpha/beta
    of the first n_lanczos steps, |b|^2 and rz0 = b^T M^{-1} b per column."""
    Bm = np.asarray(Bm, dtype=np.float64)
    if Bm.ndim == 1:
        Bm = Bm[:, None]
    n, m = Bm.shape
    X = np.zeros_like(Bm)
    R = Bm.copy()
    Z = Minv(R)
    P = Z.copy()
    rz = np.sum(R * Z, axis=0)
    rz0 = rz.copy()
    bb = np.sum(Bm * Bm, axis=0)
    rr = bb.copy()
    active = bb > 0
    iters = np.zeros(m, dtype=np.int64)
    alphas = np.zeros((m, n_lanczos))
    betas = np.zeros((m, n_lanczos))
    limit = fixed_iters if fixed_iters > 0 else max_iter
    for k in range(limit):
        if not active.any():
            break
        AP = Amul(P)
        pAp = np.sum(P * AP, axis=0)
        alpha = np.where(active, rz / np.where(active, pAp, 1.0), 0.0)
        X += alpha * P
        R -= alpha * AP
        Z = Minv(R)
        rz_new = np.sum(R * Z, axis=0)
        beta = np.where(active, rz_new / np.where(active, rz, 1.0), 0.0)
        if k < n_lanczos:
            alphas[active, k] = alpha[active]
            betas[active, k] = beta[active]
        iters[active] += 1
        P = np.where(active, Z + beta * P, P)
        rz = np.where(active, rz_new, rz)
        rr = np.where(active, np.sum(R * R, axis=0), rr)
        if fixed_iters <= 0:
            active &= np.sqrt(rr) > tol * np.sqrt(bb)
    relres = np.sqrt(rr / np.where(bb > 0, bb, 1.0))
    return dict(X=X, iters=iters, relres=relres, alphas=alphas, betas=betas, bnorm2=bb, rz0=rz0)


def probes_from(L: np.ndarray, s: float, g: np.ndarray, h: np.ndarray) -> np.ndarray:
    """Probe block z = L g + sqrt(s) h (g: k x m, h: n x m standard normals),
    distributed as N(0, L L^T + s I)."""
    return L @ g + math.sqrt(s) * h


def preconditioned_slq_logdet(alphas, betas, iters, rz0, n_lanczos, logdet_P):
    """ln|A| ~ ln|P| + (1/m) sum_j rz0_j e_1^T ln(T_j) e_1 (T_j from the PCG
    coefficients of probe j); standard error of the mean over the probes."""
    est, se, contrib = krylov.slq_logdet(alphas, betas, iters, rz0, n_lanczos)
    return logdet_P + est, se, contrib
