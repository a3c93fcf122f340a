"""Conjugate gradients, Lanczos and stochastic Lanczos quadrature (oracle, FP64).

The paper discusses (Sec. 3.3) evaluating eq. "gp-mll" with the conjugate
gradient method and a stochastic log-determinant, as in GPyTorch, and cites
Numerical Recipes Sec. 10.6 for CG. The algorithms written out here are the
textbook ones:

* CG (Hestenes-Stiefel), one independent recurrence per right-hand-side column,
  x_0 = 0; a column stops once |r_k| / |b| <= tol (or after a fixed count).
* The Lanczos tridiagonal that CG implies (Saad, Iterative Methods, Sec. 6.7):
  T_kk = 1/alpha_k + beta_{k-1}/alpha_{k-1},  T_{k,k+1} = sqrt(beta_k)/alpha_k.
* Explicit Lanczos with full re-orthogonalisation, for cross-checks.
* Lanczos quadrature: z^T f(A) z ~= |z|^2 sum_i tau_i^2 f(theta_i), theta the
  Ritz values and tau the first components of T's eigenvectors (Golub & Meurant);
  the log-determinant is tr ln A ~= (1/m) sum_j z_j^T ln(A) z_j over Hutchinson
  probes with E[z z^T] = I (Ubaru, Chen & Saad 2017).
"""
from __future__ import annotations

import math

import numpy as np


def cg(Amul, Bm, tol=1e-6, max_iter=1000, n_lanczos=30, fixed_iters=0, vec_dtype=np.float64):
    """Column-independent CG on A X = B. Returns dict with X, iters, relres,
    alpha/beta histories (first n_lanczos steps per column) and |b|^2.

    vec_dtype = np.float32 keeps X, R, P and A P in single precision, the
    arithmetic of the paper's GPU fits (Sec. 4.3 compares its posterior widths
    with the machine precision of single-precision floats), while every dot
    product and the alpha/beta scalars stay FP64;
    each vector update is rounded to vec_dtype once. Amul then receives and
    returns vec_dtype blocks."""
    vt = np.dtype(vec_dtype)
    Bm = np.asarray(Bm, dtype=np.float64)
    if Bm.ndim == 1:
        Bm = Bm[:, None]
    n, m = Bm.shape
    if vt != np.float64:
        return _cg_lowprec(Amul, Bm.astype(vt), tol, max_iter, n_lanczos, fixed_iters, vt)
    X = np.zeros_like(Bm)
    R = Bm.copy()
    P = R.copy()
    rr = np.sum(R * R, axis=0)
    bb = rr.copy()
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
        alpha = np.where(active, rr / np.where(active, pAp, 1.0), 0.0)
        X += alpha * P
        R -= alpha * AP
        rr_new = np.sum(R * R, axis=0)
        beta = np.where(active, rr_new / np.where(active, rr, 1.0), 0.0)
        if k < n_lanczos:
            alphas[active, k] = alpha[active]
            betas[active, k] = beta[active]
        iters[active] += 1
        P = np.where(active, R + beta * P, P)
        rr = np.where(active, rr_new, rr)
        if fixed_iters <= 0:
            active &= np.sqrt(rr) > tol * np.sqrt(bb)
    relres = np.sqrt(rr / np.where(bb > 0, bb, 1.0))
    return dict(X=X, iters=iters, relres=relres, alphas=alphas, betas=betas, bnorm2=bb)


def _cg_lowprec(Amul, Bm, tol, max_iter, n_lanczos, fixed_iters, vt):
    """The recurrences of `cg` with vectors in vt and FP64 scalars."""
    n, m = Bm.shape
    X = np.zeros_like(Bm)
    R = Bm.copy()
    P = R.copy()
    rr = np.sum(R.astype(np.float64) ** 2, axis=0)
    bb = rr.copy()
    active = bb > 0
    iters = np.zeros(m, dtype=np.int64)
    alphas = np.zeros((m, n_lanczos))
    betas = np.zeros((m, n_lanczos))
    limit = fixed_iters if fixed_iters > 0 else max_iter
    for k in range(limit):
        if not active.any():
            break
        AP = np.asarray(Amul(P), dtype=vt)
        pAp = np.sum(P.astype(np.float64) * AP.astype(np.float64), axis=0)
        alpha = np.where(active, rr / np.where(active, pAp, 1.0), 0.0)
        X = (X + alpha.astype(vt) * P).astype(vt)
        R = (R - alpha.astype(vt) * AP).astype(vt)
        rr_new = np.sum(R.astype(np.float64) ** 2, axis=0)
        beta = np.where(active, rr_new / np.where(active, rr, 1.0), 0.0)
        if k < n_lanczos:
            alphas[active, k] = alpha[active]
            betas[active, k] = beta[active]
        iters[active] += 1
        P = np.where(active, (R + beta.astype(vt) * P).astype(vt), P)
        rr = np.where(active, rr_new, rr)
        if fixed_iters <= 0:
            active &= np.sqrt(rr) > tol * np.sqrt(bb)
    relres = np.sqrt(rr / np.where(bb > 0, bb, 1.0))
    return dict(X=X.astype(np.float64), iters=iters, relres=relres, alphas=alphas, betas=betas, bnorm2=bb)


def cg_tridiagonal(alphas, betas, k):
    """Diagonal and off-diagonal of the k x k Lanczos matrix implied by CG."""
    a = np.asarray(alphas[:k], dtype=np.float64)
    b = np.asarray(betas[:k], dtype=np.float64)
    diag = 1.0 / a
    diag[1:] += b[:k - 1] / a[:k - 1]
    off = np.sqrt(b[:k - 1]) / a[:k - 1]
    return diag, off


def lanczos(Amul, z, m):
    """Explicit Lanczos with full re-orthogonalisation; returns (diag, off)."""
    n = z.size
    Q = np.zeros((n, m))
    diag, off = np.zeros(m), np.zeros(max(m - 1, 0))
    q = z / np.linalg.norm(z)
    beta = 0.0
    q_prev = np.zeros(n)
    k_used = m
    for k in range(m):
        Q[:, k] = q
        w = Amul(q[:, None])[:, 0] - beta * q_prev
        a = q @ w
        w = w - a * q
        w = w - Q[:, :k + 1] @ (Q[:, :k + 1].T @ w)  # full re-orthogonalisation
        diag[k] = a
        if k + 1 < m:
            beta = np.linalg.norm(w)
            if beta == 0.0:
                k_used = k + 1
                break
            off[k] = beta
            q_prev, q = q, w / beta
    return diag[:k_used], off[:k_used - 1]


def quadrature(diag, off, f=np.log):
    """sum_i tau_i^2 f(theta_i) for the tridiagonal (diag, off)."""
    if diag.size == 1:
        return float(f(diag[0]))
    T = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
    theta, V = np.linalg.eigh(T)  # dense symmetric eigensolver on the small T
    return float(np.sum(V[0] ** 2 * f(theta)))


def slq_logdet(alphas, betas, iters, bnorm2, n_lanczos, scale=None):
    """SLQ estimate of ln|A| from per-probe CG coefficients.

    Probe j contributes |z_j|^2 * quadrature(T_j), T_j of size min(iters_j, n_lanczos).
    The estimate is scale * sum_j (contribution j), scale = 1/m by default; the
    standard error is the sample standard deviation of the m contributions over sqrt(m)."""
    m = len(iters)
    contrib = np.empty(m)
    for j in range(m):
        k = int(min(iters[j], n_lanczos))
        d, o = cg_tridiagonal(alphas[j], betas[j], k)
        contrib[j] = bnorm2[j] * quadrature(d, o)
    if scale is None:
        scale = 1.0 / m
    est = scale * contrib.sum()
    stderr = scale * m * contrib.std(ddof=1) / math.sqrt(m) if m > 1 else float("nan")
    return float(est), float(stderr), contrib
