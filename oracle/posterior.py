"""Exact GP posterior at arbitrary source-plane points (oracle, FP64).

Sec. 3.7, eqs. "gp-exact-mean" and "gp-exact-var": given the data, the fluxes
are normal with mean K (K+S)^{-1} d and covariance K - K (K+S)^{-1} K. With the
observation operator B (PSF and local averaging) and the mean function mu of
Sec. 3.1, at points x that need not be the fitted points p:
    mean(x) = mu(x) + K(x, p) B^T A^{-1} r,
    var(x)  = k(x, x) - K(x, p) B^T A^{-1} B K(p, x),
with A = B K(p, p) B^T + sigma^2 I and r = d - B mu(p). Sec. 3.5 evaluates
reconstructions on a regular source-plane grid; only the diagonal of the
covariance (the pointwise variance) is formed here.

Dense: K(x, p) is formed explicitly and A^{-1} is applied through the Cholesky
factor of `evidence.solve_problem`: var = k(x, x) - |L^{-1} B K(p, x)|^2 per
column.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import kernel


def posterior_at(prob, sol, qx, qy):
    """Posterior mean and variance at the points (qx, qy).

    prob: evidence.Problem; sol: evidence.solve_problem(prob, d) (uses px, py,
    u = A^{-1} r and the Cholesky factor L of A). Returns dict(mean, var)."""
    qx = np.asarray(qx, dtype=np.float64)
    qy = np.asarray(qy, dtype=np.float64)
    px, py = sol["px"], sol["py"]
    Kqp = kernel.rbf_matrix(qx, qy, prob.ell, prob.amp, px, py)  # (G, N)
    mean = prob.mean(qx, qy) + Kqp @ prob.BT(sol["u"])
    W = prob.B(Kqp.T)  # B K(p, x): (n_pix, G)
    V = sla.solve_triangular(sol["L"], W, lower=True, check_finite=False)
    var = prob.amp ** 2 - np.sum(V * V, axis=0)
    return dict(mean=mean, var=var, W=W)
