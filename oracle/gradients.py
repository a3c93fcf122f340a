"""Gradients of the evidence and of the variational objective (oracle, FP64).

With u = A^{-1} r, r = d - B mu, A = B K B^T + sigma^2 I (reading of eq. "gp-mll"):

  d ln p / d t = u^T B (d mu/d t) + 1/2 u^T B (dK/d t) B^T u - 1/2 tr(A^{-1} B (dK/d t) B^T)
  d L_VI / d t = -2 u^T B (d mu/d t) - u^T B (dK/d t) B^T u  (+ 2 N alpha/(alpha^2+sigma^2) for t = alpha)

(App. D.1 loss, single layer). The kernel derivatives follow from eq. "grbf":
dK_ij/dp_i = -K_ij (p_i - p_j)/ell^2, dK/d ell = K |p_i - p_j|^2 / ell^3,
dK/d alpha = 2K/alpha. Positions depend on the 8 lens parameters through the
lens equation (Sec. 2.1, 2.2); the source offset enters only through mu.

Parameter vector order (12): theta_E, q, phi, slope, x0, y0, gamma1, gamma2,
xs, ys, ell, amp. Everything is dense; the position Jacobian comes from
`lens.raytrace_jacobian`. `fd_gradient` gives independent central differences
of the exact Cholesky evidence.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import evidence, kernel, lens as lensmod, source

PARAM_NAMES = ("theta_E", "q", "phi", "slope", "x0", "y0", "gamma1", "gamma2", "xs", "ys", "ell", "amp")


def pack(prob: evidence.Problem) -> np.ndarray:
    return np.array(list(prob.lens) + [prob.src[3], prob.src[4], prob.ell, prob.amp])


def unpack(prob: evidence.Problem, t) -> evidence.Problem:
    t = np.asarray(t, dtype=np.float64)
    src = (prob.src[0], prob.src[1], prob.src[2], t[8], t[9])
    return evidence.Problem(prob.n, prob.ss, prob.pix_scale, t[:8], src, t[10], t[11], prob.sigma, prob.fwhm,
                            prob.cx, prob.cy)


def analytic_gradient(prob: evidence.Problem, d: np.ndarray):
    """Dense analytic gradients of ln p and L_VI (both length 12) plus values."""
    xi_x, xi_y = prob.coords()
    px, py = lensmod.raytrace(xi_x, xi_y, prob.lens)
    N = px.size
    mu = prob.mean(px, py)
    r = d - prob.B(mu)
    A = evidence.assemble_A(prob, px, py)
    ev = evidence.exact_evidence(A, r)
    u, L = ev["u"], ev["L"]
    w = prob.BT(u)  # B^T u on the fine grid
    Bd = prob.B(np.eye(N))  # dense B (n_pix x N)
    Ainv_B = sla.cho_solve((L, True), Bd, check_finite=False)
    BtAinvB = Bd.T @ Ainv_B  # B^T A^{-1} B (N x N)

    K = kernel.rbf_matrix(px, py, prob.ell, prob.amp)
    dx = px[:, None] - px[None, :]
    dy = py[:, None] - py[None, :]
    d2 = dx * dx + dy * dy
    ell, amp = prob.ell, prob.amp

    def kernel_part(Mw):
        """Sum_ij Mw_ij dK_ij/dt for positions (N,2), ell, amp; Mw symmetric."""
        MK = Mw * K
        gpos = np.stack([-(2.0 / ell ** 2) * np.sum(MK * dx, axis=1),
                         -(2.0 / ell ** 2) * np.sum(MK * dy, axis=1)], axis=-1)
        g_ell = float(np.sum(MK * d2)) / ell ** 3
        g_amp = 2.0 * float(np.sum(MK)) / amp
        return gpos, g_ell, g_amp

    gmu = source.sersic_grad(px, py, *prob.src)  # d mu_i / d p_i
    J = lensmod.raytrace_jacobian(xi_x, xi_y, prob.lens)  # (N, 2, 8)

    def assemble(gpos_K, g_ell, g_amp, mean_weight):
        gpos = gpos_K + mean_weight[:, None] * gmu
        g = np.zeros(12)
        g[:8] = np.einsum("ia,iak->k", gpos, J)
        g[8:10] = -np.sum(mean_weight[:, None] * gmu, axis=0)
        g[10], g[11] = g_ell, g_amp
        return g

    M_lnp = 0.5 * np.outer(w, w) - 0.5 * BtAinvB
    gl = assemble(*kernel_part(M_lnp), w)
    M_vi = -np.outer(w, w)
    gv = assemble(*kernel_part(M_vi), -2.0 * w)
    gv[11] += 2.0 * N * amp / (amp * amp + prob.sigma ** 2)
    vi = evidence.vi_objective(ev["quad"], N, amp, prob.sigma)
    return dict(lnp=ev["lnp"], vi=vi, grad_lnp=gl, grad_vi=gv, quad=ev["quad"], logdet=ev["logdet"])


def values(prob: evidence.Problem, d: np.ndarray):
    """(ln p, L_VI) from the exact Cholesky evidence."""
    px, py = prob.points()
    r = d - prob.B(prob.mean(px, py))
    ev = evidence.exact_evidence(evidence.assemble_A(prob, px, py), r)
    return ev["lnp"], evidence.vi_objective(ev["quad"], px.size, prob.amp, prob.sigma)


def fd_gradient(prob: evidence.Problem, d: np.ndarray, h: float = 1e-4):
    """Central differences (absolute step h in natural units) of ln p and L_VI."""
    t0 = pack(prob)
    gl, gv = np.zeros(12), np.zeros(12)
    for k in range(12):
        tp, tm = t0.copy(), t0.copy()
        tp[k] += h
        tm[k] -= h
        lp, vp = values(unpack(prob, tp), d)
        lm, vm = values(unpack(prob, tm), d)
        gl[k] = (lp - lm) / (2 * h)
        gv[k] = (vp - vm) / (2 * h)
    return gl, gv
