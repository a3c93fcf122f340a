"""Variationally optimised GP source: the single-sample ELBO, its gradient and
one Adam step (oracle, FP64).

Model. Sec. 3.3 eqs. "gp-gen2" and "decomposition" write a GP layer as
f = T y with y ~ N(0, alpha^2 I); Sec. 3.4 eq. "transmission" gives
    T_ij = A_j N(p_i - q_j, Zt_i + Sigma / 2),  A_j = |2 pi Sigma|^{1/4} / sqrt(rho(q_j)),
with Sigma = l^2 I (eq. "grbf-layers"), rho the k-th-neighbour density of the
inducing points q (footnote there, k = 20) and Zt_i the pixel shape of Sec. 3.2
(eq. "window-kernel"). Sec. 3.5 uses two kinds of layer: image-plane layers
whose inducing points are the traced points themselves (q = p, pixel shapes
kept) and one source-plane layer on a fixed regular grid (no pixel shapes).
Layers add (eq. "grbf-layers"): f = mu(p) + sum_k T_k y_k, with the Sersic mean
mu of the evidence path; the data are d ~ N(B f, sigma^2 I) with B the PSF and
local averaging.

Guide (Sec. 4.2, eq. "guide" and Table "gparams"): the seven free lens
parameters and the source-plane parameters share a partial multivariate
normal with scale matrix [[L_l, 0], [C, diag(s_sp)]]; each image-plane layer
has a diagonal normal (Sec. 3.7 eq. "gp-guide"); the amplitudes alpha_k are
point estimates. One reparametrised sample (Sec. 3.6 eq. "reparam") with
standard normals e_l (7), e_sp, e_k:
    theta = m_l + L_l e_l,  y_sp = m_sp + C e_l + s_sp e_sp,  y_k = m_k + s_k e_k,
and the ELBO sample (eq. "elbo")
    E = ln N(d | B f, sigma^2 I) + sum_k ln N(y_k | 0, alpha_k^2 I) + ln p(theta) - ln q(theta, y).

Lens prior (Table "lens-params"): uniform boxes on theta_E, q, phi, x0, y0 and
N(0, 0.05^2) on each shear component.

Readings (the paper leaves these to its software):
  * positive quantities (s, alpha and the diagonal of L_l) are optimised as
    their logarithms, the strictly lower part of L_l directly (the exponential
    transforms of positive and lower-Cholesky constraints);
  * Adam with torch's defaults minimises -E (Sec. 4.3);
  * samples are not mapped into the prior boxes: one outside a box has
    E = -inf (the paper's post-sampling transform and its Jacobian are left out);
  * the slope, the Sersic mean and the noise level are fixed;
  * the gradient follows everything the forward pass computes from theta: the
    traced points, their pixel shapes and the k-NN densities of image-plane
    inducing points (each point's k-th neighbour held at its current index).

Parameters are a dict of FP64 arrays:
  lens_mean (7), lens_raw (7, 7), log_amp (n_layers),
  sp_mean (G), sp_logs (G), sp_cross (G, 7), ip_mean [list of (N,)], ip_logs [list].
Noise draws: e_l (7), e_sp (G), e_ip [list of (N,)].
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import grid, lens as lensmod, psf, source, window

FREE = (0, 1, 2, 4, 5, 6, 7)  # theta_E, q, phi, x0, y0, gamma1, gamma2 (slope, index 3, fixed)
BOX = (0, 1, 2, 4, 5)  # components of the 8-vector with uniform priors
SHEAR = (6, 7)


@dataclasses.dataclass
class Model:
    n: int
    ss: int
    pix_scale: float
    slope: float
    src: tuple  # Sersic (peak, R_e, n, xs, ys), fixed
    sigma: float
    fwhm: float
    layers: tuple  # ((kind, lengthscale), ...), kind "ip" or "sp" (at most one "sp")
    gx: np.ndarray = None  # source-plane grid (G,)
    gy: np.ndarray = None
    prior_lo: tuple = (0.5, 0.1, 0.0, -0.2, -0.2)  # theta_E, q, phi, x0, y0
    prior_hi: tuple = (1.7, 1.0, 2.0 * math.pi, 0.2, 0.2)
    shear_sd: float = 0.05
    knn_k: int = 20

    @property
    def M(self):
        return self.n * self.ss

    @property
    def N(self):
        return self.M ** 2

    @property
    def G(self):
        return 0 if self.gx is None else self.gx.size

    def taps(self):
        return psf.psf_taps(self.fwhm, self.pix_scale / self.ss)

    def B(self, f):
        return psf.apply_B(f, self.n, self.ss, self.taps())

    def BT(self, x):
        return psf.apply_BT(x, self.n, self.ss, self.taps())


def scale_matrix(raw):
    """Lower-triangular L_l: strictly lower part of raw, exp of its diagonal."""
    raw = np.asarray(raw, dtype=np.float64)
    return np.tril(raw, -1) + np.diag(np.exp(np.diag(raw)))


def lens_sample(model: Model, params, e_l):
    L = scale_matrix(params["lens_raw"])
    tf = params["lens_mean"] + L @ e_l
    theta = np.empty(8)
    theta[list(FREE)] = tf
    theta[3] = model.slope
    return theta, L


def _gauss(dx, dy, cxx, cxy, cyy):
    return window.gauss2(dx, dy, cxx, cxy, cyy)


def _layer_setup(model: Model, kind, ell, px, py, Z):
    """Inducing points, weights A and target shapes of one layer."""
    if kind == "ip":
        qx, qy, Zt = px, py, Z
    else:
        qx, qy, Zt = model.gx, model.gy, np.zeros((px.size, 3))
    r, nn = window.knn_radius(qx, qy, model.knn_k)
    rho = model.knn_k / (math.pi * r * r)
    A = window.transmission_weights(rho, ell)
    return qx, qy, Zt, A, r, nn


def elbo(model: Model, params, eps, d, want_grad: bool = False, points=None):
    """Single-sample ELBO E (and, with want_grad, dE/d every parameter).

    Returns (E, pieces, grads) with pieces = dict(loglik, logprior_y,
    logprior_theta, neg_logq) and grads a dict shaped like params. `points`
    (px, py), if given, replaces the traced points of the sampled lens (the
    lens Jacobian is still that of the sampled lens): it lets a comparison
    use another implementation's rounded points."""
    nl = len(model.layers)
    theta, L = lens_sample(model, params, eps["e_l"])
    xi_x, xi_y = grid.fine_coords(model.n, model.ss, model.pix_scale)
    if points is None:
        px, py = lensmod.raytrace(xi_x, xi_y, theta)
    else:
        px, py = (np.asarray(v, dtype=np.float64) for v in points)
    a, b = window.pixel_axes(px, py, model.M)
    Z = window.shape_cov(a, b)
    mu = source.sersic(px, py, *model.src)
    f = mu.copy()
    amp = np.exp(params["log_amp"])
    layers = []
    ip_i = 0
    for k, (kind, ell) in enumerate(model.layers):
        qx, qy, Zt, A, r, nn = _layer_setup(model, kind, ell, px, py, Z)
        h = 0.5 * ell * ell
        cxx = Zt[:, 0][:, None] + h
        cxy = np.broadcast_to(Zt[:, 1][:, None], (px.size, qx.size))
        cyy = Zt[:, 2][:, None] + h
        dx = px[:, None] - qx[None, :]
        dy = py[:, None] - qy[None, :]
        Gm = _gauss(dx, dy, cxx, cxy, cyy)
        if kind == "ip":
            s = np.exp(params["ip_logs"][ip_i])
            e = eps["e_ip"][ip_i]
            y = params["ip_mean"][ip_i] + s * e
            ip_i += 1
        else:
            s = np.exp(params["sp_logs"])
            e = eps["e_sp"]
            y = params["sp_mean"] + params["sp_cross"] @ eps["e_l"] + s * e
        f += (Gm * A[None, :]) @ y
        layers.append(dict(kind=kind, ell=ell, h=h, qx=qx, qy=qy, Zt=Zt, A=A, r=r, nn=nn, Gm=Gm, dx=dx, dy=dy,
                           cxx=cxx, cxy=cxy, cyy=cyy, y=y, s=s, e=e, amp=amp[k]))
    resid = d - model.B(f)
    sig = model.sigma
    n_pix = resid.size
    loglik = -0.5 * float(resid @ resid) / sig ** 2 - n_pix * math.log(sig) - 0.5 * n_pix * math.log(2 * math.pi)
    logprior_y = 0.0
    n_tot = 7
    neg_logq = 0.5 * float(eps["e_l"] @ eps["e_l"]) + float(np.sum(np.diag(params["lens_raw"])))
    for ly in layers:
        nk = ly["y"].size
        logprior_y += (-0.5 * float(ly["y"] @ ly["y"]) / ly["amp"] ** 2 - nk * math.log(ly["amp"])
                       - 0.5 * nk * math.log(2 * math.pi))
        neg_logq += 0.5 * float(ly["e"] @ ly["e"]) + float(np.sum(np.log(ly["s"])))
        n_tot += nk
    neg_logq += 0.5 * n_tot * math.log(2 * math.pi)
    inside = all(model.prior_lo[i] <= theta[j] <= model.prior_hi[i] for i, j in enumerate(BOX))
    logprior_theta = -float(np.sum(np.log(np.subtract(model.prior_hi, model.prior_lo)))) if inside else -math.inf
    sd = model.shear_sd
    for j in SHEAR:
        logprior_theta += -0.5 * (theta[j] / sd) ** 2 - math.log(sd) - 0.5 * math.log(2 * math.pi)
    E = loglik + logprior_y + logprior_theta + neg_logq
    pieces = dict(loglik=loglik, logprior_y=logprior_y, logprior_theta=logprior_theta, neg_logq=neg_logq,
                  theta=theta, f=f, resid=resid)
    if not want_grad:
        return E, pieces, None

    # ---- gradient
    g_f = model.BT(resid) / sig ** 2
    g_p = g_f[:, None] * source.sersic_grad(px, py, *model.src)
    gZ = np.zeros((px.size, 3))  # symmetric matrix gradient (xx, xy, yy) of the target shapes
    grads = dict(ip_mean=[], ip_logs=[], log_amp=np.empty(nl))
    for k, ly in enumerate(layers):
        A, Gm, y = ly["A"], ly["Gm"], ly["y"]
        g_y = (Gm * A[None, :]).T @ g_f - y / ly["amp"] ** 2
        grads["log_amp"][k] = float(y @ y) / ly["amp"] ** 2 - y.size
        if ly["kind"] == "ip":
            grads["ip_mean"].append(g_y)
            grads["ip_logs"].append(ly["s"] * g_y * ly["e"] + 1.0)
        else:
            grads["sp_mean"] = g_y
            grads["sp_logs"] = ly["s"] * g_y * ly["e"] + 1.0
            grads["sp_cross"] = np.outer(g_y, eps["e_l"])
        # pair weights W_ij = g_i A_j y_j G_ij and u_ij = C_i^{-1} d_ij
        W = g_f[:, None] * Gm * (A * y)[None, :]
        det = ly["cxx"] * ly["cyy"] - ly["cxy"] ** 2
        ixx, ixy, iyy = ly["cyy"] / det, -ly["cxy"] / det, ly["cxx"] / det
        ux = ixx * ly["dx"] + ixy * ly["dy"]
        uy = ixy * ly["dx"] + iyy * ly["dy"]
        g_p[:, 0] -= np.sum(W * ux, axis=1)
        g_p[:, 1] -= np.sum(W * uy, axis=1)
        if ly["kind"] == "ip":
            # inducing points are the traced points: q_j = p_j
            g_p[:, 0] += np.sum(W * ux, axis=0)
            g_p[:, 1] += np.sum(W * uy, axis=0)
            # target shapes: dG/dC = G (C^{-1} d d^T C^{-1} - C^{-1}) / 2
            gZ[:, 0] += np.sum(0.5 * W * (ux * ux - ixx), axis=1)
            gZ[:, 1] += np.sum(0.5 * W * (ux * uy - ixy), axis=1)
            gZ[:, 2] += np.sum(0.5 * W * (uy * uy - iyy), axis=1)
            # weights: A_j is proportional to r_j, the distance to the k-th neighbour nn_j
            gA = y * (Gm.T @ g_f)
            coef = gA * A / ly["r"] ** 2
            vx = ly["qx"] - ly["qx"][ly["nn"]]
            vy = ly["qy"] - ly["qy"][ly["nn"]]
            g_p[:, 0] += coef * vx
            g_p[:, 1] += coef * vy
            np.add.at(g_p[:, 0], ly["nn"], -coef * vx)
            np.add.at(g_p[:, 1], ly["nn"], -coef * vy)
    # pixel shapes Z = (a a^T + b b^T) / (4 pi): dE/da = Gbar a / (2 pi)
    ga = np.stack([gZ[:, 0] * a[:, 0] + gZ[:, 1] * a[:, 1], gZ[:, 1] * a[:, 0] + gZ[:, 2] * a[:, 1]], 1) / (2 * math.pi)
    gb = np.stack([gZ[:, 0] * b[:, 0] + gZ[:, 1] * b[:, 1], gZ[:, 1] * b[:, 0] + gZ[:, 2] * b[:, 1]], 1) / (2 * math.pi)
    g_p += axes_backward(ga, gb, model.M)
    J = lensmod.raytrace_jacobian(xi_x, xi_y, theta, rel_step=1e-5)  # (N, 2, 8)
    g_theta = np.einsum("nc,nck->k", g_p, J)
    for j in SHEAR:
        g_theta[j] -= theta[j] / sd ** 2
    gt = g_theta[list(FREE)]
    grads["lens_mean"] = gt
    gr = np.tril(np.outer(gt, eps["e_l"]), -1)
    gr[np.diag_indices(7)] = gt * eps["e_l"] * np.diag(L) + 1.0
    grads["lens_raw"] = gr
    pieces["g_theta"] = g_theta
    pieces["g_p"] = g_p
    return E, pieces, grads


def axes_backward(ga, gb, M: int):
    """Adjoint of `window.pixel_axes`: given dE/da and dE/db per point ((N, 2)
    each), dE/dp per point."""
    out = np.zeros((M, M, 2))
    for G, ax in ((ga.reshape(M, M, 2), 1), (gb.reshape(M, M, 2), 0)):
        if M == 1:
            continue
        Gt = np.moveaxis(G, ax, 0)  # axis of differences first
        Ot = np.moveaxis(out, ax, 0)  # a view into out
        Ot[2:] += 0.5 * Gt[1:-1]
        Ot[:-2] -= 0.5 * Gt[1:-1]
        Ot[1] += Gt[0]
        Ot[0] -= Gt[0]
        Ot[-1] += Gt[-1]
        Ot[-2] -= Gt[-1]
    return out.reshape(-1, 2)


def expected_elbo_fixed_lens(model: Model, params, e_l, d):
    """E over the source-parameter noise of the ELBO sample with the lens noise
    fixed at e_l: the textbook Gaussian expectation (expected log-likelihood of a
    linear model minus the KL divergence of diagonal normals), used to check the
    sample's algebra."""
    theta, L = lens_sample(model, params, e_l)
    xi_x, xi_y = grid.fine_coords(model.n, model.ss, model.pix_scale)
    px, py = lensmod.raytrace(xi_x, xi_y, theta)
    a, b = window.pixel_axes(px, py, model.M)
    Z = window.shape_cov(a, b)
    fm = source.sersic(px, py, *model.src)
    sig = model.sigma
    amp = np.exp(params["log_amp"])
    var_term = 0.0
    kl = 0.0
    ip_i = 0
    for k, (kind, ell) in enumerate(model.layers):
        qx, qy, Zt, A, _, _ = _layer_setup(model, kind, ell, px, py, Z)
        T = window.transmission_matrix(px, py, Zt, qx, qy, ell, A)
        if kind == "ip":
            m = params["ip_mean"][ip_i]
            s = np.exp(params["ip_logs"][ip_i])
            ip_i += 1
        else:
            m = params["sp_mean"] + params["sp_cross"] @ e_l
            s = np.exp(params["sp_logs"])
        fm = fm + T @ m
        BT_ = model.B(T)  # (n_pix, n_k)
        var_term += float(np.sum(s * s * np.sum(BT_ * BT_, axis=0)))
        # KL(N(m, s^2) || N(0, amp^2)) per component
        kl += float(np.sum(np.log(amp[k] / s) + (s * s + m * m) / (2 * amp[k] ** 2) - 0.5))
    resid = d - model.B(fm)
    n_pix = resid.size
    ell_exp = (-0.5 * float(resid @ resid) / sig ** 2 - 0.5 * var_term / sig ** 2 - n_pix * math.log(sig)
               - 0.5 * n_pix * math.log(2 * math.pi))
    # lens part at the fixed e_l: ln p(theta) + 0.5 |e_l|^2 + ln|L_l| + (7/2) ln 2 pi
    inside = all(model.prior_lo[i] <= theta[j] <= model.prior_hi[i] for i, j in enumerate(BOX))
    lp = -float(np.sum(np.log(np.subtract(model.prior_hi, model.prior_lo)))) if inside else -math.inf
    for j in SHEAR:
        lp += -0.5 * (theta[j] / model.shear_sd) ** 2 - math.log(model.shear_sd) - 0.5 * math.log(2 * math.pi)
    lens_q = 0.5 * float(e_l @ e_l) + float(np.sum(np.log(np.diag(L)))) + 3.5 * math.log(2 * math.pi)
    return ell_exp - kl + lp + lens_q


def adam_step(params, grads, state, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015, torch's defaults) that minimises -E:
    the gradient of the loss is -grads. state holds the moment estimates
    m, v shaped like params (zeros at t = 1). Returns new params and state."""
    new_p, new_s = {}, {"m": {}, "v": {}}

    def upd(p, g, m, v):
        gl = -np.asarray(g, dtype=np.float64)
        m = beta1 * m + (1 - beta1) * gl
        v = beta2 * v + (1 - beta2) * gl * gl
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        return p - lr * mh / (np.sqrt(vh) + eps), m, v

    for key, p in params.items():
        if isinstance(p, list):
            outs = [upd(pi, gi, mi, vi) for pi, gi, mi, vi in zip(p, grads[key], state["m"][key], state["v"][key])]
            new_p[key] = [o[0] for o in outs]
            new_s["m"][key] = [o[1] for o in outs]
            new_s["v"][key] = [o[2] for o in outs]
        else:
            g = grads[key]
            if key == "lens_raw":  # only the lower triangle is a parameter
                g = np.tril(g)
            new_p[key], new_s["m"][key], new_s["v"][key] = upd(p, g, state["m"][key], state["v"][key])
    return new_p, new_s


def zeros_like(params):
    return {k: ([np.zeros_like(x) for x in v] if isinstance(v, list) else np.zeros_like(v)) for k, v in params.items()}


def adam_init(params):
    """Adam state before the first step: both moment estimates zero."""
    return {"m": zeros_like(params), "v": zeros_like(params)}
