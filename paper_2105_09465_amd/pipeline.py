"""One reconstruction through the library: ray tracing, mean, residual, CG on
the solve column and the probes, SLQ log-determinant, evidence scalars,
posterior mean and predicted image.

Each step is one library call on torch's current stream; torch only provides
the buffers (and copies d and the probes into the right-hand-side block).
"""
from __future__ import annotations

import dataclasses
import math

import torch

from . import ops
from .params import Problem


@dataclasses.dataclass
class Reconstruction:
    px: torch.Tensor
    py: torch.Tensor
    mu: torch.Tensor
    rhs: torch.Tensor  # (1+m, n_pix): residual r = d - B mu, then the probes
    X: torch.Tensor  # A^{-1} rhs
    cg: dict
    logdet: torch.Tensor
    stderr: torch.Tensor
    contrib: torch.Tensor
    scalars: torch.Tensor  # quad, ln p, L_VI (float64, device)
    fhat: torch.Tensor | None
    image: torch.Tensor | None
    precond: dict | None = None  # the preconditioner of reconstruct_preconditioned

    def host(self):
        """Copy the scalar results to the host (one synchronisation)."""
        s = self.scalars.double().cpu().tolist()
        tr = self.cg.get("true_relres")
        return dict(quad=s[0], lnp=s[1], vi=s[2], logdet=float(self.logdet.item()), stderr=float(self.stderr.item()),
                    iters=self.cg["iters"].cpu().tolist(), relres=self.cg["relres"].cpu().tolist(),
                    true_relres=tr.cpu().tolist() if tr is not None else None,
                    status=self.cg["status"].cpu().tolist())


def reconstruct(problem: Problem, d: torch.Tensor, probes: torch.Tensor, prec="fp32", tol=1e-6, max_iter=1000,
                fixed_iters=0, n_lanczos=30, logdet_scale=None, want_image=True, check_every=8, ws=None):
    """Evidence and posterior mean of one image.

    d: observed image (n_pix,) float32 on the GPU; probes: (m, n_pix) float32
    (Rademacher for SLQ, or unit vectors with logdet_scale=1 for the exact trace)."""
    g = problem.grid
    dev = d.device
    pts = ops.lens_raytrace(g, problem.lens, device=dev)
    px, py = pts[0], pts[1]
    mu = ops.sersic_eval(problem.source, px, py)
    m = probes.shape[0]
    rhs = torch.empty(1 + m, g.n_pix, dtype=torch.float32, device=dev)
    rhs[0].copy_(d)
    if m:
        rhs[1:].copy_(probes)
    ops.psf_conv(g, problem.psf, mu, adjoint=False, out=rhs[0], alpha=-1.0, beta=1.0)  # r = d - B mu
    cg = ops.cg_solve(problem, px, py, rhs, tol=tol, max_iter=max_iter, fixed_iters=fixed_iters,
                      n_lanczos=n_lanczos, prec=prec, check_every=check_every, ws=ws)
    if m and cg["n_lanczos"] > 0:
        scale = (1.0 / m) if logdet_scale is None else logdet_scale
        logdet, stderr, contrib = ops.lanczos_logdet(cg["ab"][1:], cg["iters"][1:], cg["bnorm2"][1:], scale)
    else:
        logdet = torch.full((1,), math.nan, dtype=torch.float64, device=dev)
        stderr, contrib = logdet.clone(), torch.empty(0, dtype=torch.float64, device=dev)
    u = cg["X"][0]
    scalars = ops.evidence_scalars(g.n_pix, g.N, rhs[0], u, logdet, problem.kernel.amplitude, problem.noise_sigma)
    fhat = image = None
    if want_image:
        w = ops.psf_conv(g, problem.psf, u, adjoint=True)  # B^T u
        fhat = mu.clone()
        ops.kernel_mvm(problem.kernel, px, py, w, prec="fp32", out=fhat, beta=1.0, grid=g)  # mu + K B^T u
        image = ops.psf_conv(g, problem.psf, fhat, adjoint=False)
    return Reconstruction(px, py, mu, rhs, cg["X"], cg, logdet, stderr, contrib, scalars, fhat, image)


def reconstruct_preconditioned(problem: Problem, d: torch.Tensor, g: torch.Tensor, h: torch.Tensor, rank=4096,
                               prec="f16x3", tol=1e-6, max_iter=200, n_lanczos=200, want_image=True,
                               check_every=2, ws=None):
    """Evidence and posterior mean of one image with the partial pivoted
    Cholesky preconditioner of rank `rank` (a multiple of 64): ln|A| = ln|P| +
    the SLQ estimate of ln|P^{-1/2} A P^{-1/2}| from preconditioned CG on probes
    z = L g + sigma h ~ N(0, P). g: (m, rank) float64 and h: (m, n_pix) float32
    standard normals on the GPU."""
    gr = problem.grid
    dev = d.device
    pts = ops.lens_raytrace(gr, problem.lens, device=dev)
    px, py = pts[0], pts[1]
    mu = ops.sersic_eval(problem.source, px, py)
    pc = ops.pchol(problem, px, py, rank, prec=prec)
    m = g.shape[0]
    rhs = torch.empty(1 + m, gr.n_pix, dtype=torch.float32, device=dev)
    rhs[0].copy_(d)
    if m:
        rhs[1:].copy_(ops.pchol_probes(pc, problem.noise_sigma, g, h))
    ops.psf_conv(gr, problem.psf, mu, adjoint=False, out=rhs[0], alpha=-1.0, beta=1.0)  # r = d - B mu
    cg = ops.pcg_solve(problem, px, py, pc, rhs, tol=tol, max_iter=max_iter, n_lanczos=n_lanczos, prec=prec,
                       check_every=check_every, ws=ws)
    if m and cg["n_lanczos"] > 0:
        logdet, stderr, contrib = ops.lanczos_logdet(cg["ab"][1:], cg["iters"][1:], cg["rz0"][1:], 1.0 / m,
                                                     offset=pc["logdet_P"])
    else:
        logdet = torch.full((1,), math.nan, dtype=torch.float64, device=dev)
        stderr, contrib = logdet.clone(), torch.empty(0, dtype=torch.float64, device=dev)
    u = cg["X"][0]
    scalars = ops.evidence_scalars(gr.n_pix, gr.N, rhs[0], u, logdet, problem.kernel.amplitude, problem.noise_sigma)
    fhat = image = None
    if want_image:
        w = ops.psf_conv(gr, problem.psf, u, adjoint=True)
        fhat = mu.clone()
        ops.kernel_mvm(problem.kernel, px, py, w, prec="fp32", out=fhat, beta=1.0, grid=gr)
        image = ops.psf_conv(gr, problem.psf, fhat, adjoint=False)
    return Reconstruction(px, py, mu, rhs, cg["X"], cg, logdet, stderr, contrib, scalars, fhat, image, pc)


@dataclasses.dataclass
class Posterior:
    mean: torch.Tensor  # (G,) float32
    var: torch.Tensor  # (G,) float64
    W: torch.Tensor  # (G, n_pix): B K(p, x_g)
    X: torch.Tensor  # (G, n_pix): A^{-1} W
    cg: dict


def posterior_at(problem: Problem, rec: Reconstruction, qx: torch.Tensor, qy: torch.Tensor, tol=1e-6,
                 max_iter=None, prec=None, check_every=2, ws=None):
    """Exact GP posterior mean and pointwise variance (Sec. 3.7, eqs.
    "gp-exact-mean" and "gp-exact-var") at source-plane points q (float32 on
    the GPU), from a finished reconstruction:
        mean(x) = mu(x) + K(x, p) B^T u,   var(x) = alpha^2 - w_x^T A^{-1} w_x,
    w_x = B K(p, x). The columns w_x are solved together, by preconditioned CG
    with the reconstruction's preconditioner when it has one, else by CG."""
    if problem.kernel.kind != 0:
        raise ValueError("posterior_at supports the RBF kernel (kind 0)")
    gr = problem.grid
    ell, amp = problem.kernel.lengthscale, problem.kernel.amplitude
    base, norm = ell * ell, amp * amp * ell * ell
    w = ops.psf_conv(gr, problem.psf, rec.X[0], adjoint=True)  # B^T u
    mean = ops.sersic_eval(problem.source, qx, qy)
    ops.gauss_product(base, norm, qx, qy, rec.px, rec.py, w, out=mean, beta=1.0)
    Kpq = ops.gauss_matrix(base, norm, rec.px, rec.py, qx, qy)  # (G, N): row g = K(p, x_g)
    W = ops.psf_conv(gr, problem.psf, Kpq, adjoint=False)  # (G, n_pix)
    del Kpq
    if rec.precond is not None:
        cg = ops.pcg_solve(problem, rec.px, rec.py, rec.precond, W, tol=tol, max_iter=max_iter or 200, n_lanczos=0,
                           prec=prec or "f16x3", check_every=check_every, ws=ws)
    else:
        cg = ops.cg_solve(problem, rec.px, rec.py, W, tol=tol, max_iter=max_iter or 1000, n_lanczos=0,
                          prec=prec or "fp32", check_every=max(check_every, 1), ws=ws)
    var = ops.posterior_variance(W, cg["X"], amp * amp)
    return Posterior(mean, var, W, cg["X"], cg)
