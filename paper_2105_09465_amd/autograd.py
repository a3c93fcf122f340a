"""torch.autograd.Function wrappers whose forward and backward are library calls.

Gradients of the evidence follow from the reading -2 ln p = r^T A^{-1} r + ln|2 pi A|
of eq. "gp-mll" (Sec. 3.1), r = d - B mu, A = B K B^T + sigma^2 I, u = A^{-1} r:

  d ln p/dt = u^T B dmu/dt + 1/2 u^T B dK/dt B^T u - 1/2 tr(A^{-1} B dK/dt B^T)

with the trace estimated from the CG solves of the probe columns,
tr(A^{-1} B dK B^T) ~ (1/m) sum_j (B^T A^{-1} z_j)^T dK (B^T z_j) (or exactly, with
all unit probes), and of the App. D.1 loss L_VI = quad + N ln(alpha^2 + sigma^2):

  dL_VI/dt = -2 u^T B dmu/dt - u^T B dK/dt B^T u  (+ 2 N alpha/(alpha^2 + sigma^2) for alpha).

The kernel terms come from the kernel-product adjoint (tiles recomputed), the
mean term from the Sersic adjoint, and both are pulled back to the lens
parameters through the ray-tracing adjoint. Parameter order (12): theta_E, q,
phi, slope, x0, y0, gamma1, gamma2, xs, ys, lengthscale, amplitude.
"""
from __future__ import annotations

import dataclasses

import torch

from . import ops
from .params import Kernel, Lens, Problem, Sersic
from .pipeline import Reconstruction, reconstruct

PARAM_NAMES = ("theta_E", "q", "phi", "slope", "x0", "y0", "gamma1", "gamma2", "xs", "ys", "lengthscale",
               "amplitude")


def problem_with(problem: Problem, theta) -> Problem:
    t = [float(v) for v in theta]
    src = dataclasses.replace(problem.source, xs=t[8], ys=t[9])
    return problem.replace(lens=Lens(*t[:8]), source=src, kernel=Kernel(t[10], t[11]))


def theta_of(problem: Problem):
    return list(problem.lens.as_tuple()) + [problem.source.xs, problem.source.ys, problem.kernel.lengthscale,
                                             problem.kernel.amplitude]


def evidence_gradients(problem: Problem, rec: Reconstruction, probe_scale=None, want=("lnp", "vi")):
    """Gradients (float64 tensors of length 12 on the device) of ln p and L_VI for
    a finished reconstruction. probe_scale multiplies the trace estimate
    (default 1/m; 1 for all unit probes)."""
    g = problem.grid
    dev = rec.X.device
    u = rec.X[0]
    w = ops.psf_conv(g, problem.psf, u, adjoint=True)  # B^T u
    m = rec.X.shape[0] - 1
    out = {}
    amp_grads = None
    if "lnp" in want:
        scale = (1.0 / m if m else 0.0) if probe_scale is None else probe_scale
        gpx = torch.zeros(g.N, dtype=torch.float32, device=dev)
        gpy = torch.zeros_like(gpx)
        if m:
            a = ops.psf_conv(g, problem.psf, rec.X[1:], adjoint=True)  # B^T A^{-1} z_j
            b = ops.psf_conv(g, problem.psf, rec.rhs[1:], adjoint=True)  # B^T z_j
            A_ = torch.cat([w.unsqueeze(0), a], 0)
            B_ = torch.cat([w.unsqueeze(0), b], 0)
        else:
            A_ = B_ = w.unsqueeze(0)
        weights = [0.5] + [-0.5 * scale] * m
        _, _, ghyp = ops.kernel_mvm_backward(problem.kernel, rec.px, rec.py, A_, B_, weights, gpx, gpy)
        gsrc = ops.sersic_backward(problem.source, rec.px, rec.py, w, gpx, gpy)
        glens = ops.lens_raytrace_backward(g, problem.lens, gpx, gpy)
        # the amplitude derivatives come from the exact identity the library
        # evaluates with FP64 dot products (the two large kernel sums of the
        # adjoint cancel to ~1e-3); the adjoint's own amplitude entry is replaced
        ga = ops.evidence_amplitude_grad(g.N, u, rec.rhs[1:] if m else None, rec.X[1:] if m else None,
                                         rec.scalars[0:1], scale, problem.kernel.amplitude, problem.noise_sigma)
        out["lnp"] = torch.cat([glens, gsrc, ghyp[0:1], ga[0:1]])
        amp_grads = ga
    if "vi" in want:
        gpx = torch.zeros(g.N, dtype=torch.float32, device=dev)
        gpy = torch.zeros_like(gpx)
        W = w.unsqueeze(0)
        _, _, ghyp = ops.kernel_mvm_backward(problem.kernel, rec.px, rec.py, W, W, [-1.0], gpx, gpy)
        w2 = ops.psf_conv(g, problem.psf, u, adjoint=True, alpha=-2.0)  # -2 B^T u
        gsrc = ops.sersic_backward(problem.source, rec.px, rec.py, w2, gpx, gpy)
        glens = ops.lens_raytrace_backward(g, problem.lens, gpx, gpy)
        if amp_grads is None:
            amp_grads = ops.evidence_amplitude_grad(g.N, u, None, None, rec.scalars[0:1], 0.0,
                                                    problem.kernel.amplitude, problem.noise_sigma)
        out["vi"] = torch.cat([glens, gsrc, ghyp[0:1], amp_grads[1:2]])
    return out


class GPEvidence(torch.autograd.Function):
    """theta (12,) -> (ln p, L_VI); backward through the library adjoints."""

    @staticmethod
    def forward(ctx, theta, problem: Problem, d, probes, opts: dict):
        prob = problem_with(problem, theta.detach().cpu().tolist())
        rec = reconstruct(prob, d, probes, want_image=False, **opts)
        ctx.prob, ctx.rec = prob, rec
        ctx.probe_scale = opts.get("logdet_scale")
        return rec.scalars[1:3].clone().to(theta.dtype)

    @staticmethod
    def backward(ctx, gout):
        grads = evidence_gradients(ctx.prob, ctx.rec, probe_scale=ctx.probe_scale)
        gl, gv = grads["lnp"].to(gout.device, gout.dtype), grads["vi"].to(gout.device, gout.dtype)
        return gout[0] * gl + gout[1] * gv, None, None, None, None


def evidence(theta, problem: Problem, d, probes, **opts):
    """Differentiable (ln p, L_VI) of the image d at parameters theta."""
    return GPEvidence.apply(theta, problem, d, probes, opts)


class RayTrace(torch.autograd.Function):
    """lens (8,) -> source-plane points (2, N) on the problem's grid."""

    @staticmethod
    def forward(ctx, lens_params, grid):
        lens = Lens(*[float(v) for v in lens_params.detach().cpu().tolist()])
        ctx.grid, ctx.lens, ctx.dtype = grid, lens, lens_params.dtype
        return ops.lens_raytrace(grid, lens)

    @staticmethod
    def backward(ctx, gp):
        gp = gp.contiguous().float()
        g = ops.lens_raytrace_backward(ctx.grid, ctx.lens, gp[0], gp[1])
        return g.to(ctx.dtype), None


class KernelMVM(torch.autograd.Function):
    """(px, py, V (ncols, N), hyper (2,) = (lengthscale, amplitude)) -> K V."""

    @staticmethod
    def forward(ctx, px, py, V, hyper, prec="fp32"):
        kern = Kernel(*[float(v) for v in hyper.detach().cpu().tolist()])
        ctx.save_for_backward(px, py, V)
        ctx.kern, ctx.prec, ctx.hdtype = kern, prec, hyper.dtype
        return ops.kernel_mvm(kern, px.contiguous(), py.contiguous(), V.contiguous(), prec=prec)

    @staticmethod
    def backward(ctx, gY):
        px, py, V = ctx.saved_tensors
        gY = gY.contiguous()
        gV = ops.kernel_mvm(ctx.kern, px, py, gY, prec=ctx.prec)  # K symmetric
        gpx = torch.zeros_like(px)
        gpy = torch.zeros_like(py)
        _, _, ghyp = ops.kernel_mvm_backward(ctx.kern, px, py, gY, V.contiguous(), [1.0] * V.shape[0], gpx, gpy)
        return gpx, gpy, gV, ghyp.to(ctx.hdtype), None


class PSFConv(torch.autograd.Function):
    """B x (adjoint=False) or B^T x (adjoint=True) on (ncols, rows) blocks."""

    @staticmethod
    def forward(ctx, x, grid, psf, adjoint=False):
        ctx.grid, ctx.psf, ctx.adjoint = grid, psf, adjoint
        return ops.psf_conv(grid, psf, x.contiguous(), adjoint=adjoint)

    @staticmethod
    def backward(ctx, g):
        return ops.psf_conv(ctx.grid, ctx.psf, g.contiguous(), adjoint=not ctx.adjoint), None, None, None
