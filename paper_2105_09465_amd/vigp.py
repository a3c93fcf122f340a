"""Variational GP source fitting through the library (Sec. 3.3-3.7, 4.2, 4.3).

`VigpModel` describes the layers (image-plane layers on the traced points, at
most one source-plane layer on a grid) and the lens prior; `Vigp` holds the
guide's parameter blocks, their gradients and Adam's moments on the device in
the layout the library documents, and runs one step as two library calls: the
ELBO sample with its gradient, then the Adam update. The noise of each sample
is drawn by the caller and passed in.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math

import torch

from . import _lib
from .ops import _ptr, _stream
from .params import Problem

KINDS = {"ip": 0, "sp": 1}


@dataclasses.dataclass(frozen=True)
class VigpModel:
    layers: tuple  # ((kind "ip" | "sp", lengthscale), ...)
    slope: float
    prior_lo: tuple = (0.5, 0.1, 0.0, -0.2, -0.2)  # theta_E, q, phi, x0, y0
    prior_hi: tuple = (1.7, 1.0, 2.0 * math.pi, 0.2, 0.2)
    shear_sd: float = 0.05
    knn_k: int = 20

    def c(self):
        m = _lib.gpl_vigp_model()
        m.n_layers = len(self.layers)
        for k, (kind, ell) in enumerate(self.layers):
            m.kind[k] = KINDS[kind]
            m.lengthscale[k] = float(ell)
        m.knn_k = int(self.knn_k)
        m.slope = float(self.slope)
        for i in range(5):
            m.prior_lo[i] = float(self.prior_lo[i])
            m.prior_hi[i] = float(self.prior_hi[i])
        m.shear_sd = float(self.shear_sd)
        return m


class Vigp:
    """Guide parameters, gradients and Adam state for one image."""

    def __init__(self, model: VigpModel, problem: Problem, d: torch.Tensor, gx=None, gy=None):
        self.model, self.problem = model, problem
        self.d = d
        self.gx, self.gy = gx, gy
        self.G = 0 if gx is None else gx.numel()
        self._m, self._g = model.c(), problem.grid.c()
        n64, n32, ne32 = C.c_size_t(), C.c_size_t(), C.c_size_t()
        _lib.call("gpl_vigp_sizes", C.byref(self._m), C.byref(self._g), self.G, C.byref(n64), C.byref(n32),
                  C.byref(ne32))
        self.n64, self.n32, self.ne32 = n64.value, n32.value, ne32.value
        dev = d.device
        z64 = lambda: torch.zeros(self.n64, dtype=torch.float64, device=dev)  # noqa: E731
        z32 = lambda: torch.zeros(self.n32, dtype=torch.float32, device=dev)  # noqa: E731
        self.P64, self.G64, self.M64, self.V64 = z64(), z64(), z64(), z64()
        self.P32, self.G32, self.M32, self.V32 = z32(), z32(), z32(), z32()
        self.out = torch.zeros(13, dtype=torch.float64, device=dev)
        nb = _lib.lib.gpl_vigp_workspace(C.byref(self._m), C.byref(self._g), self.G)
        self.ws = torch.empty(nb, dtype=torch.uint8, device=dev)
        self.t = 0
        # block views (the library's layout)
        N = problem.grid.N
        self.lens_mean = self.P64[0:7]
        self.lens_raw = self.P64[7:56].view(7, 7)
        self.log_amp = self.P64[56:]
        o = 0
        self.sp = None
        sp_k = [k for k, (kind, _) in enumerate(model.layers) if kind == "sp"]
        if sp_k:
            G = self.G
            self.sp = dict(mean=self.P32[0:G], logs=self.P32[G:2 * G], cross=self.P32[2 * G:9 * G].view(7, G))
            o = 9 * G
        self.ip = []
        for kind, _ in model.layers:
            if kind == "ip":
                self.ip.append(dict(mean=self.P32[o:o + N], logs=self.P32[o + N:o + 2 * N]))
                o += 2 * N

    def elbo(self, e64: torch.Tensor, e32: torch.Tensor):
        """One ELBO sample and its gradient (into G64/G32); returns `out`."""
        pr = self.problem
        psf, src = pr.psf.c(), pr.source.c()
        _lib.call("gpl_vigp_elbo", C.byref(self._m), C.byref(self._g), C.byref(psf), C.byref(src),
                  float(pr.noise_sigma), self.G, _ptr(self.gx), _ptr(self.gy), _ptr(self.d), _ptr(self.P64),
                  _ptr(self.P32), _ptr(e64), _ptr(e32), _ptr(self.out), _ptr(self.G64), _ptr(self.G32),
                  _ptr(self.ws), self.ws.numel(), _stream())
        return self.out

    def adam(self, lr: float, betas=(0.9, 0.999), eps=1e-8):
        self.t += 1
        _lib.call("gpl_vigp_adam", self.n64, _ptr(self.P64), _ptr(self.G64), _ptr(self.M64), _ptr(self.V64),
                  self.n32, _ptr(self.P32), _ptr(self.G32), _ptr(self.M32), _ptr(self.V32), self.t, float(lr),
                  float(betas[0]), float(betas[1]), float(eps), _stream())

    def step(self, e64, e32, lr: float):
        out = self.elbo(e64, e32)
        self.adam(lr)
        return out
