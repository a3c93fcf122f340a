"""Shared test plumbing: workloads from synth as GPU-package and oracle problems,
and the oracle-generated observation for a workload."""
from __future__ import annotations

import functools

import numpy as np

import synth
from oracle import data as odata
from oracle import evidence as oev


def oracle_problem(w: synth.Workload, cx=0.0, cy=0.0):
    s = w.source
    return oev.Problem(w.n, w.ss, w.pix_scale, w.lens.as_tuple(), (s.peak, s.R_e, s.n_sersic, s.xs, s.ys), w.ell,
                       w.amp, w.noise_sigma, w.psf_fwhm, cx, cy)


def gpu_problem(w: synth.Workload, cx=0.0, cy=0.0):
    import paper_2105_09465_amd as G
    s = w.source
    return G.Problem(G.Grid(w.n, w.ss, w.pix_scale, cx, cy), G.Lens(*w.lens.as_tuple()),
                     G.Sersic(s.peak, s.R_e, s.n_sersic, s.xs, s.ys), G.Kernel(w.ell, w.amp), G.PSF(w.psf_fwhm),
                     w.noise_sigma)


@functools.lru_cache(maxsize=16)
def observation(index: int, sub: int = 0, n=None, ss=None, exact_max=4096):
    """Observed image of workload `index` (optionally resized), simulated by the
    oracle: exact GP draw for N <= exact_max, random Fourier features above."""
    w = synth.workload(index, sub)
    if n is not None:
        w = w.replace(n=n)
    if ss is not None:
        w = w.replace(ss=ss)
    P = oracle_problem(w)
    noise = synth.noise_normals(w.n_pix, index, sub)
    if w.N <= exact_max:
        d, truth = odata.simulate(P, noise, gp_normals=synth.gp_normals(w.N, index, sub))
    else:
        d, truth = odata.simulate(P, noise, rff=synth.rff_draws(8192, index, sub))
    return w, d, truth
