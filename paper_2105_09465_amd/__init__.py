"""MI355X (gfx950) library for the Gaussian-process evidence of a strongly
lensed source: SPLE + shear ray tracing, matrix-free RBF kernel products,
conjugate gradients, stochastic Lanczos quadrature, PSF and local averaging,
their adjoints, and a continuous-batching request loop.

The computation lives in libgplens.so (C-ABI in include/gplens.h); this
package binds it for torch tensors.
"""
from . import _lib, autograd, ops, params, pipeline, serving, vigp  # noqa: F401
from .params import Grid, Kernel, Lens, Problem, PSF, Sersic  # noqa: F401
from .pipeline import posterior_at, reconstruct, reconstruct_preconditioned  # noqa: F401
