"""FP64 CPU oracle for the lensed-source GP evidence path.

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, obviously correct
numpy/scipy implementation of what the GPU library computes. It may be
imported only by the tests, by the smoke check and by the bench's CPU-baseline
leg. It shares no code with the GPU package and imports nothing from it; the
product path never calls it.

Each function cites the passage of Karchev, Coogan & Weniger (2021),
"Strong-lensing source reconstruction with variationally optimised Gaussian
processes", that it follows. Readings of passages the paper leaves open are
stated where they are used.
"""
from . import grid, lens, source, kernel, psf, evidence, krylov, precond, gradients, data, window, posterior, vigp  # noqa: F401,E501
