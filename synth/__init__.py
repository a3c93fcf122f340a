"""Seeded synthetic inputs shared by the tests, the oracle fixtures and the bench.

This package holds only workload definitions (sizes, hyperparameter values,
prior ranges) and seeded random draws. It contains none of the method's
arithmetic: no ray tracing, kernels, solves or determinants. Random numbers
that the method consumes (probe vectors, noise, GP-draw normals, random
Fourier feature draws) are produced here and handed to both the GPU path and
the FP64 oracle as plain arrays.
"""
from .inputs import *  # noqa: F401,F403
