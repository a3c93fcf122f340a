"""Image-plane pixel grid, supersampling and local averaging (oracle).

Sec. 2 (model overview) places observations at the image-plane pixel centres;
Sec. 4.1 generates images at a finer resolution and downsamples them "by local
averaging". Reading: the image is n x n pixels of side `pix_scale`, centred on
the optical axis, each split into ss x ss sub-pixels; sub-pixel centres are at
((f - (M-1)/2) h) with M = n*ss, h = pix_scale/ss; x grows with the column
index and y with the row index; fine points are stored row-major
(j = f_y*M + f_x). Local averaging D is the plain mean over each ss x ss block.
A crop of a larger image is the same grid shifted by the position (cx, cy) of
its centre.
"""
from __future__ import annotations

import numpy as np


def fine_coords(n: int, ss: int, pix_scale: float, cx: float = 0.0, cy: float = 0.0):
    """Sub-pixel centres (x, y), each of length N = (n*ss)^2, row-major."""
    M = n * ss
    h = pix_scale / ss
    c = (np.arange(M, dtype=np.float64) - (M - 1) / 2.0) * h
    yy, xx = np.meshgrid(c, c, indexing="ij")
    return cx + xx.ravel(), cy + yy.ravel()


def coarse_of_fine(n: int, ss: int) -> np.ndarray:
    """Index of the image pixel that contains each fine point (int64, length N)."""
    M = n * ss
    fy, fx = np.divmod(np.arange(M * M, dtype=np.int64), M)
    return (fy // ss) * n + (fx // ss)


def block_mean(f: np.ndarray, n: int, ss: int) -> np.ndarray:
    """D: fine (N, ...) -> coarse (n*n, ...), mean over each ss x ss block."""
    idx = coarse_of_fine(n, ss)
    out = np.zeros((n * n,) + f.shape[1:], dtype=np.float64)
    np.add.at(out, idx, f)
    return out / (ss * ss)


def block_mean_T(x: np.ndarray, n: int, ss: int) -> np.ndarray:
    """D^T: coarse (n*n, ...) -> fine (N, ...): each fine point gets x_I / ss^2."""
    return x[coarse_of_fine(n, ss)] / (ss * ss)
