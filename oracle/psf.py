"""Observation operator B = D o P: PSF convolution on the fine grid, then local
averaging to image pixels (oracle, FP64).

The paper models the instrument as i.i.d. Gaussian noise and names a PSF as a
straightforward extension that acts on the predicted fluxes before the noise
(Sec. 2, model overview; Sec. 3.1 footnote on S; Sec. 3.3 footnote on
splitting the data sampling into a deterministic PSF step and uncorrelated
noise). Reading: Gaussian PSF of the given FWHM, sigma = FWHM / (2 sqrt(2 ln 2)),
sampled at fine-grid offsets k*h for |k| <= r = ceil(4 sigma / h), normalised to
unit sum per axis, applied as the outer product of the 1-D taps with zero
padding ("same" size). Local averaging D is the ss x ss block mean (Sec. 4.1).
"""
from __future__ import annotations

import math

import numpy as np

from . import grid


def psf_sigma(fwhm: float) -> float:
    return fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))


def psf_taps(fwhm: float, h: float, radius: int = 0) -> np.ndarray:
    """Normalised 1-D Gaussian taps w[-r..r] on spacing h; fwhm == 0 gives [1]."""
    if fwhm <= 0:
        return np.ones(1)
    s = psf_sigma(fwhm)
    r = radius if radius > 0 else int(math.ceil(4.0 * s / h))
    k = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-0.5 * (k * h / s) ** 2)
    return w / w.sum()


def conv_same(img: np.ndarray, taps: np.ndarray) -> np.ndarray:
    """2-D zero-padded 'same' convolution of img (M, M, ...) with taps (x) taps.

    out[y, x] = sum_{a, b} w[a] w[b] img[y - a, x - b], shifts |a|, |b| <= r."""
    r = (taps.size - 1) // 2
    M0, M1 = img.shape[:2]
    pad = [(r, r), (r, r)] + [(0, 0)] * (img.ndim - 2)
    src = np.pad(img, pad)
    tmp = np.zeros((M0 + 2 * r, M1) + img.shape[2:])
    for b in range(-r, r + 1):  # along x
        tmp += taps[b + r] * src[:, r - b:r - b + M1]
    out = np.zeros_like(img, dtype=np.float64)
    for a in range(-r, r + 1):  # along y
        out += taps[a + r] * tmp[r - a:r - a + M0]
    return out


def apply_B(f: np.ndarray, n: int, ss: int, taps: np.ndarray) -> np.ndarray:
    """B f: fine (N, ...) -> image pixels (n*n, ...)."""
    M = n * ss
    img = f.reshape((M, M) + f.shape[1:])
    return grid.block_mean(conv_same(img, taps).reshape(f.shape), n, ss)


def apply_BT(x: np.ndarray, n: int, ss: int, taps: np.ndarray) -> np.ndarray:
    """B^T x = P^T D^T x; the taps are symmetric, so P^T is the same convolution."""
    M = n * ss
    f = grid.block_mean_T(x, n, ss)
    img = f.reshape((M, M) + x.shape[1:])
    return conv_same(img, taps[::-1]).reshape(f.shape)


def B_matrix(n: int, ss: int, taps: np.ndarray) -> np.ndarray:
    """Dense B (n*n x N), column by column from unit fine images."""
    N = (n * ss) ** 2
    return apply_B(np.eye(N), n, ss, taps)
