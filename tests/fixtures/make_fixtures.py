"""Write the stored inputs and expected values of the full-size workload.

Runs only the FP64 oracle (and synth for the seeded draws). For the 100x100
image with 2x2 supersampling (N = 40,000 source points, the first prior draw of
that workload) it stores the simulated observation d, the exact Cholesky
evidence terms, the variational objective, the predicted image, and the exact
posterior mean and variance on the 40 x 40 source-plane grid at 30 mas centred
on the origin. For the 200x200 image with 2x2 supersampling (N = 160,000) it
stores the observation and the exact evidence of its central 100x100 crop.

    python tests/fixtures/make_fixtures.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import data, evidence, posterior  # noqa: E402


def make(index=1, sub=0):
    w = synth.workload(index, sub)
    s = w.source
    P = evidence.Problem(w.n, w.ss, w.pix_scale, w.lens.as_tuple(), (s.peak, s.R_e, s.n_sersic, s.xs, s.ys), w.ell,
                         w.amp, w.noise_sigma, w.psf_fwhm)
    t = time.time()
    d, _ = data.simulate(P, synth.noise_normals(w.n_pix, index, sub), rff=synth.rff_draws(8192, index, sub))
    out = evidence.solve_problem(P, d)
    gx, gy = synth.source_grid(40, 0.03)
    post = posterior.posterior_at(P, out, gx, gy)
    path = os.path.join(HERE, f"workload{index}_draw{sub}.npz")
    np.savez_compressed(path, d=d, image=out["image"], lnp=out["lnp"], quad=out["quad"], logdet=out["logdet"],
                        vi=out["vi"], lens=np.array(w.lens.as_tuple()), source=np.array([s.peak, s.R_e, s.n_sersic,
                                                                                         s.xs, s.ys]),
                        n=w.n, ss=w.ss, pix_scale=w.pix_scale, ell=w.ell, amp=w.amp, sigma=w.noise_sigma,
                        fwhm=w.psf_fwhm, grid_n=40, grid_spacing=0.03, grid_mean=post["mean"],
                        grid_var=post["var"])
    print(f"{path}: lnp {out['lnp']:.6f} quad {out['quad']:.6f} logdet {out['logdet']:.6f} "
          f"var [{post['var'].min():.3e}, {post['var'].max():.3e}] ({time.time() - t:.0f} s)")


def make_crop(index=2, sub=0, crop=100):
    """The 200x200 workload with 2x2 supersampling (N = 160,000): its full
    observation d (simulated with random Fourier features), and the exact
    Cholesky evidence and predicted image of the central crop x crop pixels
    (the same lens, the crop's own fine points; its pixel centres coincide with
    the full image's because the sides differ by an even number)."""
    w = synth.workload(index, sub)
    s = w.source
    src = (s.peak, s.R_e, s.n_sersic, s.xs, s.ys)
    P = evidence.Problem(w.n, w.ss, w.pix_scale, w.lens.as_tuple(), src, w.ell, w.amp, w.noise_sigma, w.psf_fwhm)
    t = time.time()
    d, _ = data.simulate(P, synth.noise_normals(w.n_pix, index, sub), rff=synth.rff_draws(8192, index, sub))
    o = (w.n - crop) // 2
    d_crop = d.reshape(w.n, w.n)[o:o + crop, o:o + crop].ravel()
    Pc = evidence.Problem(crop, w.ss, w.pix_scale, w.lens.as_tuple(), src, w.ell, w.amp, w.noise_sigma, w.psf_fwhm)
    out = evidence.solve_problem(Pc, d_crop)
    path = os.path.join(HERE, f"workload{index}_draw{sub}_crop{crop}.npz")
    np.savez_compressed(path, d=d, crop=crop, offset=o, image=out["image"], lnp=out["lnp"], quad=out["quad"],
                        logdet=out["logdet"])
    print(f"{path}: crop lnp {out['lnp']:.6f} quad {out['quad']:.6f} logdet {out['logdet']:.6f} "
          f"({time.time() - t:.0f} s)")


if __name__ == "__main__":
    make()
    make_crop()
