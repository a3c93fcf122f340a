"""Exact GP posterior mean and pointwise variance at source-plane points
(Sec. 3.7, eqs. "gp-exact-mean" and "gp-exact-var") through the C-ABI, against
the FP64 oracle.

Error bounds (per query point x, written in the tests): with s = w^T A^{-1} w,
w = B K(p, x), and a solve whose residual is res, |w^T A^{-1} res| <=
sqrt(s) |res| / sigma because every eigenvalue of A is at least sigma^2. The
solves report their true residual |res|/|rhs|, so the variance error is at most
2 sqrt(s) |w| (true_relres + 2e-6) / sigma (the 2e-6 covers the FP32 rounding of
w itself) and the mean's error from u = A^{-1} r at most sqrt(s) |r|
true_relres_u / sigma, each plus FP32 rounding of the sums."""
import os

import numpy as np
import pytest

import synth
from oracle import evidence as oev
from oracle import kernel as okernel
from oracle import posterior as opost

from helpers import gpu_problem, observation, oracle_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2105_09465_amd as G
    return G


def _say(*a):
    print("[case]", *a, flush=True)


def t64(x):
    return x.detach().double().cpu().numpy()


def cuda32(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def _oracle_on_points(P, d, px, py):
    """The oracle's exact solution for the given (GPU, FP32) points."""
    mu = P.mean(px, py)
    r = d - P.B(mu)
    A = oev.assemble_A(P, px, py)
    ev = oev.exact_evidence(A, r)
    return dict(px=px, py=py, r=r, **ev)


def _check(G, P, prob, rec, post, gx, gy, sol):
    o = opost.posterior_at(P, sol, gx, gy)
    sigma = prob.noise_sigma
    amp2 = prob.kernel.amplitude ** 2
    s = np.maximum(amp2 - o["var"], 0.0)
    W = t64(post.W)
    wn = np.linalg.norm(W, axis=1)
    tr = t64(post.cg["true_relres"])
    var = t64(post.var)
    bound_v = 2.0 * np.sqrt(s) * wn * (tr + 2e-6) / sigma + 1e-6 * amp2
    err_v = np.abs(var - o["var"])
    print(f"var: max err {err_v.max():.3e} (max bound {bound_v.max():.3e}, worst ratio "
          f"{np.max(err_v / bound_v):.3f}); var range [{o['var'].min():.3e}, {o['var'].max():.3e}]; "
          f"iters {int(t64(post.cg['iters']).max())}")
    assert np.all(err_v <= bound_v)
    # mean
    tr0 = float(rec.cg["true_relres"][0].item())
    rnorm = float(np.linalg.norm(sol["r"]))
    Kqp = okernel.rbf_matrix(gx, gy, P.ell, P.amp, sol["px"], sol["py"])
    scale = np.abs(Kqp) @ np.abs(P.BT(sol["u"])) + np.abs(P.mean(gx, gy))
    bound_m = 2.0 * np.sqrt(s) * rnorm * tr0 / sigma + 1e-5 * scale
    err_m = np.abs(t64(post.mean) - o["mean"])
    print(f"mean: max err {err_m.max():.3e} (worst ratio {np.max(err_m / bound_m):.3f}); "
          f"|mean| max {np.abs(o['mean']).max():.3e}")
    assert np.all(err_m <= bound_m)
    return o


def test_posterior_small_plain_cg(G):
    """24 x 24 workload with PSF, plain CG reconstruction; a 16 x 16 grid at
    40 mas over the source region (some points far from every fitted point)."""
    w, d, _ = observation(0)
    _say("posterior small plain", w.name)
    prob = gpu_problem(w)
    P = oracle_problem(w)
    rec = G.reconstruct(prob, cuda32(d), torch.empty(0, w.n_pix, device="cuda"), prec="fp32", tol=1e-6,
                        max_iter=1000, want_image=False)
    gx, gy = synth.source_grid(16, 0.04)
    gx32, gy32 = gx.astype(np.float32), gy.astype(np.float32)
    post = G.posterior_at(prob, rec, cuda32(gx32), cuda32(gy32))
    torch.cuda.synchronize()
    sol = _oracle_on_points(P, d, t64(rec.px), t64(rec.py))
    _check(G, P, prob, rec, post, gx32.astype(np.float64), gy32.astype(np.float64), sol)


@pytest.mark.parametrize("prec", ["fp32", "f16x3"])
def test_posterior_small_preconditioned(G, prec):
    """32 x 32 image at 2x supersampling (N = 4,096), preconditioned
    reconstruction of rank 512; a 24 x 24 grid at 30 mas."""
    w, d, _ = observation(1, n=32)
    _say("posterior small preconditioned", w.name, prec)
    prob = gpu_problem(w)
    P = oracle_problem(w)
    g, h = synth.preconditioned_probe_normals(w.n_pix, 512, 4, 1, 0)
    rec = G.reconstruct_preconditioned(prob, cuda32(d), torch.as_tensor(g, device="cuda"), cuda32(h), rank=512,
                                       prec=prec, want_image=False)
    gx, gy = synth.source_grid(24, 0.03)
    gx32, gy32 = gx.astype(np.float32), gy.astype(np.float32)
    post = G.posterior_at(prob, rec, cuda32(gx32), cuda32(gy32), prec=prec)
    torch.cuda.synchronize()
    sol = _oracle_on_points(P, d, t64(rec.px), t64(rec.py))
    _check(G, P, prob, rec, post, gx32.astype(np.float64), gy32.astype(np.float64), sol)


def test_posterior_grid_full_size_vs_stored_oracle(G):
    """100 x 100 image at 2x supersampling (N = 40,000): the 40 x 40 grid at 30
    mas against the stored FP64 oracle (computed on FP64 ray-traced points).
    The GPU's FP32 points differ from those by the ray tracer's rounding (about
    1e-7 of the deflection), which moves K(x, p) by up to |x - p| / l^2 times
    that shift; the bounds add 1e-4 alpha^2 to the variance's and 1e-4 of the
    largest |mean| to the mean's for it."""
    path = os.path.join(os.path.dirname(__file__), "fixtures", "workload1_draw0.npz")
    f = np.load(path)
    w = synth.workload(1)
    _say("posterior full size", w.name)
    prob = gpu_problem(w)
    d = f["d"]
    g, h = synth.preconditioned_probe_normals(w.n_pix, 4096, 16, 1, 0)
    rec = G.reconstruct_preconditioned(prob, cuda32(d), torch.as_tensor(g, device="cuda"), cuda32(h), rank=4096,
                                       prec="f16x3", want_image=False)
    gx, gy = synth.source_grid(int(f["grid_n"]), float(f["grid_spacing"]))
    post = G.posterior_at(prob, rec, cuda32(gx), cuda32(gy))
    torch.cuda.synchronize()
    amp2 = w.amp ** 2
    var, mean = t64(post.var), t64(post.mean)
    ev = np.abs(var - f["grid_var"])
    em = np.abs(mean - f["grid_mean"])
    tr = t64(post.cg["true_relres"])
    print(f"full size: var err max {ev.max():.3e} (alpha^2 {amp2}), mean err max {em.max():.3e} "
          f"(|mean| max {np.abs(f['grid_mean']).max():.3e}); true residual max {tr.max():.2e}; "
          f"iters {int(t64(post.cg['iters']).max())}")
    s = np.maximum(amp2 - f["grid_var"], 0.0)
    wn = np.linalg.norm(t64(post.W), axis=1)
    assert np.all(ev <= 2.0 * np.sqrt(s) * wn * (tr + 2e-6) / w.noise_sigma + 1e-4 * amp2)
    rnorm = float(torch.linalg.vector_norm(rec.rhs[0].double()).item())
    tr0 = float(rec.cg["true_relres"][0].item())
    assert np.all(em <= 2.0 * np.sqrt(s) * rnorm * tr0 / w.noise_sigma + 1e-4 * np.max(np.abs(f["grid_mean"])))
