"""Pixel shapes, the windowed kernel (kind 1), the Gaussian products of the
transmission matrix and the source reconstruction, and the k-NN density
(through the C-ABI) against the FP64 oracle."""
import math

import numpy as np
import pytest

import synth
from oracle import kernel as okernel
from oracle import psf as opsf
from oracle import window as owin

from helpers import gpu_problem

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


def _lensed(G, index=1, n=24, ss=2):
    w = synth.workload(index).replace(n=n, ss=ss)
    prob = gpu_problem(w)
    pts = G.ops.lens_raytrace(prob.grid, prob.lens)
    return w, prob, pts


@pytest.mark.parametrize("n,ss", [(24, 1), (20, 2), (13, 3)])
def test_pixel_shapes_vs_oracle(G, n, ss):
    """Z from the FP32 ray-traced grid against the oracle's FP64 axes of the same
    points: the central differences cancel the coordinates, so the bound is a
    few FP32 ulps of |p| over |a| times |Z| (2e-5 of the trace of Z here)."""
    _say("pixel shapes", n, ss)
    w, prob, pts = _lensed(G, 1, n, ss)
    z = t64(G.ops.pixel_shapes(prob.grid, pts[0], pts[1]))
    a, b = owin.pixel_axes(t64(pts[0]), t64(pts[1]), n * ss)
    zo = owin.shape_cov(a, b).T
    tr = zo[0] + zo[2]
    err = np.max(np.abs(z - zo) / tr)
    print(f"max |dZ| / tr Z = {err:.2e}")
    assert err <= 2e-5


@pytest.mark.parametrize("n,ss,nrhs", [(24, 1, 3), (20, 2, 9), (13, 3, 1)])
def test_windowed_product_vs_oracle(G, n, ss, nrhs):
    """kind = 1 product against the oracle's dense windowed K on the same FP32
    points and the library's own pixel shapes (which the test above pins), per
    entry within 1e-5 of (|K||V|)."""
    _say("windowed product", n, ss, nrhs)
    w, prob, pts = _lensed(G, 1, n, ss)
    N = w.N
    rng = np.random.default_rng(60 + n)
    V = rng.standard_normal((nrhs, N)).astype(np.float32)
    kw = G.Kernel(w.ell, w.amp, kind=1)
    Y = G.ops.kernel_mvm(kw, pts[0], pts[1], cuda32(V), prec="fp32", grid=prob.grid)
    z = t64(G.ops.pixel_shapes(prob.grid, pts[0], pts[1])).T
    px, py = t64(pts[0]), t64(pts[1])
    K = owin.windowed_kernel_matrix(px, py, z, w.ell, w.amp)
    V64 = V.astype(np.float64).T
    want = K @ V64
    scale = np.abs(K) @ np.abs(V64)
    err = np.max(np.abs(t64(Y).T - want) / scale)
    print(f"max |err| / (|K||V|) = {err:.2e}")
    assert err <= 1e-5
    # the precision form is not available for kind 1
    with pytest.raises(Exception):
        G.ops.kernel_mvm(kw, pts[0], pts[1], cuda32(V), prec="f16x3", grid=prob.grid)


def test_gauss_product_without_shapes_is_the_rbf_product(G):
    """No shape covariances, base variance l^2, norm a^2 l^2: the RBF product."""
    _say("gauss product = rbf")
    rng = np.random.default_rng(61)
    n = 1500
    px, py = rng.uniform(-0.4, 0.4, (2, n))
    V = rng.standard_normal((5, n)).astype(np.float32)
    X, Yp = cuda32(px), cuda32(py)
    Y = G.ops.gauss_product(0.04 ** 2, 0.09 * 0.04 ** 2, X, Yp, X, Yp, cuda32(V))
    P64 = (px.astype(np.float32).astype(np.float64), py.astype(np.float32).astype(np.float64))
    V64 = V.astype(np.float64).T
    want = okernel.kernel_mvm(*P64, V64, 0.04, 0.3)
    scale = okernel.kernel_abs_mvm_rows(*P64, np.arange(n), V64, 0.04, 0.3)
    assert np.max(np.abs(t64(Y).T - want) / scale) <= 1e-5


def test_knn_density_vs_oracle(G):
    _say("knn density")
    rng = np.random.default_rng(62)
    q = rng.uniform(-1, 1, (2, 3000)).astype(np.float32)
    rho = t64(G.ops.knn_density(cuda32(q[0]), cuda32(q[1]), 20))
    want = owin.knn_density(q[0].astype(np.float64), q[1].astype(np.float64), 20)
    assert np.max(np.abs(rho - want) / want) <= 1e-5


def test_knn_density_lensed_full_size(G):
    """The traced 200 x 200 fine grid of the 100 x 100 workload (N = 40,000,
    strongly non-uniform): density at 600 sampled points against brute force
    on the same FP32 points, and a regular grid (many equal distances)."""
    _say("knn density lensed full size")
    w = synth.workload(1)
    prob = gpu_problem(w)
    pts = G.ops.lens_raytrace(prob.grid, prob.lens)
    rho = t64(G.ops.knn_density(pts[0], pts[1], 20))
    rows = np.random.default_rng(65).choice(w.N, 600, replace=False)
    r, _ = owin.knn_radius(t64(pts[0]), t64(pts[1]), 20, rows=rows)
    want = 20 / (math.pi * r * r)
    err = np.max(np.abs(rho[rows] - want) / want)
    print(f"max rel err {err:.2e}")
    assert err <= 1e-5
    gx, gy = synth.source_grid(40, 0.03)
    rho = t64(G.ops.knn_density(cuda32(gx), cuda32(gy), 20))
    want = owin.knn_density(gx.astype(np.float32).astype(np.float64), gy.astype(np.float32).astype(np.float64), 20)
    assert np.max(np.abs(rho - want) / want) <= 1e-5


def test_transmission_products_vs_oracle(G):
    """T y and T^T v (eq. "transmission") for image-plane inducing points (q = p,
    the pixel shapes on the point side) and for a 40 x 40 source-plane grid
    (no shapes), with weights A_k from the k-NN density, against the oracle's
    dense T; and the reconstruction sum of eq. "gp-reconstruction" on a fine
    grid."""
    _say("transmission")
    w, prob, pts = _lensed(G, 1, 24, 2)
    N = w.N
    px, py = t64(pts[0]), t64(pts[1])
    z = G.ops.pixel_shapes(prob.grid, pts[0], pts[1])
    z64 = t64(z).T
    rng = np.random.default_rng(63)
    l2h = 0.5 * w.ell ** 2
    # image-plane layer: q = p
    rho = G.ops.knn_density(pts[0], pts[1], 20)
    A = t64(rho)
    A = owin.transmission_weights(A, w.ell)
    Ad = cuda32(A)
    y = rng.standard_normal(N).astype(np.float32)
    Ty = G.ops.gauss_product(l2h, 1.0 / (2 * math.pi), pts[0], pts[1], pts[0], pts[1], cuda32(y), tz=z, sw=Ad)
    T = owin.transmission_matrix(px, py, z64, px, py, w.ell, A)
    want = T @ y.astype(np.float64)
    scale = np.abs(T) @ np.abs(y.astype(np.float64))
    assert np.max(np.abs(t64(Ty) - want) / scale) <= 1e-5
    v = rng.standard_normal(N).astype(np.float32)
    Ttv = G.ops.gauss_product(l2h, 1.0 / (2 * math.pi), pts[0], pts[1], pts[0], pts[1], cuda32(v), tw=Ad, sz=z)
    want = T.T @ v.astype(np.float64)
    scale = np.abs(T.T) @ np.abs(v.astype(np.float64))
    assert np.max(np.abs(t64(Ttv) - want) / scale) <= 1e-5
    # source-plane layer: a 40 x 40 grid at 30 mas over the points' centre
    c = np.array([px.mean(), py.mean()])
    g1 = (np.arange(40) - 19.5) * 0.03
    gx, gy = [u.ravel() + o for u, o in zip(np.meshgrid(g1, g1), c)]
    gxd, gyd = cuda32(gx), cuda32(gy)
    rg = t64(G.ops.knn_density(gxd, gyd, 20))
    Ag = owin.transmission_weights(rg, 0.1)
    yg = rng.standard_normal(1600).astype(np.float32)
    Tg = G.ops.gauss_product(0.5 * 0.1 ** 2, 1.0 / (2 * math.pi), pts[0], pts[1], gxd, gyd, cuda32(yg),
                             sw=cuda32(Ag))
    Tgo = owin.transmission_matrix(px, py, None, gx.astype(np.float32).astype(np.float64),
                                   gy.astype(np.float32).astype(np.float64), 0.1, Ag)
    want = Tgo @ yg.astype(np.float64)
    scale = np.abs(Tgo) @ np.abs(yg.astype(np.float64))
    # points far outside the grid see only terms that underflow FP32 (the FP64
    # values are ~1e-40 and below): a floor of 1e-12 of the largest scale
    assert np.all(np.abs(t64(Tg) - want) <= 1e-5 * scale + 1e-12 * scale.max())
    # reconstruction on a fine grid from the image-plane layer
    f1 = (np.arange(64) - 31.5) * 0.02
    fx, fy = [u.ravel() + o for u, o in zip(np.meshgrid(f1, f1), c)]
    beta = G.ops.gauss_product(l2h, 1.0 / (2 * math.pi), cuda32(fx), cuda32(fy), pts[0], pts[1], cuda32(y), sw=Ad)
    want = owin.reconstruct_brightness(fx.astype(np.float32).astype(np.float64),
                                       fy.astype(np.float32).astype(np.float64), px, py, y.astype(np.float64), w.ell,
                                       A)
    Tr = owin.transmission_matrix(fx.astype(np.float32).astype(np.float64), fy.astype(np.float32).astype(np.float64),
                                  None, px, py, w.ell, A)
    scale = np.abs(Tr) @ np.abs(y.astype(np.float64))
    assert np.all(np.abs(t64(beta) - want) <= 1e-5 * scale + 1e-12 * scale.max())


def test_apply_A_windowed_vs_oracle(G):
    """A = B K B^T + sigma^2 I with the windowed K (24 x 24 workload, PSF):
    against the oracle's dense matrices (FP32 points, the library's shapes)."""
    w = synth.workload(0)
    _say("apply_A windowed", w.name)
    prob = gpu_problem(w)
    prob = prob.replace(kernel=G.Kernel(w.ell, w.amp, kind=1))
    pts = G.ops.lens_raytrace(prob.grid, prob.lens)
    rng = np.random.default_rng(64)
    X = rng.standard_normal((4, w.n_pix)).astype(np.float32)
    Y = G.ops.apply_A(prob, pts[0], pts[1], cuda32(X), prec="fp32")
    z = t64(G.ops.pixel_shapes(prob.grid, pts[0], pts[1])).T
    K = owin.windowed_kernel_matrix(t64(pts[0]), t64(pts[1]), z, w.ell, w.amp)
    Bm = opsf.B_matrix(w.n, w.ss, opsf.psf_taps(w.psf_fwhm, w.pix_scale / w.ss))
    A = Bm @ K @ Bm.T + w.noise_sigma ** 2 * np.eye(w.n_pix)
    X64 = X.astype(np.float64).T
    want = A @ X64
    scale = np.abs(A) @ np.abs(X64)
    err = np.max(np.abs(t64(Y).T - want) / scale)
    print(f"max |err| / (|A||X|) = {err:.2e}")
    assert err <= 1e-5
