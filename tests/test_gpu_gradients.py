"""Gradients through the library adjoints (ray tracing, Sersic mean, kernel
product, PSF) against the FP64 oracle: central differences of oracle
functions for the building blocks, and the oracle's analytic evidence gradient
(itself pinned to finite differences in the CPU tests) for the full chain."""
import math

import numpy as np
import pytest

import synth
from oracle import gradients as ograd
from oracle import kernel as okernel
from oracle import lens as olens
from oracle import psf as opsf
from oracle import source as osource

from helpers import gpu_problem, oracle_problem

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


@pytest.mark.parametrize("n,spread", [(700, 0.15), (4000, 1.2)])
def test_kernel_mvm_adjoint(G, n, spread):
    """F = sum_c g_c^T K V_c: gradients w.r.t. points, lengthscale, amplitude and V
    against FP64 central differences of the oracle's matrix-free product. The
    wide cloud (60 lengthscales across) has most source tiles beyond the exact-zero
    cutoff, which the adjoint skips."""
    _say("kernel mvm adjoint", n, spread)
    rng = np.random.default_rng(0)
    m = 3
    px = rng.uniform(-spread, spread, n).astype(np.float32)
    py = rng.uniform(-spread, spread, n).astype(np.float32)
    V = rng.standard_normal((m, n)).astype(np.float32)
    gY = rng.standard_normal((m, n)).astype(np.float32)
    ell, amp = 0.04, 0.3
    tpx = cuda32(px).requires_grad_()
    tpy = cuda32(py).requires_grad_()
    tV = cuda32(V).requires_grad_()
    th = torch.tensor([ell, amp], dtype=torch.float64, device="cuda", requires_grad=True)
    Y = G.autograd.KernelMVM.apply(tpx, tpy, tV, th)
    Y.backward(cuda32(gY))
    P = (px.astype(np.float64), py.astype(np.float64))
    V64, g64 = V.astype(np.float64).T, gY.astype(np.float64).T

    def F(qx, qy, l, a):
        return float(np.sum(g64 * okernel.kernel_mvm(qx, qy, V64, l, a)))

    h = 1e-6
    idx = rng.choice(n, 12, replace=False)
    for i in idx:
        for comp, tg in ((0, tpx), (1, tpy)):
            qp = [P[0].copy(), P[1].copy()]
            qm = [P[0].copy(), P[1].copy()]
            qp[comp][i] += h
            qm[comp][i] -= h
            fd = (F(*qp, ell, amp) - F(*qm, ell, amp)) / (2 * h)
            got = tg.grad[i].item()
            assert abs(got - fd) <= 2e-4 * abs(fd) + 2e-4, (i, comp, got, fd)
    gl = (F(*P, ell + 1e-7, amp) - F(*P, ell - 1e-7, amp)) / 2e-7
    ga = (F(*P, ell, amp + 1e-7) - F(*P, ell, amp - 1e-7)) / 2e-7
    assert math.isclose(th.grad[0].item(), gl, rel_tol=1e-4)
    assert math.isclose(th.grad[1].item(), ga, rel_tol=1e-4)
    # d/dV = K g (K symmetric)
    want = okernel.kernel_mvm(*P, g64, ell, amp).T
    assert np.max(np.abs(t64(tV.grad) - want)) <= 1e-5 * np.max(np.abs(want))


def test_raytrace_adjoint(G):
    """sum_i g_i . dp_i/dtheta for the 8 lens parameters vs the oracle Jacobian."""
    _say("raytrace adjoint")
    lens = synth.workload(1, 2).lens.as_tuple()
    grid = G.Grid(40, 2, 0.05, 0.9, 0.4)
    rng = np.random.default_rng(1)
    g = rng.standard_normal((2, grid.N)).astype(np.float32)
    th = torch.tensor(lens, dtype=torch.float64, device="cuda", requires_grad=True)
    p = G.autograd.RayTrace.apply(th, grid)
    p.backward(cuda32(g))
    xi_x, xi_y, _ = G.ops.grid_map(grid)
    J = olens.raytrace_jacobian(t64(xi_x), t64(xi_y), lens)  # (N, 2, 8)
    want = np.einsum("ia,iak->k", g.T.astype(np.float64), J)
    scale = np.einsum("ia,iak->k", np.abs(g.T.astype(np.float64)), np.abs(J))
    got = t64(th.grad)
    print("raytrace adjoint rel err", np.abs(got - want) / scale)
    assert np.all(np.abs(got - want) <= 2e-5 * scale)


def test_sersic_adjoint(G):
    _say("sersic adjoint")
    rng = np.random.default_rng(2)
    n = 3000
    px = rng.uniform(-0.5, 0.5, n).astype(np.float32)
    py = rng.uniform(-0.5, 0.5, n).astype(np.float32)
    gmu = rng.standard_normal(n).astype(np.float32)
    src = (0.6, 0.1, 1.5, 0.02, -0.03)
    gpx = torch.zeros(n, device="cuda")
    gpy = torch.zeros(n, device="cuda")
    gs = G.ops.sersic_backward(G.Sersic(*src), cuda32(px), cuda32(py), cuda32(gmu), gpx, gpy)
    src32 = src[:3] + tuple(float(np.float32(v)) for v in src[3:])
    grad = osource.sersic_grad(px.astype(np.float64), py.astype(np.float64), *src32)
    want = gmu[:, None].astype(np.float64) * grad
    assert np.allclose(t64(gpx), want[:, 0], rtol=2e-5, atol=1e-6 * np.abs(want).max())
    assert np.allclose(t64(gpy), want[:, 1], rtol=2e-5, atol=1e-6 * np.abs(want).max())
    assert np.allclose(t64(gs), -want.sum(axis=0), rtol=1e-4, atol=1e-5 * np.abs(want).sum())


def _crop_center(index, side):
    """Brightest noiseless image pixel of the workload, as a crop centre clamped
    so a side x side crop stays inside the image."""
    w = synth.workload(index)
    P = oracle_problem(w)
    px, py = P.points()
    img = P.B(P.mean(px, py)).reshape(w.n, w.n)
    iy, ix = np.unravel_index(np.argmax(img), img.shape)
    half = side // 2
    iy = min(max(iy, half), w.n - half)
    ix = min(max(ix, half), w.n - half)
    # centre of the crop covering pixels [i - half, i + half)
    cx = (ix - half + (side - 1) / 2 - (w.n - 1) / 2) * w.pix_scale
    cy = (iy - half + (side - 1) / 2 - (w.n - 1) / 2) * w.pix_scale
    return w, cx, cy


@pytest.mark.parametrize("side", [32])
def test_evidence_gradient_crop_exact_trace(G, side):
    """Gradient of ln p and L_VI w.r.t. the 8 lens parameters, source offset,
    lengthscale and amplitude on a 32x32 crop (2x2 supersampling, N = 4096) of the
    gradient workload, centred on its brightest noiseless pixel. Exact-trace mode
    (all 1024 unit probes) makes the GPU gradient deterministic; compared with the
    oracle's dense analytic gradient."""
    w0, cx, cy = _crop_center(3, side)
    w = w0.replace(n=side)
    _say("evidence gradient crop", side, cx, cy)
    P = oracle_problem(w, cx, cy)
    from oracle import data as odata
    d, _ = odata.simulate(P, synth.noise_normals(w.n_pix, 3), gp_normals=synth.gp_normals(w.N, 3))
    an = ograd.analytic_gradient(P, d)
    prob = gpu_problem(w, cx, cy)
    th = torch.tensor(G.autograd.theta_of(prob), dtype=torch.float64, device="cuda", requires_grad=True)
    E = torch.eye(w.n_pix, dtype=torch.float32, device="cuda")
    out = G.autograd.evidence(th, prob, cuda32(d), E, tol=1e-7, max_iter=3000, n_lanczos=3000, logdet_scale=1.0)
    gl = torch.autograd.grad(out[0], th, retain_graph=True)[0]
    gv = torch.autograd.grad(out[1], th)[0]
    for name, got, want in (("lnp", t64(gl), an["grad_lnp"]), ("vi", t64(gv), an["grad_vi"])):
        scale = np.maximum(np.abs(want), 1e-3 * np.max(np.abs(want)))
        rel = np.abs(got - want) / scale
        print(name, "max rel err", rel.max(), dict(zip(G.autograd.PARAM_NAMES, np.round(rel, 7))))
        assert rel.max() <= 5e-4, name
    assert math.isclose(out[0].item(), an["lnp"], rel_tol=1e-4)
    assert math.isclose(out[1].item(), an["vi"], rel_tol=1e-4)


def test_vi_gradient_without_probes(G):
    """The variational objective has no trace term, so its gradient needs no
    probes: 28x28 pixels, ss = 2 (N = 3136, random-Fourier-feature source draw)
    against the oracle's analytic gradient."""
    w = synth.workload(3).replace(n=28)
    _say("vi gradient 28x28 ss2")
    P = oracle_problem(w)
    from oracle import data as odata
    d, _ = odata.simulate(P, synth.noise_normals(w.n_pix, 3, 5), rff=synth.rff_draws(4096, 3, 5))
    an = ograd.analytic_gradient(P, d)
    prob = gpu_problem(w)
    th = torch.tensor(G.autograd.theta_of(prob), dtype=torch.float64, device="cuda", requires_grad=True)
    out = G.autograd.evidence(th, prob, cuda32(d), torch.empty(0, w.n_pix, device="cuda"), tol=1e-7,
                              max_iter=3000, n_lanczos=0)
    gv = torch.autograd.grad(out[1], th)[0]
    got, want = t64(gv), an["grad_vi"]
    scale = np.maximum(np.abs(want), 1e-3 * np.max(np.abs(want)))
    rel = np.abs(got - want) / scale
    print("vi max rel err", rel.max(), dict(zip(G.autograd.PARAM_NAMES, np.round(rel, 7))))
    assert rel.max() <= 1e-3
