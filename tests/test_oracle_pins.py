"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: closed forms,
library routines used as independent references (mpmath, scipy), brute force
on tiny inputs, identities, and the values the paper prints.
"""
import math
import os

import mpmath
import numpy as np
import pytest
import scipy.integrate as si
import scipy.stats as st

import synth
from oracle import (data, evidence, gradients, grid, kernel, krylov, lens, posterior, precond, psf, source, vigp,
                    window)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append([float(v) for v in line.split()])
    return np.array(rows)


# ---------------------------------------------------------------- grid (a1)

def test_grid_index_brute_force():
    for n, ss in [(3, 1), (3, 2), (4, 3), (5, 2)]:
        M = n * ss
        want = []
        for fy in range(M):
            for fx in range(M):
                want.append((fy // ss) * n + (fx // ss))
        assert np.array_equal(grid.coarse_of_fine(n, ss), np.array(want))


def test_grid_coords_centred_and_spaced():
    x, y = grid.fine_coords(4, 2, 0.05)
    M, h = 8, 0.025
    assert abs(x.mean()) < 1e-15 and abs(y.mean()) < 1e-15
    assert np.allclose(np.diff(x.reshape(M, M), axis=1), h)
    assert np.allclose(np.diff(y.reshape(M, M), axis=0), h)
    # sub-pixel centres sit at ((s + 1/2)/ss - 1/2) pix inside each pixel
    assert math.isclose(x[0], -(M - 1) / 2 * h)


def test_block_mean_adjoint_and_constant():
    rng = np.random.default_rng(1)
    f, xv = rng.standard_normal(36), rng.standard_normal(9)
    assert math.isclose(grid.block_mean(f, 3, 2) @ xv, f @ grid.block_mean_T(xv, 3, 2), rel_tol=1e-13)
    assert np.allclose(grid.block_mean(np.full(36, 2.5), 3, 2), 2.5)


# ---------------------------------------------------------------- lensing (a2)

def test_hyp2f1_series_matches_mpmath():
    rng = np.random.default_rng(2)
    for _ in range(20):
        slope = rng.uniform(1.5, 2.5)
        qq = rng.uniform(0.1, 1.0)
        ang = rng.uniform(-math.pi, math.pi)
        z = -(1 - qq) / (1 + qq) * complex(math.cos(2 * ang), math.sin(2 * ang))
        b, c = (slope - 1) / 2, (5 - slope) / 2
        got = lens.hyp2f1_one(b, c, np.array([z]))[0]
        want = complex(mpmath.hyp2f1(1, b, c, z))
        assert abs(got - want) <= 1e-14 * abs(want)


def test_sis_einstein_ring():
    """Singular isothermal sphere: every point of |xi| = theta_E maps to the origin."""
    theta_E = 0.6
    t = np.linspace(0, 2 * np.pi, 64, endpoint=False)
    px, py = lens.raytrace(theta_E * np.cos(t), theta_E * np.sin(t), (theta_E, 1.0, 0.3, 2.0, 0, 0, 0, 0))
    assert np.max(np.hypot(px, py)) < 1e-14
    # and |alpha| = theta_E everywhere (constant deflection magnitude)
    ax, ay = lens.sple_deflection(np.array([0.1, 2.0]), np.array([-0.3, 1.0]), theta_E, 1.0, 0.3, 2.0, 0, 0)
    assert np.allclose(np.hypot(ax, ay), theta_E, rtol=1e-15)


def test_circular_power_law_mass_enclosed():
    """q = 1: alpha = R <kappa>(R), the mean convergence inside R from the printed kappa."""
    for slope in (1.7, 2.0, 2.3):
        theta_E = 1.1
        for R in (0.2, 0.9, 2.3):
            kbar = 2.0 / R ** 2 * si.quad(
                lambda r: (3 - slope) / 2 * (theta_E / r) ** (slope - 1) * r, 0, R, limit=200)[0]
            ax, ay = lens.sple_deflection(np.array([R * 0.6]), np.array([R * 0.8]), theta_E, 1.0, 0.0, slope, 0, 0)
            assert math.isclose(math.hypot(ax[0], ay[0]), R * kbar, rel_tol=1e-9)


def test_sie_arctan_closed_form():
    """slope = 2: 2F1(1, 1/2; 3/2; -w^2) = arctan(w)/w (A&S 15.1.4)."""
    for q in (0.1, 0.6, 0.8, 0.95):
        ang = np.linspace(-3, 3, 13)
        z = -(1 - q) / (1 + q) * np.exp(2j * ang)
        w = np.sqrt(-z + 0j)
        want = np.arctan(w) / w
        got = lens.hyp2f1_one(0.5, 1.5, z)
        assert np.max(np.abs(got - want)) < 1e-14


@pytest.mark.parametrize("slope,q,phi", [(2.2, 0.7, 0.4), (1.85, 0.6, 2.0), (2.0, 0.8, math.radians(30))])
def test_poisson_and_curl(slope, q, phi):
    """div alpha = 2 kappa and curl alpha = 0 (FP64 central differences): pins the
    prefactor, exponent, 2F1 arguments and the rotation back to the sky frame."""
    theta_E, x0, y0 = 1.1, 0.05, -0.1
    rng = np.random.default_rng(3)
    X = rng.uniform(-2, 2, 30)
    Y = rng.uniform(-2, 2, 30)
    h = 1e-5

    def a(x, y):
        return lens.sple_deflection(x, y, theta_E, q, phi, slope, x0, y0)

    axp, _ = a(X + h, Y)
    axm, _ = a(X - h, Y)
    _, ayp = a(X, Y + h)
    _, aym = a(X, Y - h)
    _, ayxp = a(X + h, Y)
    _, ayxm = a(X - h, Y)
    axyp, _ = a(X, Y + h)
    axym, _ = a(X, Y - h)
    div = (axp - axm) / (2 * h) + (ayp - aym) / (2 * h)
    curl = (ayxp - ayxm) / (2 * h) - (axyp - axym) / (2 * h)
    kap = lens.convergence(X, Y, theta_E, q, phi, slope, x0, y0)
    assert np.allclose(div / 2, kap, rtol=2e-8)
    assert np.max(np.abs(curl)) < 1e-7


def test_shear_is_linear_about_origin():
    px, py = lens.raytrace(np.array([0.7]), np.array([-0.4]), (1e-12, 1.0, 0, 2.0, 5.0, 5.0, 0.03, -0.02))
    # negligible SPLE (tiny theta_E far away), shear only
    assert math.isclose(px[0], 0.7 - (0.03 * 0.7 - 0.02 * -0.4), rel_tol=1e-9)
    assert math.isclose(py[0], -0.4 - (-0.02 * 0.7 - 0.03 * -0.4), rel_tol=1e-9)


def test_raytrace_jacobian_identities():
    lp = (1.1, 0.7, 0.4, 2.15, 0.05, -0.1, 0.03, -0.02)
    X = np.array([0.3, -1.2, 1.7, 0.9])
    Y = np.array([1.1, 0.4, -0.8, -1.5])
    J = lens.raytrace_jacobian(X, Y, lp)
    ax, ay = lens.sple_deflection(X, Y, *lp[:6])
    # theta_E: alpha_SPLE scales as theta_E^(slope-1)
    assert np.allclose(J[:, 0, 0], -(lp[3] - 1) / lp[0] * ax, rtol=1e-9)
    assert np.allclose(J[:, 1, 0], -(lp[3] - 1) / lp[0] * ay, rtol=1e-9)
    # lens centre: dp/dx0 + dp/dy0 traces give div alpha = 2 kappa
    kap = lens.convergence(X, Y, *lp[:6])
    assert np.allclose(J[:, 0, 4] + J[:, 1, 5], 2 * kap, rtol=1e-8)
    # shear columns are exact
    assert np.allclose(J[:, 0, 6], -X) and np.allclose(J[:, 1, 6], Y)
    assert np.allclose(J[:, 0, 7], -Y) and np.allclose(J[:, 1, 7], -X)
    # q, phi, slope against mpmath high-precision differentiation at one point
    mpmath.mp.dps = 30

    def p_mp(k, comp):
        def f(t):
            v = [mpmath.mpf(x) for x in lp]
            v[k] = t
            th, q, phi, s, x0, y0 = v[:6]
            dx, dy = mpmath.mpf(X[0]) - x0, mpmath.mpf(Y[0]) - y0
            xp = mpmath.cos(phi) * dx + mpmath.sin(phi) * dy
            yp = -mpmath.sin(phi) * dx + mpmath.cos(phi) * dy
            Rx, Ry = mpmath.sqrt(q) * xp, yp / mpmath.sqrt(q)
            R = mpmath.sqrt(Rx ** 2 + Ry ** 2)
            e = mpmath.mpc(Rx, Ry) / R
            F = mpmath.hyp2f1(1, (s - 1) / 2, (5 - s) / 2, -(1 - q) / (1 + q) * e ** 2)
            a = th * 2 * mpmath.sqrt(q) / (1 + q) * (th / R) ** (s - 2) * F * e
            axs = mpmath.cos(phi) * a.real - mpmath.sin(phi) * a.imag
            ays = mpmath.sin(phi) * a.real + mpmath.cos(phi) * a.imag
            return -(axs if comp == 0 else ays)
        return float(mpmath.diff(f, mpmath.mpf(lp[k])))

    for k in (1, 2, 3):
        for comp in (0, 1):
            assert math.isclose(J[0, comp, k], p_mp(k, comp), rel_tol=1e-8, abs_tol=1e-11)


# ---------------------------------------------------------------- source (a3)

def test_sersic_bn_textbook():
    for n, bn in _golden("sersic_bn.txt"):
        assert math.isclose(source.sersic_bn(n), bn, rel_tol=2e-6)


def test_sersic_half_light_and_gradient():
    n, Re, peak = 1.5, 0.1, 0.6
    tot = si.quad(lambda r: source.sersic(r, 0.0, peak, Re, n, 0, 0) * r, 0, 50 * Re, limit=400)[0]
    half = si.quad(lambda r: source.sersic(r, 0.0, peak, Re, n, 0, 0) * r, 0, Re, limit=400)[0]
    assert math.isclose(half, tot / 2, rel_tol=1e-8)
    assert math.isclose(float(source.sersic(0.0, 0.0, peak, Re, n, 0, 0)), peak, rel_tol=1e-14)
    px, py = np.array([0.03, -0.2]), np.array([0.05, 0.11])
    g = source.sersic_grad(px, py, peak, Re, n, 0.01, -0.02)
    h = 1e-6
    fdx = (source.sersic(px + h, py, peak, Re, n, 0.01, -0.02) - source.sersic(px - h, py, peak, Re, n, 0.01, -0.02)) / (2 * h)
    fdy = (source.sersic(px, py + h, peak, Re, n, 0.01, -0.02) - source.sersic(px, py - h, peak, Re, n, 0.01, -0.02)) / (2 * h)
    assert np.allclose(g[:, 0], fdx, rtol=1e-7) and np.allclose(g[:, 1], fdy, rtol=1e-7)


# ---------------------------------------------------------------- kernel (a5)

def test_kernel_symmetric_psd_and_mvm():
    rng = np.random.default_rng(4)
    px, py = rng.uniform(-0.3, 0.3, 300), rng.uniform(-0.3, 0.3, 300)
    K = kernel.rbf_matrix(px, py, 0.04, 0.3)
    assert np.array_equal(K, K.T)
    assert np.allclose(np.diag(K), 0.09, rtol=0, atol=0)
    assert np.linalg.eigvalsh(K).min() >= -1e-12 * 0.09 * 300
    V = rng.standard_normal((300, 5))
    Y = kernel.kernel_mvm(px, py, V, 0.04, 0.3, block=37)
    # brute force on one entry with a Python loop
    i, c = 17, 3
    s = sum(0.09 * math.exp(-((px[i] - px[j]) ** 2 + (py[i] - py[j]) ** 2) / (2 * 0.04 ** 2)) * V[j, c] for j in range(300))
    assert math.isclose(Y[i, c], s, rel_tol=1e-12)
    assert np.allclose(Y, K @ V, rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------- PSF / B (a4)

def test_psf_taps_and_adjoint():
    taps = psf.psf_taps(0.1, 0.025)
    assert math.isclose(taps.sum(), 1.0, rel_tol=1e-15)
    assert taps.size == 2 * math.ceil(4 * 0.1 / (2 * math.sqrt(2 * math.log(2))) / 0.025) + 1
    rng = np.random.default_rng(5)
    for n, ss in [(6, 1), (5, 2)]:
        f = rng.standard_normal((n * ss) ** 2)
        xv = rng.standard_normal(n * n)
        lhs = psf.apply_B(f, n, ss, taps) @ xv
        rhs = f @ psf.apply_BT(xv, n, ss, taps)
        assert math.isclose(lhs, rhs, rel_tol=1e-13)


def test_psf_sigma_is_half_maximum_width():
    """The FWHM -> sigma conversion, pinned by the definition of the full width
    at half maximum rather than by its closed form: with taps on a spacing that
    puts a sample exactly at FWHM/2 from the centre, that sample is half the
    central one; the half-maximum crossing of the continuous profile, found by
    bisection, lies at FWHM/2."""
    for fwhm, h, k in [(0.1, 0.01, 5), (0.12, 0.02, 3), (0.3, 0.025, 6)]:
        taps = psf.psf_taps(fwhm, h)
        r = (taps.size - 1) // 2
        assert math.isclose(k * h, fwhm / 2, rel_tol=1e-12)
        assert math.isclose(taps[r + k] / taps[r], 0.5, rel_tol=1e-12)
        assert math.isclose(taps[r - k] / taps[r], 0.5, rel_tol=1e-12)
        s = psf.psf_sigma(fwhm)
        lo, hi = 0.0, 10 * fwhm
        for _ in range(200):  # profile(x) = 1/2 by bisection on x
            mid = 0.5 * (lo + hi)
            lo, hi = (mid, hi) if math.exp(-mid * mid / (2 * s * s)) > 0.5 else (lo, mid)
        assert math.isclose(2 * lo, fwhm, rel_tol=1e-12)


def test_psf_brute_force_and_constant():
    taps = psf.psf_taps(0.1, 0.05)
    r = (taps.size - 1) // 2
    rng = np.random.default_rng(6)
    M = 9
    img = rng.standard_normal((M, M))
    out = psf.conv_same(img, taps)
    for (y, x) in [(0, 0), (4, 4), (8, 2)]:
        s = 0.0
        for a in range(-r, r + 1):
            for b in range(-r, r + 1):
                if 0 <= y - a < M and 0 <= x - b < M:
                    s += taps[a + r] * taps[b + r] * img[y - a, x - b]
        assert math.isclose(out[y, x], s, rel_tol=1e-13)
    const = psf.conv_same(np.ones((20, 20)), taps)
    assert np.allclose(const[r:-r, r:-r], 1.0, rtol=1e-14)
    # no PSF: B is the plain block mean
    f = rng.standard_normal(36)
    assert np.allclose(psf.apply_B(f, 3, 2, psf.psf_taps(0.0, 0.025)), grid.block_mean(f, 3, 2))


# ---------------------------------------------------------------- evidence (a6-a8)

def _tiny_problem(n=8, ss=2, fwhm=0.1, seed=0, cx=0.0, cy=0.0):
    w = synth.workload(1)
    P = evidence.Problem(n, ss, 0.05, w.lens.as_tuple(), (0.6, 0.1, 1.5, 0.02, -0.01), 0.04, 0.3, 0.02, fwhm,
                         cx, cy)
    d, _ = data.simulate(P, synth.noise_normals(n * n, 9, seed), gp_normals=synth.gp_normals(P.N, 9, seed))
    return P, d


def test_evidence_matches_scipy_mvn_logpdf():
    """The sign reading of eq. gp-mll: ln p equals the Gaussian log-density of d."""
    P, d = _tiny_problem()
    out = evidence.solve_problem(P, d, want_mean=False)
    A = out["A"]
    want = st.multivariate_normal(mean=P.B(out["mu"]), cov=A).logpdf(d)
    assert math.isclose(out["lnp"], want, rel_tol=1e-12)
    assert math.isclose(out["logdet"], np.linalg.slogdet(A)[1], rel_tol=1e-12)
    # A built blockwise equals the dense B K B^T + sigma^2 I
    Bd = psf.B_matrix(P.n, P.ss, P.taps())
    Kd = kernel.rbf_matrix(out["px"], out["py"], P.ell, P.amp)
    assert np.allclose(A, Bd @ Kd @ Bd.T + P.sigma ** 2 * np.eye(P.n_pix), rtol=1e-12, atol=1e-15)


def test_sherman_morrison_block_constant():
    """App. D.1: clumps of Nc perfectly correlated points, K block = alpha^2 u u^T, B = I.
    (S0 + alpha^2 u u^T)^{-1} = sigma^-2 [I - alpha^2/(sigma^2 + Nc alpha^2) u u^T]."""
    Nc, nb, a, s = 5, 4, 0.3, 0.02
    K = np.kron(np.eye(nb), a * a * np.ones((Nc, Nc)))
    A = K + s * s * np.eye(Nc * nb)
    d = np.random.default_rng(7).standard_normal(Nc * nb)
    ev = evidence.exact_evidence(A, d)
    quad_cf = 0.0
    for b in range(nb):
        db = d[b * Nc:(b + 1) * Nc]
        quad_cf += (db @ db - a * a / (s * s + Nc * a * a) * db.sum() ** 2) / (s * s)
    logdet_cf = nb * ((Nc - 1) * math.log(s * s) + math.log(s * s + Nc * a * a))
    assert math.isclose(ev["quad"], quad_cf, rel_tol=1e-12)
    assert math.isclose(ev["logdet"], logdet_cf, rel_tol=1e-12)


def test_vi_objective_forms_and_golden_variance():
    """App. D.1: the simplified loss equals quad + ln|Omega^2| - ln|Sigma_y| + N ln sigma^2;
    the variance limit reproduces the theory lines printed in Fig. vigp."""
    assert math.isclose(evidence.vi_objective(123.4, 1000, 0.3, 0.02),
                        evidence.vi_objective_full(123.4, 1000, 0.3, 0.02), rel_tol=1e-13)
    for a1, a2, s, want in _golden("vigp_variance.txt"):
        got = math.sqrt(evidence.diag_variance_limit([a1, a2], s).sum())
        assert abs(got - want) < 5e-5


def test_posterior_mean_interpolation_limit():
    """B = I and sigma -> 0: the posterior mean interpolates the data."""
    P, d = _tiny_problem(n=6, ss=1, fwhm=0.0)
    P.sigma = 1e-5
    out = evidence.solve_problem(P, d)
    assert np.allclose(out["fhat"], d, atol=1e-6)


# ---------------------------------------------------------------- Krylov (a6, a7)

def _spd(n=40, seed=8):
    rng = np.random.default_rng(seed)
    p = rng.uniform(-0.2, 0.2, (2, n))
    return kernel.rbf_matrix(p[0], p[1], 0.1, 1.0) + 0.05 * np.eye(n)


def test_cg_equals_direct_solve():
    A = _spd()
    b = np.random.default_rng(9).standard_normal((40, 3))
    res = krylov.cg(lambda X: A @ X, b, tol=1e-12, max_iter=500)
    assert np.allclose(res["X"], np.linalg.solve(A, b), rtol=1e-9, atol=1e-10)
    assert np.all(res["relres"] <= 1e-12)


def test_cg_single_precision_vectors():
    """The FP32-vector variant: on a well-conditioned system it reaches the
    direct solve to FP32 accuracy, its vectors stay float32, and its first step
    (x_1 = alpha b, alpha = b.b / b.Ab) matches the closed form."""
    A = _spd()
    b = np.random.default_rng(9).standard_normal((40, 3))
    seen = []

    def amul(X):
        seen.append(X.dtype)
        return (A.astype(np.float32) @ X).astype(np.float32)

    res = krylov.cg(amul, b, tol=1e-6, max_iter=500, vec_dtype=np.float32)
    assert all(t == np.float32 for t in seen)
    x = np.linalg.solve(A, b)
    assert np.all(np.linalg.norm(res["X"] - x, axis=0) <= 1e-5 * np.linalg.norm(x, axis=0))
    one = krylov.cg(amul, b, fixed_iters=1, vec_dtype=np.float32)
    b32 = b.astype(np.float32).astype(np.float64)
    alpha = np.sum(b32 * b32, axis=0) / np.sum(b32 * (A @ b32), axis=0)
    assert np.allclose(one["X"], alpha * b32, rtol=1e-6)


def test_cg_tridiagonal_equals_explicit_lanczos():
    A = _spd()
    z = synth.rademacher(40, 1, 0)[:, 0]
    m = 12
    res = krylov.cg(lambda X: A @ X, z, tol=0.0, fixed_iters=m, n_lanczos=m)
    d1, o1 = krylov.cg_tridiagonal(res["alphas"][0], res["betas"][0], m)
    d2, o2 = krylov.lanczos(lambda X: A @ X, z, m)
    assert np.allclose(d1, d2, rtol=1e-10) and np.allclose(o1, np.abs(o2), rtol=1e-10)


def test_slq_all_unit_probes_is_exact():
    A = _spd(n=30)
    n = 30
    E = np.eye(n)
    res = krylov.cg(lambda X: A @ X, E, tol=0.0, fixed_iters=n, n_lanczos=n)
    est, _, _ = krylov.slq_logdet(res["alphas"], res["betas"], res["iters"], res["bnorm2"], n, scale=1.0)
    assert math.isclose(est, np.linalg.slogdet(A)[1], rel_tol=1e-10)


# ---------------------------------------------------------------- preconditioned solves and log-det

def test_pivoted_cholesky_exact_at_full_rank_and_greedy():
    M = _spd(n=40, seed=11) - 0.05 * np.eye(40)  # the kernel part, PSD
    L, piv = precond.pivoted_cholesky(M, 40)
    assert np.allclose(L @ L.T, M, rtol=0, atol=1e-12 * np.abs(M).max())
    # lower triangular in pivot order, first pivot the largest diagonal entry
    Lp = L[piv]
    assert np.allclose(np.triu(Lp, 1), 0.0)
    assert piv[0] == int(np.argmax(np.diag(M)))
    # a partial factor is exact on its pivot rows and columns and leaves a PSD rest
    L6, piv6 = precond.pivoted_cholesky(M, 6)
    assert np.allclose((L6 @ L6.T)[:, piv6], M[:, piv6], atol=1e-12)
    assert np.linalg.eigvalsh(M - L6 @ L6.T).min() > -1e-12
    # the second pivot maximises the residual diagonal after the first step
    L1, _ = precond.pivoted_cholesky(M, 1)
    assert piv6[1] == int(np.argmax(np.diag(M - L1 @ L1.T)))


def test_lowrank_logdet_and_woodbury():
    rng = np.random.default_rng(12)
    L = rng.standard_normal((50, 7))
    s = 0.3
    P = L @ L.T + s * np.eye(50)
    assert math.isclose(precond.logdet_lowrank_plus_shift(L, s), np.linalg.slogdet(P)[1], rel_tol=1e-12)
    V = rng.standard_normal((50, 3))
    assert np.allclose(P @ precond.woodbury_solver(L, s)(V), V, rtol=1e-10, atol=1e-10)


def test_pcg_solves_and_reduces_to_cg():
    A = _spd(n=60, seed=13)
    b = np.random.default_rng(14).standard_normal((60, 2))
    x = np.linalg.solve(A, b)
    M = A - 0.05 * np.eye(60)
    L, _ = precond.pivoted_cholesky(M, 10)
    res = precond.pcg(lambda X: A @ X, precond.woodbury_solver(L, 0.05), b, tol=1e-12, max_iter=200)
    assert np.allclose(res["X"], x, rtol=1e-9, atol=1e-10)
    exact = precond.pcg(lambda X: A @ X, lambda R: np.linalg.solve(A, R), b, tol=1e-12, max_iter=5)
    assert np.all(exact["iters"] == 1)  # M = A: one step
    plain = krylov.cg(lambda X: A @ X, b, tol=1e-12, max_iter=200, n_lanczos=20)
    ident = precond.pcg(lambda X: A @ X, lambda R: R.copy(), b, tol=1e-12, max_iter=200, n_lanczos=20)
    assert np.allclose(ident["alphas"], plain["alphas"]) and np.allclose(ident["betas"], plain["betas"])
    assert np.allclose(ident["rz0"], plain["bnorm2"])


def test_preconditioned_slq_whitened_unit_probes_is_exact():
    """Probes P^{1/2} e_j for every j with full-length PCG: the estimate is
    ln|P| + tr ln(P^{-1/2} A P^{-1/2}) = ln|A| exactly."""
    n = 30
    A = _spd(n=n, seed=15)
    s = 0.05
    L, _ = precond.pivoted_cholesky(A - s * np.eye(n), 5)
    P = L @ L.T + s * np.eye(n)
    w, V = np.linalg.eigh(P)
    Z = (V * np.sqrt(w)) @ V.T  # P^{1/2} e_j as columns
    res = precond.pcg(lambda X: A @ X, precond.woodbury_solver(L, s), Z, tol=0.0, fixed_iters=n, n_lanczos=n)
    est, _, _ = precond.preconditioned_slq_logdet(res["alphas"], res["betas"], res["iters"], res["rz0"], n,
                                                  precond.logdet_lowrank_plus_shift(L, s))
    # scale: slq_logdet averages over m probes; whitened unit probes sum, so times n
    ld_rest = (est - precond.logdet_lowrank_plus_shift(L, s)) * n
    assert math.isclose(precond.logdet_lowrank_plus_shift(L, s) + ld_rest, np.linalg.slogdet(A)[1], rel_tol=1e-10)


def test_preconditioned_probes_have_covariance_P():
    rng = np.random.default_rng(16)
    n, k, m = 40, 6, 20000
    L = rng.standard_normal((n, k))
    s = 0.2
    Z = precond.probes_from(L, s, rng.standard_normal((k, m)), rng.standard_normal((n, m)))
    P = L @ L.T + s * np.eye(n)
    C = Z @ Z.T / m
    assert np.max(np.abs(C - P)) <= 5 * np.sqrt(2.0 / m) * np.max(np.diag(P))
    q = np.sum(Z * np.linalg.solve(P, Z), axis=0)  # chi-square with n degrees of freedom
    assert abs(q.mean() - n) <= 5 * math.sqrt(2 * n / m)


def test_slq_rademacher_within_stderr():
    A = _spd(n=200, seed=10)
    Z = synth.rademacher(200, 64, 1)
    res = krylov.cg(lambda X: A @ X, Z, tol=1e-10, max_iter=400, n_lanczos=60)
    est, se, _ = krylov.slq_logdet(res["alphas"], res["betas"], res["iters"], res["bnorm2"], 60)
    exact = np.linalg.slogdet(A)[1]
    assert abs(est - exact) < 4 * se
    # predicted standard error from the exact off-diagonal of ln A
    w, V = np.linalg.eigh(A)
    lnA = (V * np.log(w)) @ V.T
    pred = math.sqrt(2 * (np.sum(lnA ** 2) - np.sum(np.diag(lnA) ** 2)) / 64)
    assert 0.6 * pred < se < 1.6 * pred


# ---------------------------------------------------------------- gradients (a10)

def test_gradients_analytic_vs_finite_differences():
    """A crop on the Einstein ring (away from the lens centre, where the central
    differences of both the stencil and the evidence stay accurate). The step
    h = 1e-4 leaves a truncation error of order (h/ell)^2 ~ 1e-5 in the ell entry."""
    P, d = _tiny_problem(n=6, ss=2, cx=0.9, cy=0.5)
    an = gradients.analytic_gradient(P, d)
    fl, fv = gradients.fd_gradient(P, d, h=1e-4)
    for g_an, g_fd in ((an["grad_lnp"], fl), (an["grad_vi"], fv)):
        scale = np.maximum(np.abs(g_fd), 1e-3 * np.max(np.abs(g_fd)))
        assert np.max(np.abs(g_an - g_fd) / scale) < 2e-5, (g_an, g_fd)


def test_amplitude_gradient_identity():
    """alpha d ln p/d alpha = u^T B K B^T u - tr(A^{-1} B K B^T) (K is proportional to alpha^2)."""
    P, d = _tiny_problem(n=5, ss=2)
    an = gradients.analytic_gradient(P, d)
    out = evidence.solve_problem(P, d, want_mean=False)
    BKBt = out["A"] - P.sigma ** 2 * np.eye(P.n_pix)
    u = out["u"]
    want = u @ BKBt @ u - np.trace(np.linalg.solve(out["A"], BKBt))
    assert math.isclose(P.amp * an["grad_lnp"][11], want, rel_tol=1e-9)


# ---------------------------------------------------------------- data

def test_rff_draw_covariance_is_rbf():
    """Empirical covariance of many random-Fourier-feature draws approaches K."""
    px, py = np.array([0.0, 0.02, 0.05]), np.array([0.0, 0.01, -0.03])
    draws = []
    for k in range(3000):
        om, ph, w = synth.rff_draws(512, 0, sub=k)
        draws.append(data.gp_draw_rff(px, py, 0.04, 0.3, om, ph, w))
    cov = np.cov(np.array(draws).T)
    assert np.allclose(cov, kernel.rbf_matrix(px, py, 0.04, 0.3), atol=0.08 * 0.09)


# ---------------------------------------------------------------- pixel shapes, transmission (Sec. 3.2, 3.4, 3.5)

def test_windowed_kernel_reduces_to_rbf():
    """Z -> 0: eq. "covariance" is the RBF kernel of eq. "grbf"."""
    rng = np.random.default_rng(50)
    px, py = rng.uniform(-0.3, 0.3, (2, 60))
    K0 = window.windowed_kernel_matrix(px, py, np.zeros((60, 3)), 0.04, 0.3)
    assert np.allclose(K0, kernel.rbf_matrix(px, py, 0.04, 0.3), rtol=1e-13, atol=0)
    # and continuously: a tiny shape moves K by O(|Z| / l^2)
    Zt = np.tile([1e-9, 0.0, 1e-9], (60, 1))
    Kt = window.windowed_kernel_matrix(px, py, Zt, 0.04, 0.3)
    assert np.max(np.abs(Kt - K0)) <= 1e-4 * 0.09


def test_window_square_integral_is_inverse_area():
    """App. C: int w^2 = 1/|a x b| for Z = (a a^T + b b^T)/(4 pi), by quadrature."""
    rng = np.random.default_rng(51)
    for _ in range(4):
        a, b = rng.uniform(-1, 1, 2), rng.uniform(-1, 1, 2)
        Z = window.shape_cov(a[None], b[None])[0]
        area = abs(a[0] * b[1] - a[1] * b[0])
        s = math.sqrt(max(Z[0], Z[2]))
        t = np.linspace(-12 * s, 12 * s, 1601)
        X, Y = np.meshgrid(t, t)
        w = window.gauss2(X, Y, Z[0], Z[1], Z[2])
        integral = np.sum(w * w) * (t[1] - t[0]) ** 2
        assert math.isclose(integral, 1.0 / area, rel_tol=1e-6)


def test_windowed_covariance_is_the_double_integral():
    """Eq. "covariance" against its definition, eq. "windowing": the mean of the
    RBF kernel over independent draws from the two indicator Gaussians (Monte
    Carlo, 4e6 samples, within 5 standard errors)."""
    rng = np.random.default_rng(52)
    ell, amp = 0.04, 0.3
    pi_, pj = np.array([0.01, -0.02]), np.array([0.05, 0.03])
    Zi = window.shape_cov(np.array([[0.03, 0.01]]), np.array([[-0.005, 0.02]]))[0]
    Zj = window.shape_cov(np.array([[0.02, -0.015]]), np.array([[0.01, 0.025]]))[0]
    want = window.windowed_kernel_matrix(pi_[:1], pi_[1:], Zi[None], ell, amp, pj[:1], pj[1:], Zj[None])[0, 0]
    m = 4_000_000

    def draw(mu, Z):
        Lc = np.linalg.cholesky(np.array([[Z[0], Z[1]], [Z[1], Z[2]]]))
        return mu + rng.standard_normal((m, 2)) @ Lc.T

    x1, x2 = draw(pi_, Zi), draw(pj, Zj)
    k = amp * amp * np.exp(-np.sum((x1 - x2) ** 2, axis=1) / (2 * ell * ell))
    assert abs(k.mean() - want) <= 5 * k.std() / math.sqrt(m)


def test_pixel_axes_on_a_regular_grid():
    """An undeflected grid of spacing h: a = (h, 0), b = (0, h) everywhere,
    edges included; Z = h^2 I / (4 pi), whose indicator has area h^2."""
    h, M = 0.025, 7
    x, y = grid.fine_coords(M, 1, h)
    a, b = window.pixel_axes(x, y, M)
    assert np.allclose(a, [h, 0.0]) and np.allclose(b, [0.0, h])
    Z = window.shape_cov(a, b)
    assert np.allclose(Z, [h * h / (4 * math.pi), 0.0, h * h / (4 * math.pi)])
    # a sheared grid: the central difference of a linear map is exact inside
    J = np.array([[1.3, 0.4], [-0.2, 0.7]])
    P = (J @ np.stack([x, y])).T
    a2, b2 = window.pixel_axes(P[:, 0], P[:, 1], M)
    assert np.allclose(a2, J @ [h, 0.0]) and np.allclose(b2, J @ [0.0, h])


def test_windowed_kernel_symmetric_psd_on_lensed_grid():
    w = synth.workload(0)
    P = evidence.Problem(w.n, w.ss, w.pix_scale, w.lens.as_tuple(), (1.0, 0.1, 1.5, 0.0, 0.0), w.ell, w.amp,
                         w.noise_sigma, 0.0)
    px, py = P.points()
    a, b = window.pixel_axes(px, py, w.n * w.ss)
    K = window.windowed_kernel_matrix(px, py, window.shape_cov(a, b), w.ell, w.amp)
    assert np.array_equal(K, K.T)
    assert np.linalg.eigvalsh(K).min() >= -1e-12 * w.amp ** 2 * px.size
    # the pixel shapes widen the kernel: K_ii = alpha^2 l^2 / sqrt|2 Z_i + l^2 I| <= alpha^2
    assert np.all(np.diag(K) <= w.amp ** 2 * (1 + 1e-15))


def test_transmission_factorises_the_windowed_kernel():
    """Eq. "transmission": with inducing points on a dense regular grid of
    spacing s (density 1/s^2) covering the points, alpha^2 T T^T reproduces the
    windowed K (the sum over the grid is a converged Riemann sum of a Gaussian
    product)."""
    rng = np.random.default_rng(53)
    ell, amp = 0.04, 0.3
    px, py = rng.uniform(-0.05, 0.05, (2, 12))
    Z = window.shape_cov(rng.uniform(-0.01, 0.01, (12, 2)), rng.uniform(-0.01, 0.01, (12, 2)))
    s = ell / 5
    g = np.arange(-0.35, 0.35 + s / 2, s)
    qx, qy = [v.ravel() for v in np.meshgrid(g, g)]
    A = window.transmission_weights(np.full(qx.size, 1.0 / (s * s)), ell)
    T = window.transmission_matrix(px, py, Z, qx, qy, ell, A)
    K = window.windowed_kernel_matrix(px, py, Z, ell, amp)
    assert np.allclose(amp * amp * T @ T.T, K, rtol=1e-8, atol=1e-12)


def test_knn_density():
    """k-th neighbour density: a square lattice of spacing s has its 20th
    closest other point at sqrt(5) s (4 + 4 + 4 + 8 neighbours), so the estimate
    is 20 / (5 pi s^2) away from the edges; brute force on random points."""
    s = 0.03
    g = np.arange(15) * s
    qx, qy = [v.ravel() for v in np.meshgrid(g, g)]
    rho = window.knn_density(qx, qy, 20)
    centre = 7 * 15 + 7
    assert math.isclose(rho[centre], 20 / (5 * math.pi * s * s), rel_tol=1e-12)
    rng = np.random.default_rng(54)
    q = rng.uniform(0, 1, (2, 300))
    r = window.knn_density(q[0], q[1], 5)
    i = 17
    d = np.sort(np.hypot(q[0] - q[0, i], q[1] - q[1, i]))[1:]
    assert math.isclose(r[i], 5 / (math.pi * d[4] ** 2), rel_tol=1e-12)


def test_reconstruction_is_transmission_without_shapes():
    rng = np.random.default_rng(55)
    qx, qy = rng.uniform(-0.2, 0.2, (2, 40))
    A = window.transmission_weights(window.knn_density(qx, qy, 20), 0.04)
    yk = rng.standard_normal(40)
    x, y = rng.uniform(-0.2, 0.2, (2, 30))
    want = np.array([sum(A[k] * math.exp(-((x[i] - qx[k]) ** 2 + (y[i] - qy[k]) ** 2) / (2 * 0.0008)) /
                         (2 * math.pi * 0.0008) * yk[k] for k in range(40)) for i in range(30)])
    assert np.allclose(window.reconstruct_brightness(x, y, qx, qy, yk, 0.04, A), want, rtol=1e-12)


# ---------------------------------------------------------------- posterior at new points (f4)

def _posterior_problem(n, ss, fwhm, theta_e=0.6, ell=0.04, peak=0.0):
    return evidence.Problem(n, ss, 0.05, (theta_e, 0.8, 0.5, 2.0, 0.0, 0.0, 0.03, 0.0), (peak, 0.1, 1.5, 0.0, 0.0),
                            ell, 0.3, 0.02, fwhm)


def test_posterior_matches_sklearn_gp_regression():
    """No PSF, no supersampling (B = I) and a zero mean: the posterior mean and
    variance at new points are those of scikit-learn's Gaussian-process
    regressor with the same fixed RBF kernel and noise (an independent
    implementation of eqs. "gp-exact-mean" and "gp-exact-var")."""
    from sklearn.gaussian_process import GaussianProcessRegressor
    from sklearn.gaussian_process.kernels import RBF, ConstantKernel
    P = _posterior_problem(8, 1, 0.0)
    rng = np.random.default_rng(80)
    d = 0.3 * rng.standard_normal(P.n_pix)
    sol = evidence.solve_problem(P, d)
    q = rng.uniform(-0.35, 0.35, (2, 25))
    o = posterior.posterior_at(P, sol, q[0], q[1])
    gp = GaussianProcessRegressor(ConstantKernel(P.amp ** 2, "fixed") * RBF(P.ell, "fixed"), alpha=P.sigma ** 2,
                                  optimizer=None)
    gp.fit(np.stack([sol["px"], sol["py"]], 1), d)
    m, s = gp.predict(q.T, return_std=True)
    assert np.max(np.abs(m - o["mean"])) <= 1e-12
    assert np.max(np.abs(s * s - o["var"])) <= 1e-12
    assert o["var"].min() < 0.5 * P.amp ** 2  # some query points are informed by the data


def test_posterior_information_form_with_psf_and_supersampling():
    """B = D o P (PSF, 2x2 supersampling) and a Sersic mean: the joint posterior
    of the fluxes at the fitted points and the query points from the
    information form Cov = (K_all^{-1} + H^T H / sigma^2)^{-1}, H = [B 0], mean
    = mu_all + Cov H^T r / sigma^2 (Bayes' rule for a linear Gaussian model,
    a different route from the Cholesky of A)."""
    P = _posterior_problem(4, 2, 0.1, theta_e=0.02, ell=0.015, peak=0.2)
    rng = np.random.default_rng(81)
    d = 0.3 * rng.standard_normal(P.n_pix)
    sol = evidence.solve_problem(P, d)
    px, py = sol["px"], sol["py"]
    q = np.array([[0.0125, -0.0375, 0.03], [0.0125, 0.0125, -0.06]])
    o = posterior.posterior_at(P, sol, q[0], q[1])
    ax, ay = np.concatenate([px, q[0]]), np.concatenate([py, q[1]])
    Kall = kernel.rbf_matrix(ax, ay, P.ell, P.amp)
    assert np.linalg.cond(Kall) < 1e8
    Bm = psf.B_matrix(P.n, P.ss, P.taps())
    H = np.hstack([Bm, np.zeros((P.n_pix, q.shape[1]))])
    Lam = np.linalg.inv(Kall) + H.T @ H / P.sigma ** 2
    Cov = np.linalg.inv(Lam)
    mu_all = source.sersic(ax, ay, *P.src)
    r = d - Bm @ mu_all[:px.size]
    mean_all = mu_all + Cov @ H.T @ r / P.sigma ** 2
    G = q.shape[1]
    assert np.max(np.abs(mean_all[-G:] - o["mean"])) <= 1e-8 * np.max(np.abs(mean_all))
    assert np.max(np.abs(np.diag(Cov)[-G:] - o["var"])) <= 1e-8 * P.amp ** 2


def test_posterior_far_from_data_is_the_prior():
    """Far from every fitted point (hundreds of lengthscales) the kernel
    vanishes: the mean is the mean function and the variance is alpha^2."""
    P = _posterior_problem(6, 2, 0.1, peak=0.5)
    rng = np.random.default_rng(82)
    d = 0.3 * rng.standard_normal(P.n_pix)
    sol = evidence.solve_problem(P, d)
    q = np.array([[20.0, -20.0], [20.0, 5.0]])
    o = posterior.posterior_at(P, sol, q[0], q[1])
    assert np.array_equal(o["var"], np.full(2, P.amp ** 2))
    assert np.array_equal(o["mean"], source.sersic(q[0], q[1], *P.src))


# ---------------------------------------------------------------- variational GP source (f2, f3)

def _vigp_case(seed, n=6, ss=2, gn=8):
    rng = np.random.default_rng(seed)
    gx, gy = synth.source_grid(gn, 0.06)
    m = vigp.Model(n, ss, 0.05, 2.0, (0.2, 0.1, 1.5, 0.01, -0.02), 0.02, 0.1,
                   (("ip", 0.03), ("ip", 0.06), ("sp", 0.08)), gx, gy)
    N, G = m.N, m.G
    P = dict(lens_mean=np.array([0.6, 0.8, 0.5, 0.01, -0.02, 0.03, 0.01]) + 0.01 * rng.standard_normal(7),
             lens_raw=np.tril(0.003 * rng.standard_normal((7, 7)), -1) + np.diag(np.log(0.01 * (1 + 0.1 * rng.random(7)))),
             log_amp=np.log(np.array([0.02, 0.05, 0.2])),
             sp_mean=0.05 * rng.standard_normal(G), sp_logs=np.log(0.01 * (1 + rng.random(G))),
             sp_cross=0.01 * rng.standard_normal((G, 7)),
             ip_mean=[0.01 * rng.standard_normal(N) for _ in range(2)],
             ip_logs=[np.log(0.001 * (1 + rng.random(N))) for _ in range(2)])
    eps = dict(e_l=rng.standard_normal(7), e_sp=rng.standard_normal(G), e_ip=[rng.standard_normal(N) for _ in range(2)])
    d = 0.1 * rng.standard_normal(n * n) + 0.1
    return m, P, eps, d


def _perturbed(P, key, idx, h, li):
    Q = {k: ([x.copy() for x in v] if isinstance(v, list) else v.copy()) for k, v in P.items()}
    (Q[key][li] if li is not None else Q[key])[idx] += h
    return Q


def test_vigp_gradient_vs_finite_differences():
    """The analytic ELBO gradient (through ray tracing, pixel shapes, k-NN
    weights, both guide blocks and the amplitudes) against central differences
    of the oracle's own ELBO sample (h = 1e-6)."""
    m, P, eps, d = _vigp_case(0)
    E, _, g = vigp.elbo(m, P, eps, d, want_grad=True)
    assert np.isfinite(E)
    rng = np.random.default_rng(1)
    for key in ("lens_mean", "lens_raw", "log_amp", "sp_mean", "sp_logs", "sp_cross", "ip_mean", "ip_logs"):
        for trial in range(3):
            li = trial % 2 if key.startswith("ip_") else None
            arr = P[key][li] if li is not None else P[key]
            ga = g[key][li] if li is not None else g[key]
            if key == "lens_raw":
                a = int(rng.integers(0, 7))
                idx = (a, int(rng.integers(0, a + 1)))
            else:
                idx = tuple(int(rng.integers(0, k)) for k in arr.shape)
            h = 1e-6
            fd = (vigp.elbo(m, _perturbed(P, key, idx, h, li), eps, d)[0]
                  - vigp.elbo(m, _perturbed(P, key, idx, -h, li), eps, d)[0]) / (2 * h)
            assert abs(fd - ga[idx]) <= 2e-6 * max(1.0, abs(ga[idx])), (key, idx, fd, ga[idx])
    # every lens parameter, including x0, y0 (points near the lens centre)
    for i in range(7):
        h = 1e-6
        fd = (vigp.elbo(m, _perturbed(P, "lens_mean", i, h, None), eps, d)[0]
              - vigp.elbo(m, _perturbed(P, "lens_mean", i, -h, None), eps, d)[0]) / (2 * h)
        assert abs(fd - g["lens_mean"][i]) <= 2e-6 * max(1.0, abs(g["lens_mean"][i])), (i, fd, g["lens_mean"][i])


def test_vigp_sample_expectation_is_the_gaussian_elbo():
    """With the lens noise fixed, the ELBO sample is a quadratic in the
    source-parameter noise, so its mean over that noise follows exactly from
    2n + 1 evaluations; it must equal the textbook Gaussian ELBO: the expected
    log-likelihood of the linear model minus the KL divergence of the diagonal
    guide from the prior."""
    m, P, eps, d = _vigp_case(2, n=5, ss=1, gn=5)
    e_l = eps["e_l"]
    G, N = m.G, m.N

    def sample(z):
        e = dict(e_l=e_l, e_sp=z[:G], e_ip=[z[G:G + N], z[G + N:]])
        return vigp.elbo(m, P, e, d)[0]

    n = G + 2 * N
    q0 = sample(np.zeros(n))
    acc = q0
    for j in range(n):
        ej = np.zeros(n)
        ej[j] = 1.0
        acc += 0.5 * (sample(ej) + sample(-ej) - 2.0 * q0)
    want = vigp.expected_elbo_fixed_lens(m, P, e_l, d)
    assert abs(acc - want) <= 1e-9 * abs(want)


def test_vigp_adam_matches_torch():
    """Three Adam steps (torch's defaults, lr 1e-2) on changing gradients equal
    torch.optim.Adam minimising -E."""
    import torch
    m, P, eps, d = _vigp_case(3)
    rng = np.random.default_rng(4)
    keys = ("lens_mean", "lens_raw", "sp_mean", "ip_mean")
    params = {k: P[k] for k in keys}
    state = vigp.adam_init(params)
    tp = {k: ([torch.tensor(x, requires_grad=True) for x in v] if isinstance(v, list)
              else torch.tensor(v, requires_grad=True)) for k, v in params.items()}
    flat = [t for v in tp.values() for t in (v if isinstance(v, list) else [v])]
    opt = torch.optim.Adam(flat, lr=1e-2)
    for t in range(1, 4):
        grads = {k: ([rng.standard_normal(x.shape) for x in v] if isinstance(v, list)
                     else rng.standard_normal(v.shape)) for k, v in params.items()}
        grads["lens_raw"] = np.tril(grads["lens_raw"])
        params, state = vigp.adam_step(params, grads, state, t, 1e-2)
        for k, v in tp.items():
            for tv, gv in zip(v if isinstance(v, list) else [v], grads[k] if isinstance(v, list) else [grads[k]]):
                tv.grad = torch.tensor(-gv)
        opt.step()
    for k, v in tp.items():
        for tv, pv in zip(v if isinstance(v, list) else [v], params[k] if isinstance(v, list) else [params[k]]):
            assert np.allclose(tv.detach().numpy(), pv, rtol=0, atol=1e-14)


def test_pixel_axes_adjoint():
    """axes_backward is the transpose of the linear map p -> (a, b):
    <(a, b)(p), (ga, gb)> = <p, axes_backward(ga, gb)>."""
    rng = np.random.default_rng(5)
    for M in (1, 2, 3, 7):
        p = rng.standard_normal((M * M, 2))
        a, b = window.pixel_axes(p[:, 0], p[:, 1], M)
        ga, gb = rng.standard_normal((2, M * M, 2))
        lhs = np.sum(a * ga) + np.sum(b * gb)
        rhs = np.sum(p * vigp.axes_backward(ga, gb, M))
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_knn_radius_matches_density():
    rng = np.random.default_rng(6)
    q = rng.uniform(-1, 1, (2, 300))
    r, nn = window.knn_radius(q[0], q[1], 20)
    assert np.allclose(20 / (math.pi * r * r), window.knn_density(q[0], q[1], 20), rtol=1e-12)
    assert np.allclose(np.hypot(q[0] - q[0][nn], q[1] - q[1][nn]), r, rtol=1e-14)
