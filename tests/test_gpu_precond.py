"""The partial pivoted Cholesky preconditioner, preconditioned CG and the
preconditioned SLQ evidence (through the C-ABI) against the FP64 oracle.

The GPU's pivot order is handed to the oracle, which rebuilds the factor from
the exact matrix for that order; the order itself is checked against the
selection rule (block candidates are the largest residual diagonal entries)."""
import math
import os

import numpy as np
import pytest

import synth
from oracle import evidence as oev
from oracle import precond as opc

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


def _normals(n, k, m, seed):
    g, h = synth.preconditioned_probe_normals(n, k, m, 0, seed)
    return (torch.as_tensor(g, dtype=torch.float64, device="cuda"),
            torch.as_tensor(h, dtype=torch.float32, device="cuda"))


def _small_case(G, k, prec):
    w, d, _ = observation(0)
    prob = gpu_problem(w)
    pts = G.ops.lens_raytrace(prob.grid, prob.lens)
    pc = G.ops.pchol(prob, pts[0], pts[1], k, prec=prec)
    torch.cuda.synchronize()
    P = oracle_problem(w)
    A = oev.assemble_A(P, t64(pts[0]), t64(pts[1]))
    M = A - w.noise_sigma ** 2 * np.eye(w.n_pix)
    return w, d, prob, pts, pc, A, M


@pytest.mark.parametrize("prec", ["fp32", "f16x3"])
def test_pchol_factor_vs_oracle(G, prec):
    """24x24 workload, rank 128 (two blocks). The columns of M come from the
    library's product (FP32 or precision form, ~5e-7 relative), and a partial
    Cholesky factor amplifies such perturbations by the inverse of its smaller
    pivots, so the factor is checked by what it must satisfy for the pivots it
    chose: L L^T reproduces the pivot columns of the exact M (interpolation, to
    the product's accuracy); the leading columns (largest pivots) match the
    oracle's factor for the same pivot order; ln|P| equals the determinant
    lemma on the returned factor and nearly the oracle's; the inverse of
    sigma^2 I + L^T L is exact; the selection rule holds."""
    k = 128
    _say("pchol vs oracle", prec, k)
    w, d, prob, pts, pc, A, M = _small_case(G, k, prec)
    assert int(pc["info"].item()) == 0
    piv = pc["pivots"].cpu().numpy()
    taken = piv >= 0
    Lg = t64(pc["L"]).T  # (n_pix, k)
    assert np.all(Lg[:, ~taken] == 0.0)
    assert len(set(piv[taken].tolist())) == int(taken.sum())
    Lgt = Lg[:, taken]
    S = piv[taken]
    dmax = np.max(np.diag(M))
    interp = np.max(np.abs((Lgt @ Lgt[S].T) - M[:, S])) / dmax
    Lo, _ = opc.pivoted_cholesky(M, int(taken.sum()), pivots=S)
    err_lead = np.max(np.abs(Lgt[:, :8] - Lo[:, :8])) / math.sqrt(dmax)
    print(f"taken {taken.sum()} of {k}; pivot columns of L L^T vs M {interp:.2e}; leading columns {err_lead:.2e}")
    assert interp <= 2e-6
    assert err_lead <= 2e-5
    s = w.noise_sigma ** 2
    ldp = float(pc["logdet_P"].item())
    # ln|P| is exact for the factor returned; against the oracle's factor for
    # the same pivots it moves by what the smaller pivots amplify (the SLQ part
    # of the estimate corrects for whichever P is used)
    ld_o = opc.logdet_lowrank_plus_shift(Lo, s)
    print(f"ln|P| {ldp:.6f}, oracle factor {ld_o:.6f}")
    assert math.isclose(ldp, opc.logdet_lowrank_plus_shift(Lg, s), rel_tol=1e-10)
    assert math.isclose(ldp, ld_o, rel_tol=1e-4)
    Gf = t64(pc["G"]).T
    Gm = s * np.eye(k) + Lg.T @ Lg
    Gi = np.tril(Gf) + np.tril(Gf, -1).T  # the inverse, from its lower triangle
    assert np.allclose(Gi @ Gm, np.eye(k), rtol=0, atol=1e-9)
    # selection rule: the first block's pivots are among the 64 largest diagonal
    # entries of M (ranked in FP32; rounding may swap entries at the boundary),
    # the first pivot is the largest, and the first pivot of the second block is
    # the largest residual diagonal entry after the first block
    top = set(np.argsort(-np.diag(M).astype(np.float32), kind="stable")[:64].tolist())
    first = set(piv[:64][piv[:64] >= 0].tolist())
    assert len(first & top) >= len(first) - 2
    assert piv[0] == int(np.argmax(np.diag(M)))
    j = int(taken[:64].sum())
    r = np.diag(M) - np.sum(Lgt[:, :j] ** 2, axis=1)
    assert r[piv[64]] >= (1 - 1e-3) * r.max()


def test_pchol_full_rank_is_the_matrix(G):
    """Rank = every pixel (24x24 = 576 = 9 blocks): the pivots taken reproduce
    their columns of A, the residual diagonal of M - L L^T is below the
    threshold (1e-5 of the largest diagonal entry) up to rounding, and
    preconditioned CG then converges in a few steps."""
    k = 576
    _say("pchol full rank")
    w, d, prob, pts, pc, A, M = _small_case(G, k, "fp32")
    assert int(pc["info"].item()) == 0
    piv = pc["pivots"].cpu().numpy()
    taken = piv >= 0
    Lg = t64(pc["L"]).T[:, taken]
    dmax = np.max(np.diag(M))
    interp = np.max(np.abs(Lg @ Lg[piv[taken]].T - M[:, piv[taken]])) / dmax
    resid = (np.diag(M) - np.sum(Lg ** 2, axis=1)) / dmax
    print(f"taken {taken.sum()} of {k}; pivot columns {interp:.2e}; residual diagonal {resid.max():.2e}")
    assert interp <= 2e-6
    assert resid.max() <= 1e-4
    B = np.random.default_rng(40).standard_normal((w.n_pix, 2))
    res = G.ops.pcg_solve(prob, pts[0], pts[1], pc, cuda32(B.T), tol=1e-6, max_iter=50, n_lanczos=0, prec="fp32")
    print("pcg iterations", res["iters"].cpu().tolist())
    assert max(res["iters"].cpu().tolist()) <= 8


def test_pchol_rank_beyond_sixteen_splits(G):
    """Rank 4480 on a 72 x 72 image (5184 pixels): from the 69th block on, the
    residual columns' reduction over the earlier pivots (more than 16 x 256 of
    them) is split at most as far as its scratch holds. The pivots taken still
    reproduce their columns of M, the inverse of sigma^2 I + L^T L is exact, and
    ln|P| follows the determinant lemma."""
    k = 4480
    _say("pchol rank 4480", "72x72")
    w, d, _ = observation(0)
    w = w.replace(n=72)
    prob = gpu_problem(w)
    pts = G.ops.lens_raytrace(prob.grid, prob.lens)
    pc = G.ops.pchol(prob, pts[0], pts[1], k, prec="fp32")
    torch.cuda.synchronize()
    assert int(pc["info"].item()) == 0
    P = oracle_problem(w)
    A = oev.assemble_A(P, t64(pts[0]), t64(pts[1]))
    M = A - w.noise_sigma ** 2 * np.eye(w.n_pix)
    piv = pc["pivots"].cpu().numpy()
    taken = piv >= 0
    Lg = t64(pc["L"]).T[:, taken]
    dmax = np.max(np.diag(M))
    interp = np.max(np.abs(Lg @ Lg[piv[taken]].T - M[:, piv[taken]])) / dmax
    print(f"taken {taken.sum()} of {k}; pivot columns {interp:.2e}")
    # the last block starts at column 4416 > 16 x 256 whatever the candidates taken
    assert k - 64 > 16 * 256 and taken.sum() > 4000
    assert interp <= 2e-6
    s = w.noise_sigma ** 2
    Lall = t64(pc["L"]).T
    Gf = t64(pc["G"]).T
    Gm = s * np.eye(k) + Lall.T @ Lall
    Gi = np.tril(Gf) + np.tril(Gf, -1).T  # the inverse, from its lower triangle
    assert np.allclose(Gi @ Gm, np.eye(k), rtol=0, atol=1e-9)
    assert math.isclose(float(pc["logdet_P"].item()), opc.logdet_lowrank_plus_shift(Lall, s), rel_tol=1e-10)


@pytest.mark.parametrize("prec", ["fp32", "f16x3"])
def test_pcg_vs_oracle(G, prec):
    """Preconditioned CG with the GPU factor (rank 448) against the oracle's PCG
    with the same factor on the exact matrix: solutions against a direct solve,
    iteration counts, the first recurrence coefficients and the quadrature
    weights b^T P^{-1} b."""
    k = 448
    _say("pcg vs oracle", prec)
    w, d, prob, pts, pc, A, M = _small_case(G, k, prec)
    rng = np.random.default_rng(41)
    B = rng.standard_normal((w.n_pix, 5))
    res = G.ops.pcg_solve(prob, pts[0], pts[1], pc, cuda32(B.T), tol=1e-6, max_iter=300, n_lanczos=20, prec=prec)
    Lg = t64(pc["L"]).T
    s = w.noise_sigma ** 2
    B32 = B.astype(np.float32).astype(np.float64)
    o = opc.pcg(lambda X: A @ X, opc.woodbury_solver(Lg, s), B32, tol=1e-6, max_iter=300, n_lanczos=20)
    X = t64(res["X"]).T
    xs = np.linalg.solve(A, B32)
    errx = np.max(np.linalg.norm(X - xs, axis=0) / np.linalg.norm(xs, axis=0))
    it_g = res["iters"].cpu().numpy()
    print(f"pcg iters gpu {it_g.tolist()} oracle {o['iters'].tolist()}; solution error {errx:.2e}; true residual "
          f"{t64(res['true_relres']).max():.2e}")
    assert np.all(np.abs(it_g - o["iters"]) <= 1)
    assert errx <= 1e-4
    assert np.allclose(t64(res["rz0"]), o["rz0"], rtol=1e-5)
    # the first step's coefficients are well determined (later ones act on
    # residuals at the rounding level after one or two steps)
    ab = t64(res["ab"])
    assert np.allclose(ab[:, 0, 0], o["alphas"][:, 0], rtol=1e-4)
    assert np.allclose(ab[:, 0, 1], o["betas"][:, 0], rtol=1e-3, atol=1e-9)
    assert all(v == 0 for v in res["status"].cpu().tolist())


def test_preconditioned_evidence_small_vs_cholesky(G):
    """24x24 workload: the preconditioned estimate of ln p at rank 256 with 16
    probes against the exact Cholesky value, within 4 of its standard errors;
    quad within 1e-5; the image within 1e-4 of its maximum."""
    w, d, _ = observation(0)
    _say("preconditioned evidence 24x24")
    prob = gpu_problem(w)
    g, h = _normals(w.n_pix, 256, 16, 1)
    rec = G.reconstruct_preconditioned(prob, cuda32(d), g, h, rank=256, prec="f16x3")
    hh = rec.host()
    ex = oev.solve_problem(oracle_problem(w), d)
    print(f"lnp {hh['lnp']:.5f} exact {ex['lnp']:.5f}; logdet err {hh['logdet'] - ex['logdet']:.4f} stderr "
          f"{hh['stderr']:.4f}; iters {max(hh['iters'])}")
    assert all(s == 0 for s in hh["status"])
    assert abs(hh["quad"] - ex["quad"]) <= 1e-5 * ex["quad"]
    assert abs(hh["logdet"] - ex["logdet"]) <= 4 * hh["stderr"] + 1e-6 * abs(ex["logdet"])
    im = t64(rec.image)
    assert np.max(np.abs(im - ex["image"])) <= 1e-4 * np.max(np.abs(ex["image"]))


@pytest.mark.parametrize("prec", ["f16x3", "fp32"])
def test_preconditioned_evidence_full_size_1e4(G, prec):
    """The 100x100, ss = 2 workload (N = 40,000) at rank 4096 with 16 probes,
    for four probe seeds: ln p within 1e-4 relative of the stored exact
    Cholesky value every time, the SLQ standard error of ln p within 5e-5 of
    |ln p|, quad within 1e-5."""
    path = os.path.join(os.path.dirname(__file__), "fixtures", "workload1_draw0.npz")
    z = np.load(path)
    w = synth.workload(1)
    prob = gpu_problem(w)
    dd = cuda32(z["d"])
    lnp_ref = float(z["lnp"])
    for seed in range(4):
        _say("preconditioned evidence full size", prec, "seed", seed)
        g, h = _normals(w.n_pix, 4096, 16, 10 + seed)
        rec = G.reconstruct_preconditioned(prob, dd, g, h, rank=4096, prec=prec, want_image=(seed == 0))
        hh = rec.host()
        rel = abs(hh["lnp"] - lnp_ref) / abs(lnp_ref)
        se_rel = 0.5 * hh["stderr"] / abs(lnp_ref)
        quad_rel = abs(hh["quad"] - float(z["quad"])) / float(z["quad"])
        print(f"{prec} seed {seed}: lnp rel {rel:.2e} (SE {se_rel:.2e}); logdet err "
              f"{hh['logdet'] - float(z['logdet']):.3f}; quad rel {quad_rel:.2e}; iters {max(hh['iters'])}; "
              f"true residual {max(hh['true_relres']):.2e}")
        assert all(s == 0 for s in hh["status"])
        assert rel <= 1e-4
        assert se_rel <= 5e-5
        assert quad_rel <= 1e-5
        if seed == 0:
            im = t64(rec.image)
            assert np.max(np.abs(im - z["image"])) <= 1e-4 * np.max(np.abs(z["image"]))
