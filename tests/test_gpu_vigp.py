"""The variational GP source step (single-sample ELBO, its gradient, Adam)
through the C-ABI against the FP64 oracle, on the same inputs: the same guide
parameters (rounded to FP32 where the library holds them in FP32), the same
noise draws, and the oracle evaluated at the library's FP32 traced points.

Bounds. The library sums in FP32 (products over all pairs) and folds scalars
in FP64. The residual r = d - B f cancels: |f| is up to ~25x |r| here, so FP32
rounding of f (~1e-7 relative over a few hundred terms) reaches ~3e-6 of r, and
every gradient is linear in r. Blocks are therefore compared by the norm of
their error relative to the norm of the block, within 1e-4 (30x that
estimate); scalars of the ELBO within 1e-6 of the sum of the magnitudes of its
pieces (FP64 folds of FP32 terms)."""
import math

import numpy as np
import pytest

import synth
from oracle import vigp as ov

from helpers import gpu_problem, observation

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


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


LAYERS = (("ip", 0.025), ("ip", 0.05), ("sp", 0.1))


def _setup(G, n, ss, gn, spacing, seed, layers=LAYERS):
    w, d, _ = observation(1, n=n, ss=ss)
    prob = gpu_problem(w)
    gx, gy = synth.source_grid(gn, spacing)
    gx, gy = f32(gx), f32(gy)
    lens = np.array(w.lens.as_tuple())
    om = ov.Model(n, ss, w.pix_scale, lens[3], (w.source.peak, w.source.R_e, w.source.n_sersic, w.source.xs,
                                               w.source.ys), w.noise_sigma, w.psf_fwhm, layers, gx, gy)
    gm = G.vigp.VigpModel(layers, lens[3])
    N = w.N
    Gn = gx.size
    rng = np.random.default_rng(seed)
    nip = sum(1 for k, _ in layers if k == "ip")
    has_sp = any(k == "sp" for k, _ in layers)
    P = dict(lens_mean=lens[list(ov.FREE)] + 0.005 * rng.standard_normal(7),
             lens_raw=np.tril(0.002 * rng.standard_normal((7, 7)), -1) + np.diag(np.full(7, math.log(0.005))),
             log_amp=np.log(np.array([0.02 if k == "ip" else 0.2 for k, _ in layers])),
             ip_mean=[f32(0.01 * rng.standard_normal(N)) for _ in range(nip)],
             ip_logs=[f32(np.log(0.001 * (1 + rng.random(N)))) for _ in range(nip)])
    eps = dict(e_l=rng.standard_normal(7), e_ip=[f32(rng.standard_normal(N)) for _ in range(nip)])
    if has_sp:
        P.update(sp_mean=f32(0.05 * rng.standard_normal(Gn)), sp_logs=f32(np.log(0.01 * (1 + rng.random(Gn)))),
                 sp_cross=f32(0.01 * rng.standard_normal((Gn, 7))))
        eps["e_sp"] = f32(rng.standard_normal(Gn))
    dev = "cuda"
    v = G.vigp.Vigp(gm, prob, torch.as_tensor(d, dtype=torch.float32, device=dev),
                    torch.as_tensor(gx, dtype=torch.float32, device=dev) if has_sp else None,
                    torch.as_tensor(gy, dtype=torch.float32, device=dev) if has_sp else None)
    v.lens_mean.copy_(torch.as_tensor(P["lens_mean"]))
    v.lens_raw.copy_(torch.as_tensor(P["lens_raw"]))
    v.log_amp.copy_(torch.as_tensor(P["log_amp"]))
    for blk, m, ls in zip(v.ip, P["ip_mean"], P["ip_logs"]):
        blk["mean"].copy_(torch.as_tensor(m))
        blk["logs"].copy_(torch.as_tensor(ls))
    e32 = []
    if has_sp:
        v.sp["mean"].copy_(torch.as_tensor(P["sp_mean"]))
        v.sp["logs"].copy_(torch.as_tensor(P["sp_logs"]))
        v.sp["cross"].copy_(torch.as_tensor(P["sp_cross"].T))
        e32.append(eps["e_sp"])
    e32 += eps["e_ip"]
    e64 = torch.as_tensor(eps["e_l"], dtype=torch.float64, device=dev)
    e32 = torch.as_tensor(np.concatenate(e32), dtype=torch.float32, device=dev)
    return w, d, prob, om, P, eps, v, e64, e32


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


@pytest.mark.parametrize("n,ss,gn", [(12, 2, 20), (16, 1, 24)])
def test_vigp_elbo_and_gradient_vs_oracle(G, n, ss, gn):
    """Two image-plane layers and a source-plane grid: the sampled lens, the
    ELBO pieces and every gradient block."""
    _say("vigp elbo", n, ss, gn)
    w, d, prob, om, P, eps, v, e64, e32 = _setup(G, n, ss, gn, 0.04, 90 + n)
    out = t64(v.elbo(e64, e32))
    theta = out[5:13]
    pts = G.ops.lens_raytrace(prob.grid, G.Lens(*theta))
    E, pc, g = ov.elbo(om, P, eps, d, want_grad=True, points=(t64(pts[0]), t64(pts[1])))
    assert np.max(np.abs(theta - pc["theta"])) <= 1e-12 * np.max(np.abs(pc["theta"]))
    mag = abs(pc["loglik"]) + abs(pc["logprior_y"]) + abs(pc["logprior_theta"]) + abs(pc["neg_logq"])
    errs = [abs(out[0] - E), abs(out[1] - pc["loglik"]), abs(out[2] - pc["logprior_y"]),
            abs(out[3] - pc["logprior_theta"]), abs(out[4] - pc["neg_logq"])]
    print(f"E gpu {out[0]:.6f} oracle {E:.6f}; piece errors {[f'{e:.2e}' for e in errs]} (scale {mag:.3e})")
    assert max(errs) <= 1e-6 * mag
    G64, G32 = t64(v.G64), t64(v.G32)
    rep = {}
    rep["lens_mean"] = _rel(G64[0:7], g["lens_mean"])
    rep["lens_raw"] = _rel(np.tril(G64[7:56].reshape(7, 7)), np.tril(g["lens_raw"]))
    rep["log_amp"] = _rel(G64[56:], g["log_amp"])
    o = 0
    Gn = om.G
    if "sp_mean" in g:
        rep["sp_mean"] = _rel(G32[0:Gn], g["sp_mean"])
        rep["sp_logs"] = _rel(G32[Gn:2 * Gn], g["sp_logs"])
        rep["sp_cross"] = _rel(G32[2 * Gn:9 * Gn].reshape(7, Gn).T, g["sp_cross"])
        o = 9 * Gn
    N = om.N
    for i, (gm, gl) in enumerate(zip(g["ip_mean"], g["ip_logs"])):
        rep[f"ip{i}_mean"] = _rel(G32[o:o + N], gm)
        rep[f"ip{i}_logs"] = _rel(G32[o + N:o + 2 * N], gl)
        o += 2 * N
    print("relative errors:", {k: f"{x:.2e}" for k, x in rep.items()})
    assert max(rep.values()) <= 1e-4


def test_vigp_adam_vs_oracle(G):
    """The Adam kernel fed the oracle's gradient: the parameter blocks after
    two steps equal the oracle's Adam (FP64 block to 1e-14 relative, FP32
    block to FP32 rounding of each update)."""
    _say("vigp adam")
    w, d, prob, om, P, eps, v, e64, e32 = _setup(G, 10, 1, 16, 0.05, 95)
    state = ov.adam_init(P)
    params = P
    for t in (1, 2):
        _, _, g = ov.elbo(om, params, eps, d, want_grad=True)
        gl = dict(g)
        gl["lens_raw"] = np.tril(g["lens_raw"])
        v.G64.copy_(torch.as_tensor(np.concatenate([g["lens_mean"], gl["lens_raw"].ravel(), g["log_amp"]])))
        parts = [g["sp_mean"], g["sp_logs"], g["sp_cross"].T.ravel()]
        for gm, gs in zip(g["ip_mean"], g["ip_logs"]):
            parts += [gm, gs]
        v.G32.copy_(torch.as_tensor(np.concatenate(parts), dtype=torch.float32))
        gl_r = {k: ([f32(x) for x in val] if isinstance(val, list) else
                    (val if k in ("lens_mean", "lens_raw", "log_amp") else f32(val))) for k, val in gl.items()}
        params, state = ov.adam_step(params, gl_r, state, t, 1e-2)
        v.adam(1e-2)
    torch.cuda.synchronize()
    P64 = t64(v.P64)
    want64 = np.concatenate([params["lens_mean"], np.where(np.tril(np.ones((7, 7))) > 0, params["lens_raw"],
                                                           P["lens_raw"]).ravel(), params["log_amp"]])
    assert np.max(np.abs(P64 - want64)) <= 1e-14 * np.max(np.abs(want64))
    P32 = t64(v.P32)
    want32 = np.concatenate([params["sp_mean"], params["sp_logs"], params["sp_cross"].T.ravel()]
                            + [x for pair in zip(params["ip_mean"], params["ip_logs"]) for x in pair])
    # each step moves a parameter by at most lr (1e-2); FP32 rounding of the
    # parameter and of the step
    assert np.max(np.abs(P32 - want32) / (np.abs(want32) + 1e-2)) <= 1e-6


def test_vigp_steps_raise_the_elbo(G):
    """Forty Adam steps (lr 1e-3, fresh noise each step) on the 12 x 12 image
    raise the mean ELBO of the last ten steps above that of the first ten: the
    gradient points uphill end to end."""
    _say("vigp steps")
    w, d, prob, om, P, eps, v, e64, e32 = _setup(G, 12, 2, 16, 0.05, 97)
    rng = np.random.default_rng(98)
    vals = []
    for t in range(40):
        e64.copy_(torch.as_tensor(rng.standard_normal(7)))
        e32.copy_(torch.as_tensor(rng.standard_normal(e32.numel()), dtype=torch.float32))
        vals.append(float(v.step(e64, e32, 1e-3)[0].item()))
    assert all(np.isfinite(vals))
    print(f"ELBO first ten {np.mean(vals[:10]):.3f} last ten {np.mean(vals[-10:]):.3f}")
    assert np.mean(vals[-10:]) > np.mean(vals[:10])
