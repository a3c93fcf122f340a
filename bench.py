#!/usr/bin/env python
"""Throughput of the lensed-source GP evidence path on one MI355X.

One step = one full reconstruction of the 100x100-pixel image with 2x2
supersampling (N = 40,000 source points): ray tracing, Sersic mean, residual,
CG on the solve column plus 16 Rademacher probes (tolerance 1e-6), SLQ
log-determinant over every CG step of each probe, evidence scalars, posterior
mean and predicted image. The observation comes from the stored oracle simulation of
that workload; everything in the timed region runs in the HIP library with the
inputs already in HBM.

Prints one JSON line. `value` is the kernel-pair throughput of the whole step:
the kernel values the step's products evaluate (pairs below the 2^-36 cutoff
are not evaluated), over the step time; the dense equivalent (N^2 pairs per
product) is reported beside it. Extra fields: reconstructions/s of both
arithmetic forms, the roofline of the dominant kernel and of the FP32 form's
product, the preconditioned step, the 200 x 200 image (N = 160,000) with 64
columns in both forms, the exact posterior on a 40 x 40 source-plane grid, the variational GP source fit (Adam steps) with the
roofline of its transmission product, the serving trace, and the FP64 oracle
timed on the host as a baseline.

    python bench.py [--steps K] [--warmup W] [--prec f16x3|fp32]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FIXTURE = os.path.join(ROOT, "tests", "fixtures", "workload1_draw0.npz")
# Lanczos steps in the log-determinant quadrature: every CG step of each probe
# (at most the iteration cap). The 30-step quadrature the workload names is
# biased at this spectrum width; its error is reported next to it.
N_LANCZOS = 1000
# Every k-th product launch of the timed steps is timed with HIP events.
TIMING_STRIDE = 16
# Rank of the partial pivoted Cholesky preconditioner of the preconditioned step.
PC_RANK = 4096
METRIC = "kernel-MVM Gpairs/s at N=40k; reconstructions/s + p99 latency vs plain form"

# Peak of the plain ALUs for the exp tile: 256 CUs x
# 128 FP32 lanes x 2.4 GHz = 78.6 T FP32 VALU lane-ops/s (157.3 TFLOP/s counting
# an FMA as two); v_exp_f32 at a quarter of that rate. With the exp2 scale folded
# into the coordinates once per point, one kernel pair needs at least 4 FP32 VALU
# ops (two differences, two FMAs) and one exp, i.e. 4 + 4 = 8 FP32-op
# equivalents -> 78.6e12 / 8 pairs/s.
VALU_LANE_OPS = 256 * 128 * 2.4e9
PAIR_COST = 4 + 4
ALU_PEAK_GPAIRS = VALU_LANE_OPS / PAIR_COST / 1e9
# Dense FP32 MFMA peak of MI355X (the FP32 form's tile x RHS product).
FP32_MFMA_PEAK_TFLOPS = 157.3

# HBM traffic of the dominant kernel per launch at this workload, from rocprofv3
# FETCH_SIZE / WRITE_SIZE scaled by a copy-kernel calibration (profiles/), valid
# only for the kernel source it was measured on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "mvm_f16x3_traffic_N40000_17cols.txt")


def _source_hash():
    h = hashlib.sha256()
    for f in ("mvm_mfma.hip", "mvm_mfma.hpp", "tileplan.hpp", "tileplan.hip"):
        with open(os.path.join(ROOT, "paper_2105_09465_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic():
    try:
        vals = {}
        for line in open(TRAFFIC_FILE):
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
        if vals.get("source_sha256_16") != _source_hash():
            return None
        return float(vals["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def load_workload():
    import numpy as np

    import paper_2105_09465_amd as G
    z = np.load(FIXTURE)
    src = z["source"]
    prob = G.Problem(G.Grid(int(z["n"]), int(z["ss"]), float(z["pix_scale"])), G.Lens(*z["lens"].tolist()),
                     G.Sersic(*src.tolist()), G.Kernel(float(z["ell"]), float(z["amp"])), G.PSF(float(z["fwhm"])),
                     float(z["sigma"]))
    return prob, z


def cpu_baseline(prob, px, py, budget_s=15.0):
    """The FP64 oracle's matrix-free product on a sample of rows (same points,
    17 columns), on the host's cores; Gpairs/s scaled from the sample."""
    import numpy as np
    from oracle import kernel as okernel
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max((i.get("num_threads", 1) for i in threadpool_info()), default=1)
    except Exception:  # pragma: no cover
        blas_threads = 1
    N = px.size
    V = np.random.default_rng(0).standard_normal((N, 17))
    rows_done, t0 = 0, time.time()
    block = 1024
    while time.time() - t0 < budget_s and rows_done < N:
        rows = np.arange(rows_done, min(N, rows_done + block))
        okernel.kernel_mvm_rows(px, py, rows, V, prob.kernel.lengthscale, prob.kernel.amplitude)
        rows_done += rows.size
    dt = time.time() - t0
    return {"value": rows_done * N / dt / 1e9, "unit": "Gpairs/s", "cores": int(blas_threads), "kind": "oracle",
            "sample": f"{rows_done} of {N} rows of K V with 17 columns (FP64 numpy, oracle.kernel.kernel_mvm_rows; "
                      f"exp on 1 thread, products on {blas_threads} BLAS threads), {dt:.1f} s; host has "
                      f"{os.cpu_count()} logical CPUs"}


def mock_observation(G, torch, problem, noise, field):
    """A mock lensed image for a serving request (input generation, outside any
    timed region): the Sersic mean plus a smooth random field (the kernel
    product of white noise `field` with a kernel of lengthscale l/sqrt(2),
    rescaled to the kernel amplitude), observed through B, plus i.i.d. noise of
    the problem's sigma. Large requests would take the FP64 oracle minutes each,
    so the library draws these."""
    import dataclasses
    g = problem.grid
    pts = G.ops.lens_raytrace(g, problem.lens)
    mu = G.ops.sersic_eval(problem.source, pts[0], pts[1])
    wn = torch.as_tensor(field, dtype=torch.float32, device="cuda")
    k2 = dataclasses.replace(problem.kernel, lengthscale=problem.kernel.lengthscale / math.sqrt(2.0))
    gf = G.ops.kernel_mvm(k2, pts[0], pts[1], wn, prec="fp32", grid=g)
    gf = gf * (problem.kernel.amplitude / gf.std().clamp_min(1e-30))
    d = G.ops.psf_conv(g, problem.psf, mu + gf, adjoint=False)
    return d + problem.noise_sigma * torch.as_tensor(noise, dtype=torch.float32, device="cuda")


def serving_requests(G, torch, synth, n_requests, rate_hz=1.0):
    """n_requests requests with sides and supersampling from the serving trace,
    lens and source from the priors, a mock observation made by library calls,
    and 16 Rademacher probes each. Arrival times are set by the caller."""
    trace = synth.serving_trace(n_requests, rate_hz)
    reqs = []
    for k, (t, side, ss, seed) in enumerate(trace):
        w = synth.serving_request(side, ss, seed)
        s = w.source
        prob = G.Problem(G.Grid(w.n, w.ss, w.pix_scale), G.Lens(*w.lens.as_tuple()),
                         G.Sersic(s.peak, s.R_e, s.n_sersic, s.xs, s.ys), G.Kernel(w.ell, w.amp), G.PSF(w.psf_fwhm),
                         w.noise_sigma)
        d = mock_observation(G, torch, prob, synth.noise_normals(w.n_pix, 4, seed), synth.gp_normals(w.N, 4, seed))
        Z = torch.as_tensor(synth.rademacher(w.n_pix, 16, 4, seed).T.copy(), dtype=torch.float32, device="cuda")
        reqs.append(G.serving.Request(k, t, prob, d, Z))
    torch.cuda.synchronize()
    return reqs


def serve_section(G, torch, synth, n_requests):
    """Reconstructions of uneven sizes (sides 48..160 px, 1x1 or 2x2
    supersampling, lens and source from the priors, 16 probes each) through the
    continuous-batching engine, for both arithmetic forms:
    - capacity: every request available at once, reconstructions/s of the engine;
    - stream: Poisson arrivals at 0.8 x the plain FP32 capacity, with p50/p99
      latency from arrival to result.
    The scheduling overhead is the share of the capacity run's wall time not
    covered by the device time of the grouped CG steps (event pairs around each
    round's step), i.e. host waits, admission, snapshots and retirement."""
    reqs = serving_requests(G, torch, synth, n_requests)
    out = {"requests": n_requests, "hbm_budget_GiB": 8}
    for prec in ("fp32", "f16x3"):  # capacity: all present at the start, latency counted from there
        eng = G.serving.ServingEngine(prec=prec, hbm_budget=8 << 30)
        res = eng.run(reqs, realtime=False)
        s = G.serving.summarize(res, eng.stats["wall_s"])
        out[f"capacity_{prec}"] = {"reconstructions_per_s": s["reconstructions_per_s"], "wall_s": s["wall_s"],
                                   "p50_latency_ms": s["p50_latency_ms"], "p99_latency_ms": s["p99_latency_ms"],
                                   "max_active_slots": eng.stats["max_active"],
                                   "device_step_fraction": eng.stats["step_s"] / s["wall_s"],
                                   "scheduling_overhead": 1.0 - eng.stats["step_s"] / s["wall_s"],
                                   "rounds": eng.stats["rounds"],
                                   "lnp_slq_stderr_rel_median": s["lnp_slq_stderr_rel_median"]}
    rate = 0.8 * out["capacity_fp32"]["reconstructions_per_s"]
    trace = synth.serving_trace(n_requests, rate)
    for r, (t, _, _, _) in zip(reqs, trace):
        r.arrival = t
    out["arrival_rate_per_s"] = rate
    for prec in ("fp32", "f16x3"):
        eng = G.serving.ServingEngine(prec=prec, hbm_budget=8 << 30)
        res = eng.run(reqs, realtime=True)
        s = G.serving.summarize(res, eng.stats["wall_s"])
        s.update(max_active_slots=eng.stats["max_active"], rounds=eng.stats["rounds"],
                 device_step_s=eng.stats["step_s"],
                 nonconverged=int(sum(any(st != 0 for st in r.status) for r in res)))
        out[prec] = s
    out["capacity_ratio_f16x3_vs_fp32"] = (out["capacity_f16x3"]["reconstructions_per_s"] /
                                           out["capacity_fp32"]["reconstructions_per_s"])
    return out


def run_steps(G, torch, prob, d, probes, prec, steps, ws):
    recs, times = [], []
    for _ in range(steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        rec = G.reconstruct(prob, d, probes, prec=prec, tol=1e-6, max_iter=1000, n_lanczos=N_LANCZOS, ws=ws)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
        recs.append(rec)
    return recs, times


def kernel_only(G, torch, prec, reps):
    """The dominant product alone (N = 40,000 points of the workload, 17 columns),
    then a device copy of exactly 1 GiB whose byte counters calibrate HBM traffic."""
    prob, _ = load_workload()
    pts = G.ops.lens_raytrace(prob.grid, prob.lens)
    V = torch.randn(17, prob.grid.N, device="cuda")
    Y = torch.empty_like(V)
    for _ in range(reps):
        G.ops.kernel_mvm(prob.kernel, pts[0], pts[1], V, prec=prec, out=Y, grid=prob.grid)
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"kernel_only": reps, "copy_bytes": src.numel() * 4}), flush=True)


def gauss_only(G, torch, reps):
    """The variational step's image-plane transmission product alone (N =
    40,000 traced points with their pixel shapes as targets, the same points with
    k-NN weights as sources, one column, lengthscale 0.01"), `reps` launches."""
    prob, _ = load_workload()
    pts = G.ops.lens_raytrace(prob.grid, prob.lens)
    z = G.ops.pixel_shapes(prob.grid, pts[0], pts[1])
    w = G.ops.knn_density(pts[0], pts[1], 20).rsqrt()
    y = torch.randn(prob.grid.N, device="cuda")
    out = torch.empty_like(y)
    ell = VIGP_LAYERS[0][1]
    for _ in range(reps):
        G.ops.gauss_product(0.5 * ell * ell, math.sqrt(2 * math.pi * ell * ell) / (2 * math.pi), pts[0], pts[1],
                            pts[0], pts[1], y, tz=z, sw=w, out=out)
    torch.cuda.synchronize()
    print(json.dumps({"gauss_only": reps, "pairs_per_launch": prob.grid.N ** 2}), flush=True)


def gradient_only(G, torch, synth, prec, reps):
    """Timing of the backward path at the bench shape: ray tracing of the
    40,000 points, one reconstruction, then `reps` evaluations of the 12-component
    gradients of ln p and L_VI (the adjoints of the product with its tiles
    recomputed, of ray tracing and of the Sersic mean). Prints one JSON line."""
    import time
    prob, z = load_workload()
    npix = prob.grid.n_pix
    d = torch.as_tensor(z["d"], dtype=torch.float32, device="cuda")
    probes = torch.as_tensor(synth.rademacher(npix, 16, 1).T.copy(), dtype=torch.float32, device="cuda")
    for _ in range(3):
        G.ops.lens_raytrace(prob.grid, prob.lens)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        G.ops.lens_raytrace(prob.grid, prob.lens)
    torch.cuda.synchronize()
    t_ray = (time.perf_counter() - t0) / 20
    rec = G.reconstruct(prob, d, probes, prec=prec, tol=1e-6, max_iter=1000, n_lanczos=N_LANCZOS)
    G.autograd.evidence_gradients(prob, rec)  # warmup
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g = G.autograd.evidence_gradients(prob, rec)
    torch.cuda.synchronize()
    t_grad = (time.perf_counter() - t0) / reps
    print(json.dumps({"gradient_only": reps, "prec": prec, "N": prob.grid.N, "raytrace_ms": t_ray * 1e3,
                      "gradients_ms": t_grad * 1e3, "components": int(g["lnp"].numel())}), flush=True)


def pc_only(G, torch, synth, prec, reps):
    """The preconditioned reconstruction alone at the bench shape (100x100 px,
    2x2 supersampling, rank PC_RANK, 16 probes N(0, P)): two warmups, then
    `reps` timed reconstructions and `reps` timed builds of the factor. Prints
    one JSON line."""
    import time
    prob, z = load_workload()
    npix = prob.grid.n_pix
    d = torch.as_tensor(z["d"], dtype=torch.float32, device="cuda")
    gn, hn = synth.preconditioned_probe_normals(npix, PC_RANK, 16, 1)
    gn = torch.as_tensor(gn, dtype=torch.float64, device="cuda")
    hn = torch.as_tensor(hn, dtype=torch.float32, device="cuda")
    for _ in range(2):
        G.reconstruct_preconditioned(prob, d, gn, hn, rank=PC_RANK, prec=prec)
    pts = G.ops.lens_raytrace(prob.grid, prob.lens)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        G.reconstruct_preconditioned(prob, d, gn, hn, rank=PC_RANK, prec=prec)
    torch.cuda.synchronize()
    t_rec = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        G.ops.pchol(prob, pts[0], pts[1], PC_RANK, prec=prec)
    torch.cuda.synchronize()
    t_build = (time.perf_counter() - t0) / reps
    print(json.dumps({"pc_only": reps, "prec": prec, "rank": PC_RANK, "reconstruction_ms": t_rec * 1e3,
                      "build_ms": t_build * 1e3}), flush=True)


def mfma_flops_per_launch(prec, nrhs, live_subtiles, live_lo):
    """MFMA FLOP one product launch executes, from the plan's counts of evaluated
    (16-point subtile, 32-point chunk) pairs and of those that need the lo part.
    Precision form (v_mfma_f32_16x16x32_f16, 16384 FLOP): per 16-column block 3
    MFMAs (hi.hi + hi.lo + lo.hi), 2 where the lo part is skipped; a last block of
    at most 8 columns packs hi and lo side by side: 2 MFMAs, 1 without lo. FP32
    form (v_mfma_f32_16x16x4_f32, 2048 FLOP): 8 MFMAs per 16-column block."""
    full, rem = divmod(nrhs, 16)
    if prec == "f16x3":
        packed = 1 if 0 < rem <= 8 else 0
        blocks = full + (1 if rem > 8 else 0)
        per_lo = 3 * blocks + 2 * packed
        per_hi = 2 * blocks + 1 * packed
        n_mfma = live_lo * per_lo + (live_subtiles - live_lo) * per_hi
        return n_mfma * 2 * 16 * 16 * 32
    blocks = full + (1 if rem else 0)
    return live_subtiles * blocks * 8 * 2 * 16 * 16 * 4


def product_alone(G, torch, prob, px, py, nrhs, prec, reps=10):
    """Average event-timed launch of the product alone (same shape, same stream)."""
    V = torch.randn(nrhs, px.numel(), device="cuda")
    Y = torch.empty_like(V)
    for _ in range(2):
        G.ops.kernel_mvm(prob.kernel, px, py, V, prec=prec, out=Y, grid=prob.grid)
    torch.cuda.synchronize()
    G.ops.timing_read(reset=True)
    G.ops.timing_enable(1)
    for _ in range(reps):
        G.ops.kernel_mvm(prob.kernel, px, py, V, prec=prec, out=Y, grid=prob.grid)
    G.ops.timing_enable(False)
    ms, n = G.ops.timing_read(reset=True)
    return ms / max(n, 1)


# Variational GP source fit at the same workload: two image-plane layers on the
# traced points and a source-plane layer on a 40 x 40 grid at 30 mas (Sec. 3.5,
# Sec. 4.1), lengthscales in arcsec.
VIGP_LAYERS = (("ip", 0.01), ("ip", 0.04), ("sp", 0.04))
# FP32 slots per pair of a one-column transmission product with shapes on one
# side: 2 differences, 6 for u = C^{-1} d and q = d.u, 1 scale, exp2 at a quarter
# rate (4), 1 weight, 1 accumulate.
GAUSS_PAIR_COST = 2 + 6 + 1 + 4 + 1 + 1
GAUSS_PEAK_GPAIRS = VALU_LANE_OPS / GAUSS_PAIR_COST / 1e9


C3_FIXTURE = os.path.join(ROOT, "tests", "fixtures", "workload2_draw0_crop100.npz")


def c3_section(G, torch, synth, steps):
    """The 200 x 200 image with 2 x 2 supersampling (N = 160,000) and 64 columns
    (1 solve + 63 probes): timed reconstructions in both forms, the product's
    roofline at that size, and ln p with its SLQ standard error. Its observation
    is the stored oracle simulation; the oracle's evidence exists for the central
    100 x 100 crop only (the test suite compares against it)."""
    import numpy as np
    w = synth.workload(2)
    s = w.source
    prob = G.Problem(G.Grid(w.n, w.ss, w.pix_scale), G.Lens(*w.lens.as_tuple()),
                     G.Sersic(s.peak, s.R_e, s.n_sersic, s.xs, s.ys), G.Kernel(w.ell, w.amp), G.PSF(w.psf_fwhm),
                     w.noise_sigma)
    z = np.load(C3_FIXTURE)
    d = torch.as_tensor(z["d"], dtype=torch.float32, device="cuda")
    Z = torch.as_tensor(synth.rademacher(w.n_pix, 63, 2).T.copy(), dtype=torch.float32, device="cuda")
    out = {"workload": "200x200 px, 2x2 supersampling (N=160000), 64 columns (1 + 63 probes), CG tol 1e-6",
           "N": w.N, "n_pix": w.n_pix}
    for prec in ("f16x3", "fp32"):
        G.reconstruct(prob, d, Z, prec=prec, tol=1e-6, max_iter=3000, n_lanczos=3000)  # warmup
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            rec = G.reconstruct(prob, d, Z, prec=prec, tol=1e-6, max_iter=3000, n_lanczos=3000)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
        h = rec.host()
        _, sub, lo = G.ops.kernel_mvm_live_tiles(prob.kernel, rec.px, rec.py, prec=prec, grid=prob.grid, with_lo=True)
        ms = product_alone(G, torch, prob, rec.px, rec.py, 64, prec)
        ev = sub * 512
        sec = {"ms_per_reconstruction": el * 1e3, "reconstructions_per_s": 1.0 / el, "cg_iters": max(h["iters"]),
               "lnp": h["lnp"], "lnp_slq_stderr_rel": 0.5 * h["stderr"] / abs(h["lnp"]),
               "true_relres_max": max(h["true_relres"]), "product_ms_alone": ms,
               "evaluated_pairs_per_launch": ev, "evaluated_fraction": ev / (w.N * w.N)}
        if prec == "f16x3":
            sec["roofline"] = {"bound": "alu", "unit": "Gpairs/s", "achieved": ev / (ms * 1e-3) / 1e9,
                               "peak": ALU_PEAK_GPAIRS, "frac": ev / (ms * 1e-3) / 1e9 / ALU_PEAK_GPAIRS,
                               "mfma_tflops_executed": mfma_flops_per_launch(prec, 64, sub, lo) / (ms * 1e-3) / 1e12}
        else:
            flop = mfma_flops_per_launch(prec, 64, sub, sub)
            sec["roofline"] = {"bound": "mfma", "unit": "TFLOP/s", "achieved": flop / (ms * 1e-3) / 1e12,
                               "peak": FP32_MFMA_PEAK_TFLOPS,
                               "frac": flop / (ms * 1e-3) / 1e12 / FP32_MFMA_PEAK_TFLOPS}
        out[prec] = sec
    out["reconstructions_ratio_f16x3_vs_fp32"] = (out["f16x3"]["reconstructions_per_s"] /
                                                   out["fp32"]["reconstructions_per_s"])
    return out


def vigp_section(G, torch, synth, prob, d, steps, lens):
    """Timed Adam steps of the variational fit (ELBO sample, gradient, update),
    and the dense transmission product alone with its ALU roofline."""
    import numpy as np
    gx, gy = synth.source_grid(40, 0.03)
    gxd = torch.as_tensor(gx, dtype=torch.float32, device="cuda")
    gyd = torch.as_tensor(gy, dtype=torch.float32, device="cuda")
    v = G.vigp.Vigp(G.vigp.VigpModel(VIGP_LAYERS, lens[3]), prob, d, gxd, gyd)
    v.lens_mean.copy_(torch.as_tensor(np.asarray(lens)[[0, 1, 2, 4, 5, 6, 7]]))
    v.lens_raw.copy_(torch.diag(torch.full((7,), math.log(0.01), dtype=torch.float64)))
    v.log_amp.copy_(torch.log(torch.tensor([prob.noise_sigma, prob.noise_sigma, 10 * prob.noise_sigma],
                                           dtype=torch.float64)))
    v.sp["logs"].fill_(math.log(0.01))
    for blk in v.ip:
        blk["logs"].fill_(math.log(0.001))
    noise = []
    for t in range(steps + 2):
        a, b = synth.vigp_normals(v.ne32, t)
        noise.append((torch.as_tensor(a, device="cuda"), torch.as_tensor(b, dtype=torch.float32, device="cuda")))
    for e64, e32 in noise[:2]:  # warmup
        v.step(e64, e32, 1e-3)
    torch.cuda.synchronize()
    elbos = []
    t0 = time.perf_counter()
    for e64, e32 in noise[2:]:
        elbos.append(v.step(e64, e32, 1e-3)[0].clone())
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    elbos = [float(x.item()) for x in elbos]
    # the image-plane layer's product alone: N targets with shapes, N weighted sources, one column
    N = prob.grid.N
    pts = G.ops.lens_raytrace(prob.grid, prob.lens)
    z = G.ops.pixel_shapes(prob.grid, pts[0], pts[1])
    w = G.ops.knn_density(pts[0], pts[1], 20).rsqrt()
    y = torch.randn(N, device="cuda")
    out = torch.empty(N, device="cuda")
    ell = VIGP_LAYERS[0][1]
    args_ = (0.5 * ell * ell, math.sqrt(2 * math.pi * ell * ell) / (2 * math.pi), pts[0], pts[1], pts[0], pts[1], y)
    G.ops.gauss_product(*args_, tz=z, sw=w, out=out)
    reps = 10
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        G.ops.gauss_product(*args_, tz=z, sw=w, out=out)
    e1.record()
    torch.cuda.synchronize()
    g_ms = e0.elapsed_time(e1) / reps
    achieved = N * N / (g_ms * 1e-3) / 1e9
    return {"layers": [list(x) for x in VIGP_LAYERS], "grid": "40x40 at 30 mas", "steps": steps,
            "ms_per_step": el / steps * 1e3, "steps_per_s": steps / el, "lr": 1e-3,
            "elbo_first": elbos[0], "elbo_last": elbos[-1],
            "roofline": {"kernel": "gauss_product_kernel (image-plane layer, 1 column)", "bound": "alu",
                         "unit": "Gpairs/s", "achieved": achieved, "peak": GAUSS_PEAK_GPAIRS,
                         "frac": achieved / GAUSS_PEAK_GPAIRS, "pairs_per_launch": N * N,
                         "avg_launch_ms_alone": g_ms}}


def posterior_section(G, torch, synth, prob, rec, z):
    """Exact posterior mean and variance on the 40 x 40 source-plane grid from
    the preconditioned reconstruction, against the stored FP64 oracle."""
    import numpy as np
    gx, gy = synth.source_grid(int(z["grid_n"]), float(z["grid_spacing"]))
    gxd = torch.as_tensor(gx, dtype=torch.float32, device="cuda")
    gyd = torch.as_tensor(gy, dtype=torch.float32, device="cuda")
    G.posterior_at(prob, rec, gxd, gyd)  # warmup
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        post = G.posterior_at(prob, rec, gxd, gyd)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    var = post.var.cpu().numpy()
    mean = post.mean.double().cpu().numpy()
    return {"points": int(gx.size), "ms": el * 1e3, "pcg_iters": int(post.cg["iters"].max().item()),
            "var_max_abs_err_vs_oracle": float(np.max(np.abs(var - z["grid_var"]))),
            "mean_max_abs_err_vs_oracle": float(np.max(np.abs(mean - z["grid_mean"]))),
            "var_range_oracle": [float(z["grid_var"].min()), float(z["grid_var"].max())]}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default="f16x3", choices=["f16x3", "fp32"])
    ap.add_argument("--plain-steps", type=int, default=3, help="timed steps of the plain FP32 form (0: skip)")
    ap.add_argument("--pc-steps", type=int, default=3,
                    help="timed steps with the rank-%d partial pivoted Cholesky preconditioner (0: skip)" % 4096)
    ap.add_argument("--async-steps", type=int, default=2,
                    help="steps with the fully asynchronous CG call (no host wait; 0: skip)")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle CPU work (0: skip)")
    ap.add_argument("--kernel-only", type=int, default=0,
                    help="run only the dominant kernel this many times at the bench shape, then a 1 GiB copy "
                         "(calibration of the HBM byte counters), and exit; for rocprofv3 counter runs")
    ap.add_argument("--gauss-only", type=int, default=0,
                    help="run only the variational step's transmission product this many times (for counters)")
    ap.add_argument("--gradient-only", type=int, default=0,
                    help="time ray tracing and this many evaluations of the evidence gradients at the bench shape, "
                         "print one JSON line and exit")
    ap.add_argument("--pc-only", type=int, default=0,
                    help="time only the preconditioned reconstruction and its factor build, this many times")
    ap.add_argument("--c3-steps", type=int, default=2,
                    help="timed reconstructions of the 200x200, N=160000 image per form (0: skip)")
    ap.add_argument("--vigp-steps", type=int, default=10,
                    help="timed steps of the variational GP source fit (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=512,
                    help="requests in the serving trace (0: skip)")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving section (both forms) and print its JSON; for kernel traces")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path runs on a single MI355X)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2105_09465_amd as G
    import synth

    torch.cuda.set_device(0)
    if args.kernel_only > 0:
        kernel_only(G, torch, args.prec, args.kernel_only)
        return
    if args.gauss_only > 0:
        gauss_only(G, torch, args.gauss_only)
        return
    if args.gradient_only > 0:
        gradient_only(G, torch, synth, args.prec, args.gradient_only)
        return
    if args.pc_only > 0:
        pc_only(G, torch, synth, args.prec, args.pc_only)
        return
    if args.serve_only:
        print(json.dumps(serve_section(G, torch, synth, args.serve_requests)), flush=True)
        return
    prob, z = load_workload()
    N, npix = prob.grid.N, prob.grid.n_pix
    nrhs = 17
    d = torch.as_tensor(z["d"], dtype=torch.float32, device="cuda")
    probes = torch.as_tensor(synth.rademacher(npix, 16, 1).T.copy(), dtype=torch.float32, device="cuda")
    ws = None

    # ---- precision form: warmup, then the timed region; every TIMING_STRIDE-th
    # product launch in it is bracketed by HIP events on its stream (an event
    # pair delays the stream by a few microseconds, so timing every launch would
    # slow the timed steps themselves)
    run_steps(G, torch, prob, d, probes, args.prec, args.warmup, ws)
    G.ops.timing_samples(reset=True)
    G.ops.timing_enable(TIMING_STRIDE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs, times = run_steps(G, torch, prob, d, probes, args.prec, args.steps, ws)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    G.ops.timing_enable(False)
    samples = G.ops.timing_samples(reset=True)
    hosts = [r.host() for r in recs]
    iters = [max(h["iters"]) for h in hosts]
    ms_per_step = elapsed / args.steps * 1e3
    # the dominant kernel: the 17-column product inside CG. Launches queued past
    # a step's last active iteration exit at once (a few microseconds against
    # tens); they are left out of the average by a cut at a quarter of the median
    active = [v for v in samples if v > 0.25 * float(np.median(samples))] if samples else []
    avg_ms = float(np.mean(active)) if active else float("nan")
    # work of one launch: the kernel values the product evaluates, 512 per live
    # (16-point subtile, 32-point chunk) pair of its tile plan; every other pair
    # is below 2^-36 a^2 (exactly zero in the precision form) and is not evaluated
    px, py = recs[-1].px, recs[-1].py
    live_tiles, live_subtiles, live_lo = G.ops.kernel_mvm_live_tiles(prob.kernel, px, py, prec=args.prec,
                                                                     grid=prob.grid, with_lo=True)
    evaluated = live_subtiles * 16 * 32
    achieved = evaluated / (avg_ms * 1e-3) / 1e9
    mfma_flop = mfma_flops_per_launch(args.prec, nrhs, live_subtiles, live_lo)
    # products with K per step: one per CG iteration (all 17 columns), one for the
    # true residual at exit and the posterior mean's
    products = [it + 2 for it in iters]
    value = sum(products) * evaluated / elapsed / 1e9
    dense_equivalent = sum(products) * N * N / elapsed / 1e9
    alone_avg = product_alone(G, torch, prob, px, py, nrhs, args.prec)

    # ---- accuracy of this run against the stored oracle evidence
    h = hosts[-1]
    lnp_ref = float(z["lnp"])
    lnp_rel = abs(h["lnp"] - lnp_ref) / abs(lnp_ref)
    r = recs[-1]
    ld30, se30, _ = G.ops.lanczos_logdet(r.cg["ab"][1:, :30].contiguous(), r.cg["iters"][1:], r.cg["bnorm2"][1:],
                                         1.0 / 16)
    slq30 = {"logdet_err": ld30.item() - float(z["logdet"]), "stderr": se30.item()}

    # ---- the same step with the fully asynchronous CG call (every iteration up
    # to the cap enqueued, no host wait inside the library)
    async_ms = None
    if args.async_steps > 0:
        t_async = []
        for k in range(args.async_steps + 1):  # the first is a warmup
            torch.cuda.synchronize()
            t = time.perf_counter()
            G.reconstruct(prob, d, probes, prec=args.prec, tol=1e-6, max_iter=1000, n_lanczos=N_LANCZOS,
                          check_every=0, ws=ws)
            torch.cuda.synchronize()
            if k:
                t_async.append((time.perf_counter() - t) * 1e3)
        async_ms = float(np.mean(t_async))

    # ---- the same image with the partial pivoted Cholesky preconditioner
    # (rank PC_RANK): ln|A| = ln|P| + SLQ of P^{-1/2} A P^{-1/2}, 16 probes N(0, P)
    pcsec = None
    if args.pc_steps > 0:
        gn, hn = synth.preconditioned_probe_normals(npix, PC_RANK, 16, 1)
        gn = torch.as_tensor(gn, dtype=torch.float64, device="cuda")
        hn = torch.as_tensor(hn, dtype=torch.float32, device="cuda")
        G.reconstruct_preconditioned(prob, d, gn, hn, rank=PC_RANK, prec=args.prec)  # warmup
        pts_pc = G.ops.lens_raytrace(prob.grid, prob.lens)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.pc_steps):
            rpc = G.reconstruct_preconditioned(prob, d, gn, hn, rank=PC_RANK, prec=args.prec)
        torch.cuda.synchronize()
        pc_el = time.perf_counter() - t0
        t0 = time.perf_counter()
        G.ops.pchol(prob, pts_pc[0], pts_pc[1], PC_RANK, prec=args.prec)
        torch.cuda.synchronize()
        t_build = time.perf_counter() - t0
        hp = rpc.host()
        pcsec = {"rank": PC_RANK, "probes": 16, "ms_per_step": pc_el / args.pc_steps * 1e3,
                 "reconstructions_per_s": args.pc_steps / pc_el, "preconditioner_build_ms": t_build * 1e3,
                 "pcg_iters": max(hp["iters"]), "lnp_rel_err_vs_oracle": abs(hp["lnp"] - lnp_ref) / abs(lnp_ref),
                 "lnp_slq_stderr_rel": 0.5 * hp["stderr"] / abs(lnp_ref),
                 "logdet_err_vs_oracle": hp["logdet"] - float(z["logdet"]), "slq_stderr": hp["stderr"],
                 "quad_rel_err_vs_oracle": abs(hp["quad"] - float(z["quad"])) / float(z["quad"]),
                 "true_relres_max": max(hp["true_relres"])}

    post = None
    if pcsec is not None:
        post = posterior_section(G, torch, synth, prob, rpc, z)

    c3 = None
    if args.c3_steps > 0:
        c3 = c3_section(G, torch, synth, args.c3_steps)

    vsec = None
    if args.vigp_steps > 0:
        vsec = vigp_section(G, torch, synth, prob, d, args.vigp_steps, prob.lens.as_tuple())

    # ---- plain FP32 form, same step, and its product's own roofline
    plain = None
    if args.plain_steps > 0 and args.prec != "fp32":
        run_steps(G, torch, prob, d, probes, "fp32", 1, ws)
        t0 = time.perf_counter()
        precs, ptimes = run_steps(G, torch, prob, d, probes, "fp32", args.plain_steps, ws)
        pel = time.perf_counter() - t0
        ph = [x.host() for x in precs]
        pit = [max(x["iters"]) for x in ph]
        _, p_sub, _ = G.ops.kernel_mvm_live_tiles(prob.kernel, px, py, prec="fp32", grid=prob.grid, with_lo=True)
        p_ms = product_alone(G, torch, prob, px, py, nrhs, "fp32")
        p_flop = mfma_flops_per_launch("fp32", nrhs, p_sub, p_sub)
        p_alg = p_sub * 512 * 2 * nrhs
        plain = {"value": sum(it + 2 for it in pit) * p_sub * 512 / pel / 1e9, "unit": "Gpairs/s (evaluated)",
                 "reconstructions_per_s": args.plain_steps / pel, "ms_per_step": pel / args.plain_steps * 1e3,
                 "cg_iters": pit[-1], "lnp_rel_err_vs_oracle": abs(ph[-1]["lnp"] - lnp_ref) / abs(lnp_ref),
                 "true_relres_max": max(ph[-1]["true_relres"]),
                 "roofline": {"bound": "mfma", "kernel": "mvm_f32_kernel", "unit": "TFLOP/s",
                              "achieved": p_flop / (p_ms * 1e-3) / 1e12, "peak": FP32_MFMA_PEAK_TFLOPS,
                              "frac": p_flop / (p_ms * 1e-3) / 1e12 / FP32_MFMA_PEAK_TFLOPS,
                              "executed_flop_per_launch": p_flop,
                              "algorithmic_flop_per_launch": p_alg,
                              "note": "17 columns run as two 16-column MFMA blocks (32 columns executed)",
                              "avg_launch_ms_alone": p_ms,
                              "evaluated_pairs_per_launch": p_sub * 512,
                              "alu_frac": p_sub * 512 / (p_ms * 1e-3) / 1e9 / ALU_PEAK_GPAIRS}}

    serving = None
    if args.serve_requests > 0:
        serving = serve_section(G, torch, synth, args.serve_requests)

    cpu = None
    if args.cpu_budget > 0:
        cpu = cpu_baseline(prob, px.double().cpu().numpy(), py.double().cpu().numpy(), args.cpu_budget)

    traffic = _traffic()
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "Gpairs/s (evaluated)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16x3" if args.prec == "f16x3" else "f32",
        "data": "synthetic (oracle-simulated lensed Sersic + RBF-GP source, seeded)",
        "config": {"workload": "100x100 px image, 2x2 supersampling (N=40000 points), SPLE+shear lens prior draw, "
                               "Gaussian PSF FWHM 0.1\", 1 solve + 16 Rademacher probe columns, CG tol 1e-6, "
                               "SLQ over all CG steps", "N": N, "n_pix": npix, "rhs": nrhs},
        "value_note": "kernel values evaluated by the step's products per second (the pairs of every product "
                      "whose kernel value is below 2^-36 a^2 are not evaluated)",
        "dense_equivalent_gpairs_per_s": dense_equivalent,
        "reconstructions_per_s": args.steps / elapsed,
        "async_ms_per_step": async_ms,
        "cg_iters": iters[-1],
        "true_relres_max": max(h["true_relres"]),
        "lnp_rel_err_vs_oracle": lnp_rel,
        "lnp_slq_stderr_rel": 0.5 * h["stderr"] / abs(lnp_ref),
        "logdet_err_vs_oracle": h["logdet"] - float(z["logdet"]),
        "quad_rel_err_vs_oracle": abs(h["quad"] - float(z["quad"])) / float(z["quad"]),
        "slq_stderr": h["stderr"],
        "slq_30_steps": slq30,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_GPAIRS, "unit": "Gpairs/s",
                     "frac": achieved / ALU_PEAK_GPAIRS, "traffic": traffic,
                     "kernel": "mvm_f16x3_kernel" if args.prec == "f16x3" else "mvm_f32_kernel",
                     "evaluated_pairs_per_launch": evaluated, "all_pairs_per_launch": N * N,
                     "evaluated_fraction": evaluated / (N * N),
                     "avg_launch_ms_in_step": avg_ms, "timed_launches_in_step": len(active),
                     "timing_stride": TIMING_STRIDE, "avg_launch_ms_alone": alone_avg,
                     "subtile_pairs_with_lo": live_lo, "subtile_pairs": live_subtiles,
                     "mfma_flop_per_launch": mfma_flop,
                     "mfma_tflops_executed": mfma_flop / (avg_ms * 1e-3) / 1e12},
        "preconditioned": pcsec,
        "posterior_grid": post,
        "c3_160k_64cols": c3,
        "vigp": vsec,
        "plain_fp32": plain,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    if plain:
        out["reconstructions_ratio_vs_fp32"] = out["reconstructions_per_s"] / plain["reconstructions_per_s"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
