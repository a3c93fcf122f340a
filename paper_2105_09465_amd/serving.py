"""Continuous-batching request loop over the library's serving entry points.

Requests of uneven image sizes arrive over time. Each admitted request becomes
a slot whose points, right-hand sides, CG vectors, CG state and Lanczos
coefficients live in its own device workspace (its HBM footprint, the unit of
admission). Every round the engine admits arrived requests while slots and the
memory budget allow, advances all active slots by a few CG iterations with one
grouped launch per stage, reads back which slots have finished, and retires
them (SLQ log-determinant, evidence scalars, posterior mean, image). Latency is
arrival to results on the host.
"""
from __future__ import annotations

import collections
import ctypes as C
import dataclasses
import time

import numpy as np
import torch

from . import _lib
from .params import Problem

PREC = {"fp32": _lib.PREC_FP32, "f16x3": _lib.PREC_F16X3}


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float  # seconds after the start of the run
    problem: Problem
    d: torch.Tensor  # (n_pix,) float32 on the GPU
    probes: torch.Tensor  # (m, n_pix) float32 on the GPU


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float
    quad: float
    lnp: float
    vi: float
    logdet: float
    stderr: float
    iters: list
    relres: list
    status: list
    image: torch.Tensor | None = None

    @property
    def latency(self):
        return self.finished - self.arrival


class _Slot:
    def __init__(self, req, ws, c_slot, admitted_iter, admitted_time, footprint):
        self.req, self.ws, self.c, self.it0, self.t_admit, self.footprint = req, ws, c_slot, admitted_iter, \
            admitted_time, footprint


class ServingEngine:
    def __init__(self, prec="f16x3", hbm_budget=8 << 30, max_slots=64,
                 chunk=4, tol=1e-6, max_iter=1000, n_lanczos=1000, want_image=False):
        self.prec = PREC[prec] if isinstance(prec, str) else int(prec)
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.chunk = int(chunk)
        self.tol, self.max_iter, self.n_lanczos = float(tol), int(max_iter), int(n_lanczos)
        self.want_image = want_image
        self.snap = torch.zeros(64, dtype=torch.int32, pin_memory=True)
        self.stats = dict(rounds=0, max_active=0, max_bytes=0, admitted=0, deferred_memory=0, step_s=0.0)

    def footprint(self, req: Request) -> int:
        g = req.problem.grid.c()
        return int(_lib.lib.gpl_serve_slot_workspace(C.byref(g), 1 + req.probes.shape[0], self.n_lanczos,
                                                     self.prec))

    def _admit(self, req, it, now, stream):
        fp = self.footprint(req)
        ws = torch.empty(fp, dtype=torch.uint8, device="cuda")
        slot = _lib.gpl_serve_slot()
        P = req.problem
        prob = _lib.gpl_problem(P.grid.c(), P.kernel.c(), P.psf.c(), P.noise_sigma, None, None)
        lens, src = P.lens.c(), P.source.c()
        m = req.probes.shape[0]
        _lib.call("gpl_serve_slot_init", C.byref(slot), C.byref(prob), C.byref(lens), C.byref(src),
                  C.c_void_p(req.d.data_ptr()), C.c_void_p(req.probes.data_ptr()) if m else None,
                  P.grid.n_pix, 1 + m, self.tol, self.max_iter, self.n_lanczos, self.prec,
                  C.c_void_p(ws.data_ptr()), fp, stream)
        self.stats["admitted"] += 1
        return _Slot(req, ws, slot, it, now, fp)

    def _finish(self, s: _Slot, it, stream):
        m = s.req.probes.shape[0]
        dev = "cuda"
        out = torch.empty(5, dtype=torch.float64, device=dev)
        iters = torch.empty(1 + m, dtype=torch.int32, device=dev)
        relres = torch.empty(1 + m, dtype=torch.float64, device=dev)
        status = torch.empty(1 + m, dtype=torch.int32, device=dev)
        g = s.req.problem.grid
        fhat = torch.empty(g.N, dtype=torch.float32, device=dev) if self.want_image else None
        image = torch.empty(g.n_pix, dtype=torch.float32, device=dev) if self.want_image else None
        _lib.call("gpl_serve_slot_finish", C.byref(s.c), it, (1.0 / m) if m else 0.0, C.c_void_p(out.data_ptr()),
                  C.c_void_p(iters.data_ptr()), C.c_void_p(relres.data_ptr()), C.c_void_p(status.data_ptr()),
                  C.c_void_p(fhat.data_ptr()) if fhat is not None else None,
                  C.c_void_p(image.data_ptr()) if image is not None else None, stream)
        return out, iters, relres, status, image

    def run(self, requests, realtime=True):
        """Serve `requests` (sorted or not by arrival). With realtime=True arrivals
        follow the wall clock from the start of the run; otherwise every request
        is available at once (arrival 0). Returns the list of Results."""
        stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        active: list[_Slot] = []
        results = []
        used = 0
        it = 0
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while pending or active:
            now = time.perf_counter() - t0
            while pending and (not realtime or pending[0].arrival <= now) and len(active) < self.max_slots:
                fp = self.footprint(pending[0])
                if used + fp > self.budget and active:
                    self.stats["deferred_memory"] += 1
                    break
                req = pending.popleft()
                active.append(self._admit(req, it, now, stream))
                used += fp
            if not active:
                wait = pending[0].arrival - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.05))
                continue
            self.stats["max_active"] = max(self.stats["max_active"], len(active))
            self.stats["max_bytes"] = max(self.stats["max_bytes"], used)
            arr = (C.POINTER(_lib.gpl_serve_slot) * len(active))(*[C.pointer(s.c) for s in active])
            ev0.record()
            _lib.call("gpl_serve_step", arr, len(active), self.chunk, it, stream)
            ev1.record()
            it += self.chunk
            _lib.call("gpl_serve_snapshot", arr, len(active), it, C.c_void_p(self.snap.data_ptr()), stream)
            torch.cuda.current_stream().synchronize()
            # device time of the round's grouped CG iterations (the rest of the
            # round is the scheduler: snapshot, host wait, admission, retirement)
            self.stats["step_s"] += ev0.elapsed_time(ev1) * 1e-3
            self.stats["rounds"] += 1
            snap = self.snap[:len(active)].tolist()
            keep = []
            done = []
            for s, a in zip(active, snap):
                if a == 0 or it - s.it0 >= self.max_iter + self.chunk:
                    done.append((s, self._finish(s, it, stream)))
                else:
                    keep.append(s)
            if done:
                torch.cuda.current_stream().synchronize()
                tnow = time.perf_counter() - t0
                for s, (out, iters, relres, status, image) in done:
                    o = out.cpu().tolist()
                    arrival = s.req.arrival if realtime else 0.0
                    results.append(Result(s.req.rid, arrival, s.t_admit, tnow, o[0], o[1], o[2], o[3], o[4],
                                          iters.cpu().tolist(), relres.cpu().tolist(), status.cpu().tolist(), image))
                    used -= s.footprint
            active = keep
        self.stats["wall_s"] = time.perf_counter() - t0
        return results


def summarize(results, wall_s):
    lat = np.array([r.latency for r in results])
    se = np.array([0.5 * r.stderr / abs(r.lnp) for r in results if r.lnp != 0])
    return {"requests": len(results), "reconstructions_per_s": len(results) / wall_s,
            "p50_latency_ms": float(np.percentile(lat, 50) * 1e3), "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_latency_ms": float(lat.mean() * 1e3), "wall_s": wall_s,
            "lnp_slq_stderr_rel_median": float(np.median(se)) if se.size else None}
