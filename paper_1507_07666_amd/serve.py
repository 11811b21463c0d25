"""Continuous-batching request loop for geometry-scan solves.

Requests (atoms, or scans of molecule geometries) arrive over time.  Each one
is admitted into the batch as soon as the device-memory budget allows, takes
steps in lockstep with everything else already on the GPU (one launch per
kernel for all of them), and when one of its scan points converges the next
point warm-starts in the same slot (lbks_set_nuclei keeps the orbitals
resident).  A request leaves, freeing its memory, after its last point.

The stopping rule of each solve depends only on its own chunk energies and
the relax calls are made of whole chunks, so every result is bit-for-bit what
the same request gives when solved alone (`solve_alone`).
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

from . import lbks


@dataclass
class PointResult:
    e_total: float
    eps: List[float]
    steps: int
    status: int
    ritz: Optional[List[float]] = None          # with ServeConfig.detail: Ritz values of the projected operator
    rho_sub4: Optional[np.ndarray] = None       # with ServeConfig.detail: density on every fourth node per axis


@dataclass
class RequestResult:
    rid: int
    arrival: float
    admitted: float = float("nan")
    finished: float = float("nan")
    points: List[PointResult] = field(default_factory=list)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


# Stopping rule of FP32 solves.  At the fixed point the FP32 total energy moves
# by up to about 1e-6 Ha from one check to the next, and on the way there it
# passes a turning point where two checks can agree by chance; the sum of the
# orbital energies converges linearly in the error of the orbitals and settles
# to about 3e-7.  A solve stops when the energy moved by less than 2e-6 Ha and
# the eigenvalue sum by less than 1e-6 Ha on two consecutive checks.
FP32_RULE = dict(dE_tol=2e-6, deps_tol=1e-6, stop_checks=2)


@dataclass
class ServeConfig:
    hbm_budget: int                 # bytes of device memory the solves may hold
    precision: int = lbks.LBKS_FP32_BULK
    check_every: int = 100
    dE_tol: float = FP32_RULE["dE_tol"]
    deps_tol: float = FP32_RULE["deps_tol"]
    stop_checks: int = FP32_RULE["stop_checks"]
    chunks_per_call: int = 2        # lattice steps between admissions = chunks_per_call * check_every
    max_steps_per_point: int = 20000
    detail: bool = False            # also record Ritz values and a coarse density per point (for checks)


def point_params(system, cfg: ServeConfig) -> lbks.lbks_params:
    return lbks.params_for(system, precision=cfg.precision, deps_tol=cfg.deps_tol,
                           stop_checks=cfg.stop_checks)


def point_bytes(system, cfg: ServeConfig) -> int:
    """Device bytes one slot for this system holds (0 if its parameters are invalid)."""
    p = point_params(system, cfg)
    return int(lbks.load().lbks_estimate_bytes(lbks.ctypes.byref(p)))


def point_result(s: "lbks.Solver", system, steps: int, rc: int, cfg: ServeConfig) -> PointResult:
    """Result of a finished point (energies; with cfg.detail the Ritz values and
    the density on every fourth node)."""
    e = s.energy()
    out = PointResult(e["e_total"], list(e["eps"]), steps, rc)
    if cfg.detail:
        _, ritz = s.hamiltonian()
        _, rho = s.orbitals()
        nx, ny, nz = system.dims
        out.ritz = [float(x) for x in ritz]
        out.rho_sub4 = rho.reshape(nz, ny, nx)[::4, ::4, ::4].copy()
    return out


def solve_alone(request, cfg: ServeConfig) -> List[PointResult]:
    """The same request on its own (same rule, same warm starts)."""
    out = []
    pts = request.points
    s = lbks.Solver(point_params(pts[0], cfg))
    try:
        for sy in pts:
            s.set_nuclei(sy.Z, sy.R)
            steps = 0
            rc = lbks.LBKS_NOT_CONVERGED
            while steps < cfg.max_steps_per_point:
                n = min(cfg.chunks_per_call * cfg.check_every, cfg.max_steps_per_point - steps)
                rc, k = s.relax(n, cfg.dE_tol, cfg.check_every)
                steps += k
                if rc == lbks.LBKS_OK:
                    break
            out.append(point_result(s, sy, steps, rc, cfg))
    finally:
        s.close()
    return out


class Server:
    def __init__(self, cfg: ServeConfig, clock: Optional[Callable[[], float]] = None):
        self.cfg = cfg
        self.clock = clock or time.perf_counter
        self.batch = lbks.Batch()
        self.used = 0
        self.active: Dict[int, dict] = {}
        self.log: List[str] = []
        self.peak_used = 0
        self.peak_active = 0

    def _admit(self, req, now, res: RequestResult):
        first = req.points[0]
        s = self.batch.add(point_params(first, self.cfg))
        s.set_nuclei(first.Z, first.R)
        nbytes = s.device_bytes()
        self.used += nbytes
        self.peak_used = max(self.peak_used, self.used)
        self.active[req.rid] = dict(req=req, solver=s, point=0, steps=0, bytes=nbytes, res=res)
        res.admitted = now
        self.peak_active = max(self.peak_active, len(self.active))

    def _retire(self, rid, now):
        a = self.active.pop(rid)
        self.batch.remove(a["solver"])
        a["solver"].close()
        self.used -= a["bytes"]
        a["res"].finished = now

    def run(self, requests) -> List[RequestResult]:
        cfg = self.cfg
        t0 = self.clock()
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        waiting: deque = deque()
        results = {r.rid: RequestResult(r.rid, r.arrival) for r in requests}
        while pending or waiting or self.active:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # admission in arrival order while the memory budget allows
            while waiting:
                need = point_bytes(waiting[0].points[0], cfg)
                if need > cfg.hbm_budget:
                    raise ValueError(f"request {waiting[0].rid} needs {need} B, more than the whole budget")
                if self.used + need > cfg.hbm_budget:
                    break
                r = waiting.popleft()
                self._admit(r, self.clock() - t0, results[r.rid])
            if not self.active:
                if pending:
                    time.sleep(max(0.0, min(0.05, pending[0].arrival - (self.clock() - t0))))
                continue
            rids = list(self.active)
            st, steps = self.batch.relax(cfg.chunks_per_call * cfg.check_every, cfg.dE_tol, cfg.check_every)
            order = [s for s in self.batch.solvers]
            by_solver = {id(self.active[r]["solver"]): r for r in rids}
            now = self.clock() - t0
            for s, rc, k in zip(order, st, steps):
                rid = by_solver[id(s)]
                a = self.active[rid]
                a["steps"] += k
                if rc < 0:
                    raise lbks.LbksError(rc, f"request {rid} failed")
                if rc == lbks.LBKS_OK or a["steps"] >= cfg.max_steps_per_point:
                    a["res"].points.append(point_result(s, a["req"].points[a["point"]], a["steps"], rc, cfg))
                    a["point"] += 1
                    a["steps"] = 0
                    if a["point"] < len(a["req"].points):
                        nxt = a["req"].points[a["point"]]
                        s.set_nuclei(nxt.Z, nxt.R)       # warm start: orbitals stay resident
                    else:
                        self._retire(rid, self.clock() - t0)
        return [results[r.rid] for r in requests]

    def close(self):
        for rid in list(self.active):
            self._retire(rid, float("nan"))
        self.batch.close()


def summarize(results: List[RequestResult], wall: float) -> dict:
    lat = np.array([r.latency for r in results])
    points = sum(len(r.points) for r in results)
    return {"requests": len(results), "points": points, "wall_s": wall,
            "solves_per_s": points / wall if wall > 0 else float("nan"),
            "requests_per_s": len(results) / wall if wall > 0 else float("nan"),
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_queue_s": float(np.nanmean([r.admitted - r.arrival for r in results]))}
