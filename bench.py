"""Throughput of the lattice kinetic Kohn-Sham relaxation on one MI355X.

A step is one lattice step of the whole hot path for every orbital: overlap +
Cholesky Gram-Schmidt, density, Hartree SOR sweeps, potential with local xc,
and the population stream-collide; the energy evaluation and convergence test
run every `--check-every` steps inside the timed region.

Default workload: Ne atom, 96^3 nodes at 0.2 bohr, softening 0.05, 5 orbitals,
FP64, seeded random Gaussian-enveloped start (seed 2).  Metric: orbital-site
updates per second (orbitals x nodes x steps / wall time), inputs resident in
HBM.  The same JSON line also carries the other parts of the metric: the
64-molecule H2O batch (solves/s until every member meets the FP32 rule, with the
energy error of the members that have a stored oracle reference), one rate of
the seeded serving stream (p50/p99 latency, solves/s), and CH4 128^3 time to
|E - E_oracle| < 1e-5 Ha in FP64 and in FP32 on the GPU.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
I_SERVE_GRIDS = (48, 64, 80, 96, 112, 128)


def workload(name):
    from paper_1507_07666_amd import inputs as I
    if name == "ne96":
        return I.ne_atom()
    if name == "he32":
        return I.he_atom()
    if name == "ch4":
        return I.ch4()
    if name.startswith("he") and name[2:].isdigit():     # He on n^3 nodes at 0.3 * 32 / n bohr
        n = int(name[2:])
        return I.he_atom().scaled(n, h=0.3 * 32 / n)
    raise SystemExit(f"unknown workload {name}")


def k1_bytes_per_launch(n_orb, nsite, s, scheme, wmode=False):
    """Algorithmic HBM bytes of one stream-collide launch: per orbital-site 2 Q s
    (populations in and out) + s (psi_hat stencil centre, read once) + s (psi out);
    per site s (potential).  The collapsed scheme moves only 2 s per orbital-site + s.
    With the orthogonalisation source W, psi* is read too: s more per orbital-site."""
    w = n_orb * s if wmode else 0
    if scheme == 0:
        return nsite * (n_orb * (2 * 19 * s + 2 * s) + s + w)
    return nsite * (n_orb * 2 * s + s + w)


def measured_traffic(key):
    """HBM bytes per stream-collide launch from the committed counter runs, or None
    when the kernel sources changed since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    h = hashlib.sha256()
    for p in d["kernel_sources"]:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    if h.hexdigest() != d["kernel_sha256"]:
        return None
    return d.get(key)


def cpu_baseline(system, steps, steps_1t):
    """The FP64 CPU oracle, as it stands, on a bounded sample of the same workload:
    `steps` steps on every thread the OpenMP runtime offers, then `steps_1t` steps on
    one thread (the oracle's results do not depend on the thread count)."""
    from oracle import oracle as O
    threads = O.max_threads()
    o = O.oracle_for(system)
    o.step()                      # warm caches / first-touch

    def rate(k):
        t0 = time.perf_counter()
        for _ in range(k):
            o.step()
        return system.n_orb * system.n_sites * k / (time.perf_counter() - t0)

    v = rate(steps)
    O.set_threads(1)
    try:
        v1 = rate(steps_1t)
    finally:
        O.set_threads(threads)
    return {"value": v, "unit": "orbital-site updates/s", "cores": threads, "kind": "oracle",
            "value_1_thread": v1,
            "sample": f"{steps} oracle steps of the same workload ({system.name} "
                      f"{system.dims[0]}^3, {system.n_orb} orbitals, FP64) after 1 untimed step on "
                      f"{threads} threads, then {steps_1t} steps on 1 thread"}


def copy_calibration(nbytes, iters):
    """Bandwidth of the library's plain 16-byte-per-lane copy kernel (read + write)."""
    import ctypes
    import torch
    from paper_1507_07666_amd import lbks
    L = lbks.load()
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").uniform_()
    dst = torch.empty_like(src)
    st = torch.cuda.current_stream()
    for _ in range(3):
        L.lbks_copy_kernel(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes,
                           ctypes.c_void_p(st.cuda_stream))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(iters):
        L.lbks_copy_kernel(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes,
                           ctypes.c_void_p(st.cuda_stream))
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / iters
    assert torch.equal(src, dst)
    return {"mode": "copy", "bytes_read": nbytes, "bytes_moved": 2 * nbytes, "avg_us": ms * 1e3,
            "GBps": 2 * nbytes / (ms * 1e-3) / 1e9, "frac_of_8TBps": 2 * nbytes / (ms * 1e-3) / 8e12}


def golden_energy(name):
    """Converged total energy of a stored FP64 oracle reference (tests/golden), or None."""
    path = os.path.join(ROOT, "tests", "golden", f"{name}.json")
    if not os.path.exists(path):
        return None
    return json.load(open(path))["energies"]["e_total"]


def fp32_gain_run(max_steps=6000, chunk=100, tol=1e-5):
    """CH4 128^3 (the precision workload) from its seeded start, in FP64 and in FP32
    bulk on the GPU, each relaxed in chunks of `chunk` steps until its total energy
    (Hartree potential converged, lbks_energy) is within `tol` of the converged FP64
    oracle reference.  Wall time includes the energy evaluations."""
    import torch
    from paper_1507_07666_amd import inputs as I
    from paper_1507_07666_amd import lbks
    ref = golden_energy("ch4")
    if ref is None:
        return None
    sy = I.ch4()
    out = {"workload": f"CH4 128^3 at 0.2 bohr, 5 orbitals, seed {sy.seed}; time until |E - E_oracle| < {tol:g} Ha, "
                       f"energy checked every {chunk} steps", "e_oracle": ref, "tol_Ha": tol}
    for name, prec in (("fp64", lbks.LBKS_FP64), ("fp32", lbks.LBKS_FP32_BULK)):
        s = lbks.Solver.for_system(sy, precision=prec)
        v, _ = s.autotune(reps=3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps, e = 0, None
        while steps < max_steps:
            s.relax(chunk)
            steps += chunk
            e = s.energy()["e_total"]
            if abs(e - ref) < tol:
                break
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        s.close()
        out[name] = {"wall_s": wall, "steps": steps, "dE_Ha": e - ref, "reached": abs(e - ref) < tol,
                     "update_variant": v}
    out["gain"] = out["fp64"]["wall_s"] / out["fp32"]["wall_s"]
    return out


def h2o_batch_run(count, check_every, max_steps):
    """64 H2O molecules (uneven grids) in one batch, FP32 bulk, until every one meets
    the FP32 stopping rule (energy within 2e-6 Ha and eigenvalue sum within 1e-6 Ha
    on two consecutive checks).  Returns the timing summary."""
    import torch
    from paper_1507_07666_amd import inputs as I
    from paper_1507_07666_amd import lbks
    from paper_1507_07666_amd.serve import FP32_RULE
    dE_tol = FP32_RULE["dE_tol"]
    systems = I.h2o_batch(count)
    b = lbks.Batch()
    members = [b.add_system(sy, precision=lbks.LBKS_FP32_BULK, deps_tol=FP32_RULE["deps_tol"],
                            stop_checks=FP32_RULE["stop_checks"]) for sy in systems]
    # update-kernel variant per grid size: timed on the first member of each size,
    # the others take the cached choice (outside the timed region)
    variants, tuned_us = {}, {}
    for sy, m in zip(systems, members):
        v, ms = m.autotune(reps=3)
        key = f"{sy.dims[0]}^3"
        if key not in variants:
            variants[key] = v
            tuned_us[key] = None if ms is None else [None if x is None else round(1e3 * x, 1) for x in ms]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, steps = b.relax(max_steps, dE_tol, check_every)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    upd = sum(sy.n_orb * sy.n_sites * k for sy, k in zip(systems, steps))
    # members with a stored FP64 oracle reference: their energy error
    dE = {}
    for i, m in enumerate(members):
        ref = golden_energy(f"h2o_{i}")
        if ref is not None:
            dE[i] = m.energy()["e_total"] - ref
    e = [m.energy()["e_total"] for m in members[:4]]
    b.close()
    return {"workload": f"{count} H2O, grids {{64,80,96,112}}^3 at 0.2 bohr, 5 orbitals, FP32 bulk, "
                        f"|dE| < {dE_tol:g} Ha and |d sum eps| < {FP32_RULE['deps_tol']:g} Ha per {check_every} "
                        f"steps on {FP32_RULE['stop_checks']} consecutive checks",
            "solves": count, "converged": sum(1 for x in st if x == lbks.LBKS_OK),
            "wall_s": wall, "h2o_solves_per_s": count / wall, "orbital_site_updates_per_s": upd / wall,
            "steps_min": min(steps), "steps_max": max(steps), "nodes_total": sum(sy.n_sites for sy in systems),
            "update_variants": variants,
            "update_variant_us": tuned_us,    # per-launch time of every variant timed, per grid size
            "e_total_first4": e,
            "dE_vs_oracle_Ha": {str(k): v for k, v in dE.items()},
            "max_abs_dE_vs_oracle_Ha": max((abs(v) for v in dE.values()), default=None)}


def bo_md_run(n_steps, n=80, softening=0.2):
    """Born-Oppenheimer dynamics of one H2O (80^3 at 0.2 bohr, FP32 bulk).  The
    geometry is first relaxed to zero force; then both O-H bonds are stretched by
    0.05 bohr and the molecule vibrates from rest under velocity Verlet (dt = 0.09
    fs), the electrons relaxed by the FP32 rule at every nuclear step from the
    previous step's orbitals.  The nuclear softening equals the grid spacing: with
    a much smaller one a nucleus moving between nodes sees its core density jump
    onto the nearest node (the energy falls by hartrees within a tenth of a
    spacing), which no dynamics survives.  Returns nuclear steps/s, lattice steps
    per nuclear step and the excursion of E_pot + E_kin against the swing of E_pot."""
    import numpy as np
    import torch
    from paper_1507_07666_amd import dynamics as Dy
    from paper_1507_07666_amd import inputs as I
    from paper_1507_07666_amd import lbks
    from paper_1507_07666_amd.serve import FP32_RULE
    sy = I.h2o_from_geometry(1.85, 1.75, 108.0, n, softening=softening, seed=11)
    s = lbks.Solver(lbks.params_for(sy, precision=lbks.LBKS_FP32_BULK, deps_tol=FP32_RULE["deps_tol"],
                                    stop_checks=FP32_RULE["stop_checks"]))
    s.set_nuclei(sy.Z, sy.R)
    rule = Dy.ElectronRule(dE_tol=FP32_RULE["dE_tol"], check_every=50)
    t0 = time.perf_counter()
    geo = Dy.relax_geometry(s, sy.Z, np.array(sy.R), ftol=2e-3, max_iter=300, rule=rule)
    t_geo = time.perf_counter() - t0
    R0 = geo.R.copy()
    for k in (1, 2):                                        # stretch both O-H bonds by 0.05 bohr
        u = (R0[k] - R0[0]) / np.linalg.norm(R0[k] - R0[0])
        R0[k] += 0.05 * u
    masses = [16.0 * Dy.AMU, Dy.PROTON_MASS, Dy.PROTON_MASS]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tr = Dy.bo_md(s, sy.Z, R0, np.zeros((3, 3)), masses, 0.09 * Dy.FS, n_steps, rule=rule)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s.close()
    oh = [float(np.linalg.norm(geo.R[k] - geo.R[0])) for k in (1, 2)]
    a, b = geo.R[1] - geo.R[0], geo.R[2] - geo.R[0]
    ang = float(np.degrees(np.arccos(a @ b / np.linalg.norm(a) / np.linalg.norm(b))))
    swing = float(tr.e_pot.max() - tr.e_pot.min())
    return {"metric": "Born-Oppenheimer nuclear steps/s", "value": n_steps / wall, "unit": "nuclear steps/s",
            "ms_per_nuclear_step": 1e3 * wall / n_steps,
            "lattice_steps_per_nuclear_step": float(np.mean(tr.lattice_steps[1:])),
            "e_pot_swing_Ha": swing,
            "e_total_excursion_Ha": float(np.max(np.abs(tr.e_total - tr.e_total[0]))),
            "geometry_relaxation": {"iterations": geo.iterations, "converged": geo.converged, "wall_s": t_geo,
                                    "O_H_bohr": oh, "angle_deg": ang},
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"H2O {n}^3 at 0.2 bohr, softening {softening}, FP32 bulk; relaxed to "
                                   f"|F| < 2e-3, O-H stretched by 0.05 bohr, velocity Verlet dt 0.09 fs, "
                                   f"{n_steps} steps from rest"}}


def serve_run(n_requests, rate, check_every, budget_gb, grids):
    """The seeded serving stream (seed 50) at `rate` Poisson arrivals per second,
    continuous batching under an HBM budget; p50/p99 latency from arrival to the
    last point's result, and solves (points) per second over the whole run."""
    from paper_1507_07666_amd import inputs as I
    from paper_1507_07666_amd import serve
    reqs = I.serving_stream(n_requests, rate=rate, seed=50, grids=grids)
    cfg = serve.ServeConfig(hbm_budget=int(budget_gb * (1 << 30)), check_every=check_every)
    srv = serve.Server(cfg)
    t0 = time.perf_counter()
    res = srv.run(reqs)
    wall = time.perf_counter() - t0
    srv.close()
    out = serve.summarize(res, wall)
    out.update({"rate_per_s": rate, "budget_gb": budget_gb, "peak_slots": srv.peak_active,
                "peak_bytes": srv.peak_used, "grids": list(grids),
                "workload": f"serving stream, seed 50, {n_requests} requests at {rate:g}/s (half atoms Z 1..10, "
                            f"half 8-point scans of CH4/NH3/H2O), grids {list(grids)}, h 0.2, FP32 bulk, FP32 rule",
                "all_converged": all(p.status == 0 for r in res for p in r.points)})
    return out


def cd_run(n_steps, h=0.01, restart_every=500):
    """Concurrent dynamics (complex orbitals in real time) on the Ne 96^3 FP64
    workload, nucleus fixed: the orbitals are relaxed to the ground state (|dE| <
    1e-9 Ha per 100 steps), then `n_steps` time-centred steps of h a.u. (a restart
    every `restart_every`) are timed (wall and the step kernel's HIP events; a
    restart counts as one launch).  Algorithmic bytes of one step-kernel launch:
    per orbital-site 48 B (psi^n at the node, psi^(n-1) in, psi^(n+1) out, complex
    FP64), per site 8 B (V)."""
    import torch
    from paper_1507_07666_amd import lbks
    sy = workload("ne96")
    s = lbks.Solver.for_system(sy)
    _, relax_steps = s.relax(8000, 1e-9, 100)
    s.cd_start(h, restart_every)
    e0 = s.cd_energy()["e_total"]
    s.cd_step(20)                           # warm-up
    torch.cuda.synchronize()
    s.set_timing(True)
    t0 = time.perf_counter()
    s.cd_step(n_steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms, k = s.kernel_time(1)
    e1 = s.cd_energy()["e_total"]
    s.cd_stop()
    s.close()
    alg = sy.n_sites * (sy.n_orb * 48 + 8)
    avg_s = ms / max(k, 1) * 1e-3
    return {"metric": "concurrent-dynamics steps/s", "value": n_steps / wall, "unit": "steps/s",
            "ms_per_step": 1e3 * wall / n_steps, "orbital_site_updates_per_s": sy.n_orb * sy.n_sites * n_steps / wall,
            "roofline": {"bound": "hbm", "kernel": "k_cd_step", "avg_us": avg_s * 1e6, "launches": k,
                         "alg_bytes_per_launch": alg, "achieved": alg / avg_s / 1e9, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": alg / avg_s / 1e9 / HBM_PEAK_GBS},
            "e_total_drift_Ha": e1 - e0, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"Ne atom 96^3 at 0.2 bohr, 5 orbitals, FP64, nucleus fixed, relaxed {relax_steps} "
                                   f"steps to the ground state, then time step {h} a.u. ({h / 41.341373335 * 1e3:.3f} as), "
                                   f"a restart every {restart_every} steps"}}


def sequential_run(dE_tol=1e-9, check_every=50):
    """The sequential Gram-Schmidt order against the concurrent one on the same
    Be atom (32^3 at 0.3 bohr, 2 orbitals, FP64, omega = 1 field update), both from
    the same seeded start to the same tolerances: lattice steps, wall time, and the
    difference of the converged total energies."""
    import torch
    from paper_1507_07666_amd import inputs as I
    from paper_1507_07666_amd import lbks
    sy = I.atom(4, 32, h=0.3, softening=0.3, seed=4)
    out = {"workload": "Be atom 32^3 at 0.3 bohr, softening 0.3, 2 orbitals, FP64, omega = 1 field update, "
                       f"|dE| < {dE_tol:g} Ha (and |d eps_k| < {dE_tol:g} Ha per stage) checked every {check_every} steps"}
    res = {}
    for order in ("concurrent", "sequential"):
        s = lbks.Solver(lbks.params_for(sy, init=lbks.LBKS_INIT_USER, scheme=lbks.LBKS_SCHEME_COLLAPSED))
        s.set_nuclei(sy.Z, sy.R)
        s.set_orbitals(sy.psi0())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if order == "concurrent":
            rc, steps = s.relax(200000, dE_tol, check_every)
            sweeps = None
        else:
            rc, steps, sweeps = s.relax_sequential(200000, dE_tol, dE_tol, check_every, 50)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        e = s.energy()
        s.close()
        res[order] = {"status": rc, "steps": steps, "sweeps": sweeps, "wall_s": wall, "e_total": e["e_total"],
                      "eps": [float(x) for x in e["eps"][:sy.n_orb]]}
    out.update(res)
    out["dE_sequential_minus_concurrent_Ha"] = res["sequential"]["e_total"] - res["concurrent"]["e_total"]
    out["steps_ratio"] = res["sequential"]["steps"] / max(1, res["concurrent"]["steps"])
    return out


def serve_sweep(n_requests, check_every, budget_gb, grids, factors=(0.25, 0.5, 1.0, 2.0)):
    """Saturation rate first (every request arrives at t = 0: requests/s of the
    drained queue), then Poisson arrivals of the same seeded stream at the given
    multiples of it; p50/p99 latency from arrival to the last point's result."""
    sat = serve_run(n_requests, 1e9, check_every, budget_gb, grids)
    lam = sat["requests_per_s"]
    print(f"[serve] saturation {lam:.3f} requests/s, {sat['solves_per_s']:.2f} solves/s", file=sys.stderr, flush=True)
    runs = []
    for f in factors:
        r = serve_run(n_requests, f * lam, check_every, budget_gb, grids)
        r["rate_factor"] = f
        print(f"[serve] rate {f} x saturation: p50 {r['p50_latency_s']:.2f} s, p99 {r['p99_latency_s']:.2f} s, "
              f"{r['solves_per_s']:.2f} solves/s", file=sys.stderr, flush=True)
        runs.append(r)
    return {"metric": "serving latency sweep", "saturation_requests_per_s": lam, "saturation": sat,
            "runs": runs, "data": "synthetic", "dtype": "f32",
            "config": {"workload": f"serving stream, seed 50, {n_requests} requests (half atoms Z 1..10, half "
                                   f"8-point scans of CH4/NH3/H2O), grids {list(grids)}, h 0.2"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="ne96")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--scheme", default="populations", choices=["populations", "collapsed"])
    ap.add_argument("--omega", type=float, default=1.0, help="relaxation parameter (populations only)")
    ap.add_argument("--ortho", default="gs", choices=["gs", "w"],
                    help="Cholesky Gram-Schmidt, or the paper's orthogonalisation source")
    ap.add_argument("--check-every", type=int, default=100)
    ap.add_argument("--hermite", type=int, default=2, choices=[2, 4],
                    help="order of the equilibrium and source weights")
    ap.add_argument("--fold", type=int, default=0, choices=[0, -1],
                    help="-1: the overlap and multipole totals always by their own reduction kernels")
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true", help="skip the per-kernel HIP events")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default update-kernel variant")
    ap.add_argument("--variant", type=int, default=None, help="fix the update-kernel variant (no autotuning)")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--requests", type=int, default=12)
    ap.add_argument("--rate", type=float, default=0.5, help="serving arrivals per second")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the orbital-site update rate (no H2O batch, serving or FP32-gain legs)")
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--mode", default="solve", choices=["solve", "copy"],
                    help="copy: time the library's plain copy kernel (bandwidth calibration)")
    ap.add_argument("--copy-mib", type=int, default=678, help="bytes read (= written) by one copy launch")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(independent solves would be spread over GPUs, and one large solve split "
              "into z-slabs).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1507_07666_amd import lbks

    torch.cuda.set_device(0)
    if args.mode == "copy":
        print(json.dumps(copy_calibration(args.copy_mib << 20, max(args.steps, 10))), flush=True)
        return
    if args.workload == "h2o_batch":
        print(json.dumps(h2o_batch_run(args.batch_count, 100, 20000)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(serve_run(args.requests, args.rate, 100, args.budget_gb, I_SERVE_GRIDS)), flush=True)
        return
    if args.workload == "bo_md":
        print(json.dumps(bo_md_run(max(2, args.steps // 15))), flush=True)
        return
    if args.workload == "cd":
        print(json.dumps(cd_run(args.steps)), flush=True)
        return
    if args.workload == "sequential":
        print(json.dumps(sequential_run()), flush=True)
        return
    if args.workload == "serve_sweep":
        print(json.dumps(serve_sweep(args.requests, 100, args.budget_gb, I_SERVE_GRIDS)), flush=True)
        return
    system = workload(args.workload)
    prec = lbks.LBKS_FP64 if args.precision == "fp64" else lbks.LBKS_FP32_BULK
    scheme = lbks.LBKS_SCHEME_POPULATIONS if args.scheme == "populations" else lbks.LBKS_SCHEME_COLLAPSED
    ortho = lbks.LBKS_ORTHO_GS if args.ortho == "gs" else lbks.LBKS_ORTHO_W
    solver = lbks.Solver.for_system(system, precision=prec, scheme=scheme, omega=args.omega, ortho=ortho,
                                    hermite=args.hermite, fold=args.fold)
    s_bytes = 8 if prec == lbks.LBKS_FP64 else 4

    if args.variant is not None:
        solver.set_variant(args.variant)
    if args.warmup:
        solver.relax(args.warmup)
    # the LDS-staged field update (collapsed scheme, Gram-Schmidt, at most five
    # orbitals) tunes its brick depth and workgroup order
    bricks = scheme == lbks.LBKS_SCHEME_COLLAPSED and system.n_orb <= 5 and ortho == lbks.LBKS_ORTHO_GS
    if args.no_autotune or args.variant is not None:
        variant, tune_ms = solver.variant(), None
    else:
        variant, tune_ms = solver.autotune(reps=5, force=True)
    torch.cuda.synchronize()
    if not args.no_timing:
        solver.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, steps = solver.relax(args.steps, dE_tol=1e-30, check_every=args.check_every)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    k1_ms, k1_n = solver.kernel_time() if not args.no_timing else (0.0, 0)
    e = solver.energy()
    fold_bits = solver.fold()
    solver.close()

    value = system.n_orb * system.n_sites * steps / elapsed
    out = {
        "metric": "orbital-site updates/s",
        "value": value,
        "unit": "orbital-site updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / max(1, steps),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == lbks.LBKS_FP64 else "f32",
        "data": "synthetic",
        "config": {"workload": f"{system.name} atom {system.dims[0]}^3 nodes, h={system.h} bohr, "
                               f"softening {system.softening}, {system.n_orb} orbitals, "
                               f"{args.precision} {args.scheme}, seed {system.seed}"
                               + (f", omega {args.omega}" if args.omega != 1.0 else "")
                               + (", fourth-order weights" if args.hermite == 4 else "")
                               + (", orthogonalisation source W" if args.ortho == "w" else ""),
                   "n_orb": system.n_orb, "nodes": system.n_sites, "check_every": args.check_every,
                   "omega": args.omega, "fold": fold_bits,
                   "update_variant": variant, "autotune_ms": tune_ms,
                   "parallelism": "single GPU"},
        "e_total": e["e_total"],
    }
    if k1_n:
        avg_s = k1_ms / k1_n * 1e-3
        alg = k1_bytes_per_launch(system.n_orb, system.n_sites, s_bytes, scheme, ortho == lbks.LBKS_ORTHO_W)
        ach = alg / avg_s / 1e9
        tkey = f"{args.workload}_{args.precision}_" + (f"v{variant}" if scheme == 0
                                                       else f"collapsed_v{variant}" if bricks else "")
        out["roofline"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": ach / HBM_PEAK_GBS, "traffic": measured_traffic(tkey) if tkey else None,
                           "kernel": ("k_stream_collide_wide" if variant is not None and variant & 8 and system.n_orb <= 5
                                      else "k_stream_collide") if scheme == 0
                           else "k_collapsed_brick" if bricks else "k_collapsed",
                           "avg_us": avg_s * 1e6, "launches": k1_n, "alg_bytes_per_launch": alg}
        # the same bytes against what a plain copy kernel reaches on this GPU
        cp = copy_calibration(678 << 20, 20)
        out["roofline"]["copy_GBps"] = cp["GBps"]
        out["roofline"]["frac_of_copy"] = ach / cp["GBps"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(system, args.cpu_steps, max(1, args.cpu_steps // 5))
    if not args.no_extras and args.workload == "ne96":
        # the other two parts of the metric, and the FP32-vs-FP64 time to the same accuracy
        print("[bench] 64 H2O batch", file=sys.stderr, flush=True)
        out["h2o_batch"] = h2o_batch_run(args.batch_count, 100, 20000)
        print("[bench] serving", file=sys.stderr, flush=True)
        out["serving"] = serve_run(args.requests, args.rate, 100, args.budget_gb, I_SERVE_GRIDS)
        print("[bench] FP32 gain", file=sys.stderr, flush=True)
        out["fp32_gain"] = fp32_gain_run()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
