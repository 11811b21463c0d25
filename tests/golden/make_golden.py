"""Write converged FP64 oracle references for the full-size workloads.

Calls only oracle/ and the seeded input generators; nothing here touches the
GPU library.  Usage:  python tests/golden/make_golden.py ne96 ch4 serve ...
Each solve run writes tests/golden/<name>.json (relaxation rule, steps,
energies, eigenvalues, the projected operator H_jk and its Ritz values, density
norms and seeded node samples) and <name>_rho.npz (the density on every second
node per axis, float32).  "serve" writes serve.json and serve_rho.npz: every
point of the seeded serving subset (requests 0-7 of the seed-50 stream on 48^3
and 64^3 grids: four 8-point geometry scans and four atoms), scan points
warm-started from the previous point as the server does, with the density on
every fourth node per axis.  "serve_trace" re-runs, the same way, the requests
holding a point whose relaxation reached the 40000-step limit and adds to each of
their points the energies checked every 100 steps (Hartree potential as it
stands), so that a served point is compared with how far the oracle itself moved
after the step count where the served solve stopped.

The FP32 workloads' references (CH4, H2O, serving) are relaxed with the
omega = 1 field step of the oracle (Oracle.step_fields), which is the moment of
the population step and reaches the same fixed point with less work, to
|dE| < 1e-9 Ha per 100 steps; the Ritz values are then settled far below the
1e-5 Ha bar they are compared at.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1507_07666_amd import inputs as I  # noqa: E402

# name -> (system factory, dE_tol per check, check_every, max_steps, field step)
RUNS = {
    "ne96": (I.ne_atom, 1e-8, 100, 40000, False),
    "ch4": (I.ch4, 1e-9, 100, 40000, True),
    "he32": (I.he_atom, 0.0, 2000, 2000, False),
}
# the H2O references are relaxed well past the FP32 solves' own rule, so that
# they stand for the fixed point
for i, s in enumerate(I.h2o_batch(64)):
    if i in (0, 1, 2, 3, 4, 5, 6, 7):
        RUNS[f"h2o_{i}"] = (lambda s=s: s, 1e-9, 100, 40000, True)

N_SAMPLES = 4096
SERVE_REQUESTS = 8
SERVE_TOL = 1e-9


def serving_subset():
    """The seeded serving requests with oracle references (rate does not change
    the systems, only the arrival times)."""
    return I.serving_stream(SERVE_REQUESTS, rate=1.0, seed=50, grids=(48, 64), scan_points=8)


def sample_nodes(n_sites, seed=12345):
    return np.sort(I.splitmix64(seed, np.arange(N_SAMPLES, dtype=np.uint64)) % np.uint64(n_sites)).astype(np.int64)


def energies_dict(e):
    return {k: float(getattr(e, k)) for k in ("e_total", "e_kin", "e_ext", "e_hartree", "e_x", "e_c", "e_nn",
                                               "n_electrons", "poisson_residual")}


def run(name):
    factory, tol, every, max_steps, fields = RUNS[name]
    system = factory()
    t0 = time.time()
    o = O.oracle_for(system)
    log = []

    def progress(steps, e):
        log.append((steps, e))
        print(f"[{name}] step {steps} E {e:.12f} ({time.time() - t0:.0f}s)", flush=True)

    rc, steps = o.relax(max_steps, tol, every, progress=progress, fields=fields)
    e = o.energies(converge_poisson=True)
    H, ritz = o.hamiltonian(converge_poisson=False)      # V_H converged just above
    psihat, rho = o.state()
    nx, ny, nz = system.dims
    idx = sample_nodes(system.n_sites)
    out = {
        "name": name, "system": system.name, "dims": list(system.dims), "h": system.h,
        "Z": list(system.Z), "R": [list(r) for r in system.R], "n_elec": system.n_elec,
        "n_orb": system.n_orb, "softening": system.softening, "seed": system.seed,
        "rule": {"dE_tol": tol, "check_every": every, "max_steps": max_steps},
        "path": "field step (omega = 1)" if fields else "population step",
        "rc": rc, "steps": steps,
        "energies": energies_dict(e),
        "eps": [float(x) for x in e.eps],
        "H": H.tolist(), "ritz": [float(x) for x in ritz],
        "rho_l2": float(np.linalg.norm(rho)), "rho_max": float(rho.max()),
        "sample_nodes": idx.tolist(), "rho_samples": rho[idx].tolist(),
        "trace": log, "wall_s": time.time() - t0,
        "threads": O.max_threads(),
    }
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f)
    sub = rho.reshape(nz, ny, nx)[::2, ::2, ::2].astype(np.float32)
    np.savez_compressed(os.path.join(HERE, f"{name}_rho.npz"), rho_sub=sub)
    print(f"[{name}] done rc={rc} steps={steps} E={e.e_total:.12f} ritz={ritz} in {time.time() - t0:.0f}s",
          flush=True)


def serve_request(r, t0, points, rho4, trace=False):
    """Relax every point of request r as the server does (scan points warm-started
    from the previous one); append its records to points and its density to rho4."""
    o = None
    for k, sy in enumerate(r.points):
        if o is None:
            o = O.oracle_for(sy)
        else:
            o.set_nuclei(sy.Z, sy.R)                 # warm start from the previous scan point
        checks = []
        rc, steps = o.relax(40000, SERVE_TOL, 100, fields=True,
                            progress=(lambda n, e: checks.append([int(n), float(e)])) if trace else None)
        e = o.energies(converge_poisson=True)
        H, ritz = o.hamiltonian(converge_poisson=False)
        _, rho = o.state()
        nx, ny, nz = sy.dims
        key = f"r{r.rid}_p{k}"
        rho4[key] = rho.reshape(nz, ny, nx)[::4, ::4, ::4].astype(np.float32)
        points.append({"rid": r.rid, "point": k, "system": sy.name, "dims": list(sy.dims), "h": sy.h,
                       "Z": list(sy.Z), "R": [list(x) for x in sy.R], "n_orb": sy.n_orb,
                       "n_elec": sy.n_elec, "rc": rc, "steps": steps, "energies": energies_dict(e),
                       "eps": [float(x) for x in e.eps], "ritz": [float(x) for x in ritz],
                       "rho_l2_sub4": float(np.linalg.norm(rho4[key]))})
        if trace:
            points[-1]["checks"] = checks
        print(f"[serve] r{r.rid} p{k} {sy.name} {sy.dims[0]}^3 rc={rc} steps={steps} E={e.e_total:.10f} "
              f"({time.time() - t0:.0f}s)", flush=True)


def run_serve():
    t0 = time.time()
    reqs = serving_subset()
    points, rho4 = [], {}
    for r in reqs:
        serve_request(r, t0, points, rho4)
    out = {"requests": SERVE_REQUESTS, "seed": 50, "grids": [48, 64], "scan_points": 8,
           "rule": {"dE_tol": SERVE_TOL, "check_every": 100}, "path": "field step (omega = 1)",
           "points": points, "wall_s": time.time() - t0, "threads": O.max_threads()}
    with open(os.path.join(HERE, "serve.json"), "w") as f:
        json.dump(out, f)
    np.savez_compressed(os.path.join(HERE, "serve_rho.npz"), **rho4)


def run_serve_trace():
    """Re-run the requests with a step-limited point and store their check energies
    (the records must come out as they are stored: same steps and energies)."""
    t0 = time.time()
    path = os.path.join(HERE, "serve.json")
    with open(path) as f:
        g = json.load(f)
    reqs = {r.rid: r for r in serving_subset()}
    limited = sorted({p["rid"] for p in g["points"] if p["rc"] != 0})
    for rid in limited:
        points, rho4 = [], {}
        serve_request(reqs[rid], t0, points, rho4, trace=True)
        for new in points:
            old = next(p for p in g["points"] if p["rid"] == rid and p["point"] == new["point"])
            assert old["steps"] == new["steps"] and old["energies"]["e_total"] == new["energies"]["e_total"], \
                (rid, new["point"], old["energies"]["e_total"], new["energies"]["e_total"])
            old["checks"] = new["checks"]
    with open(path, "w") as f:
        json.dump(g, f)


if __name__ == "__main__":
    for n in sys.argv[1:]:
        if n == "serve":
            run_serve()
        elif n == "serve_trace":
            run_serve_trace()
        else:
            run(n)
