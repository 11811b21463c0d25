"""Serving: requests arriving while others run are admitted as memory frees up,
share every launch with the solves already on the GPU, warm-start their scan
points in place, and give the same result as when solved alone."""
import sys

import numpy as np
import pytest

from paper_1507_07666_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_1507_07666_amd import lbks, serve
    lbks.load()
    return serve


def small_stream():
    reqs = I.serving_stream(6, rate=50.0, seed=50, grids=(20, 24), scan_points=3)
    for r in reqs:                       # coarser spacing keeps the boxes around the molecules
        for k, p in enumerate(r.points):
            r.points[k] = p.scaled(p.dims[0], h=0.4)
    return reqs


def test_served_results_equal_alone(S):
    from paper_1507_07666_amd import lbks
    print("[gpu-serve] mixed stream", file=sys.stderr, flush=True)
    reqs = small_stream()
    cfg = S.ServeConfig(hbm_budget=0, check_every=20, dE_tol=1e-7, chunks_per_call=2,
                        max_steps_per_point=3000)
    need = [S.point_bytes(r.points[0], cfg) for r in reqs]
    cfg.hbm_budget = int(sum(sorted(need)[-3:]))       # room for about three at a time
    srv = S.Server(cfg)
    res = srv.run(reqs)
    srv.close()
    assert srv.peak_active >= 2                          # work really overlapped
    assert srv.peak_used <= cfg.hbm_budget
    for r, out in zip(reqs, res):
        assert len(out.points) == len(r.points)
        ref = S.solve_alone(r, cfg)
        for a, b in zip(out.points, ref):
            assert a.steps == b.steps and a.status == b.status
            assert abs(a.e_total - b.e_total) <= 1e-5          # the contract; in practice identical
            assert a.e_total == b.e_total
            assert np.allclose(a.eps, b.eps, atol=1e-5)
        assert out.finished >= out.admitted >= out.arrival


def test_served_points_match_oracle(S):
    """The seeded serving subset (requests 0-7 of the seed-50 stream on 48^3 and
    64^3 grids: four 8-point geometry scans and four atoms), served in FP32 with
    continuous batching under a memory budget, against per-point FP64 oracle
    references (tests/golden/serve.json, written by make_golden.py from the oracle
    alone): |dE| <= 1e-5 Ha, every Ritz value of the occupied span within 1e-5 Ha,
    density relative L2 <= 1e-4 on every fourth node (open-shell atoms: the energy
    only).  A reference that stopped at the oracle's step limit is not the fixed
    point: carbon on 48^3 keeps a level 1e-4 Ha from the occupied span and its
    energy still falls by 1.5e-8 Ha per 100 steps at 40000 steps.  Such a point's
    energy bar is widened by how far the oracle's own checked energy moved after
    the step count where the served solve stopped (stored with the reference)."""
    import json
    import os
    from paper_1507_07666_amd import lbks
    path = os.path.join(os.path.dirname(__file__), "golden", "serve.json")
    if not os.path.exists(path):
        pytest.skip("serving references not generated")
    g = json.load(open(path))
    rho_ref = np.load(os.path.join(os.path.dirname(__file__), "golden", "serve_rho.npz"))
    reqs = I.serving_stream(g["requests"], rate=50.0, seed=g["seed"], grids=tuple(g["grids"]),
                            scan_points=g["scan_points"])
    print("[gpu-serve] oracle subset", len(reqs), "requests", file=sys.stderr, flush=True)
    cfg = S.ServeConfig(hbm_budget=0, detail=True)
    need = [S.point_bytes(r.points[0], cfg) for r in reqs]
    cfg.hbm_budget = int(sum(sorted(need)[-3:]))       # about three requests at a time
    srv = S.Server(cfg)
    res = srv.run(reqs)
    srv.close()
    assert srv.peak_active >= 2 and srv.peak_used <= cfg.hbm_budget
    refs = {(p["rid"], p["point"]): p for p in g["points"]}
    worst = dict(de=0.0, ritz=0.0, rho=0.0)
    for r, out in zip(reqs, res):
        assert len(out.points) == len(r.points)
        for k, pt in enumerate(out.points):
            ref = refs[(r.rid, k)]
            assert pt.status == lbks.LBKS_OK, (r.rid, k, pt.status)
            de = abs(pt.e_total - ref["energies"]["e_total"])
            dr = float(np.max(np.abs(np.asarray(pt.ritz) - np.asarray(ref["ritz"]))))
            rr = rho_ref[f"r{r.rid}_p{k}"].astype(np.float64)
            err = float(np.linalg.norm(pt.rho_sub4 - rr) / np.linalg.norm(rr))
            # atoms B..F fill a 2p level in part: in this closed-shell reading the
            # occupied p orbitals break the symmetry, which p is chosen and how fast
            # it separates from the others is not fixed, so only the energy is compared
            open_shell = ref["system"].startswith("Z") and 5 <= int(ref["system"][1:]) <= 9
            bar = 1e-5
            if ref["rc"] != 0:
                assert "checks" in ref, f"step-limited reference r{r.rid} p{k} without its checks (serve_trace)"
                checks = np.asarray(ref["checks"], dtype=np.float64)
                before = checks[checks[:, 0] <= pt.steps]
                e_then = before[-1, 1] if len(before) else checks[0, 1]
                bar += abs(e_then - checks[-1, 1])
            print(f"[gpu-serve] r{r.rid} p{k} {ref['system']} {ref['dims'][0]}^3 steps {pt.steps} "
                  f"(oracle {ref['steps']}, rc {ref['rc']}) dE {de:.1e} (bar {bar:.1e}) max|d ritz| {dr:.1e} "
                  f"rho {err:.1e}" + (" (open shell: energy only)" if open_shell else ""),
                  file=sys.stderr, flush=True)
            assert de <= bar, (r.rid, k, de, bar)
            if not open_shell:
                assert dr <= 1e-5 and err <= 1e-4, (r.rid, k, de, dr, err)
                worst = dict(de=max(worst["de"], de), ritz=max(worst["ritz"], dr), rho=max(worst["rho"], err))
    print("[gpu-serve] worst", worst, file=sys.stderr, flush=True)
