"""Full-size workloads against converged FP64 oracle references.

The references in tests/golden/ are written by tests/golden/make_golden.py,
which runs only the CPU oracle (seeded inputs, the same stopping rule).
  * Ne, 96^3 at 0.2 bohr, FP64: same number of steps to |dE| < 1e-8 per 100
    steps, total energy within 1e-10 relative, density within 1e-9 at sampled
    nodes;
  * CH4, 128^3, FP32 bulk against the FP64 oracle: |dE| <= 1e-5 Ha,
    |d eps_j| <= 1e-5 Ha, density relative L2 <= 1e-4 (on every second node);
  * the 64-molecule H2O batch, FP32, one launch per kernel: members with a
    reference meet the same FP32 bars; the others meet them against the same
    molecules relaxed in FP64 on the GPU.
The FP32 solves stop by the FP32 rule of the serving module (energy and
eigenvalue sum settled on two consecutive checks).
"""
import json
import os
import sys

import numpy as np
import pytest

from paper_1507_07666_amd import inputs as I
from paper_1507_07666_amd.serve import FP32_RULE

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    path = os.path.join(GOLD, f"{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"reference {name} not generated")
    g = json.load(open(path))
    g["rho_sub"] = np.load(os.path.join(GOLD, f"{name}_rho.npz"))["rho_sub"].astype(np.float64)
    return g


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_1507_07666_amd import lbks
    lbks.load()
    return lbks


def say(*a):
    print("[gpu-workload]", *a, file=sys.stderr, flush=True)


def solver(L, system, **kw):
    s = L.Solver(L.params_for(system, init=L.LBKS_INIT_USER, **kw))
    s.set_nuclei(system.Z, system.R)
    s.set_orbitals(system.psi0())
    return s


def rho_checks(rho, g, dims, max_abs=None, rel_l2=None):
    nx, ny, nz = dims
    flat = rho.ravel()
    idx = np.array(g["sample_nodes"])
    ref = np.array(g["rho_samples"])
    if max_abs is not None:
        assert np.max(np.abs(flat[idx] - ref)) <= max_abs
    sub = rho.reshape(nz, ny, nx)[::2, ::2, ::2]
    err = np.linalg.norm(sub - g["rho_sub"]) / np.linalg.norm(g["rho_sub"])
    if rel_l2 is not None:
        assert err <= rel_l2, err
    return err


def test_ne_fp64_converged_against_oracle(L):
    g = golden("ne96")
    system = I.ne_atom()
    rule = g["rule"]
    say("Ne 96^3 FP64, stopping rule")
    s = solver(L, system)
    rc, steps = s.relax(rule["max_steps"], rule["dE_tol"], rule["check_every"])
    assert rc == 0 and abs(steps - g["steps"]) <= rule["check_every"]
    s.close()
    say("Ne 96^3 FP64, fixed steps", g["steps"])
    s = solver(L, system)
    s.relax(g["steps"])
    e = s.energy()
    ref = g["energies"]
    assert abs(e["e_total"] - ref["e_total"]) <= 1e-10 * abs(ref["e_total"])
    for k in ("e_kin", "e_ext", "e_hartree", "e_x", "e_c", "n_electrons"):
        assert abs(e[k] - ref[k]) <= 1e-10 * max(1.0, abs(ref[k])), k
    assert np.allclose(e["eps"], g["eps"], rtol=0, atol=1e-10 * np.max(np.abs(g["eps"])))
    _, rho = s.orbitals()
    # sampled nodes are stored in FP64 (the 1e-9 bar); the every-second-node field
    # is stored in FP32, so it can only confirm agreement to its own precision
    rho_checks(rho, g, system.dims, max_abs=1e-9, rel_l2=1e-6)
    s.close()


def level_clusters(eps, gap):
    """Sorted levels grouped where neighbours lie closer than `gap`."""
    order = np.sort(np.asarray(eps))
    groups = [[order[0]]]
    for x in order[1:]:
        if x - groups[-1][-1] < gap:
            groups[-1].append(x)
        else:
            groups.append([x])
    return groups


def eps_bars(eps, eps_ref, dt, steps, tol=1e-5):
    """Two levels a gap g apart stop mixing only as exp(-dt g steps); until then the
    individual orbital energies depend on the path.  What is unique is each level
    separated from the others by g > ln(1e4) / (dt steps) and the sum over each
    cluster closer than that (the trace of the operator on the cluster's subspace).
    `steps` is that of the less relaxed of the two runs compared."""
    ref = level_clusters(eps_ref, np.log(1e4) / (dt * steps))
    got = np.sort(np.asarray(eps))
    k = 0
    for grp in ref:
        m = len(grp)
        mine = got[k:k + m]
        k += m
        if m == 1:
            assert abs(mine[0] - grp[0]) <= tol, (mine, grp)
        else:
            assert abs(mine.sum() - sum(grp)) <= tol * m, (mine, grp)


def fp32_bars(e, g, rho, dims, steps):
    assert abs(e["e_total"] - g["energies"]["e_total"]) <= 1e-5, (e["e_total"], g["energies"]["e_total"])
    eps_bars(e["eps"], g["eps"], g["h"] ** 2 / 3.0, min(steps, g["steps"]))
    return rho_checks(rho, g, dims, rel_l2=1e-4)


def test_ch4_fp32_against_fp64_oracle(L):
    g = golden("ch4")
    system = I.ch4()
    rule = g["rule"]
    say("CH4 128^3 FP32")
    s = solver(L, system, precision=L.LBKS_FP32_BULK, deps_tol=FP32_RULE["deps_tol"],
               stop_checks=FP32_RULE["stop_checks"])
    rc, steps = s.relax(4 * g["steps"], FP32_RULE["dE_tol"], rule["check_every"])
    assert rc == 0
    e = s.energy()
    _, rho = s.orbitals()
    say("CH4 FP32 eps", list(e["eps"]), "oracle", g["eps"], "E", e["e_total"], g["energies"]["e_total"])
    err = fp32_bars(e, g, rho, system.dims, steps)
    say(f"CH4 FP32: steps {steps} (oracle {g['steps']}), dE {e['e_total'] - g['energies']['e_total']:.2e}, "
        f"rho rel L2 {err:.2e}")
    s.close()


def relax_batch(L, systems, precision, max_steps=12000, tol=1e-7, every=100, **rule):
    """Relax the systems as one batch; per member (energies, density, steps)."""
    b = L.Batch()
    members = []
    for sy in systems:
        s = b.add(L.params_for(sy, init=L.LBKS_INIT_USER, precision=precision, **rule))
        s.set_nuclei(sy.Z, sy.R)
        s.set_orbitals(sy.psi0())
        members.append(s)
    st, steps = b.relax(max_steps, tol, every)
    assert all(x == L.LBKS_OK for x in st), st
    out = []
    for s, k in zip(members, steps):
        e = s.energy()
        _, rho = s.orbitals()
        out.append((e, rho, k))
    b.close()
    return out


def test_h2o_batch_fp32_against_fp64(L):
    """The 64-molecule batch in FP32, one launch per kernel.  Members with an oracle
    reference meet the FP32 bars against it; every other member is checked against
    the same molecule relaxed in FP64 on the GPU (an FP64 batch, whose members
    equal single FP64 solves bit for bit), to the same bars."""
    refs = {int(f[4:-5]): f[:-5] for f in os.listdir(GOLD) if f.startswith("h2o_") and f.endswith(".json")}
    systems = I.h2o_batch(64)
    say("64 H2O FP32 batch")
    fp32 = relax_batch(L, systems, L.LBKS_FP32_BULK, tol=FP32_RULE["dE_tol"], deps_tol=FP32_RULE["deps_tol"],
                       stop_checks=FP32_RULE["stop_checks"])
    for i, name in sorted(refs.items()):
        g = golden(name)
        e, rho, k = fp32[i]
        err = fp32_bars(e, g, rho, systems[i].dims, k)
        say(f"H2O {i} ({systems[i].dims[0]}^3): steps {k} (oracle {g['steps']}), "
            f"dE {e['e_total'] - g['energies']['e_total']:.2e}, rho rel L2 {err:.2e}")
    others = [i for i in range(64) if i not in refs]
    # the FP64 reference is relaxed further than the FP32 rule (1e-9 per 100 steps),
    # so what is measured is the FP32 result's own distance from the fixed point
    say(f"{len(others)} H2O FP64 batch")
    fp64 = relax_batch(L, [systems[i] for i in others], L.LBKS_FP64, max_steps=40000, tol=1e-9)
    rows, bad = [], []
    for i, (e64, rho64, k64) in zip(others, fp64):
        e32, rho32, k32 = fp32[i]
        de = abs(e32["e_total"] - e64["e_total"])
        err = np.linalg.norm(rho32 - rho64) / np.linalg.norm(rho64)
        deps = np.abs(np.sort(e32["eps"]) - np.sort(e64["eps"][:systems[i].n_orb]))
        rows.append((i, systems[i].dims[0], k32, k64, de, float(deps.max()), err))
        try:
            assert de <= 1e-5 and err <= 1e-4
            eps_bars(e32["eps"], e64["eps"][:systems[i].n_orb], systems[i].h ** 2 / 3.0, min(k32, k64))
        except AssertionError:
            bad.append(i)
            say(f"H2O {i}: eps fp32 {np.sort(e32['eps'])} fp64 {np.sort(e64['eps'][:systems[i].n_orb])}")
    for r in rows:
        say("H2O %2d (%d^3): steps fp32 %5d fp64 %5d  |dE| %.2e  max|d eps| %.2e  rho rel L2 %.2e" % r)
    assert not bad, f"members outside the FP32 bars: {bad}"
