"""Full-size workloads against converged FP64 oracle references.

The references in tests/golden/ are written by tests/golden/make_golden.py,
which runs only the CPU oracle (seeded inputs, the same stopping rule).
  * Ne, 96^3 at 0.2 bohr, FP64: same number of steps to |dE| < 1e-8 per 100
    steps, total energy within 1e-10 relative, density within 1e-9 at sampled
    nodes;
  * CH4, 128^3, FP32 bulk against the FP64 oracle: |dE| <= 1e-5 Ha, density
    relative L2 <= 1e-4 (on every second node), and the eigenvalues level by
    level: every Ritz value of the GPU state's projected operator within 1e-5 Ha
    of the oracle's, and every reported eps_j within 1e-5 Ha of its level where
    the run has separated that level from the others (then the run continues
    until the 0.15 Ha gap above the a1 level is separated too);
  * the 64-molecule H2O batch, FP32, one launch per kernel: members with a
    reference meet the same FP32 bars; the others meet them against the same
    molecules relaxed in FP64 on the GPU.
The FP32 solves stop by the FP32 rule of the serving module (energy and
eigenvalue sum settled on two consecutive checks).  Nearly degenerate levels
(the t2 levels of CH4 split by its unequal bonds) separate only as
exp(-dt g steps); their reported eigenvalues are Rayleigh quotients of orbitals
still rotating inside the level set, while the Ritz values are not.
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


def resolvable(levels, dt, steps, bound=1e-6):
    """Per level (ascending): can a run of `steps` steps report it alone?  An orbital
    that still mixes in level k, a gap g away, with amplitude exp(-dt g steps) (at
    most 1 after Gram-Schmidt) has a Rayleigh quotient off by up to
    sum_k g exp(-2 dt g steps); the level is resolvable when that is <= bound."""
    lv = np.sort(np.asarray(levels, dtype=np.float64))
    out = []
    for j in range(len(lv)):
        g = np.abs(np.delete(lv, j) - lv[j])
        out.append(float(np.sum(g * np.exp(-2.0 * dt * g * steps))) <= bound)
    return np.array(out)


def steps_to_resolve(levels, dt, j, bound=1e-6, every=100):
    """Smallest multiple of `every` steps at which level j is resolvable."""
    n = every
    while not resolvable(levels, dt, n, bound)[j]:
        n += every
    return n


def eigen_bars(s, e, ritz_ref, dt, steps, tol=1e-5, tag=""):
    """Every level through the Ritz values of the GPU state's projected operator
    (rotation-invariant inside nearly degenerate levels), and the reported
    eigenvalues level by level wherever the run has separated them.  Returns
    (max |d ritz|, resolvable mask, per-level |d eps| or nan)."""
    ref = np.asarray(ritz_ref, dtype=np.float64)
    n = len(ref)
    _, ritz = s.hamiltonian()
    dr = np.abs(ritz - ref)
    res = resolvable(ref, dt, steps)
    got = np.sort(np.asarray(e["eps"][:n]))
    de = np.where(res, np.abs(got - ref), np.nan)
    say(f"{tag} levels {np.round(ref, 6).tolist()} |d ritz| {['%.1e' % x for x in dr]} "
        f"resolved at {steps} steps {res.tolist()} |d eps| {['%.1e' % x for x in de]}")
    assert dr.max() <= tol, (tag, dr)
    assert np.all(de[res] <= tol), (tag, de)
    return float(dr.max()), res, de


def fp32_bars(s, e, g, rho, dims, steps, tag=""):
    assert abs(e["e_total"] - g["energies"]["e_total"]) <= 1e-5, (e["e_total"], g["energies"]["e_total"])
    eigen_bars(s, e, g["ritz"], g["h"] ** 2 / 3.0, steps, tag=tag)
    return rho_checks(rho, g, dims, rel_l2=1e-4)


def test_ch4_fp32_against_fp64_oracle(L):
    g = golden("ch4")
    if "ritz" not in g:
        pytest.skip("reference without Ritz values")
    system = I.ch4()
    rule = g["rule"]
    dt = g["h"] ** 2 / 3.0
    say("CH4 128^3 FP32")
    s = solver(L, system, precision=L.LBKS_FP32_BULK, deps_tol=FP32_RULE["deps_tol"],
               stop_checks=FP32_RULE["stop_checks"])
    rc, steps = s.relax(4 * g["steps"], FP32_RULE["dE_tol"], rule["check_every"])
    assert rc == 0
    e = s.energy()
    _, rho = s.orbitals()
    err = fp32_bars(s, e, g, rho, system.dims, steps, tag="CH4 at the FP32 rule")
    say(f"CH4 FP32: steps {steps} (oracle {g['steps']}), dE {e['e_total'] - g['energies']['e_total']:.2e}, "
        f"rho rel L2 {err:.2e}")
    # a1 is 0.15 Ha below the t2 levels: run on until the bound separates it too
    need = steps_to_resolve(g["ritz"], dt, 1)
    if need > steps:
        s.relax(need - steps)
        e = s.energy()
        _, res, de = eigen_bars(s, e, g["ritz"], dt, need, tag=f"CH4 at {need} steps")
        assert res[0] and res[1], res
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
        _, ritz = s.hamiltonian()
        out.append((e, rho, k, ritz, s))
    return b, out


def test_h2o_batch_fp32_against_fp64(L):
    """The 64-molecule batch in FP32, one launch per kernel.  Members with an oracle
    reference meet the FP32 bars against it; every other member is checked against
    the same molecule relaxed in FP64 on the GPU (an FP64 batch, whose members
    equal single FP64 solves bit for bit), to the same bars."""
    refs = {int(f[4:-5]): f[:-5] for f in os.listdir(GOLD) if f.startswith("h2o_") and f.endswith(".json")}
    systems = I.h2o_batch(64)
    say("64 H2O FP32 batch")
    b32, fp32 = relax_batch(L, systems, L.LBKS_FP32_BULK, tol=FP32_RULE["dE_tol"], deps_tol=FP32_RULE["deps_tol"],
                            stop_checks=FP32_RULE["stop_checks"])
    bad = []
    for i, name in sorted(refs.items()):
        g = golden(name)
        if "ritz" not in g:
            pytest.skip(f"reference {name} without Ritz values")
        e, rho, k, _, s = fp32[i]
        try:
            err = fp32_bars(s, e, g, rho, systems[i].dims, k, tag=f"H2O {i}")
            say(f"H2O {i} ({systems[i].dims[0]}^3): steps {k} (oracle {g['steps']}), "
                f"dE {e['e_total'] - g['energies']['e_total']:.2e}, rho rel L2 {err:.2e}")
        except AssertionError as ex:
            bad.append(i)
            say(f"H2O {i}: outside the bars against the oracle: {ex}")
    others = [i for i in range(64) if i not in refs]
    # the FP64 reference is relaxed further than the FP32 rule (1e-9 per 100 steps),
    # so what is measured is the FP32 result's own distance from the fixed point
    say(f"{len(others)} H2O FP64 batch")
    b64, fp64 = relax_batch(L, [systems[i] for i in others], L.LBKS_FP64, max_steps=40000, tol=1e-9)
    rows = []
    for i, (e64, rho64, k64, ritz64, _) in zip(others, fp64):
        e32, rho32, k32, _, s32 = fp32[i]
        de = abs(e32["e_total"] - e64["e_total"])
        err = np.linalg.norm(rho32 - rho64) / np.linalg.norm(rho64)
        try:
            assert de <= 1e-5 and err <= 1e-4, (de, err)
            dr, res, deps = eigen_bars(s32, e32, ritz64, systems[i].h ** 2 / 3.0, k32, tag=f"H2O {i}")
            rows.append((i, systems[i].dims[0], k32, k64, de, dr, int(res.sum()), err))
        except AssertionError as ex:
            bad.append(i)
            say(f"H2O {i}: outside the bars against FP64: {ex}")
    for r in rows:
        say("H2O %2d (%d^3): steps fp32 %5d fp64 %5d  |dE| %.2e  max|d ritz| %.2e  levels resolved %d  "
            "rho rel L2 %.2e" % r)
    b32.close()
    b64.close()
    assert not bad, f"members outside the FP32 bars: {bad}"
