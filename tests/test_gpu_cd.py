"""Concurrent dynamics on the GPU (lbks_cd_*) against the oracle's
ConcurrentDynamics on the same seeded inputs: the complex orbitals, the
energies and the forces after the same steps (FP64, 1e-10), with the nuclei
fixed and with the nuclei moved by the same velocity-Verlet loop on both sides;
the calls' state rules and stability check; and the H2 vibration of the
concurrent scenario next to Born-Oppenheimer dynamics on the same grid."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1507_07666_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_1507_07666_amd import lbks
    lbks.load()
    return lbks


def say(*a):
    print("[gpu-cd]", *a, file=sys.stderr, flush=True)


def relaxed_pair(L, system, steps, sweeps=4):
    """GPU solver and oracle, both relaxed the same number of steps from the seeded start."""
    p = L.params_for(system, init=L.LBKS_INIT_USER, poisson_sweeps=sweeps)
    s = L.Solver(p)
    s.set_nuclei(system.Z, system.R)
    s.set_orbitals(system.psi0())
    s.relax(steps)
    o = O.oracle_for(system, poisson_sweeps=sweeps)
    for _ in range(steps):
        o.step()
    return s, o


def compare(s, cd, tol=1e-10, energies=True):
    psi = s.cd_orbitals().reshape(cd.cur.shape)
    scale = np.max(np.abs(cd.cur))
    assert np.max(np.abs(psi - cd.cur)) <= tol * scale, np.max(np.abs(psi - cd.cur)) / scale
    if energies:
        e = s.cd_energy()
        eo = cd.energies(converge_poisson=True)
        assert abs(e["e_total"] - eo.e_total) <= tol * abs(eo.e_total), (e["e_total"], eo.e_total)
        assert np.allclose(e["eps"][:len(eo.eps)], eo.eps, rtol=0, atol=tol * max(1.0, np.abs(eo.eps).max()))
        assert abs(e["n_electrons"] - eo.n_electrons) <= tol * eo.n_electrons


@pytest.mark.parametrize("case,restart", [("he_shift", 0), ("ne_5orb", 0), ("he_shift", 20), ("ne_5orb", 7)])
def test_cd_matches_oracle_with_fixed_nuclei(L, case, restart):
    if case == "he_shift":
        system = I.System("He", (16, 16, 16), 0.35, [2.0], [(0.15, 0.0, 0.0)], 2, 1, 0.3, seed=5)
        steps, h, n = 1500, 0.015, 60
    else:
        system = I.ne_atom().scaled(18, h=0.3)
        system.softening = 0.3
        steps, h, n = 300, 0.004, 25
    say("fixed nuclei", case, "restart every", restart)
    s, o = relaxed_pair(L, system, steps)
    if case == "he_shift":                              # a sudden shift: the density sloshes
        s.set_nuclei([2.0], [[0.0, 0.0, 0.0]])
        o.set_nuclei([2.0], [[0.0, 0.0, 0.0]])
    s.cd_start(h, restart)
    cd = O.ConcurrentDynamics(o, h, restart_every=restart)
    compare(s, cd, energies=False)
    s.cd_step(n)
    for _ in range(n):
        cd.step()
    compare(s, cd)
    F = s.forces()
    Fo = cd.forces()
    assert np.max(np.abs(F - Fo)) <= 1e-10 * max(1.0, np.abs(Fo).max())
    s.cd_step(5)                                        # continues after an energy evaluation
    for _ in range(5):
        cd.step()
    compare(s, cd)
    s.cd_stop()
    s.close()


def test_cd_with_moving_nuclei_matches_oracle(L):
    """H2 (20^3 at 0.35 bohr, softening 0.3) stretched from its relaxed bond: the
    same velocity-Verlet loop drives the GPU dynamics (lbks_cd_*, lbks_forces,
    lbks_set_nuclei) and the oracle's, both restarting every 15 steps."""
    from paper_1507_07666_amd import dynamics as Dy
    system = I.System("H2", (20, 20, 20), 0.35, [1.0, 1.0], [(-0.75, 0.0, 0.0), (0.75, 0.0, 0.0)], 2, 1, 0.3,
                      seed=6)
    say("moving nuclei")
    s, o = relaxed_pair(L, system, 600)
    dt, n = 0.03, 40
    M = np.array([[Dy.PROTON_MASS], [Dy.PROTON_MASS]])
    R0 = np.array(system.R, dtype=np.float64)
    tr = Dy.cd_md(s, system.Z, R0, np.zeros((2, 3)), [Dy.PROTON_MASS] * 2, dt, n, restart_every=15)
    # the oracle with the same loop
    o.set_nuclei(system.Z, R0)
    Fo = o.forces()                                     # forces of the relaxed state
    cd = O.ConcurrentDynamics(o, dt, restart_every=15)
    R, V = R0.copy(), np.zeros((2, 3))
    for k in range(n):
        R = R + V * dt + Fo / (2.0 * M) * dt * dt
        o.set_nuclei(system.Z, R)
        Fn = cd.forces()
        V = V + (Fo + Fn) / (2.0 * M) * dt
        Fo = Fn
        if k + 1 < n:
            cd.step()
    assert np.max(np.abs(tr.R[-1] - R)) <= 1e-12 * np.abs(R).max() + 1e-14
    assert np.max(np.abs(tr.V[-1] - V)) <= 1e-9 * max(np.abs(V).max(), 1e-12)
    compare(s, cd)
    s.cd_stop()
    s.close()


def test_cd_state_rules_and_stability_check(L):
    system = I.he_atom().scaled(14, h=0.4)
    s = L.Solver.for_system(system)
    s.relax(200)
    with pytest.raises(L.LbksError):
        s.cd_step(1)                                    # not started
    with pytest.raises(L.LbksError):
        s.cd_start(1.0)                                 # far beyond the stable step
    s.cd_start(0.01)
    for call in (lambda: s.relax(1), s.energy, s.orbitals, s.hamiltonian):
        with pytest.raises(L.LbksError) as ex:
            call()
        assert ex.value.code == L.LBKS_E_STATE
    s.set_timing(True)
    s.cd_step(3)
    ms, launches = s.kernel_time(1)                    # the CD step kernel, timed per launch
    assert launches == 3 and ms > 0.0
    assert s.kernel_time(0) == (0.0, 0)                # no update-kernel launch in the dynamics
    s.set_timing(False)
    e = s.cd_energy()
    assert e["steps"] == 3 and np.isfinite(e["e_total"])
    s.cd_stop()
    s.relax(5)                                          # back to the relaxation
    s.close()
    f = L.Solver.for_system(system, precision=L.LBKS_FP32_BULK)
    with pytest.raises(L.LbksError) as ex:
        f.cd_start(0.01)
    assert ex.value.code == L.LBKS_E_INVAL
    f.close()


def test_h2_vibration_concurrent_and_born_oppenheimer(L):
    """The paper's comparison (results section, H2 on a 24^3 lattice): the bond,
    stretched by 0.1 bohr from its relaxed length, vibrates under Born-Oppenheimer
    dynamics (electrons relaxed at each nuclear step, 0.09 fs) and under the
    concurrent scheme with the paper's step of 0.0014 fs (stable here for a
    spacing of 0.45 bohr; the softening equals the spacing) and a restart every
    500 steps; the two frequencies agree within 2 % and the concurrent total
    energy stays within a tenth of the BO potential swing (3 % on the oracle)."""
    from paper_1507_07666_amd import dynamics as Dy
    n, hx, a = 24, 0.45, 0.45
    system = I.System("H2", (n, n, n), hx, [1.0, 1.0], [(-0.7, 0.0, 0.0), (0.7, 0.0, 0.0)], 2, 1, a, seed=7)
    Z = system.Z
    s = L.Solver(L.params_for(system, poisson_sweeps=4))
    s.set_nuclei(Z, system.R)
    rule = Dy.ElectronRule(dE_tol=1e-10, check_every=50)
    geo = Dy.relax_geometry(s, Z, np.array(system.R), ftol=1e-4, max_iter=200, rule=rule)
    d0 = float(np.linalg.norm(geo.R[1] - geo.R[0]))
    u = (geo.R[1] - geo.R[0]) / d0
    R0 = geo.R.copy()
    R0[0] -= 0.05 * u
    R0[1] += 0.05 * u
    masses = [Dy.PROTON_MASS] * 2
    T = 2.0 * 2 * np.pi / 0.0195                        # two periods of a 4300 cm^-1 mode
    dt_bo = 0.09 * Dy.FS
    say(f"H2 bond {d0:.4f} bohr; BO {int(T / dt_bo)} steps")
    bo = Dy.bo_md(s, Z, R0, np.zeros((2, 3)), masses, dt_bo, int(T / dt_bo), rule=rule)
    w_bo = Dy.vibration_frequency(bo.t, np.linalg.norm(bo.R[:, 1] - bo.R[:, 0], axis=1))
    dt_cd = 0.0014 * Dy.FS                              # the paper's concurrent time step
    s.set_nuclei(Z, R0)
    s.relax(40000, 1e-12, 50)                           # the ground state at the stretched geometry
    n_cd = int(T / dt_cd)
    say(f"CD {n_cd} steps of {dt_cd:.4f} a.u.")
    cd = Dy.cd_md(s, Z, R0, np.zeros((2, 3)), masses, dt_cd, n_cd, energy_every=n_cd // 20, restart_every=500)
    s.cd_stop()
    w_cd = Dy.vibration_frequency(cd.t, np.linalg.norm(cd.R[:, 1] - cd.R[:, 0], axis=1))
    cm = 219474.63                                       # cm^-1 per hartree
    swing = float(bo.e_pot.max() - bo.e_pot.min())
    etot = cd.e_pot + cd.e_kin
    say(f"H2 vibration: BO {w_bo * cm:.1f} cm^-1, CD {w_cd * cm:.1f} cm^-1; CD total-energy excursion "
        f"{np.ptp(etot):.2e} Ha against the BO potential swing {swing:.2e} Ha")
    assert np.isfinite(w_bo) and np.isfinite(w_cd)
    assert abs(w_cd / w_bo - 1.0) < 0.02
    assert np.ptp(etot) < 0.1 * swing
    s.close()
