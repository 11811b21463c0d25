"""Pins of the oracle's concurrent dynamics (section on concurrent dynamics, eq.
KSLBCD, in the reading of Oracle.ConcurrentDynamics: complex orbitals advanced by
the two-step time-centred scheme psi_j^{n+1} = psi_j^{n-1} - 2 i h (H - E_j) psi_j^n
with the relaxation's operator H = K_h + S_chi(V .) and each orbital's energy
reference E_j):

  * one step equals the same step written with the dense matrix H = (I - M)/dt,
    M = S_xi - dt S_chi diag(V), built independently (fixed potential, 12^3);
  * with V = 0, H is symmetric and the scheme conserves Re h^3 <psi^{n-1}|psi^n>
    exactly (to rounding) for every orbital;
  * an eigenstate of H started with its exact second level psi^1 = e^{-i theta}
    psi^0 rotates rigidly: psi^n = e^{-i n theta} psi^0 with
    sin(theta) = h (eps - E), eps from the dense eigenproblem (E = 0 here); with
    the default reference E = eps it stands still;
  * the reference keeps the self-consistent dynamics stable over thousands of
    steps where the plain scheme's parasitic mode grows (H2, 24^3 at 0.45 bohr,
    the paper's 0.0014 fs);
  * with the nuclei moving (the same H2 vibrating from a stretched bond) the
    fixed reference no longer suffices and the parasitic mode grows back, while
    the periodic restart (reference re-centred, one-step start) holds the total
    energy of electrons and nuclei to a few 1e-5 hartree; a restart step is the
    one-step start from psi^n written out again here;
  * self-consistent (Hartree and xc on), nuclei fixed: after a sudden shift of
    the nucleus the density oscillates while the norm and the orthonormality stay
    within 1e-6 and the Kohn-Sham energy stays within a bounded excursion that
    does not depend on the time step (halving h changes the energy trace by far
    less than the excursion): the excursion comes from the non-symmetric smearing
    of the potential source, not from the time integration.
"""
import math

import numpy as np
import pytest

from test_oracle_spectral import fixed_potential_oracle, ho_potential, relaxation_matrix


def test_cd_step_equals_dense_matrix_step(oracle_mod):
    O = oracle_mod
    dims, h, n = (12, 12, 12), 0.35, 2
    V = ho_potential(dims, h, 2.0) + 0.3 * np.sin(np.arange(12 ** 3) * 0.37)
    M, dt = relaxation_matrix(dims, h, V, O)
    H = (np.eye(M.shape[0]) - M) / dt
    o = fixed_potential_oracle(O, dims, h, n, V, seed=7)
    for _ in range(30):
        o.step()
    cd = O.ConcurrentDynamics(o, 0.01)
    psi0 = o.state()[0].astype(complex)
    E = np.array([h ** 3 * (psi0[j].conj() @ H @ psi0[j]).real for j in range(n)])
    assert np.allclose(cd.eref, E, rtol=0, atol=1e-12)
    h1 = psi0 @ H.T - E[:, None] * psi0
    h2 = h1 @ H.T - E[:, None] * h1
    assert np.allclose(cd.prev, psi0, rtol=0, atol=1e-15)
    assert np.max(np.abs(cd.cur - (psi0 - 0.01j * h1 - 0.5e-4 * h2))) < 1e-12
    prev, cur = cd.prev.copy(), cd.cur.copy()
    cd.step()
    ref = prev - 2j * 0.01 * (cur @ H.T - E[:, None] * cur)
    assert np.max(np.abs(cd.cur - ref)) < 1e-12 * np.max(np.abs(ref))
    assert np.array_equal(cd.prev, cur)


def test_cd_conserves_staggered_norm_at_zero_potential(oracle_mod):
    O = oracle_mod
    dims, h, n = (10, 11, 12), 0.4, 3
    o = fixed_potential_oracle(O, dims, h, n, np.zeros(int(np.prod(dims))), seed=8)
    for _ in range(40):
        o.step()
    step = 0.9 * o.prm.dt / (8.0 / 9.0)          # h * max eigenvalue of K_h = 0.9
    cd = O.ConcurrentDynamics(o, step)
    s0 = cd.staggered_overlap().real
    for _ in range(400):
        cd.step()
    s1 = cd.staggered_overlap().real
    assert np.max(np.abs(s1 - s0)) < 1e-13
    assert np.all(np.abs(s0 - 1.0) < 1e-2)


def test_cd_eigenstate_rotates_with_the_schemes_phase(oracle_mod):
    O = oracle_mod
    dims, h = (12, 12, 12), 0.35
    V = ho_potential(dims, h, 2.0)
    M, dt = relaxation_matrix(dims, h, V, O)
    w, vr = np.linalg.eig(M)
    k = np.argmax(w.real)
    eps = (1.0 - w[k].real) / dt
    phi = vr[:, k].real
    phi /= math.sqrt(h ** 3 * phi @ phi)
    o = fixed_potential_oracle(O, dims, h, 1, V, seed=9)
    o.set_orbitals(phi[None])
    step = 0.02
    still = O.ConcurrentDynamics(o, step)                     # reference E = eps: at rest
    psi_still = still.prev.copy()
    for _ in range(300):
        still.step()
    assert np.max(np.abs(still.cur - psi_still)) < 1e-9
    cd = O.ConcurrentDynamics(o, step, eref=[0.0])
    theta = math.asin(step * eps)
    cd.cur = np.exp(-1j * theta) * cd.prev            # the exact second time level
    psi0 = cd.prev.copy()
    for _ in range(600):
        cd.step()
    expect = np.exp(-1j * 601 * theta) * psi0
    assert np.max(np.abs(cd.cur - expect)) < 1e-9
    assert abs(eps - 3.0) < 0.2                        # the well's ground level, 3 w0 / 2 = 3


def he_shift(O, step, sweeps=4):
    from paper_1507_07666_amd import inputs as I
    s = I.he_atom().scaled(16, h=0.35)
    prm = O.Params(s.dims, s.h, 1, 2, softening=0.3, poisson_sweeps=sweeps)
    o = O.Oracle(prm)
    o.set_nuclei([2.0], [[0.15, 0.0, 0.0]])
    o.set_orbitals(s.psi0())
    assert o.relax(4000, 1e-12, 50)[0] == 0
    o.set_nuclei([2.0], [[0.0, 0.0, 0.0]])             # sudden shift: the density sloshes
    return O.ConcurrentDynamics(o, step)


def test_cd_self_consistent_energy_and_norm_with_fixed_nuclei(oracle_mod):
    O = oracle_mod
    T, every = 6.0, 0.6
    traces = {}
    for step in (0.015, 0.0075):
        cd = he_shift(O, step)
        n, k = int(round(T / step)), int(round(every / step))
        E, rho0 = [], cd.density(cd.cur).copy()
        for i in range(n + 1):
            if i % k == 0:
                E.append(cd.energies(converge_poisson=True).e_total)
            if i < n:
                cd.step()
        traces[step] = np.array(E)
        S = cd.overlap()
        assert abs(S[0, 0].real - 1.0) < 1e-6 and abs(S[0, 0].imag) < 1e-12
        assert np.max(np.abs(cd.density(cd.cur) - rho0)) > 1e-3     # the density did move
    a, b = traces[0.015], traces[0.0075]
    exc = np.max(np.abs(a - a[0]))
    assert exc < 5e-4
    assert np.max(np.abs(a - b)) < 0.1 * exc                         # not a time-step error
    half = len(a) // 2
    assert np.max(np.abs(a[half:] - a[0])) < 2.0 * np.max(np.abs(a[:half + 1] - a[0])) + 1e-6   # no drift


def test_cd_energy_reference_keeps_the_dynamics_stable(oracle_mod):
    """H2 (24^3 at 0.45 bohr, softening 0.45, Hartree and xc on), the paper's step
    0.0014 fs, nuclei fixed: with the energy reference the ground state stays put
    (energy and norm within 1e-8 over 3000 steps); without it (E = 0) the
    two-step scheme's parasitic mode, fed back through the density-dependent
    potential, has grown to a visible energy error by then."""
    O = oracle_mod
    from paper_1507_07666_amd import inputs as I
    s = I.System("H2", (24, 24, 24), 0.45, [1.0, 1.0], [(-1.232, 0.0, 0.0), (1.232, 0.0, 0.0)], 2, 1, 0.45,
                 seed=7)
    o = O.oracle_for(s, poisson_sweeps=4)
    assert o.relax(40000, 1e-12, 50)[0] == 0
    f0, vh0 = o.f.copy(), o.vh.copy()
    step = 0.0014 * 41.341373335
    drift = {}
    for eref in (None, [0.0]):
        o.f[:] = f0
        o.vh[:] = vh0
        cd = O.ConcurrentDynamics(o, step, eref=eref)
        e0 = cd.energies(converge_poisson=False).e_total
        for _ in range(3000):
            cd.step()
        drift[eref is None] = (abs(cd.energies(converge_poisson=False).e_total - e0), abs(cd.overlap()[0, 0].real - 1))
    assert drift[True][0] < 1e-8 and drift[True][1] < 1e-8, drift
    assert drift[False][0] > 1e-6, drift


def test_cd_restart_is_the_one_step_start_from_the_current_level(oracle_mod):
    O = oracle_mod
    dims, h, n = (12, 12, 12), 0.35, 2
    V = ho_potential(dims, h, 2.0) + 0.3 * np.sin(np.arange(12 ** 3) * 0.37)
    M, dt = relaxation_matrix(dims, h, V, O)
    H = (np.eye(M.shape[0]) - M) / dt
    o = fixed_potential_oracle(O, dims, h, n, V, seed=7)
    for _ in range(30):
        o.step()
    step = 0.01
    cd = O.ConcurrentDynamics(o, step, restart_every=3)
    for _ in range(2):
        cd.step()
    cur = cd.cur.copy()
    E = np.array([h ** 3 * (cur[j].conj() @ H @ cur[j]).real for j in range(n)])
    cd.step()                                         # the third step restarts
    h1 = cur @ H.T - E[:, None] * cur
    h2 = h1 @ H.T - E[:, None] * h1
    assert np.allclose(cd.eref, E, rtol=0, atol=1e-12)
    assert np.array_equal(cd.prev, cur)
    assert np.max(np.abs(cd.cur - (cur - 1j * step * h1 - 0.5 * step * step * h2))) < 1e-12


def test_cd_restarts_keep_moving_nuclei_dynamics_stable(oracle_mod):
    """H2 (24^3 at 0.45 bohr, softening 0.45), its bond stretched by 0.1 bohr from
    the relaxed 2.364 bohr, nuclei moved by velocity Verlet with the Hellmann-
    Feynman forces at the paper's 0.0014 fs: after 8000 steps the total energy of
    the plain scheme has departed by more than 3e-4 hartree (the parasitic mode);
    with a restart every 500 steps it stays within 3e-5 of its start while the
    bond swings by more than 0.1 bohr."""
    O = oracle_mod
    from paper_1507_07666_amd import dynamics as Dy
    from paper_1507_07666_amd import inputs as I
    d = 2.3643 + 0.1
    R0 = np.array([[-d / 2, 0.0, 0.0], [d / 2, 0.0, 0.0]])
    s = I.System("H2", (24, 24, 24), 0.45, [1.0, 1.0], [tuple(r) for r in R0], 2, 1, 0.45, seed=7)
    o = O.oracle_for(s, poisson_sweeps=4)
    assert o.relax(40000, 1e-12, 50)[0] == 0
    f0, vh0 = o.f.copy(), o.vh.copy()
    M = np.full((2, 1), Dy.PROTON_MASS)
    dt = 0.0014 * Dy.FS
    dev, swing = {}, {}
    for every in (0, 500):
        o.f[:] = f0
        o.vh[:] = vh0
        o.set_nuclei([1.0, 1.0], R0)
        F = o.forces()
        cd = O.ConcurrentDynamics(o, dt, restart_every=every)
        R, V = R0.copy(), np.zeros((2, 3))
        e0 = cd.energies(converge_poisson=True).e_total
        worst, bonds = 0.0, []
        for k in range(8000):
            R = R + V * dt + F / (2.0 * M) * dt * dt
            o.set_nuclei([1.0, 1.0], R)
            Fn = cd.forces()
            V = V + (F + Fn) / (2.0 * M) * dt
            F = Fn
            if (k + 1) % 1000 == 0:
                et = cd.energies(converge_poisson=True).e_total + 0.5 * np.sum(M * V * V)
                worst = max(worst, abs(et - e0))
                bonds.append(np.linalg.norm(R[1] - R[0]))
            cd.step()
        dev[every], swing[every] = worst, max(bonds) - min(bonds)
    assert dev[0] > 3e-4, dev
    assert dev[500] < 3e-5, dev
    assert swing[500] > 0.1, swing
