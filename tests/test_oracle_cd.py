"""Pins of the oracle's concurrent dynamics (section on concurrent dynamics, eq.
KSLBCD, in the reading of Oracle.ConcurrentDynamics: complex orbitals advanced by
the two-step time-centred scheme psi^{n+1} = psi^{n-1} - 2 i h H psi^n with the
relaxation's operator H = K_h + S_chi(V .)):

  * one step equals the same step written with the dense matrix H = (I - M)/dt,
    M = S_xi - dt S_chi diag(V), built independently (fixed potential, 12^3);
  * with V = 0, H is symmetric and the scheme conserves Re h^3 <psi^{n-1}|psi^n>
    exactly (to rounding) for every orbital;
  * an eigenstate of H started with its exact second level psi^1 = e^{-i theta}
    psi^0 rotates rigidly: psi^n = e^{-i n theta} psi^0 with sin(theta) = h eps
    (the time-centred scheme's phase), eps from the dense eigenproblem;
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
    h1 = psi0 @ H.T
    h2 = h1 @ H.T
    assert np.allclose(cd.prev, psi0, rtol=0, atol=1e-15)
    assert np.max(np.abs(cd.cur - (psi0 - 0.01j * h1 - 0.5e-4 * h2))) < 1e-12
    prev, cur = cd.prev.copy(), cd.cur.copy()
    cd.step()
    ref = prev - 2j * 0.01 * (cur @ H.T)
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
    cd = O.ConcurrentDynamics(o, step)
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
