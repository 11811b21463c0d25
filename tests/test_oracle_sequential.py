"""Pins of the oracle's sequential Gram-Schmidt order (the closing remark on eq.
KSLB-2: psi_0 is evolved to its ground state, then psi_1, and so on), in the
reading of relax_sequential: in stage k only orbital k takes lattice steps,
every orbital is orthonormalised in order each step and the density is that of
all orbitals in their current state.

  * one stage step leaves the other orbitals' moments unchanged bit for bit and
    gives orbital k the omega = 1 update of its orthonormalised field, M psi_hat_k
    with M = S_xi - dt S_chi diag(V) built as a dense matrix and psi_hat from a
    QR factorisation in the h^3 metric (not the oracle's Cholesky);
  * on a fixed low-symmetry well the sequential run ends where the paper says the
    procedure ends: the first k orbitals span M's k dominant eigenvectors (dense
    eigen-decomposition) and the Ritz values are (1 - lambda_k)/dt;
  * self-consistent (the same well with Hartree and xc on, four electrons in two
    orbitals, a ragged grid): the sequential order reaches the fixed point of the
    concurrent relaxation (energies, eigenvalues, density), after several sweeps
    because the second orbital's density moves the first one's potential.
"""
import numpy as np

from paper_1507_07666_amd.inputs import node_coords
from test_oracle_spectral import relaxation_matrix, subspace_distance


def anisotropic_well(dims, h):
    nx, ny, nz = dims
    x, y, z = node_coords(nx, h), node_coords(ny, h), node_coords(nz, h)
    V = (0.5 * (4.0 * x[None, None, :] ** 2 + 2.25 * y[None, :, None] ** 2 + z[:, None, None] ** 2)).ravel()
    return V + 0.2 * np.sin(np.arange(V.size) * 0.37)


def well_oracle(O, dims, h, n, seed=3):
    o = O.Oracle(O.Params(dims, h, n, 2 * n, xc=O.XC_NONE, hartree=False))
    V = anisotropic_well(dims, h)
    o.set_potential(V)
    o.set_orbitals(np.random.default_rng(seed).standard_normal((n, int(np.prod(dims)))))
    return o, V


def test_stage_step_moves_only_its_orbital(oracle_mod):
    O = oracle_mod
    dims, h, n = (12, 12, 12), 0.35, 3
    o, V = well_oracle(O, dims, h, n)
    M, dt = relaxation_matrix(dims, h, V, O)
    for _ in range(5):
        o.step()
    for k in range(n):
        before = o.moment()
        Q, R = np.linalg.qr(before.T * h ** 1.5)          # Gram-Schmidt in order, h^3 metric
        psihat = (Q * np.sign(np.diag(R))).T / h ** 1.5
        o.step(active={k})
        after = o.moment()
        for j in range(n):
            if j != k:
                assert np.array_equal(after[j], before[j]), (k, j)
        want = M @ psihat[k]
        assert np.max(np.abs(after[k] - want)) <= 1e-12 * np.max(np.abs(want)), k


def test_sequential_fixed_point_is_the_dominant_eigenspace(oracle_mod):
    O = oracle_mod
    dims, h, n = (12, 12, 12), 0.35, 3
    o, V = well_oracle(O, dims, h, n)
    M, dt = relaxation_matrix(dims, h, V, O)
    w, vr = np.linalg.eig(M)
    order = np.argsort(-w.real)
    lam = w.real[order[:n + 1]]
    assert np.all(np.abs(w.imag[order[:n]]) < 1e-12) and lam[n - 1] - lam[n] > 1e-3
    rc, steps, sweeps = O.relax_sequential(o, 60000, 1e-12, 1e-12, 50, 4)
    assert rc == 0 and sweeps >= 1
    psihat, _ = o.state()
    for k in range(1, n + 1):
        assert subspace_distance(psihat[:k].T, vr[:, order[:k]].real) < 1e-5, k
    _, ritz = o.hamiltonian(converge_poisson=False)
    assert np.allclose(ritz, np.sort((1.0 - lam[:n]) / dt), rtol=0, atol=1e-8), (ritz, (1.0 - lam[:n]) / dt)


def test_sequential_and_concurrent_orders_share_the_fixed_point(oracle_mod):
    O = oracle_mod
    dims, h = (12, 13, 14), 0.35
    V = anisotropic_well(dims, h)

    def scf():
        o = O.Oracle(O.Params(dims, h, 2, 4))         # Hartree and the default local functional on
        o.set_potential(V)
        o.set_orbitals(np.random.default_rng(3).standard_normal((2, int(np.prod(dims)))))
        return o

    seq = scf()
    rc, steps, sweeps = O.relax_sequential(seq, 40000, 1e-10, 1e-10, 50, 12)
    assert rc == 0 and sweeps >= 3
    con = scf()
    assert con.relax(40000, 1e-12, 50)[0] == 0
    es, ec = seq.energies(converge_poisson=True), con.energies(converge_poisson=True)
    assert es.e_hartree > 1.0 and es.e_x < -1.0                    # the self-consistent terms are large
    assert abs(es.e_total - ec.e_total) < 1e-10, (es.e_total, ec.e_total)
    assert np.allclose(es.eps, ec.eps, rtol=0, atol=1e-9), (es.eps, ec.eps)
    _, rs = seq.state()
    _, rcn = con.state()
    assert np.linalg.norm(rs - rcn) <= 1e-6 * np.linalg.norm(rcn)
