"""Spectral pins of the oracle's relaxation (imaginary-time eigen-expansion
argument and the time-dependent Gram-Schmidt procedure of the paper).

At omega = 1 one step maps psi_hat to M psi_hat with
M = S_xi - dt S_chi diag(V), (S_w u)(r) = sum_p w_p u(r - v_p), zero outside the
box, so the relaxation is subspace iteration on M: its steady state spans the
dominant invariant subspace and eps_j = (1 - lambda_j) / dt.  These tests build
M (or, for omega != 1, the population operator) independently of the oracle,
with dense/ARPACK eigensolvers, and compare.
"""
import itertools

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def site_index(dims):
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.ravel(), y.ravel(), z.ravel()


def sparse_stencil(dims, v, wts, diag=None):
    """Sparse matrix of u -> sum_p wts_p (diag * u)(r - v_p) with zero outside the box."""
    nx, ny, nz = dims
    x, y, z = site_index(dims)
    N = nx * ny * nz
    rows, cols, vals = [], [], []
    for p in range(len(wts)):
        sx, sy, sz = x - v[p, 0], y - v[p, 1], z - v[p, 2]
        ok = (sx >= 0) & (sx < nx) & (sy >= 0) & (sy < ny) & (sz >= 0) & (sz < nz)
        src = (sz * ny + sy) * nx + sx
        r = np.nonzero(ok)[0]
        c = src[ok]
        val = np.full(len(r), wts[p])
        if diag is not None:
            val = val * diag[c]
        rows.append(r)
        cols.append(c)
        vals.append(val)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N))


def relaxation_matrix(dims, h, V, O, D=1.0 / 3.0):
    v, _, xi, chi = O.lattice(D)
    dt = O.time_step(1.0, D, h)
    return (sparse_stencil(dims, v, xi) - dt * sparse_stencil(dims, v, chi, V)).toarray(), dt


def subspace_distance(A, B):
    """Largest sine of the principal angles between the column spaces of A and B,
    computed as ||(I - Qa Qa^T) Qb||_2 (accurate for tiny angles)."""
    Qa, _ = np.linalg.qr(A)
    Qb, _ = np.linalg.qr(B)
    R = Qb - Qa @ (Qa.T @ Qb)
    return float(np.linalg.norm(R, 2))


def fixed_potential_oracle(O, dims, h, n_orb, V, seed=0, omega=1.0, ortho="gs"):
    prm = O.Params(dims, h, n_orb, 2 * n_orb, omega=omega, ortho=ortho, xc=O.XC_NONE,
                   hartree=False)
    o = O.Oracle(prm)
    o.set_potential(V)
    rng = np.random.default_rng(seed)
    o.set_orbitals(rng.standard_normal((n_orb, prm.n_sites)))
    return o


def ho_potential(dims, h, w0):
    from paper_1507_07666_amd.inputs import radius2
    return 0.5 * w0 * w0 * radius2(dims, h).ravel()


def test_box_modes_closed_form(oracle_mod):
    """V = 0: the discrete spectrum is lambda(k) = sum_p xi_p prod_a cos(k_a v_pa) on the
    sine modes k_a = pi m_a / (N_a + 1), which vanish on the ghost layer."""
    O = oracle_mod
    dims, h, n_orb = (6, 7, 8), 0.5, 4
    v, _, xi, _ = O.lattice()
    modes = []
    for m in itertools.product(range(1, dims[0] + 1), range(1, dims[1] + 1), range(1, dims[2] + 1)):
        k = np.pi * np.array(m) / (np.array(dims) + 1)
        lam = float(np.sum(xi * np.prod(np.cos(k[None, :] * v), axis=1)))
        modes.append((lam, m))
    modes.sort(key=lambda t: -t[0])
    lam = np.array([t[0] for t in modes])
    assert lam[n_orb - 1] - lam[n_orb] > 1e-3           # top-4 block is separated
    # GS orders the block: orbital j converges at rate lambda_{j+1} / lambda_j
    worst = max(lam[j + 1] / lam[j] for j in range(n_orb))
    steps = int(np.ceil(np.log(1e-13) / np.log(worst)))
    o = fixed_potential_oracle(O, dims, h, n_orb, np.zeros(np.prod(dims)))
    for _ in range(steps):
        o.step()
    e = o.energies(converge_poisson=False)
    expect = (1.0 - lam[:n_orb]) / (O.Params(dims, h, 1, 2).D * h * h)
    assert np.allclose(e.eps, expect, rtol=0, atol=1e-12 * expect.max())
    x, y, z = site_index(dims)
    U = np.stack([np.sin(np.pi * m[0] * (x + 1) / (dims[0] + 1))
                  * np.sin(np.pi * m[1] * (y + 1) / (dims[1] + 1))
                  * np.sin(np.pi * m[2] * (z + 1) / (dims[2] + 1)) for _, m in modes[:n_orb]], 1)
    psihat, rho = o.state()
    assert subspace_distance(psihat.T, U) < 1e-8
    # psi_hat orthonormal in <a|b> = h^3 sum a b
    G = h ** 3 * psihat @ psihat.T
    assert np.allclose(G, np.eye(n_orb), atol=1e-13)


def test_dense_eigen_ho_gram_schmidt(oracle_mod):
    """12^3 harmonic well (Hartree and xc off): the GS relaxation reaches the dominant
    4-dimensional invariant subspace of M and eps_j equals the real Schur diagonal."""
    O = oracle_mod
    dims, h, n_orb = (12, 12, 12), 0.3, 4
    V = ho_potential(dims, h, 2.0)
    M, dt = relaxation_matrix(dims, h, V, O)
    T, Z, sdim = sla.schur(M, output="real", sort=lambda re, im: re > 0.0)
    evals = np.linalg.eigvals(M)
    order = np.argsort(-evals.real)
    ev = evals[order]
    assert np.max(np.abs(ev[:n_orb + 2].imag)) < 1e-12       # leading eigenvalues are real
    # Schur vectors of the leading block from the sorted real eigenvectors
    w, vr = np.linalg.eig(M)
    idx = np.argsort(-w.real)[:n_orb]
    lead = vr[:, idx].real
    ratio = ev[n_orb].real / ev[n_orb - 1].real
    steps = int(np.ceil(np.log(1e-10) / np.log(ratio)))
    o = fixed_potential_oracle(O, dims, h, n_orb, V, seed=1)
    for _ in range(steps):
        o.step()
    psihat, _ = o.state()
    assert subspace_distance(psihat.T, lead) < 1e-9
    # Rayleigh quotients of the orthonormal relaxed basis equal (1 - Schur diagonal)/dt
    Q, _ = np.linalg.qr(lead)
    Tlead = Q.T @ M @ Q
    e = o.energies(converge_poisson=False)
    Uh = psihat.T * h ** 1.5
    ray = np.array([(1.0 - Uh[:, j] @ M @ Uh[:, j]) / dt for j in range(n_orb)])
    assert np.allclose(e.eps, ray, rtol=0, atol=1e-10)
    assert abs(e.eps[0] - (1.0 - ev[0].real) / dt) < 1e-10
    assert np.allclose(np.sort(e.eps)[1:], np.sort((1 - np.linalg.eigvals(Tlead).real) / dt)[1:],
                       atol=1e-9)


def aniso_ho(dims, h, w):
    from paper_1507_07666_amd.inputs import node_coords
    nx, ny, nz = dims
    x, y, z = node_coords(nx, h), node_coords(ny, h), node_coords(nz, h)
    return 0.5 * (w[0] ** 2 * x[None, None, :] ** 2 + w[1] ** 2 * y[None, :, None] ** 2
                  + w[2] ** 2 * z[:, None, None] ** 2).ravel()


def test_w_mode_reaches_gs_subspace_on_symmetric_potential(oracle_mod):
    """The paper-literal orthogonalisation source reaches the same orbitals as exact
    Gram-Schmidt when the potential's mirror symmetries make the lowest orbitals
    mutually orthogonal (ground, z-odd, y-odd states of an anisotropic well)."""
    O = oracle_mod
    dims, h, n_orb = (12, 12, 12), 0.35, 3
    V = aniso_ho(dims, h, (2.0, 1.5, 1.0))
    gs = fixed_potential_oracle(O, dims, h, n_orb, V, seed=2, ortho="gs")
    w = fixed_potential_oracle(O, dims, h, n_orb, V, seed=2, ortho="w")
    for _ in range(2000):
        gs.step()
        w.step()
    pg, _ = gs.state()
    pw, _ = w.state()
    for j in range(n_orb):
        assert subspace_distance(pg[j:j + 1].T, pw[j:j + 1].T) < 1e-9
    eg = gs.energies(converge_poisson=False).eps
    ew = w.energies(converge_poisson=False).eps
    assert np.allclose(eg, ew, atol=1e-10)
    assert np.all(np.diff(eg) > 0.3)


def population_operator(O, dims, h, V, omega, D=1.0 / 3.0):
    """f -> stream((1 - omega) f + omega xi psi - dt chi V psi), psi = sum_p f_p,
    as a LinearOperator over [19][sites] (written here independently of the oracle)."""
    v, _, xi, chi = O.lattice(D)
    dt = O.time_step(omega, D, h)
    nx, ny, nz = dims
    N = nx * ny * nz
    Vg = V.reshape(nz, ny, nx)

    def mv(fv):
        f = fv.reshape(19, nz, ny, nx)
        psi = f.sum(0)
        out = np.zeros_like(f)
        for p in range(19):
            post = (1 - omega) * f[p] + omega * xi[p] * psi - dt * chi[p] * Vg * psi
            vx, vy, vz = v[p]
            dst = out[p]
            dst[max(vz, 0):nz + min(vz, 0), max(vy, 0):ny + min(vy, 0), max(vx, 0):nx + min(vx, 0)] = \
                post[max(-vz, 0):nz + min(-vz, 0), max(-vy, 0):ny + min(-vy, 0), max(-vx, 0):nx + min(-vx, 0)]
        return out.ravel()

    return spla.LinearOperator((19 * N, 19 * N), matvec=mv, dtype=np.float64), dt


@pytest.mark.parametrize("omega", [0.8, 1.3])
def test_population_operator_dominant_mode(oracle_mod, omega):
    """omega != 1: populations carry non-equilibrium parts; the normalised relaxation
    converges to the dominant eigenvector of the population operator and the
    per-step norm factor to its eigenvalue."""
    O = oracle_mod
    dims, h = (8, 9, 10), 0.3
    V = ho_potential(dims, h, 2.0)
    A, dt = population_operator(O, dims, h, V, omega)
    vals, vecs = spla.eigs(A, k=4, which="LR", tol=1e-14, maxiter=20000)
    order = np.argsort(-vals.real)
    lam0 = vals[order[0]]
    assert abs(lam0.imag) < 1e-12
    f0 = vecs[:, order[0]].real.reshape(19, -1)
    psi_ref = f0.sum(0)
    o = fixed_potential_oracle(O, dims, h, 1, V, seed=3, omega=omega)
    for _ in range(2500):
        o.step()
    psi = o.moment()
    S = o.overlap(psi)
    o.step()
    psi2 = o.moment()
    n_next = np.sqrt(o.overlap(psi2)[0, 0] / 1.0)      # |M psi_hat| after one step from a normalised state
    assert abs(n_next - lam0.real) < 1e-11
    psihat, _ = o.state()
    assert subspace_distance(psihat.T, psi_ref[:, None]) < 1e-8


def test_projected_operator_and_ritz_values(oracle_mod):
    """The oracle's projected operator H_jk = <psi_hat_j|K_h psi_hat_k + S_chi(V psi_hat_k)>
    equals U^T (I - M) U / dt for the orthonormal basis U = h^(3/2) psi_hat of any
    state (at omega = 1, dt = D h^2 makes K_h = (I - S_xi)/dt), written here with the
    dense M; rotating the basis inside its span leaves its eigenvalues (the Ritz
    values) unchanged while its diagonal changes; on the relaxed subspace the Ritz
    values are M's dominant eigenvalues mapped to (1 - lambda_k)/dt."""
    O = oracle_mod
    dims, h, n_orb = (12, 12, 12), 0.3, 4
    V = ho_potential(dims, h, 2.0)
    M, dt = relaxation_matrix(dims, h, V, O)
    o = fixed_potential_oracle(O, dims, h, n_orb, V, seed=4)
    for _ in range(5):
        o.step()
    psihat, _ = o.state()
    U = psihat.T * h ** 1.5
    H, ritz = o.hamiltonian(converge_poisson=False)
    Href = U.T @ ((np.eye(M.shape[0]) - M) @ U) / dt
    assert np.allclose(H, Href, rtol=0, atol=1e-10 * np.abs(Href).max())
    assert np.allclose(np.diag(H), o.energies(converge_poisson=False).eps, rtol=0, atol=1e-12)
    # rotation inside the span (GS of an orthonormal set is the identity)
    th = 0.7
    R = np.eye(n_orb)
    R[1, 1] = R[2, 2] = np.cos(th)
    R[1, 2], R[2, 1] = -np.sin(th), np.sin(th)
    o2 = fixed_potential_oracle(O, dims, h, n_orb, V, seed=4)
    o2.set_orbitals(R.T @ psihat)
    H2, ritz2 = o2.hamiltonian(converge_poisson=False)
    assert np.abs(np.diag(H2) - np.diag(H)).max() > 1e-3
    assert np.allclose(ritz2, ritz, rtol=0, atol=1e-11)
    # relaxed subspace: the dominant eigenvalues of M
    ev = np.sort(np.linalg.eigvals(M).real)[::-1]
    steps = int(np.ceil(np.log(1e-8) / np.log(ev[n_orb] / ev[n_orb - 1])))
    for _ in range(steps):
        o.step()
    _, ritz3 = o.hamiltonian(converge_poisson=False)
    assert np.allclose(ritz3, np.sort((1.0 - ev[:n_orb]) / dt), rtol=0, atol=1e-9)


def test_field_step_is_the_moment_of_the_population_step(oracle_mod):
    """At omega = 1 the oracle's field step psi <- S_xi psi_hat - dt S_chi(V psi_hat)
    gives the moment of the population step (Hartree and xc on, several orbitals,
    ragged grid), so both relax to the same fixed point; the sums differ only in
    rounding order."""
    O = oracle_mod
    from paper_1507_07666_amd import inputs as I
    system = I.ne_atom().scaled(15)
    a, b = O.oracle_for(system), O.oracle_for(system)
    for _ in range(3):
        a.step()
        b.step()
    a.step()
    b.step_fields()
    pa, pb = a.moment(), b.moment()
    assert np.max(np.abs(pa - pb)) <= 1e-14 * np.max(np.abs(pa))
    for _ in range(4):                      # and back: a population step after field steps
        b.step_fields()
        a.step()
    b.step()
    a.step()
    assert np.max(np.abs(a.moment() - b.moment())) <= 1e-13 * np.max(np.abs(pa))
    ea, eb = a.energies(), b.energies()
    assert abs(ea.e_total - eb.e_total) <= 1e-12 * abs(ea.e_total)
    with pytest.raises(ValueError):
        O.oracle_for(system, omega=0.8).step_fields()


def w_mode_reference_step(f, xi, chi, v, V, dt, omega, dims, h):
    """The paper-literal orthogonalisation source written out with numpy (independent
    of the oracle): psi_j = sum_p f_jp, S_jl = <psi_j|psi_l> = h^3 sum psi_j psi_l,
    n_j = sqrt(S_jj), psi_hat_j = psi_j / n_j, Lambda_jl =
    S_jl / (n_j n_l), psi*_j = psi_hat_j - sum_{l<j} Lambda_jl psi_hat_l,
    post = (1 - omega) f_jp / n_j + omega xi_p psi*_j - dt chi_p V psi_hat_j,
    then streamed with zero inflow."""
    nx, ny, nz = dims
    n = f.shape[0]
    psi = f.sum(1)
    S = h ** 3 * (psi @ psi.T)
    nrm = np.sqrt(np.diag(S))
    hat = psi / nrm[:, None]
    lam = S / np.outer(nrm, nrm)
    star = hat.copy()
    for j in range(n):
        for l in range(j):
            star[j] -= lam[j, l] * hat[l]
    out = np.zeros_like(f)
    for j in range(n):
        for p in range(19):
            post = ((1 - omega) * f[j, p] / nrm[j] + omega * xi[p] * star[j] - dt * chi[p] * V * hat[j])
            post = post.reshape(nz, ny, nx)
            vx, vy, vz = v[p]
            dst = out[j, p].reshape(nz, ny, nx)
            dst[max(vz, 0):nz + min(vz, 0), max(vy, 0):ny + min(vy, 0), max(vx, 0):nx + min(vx, 0)] = \
                post[max(-vz, 0):nz + min(-vz, 0), max(-vy, 0):ny + min(-vy, 0), max(-vx, 0):nx + min(-vx, 0)]
    return out


@pytest.mark.parametrize("omega", [1.0, 0.8])
def test_w_mode_on_low_symmetry_potential_follows_the_lagged_projection_map(oracle_mod, omega):
    """The oracle's W mode on a potential without mirror symmetries (a displaced,
    anisotropic well plus a random smooth bump) follows the lagged-projection map
    written out independently, step by step (30 steps, 3 orbitals), and keeps
    following it near its fixed point (after 600 more steps)."""
    O = oracle_mod
    from paper_1507_07666_amd.inputs import node_coords
    dims, h, n_orb = (9, 10, 11), 0.35, 3
    nx, ny, nz = dims
    x, y, z = node_coords(nx, h), node_coords(ny, h), node_coords(nz, h)
    X, Y, Zc = x[None, None, :], y[None, :, None], z[:, None, None]
    rng = np.random.default_rng(21)
    c = rng.uniform(-0.3, 0.3, 3)
    V = (0.5 * (4.0 * (X - c[0]) ** 2 + 2.2 * (Y - c[1]) ** 2 + 1.1 * (Zc - c[2]) ** 2)
         + 0.8 * (X - c[0]) * (Y - c[1]) + 0.5 * np.exp(-((X - 0.4) ** 2 + (Y + 0.3) ** 2 + (Zc - 0.2) ** 2))).ravel()
    o = fixed_potential_oracle(O, dims, h, n_orb, V, seed=5, omega=omega, ortho="w")
    v, _, xi, chi = O.lattice()
    f = o.f.copy()
    for k in range(30):
        f = w_mode_reference_step(f, xi, chi, v, V, o.prm.dt, omega, dims, h)
        o.step()
        assert np.max(np.abs(o.f - f)) <= 1e-12 * np.max(np.abs(f)), k
    for _ in range(600):
        o.step()
    f = o.f.copy()
    f2 = w_mode_reference_step(f, xi, chi, v, V, o.prm.dt, omega, dims, h)
    o.step()
    assert np.max(np.abs(o.f - f2)) <= 1e-12 * np.max(np.abs(f2))
