"""Pins of the oracle's Hartree and exchange-correlation pieces.

Hartree term of the KS Hamiltonian, read as the 7-point discrete Poisson
problem with multipole Dirichlet data:
  * the SOR fixed point equals the exact discrete solution by DST-I;
  * ghost values equal the exterior potential of a Gaussian charge (erf closed
    form) and of a displaced charge within the rigorous l >= 3 remainder bound.
Local xc (functional left open by the paper; Slater exchange + LYP at zero
gradient, or PZ81):
  * v = d(rho eps)/d rho by central differences;
  * Slater exchange equals the electron-gas form -3 k_F / (4 pi);
  * LYP limits and PZ81 branch continuity.
"""
import math

import numpy as np
import pytest
import scipy.fft as sfft
from scipy.special import erf

from paper_1507_07666_amd.inputs import node_coords


def gaussian_charge(dims, h, sigma, centre=(0.0, 0.0, 0.0)):
    nx, ny, nz = dims
    x = node_coords(nx, h)[None, None, :] - centre[0]
    y = node_coords(ny, h)[None, :, None] - centre[1]
    z = node_coords(nz, h)[:, None, None] - centre[2]
    r2 = x * x + y * y + z * z
    return (np.exp(-r2 / (2 * sigma * sigma)) / (2 * np.pi * sigma * sigma) ** 1.5).ravel()


def make_oracle(O, dims, h):
    prm = O.Params(dims, h, 1, 2, xc=O.XC_NONE, hartree=True)
    return O.Oracle(prm)


def ghost_positions(dims, h):
    """(index into the padded array, x, y, z) of the six ghost faces."""
    nx, ny, nz = dims
    X, Y, Z = node_coords(nx, h), node_coords(ny, h), node_coords(nz, h)
    gx = lambda i: (i - 0.5 * (nx - 1)) * h
    gy = lambda j: (j - 0.5 * (ny - 1)) * h
    gz = lambda k: (k - 0.5 * (nz - 1)) * h
    out = []
    for k in range(nz):
        for j in range(ny):
            out.append(((k + 1, j + 1, 0), gx(-1), Y[j], Z[k]))
            out.append(((k + 1, j + 1, nx + 1), gx(nx), Y[j], Z[k]))
    for k in range(nz):
        for i in range(nx):
            out.append(((k + 1, 0, i + 1), X[i], gy(-1), Z[k]))
            out.append(((k + 1, ny + 1, i + 1), X[i], gy(ny), Z[k]))
    for j in range(ny):
        for i in range(nx):
            out.append(((0, j + 1, i + 1), X[i], Y[j], gz(-1)))
            out.append(((nz + 1, j + 1, i + 1), X[i], Y[j], gz(nz)))
    return out


def test_ghost_values_spherical_gaussian(oracle_mod):
    dims, h, sigma = (32, 32, 32), 0.2, 0.5
    o = make_oracle(oracle_mod, dims, h)
    rho = gaussian_charge(dims, h, sigma)
    m = o.hartree_boundary(rho)
    assert abs(m[0] - 1.0) < 1e-8           # charge outside the box is ~1e-9
    assert np.allclose(m[1:], 0.0, atol=1e-13)
    for idx, x, y, z in ghost_positions(dims, h):
        r = math.sqrt(x * x + y * y + z * z)
        exact = erf(r / (math.sqrt(2) * sigma)) / r
        assert abs(o.vh[idx] - exact) < 1e-6 * exact


def test_ghost_values_displaced_charge_remainder_bound(oracle_mod):
    """1/|r - d| = sum_l d^l / r^(l+1) P_l(cos g); after l = 2 the remainder is at most
    (d^3 / r^4) / (1 - d/r).  A wrong sign or factor in the dipole or quadrupole term
    breaks this bound by orders of magnitude."""
    dims, h, sigma = (40, 40, 40), 0.2, 0.3
    d = np.array([0.5, -0.3, 0.4])
    o = make_oracle(oracle_mod, dims, h)
    rho = gaussian_charge(dims, h, sigma, d)
    m = o.hartree_boundary(rho)
    assert abs(m[0] - 1.0) < 1e-12
    assert np.allclose(m[1:4], d, atol=1e-12)
    dn = np.linalg.norm(d)
    worst = 0.0
    for idx, x, y, z in ghost_positions(dims, h):
        r = math.sqrt(x * x + y * y + z * z)
        exact = 1.0 / math.sqrt((x - d[0]) ** 2 + (y - d[1]) ** 2 + (z - d[2]) ** 2)
        bound = (dn ** 3 / r ** 4) / (1.0 - dn / r)
        err = abs(o.vh[idx] - exact)
        assert err <= 1.001 * bound + 1e-12
        worst = max(worst, err / bound)
    assert worst > 0.05      # the bound is reached within an order of magnitude (not vacuous)


def dst_poisson(rho, ghost_padded, dims, h):
    """Exact solution of (sum of face neighbours - 6u)/h^2 = -4 pi rho with the ghost
    layer of `ghost_padded` as Dirichlet data, by DST-I diagonalisation."""
    nx, ny, nz = dims
    g = ghost_padded
    b = -4.0 * np.pi * h * h * rho.reshape(nz, ny, nx)
    b = b.copy()
    b[:, :, 0] -= g[1:-1, 1:-1, 0]
    b[:, :, -1] -= g[1:-1, 1:-1, -1]
    b[:, 0, :] -= g[1:-1, 0, 1:-1]
    b[:, -1, :] -= g[1:-1, -1, 1:-1]
    b[0, :, :] -= g[0, 1:-1, 1:-1]
    b[-1, :, :] -= g[-1, 1:-1, 1:-1]
    bh = sfft.dstn(b, type=1)
    lam = lambda n: -4.0 * np.sin(np.pi * np.arange(1, n + 1) / (2.0 * (n + 1))) ** 2
    den = lam(nz)[:, None, None] + lam(ny)[None, :, None] + lam(nx)[None, None, :]
    return sfft.idstn(bh / den, type=1).ravel()


def test_sor_fixed_point_is_exact_discrete_solution(oracle_mod):
    dims, h = (14, 12, 10), 0.25
    o = make_oracle(oracle_mod, dims, h)
    rho = gaussian_charge(dims, h, 0.4, (0.2, -0.1, 0.15)) + 0.3 * gaussian_charge(dims, h, 0.3, (-0.4, 0.3, 0.0))
    res, sweeps = o.converge_poisson(rho, tol=1e-13)
    assert res <= 1e-13 and sweeps > 0
    ref = dst_poisson(rho, o.vh, dims, h)
    got = o.vh_interior()
    assert np.max(np.abs(got - ref)) < 1e-11 * np.max(np.abs(ref))


def test_sor_omega_cube():
    from oracle import oracle as O
    for n in (16, 32, 96):
        w = O.lib().orc_sor_omega(n, n, n)
        assert abs(w - 2.0 / (1.0 + math.sin(math.pi / (n + 1)))) < 1e-14


# ------------------------------------------------------------------------ xc

def xc(O, kind, rho):
    return O.xc_fields(kind, np.asarray(rho, dtype=np.float64))


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_xc_potential_is_derivative_of_energy_density(oracle_mod, kind):
    O = oracle_mod
    rho = np.logspace(-6, 3, 61)
    rho = rho[np.abs(rho - 3.0 / (4.0 * np.pi)) > 1e-2]      # PZ81 branch point
    ex, ec, vx, vc = xc(O, kind, rho)
    step = 1e-5 * rho
    exp_, ecp, _, _ = xc(O, kind, rho + step)
    exm, ecm, _, _ = xc(O, kind, rho - step)
    dx = ((rho + step) * exp_ - (rho - step) * exm) / (2 * step)
    assert np.allclose(vx, dx, rtol=1e-8, atol=1e-14)
    if kind != 1:
        dc = ((rho + step) * ecp - (rho - step) * ecm) / (2 * step)
        assert np.allclose(vc, dc, rtol=1e-7, atol=1e-13)
    else:
        assert np.all(ec == 0) and np.all(vc == 0)


def test_slater_exchange_is_electron_gas_exchange(oracle_mod):
    rho = np.logspace(-8, 4, 50)
    ex, _, _, _ = xc(oracle_mod, 1, rho)
    kf = (3 * np.pi ** 2 * rho) ** (1.0 / 3.0)
    assert np.allclose(ex, -3.0 * kf / (4.0 * np.pi), rtol=1e-14)


def test_lyp_uniform_limits(oracle_mod):
    a, b, d = 0.04918, 0.132, 0.349
    CF = 2.871234000188191        # Thomas-Fermi constant (3/10)(3 pi^2)^(2/3)
    _, ec, _, vc = xc(oracle_mod, 2, np.array([1e18]))
    assert abs(ec[0] + a * (1 + b * CF)) < 1e-6
    assert abs(vc[0] + a * (1 + b * CF)) < 1e-6       # g'(0) finite: v -> eps at u -> 0
    _, ec, _, _ = xc(oracle_mod, 2, np.array([1e-12]))
    u = 1e4
    assert abs(ec[0] * u + a / d) < 1e-3 * a / d


def test_pz81_branch_continuity(oracle_mod):
    rs1 = 3.0 / (4.0 * np.pi)            # rho with r_s = 1
    _, e, _, v = xc(oracle_mod, 3, np.array([rs1 * (1 + 1e-12), rs1 * (1 - 1e-12)]))
    assert abs(e[0] - e[1]) < 5e-5 and abs(e[0] + 0.0596) < 2e-4
    assert abs(v[0] - v[1]) < 5e-4


def test_density_floor(oracle_mod):
    for kind in (1, 2, 3):
        out = xc(oracle_mod, kind, np.array([0.0, 1e-15, 9.9e-15]))
        for arr in out:
            assert np.all(arr == 0.0)
