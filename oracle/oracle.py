"""Python driver of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It composes the plain C functions of lbks_oracle.c into
one relaxation step in the order the method defines it, and evaluates the
energies.  It never touches the GPU library.

One step (lattice Boltzmann equation per orbital with the orthogonalisation
source, section "The kinetic approach to Kohn-Sham theory"):
  1. psi_j = sum_p f_jp                                   (kinetic representation)
  2. S_jk = <psi_j|psi_k>                                  (orthogonality constraints)
  3. orthonormalise: GS  psi_hat = psi C, g = f C, C = L^{-T}, S = L L^T,
                     W   psi_hat = psi / n, psi* = psi_hat - sum_{l<j} Lambda_jl psi_hat_l
  4. rho = sum_j occ_j psi_hat_j^2                         (density)
  5. Hartree: multipole ghost values, K_P red/black SOR sweeps
  6. V = V_ext + V_H + v_xc(rho)                           (KS potential)
  7. collide: f^post = (1-omega) g + omega xi psi* - dt chi V psi_hat
  8. stream with zero inflow from outside the box.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# LBKS_ORACLE_LIB points the loader at another build of lbks_oracle.c (the
# sanitizer test's instrumented one)
LIB_PATH = os.environ.get("LBKS_ORACLE_LIB") or os.path.join(_HERE, "liblbks_oracle.so")
SRC_PATH = os.path.join(_HERE, "lbks_oracle.c")

XC_NONE, XC_X, XC_X_LYPLOCAL, XC_X_PZ81, XC_B88_LYP, XC_B88_LYP_POLARISED = 0, 1, 2, 3, 4, 5
Q = 19

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP, no host-specific ISA)."""
    import subprocess
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-o", tmp, SRC_PATH, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i64 = ctypes.c_longlong
        I = ctypes.c_int
        D = ctypes.c_double
        sig = {
            "orc_lattice": (I, [D, P, P, P, P, P]),
            "orc_dot": (D, [i64, P, P]),
            "orc_sum": (D, [i64, P]),
            "orc_moment": (None, [I, i64, P, P]),
            "orc_overlap": (None, [I, i64, D, P, P]),
            "orc_cholesky_inverse": (I, [I, P, P]),
            "orc_combine": (None, [I, i64, P, P, P]),
            "orc_w_fields": (None, [I, i64, P, P, P, P, P, P]),
            "orc_density": (None, [I, i64, P, P, P]),
            "orc_multipoles": (None, [I, I, I, D, P, P]),
            "orc_multipole_value": (D, [P, D, D, D]),
            "orc_boundary": (None, [I, I, I, D, P, P]),
            "orc_sor_omega": (D, [I, I, I]),
            "orc_sor_sweep": (None, [I, I, I, D, D, P, P]),
            "orc_poisson_residual": (D, [I, I, I, D, P, P]),
            "orc_vh_interior": (None, [I, I, I, P, P]),
            "orc_vext": (None, [I, I, I, D, I, P, P, D, P]),
            "orc_enn": (D, [I, P, P]),
            "orc_forces": (None, [I, I, I, D, I, P, P, D, P, P]),
            "orc_xc": (None, [I, i64, P, D, P, P, P, P]),
            "orc_gga_point": (None, [D, D, D, P, P, P, P, P, P]),
            "orc_gga": (None, [I, I, I, D, P, D, I, P, P, P, P]),
            "orc_gga_point_polarised": (None, [D, D, D, P, P, P, P, P, P]),
            "orc_collide": (None, [I, i64, D, D, P, P, P, P, P, P, P]),
            "orc_stream": (None, [I, I, I, I, P, P, P]),
            "orc_equilibrium": (None, [I, i64, P, P, P]),
            "orc_apply_sw": (None, [I, I, I, P, P, P, P]),
            "orc_set_threads": (None, [I]),
            "orc_max_threads": (I, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    """Threads of the oracle's element-wise loops (its results do not depend on it)."""
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def _p(a: np.ndarray):
    """Address of a C-contiguous array.  The caller must hold a reference to `a`
    for the duration of the C call (never pass a temporary)."""
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


# ------------------------------------------------------------------ lattice

def lattice(D: float = 1.0 / 3.0):
    """(v[19,3] int (x,y,z), w, xi, chi) of the D3Q19 reading."""
    v = np.zeros((Q, 3), dtype=np.int32)
    w = np.zeros(Q)
    xi = np.zeros(Q)
    chi = np.zeros(Q)
    n = lib().orc_lattice(D, _p(v), _p(w), _p(xi), _p(chi), None)
    assert n == Q
    return v, w, xi, chi


def lattice4(D: float = 1.0 / 3.0):
    """(v, w, xi, chi) with fourth-order Hermite weights on the D3Q19 velocities
    (the paper's He run takes fourth order for the equilibrium and the source):
    one value per speed class (rest, faces, edges) from the moment conditions
      xi:  sum_p xi_p = 1,  sum_p xi_p v_x^2 = D,  sum_p xi_p v_x^2 v_y^2 = D^2
           (zeroth, second and mixed fourth moments of a Gaussian of variance D),
      chi: sum_p chi_p = 1, sum_p chi_p v_x^2 = 0, sum_p chi_p v_x^2 v_y^2 = 0,
    solved as a 3 x 3 linear system (on D3Q19, v_x^4 = v_x^2, so these are all the
    independent even moments up to fourth order)."""
    v, w, _, _ = lattice(D)
    cls = (v.astype(np.int64) ** 2).sum(1)
    A = np.zeros((3, 3))
    for c in range(3):
        sel = cls == c
        A[0, c] = sel.sum()
        A[1, c] = float((v[sel, 0] ** 2).sum())
        A[2, c] = float((v[sel, 0] ** 2 * v[sel, 1] ** 2).sum())
    xc = np.linalg.solve(A, np.array([1.0, D, D * D]))
    cc = np.linalg.solve(A, np.array([1.0, 0.0, 0.0]))
    return v, w, np.ascontiguousarray(xc[cls]), np.ascontiguousarray(cc[cls])


def occupations(n_elec: int, n_orb: int, polarised: bool = False) -> np.ndarray:
    """Closed-shell reading: 2 electrons per orbital, the last takes the rest.  A
    fully spin-polarised density has one electron in each orbital."""
    if polarised:
        assert n_elec == n_orb, "one spin: one electron per orbital"
        return np.ones(n_orb)
    occ = np.full(n_orb, 2.0)
    occ[-1] = n_elec - 2.0 * (n_orb - 1)
    return occ


def time_step(omega: float, D: float, h: float) -> float:
    """Physical imaginary-time step of one lattice step: the lattice diffusivity
    (1/omega - 1/2) D must equal hbar/2m = 1/2 in atomic units, so
    Delta t = 2 (1/omega - 1/2) D h^2."""
    return 2.0 * (1.0 / omega - 0.5) * D * h * h


def xc_fields(kind: int, rho: np.ndarray, floor: float = 1e-14, dims=None, h=None):
    """Per-node exchange and correlation energies per particle and potentials.
    The gradient-corrected kinds (XC_B88_LYP, XC_B88_LYP_POLARISED) need the grid (dims, h)."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    n = rho.size
    ex, ec, vx, vc = (np.zeros_like(rho) for _ in range(4))
    if kind in (XC_B88_LYP, XC_B88_LYP_POLARISED):
        nx, ny, nz = dims
        lib().orc_gga(nx, ny, nz, h, _p(rho), floor, 1 if kind == XC_B88_LYP_POLARISED else 0,
                      _p(ex), _p(ec), _p(vx), _p(vc))
    else:
        lib().orc_xc(kind, n, _p(rho), floor, _p(ex), _p(ec), _p(vx), _p(vc))
    return ex, ec, vx, vc


def gga_point(rho: float, sigma: float, floor: float = 1e-14, polarised: bool = False):
    """(f_x, f_c, df_x/drho, df_c/drho, df_x/dsigma, df_c/dsigma) of B88 + LYP,
    spin-unpolarised or fully spin-polarised."""
    out = [ctypes.c_double() for _ in range(6)]
    fn = lib().orc_gga_point_polarised if polarised else lib().orc_gga_point
    fn(rho, sigma, floor, *[ctypes.byref(o) for o in out])
    return tuple(o.value for o in out)


def apply_sw(dims, v, wts, u):
    nx, ny, nz = dims
    u = np.ascontiguousarray(u, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.int32)
    wts = np.ascontiguousarray(wts, dtype=np.float64)
    out = np.empty_like(u)
    lib().orc_apply_sw(nx, ny, nz, _p(v), _p(wts), _p(u), _p(out))
    return out


# --------------------------------------------------------------------- solver

@dataclass
class Params:
    dims: tuple
    h: float
    n_orb: int
    n_elec: int
    omega: float = 1.0
    D: float = 1.0 / 3.0
    ortho: str = "gs"             # "gs" or "w"
    xc: int = XC_X_LYPLOCAL
    hartree: bool = True
    poisson_sweeps: int = 2
    softening: float = 0.05
    rho_floor: float = 1e-14
    occ: Optional[np.ndarray] = None
    deps_tol: float = 0.0           # stopping rule: > 0 also bounds the change of sum_j eps_j
    stop_checks: int = 0            # consecutive passing checks needed (0, 1: one)
    hermite: int = 2                # order of the Hermite weights: 2, or 4 (lattice4)

    @property
    def dt(self) -> float:
        return time_step(self.omega, self.D, self.h)

    @property
    def n_sites(self) -> int:
        return self.dims[0] * self.dims[1] * self.dims[2]


@dataclass
class Energies:
    e_total: float
    e_kin: float
    e_ext: float
    e_hartree: float
    e_x: float
    e_c: float
    e_nn: float
    n_electrons: float
    poisson_residual: float
    eps: np.ndarray
    steps: int
    extra: dict = field(default_factory=dict)


class Oracle:
    """State (f, V_H) of one solve, advanced one plain step at a time."""

    def __init__(self, prm: Params):
        self.prm = prm
        self.L = lib()
        nx, ny, nz = prm.dims
        self.N = prm.n_sites
        self.v, self.w, self.xi, self.chi = lattice4(prm.D) if prm.hermite == 4 else lattice(prm.D)
        self.occ = (np.asarray(prm.occ, dtype=np.float64) if prm.occ is not None
                    else occupations(prm.n_elec, prm.n_orb, prm.xc == XC_B88_LYP_POLARISED))
        self.f = np.zeros((prm.n_orb, Q, self.N))
        self.fpost = np.zeros_like(self.f)
        self.vh = np.zeros((nz + 2, ny + 2, nx + 2))
        self.vext = None
        self.e_nn = 0.0
        self.steps = 0
        self.e_prev = None          # stopping rule: (energy, sum of eps) of the previous check, kept across relax calls
        self.passes = 0             # consecutive passing checks
        self.omega_sor = self.L.orc_sor_omega(nx, ny, nz)
        self.fields = None          # orbital fields psi_j of the omega = 1 field step (step_fields), else None

    # -- inputs
    def set_nuclei(self, Z, R):
        nx, ny, nz = self.prm.dims
        Z = np.ascontiguousarray(Z, dtype=np.float64)
        R = np.ascontiguousarray(R, dtype=np.float64).reshape(-1, 3)
        self.vext = np.zeros(self.N)
        self.L.orc_vext(nx, ny, nz, self.prm.h, len(Z), _p(Z), _p(R), self.prm.softening,
                        _p(self.vext))
        self.e_nn = self.L.orc_enn(len(Z), _p(Z), _p(R))
        self.nuclei = (Z.copy(), R.copy())
        self.e_prev = None

    def set_potential(self, vext):
        self.vext = np.ascontiguousarray(vext, dtype=np.float64).reshape(self.N).copy()
        self.e_nn = 0.0
        self.nuclei = None
        self.e_prev = None

    def set_orbitals(self, psi0):
        psi0 = np.ascontiguousarray(psi0, dtype=np.float64).reshape(self.prm.n_orb, self.N)
        self.e_prev = None
        self.fields = None
        self.L.orc_equilibrium(self.prm.n_orb, self.N, _p(self.xi), _p(psi0), _p(self.f))

    # -- pieces of one step
    def moment(self):
        if self.fields is not None:
            return self.fields.copy()
        psi = np.empty((self.prm.n_orb, self.N))
        self.L.orc_moment(self.prm.n_orb, self.N, _p(self.f), _p(psi))
        return psi

    def overlap(self, psi):
        S = np.empty((self.prm.n_orb, self.prm.n_orb))
        self.L.orc_overlap(self.prm.n_orb, self.N, self.prm.h, _p(psi), _p(S))
        return S

    def orthonormalise(self, psi, with_g=True):
        """Returns (psi_hat, psi_star, g, S)."""
        n = self.prm.n_orb
        S = self.overlap(psi)
        if self.prm.ortho == "gs":
            C = np.empty((n, n))
            rc = self.L.orc_cholesky_inverse(n, _p(S), _p(C))
            if rc != 0:
                raise FloatingPointError("overlap matrix is not positive definite")
            psihat = np.empty_like(psi)
            self.L.orc_combine(n, self.N, _p(C), _p(psi), _p(psihat))
            g = None
            if with_g:
                g = np.empty_like(self.f)
                self.L.orc_combine(n, Q * self.N, _p(C), _p(self.f), _p(g))
            return psihat, psihat, g, S
        psihat = np.empty_like(psi)
        psistar = np.empty_like(psi)
        g = np.empty_like(self.f)
        self.L.orc_w_fields(n, self.N, _p(S), _p(psi), _p(self.f), _p(psihat), _p(psistar), _p(g))
        return psihat, psistar, g, S

    def density(self, psihat):
        rho = np.empty(self.N)
        self.L.orc_density(self.prm.n_orb, self.N, _p(self.occ), _p(psihat), _p(rho))
        return rho

    def hartree_boundary(self, rho):
        nx, ny, nz = self.prm.dims
        m = np.empty(10)
        self.L.orc_multipoles(nx, ny, nz, self.prm.h, _p(rho), _p(m))
        self.L.orc_boundary(nx, ny, nz, self.prm.h, _p(m), _p(self.vh))
        return m

    def sor(self, rho, sweeps):
        nx, ny, nz = self.prm.dims
        for _ in range(sweeps):
            self.L.orc_sor_sweep(nx, ny, nz, self.prm.h, self.omega_sor, _p(rho), _p(self.vh))

    def poisson_residual(self, rho):
        nx, ny, nz = self.prm.dims
        return self.L.orc_poisson_residual(nx, ny, nz, self.prm.h, _p(rho), _p(self.vh))

    def vh_interior(self):
        nx, ny, nz = self.prm.dims
        out = np.empty(self.N)
        self.L.orc_vh_interior(nx, ny, nz, _p(self.vh), _p(out))
        return out

    def potential(self, rho):
        """V = V_ext + V_H + v_x + v_c, plus the xc fields used for energies."""
        V = self.vext.copy()
        if self.prm.hartree:
            V += self.vh_interior()
        ex, ec, vx, vc = xc_fields(self.prm.xc, rho, self.prm.rho_floor, self.prm.dims, self.prm.h)
        if self.prm.xc != XC_NONE:
            V += vx
            V += vc
        return V, (ex, ec, vx, vc)

    def step(self, active=None):
        """One lattice step.  `active` (a set of orbital indices, None: all): the
        orbitals outside it keep their populations (the sequential order of the
        Gram-Schmidt procedure, relax_sequential); every orbital still enters the
        orthonormalisation and the density."""
        if self.vext is None:
            raise RuntimeError("no potential set")
        p = self.prm
        keep = None
        if active is not None:
            keep = {j: self.f[j].copy() for j in range(p.n_orb) if j not in active}
        if self.fields is not None:
            # leave the field form: the populations at equilibrium with the fields
            # (at omega = 1 the step below does not read them beyond their moment)
            self.L.orc_equilibrium(p.n_orb, self.N, _p(self.xi), _p(self.fields), _p(self.f))
            self.fields = None
        psi = self.moment()
        psihat, psistar, g, _ = self.orthonormalise(psi)
        rho = self.density(psihat)
        if p.hartree:
            self.hartree_boundary(rho)
            self.sor(rho, p.poisson_sweeps)
        V, _ = self.potential(rho)
        self.L.orc_collide(p.n_orb, self.N, p.omega, p.dt, _p(self.xi), _p(self.chi), _p(g),
                           _p(psistar), _p(psihat), _p(V), _p(self.fpost))
        nx, ny, nz = p.dims
        self.L.orc_stream(p.n_orb, nx, ny, nz, _p(self.v), _p(self.fpost), _p(self.f))
        if keep:
            for j, fj in keep.items():
                self.f[j] = fj
        self.steps += 1

    def step_fields(self):
        """One step at omega = 1 on the orbital fields alone.  With omega = 1 the
        relaxed part (1 - omega) g of the collision vanishes, so the new moment of
        the lattice Boltzmann equation depends only on the orthonormalised fields:
        summing the streamed post-collision populations over p gives
            psi_j <- S_xi psi*_j - dt S_chi(V psi_hat_j),  (S_w u)(r) = sum_p w_p u(r - v_p),
        zero outside the box (psi* = psi_hat: Gram-Schmidt mode).  Same steps 1-6 as step();
        the populations are not formed.  Used to reach the fixed point with less work."""
        if self.vext is None:
            raise RuntimeError("no potential set")
        p = self.prm
        if p.omega != 1.0:
            raise ValueError("the field step holds at omega = 1 only")
        if p.ortho != "gs":
            raise ValueError("the field step is written for Gram-Schmidt orthonormalisation")
        psi = self.moment()
        psihat, psistar, _, _ = self.orthonormalise(psi, with_g=False)
        rho = self.density(psihat)
        if p.hartree:
            self.hartree_boundary(rho)
            self.sor(rho, p.poisson_sweeps)
        V, _ = self.potential(rho)
        new = np.empty_like(psi)
        for j in range(p.n_orb):
            a = apply_sw(p.dims, self.v, self.xi, psistar[j])
            b = apply_sw(p.dims, self.v, self.chi, V * psihat[j])
            new[j] = a - p.dt * b
        self.fields = new
        self.steps += 1

    # -- results
    def state(self):
        """(psi_hat, rho) of the current populations."""
        psihat, _, _, _ = self.orthonormalise(self.moment(), with_g=False)
        return psihat, self.density(psihat)

    def converge_poisson(self, rho, tol=1e-12, block=10, max_sweeps=200000):
        """Blocks of `block` SOR sweeps until the relative residual is <= tol, or until
        it has reached the roundoff floor: <= 1e-9 and no more than 10 % below its
        value five blocks earlier."""
        self.hartree_boundary(rho)
        sweeps = 0
        res = self.poisson_residual(rho)
        hist = [res]
        while res > tol and sweeps < max_sweeps:
            k = len(hist) - 1
            if k >= 5 and res <= 1e-9 and res >= 0.9 * hist[k - 5]:
                break
            self.sor(rho, block)
            sweeps += block
            res = self.poisson_residual(rho)
            hist.append(res)
        return res, sweeps

    def energies(self, converge_poisson=True, tol=1e-12) -> Energies:
        p = self.prm
        h3 = p.h ** 3
        psihat, _, _, _ = self.orthonormalise(self.moment(), with_g=False)
        rho = self.density(psihat)
        res = 0.0
        if p.hartree:
            if converge_poisson:
                self.e_prev = None          # the Hartree relaxation changes the state
                res, _ = self.converge_poisson(rho, tol)
            else:
                res = self.poisson_residual(rho)
        V, (ex, ec, vx, vc) = self.potential(rho)
        dims = p.dims
        eps = np.empty(p.n_orb)
        e_kin = 0.0
        D = self.L.orc_dot
        for j in range(p.n_orb):
            u = np.ascontiguousarray(psihat[j])
            su = apply_sw(dims, self.v, self.xi, u)
            ku = np.ascontiguousarray(-(su - u) / (p.D * p.h * p.h))   # K_h u
            vu = apply_sw(dims, self.v, self.chi, V * u)                # S_chi (V u)
            kin = h3 * D(self.N, _p(u), _p(ku))
            pot = h3 * D(self.N, _p(u), _p(vu))
            eps[j] = kin + pot
            e_kin += self.occ[j] * kin
        e_ext = h3 * D(self.N, _p(self.vext), _p(rho))
        vhi = self.vh_interior()
        e_h = 0.5 * h3 * D(self.N, _p(vhi), _p(rho)) if p.hartree else 0.0
        e_x = h3 * D(self.N, _p(rho), _p(ex)) if p.xc != XC_NONE else 0.0
        e_c = h3 * D(self.N, _p(rho), _p(ec)) if p.xc != XC_NONE else 0.0
        ne = h3 * self.L.orc_sum(self.N, _p(rho))
        et = e_kin + e_ext + e_h + e_x + e_c + self.e_nn
        return Energies(et, e_kin, e_ext, e_h, e_x, e_c, self.e_nn, ne, res, eps, self.steps)

    def hamiltonian(self, converge_poisson=True, tol=1e-12):
        """The relaxation operator projected on the current orthonormalised orbitals,
        H_jk = <psi_hat_j | K_h psi_hat_k + S_chi(V psi_hat_k)>, with V built from
        their density exactly as in energies().  Its diagonal is eps_j (the
        Rayleigh quotients of the eigenvalue reading); its eigenvalues are the Ritz
        values of the operator (I - M)/dt on the orbitals' span, which do not
        depend on how the orbitals are rotated inside that span.  Returns
        (H, ritz) with ritz the eigenvalues' real parts in ascending order."""
        p = self.prm
        h3 = p.h ** 3
        psihat, _, _, _ = self.orthonormalise(self.moment(), with_g=False)
        rho = self.density(psihat)
        if p.hartree:
            if converge_poisson:
                self.e_prev = None
                self.converge_poisson(rho, tol)
        V, _ = self.potential(rho)
        n = p.n_orb
        W = np.empty((n, self.N))
        for k in range(n):
            u = np.ascontiguousarray(psihat[k])
            su = apply_sw(p.dims, self.v, self.xi, u)
            W[k] = -(su - u) / (p.D * p.h * p.h) + apply_sw(p.dims, self.v, self.chi, V * u)
        H = np.empty((n, n))
        for j in range(n):
            for k in range(n):
                H[j, k] = h3 * self.L.orc_dot(self.N, _p(np.ascontiguousarray(psihat[j])), _p(W[k]))
        ritz = np.sort(np.linalg.eigvals(H).real)
        return H, ritz

    def forces(self) -> np.ndarray:
        """Hellmann-Feynman forces on the nuclei, [n][3] hartree/bohr, from the
        density of the orthonormalised current orbitals (Born-Oppenheimer scenario
        of the section on concurrent dynamics; orc_forces)."""
        p = self.prm
        psihat, _, _, _ = self.orthonormalise(self.moment(), with_g=False)
        rho = np.ascontiguousarray(self.density(psihat))
        if getattr(self, "nuclei", None) is None:
            raise ValueError("forces need nuclei (set_nuclei)")
        Z, R = self.nuclei
        F = np.zeros((len(Z), 3))
        nx, ny, nz = p.dims
        self.L.orc_forces(nx, ny, nz, p.h, len(Z), _p(Z), _p(R), p.softening, _p(rho), _p(F))
        return F

    def relax(self, max_steps, dE_tol=0.0, check_every=100, progress=None, fields=False):
        """Run steps in chunks of check_every.  After each chunk (only if dE_tol > 0)
        the energies with the current Hartree potential are compared with the
        previous chunk's: the check passes if the total energy moved by less than
        dE_tol and, when prm.deps_tol > 0, the sum of the orbital energies by less
        than deps_tol; the run has converged after prm.stop_checks consecutive
        passing checks (at least one).  The previous check and the count are kept
        across calls until the state is changed by new nuclei, potential or
        orbitals, or a Poisson-converged energy evaluation.  Returns
        (0 converged | 1 step limit, steps done).  `progress(steps, energy)` is
        called after each check.  fields=True takes the omega = 1 field step
        (step_fields), which reaches the same fixed point."""
        done = 0
        advance = self.step_fields if fields else self.step
        check_every = max(1, int(check_every))
        need = max(1, int(self.prm.stop_checks))
        while done < max_steps:
            n = min(check_every, max_steps - done)
            for _ in range(n):
                advance()
            done += n
            if dE_tol > 0:
                en = self.energies(converge_poisson=False)
                e, tr = en.e_total, float(np.sum(en.eps))
                if progress is not None:
                    progress(done, e)
                ok = self.e_prev is not None and abs(e - self.e_prev[0]) < dE_tol
                if ok and self.prm.deps_tol > 0:
                    ok = abs(tr - self.e_prev[1]) < self.prm.deps_tol
                self.passes = self.passes + 1 if ok else 0
                self.e_prev = (e, tr)
                if self.passes >= need:
                    return 0, done
        return 1, done


def relax_sequential(o: "Oracle", max_steps: int, dE_tol: float, deps_tol: float, check_every: int = 50,
                     max_sweeps: int = 20, progress=None):
    """The sequential order of the time-dependent Gram-Schmidt procedure (the
    closing remark on eq. KSLB-2: evolve psi_0 to its ground state, then psi_1, and
    so on), in this reading: in stage k only orbital k takes lattice steps (the
    others keep their populations), every orbital is orthonormalised in order each
    step (so orbital k is projected against the converged lower ones) and the
    density is that of all orbitals in their current state; stage k ends when eps_k
    changed by less than deps_tol over check_every steps.  A sweep runs the stages
    k = 0 .. n-1; sweeps repeat until the total energy changed by less than dE_tol
    from the previous sweep (the density of the later orbitals drives V in the
    earlier stages, so one sweep is not self-consistent).  Returns
    (0 converged | 1 step limit, steps, sweeps)."""
    n = o.prm.n_orb
    steps, e_prev = 0, None
    for sweep in range(1, max_sweeps + 1):
        for k in range(n):
            eps_prev = None
            while steps < max_steps:
                for _ in range(check_every):
                    o.step(active={k})
                steps += check_every
                eps = o.energies(converge_poisson=False).eps[k]
                if progress is not None:
                    progress(sweep, k, steps, eps)
                if eps_prev is not None and abs(eps - eps_prev) < deps_tol:
                    break
                eps_prev = eps
        e = o.energies(converge_poisson=False).e_total
        if steps >= max_steps:
            return 1, steps, sweep
        if e_prev is not None and abs(e - e_prev) < dE_tol:
            return 0, steps, sweep
        e_prev = e
    return 1, steps, max_sweeps


def params_for(system, **kw) -> Params:
    """Oracle parameters for an inputs.System."""
    return Params(dims=tuple(system.dims), h=system.h, n_orb=system.n_orb, n_elec=system.n_elec,
                  softening=system.softening, **kw)


def oracle_for(system, **kw) -> Oracle:
    o = Oracle(params_for(system, **kw))
    o.set_nuclei(system.Z, system.R)
    o.set_orbitals(system.psi0())
    return o


class ConcurrentDynamics:
    """Electrons and nuclei moved together (the concurrent scenario of the section
    on concurrent dynamics, eq. KSLBCD), in this reading:

      * the orbitals are complex and the populations are at equilibrium with them,
        f_jp = xi_p psi_j (the omega = 1 reading of the relaxation, where the
        populations carry nothing beyond their moment), so the two-step
        time-centred lattice equation advances the moments:
            psi_j^{n+1} = psi_j^{n-1} - 2 i h (H - E_j) psi_j^n,
            H u = K_h u + S_chi(V u),  K_h u = -(S_xi u - u) / (D dx^2),
        H being the operator whose steady state the relaxation reaches (its
        Rayleigh quotients are the eps_j), with the potential and orthogonality
        sources turned by i as printed;
      * U_jp = kappa w_p q_p E_j phi_j, the source that holds the orbital's
        energy at E_j, is read as each orbital's energy reference: orbital j is advanced with
        H - E_j, E_j its Rayleigh quotient at the start.  That is a global phase
        e^{i E_j t} per orbital (densities, energies and forces are unchanged) which
        makes the ground state stationary; without it the density picks up the
        two-step scheme's parasitic (-1)^n mode and, fed back through V, it grows
        exponentially (measured on H2 at 0.45 bohr and 0.0014 fs: tenfold every
        500 steps from step 1500 on);
      * the energy reference alone does not hold once the nuclei move: the
        orbitals' energies drift away from E_j and the parasitic mode grows again
        (measured on the same H2 vibrating: the total energy departs by 2e-3
        hartree after 6000 steps).  With restart_every = R > 0, every R-th step
        (steps R, 2R, ... counted from the start) is a restart: E_j is re-centred
        on h^3 Re<psi_j^n|H psi_j^n> with that step's V, and the step is the
        one-step start below taken from psi^n, which leaves no parasitic mode;
      * W = 0: the evolution is unitary up to the scheme's own error, which keeps
        the orbitals orthonormal (the drift is measured, not corrected);
      * start: psi^0 = the orthonormalised current orbitals (a relaxed ground
        state), V_H converged for their density, E_j = <psi_j^0|H psi_j^0>, and
        psi^1 = psi^0 - i h H' psi^0 - (h^2/2) H' H' psi^0, H' = H - E_j;
      * each step first rebuilds V from rho^n = sum_j occ_j |psi_j^n|^2 (multipole
        boundary and K_P warm-started red/black sweeps, as in the relaxation),
        then takes the step above;
      * the nuclei (moved by the caller) enter through V_ext; forces are the
        Hellmann-Feynman forces of the instantaneous density.
    h is the time step in atomic units of real time.  Test infrastructure only."""

    def __init__(self, o: "Oracle", h: float, eref=None, restart_every: int = 0):
        """eref: the energy references E_j (default: the orbitals' Rayleigh
        quotients at the start); restart_every: period of the restarts (0: none)."""
        self.o = o
        self.h = float(h)
        self.restart_every = int(restart_every)
        p = o.prm
        if p.omega != 1.0 or p.ortho != "gs":
            raise ValueError("concurrent dynamics starts from the omega = 1 Gram-Schmidt relaxation")
        psihat, _ = o.state()
        self.prev = psihat.astype(np.complex128)
        rho = self.density(self.prev)
        if p.hartree:
            o.converge_poisson(rho)
        V, _ = o.potential(rho)
        if eref is None:
            eref = self.rayleigh(self.prev, V)
        self.eref = np.asarray(eref, dtype=np.float64).reshape(p.n_orb)
        h1 = self.apply_h(self.prev, V)
        h2 = self.apply_h(h1, V)
        self.cur = self.prev - 1j * self.h * h1 - 0.5 * self.h * self.h * h2
        self.steps = 0

    # -- pieces
    def density(self, psi):
        re = np.ascontiguousarray(psi.real)
        im = np.ascontiguousarray(psi.imag)
        return self.o.density(re) + self.o.density(im)

    def apply_h(self, psi, V, shift=True):
        """(H - E_j) psi_j for complex psi [n][N] (H psi with shift=False), on the
        real and imaginary parts."""
        p = self.o.prm
        out = np.empty_like(psi)
        for j in range(psi.shape[0]):
            parts = []
            for u in (np.ascontiguousarray(psi[j].real), np.ascontiguousarray(psi[j].imag)):
                su = apply_sw(p.dims, self.o.v, self.o.xi, u)
                hu = -(su - u) / (p.D * p.h * p.h) + apply_sw(p.dims, self.o.v, self.o.chi, V * u)
                if shift:
                    hu = hu - self.eref[j] * u
                parts.append(hu)
            out[j] = parts[0] + 1j * parts[1]
        return out

    def potential_now(self):
        """V of the current density after the step's Hartree sweeps."""
        p = self.o.prm
        rho = self.density(self.cur)
        if p.hartree:
            self.o.hartree_boundary(rho)
            self.o.sor(rho, p.poisson_sweeps)
        V, _ = self.o.potential(rho)
        return V

    def rayleigh(self, psi, V):
        """h^3 Re<psi_j|H psi_j> per orbital."""
        hp = self.apply_h(psi, V, shift=False)
        return np.array([self.o.prm.h ** 3 * np.vdot(psi[j], hp[j]).real for j in range(psi.shape[0])])

    def step(self):
        V = self.potential_now()
        if self.restart_every > 0 and (self.steps + 1) % self.restart_every == 0:
            self.eref = self.rayleigh(self.cur, V)
            h1 = self.apply_h(self.cur, V)
            h2 = self.apply_h(h1, V)
            new = self.cur - 1j * self.h * h1 - 0.5 * self.h * self.h * h2
        else:
            new = self.prev - 2j * self.h * self.apply_h(self.cur, V)
        self.prev, self.cur = self.cur, new
        self.steps += 1

    # -- results
    def staggered_overlap(self):
        """h^3 <psi_j^{n-1}|psi_j^n> per orbital (complex): its real part is exactly
        conserved by the time-centred step when H is symmetric."""
        h3 = self.o.prm.h ** 3
        return np.array([h3 * np.vdot(self.prev[j], self.cur[j]) for j in range(self.cur.shape[0])])

    def overlap(self):
        """h^3 <psi_j^n|psi_k^n> (complex Hermitian matrix)."""
        h3 = self.o.prm.h ** 3
        return h3 * (self.cur.conj() @ self.cur.T)

    def energies(self, converge_poisson=True, tol=1e-12) -> Energies:
        """Kohn-Sham energies of psi^n (as Oracle.energies, with Re<psi|.|psi>)."""
        o, p = self.o, self.o.prm
        h3 = p.h ** 3
        rho = self.density(self.cur)
        res = 0.0
        if p.hartree:
            if converge_poisson:
                res, _ = o.converge_poisson(rho, tol)
            else:
                res = o.poisson_residual(rho)
        V, (ex, ec, vx, vc) = o.potential(rho)
        eps = np.empty(p.n_orb)
        e_kin = 0.0
        for j in range(p.n_orb):
            kin = pot = 0.0
            for u in (np.ascontiguousarray(self.cur[j].real), np.ascontiguousarray(self.cur[j].imag)):
                su = apply_sw(p.dims, o.v, o.xi, u)
                ku = np.ascontiguousarray(-(su - u) / (p.D * p.h * p.h))
                vu = apply_sw(p.dims, o.v, o.chi, V * u)
                kin += h3 * o.L.orc_dot(o.N, _p(u), _p(ku))
                pot += h3 * o.L.orc_dot(o.N, _p(u), _p(vu))
            eps[j] = kin + pot
            e_kin += o.occ[j] * kin
        rho = np.ascontiguousarray(rho)
        e_ext = h3 * o.L.orc_dot(o.N, _p(o.vext), _p(rho))
        vhi = o.vh_interior()
        e_h = 0.5 * h3 * o.L.orc_dot(o.N, _p(vhi), _p(rho)) if p.hartree else 0.0
        e_x = h3 * o.L.orc_dot(o.N, _p(rho), _p(ex)) if p.xc != XC_NONE else 0.0
        e_c = h3 * o.L.orc_dot(o.N, _p(rho), _p(ec)) if p.xc != XC_NONE else 0.0
        ne = h3 * o.L.orc_sum(o.N, _p(rho))
        et = e_kin + e_ext + e_h + e_x + e_c + o.e_nn
        return Energies(et, e_kin, e_ext, e_h, e_x, e_c, o.e_nn, ne, res, eps, self.steps)

    def forces(self) -> np.ndarray:
        """Hellmann-Feynman forces of the current density on the nuclei, [n][3]."""
        o, p = self.o, self.o.prm
        rho = np.ascontiguousarray(self.density(self.cur))
        Z, R = o.nuclei
        F = np.zeros((len(Z), 3))
        nx, ny, nz = p.dims
        o.L.orc_forces(nx, ny, nz, p.h, len(Z), _p(Z), _p(R), p.softening, _p(rho), _p(F))
        return F
