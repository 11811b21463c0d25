"""Seeded synthetic inputs: nuclei, grids and initial orbitals.

This module is the only code shared by the GPU library's callers and the CPU
oracle.  It draws random numbers and lays out geometry; it holds none of the
lattice-Boltzmann Kohn-Sham arithmetic (no lattice constants, potentials,
orthonormalisation, density or energies).

Random numbers come from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014, as
published in Vigna's reference splitmix64.c) used as a counter-based generator:
draw k (k = 0, 1, ...) under seed s is mix(s + (k + 1) * 0x9E3779B97F4A7C15),
which is exactly the (k+1)-th output of the sequential generator seeded with s.
A uniform double in [0, 1) is (draw >> 11) * 2**-53.

Workloads (sizes and spacings are the ones the solver is exercised on):
  * He atom, 32^3 nodes at 0.3 bohr, softening 0.1 bohr, Gaussian + noise start;
  * Ne atom, 96^3 at 0.2 bohr, softening 0.05 bohr, random Gaussian-enveloped start;
  * CH4, 128^3 at 0.2 bohr, C-H lengths uniform in [1.9, 2.2] bohr;
  * a batch of 64 H2O molecules (O-H in [1.7, 1.9] bohr, H-O-H in [95, 115] deg,
    grids drawn from {64, 80, 96, 112}^3 at 0.2 bohr);
  * a Poisson-arrival request stream mixing atoms Z = 1..10 and CH4/NH3/H2O
    geometry-scan points on grids 48^3..128^3.
Positions are in bohr relative to the grid centre.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, k) -> np.ndarray:
    """Draw(s) number k of SplitMix64 seeded with ``seed`` (uint64, vectorised over k)."""
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (k + np.uint64(1)) * GOLDEN_GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, k) -> np.ndarray:
    """Uniform doubles in [0, 1) from the 53 high bits of draw k."""
    return (splitmix64(seed, k) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# --------------------------------------------------------------------------- grid

def node_coords(n: int, h: float) -> np.ndarray:
    """Node coordinates x_i = (i - (n-1)/2) h; the origin is the box centre."""
    return (np.arange(n, dtype=np.float64) - 0.5 * (n - 1)) * h


def radius2(dims: Tuple[int, int, int], h: float) -> np.ndarray:
    """|r|^2 on the grid, array shaped [nz][ny][nx] (x fastest)."""
    nx, ny, nz = dims
    x = node_coords(nx, h)
    y = node_coords(ny, h)
    z = node_coords(nz, h)
    return z[:, None, None] ** 2 + y[None, :, None] ** 2 + x[None, None, :] ** 2


# ------------------------------------------------------------------ initial orbitals

def init_gauss_noise(dims, h, n_orb, sigma, noise, seed) -> np.ndarray:
    """psi0_j = exp(-|r|^2 / 2 sigma^2) + noise * (2u - 1); array [n_orb][nz][ny][nx].

    u is draw k with k running over (orbital, z, y, x), x fastest.
    """
    nx, ny, nz = dims
    env = np.exp(-radius2(dims, h) / (2.0 * sigma * sigma))
    k = np.arange(n_orb * nx * ny * nz, dtype=np.uint64)
    u = uniform(seed, k).reshape(n_orb, nz, ny, nx)
    return env[None] + noise * (2.0 * u - 1.0)


def init_random_gauss(dims, h, n_orb, sigma, seed) -> np.ndarray:
    """psi0_j = exp(-|r|^2 / 2 sigma^2) * (2u_j - 1); array [n_orb][nz][ny][nx]."""
    nx, ny, nz = dims
    env = np.exp(-radius2(dims, h) / (2.0 * sigma * sigma))
    k = np.arange(n_orb * nx * ny * nz, dtype=np.uint64)
    u = uniform(seed, k).reshape(n_orb, nz, ny, nx)
    return env[None] * (2.0 * u - 1.0)


# ------------------------------------------------------------------------ systems

@dataclass
class System:
    """One solve: grid, nuclei and electron count (positions in bohr)."""
    name: str
    dims: Tuple[int, int, int]
    h: float
    Z: List[float]
    R: List[Tuple[float, float, float]]
    n_elec: int
    n_orb: int
    softening: float
    seed: int
    init: str = "random_gauss"       # or "gauss_noise"
    init_sigma: float = 1.0
    init_noise: float = 0.0
    tag: dict = field(default_factory=dict)

    @property
    def n_sites(self) -> int:
        return self.dims[0] * self.dims[1] * self.dims[2]

    def psi0(self) -> np.ndarray:
        if self.init == "gauss_noise":
            return init_gauss_noise(self.dims, self.h, self.n_orb, self.init_sigma,
                                    self.init_noise, self.seed)
        return init_random_gauss(self.dims, self.h, self.n_orb, self.init_sigma, self.seed)

    def scaled(self, n: int, h: Optional[float] = None) -> "System":
        """Same chemistry on an n^3 grid (for small parity cases)."""
        s = System(**{**self.__dict__})
        s.dims = (n, n, n)
        if h is not None:
            s.h = h
        s.tag = dict(self.tag)
        return s


def n_orb_closed_shell(n_elec: int) -> int:
    return (n_elec + 1) // 2


def he_atom() -> System:
    """He at the centre of 32^3 nodes, h = 0.3, softening 0.1, Gaussian + 1e-3 noise."""
    return System("He", (32, 32, 32), 0.3, [2.0], [(0.0, 0.0, 0.0)], 2, 1, 0.1, seed=1,
                  init="gauss_noise", init_sigma=1.0, init_noise=1e-3)


def ne_atom() -> System:
    """Ne at the centre of 96^3 nodes, h = 0.2, softening 0.05, 5 orbitals."""
    return System("Ne", (96, 96, 96), 0.2, [10.0], [(0.0, 0.0, 0.0)], 10, 5, 0.05, seed=2)


def atom(Z: int, n: int, h: float = 0.2, softening: float = 0.05, seed: int = 0) -> System:
    return System(f"Z{Z}", (n, n, n), h, [float(Z)], [(0.0, 0.0, 0.0)], Z,
                  n_orb_closed_shell(Z), softening, seed=seed)


_TETRA = [(1, 1, 1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1)]


def ch4_from_lengths(L: Sequence[float], n: int = 128, h: float = 0.2,
                     softening: float = 0.05, seed: int = 3) -> System:
    s3 = 1.0 / math.sqrt(3.0)
    R = [(0.0, 0.0, 0.0)] + [(L[k] * d[0] * s3, L[k] * d[1] * s3, L[k] * d[2] * s3)
                             for k, d in enumerate(_TETRA)]
    return System("CH4", (n, n, n), h, [6.0, 1.0, 1.0, 1.0, 1.0], R, 10, 5, softening,
                  seed=seed, tag={"L": list(L)})


def ch4(seed: int = 3, n: int = 128) -> System:
    """CH4: C at the origin, H along the even-parity tetrahedral directions,
    C-H lengths uniform in [1.9, 2.2] bohr (draws 0..3 of ``seed``)."""
    u = uniform(seed, np.arange(4, dtype=np.uint64))
    return ch4_from_lengths([1.9 + 0.3 * float(x) for x in u], n=n, seed=seed)


def h2o_from_geometry(L1: float, L2: float, theta_deg: float, n: int, h: float = 0.2,
                      softening: float = 0.05, seed: int = 4) -> System:
    t = math.radians(theta_deg) / 2.0
    R = [(0.0, 0.0, 0.0), (-L1 * math.sin(t), L1 * math.cos(t), 0.0),
         (L2 * math.sin(t), L2 * math.cos(t), 0.0)]
    return System("H2O", (n, n, n), h, [8.0, 1.0, 1.0], R, 10, 5, softening, seed=seed,
                  tag={"L1": L1, "L2": L2, "theta": theta_deg})


H2O_GRIDS = (64, 80, 96, 112)


def h2o_batch(count: int = 64, seed: int = 4) -> List[System]:
    """Instance i uses draws 4i..4i+3 of ``seed``: L1, L2 ~ U[1.7, 1.9] bohr,
    theta ~ U[95, 115] deg, grid edge ~ U{64, 80, 96, 112}; its orbitals use seed
    1000 * seed + i."""
    out = []
    for i in range(count):
        u = uniform(seed, np.arange(4 * i, 4 * i + 4, dtype=np.uint64))
        L1 = 1.7 + 0.2 * float(u[0])
        L2 = 1.7 + 0.2 * float(u[1])
        th = 95.0 + 20.0 * float(u[2])
        n = H2O_GRIDS[min(3, int(4.0 * float(u[3])))]
        s = h2o_from_geometry(L1, L2, th, n, seed=1000 * seed + i)
        s.tag["index"] = i
        out.append(s)
    return out


def nh3_from_geometry(L: float, alpha_deg: float, n: int, h: float = 0.2,
                      softening: float = 0.05, seed: int = 5) -> System:
    """NH3 with C3v symmetry about z: N at the origin, three H at bond length L with
    H-N-H angle alpha.  The polar angle b of each N-H bond from -z obeys
    cos(alpha) = 1 - 1.5 sin^2(b)."""
    a = math.radians(alpha_deg)
    sb = math.sqrt(max(0.0, (2.0 / 3.0) * (1.0 - math.cos(a))))
    cb = math.sqrt(max(0.0, 1.0 - sb * sb))
    R = [(0.0, 0.0, 0.0)]
    for k in range(3):
        phi = 2.0 * math.pi * k / 3.0
        R.append((L * sb * math.cos(phi), L * sb * math.sin(phi), -L * cb))
    return System("NH3", (n, n, n), h, [7.0, 1.0, 1.0, 1.0], R, 10, 5, softening,
                  seed=seed, tag={"L": L, "alpha": alpha_deg})


# ------------------------------------------------------------------- serving stream

SERVE_GRIDS = (48, 64, 80, 96, 112, 128)


@dataclass
class Request:
    """One solve request in the serving stream; a scan is a list of systems that
    must be solved in order (each point warm-starts from the previous one)."""
    rid: int
    arrival: float
    points: List[System]


def serving_stream(n_requests: int, rate: float, seed: int = 50,
                   grids: Sequence[int] = SERVE_GRIDS, scan_points: int = 8) -> List[Request]:
    """Poisson arrivals at ``rate`` per second.  Request r uses draws 8r..8r+7 of
    ``seed``: [0] inter-arrival time, [1] atom-or-scan, [2] Z or molecule,
    [3] grid, [4..5] unused by atoms; scans sweep the bond length over
    1.9 (1 +- 0.1) bohr and, for NH3/H2O, the angle over 107 +- 10 deg."""
    reqs = []
    t = 0.0
    for r in range(n_requests):
        u = uniform(seed, np.arange(8 * r, 8 * r + 8, dtype=np.uint64))
        t += -math.log(1.0 - float(u[0])) / rate
        n = grids[min(len(grids) - 1, int(len(grids) * float(u[3])))]
        oseed = 100000 + r
        if float(u[1]) < 0.5:
            Z = 1 + min(9, int(10.0 * float(u[2])))
            pts = [atom(Z, n, seed=oseed)]
        else:
            mol = ("CH4", "NH3", "H2O")[min(2, int(3.0 * float(u[2])))]
            pts = []
            for k in range(scan_points):
                f = -1.0 + 2.0 * k / max(1, scan_points - 1)
                L = 1.9 * (1.0 + 0.1 * f)
                ang = 107.0 + 10.0 * f
                if mol == "CH4":
                    s = ch4_from_lengths([L] * 4, n=n, seed=oseed)
                elif mol == "NH3":
                    s = nh3_from_geometry(L, ang, n, seed=oseed)
                else:
                    s = h2o_from_geometry(L, L, ang, n, seed=oseed)
                pts.append(s)
        reqs.append(Request(r, t, pts))
    return reqs
