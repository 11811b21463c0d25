"""Born-Oppenheimer nuclear motion around the electronic relaxation.

In the Born-Oppenheimer scenario of the paper's section on concurrent dynamics
the ions move on the surface of the electronic ground state: at every nuclear
configuration the orbitals relax to the ground state and the ions feel the
forces of that state.  Here each configuration is entered with
lbks_set_nuclei, which keeps the orbitals of the previous one (a warm start),
the relaxation runs until the total energy changes by less than dE_tol per
check_every lattice steps, and the forces are the Hellmann-Feynman forces of
the relaxed density (lbks_forces).  All lattice work runs in the library; this
module only moves the nuclei.

  * relax_geometry: steepest descent to zero force with an adaptive step, for
    building a molecule
    from a rough start (the paper relaxes water from random hydrogen
    positions);
  * bo_md: velocity-Verlet molecular dynamics on the ground-state surface (the
    paper's H2 vibration);
  * cd_md: the concurrent scenario, electrons (complex orbitals in real time)
    and nuclei advanced together with one small time step.

Units are atomic: bohr, hartree, electron masses, and atomic time
(1 fs = 41.341 a.u.).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

from . import lbks

PROTON_MASS = 1836.15267343          # electron masses
AMU = 1822.888486                    # electron masses per dalton
FS = 41.341373335                    # atomic time units per femtosecond


@dataclass
class ElectronRule:
    """How far the orbitals relax at each nuclear configuration."""
    max_steps: int = 40000
    dE_tol: float = 1e-9
    check_every: int = 50
    fixed_steps: int = 0             # > 0: exactly this many lattice steps instead of the rule


@dataclass
class GroundState:
    R: np.ndarray
    energy: float
    forces: np.ndarray
    steps: int
    status: int


def ground_state(solver: lbks.Solver, Z: Sequence[float], R: np.ndarray,
                 rule: Optional[ElectronRule] = None) -> GroundState:
    """Relax the electrons at nuclear positions R (warm start) and return the
    total energy and forces there."""
    rule = rule or ElectronRule()
    R = np.asarray(R, dtype=np.float64).reshape(-1, 3)
    solver.set_nuclei(Z, R)
    if rule.fixed_steps > 0:
        rc, steps = solver.relax(rule.fixed_steps)
    else:
        rc, steps = solver.relax(rule.max_steps, rule.dE_tol, rule.check_every)
    e = solver.energy()
    F = solver.forces()
    return GroundState(R.copy(), float(e["e_total"]), F, int(steps), int(rc))


def _free(F: np.ndarray, fixed: Optional[Sequence[bool]]) -> np.ndarray:
    if fixed is None:
        return F
    F = F.copy()
    F[np.asarray(fixed, dtype=bool)] = 0.0
    return F


@dataclass
class GeometryResult:
    R: np.ndarray
    energy: float
    forces: np.ndarray
    iterations: int
    converged: bool
    history: List[tuple] = field(default_factory=list)   # (energy, max |F|, step factor) per iteration


def relax_geometry(solver: lbks.Solver, Z: Sequence[float], R0, fixed: Optional[Sequence[bool]] = None,
                   ftol: float = 1e-3, max_iter: int = 200, step: float = 0.5, max_disp: float = 0.1,
                   rule: Optional[ElectronRule] = None) -> GeometryResult:
    """Steepest descent to zero force: R <- R + alpha F, each atom's move capped at
    max_disp bohr.  alpha grows by 1.2 while consecutive forces point the same way
    (F_new . F_old > 0) and halves when a move overshoots.  Moves are judged by
    the forces, not the energy: the forces of the lattice fixed point differ from
    the exact energy gradient by the smoothing of the potential source (about 1e-3
    relative), so near the minimum an energy test would reject moves toward zero
    force.  Stops when every free force component is below ftol hartree/bohr."""
    rule = rule or ElectronRule()
    gs = ground_state(solver, Z, R0, rule)
    alpha = step
    hist = []
    for it in range(max_iter):
        F = _free(gs.forces, fixed)
        fmax = float(np.max(np.abs(F)))
        hist.append((gs.energy, fmax, alpha))
        if fmax < ftol:
            return GeometryResult(gs.R, gs.energy, gs.forces, it, True, hist)
        move = alpha * F
        norms = np.linalg.norm(move, axis=1)
        scale = np.where(norms > max_disp, max_disp / np.maximum(norms, 1e-300), 1.0)
        gs = ground_state(solver, Z, gs.R + move * scale[:, None], rule)
        alpha *= 1.2 if float(np.sum(_free(gs.forces, fixed) * F)) > 0.0 else 0.5
    F = _free(gs.forces, fixed)
    return GeometryResult(gs.R, gs.energy, gs.forces, max_iter, bool(np.max(np.abs(F)) < ftol), hist)


@dataclass
class Trajectory:
    t: np.ndarray            # [n+1] atomic time
    R: np.ndarray            # [n+1][nuclei][3]
    V: np.ndarray            # [n+1][nuclei][3]
    e_pot: np.ndarray        # [n+1] electronic + ion-ion energy
    e_kin: np.ndarray        # [n+1] nuclear kinetic energy
    lattice_steps: np.ndarray

    @property
    def e_total(self) -> np.ndarray:
        return self.e_pot + self.e_kin


def bo_md(solver: lbks.Solver, Z: Sequence[float], R0, V0, masses: Sequence[float], dt: float,
          n_steps: int, fixed: Optional[Sequence[bool]] = None,
          rule: Optional[ElectronRule] = None) -> Trajectory:
    """Velocity Verlet on the ground-state surface:
        R(t+dt) = R + V dt + F/(2M) dt^2,  V(t+dt) = V + (F(t) + F(t+dt))/(2M) dt,
    with the electrons relaxed at every R (warm start).  masses in electron masses,
    dt in atomic time units; fixed nuclei do not move."""
    rule = rule or ElectronRule()
    M = np.asarray(masses, dtype=np.float64)[:, None]
    R = np.asarray(R0, dtype=np.float64).reshape(-1, 3).copy()
    V = np.asarray(V0, dtype=np.float64).reshape(-1, 3).copy()
    if fixed is not None:
        V[np.asarray(fixed, dtype=bool)] = 0.0
    gs = ground_state(solver, Z, R, rule)
    F = _free(gs.forces, fixed)
    ts, Rs, Vs, ep, ek, ls = [0.0], [R.copy()], [V.copy()], [gs.energy], [0.5 * float(np.sum(M * V * V))], [gs.steps]
    for k in range(n_steps):
        R = R + V * dt + F / (2.0 * M) * dt * dt
        gs = ground_state(solver, Z, R, rule)
        Fn = _free(gs.forces, fixed)
        V = V + (F + Fn) / (2.0 * M) * dt
        F = Fn
        ts.append((k + 1) * dt)
        Rs.append(R.copy())
        Vs.append(V.copy())
        ep.append(gs.energy)
        ek.append(0.5 * float(np.sum(M * V * V)))
        ls.append(gs.steps)
    return Trajectory(np.array(ts), np.array(Rs), np.array(Vs), np.array(ep), np.array(ek), np.array(ls))


@dataclass
class CDTrajectory:
    t: np.ndarray            # [n+1] atomic time
    R: np.ndarray            # [n+1][nuclei][3]
    V: np.ndarray            # [n+1][nuclei][3]
    e_t: np.ndarray          # times of the energy records
    e_pot: np.ndarray        # electronic + ion-ion energy at those times
    e_kin: np.ndarray        # nuclear kinetic energy at those times


def cd_md(solver: lbks.Solver, Z: Sequence[float], R0, V0, masses: Sequence[float], dt: float, n_steps: int,
          energy_every: int = 0, fixed: Optional[Sequence[bool]] = None,
          restart_every: int = 500) -> CDTrajectory:
    """Concurrent dynamics (the paper's concurrent scenario, eq. KSLBCD): the
    electrons, complex orbitals advanced by the library's time-centred step
    (lbks_cd_*), and the nuclei, moved by velocity Verlet with the
    Hellmann-Feynman forces of the instantaneous density, share one time step dt.
    The solver must hold the electronic ground state at R0 (relaxed there); the
    electrons start from it (lbks_cd_start).  Step n: R^{n+1} = R^n + V^n dt +
    F^n dt^2/(2M); the nuclei are set to R^{n+1}; F^{n+1} comes from psi^{n+1};
    V^{n+1} = V^n + (F^n + F^{n+1}) dt/(2M); then the electrons take the step from
    psi^{n+1} to psi^{n+2} with the potential of R^{n+1} (centred in time).  With
    energy_every > 0 the energies are recorded every that many steps
    (lbks_cd_energy, which also converges V_H).  Every restart_every-th electron
    step restarts the two-step scheme (energy references re-centred, one-step
    start), which keeps its parasitic mode from growing while the nuclei move;
    0 turns the restarts off.  The dynamics is left running; call
    solver.cd_stop() to return to the relaxation."""
    M = np.asarray(masses, dtype=np.float64)[:, None]
    R = np.asarray(R0, dtype=np.float64).reshape(-1, 3).copy()
    V = np.asarray(V0, dtype=np.float64).reshape(-1, 3).copy()
    if fixed is not None:
        V[np.asarray(fixed, dtype=bool)] = 0.0
    solver.set_nuclei(Z, R)
    F = _free(solver.forces(), fixed)
    solver.cd_start(dt, restart_every)
    ts, Rs, Vs = [0.0], [R.copy()], [V.copy()]
    et, ep, ek = [], [], []

    def record(k):
        e = solver.cd_energy()
        et.append(k * dt)
        ep.append(float(e["e_total"]))
        ek.append(0.5 * float(np.sum(M * V * V)))

    if energy_every > 0:
        record(0)
    for k in range(n_steps):
        R = R + V * dt + F / (2.0 * M) * dt * dt
        solver.set_nuclei(Z, R)
        Fn = _free(solver.forces(), fixed)
        V = V + (F + Fn) / (2.0 * M) * dt
        F = Fn
        ts.append((k + 1) * dt)
        Rs.append(R.copy())
        Vs.append(V.copy())
        if energy_every > 0 and (k + 1) % energy_every == 0:
            record(k + 1)
        if k + 1 < n_steps:
            solver.cd_step(1)
    return CDTrajectory(np.array(ts), np.array(Rs), np.array(Vs), np.array(et), np.array(ep), np.array(ek))


def vibration_frequency(t: np.ndarray, d: np.ndarray) -> float:
    """Angular frequency of an oscillating signal from its crossings of the mean of
    its extremes (linear interpolation between samples; successive crossings are
    half a period apart); nan with fewer than two crossings."""
    d = np.asarray(d, dtype=np.float64)
    x = d - 0.5 * (d.max() + d.min())
    cr = [t[i] - x[i] * (t[i + 1] - t[i]) / (x[i + 1] - x[i]) for i in range(len(x) - 1)
          if (x[i] < 0.0) != (x[i + 1] < 0.0)]
    if len(cr) < 2:
        return float("nan")
    return np.pi * (len(cr) - 1) / (cr[-1] - cr[0])
