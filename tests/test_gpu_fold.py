"""Folded reductions (lbks_params.fold).  On small grids the orthonormalisation
sums the overlap S from the tile partials itself, and the ghost-face kernel the
multipoles, in the order of the separate reduction kernels; a run with fold = 0
must equal the run with fold = -1 (the separate kernels) bit for bit, orbitals,
density, energies, Ritz values and forces alike.  The cases straddle the
threshold: both folds (at most 256 tiles of 256 nodes, at most five orbitals;
the first-level groups of 8 tiles or fewer take the smaller tree), the
multipoles alone (more orbitals), neither (more tiles); Gram-Schmidt and W, FP64
and FP32, both update schemes, a batch that
mixes folded and unfolded members, and concurrent dynamics.  Accuracy against
the oracle is the other parity tests' business: they run the folded path
wherever their grids are small.
"""
import sys

import numpy as np
import pytest

from paper_1507_07666_amd import inputs as I

pytestmark = pytest.mark.gpu

FOLD_S, FOLD_M = 1, 2


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    from paper_1507_07666_amd import lbks
    lbks.load()
    return lbks


def say(*a):
    print("[gpu-fold]", *a, file=sys.stderr, flush=True)


def same(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return a.shape == b.shape and a.dtype == b.dtype and a.tobytes() == b.tobytes()


def run(L, system, kw, fold, steps):
    s = L.Solver.for_system(system, fold=fold, **kw)
    bits = s.fold()
    out = s.relax(steps, dE_tol=0.0, check_every=10)
    psi, rho = s.orbitals()
    e = s.energy()
    H, ritz = s.hamiltonian()
    F = s.forces()
    s.close()
    return bits, out, psi, rho, e, H, ritz, F


def he_slab(nz):
    return I.System("He", (64, 64, nz), 0.25, [2.0], [(0.0, 0.0, 0.0)], 2, 1, 0.3, seed=1)


CASES = [
    # name, system, params, fold bits expected with fold = 0
    ("ne20", lambda: I.ne_atom().scaled(20, h=0.3), {}, FOLD_S | FOLD_M),                      # 32 tiles
    ("ne20_w", lambda: I.ne_atom().scaled(20, h=0.3), dict(ortho=1), FOLD_S | FOLD_M),
    ("ne_6x17x17_fp32", lambda: I.System("Ne", (6, 17, 17), 0.3, [10.0], [(0.0, 0.0, 0.0)], 10, 5, 0.3, seed=4),
     dict(precision=1), FOLD_S | FOLD_M),
    ("ne21_collapsed_fp32", lambda: I.ne_atom().scaled(21, h=0.3), dict(scheme=1, precision=1), FOLD_S | FOLD_M),
    ("he32", lambda: I.he_atom(), {}, FOLD_S | FOLD_M),                                         # 128 tiles
    ("he40", lambda: I.he_atom().scaled(40, h=0.25), {}, FOLD_S | FOLD_M),                      # 250 tiles
    ("he_64x64x16", lambda: he_slab(16), dict(scheme=1), FOLD_S | FOLD_M),                      # 256 tiles
    ("he_64x64x17", lambda: he_slab(17), dict(scheme=1), 0),                                    # 272 tiles
    ("he41", lambda: I.he_atom().scaled(41, h=0.25), {}, 0),                                    # 270 tiles
    ("z15_20", lambda: I.atom(15, 20, h=0.35, softening=0.3, seed=8), {}, FOLD_M),              # 8 orbitals
]


@pytest.mark.parametrize("name,make,kw,bits", CASES, ids=[c[0] for c in CASES])
def test_fold_equals_separate_reductions(L, name, make, kw, bits):
    system = make()
    say(name, system.dims, kw)
    b0, out0, psi0, rho0, e0, H0, r0, F0 = run(L, system, kw, 0, 30)
    b1, out1, psi1, rho1, e1, H1, r1, F1 = run(L, system, kw, -1, 30)
    assert b0 == bits and b1 == 0, (b0, b1)
    assert out0 == out1
    assert same(psi0, psi1) and same(rho0, rho1), name
    for k in ("e_total", "e_kin", "e_ext", "e_hartree", "e_x", "e_c", "n_electrons", "poisson_residual"):
        assert same(e0[k], e1[k]), (k, e0[k], e1[k])
    assert same(e0["eps"], e1["eps"])
    assert same(H0, H1) and same(r0, r1) and same(F0, F1)
    assert np.isfinite(e0["e_total"])


def test_fold_in_a_mixed_batch(L):
    """Members that fold alone and members that do not, in one group: the launch
    folds only when every member does, so here the separate kernels serve them
    all, and every member still equals its run alone bit for bit."""
    members = [
        (I.ne_atom().scaled(20, h=0.3), dict(fold=0)),
        (I.ne_atom().scaled(18, h=0.3), dict(fold=-1)),
        (I.he_atom().scaled(48, h=0.25), dict(fold=0)),     # 432 tiles: no fold
        (I.atom(3, 17, h=0.35, seed=6), dict(fold=0)),
    ]
    b = L.Batch()
    solvers = [b.add_system(sy, **kw) for sy, kw in members]
    assert [s.fold() for s in solvers] == [FOLD_S | FOLD_M, 0, 0, FOLD_S | FOLD_M]
    st, steps = b.relax(25, dE_tol=0.0, check_every=10)
    assert steps == [25] * len(members)
    for (sy, kw), s in zip(members, solvers):
        say("batch member", sy.name, sy.dims, kw)
        psi, rho = s.orbitals()
        a = L.Solver.for_system(sy, **kw)
        a.relax(25, dE_tol=0.0, check_every=10)
        psi_a, rho_a = a.orbitals()
        a.close()
        assert same(psi, psi_a) and same(rho, rho_a), sy.name
    b.close()


def test_fold_in_concurrent_dynamics(L):
    """The dynamics step rebuilds the Hartree boundary each step from the
    multipoles; H2 on 20^3 folds them."""
    system = I.System("H2", (20, 20, 20), 0.35, [1.0, 1.0], [(-0.75, 0.0, 0.0), (0.75, 0.0, 0.0)], 2, 1, 0.3, seed=3)
    res = []
    for fold in (0, -1):
        s = L.Solver.for_system(system, fold=fold, poisson_sweeps=4)
        s.relax(300)
        s.cd_start(0.02, 15)
        s.cd_step(40)
        e = s.cd_energy()
        res.append((s.fold(), s.cd_orbitals(), e["e_total"], s.forces()))
        s.cd_stop()
        s.close()
    (b0, psi0, E0, F0), (b1, psi1, E1, F1) = res
    assert b0 == FOLD_S | FOLD_M and b1 == 0
    assert same(psi0, psi1) and same(E0, E1) and same(F0, F1)


def test_small_grid_defaults(L):
    """Grids of at most 256 tiles start from the node-per-lane population update
    (0 in FP64, 1 in FP32) and fold; larger ones start from the rolled wide form
    (13) and do not; the brick update keeps its own defaults."""
    cases = [
        (I.he_atom(), {}, 0, FOLD_S | FOLD_M),                                  # 128 tiles
        (I.he_atom(), dict(precision=1), 1, FOLD_S | FOLD_M),
        (he_slab(16), {}, 0, FOLD_S | FOLD_M),                                  # 256 tiles
        (he_slab(17), {}, 13, 0),                                               # 272 tiles
        (he_slab(17), dict(precision=1), 13, 0),
        (I.he_atom(), dict(fold=-1), 0, 0),
        (I.he_atom(), dict(scheme=1), 0, FOLD_S | FOLD_M),                      # the brick update
        (he_slab(17), dict(scheme=1, precision=1), 1, 0),
        (I.atom(15, 20, h=0.35, softening=0.3, seed=8), {}, 4, FOLD_M),         # 8 orbitals
    ]
    for system, kw, variant, bits in cases:
        s = L.Solver.for_system(system, **kw)
        got = (s.variant(), s.fold())
        s.close()
        assert got == (variant, bits), (system.dims, kw, got)
