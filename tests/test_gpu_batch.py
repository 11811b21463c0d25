"""Batched solves: one launch per kernel for many solves of uneven grids, orbital
counts and precisions, each step captured in a HIP graph.  Every member's result
must be the same as that solve run alone (bitwise: tile work and reduction order
depend only on the solve), and the stopping rule must act per member."""
import sys

import numpy as np
import pytest

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
    print("[gpu-batch]", *a, file=sys.stderr, flush=True)


def mixed_systems():
    return [
        (I.he_atom().scaled(16), {}),
        (I.ne_atom().scaled(20), {}),
        (I.atom(7, 18, h=0.3, seed=5), {}),
        (I.h2o_batch(2)[1].scaled(24, h=0.35), dict(precision=1)),
        (I.ne_atom().scaled(20), dict(precision=1)),
        (I.atom(3, 17, h=0.35, seed=6), dict(ortho=1)),
        (I.he_atom().scaled(18, h=0.3), dict(xc=4)),          # gradient-corrected xc: its own group
        (I.ne_atom().scaled(21, h=0.3), dict(scheme=1)),      # omega = 1 field update (LDS bricks)
        (I.ne_atom().scaled(19, h=0.3), dict(scheme=1)),      # same group; more bricks than tiles
        (I.atom(6, 19, h=0.32, seed=7), dict(scheme=1, precision=1)),
    ]


def alone(L, system, kw, steps, tol=0.0, every=10, variant=None):
    s = L.Solver.for_system(system, **kw)
    if variant is not None:
        s.set_variant(variant)
    out = s.relax(steps, dE_tol=tol, check_every=every)
    psi, rho = s.orbitals()
    e = s.energy()
    s.close()
    return out, psi, rho, e


def test_batch_equals_alone_fixed_steps(L):
    say("batch fixed steps")
    systems = mixed_systems()
    b = L.Batch()
    members = [b.add_system(sy, **kw) for sy, kw in systems]
    variants = [0, 5, 2, 7, 3, 6] + [None] * (len(systems) - 6)
    for m, v in zip(members, variants):
        if v is not None:
            m.set_variant(v)
    st, steps = b.relax(25, dE_tol=0.0, check_every=10)
    assert steps == [25] * len(systems)
    assert all(x == L.LBKS_NOT_CONVERGED for x in st)
    assert len(variants) == len(members) == len(systems)
    for (sy, kw), s, v in zip(systems, members, variants):
        say("member", sy.name, kw)
        psi, rho = s.orbitals()
        _, psi_a, rho_a, _ = alone(L, sy, kw, 25, variant=v)
        assert np.array_equal(psi, psi_a) and np.array_equal(rho, rho_a), sy.name
    # members stay usable one by one, and continue in the batch
    e0 = members[0].energy()
    st, steps = b.relax(6, dE_tol=0.0, check_every=4)
    assert steps == [6] * len(systems)
    b.close()
    assert np.isfinite(e0["e_total"])


@pytest.mark.parametrize("rule", ["energy", "eigenvalue_sum_confirmed"])
def test_batch_stopping_rule_per_member(L, rule):
    say("batch convergence", rule)
    r = {} if rule == "energy" else dict(deps_tol=1e-7, stop_checks=2)
    systems = [(I.he_atom().scaled(12, h=0.4), dict(r)), (I.atom(4, 14, h=0.35, seed=9), dict(r)),
               (I.he_atom().scaled(14, h=0.4), dict(precision=1, **r))]
    b = L.Batch()
    members = [b.add_system(sy, **kw) for sy, kw in systems]
    st, steps = b.relax(4000, dE_tol=1e-8, check_every=20)
    for (sy, kw), s, rc, n in zip(systems, members, st, steps):
        (rc_a, n_a), _, _, e_a = alone(L, sy, kw, 4000, tol=1e-8, every=20)
        assert (rc, n) == (rc_a, n_a), (sy.name, rc, n, rc_a, n_a)
        e = s.energy()
        assert e["e_total"] == e_a["e_total"], sy.name
    b.close()


def test_batch_relax_without_steps_reports_statuses(L):
    """A relax that steps nothing still reports every member: max_steps = 0, a
    member without a potential, and a member attached after the last build all
    read back through a pointer table built for the current members."""
    say("batch relax without steps")
    b = L.Batch()
    with_nuc = b.add_system(I.he_atom().scaled(12, h=0.4))
    without = b.add_system(I.he_atom().scaled(12, h=0.4), set_nuclei=False)
    st, steps = b.relax(0, dE_tol=0.0, check_every=10)
    assert st == [L.LBKS_NOT_CONVERGED, L.LBKS_E_STATE] and steps == [0, 0]
    st, steps = b.relax(5, dE_tol=0.0, check_every=10)
    assert st == [L.LBKS_NOT_CONVERGED, L.LBKS_E_STATE] and steps == [5, 0]
    late = b.add_system(I.atom(3, 12, h=0.4, seed=9))          # attached after the last build
    st, steps = b.relax(0, dE_tol=0.0, check_every=10)
    assert st == [L.LBKS_NOT_CONVERGED, L.LBKS_E_STATE, L.LBKS_NOT_CONVERGED] and steps == [0, 0, 0]
    b.remove(without)
    without.close()
    st, steps = b.relax(0, dE_tol=0.0, check_every=10)
    assert st == [L.LBKS_NOT_CONVERGED, L.LBKS_NOT_CONVERGED] and steps == [0, 0]
    only = L.Batch()
    only.add_system(I.he_atom().scaled(12, h=0.4), set_nuclei=False)
    st, steps = only.relax(3, dE_tol=1e-8, check_every=1)
    assert st == [L.LBKS_E_STATE] and steps == [0]
    assert np.isfinite(with_nuc.energy()["e_total"]) and np.isfinite(late.energy()["e_total"])
    only.close()
    b.close()
