"""lbks_batch_relax_static, the batch relaxation for callers that cannot allocate
device memory, against lbks_batch_relax on identical batches: the same statuses,
step counts and orbitals bit for bit (same kernels in the same order; the static
form launches them one by one instead of from graphs), on two calls in a row, the
second with fewer and smaller members; and a batch whose tables exceed the static
workspace is refused with a clear error, leaving the allocating call usable."""
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
    print("[gpu-no-alloc]", *a, file=sys.stderr, flush=True)


def make_batch(L, systems):
    b = L.Batch()
    members = []
    for sy, kw in systems:
        m = b.add(L.params_for(sy, init=L.LBKS_INIT_USER, **kw))
        m.set_nuclei(sy.Z, sy.R)
        m.set_orbitals(sy.psi0())
        members.append(m)
    return b, members


def outcome(members):
    return [(m.orbitals()[0], m.energy()["e_total"]) for m in members]


def compare(L, systems, steps, tol, every):
    b_ref, m_ref = make_batch(L, systems)
    b_st, m_st = make_batch(L, systems)
    st_ref, k_ref = b_ref.relax(steps, tol, every)
    st_st, k_st = b_st.relax(steps, tol, every, static=True)
    assert st_st == st_ref and k_st == k_ref, (st_st, st_ref, k_st, k_ref)
    for (p_ref, e_ref), (p_st, e_st), (sy, _) in zip(outcome(m_ref), outcome(m_st), systems):
        assert np.array_equal(p_ref, p_st) and e_ref == e_st, sy.name
    b_ref.close()
    b_st.close()
    return st_ref, k_ref


def test_static_workspace_equals_allocating_relax_twice(L):
    big = [(I.ne_atom().scaled(22), dict(precision=0)),
           (I.h2o_batch(2)[1].scaled(24, h=0.35), dict(precision=1)),
           (I.ne_atom().scaled(21, h=0.3), dict(scheme=1)),
           (I.atom(3, 17, h=0.35, seed=6), dict(ortho=1))]
    small = [(I.he_atom().scaled(14, h=0.4), dict(precision=0)),
             (I.atom(4, 13, h=0.4, seed=9), dict(precision=1))]
    say("four members, fixed steps")
    st, k = compare(L, big, 30, 0.0, 10)
    assert k == [30] * 4
    say("two smaller members, stopping rule")
    st, k = compare(L, small, 3000, 1e-8, 20)
    assert all(x == L.LBKS_OK for x in st) and all(n < 3000 for n in k), (st, k)
    # the same batch on both entry points in turn: the allocating call rebuilds its
    # own tables after the static one
    b, ms = make_batch(L, small)
    b.relax(10, static=True)
    b.relax(10)
    b.relax(0, static=True)
    b2, ms2 = make_batch(L, small)
    b2.relax(20)
    assert all(np.array_equal(a[0], c[0]) for a, c in zip(outcome(ms), outcome(ms2)))
    b.close()
    b2.close()


def test_static_workspace_refuses_oversized_tables(L):
    """Twenty 128^3 members (omega = 1 field update, no populations) need about
    2.4 MB of tables (118 KB each: site, ghost, SOR, brick and wide-update tile
    entries), more than the 2 MiB workspace."""
    systems = [(I.he_atom().scaled(128, h=0.15), dict(precision=1, scheme=1)) for _ in range(20)]
    b, members = make_batch(L, systems)
    say("oversized batch")
    with pytest.raises(L.LbksError) as ex:
        b.relax(5, static=True)
    assert "static workspace" in str(ex.value) and ex.value.code == L.LBKS_E_INVAL
    st, k = b.relax(5)                      # the allocating call still serves this batch
    assert k == [5] * 20
    b.close()
