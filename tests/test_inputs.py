"""Seeded input generators: SplitMix64 against its published outputs, geometry recipes."""
import math
import os

import numpy as np

from paper_1507_07666_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.txt")


def test_splitmix64_reference_vectors():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) >= 8
    for seed, k, val in rows:
        got = int(I.splitmix64(int(seed), np.array([int(k)], dtype=np.uint64))[0])
        assert got == int(val), (seed, k)


def test_uniform_range_and_determinism():
    u = I.uniform(7, np.arange(100000, dtype=np.uint64))
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.01
    assert np.array_equal(u, I.uniform(7, np.arange(100000, dtype=np.uint64)))


def test_initial_orbitals_counter_layout():
    dims = (5, 4, 3)
    psi = I.init_random_gauss(dims, 0.3, 2, 1.0, seed=9)
    assert psi.shape == (2, 3, 4, 5)
    # draw k runs over (orbital, z, y, x) with x fastest
    j, z, y, x = 1, 2, 3, 4
    k = ((j * 3 + z) * 4 + y) * 5 + x
    u = I.uniform(9, np.array([k], dtype=np.uint64))[0]
    r2 = sum(c ** 2 for c in ((x - 2.0) * 0.3, (y - 1.5) * 0.3, (z - 1.0) * 0.3))
    assert psi[j, z, y, x] == math.exp(-r2 / 2.0) * (2.0 * u - 1.0)


def test_ch4_geometry():
    s = I.ch4()
    assert s.dims == (128, 128, 128) and s.n_orb == 5 and s.n_elec == 10
    C = np.array(s.R[0])
    Hs = np.array(s.R[1:])
    L = np.linalg.norm(Hs - C, axis=1)
    assert np.all((L >= 1.9) & (L <= 2.2))
    d = Hs / L[:, None]
    for a in range(4):
        for b in range(a + 1, 4):
            assert abs(np.dot(d[a], d[b]) + 1.0 / 3.0) < 1e-12   # tetrahedral angle


def test_h2o_batch_recipe():
    b = I.h2o_batch(64)
    assert len(b) == 64
    sizes = set()
    for s in b:
        O, H1, H2 = (np.array(r) for r in s.R)
        L1, L2 = np.linalg.norm(H1 - O), np.linalg.norm(H2 - O)
        ang = math.degrees(math.acos(np.dot(H1, H2) / (L1 * L2)))
        assert 1.7 <= L1 <= 1.9 and 1.7 <= L2 <= 1.9
        assert 95.0 <= ang <= 115.0
        sizes.add(s.dims[0])
    assert sizes <= set(I.H2O_GRIDS) and len(sizes) >= 3
    total = sum(s.n_sites for s in b)
    assert 16.8e6 <= total <= 89.9e6


def test_nh3_geometry():
    s = I.nh3_from_geometry(1.9, 107.0, 64)
    Hs = np.array(s.R[1:])
    for a in range(3):
        for b in range(a + 1, 3):
            c = np.dot(Hs[a], Hs[b]) / (np.linalg.norm(Hs[a]) * np.linalg.norm(Hs[b]))
            assert abs(math.degrees(math.acos(c)) - 107.0) < 1e-9
    assert np.allclose(np.linalg.norm(Hs, axis=1), 1.9)


def test_serving_stream_recipe():
    reqs = I.serving_stream(40, rate=2.0)
    t = [r.arrival for r in reqs]
    assert all(b > a for a, b in zip(t, t[1:]))
    kinds = {len(r.points) for r in reqs}
    assert kinds == {1, 8}
    for r in reqs:
        for p in r.points:
            assert p.dims[0] in I.SERVE_GRIDS and 1 <= p.n_orb <= 5
