"""Pins of the oracle's lattice constants by the moment identities the method
requires (equilibrium and potential source of the lattice Boltzmann equation):
  sum xi = 1, sum xi v = 0, sum xi v v = D I         (mass conservation, diffusivity D)
  sum chi = 1, sum chi v = 0, sum chi v v = 0         (source leaves momentum and energy)
and fourth-order isotropy of the weights, which the zero second moment of chi needs."""
import itertools

import numpy as np
import pytest


@pytest.mark.parametrize("D", [1.0 / 3.0, 0.25, 0.3])
def test_equilibrium_and_source_moments(oracle_mod, D):
    v, w, xi, chi = oracle_mod.lattice(D)
    v = v.astype(float)
    assert len({tuple(r) for r in v.astype(int)}) == 19
    assert np.all((v ** 2).sum(1) <= 2)
    assert abs(w.sum() - 1) < 1e-15
    assert abs(xi.sum() - 1) < 1e-15
    assert np.allclose((xi[:, None] * v).sum(0), 0, atol=1e-16)
    assert np.allclose(np.einsum("p,pa,pb->ab", xi, v, v), D * np.eye(3), atol=1e-15)
    assert abs(chi.sum() - 1) < 1e-15
    assert np.allclose((chi[:, None] * v).sum(0), 0, atol=1e-16)
    assert np.allclose(np.einsum("p,pa,pb->ab", chi, v, v), 0, atol=1e-15)


def test_weights_fourth_order_isotropic(oracle_mod):
    v, w, _, _ = oracle_mod.lattice()
    v = v.astype(float)
    cs2 = np.einsum("p,pa,pa->", w, v, v) / 3.0
    assert abs(cs2 - 1.0 / 3.0) < 1e-15
    d = np.eye(3)
    T = np.einsum("p,pa,pb,pc,pd->abcd", w, v, v, v, v)
    iso = cs2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                      + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(T, iso, atol=1e-15)
    # odd moments vanish
    for a, b, c in itertools.product(range(3), repeat=3):
        assert abs(np.sum(w * v[:, a] * v[:, b] * v[:, c])) < 1e-16


def test_default_equilibrium_is_weights(oracle_mod):
    _, w, xi, chi = oracle_mod.lattice(1.0 / 3.0)
    assert np.allclose(xi, w, rtol=0, atol=1e-16)
    # chi by speed class: rest 5/6, faces 1/18, edges -1/72
    assert sorted(set(np.round(chi, 14))) == sorted({round(5 / 6, 14), round(1 / 18, 14), round(-1 / 72, 14)})
