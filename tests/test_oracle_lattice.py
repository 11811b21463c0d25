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


@pytest.mark.parametrize("D", [1.0 / 3.0, 0.25, 0.5])
def test_fourth_order_weights_moments(oracle_mod, D):
    """Fourth-order Hermite weights (the paper's He run): xi carries the zeroth,
    second and mixed fourth moments of a Gaussian of variance D, chi only a zeroth
    moment; both have no odd moments; the closed forms rest 1 - 3D + 3D^2, faces
    D/2 - D^2, edges D^2/4 follow; at D = c_s^2 = 1/3 xi is the second-order set."""
    v, w, xi, chi = oracle_mod.lattice4(D)
    v = v.astype(float)
    d = np.eye(3)
    assert abs(xi.sum() - 1) < 1e-15 and abs(chi.sum() - 1) < 1e-15
    assert np.allclose(np.einsum("p,pa,pb->ab", xi, v, v), D * d, atol=1e-15)
    assert np.allclose(np.einsum("p,pa,pb->ab", chi, v, v), 0, atol=1e-15)
    for a, b in ((0, 1), (0, 2), (1, 2)):
        assert abs(np.sum(xi * v[:, a] ** 2 * v[:, b] ** 2) - D * D) < 1e-15
        assert abs(np.sum(chi * v[:, a] ** 2 * v[:, b] ** 2)) < 1e-15
    for wts in (xi, chi):
        assert np.allclose((wts[:, None] * v).sum(0), 0, atol=1e-16)
        for a, b, c in itertools.product(range(3), repeat=3):
            assert abs(np.sum(wts * v[:, a] * v[:, b] * v[:, c])) < 1e-16
    speed = (v ** 2).sum(1)
    expect = np.where(speed == 0, 1 - 3 * D + 3 * D * D, np.where(speed == 1, D / 2 - D * D, D * D / 4))
    assert np.allclose(xi, expect, rtol=0, atol=1e-15)
    assert np.allclose(chi, (speed == 0).astype(float), rtol=0, atol=1e-15)
    if abs(D - 1.0 / 3.0) < 1e-15:
        assert np.allclose(xi, oracle_mod.lattice(D)[2], rtol=0, atol=1e-15)


def test_fourth_order_symbol_non_negative_up_to_one_half(oracle_mod):
    """The symbol sum_p xi_p cos(k . v_p) of the fourth-order equilibrium stays
    non-negative for D <= 1/2 (its minimum (1 - 2D) sits at k = (0, pi, pi)), so the
    relaxation is stable there; beyond it the symbol turns negative."""
    k1 = np.linspace(0.0, np.pi, 17)
    K = np.stack(np.meshgrid(k1, k1, k1, indexing="ij"), -1).reshape(-1, 3)
    for D, ok in ((0.25, True), (1.0 / 3.0, True), (0.5, True), (0.55, False)):
        v, _, xi, _ = oracle_mod.lattice4(D)
        sym = np.cos(K @ v.T.astype(float)) @ xi
        assert (sym.min() >= -1e-15) == ok, (D, sym.min())
        assert abs(sym.min() - min(1.0 - 2 * D, (1.0 - 2 * D) ** 2, 1 - 6 * D + 12 * D * D)) < 1e-12
