"""The gradient-corrected functional (Becke 88 exchange + Lee-Yang-Parr
correlation) against the exchange and correlation energies the paper's Table 1
lists (tests/golden/table1_xc.txt): the closed-shell atoms He and Be
spin-unpolarised, and the one-electron H fully spin-polarised.

Each atom is relaxed with the local functional first and then with the
gradient-corrected one from those orbitals (a rough start makes the explicit
potential step of a gradient-corrected functional unstable).  Grid 96^3 at
0.1 bohr with nuclear softening 0.01 bohr; the paper reports its own lattice
values within about 1 % of these; the softened, finitely resolved nuclear cusp
moves ours by about 1.5 %, so the bar is 2 %.
"""
import os
import sys

import numpy as np
import pytest

from paper_1507_07666_amd import inputs as I

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(__file__)


def table1():
    rows = {}
    for line in open(os.path.join(HERE, "golden", "table1_xc.txt")):
        if line.strip() and not line.startswith("#"):
            name, Z, ne, vx, vc = line.split()
            rows[name] = (int(Z), int(ne), float(vx), float(vc))
    return rows


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_1507_07666_amd import lbks
    lbks.load()
    return lbks


@pytest.mark.parametrize("atom", ["H", "He", "Be"])
def test_exchange_correlation_energies_against_table1(L, atom):
    Z, ne, vx_ref, vc_ref = table1()[atom]
    sy = I.System(atom, (96, 96, 96), 0.1, [float(Z)], [(0.0, 0.0, 0.0)], ne, (ne + 1) // 2, 0.01, seed=1,
                  init="gauss_noise", init_sigma=1.0, init_noise=1e-3)
    xc = L.LBKS_XC_B88_LYP_POLARISED if ne == 1 else L.LBKS_XC_B88_LYP
    lda = L.Solver.for_system(sy)
    lda.relax(40000, 1e-8, 100)
    psi, _ = lda.orbitals()
    lda.close()
    s = L.Solver(L.params_for(sy, init=L.LBKS_INIT_USER, xc=xc))
    s.set_nuclei(sy.Z, sy.R)
    s.set_orbitals(psi)
    rc, steps = s.relax(40000, 1e-10, 100)
    e = s.energy()
    s.close()
    print(f"[table1] {atom}: E_x {e['e_x']:.5f} (table {vx_ref}), E_c {e['e_c']:.5f} (table {vc_ref}), "
          f"E {e['e_total']:.5f}, eps {np.round(e['eps'], 5)}, {steps} steps", file=sys.stderr, flush=True)
    assert rc == L.LBKS_OK
    assert abs(e["e_x"] - vx_ref) <= 0.02 * abs(vx_ref)
    if vc_ref == 0.0:
        assert e["e_c"] == 0.0                       # one spin: no Lee-Yang-Parr correlation
    else:
        assert abs(e["e_c"] - vc_ref) <= 0.02 * abs(vc_ref)
