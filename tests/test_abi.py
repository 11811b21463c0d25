"""The C-ABI library loads, exports every symbol include/lbks.h declares, and its
host-only parameter logic behaves as documented (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbks.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = set(re.findall(r"\b(lbks_[a-z_]+)\s*\(", txt))
    return names


@pytest.fixture(scope="module")
def L():
    from paper_1507_07666_amd import lbks
    return lbks.load()


def test_header_declares_the_core_calls():
    names = declared_functions()
    for n in ("lbks_create", "lbks_set_nuclei", "lbks_relax", "lbks_energy", "lbks_orbitals",
              "lbks_destroy", "lbks_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(L):
    from paper_1507_07666_amd import lbks
    names = declared_functions()
    for n in names:
        assert hasattr(L, n), n
    assert names == set(lbks.SIGNATURES), names ^ set(lbks.SIGNATURES)


def test_struct_layouts_match_the_header(tmp_path):
    """Compile a probe against include/lbks.h with gcc and compare sizes and offsets
    with the ctypes mirrors."""
    import subprocess
    from paper_1507_07666_amd import lbks
    probe = tmp_path / "probe.c"
    fields = {"lbks_params": [f for f, _ in lbks.lbks_params._fields_],
              "lbks_energies": [f for f, _ in lbks.lbks_energies._fields_],
              "lbks_device": [f for f, _ in lbks.lbks_device._fields_]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lbks.h"', "int main(void){"]
    for st, fl in fields.items():
        lines.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in fl:
            lines.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines.append("return 0;}")
    probe.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(probe), "-o", str(exe)])
    out = dict(l.split() for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for st, fl in fields.items():
        cls = getattr(lbks, st)
        assert int(out[st]) == ctypes.sizeof(cls), st
        for f in fl:
            assert int(out[f"{st}.{f}"]) == getattr(cls, f).offset, (st, f)


def test_defaults(L):
    from paper_1507_07666_amd import lbks
    p = lbks.lbks_params_default()
    assert p.omega == 1.0 and abs(p.D - 1.0 / 3.0) < 1e-16 and p.poisson_sweeps == 2
    assert p.xc == lbks.LBKS_XC_X_LYPLOCAL and p.hartree == 1 and p.precision == lbks.LBKS_FP64


def test_parameter_validation_host_side(L):
    from paper_1507_07666_amd import lbks
    ok = lbks.params(32, 0.3, 1, 2)
    est = L.lbks_estimate_bytes(ctypes.byref(ok))
    N = 32 ** 3
    assert est >= 2 * 19 * N * 8 and est < 2 * 19 * N * 8 * 1.6
    bad = [dict(D=0.5), dict(omega=2.0), dict(omega=0.0), dict(scheme=1, omega=0.8),
           dict(n_elec=3), dict(n_orb=0), dict(h=-1.0), dict(poisson_sweeps=-1)]
    for kw in bad:
        kw = dict(kw)
        p = lbks.params(32, kw.pop("h", 0.3), kw.pop("n_orb", 1), kw.pop("n_elec", 2), **kw)
        assert L.lbks_estimate_bytes(ctypes.byref(p)) == 0, kw
    p = lbks.params(16, 0.3, 1, 2)
    p.reserved[0] = 1
    assert L.lbks_estimate_bytes(ctypes.byref(p)) == 0
    for fold, ok_ in ((0, True), (-1, True), (1, False), (2, False)):
        p = lbks.params(16, 0.3, 1, 2, fold=fold)
        assert (L.lbks_estimate_bytes(ctypes.byref(p)) > 0) == ok_, fold
    fp32 = lbks.params(32, 0.3, 1, 2, precision=lbks.LBKS_FP32_BULK)
    assert L.lbks_estimate_bytes(ctypes.byref(fp32)) < est
    coll = lbks.params(32, 0.3, 1, 2, scheme=lbks.LBKS_SCHEME_COLLAPSED)
    assert L.lbks_estimate_bytes(ctypes.byref(coll)) < est / 4
    # exchange-correlation kinds: the gradient-corrected ones need 32 more bytes per node;
    # the fully spin-polarised one holds one electron per orbital
    gga = lbks.params(32, 0.3, 1, 2, xc=lbks.LBKS_XC_B88_LYP)
    assert L.lbks_estimate_bytes(ctypes.byref(gga)) >= est + 32 * N
    pol = lbks.params(32, 0.3, 3, 3, xc=lbks.LBKS_XC_B88_LYP_POLARISED)
    assert L.lbks_estimate_bytes(ctypes.byref(pol)) > 0
    for n_orb, n_elec, xc in ((1, 2, lbks.LBKS_XC_B88_LYP_POLARISED), (3, 5, lbks.LBKS_XC_B88_LYP_POLARISED),
                              (1, 2, lbks.LBKS_XC_B88_LYP_POLARISED + 1), (1, 2, -1)):
        q = lbks.params(32, 0.3, n_orb, n_elec, xc=xc)
        assert L.lbks_estimate_bytes(ctypes.byref(q)) == 0, (n_orb, n_elec, xc)


def test_create_rejects_invalid_params_before_touching_a_device(L):
    from paper_1507_07666_amd import lbks
    p = lbks.params(16, 0.3, 1, 2, D=1.0)
    with pytest.raises(lbks.LbksError) as ei:
        lbks.lbks_create(p)
    assert ei.value.code == lbks.LBKS_E_INVAL
    assert "7/18" in str(ei.value)
    p = lbks.params(16, 0.3, 1, 2, fold=3)
    with pytest.raises(lbks.LbksError) as ei:
        lbks.lbks_create(p)
    assert ei.value.code == lbks.LBKS_E_INVAL and "fold" in str(ei.value)
    # the queries of a context refuse a NULL one without a device
    assert lbks.load().lbks_get_fold(None) == lbks.LBKS_E_INVAL
    assert lbks.load().lbks_get_variant(None) == lbks.LBKS_E_INVAL


def test_bench_refuses_several_gpus():
    """The bench runs on one GPU; asked for more it exits with a message."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=root)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
