"""Address and undefined-behaviour sanitizer runs of the CPU code (no GPU).

  * the oracle (oracle/lbks_oracle.c) built with gcc -fsanitize=address,undefined
    and driven through every C entry point the tests use: population and field
    steps with Hartree and the local functional, the W mode, omega != 1, the
    gradient-corrected functional (both spin kinds), forces, the sequential order
    and concurrent dynamics, on a ragged grid;
  * the host side of the C-ABI library (lbks_capi.hip, host code only, built with
    AddressSanitizer and UBSan; the device code is the normal build) through the
    calls that run without a GPU: defaults, the parameter validation of
    lbks_estimate_bytes and lbks_create, and the error paths when no device is
    present.

Each runs in a child process with the sanitizer runtime preloaded; any report
(or a non-zero exit) fails the test.
"""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REPORTS = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer", "SUMMARY: UndefinedBehavior")


def runtime(cc, name):
    r = subprocess.run([cc, f"-print-file-name={name}"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def run_child(script, env_extra, timeout):
    env = dict(os.environ)
    env.update(env_extra)
    env.update(ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2",
               PYTHONPATH=ROOT + os.pathsep + env.get("PYTHONPATH", ""))
    r = subprocess.run([sys.executable, "-c", textwrap.dedent(script)], capture_output=True, text=True,
                       timeout=timeout, env=env, cwd=ROOT)
    found = [m for m in REPORTS if m in r.stderr]
    assert r.returncode == 0 and not found and "SANITIZED RUN OK" in r.stdout, \
        (r.returncode, found, r.stdout[-2000:], r.stderr[-6000:])


ORACLE_SCRIPT = """
import numpy as np
from oracle import oracle as O
from paper_1507_07666_amd import inputs as I
assert O.LIB_PATH.endswith("liblbks_oracle_san.so"), O.LIB_PATH
s = I.ne_atom().scaled(13)
s.dims = (13, 11, 9)
for kw in (dict(), dict(ortho="w"), dict(omega=0.8), dict(xc=O.XC_X_PZ81), dict(hartree=False, xc=O.XC_NONE)):
    o = O.oracle_for(s, **kw)
    for _ in range(3):
        o.step()
    e = o.energies(converge_poisson=True)
    assert np.isfinite(e.e_total)
o = O.oracle_for(s)
o.relax(20, 1e-9, 10, fields=True)
F = o.forces()
H, ritz = o.hamiltonian()
assert np.all(np.isfinite(F)) and np.all(np.isfinite(ritz))
for xc in (O.XC_B88_LYP,):
    g = O.oracle_for(s, xc=xc)
    g.step()
    assert np.isfinite(g.energies(converge_poisson=True).e_total)
h = I.System("H3", (11, 10, 9), 0.4, [1.0, 1.0, 1.0], [(-0.8, 0.0, 0.0), (0.8, 0.0, 0.0), (0.0, 0.9, 0.0)], 3, 3,
             0.4, seed=3)
p = O.oracle_for(h, xc=O.XC_B88_LYP_POLARISED)
p.step()
assert np.isfinite(p.energies(converge_poisson=True).e_total)
q = O.oracle_for(s)
O.relax_sequential(q, 60, 1e-6, 1e-6, 10, 2)
cd = O.ConcurrentDynamics(O.oracle_for(s), 0.002, restart_every=3)
for _ in range(7):
    cd.step()
assert np.isfinite(cd.energies(converge_poisson=True).e_total) and np.all(np.isfinite(cd.forces()))
print("SANITIZED RUN OK")
"""


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    asan = runtime("gcc", "libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = tmp_path / "liblbks_oracle_san.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-o", str(lib), os.path.join(ROOT, "oracle", "lbks_oracle.c"), "-lm"])
    run_child(ORACLE_SCRIPT, {"LD_PRELOAD": asan, "LBKS_ORACLE_LIB": str(lib)}, timeout=600)


HOST_SCRIPT = """
import ctypes, sys
from paper_1507_07666_amd import lbks
L = ctypes.CDLL(sys.argv[1] if len(sys.argv) > 1 else LIB)
for name, (res, args) in lbks.SIGNATURES.items():
    fn = getattr(L, name)
    fn.restype = res
    fn.argtypes = args
p = lbks.lbks_params()
assert L.lbks_params_default(ctypes.byref(p)) == 0
ok = lbks.params(24, 0.3, 2, 4)
assert L.lbks_estimate_bytes(ctypes.byref(ok)) > 0
bad = [dict(D=0.5), dict(omega=2.0), dict(scheme=1, omega=0.8), dict(poisson_sweeps=-1), dict(hermite=3),
       dict(hermite=4, D=0.6), dict(xc=99), dict(precision=7), dict(ortho=5)]
for kw in bad:
    q = lbks.params(24, 0.3, 2, 4, **kw)
    assert L.lbks_estimate_bytes(ctypes.byref(q)) == 0, kw
for n_orb, n_elec in ((0, 2), (17, 34), (2, 5), (2, 0)):
    q = lbks.params(24, 0.3, 1, 2)
    q.n_orb, q.n_elec = n_orb, n_elec
    assert L.lbks_estimate_bytes(ctypes.byref(q)) == 0, (n_orb, n_elec)
ctx = ctypes.c_void_p()
q = lbks.params(16, 0.3, 1, 2, D=1.0)
assert L.lbks_create(ctypes.byref(q), None, ctypes.byref(ctx)) == lbks.LBKS_E_INVAL
assert b"7/18" in L.lbks_last_error(None)
assert L.lbks_create(None, None, ctypes.byref(ctx)) != 0
rc = L.lbks_create(ctypes.byref(ok), None, ctypes.byref(ctx))   # no GPU here: an error, not a crash
assert rc != 0 and not ctx.value and L.lbks_last_error(None)
b = ctypes.c_void_p()
assert L.lbks_batch_create(None, ctypes.byref(b)) != 0 and not b.value
assert L.lbks_energy(None, None) == lbks.LBKS_E_INVAL
assert L.lbks_cd_step(None, 1) == lbks.LBKS_E_INVAL
assert L.lbks_batch_size(None) == 0
assert L.lbks_get_fold(None) == lbks.LBKS_E_INVAL
q = lbks.params(24, 0.3, 2, 4, fold=-2)
assert L.lbks_estimate_bytes(ctypes.byref(q)) == 0
L.lbks_destroy(None)
L.lbks_batch_destroy(None)
print("SANITIZED RUN OK")
"""


def test_host_library_under_address_and_undefined_sanitizers(tmp_path):
    """lbks_capi.hip's host code with AddressSanitizer and UBSan (each -fsanitize
    applies to the host pass only), linked with the normal objects of the other
    sources."""
    from paper_1507_07666_amd import build as B
    hipcc = B.HIPCC
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    asan = runtime(os.path.join(os.path.dirname(os.path.realpath(hipcc)), "..", "llvm", "bin", "clang"),
                   "libclang_rt.asan-x86_64.so")
    if asan is None:
        import glob
        hits = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        asan = hits[0] if hits else None
    if asan is None:
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    objs = []
    for src in B.SOURCES:
        if src == "lbks_capi.hip":
            continue
        o = os.path.join(B.BUILD, os.path.splitext(src)[0] + ".o")
        if not os.path.exists(o):
            B.build()
        objs.append(o)
    capi = tmp_path / "lbks_capi_san.o"
    subprocess.check_call([hipcc] + B.FLAGS + ["-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                                               "-fsanitize=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
                                               "-c", os.path.join(B.CSRC, "lbks_capi.hip"), "-o", str(capi)])
    lib = tmp_path / "liblbks_san.so"
    subprocess.check_call([hipcc, "--offload-arch=" + B.ARCH, "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
                           "-Xarch_host", "-fsanitize=undefined", "-o", str(lib), str(capi)] + objs)
    script = "LIB = %r\n" % str(lib) + HOST_SCRIPT
    run_child(script, {"LD_PRELOAD": asan, "HIP_VISIBLE_DEVICES": ""}, timeout=600)
