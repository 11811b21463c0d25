"""ctypes binding of liblbks.so (the C ABI in include/lbks.h).

Argument marshalling only: every step of the relaxation runs in the library's
HIP kernels.  The functions keep the C names (lbks_create, lbks_set_nuclei,
lbks_relax, lbks_energy, lbks_orbitals, ...); `Solver` is a thin owner of one
context.  PyTorch, when present, supplies the stream and the device
allocator; the library never falls back to anything but its own kernels and
raises if it is not built.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import (CFUNCTYPE, POINTER, Structure, c_char_p, c_double, c_int32, c_int64,
                    c_size_t, c_uint64, c_void_p)
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbks.so")

LBKS_OK, LBKS_NOT_CONVERGED = 0, 1
N_VARIANTS = 16           # update-kernel variants (bit 3: 16 bytes of nodes per lane in the population update)
LBKS_E_INVAL, LBKS_E_NOMEM, LBKS_E_HIP, LBKS_E_NUMERIC, LBKS_E_STATE = -1, -2, -3, -4, -5
LBKS_ORTHO_GS, LBKS_ORTHO_W = 0, 1
LBKS_XC_NONE, LBKS_XC_X, LBKS_XC_X_LYPLOCAL, LBKS_XC_X_PZ81, LBKS_XC_B88_LYP = 0, 1, 2, 3, 4
LBKS_XC_B88_LYP_POLARISED = 5
LBKS_FP64, LBKS_FP32_BULK = 0, 1
LBKS_INIT_GAUSS_NOISE, LBKS_INIT_RANDOM_GAUSS, LBKS_INIT_USER = 0, 1, 2
LBKS_SCHEME_POPULATIONS, LBKS_SCHEME_COLLAPSED = 0, 1
LBKS_MAX_ORB = 16


class lbks_params(Structure):
    _fields_ = [("N", c_int32 * 3), ("h", c_double), ("n_orb", c_int32), ("n_elec", c_int32),
                ("omega", c_double), ("D", c_double), ("ortho", c_int32), ("xc", c_int32),
                ("hartree", c_int32), ("poisson_sweeps", c_int32), ("precision", c_int32),
                ("softening", c_double), ("init", c_int32), ("init_sigma", c_double),
                ("init_noise", c_double), ("seed", c_uint64), ("rho_floor", c_double),
                ("scheme", c_int32), ("stop_checks", c_int32), ("deps_tol", c_double),
                ("hermite", c_int32), ("fold", c_int32), ("reserved", c_int32 * 2)]


ALLOC_FN = CFUNCTYPE(c_void_p, c_size_t, c_void_p)
FREE_FN = CFUNCTYPE(None, c_void_p, c_void_p)


class lbks_device(Structure):
    _fields_ = [("stream", c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN), ("user", c_void_p),
                ("device", c_int32), ("reserved", c_int32 * 3)]


class lbks_energies(Structure):
    _fields_ = [("e_total", c_double), ("e_kin", c_double), ("e_ext", c_double),
                ("e_hartree", c_double), ("e_x", c_double), ("e_c", c_double), ("e_nn", c_double),
                ("n_electrons", c_double), ("poisson_residual", c_double),
                ("eps", c_double * LBKS_MAX_ORB), ("steps", c_int64)]

    def as_dict(self, n_orb: int) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "eps"}
        d["eps"] = np.array(self.eps[:n_orb])
        return d


# exported symbol -> (restype, argtypes); the ABI test checks this list against include/lbks.h
SIGNATURES = {
    "lbks_params_default": (c_int32, [POINTER(lbks_params)]),
    "lbks_create": (c_int32, [POINTER(lbks_params), POINTER(lbks_device), POINTER(c_void_p)]),
    "lbks_set_nuclei": (c_int32, [c_void_p, c_int32, POINTER(c_double), POINTER(c_double)]),
    "lbks_relax": (c_int32, [c_void_p, c_int64, c_double, c_int32, POINTER(c_int64)]),
    "lbks_energy": (c_int32, [c_void_p, POINTER(lbks_energies)]),
    "lbks_orbitals": (c_int32, [c_void_p, POINTER(c_double), c_size_t, POINTER(c_double), c_size_t]),
    "lbks_forces": (c_int32, [c_void_p, POINTER(c_double), c_size_t]),
    "lbks_hamiltonian": (c_int32, [c_void_p, POINTER(c_double), c_size_t]),
    "lbks_relax_sequential": (c_int32, [c_void_p, c_int64, c_double, c_double, c_int32, c_int32,
                                        POINTER(c_int64), POINTER(c_int32)]),
    "lbks_cd_start": (c_int32, [c_void_p, c_double, c_int64]),
    "lbks_cd_step": (c_int32, [c_void_p, c_int64]),
    "lbks_cd_energy": (c_int32, [c_void_p, POINTER(lbks_energies)]),
    "lbks_cd_orbitals": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_double), c_size_t]),
    "lbks_cd_stop": (c_int32, [c_void_p]),
    "lbks_destroy": (None, [c_void_p]),
    "lbks_last_error": (c_char_p, [c_void_p]),
    "lbks_set_potential": (c_int32, [c_void_p, POINTER(c_double)]),
    "lbks_set_orbitals": (c_int32, [c_void_p, POINTER(c_double)]),
    "lbks_shape": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32)]),
    "lbks_device_bytes": (c_size_t, [c_void_p]),
    "lbks_estimate_bytes": (c_size_t, [POINTER(lbks_params)]),
    "lbks_set_timing": (c_int32, [c_void_p, c_int32]),
    "lbks_kernel_time": (c_int32, [c_void_p, c_int32, POINTER(c_double), POINTER(c_int64)]),
    "lbks_copy_kernel": (c_int32, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "lbks_set_variant": (c_int32, [c_void_p, c_int32]),
    "lbks_get_variant": (c_int32, [c_void_p]),
    "lbks_get_fold": (c_int32, [c_void_p]),
    "lbks_autotune": (c_int32, [c_void_p, c_int32, c_int32, POINTER(c_int32), POINTER(c_double)]),
    "lbks_batch_create": (c_int32, [POINTER(lbks_device), POINTER(c_void_p)]),
    "lbks_batch_attach": (c_int32, [c_void_p, c_void_p]),
    "lbks_batch_detach": (c_int32, [c_void_p, c_void_p]),
    "lbks_batch_relax": (c_int32, [c_void_p, c_int64, c_double, c_int32, POINTER(c_int32),
                                   POINTER(c_int64)]),
    "lbks_batch_relax_static": (c_int32, [c_void_p, c_int64, c_double, c_int32, POINTER(c_int32),
                                          POINTER(c_int64)]),
    "lbks_batch_size": (c_int32, [c_void_p]),
    "lbks_batch_stream": (c_void_p, [c_void_p]),
    "lbks_batch_destroy": (None, [c_void_p]),
}

_lib = None


def load():
    """Load liblbks.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1507_07666_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class LbksError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbks error {code}: {msg}")
        self.code = code


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(POINTER(c_double))


# ------------------------------------------------------------- thin wrappers

def lbks_params_default() -> lbks_params:
    p = lbks_params()
    load().lbks_params_default(ctypes.byref(p))
    return p


def lbks_create(p: lbks_params, dev: Optional[lbks_device] = None):
    L = load()
    out = c_void_p()
    rc = L.lbks_create(ctypes.byref(p), ctypes.byref(dev) if dev is not None else None, ctypes.byref(out))
    if rc != 0:
        raise LbksError(rc, L.lbks_last_error(None).decode())
    return out


def lbks_last_error(ctx) -> str:
    return load().lbks_last_error(ctx).decode()


def _check(ctx, rc, ok=(0,)):
    if rc not in ok:
        raise LbksError(rc, lbks_last_error(ctx))
    return rc


def lbks_set_nuclei(ctx, Z, R):
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    R = np.ascontiguousarray(R, dtype=np.float64).reshape(-1)
    return _check(ctx, load().lbks_set_nuclei(ctx, len(Z), _dptr(Z), _dptr(R)))


def lbks_set_potential(ctx, v):
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
    return _check(ctx, load().lbks_set_potential(ctx, _dptr(v)))


def lbks_set_orbitals(ctx, psi):
    psi = np.ascontiguousarray(psi, dtype=np.float64).reshape(-1)
    return _check(ctx, load().lbks_set_orbitals(ctx, _dptr(psi)))


def lbks_relax(ctx, max_steps, dE_tol=0.0, check_every=100):
    done = c_int64(0)
    rc = load().lbks_relax(ctx, int(max_steps), float(dE_tol), int(check_every), ctypes.byref(done))
    _check(ctx, rc, ok=(LBKS_OK, LBKS_NOT_CONVERGED))
    return rc, done.value


def lbks_energy(ctx) -> lbks_energies:
    e = lbks_energies()
    _check(ctx, load().lbks_energy(ctx, ctypes.byref(e)))
    return e


def lbks_shape(ctx):
    N = (c_int32 * 3)()
    n = c_int32()
    _check(ctx, load().lbks_shape(ctx, N, ctypes.byref(n)))
    return (N[0], N[1], N[2]), n.value


def lbks_orbitals(ctx, with_rho=True):
    (nx, ny, nz), n = lbks_shape(ctx)
    psi = np.empty((n, nz, ny, nx))
    rho = np.empty((nz, ny, nx)) if with_rho else None
    rc = load().lbks_orbitals(ctx, _dptr(psi), psi.size, _dptr(rho) if with_rho else None,
                              rho.size if with_rho else 0)
    _check(ctx, rc)
    return psi, rho


def lbks_forces(ctx, n_nuc):
    """Forces on the nuclei, [n_nuc][3] hartree/bohr."""
    F = np.zeros((max(int(n_nuc), 1), 3))
    rc = load().lbks_forces(ctx, _dptr(F), 3 * int(n_nuc))
    _check(ctx, rc)
    return F[:n_nuc]


def lbks_hamiltonian(ctx, n_orb):
    """Projected relaxation operator H_jk (n_orb x n_orb, FP64) of the current state."""
    H = np.zeros((int(n_orb), int(n_orb)))
    _check(ctx, load().lbks_hamiltonian(ctx, _dptr(H), H.size))
    return H


def ritz_values(H):
    """Ascending real parts of the eigenvalues of a projected operator."""
    return np.sort(np.linalg.eigvals(np.asarray(H)).real)


def lbks_destroy(ctx):
    if ctx:
        load().lbks_destroy(ctx)


# ------------------------------------------------------------ torch plumbing

def torch_device_binding(device: int = 0, stream=None, use_allocator: bool = True):
    """lbks_device on torch's current stream (or `stream`), with allocations served
    by the PyTorch caching allocator.  Returns (struct, keepalive)."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream(device)
    dev = lbks_device()
    dev.stream = c_void_p(s.cuda_stream)
    dev.device = device
    keep = [s]
    if use_allocator:
        def _alloc(nbytes, user):
            return torch.cuda.caching_allocator_alloc(int(nbytes), device, s)

        def _free(ptr, user):
            torch.cuda.caching_allocator_delete(ptr)

        a, f = ALLOC_FN(_alloc), FREE_FN(_free)
        dev.alloc, dev.free = a, f
        keep += [a, f]
    return dev, keep


def params(N, h, n_orb, n_elec, **kw) -> lbks_params:
    p = lbks_params_default()
    if isinstance(N, int):
        N = (N, N, N)
    p.N[0], p.N[1], p.N[2] = N
    p.h, p.n_orb, p.n_elec = h, n_orb, n_elec
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def params_for(system, **kw) -> lbks_params:
    """Parameters for an inputs.System (grid, spacing, electrons, softening, start)."""
    init = LBKS_INIT_GAUSS_NOISE if system.init == "gauss_noise" else LBKS_INIT_RANDOM_GAUSS
    base = dict(softening=system.softening, init=init, init_sigma=system.init_sigma,
                init_noise=system.init_noise, seed=system.seed)
    base.update(kw)
    return params(tuple(system.dims), system.h, system.n_orb, system.n_elec, **base)


class Solver:
    """One solve context on one GPU."""

    def __init__(self, p: lbks_params, device: int = 0, use_torch: bool = True, stream=None,
                 use_allocator: bool = True):
        self._keep = []
        dev = None
        if use_torch:
            if stream is None:
                # a stream of its own: the caching allocator then tags this context's
                # blocks to the stream its kernels run on, so no block is handed out
                # while work of another stream may still use it
                import torch
                stream = torch.cuda.Stream(device=device)      # default priority
                stream.wait_stream(torch.cuda.current_stream(device))
            dev, self._keep = torch_device_binding(device, stream, use_allocator)
        self.p = p
        self.ctx = lbks_create(p, dev)
        self.n_orb = p.n_orb

    @classmethod
    def for_system(cls, system, set_nuclei=True, **kw):
        use_torch = kw.pop("use_torch", True)
        s = cls(params_for(system, **kw), use_torch=use_torch)
        if set_nuclei:
            s.set_nuclei(system.Z, system.R)
        return s

    def set_nuclei(self, Z, R):
        lbks_set_nuclei(self.ctx, Z, R)
        self.n_nuc = len(Z)

    def set_potential(self, v):
        lbks_set_potential(self.ctx, v)
        self.n_nuc = 0

    def forces(self):
        """Hellmann-Feynman forces on the nuclei of the current state, [n][3]."""
        return lbks_forces(self.ctx, getattr(self, "n_nuc", 0))

    def set_orbitals(self, psi):
        lbks_set_orbitals(self.ctx, psi)

    def relax(self, max_steps, dE_tol=0.0, check_every=100):
        return lbks_relax(self.ctx, max_steps, dE_tol, check_every)

    def energy(self) -> dict:
        return lbks_energy(self.ctx).as_dict(self.n_orb)

    def orbitals(self):
        return lbks_orbitals(self.ctx)

    def relax_sequential(self, max_steps, dE_tol, deps_tol, check_every=50, max_sweeps=20):
        """Sequential Gram-Schmidt order (lbks_relax_sequential): (rc, steps, sweeps)."""
        n = c_int64()
        sw = c_int32()
        rc = load().lbks_relax_sequential(self.ctx, int(max_steps), float(dE_tol), float(deps_tol),
                                          int(check_every), int(max_sweeps), ctypes.byref(n), ctypes.byref(sw))
        _check(self.ctx, rc, ok=(LBKS_OK, LBKS_NOT_CONVERGED))
        return rc, n.value, sw.value

    # -- concurrent dynamics (complex orbitals in real time; lbks_cd_*)
    def cd_start(self, h, restart_every=0):
        """Start concurrent dynamics with time step h (atomic units); every
        restart_every-th step restarts the two-step scheme (0: never)."""
        _check(self.ctx, load().lbks_cd_start(self.ctx, float(h), int(restart_every)))

    def cd_step(self, steps=1):
        _check(self.ctx, load().lbks_cd_step(self.ctx, int(steps)))

    def cd_energy(self) -> dict:
        e = lbks_energies()
        _check(self.ctx, load().lbks_cd_energy(self.ctx, ctypes.byref(e)))
        return e.as_dict(self.n_orb)

    def cd_orbitals(self):
        """psi^n as a complex array [n_orb][z][y][x]."""
        nx, ny, nz = self.p.N[0], self.p.N[1], self.p.N[2]
        re = np.zeros((self.n_orb, nz, ny, nx))
        im = np.zeros_like(re)
        _check(self.ctx, load().lbks_cd_orbitals(self.ctx, _dptr(re), _dptr(im), re.size))
        return re + 1j * im

    def cd_stop(self):
        _check(self.ctx, load().lbks_cd_stop(self.ctx))

    def hamiltonian(self):
        """(H, Ritz values) of the current state: H_jk = <psi_hat_j|K_h psi_hat_k + S_chi(V psi_hat_k)>."""
        H = lbks_hamiltonian(self.ctx, self.n_orb)
        return H, ritz_values(H)

    def device_bytes(self) -> int:
        return load().lbks_device_bytes(self.ctx)

    def set_timing(self, on: bool):
        _check(self.ctx, load().lbks_set_timing(self.ctx, 1 if on else 0))

    def set_variant(self, v: int):
        _check(self.ctx, load().lbks_set_variant(self.ctx, int(v)))

    def variant(self) -> int:
        return load().lbks_get_variant(self.ctx)

    def fold(self) -> int:
        """Bit 0: the overlap totals are summed by the orthonormalisation; bit 1:
        the multipole totals by the ghost-face kernel."""
        return load().lbks_get_fold(self.ctx)

    def autotune(self, reps: int = 5, force: bool = False):
        """Pick the fastest update-kernel variant on the current state; returns
        (variant, per-variant ms or None when the process cache answered)."""
        ch = c_int32()
        ms = (c_double * N_VARIANTS)()
        _check(self.ctx, load().lbks_autotune(self.ctx, int(reps), 1 if force else 0, ctypes.byref(ch), ms))
        times = list(ms)
        if all(t < 0 for t in times):
            return ch.value, None                     # the process cache answered
        return ch.value, [None if t < 0 else t for t in times]

    def kernel_time(self, kernel=0):
        """(summed ms, launches) of the timed launches: kernel 0 = the update kernel,
        1 = the concurrent-dynamics step."""
        ms = c_double()
        n = c_int64()
        _check(self.ctx, load().lbks_kernel_time(self.ctx, int(kernel), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def close(self):
        if self.ctx:
            lbks_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Batch:
    """Many solves advanced together: one launch per kernel per group of alike
    solves, each step captured in a HIP graph (lbks_batch_* in the C ABI)."""

    def __init__(self, device: int = 0, use_torch_allocator: bool = True):
        import torch
        self.device = device
        self.stream = torch.cuda.Stream(device=device)      # default priority
        dev, self._keep = torch_device_binding(device, self.stream, use_torch_allocator)
        self._use_alloc = use_torch_allocator
        out = c_void_p()
        rc = load().lbks_batch_create(ctypes.byref(dev), ctypes.byref(out))
        if rc != 0:
            raise LbksError(rc, "lbks_batch_create failed")
        self.handle = out
        self.solvers = []

    def add(self, p: lbks_params) -> "Solver":
        s = Solver(p, device=self.device, stream=self.stream, use_allocator=self._use_alloc)
        rc = load().lbks_batch_attach(self.handle, s.ctx)
        _check(s.ctx, rc)
        self.solvers.append(s)
        return s

    def add_system(self, system, set_nuclei=True, **kw) -> "Solver":
        s = self.add(params_for(system, **kw))
        if set_nuclei:
            s.set_nuclei(system.Z, system.R)
        return s

    def remove(self, s: "Solver"):
        _check(s.ctx, load().lbks_batch_detach(self.handle, s.ctx))
        self.solvers.remove(s)

    def relax(self, max_steps, dE_tol=0.0, check_every=100, static=False):
        """Advance every member; static=True takes lbks_batch_relax_static (tables in
        the library's fixed device workspace, no allocation, no graphs)."""
        m = len(self.solvers)
        st = (c_int32 * max(1, m))()
        steps = (c_int64 * max(1, m))()
        fn = load().lbks_batch_relax_static if static else load().lbks_batch_relax
        rc = fn(self.handle, int(max_steps), float(dE_tol), int(check_every), st, steps)
        if rc < 0:
            msg = load().lbks_last_error(None)
            raise LbksError(rc, (msg.decode() if msg else "") or "batch relaxation failed")
        return list(st[:m]), list(steps[:m])

    def close(self):
        if getattr(self, "handle", None):
            load().lbks_batch_destroy(self.handle)
            self.handle = None
        for s in self.solvers:
            s.close()
        self.solvers = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
