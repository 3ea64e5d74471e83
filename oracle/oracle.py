"""ctypes wrapper of the FP64 CPU oracle (``tfl_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py``.  The product library never imports it.

Arrays are NumPy float64, shape (nz, ny, nx), x fastest, one array per
component.  The oracle's state is the integer-time state (E^n, B^n, Js^n) of
Algorithm 1; B = mu0 H.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# TFL_ORACLE_LIB points the wrapper at another build of the same source (the planted-mistake tests
# build altered copies and run the pins against them)
LIB_PATH = os.environ.get("TFL_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "tfl_oracle.c")
SRC_ADJ_PATH = os.path.join(HERE, "tfl_oracle_adjoint.c")

SRC_SIN, SRC_GAUSS, SRC_MOD_GAUSS = 0, 1, 2


def build(force=True):
    """Compile the oracle with gcc (plain -O2, no FMA contraction, OpenMP)."""
    srcs = [SRC_PATH] + ([SRC_ADJ_PATH] if os.path.exists(SRC_ADJ_PATH) else [])
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           "-o", LIB_PATH] + srcs + ["-lm"]
    subprocess.check_call(cmd)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        D = ctypes.c_double
        I = ctypes.c_int
        Lg = ctypes.c_long
        pl = ctypes.POINTER(ctypes.c_long)
        pd = ctypes.POINTER(ctypes.c_double)
        pi = ctypes.POINTER(ctypes.c_int)
        L.oracle_create.restype = P
        L.oracle_create.argtypes = [pl, pd, D, D, pi, pl, pl, D, D, D, D]
        L.oracle_destroy.argtypes = [P]
        L.oracle_set_materials.argtypes = [P, pd, pd, pd]
        L.oracle_set_fields.argtypes = [P, ctypes.POINTER(pd), ctypes.POINTER(pd), ctypes.POINTER(pd)]
        L.oracle_get_fields.argtypes = [P, ctypes.POINTER(pd), ctypes.POINTER(pd), ctypes.POINTER(pd)]
        L.oracle_get_edge_materials.argtypes = [P, ctypes.POINTER(pd), ctypes.POINTER(pd), ctypes.POINTER(pd)]
        L.oracle_add_source.restype = I
        L.oracle_add_source.argtypes = [P, I, pl, D, I, D, D, D]
        L.oracle_add_probe.restype = I
        L.oracle_add_probe.argtypes = [P, I, pl, Lg, I, pd]
        L.oracle_probe_read.argtypes = [P, I, pd, pd, pd]
        L.oracle_step.argtypes = [P, Lg]
        L.oracle_step_index.restype = Lg
        L.oracle_step_index.argtypes = [P]
        L.oracle_threads.restype = I
        L.oracle_threads.argtypes = []
        L.oracle_energy.restype = D
        L.oracle_energy.argtypes = [P]
        if hasattr(L, "oracle_adjoint"):
            L.oracle_adjoint.restype = I
            L.oracle_adjoint.argtypes = [P, Lg, I, D, pd, pd, pd]
            L.oracle_adjoint_state.restype = I
            L.oracle_adjoint_state.argtypes = [P, Lg, I, D, pd, pd, pd, ctypes.POINTER(pd), ctypes.POINTER(pd),
                                               ctypes.POINTER(pd)]
        _lib = L
    return _lib


def threads():
    """OpenMP threads of the oracle's grid sweeps."""
    return int(lib().oracle_threads())


def _pd(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _arr3(arrs):
    t = ctypes.POINTER(ctypes.c_double) * 3
    return t(*[_pd(a) for a in arrs])


class OracleSim:
    """FP64 CPU oracle run of Algorithm 1 on an nx x ny x nz Yee grid.

    ``pml`` is a 3-tuple of 0/1 per axis; ``npml`` a 3-tuple of (lo, hi) cell
    counts.  Axes without PML are periodic.
    """

    def __init__(self, shape, spacing, dt, theta=1.0, pml=(0, 0, 0), npml=((0, 0), (0, 0), (0, 0)),
                 pml_order=3.0, pml_scale=1.0, kappa_max=1.0, alpha_max=0.0):
        self.nx, self.ny, self.nz = (int(v) for v in shape)
        self.shape3 = (self.nz, self.ny, self.nx)
        self.spacing = tuple(float(v) for v in spacing)
        self.dt = float(dt)
        self.theta = float(theta)
        L = lib()
        n = (ctypes.c_long * 3)(self.nx, self.ny, self.nz)
        d = (ctypes.c_double * 3)(*self.spacing)
        p = (ctypes.c_int * 3)(*[int(v) for v in pml])
        lo = (ctypes.c_long * 3)(*[int(v[0]) for v in npml])
        hi = (ctypes.c_long * 3)(*[int(v[1]) for v in npml])
        self._h = L.oracle_create(n, d, self.dt, self.theta, p, lo, hi,
                                  float(pml_order), float(pml_scale), float(kappa_max), float(alpha_max))
        self._probes = []

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().oracle_destroy(h)
            self._h = None

    def _c(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        assert a.shape == self.shape3, (a.shape, self.shape3)
        return a

    def set_materials(self, eps_r, sigma, ell):
        e, s, l = self._c(eps_r), self._c(sigma), self._c(ell)
        lib().oracle_set_materials(self._h, _pd(e), _pd(s), _pd(l))

    def set_fields(self, E, B, J=None):
        E = [self._c(a) for a in E]
        B = [self._c(a) for a in B]
        J = [self._c(a) for a in J] if J is not None else [np.zeros(self.shape3) for _ in range(3)]
        lib().oracle_set_fields(self._h, _arr3(E), _arr3(B), _arr3(J))

    def get_fields(self):
        E = [np.empty(self.shape3) for _ in range(3)]
        B = [np.empty(self.shape3) for _ in range(3)]
        J = [np.empty(self.shape3) for _ in range(3)]
        lib().oracle_get_fields(self._h, _arr3(E), _arr3(B), _arr3(J))
        return E, B, J

    def edge_materials(self):
        e = [np.empty(self.shape3) for _ in range(3)]
        s = [np.empty(self.shape3) for _ in range(3)]
        l = [np.empty(self.shape3) for _ in range(3)]
        lib().oracle_get_edge_materials(self._h, _arr3(e), _arr3(s), _arr3(l))
        return e, s, l

    def add_source(self, comp, box, amp, kind, f=0.0, t0=0.0, tw=1.0):
        b = (ctypes.c_long * 6)(*[int(v) for v in box])
        return lib().oracle_add_source(self._h, int(comp), b, float(amp), int(kind), float(f), float(t0), float(tw))

    def add_probe(self, comp, box, cap, freqs=()):
        b = (ctypes.c_long * 6)(*[int(v) for v in box])
        fr = np.ascontiguousarray(np.asarray(freqs, dtype=np.float64).reshape(-1))
        pid = lib().oracle_add_probe(self._h, int(comp), b, int(cap), int(fr.size), _pd(fr) if fr.size else None)
        self._probes.append((int(cap), int(fr.size)))
        return pid

    def probe(self, pid):
        cap, nf = self._probes[pid]
        s = np.empty(max(cap, 1))
        re = np.empty(max(nf, 1))
        im = np.empty(max(nf, 1))
        lib().oracle_probe_read(self._h, int(pid), _pd(s), _pd(re), _pd(im))
        return s[:cap], (re + 1j * im)[:nf]

    def step(self, n):
        lib().oracle_step(self._h, int(n))

    @property
    def step_index(self):
        return lib().oracle_step_index(self._h)

    def energy(self):
        return lib().oracle_energy(self._h)

    def adjoint(self, nsteps, pid, f0):
        """Run nsteps forward from the current state and return (J, F, dJ/d ell, dJ/d sigma) for
        J = |sum_n dt exp(-i 2 pi f0 n dt) s_n|^2 of probe `pid` (per-cell FP64 gradients)."""
        gl = np.zeros(self.shape3)
        gs = np.zeros(self.shape3)
        out = np.zeros(3)
        rc = lib().oracle_adjoint(self._h, int(nsteps), int(pid), float(f0), _pd(gl), _pd(gs), _pd(out))
        if rc != 0:
            raise ValueError("oracle_adjoint: bad arguments")
        return out[0], out[1] + 1j * out[2], gl, gs

    def adjoint_state(self, nsteps, pid, f0):
        """adjoint() plus the adjoint of the state the run started from: (J, F, dJ/d ell, dJ/d sigma,
        dJ/dE^0, dJ/dB^0, dJ/dJs^0), the last three as lists of three arrays (PML variables held fixed)."""
        gl = np.zeros(self.shape3)
        gs = np.zeros(self.shape3)
        out = np.zeros(3)
        aE, aB, aJ = ([np.zeros(self.shape3) for _ in range(3)] for _ in range(3))
        rc = lib().oracle_adjoint_state(self._h, int(nsteps), int(pid), float(f0), _pd(gl), _pd(gs), _pd(out),
                                        _arr3(aE), _arr3(aB), _arr3(aJ))
        if rc != 0:
            raise ValueError("oracle_adjoint: bad arguments")
        return out[0], out[1] + 1j * out[2], gl, gs, aE, aB, aJ
