"""ctypes wrapper of the FP64 CPU oracle (sph_oracle.c).

TEST INFRASTRUCTURE: imported only by the tests, the smoke check and the
benchmark's CPU-baseline leg. It imports nothing from the HIP package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sph_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-Wall", "-Wextra"]


def build(force=True):
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


class OrcParams(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("n_avg", C.c_int32), ("flags", C.c_int32),
        ("periodic", C.c_int32 * 3),
        ("h", C.c_double), ("dx", C.c_double), ("rho0", C.c_double), ("c", C.c_double),
        ("U", C.c_double), ("nu", C.c_double), ("alpha", C.c_double), ("eta", C.c_double),
        ("dt", C.c_double), ("pb", C.c_double),
        ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("x_inlet", C.c_double), ("x_outlet", C.c_double), ("x_outlet_end", C.c_double),
        ("inlet_len", C.c_double), ("noise_amp", C.c_double), ("noise_seed", C.c_uint64),
        ("outlet", C.c_int32),
    ]


def make_params(prm):
    q = OrcParams()
    q.dim, q.n_avg, q.flags = prm["dim"], prm["n_avg"], prm["flags"]
    for d in range(3):
        q.periodic[d] = int(prm["periodic"][d])
        q.lo[d] = float(prm["lo"][d])
        q.hi[d] = float(prm["hi"][d])
    for k in ("h", "dx", "rho0", "c", "U", "nu", "alpha", "eta", "dt", "pb", "x_inlet",
              "x_outlet", "x_outlet_end", "inlet_len", "noise_amp"):
        setattr(q, k, float(prm[k]))
    q.noise_seed = int(prm["noise_seed"])
    q.outlet = int(prm.get("outlet", 0))
    return q


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.orc_create.restype = P
        L.orc_create.argtypes = [C.POINTER(OrcParams), C.c_int64] + [P] * 12
        L.orc_destroy.argtypes = [P]
        L.orc_count.restype = C.c_int64
        L.orc_count.argtypes = [P]
        L.orc_get.argtypes = [P] * 13
        L.orc_get_derived.argtypes = [P] * 10
        L.orc_get_abs.argtypes = [P] * 4
        L.orc_rhs.argtypes = [P, C.c_int, P]
        L.orc_set_uin.argtypes = [P, P]
        L.orc_step.argtypes = [P, C.c_int32, C.c_int, P]
        L.orc_neighbors.restype = C.c_int64
        L.orc_neighbors.argtypes = [P, C.c_int, P, P, C.c_int64]
        L.orc_w.restype = C.c_double
        L.orc_w.argtypes = [C.c_double, C.c_double, C.c_int]
        L.orc_gradw_factor.restype = C.c_double
        L.orc_gradw_factor.argtypes = [C.c_double, C.c_double, C.c_int]
        L.orc_quintic_w.restype = C.c_double
        L.orc_quintic_w.argtypes = [C.c_double, C.c_double, C.c_int]
        L.orc_quintic_gradw_factor.restype = C.c_double
        L.orc_quintic_gradw_factor.argtypes = [C.c_double, C.c_double, C.c_int]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_splitmix_uniform.restype = C.c_double
        L.orc_splitmix_uniform.argtypes = [C.c_uint64, C.c_int64, C.c_int]
        L.orc_inlet_velocity.argtypes = [C.POINTER(OrcParams), C.c_int64, P, P]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


_LAYOUT = [("x", np.float64, 3), ("u", np.float64, 3), ("ut", np.float64, 3),
           ("p", np.float64, None), ("uin", np.float64, 3), ("ring", np.float64, (6, 4)),
           ("head", np.int32, None), ("avg", np.float64, 4), ("jprev", np.float64, 3),
           ("red_prev", np.uint8, None), ("type", np.uint8, None), ("id", np.int64, None)]


def w(r, h, dim):
    return lib().orc_w(r, h, dim)


def gradw_factor(r, h, dim):
    return lib().orc_gradw_factor(r, h, dim)


def quintic_w(r, h, dim):
    return lib().orc_quintic_w(r, h, dim)


def quintic_gradw_factor(r, h, dim):
    return lib().orc_quintic_gradw_factor(r, h, dim)


def splitmix_uniform(seed, pid, k):
    """The k-th uniform in [0, 1) of particle pid under the seeded generator."""
    return lib().orc_splitmix_uniform(int(seed), int(pid), int(k))


def inlet_velocity(prm, pid, parent=(0.0, 0.0, 0.0)):
    """Prescribed velocity of a re-spawned inlet particle with id pid."""
    q = make_params(prm)
    par = np.ascontiguousarray(parent, dtype=np.float64)
    out = np.zeros(3)
    lib().orc_inlet_velocity(C.byref(q), int(pid), _ptr(par), _ptr(out))
    return out


def num_threads():
    return lib().orc_num_threads()


def set_threads(n):
    """OpenMP threads of later oracle calls (results do not depend on it)."""
    lib().orc_set_threads(int(n))


class Oracle:
    """An oracle simulation holding its own copy of a particle set."""

    def __init__(self, prm, state):
        self.prm = prm
        self._q = make_params(prm)
        n = len(state["p"])
        arrs = []
        for k, dt, shp in _LAYOUT:
            a = np.ascontiguousarray(state[k], dtype=dt)
            arrs.append(a)
        self._keep = arrs
        self.h = lib().orc_create(C.byref(self._q), n, *[_ptr(a) for a in arrs])

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    @property
    def n(self):
        return lib().orc_count(self.h)

    def state(self):
        n = self.n
        out = {}
        for k, dt, shp in _LAYOUT:
            shape = (n,) if shp is None else ((n, shp) if isinstance(shp, int) else (n, *shp))
            out[k] = np.zeros(shape, dt)
        lib().orc_get(self.h, *[_ptr(out[k]) for k, _, _ in _LAYOUT])
        return out

    def derived(self):
        n = self.n
        d = dict(rho=np.zeros(n), vol=np.zeros(n), pavg=np.zeros(n), a=np.zeros((n, 3)),
                 b=np.zeros((n, 3)), pdot=np.zeros(n), jcur=np.zeros((n, 3)),
                 red=np.zeros(n, np.uint8), force=np.zeros((n, 3)))
        lib().orc_get_derived(self.h, *[_ptr(d[k]) for k in
                                        ("rho", "vol", "pavg", "a", "b", "pdot", "jcur",
                                         "red", "force")])
        d["abs_a"], d["abs_b"], d["abs_pdot"] = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros(n)
        lib().orc_get_abs(self.h, _ptr(d["abs_a"]), _ptr(d["abs_b"]), _ptr(d["abs_pdot"]))
        return d

    def set_uin(self, uin):
        """Prescribed inlet velocities, one row of 3 per particle in state() order."""
        a = np.ascontiguousarray(uin, dtype=np.float64)
        assert a.shape == (self.n, 3)
        lib().orc_set_uin(self.h, _ptr(a))

    def rhs(self, brute=False):
        F = np.zeros(3)
        lib().orc_rhs(self.h, int(brute), _ptr(F))
        return F

    def step(self, nsteps, brute=False):
        drag = np.zeros((max(nsteps, 1), 3))
        lib().orc_step(self.h, int(nsteps), int(brute), _ptr(drag))
        return drag[:nsteps]

    def neighbors(self, brute=False):
        nnz = lib().orc_neighbors(self.h, int(brute), None, None, 0)
        row = np.zeros(self.n + 1, np.int64)
        col = np.zeros(max(nnz, 1), np.int32)
        lib().orc_neighbors(self.h, int(brute), _ptr(row), _ptr(col), nnz)
        return row, col[:nnz]


def rhs_once(prm, state, brute=False):
    """Evaluate one right-hand side on a copy of `state`; returns (state, derived, F)."""
    o = Oracle(prm, state)
    F = o.rhs(brute=brute)
    return o.state(), o.derived(), F
