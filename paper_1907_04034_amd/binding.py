"""ctypes binding of libsph (the C ABI in include/sph.h).

Argument marshalling only: device memory comes from torch tensors, the stream
is torch's current HIP stream, and every step of the path runs in libsph's HIP
kernels. Importing this module does not touch the GPU; loading fails loudly
if libsph.so has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsph.so")

FP64, FP32 = 0, 1
FLUID, INLET, OUTLET, WALL_SLIP, WALL_NOSLIP, BODY, DEAD = 0, 1, 2, 3, 4, 5, 255
ERR_BITS = {1: "NBR_OVERFLOW", 2: "CAPACITY", 4: "NONFINITE", 8: "SKIN", 16: "ESCAPE",
            32: "CELL_RANGE", 64: "NNZ_CAPACITY"}

EXPORTED = ["sph_workspace_size", "sph_workspace_bytes", "sph_default_maxnb", "sph_bin",
            "sph_neighbors", "sph_neighbor_table", "sph_get_cells", "sph_cell_key",
            "sph_density", "sph_outlet_extrapolate", "sph_rhs", "sph_force", "sph_step",
            "sph_rhs_adjoint", "sph_outlet_extrapolate_adjoint", "sph_step_record", "sph_step_adjoint_scratch_size",
            "sph_step_adjoint", "sph_step_record_store", "sph_step_adjoint_stored",
            "sph_inlet_profile_grad", "sph_poll_error", "sph_live_count", "sph_last_error",
            "sph_step_static", "sph_launch_config"]
EV_PUSH, EV_TO_OUTLET, EV_DELETE, EV_SPAWN = 1, 2, 4, 8
FLAG_REUSE_BINS = 8


class SphParams(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("n_avg", C.c_int32), ("flags", C.c_int32),
        ("periodic", C.c_int32 * 3),
        ("h", C.c_double), ("dx", C.c_double), ("rho0", C.c_double), ("c", C.c_double),
        ("U", C.c_double), ("nu", C.c_double), ("alpha", C.c_double), ("eta", C.c_double),
        ("dt", C.c_double), ("pb", C.c_double),
        ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("x_inlet", C.c_double), ("x_outlet", C.c_double), ("x_outlet_end", C.c_double),
        ("inlet_len", C.c_double), ("noise_amp", C.c_double), ("noise_seed", C.c_uint64),
        ("group_force", C.c_int32), ("group_nbr", C.c_int32),
        ("list_cap", C.c_int32), ("outlet", C.c_int32),
    ]


_P = C.c_void_p


class SphLaunchInfo(C.Structure):
    _fields_ = [("cells", C.c_int32 * 3), ("tiles", C.c_int32), ("tile_cells", C.c_int32 * 3),
                ("halo_cells", C.c_int32), ("group_force", C.c_int32),
                ("group_search", C.c_int32), ("lists", C.c_int32)]


class SphState(C.Structure):
    _fields_ = [("cap", C.c_int64), ("prec", C.c_int32), ("dim", C.c_int32), ("n", _P),
                ("x", _P), ("u", _P), ("ut", _P), ("p", _P), ("uin", _P), ("ring", _P),
                ("head", _P), ("avg", _P), ("jprev", _P), ("red_prev", _P), ("type", _P),
                ("id", _P)]


class SphNlist(C.Structure):
    _fields_ = [("maxnb", C.c_int32), ("count", _P), ("nbr", _P)]


class SphCsr(C.Structure):
    _fields_ = [("row_ptr", _P), ("col", _P), ("cap_nnz", C.c_int64), ("nnz_out", _P)]


class SphCells(C.Structure):
    _fields_ = [("ncell", C.c_int32 * 3), ("cs", C.c_double * 3), ("nkeys", C.c_int64),
                ("cell_start", _P), ("key", _P)]


class SphAdjoint(C.Structure):
    _fields_ = [("abar", _P), ("bbar", _P), ("pdbar", _P), ("pseed", _P), ("useed", _P),
                ("jseed", _P), ("fbar", C.c_double * 3),
                ("xbar", _P), ("ubar", _P), ("utbar", _P), ("pbar", _P), ("uinbar", _P),
                ("avgbar", _P), ("jprevbar", _P), ("scratch", _P)]


class SphStateAdjoint(C.Structure):
    _fields_ = [("cap", C.c_int64), ("x", _P), ("u", _P), ("ut", _P), ("p", _P), ("uin", _P),
                ("ring", _P), ("avg", _P), ("jprev", _P)]


class SphDerived(C.Structure):
    _fields_ = [("rho", _P), ("vol", _P), ("pavg", _P), ("a", _P), ("b", _P), ("pdot", _P),
                ("jcur", _P), ("red", _P), ("force", _P), ("drag", _P), ("sfl", _P)]


class SphStepStore(C.Structure):
    _fields_ = [("start", SphState), ("perm", _P), ("cell", _P), ("nl1", SphNlist),
                ("nl2", SphNlist), ("d1", SphDerived), ("d2", SphDerived), ("half_x", _P),
                ("half_u", _P), ("half_ut", _P), ("half_p", _P), ("off1", _P), ("off2", _P)]


_lib = None


def lib():
    """Load libsph.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is None:
        # torch brings its own HIP runtime: it must be the process's runtime
        # before libsph.so binds to one, or the library's launches and torch's
        # device memory would belong to different runtimes
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libsph.so not built ({LIB_PATH}); run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        SP, ST, NL, DE = (C.POINTER(SphParams), C.POINTER(SphState), C.POINTER(SphNlist),
                          C.POINTER(SphDerived))
        sz = C.c_size_t
        L.sph_workspace_size.argtypes = [SP, C.c_int64, C.POINTER(C.c_size_t)]
        L.sph_default_maxnb.argtypes = [SP]
        L.sph_default_maxnb.restype = C.c_int32
        L.sph_bin.argtypes = [SP, ST, ST, _P, sz, _P]
        L.sph_workspace_bytes.argtypes = [SP, C.c_int64]
        L.sph_workspace_bytes.restype = C.c_size_t
        L.sph_neighbors.argtypes = [SP, ST, C.POINTER(SphCsr), _P, sz, _P]
        L.sph_neighbor_table.argtypes = [SP, ST, NL, DE, _P, sz, _P]
        L.sph_get_cells.argtypes = [SP, ST, C.POINTER(SphCells), _P, sz, _P]
        L.sph_cell_key.argtypes = [SP, C.c_int64, C.c_int32, C.c_int32, C.c_int32]
        L.sph_cell_key.restype = C.c_int64
        L.sph_density.argtypes = [SP, ST, NL, DE, _P, sz, _P]
        L.sph_outlet_extrapolate.argtypes = [SP, ST, NL, DE, _P, sz, _P]
        L.sph_rhs.argtypes = [SP, ST, NL, DE, _P, sz, _P]
        L.sph_force.argtypes = [SP, ST, NL, DE, _P, sz, _P]
        L.sph_step.argtypes = [SP, ST, ST, NL, DE, C.c_int32, _P, _P, sz, _P]
        L.sph_step_static.argtypes = [SP, ST, ST, NL, DE, C.c_int32, _P, _P, _P]
        L.sph_launch_config.argtypes = [SP, C.c_int64, C.c_int32, C.POINTER(SphLaunchInfo)]
        L.sph_rhs_adjoint.argtypes = [SP, ST, NL, DE, C.POINTER(SphAdjoint), _P, sz, _P]
        L.sph_outlet_extrapolate_adjoint.argtypes = L.sph_rhs_adjoint.argtypes
        LA = C.POINTER(SphStateAdjoint)
        L.sph_step_record.argtypes = [SP, ST, ST, NL, DE, _P, _P, _P, _P, sz, _P]
        L.sph_step_adjoint_scratch_size.argtypes = [SP, C.c_int64, C.POINTER(C.c_size_t)]
        L.sph_step_adjoint.argtypes = [SP, ST, ST, _P, _P, NL, NL, DE, DE,
                                       C.POINTER(C.c_double * 3), LA, LA, _P, sz, _P, sz, _P]
        SS = C.POINTER(SphStepStore)
        L.sph_step_record_store.argtypes = [SP, ST, ST, SS, C.c_int32, _P, _P, _P, _P, sz, _P]
        L.sph_step_adjoint_stored.argtypes = [SP, ST, SS, _P, _P, C.POINTER(C.c_double * 3), LA,
                                              LA, _P, sz, _P, sz, _P]
        L.sph_inlet_profile_grad.argtypes = [SP, ST, LA, _P, C.c_int32, _P, _P]
        L.sph_poll_error.argtypes = [_P, sz, C.POINTER(C.c_uint32), _P]
        L.sph_live_count.argtypes = [ST, C.POINTER(C.c_int64), _P]
        L.sph_last_error.restype = C.c_char_p
        for name in EXPORTED:
            if name != "sph_default_maxnb" and name != "sph_last_error":
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


class SphError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        raise SphError(f"{what} failed ({rc}): {lib().sph_last_error().decode()}")


def make_params(prm):
    q = SphParams()
    q.dim, q.n_avg, q.flags = int(prm["dim"]), int(prm["n_avg"]), int(prm["flags"])
    for d in range(3):
        q.periodic[d] = int(prm["periodic"][d])
        q.lo[d] = float(prm["lo"][d])
        q.hi[d] = float(prm["hi"][d])
    for k in ("h", "dx", "rho0", "c", "U", "nu", "alpha", "eta", "dt", "pb", "x_inlet",
              "x_outlet", "x_outlet_end", "inlet_len", "noise_amp"):
        setattr(q, k, float(prm[k]))
    q.noise_seed = int(prm["noise_seed"])
    q.group_force = int(prm.get("group_force", 0))
    q.group_nbr = int(prm.get("group_nbr", 0))
    q.list_cap = int(prm.get("list_cap", 0))
    q.outlet = int(prm.get("outlet", 0))
    return q


def launch_config(prm, cap, prec="fp64"):
    """The launch configuration the library derives (dict; no GPU needed)."""
    q = make_params(prm)
    out = SphLaunchInfo()
    _check(lib().sph_launch_config(C.byref(q), int(cap), FP64 if prec == "fp64" else FP32,
                                   C.byref(out)), "sph_launch_config")
    return dict(cells=tuple(out.cells), tiles=bool(out.tiles), tile_cells=tuple(out.tile_cells),
                halo_cells=out.halo_cells, group_force=out.group_force,
                group_search=out.group_search, lists=bool(out.lists))


def workspace_size(prm, cap):
    q = make_params(prm)
    out = C.c_size_t(0)
    _check(lib().sph_workspace_size(C.byref(q), int(cap), C.byref(out)), "sph_workspace_size")
    return out.value


class Simulation:
    """Particle state, neighbour table, derived fields and workspace on one GPU.

    `state` is the host exchange format of the input generators (a dict of
    numpy arrays, one row per particle); rows are re-ordered on the device by
    every bin, so results are matched by id.
    """

    def __init__(self, prm, state, prec="fp64", cap=None, maxnb=None, device="cuda"):
        import torch
        self.torch = torch
        self.prm = dict(prm)
        self.q = make_params(prm)
        self.dim = int(prm["dim"])
        self.prec = FP64 if prec == "fp64" else FP32
        self.rdt = torch.float64 if self.prec == FP64 else torch.float32
        self.dev = torch.device(device)
        n = len(state["p"])
        self.cap = int(cap) if cap else int(n * 1.25) + 256
        if n > self.cap:
            raise SphError("state larger than capacity")
        self.maxnb = int(maxnb) if maxnb else int(lib().sph_default_maxnb(C.byref(self.q)))
        self.n_dev = torch.zeros(1, dtype=torch.int64, device=self.dev)
        self.bufs = [self._alloc() for _ in range(2)]
        self.nl_count = torch.zeros(self.cap, dtype=torch.int32, device=self.dev)
        self.nl_nbr = torch.zeros(self.maxnb * self.cap, dtype=torch.int32, device=self.dev)
        cap = self.cap
        self.der = dict(
            rho=torch.zeros(cap, dtype=self.rdt, device=self.dev),
            vol=torch.zeros(cap, dtype=self.rdt, device=self.dev),
            pavg=torch.zeros(cap, dtype=self.rdt, device=self.dev),
            a=torch.zeros(3 * cap, dtype=self.rdt, device=self.dev),
            b=torch.zeros(3 * cap, dtype=self.rdt, device=self.dev),
            pdot=torch.zeros(cap, dtype=self.rdt, device=self.dev),
            jcur=torch.zeros(3 * cap, dtype=torch.float64, device=self.dev),
            red=torch.zeros(cap, dtype=torch.uint8, device=self.dev),
            force=torch.zeros(3 * cap, dtype=torch.float64, device=self.dev),
            drag=torch.zeros(3, dtype=torch.float64, device=self.dev),
            sfl=torch.zeros(cap, dtype=torch.float64, device=self.dev),
        )
        self.ws_bytes = workspace_size(prm, cap)
        self.ws = torch.zeros(self.ws_bytes, dtype=torch.uint8, device=self.dev)
        self._upload(self.bufs[0], state)
        self.st = self._state_struct(self.bufs[0])
        self.alt = self._state_struct(self.bufs[1])
        self.nl = SphNlist(self.maxnb, self.nl_count.data_ptr(), self.nl_nbr.data_ptr())
        d = self.der
        self.out = SphDerived(*[d[k].data_ptr() for k in
                                ("rho", "vol", "pavg", "a", "b", "pdot", "jcur", "red", "force",
                                 "drag", "sfl")])
        self.binned = False

    # ------------------------------------------------------------ memory
    def _alloc(self):
        """One state buffer set: every array is a 256-byte aligned view of one
        device allocation ("_buf"), so a whole state copies in one call."""
        t, cap, D = self.torch, self.cap, self.dim
        f64, rdt, u8, i64 = t.float64, self.rdt, t.uint8, t.int64
        spec = [("x", 3, f64), ("u", 3, rdt), ("ut", 3, rdt), ("p", 1, rdt), ("uin", 3, f64),
                ("ring", 6 * (D + 1), f64), ("head", 1, u8), ("avg", D + 1, f64),
                ("jprev", 3, f64), ("red_prev", 1, u8), ("type", 1, u8), ("id", 1, i64)]
        offs, total = [], 0
        for name, comps, dt in spec:
            nbytes = comps * cap * t.empty((), dtype=dt).element_size()
            offs.append((name, total, nbytes, dt))
            total += (nbytes + 255) // 256 * 256
        buf = t.zeros(total, dtype=u8, device=self.dev)
        out = {name: buf[o:o + nb].view(dt) for name, o, nb, dt in offs}
        out["type"].fill_(DEAD)
        out["_buf"] = buf
        return out

    def _state_struct(self, b):
        return SphState(self.cap, self.prec, self.dim, self.n_dev.data_ptr(),
                        *[b[k].data_ptr() for k in ("x", "u", "ut", "p", "uin", "ring", "head",
                                                    "avg", "jprev", "red_prev", "type", "id")])

    def _upload(self, b, s):
        t, cap, D = self.torch, self.cap, self.dim
        n = len(s["p"])

        def put(name, arr, comps):
            host = np.ascontiguousarray(np.asarray(arr).T if comps > 1 else arr)
            view = b[name].view(comps, cap) if comps > 1 else b[name]
            view[..., :n].copy_(t.from_numpy(host).to(view.dtype))

        put("x", s["x"], 3)
        put("u", s["u"], 3)
        put("ut", s["ut"], 3)
        put("uin", s["uin"], 3)
        put("jprev", s["jprev"], 3)
        put("p", s["p"], 1)
        ring = np.concatenate([s["ring"][:, :, :D], s["ring"][:, :, 3:4]], axis=2)  # n,6,D+1
        b["ring"].view(6, D + 1, cap)[:, :, :n].copy_(
            t.from_numpy(np.ascontiguousarray(ring.transpose(1, 2, 0))))
        avg = np.concatenate([s["avg"][:, :D], s["avg"][:, 3:4]], axis=1)
        b["avg"].view(D + 1, cap)[:, :n].copy_(t.from_numpy(np.ascontiguousarray(avg.T)))
        b["head"][:n].copy_(t.from_numpy(np.asarray(s["head"], np.uint8)))
        b["red_prev"][:n].copy_(t.from_numpy(np.asarray(s["red_prev"], np.uint8)))
        b["type"][:n].copy_(t.from_numpy(np.asarray(s["type"], np.uint8)))
        b["id"][:n].copy_(t.from_numpy(np.asarray(s["id"], np.int64)))
        self.n_dev.fill_(n)

    def _current(self):
        for b in self.bufs:
            if b["x"].data_ptr() == self.st.x:
                return b
        raise SphError("state pointers do not match any buffer set")

    @staticmethod
    def copy_state(dst, src):
        """Device copy of a whole state buffer set (one call)."""
        dst["_buf"].copy_(src["_buf"])

    # ------------------------------------------------------------ calls
    @property
    def stream(self):
        return self.torch.cuda.current_stream(self.dev).cuda_stream

    def _ws(self):
        return self.ws.data_ptr(), self.ws_bytes

    def bin(self):
        ws, nb = self._ws()
        _check(lib().sph_bin(C.byref(self.q), C.byref(self.st), C.byref(self.alt), ws, nb,
                             self.stream), "sph_bin")
        self.binned = True

    def neighbors(self):
        if not self.binned:
            self.bin()
        ws, nb = self._ws()
        _check(lib().sph_neighbor_table(C.byref(self.q), C.byref(self.st), C.byref(self.nl),
                                        C.byref(self.out), ws, nb, self.stream),
               "sph_neighbor_table")

    def cells(self):
        """The cell structure of the last bin (sph_get_cells) as host arrays:
        ncell, cs, nkeys, cell_start [nkeys + 1] and the key of every live
        row."""
        t = self.torch
        out = SphCells()
        ws, nb = self._ws()
        _check(lib().sph_get_cells(C.byref(self.q), C.byref(self.st), C.byref(out), ws, nb,
                                   self.stream), "sph_get_cells")
        cs = t.full((out.nkeys + 1,), -1, dtype=t.int32, device=self.dev)
        key = t.zeros((self.cap,), dtype=t.int32, device=self.dev)
        out.cell_start, out.key = cs.data_ptr(), key.data_ptr()
        _check(lib().sph_get_cells(C.byref(self.q), C.byref(self.st), C.byref(out), ws, nb,
                                   self.stream), "sph_get_cells")
        n = self.live_count()
        return dict(ncell=tuple(out.ncell), cs=tuple(out.cs), nkeys=int(out.nkeys),
                    cell_start=cs.cpu().numpy(), key=key[:n].cpu().numpy().view(np.uint32))

    def neighbors_csr(self, cap_nnz=None):
        """sph_neighbors on the cells of the last bin: row_ptr [n+1] (int64)
        and the first min(nnz, cap_nnz) entries of col (int32) as host arrays,
        the total nnz and the device error bits of the call.
        cap_nnz defaults to the padded table's capacity (cap x maxnb)."""
        if not self.binned:
            self.bin()
        t = self.torch
        if cap_nnz is None:
            cap_nnz = self.cap * self.maxnb
        row_ptr = t.full((self.cap + 1,), -1, dtype=t.int64, device=self.dev)
        col = t.full((max(cap_nnz, 1),), -1, dtype=t.int32, device=self.dev)
        nnz = t.full((1,), -1, dtype=t.int64, device=self.dev)
        csr = SphCsr(row_ptr.data_ptr(), col.data_ptr() if cap_nnz > 0 else None, cap_nnz,
                     nnz.data_ptr())
        ws, nb = self._ws()
        _check(lib().sph_neighbors(C.byref(self.q), C.byref(self.st), C.byref(csr), ws, nb,
                                   self.stream), "sph_neighbors")
        bits = self.poll_error()
        n = self.live_count()
        rp = row_ptr[:n + 1].cpu().numpy()
        total = int(nnz.item())
        return rp, col[:min(total, cap_nnz)].cpu().numpy(), total, bits

    def density(self):
        ws, nb = self._ws()
        _check(lib().sph_density(C.byref(self.q), C.byref(self.st), C.byref(self.nl),
                                 C.byref(self.out), ws, nb, self.stream), "sph_density")

    def outlet_extrapolate(self):
        ws, nb = self._ws()
        _check(lib().sph_outlet_extrapolate(C.byref(self.q), C.byref(self.st), C.byref(self.nl),
                                            C.byref(self.out), ws, nb, self.stream),
               "sph_outlet_extrapolate")

    def rhs(self):
        ws, nb = self._ws()
        _check(lib().sph_rhs(C.byref(self.q), C.byref(self.st), C.byref(self.nl),
                             C.byref(self.out), ws, nb, self.stream), "sph_rhs")

    def force(self, reduce_drag=True):
        ws, nb = self._ws()
        out = self.out
        if not reduce_drag:
            out = SphDerived.from_buffer_copy(self.out)
            out.drag = None
        _check(lib().sph_force(C.byref(self.q), C.byref(self.st), C.byref(self.nl),
                               C.byref(out), ws, nb, self.stream), "sph_force")

    def step(self, nsteps, drag_hist=None):
        """Run nsteps RK2 steps; drag_hist: optional device float64 tensor [nsteps, 3]."""
        ws, nb = self._ws()
        dh = drag_hist.data_ptr() if drag_hist is not None else None
        _check(lib().sph_step(C.byref(self.q), C.byref(self.st), C.byref(self.alt),
                              C.byref(self.nl), C.byref(self.out), int(nsteps), dh, ws, nb,
                              self.stream), "sph_step")
        self.binned = True

    def step_static(self, nsteps, drag_hist=None):
        """sph_step on the library's static scratch (no workspace argument); the
        call's device error bits land in a device word read by static_error()."""
        t = self.torch
        if not hasattr(self, "static_err"):
            self.static_err = t.zeros(1, dtype=t.int32, device=self.dev)
        dh = drag_hist.data_ptr() if drag_hist is not None else None
        _check(lib().sph_step_static(C.byref(self.q), C.byref(self.st), C.byref(self.alt),
                                     C.byref(self.nl), C.byref(self.out), int(nsteps), dh,
                                     self.static_err.data_ptr(), self.stream),
               "sph_step_static")
        self.binned = True

    def static_error(self):
        """Device error bits of the last step_static call (synchronises)."""
        return int(self.static_err.item()) & 0xFFFFFFFF

    def poll_error(self):
        bits = C.c_uint32(0)
        ws, nb = self._ws()
        _check(lib().sph_poll_error(ws, nb, C.byref(bits), self.stream), "sph_poll_error")
        return bits.value

    def live_count(self):
        n = C.c_int64(0)
        _check(lib().sph_live_count(C.byref(self.st), C.byref(n), self.stream), "sph_live_count")
        return n.value

    def outlet_extrapolate_adjoint(self, pseed=None, useed=None, jseed=None):
        """Reverse of the boundary values alone (sph_outlet_extrapolate_adjoint); same
        seeds and outputs as rhs_adjoint."""
        return self.rhs_adjoint(pseed=pseed, useed=useed, jseed=jseed, boundary_only=True)

    def rhs_adjoint(self, abar=None, bbar=None, pdbar=None, fbar=(0.0, 0.0, 0.0), pseed=None,
                    useed=None, jseed=None, boundary_only=False):
        """Gradient of L = sum_fluid(abar.a + bbar.b + pdbar*pdot) + fbar.drag
        + sum_nonfluid(pseed*p + useed.u) + sum_inlet/outlet(jseed.J) for the current
        stage (sph_neighbor_table and sph_rhs must have run). Weights are host arrays in
        the current device row order ((n, 3) or (n,)); returns host gradients in the
        same order (xbar, ubar, utbar, uinbar, jprevbar: (n, 3); pbar: (n,); avgbar:
        (n, 4) with the pressure in the last column)."""
        t, cap, D = self.torch, self.cap, self.dim
        n = self.live_count()
        if not hasattr(self, "adj"):
            z = lambda k: t.zeros(k * cap, dtype=t.float64, device=self.dev)  # noqa: E731
            self.adj = dict(xbar=z(3), ubar=z(3), utbar=z(3), pbar=z(1), uinbar=z(3),
                            avgbar=z(D + 1), jprevbar=z(3), scratch=z(10), pseed=z(1),
                            useed=z(3), jseed=z(3),
                            abar=t.zeros(3 * cap, dtype=self.rdt, device=self.dev),
                            bbar=t.zeros(3 * cap, dtype=self.rdt, device=self.dev),
                            pdbar=t.zeros(cap, dtype=self.rdt, device=self.dev))
        A = self.adj
        for name, w, comps in (("abar", abar, 3), ("bbar", bbar, 3), ("pdbar", pdbar, 1),
                               ("pseed", pseed, 1), ("useed", useed, 3), ("jseed", jseed, 3)):
            A[name].zero_()
            if w is not None:
                w = np.asarray(w, np.float64)
                view = A[name].view(comps, cap) if comps > 1 else A[name]
                host = np.ascontiguousarray(w.T if comps > 1 else w)
                view[..., :n].copy_(t.from_numpy(host).to(view.dtype))
        st = self._adj_struct(fbar)
        self.rhs_adjoint_launch(st, boundary_only)
        out = {}
        for k in ("xbar", "ubar", "utbar", "uinbar", "jprevbar"):
            out[k] = A[k].view(3, cap)[:, :n].cpu().numpy().T.copy()
        out["pbar"] = A["pbar"][:n].cpu().numpy().copy()
        av = A["avgbar"].view(D + 1, cap)[:, :n].cpu().numpy().T
        out["avgbar"] = np.zeros((n, 4))
        out["avgbar"][:, :D] = av[:, :D]
        out["avgbar"][:, 3] = av[:, D]
        return out

    def _adj_struct(self, fbar=(0.0, 0.0, 0.0)):
        A = self.adj
        st = SphAdjoint()
        st.abar, st.bbar, st.pdbar = A["abar"].data_ptr(), A["bbar"].data_ptr(), A["pdbar"].data_ptr()
        for d in range(3):
            st.fbar[d] = float(fbar[d])
        for k in ("pseed", "useed", "jseed", "xbar", "ubar", "utbar", "pbar", "uinbar", "avgbar",
                  "jprevbar", "scratch"):
            setattr(st, k, A[k].data_ptr())
        return st

    def rhs_adjoint_launch(self, st, boundary_only=False):
        """Enqueue sph_rhs_adjoint (or the boundary-values reverse alone) with a
        prepared argument block (weights already on the device); nothing is copied
        back."""
        ws, nb = self._ws()
        fn = lib().sph_outlet_extrapolate_adjoint if boundary_only else lib().sph_rhs_adjoint
        name = "sph_outlet_extrapolate_adjoint" if boundary_only else "sph_rhs_adjoint"
        _check(fn(C.byref(self.q), C.byref(self.st), C.byref(self.nl), C.byref(self.out),
                  C.byref(st), ws, nb, self.stream), name)

    # ------------------------------------------------------------ results
    def state(self):
        """Host copy of the live particles in the exchange format (device order)."""
        n = self.live_count()
        b = self._current()
        cap, D = self.cap, self.dim

        def get(name, comps):
            v = b[name].view(comps, cap)[:, :n] if comps > 1 else b[name][:n]
            a = v.to(self.torch.float64 if v.is_floating_point() else v.dtype).cpu().numpy()
            return a.T.copy() if comps > 1 else a.copy()

        s = dict(x=get("x", 3), u=get("u", 3), ut=get("ut", 3), uin=get("uin", 3),
                 jprev=get("jprev", 3), p=get("p", 1),
                 head=b["head"][:n].cpu().numpy().astype(np.int32),
                 red_prev=b["red_prev"][:n].cpu().numpy(), type=b["type"][:n].cpu().numpy(),
                 id=b["id"][:n].cpu().numpy())
        ring = b["ring"].view(6, D + 1, cap)[:, :, :n].cpu().numpy().transpose(2, 0, 1)
        s["ring"] = np.zeros((n, 6, 4))
        s["ring"][:, :, :D] = ring[:, :, :D]
        s["ring"][:, :, 3] = ring[:, :, D]
        avg = b["avg"].view(D + 1, cap)[:, :n].cpu().numpy().T
        s["avg"] = np.zeros((n, 4))
        s["avg"][:, :D] = avg[:, :D]
        s["avg"][:, 3] = avg[:, D]
        return s

    def derived(self):
        n = self.live_count()
        cap = self.cap
        out = {}
        for k in ("rho", "vol", "pavg", "pdot"):
            out[k] = self.der[k][:n].double().cpu().numpy()
        for k in ("a", "b", "jcur", "force"):
            out[k] = self.der[k].view(3, cap)[:, :n].double().cpu().numpy().T.copy()
        out["red"] = self.der["red"][:n].cpu().numpy()
        out["drag"] = self.der["drag"].cpu().numpy()
        return out

    def neighbor_table(self):
        n = self.live_count()
        cnt = self.nl_count[:n].cpu().numpy()
        nbr = self.nl_nbr.view(self.cap, self.maxnb)[:n].cpu().numpy()
        return cnt, nbr


def rhs_once(prm, state, prec="fp64", **kw):
    """Bin, build the neighbour table and evaluate one right-hand side.
    Returns (state, derived, sim) with rows in the device's sorted order."""
    sim = Simulation(prm, state, prec=prec, **kw)
    sim.bin()
    sim.neighbors()
    sim.rhs()
    return sim.state(), sim.derived(), sim
