"""Discrete adjoint of a run of time steps on the GPU.

The forward run keeps a copy of the state every `segment` steps. The reverse
goes segment by segment from the end: it restores the segment's checkpoint,
replays the segment with sph_step_record_store (keeping the state before every
step, the step's recorded events and its stage values: sorted start state,
tables, derived values, half state), then runs sph_step_adjoint_stored from the
last step of the segment to the first. The replay is bit-identical to the
forward run (deterministic kernels, fixed summation orders), so the reverse
sees the forward's discrete events. With stored=False the tape keeps only the
states and events, and sph_step_adjoint recomputes each step's stage values
(the same result, bit for bit, for about a third more work and a few tens of
MB per step less memory).

Objective used by the wind-tunnel workload with a cylinder: the time-averaged
stage-1 drag J = (1/N) sum_n F_x^n (the force of eq:tvf-momentum_solid on the
body), differentiated with respect to the inlet velocity profile theta (one
value per inlet lattice row).

Argument marshalling and buffer management only: the forward steps, the
replay and every reverse step run in libsph's HIP kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import binding as Bd
from . import inputs as I

_LAM_FIELDS = ("x", "u", "ut", "p", "uin", "ring", "avg", "jprev")


class StepTape:
    """Recording and reverse buffers of one Simulation (FP64 adjoint arrays)."""

    def __init__(self, sim, segment, stored=True):
        t = sim.torch
        self.sim, self.segment, self.stored = sim, int(segment), bool(stored)
        self.stores = []
        cap, D, dev = sim.cap, sim.dim, sim.dev
        self.work = sim._alloc()
        self.work_n = t.zeros(1, dtype=t.int64, device=dev)
        self.work_st = self._struct(self.work, self.work_n)
        self.nl2_count = t.zeros(cap, dtype=t.int32, device=dev)
        self.nl2_nbr = t.zeros(sim.maxnb * cap, dtype=t.int32, device=dev)
        self.nl2 = Bd.SphNlist(sim.maxnb, self.nl2_count.data_ptr(), self.nl2_nbr.data_ptr())
        self.d2 = {k: t.zeros_like(v) for k, v in sim.der.items()}
        self.out2 = Bd.SphDerived(*[self.d2[k].data_ptr() for k in
                                    ("rho", "vol", "pavg", "a", "b", "pdot", "jcur", "red",
                                     "force", "drag", "sfl")])
        nbytes = C.c_size_t(0)
        Bd._check(Bd.lib().sph_step_adjoint_scratch_size(C.byref(sim.q), cap, C.byref(nbytes)),
                  "sph_step_adjoint_scratch_size")
        self.scratch_bytes = nbytes.value
        self.scratch = t.zeros(self.scratch_bytes // 8, dtype=t.float64, device=dev)
        self.lam = [self._lam_alloc(), self._lam_alloc()]
        self.slots, self.slot_n, self.slot_st = [], [], []
        self.child = t.zeros((self.segment, cap), dtype=t.int32, device=dev)
        self.events = t.zeros((self.segment, cap), dtype=t.uint8, device=dev)

    # ------------------------------------------------------------ buffers
    def _struct(self, b, n):
        s = self.sim
        return Bd.SphState(s.cap, s.prec, s.dim, n.data_ptr(),
                           *[b[k].data_ptr() for k in ("x", "u", "ut", "p", "uin", "ring", "head",
                                                       "avg", "jprev", "red_prev", "type", "id")])

    def _lam_alloc(self):
        t, cap, D, dev = self.sim.torch, self.sim.cap, self.sim.dim, self.sim.dev
        comps = dict(x=3, u=3, ut=3, p=1, uin=3, ring=6 * (D + 1), avg=D + 1, jprev=3)
        lam = {k: t.zeros(comps[k] * cap, dtype=t.float64, device=dev) for k in _LAM_FIELDS}
        lam["_s"] = Bd.SphStateAdjoint(cap, *[lam[k].data_ptr() for k in _LAM_FIELDS])
        return lam

    def _slot(self, j):
        while len(self.slots) <= j:
            b = self.sim._alloc()
            n = self.sim.torch.zeros(1, dtype=self.sim.torch.int64, device=self.sim.dev)
            self.slots.append(b)
            self.slot_n.append(n)
            self.slot_st.append(self._struct(b, n))
        return self.slots[j], self.slot_n[j], self.slot_st[j]

    def reserve(self):
        """Allocates the buffers of every slot of a segment up front (state
        copies and, stored, stage values), so that runs allocate nothing."""
        for j in range(self.segment):
            self._slot(j)
            if self.stored:
                self._store(j)

    def _store(self, j):
        """Stage-value buffers of slot j (sph_step_store)."""
        while len(self.stores) <= j:
            self.stores.append(self._store_alloc())
        return self.stores[j]

    def _store_alloc(self):
        s, t = self.sim, self.sim.torch
        cap, dev, rdt = s.cap, s.dev, s.rdt
        i32, f64, f32 = t.int32, t.float64, t.float32
        b = dict(start=s._alloc(), n=t.zeros(1, dtype=t.int64, device=dev),
                 perm=t.zeros(cap, dtype=i32, device=dev), cell=t.zeros(cap, dtype=i32, device=dev),
                 half_x=t.zeros(3 * cap, dtype=f64, device=dev),
                 half_u=t.zeros(3 * cap, dtype=rdt, device=dev),
                 half_ut=t.zeros(3 * cap, dtype=rdt, device=dev),
                 half_p=t.zeros(cap, dtype=rdt, device=dev))
        nls, ders = [], []
        for _ in range(2):
            cnt = t.zeros(cap, dtype=i32, device=dev)
            nbr = t.zeros(s.maxnb * cap, dtype=i32, device=dev)
            nls.append((cnt, nbr, Bd.SphNlist(s.maxnb, cnt.data_ptr(), nbr.data_ptr())))
            # a, b, pdot, force, drag are not read by the reverse: shared
            d = {k: t.zeros_like(s.der[k]) for k in ("rho", "vol", "pavg", "jcur", "red", "sfl")}
            d.update({k: s.der[k] for k in ("a", "b", "pdot", "force", "drag")})
            ders.append((d, Bd.SphDerived(*[d[k].data_ptr() for k in
                                           ("rho", "vol", "pavg", "a", "b", "pdot", "jcur", "red",
                                            "force", "drag", "sfl")])))
        offs = [t.zeros(3 * cap, dtype=f32, device=dev) if s.prec == Bd.FP32 else None
                for _ in range(2)]
        b.update(nls=nls, ders=ders, offs=offs)
        b["_s"] = Bd.SphStepStore(
            self._struct(b["start"], b["n"]), b["perm"].data_ptr(), b["cell"].data_ptr(),
            nls[0][2], nls[1][2], ders[0][1], ders[1][1], b["half_x"].data_ptr(),
            b["half_u"].data_ptr(), b["half_ut"].data_ptr(), b["half_p"].data_ptr(),
            offs[0].data_ptr() if offs[0] is not None else None,
            offs[1].data_ptr() if offs[1] is not None else None)
        return b

    def snapshot(self):
        """Device copy of the simulation's current state."""
        b = self.sim._alloc()
        Bd.Simulation.copy_state(b, self.sim._current())
        return b, self.sim.n_dev.clone()

    def restore(self, snap):
        b, n = snap
        Bd.Simulation.copy_state(self.sim._current(), b)
        self.sim.n_dev.copy_(n)

    # ------------------------------------------------------------ steps
    def record(self, j, drag=None, first=True):
        """Keep the current state in slot j, then one recorded step (first:
        the step starts a run and sorts; otherwise, with the simulation's
        bin-reuse flag, it keeps the cell order while the skin allows)."""
        s = self.sim
        b, n, _ = self._slot(j)
        Bd.Simulation.copy_state(b, s._current())
        n.copy_(s.n_dev)
        ws, nb = s._ws()
        dp = drag.data_ptr() if drag is not None else None
        if self.stored:
            Bd._check(Bd.lib().sph_step_record_store(
                C.byref(s.q), C.byref(s.st), C.byref(s.alt), C.byref(self._store(j)["_s"]),
                1 if first else 0, dp, self.child[j].data_ptr(), self.events[j].data_ptr(), ws,
                nb, s.stream), "sph_step_record_store")
        else:
            Bd._check(Bd.lib().sph_step_record(
                C.byref(s.q), C.byref(s.st), C.byref(s.alt), C.byref(s.nl), C.byref(s.out), dp,
                self.child[j].data_ptr(), self.events[j].data_ptr(), ws, nb, s.stream),
                "sph_step_record")
        s.binned = True

    def reverse(self, j, fbar, lam_next, lam):
        """Adjoint of the state before recorded step j from that after it."""
        s = self.sim
        _, _, st = self._slot(j)
        fb = (C.c_double * 3)(*[float(v) for v in fbar])
        ws, nb = s._ws()
        if self.stored:
            Bd._check(Bd.lib().sph_step_adjoint_stored(
                C.byref(s.q), C.byref(st), C.byref(self._store(j)["_s"]),
                self.child[j].data_ptr(), self.events[j].data_ptr(), C.byref(fb),
                C.byref(lam_next["_s"]), C.byref(lam["_s"]), self.scratch.data_ptr(),
                self.scratch_bytes, ws, nb, s.stream), "sph_step_adjoint_stored")
            return
        Bd._check(Bd.lib().sph_step_adjoint(
            C.byref(s.q), C.byref(st), C.byref(self.work_st), self.child[j].data_ptr(),
            self.events[j].data_ptr(), C.byref(s.nl), C.byref(self.nl2), C.byref(s.out),
            C.byref(self.out2), C.byref(fb), C.byref(lam_next["_s"]), C.byref(lam["_s"]),
            self.scratch.data_ptr(), self.scratch_bytes, ws, nb, s.stream), "sph_step_adjoint")


class DragAdjoint:
    """Per-step stage-1 body force over nsteps steps and its discrete adjoint.

    forward() runs nsteps steps from the simulation's current state (a
    checkpoint every `segment` steps) and returns the drag history, a device
    tensor [nsteps, 3]. backward(fbar) takes the weights of the per-step
    forces ([nsteps, 3]) and returns the adjoint of the initial state: a dict
    of device FP64 tensors in the state's layout ([comp * cap]), rows in the
    initial state's order, plus a final-state adjoint `lam_final` if given.
    """

    def __init__(self, sim, nsteps, segment=50, stored=True, keep_order=None):
        # the replays must match the checkpointed forward row for row: both
        # sort at the first step of every segment and, with stored stage
        # values (keep_order, default), keep the cell order while the skin
        # allows after it; the recomputing reverse needs a sort at every step
        keep_order = stored if keep_order is None else bool(keep_order)
        if keep_order and not stored:
            raise ValueError("keeping the cell order needs stored stage values")
        if keep_order:
            sim.q.flags |= Bd.FLAG_REUSE_BINS
        else:
            sim.q.flags &= ~Bd.FLAG_REUSE_BINS
        self.sim, self.nsteps = sim, int(nsteps)
        self.segment = max(1, min(int(segment), self.nsteps))
        self.tape = StepTape(sim, self.segment, stored=stored)
        self.tape.reserve()
        self.ckpts = []
        self._tape_holds_last = False

    def forward(self):
        """The last segment is recorded as it runs, so the reverse starts
        without a replay (with segment >= nsteps nothing is replayed)."""
        t = self.sim.torch
        hist = t.zeros((self.nsteps, 3), dtype=t.float64, device=self.sim.dev)
        self.ckpts = []
        starts = list(range(0, self.nsteps, self.segment))
        for s0 in starts:
            self.ckpts.append(self.tape.snapshot())
            k = min(self.segment, self.nsteps - s0)
            if s0 == starts[-1]:
                for j in range(k):
                    self.tape.record(j, drag=hist[s0 + j], first=(j == 0))
            else:
                self.sim.step(k, drag_hist=hist[s0:s0 + k])
        self._tape_holds_last = True
        return hist

    def backward(self, fbar, lam_final=None):
        """lam_final: optional callable(ids) -> dict of host arrays, the adjoint of
        the final state for the particles `ids` in that order (x, u, ut, uin, jprev:
        (n, 3); p: (n,); ring: (n, 6, dim+1); avg: (n, dim+1)); it is called with
        the final state's ids in row order (the replay reproduces the forward run
        row for row)."""
        fbar = np.asarray(fbar, np.float64).reshape(self.nsteps, 3)
        tape = self.tape
        nxt, cur = tape.lam
        for k in _LAM_FIELDS:
            nxt[k].zero_()
        last = len(self.ckpts) - 1
        for seg in reversed(range(len(self.ckpts))):
            s0 = seg * self.segment
            k = min(self.segment, self.nsteps - s0)
            if seg != last or not self._tape_holds_last:
                tape.restore(self.ckpts[seg])
                for j in range(k):
                    tape.record(j, first=(j == 0))
            if lam_final is not None and seg == last:
                self._upload_lam(nxt, lam_final)
            for j in reversed(range(k)):
                tape.reverse(j, fbar[s0 + j], nxt, cur)
                nxt, cur = cur, nxt
        self._tape_holds_last = False
        self.lam0 = nxt
        return nxt

    def _upload_lam(self, lam, fn):
        sim = self.sim
        t, cap, D = sim.torch, sim.cap, sim.dim
        n = sim.live_count()
        ids = sim._current()["id"][:n].cpu().numpy()
        host = fn(ids)
        comps = dict(x=3, u=3, ut=3, p=1, uin=3, ring=6 * (D + 1), avg=D + 1, jprev=3)
        for k in _LAM_FIELDS:
            if k not in host:
                continue
            a = np.asarray(host[k], np.float64).reshape(n, comps[k])
            lam[k].view(comps[k], cap)[:, :n].copy_(t.from_numpy(np.ascontiguousarray(a.T)))

    def initial_state_struct(self):
        """sph_state of the initial checkpoint (its live count is n_0)."""
        b, n = self.ckpts[0]
        return self.tape._struct(b, n), (b, n)


def lam_to_host(lam, n, dim, cap):
    """Host copy of rows [0, n) of an adjoint state (shapes as for lam_final)."""
    comps = dict(x=3, u=3, ut=3, p=1, uin=3, ring=6 * (dim + 1), avg=dim + 1, jprev=3)
    out = {}
    for k in _LAM_FIELDS:
        a = lam[k].view(comps[k], cap)[:, :n].cpu().numpy().T.copy()
        out[k] = a[:, 0] if comps[k] == 1 else a
    out["ring"] = out["ring"].reshape(n, 6, dim + 1)
    return out


class InletProfileDrag:
    """J(theta) = (1/nsteps) sum_n F_x^n for an inlet velocity profile theta
    (theta[k] = streamwise velocity of inlet lattice row k, also the initial u,
    ut, ring and mean of those particles), and dJ/dtheta by the adjoint."""

    def __init__(self, prm, state, nsteps, segment=50, prec="fp64", cap=None):
        self.prm, self.base, self.nsteps = prm, state, int(nsteps)
        self.segment, self.prec, self.cap = segment, prec, cap
        self.rows = I.inlet_rows(prm, state)
        self.ntheta = int(self.rows.max()) + 1
        self.sim = self.run = None

    def theta0(self):
        return I.inlet_profile(self.prm, self.base, self.rows)

    def forward(self, theta):
        """One forward run at theta: (J, drag history, tape), where the tape
        (the run's Simulation and DragAdjoint) is what gradient() reverses."""
        s = I.set_inlet_profile(self.prm, self.base, self.rows, theta)
        sim = Bd.Simulation(self.prm, s, prec=self.prec, cap=self.cap)
        run = DragAdjoint(sim, self.nsteps, self.segment)
        hist = run.forward()
        if sim.poll_error():
            raise Bd.SphError("device error during the forward run")
        return float(hist[:, 0].mean().item()), hist, (sim, run)

    def value(self, theta, keep=True):
        """J(theta) and the drag history; keep=True makes this run the one
        gradient() reverses by default."""
        J, hist, tape = self.forward(theta)
        if keep:
            self.sim, self.run = tape
        return J, hist

    def gradient(self, gJ=1.0, tape=None):
        """gJ dJ/dtheta (device FP64 tensor [ntheta]) for the run of `tape`
        (default: the last value() call that kept its run)."""
        sim, run = tape if tape is not None else (self.sim, self.run)
        t = sim.torch
        fbar = np.zeros((self.nsteps, 3))
        fbar[:, 0] = float(gJ) / self.nsteps
        lam = run.backward(fbar)
        st0, _ = run.initial_state_struct()
        index = t.full((sim.cap,), -1, dtype=t.int32, device=sim.dev)
        index[:len(self.rows)].copy_(t.from_numpy(self.rows.astype(np.int32)))
        grad = t.zeros(self.ntheta, dtype=t.float64, device=sim.dev)
        Bd._check(Bd.lib().sph_inlet_profile_grad(
            C.byref(sim.q), C.byref(st0), C.byref(lam["_s"]), index.data_ptr(), self.ntheta,
            grad.data_ptr(), sim.stream), "sph_inlet_profile_grad")
        if sim.poll_error():
            raise Bd.SphError("device error during the reverse run")
        return grad


def inlet_drag_objective():
    """torch.autograd.Function computing J(theta) with the adjoint as backward."""
    import torch

    class InletDragObjective(torch.autograd.Function):
        # each application keeps its own forward run (Simulation and tape) in
        # ctx, so several evaluations may precede their backward passes; the
        # run is released after its backward
        @staticmethod
        def forward(ctx, theta, problem):
            J, _, tape = problem.forward(theta.detach().cpu().numpy())
            ctx.problem, ctx.tape = problem, tape
            return theta.new_tensor(J)

        @staticmethod
        def backward(ctx, gJ):
            if ctx.tape is None:
                raise RuntimeError("InletDragObjective: backward called twice for one forward")
            g = ctx.problem.gradient(float(gJ), tape=ctx.tape)
            ctx.tape = None
            return g.to(gJ.device, gJ.dtype), None

    return InletDragObjective
