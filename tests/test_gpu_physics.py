"""Invariants and physics checks of the HIP path at the workload sizes.

* A uniform channel (no pulse) stays uniform: the inlet, the hybrid outlet,
  transfers and re-spawns must not disturb u = U, p = 0 (all characteristic
  values vanish and the outlet reproduces its averages).
* Momentum: with the neighbour average of eq:pavg off, pair forces are
  antisymmetric and the total momentum rate vanishes to rounding.
* Determinism: two runs agree bit for bit at every lane-group size.
* Acoustic pulse (2D channel, 2000 steps): the outlet reflection
  R = max|p| over probes x in [3.0, 3.5] for t in [0.18, 0.4545] s divided by
  the right-going half amplitude A/2. The window sees only outlet reflections
  (the incident half has passed x = 3.5 by t = 0.16 s; the inlet's reflection of
  the left-going half reaches x = 3 only after t = 0.495 s). The paper gives no
  bound for this configuration, so R is reported (measured 0.0247), checked
  against the oracle's R, and bounded well below a reflecting wall's (R = 1).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1907_04034_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def B():
    from paper_1907_04034_amd import binding
    return binding


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_uniform_channel_stays_uniform(prec, tol):
    print(f"uniform channel {prec}", flush=True)
    prm, s = I.channel(Lx=4.0, Ly=1.0, dx=0.01, name="uniform channel")
    sim = B().Simulation(prm, s, prec=prec)
    sim.step(2000)
    assert sim.poll_error() == 0
    st = sim.state()
    fl = st["type"] == I.FLUID
    dp = np.abs(st["p"][fl]).max()
    du = np.abs(st["u"][fl, 0] - 1.0).max()
    dv = np.abs(st["u"][fl, 1]).max()
    print(f"  max|p| = {dp:.2e}, max|u-1| = {du:.2e}, max|v| = {dv:.2e}", flush=True)
    assert (st["id"] >= I.ID_GENERATION).any()  # inlet particles re-spawned
    assert dp <= tol and du <= tol and dv <= tol


def test_momentum_conservation_without_pavg():
    prm, s = I.config("C1")
    prm = dict(prm, flags=I.FLAG_NO_PAVG)
    s = I.random_fields(prm, I.jitter(prm, s, 0.3, 8), 9)
    gs, gd, sim = B().rhs_once(prm, s)
    assert sim.poll_error() == 0
    m = prm["rho0"] * prm["dx"] ** 2
    for key in ("a", "b"):
        tot = m * gd[key][:, :2].sum(axis=0)
        scale = m * np.abs(gd[key][:, :2]).sum()
        print(f"  sum m {key} = {tot}, scale {scale:.3e}", flush=True)
        assert np.abs(tot).max() <= 1e-13 * scale


@pytest.mark.parametrize("g", [1, 2, 8, 32])
def test_determinism_every_group_size(g):
    prm, s = I.config("C4", small=True)
    prm = dict(prm, group_force=g, group_nbr=g)
    out = []
    for _ in range(2):
        sim = B().Simulation(prm, s)
        drag = torch.zeros((60, 3), dtype=torch.float64, device="cuda")
        sim.step(60, drag_hist=drag)
        st = sim.state()
        out.append(np.concatenate([st["x"].ravel(), st["u"].ravel(), st["p"],
                                   st["id"].astype(np.float64), drag.cpu().numpy().ravel()]))
    assert np.array_equal(out[0], out[1])


def _probe_window(prm):
    dt = prm["dt"]
    first = int(np.ceil(0.18 / dt))
    return first, 2000


def test_pulse_reflection_against_oracle():
    prm, s = I.config("C2")
    first, last = _probe_window(prm)
    amp = 0.5 * 0.1  # right-going half of the A = 0.01 rho0 c U pulse
    print(f"pulse reflection: probe steps {first}..{last}", flush=True)
    sim = B().Simulation(prm, s)
    sim.step(first)
    peak = torch.zeros((), dtype=torch.float64, device="cuda")
    for _ in range(first, last):
        sim.step(1)
        n = sim.live_count()
        b = sim._current()
        x = b["x"][:n]
        p = b["p"][:n]
        typ = b["type"][:n]
        win = (x >= 3.0) & (x <= 3.5) & (typ == I.FLUID)
        peak = torch.maximum(peak, torch.where(win, p.abs(), torch.zeros_like(p)).max())
    assert sim.poll_error() == 0
    R_gpu = float(peak.item()) / amp
    o = O.Oracle(prm, s)
    o.step(first)
    pk = 0.0
    for _ in range(first, last):
        o.step(1)
        st = o.state()
        x = st["x"][:, 0]
        win = (x >= 3.0) & (x <= 3.5) & (st["type"] == I.FLUID)
        if win.any():
            pk = max(pk, float(np.abs(st["p"][win]).max()))
    R_orc = pk / amp
    print(f"  reflection R = {R_gpu:.6f} (GPU), {R_orc:.6f} (oracle)", flush=True)
    # the workload is an exact lattice: pairs at r = 2h switch the neighbour
    # count of eq:pavg on rounding, which both sides resolve in their own
    # summation order, so the two runs differ far above rounding (measured
    # 8e-5 relative in R) while staying the same flow
    assert abs(R_gpu - R_orc) <= 1e-3 * R_orc
    assert R_gpu < 0.5
