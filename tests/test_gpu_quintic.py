"""The paper's own kernel (quintic spline, support 3h, h = 1.2 dx): HIP path
against the oracle, to the same bars as the Wendland C2 runs.

* neighbour sets (|r|^2 < (3h)^2) bitwise equal to the oracle's brute force;
* one right-hand side, FP64 to 1e-12 and FP32 to 1e-5 of the field scale, on
  the small channel, the small 3D duct with no-slip walls, and the full 41k
  particle channel;
* trajectories with the cell order kept between sorts, within 20 times the
  oracle's own one-ulp sensitivity;
* every lane-group size gives the same neighbour tables and right-hand side.
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


def _match(gs, os_):
    idx = {int(v): k for k, v in enumerate(os_["id"])}
    return np.array([idx[int(v)] for v in gs["id"]])


def _nerr(got, ref, floor=0.0):
    scale = max(np.abs(ref).max() if ref.size else 0.0, floor, 1e-300)
    return np.abs(got - ref).max() / scale if ref.size else 0.0


def _case(name, small=True):
    prm, s = I.config(name, small=small)
    s = I.random_fields(prm, I.jitter(prm, s, 0.15, 7), 11)
    return prm, s


@pytest.mark.parametrize("name", ["C2Q", "C5Q"])
def test_quintic_neighbor_sets_bitwise(name):
    print(f"quintic neighbours {name}", flush=True)
    prm, s = _case(name)
    sim = B().Simulation(prm, s)
    sim.bin()
    sim.neighbors()
    assert sim.poll_error() == 0
    gs = sim.state()
    cnt, nbr = sim.neighbor_table()
    o = O.Oracle(prm, s)
    row, col = o.neighbors(brute=True)
    ids = s["id"]
    ref = {int(ids[i]): set(int(v) for v in ids[col[row[i]:row[i + 1]]])
           for i in range(len(row) - 1)}
    gid = gs["id"]
    for r in range(len(gid)):
        assert set(int(v) for v in gid[nbr[r, :cnt[r]]]) == ref[int(gid[r])], int(gid[r])
    assert np.diff(row).max() > 30


def _rhs_errors(prm, s, prec, **kw):
    gs, gd, sim = B().rhs_once(prm, s, prec=prec, **kw)
    assert sim.poll_error() == 0
    os_, od, F = O.rhs_once(prm, s)
    perm = _match(gs, os_)
    t = gs["type"]
    fl = t == I.FLUID
    D = prm["dim"]
    e = {"rho": _nerr(gd["rho"], od["rho"][perm]), "vol": _nerr(gd["vol"], od["vol"][perm])}
    for key in ("a", "b"):
        e[key] = _nerr(gd[key][fl, :D], od[key][perm][fl, :D],
                       np.abs(od["abs_" + key][perm][fl]).max())
    e["pdot"] = _nerr(gd["pdot"][fl], od["pdot"][perm][fl], np.abs(od["abs_pdot"][perm][fl]).max())
    nf = ~fl
    if nf.any():
        e["p_bnd"] = _nerr(gs["p"][nf], os_["p"][perm][nf])
        e["u_bnd"] = _nerr(gs["u"][nf, :D], os_["u"][perm][nf, :D])
    io = (t == I.INLET) | (t == I.OUTLET)
    if io.any():
        assert np.array_equal(gd["red"][io], od["red"][perm][io])
        e["jcur"] = _nerr(gd["jcur"][io], od["jcur"][perm][io])
    return e, gd


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("name", ["C2Q", "C5Q"])
def test_quintic_rhs_parity(name, prec, tol):
    print(f"quintic rhs {name} {prec}", flush=True)
    prm, s = _case(name)
    e, _ = _rhs_errors(prm, s, prec)
    print({k: f"{v:.2e}" for k, v in e.items()}, flush=True)
    for key, v in e.items():
        assert v <= tol, (key, v)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_quintic_full_size_rhs_parity(prec, tol):
    """The 4x1 channel at dx = 0.01 (41k particles, about 40 neighbours each)."""
    print(f"quintic full-size rhs C2Q {prec}", flush=True)
    prm, s = I.config("C2Q")
    s = I.random_fields(prm, I.jitter(prm, s, 0.1, 1), 2)
    e, _ = _rhs_errors(prm, s, prec)
    print({k: f"{v:.2e}" for k, v in e.items()}, flush=True)
    for key, v in e.items():
        assert v <= tol, (key, v)


TRAJ_KEYS = (("x", True), ("u", True), ("p", False), ("avg", False), ("jprev", False))


def _by_id(st):
    """Live rows sorted by id. Rows a step's end deleted stay in the device
    state, of kind DEAD, until the next bin drops them; they are not
    particles."""
    live = np.flatnonzero(st["type"] != I.DEAD)
    idx = live[np.argsort(st["id"][live])]
    return {k: v[idx] for k, v in st.items()}


def _traj_errors(prm, a, b):
    D = prm["dim"]
    return {key: _nerr(a[key][:, :D], b[key][:, :D]) if vec else _nerr(a[key], b[key])
            for key, vec in TRAJ_KEYS}


def _oracle_state(prm, s, steps):
    o = O.Oracle(prm, s)
    o.step(steps)
    return _by_id(o.state())


@pytest.mark.parametrize("name,steps", [("C2Q", 300), ("C5Q", 40)])
def test_quintic_trajectory_parity(name, steps):
    print(f"quintic trajectory {name} {steps}", flush=True)
    prm, s = I.config(name, small=True)
    prm = dict(prm, flags=prm["flags"] | I.FLAG_REUSE_BINS)
    s = I.jitter(prm, s, 1e-3, 5, types=(I.FLUID, I.INLET, I.OUTLET))
    sim = B().Simulation(prm, s)
    sim.step(steps)
    assert sim.poll_error() == 0
    gs = _by_id(sim.state())
    ref = _oracle_state(prm, s, steps)
    assert np.array_equal(gs["id"], ref["id"])
    assert np.array_equal(gs["type"], ref["type"])
    s2 = I.snapshot_copy(s)
    s2["x"][:, :prm["dim"]] *= 1.0 + 2.0 ** -52
    sens = _traj_errors(prm, _oracle_state(prm, s2, steps), ref)
    err = _traj_errors(prm, gs, ref)
    print({k: f"{err[k]:.2e} (sens {sens[k]:.2e})" for k in err}, flush=True)
    for key in err:
        assert err[key] <= max(1e-10, 20 * sens[key]), (key, err[key], sens[key])


@pytest.mark.parametrize("g", [1, 4, 16, 32])
def test_quintic_lane_group_variants(g):
    prm, s = _case("C2Q")
    prm = dict(prm, group_force=g, group_nbr=g)
    e, _ = _rhs_errors(prm, s, "fp64")
    for key, v in e.items():
        assert v <= 1e-12, (g, key, v)
