"""The paper's cylinder tunnel (Sec. 4.6: the quintic spline at h = 1.2 dx, a
body filled with rings, 6 layers of inlet, outlet and slip-wall particles;
97k particles at dx = 0.1) through the HIP path against the FP64 oracle.

* One right-hand side on jittered positions with seeded fields: FP64 within
  1e-12 and FP32 within 1e-5 of the per-field scale max_i sum_j |t_ij| (the
  pair sums) or of max |reference| (densities, boundary values, the body
  force); the FP32 pair sums are also reported against max |reference|.
* A 150-step FP64 trajectory from the tunnel's initial state (fluid at rest
  against the body, the inlet at U), with and without the cell order kept
  between sorts: the same particles, kinds and ring heads, fields within 20
  times the oracle's own sensitivity to a one-ulp change of the positions
  (floor 1e-10), and the drag history to the same bar.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1907_04034_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MOVING = (I.FLUID, I.INLET, I.OUTLET)


def B():
    from paper_1907_04034_amd import binding
    return binding


def _match(gs, os_):
    idx = {int(v): k for k, v in enumerate(os_["id"])}
    return np.array([idx[int(v)] for v in gs["id"]])


def _nerr(got, ref, floor=0.0):
    scale = max(np.abs(ref).max() if ref.size else 0.0, floor, 1e-300)
    return np.abs(got - ref).max() / scale if ref.size else 0.0


def _by_id(st):
    """Live rows sorted by id. Rows a step's end deleted stay in the device
    state, of kind DEAD, until the next bin drops them; they are not
    particles."""
    live = np.flatnonzero(st["type"] != I.DEAD)
    idx = live[np.argsort(st["id"][live])]
    return {k: v[idx] for k, v in st.items()}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_cylinder_tunnel_rhs(prec):
    prm, s = I.cylinder_tunnel(dx=0.1)
    s = I.random_fields(prm, I.jitter(prm, s, 0.1, 3, types=MOVING), 4)
    print(f"cylinder tunnel rhs {prec} n={len(s['p'])}", flush=True)
    gs, gd, sim = B().rhs_once(prm, s, prec=prec)
    assert sim.poll_error() == 0
    os_, od, F = O.rhs_once(prm, s)
    perm = _match(gs, os_)
    t = gs["type"]
    fl = t == I.FLUID
    D = prm["dim"]
    tol = 1e-12 if prec == "fp64" else 1e-5
    e = {}
    for key in ("a", "b"):
        e[key] = _nerr(gd[key][fl, :D], od[key][perm][fl, :D],
                       np.abs(od["abs_" + key][perm][fl]).max())
    e["pdot"] = _nerr(gd["pdot"][fl], od["pdot"][perm][fl], np.abs(od["abs_pdot"][perm][fl]).max())
    e["rho"] = _nerr(gd["rho"], od["rho"][perm])
    e["vol"] = _nerr(gd["vol"], od["vol"][perm])
    nf = ~fl
    e["p_bnd"] = _nerr(gs["p"][nf], os_["p"][perm][nf])
    e["u_bnd"] = _nerr(gs["u"][nf, :D], os_["u"][perm][nf, :D])
    io = (t == I.INLET) | (t == I.OUTLET)
    assert np.array_equal(gd["red"][io], od["red"][perm][io])
    e["jcur"] = _nerr(gd["jcur"][io], od["jcur"][perm][io])
    body = t == I.BODY
    assert body.sum() == 314
    e["force"] = _nerr(gd["force"][body, :D], od["force"][perm][body, :D])
    e["drag"] = np.abs(gd["drag"] - F).max() / np.abs(F).max()
    # the pair sums against their own largest value (a stricter scale where
    # the sums cancel), reported
    rel = {k: _nerr(gd[k][fl, :D], od[k][perm][fl, :D]) for k in ("a", "b")}
    rel["pdot"] = _nerr(gd["pdot"][fl], od["pdot"][perm][fl])
    print("  errors:", {k: f"{v:.2e}" for k, v in e.items()}, flush=True)
    print("  pair sums / max |reference|:", {k: f"{v:.2e}" for k, v in rel.items()}, flush=True)
    for key, v in e.items():
        assert v <= tol, (key, v)


def _oracle_run(prm, s, steps):
    o = O.Oracle(prm, s)
    drag = o.step(steps)
    return _by_id(o.state()), drag


def _errors(prm, a, b):
    D = prm["dim"]
    out = {}
    for key, vec in (("x", True), ("u", True), ("p", False), ("avg", False), ("jprev", False)):
        x, y = (a[key][:, :D], b[key][:, :D]) if vec else (a[key], b[key])
        out[key] = _nerr(x, y)
    return out


@pytest.mark.parametrize("reuse", [False, True])
def test_cylinder_tunnel_trajectory_fp64(reuse):
    steps = 150
    prm, s = I.cylinder_tunnel(dx=0.1)
    if reuse:
        prm = dict(prm, flags=prm["flags"] | I.FLAG_REUSE_BINS)
    print(f"cylinder tunnel trajectory fp64 {steps} steps reuse={reuse}", flush=True)
    sim = B().Simulation(prm, s)
    drag = torch.zeros((steps, 3), dtype=torch.float64, device="cuda")
    sim.step(steps, drag_hist=drag)
    assert sim.poll_error() == 0
    gs = _by_id(sim.state())
    g_drag = drag.cpu().numpy()
    ref, ref_drag = _oracle_run(prm, s, steps)
    for key in ("id", "type", "head", "red_prev"):
        assert np.array_equal(gs[key], ref[key]), key
    s2 = I.snapshot_copy(s)
    s2["x"][:, :prm["dim"]] *= 1.0 + 2.0 ** -52
    pert, pdrag = _oracle_run(prm, s2, steps)
    sens = _errors(prm, pert, ref)
    dsens = np.abs(pdrag - ref_drag).max() / np.abs(ref_drag).max()
    err = _errors(prm, gs, ref)
    derr = np.abs(g_drag - ref_drag).max() / np.abs(ref_drag).max()
    print(f"  errors {err}\n  oracle one-ulp sensitivity {sens}\n  drag {derr:.2e} "
          f"(sensitivity {dsens:.2e}); c_d at the last step "
          f"{ref_drag[-1, 0] / (0.5 * prm['rho0'] * prm['U'] ** 2 * 2.0):.4f}", flush=True)
    for key in err:
        assert err[key] <= max(1e-10, 20 * sens[key]), (key, err[key], sens[key])
    assert derr <= max(1e-10, 20 * dsens), (derr, dsens)
