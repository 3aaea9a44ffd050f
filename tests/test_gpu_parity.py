"""GPU (libsph, FP64) against the CPU oracle on identical seeded inputs.

Neighbour sets must be bitwise equal (matched by particle id). FP64 fields
must agree to 1e-12 of the field's scale: for pair sums (a, b, pdot) the
largest sum of absolute pair contributions max_i sum_j |t_ij| that the oracle
reports (rounding in a sum is bounded relative to that, and fields that cancel
to rounding level on a perfect lattice are not judged against their own
noise); for every other field max|reference|.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1907_04034_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


def B():
    from paper_1907_04034_amd import binding
    return binding


def _match(gs, os_):
    idx = {int(v): k for k, v in enumerate(os_["id"])}
    return np.array([idx[int(v)] for v in gs["id"]])


def _floors(od, sel):
    """Per-field scale max_i sum_j |t_ij| over the selected rows."""
    return dict(a=np.abs(od["abs_a"][sel]).max(), b=np.abs(od["abs_b"][sel]).max(),
                pdot=np.abs(od["abs_pdot"][sel]).max())


def _nerr(got, ref, floor=0.0):
    scale = max(np.abs(ref).max() if ref.size else 0.0, floor, 1e-300)
    return np.abs(got - ref).max() / scale if ref.size else 0.0


def _case(name):
    if name == "C1":
        return I.config("C1")
    if name == "C1-jit":
        prm, s = I.config("C1")
        s = I.random_fields(prm, I.jitter(prm, s, 0.2, 3), 5)
        return prm, s
    if name == "lattice3d":
        prm, s = I.periodic_lattice(n_side=8, dim=3, dx=0.125)
        s = I.random_fields(prm, I.jitter(prm, s, 0.1, 2), 9)
        return prm, s
    cfg, _ = name.split("-", 1)
    prm, s = I.config(cfg, small=True)
    s = I.random_fields(prm, I.jitter(prm, s, 0.15, 7), 11)
    return prm, s


CASES = ["C1", "C1-jit", "lattice3d", "C2-small", "C3-small", "C4-small", "C5-small"]


def _print_case(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("name", CASES)
def test_neighbor_sets_bitwise(name):
    _print_case(f"neighbours {name}")
    prm, s = _case(name)
    sim = B().Simulation(prm, s)
    sim.bin()
    sim.neighbors()
    assert sim.poll_error() == 0
    gs = sim.state()
    cnt, nbr = sim.neighbor_table()
    o = O.Oracle(prm, s)
    row, col = o.neighbors(brute=len(s["p"]) <= 6000)
    ids_o = s["id"]
    ref = {int(ids_o[i]): set(int(v) for v in ids_o[col[row[i]:row[i + 1]]])
           for i in range(len(row) - 1)}
    gid = gs["id"]
    for r in range(len(gid)):
        got = set(int(v) for v in gid[nbr[r, :cnt[r]]])
        assert got == ref[int(gid[r])], (name, int(gid[r]))


@pytest.mark.parametrize("name", CASES)
def test_rhs_parity_fp64(name):
    _print_case(f"rhs fp64 {name}")
    prm, s = _case(name)
    gs, gd, sim = B().rhs_once(prm, s)
    assert sim.poll_error() == 0
    os_, od, F = O.rhs_once(prm, s)
    perm = _match(gs, os_)
    t = gs["type"]
    fl = t == I.FLUID
    D = prm["dim"]
    fl_or_body = fl | (t == I.BODY)
    floors = _floors(od, perm[fl])
    assert _nerr(gd["rho"], od["rho"][perm]) < TOL
    assert _nerr(gd["vol"], od["vol"][perm]) < TOL
    assert _nerr(gd["pavg"][fl_or_body], od["pavg"][perm][fl_or_body]) < TOL
    for key in ("a", "b"):
        e = _nerr(gd[key][fl, :D], od[key][perm][fl, :D], floors[key])
        assert e < TOL, (key, e)
    assert _nerr(gd["pdot"][fl], od["pdot"][perm][fl], floors["pdot"]) < TOL
    nf = ~fl
    if nf.any():
        assert _nerr(gs["p"][nf], os_["p"][perm][nf]) < TOL
        assert _nerr(gs["u"][nf, :D], os_["u"][perm][nf, :D]) < TOL
    io = (t == I.INLET) | (t == I.OUTLET)
    if io.any():
        assert np.array_equal(gd["red"][io], od["red"][perm][io])
        assert _nerr(gd["jcur"][io], od["jcur"][perm][io]) < TOL
    if (t == I.BODY).any():
        assert np.abs(gd["drag"] - F).max() <= TOL * np.abs(F).max()


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
    out = {}
    for key, vec in TRAJ_KEYS:
        x, y = (a[key][:, :D], b[key][:, :D]) if vec else (a[key], b[key])
        out[key] = _nerr(x, y)
    return out


def _oracle_run(prm, s, steps):
    o = O.Oracle(prm, s)
    drag = o.step(steps)
    return _by_id(o.state()), drag


def _ulp_sensitivity(prm, s, steps, ref, ref_drag):
    """Oracle against itself with positions perturbed by one ulp: the scale at
    which the discontinuous neighbour count of eq:pavg amplifies rounding."""
    s2 = I.snapshot_copy(s)
    s2["x"][:, :prm["dim"]] *= 1.0 + 2.0 ** -52
    pert, pdrag = _oracle_run(prm, s2, steps)
    sens = _traj_errors(prm, pert, ref)
    dsens = np.abs(pdrag - ref_drag).max() / max(np.abs(ref_drag).max(), 1e-300)
    return sens, dsens


TRAJ_CASES = [("C1", 100, 0.0), ("C2-small", 300, 1e-3), ("C3-small", 100, 1e-3),
              ("C4-small", 150, 1e-3), ("C5-small", 60, 1e-3)]


@pytest.mark.parametrize("reuse", [False, True])
@pytest.mark.parametrize("name,steps,jit", TRAJ_CASES)
def test_trajectory_parity_fp64(name, steps, jit, reuse):
    """GPU vs oracle after many steps, within a small multiple of the oracle's
    own one-ulp sensitivity (floor 1e-10); also with the cell order kept
    across steps while the skin allows."""
    _print_case(f"trajectory fp64 {name} {steps} reuse={reuse}")
    prm, s = I.config("C1") if name == "C1" else I.config(name.split("-")[0], small=True)
    if reuse:
        prm = dict(prm, flags=prm["flags"] | I.FLAG_REUSE_BINS)
    if jit:
        s = I.jitter(prm, s, jit, 5, types=(I.FLUID, I.INLET, I.OUTLET))
    sim = B().Simulation(prm, s)
    drag = torch.zeros((steps, 3), dtype=torch.float64, device="cuda")
    sim.step(steps, drag_hist=drag)
    assert sim.poll_error() == 0
    gs = _by_id(sim.state())
    ref, ref_drag = _oracle_run(prm, s, steps)
    assert np.array_equal(gs["id"], ref["id"])
    assert np.array_equal(gs["type"], ref["type"])
    assert np.array_equal(gs["head"], ref["head"])
    assert np.array_equal(gs["red_prev"], ref["red_prev"])
    sens, dsens = _ulp_sensitivity(prm, s, steps, ref, ref_drag)
    err = _traj_errors(prm, gs, ref)
    for key in err:
        assert err[key] <= max(1e-10, 20 * sens[key]), (key, err[key], sens[key])
    if (s["type"] == I.BODY).any():
        g = drag.cpu().numpy()
        derr = np.abs(g - ref_drag).max() / np.abs(ref_drag).max()
        assert derr <= max(1e-10, 20 * dsens), (derr, dsens)
    if name == "C2-small":
        assert (gs["id"] >= I.ID_GENERATION).any()  # re-spawns happened


def test_trajectory_exact_lattice_without_pavg():
    """Exact lattice (ties at r = 2h) with the neighbour average off: the
    right-hand side is continuous and GPU and oracle agree to 1e-11."""
    prm, s = I.config("C2", small=True)
    prm = dict(prm, flags=I.FLAG_NO_PAVG)
    sim = B().Simulation(prm, s)
    sim.step(300)
    assert sim.poll_error() == 0
    gs = _by_id(sim.state())
    ref, _ = _oracle_run(prm, s, 300)
    assert np.array_equal(gs["id"], ref["id"])
    err = _traj_errors(prm, gs, ref)
    assert all(v < 1e-11 for v in err.values()), err


def test_determinism_bitwise():
    prm, s = I.config("C2", small=True)
    out = []
    for _ in range(2):
        sim = B().Simulation(prm, s)
        sim.step(80)
        st = sim.state()
        out.append(np.concatenate([st["x"].ravel(), st["u"].ravel(), st["p"],
                                   st["id"].astype(np.float64)]))
    assert np.array_equal(out[0], out[1])


def test_neighbor_overflow_sets_error_bit():
    prm, s = I.config("C1")
    sim = B().Simulation(prm, s, maxnb=4)
    sim.bin()
    sim.neighbors()
    bits = sim.poll_error()
    assert bits & 1
    cnt, _ = sim.neighbor_table()
    assert cnt.max() == 4


@pytest.mark.parametrize("cfg", ["C2", "C3", "C5"])
def test_full_size_rhs_parity(cfg):
    """Full workload size (41k, 1.2M and 4.6M particles), single right-hand
    side, every particle."""
    _print_case(f"full-size rhs {cfg}")
    prm, s = I.config(cfg)
    s = I.random_fields(prm, I.jitter(prm, s, 0.1, 1), 2)
    gs, gd, sim = B().rhs_once(prm, s)
    assert sim.poll_error() == 0
    os_, od, F = O.rhs_once(prm, s)
    perm = _match(gs, os_)
    fl = gs["type"] == I.FLUID
    floors = _floors(od, perm[fl])
    D = prm["dim"]
    assert _nerr(gd["rho"], od["rho"][perm]) < TOL
    for key in ("a", "b"):
        assert _nerr(gd[key][fl, :D], od[key][perm][fl, :D], floors[key]) < TOL
    assert _nerr(gd["pdot"][fl], od["pdot"][perm][fl], floors["pdot"]) < TOL


@pytest.mark.parametrize("g", [1, 2, 4, 8, 16, 32])
@pytest.mark.parametrize("name", ["C2-small", "C5-small"])
def test_lane_group_variants(name, g):
    """Every lanes-per-target variant of the neighbour search and the force
    pass gives the same neighbour sets and FP64 forces (to rounding)."""
    _print_case(f"lane groups {name} g={g}")
    prm, s = _case(name)
    prm = dict(prm, group_force=g, group_nbr=g)
    gs, gd, sim = B().rhs_once(prm, s)
    assert sim.poll_error() == 0
    os_, od, F = O.rhs_once(prm, s)
    perm = _match(gs, os_)
    fl = gs["type"] == I.FLUID
    floors = _floors(od, perm[fl])
    D = prm["dim"]
    for key in ("a", "b"):
        assert _nerr(gd[key][fl, :D], od[key][perm][fl, :D], floors[key]) < TOL
    assert _nerr(gd["pdot"][fl], od["pdot"][perm][fl], floors["pdot"]) < TOL
    cnt, nbr = sim.neighbor_table()
    row, col = O.Oracle(prm, s).neighbors(brute=True)
    ids = s["id"]
    ref = {int(ids[i]): set(ids[col[row[i]:row[i + 1]]].tolist()) for i in range(len(row) - 1)}
    for r in range(len(cnt)):
        assert set(gs["id"][nbr[r, :cnt[r]]].tolist()) == ref[int(gs["id"][r])]


def test_bin_reuse_matches_sorting_every_step():
    """Full 2D channel (jittered), 300 steps: keeping the cell order across
    steps gives the same flow as sorting every step (same neighbour sets; only
    the summation order differs), and the same particles."""
    prm, s = I.config("C2")
    s = I.jitter(prm, s, 1e-3, 5, types=(I.FLUID, I.INLET, I.OUTLET))
    out = []
    for flags in (prm["flags"], prm["flags"] | I.FLAG_REUSE_BINS):
        sim = B().Simulation(dict(prm, flags=flags), s)
        sim.step(300)
        assert sim.poll_error() == 0
        out.append(_by_id(sim.state()))
    assert np.array_equal(out[0]["id"], out[1]["id"])
    assert np.array_equal(out[0]["type"], out[1]["type"])
    err = _traj_errors(prm, out[1], out[0])
    print(err, flush=True)
    assert all(v < 1e-9 for v in err.values()), err


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("tiles", [False, True])
@pytest.mark.parametrize("name,caps", [("C4", (1, 14)), ("C5", (1, 52))])
def test_candidate_lists_match_stencil_search(name, caps, tiles, prec):
    """The step path's searches through stored candidate lists give the same
    neighbour tables, in the same order, as walking the cell stencil: the
    trajectory with the lists (automatic capacity) is bit-identical to one
    where every particle overflows its list (capacity 1: every search walks
    the stencil) and to one where only some do. Both for the gather search
    (lists of rows) and the LDS-tiled one (lists of halo slots), in FP64 and
    FP32."""
    _print_case(f"candidate lists {name} tiles={tiles} {prec}")
    prm, s = I.config(name, small=True)
    s = I.jitter(prm, s, 0.05, 3, types=(I.FLUID, I.INLET, I.OUTLET))
    flags = prm["flags"] | I.FLAG_REUSE_BINS | (I.FLAG_TILES if tiles else 0)
    out = []
    for cap in (0,) + tuple(caps):
        q = dict(prm, flags=flags, list_cap=cap)
        sim = B().Simulation(q, s, prec=prec)
        drag = torch.zeros((80, 3), dtype=torch.float64, device="cuda")
        sim.step(80, drag_hist=drag)
        assert sim.poll_error() == 0
        st = sim.state()
        out.append(np.concatenate([st["x"].ravel(), st["u"].ravel(), st["p"],
                                   st["id"].astype(np.float64), drag.cpu().numpy().ravel()]))
    for o in out[1:]:
        assert np.array_equal(out[0], o)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["C4", "C5"])
def test_empty_state(name, prec):
    """No particles: every entry point runs, finds nothing and raises no
    error bit (the degenerate case of the bin, the searches, the boundary
    values, the force pass and the bookkeeping)."""
    _print_case(f"empty state {name} {prec}")
    prm, s = I.config(name, small=True)
    s0 = {k: v[:0] for k, v in s.items()}
    sim = B().Simulation(prm, s0, prec=prec)
    sim.bin()
    sim.neighbors()
    rp, _, nnz, bits = sim.neighbors_csr()
    assert bits == 0 and nnz == 0 and rp.tolist() == [0]
    sim.rhs()
    drag = torch.zeros((5, 3), dtype=torch.float64, device="cuda")
    sim.step(5, drag_hist=drag)
    assert sim.poll_error() == 0
    assert sim.live_count() == 0
    assert float(drag.abs().max().item()) == 0.0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_capacity_exhausted_sets_error_bit(prec):
    """Capacity equal to the initial count: an inlet re-spawn finds no free
    row, so the step raises SPH_ERR_CAPACITY (bit 2), writes no row past the
    capacity and never counts more live rows than it holds; with room for the
    re-spawns the same run raises nothing."""
    _print_case(f"capacity exhausted C2-small {prec}")
    prm, s = I.config("C2", small=True)
    # without the outermost outlet column the first deletion (step 66 in the
    # oracle) comes well after the first inlet re-spawn (step 23), so no row
    # is freed before the re-spawn needs one
    out = s["type"] == I.OUTLET
    xo = s["x"][:, 0]
    keep = ~(out & (xo > xo[out].max() - 0.5 * prm["dx"]))
    s = {k: v[keep] for k, v in s.items()}
    n = len(s["p"])
    steps = int(np.ceil(prm["dx"] / (prm["U"] * prm["dt"]))) + 5  # 49: one inlet column crosses
    full = B().Simulation(prm, s, prec=prec, cap=n)
    full.step(steps)
    assert full.poll_error() & 2
    assert full.live_count() <= n
    roomy = B().Simulation(prm, s, prec=prec, cap=2 * n)
    roomy.step(steps)
    assert roomy.poll_error() == 0
    assert roomy.live_count() > n  # the re-spawned inlet column


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_nonfinite_value_sets_error_bit(prec):
    """A NaN pressure on one fluid particle: the stage update flags the
    non-finite result (SPH_ERR_NONFINITE, bit 4), and the step completes (NaN
    positions are clamped into a valid cell by the bin, which flags them)."""
    _print_case(f"non-finite pressure C2-small {prec}")
    prm, s = I.config("C2", small=True)
    s = I.snapshot_copy(s)
    fl = np.flatnonzero(s["type"] == I.FLUID)
    s["p"][fl[len(fl) // 2]] = np.nan
    sim = B().Simulation(prm, s, prec=prec)
    sim.step(2)
    assert sim.poll_error() & 4
    clean = B().Simulation(prm, I.config("C2", small=True)[1], prec=prec)
    clean.step(2)
    assert clean.poll_error() == 0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_escaped_particle_sets_error_bit(prec):
    """A fluid particle outside the box along a closed axis (the 3D duct's
    walls): the bin clamps it into the edge cell and raises SPH_ERR_ESCAPE
    (bit 16); the step completes."""
    _print_case(f"escaped particle C5-small {prec}")
    prm, s = I.config("C5", small=True)
    closed = [d for d in range(1, prm["dim"]) if not prm["periodic"][d]]
    assert closed, "the duct's transverse axes are closed"
    d = closed[0]
    s = I.snapshot_copy(s)
    fl = np.flatnonzero(s["type"] == I.FLUID)
    s["x"][fl[len(fl) // 2], d] = prm["hi"][d] + 0.5
    sim = B().Simulation(prm, s, prec=prec)
    sim.step(1)
    assert sim.poll_error() & 16
