"""The LDS-tiled neighbour search and force pass (SPH_FLAG_TILES) against the
gather kernels (the default).

With the same lanes per target, the tiled kernels reproduce the gather
kernels' neighbour table bit for bit (same entries in the same order) and
their densities (summed in table order). The force pass evaluates the same
pair terms in the same order through the same inline functions, but the
compiler may fuse multiplies and adds differently inside the two kernels, so
its outputs agree to rounding (a wrong neighbour or slot would show at the
size of a pair term); so do trajectories over 30 steps. The body-force total
is summed over a different block decomposition. Cases
cover 2D and 3D, both precisions, periodic axes with three cells (a tile's
halo then holds one cell twice), inlet/outlet/wall/body rows, and the small
3D duct, whose halos overflow the LDS capacity in places (those rows are
read from global memory).
"""
import numpy as np
import pytest

from paper_1907_04034_amd import inputs as I


def B():
    from paper_1907_04034_amd import binding
    return binding


def _case(name):
    if name == "lattice2d-nc3":
        prm, s = I.periodic_lattice(n_side=8, dim=2, dx=0.1)
    elif name == "lattice3d":
        prm, s = I.periodic_lattice(n_side=11, dim=3, dx=0.1)
    elif name == "C1":
        prm, s = I.config("C1")
    elif name == "C5-small":
        prm, s = I.config("C5", small=True)
    else:
        prm, s = I.config(name, small=True)
    s = I.random_fields(prm, I.jitter(prm, s, 0.2, 7), 8, p_range=(-0.2, 0.2),
                        u_range=(0.8, 1.2), ut_dev=0.02)
    prm["group_force"], prm["group_nbr"] = 4, 8
    return prm, s


CASES = ["lattice2d-nc3", "lattice3d", "C1", "C2", "C3", "C4", "C5-small"]


@pytest.mark.parametrize("name", CASES)
def test_tiles_are_used(name):
    """The library takes the tiled path on request only (host query, no GPU)."""
    prm, s = _case(name)
    cap = int(len(s["p"]) * 1.25) + 256
    for prec in ("fp64", "fp32"):
        assert not B().launch_config(prm, cap, prec)["tiles"]
        on = dict(prm, flags=prm["flags"] | I.FLAG_TILES)
        assert B().launch_config(on, cap, prec)["tiles"]


def test_tile_shapes_of_the_workloads():
    for name in ("C1", "C2", "C3", "C4", "C5"):
        prm, s = I.config(name)
        prm["flags"] |= I.FLAG_TILES
        cap = int(len(s["p"]) * 1.25) + 256
        cfg = B().launch_config(prm, cap)
        assert cfg["tiles"], name
        assert cfg["tile_cells"][:prm["dim"]] == ((2, 2, 2) if prm["dim"] == 3 else (4, 4))
        assert cfg["halo_cells"] == (64 if prm["dim"] == 3 else 36)


def _rhs(prm, s, prec, tiles):
    p = dict(prm)
    if tiles:
        p["flags"] |= I.FLAG_TILES
    st, dv, sim = B().rhs_once(p, s, prec=prec)
    cnt, nbr = sim.neighbor_table()
    assert sim.poll_error() == 0
    return st, dv, cnt, nbr


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", CASES)
def test_tiled_rhs_equals_gather_kernels(name, prec):
    prm, s = _case(name)
    print(f"tiles rhs: {name} {prec} n={len(s['p'])}", flush=True)
    a = _rhs(prm, s, prec, False)
    b = _rhs(prm, s, prec, True)
    assert np.array_equal(a[0]["id"], b[0]["id"])
    assert np.array_equal(a[2], b[2])
    for i in range(len(a[2])):
        assert np.array_equal(a[3][i, :a[2][i]], b[3][i, :a[2][i]]), i
    for key in ("rho", "vol", "jcur", "red"):
        assert np.array_equal(a[1][key], b[1][key]), key
    for key in ("p", "u", "ut"):
        assert np.array_equal(a[0][key], b[0][key]), key
    tol = 1e-12 if prec == "fp64" else 2e-5
    for key in ("pavg", "a", "b", "pdot", "force", "drag"):
        scale = max(np.abs(a[1][key]).max(), 1e-300)
        err = np.abs(a[1][key] - b[1][key]).max() / scale
        print(f"  {key}: max diff / max |value| = {err:.2e}")
        assert err <= tol, key


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["C2", "C4", "C5-small", "lattice3d"])
def test_tiled_steps_equal_gather_kernels(name, prec):
    """Whole steps (bin with the cell order kept while the skin allows,
    both stages, bookkeeping): the tiled run follows the gather run to rounding."""
    import torch
    prm, s = _case(name)
    prm["flags"] |= I.FLAG_REUSE_BINS
    steps = 30
    out = []
    for tiles in (False, True):
        p = dict(prm)
        if tiles:
            p["flags"] |= I.FLAG_TILES
        print(f"tiles steps: {name} {prec} tiles={tiles}", flush=True)
        sim = B().Simulation(p, s, prec=prec)
        dh = torch.zeros((steps, 3), dtype=torch.float64, device="cuda")
        sim.step(steps, dh)
        assert sim.poll_error() == 0
        out.append((sim.state(), dh.cpu().numpy()))
    (sa, da), (sb, db) = out
    for key in ("id", "type", "head", "red_prev"):
        assert np.array_equal(sa[key], sb[key]), key
    tol = 1e-10 if prec == "fp64" else 1e-4
    dx = prm["dx"]
    for key, scale in (("x", dx), ("u", None), ("ut", None), ("p", None), ("avg", None)):
        sc = scale or max(np.abs(sa[key]).max(), 1e-300)
        err = np.abs(sa[key] - sb[key]).max() / sc
        print(f"  {key}: max diff / scale = {err:.2e}")
        assert err <= tol, key
    assert np.abs(da - db).max() <= tol * max(np.abs(da).max(), 1e-300)
