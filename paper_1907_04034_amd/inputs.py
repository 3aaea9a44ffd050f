"""Seeded synthetic inputs for the EDAC-SPH wind-tunnel path.

This module builds particle sets (lattices, inlet/outlet/wall layers, cylinders)
and the configuration parameters of the five workloads. It holds none of the
method's arithmetic: no kernel, no neighbour search, no pair term, no boundary
rule. Both the HIP path and the CPU oracle consume its output, so that they see
bit-identical FP64 inputs.

Particle-set format (a dict of numpy arrays, one row per particle):

    x, u, ut, uin : float64 (n, 3)   position, momentum velocity, transport
                                     velocity, prescribed inlet velocity
    p             : float64 (n,)     gauge pressure
    ring          : float64 (n, 6, 4) time-average window of (u, v, w, p)
    head          : int32   (n,)     next ring slot to overwrite
    avg           : float64 (n, 4)   mean of the ring
    jprev         : float64 (n, 3)   characteristic variables of the previous step
    red_prev      : uint8   (n,)     1 if the particle had fluid support last step
    type          : uint8   (n,)     FLUID/INLET/OUTLET/WALL_SLIP/WALL_NOSLIP/BODY
    id            : int64   (n,)     stable particle identity

In 2D the third components are zero. Parameters follow the paper's EDAC setup
(Sec. 2): c_s = 10 U, alpha = 0.5, the 0.01 regulariser of the viscous term, and
a 6-step averaging window (Sec. 3.4, eq:N). The time step and background
pressure are chosen by the usual EDAC-TVF rule (acoustic CFL 0.25, viscous
limit 0.125 h^2/nu, p_b = rho0 c^2) and are passed to both sides as inputs.
"""
from __future__ import annotations

import math

import numpy as np

FLUID, INLET, OUTLET, WALL_SLIP, WALL_NOSLIP, BODY, DEAD = 0, 1, 2, 3, 4, 5, 255
N_AVG = 6

# flag bits shared by both sides' parameter blocks
FLAG_NO_PAVG = 1   # drop the neighbour-average pressure (conservation tests)
FLAG_DAMP_NU = 2   # use the physical viscosity in the pressure damping term
FLAG_NOISE = 4     # add seeded velocity noise to inlet particles at spawn
FLAG_REUSE_BINS = 8  # GPU stepping option: keep the cell order while the skin allows
                     # (same neighbour sets; the oracle ignores it)
FLAG_QUINTIC = 16  # the paper's quintic spline (support 3h) instead of Wendland C2 (2h)
FLAG_MIRROR_INLET = 32  # inlet pressure mirrored from the fluid instead of the characteristic J3
FLAG_TILES = 128  # GPU option: the LDS-tiled pair passes instead of the gather kernels (same results)

ID_GENERATION = 1 << 40   # a spawned inlet particle's id is its parent's + this

# outlet rules (the "outlet" entry of a parameter dict; absent = hybrid)
OUTLET_HYBRID, OUTLET_MOC, OUTLET_DO_NOTHING, OUTLET_MOD_DO_NOTHING, OUTLET_MIRROR = 0, 1, 2, 3, 4
OUTLETS = {"hybrid": OUTLET_HYBRID, "moc": OUTLET_MOC, "do-nothing": OUTLET_DO_NOTHING,
           "mod-do-nothing": OUTLET_MOD_DO_NOTHING, "mirror": OUTLET_MIRROR}


def base_params(*, dim, dx, U=1.0, c_factor=10.0, rho0=1.0, nu=0.01, alpha=0.5,
                h_over_dx=1.0, name="custom"):
    h = h_over_dx * dx
    c = c_factor * U
    dt = min(0.25 * h / (c + U), 0.125 * h * h / nu) if nu > 0 else 0.25 * h / (c + U)
    return dict(
        name=name, dim=dim, dx=dx, h=h, rho0=rho0, c=c, U=U, nu=nu, alpha=alpha,
        eta=0.01, dt=dt, pb=rho0 * c * c, n_avg=N_AVG, flags=0,
        lo=[0.0, 0.0, 0.0], hi=[1.0, 1.0, 1.0], periodic=[0, 0, 0],
        x_inlet=-1e30, x_outlet=1e30, x_outlet_end=1e30, inlet_len=0.0,
        noise_amp=0.0, noise_seed=0, D=0.0, steps=1,
    )


def _empty(n):
    return dict(
        x=np.zeros((n, 3)), u=np.zeros((n, 3)), ut=np.zeros((n, 3)),
        uin=np.zeros((n, 3)), p=np.zeros(n), ring=np.zeros((n, N_AVG, 4)),
        head=np.zeros(n, np.int32), avg=np.zeros((n, 4)), jprev=np.zeros((n, 3)),
        red_prev=np.zeros(n, np.uint8), type=np.zeros(n, np.uint8),
        id=np.arange(n, dtype=np.int64),
    )


def _finish(parts):
    """Concatenate blocks, fill rings/averages with the initial (u, v, w, p)."""
    keys = parts[0].keys()
    s = {k: np.concatenate([b[k] for b in parts]) for k in keys}
    n = len(s["p"])
    s["id"] = np.arange(n, dtype=np.int64)
    s["ut"] = s["u"].copy()
    init = np.concatenate([s["u"], s["p"][:, None]], axis=1)
    s["ring"] = np.repeat(init[:, None, :], N_AVG, axis=1).copy()
    s["avg"] = init.copy()
    s["head"] = np.zeros(n, np.int32)
    s["jprev"] = np.zeros((n, 3))
    s["red_prev"] = np.zeros(n, np.uint8)
    return s


def _block(xs, ys, zs, typ):
    g = np.meshgrid(xs, ys, zs, indexing="ij")
    pts = np.stack([a.ravel() for a in g], axis=1)
    b = _empty(len(pts))
    b["x"] = pts
    b["type"][:] = typ
    return b


def centres(i0, i1, dx, origin=0.0):
    return origin + (np.arange(i0, i1) + 0.5) * dx


def taylor_green_box(n_side=40, L=1.0, U=1.0, nu=0.01):
    """Periodic unit box, square lattice, Taylor-Green vortex initial state."""
    dx = L / n_side
    prm = base_params(dim=2, dx=dx, U=U, nu=nu, name=f"tgv{n_side}")
    prm.update(lo=[0.0, 0.0, 0.0], hi=[L, L, 0.0], periodic=[1, 1, 0])
    b = _block(centres(0, n_side, dx), centres(0, n_side, dx), [0.0], FLUID)
    x, y = b["x"][:, 0], b["x"][:, 1]
    k = 2.0 * math.pi / L
    b["u"][:, 0] = -U * np.cos(k * x) * np.sin(k * y)
    b["u"][:, 1] = U * np.sin(k * x) * np.cos(k * y)
    b["p"] = -0.25 * prm["rho0"] * U * U * (np.cos(2 * k * x) + np.cos(2 * k * y))
    return prm, _finish([b])


def periodic_lattice(n_side=12, dim=2, dx=0.1, U=0.0, quintic=False):
    """Perfect periodic lattice with zero fields (used for closed-form checks);
    quintic: the paper's kernel and h/dx = 1.2."""
    L = n_side * dx
    prm = base_params(dim=dim, dx=dx, U=max(U, 1.0), h_over_dx=1.2 if quintic else 1.0,
                      name=f"lattice{dim}d")
    if quintic:
        prm["flags"] |= FLAG_QUINTIC
    prm.update(lo=[0.0] * 3, hi=[L, L, L if dim == 3 else 0.0],
               periodic=[1, 1, 1 if dim == 3 else 0])
    zs = centres(0, n_side, dx) if dim == 3 else [0.0]
    b = _block(centres(0, n_side, dx), centres(0, n_side, dx), zs, FLUID)
    return prm, _finish([b])


def channel(Lx=4.0, Ly=1.0, Lz=None, dx=0.01, layers=5, U=1.0, nu=0.01,
            pulse_amp=None, pulse_x=None, pulse_w=0.1, cyl=None,
            side_walls=None, wall_layers=3, noise=0.0, noise_seed=1907,
            quintic=False, cyl_layers=None, name="channel"):
    """Wind-tunnel channel: inlet layers | fluid | hybrid outlet layers.

    Lz=None gives 2D. side_walls: None (periodic lateral directions),
    'slip' or 'noslip' (wall_layers layers of wall particles on every lateral
    face, spanning the whole x range). cyl=(xc, yc, D) adds a no-slip body
    made of cyl_layers (default wall_layers; 0 = down to the centre)
    concentric rings spaced dx inward from D/2 - dx/2, each with particles
    about dx apart.
    pulse_amp adds p = A exp(-((x - pulse_x)/pulse_w)^2) to the fluid.
    quintic: the paper's kernel with its h/dx = 1.2 (support 3.6 dx, within the
    5 inlet and outlet layers; walls need 4 layers).
    """
    dim = 2 if Lz is None else 3
    prm = base_params(dim=dim, dx=dx, U=U, nu=nu, h_over_dx=1.2 if quintic else 1.0, name=name)
    if quintic:
        prm["flags"] |= FLAG_QUINTIC
    nx, ny = int(round(Lx / dx)), int(round(Ly / dx))
    nz = int(round(Lz / dx)) if dim == 3 else 0
    wl = wall_layers if side_walls else 0
    pad = 2 * dx
    prm.update(
        x_inlet=0.0, x_outlet=Lx, x_outlet_end=Lx + layers * dx, inlet_len=layers * dx,
        lo=[-layers * dx - pad, -wl * dx - (pad if wl else 0.0),
            (-wl * dx - (pad if wl else 0.0)) if dim == 3 else 0.0],
        hi=[Lx + layers * dx + pad, Ly + wl * dx + (pad if wl else 0.0),
            (Lz + wl * dx + (pad if wl else 0.0)) if dim == 3 else 0.0],
        periodic=[0, 0 if side_walls else 1, (0 if side_walls else 1) if dim == 3 else 0],
    )
    ys = centres(0, ny, dx)
    zs = centres(0, nz, dx) if dim == 3 else [0.0]
    blocks = []
    inl = _block(centres(-layers, 0, dx), ys, zs, INLET)
    inl["uin"][:, 0] = U
    inl["u"][:, 0] = U
    blocks.append(inl)
    fl = _block(centres(0, nx, dx), ys, zs, FLUID)
    fl["u"][:, 0] = U
    if pulse_amp is not None:
        px = Lx / 2 if pulse_x is None else pulse_x
        fl["p"] = pulse_amp * np.exp(-(((fl["x"][:, 0] - px) / pulse_w) ** 2))
    if cyl is not None:
        xc, yc, D = cyl
        r = np.hypot(fl["x"][:, 0] - xc, fl["x"][:, 1] - yc)
        keep = r >= 0.5 * D
        fl = {k: v[keep] for k, v in fl.items()}
        prm["D"] = D
    blocks.append(fl)
    out = _block(centres(nx, nx + layers, dx), ys, zs, OUTLET)
    out["u"][:, 0] = U
    blocks.append(out)
    if side_walls:
        wt = WALL_SLIP if side_walls == "slip" else WALL_NOSLIP
        xs_all = centres(-layers, nx + layers, dx)
        if dim == 2:
            blocks.append(_block(xs_all, centres(-wl, 0, dx), [0.0], wt))
            blocks.append(_block(xs_all, centres(ny, ny + wl, dx), [0.0], wt))
        else:
            yy = centres(-wl, ny + wl, dx)
            zz = centres(-wl, nz + wl, dx)
            g = np.meshgrid(yy, zz, indexing="ij")
            yz = np.stack([g[0].ravel(), g[1].ravel()], axis=1)
            inside = ((yz[:, 0] > 0) & (yz[:, 0] < Ly) & (yz[:, 1] > 0) & (yz[:, 1] < Lz))
            yz = yz[~inside]
            pts = np.concatenate([
                np.stack([np.full(len(yz), xv), yz[:, 0], yz[:, 1]], axis=1)
                for xv in xs_all])
            wb = _empty(len(pts))
            wb["x"] = pts
            wb["type"][:] = wt
            blocks.append(wb)
    if cyl is not None:
        xc, yc, D = cyl
        pts = []
        nring = wall_layers if cyl_layers is None else (cyl_layers or 1 << 30)
        for k in range(nring):
            rk = 0.5 * D - (k + 0.5) * dx
            if rk <= 0:
                break
            nk = max(1, int(round(2 * math.pi * rk / dx)))
            th = 2 * math.pi * (np.arange(nk) + 0.5) / nk
            pts.append(np.stack([xc + rk * np.cos(th), yc + rk * np.sin(th),
                                 np.zeros(nk)], axis=1))
        pts = np.concatenate(pts)
        cb = _empty(len(pts))
        cb["x"] = pts
        cb["type"][:] = BODY
        blocks.append(cb)
    s = _finish(blocks)
    if noise:
        prm["flags"] |= FLAG_NOISE
        prm["noise_amp"] = noise
        prm["noise_seed"] = noise_seed
    return prm, s


def cylinder_tunnel(D=2.0, Re=20.0, dx=0.1, U=1.0, quintic=True, outlet=None):
    """The paper's flow past a circular cylinder (Sec. 4.6): a 15D x 15D fluid
    region, the cylinder centred 5D behind the inlet interface and midway
    between slip walls, 6 layers of inlet, outlet and wall particles, the
    body filled with rings down to its centre, nu = U D / Re, and the paper's
    kernel at h = 1.2 dx (quintic=False: Wendland C2 at h = dx)."""
    L = 15.0 * D
    prm, s = channel(Lx=L, Ly=L, dx=dx, layers=6, U=U, nu=U * D / Re,
                     cyl=(5.0 * D, 0.5 * L, D), side_walls="slip", wall_layers=6,
                     cyl_layers=0, quintic=quintic,
                     name=f"cylinder tunnel D={D} Re={Re:g} dx={dx:g}")
    if outlet is not None:
        prm["outlet"] = outlet
    return prm, s


def vortex_tunnel(dx=0.1, L=2.0, W=4.0, T=4.0, probe=1.7, long=False, U=1.0):
    """The paper's moving-vortex problem (Sec. 4.4): a fluid region L long and
    W wide between inviscid (slip) walls, 6 layers of inlet, outlet and wall
    particles, inviscid fluid, the paper's kernel at h = 1.2 dx. long=True
    gives the reference domain of length probe + c T (Sec. 4), whose outlet
    no wave from the probe region reaches within the time T."""
    c = 10.0 * U
    Lx = probe + c * T if long else L
    prm, s = channel(Lx=Lx, Ly=W, dx=dx, layers=6, U=U, nu=0.0, side_walls="slip",
                     wall_layers=6, quintic=True,
                     name=f"vortex tunnel {Lx:g}x{W:g} dx={dx:g}")
    prm["probe"] = [probe, 0.5 * W, 0.0]
    return prm, s


def ramp_tunnel(dx=0.1, L=2.0, W=2.0, T=3.0, probe=1.7, long=False, U=1.0):
    """The paper's ramp-inlet problem (Sec. 4.3): the 2D-pulse tunnel (L x W
    fluid, slip walls, 6 layers of inlet, outlet and wall particles, inviscid,
    the paper's kernel at h = 1.2 dx) with everything at rest at t = 0; the
    inlet velocity then follows ramp_inlet_velocity. long=True: the reference
    domain of length probe + c T."""
    c = 10.0 * U
    Lx = probe + c * T if long else L
    prm, s = channel(Lx=Lx, Ly=W, dx=dx, layers=6, U=U, nu=0.0, side_walls="slip",
                     wall_layers=6, quintic=True, name=f"ramp tunnel {Lx:g}x{W:g} dx={dx:g}")
    s["u"][:] = 0.0
    s["ut"][:] = 0.0
    s["uin"][:] = 0.0
    s["ring"][:] = 0.0
    s["avg"][:] = 0.0
    prm["probe"] = [probe, 0.5 * W, 0.0]
    return prm, s


def bump_tunnel(dx=0.005, L=1.0, W=0.1, T=0.2, long=False, U=1.0, alpha=0.1, rho0=1000.0):
    """The paper's 1D pressure bump (Sec. 4.1, eq:pressurebump, after
    Lastiwka et al.): fluid of density rho0 moving at U through an L long
    tunnel, 6 layers of inlet and outlet particles, periodic across (a 1D
    problem in a 2D domain, W wide), inviscid, the paper's kernel at
    h = 1.2 dx, EDAC alpha = 0.1. Pressure p(x) = 1 - 0.2 exp(-(x - 0.5)^2 /
    0.001) in the fluid and 1 at inlet and outlet, here shifted by -1 Pa (the
    scheme sees pressure only through differences, apart from the acoustic
    gate at rho0 U^2 / 2 = 500 Pa, which this bump never reaches; the
    characteristics outlet's p_ref = 1 Pa of the paper is then its 0). The
    spacing is not given for this case (the paper's default 0.1 m cannot
    resolve a bump of width 0.03 m); 0.005 m puts 6 particles in its width.
    long=True: a tunnel of length L + (c + U) T, which the right-going wave
    does not leave within T."""
    c = 10.0 * U
    Lx = L + (c + U) * T if long else L
    prm, s = channel(Lx=Lx, Ly=W, dx=dx, layers=6, U=U, nu=0.0, side_walls=None,
                     quintic=True, name=f"1D bump tunnel {Lx:g}x{W:g} dx={dx:g}")
    prm.update(alpha=alpha, rho0=rho0)
    prm["pb"] = rho0 * prm["c"] ** 2
    fl = s["type"] == FLUID
    s["p"][:] = 0.0
    s["p"][fl] = -0.2 * np.exp(-((s["x"][fl, 0] - 0.5) ** 2) / 0.001)
    s["ring"][:, :, 3] = s["p"][:, None]
    s["avg"][:, 3] = s["p"]
    return prm, s


def pulse2d_tunnel(dx=0.1, L=2.0, W=2.0, T=3.0, probe=1.7, long=False, U=1.0, alpha=0.5):
    """The paper's 2D pulse (Sec. 4.2): the ramp problem's tunnel (L x W fluid,
    slip walls, 6 layers of inlet, outlet and wall particles, inviscid, the
    paper's kernel at h = 1.2 dx) in uniform flow U; the inlet velocity then
    follows pulse2d_inlet_velocity. alpha is the EDAC damping coefficient
    (the paper's tables use 0.5 and sweep 0.1 to 1.0). long=True: the
    reference domain of length probe + c T."""
    c = 10.0 * U
    Lx = probe + c * T if long else L
    prm, s = channel(Lx=Lx, Ly=W, dx=dx, layers=6, U=U, nu=0.0, side_walls="slip",
                     wall_layers=6, quintic=True, name=f"2D pulse tunnel {Lx:g}x{W:g} dx={dx:g}")
    prm["alpha"] = alpha
    prm["probe"] = [probe, 0.5 * W, 0.0]
    return prm, s


def pulse2d_inlet_velocity(y, t, W=2.0, U=1.0, delta=1e-3):
    """Inlet x velocity of the 2D pulse (Sec. 4.2 eq:velfunc2, as read here):
    U + 0.5 U cos(pi y' / 12) exp(-(t - 1)^2 / delta) for 1 < t < 1.1 s, else U,
    with y' = y - W/2 measured from the channel's centre line. The printed
    exponent has no minus sign and delta is not given; delta = 1e-3 makes the
    pulse a half-Gaussian of about 0.03 s that has decayed to 5e-5 of its
    height where the printed window closes. Works on numpy arrays and torch
    tensors alike (y), t a float."""
    if not (1.0 < t < 1.1):
        return y * 0.0 + U
    g = 0.5 * U * float(np.exp(-(t - 1.0) ** 2 / delta))
    yc = y - 0.5 * W
    try:
        import torch
        if isinstance(yc, torch.Tensor):
            return U + g * torch.cos(np.pi * yc / 12.0)
    except ImportError:
        pass
    return U + g * np.cos(np.pi * yc / 12.0)


def ramp_inlet_velocity(t, U=1.0):
    """Inlet x velocity of the ramp problem: U t for t < 1 s, then U."""
    return U * min(max(t, 0.0), 1.0)


def vortex_inlet_velocity(y, t, W=4.0, U=1.0, gamma=0.1):
    """Prescribed inlet velocity of the vortex problem at time t (Sec. 4.4
    eq:vortex with eq:vortexx): (u, v) = (U + G y'/(r^2 + 0.2), -G x'/(r^2 + 0.2))
    with x' = U (1 - t), the distance of the vortex centre from the start of
    the inlet, y' = y - W/2 and r^2 = x'^2 + y'^2. Works on numpy arrays and
    torch tensors alike."""
    xv = U * (1.0 - t)
    yv = y - 0.5 * W
    den = xv * xv + yv * yv + 0.2
    return U + gamma * yv / den, -gamma * xv / den


# ---------------------------------------------------------------- workloads

def config(name, small=False):
    """The five workloads. small=True gives a reduced-size variant with the
    same structure (layers, boundary kinds, pulse/cylinder) for parity tests."""
    if name == "C1":
        prm, s = taylor_green_box(n_side=40, L=1.0, U=1.0, nu=0.01)
        prm.update(name="C1 tgv 40x40", steps=100)
        return prm, s
    if name == "C2":
        if small:
            prm, s = channel(Lx=0.4, Ly=0.1, dx=0.01, pulse_amp=0.1, pulse_x=0.2,
                             pulse_w=0.02, name="C2-small channel")
        else:
            prm, s = channel(Lx=4.0, Ly=1.0, dx=0.01, pulse_amp=0.1, pulse_x=2.0,
                             pulse_w=0.1, name="C2 channel 4x1 dx0.01 pulse")
        prm["steps"] = 2000
        return prm, s
    if name == "C2Q":
        # the 2D channel with the paper's own kernel and resolution ratio
        if small:
            prm, s = channel(Lx=0.4, Ly=0.2, dx=0.01, pulse_amp=0.1, pulse_x=0.2,
                             pulse_w=0.02, quintic=True, name="C2Q-small channel quintic")
        else:
            prm, s = channel(Lx=4.0, Ly=1.0, dx=0.01, pulse_amp=0.1, pulse_x=2.0,
                             pulse_w=0.1, quintic=True,
                             name="C2Q channel 4x1 dx0.01 pulse quintic h/dx1.2")
        prm["steps"] = 2000
        return prm, s
    if name == "C5Q":
        # small 3D duct with the paper's kernel (parity only)
        prm, s = channel(Lx=0.16, Ly=0.08, Lz=0.08, dx=0.01, side_walls="noslip",
                         wall_layers=4, noise=0.01, quintic=True, name="C5Q-small duct quintic")
        prm["steps"] = 500
        return prm, s
    if name == "C3":
        if small:
            prm, s = channel(Lx=1.2, Ly=0.64, dx=0.04 / 2.5, cyl=(0.3, 0.32, 0.16),
                             side_walls="slip", nu=0.008, name="C3-small cylinder")
        else:
            D = 2.0
            prm, s = channel(Lx=60.0, Ly=32.0, dx=D / 50, cyl=(5 * D, 16.0, D),
                             side_walls="slip", nu=1.0 * D / 200.0,
                             name="C3 cylinder Re200 60x32 dx0.04")
        prm["steps"] = 5000
        return prm, s
    if name == "C4":
        if small:
            prm, s = channel(Lx=0.5, Ly=0.2, dx=0.01, cyl=(0.2, 0.1, 0.06),
                             name="C4-small channel+cylinder")
        else:
            prm, s = channel(Lx=4.0, Ly=1.0, dx=0.01, cyl=(1.0, 0.5, 0.2),
                             nu=1.0 * 0.2 / 20.0, name="C4 channel+cylinder D0.2 Re20")
        prm["steps"] = 500
        return prm, s
    if name == "C5":
        if small:
            prm, s = channel(Lx=0.16, Ly=0.08, Lz=0.08, dx=0.01, side_walls="noslip",
                             noise=0.01, name="C5-small duct")
        else:
            prm, s = channel(Lx=4.0, Ly=1.0, Lz=1.0, dx=0.01, side_walls="noslip",
                             noise=0.01, name="C5 duct 4x1x1 dx0.01")
        prm["steps"] = 500
        return prm, s
    raise KeyError(name)


def jitter(prm, s, amp, seed, types=(FLUID,)):
    """Seeded uniform jitter of +-amp*dx on positions of the given types."""
    rng = np.random.default_rng(seed)
    s = {k: v.copy() for k, v in s.items()}
    m = np.isin(s["type"], types)
    d = prm["dim"]
    s["x"][m, :d] += amp * prm["dx"] * rng.uniform(-1, 1, size=(m.sum(), d))
    return s


def random_fields(prm, s, seed, p_range=(-0.5, 0.5), u_range=(0.0, 1.5), ut_dev=0.05):
    """Seeded random p, u and transport-velocity perturbation on fluid particles,
    and random averages/previous characteristic values on every particle."""
    rng = np.random.default_rng(seed)
    s = {k: v.copy() for k, v in s.items()}
    n, d = len(s["p"]), prm["dim"]
    fl = s["type"] == FLUID
    s["p"][fl] = rng.uniform(*p_range, size=fl.sum())
    s["u"][fl, :d] = rng.uniform(*u_range, size=(fl.sum(), d))
    s["ut"][fl, :d] = s["u"][fl, :d] + rng.uniform(-ut_dev, ut_dev, size=(fl.sum(), d))
    s["avg"][:, :d] = rng.uniform(*u_range, size=(n, d))
    s["avg"][:, 3] = rng.uniform(*p_range, size=n)
    s["jprev"][:] = rng.uniform(-0.5, 0.5, size=(n, 3))
    s["red_prev"][:] = (rng.uniform(size=n) < 0.5).astype(np.uint8)
    return s


def snapshot_copy(s):
    return {k: np.array(v, copy=True) for k, v in s.items()}


# ------------------------------------------------------- inlet profile

def inlet_rows(prm, s):
    """Lattice row of every inlet particle (-1 for other kinds): rows are
    numbered by the transverse lattice position ((j + 1/2) dx in y, and z in
    3D, row = jy * nz + jz)."""
    n, dx = len(s["p"]), prm["dx"]
    rows = np.full(n, -1, np.int64)
    m = s["type"] == INLET
    if not m.any():
        return rows
    jy = np.rint(s["x"][m, 1] / dx - 0.5).astype(np.int64)
    if prm["dim"] == 3:
        jz = np.rint(s["x"][m, 2] / dx - 0.5).astype(np.int64)
        jy = jy - jy.min()
        jz = jz - jz.min()
        rows[m] = jy * (jz.max() + 1) + jz
    else:
        rows[m] = jy - jy.min()
    return rows


def inlet_profile(prm, s, rows):
    """The streamwise inlet velocity of every row (first particle found)."""
    theta = np.zeros(int(rows.max()) + 1)
    for k in range(len(theta)):
        theta[k] = s["uin"][np.flatnonzero(rows == k)[0], 0]
    return theta


def set_inlet_profile(prm, s, rows, theta):
    """Copy of s whose inlet row k has streamwise u_in = u = ut = ring = mean
    = theta[k]."""
    s = snapshot_copy(s)
    m = rows >= 0
    v = np.asarray(theta, np.float64)[rows[m]]
    for key in ("uin", "u", "ut", "avg"):
        s[key][m, 0] = v
    s["ring"][m, :, 0] = v[:, None]
    return s
