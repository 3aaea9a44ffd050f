"""Pins of the oracle parts that uniform lattices leave open.

1. The density weights of the pair pressure (Sec. 2 eq:tvf-p-ij-basa) and of
   the divergence term of the pressure rate (eq:p-edac, m_j rho_i / rho_j).
   On a uniform lattice every rho is equal, so a transposed rho_i / rho_j, or
   an unweighted mean, would pass every closed form there. Here the right-hand
   side is linear in the pressures (with u = 0 and no neighbour average) and
   in the velocities (with p = 0), and the coefficients the oracle produces
   must obey identities that follow from the weights alone:
     * pair pressure: K_ij rho_j + K_ji rho_i = 0 and
       K_jj = sum_k (rho_k / rho_j) K_jk, where K_ij = d a_i / d p_j;
     * pressure rate: L_ij rho_j^2 + L_ji rho_i^2 = 0, where
       L_ij = d pdot_i / d u_j,x.
   The inputs are a jittered block of fluid in a closed box with empty space
   around it, so rho falls to about 0.6 rho0 at its corners.
2. The body force of Sec. 4.6 eq:tvf-momentum_solid on one body particle of a
   periodic lattice: in the linear pressure field p = G x it equals
   -G g dx^d / s^2 (the fluid's own lattice response times the particle mass;
   s and g are the lattice sums pinned elsewhere), and in the shear flow
   u_x = gamma y with the no-slip ghost velocity it equals
   4 rho0 nu gamma y_i delta dx^(d-2) / s, with delta = -sum F^ |o|^2 /
   (|o|^2 + 0.01) over the lattice offsets (F^ = W'(q)/q at h = 1), evaluated
   here in 30-digit arithmetic.
3. The seeded inlet noise: the generator against published SplitMix64 outputs,
   the velocity distribution (uniform, mean U e_x, standard deviation amp U,
   support +-sqrt(3) amp U per component, uncorrelated components) over 10^5
   identities, and a re-spawned particle of a stepped 3D duct taking the noise
   of its own identity.
"""
import itertools

import mpmath as mp
import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O
from paper_1907_04034_amd import inputs as I

mp.mp.dps = 30


# ------------------------------------------------------------ unequal densities

def _closed_block(seed=3, n=9, dim=2):
    """A jittered n^dim block of fluid particles with empty space around it in a
    closed (non-periodic) box, so that densities differ near its faces."""
    dx = 0.1
    prm = I.base_params(dim=dim, dx=dx, name="closed block")
    L = (n + 8) * dx
    prm.update(lo=[0.0] * 3, hi=[L, L, L if dim == 3 else 0.0], periodic=[0, 0, 0],
               flags=I.FLAG_NO_PAVG)
    xs = I.centres(4, 4 + n, dx)
    zs = xs if dim == 3 else [0.0]
    b = I._block(xs, xs, zs, I.FLUID)
    s = I._finish([b])
    s = I.jitter(prm, s, 0.2, seed)
    return prm, s


def _coefficients(prm, s, field, comp=0):
    """Column k of the linear map field -> (a, pdot): the oracle's a and pdot
    with the field set to the unit vector e_k (component comp for velocities)
    and every other input field zero."""
    n = len(s["p"])
    A = np.zeros((n, n, 3))
    P = np.zeros((n, n))
    base = I.snapshot_copy(s)
    base["p"][:] = 0.0
    base["u"][:] = 0.0
    base["ut"][:] = 0.0
    for k in range(n):
        t = I.snapshot_copy(base)
        if field == "p":
            t["p"][k] = 1.0
        else:
            t["u"][k, comp] = 1.0
            t["ut"][k, comp] = 1.0
        _, d, _ = O.rhs_once(prm, t)
        A[:, k] = d["a"]
        P[:, k] = d["pdot"]
    _, d0, _ = O.rhs_once(prm, base)
    return A, P, d0


def _pairs(prm, s):
    o = O.Oracle(prm, s)
    row, col = o.neighbors(brute=True)
    return [(i, int(j)) for i in range(len(row) - 1) for j in col[row[i]:row[i + 1]] if j != i]


@pytest.fixture(scope="module")
def block2d():
    prm, s = _closed_block()
    return prm, s, _pairs(prm, s)


def test_block_densities_are_unequal(block2d):
    """The input does what the identities below need: neighbours whose
    densities differ by tens of percent."""
    prm, s, pairs = block2d
    _, d, _ = O.rhs_once(prm, s)
    rho = d["rho"]
    ratio = max(rho[i] / rho[j] for i, j in pairs)
    assert ratio > 1.4
    assert rho.min() < 0.7 * prm["rho0"]


def test_pair_pressure_density_weights(block2d):
    """eq:tvf-p-ij-basa weights p_i by rho_j and p_j by rho_i: the coefficient
    of p_j in a_i and that of p_i in a_j stand in the ratio -rho_i / rho_j, and
    the coefficient of p_j in a_j is the rho_k / rho_j-weighted sum of its
    cross coefficients (a transposed or unweighted mean fails both)."""
    prm, s, pairs = block2d
    K, _, d0 = _coefficients(prm, s, "p")
    rho = d0["rho"]
    assert np.abs(d0["a"]).max() == 0.0  # zero fields: the map is linear
    scale = np.abs(K).max()
    worst = 0.0
    for i, j in pairs:
        r = K[i, j] * rho[j] + K[j, i] * rho[i]
        worst = max(worst, np.abs(r).max())
    assert worst < 1e-12 * scale * rho.max()
    nbrs = {}
    for i, j in pairs:
        nbrs.setdefault(j, []).append(i)
    for j, ks in nbrs.items():
        # K[j, k] is the coefficient of p_k in a_j
        ref = sum(rho[k] / rho[j] * K[j, k] for k in ks)
        assert np.abs(K[j, j] - ref).max() < 1e-12 * scale
    # the identities are not vacuous: cross coefficients are far from the
    # unweighted ones
    i, j = max(pairs, key=lambda q: rho[q[0]] / rho[q[1]])
    assert np.abs(K[i, j] + K[j, i]).max() > 0.1 * np.abs(K[i, j]).max()


def test_pressure_rate_density_weights(block2d):
    """The divergence term of eq:p-edac carries m_j rho_i / rho_j: the
    coefficient of u_j in pdot_i and that of u_i in pdot_j satisfy
    L_ij rho_j^2 + L_ji rho_i^2 = 0 (m_j rho_j / rho_i, or no weight, fails)."""
    prm, s, pairs = block2d
    for comp in (0, 1):
        _, L, d0 = _coefficients(prm, s, "u", comp)
        rho = d0["rho"]
        scale = np.abs(L).max() * rho.max() ** 2
        worst = max(abs(L[i, j] * rho[j] ** 2 + L[j, i] * rho[i] ** 2) for i, j in pairs)
        assert worst < 1e-12 * scale
        i, j = max(pairs, key=lambda q: rho[q[0]] / rho[q[1]])
        assert abs(L[i, j] * rho[j] + L[j, i] * rho[i]) > 0.1 * abs(L[i, j] * rho[j])


def test_pair_pressure_weights_in_3d():
    """The first identity on a small 3D block."""
    prm, s = _closed_block(seed=5, n=4, dim=3)
    pairs = _pairs(prm, s)
    K, _, d0 = _coefficients(prm, s, "p")
    rho = d0["rho"]
    assert max(rho[i] / rho[j] for i, j in pairs) > 1.3
    scale = np.abs(K).max() * rho.max()
    for i, j in pairs:
        assert np.abs(K[i, j] * rho[j] + K[j, i] * rho[i]).max() < 1e-12 * scale


# ------------------------------------------------------------------ body force

def _fhat(q, dim):
    """F^ = W'(q)/q of the Wendland C2 kernel at h = 1 (mpmath), from its
    published definition, W = a (1 - q/2)^4 (2q + 1)."""
    a = mp.mpf(7) / (4 * mp.pi) if dim == 2 else mp.mpf(21) / (16 * mp.pi)
    w = lambda z: a * (1 - z / 2) ** 4 * (2 * z + 1) if z < 2 else mp.mpf(0)
    return mp.diff(w, q) / q


def _body_constants(dim):
    """s = sum W^, g = -sum F^ o_x^2 and delta = -sum F^ |o|^2/(|o|^2 + 0.01)
    over the lattice offsets within the support (h = dx = 1)."""
    a = mp.mpf(7) / (4 * mp.pi) if dim == 2 else mp.mpf(21) / (16 * mp.pi)
    s = g = delta = mp.mpf(0)
    for o in itertools.product(range(-2, 3), repeat=dim):
        r2 = sum(v * v for v in o)
        if r2 >= 4:
            continue
        r = mp.sqrt(r2)
        s += a * (1 - r / 2) ** 4 * (2 * r + 1)
        if r2 == 0:
            continue
        F = _fhat(r, dim)
        g += -F * o[0] ** 2
        delta += -F * r2 / (r2 + mp.mpf("0.01"))
    return float(s), float(g), float(delta)


def _lattice_with_body(dim):
    n = 16 if dim == 2 else 8
    prm, s = I.periodic_lattice(n_side=n, dim=dim, dx=1.0 / n)
    centre = np.full(dim, n // 2 + 0.5) / n
    k = int(np.argmin(((s["x"][:, :dim] - centre) ** 2).sum(axis=1)))
    s["type"][k] = I.BODY
    return prm, s, k


@pytest.mark.parametrize("dim", [2, 3])
def test_body_force_in_linear_pressure(dim):
    """p = G x in the fluid (the body takes its Shepard value, G x_i on the
    symmetric stencil): F_x = -(g/s^2) G dx^d, F_y = F_z = 0."""
    prm, s, k = _lattice_with_body(dim)
    G = 0.7
    fl = s["type"] == I.FLUID
    s["p"][fl] = G * s["x"][fl, 0]
    st, d, F = O.rhs_once(prm, s)
    sv, g, _ = _body_constants(dim)
    dx = prm["dx"]
    ref = -(g / sv ** 2) * G * dx ** dim
    assert abs(F[0] - ref) < 1e-11 * abs(ref)
    assert np.abs(F[1:dim]).max() < 1e-12 * abs(ref)
    # the body particle's pressure is the Shepard value G x_i
    kb = int(np.flatnonzero(st["type"] == I.BODY)[0])
    assert abs(st["p"][kb] - G * st["x"][kb, 0]) < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_body_force_in_shear_flow(dim):
    """u_x = gamma y in the fluid, p = 0: the no-slip ghost velocity of the
    body is -gamma y_i and the viscous part of eq:tvf-momentum_solid gives
    F_x = 4 rho0 nu gamma y_i delta dx^(d-2) / s."""
    prm, s, k = _lattice_with_body(dim)
    gam = 0.3
    fl = s["type"] == I.FLUID
    s["u"][fl, 0] = gam * s["x"][fl, 1]
    s["ut"] = s["u"].copy()
    st, d, F = O.rhs_once(prm, s)
    sv, _, delta = _body_constants(dim)
    yi = s["x"][k, 1]
    dx = prm["dx"]
    ref = 4 * prm["rho0"] * prm["nu"] * gam * yi * delta * dx ** (dim - 2) / sv
    assert abs(F[0] - ref) < 1e-10 * abs(ref)
    assert np.abs(F[1:dim]).max() < 1e-12 * abs(ref)
    kb = int(np.flatnonzero(st["type"] == I.BODY)[0])
    assert abs(st["u"][kb, 0] + gam * yi) < 1e-13


def test_body_force_is_additive_over_body_particles():
    """Two body particles far apart in p = G x: the total is twice the single
    particle's force (the sum runs over body particles)."""
    prm, s = I.periodic_lattice(n_side=16, dim=2, dx=1.0 / 16)
    ks = [4 * 16 + 4, 11 * 16 + 10]
    for k in ks:
        s["type"][k] = I.BODY
    fl = s["type"] == I.FLUID
    s["p"][fl] = 0.7 * s["x"][fl, 0]
    _, d, F = O.rhs_once(prm, s)
    sv, g, _ = _body_constants(2)
    ref = -2 * (g / sv ** 2) * 0.7 * prm["dx"] ** 2
    assert abs(F[0] - ref) < 1e-11 * abs(ref)
    assert np.allclose(d["force"][ks, 0], ref / 2, rtol=1e-11)


# ------------------------------------------------------------------ inlet noise

# Published SplitMix64 outputs (Steele, Lea & Flood 2014; the reference
# generator of Vigna) for the initial state 1234567: out_n = mix(state + n gamma).
SPLITMIX64_1234567 = [6457827717110365317, 3203168211198807973, 9817491932198370423,
                      4593380528125082431, 16408922859458223821]


def test_generator_matches_published_splitmix64():
    """The k-th uniform of particle id is mix(seed + (3 id + k + 1) gamma) >> 11
    scaled to [0, 1): ids 0 and 1 give the published outputs 1-3 and 4-5."""
    for n, out in enumerate(SPLITMIX64_1234567, start=1):
        pid, k = divmod(n - 1, 3)
        assert O.splitmix_uniform(1234567, pid, k) == (out >> 11) * 2.0 ** -53


def _noise_params(dim=3, amp=0.01, U=1.0):
    prm = I.base_params(dim=dim, dx=0.01, U=U)
    prm.update(flags=I.FLAG_NOISE, noise_amp=amp, noise_seed=1907)
    return prm


def test_inlet_noise_distribution():
    """Uniform per component with mean U e_x, standard deviation amp U and
    support +-sqrt(3) amp U, components uncorrelated (10^5 identities)."""
    U, amp = 1.3, 0.01
    prm = _noise_params(U=U, amp=amp)
    n = 100_000
    v = np.array([O.inlet_velocity(prm, i) for i in range(n)])
    e = v - np.array([U, 0.0, 0.0])
    half = np.sqrt(3.0) * amp * U
    assert np.abs(e).max() <= half
    assert np.abs(e).max() > 0.999 * half
    sd = amp * U
    assert np.abs(e.mean(axis=0)).max() < 5 * sd / np.sqrt(n)
    assert np.allclose(e.std(axis=0), sd, rtol=0.01)
    for c in range(3):
        assert stats.kstest(e[:, c], stats.uniform(loc=-half, scale=2 * half).cdf).pvalue > 1e-3
    cc = np.corrcoef(e.T)
    assert np.abs(cc - np.eye(3)).max() < 5 / np.sqrt(n)


def test_inlet_noise_2d_and_flag_off():
    """In 2D the third component is zero; without the flag a re-spawned
    particle takes its parent's velocity."""
    prm = _noise_params(dim=2)
    v = O.inlet_velocity(prm, 12345)
    assert v[2] == 0.0 and v[0] != 1.0 and v[1] != 0.0
    prm["flags"] = 0
    assert np.array_equal(O.inlet_velocity(prm, 12345, (0.8, 0.1, 0.0)), [0.8, 0.1, 0.0])


def test_respawned_particle_takes_noise_of_its_identity():
    """A stepped 3D duct with noise: every new inlet particle's prescribed
    velocity is the noise of its own id (parent id + 2^40)."""
    prm, s = I.config("C5", small=True)
    inl = s["type"] == I.INLET
    s["x"][inl, 0] += 0.45 * prm["dx"]  # the last inlet layer crosses in step 3
    o = O.Oracle(prm, s)
    o.step(4)
    st = o.state()
    new = st["id"] >= I.ID_GENERATION
    assert new.sum() > 10
    for k in np.flatnonzero(new):
        assert np.array_equal(st["uin"][k], O.inlet_velocity(prm, int(st["id"][k])))
    # the noise is not the parent's velocity
    assert np.abs(st["uin"][new, 1]).max() > 0.001
