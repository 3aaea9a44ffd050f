// adjoint.hip -- hand-written reverse (vector-Jacobian product) of one
// right-hand side for gfx950: force pass, neighbour-average pressure,
// boundary values (walls, hybrid outlet, inlet) and summation density.
//
// Given weights (abar, bbar, pdbar) on the fluid outputs (a, b, pdot) and a
// weight fbar on the body force, the kernels return the gradient of
//     L = sum_fluid (abar . a + bbar . b + pdbar pdot) + fbar . F_body
// with respect to positions x, velocities u, transport velocities ut,
// pressures p of the fluid, the prescribed inlet velocities and the outlet
// time averages. Everything is gather-only (each particle sums what every
// pair contributes to it; no float atomics), so results are deterministic:
//   R1  pairs:     each particle k reverses every pair term twice, once as the
//                  target (its own weights) and once as the neighbour of a
//                  fluid/body target j (j's weights);
//   R2a pbar:      the adjoint of the neighbour average pbar_i = sum_j p_j / N_i
//                  is spread to the p_j of its neighbours;
//   R2b boundary:  the adjoints of the boundary values flow back through the
//                  Shepard averages to the fluid (p, u, rho, x), to the inlet
//                  velocity and the outlet averages; then Sbar = m rhobar - V^2 Vbar;
//   R3  density:   xbar_k += sum_j (Sbar_k + Sbar_j) F_kj r_kj.
// Boundary values may also carry seeds (pseed, useed on p and u of non-fluid
// rows, jseed on J of inlet/outlet rows) from a stage update or the next
// step that reads them. Inlet/outlet particles without fluid support take J
// from the previous step's values; by the symmetry of the neighbour predicate
// no fluid particle has such a particle in its support, so only seeds reach
// them, and their adjoint goes to the previous-step values (jprevbar).
#include "sph_launch.h"

namespace sph {

template <typename T>
struct Ep {  // endpoint of a pair as the force pass sees it
    T u[3], w[3], p, rho, vol;
    int t;
};

template <typename T>
struct EpBar {  // adjoint accumulators of an endpoint
    T u[3] = {0, 0, 0}, w[3] = {0, 0, 0}, p = 0, rho = 0, vol = 0;
};

template <int DIM, typename T>
__device__ inline void load_ep(const Dev &k, const DevState &m, const Fields &R,
                               const DevDerived &o, int64_t i, Ep<T> &e)
{
    const int64_t C = k.cap;
    e.t = m.type[i];
#pragma unroll
    for (int d = 0; d < 3; ++d) e.u[d] = e.w[d] = T(0);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        e.u[d] = ld<T>(R.u, d * C + i);
        e.w[d] = ld<T>(R.ut, d * C + i) - e.u[d];
    }
    e.p = ld<T>(R.p, i);
    e.rho = ld<T>(o.rho, i);
    e.vol = ld<T>(o.vol, i);
}

// Quantities of the forward pair term shared by the fluid and body reverses.
template <int DIM, typename T>
struct PairFwd {
    T F, G, gw[3], V2, inv, pt, hm, E, D;
    __device__ inline PairFwd(const Dev &k, const T r[3], T r2, const Ep<T> &I, const Ep<T> &J,
                              T P)
    {
        const T q = T(sqrt(r2)) * T(k.inv_h);
        const T gn = T(k.gnorm);
        F = kernel_f<T>(k, q, gn);
        G = kernel_g<T>(k, q, gn, T(k.inv_h));  // (dF/dr)/|r|
#pragma unroll
        for (int d = 0; d < 3; ++d) gw[d] = F * r[d];
        V2 = I.vol * I.vol + J.vol * J.vol;
        inv = T(1) / (I.rho + J.rho);
        pt = (J.rho * (I.p - P) + I.rho * (J.p - P)) * inv;
        hm = T(2) * I.rho * J.rho * inv;
        E = r2 + T(k.eta_h2);
        D = F * r2 / E;
    }
};

// From the adjoints of V2, pt, hm, D, F and gw to the endpoints and r.
template <int DIM, typename T>
__device__ inline void pair_tail(const Dev &k, const T r[3], T r2, const Ep<T> &I,
                                 const Ep<T> &J, T P, const PairFwd<DIM, T> &f, T V2b, T ptb,
                                 T hmb, T Db, T Fb, const T gwb[3], EpBar<T> &Ib, EpBar<T> &Jb,
                                 T &Pb, T rb[3])
{
    Ib.vol += T(2) * I.vol * V2b;
    Jb.vol += T(2) * J.vol * V2b;
    Ib.p += ptb * J.rho * f.inv;
    Jb.p += ptb * I.rho * f.inv;
    Pb -= ptb;  // d pt / d P = -(rho_i + rho_j) / (rho_i + rho_j)
    Ib.rho += ptb * ((J.p - P) - f.pt) * f.inv + hmb * (T(2) * J.rho - f.hm) * f.inv;
    Jb.rho += ptb * ((I.p - P) - f.pt) * f.inv + hmb * (T(2) * I.rho - f.hm) * f.inv;
    Fb += Db * r2 / f.E;
    const T r2b = Db * f.F * T(k.eta_h2) / (f.E * f.E);
#pragma unroll
    for (int d = 0; d < DIM; ++d) Fb += gwb[d] * r[d];
#pragma unroll
    for (int d = 0; d < DIM; ++d) rb[d] += f.F * gwb[d] + Fb * f.G * r[d] + T(2) * r2b * r[d];
}

// Reverse of the fluid-target pair term (target I, neighbour J, r = x_I - x_J)
// for output weights ab (on a), bb (on b), pdb (on pdot).
template <int DIM, typename T>
__device__ inline void pair_adj_fluid(const Dev &k, const T r[3], T r2, const Ep<T> &I,
                                      const Ep<T> &J, T P, const T ab[3], const T bb[3], T pdb,
                                      EpBar<T> &Ib, EpBar<T> &Jb, T &Pb, T rb[3])
{
    const PairFwd<DIM, T> f(k, r, r2, I, J, P);
    const T nu = T(k.nu), nud = T(k.nu_damp), im = T(k.inv_mass), pbg = T(k.pb);
    T si = T(0), sj = T(0);
    const bool jfl = J.t == SPH_FLUID;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        si += I.w[d] * f.gw[d];
        if (jfl) sj += J.w[d] * f.gw[d];
    }
    const bool cv = J.t != SPH_WALL_SLIP;
    const T visc = cv ? f.hm * nu * f.D : T(0);
    const T ff = f.V2 * im;
    const bool wall = is_wall(J.t);
    T udiv = T(0), ujd[3] = {0, 0, 0}, A[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        ujd[d] = wall ? T(0) : J.u[d];
        udiv += (I.u[d] - ujd[d]) * f.gw[d];
        A[d] = -f.pt * f.gw[d] + T(0.5) * (I.rho * I.u[d] * si + J.rho * J.u[d] * sj) +
               visc * (I.u[d] - J.u[d]);
    }
    // a_I += ff * A
    T ffb = T(0), Av[3] = {0, 0, 0}, ptb = T(0), gwb[3] = {0, 0, 0}, uiAv = T(0), ujAv = T(0),
      viscb = T(0);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        ffb += ab[d] * A[d];
        Av[d] = ff * ab[d];
        ptb -= Av[d] * f.gw[d];
        gwb[d] = -f.pt * Av[d];
        uiAv += I.u[d] * Av[d];
        ujAv += J.u[d] * Av[d];
        viscb += Av[d] * (I.u[d] - J.u[d]);
    }
    const T sib = T(0.5) * I.rho * uiAv, sjb = T(0.5) * J.rho * ujAv;
    Ib.rho += T(0.5) * si * uiAv;
    Jb.rho += T(0.5) * sj * ujAv;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        Ib.u[d] += T(0.5) * I.rho * si * Av[d] + visc * Av[d];
        Jb.u[d] += T(0.5) * J.rho * sj * Av[d] - visc * Av[d];
    }
    // b_I += -(pb/m) V2 gw
    T V2b = T(0);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        V2b -= pbg * im * bb[d] * f.gw[d];
        gwb[d] -= pbg * im * f.V2 * bb[d];
    }
    // pdot_I += m (rho_I / rho_J) c^2 udiv + ff hm nu_d D (p_I - p_J)
    const T c1 = T(k.mass) * T(k.c2) / J.rho;
    Ib.rho += pdb * c1 * udiv;
    Jb.rho -= pdb * c1 * I.rho * udiv / J.rho;
    const T udivb = pdb * c1 * I.rho;
    const T dp = I.p - J.p;
    ffb += pdb * f.hm * nud * f.D * dp;
    T hmb = pdb * ff * nud * f.D * dp;
    T Db = pdb * ff * f.hm * nud * dp;
    Ib.p += pdb * ff * f.hm * nud * f.D;
    Jb.p -= pdb * ff * f.hm * nud * f.D;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        Ib.u[d] += udivb * f.gw[d];
        if (!wall) Jb.u[d] -= udivb * f.gw[d];
        gwb[d] += udivb * (I.u[d] - ujd[d]) + sib * I.w[d] + (jfl ? sjb * J.w[d] : T(0));
        Ib.w[d] += sib * f.gw[d];
        if (jfl) Jb.w[d] += sjb * f.gw[d];
    }
    if (cv) {
        hmb += viscb * nu * f.D;
        Db += viscb * f.hm * nu;
    }
    V2b += ffb * im;
    T Fb = T(0);
    pair_tail<DIM, T>(k, r, r2, I, J, P, f, V2b, ptb, hmb, Db, Fb, gwb, Ib, Jb, Pb, rb);
}

// Reverse of the body-force pair term (body I, fluid J) for the weight fb.
template <int DIM, typename T>
__device__ inline void pair_adj_body(const Dev &k, const T r[3], T r2, const Ep<T> &I,
                                     const Ep<T> &J, T P, const T fb[3], EpBar<T> &Ib,
                                     EpBar<T> &Jb, T &Pb, T rb[3])
{
    const PairFwd<DIM, T> f(k, r, r2, I, J, P);
    const T nu = T(k.nu);
    T V2b = T(0), ptb = T(0), gwb[3] = {0, 0, 0}, du_av = T(0);
    T Av[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const T du = I.u[d] - J.u[d];
        V2b += fb[d] * (-f.pt * f.gw[d] + f.hm * nu * f.D * du);
        Av[d] = f.V2 * fb[d];
        ptb -= Av[d] * f.gw[d];
        gwb[d] = -f.pt * Av[d];
        du_av += Av[d] * du;
        Ib.u[d] += f.hm * nu * f.D * Av[d];
        Jb.u[d] -= f.hm * nu * f.D * Av[d];
    }
    const T hmb = nu * f.D * du_av, Db = f.hm * nu * du_av;
    T Fb = T(0);
    pair_tail<DIM, T>(k, r, r2, I, J, P, f, V2b, ptb, hmb, Db, Fb, gwb, Ib, Jb, Pb, rb);
}

template <typename T>
__device__ inline T ldw(const void *p, int64_t i)
{
    return p ? ld<T>(p, i) : T(0);
}

// Lane groups: G lanes per particle (the force pass's choice), each lane a
// subset of the neighbours; per-particle sums are reduced with lane shuffles
// and written by lane 0. Blocks map to the XCDs in contiguous slabs.
template <int G>
__device__ inline int64_t adj_row(int64_t n, int &lane)
{
    constexpr int PB = kBlock / G;
    lane = threadIdx.x & (G - 1);
    const int64_t lb = xcd_block((n + PB - 1) / PB);
    const int64_t i = lb * PB + threadIdx.x / G;
    return lb < 0 || i >= n ? -1 : i;
}

// Neighbour slots q0, q0 + G, q0 + 2G, q0 + 3G of row i, read together so
// that the loads which depend on them go out in one round trip: ok[u] says
// the slot exists and holds a valid row (an invalid row raises the error
// word), js[u] is that row or, where not ok, row i itself (always valid, so
// dependent loads need no branch).
constexpr int kAdjBatch = 4;
template <int G>
__device__ inline void adj_slots(const DevNlist &nl, int64_t i, int cnt, int q0, int64_t n,
                                 uint32_t *err, int32_t jj[kAdjBatch], bool ok[kAdjBatch],
                                 int32_t js[kAdjBatch])
{
#pragma unroll
    for (int u = 0; u < kAdjBatch; ++u) {
        const int q = q0 + u * G;
        jj[u] = q < cnt ? nl.nbr[i * nl.maxnb + q] : int32_t(i);
    }
#pragma unroll
    for (int u = 0; u < kAdjBatch; ++u) {
        const bool in = q0 + u * G < cnt;
        const bool bad = bad_index(jj[u], n);
        if (in && bad) raise_error(err, SPH_ERR_CELL_RANGE);
        ok[u] = in && !bad;
        js[u] = ok[u] ? jj[u] : int32_t(i);
    }
}

// R1: pair reverses, gathered per particle.
template <int DIM, typename T, int G>
__global__ void __launch_bounds__(kBlock) k_adj_pairs(Dev k, DevState m, Fields R, DevNlist nl,
                                                      DevDerived o, DevAdj A, const float *off,
                                                      const uint32_t *cpos, uint32_t *err)
{
    int lane;
    const int64_t n = *m.n;
    const int64_t i = adj_row<G>(n, lane);
    if (i < 0) return;
    const int64_t C = k.cap;
    Ep<T> K;
    load_ep<DIM, T>(k, m, R, o, i, K);
    const T PK = ld<T>(o.pavg, i);
    T abK[3] = {0, 0, 0}, bbK[3] = {0, 0, 0}, pdbK = T(0), fbar[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) fbar[d] = T(A.fbar[d]);
    if (K.t == SPH_FLUID) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            abK[d] = ldw<T>(A.abar, d * C + i);
            bbK[d] = ldw<T>(A.bbar, d * C + i);
        }
        pdbK = ldw<T>(A.pdbar, i);
    }
    Sep<DIM, T> sep;
    sep.load_i(k, R, off, cpos, i);
    EpBar<T> Kb;
    T Pb = T(0), xb[3] = {0, 0, 0};
    // without weights on the pair outputs (the boundary-values reverse alone)
    // only the seeds pass through
    const bool weighted = A.abar || A.bbar || A.pdbar || A.fbar[0] != 0.0 || A.fbar[1] != 0.0 ||
                          A.fbar[2] != 0.0;
    const int cnt = weighted ? nl.count[i] : 0;
    bool nonfluid = false;  // a neighbour that is not fluid (bflag)
    for (int q = lane; q < cnt; q += G) {
        const int32_t j = nl.nbr[i * nl.maxnb + q];
        if (bad_index(j, n)) {
            raise_error(err, SPH_ERR_CELL_RANGE);
            continue;
        }
        if (j == i) continue;
        Ep<T> J;
        load_ep<DIM, T>(k, m, R, o, j, J);
        nonfluid = nonfluid || J.t != SPH_FLUID;
        T r[3], rn[3];
        const T r2 = sep.get(k, R, off, cpos, j, r);
#pragma unroll
        for (int d = 0; d < 3; ++d) rn[d] = -r[d];
        EpBar<T> dummy;
        T Pdummy = T(0);
        // i as the target
        if (K.t == SPH_FLUID || (K.t == SPH_BODY && J.t == SPH_FLUID)) {
            T rb[3] = {0, 0, 0};
            if (K.t == SPH_FLUID)
                pair_adj_fluid<DIM, T>(k, r, r2, K, J, PK, abK, bbK, pdbK, Kb, dummy, Pb, rb);
            else
                pair_adj_body<DIM, T>(k, r, r2, K, J, PK, fbar, Kb, dummy, Pb, rb);
#pragma unroll
            for (int d = 0; d < DIM; ++d) xb[d] += rb[d];
        }
        // i as the neighbour of target j
        if (J.t == SPH_FLUID || (J.t == SPH_BODY && K.t == SPH_FLUID)) {
            const T PJ = ld<T>(o.pavg, j);
            T rb[3] = {0, 0, 0};
            if (J.t == SPH_FLUID) {
                T abJ[3] = {0, 0, 0}, bbJ[3] = {0, 0, 0};
#pragma unroll
                for (int d = 0; d < DIM; ++d) {
                    abJ[d] = ldw<T>(A.abar, d * C + j);
                    bbJ[d] = ldw<T>(A.bbar, d * C + j);
                }
                pair_adj_fluid<DIM, T>(k, rn, r2, J, K, PJ, abJ, bbJ, ldw<T>(A.pdbar, j), dummy, Kb,
                                       Pdummy, rb);
            } else {
                pair_adj_body<DIM, T>(k, rn, r2, J, K, PJ, fbar, dummy, Kb, Pdummy, rb);
            }
#pragma unroll
            for (int d = 0; d < DIM; ++d) xb[d] -= rb[d];
        }
    }
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        xb[d] = gsum<G>(xb[d]);
        Kb.u[d] = gsum<G>(Kb.u[d]);
        Kb.w[d] = gsum<G>(Kb.w[d]);
    }
    Kb.p = gsum<G>(Kb.p);
    Kb.rho = gsum<G>(Kb.rho);
    Kb.vol = gsum<G>(Kb.vol);
    Pb = gsum<G>(Pb);
    const double nf = gsum<G>(nonfluid ? 1.0 : 0.0);
    if (lane != 0) return;
    // without the walk (no weights) the neighbours are unknown: flag the row
    if (A.bflag) A.bflag[i] = (!weighted || nf > 0.0) ? 1 : 0;
    // boundary values may carry adjoints from outside this right-hand side
    // (a stage update that reads them)
    const bool seeded = K.t != SPH_FLUID;
    // the seeds are read before any store (the stores could alias them)
    double us[3] = {0, 0, 0}, ps = 0.0;
    if (seeded && A.useed)
#pragma unroll
        for (int d = 0; d < DIM; ++d) us[d] = A.useed[d * C + i];
    if (seeded && A.pseed) ps = A.pseed[i];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        A.xbar[d * C + i] = double(xb[d]);
        A.ubar[d * C + i] = double(Kb.u[d]) + us[d];
        A.wbar[d * C + i] = double(Kb.w[d]);
    }
    A.pbar[i] = double(Kb.p) + ps;
    A.rhobar[i] = double(Kb.rho);
    A.volbar[i] = double(Kb.vol);
    A.Pbar[i] = double(Pb);
}

// R2a: pbar_i = (1/N_i) sum_{j in N(i)} p_j  ->  pbar_j += Pbar_i / N_i, for
// fluid targets i (body rows take p~ about zero: no neighbour average).
template <int DIM, int G>
__global__ void __launch_bounds__(kBlock) k_adj_pavg(Dev k, DevState m, DevNlist nl, DevAdj A,
                                                     uint32_t *err)
{
    int lane;
    const int64_t n = *m.n;
    const int64_t i = adj_row<G>(n, lane);
    if (i < 0) return;
    if (k.flags & SPH_FLAG_NO_PAVG) return;
    double acc = 0.0;
    const int cnt = nl.count[i];
    for (int q0 = lane; q0 < cnt; q0 += kAdjBatch * G) {
        int32_t jj[kAdjBatch], js[kAdjBatch];
        bool ok[kAdjBatch];
        adj_slots<G>(nl, i, cnt, q0, n, err, jj, ok, js);
        int tj[kAdjBatch], cj[kAdjBatch];
        double pj[kAdjBatch];
#pragma unroll
        for (int u = 0; u < kAdjBatch; ++u) {
            tj[u] = m.type[js[u]];
            pj[u] = A.Pbar[js[u]];
            cj[u] = nl.count[js[u]];
        }
#pragma unroll
        for (int u = 0; u < kAdjBatch; ++u)
            if (ok[u] && tj[u] == SPH_FLUID) acc += pj[u] / double(cj[u]);
    }
    acc = gsum<G>(acc);
    if (lane == 0) A.pbar[i] += acc;
}

// Adjoint of boundary particle b's characteristic values J = (J1, J2, J3)
// (stored as jcur[0..2]) from the adjoints of its pressure and velocity and a
// seed on J itself (J becomes the next step's previous-step value). Outlet:
// p = <p> + (J2 + J3)/2, u = <u> + (J2 - J3)/(2 rho0 c) (eq:acou) with J3
// forced to zero when J comes from the Shepard sums; inlet: p = J3.
struct BndIn {
    int t;
    double S, pbar, ubar[3], p, u[3], J[3], Jb[3], uin0;
};

// Reverse of the Shepard weight W_bf of boundary particle b and fluid f
// given the adjoints of b's values: returns Wbar and adds the fluid-side
// adjoints (p, u_x, rho, averages) and the inlet velocity adjoint of b.
template <int DIM>
__device__ inline double bnd_weight_adj(const Dev &k, const BndIn &b, double w, double pf,
                                        const double uf[3], double rhof, const double avgf[4],
                                        double &pfb, double ufb[3], double &rhofb,
                                        double avgfb[4], double &uinb0)
{
    if (is_wall(b.t)) {
        pfb += b.pbar * w / b.S;
        double Wb = b.pbar * (pf - b.p);
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            ufb[d] -= b.ubar[d] * w / b.S;
            Wb -= b.ubar[d] * (uf[d] + b.u[d]);
        }
        return Wb / b.S;
    }
    if (b.t == SPH_OUTLET) {
        // J1_f = -c^2 (rho_f - rho0) + dp, J2_f = rho_f c du + dp (eq:characteristic-vars)
        const double du = uf[0] - avgf[0], dp = pf - avgf[DIM];
        const double J1f = -k.c2 * (rhof - k.rho0) + dp;
        const double J2f = rhof * k.c * du + dp;
        const double J1fb = b.Jb[0] * w / b.S, J2fb = b.Jb[1] * w / b.S;
        rhofb += J2fb * k.c * du - J1fb * k.c2;
        ufb[0] += J2fb * rhof * k.c;
        pfb += J1fb + J2fb;
        avgfb[0] -= J2fb * rhof * k.c;
        avgfb[DIM] -= J1fb + J2fb;
        return (b.Jb[0] * (J1f - b.J[0]) + b.Jb[1] * (J2f - b.J[1])) / b.S;
    }
    // inlet: J3_f = -rho_f c (u_f - u_in,b) + p_f
    const double J3f = -rhof * k.c * (uf[0] - b.uin0) + pf;
    const double J3fb = b.Jb[2] * w / b.S;
    rhofb -= J3fb * k.c * (uf[0] - b.uin0);
    ufb[0] -= J3fb * rhof * k.c;
    pfb += J3fb;
    uinb0 += J3fb * rhof * k.c;
    return b.Jb[2] * (J3f - b.J[2]) / b.S;
}

template <int DIM, typename T>
__device__ inline void load_bnd(const Dev &k, const DevState &m, const Fields &R,
                                const DevDerived &o, const DevAdj &A, int64_t b, BndIn &B)
{
    const int64_t C = k.cap;
    B.t = m.type[b];
    B.S = o.sfl[b];
    B.pbar = A.pbar[b];
    B.p = double(ld<T>(R.p, b));
#pragma unroll
    for (int d = 0; d < 3; ++d) B.ubar[d] = B.u[d] = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        B.ubar[d] = A.ubar[d * C + b];
        B.u[d] = double(ld<T>(R.u, d * C + b));
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        B.J[a] = o.jcur[a * C + b];
        B.Jb[a] = A.jseed ? A.jseed[a * C + b] : 0.0;
    }
    if (B.t == SPH_OUTLET) {
        const double ub = B.ubar[0] / (2.0 * k.rho0 * k.c);
        B.Jb[1] += 0.5 * B.pbar + ub;
        B.Jb[2] = B.S > 0.0 ? 0.0 : B.Jb[2] + 0.5 * B.pbar - ub;
    } else if (B.t == SPH_INLET) {
        B.Jb[2] += B.pbar;
    }
    B.uin0 = m.uin[b];
}

// R2b: boundary reverses, then Sbar = m rhobar - V^2 Vbar. A boundary row
// without fluid support took J from the previous-step values of same-kind
// neighbours (or its own): its J adjoint is split over those, here as
// jg = Jbar / M for the neighbours to gather in R3 (or straight into its own
// jprevbar when M = 0).
template <int DIM, typename T, int G>
__global__ void __launch_bounds__(kBlock) k_adj_bnd(Dev k, DevState m, Fields R, DevNlist nl,
                                                    DevDerived o, DevAdj A, uint32_t *err)
{
    int lane;
    const int64_t n = *m.n;
    const int64_t i = adj_row<G>(n, lane);
    if (i < 0) return;
    const int64_t C = k.cap;
    const int t = m.type[i];
    const int cnt = nl.count[i];
    // per-lane parts of the sums over neighbours
    double xi[3] = {0, 0, 0}, dx[3] = {0, 0, 0}, du[3] = {0, 0, 0}, davg[4] = {0, 0, 0, 0};
    double dp = 0.0, drho = 0.0, duin0 = 0.0, M = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) xi[d] = R.x[d * C + i];
    const bool red = o.sfl[i] > 0.0;
    const bool blue_io = !red && (t == SPH_INLET || t == SPH_OUTLET) && A.jprevbar;
    // a fluid row without a non-fluid neighbour (bflag 0, from the pair
    // reverse) has no boundary row to gather from: its sums stay zero
    const int fcnt = (!A.bflag || A.bflag[i]) ? cnt : 0;
    if (t == SPH_FLUID) {
        const double pf = double(ld<T>(R.p, i)), rhof = double(ld<T>(o.rho, i));
        double uf[3] = {0, 0, 0}, avgf[4] = {0, 0, 0, 0};
#pragma unroll
        for (int d = 0; d < DIM; ++d) uf[d] = double(ld<T>(R.u, d * C + i));
#pragma unroll
        for (int c = 0; c <= DIM; ++c) avgf[c] = m.avg[c * C + i];
        for (int q0 = lane; q0 < fcnt; q0 += kAdjBatch * G) {
            int32_t jj[kAdjBatch], js[kAdjBatch];
            bool ok[kAdjBatch];
            adj_slots<G>(nl, i, cnt, q0, n, err, jj, ok, js);
            int tb[kAdjBatch];
            double sb[kAdjBatch];
#pragma unroll
            for (int u = 0; u < kAdjBatch; ++u) {
                tb[u] = m.type[js[u]];
                sb[u] = o.sfl[js[u]];
            }
            // boundary neighbours with fluid support, in slot order
            uint32_t hit = 0;
#pragma unroll
            for (int u = 0; u < kAdjBatch; ++u)
                if (ok[u] && tb[u] != SPH_FLUID && sb[u] > 0.0) hit |= 1u << u;
            while (hit) {
                const int u = __builtin_ctz(hit);
                hit &= hit - 1;
                const int32_t b = u == 0 ? jj[0] : u == 1 ? jj[1] : u == 2 ? jj[2] : jj[3];
                BndIn B;
                load_bnd<DIM, T>(k, m, R, o, A, b, B);
                double xj[3] = {0, 0, 0}, r[3];
#pragma unroll
                for (int d = 0; d < DIM; ++d) xj[d] = R.x[d * C + b];
                const double r2 = dist2_exact<DIM>(k, xj, xi, r);  // r = x_b - x_f
                const double q2 = sqrt(r2) * k.inv_h;
                const double w = kernel_w<double>(k, q2, k.wnorm);
                const double F = kernel_f<double>(k, q2, k.gnorm);
                double dummy_uin = 0.0;
                const double Wb = bnd_weight_adj<DIM>(k, B, w, pf, uf, rhof, avgf, dp, du, drho,
                                                      davg, dummy_uin);
#pragma unroll
                for (int d = 0; d < DIM; ++d) dx[d] -= Wb * F * r[d];
            }
        }
    } else if (red) {
        BndIn B;
        load_bnd<DIM, T>(k, m, R, o, A, i, B);
        for (int q0 = lane; q0 < cnt; q0 += kAdjBatch * G) {
            int32_t jj[kAdjBatch], js[kAdjBatch];
            bool ok[kAdjBatch];
            adj_slots<G>(nl, i, cnt, q0, n, err, jj, ok, js);
            // every fluid value of the batch in one round trip
            int tf[kAdjBatch];
            double xf[kAdjBatch][3], pf[kAdjBatch], rhof[kAdjBatch], uf[kAdjBatch][3],
                avgf[kAdjBatch][4];
#pragma unroll
            for (int u = 0; u < kAdjBatch; ++u) {
                const int32_t f = js[u];
                tf[u] = m.type[f];
                pf[u] = double(ld<T>(R.p, f));
                rhof[u] = double(ld<T>(o.rho, f));
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    xf[u][d] = d < DIM ? R.x[d * C + f] : 0.0;
                    uf[u][d] = d < DIM ? double(ld<T>(R.u, d * C + f)) : 0.0;
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) avgf[u][c] = c <= DIM ? m.avg[c * C + f] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kAdjBatch; ++u) {
                if (!ok[u] || tf[u] != SPH_FLUID) continue;
                double r[3];
                const double r2 = dist2_exact<DIM>(k, xi, xf[u], r);  // r = x_b - x_f
                const double q2 = sqrt(r2) * k.inv_h;
                const double w = kernel_w<double>(k, q2, k.wnorm);
                const double F = kernel_f<double>(k, q2, k.gnorm);
                double sink_u[3] = {0, 0, 0}, sink_avg[4] = {0, 0, 0, 0}, sink_p = 0.0,
                       sink_rho = 0.0;
                const double Wb = bnd_weight_adj<DIM>(k, B, w, pf[u], uf[u], rhof[u], avgf[u],
                                                      sink_p, sink_u, sink_rho, sink_avg, duin0);
#pragma unroll
                for (int d = 0; d < DIM; ++d) dx[d] += Wb * F * r[d];
            }
        }
    } else if (blue_io) {
        // no fluid support: J = mean of the previous-step values of same-kind
        // neighbours that had support (eq:average_old), else the own value
        for (int q = lane; q < cnt; q += G) {
            const int32_t j = nl.nbr[i * nl.maxnb + q];
            if (bad_index(j, n)) continue;
            if (m.type[j] == t && m.red_prev[j]) M += 1.0;
        }
    }
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        dx[d] = gsum<G>(dx[d]);
        du[d] = gsum<G>(du[d]);
    }
#pragma unroll
    for (int c = 0; c <= DIM; ++c) davg[c] = gsum<G>(davg[c]);
    dp = gsum<G>(dp);
    drho = gsum<G>(drho);
    duin0 = gsum<G>(duin0);
    M = gsum<G>(M);
    if (lane != 0) return;
    double xb[3] = {0, 0, 0}, ub[3] = {0, 0, 0}, avgb[4] = {0, 0, 0, 0}, uinb[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        xb[d] = A.xbar[d * C + i] + dx[d];
        ub[d] = A.ubar[d * C + i] + du[d];
    }
#pragma unroll
    for (int c = 0; c <= DIM; ++c) avgb[c] = davg[c];
    uinb[0] = duin0;
    const double pb = A.pbar[i] + dp, rhob = A.rhobar[i] + drho;
    double jg[3] = {0, 0, 0}, jown[3] = {0, 0, 0};
    if (blue_io) {
        BndIn B;
        load_bnd<DIM, T>(k, m, R, o, A, i, B);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (M > 0.0) jg[a] = B.Jb[a] / M;
            else jown[a] = B.Jb[a];
        }
    }
    if (t == SPH_INLET) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) uinb[d] += ub[d];  // u = u_in
    } else if (t == SPH_OUTLET) {
        // u_o = <u> + u_ac, v_o = <v>, p_o = <p> + p_ac
#pragma unroll
        for (int d = 0; d < DIM; ++d) avgb[d] += ub[d];
        avgb[DIM] += pb;
    }
    const double vol = double(ld<T>(o.vol, i));
    const double Sb = k.mass * rhob - vol * vol * A.volbar[i];
    // boundary rows' pbar and ubar are read by their fluid neighbours in this
    // launch, so only fluid rows write theirs back
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        A.xbar[d * C + i] = xb[d];
        if (t == SPH_FLUID) A.ubar[d * C + i] = ub[d];
        A.uinbar[d * C + i] = uinb[d];
    }
#pragma unroll
    for (int c = 0; c <= DIM; ++c) A.avgbar[c * C + i] = avgb[c];
    if (A.jprevbar) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            A.jg[a * C + i] = jg[a];
            A.jprevbar[a * C + i] = jown[a];
        }
    }
    if (t == SPH_FLUID) A.pbar[i] = pb;
    A.rhobar[i] = rhob;
    A.Sbar[i] = Sb;
}

// R3: density reverse, xbar_k += sum_j (Sbar_k + Sbar_j) F_kj r_kj; final
// velocity adjoints (u enters directly and through w = ut - u).
template <int DIM, typename T, int G>
__global__ void __launch_bounds__(kBlock) k_adj_dens(Dev k, DevState m, Fields R, DevNlist nl,
                                                     DevAdj A, uint32_t *err)
{
    int lane;
    const int64_t n = *m.n;
    const int64_t i = adj_row<G>(n, lane);
    if (i < 0) return;
    const int64_t C = k.cap;
    const int t = m.type[i];
    double xi[3] = {0, 0, 0}, dx[3] = {0, 0, 0}, g[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) xi[d] = R.x[d * C + i];
    const double Si = A.Sbar[i];
    // previous-step values of i read by unsupported same-kind neighbours
    // (i itself included), reverse of the mean taken in R2b
    const bool gather_j = A.jprevbar && (t == SPH_INLET || t == SPH_OUTLET) && m.red_prev[i];
    const int cnt = nl.count[i];
    for (int q0 = lane; q0 < cnt; q0 += kAdjBatch * G) {
        int32_t jj[kAdjBatch], js[kAdjBatch];
        bool ok[kAdjBatch];
        adj_slots<G>(nl, i, cnt, q0, n, err, jj, ok, js);
        double xs[kAdjBatch][3], Sj[kAdjBatch];
#pragma unroll
        for (int u = 0; u < kAdjBatch; ++u) {
#pragma unroll
            for (int d = 0; d < 3; ++d) xs[u][d] = d < DIM ? R.x[d * C + js[u]] : 0.0;
            Sj[u] = A.Sbar[js[u]];
        }
#pragma unroll
        for (int u = 0; u < kAdjBatch; ++u) {
            if (!ok[u]) continue;
            const int32_t j = jj[u];
            if (gather_j && m.type[j] == t) {
#pragma unroll
                for (int a = 0; a < 3; ++a) g[a] += A.jg[a * C + j];
            }
            if (j == i) continue;
            double r[3];
            const double r2 = dist2_exact<DIM>(k, xi, xs[u], r);
            const double F = kernel_f<double>(k, sqrt(r2) * k.inv_h, k.gnorm);
            const double s = (Si + Sj[u]) * F;
#pragma unroll
            for (int d = 0; d < DIM; ++d) dx[d] += s * r[d];
        }
    }
#pragma unroll
    for (int d = 0; d < DIM; ++d) dx[d] = gsum<G>(dx[d]);
#pragma unroll
    for (int a = 0; a < 3; ++a) g[a] = gsum<G>(g[a]);
    if (lane != 0) return;
    const bool fl = t == SPH_FLUID;
    // every read of the write-out before its first store (they could alias)
    double xb[3] = {0, 0, 0}, wb[3] = {0, 0, 0}, ub[3] = {0, 0, 0}, jb[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        xb[d] = A.xbar[d * C + i];
        wb[d] = A.wbar[d * C + i];
        if (fl) ub[d] = A.ubar[d * C + i];
    }
    if (gather_j)
#pragma unroll
        for (int a = 0; a < 3; ++a) jb[a] = A.jprevbar[a * C + i];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        A.xbar[d * C + i] = xb[d] + dx[d];
        A.utbar[d * C + i] = fl ? wb[d] : 0.0;
        if (fl) A.ubar[d * C + i] = ub[d] - wb[d];
    }
    if (gather_j) {
#pragma unroll
        for (int a = 0; a < 3; ++a) A.jprevbar[a * C + i] = jb[a] + g[a];
    }
}

// ------------------------------------------------------------------ launchers
template <int DIM, typename T, int G>
static void rhs_adjoint_g(const Dev &k, const DevState &m, const Fields &R, const DevNlist &nl,
                          const DevDerived &o, const DevAdj &A, const float *off,
                          const uint32_t *cpos, uint32_t *err, hipStream_t s)
{
    const dim3 g(xcd_grid((k.cap + kBlock / G - 1) / (kBlock / G))), b(kBlock);
    hipLaunchKernelGGL((k_adj_pairs<DIM, T, G>), g, b, 0, s, k, m, R, nl, o, A, off, cpos, err);
    hipLaunchKernelGGL((k_adj_pavg<DIM, G>), g, b, 0, s, k, m, nl, A, err);
    hipLaunchKernelGGL((k_adj_bnd<DIM, T, G>), g, b, 0, s, k, m, R, nl, o, A, err);
    hipLaunchKernelGGL((k_adj_dens<DIM, T, G>), g, b, 0, s, k, m, R, nl, A, err);
}

template <int DIM, typename T>
static void rhs_adjoint_dt(const Dev &k, const DevState &m, const Fields &R, const DevNlist &nl,
                           const DevDerived &o, const DevAdj &A, const float *off,
                           const uint32_t *cpos, uint32_t *err, hipStream_t s)
{
    switch (force_group(k)) {
    case 1: rhs_adjoint_g<DIM, T, 1>(k, m, R, nl, o, A, off, cpos, err, s); break;
    case 2: rhs_adjoint_g<DIM, T, 2>(k, m, R, nl, o, A, off, cpos, err, s); break;
    case 4: rhs_adjoint_g<DIM, T, 4>(k, m, R, nl, o, A, off, cpos, err, s); break;
    case 8: rhs_adjoint_g<DIM, T, 8>(k, m, R, nl, o, A, off, cpos, err, s); break;
    case 16: rhs_adjoint_g<DIM, T, 16>(k, m, R, nl, o, A, off, cpos, err, s); break;
    default: rhs_adjoint_g<DIM, T, 32>(k, m, R, nl, o, A, off, cpos, err, s); break;
    }
}

void launch_rhs_adjoint(const Dev &k, const DevState &m, const Fields &R, const DevNlist &nl,
                        const DevDerived &o, const DevAdj &A, const float *off,
                        const uint32_t *cpos, uint32_t *err, hipStream_t s)
{
    if (k.dim == 2 && k.prec == SPH_FP64)
        rhs_adjoint_dt<2, double>(k, m, R, nl, o, A, off, cpos, err, s);
    else if (k.dim == 3 && k.prec == SPH_FP64)
        rhs_adjoint_dt<3, double>(k, m, R, nl, o, A, off, cpos, err, s);
    else if (k.dim == 2)
        rhs_adjoint_dt<2, float>(k, m, R, nl, o, A, off, cpos, err, s);
    else
        rhs_adjoint_dt<3, float>(k, m, R, nl, o, A, off, cpos, err, s);
}

}  // namespace sph
