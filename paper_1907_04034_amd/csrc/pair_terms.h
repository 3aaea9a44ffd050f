// pair_terms.h -- device pieces shared by the pair kernels of libsph (the
// gather kernels of pairs.hip and the LDS-tiled kernels of tiles.hip):
// per-lane accumulation, the FP32 neighbour record, one neighbour's data,
// the pair terms of the force pass and the fused RK2 stage updates. Both
// kernel families evaluate every formula through these functions, so their
// arithmetic is the same operation for operation.
#pragma once

#include "sph_dev.h"

namespace sph {

// ----------------------------------------------------------------- helpers
template <int DIM>
struct Grp {
    static constexpr int G = DIM == 2 ? 16 : 32;   // lanes per target
    static constexpr int NS = DIM == 2 ? 9 : 27;   // stencil cells
    static constexpr int PER_BLOCK = kBlock / G;   // targets per block
};

// Lanes per target of the neighbour search and the force pass are template
// parameters: many lanes per target keep small systems busy (every gather of
// a target in flight at once), few lanes (down to one) spend no issue slots on
// idle lanes and cross-lane reductions when the particle count alone fills
// the chip. The host picks them from the capacity (override in sph_params).

// Per-lane accumulator and its group reduction: plain sums in FP64; in FP32
// the FP32 terms are summed in an FP64 accumulator (one conversion and one
// FP64 addition per term, which costs fewer VALU issue slots than carrying a
// compensated FP32 pair through TwoSum, and keeps more bits), rounded to FP32
// once after the group reduction.
template <typename T>
struct Acc {
    T s = T(0);
    __device__ inline void add(T v) { s += v; }
    template <int G>
    __device__ inline T reduce() { return gsum<G>(s); }
};

template <>
struct Acc<float> {
    double s = 0.0;
    __device__ inline void add(float v) { s += double(v); }
    template <int G>
    __device__ inline float reduce() { return float(gsum<G>(s)); }
};

// Writes the FP32 neighbour record of row i (lanes of the group split the
// 16-byte chunks): the cell offset (the same value as the offset array), p,
// u, w = ut - u, rho and V or S, the kind and the packed cell. (FP64 records
// are written by k_pack_rec.)
template <int DIM, typename T, int G>
__device__ inline void write_rec(const Dev &k, const DevState &m, const Fields &R, void *rec,
                                 int64_t i, T S, const double xi[3], const int c[3],
                                 uint32_t cposi, int lane)
{
    using L = Rec<DIM, T>;
    static_assert(L::F32, "FP64 records are written by k_pack_rec");
    const int64_t C = k.cap;
    T v[L::NC * L::PER];
#pragma unroll
    for (int q = 0; q < L::NC * L::PER; ++q) v[q] = T(0);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        v[L::X + d] = T(cell_offset(k, d, xi[d], c[d]));
        const T u = ld<T>(R.u, d * C + i);
        v[L::U + d] = u;
        v[L::W + d] = ld<T>(R.ut, d * C + i) - u;
    }
    v[L::P] = ld<T>(R.p, i);
    if constexpr (L::PACKED) {
        v[L::VOL] = S;
        v[L::AUX] = rec_word<T>(cposi | (kind_class(m.type[i]) << 30));
    } else {
        v[L::RHO] = T(k.mass) * S;
        v[L::VOL] = T(1) / S;
        v[L::AUX] = rec_word<T>(cposi);
        v[L::AUX + 1] = rec_word<T>(uint32_t(m.type[i]));
    }
#pragma unroll
    for (int ch = 0; ch < L::NC; ++ch)
        if ((ch & (G - 1)) == (lane & (G - 1)))
            *rec_chunk<DIM, T>(rec, C, i, ch) = Chunk<T>::make(v + ch * L::PER);
}

// ------------------------------------------------------------ stage updates
// Cell skin. The neighbour search finds every pair within 2h as long as each
// particle stays within disp_max (Euclidean) of the position it had at the
// last sort: cells are at least 2h + 2 disp_max wide, and the step path's
// candidate lists hold every pair within 2h + 2 disp_max at the binned
// positions. Half update (mode 1): the stage-1 position xs and the half
// position v must stay inside, else an error. Full update (mode 2, bin reuse
// only): ask the next bin to sort unless the new position plus one more
// step's displacement (from the start value x0) stays inside.
template <int DIM>
__device__ inline void skin_check(const Dev &k, int mode, const double xs[3], const double v[3],
                                  const double x0[3], const double xb[3], int32_t *rebin,
                                  uint32_t *err)
{
#pragma clang fp contract(off)
    double a2 = 0.0, b2 = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const double r = mode == 1 ? xs[d] : v[d];
        const double s = mode == 1 ? v[d] : x0[d];
        const double da = min_image(r - xb[d], k.periodic[d], k.L[d], k.halfL[d]);
        const double db = min_image(v[d] - (mode == 1 ? xb[d] : s), k.periodic[d], k.L[d],
                                    k.halfL[d]);
        a2 = a2 + da * da;
        b2 = b2 + db * db;
    }
    if (mode == 1) {
        const double lim2 = k.disp_max * k.disp_max;
        if (!(a2 <= lim2 && b2 <= lim2)) raise_error(err, SPH_ERR_SKIN);
    } else if (k.reuse) {
        if (!(sqrt(a2) + sqrt(b2) <= k.disp_max)) *rebin = 1;
    }
}

// The same for rows that move along x only (inlet and outlet): their
// displacement is the x offset.
__device__ inline void skin_check_x(const Dev &k, int mode, double xs, double v, double x0,
                                    double xb, int32_t *rebin, uint32_t *err)
{
#pragma clang fp contract(off)
    if (mode == 1) {
        const double ds = min_image(xs - xb, k.periodic[0], k.L[0], k.halfL[0]);
        const double dh = min_image(v - xb, k.periodic[0], k.L[0], k.halfL[0]);
        if (!(fabs(ds) <= k.disp_max && fabs(dh) <= k.disp_max)) raise_error(err, SPH_ERR_SKIN);
    } else if (k.reuse) {
        const double db = min_image(v - xb, k.periodic[0], k.L[0], k.halfL[0]);
        const double dn = min_image(v - x0, k.periodic[0], k.L[0], k.halfL[0]);
        if (!(fabs(db) + fabs(dn) <= k.disp_max)) *rebin = 1;
    }
}


// Explicit-midpoint RK2 (the integrator is the implementation's reading; the
// paper defers time stepping to the EDAC paper) with eq:transport-vel applied
// per stage and eq:advection for positions. Contraction is off so that the
// update evaluates the formula as written. Every load comes before the first
// store: the stores could alias the arrays read as far as the compiler knows,
// and a load placed after a store waits for it.
template <int DIM, typename T>
__device__ inline void stage_fluid(const Dev &k, const Fields &R, const Fields &W, int64_t i,
                                   int mode, const T ui[3], T pi, const T a[3], const T b[3],
                                   T pd, const double *xbin, int32_t *rebin, uint32_t *err)
{
#pragma clang fp contract(off)
    const int64_t C = k.cap;
    const double dt = mode == 2 ? k.dt : k.hdt;
    // stage position xs, start position xw (full update), skin reference xb,
    // start velocity u0 and, in the full update, the half-state advection
    // velocity and start pressure
    double xs[3] = {0, 0, 0}, xw[3] = {0, 0, 0}, xb[3] = {0, 0, 0}, u0[3] = {0, 0, 0},
           uth[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        xs[d] = R.x[d * C + i];
        xb[d] = xbin[d * C + i];
        if (mode == 2) {
            xw[d] = W.x[d * C + i];
            u0[d] = double(ld<T>(W.u, d * C + i));
            uth[d] = double(ld<T>(R.ut, d * C + i));
        } else {
            u0[d] = double(ui[d]);
        }
    }
    const double p0 = mode == 2 ? double(ld<T>(W.p, i)) : double(pi);
    bool fin = true;
    double xn[3] = {0, 0, 0}, un[3] = {0, 0, 0}, utn[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const double x0 = mode == 2 ? xw[d] : xs[d];
        un[d] = u0[d] + dt * double(a[d]);
        utn[d] = un[d] + dt * double(b[d]);
        const double adv = mode == 2 ? uth[d] : utn[d];
        xn[d] = x0 + dt * adv;
        fin = fin && isfinite(un[d]) && isfinite(utn[d]);
    }
    const double pn = p0 + dt * double(pd);
    fin = fin && isfinite(pn);
    double xv[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        double v = xn[d];
        if (k.periodic[d]) {
            const double hi = k.lo[d] + k.L[d];
            if (v >= hi) v -= k.L[d];
            else if (v < k.lo[d]) v += k.L[d];
        }
        xv[d] = v;
        fin = fin && isfinite(v);
        W.x[d * C + i] = v;
        st<T>(W.u, d * C + i, T(un[d]));
        st<T>(W.ut, d * C + i, T(utn[d]));
    }
    skin_check<DIM>(k, mode, xs, xv, xw, xb, rebin, err);
    st<T>(W.p, i, T(pn));
    if (!fin) raise_error(err, SPH_ERR_NONFINITE);
}

// Inlet rows move with their prescribed velocity and outlet rows along x with
// the speed of their rule (Sec. 3.4: no transverse motion); walls are fixed.
// The full update also makes the half state's boundary values the step's.
template <int DIM, typename T>
__device__ inline void stage_boundary(const Dev &k, const DevState &m, const Fields &R,
                                      const Fields &W, int64_t i, int t, int mode,
                                      const double *jcur, const double *xbin, int32_t *rebin,
                                      uint32_t *err)
{
#pragma clang fp contract(off)
    const int64_t C = k.cap;
    const double dt = mode == 2 ? k.dt : k.hdt;
    // outlet rules other than the hybrid and a mirrored inlet keep (part of)
    // the start values: the half state carries them into stage 2
    const bool keep = mode == 1 && ((t == SPH_OUTLET && k.outlet != SPH_OUTLET_HYBRID) ||
                                    (t == SPH_INLET && (k.flags & SPH_FLAG_MIRROR_INLET)));
    const bool copy = mode == 2 || keep;  // u, ut, p of R carried into W
    const bool moves = t == SPH_INLET || t == SPH_OUTLET;
    // every load before the first store (as in stage_fluid)
    double x0[3] = {0, 0, 0};
    T uc[3] = {T(0), T(0), T(0)}, utc[3] = {T(0), T(0), T(0)}, pc = T(0);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        x0[d] = mode == 2 ? W.x[d * C + i] : R.x[d * C + i];
        if (copy) {
            uc[d] = ld<T>(R.u, d * C + i);
            utc[d] = ld<T>(R.ut, d * C + i);
        }
    }
    if (copy) pc = ld<T>(R.p, i);
    double vx = 0.0, xs0 = 0.0, xb0 = 0.0;
    if (moves) {
        // outlet speed: its own x velocity, or the extrapolated fluid
        // velocity of the modified do-nothing rule
        vx = t == SPH_INLET ? m.uin[i]
             : k.outlet == SPH_OUTLET_MOD_DO_NOTHING ? jcur[i]
                                                     : double(ld<T>(R.u, i));
        xs0 = R.x[i];
        xb0 = xbin[i];
    }
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        double v = x0[d];
        if (d == 0 && moves) {
            v = x0[0] + dt * vx;
            skin_check_x(k, mode, xs0, v, x0[0], xb0, rebin, err);
            if (!isfinite(v)) raise_error(err, SPH_ERR_NONFINITE);
        }
        W.x[d * C + i] = v;
        if (copy) {
            st<T>(W.u, d * C + i, uc[d]);
            st<T>(W.ut, d * C + i, utc[d]);
        }
    }
    if (copy) st<T>(W.p, i, pc);
}

// One neighbour's data as a lane of the force pass needs it.
template <int DIM, typename T>
struct Nbr {
    int32_t j;
    int tj;
    T r[3], r2, u[3], w[3], p, rho, vol;  // w = ut - u
};

// Division and square root of the pair terms: exact in FP64; in FP32 the
// hardware reciprocal and square root (v_rcp_f32, v_sqrt_f32, within about one
// ulp) instead of the correctly rounded sequences, which cost several times the
// issue slots in this arithmetic-bound pass.
__device__ inline double pdiv(double a, double b) { return a / b; }
__device__ inline float pdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ inline double psqrt(double x) { return sqrt(x); }
__device__ inline float psqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// One neighbour's data from its record (Rec) in a few 16-byte loads (measured
// on the 4.6M-particle duct: FP32 records cut the force pass 1.67 -> 1.23 ms;
// row-major FP64 records of 128 and 80 bytes made it slower, 1.93 -> 2.11 ms,
// where the chunk-major ones of rec_chunk do not).
// fetch_nbr only issues the loads and finish_nbr does the arithmetic on them,
// so a lane that prefetches several neighbours issues every fetch before the
// first finish and their gathers overlap (a separation computed right after
// its loads makes the next neighbour's loads wait for them).
template <int DIM, typename T>
struct NbrRaw {
    using L = Rec<DIM, T>;
    T v[L::USE ? L::NC * L::PER : 1];  // the record
    double xj[L::USE ? 1 : 3];         // 2D FP64: the fields and the Shepard sum
    T u[L::USE ? 1 : 3], ut[L::USE ? 1 : 3], p, s;
    int tj;
    int32_t j;
};

template <int DIM, typename T>
__device__ inline void fetch_nbr(const Dev &k, const DevState &m, const Fields &R,
                                 const DevDerived &o, int32_t j, NbrRaw<DIM, T> &w)
{
    using L = Rec<DIM, T>;
    w.j = j;
    if constexpr (L::USE) {
#pragma unroll
        for (int ch = 0; ch < L::NC; ++ch)
            Chunk<T>::get(*rec_chunk<DIM, T>(o.rec, k.cap, j, ch), w.v + ch * L::PER);
    } else {
        const int64_t C = k.cap;
        w.tj = m.type[j];
        w.xj[2] = 0.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            w.xj[d] = R.x[d * C + j];
            w.u[d] = ld<T>(R.u, d * C + j);
            w.ut[d] = ld<T>(R.ut, d * C + j);
        }
        w.p = ld<T>(R.p, j);
        w.s = ld<T>(o.shep, j);
    }
}

template <int DIM, typename T>
__device__ inline void finish_nbr(const Dev &k, const Sep<DIM, T> &sep, const NbrRaw<DIM, T> &w,
                                  Nbr<DIM, T> &nb)
{
    using L = Rec<DIM, T>;
    const T *v = w.v;
    nb.j = w.j;
    if constexpr (L::PACKED) {
        const uint32_t word = rec_uint<T>(v[L::AUX]);
        nb.tj = class_kind(word >> 30);
        nb.r2 = sep.get_rec(k, v + L::X, word & kCellBits, nb.r);
        const T S = v[L::VOL];
        nb.rho = T(k.mass) * S;
        nb.vol = pdiv(T(1), S);
    } else if constexpr (L::F32) {
        nb.tj = int(rec_uint<T>(v[L::AUX + 1]));
        nb.r2 = sep.get_rec(k, v + L::X, rec_uint<T>(v[L::AUX]), nb.r);
        nb.rho = v[L::RHO];
        nb.vol = v[L::VOL];
    } else if constexpr (L::USE) {
        nb.tj = int(rec_uint<T>(v[L::AUX]));
        nb.r2 = sep.get_rec(k, v + L::X, nb.r);
        const T S = v[L::VOL];
        nb.rho = T(k.mass) * S;  // as the density pass forms the stored fields
        nb.vol = T(1) / S;
    } else {
        nb.tj = w.tj;
        nb.r2 = dist2_exact<DIM>(k, sep.xi, w.xj, nb.r);
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            nb.u[d] = w.u[d];
            nb.w[d] = w.ut[d] - w.u[d];
        }
        nb.p = w.p;
        nb.rho = T(k.mass) * w.s;
        nb.vol = T(1) / w.s;
        return;
    }
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        nb.u[d] = v[L::U + d];
        nb.w[d] = v[L::W + d];
    }
    nb.p = v[L::P];
}

template <int DIM, typename T>
__device__ inline void load_nbr(const Dev &k, const DevState &m, const Fields &R,
                                const DevDerived &o, const Sep<DIM, T> &sep, int32_t j,
                                Nbr<DIM, T> &nb)
{
    NbrRaw<DIM, T> w;
    fetch_nbr<DIM, T>(k, m, R, o, j, w);
    finish_nbr<DIM, T>(k, sep, w, nb);
}


// Contribution of neighbour nb to target i. The pressure of eq:tvf-p-ij-basa
// is split as p~_ij = (p_i - pbar_i) + rho_i (p_j - p_i) / (rho_i + rho_j)
// (the same value: the density weights sum to one), so a fluid target sums
// only the pair-dependent part here and g = sum_j (V_i^2 + V_j^2)/m_i grad W_ij;
// the caller adds -(p_i - pbar_i) g to the momentum rate once pbar_i, summed
// over the same pairs, is known, and forms b = -p_b g (the background term of
// eq:tvf-momentum). One sweep over the neighbours thus gives every sum, and
// each rounding error stays proportional to a pressure difference, as in the
// unsplit form. A body target takes p~ about zero (pbar = 0, the unsplit form)
// and sums the force of eq:tvf-momentum_solid in acc, which it does not use
// otherwise.
template <int DIM, typename T>
__device__ inline void pair_acc(const Dev &k, int t, const T ui[3], const T wi[3], T pi, T rhoi,
                                T vi2, const Nbr<DIM, T> &nb, Acc<T> acc[3], Acc<T> gacc[3],
                                Acc<T> &pdot)
{
    const T F = kernel_f<T>(k, psqrt(nb.r2) * T(k.inv_h), T(k.gnorm));
    T gw[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) gw[d] = F * nb.r[d];
    const T vsq = vi2 + nb.vol * nb.vol;
    const T inv_rs = pdiv(T(1), rhoi + nb.rho);
    const T hm = T(2) * rhoi * nb.rho * inv_rs;  // eta~ / nu
    const T dfac = pdiv(F * nb.r2, nb.r2 + T(k.eta_h2));
    const T nu = T(k.nu);
    if (t == SPH_FLUID) {
        const T pdif = rhoi * (nb.p - pi) * inv_rs;
        T si = T(0), sj = T(0);
#pragma unroll
        for (int d = 0; d < DIM; ++d) si += wi[d] * gw[d];
        if (nb.tj == SPH_FLUID)
#pragma unroll
            for (int d = 0; d < DIM; ++d) sj += nb.w[d] * gw[d];
        const T visc = nb.tj == SPH_WALL_SLIP ? T(0) : hm * nu * dfac;
        const T f = vsq * T(k.inv_mass);
        const bool wall = is_wall(nb.tj);
        T udiv = T(0);
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            const T aterm = T(0.5) * (rhoi * ui[d] * si + nb.rho * nb.u[d] * sj);
            acc[d].add(f * (-pdif * gw[d] + aterm + visc * (ui[d] - nb.u[d])));
            gacc[d].add(f * gw[d]);
            udiv += (ui[d] - (wall ? T(0) : nb.u[d])) * gw[d];
        }
        // m_j rho_i / rho_j of eq:p-edac is rho_i V_j: every particle has
        // mass m and V = 1/S = m/rho
        pdot.add(rhoi * nb.vol * T(k.c2) * udiv + f * (hm * T(k.nu_damp)) * dfac * (pi - nb.p));
    } else {
        const T ptil = (nb.rho * pi + rhoi * nb.p) * inv_rs;
#pragma unroll
        for (int d = 0; d < DIM; ++d)
            acc[d].add(vsq * (-ptil * gw[d] + hm * nu * dfac * (ui[d] - nb.u[d])));
    }
}

// The group's sums: for a fluid target the momentum and background rates
// a = sum_j(...) - (p_i - pbar_i) g and b = -p_b g, formed in FP64 and
// rounded once to the field type; for a body target the body force fb (a and
// b zero).
template <int DIM, typename T, int G>
__device__ inline void finish_rates(const Dev &k, int t, Acc<T> acc[3], Acc<T> gacc[3],
                                    double dp, T a[3], T b[3], double fb[3])
{
    const bool body = t == SPH_BODY;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const double s = gsum<G>(acc[d].s);
        const double g = gsum<G>(gacc[d].s);
        fb[d] = body ? s : 0.0;
        a[d] = body ? T(0) : T(s - dp * g);
        b[d] = body ? T(0) : T(-k.pb * g);
    }
}

}  // namespace sph
