// tiles.hip -- LDS-tiled neighbour search and force pass of libsph (gfx950).
//
// A block owns one tile: an aligned block of 2^tb Morton keys, i.e. a box of
// cells (2 x 2 x 2 in 3D, 4 x 4 in 2D) whose rows are contiguous in the
// sorted state. It reads the row ranges of the tile's halo (the box grown by
// one cell on every side, which holds every neighbour of every row of the
// tile), scans their lengths into LDS offsets with one wave, and copies the
// halo's rows into LDS with coalesced loads: FP64 positions for the search;
// the packed neighbour record (FP32) or the FP64 fields for the force pass.
// Groups of G lanes then take the tile's rows in turn and read every
// neighbour from LDS instead of gathering it row by row from global memory
// (rows past the LDS capacity are read from global memory).
//
// Search: a row's candidates are the members of its 3^d stencil cells in
// stencil order, walked as one sequence with the FMA-free FP64 predicate and
// compacted by ballot, so its table row is the gather kernel's row, entry for
// entry; the density is summed in table order (lane l adds entries l, l + G,
// ...), as there. Force: a lane's table entries visit the row's stencil cells
// in order (the table is stencil-then-cell ordered), so a cursor over those
// cells maps each entry to its LDS slot; the pair terms, their order and the
// reductions are those of the gather kernel.
#include "pair_terms.h"
#include "sph_launch.h"

namespace sph {

// Halo of one tile, in LDS.
struct TileHalo {
    int32_t gbeg[kHaloCellsMax];  // first row of each halo cell (global)
    int32_t len[kHaloCellsMax];   // rows in it
    int32_t off[kHaloCellsMax];   // its first LDS slot (exclusive scan of len)
    int32_t total;                // rows in the halo
    int32_t r0, r1;               // the tile's own rows
    int32_t org[3];               // the tile's first cell
    int32_t ok;                   // 0: empty tile
};

// Row ranges and LDS offsets of the halo of `tile` (every thread of the block
// calls it). Returns false, for the whole block, for an empty tile.
template <int DIM>
__device__ inline bool tile_setup(const Dev &k, int64_t tile, int64_t n,
                                  const int32_t *cell_start, const uint32_t *spread,
                                  const uint32_t *cpos, TileHalo &H, uint32_t *err)
{
    const int t = threadIdx.x;
    if (t == 0) {
        const int64_t key0 = tile << k.tb;
        const int32_t a = cell_start[key0], b = cell_start[key0 + (int64_t(1) << k.tb)];
        const bool sane = a >= 0 && a <= b && int64_t(b) <= n;
        if (!sane) raise_error(err, SPH_ERR_CELL_RANGE);
        H.ok = sane && a < b;
        H.r0 = a;
        H.r1 = b;
        if (H.ok) {
            int c[3] = {0, 0, 0};
            unpack_cell<DIM>(cpos[a], c);
#pragma unroll
            for (int d = 0; d < 3; ++d) H.org[d] = c[d] & ~(k.text[d] - 1);
        }
    }
    __syncthreads();
    if (!H.ok) return false;
    if (t < k.nhalo) {
        const int hx = k.hext[0], hy = k.hext[1];
        const int tt[3] = {t % hx, (t / hx) % hy, t / (hx * hy)};
        int cc[3] = {0, 0, 0};
        bool valid = true;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            int v = H.org[d] - 1 + tt[d];
            if (v < 0 || v >= k.nc[d]) {
                // the cell beyond either end wraps on a periodic axis; cells of
                // the padded key space past it hold no rows
                if (k.periodic[d] && (v == -1 || v == k.nc[d])) v = v < 0 ? k.nc[d] - 1 : 0;
                else valid = false;
            }
            cc[d] = v;
        }
        int32_t b = 0, e = 0;
        if (valid) {
            const uint32_t key = morton_key<DIM>(spread, cc);
            b = cell_start[key];
            e = cell_start[key + 1];
            if (b < 0 || b > e || int64_t(e) > n) {
                raise_error(err, SPH_ERR_CELL_RANGE);
                b = e = 0;
            }
        }
        H.gbeg[t] = b;
        H.len[t] = e - b;
    }
    __syncthreads();
    // exclusive scan of the lengths: one wave, two cells per lane
    if (t < 64) {
        const int i0 = 2 * t, i1 = 2 * t + 1;
        const int v0 = i0 < k.nhalo ? H.len[i0] : 0, v1 = i1 < k.nhalo ? H.len[i1] : 0;
        int incl = v0 + v1;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o);
            if (t >= o) incl += y;
        }
        const int excl = incl - v0 - v1;
        if (i0 < k.nhalo) H.off[i0] = excl;
        if (i1 < k.nhalo) H.off[i1] = excl + v0;
        if (t == 63) H.total = incl;
    }
    __syncthreads();
    return true;
}

// Halo cell holding LDS slot f (the last cell whose offset is <= f).
__device__ inline int halo_cell_of(const TileHalo &H, int nhalo, int f)
{
    int lo = 0, hi = nhalo;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (H.off[mid] <= f) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Halo index of stencil cell sc ((dz, dy, dx) order, dx fastest) of a row in
// tile-local cell lc.
template <int DIM>
__device__ inline int halo_index(const Dev &k, const int lc[3], int sc)
{
    if (DIM == 2) return (lc[1] + sc / 3) * k.hext[0] + lc[0] + sc % 3;
    return ((lc[2] + sc / 9) * k.hext[1] + lc[1] + (sc / 3) % 3) * k.hext[0] + lc[0] + sc % 3;
}

// ---------------------------------------------------------------- search
// Candidates of one lane, NB at a time: global row and LDS slot of entries
// lane, lane + G, ... of the row's stencil sequence.
template <int DIM, int NB, int G>
struct TileWalk {
    const Dev &k;
    const TileHalo &H;
    int lc[3];
    int sc, mo, h;
    static constexpr int NS = DIM == 2 ? 9 : 27;
    __device__ inline TileWalk(const Dev &kk, const TileHalo &HH, const int l[3], int lane)
        : k(kk), H(HH)
    {
        lc[0] = l[0];
        lc[1] = l[1];
        lc[2] = l[2];
        sc = 0;
        mo = lane;
        h = halo_index<DIM>(k, lc, 0);
        advance();
    }
    __device__ inline void advance()
    {
        while (sc < NS && mo >= H.len[h]) {
            mo -= H.len[h];
            if (++sc < NS) h = halo_index<DIM>(k, lc, sc);
        }
    }
    __device__ inline void next(int32_t jj[NB], int32_t ss[NB], bool hv[NB])
    {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            hv[b] = sc < NS;
            jj[b] = hv[b] ? H.gbeg[h] + mo : 0;  // row 0 as a harmless dummy
            ss[b] = hv[b] ? H.off[h] + mo : 0;
            mo += G;
            advance();
        }
    }
};

template <int DIM, typename T, int G>
__global__ void __launch_bounds__(kBlock) k_tsearch(Dev k, DevState m, Fields R, DevNlist nl,
                                                    DevDerived o, int dens,
                                                    const uint32_t *spread,
                                                    const int32_t *cell_start,
                                                    const uint32_t *cpos, float *off,
                                                    int32_t *rebin_clear, uint32_t *err)
{
    // the step's bin has run: later updates of this step may request the next
    if (rebin_clear && blockIdx.x == 0 && threadIdx.x == 0) *rebin_clear = 0;
    constexpr int CAP = tile_cap_search(DIM);
    constexpr int NS = DIM == 2 ? 9 : 27;
    constexpr int PB = kBlock / G;
    constexpr int NB = 4;
    __shared__ TileHalo H;
    __shared__ double s_x[DIM][CAP];
    __shared__ T s_w[PB][G];
    const int64_t tile = xcd_block(k.ntiles);
    if (tile < 0) return;
    const int64_t n = *m.n;
    const int64_t C = k.cap;
    if (!tile_setup<DIM>(k, tile, n, cell_start, spread, cpos, H, err)) return;
    const int nst = H.total < CAP ? H.total : CAP;
    for (int f = threadIdx.x; f < nst; f += kBlock) {
        const int c = halo_cell_of(H, k.nhalo, f);
        const int64_t j = H.gbeg[c] + (f - H.off[c]);
#pragma unroll
        for (int d = 0; d < DIM; ++d) s_x[d][f] = R.x[d * C + j];
    }
    __syncthreads();
    const int lane = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int gshift = (threadIdx.x & 63) & ~(G - 1);
    const uint64_t gmask = G == 64 ? ~0ull : ((1ull << (G & 63)) - 1);
    const uint64_t below = (1ull << lane) - 1;
    for (int64_t i = H.r0 + grp; i < H.r1; i += PB) {
        double xi[3] = {0, 0, 0};
        int c[3] = {0, 0, 0}, lc[3] = {0, 0, 0};
        const uint32_t cposi = cpos[i];
#pragma unroll
        for (int d = 0; d < DIM; ++d) xi[d] = R.x[d * C + i];
        unpack_cell<DIM>(cposi, c);
#pragma unroll
        for (int d = 0; d < DIM; ++d) lc[d] = c[d] - H.org[d];
        int total = 0;
        for (int sc = lane; sc < NS; sc += G) total += H.len[halo_index<DIM>(k, lc, sc)];
        total = gsum<G>(total);
        int32_t *row = nl.nbr + i * nl.maxnb;
        Acc<T> sw;
        int cnt = 0;
        TileWalk<DIM, NB, G> w(k, H, lc, lane);
        for (int base = 0; base < total; base += NB * G) {
            int32_t jj[NB], ss[NB];
            bool hv[NB];
            w.next(jj, ss, hv);
            double xj[NB][3];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const bool lds = ss[b] < nst;
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    xj[b][d] = d < DIM ? (lds ? s_x[d][ss[b]] : R.x[d * C + jj[b]]) : 0.0;
            }
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                double r[3];
                const double r2 = dist2_exact<DIM>(k, xi, xj[b], r);
                const bool hit = hv[b] && r2 < k.sup2;
                int pos = cnt, nhit = hit ? 1 : 0;
                if (G > 1) {
                    const uint64_t bal = (uint64_t(__ballot(hit)) >> gshift) & gmask;
                    pos = cnt + __popcll(bal & below);
                    nhit = __popcll(bal);
                }
                if (hit && pos < nl.maxnb) row[pos] = jj[b];
                if (dens && nhit > 0) {
                    const T wv = hit ? kernel_w<T>(k, T(sqrt(r2) * k.inv_h), T(k.wnorm)) : T(0);
                    if (G == 1) {
                        sw.add(wv);
                    } else {
                        // route each kernel value to the lane of its table
                        // position, so that lane l sums entries l, l + G, ...
                        if (hit) s_w[grp][pos & (G - 1)] = wv;
                        __builtin_amdgcn_wave_barrier();
                        const T got = s_w[grp][lane];
                        __builtin_amdgcn_wave_barrier();
                        if (((lane - cnt) & (G - 1)) < nhit) sw.add(got);
                    }
                }
                cnt += nhit;
            }
        }
        const T S = sw.template reduce<G>();
        if (lane == 0) {
            if (cnt > nl.maxnb) {
                raise_error(err, SPH_ERR_NBR_OVERFLOW);
                cnt = nl.maxnb;
            }
            nl.count[i] = cnt;
            if (dens) {
                st<T>(o.rho, i, T(k.mass) * S);
                st<T>(o.vol, i, T(1) / S);
            }
        }
        if (dens && o.rec) write_rec<DIM, T, G>(k, m, R, o.rec, i, S, xi, c, cposi, lane);
        if (sizeof(T) == 4) {
            // offsets from the bin cell's corner, for the FP32 pair arithmetic
            for (int d = lane; d < DIM; d += G)
                off[d * C + i] = float(xi[d] - (k.lo[d] + double(c[d]) * k.cs[d]));
        }
    }
}

// ----------------------------------------------------------------- force
// Halo rows of the force pass in LDS: the packed record (FP32) or the FP64
// fields a neighbour contributes (x, u, ut, p, rho, V, kind).
template <int DIM, typename T>
struct ForceStage;

template <int DIM>
struct ForceStage<DIM, float> {
    using L = Rec<DIM, float>;
    static constexpr int CAP = tile_cap_force(DIM, SPH_FP32);
    float4 rec[CAP][L::NC];
    __device__ inline void put(const Dev &, const DevState &, const Fields &,
                               const DevDerived &o, int f, int64_t j)
    {
        const float4 *src = reinterpret_cast<const float4 *>(static_cast<const float *>(o.rec) +
                                                              j * L::N);
        float4 v[L::NC];
#pragma unroll
        for (int ch = 0; ch < L::NC; ++ch) v[ch] = src[ch];
#pragma unroll
        for (int ch = 0; ch < L::NC; ++ch) rec[f][ch] = v[ch];
    }
    __device__ inline void get(int f, int32_t j, NbrRaw<DIM, float> &w) const
    {
        w.j = j;
#pragma unroll
        for (int ch = 0; ch < L::NC; ++ch) Chunk<float>::get(rec[f][ch], w.v + ch * L::PER);
    }
    __device__ inline float pres(int f) const
    {
        const float *r = reinterpret_cast<const float *>(rec[f]);
        return r[L::P];
    }
};

template <int DIM>
struct ForceStage<DIM, double> {
    static constexpr int CAP = tile_cap_force(DIM, SPH_FP64);
    static constexpr int X = 0, U = DIM, UT = 2 * DIM, P = 3 * DIM, RHO = 3 * DIM + 1,
                         VOL = 3 * DIM + 2, NF = 3 * DIM + 3;
    double f64[NF][CAP];
    uint8_t kind[CAP];
    __device__ inline void put(const Dev &k, const DevState &m, const Fields &R,
                               const DevDerived &o, int f, int64_t j)
    {
        const int64_t C = k.cap;
        double v[NF];
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            v[X + d] = R.x[d * C + j];
            v[U + d] = ld<double>(R.u, d * C + j);
            v[UT + d] = ld<double>(R.ut, d * C + j);
        }
        v[P] = ld<double>(R.p, j);
        v[RHO] = ld<double>(o.rho, j);
        v[VOL] = ld<double>(o.vol, j);
        const uint8_t t = m.type[j];
#pragma unroll
        for (int q = 0; q < NF; ++q) f64[q][f] = v[q];
        kind[f] = t;
    }
    __device__ inline void get(int f, int32_t j, NbrRaw<DIM, double> &w) const
    {
        w.j = j;
        w.tj = kind[f];
        w.xj[2] = 0.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            w.xj[d] = f64[X + d][f];
            w.u[d] = f64[U + d][f];
            w.ut[d] = f64[UT + d][f];
        }
        w.p = f64[P][f];
        w.rho = f64[RHO][f];
        w.vol = f64[VOL][f];
    }
    __device__ inline double pres(int f) const { return f64[P][f]; }
};

// Maps a lane's table entries, which visit the row's stencil cells in order,
// to LDS slots (or -1 for a row past the LDS capacity); entries outside the
// row's stencil (a table of another bin) are reported and skipped.
template <int DIM>
struct Cursor {
    const Dev &k;
    const TileHalo &H;
    int lc[3];
    int sc;
    int32_t gb, ln, so;
    static constexpr int NS = DIM == 2 ? 9 : 27;
    __device__ inline Cursor(const Dev &kk, const TileHalo &HH, const int l[3]) : k(kk), H(HH)
    {
        lc[0] = l[0];
        lc[1] = l[1];
        lc[2] = l[2];
        reset();
    }
    __device__ inline void reset()
    {
        sc = 0;
        const int h = halo_index<DIM>(k, lc, 0);
        gb = H.gbeg[h];
        ln = H.len[h];
        so = H.off[h];
    }
    // returns false if j lies in none of the remaining stencil cells
    __device__ inline bool find(int32_t j, int nst, int &slot)
    {
        while (!(j >= gb && j - gb < ln)) {
            if (++sc >= NS) return false;
            const int h = halo_index<DIM>(k, lc, sc);
            gb = H.gbeg[h];
            ln = H.len[h];
            so = H.off[h];
        }
        const int f = so + (j - gb);
        slot = f < nst ? f : -1;
        return true;
    }
};

template <int DIM, typename T, int G>
__global__ void __launch_bounds__(kBlock) k_tforce(Dev k, DevState m, Fields R, Fields W,
                                                   DevNlist nl, DevDerived o, const float *off,
                                                   const uint32_t *cpos, const uint32_t *spread,
                                                   const int32_t *cell_start, int mode,
                                                   int want_drag, double *dragpart,
                                                   const double *xbin, int32_t *rebin,
                                                   uint32_t *err)
{
    using FS = ForceStage<DIM, T>;
    constexpr int PB = kBlock / G;
    constexpr int NB = 4;
    __shared__ TileHalo H;
    __shared__ FS S;
    __shared__ double red_lds[3][PB];
    const int lane = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int64_t tile = xcd_block(k.ntiles);
    const int64_t n = *m.n;
    const int64_t C = k.cap;
    bool have = tile >= 0;
    if (have) have = tile_setup<DIM>(k, tile, n, cell_start, spread, cpos, H, err);
    double fbg[3] = {0, 0, 0};  // this group's body force over its rows
    if (have) {
        const int nst = H.total < FS::CAP ? H.total : FS::CAP;
        for (int f = threadIdx.x; f < nst; f += kBlock) {
            const int c = halo_cell_of(H, k.nhalo, f);
            S.put(k, m, R, o, f, int64_t(H.gbeg[c]) + (f - H.off[c]));
        }
        __syncthreads();
        for (int64_t i = H.r0 + grp; i < H.r1; i += PB) {
            const int t = m.type[i];
            if (t == SPH_FLUID || t == SPH_BODY) {
                const int cnt = nl.count[i];
                Sep<DIM, T> sep;
                sep.load_i(k, R, off, cpos, i);
                int c[3] = {0, 0, 0}, lc[3] = {0, 0, 0};
                unpack_cell<DIM>(cpos[i], c);
#pragma unroll
                for (int d = 0; d < DIM; ++d) lc[d] = c[d] - H.org[d];
                T ui[3] = {0, 0, 0}, wi[3] = {0, 0, 0};
#pragma unroll
                for (int d = 0; d < DIM; ++d) {
                    ui[d] = ld<T>(R.u, d * C + i);
                    wi[d] = ld<T>(R.ut, d * C + i) - ui[d];
                }
                const T pi = ld<T>(R.p, i);
                const T rhoi = ld<T>(o.rho, i);
                const T vi = ld<T>(o.vol, i);
                const T vi2 = vi * vi;
                const int32_t *row = nl.nbr + i * nl.maxnb;
                // the neighbour average of eq:pavg enters the fluid's momentum;
                // the body force takes p~ about zero
                T pavg = T(0);
                if (t == SPH_FLUID && !(k.flags & SPH_FLAG_NO_PAVG)) {
                    Acc<T> sp;
                    Cursor<DIM> cur(k, H, lc);
                    bool bad = false;
                    for (int q0 = lane; q0 < cnt; q0 += NB * G) {
                        int32_t jb[NB];
#pragma unroll
                        for (int f = 0; f < NB; ++f)
                            jb[f] = q0 + f * G < cnt ? row[q0 + f * G] : -1;
#pragma unroll
                        for (int f = 0; f < NB; ++f) {
                            if (q0 + f * G >= cnt) continue;
                            int slot;
                            if (bad_index(jb[f], n) || !cur.find(jb[f], nst, slot)) {
                                bad = true;
                                continue;
                            }
                            sp.add(slot >= 0 ? S.pres(slot) : ld<T>(R.p, jb[f]));
                        }
                    }
                    if (bad) raise_error(err, SPH_ERR_CELL_RANGE);
                    pavg = sp.template reduce<G>() / T(cnt);
                }
                Acc<T> acc[3], bacc[3], pdot;
                double fb[3] = {0, 0, 0};
                {
                    Cursor<DIM> cur(k, H, lc);
                    bool bad = false;
                    for (int q0 = lane; q0 < cnt; q0 += NB * G) {
                        int32_t jb[NB];
#pragma unroll
                        for (int f = 0; f < NB; ++f)
                            jb[f] = q0 + f * G < cnt ? row[q0 + f * G] : -1;
#pragma unroll
                        for (int f = 0; f < NB; ++f) {
                            if (q0 + f * G >= cnt) continue;
                            int slot;
                            if (bad_index(jb[f], n) || !cur.find(jb[f], nst, slot)) {
                                bad = true;
                                continue;
                            }
                            if (jb[f] == i) continue;
                            NbrRaw<DIM, T> raw;
                            if (slot >= 0) S.get(slot, jb[f], raw);
                            else fetch_nbr<DIM, T>(k, m, R, o, jb[f], raw);
                            Nbr<DIM, T> nb;
                            finish_nbr<DIM, T>(k, sep, raw, nb);
                            if (t == SPH_BODY && nb.tj != SPH_FLUID) continue;
                            pair_acc<DIM, T>(k, t, ui, wi, pi, rhoi, vi2, pavg, nb, acc, bacc,
                                             pdot, fb);
                        }
                    }
                    if (bad) raise_error(err, SPH_ERR_CELL_RANGE);
                }
                T a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
#pragma unroll
                for (int d = 0; d < DIM; ++d) {
                    a[d] = acc[d].template reduce<G>();
                    b[d] = bacc[d].template reduce<G>();
                    fb[d] = gsum<G>(fb[d]);
                }
                const T pd = pdot.template reduce<G>();
                if (lane == 0) {
                    if (mode == 0) {
#pragma unroll
                        for (int d = 0; d < DIM; ++d) {
                            st<T>(o.a, d * C + i, a[d]);
                            st<T>(o.b, d * C + i, b[d]);
                        }
                        st<T>(o.pdot, i, pd);
                        st<T>(o.pavg, i, pavg);
                        if (t == SPH_BODY)
#pragma unroll
                            for (int d = 0; d < DIM; ++d) o.force[d * C + i] = fb[d];
                    } else {
                        if (t == SPH_FLUID)
                            stage_fluid<DIM, T>(k, R, W, i, mode, ui, pi, a, b, pd, xbin, rebin,
                                                err);
                        st<T>(o.pavg, i, pavg);  // kept for a reverse pass
                    }
                }
#pragma unroll
                for (int d = 0; d < 3; ++d) fbg[d] += fb[d];
            }
            // every non-fluid row (walls, bodies, inlet, outlet) takes its stage
            // position and, in the full update, its half-state boundary values
            if (mode != 0 && t != SPH_FLUID && lane == 0)
                stage_boundary<DIM, T>(k, m, R, W, i, t, mode, o.jcur, xbin, rebin, err);
        }
    }
    if (!want_drag) return;
    // deterministic per-block partial of the body force (groups in order)
    if (lane == 0)
#pragma unroll
        for (int d = 0; d < 3; ++d) red_lds[d][grp] = fbg[d];
    __syncthreads();
    if (threadIdx.x == 0) {
        double s[3] = {0, 0, 0};
        for (int q = 0; q < PB; ++q)
#pragma unroll
            for (int d = 0; d < 3; ++d) s[d] += red_lds[d][q];
#pragma unroll
        for (int d = 0; d < 3; ++d) dragpart[d * gridDim.x + blockIdx.x] = s[d];
    }
}

// ------------------------------------------------------------------ launchers
int tile_grid(const Dev &k) { return xcd_grid(k.ntiles); }

template <int DIM, typename T, int G>
static void tsearch_g(const Dev &k, const DevState &m, const Fields &R, const DevNlist &nl,
                      const DevDerived &o, int dens, const uint32_t *spread,
                      const int32_t *cell_start, const uint32_t *cpos, float *off,
                      int32_t *rebin_clear, uint32_t *err, hipStream_t s)
{
    hipLaunchKernelGGL((k_tsearch<DIM, T, G>), dim3(tile_grid(k)), dim3(kBlock), 0, s, k, m, R,
                       nl, o, dens, spread, cell_start, cpos, off, rebin_clear, err);
}

template <int DIM, typename T>
static void tsearch_dt(const Dev &k, const DevState &m, const Fields &R, const DevNlist &nl,
                       const DevDerived &o, int dens, const uint32_t *spread,
                       const int32_t *cell_start, const uint32_t *cpos, float *off,
                       int32_t *rebin_clear, uint32_t *err, hipStream_t s)
{
#define SPH_TS_G(G) \
    tsearch_g<DIM, T, G>(k, m, R, nl, o, dens, spread, cell_start, cpos, off, rebin_clear, err, s)
    switch (nbr_group(k)) {
    case 1: SPH_TS_G(1); break;
    case 2: SPH_TS_G(2); break;
    case 4: SPH_TS_G(4); break;
    case 8: SPH_TS_G(8); break;
    case 16: SPH_TS_G(16); break;
    default: SPH_TS_G(32); break;
    }
#undef SPH_TS_G
}

void launch_tsearch(const Dev &k, const DevState &m, const Fields &R, const DevNlist &nl,
                    const DevDerived &o, int dens, const uint32_t *spread,
                    const int32_t *cell_start, const uint32_t *cpos, float *off,
                    int32_t *rebin_clear, uint32_t *err, hipStream_t s)
{
    if (k.dim == 2 && k.prec == SPH_FP64)
        tsearch_dt<2, double>(k, m, R, nl, o, dens, spread, cell_start, cpos, off, rebin_clear,
                              err, s);
    else if (k.dim == 3 && k.prec == SPH_FP64)
        tsearch_dt<3, double>(k, m, R, nl, o, dens, spread, cell_start, cpos, off, rebin_clear,
                              err, s);
    else if (k.dim == 2)
        tsearch_dt<2, float>(k, m, R, nl, o, dens, spread, cell_start, cpos, off, rebin_clear,
                             err, s);
    else
        tsearch_dt<3, float>(k, m, R, nl, o, dens, spread, cell_start, cpos, off, rebin_clear,
                             err, s);
}

template <int DIM, typename T, int G>
static void tforce_g(const Dev &k, const DevState &m, const Fields &R, const Fields &W,
                     const DevNlist &nl, const DevDerived &o, const float *off,
                     const uint32_t *cpos, const uint32_t *spread, const int32_t *cell_start,
                     int mode, int want_drag, double *dragpart, const double *xbin,
                     int32_t *rebin, uint32_t *err, hipStream_t s)
{
    hipLaunchKernelGGL((k_tforce<DIM, T, G>), dim3(tile_grid(k)), dim3(kBlock), 0, s, k, m, R, W,
                       nl, o, off, cpos, spread, cell_start, mode, want_drag, dragpart, xbin,
                       rebin, err);
}

template <int DIM, typename T>
static void tforce_dt(const Dev &k, const DevState &m, const Fields &R, const Fields &W,
                      const DevNlist &nl, const DevDerived &o, const float *off,
                      const uint32_t *cpos, const uint32_t *spread, const int32_t *cell_start,
                      int mode, int want_drag, double *dragpart, const double *xbin,
                      int32_t *rebin, uint32_t *err, hipStream_t s)
{
#define SPH_TF_G(G)                                                                             \
    tforce_g<DIM, T, G>(k, m, R, W, nl, o, off, cpos, spread, cell_start, mode, want_drag,   \
                        dragpart, xbin, rebin, err, s)
    switch (force_group(k)) {
    case 1: SPH_TF_G(1); break;
    case 2: SPH_TF_G(2); break;
    case 4: SPH_TF_G(4); break;
    case 8: SPH_TF_G(8); break;
    case 16: SPH_TF_G(16); break;
    default: SPH_TF_G(32); break;
    }
#undef SPH_TF_G
}

void launch_tforce(const Dev &k, const DevState &m, const Fields &R, const Fields &W,
                   const DevNlist &nl, const DevDerived &o, const float *off,
                   const uint32_t *cpos, const uint32_t *spread, const int32_t *cell_start,
                   int mode, int want_drag, double *dragpart, const double *xbin,
                   int32_t *rebin, uint32_t *err, hipStream_t s)
{
    if (k.dim == 2 && k.prec == SPH_FP64)
        tforce_dt<2, double>(k, m, R, W, nl, o, off, cpos, spread, cell_start, mode, want_drag,
                             dragpart, xbin, rebin, err, s);
    else if (k.dim == 3 && k.prec == SPH_FP64)
        tforce_dt<3, double>(k, m, R, W, nl, o, off, cpos, spread, cell_start, mode, want_drag,
                             dragpart, xbin, rebin, err, s);
    else if (k.dim == 2)
        tforce_dt<2, float>(k, m, R, W, nl, o, off, cpos, spread, cell_start, mode, want_drag,
                            dragpart, xbin, rebin, err, s);
    else
        tforce_dt<3, float>(k, m, R, W, nl, o, off, cpos, spread, cell_start, mode, want_drag,
                            dragpart, xbin, rebin, err, s);
}

}  // namespace sph
