// tiles.hip -- LDS-tiled neighbour search and force pass of libsph (gfx950).
//
// A tile is an aligned block of 2^tb Morton keys, i.e. a box of cells
// (2 x 2 x 2 in 3D, 4 x 4 in 2D) whose rows are contiguous in the sorted
// state; its halo (the box grown by one cell on every side) holds every
// neighbour of every row of the tile. After each sort k_tile_table writes one
// record per tile: the tile's rows, its first cell, and for every halo cell
// the first row and the LDS slot of its first row (an exclusive scan of the
// cell lengths, in halo-index order, x fastest). A block of the pair passes
// owns one tile: it reads the tile's record in one coalesced load, copies the
// halo's rows into LDS (a few threads per halo cell, coalesced along the
// cell's rows): FP64 positions for the search; the packed neighbour record
// (FP32) or the FP64 fields for the force pass. Groups of G lanes then take
// the tile's rows in turn and read every neighbour from LDS instead of
// gathering it row by row from global memory (rows past the LDS capacity are
// read from global memory).
//
// The three cells of a row's stencil along x are consecutive halo indices and
// so consecutive LDS slots: the stencil is 9 runs of contiguous slots in 3D
// (3 in 2D), and walking them in order visits the candidates in
// stencil-then-cell order.
//
// Search: lanes test the candidates of each run in chunks of G with the
// FMA-free FP64 predicate, and a ballot compacts the hits, so a row's table
// entries are the gather kernel's, in the same order; the density is summed
// in table order (lane l adds entries l, l + G, ...), as there. Besides the
// global row of every entry the search writes its LDS slot (a 16-bit table in
// the workspace), from which the force pass of the same bin reads each
// neighbour without looking its row up again; the pair terms, their order
// and the reductions are those of the gather kernel.
#include "pair_terms.h"
#include "sph_launch.h"

namespace sph {

// Tile record (int32): [0] first row, [1] end row, [2] packed first cell,
// [3] halo rows, [4 + c] first row of halo cell c, [4 + nhalo + c] its first
// LDS slot for c <= nhalo (the last entry is the halo's row count).
__host__ __device__ constexpr int tile_rec_ints(int nhalo) { return (5 + 2 * nhalo + 3) & ~3; }
int64_t tile_table_ints(const Dev &k) { return k.ntiles * tile_rec_ints(k.nhalo); }

// ------------------------------------------------------------- tile table
// One wave per tile (two halo cells per lane). Runs after every bin and
// returns at once when the bin kept the order (the table stays valid).
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_tile_table(Dev k, const int64_t *nrows,
                                                       const int32_t *cell_start,
                                                       const uint32_t *spread,
                                                       const uint32_t *cpos,
                                                       const int32_t *sorted, int32_t *table,
                                                       uint32_t *err)
{
    if (*sorted == 0) return;
    const int lane = threadIdx.x & 63;
    const int64_t tile = int64_t(blockIdx.x) * (kBlock / 64) + threadIdx.x / 64;
    if (tile >= k.ntiles) return;
    const int64_t n = *nrows;
    const int RI = tile_rec_ints(k.nhalo);
    int32_t *rec = table + tile * RI;
    const int64_t key0 = tile << k.tb;
    int32_t a = cell_start[key0], b = cell_start[key0 + (int64_t(1) << k.tb)];
    if (!(a >= 0 && a <= b && int64_t(b) <= n)) {
        if (lane == 0) raise_error(err, SPH_ERR_CELL_RANGE);
        a = b = 0;
    }
    if (a == b) {  // empty tile: its record says so
        if (lane == 0) {
            rec[0] = a;
            rec[1] = b;
        }
        return;
    }
    int org[3] = {0, 0, 0};
    unpack_cell<DIM>(cpos[a], org);
#pragma unroll
    for (int d = 0; d < 3; ++d) org[d] &= ~(k.text[d] - 1);
    int32_t gb[2] = {0, 0}, ln[2] = {0, 0};
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int t = 2 * lane + u;
        if (t >= k.nhalo) continue;
        const int hx = k.hext[0], hy = k.hext[1];
        const int tt[3] = {t % hx, (t / hx) % hy, t / (hx * hy)};
        int cc[3] = {0, 0, 0};
        bool valid = true;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            int v = org[d] - 1 + tt[d];
            if (v < 0 || v >= k.nc[d]) {
                // the cell beyond either end wraps on a periodic axis; cells of
                // the padded key space past it hold no rows
                if (k.periodic[d] && (v == -1 || v == k.nc[d])) v = v < 0 ? k.nc[d] - 1 : 0;
                else valid = false;
            }
            cc[d] = v;
        }
        if (valid) {
            const uint32_t key = morton_key<DIM>(spread, cc);
            const int32_t cb = cell_start[key], ce = cell_start[key + 1];
            if (cb < 0 || cb > ce || int64_t(ce) > n) {
                raise_error(err, SPH_ERR_CELL_RANGE);
            } else {
                gb[u] = cb;
                ln[u] = ce - cb;
            }
        }
    }
    // exclusive scan of the lengths over the wave
    const int v0 = ln[0], v1 = ln[1];
    int incl = v0 + v1;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    const int excl = incl - v0 - v1;
    const int total = __shfl(incl, 63, 64);
    if (total > 65535) {
        // slots are 16-bit: a halo this crowded (a thousand rows per cell)
        // is flagged and its tile skipped
        if (lane == 0) {
            raise_error(err, SPH_ERR_NBR_OVERFLOW);
            rec[0] = rec[1] = a;
        }
        return;
    }
    const int i0 = 2 * lane, i1 = 2 * lane + 1;
    if (i0 < k.nhalo) {
        rec[4 + i0] = gb[0];
        rec[4 + k.nhalo + i0] = excl;
    }
    if (i1 < k.nhalo) {
        rec[4 + i1] = gb[1];
        rec[4 + k.nhalo + i1] = excl + v0;
    }
    if (lane == 0) {
        rec[0] = a;
        rec[1] = b;
        rec[2] = int32_t(pack_cell<DIM>(org));
        rec[3] = total;
        rec[4 + 2 * k.nhalo] = total;
    }
}

// Tile of hardware block blockIdx.x. The 8 XCDs receive consecutive hardware
// blocks round-robin; they take chunks of kTileChunk consecutive tiles in turn
// (XCD x the chunks x, x + 8, ...), so that the tiles of a chunk, which share
// most of their halos, meet in one L2, and every XCD gets a share of the
// occupied tiles (a contiguous eighth of the tile index range per XCD would
// leave some XCDs only the empty padding of the Morton key space). -1 past
// the last tile.
constexpr int kTileChunk = 16;
__device__ inline int64_t tile_of_block(int64_t ntiles)
{
    const int64_t b = blockIdx.x, x = b % 8, w = b / 8;
    const int64_t t = ((w / kTileChunk) * 8 + x) * kTileChunk + w % kTileChunk;
    return t < ntiles ? t : -1;
}

// The record of one tile in LDS, with its accessors.
struct TileHalo {
    int32_t rec[(5 + 2 * kHaloCellsMax + 3) & ~3];
    int nh;
    __device__ inline int r0() const { return rec[0]; }
    __device__ inline int r1() const { return rec[1]; }
    __device__ inline int total() const { return rec[3]; }
    __device__ inline int gbeg(int c) const { return rec[4 + c]; }
    __device__ inline int off(int c) const { return rec[4 + nh + c]; }  // c <= nh
    __device__ inline int len(int c) const { return off(c + 1) - off(c); }
};

// Loads the tile's record (every thread of the block calls it); false, for
// the whole block, for an empty tile.
template <int DIM>
__device__ inline bool tile_load(const Dev &k, int64_t tile, const int32_t *table, TileHalo &H,
                                 int org[3])
{
    const int RI = tile_rec_ints(k.nhalo);
    const int32_t *src = table + tile * RI;
    for (int t = threadIdx.x; t < RI; t += kBlock) H.rec[t] = src[t];
    H.nh = k.nhalo;
    __syncthreads();
    if (H.r0() >= H.r1()) return false;
    unpack_cell<DIM>(uint32_t(H.rec[2]), org);
    return true;
}

// Copies the halo's rows into LDS slots below cap: threads in groups per
// halo cell, each group walking its cell's rows. put(f, j): slot f, row j.
template <typename Put>
__device__ inline void tile_stage(const TileHalo &H, int cap, Put put)
{
    const int per = kBlock / H.nh;  // threads per halo cell
    const int t = threadIdx.x;
    const int c = t / per;
    if (c >= H.nh) return;
    const int o = H.off(c), l = H.len(c), g = H.gbeg(c);
    for (int q = t - c * per; q < l && o + q < cap; q += per) put(o + q, int64_t(g) + q);
}

// Global row of LDS slot f (any slot below the halo's row count).
__device__ inline int32_t halo_row(const TileHalo &H, int f)
{
    int lo = 0, hi = H.nh;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (H.off(mid) <= f) lo = mid;
        else hi = mid;
    }
    return H.gbeg(lo) + (f - H.off(lo));
}

// Halo index of stencil cell sc ((dz, dy, dx) order, dx fastest) of a row in
// tile-local cell lc.
template <int DIM>
__device__ inline int halo_index(const Dev &k, const int lc[3], int sc)
{
    if (DIM == 2) return (lc[1] + sc / 3) * k.hext[0] + lc[0] + sc % 3;
    return ((lc[2] + sc / 9) * k.hext[1] + lc[1] + (sc / 3) % 3) * k.hext[0] + lc[0] + sc % 3;
}

// First halo cell of run r (the cells dx = -1, 0, 1 of stencil row (dy, dz),
// r = 3 (dz + 1) + dy + 1 in 3D, dy + 1 in 2D) of a row in tile-local cell lc.
template <int DIM>
__device__ inline int run_cell(const Dev &k, const int lc[3], int r)
{
    if (DIM == 2) return (lc[1] + r) * k.hext[0] + lc[0];
    return ((lc[2] + r / 3) * k.hext[1] + lc[1] + r % 3) * k.hext[0] + lc[0];
}

// ---------------------------------------------------------------- search
// Step path (vmode 1, 2): per-row candidate lists of LDS slots, recorded by
// the first search after a sort (vmode 1 with *v.fresh: the stencil walk,
// which also keeps every candidate within Dev::rv2 of the row) and walked by
// every later search until the next sort. A list is a subsequence of the
// stencil sequence that holds every hit (rows stay within the cell skin of
// their binned positions, checked by the stage updates), and the tile layout
// does not change between sorts, so its slots stay valid and the walk gives
// the same table in the same order. vmode 0 walks the stencil only.
template <int DIM, typename T, int G>
__global__ void __launch_bounds__(kBlock) k_tsearch(Dev k, DevState m, Fields R, DevNlist nl,
                                                    DevDerived o, int dens,
                                                    const int32_t *table, const uint32_t *cpos,
                                                    float *off, uint16_t *lslot,
                                                    int32_t *rebin_clear, VList v, int vmode,
                                                    uint32_t *err)
{
    // the step's bin has run: later updates of this step may request the next
    if (rebin_clear && blockIdx.x == 0 && threadIdx.x == 0) *rebin_clear = 0;
    constexpr int CAP = tile_cap_search(DIM);
    constexpr int NR = DIM == 2 ? 3 : 9;  // runs of three cells along x
    constexpr int PB = kBlock / G;
    constexpr int NB = 2;                 // chunks of G candidates per round
    __shared__ TileHalo H;
    __shared__ double s_x[DIM][CAP];
    __shared__ int32_t s_row[CAP];
    __shared__ T s_w[PB][G];
    const int64_t tile = tile_of_block(k.ntiles);
    if (tile < 0) return;
    const int64_t C = k.cap;
    int org[3] = {0, 0, 0};
    if (!tile_load<DIM>(k, tile, table, H, org)) return;
    const int total = H.total();
    const int nst = total < CAP ? total : CAP;  // >= 1: the tile has rows
    tile_stage(H, CAP, [&](int f, int64_t j) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) s_x[d][f] = R.x[d * C + j];
        s_row[f] = int32_t(j);
    });
    __syncthreads();
    const bool build = vmode == 1 && *v.fresh != 0;
    const int lane = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int gshift = (threadIdx.x & 63) & ~(G - 1);
    const uint64_t gmask = G == 64 ? ~0ull : ((1ull << (G & 63)) - 1);
    const uint64_t below = (1ull << lane) - 1;
    const int lmax = nl.maxnb < k.lmax ? nl.maxnb : k.lmax;
    for (int64_t i = H.r0() + grp; i < H.r1(); i += PB) {
        // the walk of this row: its stored list (vc >= 0) or the stencil
        const int vc = (vmode != 0 && !build) ? v.count[i] : -1;
        double xi[3] = {0, 0, 0};
        int c[3] = {0, 0, 0}, lc[3] = {0, 0, 0};
        const uint32_t cposi = cpos[i];
#pragma unroll
        for (int d = 0; d < DIM; ++d) xi[d] = R.x[d * C + i];
        unpack_cell<DIM>(cposi, c);
#pragma unroll
        for (int d = 0; d < DIM; ++d) lc[d] = c[d] - org[d];
        int32_t *row = nl.nbr + i * nl.maxnb;
        uint16_t *lrow = lslot + i * k.lmax;
        uint16_t *vrow = v.slot + i * int64_t(k.vmax);
        Acc<T> sw;
        int cnt = 0, vcnt = 0;
        // tests NB chunks of G candidates (global rows jj, LDS slots ss,
        // positions xj) in sequence order: table entries by ballot and, when
        // recording, list entries within rv
        auto test = [&](const int32_t *jj, const int *ss, const bool *hv, double (*xj)[3],
                        bool rec) {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                double rr[3];
                const double r2 = dist2_exact<DIM>(k, xi, xj[b], rr);
                const bool hit = hv[b] && r2 < k.sup2;
                int pos = cnt, nhit = hit ? 1 : 0;
                if (G > 1) {
                    const uint64_t bal = (uint64_t(__ballot(hit)) >> gshift) & gmask;
                    pos = cnt + __popcll(bal & below);
                    nhit = __popcll(bal);
                }
                if (hit && pos < lmax) {
                    row[pos] = jj[b];
                    lrow[pos] = uint16_t(ss[b]);
                }
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
                if (rec) {
                    const bool vhit = hv[b] && r2 < k.rv2;
                    int vpos = vcnt, nv = vhit ? 1 : 0;
                    if (G > 1) {
                        const uint64_t bal = (uint64_t(__ballot(vhit)) >> gshift) & gmask;
                        vpos = vcnt + __popcll(bal & below);
                        nv = __popcll(bal);
                    }
                    if (vhit && vpos < k.vmax) vrow[vpos] = uint16_t(ss[b]);
                    vcnt += nv;
                }
            }
        };
        // positions of slot f (LDS; past the capacity from global memory,
        // under a branch: two unconditional loads would be merged into one
        // generic load through a selected pointer)
        auto position = [&](bool h, int f, int32_t j, double *x) {
            const int fs = h && f < nst ? f : 0;
            x[2] = 0.0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) x[d] = s_x[d][fs];
            if (h && f >= nst) {
#pragma unroll
                for (int d = 0; d < DIM; ++d) x[d] = R.x[d * C + j];
            }
        };
        if (vc >= 0) {
            // the stored list; the next round's entries are read while this
            // round is tested (entries past the list are not used)
            bool bad = false;
            int fc[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int q = b * G + lane;
                fc[b] = q < vc ? int(vrow[q]) : 0;
            }
            for (int base = 0; base < vc; base += NB * G) {
                int fn[NB];
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const int q = base + NB * G + b * G + lane;
                    fn[b] = q < vc ? int(vrow[q]) : 0;
                }
                int32_t jj[NB];
                int ss[NB];
                bool hv[NB];
                double xj[NB][3];
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const int q = base + b * G + lane;
                    const int f = fc[b];
                    const bool ok = f < total;
                    bad = bad || (q < vc && !ok);
                    hv[b] = q < vc && ok;
                    ss[b] = f;
                    jj[b] = !hv[b] ? 0 : (f < nst ? s_row[f] : halo_row(H, f));
                    position(hv[b], f, jj[b], xj[b]);
                }
                test(jj, ss, hv, xj, false);
#pragma unroll
                for (int b = 0; b < NB; ++b) fc[b] = fn[b];
            }
            if (bad) raise_error(err, SPH_ERR_CELL_RANGE);
        } else {
            for (int r = 0; r < NR; ++r) {
                // the run's three cells are consecutive halo indices and slots
                const int h0 = run_cell<DIM>(k, lc, r);
                const int o0 = H.off(h0), o1 = H.off(h0 + 1), o2 = H.off(h0 + 2);
                const int32_t g0 = H.gbeg(h0), g1 = H.gbeg(h0 + 1), g2 = H.gbeg(h0 + 2);
                const int rl = H.off(h0 + 3) - o0;
                for (int base = 0; base < rl; base += NB * G) {
                    int32_t jj[NB];
                    int ss[NB];
                    bool hv[NB];
                    double xj[NB][3];
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const int q = base + b * G + lane;
                        hv[b] = q < rl;
                        const int f = o0 + q;
                        ss[b] = f;
                        jj[b] = f + (f < o1 ? g0 - o0 : (f < o2 ? g1 - o1 : g2 - o2));
                        position(hv[b], f, jj[b], xj[b]);
                    }
                    test(jj, ss, hv, xj, build);
                }
            }
        }
        const T S = sw.template reduce<G>();
        if (lane == 0) {
            if (cnt > lmax) {
                raise_error(err, SPH_ERR_NBR_OVERFLOW);
                cnt = lmax;
            }
            nl.count[i] = cnt;
            if (build) v.count[i] = vcnt <= k.vmax ? vcnt : -1;
            if (dens) {
                st<T>(o.rho, i, T(k.mass) * S);
                st<T>(o.vol, i, T(1) / S);
                if (o.shep) st<T>(o.shep, i, S);
            }
        }
        if constexpr (sizeof(T) == 4 && DIM == 2)
            if (dens && o.rec) write_rec<DIM, T, G>(k, m, R, o.rec, i, S, xi, c, cposi, lane);
        if (sizeof(T) == 4) {
            // offsets from the bin cell's corner, for the FP32 pair arithmetic
            for (int d = lane; d < DIM; d += G)
                off[d * C + i] = cell_offset(k, d, xi[d], c[d]);
        }
    }
}

// ----------------------------------------------------------------- force
// Halo rows of the force pass in LDS: the packed record (FP32) or the FP64
// fields a neighbour contributes (x, u, ut, p, the Shepard sum, kind).
template <int DIM, typename T>
struct ForceStage;

template <int DIM>
struct ForceStage<DIM, float> {
    using L = Rec<DIM, float>;
    static constexpr int CAP = tile_cap_force(DIM, SPH_FP32);
    float4 rec[CAP][L::NC];
    __device__ inline void put(const Dev &k, const DevState &, const Fields &,
                               const DevDerived &o, int f, int64_t j)
    {
        float4 v[L::NC];
#pragma unroll
        for (int ch = 0; ch < L::NC; ++ch) v[ch] = *rec_chunk<DIM, float>(o.rec, k.cap, j, ch);
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
    static constexpr int X = 0, U = DIM, UT = 2 * DIM, P = 3 * DIM, SH = 3 * DIM + 1,
                         NF = 3 * DIM + 2;
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
        v[SH] = ld<double>(o.shep, j);
        const uint8_t t = m.type[j];
#pragma unroll
        for (int q = 0; q < NF; ++q) f64[q][f] = v[q];
        kind[f] = t;
    }
    // the staged fields in the record's layout (w = ut - u formed as the
    // record writer forms it)
    __device__ inline void get(int f, int32_t j, NbrRaw<DIM, double> &w) const
    {
        using L = Rec<DIM, double>;
        w.j = j;
        if constexpr (L::USE) {
#pragma unroll
            for (int q = 0; q < L::NC * L::PER; ++q) w.v[q] = 0.0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                w.v[L::X + d] = f64[X + d][f];
                const double u = f64[U + d][f];
                w.v[L::U + d] = u;
                w.v[L::W + d] = f64[UT + d][f] - u;
            }
            w.v[L::P] = f64[P][f];
            w.v[L::VOL] = f64[SH][f];
            w.v[L::AUX] = rec_word<double>(uint32_t(kind[f]));
        } else {
            w.tj = kind[f];
            w.xj[2] = 0.0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                w.xj[d] = f64[X + d][f];
                w.u[d] = f64[U + d][f];
                w.ut[d] = f64[UT + d][f];
            }
            w.p = f64[P][f];
            w.s = f64[SH][f];
        }
    }
    __device__ inline double pres(int f) const { return f64[P][f]; }
};

template <int DIM, typename T, int G>
__global__ void __launch_bounds__(kBlock) k_tforce(Dev k, DevState m, Fields R, Fields W,
                                                   DevNlist nl, DevDerived o, const float *off,
                                                   const uint32_t *cpos, const int32_t *table,
                                                   const uint16_t *lslot, int mode,
                                                   int want_drag, double *dragpart,
                                                   const double *xbin, int32_t *rebin,
                                                   uint32_t *err)
{
    using FS = ForceStage<DIM, T>;
    constexpr int PB = kBlock / G;
    constexpr int CENTRE = DIM == 2 ? 4 : 13;  // the row's own cell in its stencil
    constexpr int NQ = 8;                      // slots read per lane at a time
    __shared__ TileHalo H;
    __shared__ FS S;
    __shared__ double red_lds[3][PB];
    const int lane = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int64_t tile = tile_of_block(k.ntiles);
    const int64_t n = *m.n;
    const int64_t C = k.cap;
    int org[3] = {0, 0, 0};
    bool have = tile >= 0;
    if (have) have = tile_load<DIM>(k, tile, table, H, org);
    double fbg[3] = {0, 0, 0};  // this group's body force over its rows
    if (have) {
        const int total = H.total();
        const int nst = total < FS::CAP ? total : FS::CAP;
        tile_stage(H, FS::CAP, [&](int f, int64_t j) { S.put(k, m, R, o, f, j); });
        __syncthreads();
        for (int64_t i = H.r0() + grp; i < H.r1(); i += PB) {
            const int t = m.type[i];
            if (t == SPH_FLUID || t == SPH_BODY) {
                const int cnt = nl.count[i];
                // LDS slots of the row's neighbours, written by the search of
                // this bin: the first batch of the lane's entries (lane,
                // lane + G, ...) is read with the count, whatever the count
                // (the row holds lmax entries; those past the count are unused)
                const uint16_t *lrow = lslot + i * k.lmax;
                int fq0[NQ];
#pragma unroll
                for (int b = 0; b < NQ; ++b)
                    fq0[b] = lane + b * G < k.lmax ? int(lrow[lane + b * G]) : 0;
                Sep<DIM, T> sep;
                sep.load_i(k, R, off, cpos, i);
                int c[3] = {0, 0, 0}, lc[3] = {0, 0, 0};
                unpack_cell<DIM>(cpos[i], c);
#pragma unroll
                for (int d = 0; d < DIM; ++d) lc[d] = c[d] - org[d];
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
                // the row's own slot, in its stencil's centre cell
                const int hc = halo_index<DIM>(k, lc, CENTRE);
                const int self = H.off(hc) + int(i - H.gbeg(hc));
                bool bad = false;
                // the neighbour average of eq:pavg enters the fluid's momentum;
                // the body force takes p~ about zero
                double pbar = 0.0;
                if (t == SPH_FLUID && !(k.flags & SPH_FLAG_NO_PAVG)) {
                    Acc<T> sp;
                    for (int q0 = lane; q0 < cnt; q0 += NQ * G) {
                        int fq[NQ];
#pragma unroll
                        for (int b = 0; b < NQ; ++b)
                            fq[b] = q0 == lane ? fq0[b]
                                               : (q0 + b * G < cnt ? int(lrow[q0 + b * G]) : 0);
#pragma unroll
                        for (int b = 0; b < NQ; ++b) {
                            if (q0 + b * G >= cnt) continue;
                            const int f = fq[b];
                            if (f >= total) {
                                bad = true;
                                continue;
                            }
                            T pj = S.pres(f < nst ? f : 0);
                            if (f >= nst) pj = ld<T>(R.p, halo_row(H, f));
                            sp.add(pj);
                        }
                    }
                    pbar = gsum<G>(sp.s) / double(cnt);
                }
                const T pavg = T(pbar);
                Acc<T> acc[3], gacc[3], pdot;
                double fb[3] = {0, 0, 0};
                for (int q0 = lane; q0 < cnt; q0 += NQ * G) {
                    int fq[NQ];
#pragma unroll
                    for (int b = 0; b < NQ; ++b)
                        fq[b] = q0 == lane ? fq0[b]
                                           : (q0 + b * G < cnt ? int(lrow[q0 + b * G]) : 0);
                    const int left = (cnt - q0 + G - 1) / G;  // the lane's entries left
                    const int nq = left < NQ ? left : NQ;
                    // one neighbour at a time (the batch is shifted down), so
                    // that the pair terms are not replicated per slot
#pragma unroll 1
                    for (int b = 0; b < nq; ++b) {
                        const int f = fq[0];
#pragma unroll
                        for (int x = 0; x + 1 < NQ; ++x) fq[x] = fq[x + 1];
                        if (f >= total) {
                            bad = true;
                            continue;
                        }
                        if (f == self) continue;
                        NbrRaw<DIM, T> raw;
                        if (f < nst) S.get(f, 0, raw);
                        else fetch_nbr<DIM, T>(k, m, R, o, halo_row(H, f), raw);
                        Nbr<DIM, T> nb;
                        finish_nbr<DIM, T>(k, sep, raw, nb);
                        if (t == SPH_BODY && nb.tj != SPH_FLUID) continue;
                        pair_acc<DIM, T>(k, t, ui, wi, pi, rhoi, vi2, nb, acc, gacc, pdot);
                    }
                }
                if (bad) raise_error(err, SPH_ERR_CELL_RANGE);
                T a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
                finish_rates<DIM, T, G>(k, t, acc, gacc, double(pi) - pbar, a, b, fb);
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
int tile_grid(const Dev &k)
{
    const int64_t per = int64_t(8) * kTileChunk;
    return int((k.ntiles + per - 1) / per * per);
}

void launch_tile_table(const Dev &k, const int64_t *nrows, const int32_t *cell_start,
                       const uint32_t *spread, const uint32_t *cpos, const int32_t *sorted,
                       int32_t *table, uint32_t *err, hipStream_t s)
{
    const dim3 g(unsigned((k.ntiles + kBlock / 64 - 1) / (kBlock / 64))), b(kBlock);
    if (k.dim == 2)
        hipLaunchKernelGGL(k_tile_table<2>, g, b, 0, s, k, nrows, cell_start, spread, cpos, sorted,
                           table, err);
    else
        hipLaunchKernelGGL(k_tile_table<3>, g, b, 0, s, k, nrows, cell_start, spread, cpos, sorted,
                           table, err);
}

template <int DIM, typename T>
static void tsearch_dt(const Dev &k, const DevState &m, const Fields &R, const DevNlist &nl,
                       const DevDerived &o, int dens, const int32_t *table, const uint32_t *cpos,
                       float *off, uint16_t *lslot, int32_t *rebin_clear, const VList &v,
                       int vmode, uint32_t *err, hipStream_t s)
{
#define SPH_TS_G(G)                                                                        \
    hipLaunchKernelGGL((k_tsearch<DIM, T, G>), dim3(tile_grid(k)), dim3(kBlock), 0, s, k, m, R, \
                       nl, o, dens, table, cpos, off, lslot, rebin_clear, v, vmode, err)
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
                    const DevDerived &o, int dens, const int32_t *table, const uint32_t *cpos,
                    float *off, uint16_t *lslot, int32_t *rebin_clear, const VList &v, int vmode,
                    uint32_t *err, hipStream_t s)
{
#define SPH_TS(D, TT) \
    tsearch_dt<D, TT>(k, m, R, nl, o, dens, table, cpos, off, lslot, rebin_clear, v, vmode, err, s)
    if (k.dim == 2 && k.prec == SPH_FP64) SPH_TS(2, double);
    else if (k.dim == 3 && k.prec == SPH_FP64) SPH_TS(3, double);
    else if (k.dim == 2) SPH_TS(2, float);
    else SPH_TS(3, float);
#undef SPH_TS
}

template <int DIM, typename T>
static void tforce_dt(const Dev &k, const DevState &m, const Fields &R, const Fields &W,
                      const DevNlist &nl, const DevDerived &o, const float *off,
                      const uint32_t *cpos, const int32_t *table, const uint16_t *lslot,
                      int mode, int want_drag, double *dragpart, const double *xbin,
                      int32_t *rebin, uint32_t *err, hipStream_t s)
{
#define SPH_TF_G(G)                                                                        \
    hipLaunchKernelGGL((k_tforce<DIM, T, G>), dim3(tile_grid(k)), dim3(kBlock), 0, s, k, m, R, \
                       W, nl, o, off, cpos, table, lslot, mode, want_drag, dragpart, xbin,     \
                       rebin, err)
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
                   const uint32_t *cpos, const int32_t *table, const uint16_t *lslot, int mode,
                   int want_drag, double *dragpart, const double *xbin, int32_t *rebin,
                   uint32_t *err, hipStream_t s)
{
#define SPH_TF(D, TT)                                                                    \
    tforce_dt<D, TT>(k, m, R, W, nl, o, off, cpos, table, lslot, mode, want_drag, dragpart, \
                     xbin, rebin, err, s)
    if (k.dim == 2 && k.prec == SPH_FP64) SPH_TF(2, double);
    else if (k.dim == 3 && k.prec == SPH_FP64) SPH_TF(3, double);
    else if (k.dim == 2) SPH_TF(2, float);
    else SPH_TF(3, float);
#undef SPH_TF
}

}  // namespace sph
