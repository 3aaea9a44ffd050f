// pairs.hip -- neighbour-pair passes of libsph for gfx950: fused neighbour
// table + summation density, boundary values (walls, hybrid outlet, MOC
// inlet) and the EDAC-TVF force pass (optionally fused with the RK2 stage
// update) with the body force.
//
// Work decomposition: a group of G lanes (a template parameter the host picks
// from the particle count) owns one target particle and each lane a subset of
// its neighbours, so several neighbour gathers of a target are in flight at
// once and small particle counts still put thousands of waves on the 256 CUs. Per-target sums are
// reduced across the group with lane shuffles; in FP32 the terms are summed
// in FP64 per lane and across the group, then rounded once. Particles are Morton-sorted, the neighbour table is row-major
// (the neighbours of one target are contiguous, one coalesced load per group)
// and the block -> particle-range mapping is XCD-aware so that each of the 8
// XCDs works on a contiguous slab and its L2 serves the neighbour re-reads.
#include "pair_terms.h"
#include "sph_launch.h"

namespace sph {

// ---------------------------------------------- neighbour table + density
// The 3^d stencil cells, taken in (dz, dy, dx) order and each in member
// order, form one candidate sequence per target; the group's lanes test
// candidates lane, lane + G, ... of that sequence with the FMA-free FP64
// predicate |r|^2 < (2h)^2 and hits are compacted with a ballot, so the table
// keeps the stencil-then-cell order. Walking the concatenated sequence (cell
// ranges staged in LDS by the group) leaves no lane idle at cell ends and
// loads all cell ranges of a target at once. The density (Sec. 2
// eq:summation-density, V = 1/sum W) is summed from the same pairs when `dens`
// is set. FP32 mode records the cell-relative offsets the force pass uses.
//
// Step path (vmode 1, 2): the candidate lists of VList. vmode 1 is the first
// search of a step: after a sort (*v.fresh) it walks the stencil and also
// records every candidate within rv of the target (a second ballot), else it
// walks the stored list; vmode 2 always walks the stored list. A list is a
// subsequence of the stencil sequence that holds every hit, so both walks
// produce the same table in the same order. vmode 0 walks the stencil only.

// candidates of one lane, NB at a time, from the stencil sequence
template <int NS, int NB, int G>
struct StencilWalk {
    const int32_t *beg, *len;  // the group's cell ranges (LDS)
    int sc, mo;
    __device__ inline StencilWalk(const int32_t *b, const int32_t *l, int lane) : beg(b), len(l)
    {
        sc = 0;
        mo = lane;
        while (sc < NS && mo >= len[sc]) mo -= len[sc++];
    }
    __device__ inline void next(int32_t jj[NB], bool hv[NB])
    {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            hv[b] = sc < NS;
            jj[b] = hv[b] ? beg[sc] + mo : 0;  // row 0 as a harmless dummy
            mo += G;
            while (sc < NS && mo >= len[sc]) mo -= len[sc++];
        }
    }
};

// candidates of one lane, NB at a time, from a stored list (entries beyond the
// live rows are reported and skipped). Entries are read up to the row's
// capacity whatever the count, so that the loads need not wait for it;
// entries past the count are not used.
template <int NB, int G>
struct ListWalk {
    const int32_t *list;
    int32_t pre[NB];  // the first batch, read ahead by the caller
    bool first;
    int q, cnt, cap;
    int64_t n;
    uint32_t *err;
    __device__ inline ListWalk(const int32_t *l, const int32_t ahead[NB], int c, int rowcap,
                               int lane, int64_t nrows, uint32_t *e)
        : list(l), first(true), q(lane), cnt(c), cap(rowcap), n(nrows), err(e)
    {
#pragma unroll
        for (int b = 0; b < NB; ++b) pre[b] = ahead[b];
    }
    __device__ inline void next(int32_t jj[NB], bool hv[NB])
    {
        const bool use_pre = first;
        first = false;
        // every entry loaded before the error word is touched (an atomic
        // between them would keep each load behind the one before)
        int32_t j[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int qb = q + b * G;
            j[b] = use_pre ? pre[b] : (qb < cap ? list[qb] : 0);
        }
        bool any_bad = false;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const bool bad = q < cnt && bad_index(j[b], n);
            any_bad = any_bad || bad;
            hv[b] = q < cnt && !bad;
            jj[b] = hv[b] ? j[b] : 0;
            q += G;
        }
        if (any_bad) raise_error(err, SPH_ERR_CELL_RANGE);
    }
};

// Tests the candidates of one walk (total of them over the group), appends
// hits to the table row and, with `rec`, candidates within rv to the list
// row; returns the group's hit count. The kernel sum is accumulated in table
// order: lane l adds the entries l, l + G, l + 2G, ... (each round's kernel
// values are routed through the group's G slots of LDS to the lane of their
// table position), so the density does not depend on which walk found them.
template <int DIM, typename T, int G, int NB, typename Walk>
__device__ inline int walk_candidates(const Dev &k, const Fields &R, Walk &w, int total,
                                      const double xi[3], int lane, int32_t *row, int maxnb,
                                      bool rec, int32_t *vrow, int &vcnt, int dens, Acc<T> &sw,
                                      T *slots)
{
    const int64_t C = k.cap;
    const int gshift = (threadIdx.x & 63) & ~(G - 1);
    const uint64_t gmask = G == 64 ? ~0ull : ((1ull << (G & 63)) - 1);
    const uint64_t below = (1ull << lane) - 1;
    int cnt = 0;
    for (int base = 0; base < total; base += NB * G) {
        int32_t jj[NB];
        bool hv[NB];
        w.next(jj, hv);
        double xj[NB][3];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
#pragma unroll
            for (int d = 0; d < 3; ++d) xj[b][d] = d < DIM ? R.x[d * C + jj[b]] : 0.0;
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
            if (hit && pos < maxnb) row[pos] = jj[b];
            if (dens && nhit > 0) {
                const T wv = hit ? kernel_w<T>(k, T(sqrt(r2) * k.inv_h), T(k.wnorm)) : T(0);
                if (G == 1) {
                    sw.add(wv);
                } else {
                    if (hit) slots[pos & (G - 1)] = wv;
                    __builtin_amdgcn_wave_barrier();
                    const T got = slots[lane];
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
                if (vhit && vpos < k.vmax) vrow[vpos] = jj[b];
                vcnt += nv;
            }
        }
    }
    return cnt;
}

template <int DIM, typename T, int G>
__global__ void __launch_bounds__(kBlock) k_nbrdens(Dev k, DevState m, Fields R, DevNlist nl,
                                                    DevDerived o, int dens,
                                                    const uint32_t *spread,
                                                    const int32_t *cell_start,
                                                    const uint32_t *cpos, float *off,
                                                    int32_t *rebin_clear, VList v, int vmode,
                                                    uint32_t *err)
{
    // the step's bin has run: later updates of this step may request the next
    if (rebin_clear && blockIdx.x == 0 && threadIdx.x == 0) *rebin_clear = 0;
    constexpr int PB = kBlock / G;
    constexpr int NS = DIM == 2 ? 9 : 27;
    constexpr int NB = 4;
    __shared__ int32_t s_beg[PB][NS], s_len[PB][NS];
    __shared__ T s_w[PB][G];
    const int lane = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int64_t n = *m.n;
    const int64_t lb = xcd_block((n + PB - 1) / PB);
    const int64_t i = lb * PB + grp;
    const bool active = lb >= 0 && i < n;  // uniform across the group
    const int64_t C = k.cap;
    // walk of this target: the stored list (vc >= 0) or the stencil
    const bool build = vmode == 1 && *v.fresh != 0;
    int vc = -1;
    if (active && vmode != 0 && !build) vc = v.count[i];
    double xi[3] = {0, 0, 0};
    int c[3] = {0, 0, 0};
    if (active) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) xi[d] = R.x[d * C + i];
        unpack_cell<DIM>(cpos[i], c);
    }
    // first batch of a stored list, read in the same round trip as its count
    int32_t *vrow = v.nbr + i * int64_t(k.vmax);
    int32_t vpre[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
        vpre[b] = (active && vmode != 0 && !build && lane + b * G < k.vmax) ? vrow[lane + b * G]
                                                                            : 0;
    if (active && vc < 0) {
        // cell ranges of the stencil, one cell per lane at a time; all ranges
        // of a lane are loaded before the error word is touched (an atomic
        // between them would keep each load behind the one before)
        constexpr int NSL = (NS + G - 1) / G;  // stencil cells per lane, at most
        int32_t cb[NSL], ce[NSL];
#pragma unroll
        for (int u = 0; u < NSL; ++u) {
            const int sc = lane + u * G;
            cb[u] = ce[u] = 0;
            if (sc >= NS) continue;
            const int dxs = sc % 3 - 1, dys = (sc / 3) % 3 - 1, dzs = DIM == 3 ? sc / 9 - 1 : 0;
            int cc[3] = {c[0] + dxs, c[1] + dys, c[2] + dzs};
            bool ok = true;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                if (cc[d] < 0 || cc[d] >= k.nc[d]) {
                    if (k.periodic[d]) cc[d] = cc[d] < 0 ? cc[d] + k.nc[d] : cc[d] - k.nc[d];
                    else ok = false;
                }
            }
            if (ok) {
                const uint32_t key = morton_key<DIM>(spread, cc);
                cb[u] = cell_start[key];
                ce[u] = cell_start[key + 1];
            }
        }
        bool any_bad = false;
#pragma unroll
        for (int u = 0; u < NSL; ++u) {
            const int sc = lane + u * G;
            if (sc >= NS) continue;
            int32_t b = cb[u], e = ce[u];
            if (b < 0 || e > n || b > e) {
                any_bad = true;
                b = e = 0;
            }
            s_beg[grp][sc] = b;
            s_len[grp][sc] = e - b;
        }
        if (any_bad) raise_error(err, SPH_ERR_CELL_RANGE);
    }
    __syncthreads();
    if (!active) return;
    int32_t *row = nl.nbr + i * nl.maxnb;
    Acc<T> sw;
    int cnt, vcnt = 0;
    if (vc >= 0) {
        ListWalk<NB, G> w(vrow, vpre, vc, k.vmax, lane, n, err);
        cnt = walk_candidates<DIM, T, G, NB>(k, R, w, vc, xi, lane, row, nl.maxnb, false, vrow,
                                             vcnt, dens, sw, s_w[grp]);
    } else {
        int total = 0;
#pragma unroll
        for (int sc = 0; sc < NS; ++sc) total += s_len[grp][sc];
        StencilWalk<NS, NB, G> w(s_beg[grp], s_len[grp], lane);
        cnt = walk_candidates<DIM, T, G, NB>(k, R, w, total, xi, lane, row, nl.maxnb, build, vrow,
                                             vcnt, dens, sw, s_w[grp]);
    }
    const T S = sw.template reduce<G>();
    if (lane == 0) {
        if (cnt > nl.maxnb) {
            raise_error(err, SPH_ERR_NBR_OVERFLOW);
            cnt = nl.maxnb;
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
        if (dens && o.rec) write_rec<DIM, T, G>(k, m, R, o.rec, i, S, xi, c, cpos[i], lane);
    if (sizeof(T) == 4) {
        // offsets from the bin cell's corner, for the FP32 pair arithmetic
        for (int d = lane; d < DIM; d += G)
            off[d * C + i] = cell_offset(k, d, xi[d], c[d]);
    }
}

// Summation density from an existing neighbour table (the API path; the step
// path sums it while building the table).
template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_density(Dev k, DevState m, Fields R, DevNlist nl,
                                                    DevDerived o, const uint32_t *cpos,
                                                    uint32_t *err)
{
    using P = Grp<DIM>;
    constexpr int G = P::G;
    const int lane = threadIdx.x & (G - 1);
    const int64_t n = *m.n;
    const int64_t lb = xcd_block((n + P::PER_BLOCK - 1) / P::PER_BLOCK);
    const int64_t i = lb * P::PER_BLOCK + threadIdx.x / G;
    if (lb < 0 || i >= n) return;
    const int64_t C = k.cap;
    double xi[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) xi[d] = R.x[d * C + i];
    const int cnt = nl.count[i];
    Acc<T> sw;
    for (int q = lane; q < cnt; q += G) {
        const int32_t j = nl.nbr[i * nl.maxnb + q];
        if (bad_index(j, n)) {
            raise_error(err, SPH_ERR_CELL_RANGE);
            continue;
        }
        double xj[3] = {0, 0, 0};
#pragma unroll
        for (int d = 0; d < DIM; ++d) xj[d] = R.x[d * C + j];
        double r[3];
        sw.add(kernel_w<T>(k, T(sqrt(dist2_exact<DIM>(k, xi, xj, r)) * k.inv_h), T(k.wnorm)));
    }
    const T S = sw.template reduce<G>();
    if (lane == 0) {
        st<T>(o.rho, i, T(k.mass) * S);
        st<T>(o.vol, i, T(1) / S);
        if (o.shep) st<T>(o.shep, i, S);
    }
    if constexpr (sizeof(T) == 4 && DIM == 2) {
        if (o.rec) {
            int c[3] = {0, 0, 0};
            const uint32_t cp = cpos[i];
            unpack_cell<DIM>(cp, c);
            write_rec<DIM, T, G>(k, m, R, o.rec, i, S, xi, c, cp, lane);
        }
    }
}

// 3D neighbour records of every live row from the stage's fields, after the
// boundary pass has set its rows' values, and the Shepard sums of the density
// pass: FP64 chunk-major (x, p, u, w, S, kind), FP32 row-major (cell offsets
// as the offset array holds them, p, u, w, S, kind class and packed cell).
// One thread per row, so that each field load and each chunk store is
// coalesced across the wave: written inside the neighbour search, whose
// gathers already saturate the vector memory path, the same records cost
// about twice as long, and the boundary pass would have to patch its rows'
// slots. Every load is issued before the first store.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_pack_rec(Dev k, DevState m, Fields R, DevDerived o,
                                                     const uint32_t *cpos)
{
    using L = Rec<3, T>;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= *m.n) return;
    const int64_t C = k.cap;
    T v[L::NC * L::PER];
#pragma unroll
    for (int q = 0; q < L::NC * L::PER; ++q) v[q] = T(0);
    double x[3];
    T ut[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        x[d] = R.x[d * C + i];
        v[L::U + d] = ld<T>(R.u, d * C + i);
        ut[d] = ld<T>(R.ut, d * C + i);
    }
    v[L::P] = ld<T>(R.p, i);
    v[L::VOL] = ld<T>(o.shep, i);
    const uint32_t t = m.type[i];
    uint32_t cp = 0;
    if constexpr (L::F32) cp = cpos[i];
#pragma unroll
    for (int d = 0; d < 3; ++d) v[L::W + d] = ut[d] - v[L::U + d];
    if constexpr (L::F32) {
        int c[3] = {0, 0, 0};
        unpack_cell<3>(cp, c);
#pragma unroll
        for (int d = 0; d < 3; ++d) v[L::X + d] = cell_offset(k, d, x[d], c[d]);
        v[L::AUX] = rec_word<T>(cp | (kind_class(int(t)) << 30));
    } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) v[L::X + d] = x[d];
        v[L::AUX] = rec_word<T>(t);
    }
#pragma unroll
    for (int ch = 0; ch < L::NC; ++ch)
        *rec_chunk<3, T>(o.rec, C, i, ch) = Chunk<T>::make(v + ch * L::PER);
}

// Record slots of the boundary values of row i (p, u, ut - u), from the very
// values the state receives, so that record and state agree bit for bit.
template <int DIM, typename T>
__device__ inline void rec_put_pu(void *rec, int64_t cap, int64_t i, T p, const T u[3],
                                  const T ut[3])
{
    using L = Rec<DIM, T>;
    static_assert(L::USE, "no records in this form");
    *rec_slot<DIM, T>(rec, cap, i, L::P) = p;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        *rec_slot<DIM, T>(rec, cap, i, L::U + d) = u[d];
        *rec_slot<DIM, T>(rec, cap, i, L::W + d) = ut[d] - u[d];
    }
}

// ------------------------------------------------------------------ mirror
// Sec. 3.2, eq:matform: first-order corrected estimate of p and the velocity
// components and their gradients at the point xk from the fluid particles l
// within the kernel support of xk (x_lk = x_l - x_k, W_b = F (x_l - x_k)_b,
// V_l = 1/S_l), found by walking the 3^d cells around xk's cell (cells are
// at least support + 2 disp_max wide, so binned rows within the skin are
// covered); the group's lanes take cells in turn and the sums are reduced
// over the group. Gaussian elimination with partial pivoting on the
// dimensionless system (x_lk / h in the columns, the derivative rows times
// h); where a pivot falls below 1e-3 of the largest entry (sources nearly on
// a line), the zeroth-order Shepard value with zero gradient. Returns false
// without fluid in the support; sol[f][0] is field f (p, u_x, u_y[, u_z]),
// sol[f][1 + b] its derivative along b.
template <int DIM, typename T, int G>
__device__ inline bool mirror_fit(const Dev &k, const DevState &m, const Fields &R,
                                  const DevDerived &o, const uint32_t *spread,
                                  const int32_t *cell_start, int64_t n, const double xk[3],
                                  int lane, uint32_t *err, double sol[DIM + 1][DIM + 1])
{
    constexpr int NE = DIM + 1;
    constexpr int NS = DIM == 2 ? 9 : 27;
    const int64_t C = k.cap;
    double A[NE][NE], B[NE][NE];  // B[row][field]
#pragma unroll
    for (int a = 0; a < NE; ++a)
#pragma unroll
        for (int c = 0; c < NE; ++c) A[a][c] = B[a][c] = 0.0;
    int ck[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const double f = floor((xk[d] - k.lo[d]) * k.inv_cs[d]);
        ck[d] = !(f >= 0.0) ? 0 : (f >= double(k.nc[d]) ? k.nc[d] - 1 : int(f));
    }
    for (int sc = lane; sc < NS; sc += G) {
        const int dxs = sc % 3 - 1, dys = (sc / 3) % 3 - 1, dzs = DIM == 3 ? sc / 9 - 1 : 0;
        int cc[3] = {ck[0] + dxs, ck[1] + dys, ck[2] + dzs};
        bool ok = true;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            if (cc[d] < 0 || cc[d] >= k.nc[d]) {
                if (k.periodic[d]) cc[d] = cc[d] < 0 ? cc[d] + k.nc[d] : cc[d] - k.nc[d];
                else ok = false;
            }
        }
        if (!ok) continue;
        const uint32_t key = morton_key<DIM>(spread, cc);
        const int32_t b = cell_start[key], e = cell_start[key + 1];
        if (b < 0 || e > n || b > e) {
            raise_error(err, SPH_ERR_CELL_RANGE);
            continue;
        }
        for (int32_t l = b; l < e; ++l) {
            if (m.type[l] != SPH_FLUID) continue;
            double xl[3] = {0, 0, 0}, r[3];
#pragma unroll
            for (int d = 0; d < DIM; ++d) xl[d] = R.x[d * C + l];
            const double r2 = dist2_exact<DIM>(k, xl, xk, r);  // r = x_l - x_k
            if (!(r2 < k.sup2)) continue;
            const double q = sqrt(r2) * k.inv_h;
            const double V = double(ld<T>(o.vol, l));
            const double w = kernel_w<double>(k, q, k.wnorm) * V;
            const double F = k.h * kernel_f<double>(k, q, k.gnorm) * V;
            double rowm[NE], col[NE], fl[NE];
            rowm[0] = w;
            col[0] = 1.0;
            fl[0] = double(ld<T>(R.p, l));
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                rowm[1 + d] = F * r[d];
                col[1 + d] = r[d] * k.inv_h;
                fl[1 + d] = double(ld<T>(R.u, d * C + l));
            }
#pragma unroll
            for (int a = 0; a < NE; ++a)
#pragma unroll
                for (int c = 0; c < NE; ++c) {
                    A[a][c] += rowm[a] * col[c];
                    B[a][c] += rowm[a] * fl[c];
                }
        }
    }
#pragma unroll
    for (int a = 0; a < NE; ++a)
#pragma unroll
        for (int c = 0; c < NE; ++c) {
            A[a][c] = gsum<G>(A[a][c]);
            B[a][c] = gsum<G>(B[a][c]);
        }
    if (!(A[0][0] > 0.0)) return false;
    double amax = 0.0;
#pragma unroll
    for (int a = 0; a < NE; ++a)
#pragma unroll
        for (int c = 0; c < NE; ++c) amax = fmax(amax, fabs(A[a][c]));
    double shep[NE];
#pragma unroll
    for (int f = 0; f < NE; ++f) shep[f] = B[0][f] / A[0][0];
    bool singular = false;
#pragma unroll
    for (int c = 0; c < NE; ++c) {
        if (singular) break;
        int pr = c;
#pragma unroll
        for (int a = c + 1; a < NE; ++a)
            if (fabs(A[a][c]) > fabs(A[pr][c])) pr = a;
        if (!(fabs(A[pr][c]) > 1e-3 * amax)) {
            singular = true;
            break;
        }
        if (pr != c) {
#pragma unroll
            for (int x = 0; x < NE; ++x) {
                double t = A[c][x];
                A[c][x] = A[pr][x];
                A[pr][x] = t;
                t = B[c][x];
                B[c][x] = B[pr][x];
                B[pr][x] = t;
            }
        }
#pragma unroll
        for (int a = c + 1; a < NE; ++a) {
            const double mul = A[a][c] / A[c][c];
#pragma unroll
            for (int x = 0; x < NE; ++x) {
                if (x >= c) A[a][x] -= mul * A[c][x];
                B[a][x] -= mul * B[c][x];
            }
        }
    }
#pragma unroll
    for (int f = 0; f < NE; ++f) {
        if (singular) {
            sol[f][0] = shep[f];
#pragma unroll
            for (int d = 0; d < DIM; ++d) sol[f][1 + d] = 0.0;
            continue;
        }
        double xs[NE];
#pragma unroll
        for (int a = NE - 1; a >= 0; --a) {
            double v = B[a][f];
#pragma unroll
            for (int c = a + 1; c < NE; ++c) v -= A[a][c] * xs[c];
            xs[a] = v / A[a][a];
        }
        sol[f][0] = xs[0];
#pragma unroll
        for (int d = 0; d < DIM; ++d) sol[f][1 + d] = xs[1 + d] * k.inv_h;
    }
    return true;
}

// ---------------------------------------------------------- boundary values
// Over the non-fluid rows listed at bin time. Walls: Shepard-averaged fluid
// pressure and ghost velocity u_g = -<u_f> (static walls, no body force).
// Outlet: characteristic variables of the fluid with the fluid's own time
// averages as references (Sec. 3.3 eq:characteristic-vars, Sec. 3.4),
// Shepard-interpolated (eq:shepard), J3 = 0; without fluid support the mean
// previous-step value of same-kind neighbours that had support
// (eq:average_old), else the particle's own; then u, p = time average +
// acoustic part (eq:acou) with rho_ref = rho0. The other outlet rules: fixed
// references u = U, p = 0 with the transverse velocity unchanged (Sec. 3.3);
// u, p frozen (Sec. 3.1), with the Shepard mean of the fluid x velocity as
// the advection speed (Sec. 3.1.1, eq:shepard0; the blue fallback as above).
// Inlet: prescribed velocity, p = Shepard J3 with reference (u_in, 0). Always
// FP64 arithmetic.
template <int DIM, typename T, int G, bool MIR>
__global__ void __launch_bounds__(kBlock) k_boundary(Dev k, DevState m, Fields R, DevNlist nl,
                                                     DevDerived o, const int32_t *blist,
                                                     const int32_t *bcount,
                                                     const uint32_t *spread,
                                                     const int32_t *cell_start, uint32_t *err)
{
    constexpr int PB = kBlock / G;
    const int lane = threadIdx.x & (G - 1);
    const int64_t n = *m.n;
    const int64_t nbnd = *bcount;
    const int64_t C = k.cap;
    const int64_t stride = int64_t(gridDim.x) * PB;
    // each row index is read one iteration ahead (the first before the count
    // of rows arrives; the list holds cap entries, those past the count are
    // not used)
    int64_t g = int64_t(blockIdx.x) * PB + threadIdx.x / G;
    int32_t inext = g < C ? blist[g] : -1;
    for (; g < nbnd; g += stride) {
        const int64_t i = inext;
        inext = g + stride < C ? blist[g + stride] : -1;
        if (bad_index(int32_t(i), n)) {
            raise_error(err, SPH_ERR_CELL_RANGE);
            continue;
        }
        // the row's kind, values, neighbour count and first neighbour index
        // in one round trip
        const int t = m.type[i];
        double xi[3] = {0, 0, 0};
#pragma unroll
        for (int d = 0; d < DIM; ++d) xi[d] = R.x[d * C + i];
        const double uin0 = m.uin[i];
        const int cnt = nl.count[i];
        const int32_t j0 = lane < nl.maxnb ? nl.nbr[i * nl.maxnb + lane] : -1;
        if (t == SPH_FLUID) continue;
        const bool io = t == SPH_INLET || t == SPH_OUTLET;
        // What the write-out below reads of the row itself, loaded with the
        // neighbours: loads placed after its stores would each wait for them
        // (the compiler cannot rule out aliasing). Inlet/outlet rows: p, u,
        // u_in, the averages and the previous-step J; walls with records: ut.
        T p_old = T(0), u_old[3] = {T(0), T(0), T(0)}, ut_old[3] = {T(0), T(0), T(0)};
        double avg_i[4] = {0, 0, 0, 0}, uin_i[3] = {0, 0, 0}, jprev_i[3] = {0, 0, 0};
        if (io) {
            p_old = ld<T>(R.p, i);
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                u_old[d] = ld<T>(R.u, d * C + i);
                uin_i[d] = m.uin[d * C + i];
            }
#pragma unroll
            for (int c = 0; c <= DIM; ++c) avg_i[c] = m.avg[c * C + i];
#pragma unroll
            for (int a = 0; a < 3; ++a) jprev_i[a] = m.jprev[a * C + i];
        } else if (o.rec) {
#pragma unroll
            for (int d = 0; d < DIM; ++d) ut_old[d] = ld<T>(R.ut, d * C + i);
        }
        // the hybrid outlet's characteristic references are the neighbours'
        // time averages
        const bool hyb_avg = t == SPH_OUTLET && k.outlet == SPH_OUTLET_HYBRID;
        // Shepard sums over fluid neighbours and, in the same sweep, the
        // fallback sums over same-kind neighbours that had support
        double sw = 0.0, sp = 0.0, su[3] = {0, 0, 0}, sJ[3] = {0, 0, 0};
        double bacc[3] = {0, 0, 0}, bM = 0.0;
        for (int q = lane; q < cnt; q += G) {
            const int32_t j = q == lane ? j0 : nl.nbr[i * nl.maxnb + q];
            if (bad_index(j, n)) {
                raise_error(err, SPH_ERR_CELL_RANGE);
                continue;
            }
            // the neighbour's kind and the fluid values are loaded together
            // (one round trip); the values of non-fluid rows are not used
            const int tj = m.type[j];
            double xj[3] = {0, 0, 0}, uj[3] = {0, 0, 0};
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                xj[d] = R.x[d * C + j];
                uj[d] = double(ld<T>(R.u, d * C + j));
            }
            const double pj = double(ld<T>(R.p, j));
            const double rhoj = double(ld<T>(o.rho, j));
            // inlet/outlet rows: the neighbour's red flag, previous-step J and
            // (hybrid outlet) time averages go out with its kind, so that no
            // load waits for it; wall rows skip them
            uint8_t rpj = 0;
            double jpj[3] = {0, 0, 0}, avu = 0.0, avp = 0.0;
            if (io) {
                rpj = m.red_prev[j];
#pragma unroll
                for (int a = 0; a < 3; ++a) jpj[a] = m.jprev[a * C + j];
                if (hyb_avg) {
                    avu = m.avg[j];
                    avp = m.avg[DIM * C + j];
                }
            }
            if (io && tj == t && rpj) {
#pragma unroll
                for (int a = 0; a < 3; ++a) bacc[a] += jpj[a];
                bM += 1.0;
            }
            if (tj != SPH_FLUID) continue;
            double r[3];
            const double w =
                kernel_w<double>(k, sqrt(dist2_exact<DIM>(k, xi, xj, r)) * k.inv_h, k.wnorm);
            const double uj0 = uj[0];
            sw += w;
            sp += pj * w;
#pragma unroll
            for (int d = 0; d < DIM; ++d) su[d] += uj[d] * w;
            if (t == SPH_INLET && !(k.flags & SPH_FLAG_MIRROR_INLET)) {
                sJ[2] += (-rhoj * k.c * (uj0 - uin0) + pj) * w;
            } else if (t == SPH_OUTLET && k.outlet == SPH_OUTLET_MOD_DO_NOTHING) {
                sJ[0] += uj0 * w;  // eq:shepard0, the fluid x velocity
            } else if (t == SPH_OUTLET && k.outlet != SPH_OUTLET_DO_NOTHING &&
                       k.outlet != SPH_OUTLET_MIRROR) {
                // references: the fluid particle's time averages (hybrid) or
                // the fixed u = U, p = 0 (characteristics)
                const bool moc = k.outlet == SPH_OUTLET_MOC;
                const double dp = pj - (moc ? 0.0 : avp);
                const double du = uj0 - (moc ? k.U : avu);
                sJ[0] += (-k.c2 * (rhoj - k.rho0) + dp) * w;
                sJ[1] += (rhoj * k.c * du + dp) * w;
                sJ[2] += (-rhoj * k.c * du + dp) * w;
            }
        }
        // group reductions of the sums this kind uses (the kind is uniform
        // across the group)
        sw = gsum<G>(sw);
        if (is_wall(t)) {
            sp = gsum<G>(sp);
#pragma unroll
            for (int d = 0; d < DIM; ++d) su[d] = gsum<G>(su[d]);
        } else if (t == SPH_OUTLET) {
#pragma unroll
            for (int a = 0; a < 3; ++a) sJ[a] = gsum<G>(sJ[a]);
        } else {
            sJ[2] = gsum<G>(sJ[2]);
        }
        if (is_wall(t)) {
            if (lane == 0) {
                double pw = 0.0;
                double ug[3] = {0, 0, 0};
                if (sw > 0.0) {
                    pw = sp / sw;
#pragma unroll
                    for (int d = 0; d < DIM; ++d) ug[d] = -(su[d] / sw);
                }
                T uw[3] = {T(0), T(0), T(0)};
#pragma unroll
                for (int d = 0; d < DIM; ++d) uw[d] = T(ug[d]);
                o.sfl[i] = sw;
                st<T>(R.p, i, T(pw));
#pragma unroll
                for (int d = 0; d < DIM; ++d) st<T>(R.u, d * C + i, uw[d]);
                if constexpr (Rec<DIM, T>::USE) {
                    if (o.rec) rec_put_pu<DIM, T>(o.rec, C, i, T(pw), uw, ut_old);
                }
            }
            continue;
        }
        double J[3];
        uint8_t red;
        if (sw > 0.0) {
            red = 1;
#pragma unroll
            for (int a = 0; a < 3; ++a) J[a] = sJ[a] / sw;
            if (t == SPH_OUTLET) J[2] = 0.0;
        } else {
            red = 0;
            const double M = gsum<G>(bM);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double acc = gsum<G>(bacc[a]);
                J[a] = M > 0.0 ? acc / M : jprev_i[a];
            }
        }
        // mirroring (Sec. 3.2): the row reflected about its interface into
        // the fluid; the group fits p and u there (eq:matform). A separate
        // instantiation (MIR) keeps the fit's registers out of the other runs
        // (measured: 215 VGPRs in 3D, the 4.6M-particle pass 223 -> 380 us).
        const bool mir = MIR && ((t == SPH_OUTLET && k.outlet == SPH_OUTLET_MIRROR) ||
                                 (t == SPH_INLET && (k.flags & SPH_FLAG_MIRROR_INLET)));
        double mval[4] = {0, 0, 0, 0};
        bool mok = false;
        if constexpr (MIR) if (mir) {
            double xk[3] = {xi[0], xi[1], xi[2]};
            xk[0] = 2.0 * (t == SPH_OUTLET ? k.x_outlet : k.x_inlet) - xi[0];
            double sol[DIM + 1][DIM + 1];
            mok = mirror_fit<DIM, T, G>(k, m, R, o, spread, cell_start, n, xk, lane, err, sol);
            if (mok) {
                // eq:taylor2: f_i = f_k - (r_i - r_k) . grad f_k
#pragma unroll
                for (int f = 0; f <= DIM; ++f) {
                    double v = sol[f][0];
#pragma unroll
                    for (int d = 0; d < DIM; ++d) v -= (xi[d] - xk[d]) * sol[f][1 + d];
                    mval[f] = v;
                }
            }
        }
        if (lane == 0) {
            // the row's new p, u, ut (kept where the rule leaves them)
            T pv = p_old, uv[3], utv[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) uv[d] = utv[d] = u_old[d];
            if (t == SPH_OUTLET && k.outlet == SPH_OUTLET_HYBRID) {
                const double p_ac = 0.5 * (J[1] + J[2]);
                const double u_ac = (J[1] - J[2]) / (2.0 * k.rho0 * k.c);
                pv = T(avg_i[DIM] + p_ac);
                uv[0] = utv[0] = T(avg_i[0] + u_ac);
#pragma unroll
                for (int d = 1; d < DIM; ++d) uv[d] = utv[d] = T(avg_i[d]);
            } else if (t == SPH_OUTLET && k.outlet == SPH_OUTLET_MOC) {
                // about the fixed references; transverse velocity unchanged
                const double p_ac = 0.5 * (J[1] + J[2]);
                const double u_ac = (J[1] - J[2]) / (2.0 * k.rho0 * k.c);
                pv = T(0.0 + p_ac);
                uv[0] = utv[0] = T(k.U + u_ac);
            } else if (t == SPH_OUTLET) {
                // mirror: p and u from the mirror point (kept without fluid
                // there); do-nothing rules: u, p stay frozen
                if (mok) {
                    pv = T(mval[0]);
#pragma unroll
                    for (int d = 0; d < DIM; ++d) uv[d] = T(mval[1 + d]);
                }
#pragma unroll
                for (int d = 0; d < DIM; ++d) utv[d] = uv[d];
            } else {  // inlet: prescribed velocity, p = J3 or mirrored
                if (!mir) pv = T(J[2]);
                else if (mok) pv = T(mval[0]);
#pragma unroll
                for (int d = 0; d < DIM; ++d) uv[d] = utv[d] = T(uin_i[d]);
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) o.jcur[a * C + i] = J[a];
            o.red[i] = red;
            o.sfl[i] = sw;
            st<T>(R.p, i, pv);
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                st<T>(R.u, d * C + i, uv[d]);
                st<T>(R.ut, d * C + i, utv[d]);
            }
            if constexpr (Rec<DIM, T>::USE) {
                if (o.rec) rec_put_pu<DIM, T>(o.rec, C, i, pv, uv, utv);
            }
        }
    }
}

// ---------------------------------------------------------------- force pass
// Fluid i, in one sweep over its neighbours: pbar_i (eq:pavg, self included)
// and over j != i the momentum rate of eq:tvf-momentum with p~_ij of
// eq:tvf-p-ij-basa (its pbar_i part applied after the sweep, see pair_acc),
// the background term of eq:transport-vel and the pressure rate of eq:p-edac. A = rho u (ut - u)
// for fluid, 0 otherwise; slip walls take no viscous part; walls enter the
// divergence with zero wall velocity and the viscous term with u_g.
// Body i: force of eq:tvf-momentum_solid from fluid neighbours.
//
// mode 0 writes a, b, pdot, pavg (and force for body rows). Modes 1 (half)
// and 2 (full) instead apply the explicit-midpoint stage update from the
// start-of-step values,
//     u = u0 + dt a,  p = p0 + dt pdot,  ut = u + dt b,  x = x0 + dt ut_half,
// reading the stage state R and writing W. Half: R is the start state and W
// the half state. Full: R is the half state and W the start state, whose own
// row each target reads before overwriting it (no other lane reads W).
// Inlet particles move with their prescribed velocity, outlet particles along
// x with their composed velocity, walls are fixed; in the full update the
// boundary values of the half state become those of the step.
template <int DIM, typename T, int G, int PF>
__global__ void __launch_bounds__(kBlock) k_force(Dev k, DevState m, Fields R, Fields W,
                                                  DevNlist nl, DevDerived o, const float *off,
                                                  const uint32_t *cpos, int mode, int want_drag,
                                                  double *dragpart, const double *xbin,
                                                  int32_t *rebin, uint32_t *err)
{
    constexpr int PB = kBlock / G;
    constexpr bool kBatchTail = DIM == 3 || sizeof(T) == 4;
    __shared__ double red_lds[3][PB];
    const int lane = threadIdx.x & (G - 1);
    const int64_t n = *m.n;
    const int64_t lb = xcd_block((n + PB - 1) / PB);
    const int64_t i = lb * PB + threadIdx.x / G;
    const int64_t C = k.cap;
    double fb[3] = {0, 0, 0};
    if (lb >= 0 && i < n) {
        const int t = m.type[i];
        if (t == SPH_FLUID || t == SPH_BODY) {
            const int cnt = nl.count[i];
            Sep<DIM, T> sep;
            sep.load_i(k, R, off, cpos, i);
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
            // one sweep over the neighbours gives every sum (pair_acc): the
            // lane's first PF neighbours are fetched at once, all indices
            // first (read whatever the count, within the row's maxnb entries;
            // entries past the count are not used), then all rows
            const int32_t *row = nl.nbr + i * nl.maxnb;
            int32_t jp[PF];
            bool okp[PF];
#pragma unroll
            for (int f = 0; f < PF; ++f) jp[f] = lane + f * G < nl.maxnb ? row[lane + f * G] : -1;
            bool badp = false;
#pragma unroll
            for (int f = 0; f < PF; ++f) {
                const bool have = lane + f * G < cnt;
                okp[f] = have && !bad_index(jp[f], n);
                badp = badp || (have && !okp[f]);
            }
            if (badp) raise_error(err, SPH_ERR_CELL_RANGE);
            // rows fetched without a branch (row i itself stands in for an
            // absent slot, whose data is never used) and all before the first
            // is used, so that the gathers of all PF slots go out together
            NbrRaw<DIM, T> raw[PF];
#pragma unroll
            for (int f = 0; f < PF; ++f)
                fetch_nbr<DIM, T>(k, m, R, o, okp[f] ? jp[f] : int32_t(i), raw[f]);
            // psum: the pressures of eq:pavg (every neighbour, self included)
            Acc<T> acc[3], gacc[3], pdot, psum;
#pragma unroll
            for (int f = 0; f < PF; ++f) {
                if (!okp[f]) continue;
                Nbr<DIM, T> nb;
                finish_nbr<DIM, T>(k, sep, raw[f], nb);
                psum.add(nb.p);
                if (jp[f] != i && !(t == SPH_BODY && nb.tj != SPH_FLUID))
                    pair_acc<DIM, T>(k, t, ui, wi, pi, rhoi, vi2, nb, acc, gacc, pdot);
            }
            // the rest: in batches of PF slots (indices, then every row, then
            // the arithmetic in slot order) where the tail is long (3D) or the
            // rows are records (FP32); in 2D FP64 the batch's registers cost
            // more than it saves (1.2M particles: 4 -> 3 waves per SIMD)
            if constexpr (!kBatchTail)
                for (int q = lane + PF * G; q < cnt; q += G) {
                    const int32_t j = row[q];
                    if (bad_index(j, n)) {
                        raise_error(err, SPH_ERR_CELL_RANGE);
                        continue;
                    }
                    Nbr<DIM, T> nb;
                    load_nbr<DIM, T>(k, m, R, o, sep, j, nb);
                    psum.add(nb.p);
                    if (j == i || (t == SPH_BODY && nb.tj != SPH_FLUID)) continue;
                    pair_acc<DIM, T>(k, t, ui, wi, pi, rhoi, vi2, nb, acc, gacc, pdot);
                }
            else
            for (int q0 = lane + PF * G; q0 < cnt; q0 += PF * G) {
                int32_t jb[PF];
                bool okb[PF];
                bool bad = false;
#pragma unroll
                for (int f = 0; f < PF; ++f) jb[f] = q0 + f * G < cnt ? row[q0 + f * G] : -1;
#pragma unroll
                for (int f = 0; f < PF; ++f) {
                    const bool have = q0 + f * G < cnt;
                    okb[f] = have && !bad_index(jb[f], n);
                    bad = bad || (have && !okb[f]);
                }
                if (bad) raise_error(err, SPH_ERR_CELL_RANGE);
                NbrRaw<DIM, T> rb[PF];
#pragma unroll
                for (int f = 0; f < PF; ++f)
                    fetch_nbr<DIM, T>(k, m, R, o, okb[f] ? jb[f] : int32_t(i), rb[f]);
#pragma unroll
                for (int f = 0; f < PF; ++f) {
                    if (!okb[f]) continue;
                    Nbr<DIM, T> nb;
                    finish_nbr<DIM, T>(k, sep, rb[f], nb);
                    psum.add(nb.p);
                    if (jb[f] == i || (t == SPH_BODY && nb.tj != SPH_FLUID)) continue;
                    pair_acc<DIM, T>(k, t, ui, wi, pi, rhoi, vi2, nb, acc, gacc, pdot);
                }
            }
            // the neighbour average of eq:pavg enters the fluid's momentum;
            // the body force takes p~ about zero (the average of a surface
            // particle's neighbours would cancel the pressure on the body)
            double pbar = 0.0;
            const double ps = gsum<G>(psum.s);
            if (t == SPH_FLUID && !(k.flags & SPH_FLAG_NO_PAVG)) pbar = ps / double(cnt);
            const T pavg = T(pbar);
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
                        stage_fluid<DIM, T>(k, R, W, i, mode, ui, pi, a, b, pd, xbin, rebin, err);
                    st<T>(o.pavg, i, pavg);  // kept for a reverse pass
                }
            }
        }
        // every non-fluid row (walls, bodies, inlet, outlet) takes its stage
        // position and, in the full update, its half-state boundary values
        if (mode != 0 && t != SPH_FLUID && lane == 0)
            stage_boundary<DIM, T>(k, m, R, W, i, t, mode, o.jcur, xbin, rebin, err);
    }
    if (!want_drag) return;
    // deterministic per-block partial of the body force (fixed order)
    const int gid = threadIdx.x / G;
    if (lane == 0)
#pragma unroll
        for (int d = 0; d < 3; ++d) red_lds[d][gid] = fb[d];
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

__global__ void __launch_bounds__(kBlock) k_drag_final(int nb, const double *dragpart,
                                                       double *drag, double *hist)
{
    __shared__ double lds[3][kBlock];
    double acc[3] = {0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += kBlock)
#pragma unroll
        for (int d = 0; d < 3; ++d) acc[d] += dragpart[d * nb + b];
#pragma unroll
    for (int d = 0; d < 3; ++d) lds[d][threadIdx.x] = acc[d];
    __syncthreads();
    for (int offs = kBlock / 2; offs > 0; offs >>= 1) {
        if (int(threadIdx.x) < offs)
#pragma unroll
            for (int d = 0; d < 3; ++d) lds[d][threadIdx.x] += lds[d][threadIdx.x + offs];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (drag) drag[d] = lds[d][0];
            if (hist) hist[d] = lds[d][0];
        }
    }
}

// ------------------------------------------------------------------ launchers
static int grid_for(const Dev &k, int G) { return xcd_grid((k.cap + (kBlock / G) - 1) / (kBlock / G)); }

// Lanes per target from the capacity (measured on MI355X): a few lanes per
// target keep gathers in flight without idling many lanes; below ~300k
// particles a few more lanes help fill the chip. Powers of two only.
static int pick(int override, int64_t cap, int small, int large)
{
    if (override == 1 || override == 2 || override == 4 || override == 8 || override == 16 ||
        override == 32)
        return override;
    return cap < 300000 ? small : large;
}

int force_group(const Dev &k) { return pick(k.g_force, k.cap, k.dim == 2 ? 4 : 8, 4); }
int nbr_group(const Dev &k) { return pick(k.g_nbr, k.cap, 8, k.lists ? 8 : (k.dim == 2 ? 2 : 4)); }
int force_grid(const Dev &k) { return k.tiles ? tile_grid(k) : grid_for(k, force_group(k)); }
// the most blocks any variant launches (fewest targets per block): sizes the
// per-block drag partials
int force_grid_max(const Dev &k)
{
    const int g = grid_for(k, 32);
    return k.tiles && tile_grid(k) > g ? tile_grid(k) : g;
}

// Lanes per boundary row and grid cap of the boundary pass (grid-stride over
// the device-side count of boundary rows; blocks past the count exit at
// once). Measured (us, FP64/FP32): 4.6M-particle duct, 8 lanes 174/191 with
// 16384 blocks, 204/224 with 1024; 16 lanes 200/234; 32 lanes 280/336 (the
// group reductions dominate). Small systems, latency-bound, keep 16 lanes
// (one round over a 2D row's neighbours).
constexpr int64_t kBndBlocks = 16384;
static int bnd_group(const Dev &k) { return k.cap < 300000 ? 16 : 8; }
static int bnd_grid(const Dev &k)
{
    const int64_t per = kBlock / bnd_group(k);
    const int64_t want = (k.cap + per - 1) / per;
    return int(want < kBndBlocks ? want : kBndBlocks);
}

template <int G, bool MIR>
static void boundary_g(const Dev &k, const DevState &m, const Fields &R, const DevNlist &nl,
                       const DevDerived &o, const int32_t *blist, const int32_t *bcount,
                       const uint32_t *spread, const int32_t *cell_start, uint32_t *err,
                       hipStream_t s)
{
    const dim3 g(bnd_grid(k)), b(kBlock);
    if (k.dim == 2 && k.prec == SPH_FP64)
        hipLaunchKernelGGL((k_boundary<2, double, G, MIR>), g, b, 0, s, k, m, R, nl, o, blist,
                           bcount, spread, cell_start, err);
    else if (k.dim == 3 && k.prec == SPH_FP64)
        hipLaunchKernelGGL((k_boundary<3, double, G, MIR>), g, b, 0, s, k, m, R, nl, o, blist,
                           bcount, spread, cell_start, err);
    else if (k.dim == 2)
        hipLaunchKernelGGL((k_boundary<2, float, G, MIR>), g, b, 0, s, k, m, R, nl, o, blist,
                           bcount, spread, cell_start, err);
    else
        hipLaunchKernelGGL((k_boundary<3, float, G, MIR>), g, b, 0, s, k, m, R, nl, o, blist,
                           bcount, spread, cell_start, err);
}

#define SPH_PREC_DIM(KERNEL, GRID, ...)                                                       \
    do {                                                                                      \
        if (k.dim == 2 && k.prec == SPH_FP64)                                                 \
            hipLaunchKernelGGL((KERNEL<2, double>), dim3(GRID), dim3(kBlock), 0, s,           \
                               __VA_ARGS__);                                                  \
        else if (k.dim == 3 && k.prec == SPH_FP64)                                            \
            hipLaunchKernelGGL((KERNEL<3, double>), dim3(GRID), dim3(kBlock), 0, s,           \
                               __VA_ARGS__);                                                  \
        else if (k.dim == 2)                                                                  \
            hipLaunchKernelGGL((KERNEL<2, float>), dim3(GRID), dim3(kBlock), 0, s,            \
                               __VA_ARGS__);                                                  \
        else                                                                                  \
            hipLaunchKernelGGL((KERNEL<3, float>), dim3(GRID), dim3(kBlock), 0, s,            \
                               __VA_ARGS__);                                                  \
    } while (0)

template <int DIM, typename T, int G>
static void nbrdens_g(const Dev &k, const DevState &m, const Fields &R, const DevNlist &nl,
                      const DevDerived &o, int dens, const uint32_t *spread,
                      const int32_t *cell_start, const uint32_t *cpos, float *off,
                      int32_t *rebin_clear, const VList &v, int vmode, uint32_t *err,
                      hipStream_t s)
{
    hipLaunchKernelGGL((k_nbrdens<DIM, T, G>), dim3(grid_for(k, G)), dim3(kBlock), 0, s, k, m, R,
                       nl, o, dens, spread, cell_start, cpos, off, rebin_clear, v, vmode, err);
}

template <int DIM, typename T>
static void nbrdens_dt(const Dev &k, const DevState &m, const Fields &R, const DevNlist &nl,
                       const DevDerived &o, int dens, const uint32_t *spread,
                       const int32_t *cell_start, const uint32_t *cpos, float *off,
                       int32_t *rebin_clear, const VList &v, int vmode, uint32_t *err,
                       hipStream_t s)
{
#define SPH_NBR_G(G)                                                                         \
    nbrdens_g<DIM, T, G>(k, m, R, nl, o, dens, spread, cell_start, cpos, off, rebin_clear, v, \
                         vmode, err, s)
    switch (nbr_group(k)) {
    case 1: SPH_NBR_G(1); break;
    case 2: SPH_NBR_G(2); break;
    case 4: SPH_NBR_G(4); break;
    case 8: SPH_NBR_G(8); break;
    case 16: SPH_NBR_G(16); break;
    default: SPH_NBR_G(32); break;
    }
#undef SPH_NBR_G
}

void launch_nbrdens(const Dev &k, const DevState &m, const Fields &R, const DevNlist &nl,
                    const DevDerived &o, int dens, const uint32_t *spread,
                    const int32_t *cell_start, const uint32_t *cpos, float *off,
                    uint16_t *lslot, const int32_t *ttab, int32_t *rebin_clear, const VList &v,
                    int vmode, uint32_t *err, hipStream_t s)
{
    if (k.tiles) {
        launch_tsearch(k, m, R, nl, o, dens, ttab, cpos, off, lslot, rebin_clear, v, vmode, err,
                       s);
        return;
    }
    if (k.dim == 2 && k.prec == SPH_FP64)
        nbrdens_dt<2, double>(k, m, R, nl, o, dens, spread, cell_start, cpos, off, rebin_clear, v,
                              vmode, err, s);
    else if (k.dim == 3 && k.prec == SPH_FP64)
        nbrdens_dt<3, double>(k, m, R, nl, o, dens, spread, cell_start, cpos, off, rebin_clear, v,
                              vmode, err, s);
    else if (k.dim == 2)
        nbrdens_dt<2, float>(k, m, R, nl, o, dens, spread, cell_start, cpos, off, rebin_clear, v,
                             vmode, err, s);
    else
        nbrdens_dt<3, float>(k, m, R, nl, o, dens, spread, cell_start, cpos, off, rebin_clear, v,
                             vmode, err, s);
}

void launch_density(const Dev &k, const DevState &m, const Fields &R, const DevNlist &nl,
                    const DevDerived &o, const uint32_t *cpos, uint32_t *err, hipStream_t s)
{
    SPH_PREC_DIM(k_density, (k.dim == 2 ? grid_for(k, Grp<2>::G) : grid_for(k, Grp<3>::G)), k, m,
                 R, nl, o, cpos, err);
}

void launch_pack_rec(const Dev &k, const DevState &m, const Fields &R, const DevDerived &o,
                     const uint32_t *cpos, hipStream_t s)
{
    // 3D only: 2D FP64 gathers the fields (Rec::USE), 2D FP32 records are
    // written by the density pass (a dispatch of their own cost the small 2D
    // systems more than it saved)
    if (k.dim != 3 || !o.rec || !o.shep) return;
    if (k.prec == SPH_FP64)
        hipLaunchKernelGGL(k_pack_rec<double>, dim3(nblocks(k.cap)), dim3(kBlock), 0, s, k, m, R,
                           o, cpos);
    else
        hipLaunchKernelGGL(k_pack_rec<float>, dim3(nblocks(k.cap)), dim3(kBlock), 0, s, k, m, R,
                           o, cpos);
}

void launch_boundary(const Dev &k, const DevState &m, const Fields &R, const DevNlist &nl,
                     const DevDerived &o, const int32_t *blist, const int32_t *bcount,
                     const uint32_t *spread, const int32_t *cell_start, uint32_t *err,
                     hipStream_t s)
{
    const bool mir = k.outlet == SPH_OUTLET_MIRROR || (k.flags & SPH_FLAG_MIRROR_INLET);
    if (bnd_group(k) == 16) {
        if (mir) boundary_g<16, true>(k, m, R, nl, o, blist, bcount, spread, cell_start, err, s);
        else boundary_g<16, false>(k, m, R, nl, o, blist, bcount, spread, cell_start, err, s);
    } else {
        if (mir) boundary_g<8, true>(k, m, R, nl, o, blist, bcount, spread, cell_start, err, s);
        else boundary_g<8, false>(k, m, R, nl, o, blist, bcount, spread, cell_start, err, s);
    }
}

template <int DIM, typename T, int G, int PF>
static void force_g(const Dev &k, const DevState &m, const Fields &R, const Fields &W,
                    const DevNlist &nl, const DevDerived &o, const float *off,
                    const uint32_t *cpos, int mode, int want_drag, double *dragpart,
                    const double *xbin, int32_t *rebin, uint32_t *err, hipStream_t s)
{
    hipLaunchKernelGGL((k_force<DIM, T, G, PF>), dim3(grid_for(k, G)), dim3(kBlock), 0, s, k, m,
                       R, W, nl, o, off, cpos, mode, want_drag, dragpart, xbin, rebin, err);
}

// Two neighbours prefetched per lane (one from 16 lanes up; three for small
// 2D systems at 4 lanes, which covers a typical 2D neighbour count at 150
// registers: 0.5 % off the 41k-particle channel's step). Measured: four per
// lane slows that channel's force pass from 14.4 to 16.9 us, as 173
// registers allow two waves per SIMD and the grid then needs a second round.
template <int DIM, typename T>
static void force_dt(const Dev &k, const DevState &m, const Fields &R, const Fields &W,
                     const DevNlist &nl, const DevDerived &o, const float *off,
                     const uint32_t *cpos, int mode, int want_drag, double *dragpart,
                     const double *xbin, int32_t *rebin, uint32_t *err, hipStream_t s)
{
#define SPH_FORCE_G(G, PF)                                                                   \
    force_g<DIM, T, G, PF>(k, m, R, W, nl, o, off, cpos, mode, want_drag, dragpart, xbin, rebin, \
                           err, s)
    switch (force_group(k)) {
    case 1: SPH_FORCE_G(1, 2); break;
    case 2: SPH_FORCE_G(2, 2); break;
    case 4:
        if (DIM == 2 && k.cap < 300000) SPH_FORCE_G(4, 3); else SPH_FORCE_G(4, 2);
        break;
    case 8: SPH_FORCE_G(8, 2); break;
    case 16: SPH_FORCE_G(16, 1); break;
    default: SPH_FORCE_G(32, 1); break;
    }
#undef SPH_FORCE_G
}

void launch_force(const Dev &k, const DevState &m, const Fields &R, const Fields &W,
                  const DevNlist &nl, const DevDerived &o, const float *off,
                  const uint32_t *cpos, const int32_t *ttab, const uint16_t *lslot, int mode,
                  int want_drag, double *dragpart, const double *xbin, int32_t *rebin,
                  uint32_t *err, hipStream_t s)
{
    if (k.tiles) {
        launch_tforce(k, m, R, W, nl, o, off, cpos, ttab, lslot, mode, want_drag, dragpart, xbin,
                      rebin, err, s);
        return;
    }
    if (k.dim == 2 && k.prec == SPH_FP64)
        force_dt<2, double>(k, m, R, W, nl, o, off, cpos, mode, want_drag, dragpart, xbin, rebin,
                            err, s);
    else if (k.dim == 3 && k.prec == SPH_FP64)
        force_dt<3, double>(k, m, R, W, nl, o, off, cpos, mode, want_drag, dragpart, xbin, rebin,
                            err, s);
    else if (k.dim == 2)
        force_dt<2, float>(k, m, R, W, nl, o, off, cpos, mode, want_drag, dragpart, xbin, rebin,
                           err, s);
    else
        force_dt<3, float>(k, m, R, W, nl, o, off, cpos, mode, want_drag, dragpart, xbin, rebin,
                           err, s);
}

void launch_drag_final(const Dev &k, const double *dragpart, double *drag, double *hist,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_drag_final, dim3(1), dim3(kBlock), 0, s, force_grid(k), dragpart, drag,
                       hist);
}

}  // namespace sph
