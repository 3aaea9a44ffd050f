// bin.hip -- cell binning of libsph: Morton keys with an integer histogram,
// one-launch exclusive scan, scatter, per-cell ordering by particle id, and
// the gather that moves every per-particle array into sorted order.
//
// The sort is deterministic and stable without a radix sort: histogram and
// scan are integer (exact), the scatter writes each cell's members in
// arbitrary order, and every member then takes its place in the cell by
// counting the members with a smaller id, so the result depends only on
// (cell, id), never on the order in which atomics land. No launch is spent on clearing: every counter
// is zeroed by the kernel that consumes it (the workspace starts zeroed).
#include "sph_launch.h"

namespace sph {

// spread[a * kSpreadStride + c]: coordinate c of axis a with its bits moved to
// the positions that axis occupies in the interleaved key. Bit b of every axis
// is placed before bit b + 1 of any axis; axes with fewer bits drop out once
// exhausted, so the key space is exactly the product of the padded extents.
__global__ void k_spread(Dev k, uint32_t *spread, int32_t *rebin)
{
    int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t == 0) *rebin = 1;
    if (t >= int64_t(3) * kSpreadStride) return;
    int axis = int(t / kSpreadStride);
    int c = int(t % kSpreadStride);
    uint32_t v = 0;
    if (axis < k.dim && c < k.nc[axis]) {
        int maxb = 0;
        for (int a = 0; a < k.dim; ++a) maxb = max(maxb, k.bits[a]);
        int pos = 0;
        for (int b = 0; b < maxb; ++b)
            for (int a = 0; a < k.dim; ++a)
                if (b < k.bits[a]) {
                    if (a == axis && ((c >> b) & 1)) v |= 1u << pos;
                    ++pos;
                }
    }
    spread[t] = v;
}

constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;
constexpr int kTileSlots = 8;  // sub-counters per tile total (spreads the atomics)

int64_t scan_tiles(int64_t n) { return (n + kScanTile - 1) / kScanTile; }
int64_t tilesum_len(int64_t n) { return scan_tiles(n) * kTileSlots; }

// With bin reuse, a bin that finds no request to sort keeps the current order
// (every kernel of the bin checks the same word, written before the bin).
__device__ inline bool bin_skips(const Dev &k, const int32_t *rebin)
{
    return k.reuse && *rebin == 0;
}

// live rows this bin sees: the last count plus rows re-spawned since
__device__ inline int64_t rows_to_bin(const Dev &k, const DevState &s, const int32_t *nspawn)
{
    int64_t n = *s.n + *nspawn;
    return n < k.cap ? n : k.cap;
}

template <int DIM>
__global__ void __launch_bounds__(kBlock) k_keys(Dev k, DevState s, const int32_t *nspawn,
                                                 const uint32_t *spread, uint32_t *keys,
                                                 uint32_t *cpos, int32_t *counts,
                                                 int32_t *tilesum, int32_t *bcount,
                                                 const int32_t *rebin, uint32_t *err)
{
    if (bin_skips(k, rebin)) return;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    if (i == 0) *bcount = 0;
    const int64_t n = rows_to_bin(k, s, nspawn);
    uint32_t key = k.nkeys;
    if (i < n) {
        if (s.type[i] != SPH_DEAD) {
            int c[3] = {0, 0, 0};
            bool escaped = false;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                const double f = floor((s.x[d * k.cap + i] - k.lo[d]) * k.inv_cs[d]);
                int v;  // NaN and out-of-box values are clamped and flagged
                if (!(f >= 0.0)) v = -1;
                else if (f >= double(k.nc[d])) v = k.nc[d];
                else v = int(f);
                if (v < 0 || v >= k.nc[d]) {
                    if (!k.periodic[d]) escaped = true;
                    v = v < 0 ? 0 : k.nc[d] - 1;
                }
                c[d] = v;
            }
            if (escaped) raise_error(err, SPH_ERR_ESCAPE);
            key = morton_key<DIM>(spread, c);
            cpos[i] = pack_cell<DIM>(c);
        }
        keys[i] = key;
        atomicAdd(&counts[key], 1);
    }
    // Tile totals for the scan. Rows arrive almost sorted, so lanes of a wave
    // mostly share a tile: only the first lane of each run of equal tiles
    // adds the run length (about one atomic per wave instead of per row).
    const uint32_t tile = i < n ? key / kScanTile : 0xFFFFFFFFu;
    const uint32_t prev = __shfl_up(tile, 1);
    const bool leader = i < n && (lane == 0 || prev != tile);
    const uint64_t lead = __ballot(leader);
    if (leader) {
        const uint64_t above = lane == 63 ? 0ull : (lead & ~((2ull << lane) - 1));
        const int64_t wave_end = (i - lane) + 64 < n ? 64 : n - (i - lane);
        const int next = above ? __ffsll((long long)above) - 1 : int(wave_end);
        atomicAdd(&tilesum[int64_t(tile) * kTileSlots + (blockIdx.x % kTileSlots)], next - lane);
    }
}

// cell_start = exclusive scan of counts (n entries); every tile adds the sum
// of the tile totals before it, so one launch suffices. Consumed counts are
// zeroed for the next bin.
__global__ void __launch_bounds__(kBlock) k_scan(Dev k, int32_t *counts, int32_t *cell_start,
                                                 int64_t n, const int32_t *tilesum,
                                                 const int32_t *rebin)
{
    if (bin_skips(k, rebin)) return;
    __shared__ int32_t lds[kBlock];
    int32_t pre = 0;
    for (int64_t t = threadIdx.x; t < int64_t(blockIdx.x) * kTileSlots; t += kBlock) pre += tilesum[t];
    int32_t total;
    block_exclusive_scan(pre, lds, &total);
    const int32_t tile_off = total;
    const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
    int32_t v[kScanItems];
    int32_t s = 0;
    for (int q = 0; q < kScanItems; ++q) {
        v[q] = base + q < n ? counts[base + q] : 0;
        s += v[q];
    }
    int32_t run = block_exclusive_scan(s, lds, &total) + tile_off;
    for (int q = 0; q < kScanItems; ++q) {
        if (base + q < n) {
            cell_start[base + q] = run;
            counts[base + q] = 0;
        }
        run += v[q];
    }
}

__global__ void k_scatter(Dev k, DevState s, const int32_t *nspawn, const uint32_t *keys,
                          const int32_t *cell_start, int32_t *cursor, int32_t *scat,
                          const int32_t *rebin)
{
    if (bin_skips(k, rebin)) return;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= rows_to_bin(k, s, nspawn)) return;
    const uint32_t key = keys[i];
    const int32_t slot = cell_start[key] + atomicAdd(&cursor[key], 1);
    scat[slot] = int32_t(i);
}

// One thread per slot of the scatter: its row goes to the cell's start plus
// the number of the cell's rows with a smaller id (ids are unique; equal ids,
// which valid input does not hold, are ranked by slot so the result is still
// a permutation). O(m) independent loads per row for a cell of m rows, so the
// quintic kernel's larger cells (about 22 rows in 2D, 60 in 3D) cost no more
// than a few extra loads. The same threads clear the scatter cursor and the
// scan's tile sums for the next bin.
__global__ void __launch_bounds__(kBlock) k_cellrank(Dev k, DevState s, const int32_t *nspawn,
                                                     const uint32_t *keys,
                                                     const int32_t *cell_start,
                                                     const int32_t *scat, int32_t *tmp,
                                                     int32_t *cursor, int32_t *tilesum,
                                                     int64_t ntiles, const int32_t *rebin)
{
    if (bin_skips(k, rebin)) return;
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < ntiles * kTileSlots) tilesum[t] = 0;
    if (t <= int64_t(k.nkeys)) cursor[t] = 0;
    if (t >= rows_to_bin(k, s, nspawn)) return;
    const int32_t v = scat[t];
    const uint32_t key = keys[v];
    if (key == k.nkeys) {  // dead rows need no order
        tmp[t] = v;
        return;
    }
    const int32_t b = cell_start[key], e = cell_start[key + 1];
    const int64_t mine = s.id[v];
    int32_t rank = 0;
#pragma unroll 4
    for (int32_t q = b; q < e; ++q) {
        const int64_t other = s.id[scat[q]];
        rank += (other < mine || (other == mine && q < t)) ? 1 : 0;
    }
    tmp[b + rank] = v;
}

// Slice `slice` (0: x, u, ut, u_in, p, head, red_prev, kind, id; 1 and 2:
// the two halves of the ring; 3: the averages and previous-step J) of row i
// of a, copied to row r of b. Every load of the slice is issued before its
// first store: as far as the compiler knows a and b may alias, and a load
// placed after a store waits for it, one round trip per field. Slice 0
// returns the row's position and kind through x_out and t_out.
template <int DIM, typename T>
__device__ inline void copy_slice(const Dev &k, const DevState &a, int64_t i, const DevState &b,
                                  int64_t r, int slice, double x_out[3], int &t_out)
{
    const int64_t C = k.cap;
    constexpr int NR = kNavg * (DIM + 1);  // ring words, an even count
    constexpr int H = NR / 2;
    if (slice == 0) {
        double x[DIM], uin[DIM];
        T u[DIM], ut[DIM];
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            x[d] = a.x[d * C + i];
            u[d] = ld<T>(a.u, d * C + i);
            ut[d] = ld<T>(a.ut, d * C + i);
            uin[d] = a.uin[d * C + i];
        }
        const T p = ld<T>(a.p, i);
        const uint8_t hd = a.head[i], rp = a.red_prev[i], t = a.type[i];
        const int64_t id = a.id[i];
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            b.x[d * C + r] = x[d];
            st<T>(b.u, d * C + r, u[d]);
            st<T>(b.ut, d * C + r, ut[d]);
            b.uin[d * C + r] = uin[d];
            x_out[d] = x[d];
        }
        st<T>(b.p, r, p);
        b.head[r] = hd;
        b.red_prev[r] = rp;
        b.type[r] = t;
        b.id[r] = id;
        t_out = t;
    } else if (slice <= 2) {
        const int q0 = slice == 1 ? 0 : H;
        double v[H];
#pragma unroll
        for (int q = 0; q < H; ++q) v[q] = a.ring[int64_t(q0 + q) * C + i];
#pragma unroll
        for (int q = 0; q < H; ++q) b.ring[int64_t(q0 + q) * C + r] = v[q];
    } else {
        double v[DIM + 1], j[3];
#pragma unroll
        for (int q = 0; q < DIM + 1; ++q) v[q] = a.avg[q * C + i];
#pragma unroll
        for (int q = 0; q < 3; ++q) j[q] = a.jprev[q * C + i];
#pragma unroll
        for (int q = 0; q < DIM + 1; ++q) b.avg[q * C + r] = v[q];
#pragma unroll
        for (int q = 0; q < 3; ++q) b.jprev[q * C + r] = j[q];
    }
}

// Row r of the sorted state is row tmp[r] of the old one. Non-fluid rows are
// listed for the boundary pass, the positions kept as the reference of the
// cell skin; the live count is published and the re-spawn counter cleared.
// A bin that keeps the order copies row for row.
template <int DIM, typename T>
__global__ void k_gather(Dev k, DevState a, DevState b, const int32_t *tmp,
                         const int32_t *cell_start, const uint32_t *cpos_in, uint32_t *cpos_out,
                         int32_t *blist, int32_t *bcount, int32_t *nspawn,
                         const int32_t *rebin, double *xbin, int32_t *vfresh)
{
    // a sort gathers a -> b; a kept order leaves the rows where they are
    const bool sorted = !bin_skips(k, rebin);
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n = sorted ? int64_t(cell_start[k.nkeys]) : *a.n;
    if (r == 0 && blockIdx.y == 0) {
        *a.n = n;
        *nspawn = 0;
        *vfresh = sorted ? 1 : 0;
    }
    // a kept order needs no copy: the state stays where it is
    if (!sorted || r >= n) return;
    const int64_t i = int64_t(tmp[r]);
    const uint32_t cp = blockIdx.y == 0 ? cpos_in[i] : 0u;
    double x[3];
    int t = SPH_DEAD;
    copy_slice<DIM, T>(k, a, i, b, r, int(blockIdx.y), x, t);
    if (blockIdx.y == 0) {
        const int64_t C = k.cap;
        cpos_out[r] = cp;
        if (t != SPH_FLUID) blist[atomicAdd(bcount, 1)] = int32_t(r);
#pragma unroll
        for (int d = 0; d < DIM; ++d) xbin[d * C + r] = x[d];
    }
}

// The cell structure for the API: cell_start copied, each live row's key from
// its packed cell.
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_cells_out(Dev k, const int64_t *nptr,
                                                      const uint32_t *spread,
                                                      const int32_t *cell_start,
                                                      const uint32_t *cpos, int32_t *cs_out,
                                                      uint32_t *key_out)
{
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (cs_out && t <= int64_t(k.nkeys)) cs_out[t] = cell_start[t];
    if (key_out && t < *nptr) {
        int c[3] = {0, 0, 0};
        unpack_cell<DIM>(cpos[t], c);
        key_out[t] = morton_key<DIM>(spread, c);
    }
}

void launch_cells_out(const Dev &k, const int64_t *n, const uint32_t *spread,
                      const int32_t *cell_start, const uint32_t *cpos, int32_t *cs_out,
                      uint32_t *key_out, hipStream_t s)
{
    const int64_t m = (int64_t(k.nkeys) + 1) > k.cap ? (int64_t(k.nkeys) + 1) : k.cap;
    if (k.dim == 2)
        hipLaunchKernelGGL(k_cells_out<2>, dim3(nblocks(m)), dim3(kBlock), 0, s, k, n, spread,
                           cell_start, cpos, cs_out, key_out);
    else
        hipLaunchKernelGGL(k_cells_out<3>, dim3(nblocks(m)), dim3(kBlock), 0, s, k, n, spread,
                           cell_start, cpos, cs_out, key_out);
}

// ------------------------------------------------------------------ launchers
void launch_spread(const Dev &k, uint32_t *spread, int32_t *rebin, hipStream_t s)
{
    hipLaunchKernelGGL(k_spread, dim3(nblocks(3 * int64_t(kSpreadStride))), dim3(kBlock), 0, s,
                       k, spread, rebin);
}

// The sorted rows back into the state they came from (a sort gathers into the
// second buffer set; this returns them, so the caller's state keeps its
// buffers). Nothing to do when the bin kept the order (*sorted == 0).
template <int DIM, typename T>
__global__ void k_copy_back(Dev k, DevState src, DevState dst, const int32_t *sorted)
{
    if (*sorted == 0) return;
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= *dst.n) return;
    double x[3];
    int t = 0;
    copy_slice<DIM, T>(k, src, r, dst, r, int(blockIdx.y), x, t);
}

void launch_copy_back(const Dev &k, const DevState &src, const DevState &dst,
                      const int32_t *sorted, hipStream_t s)
{
    const dim3 g(nblocks(k.cap), 4), blk(kBlock);
    if (k.dim == 2 && k.prec == SPH_FP64)
        hipLaunchKernelGGL((k_copy_back<2, double>), g, blk, 0, s, k, src, dst, sorted);
    else if (k.dim == 3 && k.prec == SPH_FP64)
        hipLaunchKernelGGL((k_copy_back<3, double>), g, blk, 0, s, k, src, dst, sorted);
    else if (k.dim == 2)
        hipLaunchKernelGGL((k_copy_back<2, float>), g, blk, 0, s, k, src, dst, sorted);
    else
        hipLaunchKernelGGL((k_copy_back<3, float>), g, blk, 0, s, k, src, dst, sorted);
}

// Row-for-row copy of the live rows of a into b (every state array and the
// live count), plus the sort permutation (the identity if the last bin kept
// the order: *sorted == 0) and the packed cells of those rows.
template <int DIM, typename T>
__global__ void k_copy_rows(Dev k, DevState a, DevState b, const int32_t *perm_in,
                            const int32_t *sorted, int32_t *perm_out, const uint32_t *cell_in,
                            uint32_t *cell_out)
{
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n = *a.n;
    const bool moved = *sorted != 0;
    if (r == 0 && blockIdx.y == 0) *b.n = n;
    if (r >= n) return;
    int32_t pr = int32_t(r);
    uint32_t cell = 0u;
    if (blockIdx.y == 0) {
        if (moved) pr = perm_in[r];
        cell = cell_in[r];
    }
    double x[3];
    int t = 0;
    copy_slice<DIM, T>(k, a, r, b, r, int(blockIdx.y), x, t);
    if (blockIdx.y == 0) {
        perm_out[r] = pr;
        cell_out[r] = cell;
    }
}

void launch_copy_rows(const Dev &k, const DevState &a, const DevState &b, const int32_t *perm_in,
                      const int32_t *sorted, int32_t *perm_out, const uint32_t *cell_in,
                      uint32_t *cell_out, hipStream_t s)
{
    const dim3 g(nblocks(k.cap), 4), blk(kBlock);
    if (k.dim == 2 && k.prec == SPH_FP64)
        hipLaunchKernelGGL((k_copy_rows<2, double>), g, blk, 0, s, k, a, b, perm_in, sorted,
                           perm_out, cell_in, cell_out);
    else if (k.dim == 3 && k.prec == SPH_FP64)
        hipLaunchKernelGGL((k_copy_rows<3, double>), g, blk, 0, s, k, a, b, perm_in, sorted,
                           perm_out, cell_in, cell_out);
    else if (k.dim == 2)
        hipLaunchKernelGGL((k_copy_rows<2, float>), g, blk, 0, s, k, a, b, perm_in, sorted,
                           perm_out, cell_in, cell_out);
    else
        hipLaunchKernelGGL((k_copy_rows<3, float>), g, blk, 0, s, k, a, b, perm_in, sorted,
                           perm_out, cell_in, cell_out);
}

void launch_bin(const Dev &k, const DevState &a, const DevState &b, const BinBufs &w,
                uint32_t *err, hipStream_t s)
{
    const dim3 g(nblocks(k.cap)), blk(kBlock);
    const int64_t nscan = int64_t(k.nkeys) + 2;
    const int64_t ntiles = scan_tiles(nscan);
    if (k.dim == 2)
        hipLaunchKernelGGL(k_keys<2>, g, blk, 0, s, k, a, w.nspawn, w.spread, w.keys, w.cpos,
                           w.counts, w.tilesum, w.bcount, w.rebin, err);
    else
        hipLaunchKernelGGL(k_keys<3>, g, blk, 0, s, k, a, w.nspawn, w.spread, w.keys, w.cpos,
                           w.counts, w.tilesum, w.bcount, w.rebin, err);
    hipLaunchKernelGGL(k_scan, dim3(ntiles), blk, 0, s, k, w.counts, w.cell_start, nscan,
                       w.tilesum, w.rebin);
    hipLaunchKernelGGL(k_scatter, g, blk, 0, s, k, a, w.nspawn, w.keys, w.cell_start, w.cursor,
                       w.scat, w.rebin);
    int64_t nrank = int64_t(k.nkeys) + 1;  // rows, cursor entries and tile sums
    if (nrank < ntiles * kTileSlots) nrank = ntiles * kTileSlots;
    if (nrank < k.cap) nrank = k.cap;
    hipLaunchKernelGGL(k_cellrank, dim3(nblocks(nrank)), blk, 0, s, k, a, w.nspawn, w.keys,
                       w.cell_start, w.scat, w.tmp, w.cursor, w.tilesum, ntiles, w.rebin);
    const dim3 gg(nblocks(k.cap), 4);
    if (k.dim == 2 && k.prec == SPH_FP64)
        hipLaunchKernelGGL((k_gather<2, double>), gg, blk, 0, s, k, a, b, w.tmp, w.cell_start,
                           w.cpos, w.cpos_s, w.blist, w.bcount, w.nspawn, w.rebin, w.xbin,
                           w.vfresh);
    else if (k.dim == 3 && k.prec == SPH_FP64)
        hipLaunchKernelGGL((k_gather<3, double>), gg, blk, 0, s, k, a, b, w.tmp, w.cell_start,
                           w.cpos, w.cpos_s, w.blist, w.bcount, w.nspawn, w.rebin, w.xbin,
                           w.vfresh);
    else if (k.dim == 2)
        hipLaunchKernelGGL((k_gather<2, float>), gg, blk, 0, s, k, a, b, w.tmp, w.cell_start,
                           w.cpos, w.cpos_s, w.blist, w.bcount, w.nspawn, w.rebin, w.xbin,
                           w.vfresh);
    else
        hipLaunchKernelGGL((k_gather<3, float>), gg, blk, 0, s, k, a, b, w.tmp, w.cell_start,
                           w.cpos, w.cpos_s, w.blist, w.bcount, w.nspawn, w.rebin, w.xbin,
                           w.vfresh);
    // tile records of the LDS-tiled pair passes (only when this bin sorted)
    if (k.tiles)
        launch_tile_table(k, a.n, w.cell_start, w.spread, w.cpos_s, w.vfresh, w.ttab, err, s);
}

}  // namespace sph
