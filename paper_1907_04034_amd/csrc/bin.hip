// bin.hip -- cell binning of libsph: Morton keys, integer histogram, exclusive
// scan, scatter, per-cell ordering by particle id, and the gather that moves
// every per-particle array into sorted order.
//
// The sort is deterministic and stable without a radix sort: the histogram
// and the scan are integer (exact), the scatter writes each cell's members in
// arbitrary order, and one thread per cell then orders its few members by
// their unique id. The result depends only on (cell, id), never on the order
// in which atomics land.
#include "sph_launch.h"

namespace sph {

// spread[a * kSpreadStride + c]: coordinate c of axis a with its bits moved to
// the positions that axis occupies in the interleaved key. Bit b of every axis
// is placed before bit b + 1 of any axis; axes with fewer bits drop out once
// exhausted, so the key space is exactly the product of the padded extents.
__global__ void k_spread(Dev k, uint32_t *spread)
{
    int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
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

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

template <int DIM>
__global__ void k_keys(Dev k, DevState s, const uint32_t *spread, uint32_t *keys,
                       uint32_t *cpos, int32_t *counts, uint32_t *err)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t n = *s.n;
    if (i >= n) return;
    uint32_t key = k.nkeys;
    if (s.type[i] != SPH_DEAD) {
        int c[3] = {0, 0, 0};
        bool escaped = false;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            double f = floor((s.x[d * k.cap + i] - k.lo[d]) * k.inv_cs[d]);
            int v;  // NaN and out-of-box values are clamped and flagged below
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

// ------------------------------------------------------------------- scan
// Exclusive scan of int32 in place, three launches: per-tile sums, a scan of
// the tile sums in one block, then per-tile scans with the tile offset.
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

int64_t scan_blocksum_len(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

__device__ inline int32_t block_exclusive_scan(int32_t v, int32_t *lds, int32_t *total)
{
    int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        int32_t add = t >= off ? lds[t - off] : 0;
        __syncthreads();
        lds[t] += add;
        __syncthreads();
    }
    int32_t incl = lds[t];
    *total = lds[kBlock - 1];
    __syncthreads();
    return incl - v;
}

__global__ void __launch_bounds__(kBlock) k_scan_reduce(const int32_t *data, int64_t n,
                                                        int32_t *blocksum)
{
    __shared__ int32_t lds[kBlock];
    int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
    int32_t s = 0;
    for (int q = 0; q < kScanItems; ++q)
        if (base + q < n) s += data[base + q];
    int32_t total;
    block_exclusive_scan(s, lds, &total);
    if (threadIdx.x == 0) blocksum[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kBlock) k_scan_blocks(int32_t *blocksum, int64_t nb)
{
    __shared__ int32_t lds[kBlock];
    int32_t carry = 0;
    for (int64_t base = 0; base < nb; base += kBlock) {
        int64_t i = base + threadIdx.x;
        int32_t v = i < nb ? blocksum[i] : 0;
        int32_t total;
        int32_t ex = block_exclusive_scan(v, lds, &total);
        if (i < nb) blocksum[i] = ex + carry;
        carry += total;
    }
}

__global__ void __launch_bounds__(kBlock) k_scan_apply(int32_t *data, int64_t n,
                                                       const int32_t *blocksum)
{
    __shared__ int32_t lds[kBlock];
    int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
    int32_t v[kScanItems];
    int32_t s = 0;
    for (int q = 0; q < kScanItems; ++q) {
        v[q] = base + q < n ? data[base + q] : 0;
        s += v[q];
    }
    int32_t total;
    int32_t run = block_exclusive_scan(s, lds, &total) + blocksum[blockIdx.x];
    for (int q = 0; q < kScanItems; ++q) {
        if (base + q < n) data[base + q] = run;
        run += v[q];
    }
}

// ------------------------------------------------------------ scatter, sort
__global__ void k_scatter(Dev k, DevState s, const uint32_t *keys, const int32_t *cell_start,
                          int32_t *cursor, int32_t *tmp)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t n = *s.n;
    if (i >= n) return;
    uint32_t key = keys[i];
    int32_t slot = cell_start[key] + atomicAdd(&cursor[key], 1);
    tmp[slot] = int32_t(i);
}

// One thread per cell: insertion sort of the members by id (ids are unique).
__global__ void k_cellsort(Dev k, DevState s, const int32_t *cell_start, int32_t *tmp)
{
    int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= int64_t(k.nkeys)) return;
    int32_t b = cell_start[c], e = cell_start[c + 1];
    for (int32_t q = b + 1; q < e; ++q) {
        int32_t v = tmp[q];
        int64_t key = s.id[v];
        int32_t r = q - 1;
        while (r >= b && s.id[tmp[r]] > key) {
            tmp[r + 1] = tmp[r];
            --r;
        }
        tmp[r + 1] = v;
    }
}

// Row k of the sorted state is row tmp[k] of the old one. Also records the
// start-of-step copies of x, u, p used by the two-stage update.
template <int DIM, typename T>
__global__ void k_gather(Dev k, DevState a, DevState b, const int32_t *tmp,
                         const int32_t *cell_start, const uint32_t *cpos_in,
                         uint32_t *cpos_out, double *x0, T *u0, T *p0)
{
    int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t n = cell_start[k.nkeys];
    if (r >= n) return;
    int64_t i = tmp[r];
    const int64_t C = k.cap;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        double xv = a.x[d * C + i];
        T uv = ld<T>(a.u, d * C + i);
        b.x[d * C + r] = xv;
        x0[d * C + r] = xv;
        st<T>(b.u, d * C + r, uv);
        u0[d * C + r] = uv;
        st<T>(b.ut, d * C + r, ld<T>(a.ut, d * C + i));
        b.uin[d * C + r] = a.uin[d * C + i];
    }
    T pv = ld<T>(a.p, i);
    st<T>(b.p, r, pv);
    p0[r] = pv;
#pragma unroll
    for (int q = 0; q < kNavg * (DIM + 1); ++q) b.ring[q * C + r] = a.ring[q * C + i];
#pragma unroll
    for (int q = 0; q < DIM + 1; ++q) b.avg[q * C + r] = a.avg[q * C + i];
#pragma unroll
    for (int q = 0; q < 3; ++q) b.jprev[q * C + r] = a.jprev[q * C + i];
    b.head[r] = a.head[i];
    b.red_prev[r] = a.red_prev[i];
    b.type[r] = a.type[i];
    b.id[r] = a.id[i];
    cpos_out[r] = cpos_in[i];
}

__global__ void k_set_count(Dev k, DevState s, const int32_t *cell_start)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *s.n = cell_start[k.nkeys];
}

// ------------------------------------------------------------------ launchers
void launch_spread(const Dev &k, uint32_t *spread, hipStream_t s)
{
    hipLaunchKernelGGL(k_spread, dim3(nblocks(3 * int64_t(kSpreadStride))), dim3(kBlock), 0, s,
                       k, spread);
}

void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(n)), dim3(kBlock), 0, s, p, n, v);
}

void launch_keys(const Dev &k, const DevState &st, const uint32_t *spread, uint32_t *keys,
                 uint32_t *cpos, int32_t *counts, uint32_t *err, hipStream_t s)
{
    if (k.dim == 2)
        hipLaunchKernelGGL(k_keys<2>, dim3(nblocks(k.cap)), dim3(kBlock), 0, s, k, st, spread,
                           keys, cpos, counts, err);
    else
        hipLaunchKernelGGL(k_keys<3>, dim3(nblocks(k.cap)), dim3(kBlock), 0, s, k, st, spread,
                           keys, cpos, counts, err);
}

void launch_scan(int32_t *data, int64_t n, int32_t *blocksum, hipStream_t s)
{
    int64_t nb = scan_blocksum_len(n);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlock), 0, s, data, n, blocksum);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kBlock), 0, s, blocksum, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kBlock), 0, s, data, n, blocksum);
}

void launch_scatter(const Dev &k, const DevState &st, const uint32_t *keys,
                    const int32_t *cell_start, int32_t *cursor, int32_t *tmp, hipStream_t s)
{
    hipLaunchKernelGGL(k_scatter, dim3(nblocks(k.cap)), dim3(kBlock), 0, s, k, st, keys,
                       cell_start, cursor, tmp);
}

void launch_cellsort(const Dev &k, const DevState &st, const int32_t *cell_start, int32_t *tmp,
                     hipStream_t s)
{
    hipLaunchKernelGGL(k_cellsort, dim3(nblocks(k.nkeys)), dim3(kBlock), 0, s, k, st,
                       cell_start, tmp);
}

void launch_gather(const Dev &k, const DevState &src, const DevState &dst, const int32_t *tmp,
                   const int32_t *cell_start, const uint32_t *cpos_in, uint32_t *cpos_out,
                   double *x0, void *u0, void *p0, hipStream_t s)
{
    dim3 g(nblocks(k.cap)), b(kBlock);
    if (k.dim == 2 && k.prec == SPH_FP64)
        hipLaunchKernelGGL((k_gather<2, double>), g, b, 0, s, k, src, dst, tmp, cell_start,
                           cpos_in, cpos_out, x0, (double *)u0, (double *)p0);
    else if (k.dim == 3 && k.prec == SPH_FP64)
        hipLaunchKernelGGL((k_gather<3, double>), g, b, 0, s, k, src, dst, tmp, cell_start,
                           cpos_in, cpos_out, x0, (double *)u0, (double *)p0);
    else if (k.dim == 2)
        hipLaunchKernelGGL((k_gather<2, float>), g, b, 0, s, k, src, dst, tmp, cell_start,
                           cpos_in, cpos_out, x0, (float *)u0, (float *)p0);
    else
        hipLaunchKernelGGL((k_gather<3, float>), g, b, 0, s, k, src, dst, tmp, cell_start,
                           cpos_in, cpos_out, x0, (float *)u0, (float *)p0);
}

void launch_set_count(const Dev &k, const DevState &st, const int32_t *cell_start,
                      hipStream_t s)
{
    hipLaunchKernelGGL(k_set_count, dim3(1), dim3(64), 0, s, k, st, cell_start);
}

}  // namespace sph
