// Compressed-row form of the neighbour relation (the API's sph_neighbors):
// j is a neighbour of i iff |r_i - r_j|^2 < (2h)^2 (3h with the quintic
// spline, Sec. 2 eq:quintic-spline), computed in FP64 without fused
// multiply-add, minimum image on periodic axes, i itself included.
//
// Three passes over the cells of the last bin: a count pass, an exclusive
// scan of the counts into 64-bit row offsets, and a fill pass that walks the
// same stencil again. Both walks visit the 3^d stencil cells in the same
// order as the gather search (x fastest, then y, z) and each cell's rows in
// their sorted order, with hits compacted by ballot, so row i of the CSR is
// row i of the padded table in the same order. The number of entries is
// known only after the scan: when it exceeds the caller's capacity the fill
// pass writes nothing and the error word gets SPH_ERR_NNZ_CAPACITY; the row
// offsets and the total are written either way.
#include "sph_launch.h"

namespace sph {
namespace {

constexpr int kCsrG = 16;     // lanes per row
constexpr int kScanItems = 8; // consecutive rows per thread in the scan
constexpr int kScanSpan = kBlock * kScanItems;

template <int DIM, bool FILL>
__global__ void __launch_bounds__(kBlock) k_csr_walk(Dev k, DevState m,
                                                     const uint32_t *spread,
                                                     const int32_t *cell_start,
                                                     const uint32_t *cpos, int64_t *row_ptr,
                                                     int32_t *col, int64_t cap_nnz,
                                                     uint32_t *err)
{
    constexpr int G = kCsrG, PB = kBlock / G, NS = DIM == 2 ? 9 : 27;
    __shared__ int32_t s_beg[PB][NS], s_len[PB][NS];
    const int lane = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int64_t n = *m.n;
    // the fill pass runs only where every entry fits (uniform over the grid)
    if (FILL && row_ptr[n] > cap_nnz) return;
    const int64_t i = int64_t(blockIdx.x) * PB + grp;
    const bool active = i < n;  // uniform across the group
    const int64_t C = k.cap;
    double xi[3] = {0, 0, 0};
    int c[3] = {0, 0, 0};
    if (active) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) xi[d] = m.x[d * C + i];
        unpack_cell<DIM>(cpos[i], c);
        bool bad = false;
        for (int sc = lane; sc < NS; sc += G) {
            const int o[3] = {sc % 3 - 1, (sc / 3) % 3 - 1, DIM == 3 ? sc / 9 - 1 : 0};
            int cc[3] = {c[0] + o[0], c[1] + o[1], c[2] + o[2]};
            bool ok = true;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                if (cc[d] < 0 || cc[d] >= k.nc[d]) {
                    if (k.periodic[d]) cc[d] = cc[d] < 0 ? cc[d] + k.nc[d] : cc[d] - k.nc[d];
                    else ok = false;
                }
            }
            int32_t b = 0, e = 0;
            if (ok) {
                const uint32_t key = morton_key<DIM>(spread, cc);
                b = cell_start[key];
                e = cell_start[key + 1];
                if (b < 0 || e > n || b > e) {
                    bad = true;
                    b = e = 0;
                }
            }
            s_beg[grp][sc] = b;
            s_len[grp][sc] = e - b;
        }
        if (bad) raise_error(err, SPH_ERR_CELL_RANGE);
    }
    __syncthreads();
    if (!active) return;
    int total = 0;
#pragma unroll
    for (int sc = 0; sc < NS; ++sc) total += s_len[grp][sc];
    // this lane's candidate: offset mo in stencil cell sc
    int sc = 0, mo = lane;
    while (sc < NS && mo >= s_len[grp][sc]) mo -= s_len[grp][sc++];
    const int gshift = (threadIdx.x & 63) & ~(G - 1);
    const uint64_t below = (1ull << lane) - 1;
    int64_t base_out = 0, room = 0;
    if (FILL) {
        base_out = row_ptr[i];
        room = row_ptr[i + 1] - base_out;
    }
    int cnt = 0;
    for (int q0 = 0; q0 < total; q0 += G) {
        const bool has = sc < NS;
        const int32_t j = has ? s_beg[grp][sc] + mo : 0;
        bool hit = false;
        if (has) {
            double xj[3] = {0, 0, 0}, r[3];
#pragma unroll
            for (int d = 0; d < DIM; ++d) xj[d] = m.x[d * C + j];
            hit = dist2_exact<DIM>(k, xi, xj, r) < k.sup2;
        }
        const uint64_t bal = (uint64_t(__ballot(hit)) >> gshift) & ((1ull << G) - 1);
        if (FILL && hit) {
            const int pos = cnt + __popcll(bal & below);
            if (pos < room) col[base_out + pos] = j;
        }
        cnt += __popcll(bal);
        mo += G;
        while (sc < NS && mo >= s_len[grp][sc]) mo -= s_len[grp][sc++];
    }
    if (lane == 0) {
        if (!FILL) row_ptr[i] = cnt;
        else if (cnt != room) raise_error(err, SPH_ERR_CELL_RANGE);  // positions changed between passes
    }
}

// Block sum of one 64-bit value per thread: exclusive prefix in place of v,
// the total returned to every thread.
__device__ inline int64_t block_scan64(int64_t &v, int64_t *lds)
{
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {
        const int64_t add = t >= o ? lds[t - o] : 0;
        __syncthreads();
        lds[t] += add;
        __syncthreads();
    }
    const int64_t incl = lds[t], tot = lds[kBlock - 1];
    __syncthreads();
    v = incl - v;
    return tot;
}

// Pass 1 of the scan: the count total of each span of kScanSpan rows.
__global__ void __launch_bounds__(kBlock) k_csr_spans(const int64_t *nptr, const int64_t *row_ptr,
                                                      int64_t *span_sum)
{
    __shared__ int64_t lds[kBlock];
    const int64_t n = *nptr;
    const int64_t r0 = int64_t(blockIdx.x) * kScanSpan + int64_t(threadIdx.x) * kScanItems;
    int64_t v = 0;
    for (int u = 0; u < kScanItems; ++u)
        if (r0 + u < n) v += row_ptr[r0 + u];
    const int64_t tot = block_scan64(v, lds);
    if (threadIdx.x == 0) span_sum[blockIdx.x] = tot;
}

// Pass 2 (one block): exclusive scan of the span totals; the grand total at
// span_sum[nspan], in *nnz_out, and the capacity check.
__global__ void __launch_bounds__(kBlock) k_csr_span_scan(const int64_t *nptr, int64_t *span_sum,
                                                          int64_t *nnz_out, int64_t cap_nnz,
                                                          uint32_t *err)
{
    __shared__ int64_t lds[kBlock];
    const int64_t n = *nptr;
    const int64_t nspan = (n + kScanSpan - 1) / kScanSpan;
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nspan; b0 += kBlock) {
        const int64_t b = b0 + threadIdx.x;
        int64_t v = b < nspan ? span_sum[b] : 0;
        const int64_t tot = block_scan64(v, lds);
        if (b < nspan) span_sum[b] = carry + v;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        span_sum[nspan] = carry;
        *nnz_out = carry;
        if (carry > cap_nnz) raise_error(err, SPH_ERR_NNZ_CAPACITY);
    }
}

// Pass 3: counts -> exclusive row offsets in place; row_ptr[n] = total.
__global__ void __launch_bounds__(kBlock) k_csr_offsets(const int64_t *nptr, int64_t *row_ptr,
                                                        const int64_t *span_sum)
{
    __shared__ int64_t lds[kBlock];
    const int64_t n = *nptr;
    const int64_t r0 = int64_t(blockIdx.x) * kScanSpan + int64_t(threadIdx.x) * kScanItems;
    int64_t c[kScanItems];
    int64_t v = 0;
#pragma unroll
    for (int u = 0; u < kScanItems; ++u) {
        c[u] = r0 + u < n ? row_ptr[r0 + u] : 0;
        v += c[u];
    }
    block_scan64(v, lds);
    int64_t run = span_sum[blockIdx.x] + v;
#pragma unroll
    for (int u = 0; u < kScanItems; ++u) {
        if (r0 + u < n) row_ptr[r0 + u] = run;
        run += c[u];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int64_t nspan = (n + kScanSpan - 1) / kScanSpan;
        row_ptr[n] = span_sum[nspan];
    }
}

template <int DIM>
void csr_dim(const Dev &k, const DevState &m, const uint32_t *spread, const int32_t *cell_start,
             const uint32_t *cpos, int64_t *row_ptr, int32_t *col, int64_t cap_nnz,
             int64_t *nnz_out, int64_t *span_sum, uint32_t *err, hipStream_t s)
{
    const int rows_grid = nblocks(k.cap, kBlock / kCsrG);
    const int span_grid = csr_spans(k.cap);
    hipLaunchKernelGGL((k_csr_walk<DIM, false>), dim3(rows_grid), dim3(kBlock), 0, s, k, m,
                       spread, cell_start, cpos, row_ptr, col, cap_nnz, err);
    hipLaunchKernelGGL(k_csr_spans, dim3(span_grid), dim3(kBlock), 0, s, m.n, row_ptr, span_sum);
    hipLaunchKernelGGL(k_csr_span_scan, dim3(1), dim3(kBlock), 0, s, m.n, span_sum, nnz_out,
                       cap_nnz, err);
    hipLaunchKernelGGL(k_csr_offsets, dim3(span_grid), dim3(kBlock), 0, s, m.n, row_ptr,
                       span_sum);
    hipLaunchKernelGGL((k_csr_walk<DIM, true>), dim3(rows_grid), dim3(kBlock), 0, s, k, m,
                       spread, cell_start, cpos, row_ptr, col, cap_nnz, err);
}

}  // namespace

int csr_spans(int64_t cap) { return nblocks(cap, kScanSpan); }

void launch_csr(const Dev &k, const DevState &m, const uint32_t *spread,
                const int32_t *cell_start, const uint32_t *cpos, int64_t *row_ptr, int32_t *col,
                int64_t cap_nnz, int64_t *nnz_out, int64_t *span_sum, uint32_t *err,
                hipStream_t s)
{
    if (k.dim == 2)
        csr_dim<2>(k, m, spread, cell_start, cpos, row_ptr, col, cap_nnz, nnz_out, span_sum, err,
                   s);
    else
        csr_dim<3>(k, m, spread, cell_start, cpos, row_ptr, col, cap_nnz, nnz_out, span_sum, err,
                   s);
}

}  // namespace sph
