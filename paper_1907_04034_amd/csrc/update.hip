// update.hip -- end-of-step bookkeeping of the hybrid outlet for gfx950:
// gated time averages, transfers, deletion and inlet re-spawn. (The RK2
// stage updates are fused into the force pass.)
#include "sph_launch.h"

namespace sph {

// SplitMix64 (Steele, Lea & Flood 2014) used as a counter-based generator:
// uniform k of particle `id` = mix(seed + (3 id + k + 1) * golden gamma).
__device__ inline double splitmix_uniform(uint64_t seed, int64_t id, int k)
{
    uint64_t z = seed + uint64_t(3 * id + k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return double(z >> 11) * (1.0 / 9007199254740992.0);
}

// End of step (Sec. 3.4): characteristic values become previous-step values;
// time averages of fluid and inlet particles take the new sample unless the
// acoustic intensity p^2/(2 rho c) exceeds (rho U^2/2)^2/(2 rho c)
// (eq:acouinten, i.e. |p| > rho0 U^2 / 2); particles are transferred across
// the inlet and outlet interfaces and deleted past the outlet end. Every
// inlet particle entering the fluid is flagged (sflag) and counted per block
// (stile); k_spawn then appends its new inlet particle. When `child` /
// `events` are given (recording a step for the reverse pass), every row
// records its events and (in k_spawn) the row of the particle it left behind.
template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_end_of_step(Dev k, DevState s, DevDerived o,
                                                        uint8_t *sflag, int32_t *stile,
                                                        int32_t *child, uint8_t *events,
                                                        int32_t *rebin)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n = *s.n;
    const int64_t C = k.cap;
    bool spawn = false;
    if (i < n) {
        // Every load before the first store: the stores below could alias
        // the arrays read, so loads placed after them would each wait for the
        // store before (one round trip per load instead of two in all).
        const int t = s.type[i];
        const double x = s.x[i];
        const double pv = double(ld<T>(s.p, i));
        const int h = s.head[i];
        double v[DIM + 1];
#pragma unroll
        for (int d = 0; d < DIM; ++d) v[d] = double(ld<T>(s.u, d * C + i));
        v[DIM] = pv;
        const bool io = t == SPH_OUTLET || t == SPH_INLET;
        const bool push = (t == SPH_FLUID || t == SPH_INLET) && !(fabs(pv) > k.pgate);
        double jc[3] = {0, 0, 0};
        uint8_t rd = 0;
        if (io) {
#pragma unroll
            for (int a = 0; a < 3; ++a) jc[a] = o.jcur[a * C + i];
            rd = o.red[i];
        }
        double old[kNavg][DIM + 1];  // the window but slot h, which is overwritten
        if (push) {
#pragma unroll
            for (int q = 0; q < kNavg; ++q)
#pragma unroll
                for (int c = 0; c <= DIM; ++c)
                    old[q][c] = q == h ? 0.0 : s.ring[(int64_t(q) * (DIM + 1) + c) * C + i];
        }
        uint8_t ev = 0;
        if (child) child[i] = -1;
        if (io) {
#pragma unroll
            for (int a = 0; a < 3; ++a) s.jprev[a * C + i] = jc[a];
            s.red_prev[i] = rd;
        }
        if (push) {
#pragma unroll
            for (int c = 0; c <= DIM; ++c) {
                s.ring[(int64_t(h) * (DIM + 1) + c) * C + i] = v[c];
                double sum = 0.0;
#pragma unroll
                for (int q = 0; q < kNavg; ++q) sum += q == h ? v[c] : old[q][c];
                s.avg[c * C + i] = sum / double(kNavg);
            }
            s.head[i] = uint8_t((h + 1) % kNavg);
            ev |= kEvPush;
        }
        if (t == SPH_FLUID && x > k.x_outlet) {
            s.type[i] = SPH_OUTLET;
#pragma unroll
            for (int a = 0; a < 3; ++a) s.jprev[a * C + i] = 0.0;
            s.red_prev[i] = 0;
            ev |= kEvToOutlet;
        } else if (t == SPH_OUTLET && x > k.x_outlet_end) {
            s.type[i] = SPH_DEAD;
            ev |= kEvDelete;
        } else if (t == SPH_INLET && x >= k.x_inlet) {
            s.type[i] = SPH_FLUID;
            spawn = true;
            ev |= kEvSpawn;
        }
        sflag[i] = spawn ? 1 : 0;
        if (events) events[i] = ev;
        // a kind change or a new row needs a fresh sort (boundary list, cells)
        if (k.reuse && (ev & (kEvToOutlet | kEvDelete | kEvSpawn))) *rebin = 1;
    }
    const int cnt = __syncthreads_count(spawn);
    if (threadIdx.x == 0) stile[blockIdx.x] = cnt;
}

// Appends the new inlet particles in the order of their parents' rows, so
// that the state after a step is reproducible row for row: parent i's new
// particle goes to row n + (number of flagged rows before i), at x - inlet_len
// (x only) with the parent's prescribed velocity (or a seeded noisy one),
// its pressure, and a ring and mean filled with those values. Block 0 also
// publishes the total in *nspawn.
template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_spawn(Dev k, DevState s, const uint8_t *sflag,
                                                  const int32_t *stile, int32_t *nspawn,
                                                  int32_t *child, uint32_t *err)
{
    __shared__ int32_t lds[kBlock];
    const int nb = gridDim.x;
    if (blockIdx.x == 0) {
        int32_t part = 0;
        for (int b = threadIdx.x; b < nb; b += kBlock) part += stile[b];
        int32_t total;
        block_exclusive_scan(part, lds, &total);
        if (threadIdx.x == 0) *nspawn = total;
    }
    if (stile[blockIdx.x] == 0) return;  // uniform over the block
    int32_t part = 0;
    for (int b = threadIdx.x; b < int(blockIdx.x); b += kBlock) part += stile[b];
    int32_t base;
    block_exclusive_scan(part, lds, &base);
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n = *s.n;
    const int f = i < n ? sflag[i] : 0;
    int32_t cnt;
    const int32_t rank = block_exclusive_scan(f, lds, &cnt);
    if (!f) return;
    const int64_t C = k.cap;
    const int64_t r = n + base + rank;
    if (r >= C) {
        raise_error(err, SPH_ERR_CAPACITY);
        return;
    }
    if (child) child[i] = int32_t(r);
    const int64_t cid = s.id[i] + kIdGeneration;
    double uin[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) uin[d] = s.uin[d * C + i];
    if (k.flags & SPH_FLAG_NOISE) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            const double xi = splitmix_uniform(k.noise_seed, cid, d);
            uin[d] = (d == 0 ? k.U : 0.0) + k.noise_amp * k.U * sqrt(3.0) * (2.0 * xi - 1.0);
        }
    }
    const double pv = double(ld<T>(s.p, i));
    const double x = s.x[i];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        s.x[d * C + r] = d == 0 ? x - k.inlet_len : s.x[d * C + i];
        s.uin[d * C + r] = uin[d];
        st<T>(s.u, d * C + r, T(uin[d]));
        st<T>(s.ut, d * C + r, T(uin[d]));
    }
    st<T>(s.p, r, T(pv));
#pragma unroll
    for (int c = 0; c <= DIM; ++c) {
        const double v = c < DIM ? uin[c] : pv;
#pragma unroll
        for (int q = 0; q < kNavg; ++q) s.ring[(int64_t(q) * (DIM + 1) + c) * C + r] = v;
        s.avg[c * C + r] = v;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) s.jprev[a * C + r] = 0.0;
    s.head[r] = 0;
    s.red_prev[r] = 0;
    s.type[r] = SPH_INLET;
    s.id[r] = cid;
}

__global__ void k_finish_spawn(Dev k, DevState s, int32_t *nspawn)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        int64_t n = *s.n + *nspawn;
        *s.n = n < k.cap ? n : k.cap;
        *nspawn = 0;
    }
}

// ------------------------------------------------------------------ launchers
void launch_end_of_step(const Dev &k, const DevState &st, const DevDerived &o,
                        int32_t *nspawn, uint8_t *sflag, int32_t *stile, int32_t *child,
                        uint8_t *events, int32_t *rebin, uint32_t *err, hipStream_t s)
{
    const dim3 g(nblocks(k.cap)), b(kBlock);
#define SPH_EOS(D, T)                                                                           \
    do {                                                                                        \
        hipLaunchKernelGGL((k_end_of_step<D, T>), g, b, 0, s, k, st, o, sflag, stile, child,    \
                           events, rebin);                                                      \
        hipLaunchKernelGGL((k_spawn<D, T>), g, b, 0, s, k, st, sflag, stile, nspawn, child, err); \
    } while (0)
    if (k.dim == 2 && k.prec == SPH_FP64) SPH_EOS(2, double);
    else if (k.dim == 3 && k.prec == SPH_FP64) SPH_EOS(3, double);
    else if (k.dim == 2) SPH_EOS(2, float);
    else SPH_EOS(3, float);
#undef SPH_EOS
}

void launch_finish_spawn(const Dev &k, const DevState &st, int32_t *nspawn, hipStream_t s)
{
    hipLaunchKernelGGL(k_finish_spawn, dim3(1), dim3(64), 0, s, k, st, nspawn);
}

}  // namespace sph
