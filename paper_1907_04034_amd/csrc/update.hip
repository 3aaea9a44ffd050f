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
// the inlet and outlet interfaces, deleted past the outlet end, and every
// inlet particle entering the fluid leaves a new inlet particle inlet_len
// behind it.
template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_end_of_step(Dev k, DevState s, DevDerived o,
                                                        int32_t *nspawn, uint32_t *err)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n = *s.n;
    if (i >= n) return;
    const int64_t C = k.cap;
    int t = s.type[i];
    if (t == SPH_OUTLET || t == SPH_INLET) {
#pragma unroll
        for (int a = 0; a < 3; ++a) s.jprev[a * C + i] = o.jcur[a * C + i];
        s.red_prev[i] = o.red[i];
    }
    if (t == SPH_FLUID || t == SPH_INLET) {
        double pv = double(ld<T>(s.p, i));
        if (!(fabs(pv) > k.pgate)) {
            int h = s.head[i];
            double v[DIM + 1];
#pragma unroll
            for (int d = 0; d < DIM; ++d) v[d] = double(ld<T>(s.u, d * C + i));
            v[DIM] = pv;
#pragma unroll
            for (int c = 0; c <= DIM; ++c) {
                s.ring[(int64_t(h) * (DIM + 1) + c) * C + i] = v[c];
                double sum = 0.0;
#pragma unroll
                for (int q = 0; q < kNavg; ++q)
                    sum += q == h ? v[c] : s.ring[(int64_t(q) * (DIM + 1) + c) * C + i];
                s.avg[c * C + i] = sum / double(kNavg);
            }
            s.head[i] = uint8_t((h + 1) % kNavg);
        }
    }
    const double x = s.x[i];
    if (t == SPH_FLUID && x > k.x_outlet) {
        s.type[i] = SPH_OUTLET;
#pragma unroll
        for (int a = 0; a < 3; ++a) s.jprev[a * C + i] = 0.0;
        s.red_prev[i] = 0;
    } else if (t == SPH_OUTLET && x > k.x_outlet_end) {
        s.type[i] = SPH_DEAD;
    } else if (t == SPH_INLET && x >= k.x_inlet) {
        s.type[i] = SPH_FLUID;
        int64_t r = n + atomicAdd(nspawn, 1);
        if (r >= C) {
            raise_error(err, SPH_ERR_CAPACITY);
            return;
        }
        int64_t cid = s.id[i] + kIdGeneration;
        double uin[3] = {0, 0, 0};
#pragma unroll
        for (int d = 0; d < DIM; ++d) uin[d] = s.uin[d * C + i];
        if (k.flags & SPH_FLAG_NOISE) {
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                double xi = splitmix_uniform(k.noise_seed, cid, d);
                uin[d] = (d == 0 ? k.U : 0.0) + k.noise_amp * k.U * sqrt(3.0) * (2.0 * xi - 1.0);
            }
        }
        double pv = double(ld<T>(s.p, i));
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
            double v = c < DIM ? uin[c] : pv;
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
                        int32_t *nspawn, uint32_t *err, hipStream_t s)
{
    dim3 g(nblocks(k.cap)), b(kBlock);
    if (k.dim == 2 && k.prec == SPH_FP64)
        hipLaunchKernelGGL((k_end_of_step<2, double>), g, b, 0, s, k, st, o, nspawn, err);
    else if (k.dim == 3 && k.prec == SPH_FP64)
        hipLaunchKernelGGL((k_end_of_step<3, double>), g, b, 0, s, k, st, o, nspawn, err);
    else if (k.dim == 2)
        hipLaunchKernelGGL((k_end_of_step<2, float>), g, b, 0, s, k, st, o, nspawn, err);
    else
        hipLaunchKernelGGL((k_end_of_step<3, float>), g, b, 0, s, k, st, o, nspawn, err);
}

void launch_finish_spawn(const Dev &k, const DevState &st, int32_t *nspawn, hipStream_t s)
{
    hipLaunchKernelGGL(k_finish_spawn, dim3(1), dim3(64), 0, s, k, st, nspawn);
}

}  // namespace sph
