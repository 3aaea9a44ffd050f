// update.hip -- explicit-midpoint RK2 stage updates and the end-of-step
// bookkeeping of the hybrid outlet (gated time averages, transfers,
// deletion, inlet re-spawn) for gfx950.
#include "sph_launch.h"

namespace sph {

__global__ void k_save_start_d(Dev k, DevState s, double *x0, double *u0, double *p0)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= *s.n) return;
    const int64_t C = k.cap;
    for (int d = 0; d < k.dim; ++d) {
        x0[d * C + i] = s.x[d * C + i];
        u0[d * C + i] = ld<double>(s.u, d * C + i);
    }
    p0[i] = ld<double>(s.p, i);
}

__global__ void k_save_start_f(Dev k, DevState s, double *x0, float *u0, float *p0)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= *s.n) return;
    const int64_t C = k.cap;
    for (int d = 0; d < k.dim; ++d) {
        x0[d * C + i] = s.x[d * C + i];
        u0[d * C + i] = ld<float>(s.u, d * C + i);
    }
    p0[i] = ld<float>(s.p, i);
}

// Half (full = 0) or full (full = 1) update from the start-of-step copies.
// Fluid: u = u0 + dt a, p = p0 + dt pdot, ut = u + dt b (eq:transport-vel
// with the stage's sub-step), x = x0 + dt ut evaluated with the transport
// velocity of the half state (eq:advection). Inlet particles move with their
// prescribed velocity, outlet particles along x only with their composed
// velocity; walls are fixed.
template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_stage(Dev k, DevState s, DevDerived o,
                                                  const double *x0, const T *u0, const T *p0,
                                                  int full, uint32_t *err)
{
#pragma clang fp contract(off)
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= *s.n) return;
    const int64_t C = k.cap;
    const int t = s.type[i];
    const double dt = full ? k.dt : k.hdt;
    double xn[3] = {0, 0, 0};
    bool finite = true;
    if (t == SPH_FLUID) {
        double utn[3];
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            double xs = x0[d * C + i];
            double un = double(u0[d * C + i]) + dt * double(ld<T>(o.a, d * C + i));
            double bn = double(ld<T>(o.b, d * C + i));
            if (full) xn[d] = xs + dt * double(ld<T>(s.ut, d * C + i));
            utn[d] = un + dt * bn;
            if (!full) xn[d] = xs + dt * utn[d];
            st<T>(s.u, d * C + i, T(un));
            finite = finite && isfinite(un) && isfinite(utn[d]);
        }
#pragma unroll
        for (int d = 0; d < DIM; ++d) st<T>(s.ut, d * C + i, T(utn[d]));
        double pn = double(p0[i]) + dt * double(ld<T>(o.pdot, i));
        finite = finite && isfinite(pn);
        st<T>(s.p, i, T(pn));
    } else if (t == SPH_INLET || t == SPH_OUTLET) {
        double vx = t == SPH_INLET ? s.uin[i] : double(ld<T>(s.u, i));
#pragma unroll
        for (int d = 0; d < DIM; ++d) xn[d] = x0[d * C + i];
        xn[0] = x0[i] + dt * vx;
    } else {
        return;
    }
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        double v = xn[d];
        if (k.periodic[d]) {
            double hi = k.lo[d] + k.L[d];
            if (v >= hi) v -= k.L[d];
            else if (v < k.lo[d]) v += k.L[d];
        }
        finite = finite && isfinite(v);
        if (!full) {
            double disp = min_image(v - x0[d * C + i], k.periodic[d], k.L[d], k.halfL[d]);
            if (!(fabs(disp) <= k.disp_max)) raise_error(err, SPH_ERR_SKIN);
        }
        s.x[d * C + i] = v;
    }
    if (!finite) raise_error(err, SPH_ERR_NONFINITE);
}

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
void launch_save_start(const Dev &k, const DevState &st, double *x0, void *u0, void *p0,
                       hipStream_t s)
{
    if (k.prec == SPH_FP64)
        hipLaunchKernelGGL(k_save_start_d, dim3(nblocks(k.cap)), dim3(kBlock), 0, s, k, st, x0,
                           (double *)u0, (double *)p0);
    else
        hipLaunchKernelGGL(k_save_start_f, dim3(nblocks(k.cap)), dim3(kBlock), 0, s, k, st, x0,
                           (float *)u0, (float *)p0);
}

void launch_stage(const Dev &k, const DevState &st, const DevDerived &o, const double *x0,
                  const void *u0, const void *p0, int full, uint32_t *err, hipStream_t s)
{
    dim3 g(nblocks(k.cap)), b(kBlock);
    if (k.dim == 2 && k.prec == SPH_FP64)
        hipLaunchKernelGGL((k_stage<2, double>), g, b, 0, s, k, st, o, x0, (const double *)u0,
                           (const double *)p0, full, err);
    else if (k.dim == 3 && k.prec == SPH_FP64)
        hipLaunchKernelGGL((k_stage<3, double>), g, b, 0, s, k, st, o, x0, (const double *)u0,
                           (const double *)p0, full, err);
    else if (k.dim == 2)
        hipLaunchKernelGGL((k_stage<2, float>), g, b, 0, s, k, st, o, x0, (const float *)u0,
                           (const float *)p0, full, err);
    else
        hipLaunchKernelGGL((k_stage<3, float>), g, b, 0, s, k, st, o, x0, (const float *)u0,
                           (const float *)p0, full, err);
}

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
