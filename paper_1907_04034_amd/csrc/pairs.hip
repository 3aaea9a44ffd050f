// pairs.hip -- neighbour-pair passes of libsph for gfx950: neighbour table,
// summation density, boundary values (walls, hybrid outlet, MOC inlet) and the
// EDAC-TVF force pass with the body force.
//
// One work-item per target particle; particles are Morton-sorted so the
// neighbours of a wave's 64 targets lie in a handful of cells and their
// gathers are served from L2. The neighbour table is column-major
// (nbr[k * cap + i]) so the k-th neighbour of 64 consecutive targets is one
// coalesced 256-byte load.
#include "sph_launch.h"

namespace sph {

// ---------------------------------------------------------- neighbour table
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_neighbors(Dev k, DevState s, DevNlist nl,
                                                      const uint32_t *spread,
                                                      const int32_t *cell_start,
                                                      const uint32_t *cpos, uint32_t *err)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t n = *s.n;
    if (i >= n) return;
    const int64_t C = k.cap;
    double xi[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) xi[d] = s.x[d * C + i];
    int c[3];
    unpack_cell<DIM>(cpos[i], c);
    int cnt = 0;
    const int zlo = DIM == 3 ? -1 : 0, zhi = DIM == 3 ? 1 : 0;
    for (int dz = zlo; dz <= zhi; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int cc[3] = {c[0] + dx, c[1] + dy, c[2] + dz};
                bool ok = true;
#pragma unroll
                for (int d = 0; d < DIM; ++d) {
                    if (cc[d] < 0 || cc[d] >= k.nc[d]) {
                        if (k.periodic[d]) cc[d] = cc[d] < 0 ? cc[d] + k.nc[d] : cc[d] - k.nc[d];
                        else ok = false;
                    }
                }
                if (!ok) continue;
                uint32_t key = morton_key<DIM>(spread, cc);
                int32_t b = cell_start[key], e = cell_start[key + 1];
                if (b < 0 || e > n || b > e) {
                    raise_error(err, SPH_ERR_CELL_RANGE);
                    continue;
                }
                for (int32_t j = b; j < e; ++j) {
                    double xj[3] = {0, 0, 0};
#pragma unroll
                    for (int d = 0; d < DIM; ++d) xj[d] = s.x[d * C + j];
                    double r[3];
                    double r2 = dist2_exact<DIM>(k, xi, xj, r);
                    if (r2 < k.sup2) {
                        if (cnt < nl.maxnb) nl.nbr[int64_t(cnt) * C + i] = j;
                        ++cnt;
                    }
                }
            }
    if (cnt > nl.maxnb) {
        raise_error(err, SPH_ERR_NBR_OVERFLOW);
        cnt = nl.maxnb;
    }
    nl.count[i] = cnt;
}

// Neighbour index check: a table from the wrong workspace or a stale count
// must not send a gather out of bounds.
__device__ inline bool bad_index(int32_t j, int64_t n) { return uint64_t(j) >= uint64_t(n); }

// ------------------------------------------------------------------ density
// Sec. 2 eq:summation-density with m_j = m, and V_i = 1 / sum_j W_ij.
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_density(Dev k, DevState s, DevNlist nl,
                                                    DevDerived o, uint32_t *err)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t n = *s.n;
    if (i >= n) return;
    const int64_t C = k.cap;
    double xi[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) xi[d] = s.x[d * C + i];
    int cnt = nl.count[i];
    double sw = 0.0;
    for (int q = 0; q < cnt; ++q) {
        int32_t j = nl.nbr[int64_t(q) * C + i];
        if (bad_index(j, n)) {
            raise_error(err, SPH_ERR_CELL_RANGE);
            continue;
        }
        double xj[3] = {0, 0, 0};
#pragma unroll
        for (int d = 0; d < DIM; ++d) xj[d] = s.x[d * C + j];
        double r[3];
        double r2 = dist2_exact<DIM>(k, xi, xj, r);
        sw += wendland_w(sqrt(r2) / k.h, k.wnorm);
    }
    st<double>(o.rho, i, k.mass * sw);
    st<double>(o.vol, i, 1.0 / sw);
}

// ---------------------------------------------------------- boundary values
// Walls: Shepard-averaged fluid pressure and ghost velocity u_g = -<u_f>
// (static walls, no body force). Outlet: characteristic variables of the
// fluid with the fluid's own time averages as references (Sec. 3.3
// eq:characteristic-vars, Sec. 3.4), Shepard-interpolated (eq:shepard), J3 = 0;
// particles with no fluid in support take the mean previous-step value of
// same-kind neighbours that had support (eq:average_old), else their own;
// then u, p = time average + acoustic part (eq:acou) with rho_ref = rho0.
// Inlet: prescribed velocity, p = Shepard J3 with reference (u_in, 0).
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_boundary(Dev k, DevState s, DevNlist nl,
                                                     DevDerived o, uint32_t *err)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t n = *s.n;
    if (i >= n) return;
    const int t = s.type[i];
    if (t == SPH_FLUID) return;
    const int64_t C = k.cap;
    double xi[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) xi[d] = s.x[d * C + i];
    const double uin0 = s.uin[i];
    double sw = 0.0, sp = 0.0, su[3] = {0, 0, 0}, sJ[3] = {0, 0, 0};
    int cnt = nl.count[i];
    for (int q = 0; q < cnt; ++q) {
        int32_t j = nl.nbr[int64_t(q) * C + i];
        if (bad_index(j, n)) {
            raise_error(err, SPH_ERR_CELL_RANGE);
            continue;
        }
        if (s.type[j] != SPH_FLUID) continue;
        double xj[3] = {0, 0, 0};
#pragma unroll
        for (int d = 0; d < DIM; ++d) xj[d] = s.x[d * C + j];
        double r[3];
        double w = wendland_w(sqrt(dist2_exact<DIM>(k, xi, xj, r)) / k.h, k.wnorm);
        double pj = ld<double>(s.p, j);
        double rhoj = ld<double>(o.rho, j);
        double uj0 = ld<double>(s.u, j);
        sw += w;
        sp += pj * w;
#pragma unroll
        for (int d = 0; d < DIM; ++d) su[d] += ld<double>(s.u, d * C + j) * w;
        if (t == SPH_INLET) {
            sJ[2] += (-rhoj * k.c * (uj0 - uin0) + pj) * w;
        } else if (t == SPH_OUTLET) {
            double dp = pj - s.avg[DIM * C + j];
            double du = uj0 - s.avg[j];
            sJ[0] += (-k.c2 * (rhoj - k.rho0) + dp) * w;
            sJ[1] += (rhoj * k.c * du + dp) * w;
            sJ[2] += (-rhoj * k.c * du + dp) * w;
        }
    }
    if (is_wall(t)) {
        double pw = 0.0, ug[3] = {0, 0, 0};
        if (sw > 0.0) {
            pw = sp / sw;
#pragma unroll
            for (int d = 0; d < DIM; ++d) ug[d] = -(su[d] / sw);
        }
        st<double>(s.p, i, pw);
#pragma unroll
        for (int d = 0; d < DIM; ++d) st<double>(s.u, d * C + i, ug[d]);
        return;
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
        double acc[3] = {0, 0, 0};
        int M = 0;
        for (int q = 0; q < cnt; ++q) {
            int32_t j = nl.nbr[int64_t(q) * C + i];
            if (bad_index(j, n)) continue;
            if (s.type[j] == t && s.red_prev[j]) {
#pragma unroll
                for (int a = 0; a < 3; ++a) acc[a] += s.jprev[a * C + j];
                ++M;
            }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) J[a] = M ? acc[a] / double(M) : s.jprev[a * C + i];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) o.jcur[a * C + i] = J[a];
    o.red[i] = red;
    if (t == SPH_OUTLET) {
        double p_ac = 0.5 * (J[1] + J[2]);
        double u_ac = (J[1] - J[2]) / (2.0 * k.rho0 * k.c);
        st<double>(s.p, i, s.avg[DIM * C + i] + p_ac);
        double u0v = s.avg[i] + u_ac;
        st<double>(s.u, i, u0v);
        st<double>(s.ut, i, u0v);
#pragma unroll
        for (int d = 1; d < DIM; ++d) {
            st<double>(s.u, d * C + i, s.avg[d * C + i]);
            st<double>(s.ut, d * C + i, s.avg[d * C + i]);
        }
    } else {  // inlet
        st<double>(s.p, i, J[2]);
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            st<double>(s.u, d * C + i, s.uin[d * C + i]);
            st<double>(s.ut, d * C + i, s.uin[d * C + i]);
        }
    }
}

// ---------------------------------------------------------------- force pass
// Fluid i: pbar_i (eq:pavg, self included), then over j != i the momentum
// rate of eq:tvf-momentum with p~_ij of eq:tvf-p-ij-basa, the background term
// of eq:transport-vel and the pressure rate of eq:p-edac. A = rho u (ut - u)
// for fluid, 0 otherwise; slip walls take no viscous part; walls enter the
// divergence with zero wall velocity and the viscous term with u_g.
// Body i: force of eq:tvf-momentum_solid from fluid neighbours.
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_force(Dev k, DevState s, DevNlist nl, DevDerived o,
                                                  double *dragpart, uint32_t *err)
{
    __shared__ double red_lds[3][kBlock];
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t n = *s.n;
    const int64_t C = k.cap;
    double fb[3] = {0, 0, 0};
    if (i < n) {
        const int t = s.type[i];
        double acc[3] = {0, 0, 0}, bacc[3] = {0, 0, 0}, pdot = 0.0, pavg = 0.0;
        if (t == SPH_FLUID || t == SPH_BODY) {
            const int cnt = nl.count[i];
            if (!(k.flags & SPH_FLAG_NO_PAVG)) {
                double sp = 0.0;
                for (int q = 0; q < cnt; ++q) {
                    int32_t j = nl.nbr[int64_t(q) * C + i];
                    if (bad_index(j, n)) continue;
                    sp += ld<double>(s.p, j);
                }
                pavg = sp / double(cnt);
            }
            double xi[3] = {0, 0, 0}, ui[3] = {0, 0, 0}, wi[3] = {0, 0, 0};
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                xi[d] = s.x[d * C + i];
                ui[d] = ld<double>(s.u, d * C + i);
                wi[d] = ld<double>(s.ut, d * C + i) - ui[d];
            }
            const double pi = ld<double>(s.p, i);
            const double rhoi = ld<double>(o.rho, i);
            const double vi = ld<double>(o.vol, i);
            const double vi2 = vi * vi;
            const double inv_m = 1.0 / k.mass;
            for (int q = 0; q < cnt; ++q) {
                int32_t j = nl.nbr[int64_t(q) * C + i];
                if (bad_index(j, n)) {
                    raise_error(err, SPH_ERR_CELL_RANGE);
                    continue;
                }
                if (j == i) continue;
                const int tj = s.type[j];
                if (t == SPH_BODY && tj != SPH_FLUID) continue;
                double xj[3] = {0, 0, 0};
#pragma unroll
                for (int d = 0; d < DIM; ++d) xj[d] = s.x[d * C + j];
                double r[3];
                const double r2 = dist2_exact<DIM>(k, xi, xj, r);
                const double F = wendland_f(sqrt(r2) / k.h, k.gnorm);
                double gw[3] = {0, 0, 0}, uj[3] = {0, 0, 0};
#pragma unroll
                for (int d = 0; d < DIM; ++d) {
                    gw[d] = F * r[d];
                    uj[d] = ld<double>(s.u, d * C + j);
                }
                const double vj = ld<double>(o.vol, j);
                const double vsq = vi2 + vj * vj;
                const double rhoj = ld<double>(o.rho, j);
                const double pj = ld<double>(s.p, j);
                const double inv_rs = 1.0 / (rhoi + rhoj);
                const double ptil = (rhoj * (pi - pavg) + rhoi * (pj - pavg)) * inv_rs;
                const double hm = 2.0 * rhoi * rhoj * inv_rs;  // eta~ / nu
                const double dfac = F * r2 / (r2 + k.eta_h2);
                if (t == SPH_FLUID) {
                    double si = 0.0, sj = 0.0;
#pragma unroll
                    for (int d = 0; d < DIM; ++d) si += wi[d] * gw[d];
                    if (tj == SPH_FLUID) {
#pragma unroll
                        for (int d = 0; d < DIM; ++d)
                            sj += (ld<double>(s.ut, d * C + j) - uj[d]) * gw[d];
                    }
                    const double visc = tj == SPH_WALL_SLIP ? 0.0 : hm * k.nu * dfac;
                    const double f = vsq * inv_m;
                    double udiv = 0.0;
                    const bool wall = is_wall(tj);
#pragma unroll
                    for (int d = 0; d < DIM; ++d) {
                        const double aterm = 0.5 * (rhoi * ui[d] * si + rhoj * uj[d] * sj);
                        acc[d] += f * (-ptil * gw[d] + aterm + visc * (ui[d] - uj[d]));
                        bacc[d] += -k.pb * inv_m * vsq * gw[d];
                        udiv += (ui[d] - (wall ? 0.0 : uj[d])) * gw[d];
                    }
                    pdot += k.mass * rhoi / rhoj * k.c2 * udiv +
                            f * (hm * k.nu_damp) * dfac * (pi - pj);
                } else {
#pragma unroll
                    for (int d = 0; d < DIM; ++d)
                        fb[d] += vsq * (-ptil * gw[d] + hm * k.nu * dfac * (ui[d] - uj[d]));
                }
            }
        }
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            st<double>(o.a, d * C + i, acc[d]);
            st<double>(o.b, d * C + i, bacc[d]);
            if (t == SPH_BODY) o.force[d * C + i] = fb[d];
        }
        st<double>(o.pdot, i, pdot);
        st<double>(o.pavg, i, pavg);
    }
    // deterministic per-block partial of the body force (fixed tree order)
#pragma unroll
    for (int d = 0; d < 3; ++d) red_lds[d][threadIdx.x] = fb[d];
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (int(threadIdx.x) < off)
#pragma unroll
            for (int d = 0; d < 3; ++d) red_lds[d][threadIdx.x] += red_lds[d][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int d = 0; d < 3; ++d) dragpart[d * gridDim.x + blockIdx.x] = red_lds[d][0];
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
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (int(threadIdx.x) < off)
#pragma unroll
            for (int d = 0; d < 3; ++d) lds[d][threadIdx.x] += lds[d][threadIdx.x + off];
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
#define SPH_DIM_DISPATCH(KERNEL, ...)                                                         \
    do {                                                                                      \
        if (k.dim == 2)                                                                       \
            hipLaunchKernelGGL(KERNEL<2>, dim3(nblocks(k.cap)), dim3(kBlock), 0, s,           \
                               __VA_ARGS__);                                                  \
        else                                                                                  \
            hipLaunchKernelGGL(KERNEL<3>, dim3(nblocks(k.cap)), dim3(kBlock), 0, s,           \
                               __VA_ARGS__);                                                  \
    } while (0)

void launch_neighbors(const Dev &k, const DevState &st, const DevNlist &nl,
                      const uint32_t *spread, const int32_t *cell_start, const uint32_t *cpos,
                      uint32_t *err, hipStream_t s)
{
    SPH_DIM_DISPATCH(k_neighbors, k, st, nl, spread, cell_start, cpos, err);
}

void launch_density(const Dev &k, const DevState &st, const DevNlist &nl, const DevDerived &o,
                    uint32_t *err, hipStream_t s)
{
    SPH_DIM_DISPATCH(k_density, k, st, nl, o, err);
}

void launch_boundary(const Dev &k, const DevState &st, const DevNlist &nl, const DevDerived &o,
                     uint32_t *err, hipStream_t s)
{
    SPH_DIM_DISPATCH(k_boundary, k, st, nl, o, err);
}

void launch_force(const Dev &k, const DevState &st, const DevNlist &nl, const DevDerived &o,
                  double *dragpart, uint32_t *err, hipStream_t s)
{
    SPH_DIM_DISPATCH(k_force, k, st, nl, o, dragpart, err);
}

void launch_drag_final(const Dev &k, const double *dragpart, double *drag, double *hist,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_drag_final, dim3(1), dim3(kBlock), 0, s, nblocks(k.cap), dragpart,
                       drag, hist);
}

}  // namespace sph
