// step_adjoint.hip -- hand-written reverse of one explicit-midpoint step for
// gfx950, built on the reverse of the right-hand side (adjoint.hip).
//
// A step maps the state S_n (rows in the order the previous step left them)
// to S_{n+1}:
//   bin        S'_n = S_n gathered in cell order (dead rows dropped);
//   stage 1    boundary values of S'_n, force pass, half update -> H;
//   stage 2    boundary values of H, force pass, full update -> S_{n+1};
//   end        characteristic values become previous-step values, gated ring
//              push with its mean, transfers, inlet re-spawn (children are
//              appended after the live rows).
// Given the adjoint of S_{n+1} (lam_next) and the weight of the stage-1 body
// force, the reverse returns the adjoint of S_n, for fixed discrete events
// (neighbour sets, supported / unsupported boundary particles, gates,
// transfers), which the forward recorded. The reverse recomputes the stage
// values from S_n and runs, per row:
//   end    reverse of the end-of-step bookkeeping (children -> parents, ring
//          push and mean, J -> previous-step values), then of the full
//          update: weights on stage-2 rates, seeds on the stage-2 boundary
//          values, direct position/velocity/pressure parts;
//   (reverse of the stage-2 right-hand side)
//   half   reverse of the half update: weights on stage-1 rates and seeds;
//   (reverse of the stage-1 right-hand side, with the drag weight)
//   finish sum of the start-state parts, written to the row of S_n that the
//          bin moved (a permutation, so no two rows collide); rows of S_n the
//          bin dropped get zero.
#include "sph_launch.h"

namespace sph {

// ------------------------------------------------------------ bookkeeping
__global__ void k_adj_prep(const int64_t *n_src, int64_t *n_dst, int32_t *nspawn)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *n_dst = *n_src;
        *nspawn = 0;
    }
}

// ------------------------------------------------------------ end of step
// Reverse of the bookkeeping, then of the full update
//   fluid:   u' = u + dt a2, ut' = u' + dt b2, x' = x + dt ut_H, p' = p + dt pdot2
//   inlet:   x' = x + dt u_in (x only); u', ut', p' = stage-2 boundary values
//   outlet:  x' = x + dt u_H (x only, u_H its stage-2 boundary value); same
//   walls:   x' = x; u', p' = stage-2 boundary values
template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_adj_end(Dev k, DevState m, StepAdj S, DevAdj A)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= *m.n) return;
    constexpr int NC = DIM + 1, NR = kNavg * NC;
    const int64_t C = k.cap;
    const int t = m.type[i];
    const uint8_t ev = S.events[i];
    const int32_t r = S.child[i];
    const DevLam &N = S.next;
    double Lx[3] = {0, 0, 0}, Lu[3] = {0, 0, 0}, Lut[3] = {0, 0, 0}, uin[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        Lx[d] = N.x[d * C + i];
        Lu[d] = N.u[d * C + i];
        Lut[d] = N.ut[d * C + i];
        uin[d] = N.uin[d * C + i];
    }
    double Lp = N.p[i];
    double ring[NR], avg[NC], jp[3];
#pragma unroll
    for (int q = 0; q < NR; ++q) ring[q] = N.ring[q * C + i];
#pragma unroll
    for (int c = 0; c < NC; ++c) avg[c] = N.avg[c * C + i];
#pragma unroll
    for (int a = 0; a < 3; ++a) jp[a] = N.jprev[a * C + i];
    if ((ev & kEvSpawn) && r >= 0 && r < C) {
        // the re-spawned inlet particle: x = parent x - inlet_len (x only),
        // u = ut = ring = mean = u_in of the parent, p and the p-slots = parent p
#pragma unroll
        for (int d = 0; d < DIM; ++d) Lx[d] += N.x[d * C + r];
        double cp = N.p[r] + N.avg[DIM * C + r];
#pragma unroll
        for (int q = 0; q < kNavg; ++q) cp += N.ring[(q * NC + DIM) * C + r];
        Lp += cp;
        if (!(k.flags & SPH_FLAG_NOISE)) {
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                double cu = N.uin[d * C + r] + N.u[d * C + r] + N.ut[d * C + r] + N.avg[d * C + r];
#pragma unroll
                for (int q = 0; q < kNavg; ++q) cu += N.ring[(q * NC + d) * C + r];
                uin[d] += cu;
            }
        }
    }
    if (ev & kEvPush) {
        // ring[h] = (u, p) after the step; mean = sum of the ring / N
        const int h = m.head[i];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double share = avg[c] / double(kNavg);
            double v = 0.0;
#pragma unroll
            for (int q = 0; q < kNavg; ++q) {
                const double tot = ring[q * NC + c] + share;
                if (q == h) v = tot;
                ring[q * NC + c] = q == h ? 0.0 : tot;
            }
            avg[c] = 0.0;
            if (c < DIM) Lu[c] += v;
            else Lp += v;
        }
    }
    double js[3] = {0, 0, 0};
    if (t == SPH_INLET || t == SPH_OUTLET) {
        // previous-step values of the next step = this step's stage-2 J
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            js[a] = jp[a];
            jp[a] = 0.0;
        }
    } else if (ev & kEvToOutlet) {
#pragma unroll
        for (int a = 0; a < 3; ++a) jp[a] = 0.0;
    }
    // full update
    const double dt = k.dt;
    double *useed = const_cast<double *>(A.useed), *pseed = const_cast<double *>(A.pseed);
    double us[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const bool on = d < DIM;
        double au = 0.0, ab = 0.0, hut = 0.0, uacc = 0.0;
        if (t == SPH_FLUID) {
            uacc = Lu[d] + Lut[d];
            au = dt * uacc;
            ab = dt * Lut[d];
            hut = dt * Lx[d];
        } else if (t == SPH_INLET || t == SPH_OUTLET) {
            us[d] = Lu[d] + Lut[d];  // the boundary value is written to u and ut
            if (d == 0 && t == SPH_INLET) uin[0] += dt * Lx[0];
            if (d == 0 && t == SPH_OUTLET) us[0] += dt * Lx[0];
        } else {
            us[d] = Lu[d];
        }
        S.acc.x[d * C + i] = Lx[d];
        S.acc.u[d * C + i] = uacc;
        S.acc.ut[d * C + i] = 0.0;
        S.acc.uin[d * C + i] = uin[d];
        S.acc.jprev[d * C + i] = jp[d];
        S.jseed[d * C + i] = js[d];
        S.hut[d * C + i] = hut;
        if (on) {
            st<T>(const_cast<void *>(A.abar), d * C + i, T(au));
            st<T>(const_cast<void *>(A.bbar), d * C + i, T(ab));
        }
        useed[d * C + i] = us[d];
    }
    const bool fl = t == SPH_FLUID;
    st<T>(const_cast<void *>(A.pdbar), i, T(fl ? dt * Lp : 0.0));
    pseed[i] = fl ? 0.0 : Lp;
    S.acc.p[i] = fl ? Lp : 0.0;
#pragma unroll
    for (int q = 0; q < NR; ++q) S.acc.ring[q * C + i] = ring[q];
#pragma unroll
    for (int c = 0; c < NC; ++c) S.acc.avg[c * C + i] = avg[c];
}

// ------------------------------------------------------------ half update
// fluid:   u_H = u + hdt a1, ut_H = u_H + hdt b1, x_H = x + hdt ut_H,
//          p_H = p + hdt pdot1
// inlet:   x_H = x + hdt u_in (x only); outlet: x_H = x + hdt u_1 (x only,
//          u_1 its stage-1 boundary value); walls: x_H = x
template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_adj_half(Dev k, DevState m, StepAdj S, DevAdj A)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= *m.n) return;
    constexpr int NC = DIM + 1;
    const int64_t C = k.cap;
    const int t = m.type[i];
    const bool fl = t == SPH_FLUID;
    const double hdt = k.hdt;
    double *useed = const_cast<double *>(A.useed), *pseed = const_cast<double *>(A.pseed);
    // every load before the first store: the stores could alias the arrays
    // read, and a load after a store waits for it
    double avg[NC], avgb[NC], jp[3], jpb[3];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        avg[c] = S.acc.avg[c * C + i];
        avgb[c] = A.avgbar[c * C + i];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        jp[a] = S.acc.jprev[a * C + i];
        jpb[a] = A.jprevbar[a * C + i];
    }
    double xH[3] = {0, 0, 0}, ax[3] = {0, 0, 0}, ain[3] = {0, 0, 0}, uinb[3] = {0, 0, 0},
           utb[3] = {0, 0, 0}, hut[3] = {0, 0, 0}, ubr[3] = {0, 0, 0}, au_acc[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        xH[d] = A.xbar[d * C + i];
        ax[d] = S.acc.x[d * C + i];
        ain[d] = S.acc.uin[d * C + i];
        uinb[d] = A.uinbar[d * C + i];
        if (fl) {
            utb[d] = A.utbar[d * C + i];
            hut[d] = S.hut[d * C + i];
            ubr[d] = A.ubar[d * C + i];
            au_acc[d] = S.acc.u[d * C + i];
        }
    }
    double pH = 0.0, ap = 0.0;
    if (fl) {
        pH = A.pbar[i];
        ap = S.acc.p[i];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) S.acc.avg[c * C + i] = avg[c] + avgb[c];
#pragma unroll
    for (int a = 0; a < 3; ++a) S.acc.jprev[a * C + i] = jp[a] + jpb[a];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        S.acc.x[d * C + i] = ax[d] + xH[d];
        double uin_acc = ain[d] + uinb[d];
        double au = 0.0, ab = 0.0, us = 0.0;
        if (fl) {
            const double utot = utb[d] + hut[d] + hdt * xH[d];
            const double uu = ubr[d] + utot;
            au = hdt * uu;
            ab = hdt * utot;
            S.acc.u[d * C + i] = au_acc[d] + uu;
        } else if (d == 0 && t == SPH_INLET) {
            uin_acc += hdt * xH[d];
        } else if (d == 0 && t == SPH_OUTLET) {
            us = hdt * xH[d];
        }
        S.acc.uin[d * C + i] = uin_acc;
        st<T>(const_cast<void *>(A.abar), d * C + i, T(au));
        st<T>(const_cast<void *>(A.bbar), d * C + i, T(ab));
        useed[d * C + i] = us;
    }
    double pd = 0.0;
    if (fl) {
        pd = hdt * pH;
        S.acc.p[i] = ap + pH;
    }
    st<T>(const_cast<void *>(A.pdbar), i, T(pd));
    pseed[i] = 0.0;
}

// ------------------------------------------------------------ finish
// Sum of the start-state parts of sorted row r, written to row perm[r] of
// S_n; rows of S_n the bin dropped (deleted particles) get zero. Boundary
// rows' u, ut, p of the start state are overwritten by the stage-1 boundary
// values before any use, so only fluid rows take those parts.
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_adj_finish(Dev k, DevState m, DevState pre,
                                                       const int32_t *perm, StepAdj S, DevAdj A)
{
    const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t npre = *S.n_pre, npost = *m.n;
    constexpr int NC = DIM + 1, NR = kNavg * NC;
    const int64_t C = k.cap;
    const DevLam &O = S.out;
    if (q < npre && pre.type[q] == SPH_DEAD) {
#pragma unroll
        for (int d = 0; d < 3; ++d)
            O.x[d * C + q] = O.u[d * C + q] = O.ut[d * C + q] = O.uin[d * C + q] =
                O.jprev[d * C + q] = 0.0;
        O.p[q] = 0.0;
#pragma unroll
        for (int s = 0; s < NR; ++s) O.ring[s * C + q] = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) O.avg[c * C + q] = 0.0;
    }
    if (q >= npost) return;
    const int64_t r = q;  // sorted row
    const int32_t dst = perm[r];
    if (dst < 0 || dst >= npre) return;
    const bool fl = m.type[r] == SPH_FLUID;
    const DevLam &Ac = S.acc;
    // every load before the first store (the stores could alias them, and a
    // load after a store waits for it)
    double x[3] = {0, 0, 0}, u[3] = {0, 0, 0}, ut[3] = {0, 0, 0}, uin[3] = {0, 0, 0}, jp[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (d < DIM) {
            x[d] = Ac.x[d * C + r] + A.xbar[d * C + r];
            u[d] = Ac.u[d * C + r] + (fl ? A.ubar[d * C + r] : 0.0);
            ut[d] = Ac.ut[d * C + r] + (fl ? A.utbar[d * C + r] : 0.0);
            uin[d] = Ac.uin[d * C + r] + A.uinbar[d * C + r];
        }
        jp[d] = Ac.jprev[d * C + r] + A.jprevbar[d * C + r];
    }
    const double p = Ac.p[r] + (fl ? A.pbar[r] : 0.0);
    double ring[NR], avg[NC];
#pragma unroll
    for (int s = 0; s < NR; ++s) ring[s] = Ac.ring[s * C + r];
#pragma unroll
    for (int c = 0; c < NC; ++c) avg[c] = Ac.avg[c * C + r] + A.avgbar[c * C + r];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        O.x[d * C + dst] = x[d];
        O.u[d * C + dst] = u[d];
        O.ut[d * C + dst] = ut[d];
        O.uin[d * C + dst] = uin[d];
        O.jprev[d * C + dst] = jp[d];
    }
    O.p[dst] = p;
#pragma unroll
    for (int s = 0; s < NR; ++s) O.ring[s * C + dst] = ring[s];
#pragma unroll
    for (int c = 0; c < NC; ++c) O.avg[c * C + dst] = avg[c];
}

// ------------------------------------------------------------ inlet profile
// grad[k] = sum over rows q with index[q] = k of the adjoint of the x
// components the initial state takes from the profile value (u_in, u, ut,
// every ring slot and the mean). One block per profile entry; fixed order.
__global__ void __launch_bounds__(kBlock) k_profile_grad(Dev k, const int64_t *n, DevLam L,
                                                         const int32_t *index, double *grad)
{
    __shared__ double lds[kBlock];
    const int32_t e = blockIdx.x;
    const int64_t C = k.cap, rows = *n;
    const int NC = k.dim + 1;
    double acc = 0.0;
    for (int64_t q = threadIdx.x; q < rows; q += blockDim.x) {
        if (index[q] != e) continue;
        double v = L.uin[q] + L.u[q] + L.ut[q] + L.avg[q];
        for (int s = 0; s < kNavg; ++s) v += L.ring[int64_t(s) * NC * C + q];
        acc += v;
    }
    lds[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) lds[threadIdx.x] += lds[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) grad[e] = lds[0];
}

// ------------------------------------------------------------ launchers
#define SPH_STEP_DISPATCH(KERNEL, ...)                                                        \
    do {                                                                                      \
        const dim3 g(nblocks(k.cap)), b(kBlock);                                              \
        if (k.dim == 2 && k.prec == SPH_FP64)                                                 \
            hipLaunchKernelGGL((KERNEL<2, double>), g, b, 0, s, __VA_ARGS__);                 \
        else if (k.dim == 3 && k.prec == SPH_FP64)                                            \
            hipLaunchKernelGGL((KERNEL<3, double>), g, b, 0, s, __VA_ARGS__);                 \
        else if (k.dim == 2)                                                                  \
            hipLaunchKernelGGL((KERNEL<2, float>), g, b, 0, s, __VA_ARGS__);                  \
        else                                                                                  \
            hipLaunchKernelGGL((KERNEL<3, float>), g, b, 0, s, __VA_ARGS__);                  \
    } while (0)

void launch_adj_prep(const int64_t *n_src, int64_t *n_dst, int32_t *nspawn, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_prep, dim3(1), dim3(64), 0, s, n_src, n_dst, nspawn);
}

void launch_adj_end(const Dev &k, const DevState &m, const StepAdj &S, const DevAdj &A,
                    hipStream_t s)
{
    SPH_STEP_DISPATCH(k_adj_end, k, m, S, A);
}

void launch_adj_half(const Dev &k, const DevState &m, const StepAdj &S, const DevAdj &A,
                     hipStream_t s)
{
    SPH_STEP_DISPATCH(k_adj_half, k, m, S, A);
}

void launch_adj_finish(const Dev &k, const DevState &m, const DevState &pre,
                       const int32_t *perm, const StepAdj &S, const DevAdj &A, hipStream_t s)
{
    const dim3 g(nblocks(k.cap)), b(kBlock);
    if (k.dim == 2) hipLaunchKernelGGL(k_adj_finish<2>, g, b, 0, s, k, m, pre, perm, S, A);
    else hipLaunchKernelGGL(k_adj_finish<3>, g, b, 0, s, k, m, pre, perm, S, A);
}

void launch_profile_grad(const Dev &k, const int64_t *n, const DevLam &L, const int32_t *index,
                         int32_t ntheta, double *grad, hipStream_t s)
{
    hipLaunchKernelGGL(k_profile_grad, dim3(ntheta), dim3(kBlock), 0, s, k, n, L, index, grad);
}

}  // namespace sph
