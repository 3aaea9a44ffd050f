/*
 * sph_oracle.c -- plain FP64 CPU oracle of the EDAC-SPH wind-tunnel hot path of
 * Negi, Ramachandran & Haftu, "An improved non-reflecting outlet boundary
 * condition for weakly-compressible SPH" (arXiv 1907.04034).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg load this library. It shares no code, header or table with
 * the HIP path. It is deliberately slow and literal: particles are an array of
 * structs, every pass is a plain loop over targets with an inner loop over a
 * neighbour list rebuilt at every right-hand-side evaluation, and all
 * arithmetic is FP64, compiled with -ffp-contract=off and no fast-math.
 * OpenMP only splits the outer loop over targets (gather only), so results do
 * not depend on the thread count.
 *
 * What is computed (symbols of the paper):
 *   kernel        Wendland C2 quintic, support 2h (the workloads' kernel), or
 *                 the paper's own quintic spline of Sec. 2 eq:quintic-spline,
 *                 support 3h (flag F_QUINTIC)
 *   density       Sec. 2 eq:summation-density and the number-density volume
 *                 V_i = 1 / sum_j W_ij given below eq:tvf-momentum
 *   walls         ghost pressure / velocity by Shepard averaging of the fluid
 *                 (Sec. 2 defers to Adami et al. 2012; static walls, g = 0)
 *   outlet        Sec. 3.3 (method of characteristics): J1, J2, J3 of
 *                 eq:characteristic-vars, Shepard interpolation eq:shepard,
 *                 previous-step red average eq:average_old; Sec. 3.4 (hybrid):
 *                 time-average references eq:timeevg, acoustic-intensity gate
 *                 eq:acouinten, composition eq:acou, x-only advection
 *   other outlets selected by orc_params.outlet: pure method of
 *                 characteristics with fixed references (Sec. 3.3),
 *                 do-nothing (Sec. 3.1, eq:nrbc2), modified do-nothing
 *                 (Sec. 3.1.1, eq:shepard0) and mirroring (Sec. 3.2,
 *                 eq:matform, eq:taylor2), which can also give the inlet
 *                 pressure (flag F_MIRROR_INLET)
 *   inlet         prescribed velocity; pressure from the incoming
 *                 characteristic J3 (reference: inlet velocity, zero pressure)
 *   force pass    Sec. 2: eq:pavg, eq:tvf-p-ij-basa, eq:tvf-momentum,
 *                 eq:p-edac, background-pressure part of eq:transport-vel
 *   drag          Sec. 4.6 eq:tvf-momentum_solid over the body particles
 *   time step     explicit midpoint RK2 with eq:advection / eq:transport-vel
 *                 applied per stage
 *   bookkeeping   Sec. 3.4 last paragraph: inlet->fluid and fluid->outlet
 *                 transfer, deletion past the outlet end, inlet re-spawn
 *
 * Readings where the paper is silent or ambiguous are listed in the repository
 * design notes; each is marked "reading:" below.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define T_FLUID 0
#define T_INLET 1
#define T_OUTLET 2
#define T_WALL_SLIP 3
#define T_WALL_NOSLIP 4
#define T_BODY 5
#define T_DEAD 255

#define NAVG 6
#define F_NO_PAVG 1
#define F_DAMP_NU 2
#define F_NOISE 4
#define F_QUINTIC 16 /* the paper's quintic spline instead of Wendland C2 */
#define F_MIRROR_INLET 32 /* inlet pressure by mirroring (Sec. 3, Sec. 3.2) */
#define ID_GENERATION ((int64_t)1 << 40)

/* outlet rules */
#define OUT_HYBRID 0
#define OUT_MOC 1
#define OUT_DO_NOTHING 2
#define OUT_MOD_DO_NOTHING 3
#define OUT_MIRROR 4

typedef struct {
    int32_t dim, n_avg, flags, periodic[3];
    double h, dx, rho0, c, U, nu, alpha, eta, dt, pb;
    double lo[3], hi[3];
    double x_inlet, x_outlet, x_outlet_end, inlet_len;
    double noise_amp;
    uint64_t noise_seed;
    int32_t outlet;
} orc_params;

typedef struct {
    double x[3], u[3], ut[3], p, uin[3];
    double ring[NAVG][4];
    int32_t head;
    double avg[4];
    double jprev[3], jcur[3];
    int32_t red_prev, red;
    double rho, vol, pavg;
    double a[3], b[3], pdot;
    double abs_a[3], abs_b[3], abs_pdot; /* sums of |pair contribution| (error scale) */
    double force[3];       /* per-body-particle drag contribution */
    double x0[3], u0[3], p0; /* state at the start of the step */
    int32_t type;
    int64_t id;
} part;

typedef struct {
    orc_params q;
    int64_t n, cap;
    part *P;
    int64_t *row;           /* CSR neighbour list (self included) */
    int32_t *col;
    int64_t nnz_cap;
    double drag[3];
    int32_t nthreads_used;
} sim;

/* ------------------------------------------------------------------ kernel */

/* Wendland C2 quintic: W = a_d (1 - q/2)^4 (2q + 1), q = r/h < 2.
 * a_2 = 7 / (4 pi h^2), a_3 = 21 / (16 pi h^3). */
static double wendland_norm(int dim, double h)
{
    if (dim == 2) return 7.0 / (4.0 * M_PI * h * h);
    if (dim == 3) return 21.0 / (16.0 * M_PI * h * h * h);
    return 3.0 / (4.0 * h); /* 1D, used only by the normalisation pin */
}

double orc_w(double r, double h, int dim)
{
    double q = r / h;
    if (q >= 2.0) return 0.0;
    double t = 1.0 - 0.5 * q;
    return wendland_norm(dim, h) * t * t * t * t * (2.0 * q + 1.0);
}

/* dW/dr divided by r, so that grad_i W_ij = F * (r_i - r_j). */
double orc_gradw_factor(double r, double h, int dim)
{
    double q = r / h;
    if (q >= 2.0) return 0.0;
    double t = 1.0 - 0.5 * q;
    return -5.0 * wendland_norm(dim, h) * t * t * t / (h * h);
}

/* The paper's own quintic spline, Sec. 2 eq:quintic-spline, support 3h:
 * W = a [(3-q)^5 - 6 (2-q)^5 + 15 (1-q)^5] with each bracket dropped past its
 * range. a_2 = 7 / (478 pi h^2) as printed; reading: a_3 = 1 / (120 pi h^3),
 * the constant that normalises it in 3D (the paper gives the 2D one only). */
static double quintic_norm(int dim, double h)
{
    if (dim == 3) return 1.0 / (120.0 * M_PI * h * h * h);
    return 7.0 / (478.0 * M_PI * h * h);
}

double orc_quintic_w(double r, double h, int dim)
{
    double q = r / h;
    double t3 = 3.0 - q, t2 = 2.0 - q, t1 = 1.0 - q;
    if (q > 3.0) return 0.0;
    double w = t3 * t3 * t3 * t3 * t3;
    if (q <= 2.0) w -= 6.0 * t2 * t2 * t2 * t2 * t2;
    if (q <= 1.0) w += 15.0 * t1 * t1 * t1 * t1 * t1;
    return quintic_norm(dim, h) * w;
}

/* dW/dr divided by r for the quintic spline: a w'(q) / (h^2 q), with
 * w'(q) = -5 [(3-q)^4 - 6 (2-q)^4 + 15 (1-q)^4] (brackets dropped as in W);
 * at r = 0 its limit, -120 a / h^2 (w' vanishes there like -120 q). */
double orc_quintic_gradw_factor(double r, double h, int dim)
{
    double q = r / h;
    double t3 = 3.0 - q, t2 = 2.0 - q, t1 = 1.0 - q;
    double a = quintic_norm(dim, h);
    if (q >= 3.0) return 0.0;
    if (q == 0.0) return -120.0 * a / (h * h);
    double dw = t3 * t3 * t3 * t3;
    if (q <= 2.0) dw -= 6.0 * t2 * t2 * t2 * t2;
    if (q <= 1.0) dw += 15.0 * t1 * t1 * t1 * t1;
    return a * (-5.0 * dw) / (h * h * q);
}

/* The kernel of the run and its support radius in units of h. */
static double support_factor(const orc_params *q)
{
    return (q->flags & F_QUINTIC) ? 3.0 : 2.0;
}

static double kernel_w(const orc_params *q, double r)
{
    return (q->flags & F_QUINTIC) ? orc_quintic_w(r, q->h, q->dim) : orc_w(r, q->h, q->dim);
}

static double kernel_f(const orc_params *q, double r)
{
    return (q->flags & F_QUINTIC) ? orc_quintic_gradw_factor(r, q->h, q->dim)
                                  : orc_gradw_factor(r, q->h, q->dim);
}

/* ------------------------------------------------------- geometry helpers */

/* Minimum-image difference r_i - r_j with one +-L wrap per periodic axis. */
static void diff(const orc_params *q, const double *xi, const double *xj, double r[3])
{
    r[0] = r[1] = r[2] = 0.0;
    for (int d = 0; d < q->dim; ++d) {
        double v = xi[d] - xj[d];
        if (q->periodic[d]) {
            double L = q->hi[d] - q->lo[d];
            double half = 0.5 * L;
            if (v > half) v -= L;
            else if (v < -half) v += L;
        }
        r[d] = v;
    }
}

/* |r|^2 summed left to right; the file is built without FMA contraction. */
static double dot_self(int dim, const double r[3])
{
    double s = r[0] * r[0];
    s = s + r[1] * r[1];
    if (dim == 3) s = s + r[2] * r[2];
    return s;
}

static double dotv(int dim, const double *a, const double *b)
{
    double s = 0.0;
    for (int d = 0; d < dim; ++d) s += a[d] * b[d];
    return s;
}

static int is_wall(int t) { return t == T_WALL_SLIP || t == T_WALL_NOSLIP || t == T_BODY; }

static double support2(const orc_params *q)
{
    double s = support_factor(q) * q->h;
    return s * s;
}

static int in_range(const orc_params *q, const part *a, const part *b, double r[3], double *r2)
{
    diff(q, a->x, b->x, r);
    *r2 = dot_self(q->dim, r);
    return *r2 < support2(q);
}

/* -------------------------------------------------------- neighbour lists */

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static void ensure_nnz(sim *S, int64_t need)
{
    if (need <= S->nnz_cap) return;
    S->nnz_cap = need + need / 4 + 1024;
    S->col = (int32_t *)realloc(S->col, sizeof(int32_t) * S->nnz_cap);
}

/* O(N^2) search: j is a neighbour of i iff |r_ij|^2 < (k h)^2 with k h the
 * kernel's support (self included). */
static void neighbours_brute(sim *S)
{
    int64_t n = S->n;
    S->row = (int64_t *)realloc(S->row, sizeof(int64_t) * (n + 1));
    int64_t *cnt = (int64_t *)calloc(n + 1, sizeof(int64_t));
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double r[3], r2;
        int64_t c = 0;
        for (int64_t j = 0; j < n; ++j) c += in_range(&S->q, &S->P[i], &S->P[j], r, &r2);
        cnt[i] = c;
    }
    S->row[0] = 0;
    for (int64_t i = 0; i < n; ++i) S->row[i + 1] = S->row[i] + cnt[i];
    ensure_nnz(S, S->row[n]);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double r[3], r2;
        int64_t k = S->row[i];
        for (int64_t j = 0; j < n; ++j)
            if (in_range(&S->q, &S->P[i], &S->P[j], r, &r2)) S->col[k++] = (int32_t)j;
    }
    free(cnt);
}

/* Uniform bucket grid with cells of at least the support; each target scans the 3^d
 * surrounding buckets and keeps the same predicate as the brute-force search.
 * Rows are sorted by particle index so both searches give identical lists. */
static void neighbours_cells(sim *S)
{
    const orc_params *q = &S->q;
    int64_t n = S->n;
    int nc[3] = {1, 1, 1};
    double cs[3] = {1, 1, 1};
    for (int d = 0; d < q->dim; ++d) {
        double L = q->hi[d] - q->lo[d];
        /* cells strictly wider than the support so a 3^d stencil suffices */
        nc[d] = (int)floor(L / (support_factor(q) * q->h * (1.0 + 1e-9)));
        if (nc[d] < 1) nc[d] = 1;
        if (q->periodic[d] && nc[d] < 3) {
            fprintf(stderr, "oracle: periodic axis needs at least 3 cells\n");
            abort();
        }
        cs[d] = L / nc[d];
    }
    int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int32_t *cell = (int32_t *)malloc(sizeof(int32_t) * (n ? n : 1));
    int64_t *head = (int64_t *)calloc(ncell + 1, sizeof(int64_t));
    int64_t *items = (int64_t *)malloc(sizeof(int64_t) * (n ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        int c[3] = {0, 0, 0};
        for (int d = 0; d < q->dim; ++d) {
            int v = (int)floor((S->P[i].x[d] - q->lo[d]) / cs[d]);
            if (v < 0) v = 0;
            if (v >= nc[d]) v = nc[d] - 1;
            c[d] = v;
        }
        cell[i] = (int32_t)(((int64_t)c[2] * nc[1] + c[1]) * nc[0] + c[0]);
        head[cell[i] + 1]++;
    }
    for (int64_t k = 0; k < ncell; ++k) head[k + 1] += head[k];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (ncell ? ncell : 1));
    for (int64_t k = 0; k < ncell; ++k) fill[k] = head[k];
    for (int64_t i = 0; i < n; ++i) items[fill[cell[i]]++] = i;
    free(fill);

    int64_t *cnt = (int64_t *)calloc(n + 1, sizeof(int64_t));
    int32_t **lists = (int32_t **)calloc(n ? n : 1, sizeof(int32_t *));
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        int ci[3] = {(int)(cell[i] % nc[0]), (int)((cell[i] / nc[0]) % nc[1]),
                     (int)(cell[i] / ((int64_t)nc[0] * nc[1]))};
        int lo3[3], hi3[3];
        for (int d = 0; d < 3; ++d) {
            lo3[d] = (d < q->dim) ? -1 : 0;
            hi3[d] = (d < q->dim) ? 1 : 0;
        }
        int32_t cap = 64, k = 0;
        int32_t *lst = (int32_t *)malloc(sizeof(int32_t) * cap);
        for (int dz = lo3[2]; dz <= hi3[2]; ++dz)
            for (int dy = lo3[1]; dy <= hi3[1]; ++dy)
                for (int dx = lo3[0]; dx <= hi3[0]; ++dx) {
                    int cc[3] = {ci[0] + dx, ci[1] + dy, ci[2] + dz};
                    int ok = 1;
                    for (int d = 0; d < q->dim; ++d) {
                        if (cc[d] < 0 || cc[d] >= nc[d]) {
                            if (q->periodic[d]) cc[d] = (cc[d] + nc[d]) % nc[d];
                            else ok = 0;
                        }
                    }
                    if (!ok) continue;
                    int64_t cid = ((int64_t)cc[2] * nc[1] + cc[1]) * nc[0] + cc[0];
                    for (int64_t t = head[cid]; t < head[cid + 1]; ++t) {
                        int64_t j = items[t];
                        double r[3], r2;
                        if (in_range(q, &S->P[i], &S->P[j], r, &r2)) {
                            if (k == cap) {
                                cap *= 2;
                                lst = (int32_t *)realloc(lst, sizeof(int32_t) * cap);
                            }
                            lst[k++] = (int32_t)j;
                        }
                    }
                }
        qsort(lst, k, sizeof(int32_t), cmp_i32);
        lists[i] = lst;
        cnt[i] = k;
    }
    S->row = (int64_t *)realloc(S->row, sizeof(int64_t) * (n + 1));
    S->row[0] = 0;
    for (int64_t i = 0; i < n; ++i) S->row[i + 1] = S->row[i] + cnt[i];
    ensure_nnz(S, S->row[n]);
    for (int64_t i = 0; i < n; ++i) {
        memcpy(S->col + S->row[i], lists[i], sizeof(int32_t) * cnt[i]);
        free(lists[i]);
    }
    free(lists);
    free(cnt);
    free(cell);
    free(head);
    free(items);
}

/* ---------------------------------------------------------------- density */

static double particle_mass(const orc_params *q)
{
    /* reading: every particle carries m = rho0 dx^d */
    return q->dim == 3 ? q->rho0 * q->dx * q->dx * q->dx : q->rho0 * q->dx * q->dx;
}

/* Sec. 2 eq:summation-density, rho_i = sum_j m_j W_ij, and the number-density
 * volume V_i = 1 / sum_j W_ij, for every particle of every kind (self included). */
static void density(sim *S)
{
    const orc_params *q = &S->q;
    double m = particle_mass(q);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < S->n; ++i) {
        part *pi = &S->P[i];
        double sw = 0.0;
        for (int64_t k = S->row[i]; k < S->row[i + 1]; ++k) {
            part *pj = &S->P[S->col[k]];
            double r[3];
            diff(q, pi->x, pj->x, r);
            sw += kernel_w(q, sqrt(dot_self(q->dim, r)));
        }
        pi->rho = m * sw;
        pi->vol = 1.0 / sw;
    }
}

/* ------------------------------------------------------- boundary values */

/* Sec. 3.3 eq:characteristic-vars at a fluid particle, with the hybrid
 * references of Sec. 3.4: u_ref, p_ref are the particle's own time averages
 * and rho_ref = rho0.  Only the x (outlet-normal) velocity enters.
 * reading: the pure method of characteristics takes the fixed references
 * u_ref = U (the inlet speed), p_ref = 0, rho_ref = rho0. */
static void fluid_J(const orc_params *q, const part *f, double J[3])
{
    int moc = q->outlet == OUT_MOC;
    double dp = f->p - (moc ? 0.0 : f->avg[3]);
    double du = f->u[0] - (moc ? q->U : f->avg[0]);
    J[0] = -q->c * q->c * (f->rho - q->rho0) + dp;
    J[1] = f->rho * q->c * du + dp;
    J[2] = -f->rho * q->c * du + dp;
}

/* Blue-particle fallback, Sec. 3.3 eq:average_old: mean of the previous-step
 * values of the same-kind neighbours that had fluid support at that step.
 * reading: with no such neighbour the particle keeps its own previous value. */
static void fallback_J(const sim *S, int64_t i, double J[3])
{
    const part *pi = &S->P[i];
    double s[3] = {0, 0, 0};
    int64_t M = 0;
    for (int64_t k = S->row[i]; k < S->row[i + 1]; ++k) {
        const part *pj = &S->P[S->col[k]];
        if (pj->type == pi->type && pj->red_prev) {
            for (int a = 0; a < 3; ++a) s[a] += pj->jprev[a];
            ++M;
        }
    }
    for (int a = 0; a < 3; ++a) J[a] = M ? s[a] / (double)M : pi->jprev[a];
}

/* Sec. 3.2, eq:matform: first-order corrected SPH estimate of a field and
 * its gradient at the point xk from the fluid particles l within the
 * kernel support of xk: sum_l [W, x_lk W, ...; W_x, x_lk W_x, ...; ...] V_l
 * times (f_k, grad f_k) equals sum_l f_l [W, W_x, ...] V_l, with
 * x_lk = x_l - x_k, W_b = dW/dx_b at x_l - x_k and V_l = 1 / sum_j W_lj,
 * for the fields p, u_x, u_y (, u_z). Solved by Gaussian elimination with
 * partial pivoting on the dimensionless system (x_lk / h in the columns, the
 * derivative rows times h, so that every entry is of order one). reading:
 * where a pivot falls below 1e-3 of the largest entry (sources nearly on a
 * line, as for a point about one spacing beyond the last fluid column with
 * a 2h support) the zeroth-order Shepard value with zero gradient is taken.
 * Returns 0 when no fluid particle lies within the support of xk. sol[f][0]
 * is the value of field f, sol[f][1 + b] its derivative along b. */
static int mirror_fit(const sim *S, const double xk[3], double sol[4][4])
{
    const orc_params *q = &S->q;
    const int dim = q->dim, ne = dim + 1;
    double A[4][4] = {{0}}, B[4][4] = {{0}}; /* B[row][field] */
    for (int64_t l = 0; l < S->n; ++l) {
        const part *pl = &S->P[l];
        if (pl->type != T_FLUID) continue;
        double r[3];
        diff(q, pl->x, xk, r); /* x_l - x_k */
        double r2 = dot_self(dim, r);
        if (!(r2 < support2(q))) continue;
        double w = kernel_w(q, sqrt(r2)), F = kernel_f(q, sqrt(r2));
        double rowm[4] = {w * pl->vol, 0, 0, 0}, col[4] = {1.0, 0, 0, 0};
        double fl[4] = {pl->p, 0, 0, 0};
        for (int b = 0; b < dim; ++b) {
            rowm[1 + b] = q->h * F * r[b] * pl->vol;
            col[1 + b] = r[b] / q->h;
            fl[1 + b] = pl->u[b];
        }
        for (int a = 0; a < ne; ++a) {
            for (int c = 0; c < ne; ++c) A[a][c] += rowm[a] * col[c];
            for (int f = 0; f < ne; ++f) B[a][f] += rowm[a] * fl[f];
        }
    }
    if (!(A[0][0] > 0.0)) return 0;
    double shep[4];
    for (int f = 0; f < ne; ++f) shep[f] = B[0][f] / A[0][0];
    double amax = 0.0;
    for (int a = 0; a < ne; ++a)
        for (int c = 0; c < ne; ++c) amax = fmax(amax, fabs(A[a][c]));
    int singular = 0;
    for (int c = 0; c < ne && !singular; ++c) {
        int pr = c;
        for (int a = c + 1; a < ne; ++a)
            if (fabs(A[a][c]) > fabs(A[pr][c])) pr = a;
        if (!(fabs(A[pr][c]) > 1e-3 * amax)) {
            singular = 1;
            break;
        }
        if (pr != c) {
            for (int x = 0; x < ne; ++x) {
                double t = A[c][x]; A[c][x] = A[pr][x]; A[pr][x] = t;
                t = B[c][x]; B[c][x] = B[pr][x]; B[pr][x] = t;
            }
        }
        for (int a = c + 1; a < ne; ++a) {
            double m = A[a][c] / A[c][c];
            for (int x = c; x < ne; ++x) A[a][x] -= m * A[c][x];
            for (int f = 0; f < ne; ++f) B[a][f] -= m * B[c][f];
        }
    }
    for (int f = 0; f < ne; ++f) {
        if (singular) {
            sol[f][0] = shep[f];
            for (int b = 0; b < dim; ++b) sol[f][1 + b] = 0.0;
            continue;
        }
        double x[4] = {0, 0, 0, 0};
        for (int a = ne - 1; a >= 0; --a) {
            double v = B[a][f];
            for (int c = a + 1; c < ne; ++c) v -= A[a][c] * x[c];
            x[a] = v / A[a][a];
        }
        sol[f][0] = x[0];
        for (int b = 0; b < dim; ++b) sol[f][1 + b] = x[1 + b] / q->h;
    }
    return 1;
}

/* Sec. 3.2: boundary particle i mirrored about the interface x = xif into the
 * fluid (x_k = 2 xif - x_i, other coordinates kept); its fields are those of
 * the mirror point extrapolated with the paper's sign-flipped expansion
 * eq:taylor2, f_i = f_k - (r_i - r_k) . grad f_k. out[0] = p, out[1 + b] =
 * u_b. Returns 0 (out untouched) without fluid at the mirror point. */
static int mirror_value(const sim *S, int64_t i, double xif, double out[4])
{
    const part *pi = &S->P[i];
    const int dim = S->q.dim;
    double xk[3] = {pi->x[0], pi->x[1], pi->x[2]};
    xk[0] = 2.0 * xif - pi->x[0];
    double sol[4][4];
    if (!mirror_fit(S, xk, sol)) return 0;
    for (int f = 0; f <= dim; ++f) {
        double v = sol[f][0];
        for (int b = 0; b < dim; ++b) v -= (pi->x[b] - xk[b]) * sol[f][1 + b];
        out[f] = v;
    }
    return 1;
}

static void boundary_values(sim *S)
{
    const orc_params *q = &S->q;
    const int dim = q->dim;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < S->n; ++i) {
        part *pi = &S->P[i];
        int t = pi->type;
        if (t == T_FLUID) continue;
        /* Shepard sums over fluid neighbours (Sec. 3.3 eq:shepard) */
        double sw = 0.0, sp = 0.0, su[3] = {0, 0, 0}, sJ[3] = {0, 0, 0};
        for (int64_t k = S->row[i]; k < S->row[i + 1]; ++k) {
            const part *f = &S->P[S->col[k]];
            if (f->type != T_FLUID) continue;
            double r[3];
            diff(q, pi->x, f->x, r);
            double w = kernel_w(q, sqrt(dot_self(dim, r)));
            sw += w;
            sp += f->p * w;
            for (int d = 0; d < dim; ++d) su[d] += f->u[d] * w;
            double J[3];
            if (t == T_INLET && (q->flags & F_MIRROR_INLET)) {
                J[0] = J[1] = J[2] = 0.0; /* the pressure comes from the mirror */
            } else if (t == T_INLET) {
                /* reading: incoming characteristic J3 with reference
                 * (u, p) = (prescribed inlet velocity of i, 0) */
                J[0] = 0.0;
                J[1] = 0.0;
                J[2] = -f->rho * q->c * (f->u[0] - pi->uin[0]) + f->p;
            } else if (q->outlet == OUT_MOD_DO_NOTHING) {
                /* Sec. 3.1.1 eq:shepard0: the fluid x velocity, carried in
                 * the first slot */
                J[0] = f->u[0];
                J[1] = 0.0;
                J[2] = 0.0;
            } else if (q->outlet == OUT_DO_NOTHING || q->outlet == OUT_MIRROR) {
                J[0] = J[1] = J[2] = 0.0; /* no characteristic values */
            } else {
                fluid_J(q, f, J);
            }
            for (int a = 0; a < 3; ++a) sJ[a] += J[a] * w;
        }
        if (is_wall(t)) {
            /* ghost values from the fluid (static wall, no body force):
             * p_w = sum p_f W / sum W,  u_g = 2 u_w - sum u_f W / sum W, u_w = 0 */
            if (sw > 0.0) {
                pi->p = sp / sw;
                for (int d = 0; d < dim; ++d) pi->u[d] = -(su[d] / sw);
            } else {
                pi->p = 0.0;
                for (int d = 0; d < dim; ++d) pi->u[d] = 0.0;
            }
            continue;
        }
        double Jh[3];
        if (sw > 0.0) {
            pi->red = 1;
            for (int a = 0; a < 3; ++a) Jh[a] = sJ[a] / sw;
            if (t == T_OUTLET) Jh[2] = 0.0; /* outflow: J3 = 0, Sec. 3.3 */
        } else {
            pi->red = 0;
            fallback_J(S, i, Jh);
        }
        for (int a = 0; a < 3; ++a) pi->jcur[a] = Jh[a];
        if (t == T_OUTLET && q->outlet == OUT_HYBRID) {
            /* invert eq:characteristic-vars with rho_ref = rho0, then compose
             * with the frozen time averages, Sec. 3.4 eq:acou */
            double p_ac = 0.5 * (Jh[1] + Jh[2]);
            double u_ac = (Jh[1] - Jh[2]) / (2.0 * q->rho0 * q->c);
            pi->p = pi->avg[3] + p_ac;
            pi->u[0] = pi->avg[0] + u_ac;
            for (int d = 1; d < dim; ++d) pi->u[d] = pi->avg[d];
        } else if (t == T_OUTLET && q->outlet == OUT_MOC) {
            /* Sec. 3.3: invert eq:characteristic-vars about the fixed
             * references; the transverse velocity passes unchanged */
            double p_ac = 0.5 * (Jh[1] + Jh[2]);
            double u_ac = (Jh[1] - Jh[2]) / (2.0 * q->rho0 * q->c);
            pi->p = 0.0 + p_ac;
            pi->u[0] = q->U + u_ac;
        } else if (t == T_OUTLET && q->outlet == OUT_MIRROR) {
            /* Sec. 3.2: p and every velocity component from the mirror
             * point, extrapolated with eq:taylor2; no fluid there: kept */
            double f[4];
            if (mirror_value(S, i, q->x_outlet, f)) {
                pi->p = f[0];
                for (int d = 0; d < dim; ++d) pi->u[d] = f[1 + d];
            }
        } else if (t == T_OUTLET) {
            /* Sec. 3.1 and 3.1.1: velocity and pressure stay frozen */
        } else if (t == T_INLET) {
            if (q->flags & F_MIRROR_INLET) {
                /* Sec. 3: the inlet pressure mirrored from the fluid */
                double f[4];
                if (mirror_value(S, i, q->x_inlet, f)) pi->p = f[0];
            } else {
                /* prescribed velocity: u - u_ref = 0, so p = J3 */
                pi->p = Jh[2];
            }
            for (int d = 0; d < dim; ++d) pi->u[d] = pi->uin[d];
        }
        for (int d = 0; d < dim; ++d) pi->ut[d] = pi->u[d];
    }
}

/* ------------------------------------------------------------- force pass */

/* One (i, j) pair of Sec. 2: eq:tvf-p-ij-basa, eq:tvf-momentum, eq:p-edac and
 * the background-pressure sum of eq:transport-vel.  Adds into acc, bacc, pdot.
 * reading: A = rho u (ut - u) for fluid and 0 for every other kind, and
 * (A . gradW)_a = sum_b A_ab dW/dx_b; slip walls take no viscous part; walls
 * enter the divergence term with their (zero) wall velocity and the viscous
 * term with their ghost velocity; eta_i = rho_i nu. */
static void pair_terms(const orc_params *q, const part *pi, const part *pj,
                       double pavg_i, double acc[3], double bacc[3], double *pdot,
                       double abs_acc[3], double abs_bacc[3], double *abs_pdot)
{
    const int dim = q->dim;
    const double m = particle_mass(q);
    double r[3];
    diff(q, pi->x, pj->x, r);
    double r2 = dot_self(dim, r);
    double F = kernel_f(q, sqrt(r2));
    double gw[3] = {F * r[0], F * r[1], F * r[2]};
    double vsq = pi->vol * pi->vol + pj->vol * pj->vol;
    double ri = pi->rho, rj = pj->rho;
    double ptil = (rj * (pi->p - pavg_i) + ri * (pj->p - pavg_i)) / (ri + rj);
    double nu_edac = q->alpha * q->h * q->c / 8.0; /* Sec. 2 eq:edac-nu */
    double nu_damp = (q->flags & F_DAMP_NU) ? q->nu : nu_edac;
    /* eta~_ij = 2 eta_i eta_j / (eta_i + eta_j) with eta = rho nu and one
     * viscosity for all particles, i.e. 2 rho_i rho_j nu / (rho_i + rho_j) */
    double eta_ij = 2.0 * ri * rj * q->nu / (ri + rj);
    double eta_edac = 2.0 * ri * rj * nu_damp / (ri + rj);
    /* grad W . r / (r^2 + eta h^2) */
    double dfac = dotv(dim, gw, r) / (r2 + q->eta * q->h * q->h);

    /* A_i . gradW and A_j . gradW */
    double Ai[3] = {0, 0, 0}, Aj[3] = {0, 0, 0};
    if (pi->type == T_FLUID) {
        double s = 0.0;
        for (int d = 0; d < dim; ++d) s += (pi->ut[d] - pi->u[d]) * gw[d];
        for (int d = 0; d < dim; ++d) Ai[d] = pi->rho * pi->u[d] * s;
    }
    if (pj->type == T_FLUID) {
        double s = 0.0;
        for (int d = 0; d < dim; ++d) s += (pj->ut[d] - pj->u[d]) * gw[d];
        for (int d = 0; d < dim; ++d) Aj[d] = pj->rho * pj->u[d] * s;
    }
    int visc = pj->type != T_WALL_SLIP;
    for (int d = 0; d < dim; ++d) {
        double uij = pi->u[d] - pj->u[d];
        double term = -ptil * gw[d] + 0.5 * (Ai[d] + Aj[d]);
        if (visc) term += eta_ij * dfac * uij;
        acc[d] += vsq / m * term;
        bacc[d] += -q->pb / m * vsq * gw[d];
        abs_acc[d] += fabs(vsq / m * term);
        abs_bacc[d] += fabs(q->pb / m * vsq * gw[d]);
    }
    /* divergence part: walls move with their wall velocity, which is zero */
    double udiv = 0.0;
    for (int d = 0; d < dim; ++d) {
        double uj = is_wall(pj->type) ? 0.0 : pj->u[d];
        udiv += (pi->u[d] - uj) * gw[d];
    }
    double dp = m * ri / rj * q->c * q->c * udiv + vsq / m * eta_edac * dfac * (pi->p - pj->p);
    *pdot += dp;
    *abs_pdot += fabs(dp);
}

/* Sec. 2 eq:pavg: mean pressure over all neighbours (fluid and boundary),
 * self included. */
static double neighbour_pavg(const sim *S, int64_t i)
{
    if (S->q.flags & F_NO_PAVG) return 0.0;
    double s = 0.0;
    int64_t Ni = S->row[i + 1] - S->row[i];
    for (int64_t k = S->row[i]; k < S->row[i + 1]; ++k) s += S->P[S->col[k]].p;
    return s / (double)Ni;
}

static void forces(sim *S)
{
    const orc_params *q = &S->q;
    const int dim = q->dim;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < S->n; ++i) {
        part *pi = &S->P[i];
        for (int d = 0; d < 3; ++d)
            pi->a[d] = pi->b[d] = pi->force[d] = pi->abs_a[d] = pi->abs_b[d] = 0.0;
        pi->pdot = pi->abs_pdot = 0.0;
        pi->pavg = 0.0;
        if (pi->type != T_FLUID && pi->type != T_BODY) continue;
        /* reading: the body force of eq:tvf-momentum_solid takes p~ with a
         * zero average; subtracting the body particle's own neighbour mean
         * would cancel the pressure it integrates (and the paper's printed
         * drag coefficients include that pressure) */
        double pavg = pi->type == T_FLUID ? neighbour_pavg(S, i) : 0.0;
        pi->pavg = pavg;
        for (int64_t k = S->row[i]; k < S->row[i + 1]; ++k) {
            int64_t j = S->col[k];
            if (j == i) continue;
            const part *pj = &S->P[j];
            if (pi->type == T_FLUID) {
                pair_terms(q, pi, pj, pavg, pi->a, pi->b, &pi->pdot, pi->abs_a, pi->abs_b,
                           &pi->abs_pdot);
            } else if (pj->type == T_FLUID) {
                /* Sec. 4.6 eq:tvf-momentum_solid: force on the body from
                 * fluid j, with u_ij = u_g,i - u_j */
                double r[3];
                diff(q, pi->x, pj->x, r);
                double r2 = dot_self(dim, r);
                double F = kernel_f(q, sqrt(r2));
                double vsq = pi->vol * pi->vol + pj->vol * pj->vol;
                double ri = pi->rho, rj = pj->rho;
                double ptil = (rj * (pi->p - pavg) + ri * (pj->p - pavg)) / (ri + rj);
                double eta_ij = 2.0 * ri * rj * q->nu / (ri + rj);
                double gw[3] = {F * r[0], F * r[1], F * r[2]};
                double dfac = dotv(dim, gw, r) / (r2 + q->eta * q->h * q->h);
                for (int d = 0; d < dim; ++d)
                    pi->force[d] += vsq * (-ptil * gw[d] + eta_ij * dfac * (pi->u[d] - pj->u[d]));
            }
        }
    }
    double F[3] = {0, 0, 0};
    for (int64_t i = 0; i < S->n; ++i)
        if (S->P[i].type == T_BODY)
            for (int d = 0; d < 3; ++d) F[d] += S->P[i].force[d];
    for (int d = 0; d < 3; ++d) S->drag[d] = F[d];
}

/* one right-hand-side evaluation at the current positions */
static void rhs(sim *S, int brute)
{
    if (brute) neighbours_brute(S);
    else neighbours_cells(S);
    density(S);
    boundary_values(S);
    forces(S);
}

/* ------------------------------------------------------------- time step */

static void wrap(const orc_params *q, double *x)
{
    for (int d = 0; d < q->dim; ++d) {
        if (!q->periodic[d]) continue;
        double L = q->hi[d] - q->lo[d];
        if (x[d] >= q->hi[d]) x[d] -= L;
        else if (x[d] < q->lo[d]) x[d] += L;
    }
}

/* SplitMix64 (Steele, Lea & Flood 2014) as a counter-based generator:
 * the k-th uniform of particle `id` is mix(seed + (3 id + k + 1) * gamma). */
static double splitmix_uniform(uint64_t seed, int64_t id, int k)
{
    uint64_t z = seed + ((uint64_t)(3 * id + k + 1)) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

/* reading: the prescribed inlet velocity of a particle with seeded noise is
 * U e_x + amp*sqrt(3)*(2 xi - 1) per component (uniform, standard deviation
 * amp*U). */
static void inlet_velocity(const orc_params *q, int64_t id, const double *parent, double *out)
{
    if (!(q->flags & F_NOISE)) {
        for (int d = 0; d < 3; ++d) out[d] = parent[d];
        return;
    }
    for (int d = 0; d < 3; ++d) {
        double base = d == 0 ? q->U : 0.0;
        double xi = splitmix_uniform(q->noise_seed, id, d);
        out[d] = d < q->dim ? base + q->noise_amp * q->U * sqrt(3.0) * (2.0 * xi - 1.0) : 0.0;
    }
}

static void ring_push(part *pi, const double v[4])
{
    for (int a = 0; a < 4; ++a) pi->ring[pi->head][a] = v[a];
    pi->head = (pi->head + 1) % NAVG;
    /* Sec. 3.4 eq:timeevg over the N = 6 most recent accepted steps */
    for (int a = 0; a < 4; ++a) {
        double s = 0.0;
        for (int k = 0; k < NAVG; ++k) s += pi->ring[k][a];
        pi->avg[a] = s / (double)NAVG;
    }
}

static void push_particle(sim *S, const part *src)
{
    if (S->n == S->cap) {
        S->cap = S->cap * 2 + 16;
        S->P = (part *)realloc(S->P, sizeof(part) * S->cap);
    }
    S->P[S->n++] = *src;
}

/* Sec. 3.4, last two paragraphs, with the gate of eq:acouinten. */
static void end_of_step(sim *S)
{
    const orc_params *q = &S->q;
    const int dim = q->dim;
    int64_t n = S->n;
    /* (a) characteristic values of this step become the previous-step values */
    for (int64_t i = 0; i < n; ++i) {
        part *pi = &S->P[i];
        if (pi->type == T_OUTLET || pi->type == T_INLET) {
            for (int a = 0; a < 3; ++a) pi->jprev[a] = pi->jcur[a];
            pi->red_prev = pi->red;
        }
    }
    /* (b) time averages, frozen while p^2/(2 rho c) exceeds
     * I = (rho u_in^2 / 2)^2 / (2 rho c), i.e. |p| > rho0 U^2 / 2 */
    double pgate = 0.5 * q->rho0 * q->U * q->U;
    for (int64_t i = 0; i < n; ++i) {
        part *pi = &S->P[i];
        if (pi->type != T_FLUID && pi->type != T_INLET) continue;
        if (fabs(pi->p) > pgate) continue;
        double v[4] = {pi->u[0], dim > 1 ? pi->u[1] : 0.0, dim > 2 ? pi->u[2] : 0.0, pi->p};
        ring_push(pi, v);
    }
    /* (c) transfers */
    for (int64_t i = 0; i < n; ++i) {
        part *pi = &S->P[i];
        if (pi->type == T_FLUID && pi->x[0] > q->x_outlet) {
            pi->type = T_OUTLET;
            for (int a = 0; a < 3; ++a) pi->jprev[a] = 0.0;
            pi->red_prev = 0;
        } else if (pi->type == T_OUTLET && pi->x[0] > q->x_outlet_end) {
            pi->type = T_DEAD;
        } else if (pi->type == T_INLET && pi->x[0] >= q->x_inlet) {
            part child = *pi;
            pi->type = T_FLUID;
            child.id = pi->id + ID_GENERATION;
            child.x[0] = pi->x[0] - q->inlet_len;
            inlet_velocity(q, child.id, pi->uin, child.uin);
            for (int d = 0; d < 3; ++d) child.u[d] = child.ut[d] = child.uin[d];
            double v[4] = {child.uin[0], child.uin[1], child.uin[2], pi->p};
            for (int k = 0; k < NAVG; ++k)
                for (int a = 0; a < 4; ++a) child.ring[k][a] = v[a];
            for (int a = 0; a < 4; ++a) child.avg[a] = v[a];
            child.head = 0;
            for (int a = 0; a < 3; ++a) child.jprev[a] = child.jcur[a] = 0.0;
            child.red_prev = child.red = 0;
            push_particle(S, &child);
            pi = &S->P[i]; /* the array may have moved */
        }
    }
    /* (d) delete particles that left the outlet, keeping the order */
    int64_t w = 0;
    for (int64_t i = 0; i < S->n; ++i)
        if (S->P[i].type != T_DEAD) S->P[w++] = S->P[i];
    S->n = w;
}

/* Speed along x of an outlet particle at this stage: its own x velocity
 * (hybrid eq:acou, characteristics, do-nothing eq:nrbc2) or, for the modified
 * do-nothing rule, the extrapolated fluid velocity of Sec. 3.1.1. */
static double outlet_speed(const orc_params *q, const part *pi)
{
    return q->outlet == OUT_MOD_DO_NOTHING ? pi->jcur[0] : pi->u[0];
}

/* Explicit midpoint RK2 (reading of the integrator, which the paper defers to
 * the EDAC paper): stage 1 at t^n, half state, stage 2 at t^{n+1/2}. The
 * transport velocity of eq:transport-vel is formed with the stage's sub-step
 * and positions follow eq:advection.  Inlet particles move with their
 * prescribed velocity, outlet particles along x with the speed of their
 * outlet rule (outlet_speed), walls stay fixed. */
static void step(sim *S, int brute, double *drag_out)
{
    const orc_params *q = &S->q;
    const int dim = q->dim;
    const double dt = q->dt, hdt = 0.5 * q->dt;
    for (int64_t i = 0; i < S->n; ++i) {
        part *pi = &S->P[i];
        for (int d = 0; d < 3; ++d) { pi->x0[d] = pi->x[d]; pi->u0[d] = pi->u[d]; }
        pi->p0 = pi->p;
    }
    rhs(S, brute);
    if (drag_out) for (int d = 0; d < 3; ++d) drag_out[d] = S->drag[d];
    for (int64_t i = 0; i < S->n; ++i) {
        part *pi = &S->P[i];
        if (pi->type == T_FLUID) {
            for (int d = 0; d < dim; ++d) {
                pi->u[d] = pi->u0[d] + hdt * pi->a[d];
                pi->ut[d] = pi->u[d] + hdt * pi->b[d];
                pi->x[d] = pi->x0[d] + hdt * pi->ut[d];
            }
            pi->p = pi->p0 + hdt * pi->pdot;
            wrap(q, pi->x);
        } else if (pi->type == T_INLET) {
            pi->x[0] = pi->x0[0] + hdt * pi->uin[0];
        } else if (pi->type == T_OUTLET) {
            pi->x[0] = pi->x0[0] + hdt * outlet_speed(q, pi);
        }
    }
    rhs(S, brute);
    for (int64_t i = 0; i < S->n; ++i) {
        part *pi = &S->P[i];
        if (pi->type == T_FLUID) {
            for (int d = 0; d < dim; ++d) {
                pi->x[d] = pi->x0[d] + dt * pi->ut[d];
                pi->u[d] = pi->u0[d] + dt * pi->a[d];
                pi->ut[d] = pi->u[d] + dt * pi->b[d];
            }
            pi->p = pi->p0 + dt * pi->pdot;
            wrap(q, pi->x);
        } else if (pi->type == T_INLET) {
            pi->x[0] = pi->x0[0] + dt * pi->uin[0];
        } else if (pi->type == T_OUTLET) {
            pi->x[0] = pi->x0[0] + dt * outlet_speed(q, pi);
        }
    }
    end_of_step(S);
}

/* ------------------------------------------------------------- C interface */

void *orc_create(const orc_params *q, int64_t n, const double *x, const double *u,
                 const double *ut, const double *p, const double *uin, const double *ring,
                 const int32_t *head, const double *avg, const double *jprev,
                 const uint8_t *red_prev, const uint8_t *type, const int64_t *id)
{
    sim *S = (sim *)calloc(1, sizeof(sim));
    S->q = *q;
    S->n = n;
    S->cap = n + 16;
    S->P = (part *)calloc(S->cap, sizeof(part));
    for (int64_t i = 0; i < n; ++i) {
        part *pi = &S->P[i];
        for (int d = 0; d < 3; ++d) {
            pi->x[d] = x[3 * i + d];
            pi->u[d] = u[3 * i + d];
            pi->ut[d] = ut[3 * i + d];
            pi->uin[d] = uin[3 * i + d];
            pi->jprev[d] = jprev[3 * i + d];
        }
        pi->p = p[i];
        for (int k = 0; k < NAVG; ++k)
            for (int a = 0; a < 4; ++a) pi->ring[k][a] = ring[(i * NAVG + k) * 4 + a];
        pi->head = head[i];
        for (int a = 0; a < 4; ++a) pi->avg[a] = avg[4 * i + a];
        pi->red_prev = red_prev[i];
        pi->type = type[i];
        pi->id = id[i];
    }
    return S;
}

void orc_destroy(void *h)
{
    sim *S = (sim *)h;
    if (!S) return;
    free(S->P);
    free(S->row);
    free(S->col);
    free(S);
}

int64_t orc_count(void *h) { return ((sim *)h)->n; }

void orc_get(void *h, double *x, double *u, double *ut, double *p, double *uin, double *ring,
             int32_t *head, double *avg, double *jprev, uint8_t *red_prev, uint8_t *type,
             int64_t *id)
{
    sim *S = (sim *)h;
    for (int64_t i = 0; i < S->n; ++i) {
        part *pi = &S->P[i];
        for (int d = 0; d < 3; ++d) {
            x[3 * i + d] = pi->x[d];
            u[3 * i + d] = pi->u[d];
            ut[3 * i + d] = pi->ut[d];
            uin[3 * i + d] = pi->uin[d];
            jprev[3 * i + d] = pi->jprev[d];
        }
        p[i] = pi->p;
        for (int k = 0; k < NAVG; ++k)
            for (int a = 0; a < 4; ++a) ring[(i * NAVG + k) * 4 + a] = pi->ring[k][a];
        head[i] = pi->head;
        for (int a = 0; a < 4; ++a) avg[4 * i + a] = pi->avg[a];
        red_prev[i] = (uint8_t)pi->red_prev;
        type[i] = (uint8_t)pi->type;
        id[i] = pi->id;
    }
}

/* Prescribed inlet velocities for the following steps, one row of 3 per
 * particle in the order of orc_get (a boundary condition that changes in time
 * is set between steps). */
void orc_set_uin(void *h, const double *uin)
{
    sim *S = (sim *)h;
    for (int64_t i = 0; i < S->n; ++i)
        for (int d = 0; d < 3; ++d) S->P[i].uin[d] = uin[3 * i + d];
}

/* Derived fields of the last right-hand-side evaluation. */
void orc_get_derived(void *h, double *rho, double *vol, double *pavg, double *a, double *b,
                     double *pdot, double *jcur, uint8_t *red, double *force)
{
    sim *S = (sim *)h;
    for (int64_t i = 0; i < S->n; ++i) {
        part *pi = &S->P[i];
        rho[i] = pi->rho;
        vol[i] = pi->vol;
        pavg[i] = pi->pavg;
        pdot[i] = pi->pdot;
        red[i] = (uint8_t)pi->red;
        for (int d = 0; d < 3; ++d) {
            a[3 * i + d] = pi->a[d];
            b[3 * i + d] = pi->b[d];
            jcur[3 * i + d] = pi->jcur[d];
            force[3 * i + d] = pi->force[d];
        }
    }
}

/* Sums over j of |pair contribution| to a, b, pdot of the last evaluation:
 * the scale against which rounding in those sums is judged. */
void orc_get_abs(void *h, double *abs_a, double *abs_b, double *abs_pdot)
{
    sim *S = (sim *)h;
    for (int64_t i = 0; i < S->n; ++i) {
        part *pi = &S->P[i];
        abs_pdot[i] = pi->abs_pdot;
        for (int d = 0; d < 3; ++d) {
            abs_a[3 * i + d] = pi->abs_a[d];
            abs_b[3 * i + d] = pi->abs_b[d];
        }
    }
}

/* One right-hand-side evaluation at the current state; drag -> F[3]. */
int orc_rhs(void *h, int brute, double *F)
{
    sim *S = (sim *)h;
    rhs(S, brute);
    if (F) for (int d = 0; d < 3; ++d) F[d] = S->drag[d];
    return 0;
}

/* nsteps RK2 steps; drag at stage 1 of each step -> drag[3*nsteps] (optional). */
int orc_step(void *h, int32_t nsteps, int brute, double *drag)
{
    sim *S = (sim *)h;
    for (int32_t s = 0; s < nsteps; ++s) step(S, brute, drag ? drag + 3 * s : NULL);
    return 0;
}

/* Neighbour lists at the current positions (rows sorted by index). Returns nnz;
 * row_ptr/col are written only if col_cap >= nnz. */
int64_t orc_neighbors(void *h, int brute, int64_t *row_ptr, int32_t *col, int64_t col_cap)
{
    sim *S = (sim *)h;
    if (brute) neighbours_brute(S);
    else neighbours_cells(S);
    int64_t nnz = S->row[S->n];
    if (row_ptr && col && col_cap >= nnz) {
        memcpy(row_ptr, S->row, sizeof(int64_t) * (S->n + 1));
        memcpy(col, S->col, sizeof(int32_t) * nnz);
    }
    return nnz;
}

/* Test access to the seeded inlet noise: the k-th uniform of particle `id`
 * (splitmix_uniform) and the prescribed velocity a re-spawned inlet particle
 * with this id receives (inlet_velocity, parent velocity `parent`). */
double orc_splitmix_uniform(uint64_t seed, int64_t id, int k)
{
    return splitmix_uniform(seed, id, k);
}

void orc_inlet_velocity(const orc_params *q, int64_t id, const double *parent, double *out)
{
    inlet_velocity(q, id, parent, out);
}

/* Threads of the OpenMP loops of later calls (benchmark timing of the oracle
 * on one and on all host cores); results do not depend on it. */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
