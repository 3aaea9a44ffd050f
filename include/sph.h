/*
 * sph.h -- C ABI of the MI355X (gfx950) EDAC-SPH wind-tunnel hot path.
 *
 * Method: Negi, Ramachandran & Haftu, "An improved non-reflecting outlet
 * boundary condition for weakly-compressible SPH" (arXiv 1907.04034).
 * Sec. 2 gives the EDAC-TVF scheme (summation density, number-density
 * momentum equation with the neighbour-average pressure, EDAC pressure rate,
 * transport velocity); Sec. 3.3 the characteristic variables and their
 * Shepard extrapolation with the red/blue fallback; Sec. 3.4 the hybrid
 * outlet (time-averaged references, acoustic-intensity gate, composition
 * f_o = f_ac + f_avg, x-only advection, particle transfer); Sec. 4.6 the
 * force on a solid body.
 *
 * Conventions for every entry point:
 *  - All array pointers in sph_state, sph_nlist and sph_derived are DEVICE
 *    pointers owned by the caller; the library never allocates or frees them.
 *    Per-particle arrays are component-major: component k of particle i is
 *    at [k * cap + i]. The workspace is caller-owned device memory of at
 *    least sph_workspace_size() bytes, zero-filled before first use.
 *  - `stream` is a hipStream_t (0 = the null stream). Every call only
 *    enqueues work on it and returns; nothing synchronises except
 *    sph_poll_error() and sph_live_count().
 *  - Argument errors are detected on the host before any launch and return a
 *    negative sph_status; sph_last_error() then gives a message. Conditions
 *    found on the device (capacity, non-finite values, skin violation) set
 *    bits of the device error word, read with sph_poll_error().
 *  - The first *st->n rows of every state array are the live particles. After
 *    sph_bin / sph_step they are sorted by Morton cell key, ties by id.
 */
#ifndef SPH_H
#define SPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPH_OK = 0,
    SPH_EINVAL = -1,       /* bad argument, detected on the host */
    SPH_ECAPACITY = -2,    /* a size exceeds a capacity, detected on the host */
    SPH_ENONFINITE = -3,   /* a parameter is NaN or infinite (values that become
                              non-finite on the device set SPH_ERR_NONFINITE) */
    SPH_ECFL = -4,         /* dt above the acoustic bound 0.5 h / (c + U) */
    SPH_EHIP = -5,         /* a HIP runtime call failed */
    SPH_EUNSUPPORTED = -6  /* valid but not provided (e.g. dim 1) */
} sph_status;

typedef enum { SPH_FP64 = 0, SPH_FP32 = 1 } sph_precision;

/* particle kinds (byte per particle) */
enum {
    SPH_FLUID = 0, SPH_INLET = 1, SPH_OUTLET = 2,
    SPH_WALL_SLIP = 3, SPH_WALL_NOSLIP = 4, SPH_BODY = 5, /* BODY: no-slip, drag */
    SPH_DEAD = 255
};

/* sph_params.flags. SPH_FLAG_REUSE_BINS lets sph_step keep the cell order of
 * its last bin while every particle stays within the cell skin of its binned
 * position and no particle was transferred, deleted or re-spawned (the
 * neighbour sets are the same; sums run in a different row order). Steps
 * recorded for the reverse pass always bin. SPH_FLAG_QUINTIC selects the
 * paper's quintic spline (Sec. 2 eq:quintic-spline, support 3h, alpha =
 * 7/(478 pi h^2) in 2D and the normalising 1/(120 pi h^3) in 3D) instead of
 * Wendland C2 (support 2h); the neighbour predicate becomes |r|^2 < (3h)^2
 * (the reverse passes use the kernel's own derivatives).
 * SPH_FLAG_MIRROR_INLET gives inlet particles the pressure mirrored from the
 * fluid (Sec. 3 with Sec. 3.2, as SPH_OUTLET_MIRROR describes, pressure
 * only) instead of the characteristic J3 (forward only). SPH_FLAG_TILES runs
 * the neighbour search and the force pass on their LDS-tiled kernels (each
 * tile of cells and its halo staged in LDS, halo rows past the capacity read
 * from global memory) instead of the gather kernels (neighbours read from
 * global memory row by row, through the caches); both produce the same
 * neighbour table and densities and the same forces to rounding. The gather
 * kernels are the default: on the workloads measured they are the faster. */
enum { SPH_FLAG_NO_PAVG = 1, SPH_FLAG_DAMP_NU = 2, SPH_FLAG_NOISE = 4, SPH_FLAG_REUSE_BINS = 8,
       SPH_FLAG_QUINTIC = 16, SPH_FLAG_MIRROR_INLET = 32, SPH_FLAG_TILES = 128 };

/* sph_params.outlet: how outlet particles get their values and move. Every
 * rule advects outlet particles along x only; u, p are those of the rule, ut = u.
 *   HYBRID (default, Sec. 3.4): fluid characteristic variables with each fluid
 *     particle's own time averages as references (eq:characteristic-vars),
 *     Shepard-interpolated (eq:shepard), J3 = 0, previous-step red mean
 *     without fluid support (eq:average_old); u, p = the particle's frozen
 *     time average + acoustic part (eq:acou); advected with that u.
 *   MOC (Sec. 3.3): the same interpolation with fixed references u_ref = U,
 *     p_ref = 0, rho_ref = rho0; u, p = reference + acoustic part, transverse
 *     velocity unchanged; advected with that u.
 *   DO_NOTHING (Sec. 3.1, eq:nrbc2): u, p frozen at the values the particle
 *     had when it left the fluid; advected with its frozen u.
 *   MOD_DO_NOTHING (Sec. 3.1.1): u, p frozen; advected with the Shepard mean
 *     of the fluid x velocity (eq:shepard0), without fluid support with the
 *     previous-step red mean of that velocity (as eq:average_old).
 *   MIRROR (Sec. 3.2): the particle reflected about x_outlet into the fluid;
 *     p and u and their gradients at that point from the first-order
 *     corrected system eq:matform over fluid particles within the support
 *     (x_lk = x_l - x_k, V_l = 1/sum W), extrapolated back with the paper's
 *     eq:taylor2, f = f_k - (r - r_k) . grad f_k; a near-singular system (a
 *     pivot below 1e-3 of the largest entry of the system made dimensionless
 *     with h) gives the Shepard value, no fluid at the mirror point keeps
 *     the previous values; advected with u.
 * jcur holds (J1, J2, J3) for HYBRID and MOC and (u_ex, 0, 0) for
 * MOD_DO_NOTHING; DO_NOTHING and MIRROR keep no characteristic values (red
 * particles hold zeros).
 * Inlets use the characteristic inlet in all four. */
enum { SPH_OUTLET_HYBRID = 0, SPH_OUTLET_MOC = 1, SPH_OUTLET_DO_NOTHING = 2,
       SPH_OUTLET_MOD_DO_NOTHING = 3, SPH_OUTLET_MIRROR = 4 };

/* device error-word bits */
enum {
    SPH_ERR_NBR_OVERFLOW = 1u,  /* a particle has more than maxnb neighbours */
    SPH_ERR_CAPACITY = 2u,      /* a re-spawn found no free row below cap */
    SPH_ERR_NONFINITE = 4u,     /* a non-finite value after a stage update */
    SPH_ERR_SKIN = 8u,          /* a particle moved more than the cell skin in a step */
    SPH_ERR_ESCAPE = 16u,       /* a particle left the box along a closed axis */
    SPH_ERR_CELL_RANGE = 32u,   /* corrupt cell/neighbour index found (input misuse) */
    SPH_ERR_NNZ_CAPACITY = 64u  /* sph_neighbors: more entries than csr->cap_nnz */
};

/* per-row events of one step, recorded by sph_step_record for the reverse */
enum {
    SPH_EV_PUSH = 1,       /* the time-average ring took this step's sample */
    SPH_EV_TO_OUTLET = 2,  /* fluid particle crossed into the outlet */
    SPH_EV_DELETE = 4,     /* outlet particle passed the outlet end */
    SPH_EV_SPAWN = 8       /* inlet particle entered the fluid and left a child */
};

/* Host parameter block (copied by value). Symbols follow Sec. 2 of the paper:
 * h smoothing length (support 2h of the Wendland C2 kernel, 3h of the quintic
 * spline), c the artificial speed of sound c_s, nu the kinematic viscosity,
 * alpha the EDAC damping
 * coefficient (nu_edac = alpha h c / 8), eta the 0.01 regulariser, pb the
 * background pressure of the transport velocity, U the inlet reference speed
 * (also sets the acoustic-intensity gate |p| > rho0 U^2 / 2). */
typedef struct sph_params {
    int32_t dim;          /* 2 or 3 */
    int32_t n_avg;        /* time-average window, must be 6 */
    int32_t flags;        /* SPH_FLAG_* */
    int32_t periodic[3];  /* 1 = periodic axis */
    double h, dx, rho0, c, U, nu, alpha, eta, dt, pb;
    double lo[3], hi[3];  /* box; periodic axes have length hi - lo */
    double x_inlet;       /* inlet | fluid interface */
    double x_outlet;      /* fluid | outlet interface */
    double x_outlet_end;  /* outlet particles beyond are deleted */
    double inlet_len;     /* re-spawn offset of inlet particles */
    double noise_amp;     /* relative inlet velocity noise (SPH_FLAG_NOISE) */
    uint64_t noise_seed;
    int32_t group_force;  /* lanes per target in the force pass: 0 = automatic, or 1..32 (power of 2) */
    int32_t group_nbr;    /* lanes per target in the neighbour search: same convention */
    int32_t list_cap;     /* candidate-list entries per particle of the step path
                             (0 = automatic; a particle with more candidates is
                             searched through its cell stencil instead) */
    int32_t outlet;       /* SPH_OUTLET_*: the outlet rule (forward only; the
                             adjoint entry points accept the hybrid alone) */
} sph_params;

/* Particle state. Element type of u, ut, p is double for SPH_FP64 and float
 * for SPH_FP32; every other array has the type given. ring holds the last
 * n_avg accepted (u_1..u_dim, p) samples as [n_avg][dim+1][cap]; avg their
 * mean as [dim+1][cap]; head the next slot to overwrite. */
typedef struct sph_state {
    int64_t cap;          /* rows in every array */
    int32_t prec;         /* sph_precision */
    int32_t dim;          /* must equal sph_params.dim */
    int64_t *n;           /* device scalar: live particle count */
    double *x;            /* [3][cap] positions (always FP64) */
    void *u, *ut;         /* [3][cap] momentum and transport velocity */
    void *p;              /* [cap] pressure */
    double *uin;          /* [3][cap] prescribed inlet velocity */
    double *ring;         /* [n_avg][dim+1][cap] */
    uint8_t *head;        /* [cap] */
    double *avg;          /* [dim+1][cap] */
    double *jprev;        /* [3][cap] characteristic variables of the last step */
    uint8_t *red_prev;    /* [cap] fluid support at the last step */
    uint8_t *type;        /* [cap] SPH_FLUID ... */
    int64_t *id;          /* [cap] */
} sph_state;

/* Neighbour table, row-major: the neighbours of particle i (itself included)
 * are nbr[i * maxnb + k] for k < count[i], in stencil-then-cell order. */
typedef struct sph_nlist {
    int32_t maxnb;        /* rows of nbr */
    int32_t *count;       /* [cap] */
    int32_t *nbr;         /* [cap][maxnb] */
} sph_nlist;

/* Neighbour relation in compressed rows (sph_neighbors): the neighbours of
 * particle i (itself included) are col[row_ptr[i] .. row_ptr[i+1]) for
 * i < *st->n, in the same order as the rows of sph_neighbor_table. row_ptr
 * has room for cap + 1 entries, col for cap_nnz; *nnz_out receives
 * row_ptr[n] (device memory). */
typedef struct sph_csr {
    int64_t *row_ptr;     /* [cap + 1] */
    int32_t *col;         /* [cap_nnz] (may be NULL when cap_nnz is 0) */
    int64_t cap_nnz;      /* entries col can hold */
    int64_t *nnz_out;     /* [1] total entries */
} sph_csr;

/* Results of one right-hand-side evaluation. rho, vol, pavg, a, b, pdot have
 * the state's element type. a, b, pdot are written for fluid particles (zero
 * elsewhere); force only for body particles (other rows are left as they
 * are); drag is the body total. */
typedef struct sph_derived {
    void *rho, *vol, *pavg;   /* [cap] */
    void *a, *b;              /* [3][cap] momentum rate and background term */
    void *pdot;               /* [cap] */
    double *jcur;             /* [3][cap] characteristic variables this stage */
    uint8_t *red;             /* [cap] */
    double *force;            /* [3][cap] per body particle */
    double *drag;             /* [3] */
    double *sfl;              /* [cap] sum of W over fluid neighbours (non-fluid rows) */
} sph_derived;

/* Bytes of workspace needed for capacity `cap` (cell grid, sort buffers,
 * half-state copy, scan scratch, the step path's candidate lists of
 * list_cap (or the automatic count) entries per particle, the FP32 force
 * pass's packed neighbour records, error word); the same for both precisions. */
int sph_workspace_size(const sph_params *prm, int64_t cap, size_t *bytes);
/* The same figure as a return value; 0 when the parameters are invalid
 * (sph_last_error() says why). */
size_t sph_workspace_bytes(const sph_params *prm, int64_t cap);

/* Launch configuration the library derives from the parameters for a
 * capacity and precision (no GPU needed): the cell grid; whether the
 * neighbour search and the force pass stage each tile of cells and its halo
 * in LDS (tiles = 1) or gather neighbours from global memory; the tile extent
 * and halo size in cells; the lanes per target of the force pass and of the
 * search; whether the step path keeps candidate lists between sorts. */
typedef struct sph_launch_info {
    int32_t cells[3];
    int32_t tiles;
    int32_t tile_cells[3];
    int32_t halo_cells;
    int32_t group_force, group_search;
    int32_t lists;
} sph_launch_info;
int sph_launch_config(const sph_params *prm, int64_t cap, int32_t prec, sph_launch_info *out);

/* The cell structure of the last bin on this workspace (sph_bin, or the bin
 * that opens each sph_step; the neighbour structure is the implementation's,
 * no paper passage). Cells are cs[d] = (hi - lo)[d] / ncell[d] wide, at least
 * 1.3 (2D) or 1.2 (3D) times the kernel's support; a row's cell is
 * floor((x - lo) / cs) at the position it had when the rows were last sorted.
 * Cells are numbered by the Morton key of sph_cell_key, and the rows of key k
 * are [cell_start[k], cell_start[k + 1]) of the sorted state (valid while the
 * cell order is kept, i.e. until the next sorting bin). */
typedef struct sph_cells {
    int32_t ncell[3];     /* out: cells per axis (1 past dim) */
    double cs[3];         /* out: cell widths */
    int64_t nkeys;        /* out: keys are 0 .. nkeys - 1 (a power of two) */
    int32_t *cell_start;  /* device, [nkeys + 1], caller-owned; NULL: not copied */
    uint32_t *key;        /* device, [cap]: the key of each live row; NULL: not written */
} sph_cells;
int sph_get_cells(const sph_params *prm, const sph_state *st, sph_cells *out, void *ws,
                  size_t ws_bytes, void *stream);

/* Morton key of cell (cx, cy, cz) (cz = 0 in 2D) for these parameters and
 * capacity: bit b of every axis comes before bit b + 1 of any axis, in axis
 * order, an axis contributing only its ceil(log2(ncell)) bits. Returns -1 for
 * invalid parameters or a cell outside the grid. Host only. */
int64_t sph_cell_key(const sph_params *prm, int64_t cap, int32_t cx, int32_t cy, int32_t cz);

/* Default neighbour-table depth for the parameters (32 in 2D, 80 in 3D; with
 * SPH_FLAG_QUINTIC 1.6 times the lattice count of the 3h ball plus 12, in
 * multiples of 16: 80 in 2D and 336 in 3D at h = 1.2 dx). */
int32_t sph_default_maxnb(const sph_params *prm);

/* Cell-linked list (no paper passage; the neighbour structure is the
 * implementation's): cell = floor((x - lo) / cs) with cells at least 1.3 (2D)
 * or 1.2 (3D) times the kernel's support wide, Morton key, counting sort with ties ordered by
 * id; every state array
 * is gathered into *alt's buffers (scratch of the same capacity and
 * precision) and the sorted rows are copied back, so *st is sorted in place
 * and keeps its buffers. Dead particles are dropped and *st->n updated. */
int sph_bin(const sph_params *prm, sph_state *st, sph_state *alt, void *ws,
            size_t ws_bytes, void *stream);

/* Neighbour relation at the current positions from the cells of the last
 * sph_bin on this workspace (the neighbour structure is the implementation's;
 * the relation is the support of the kernel, Sec. 2 eq:summation-density): j
 * is a neighbour of i iff |r_i - r_j|^2 < (2h)^2 ((3h)^2 with
 * SPH_FLAG_QUINTIC) in FP64 without fused multiply-add, minimum image on
 * periodic axes, i itself included. Written in compressed rows: a count
 * pass, the row offsets (a scan of the counts) and a fill pass. row_ptr and
 * *nnz_out are always written; when the total exceeds csr->cap_nnz nothing is
 * written to col and SPH_ERR_NNZ_CAPACITY is set (call again with room for
 * *nnz_out entries; no row is truncated). Particles must not have moved more
 * than the cell skin since the bin. */
int sph_neighbors(const sph_params *prm, const sph_state *st, sph_csr *csr, void *ws,
                  size_t ws_bytes, void *stream);

/* The same relation as a padded table of nl->maxnb entries per row, the
 * layout the right-hand-side passes read (entries past maxnb are dropped and
 * SPH_ERR_NBR_OVERFLOW is set). If out is not NULL the summation density of
 * sph_density is written from the same pairs. With LDS tiles the table holds
 * at most sph_default_maxnb entries per row (a deeper nl is rejected). */
int sph_neighbor_table(const sph_params *prm, const sph_state *st, sph_nlist *nl,
                       sph_derived *out, void *ws, size_t ws_bytes, void *stream);

/* Summation density, Sec. 2 eq:summation-density, and the number-density
 * volume V_i = 1 / sum_j W_ij, for every particle, from the neighbour table. */
int sph_density(const sph_params *prm, const sph_state *st, const sph_nlist *nl,
                sph_derived *out, void *ws, size_t ws_bytes, void *stream);

/* Boundary values from the fluid (needs sph_bin, sph_neighbor_table and
 * sph_density first, in the same workspace: the rows and cells of the last
 * bin are used): wall ghost pressure/velocity by Shepard averaging; outlet
 * particles by the rule in prm->outlet, by default the hybrid rule of
 * Sec. 3.4 (J1, J2 of eq:characteristic-vars with time-average references,
 * Shepard eq:shepard, J3 = 0, previous-step red average eq:average_old,
 * f_o = f_ac + f_avg eq:acou; the other rules are described at
 * SPH_OUTLET_*); inlet particles keep their prescribed velocity and take p
 * from the Shepard-extrapolated J3 (or the mirror, SPH_FLAG_MIRROR_INLET).
 * Computed in FP64 for both precisions. Writes u, ut, p of non-fluid
 * particles and jcur, red. */
int sph_outlet_extrapolate(const sph_params *prm, sph_state *st, const sph_nlist *nl,
                           sph_derived *out, void *ws, size_t ws_bytes, void *stream);

/* One right-hand side: sph_density, sph_outlet_extrapolate, then the force
 * pass of Sec. 2 (eq:pavg, eq:tvf-p-ij-basa, eq:tvf-momentum, eq:p-edac and
 * the background term of eq:transport-vel) for fluid particles and the body
 * force of Sec. 4.6 eq:tvf-momentum_solid, reduced into out->drag. nl must be
 * the table the last sph_neighbor_table on this workspace wrote, unchanged: with
 * LDS tiles (sph_launch_config) the force pass reads the LDS slot of each of
 * its entries, which that search keeps in the workspace. */
int sph_rhs(const sph_params *prm, sph_state *st, const sph_nlist *nl, sph_derived *out,
            void *ws, size_t ws_bytes, void *stream);

/* The force pass alone (needs sph_density, or sph_neighbor_table with out, and
 * sph_outlet_extrapolate on the same neighbour table, state and workspace
 * first; those passes leave in the workspace what this pass gathers of a
 * neighbour, packed copies of each particle's values (FP32 states, and 3D FP64
 * states, whose copies sph_outlet_extrapolate writes) or the Shepard sums (2D
 * FP64 states), so the state must not change in between): eq:pavg, eq:tvf-p-ij-basa, eq:tvf-momentum,
 * eq:p-edac and the background term of eq:transport-vel for fluid particles;
 * eq:tvf-momentum_solid for body particles, reduced into out->drag (skipped
 * when out->drag is NULL, so that the call is exactly one kernel launch).
 * As for sph_rhs, nl must be the last sph_neighbor_table of this workspace. */
int sph_force(const sph_params *prm, const sph_state *st, const sph_nlist *nl,
              sph_derived *out, void *ws, size_t ws_bytes, void *stream);

/* nsteps explicit-midpoint RK2 steps: bin, stage 1 (neighbours + density,
 * boundary values, force pass fused with the half update into an internal
 * half state), stage 2 (the same at the half state, fused with the full
 * update), then the end-of-step bookkeeping of Sec. 3.4 (gated time-average
 * push, fluid->outlet, outlet deletion, inlet->fluid with re-spawn).
 * drag_hist (device, [nsteps][3], may be NULL) receives the body force of
 * stage 1 of every step. out receives the density and boundary data of the
 * last stage (a, b, pdot are not written). In 3D, and in 2D below a
 * capacity of 300000, the first search after each sort also records, per
 * particle, the stencil members within
 * 2h + 2 sqrt(dim) disp_max of it (disp_max: the per-axis displacement the
 * cell width allows beyond 2h); later searches until the next sort test only
 * those, which give the same neighbour table in the same order as long as no
 * particle has moved more than disp_max per axis from its sorted position
 * (checked; a violation sets SPH_ERR_SKIN). */
int sph_step(const sph_params *prm, sph_state *st, sph_state *alt, sph_nlist *nl,
             sph_derived *out, int32_t nsteps, double *drag_hist, void *ws,
             size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): sph_step
 * with the library's own scratch in place of the caller's workspace. The
 * scratch is a static device array of SPH_STATIC_SCRATCH_BYTES (32 MiB) that
 * every GPU the library runs on holds from the library's load until the
 * process ends; this call allocates nothing. It clears the part it uses, runs
 * the steps exactly as sph_step does with a freshly zeroed workspace (same
 * kernels, same results bit for bit), and writes the call's device error bits
 * (SPH_ERR_*) to *err_out (device memory, may be NULL) at the end of the call,
 * on the stream. Returns SPH_ECAPACITY, before any launch, when the capacity
 * and cell grid need a larger workspace than the scratch holds (sph_workspace
 * _size > SPH_STATIC_SCRATCH_BYTES; about 65k particles in a 2D channel).
 * Every call on one GPU shares that GPU's scratch: calls that overlap in time
 * on one GPU (other streams or threads) race and must be serialised by the
 * caller. */
#define SPH_STATIC_SCRATCH_BYTES (32u << 20)
int sph_step_static(const sph_params *prm, sph_state *st, sph_state *alt, sph_nlist *nl,
                    sph_derived *out, int32_t nsteps, double *drag_hist, uint32_t *err_out,
                    void *stream);

/* Reverse pass (vector-Jacobian product) of one right-hand side, written by
 * hand from the forward formulas (no automatic differentiation): the
 * gradient of
 *     L = sum over fluid rows (abar . a + bbar . b + pdbar pdot) + fbar . drag
 * with respect to the fluid's x, u, ut, p, the inlet rows' prescribed velocity
 * and the outlet rows' time averages, through the force pass, the neighbour
 * average pressure (eq:pavg), the boundary values (walls, hybrid outlet
 * eq:characteristic-vars / eq:shepard / eq:acou, inlet J3) and the summation
 * density. Preconditions: sph_neighbor_table and sph_rhs have run on the same
 * state, table, derived buffers and workspace (the reverse reads the stored
 * rho, V, pbar, boundary values, J and Shepard sums). Optional seeds add
 *     + sum over non-fluid rows (pseed p + useed . u) + sum over inlet/outlet
 *       rows jseed . J
 * to L, where p, u are the boundary values and J the characteristic values
 * (jcur) this right-hand side computed; inlet/outlet rows without fluid
 * support took J from the previous-step values (eq:average_old), whose
 * gradient goes to jprevbar. Gather-only, deterministic. */
typedef struct sph_adjoint {
    const void *abar, *bbar;  /* [3][cap] weights, state element type (may be NULL) */
    const void *pdbar;        /* [cap] (may be NULL) */
    const double *pseed;      /* [cap] adjoint added to non-fluid rows' p (may be NULL) */
    const double *useed;      /* [3][cap] adjoint added to non-fluid rows' u (may be NULL) */
    const double *jseed;      /* [3][cap] weight of inlet/outlet rows' J (may be NULL) */
    double fbar[3];           /* weight of the body force */
    double *xbar;             /* out [3][cap] dL/dx (every row) */
    double *ubar, *utbar;     /* out [3][cap] dL/du, dL/dut (fluid rows) */
    double *pbar;             /* out [cap] dL/dp (fluid rows) */
    double *uinbar;           /* out [3][cap] dL/du_in (inlet rows) */
    double *avgbar;           /* out [dim+1][cap] dL/d<u,p> (fluid and outlet rows) */
    double *jprevbar;         /* out [3][cap] dL/d jprev (inlet/outlet rows; may be NULL,
                                 then the previous-step values are not differentiated) */
    double *scratch;          /* [10][cap] work space */
} sph_adjoint;

int sph_rhs_adjoint(const sph_params *prm, const sph_state *st, const sph_nlist *nl,
                    const sph_derived *fwd, sph_adjoint *adj, void *ws, size_t ws_bytes,
                    void *stream);

/* ---------------------------------------------------------------------------
 * Reverse of time steps (discrete adjoint of the explicit-midpoint step).
 *
 * Adjoint of a particle state: one FP64 device array per continuous state
 * field, in the state's layout ([3][cap] for x, u, ut, uin, jprev; [cap] for
 * p; [n_avg][dim+1][cap] ring; [dim+1][cap] avg), rows in the state's order.
 */
typedef struct sph_state_adjoint {
    int64_t cap;
    double *x, *u, *ut, *p, *uin, *ring, *avg, *jprev;
} sph_state_adjoint;

/* One step exactly as sph_step (bit-identical result), recording for the
 * reverse: child[r] = row of the inlet particle that sorted row r left behind
 * (-1 if none) and events[r] = SPH_EV_* bits, for r < the live count after
 * the step's bin (device arrays of cap entries). drag (device [3], may be
 * NULL) receives the stage-1 body force. */
int sph_step_record(const sph_params *prm, sph_state *st, sph_state *alt, sph_nlist *nl,
                    sph_derived *out, double *drag, int32_t *child, uint8_t *events,
                    void *ws, size_t ws_bytes, void *stream);

/* Bytes of the scratch buffer sph_step_adjoint needs for capacity cap. */
int sph_step_adjoint_scratch_size(const sph_params *prm, int64_t cap, size_t *bytes);

/* Reverse of one step. st is the state the step started from (unchanged;
 * typically a stored copy), child / events what sph_step_record wrote for
 * that step. Given lam_next, the adjoint of the state after the step (rows in
 * that state's order: the step's sorted rows, then its children), and fbar,
 * the weight of the stage-1 body force, writes lam, the adjoint of st (rows
 * in st's order; rows the bin dropped get zero), with the discrete events of
 * the recorded step held fixed. The stage values are recomputed from st:
 * work is a scratch state (own live-count pointer), nl1/nl2 and d1/d2 scratch
 * neighbour tables and derived buffers of the two stages; scratch holds
 * sph_step_adjoint_scratch_size() bytes. lam and lam_next must not share
 * arrays. The reverse runs back through the stage updates (explicit midpoint
 * with eq:transport-vel and eq:advection), the right-hand side
 * (eq:summation-density, eq:pavg, eq:tvf-p-ij-basa, eq:tvf-momentum,
 * eq:p-edac, eq:tvf-momentum_solid), the boundary values
 * (eq:characteristic-vars, eq:shepard, eq:average_old, eq:acou, inlet J3) and
 * the bookkeeping of Sec. 3.4 (gated average eq:acouinten, transfers,
 * re-spawn). Gather-only, deterministic. */
int sph_step_adjoint(const sph_params *prm, const sph_state *st, sph_state *work,
                     const int32_t *child, const uint8_t *events, sph_nlist *nl1,
                     sph_nlist *nl2, sph_derived *d1, sph_derived *d2, const double fbar[3],
                     const sph_state_adjoint *lam_next, sph_state_adjoint *lam, void *scratch,
                     size_t scratch_bytes, void *ws, size_t ws_bytes, void *stream);

/* Stage values of one recorded step, kept so that its reverse need not
 * recompute the step (caller-owned device buffers, capacity and precision of
 * the simulation's state; a checkpointed reverse keeps one per step of a
 * segment). start: the step's sorted start state with its stage-1 boundary
 * values (own live-count pointer); perm[r]: row before the sort of sorted row
 * r; cell[r]: packed bin cell of sorted row r; nl1/d1, nl2/d2: the stage
 * neighbour tables and derived values (a, b, pdot, force, drag may be NULL);
 * half_*: the half state ([3][cap] x in FP64, [3][cap] u, ut and [cap] p in
 * the state's element type); off1/off2: [3][cap] FP32 cell offsets of the
 * two stages' positions (FP32 states only; NULL for FP64). */
typedef struct sph_step_store {
    sph_state start;
    int32_t *perm;
    uint32_t *cell;
    sph_nlist nl1, nl2;
    sph_derived d1, d2;
    double *half_x;
    void *half_u, *half_ut, *half_p;
    float *off1, *off2;
} sph_step_store;

/* sph_step_record that also fills *store with the step's stage values (nl
 * and out are not written: the step's tables and derived values go to the
 * store). With first != 0 or without SPH_FLAG_REUSE_BINS the step sorts, as
 * sph_step_record's does (bit-identical step). With the flag and first == 0
 * it continues a run as sph_step does from its second step on: the cell
 * order is kept while the cell skin allows, so a sequence of calls with first
 * set on the first one reproduces one sph_step call row for row (store->perm
 * is then the identity for steps that kept the order). */
int sph_step_record_store(const sph_params *prm, sph_state *st, sph_state *alt,
                          sph_step_store *store, int32_t first, double *drag, int32_t *child,
                          uint8_t *events, void *ws, size_t ws_bytes, void *stream);

/* sph_step_adjoint from stored stage values instead of a recomputation: st
 * is the state the step started from (as for sph_step_adjoint), store what
 * sph_step_record_store kept for that step. Same result, bit for bit, as
 * sph_step_adjoint on the same step. */
int sph_step_adjoint_stored(const sph_params *prm, const sph_state *st,
                            const sph_step_store *store, const int32_t *child,
                            const uint8_t *events, const double fbar[3],
                            const sph_state_adjoint *lam_next, sph_state_adjoint *lam,
                            void *scratch, size_t scratch_bytes, void *ws, size_t ws_bytes,
                            void *stream);

/* Gradient with respect to an inlet velocity profile theta[ntheta] that set,
 * for every row q of st with index[q] = k >= 0, the x components of u_in, u,
 * ut, every ring slot and the mean to theta[k]:
 *     grad[k] = sum over those rows of the corresponding entries of lam.
 * index: device int32 [cap] (-1 = not a profile row); grad: device [ntheta].
 * One block per entry, fixed summation order. */
int sph_inlet_profile_grad(const sph_params *prm, const sph_state *st,
                           const sph_state_adjoint *lam, const int32_t *index, int32_t ntheta,
                           double *grad, void *stream);

/* Reverse of the boundary values alone (sph_outlet_extrapolate: walls'
 * Shepard p and ghost velocity, outlet and inlet characteristic values
 * eq:characteristic-vars, eq:shepard, eq:average_old, eq:acou) through the
 * summation density the extrapolation weights use: the gradient of
 *     L = sum over non-fluid rows (pseed p + useed . u) + sum over inlet/outlet
 *         rows jseed . J
 * with respect to the fluid's x, u, p, the inlet velocities, the averages and
 * the previous-step J. Arguments as sph_rhs_adjoint; abar, bbar, pdbar and
 * fbar are ignored. Preconditions: sph_neighbor_table (with density) and
 * sph_outlet_extrapolate have run on the same state, table and buffers. */
int sph_outlet_extrapolate_adjoint(const sph_params *prm, const sph_state *st,
                                   const sph_nlist *nl, const sph_derived *fwd,
                                   sph_adjoint *adj, void *ws, size_t ws_bytes, void *stream);

/* Synchronises `stream`, returns the accumulated device error bits in *bits
 * and clears them. */
int sph_poll_error(void *ws, size_t ws_bytes, uint32_t *bits, void *stream);

/* Synchronises `stream` and returns *st->n. */
int sph_live_count(const sph_state *st, int64_t *n, void *stream);

/* Thread-local message of the last non-OK return. */
const char *sph_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SPH_H */
