// sph_launch.h -- host launchers of the libsph kernels (internal).
#pragma once

#include "sph_dev.h"

namespace sph {

inline int nblocks(int64_t n, int per = kBlock) { return int((n + per - 1) / per); }

// workspace buffers of the binning pipeline
struct BinBufs {
    int32_t *nspawn, *bcount, *counts, *cell_start, *cursor, *tilesum, *blist;
    int32_t *scat;  // scatter output: each cell's rows in arbitrary order
    int32_t *tmp;   // sorted row -> row of the state before the sort
    uint32_t *spread, *keys, *cpos, *cpos_s;
    int32_t *rebin;  // 1: the next bin sorts; 0: it keeps the order (Dev::reuse)
    double *xbin;    // [3][cap] positions at the last sort, sorted order
    int32_t *vfresh; // set by the gather: 1 if it sorted
    int32_t *ttab;   // tile records of the LDS-tiled pair passes (Dev::tiles)
};

int64_t scan_tiles(int64_t n);
int64_t tilesum_len(int64_t n);
// Morton spread tables; also asks the next bin to sort (rebin = 1)
void launch_spread(const Dev &k, uint32_t *spread, int32_t *rebin, hipStream_t s);
// keys + histogram, scan, scatter, per-cell id order, gather a -> b
void launch_bin(const Dev &k, const DevState &a, const DevState &b, const BinBufs &w,
                uint32_t *err, hipStream_t s);

// the sorted rows back from the second buffer set when the bin sorted
void launch_copy_back(const Dev &k, const DevState &src, const DevState &dst,
                      const int32_t *sorted, hipStream_t s);
// copy of the live rows of a into b, with the sort permutation and cells
void launch_copy_rows(const Dev &k, const DevState &a, const DevState &b, const int32_t *perm_in,
                      const int32_t *sorted, int32_t *perm_out, const uint32_t *cell_in,
                      uint32_t *cell_out, hipStream_t s);

// pair passes
int force_group(const Dev &k);
int force_grid(const Dev &k);
int force_grid_max(const Dev &k);
// lslot: the tiled search's table of LDS slots (workspace, [cap][lmax]);
// ttab: the tile records (workspace)
void launch_nbrdens(const Dev &k, const DevState &m, const Fields &R, const DevNlist &nl,
                    const DevDerived &o, int dens, const uint32_t *spread,
                    const int32_t *cell_start, const uint32_t *cpos, float *off,
                    uint16_t *lslot, const int32_t *ttab, int32_t *rebin_clear, const VList &v,
                    int vmode, uint32_t *err, hipStream_t s);
void launch_pack_rec(const Dev &k, const DevState &m, const Fields &R, const DevDerived &o,
                     const uint32_t *cpos, hipStream_t s);
void launch_density(const Dev &k, const DevState &m, const Fields &R, const DevNlist &nl,
                    const DevDerived &o, const uint32_t *cpos, uint32_t *err, hipStream_t s);
void launch_boundary(const Dev &k, const DevState &m, const Fields &R, const DevNlist &nl,
                     const DevDerived &o, const int32_t *blist, const int32_t *bcount,
                     const uint32_t *spread, const int32_t *cell_start, uint32_t *err,
                     hipStream_t s);
void launch_force(const Dev &k, const DevState &m, const Fields &R, const Fields &W,
                  const DevNlist &nl, const DevDerived &o, const float *off,
                  const uint32_t *cpos, const int32_t *ttab, const uint16_t *lslot, int mode,
                  int want_drag, double *dragpart, const double *xbin, int32_t *rebin,
                  uint32_t *err, hipStream_t s);
int nbr_group(const Dev &k);
void launch_drag_final(const Dev &k, const double *dragpart, double *drag, double *hist,
                       hipStream_t s);

// LDS-tiled pair passes (Dev::tiles): same arguments and results as the
// gather kernels launched by launch_nbrdens (stencil walk) and launch_force;
// table: the tile records k_tile_table writes after every sort
int tile_grid(const Dev &k);
int64_t tile_table_ints(const Dev &k);
void launch_tile_table(const Dev &k, const int64_t *nrows, const int32_t *cell_start,
                       const uint32_t *spread, const uint32_t *cpos, const int32_t *sorted,
                       int32_t *table, uint32_t *err, hipStream_t s);
// the cell structure of the last bin (API copy)
void launch_cells_out(const Dev &k, const int64_t *n, const uint32_t *spread,
                      const int32_t *cell_start, const uint32_t *cpos, int32_t *cs_out,
                      uint32_t *key_out, hipStream_t s);
// CSR neighbour relation (count, scan, fill); span_sum holds
// csr_spans(cap) + 1 entries
int csr_spans(int64_t cap);
void launch_csr(const Dev &k, const DevState &m, const uint32_t *spread,
                const int32_t *cell_start, const uint32_t *cpos, int64_t *row_ptr, int32_t *col,
                int64_t cap_nnz, int64_t *nnz_out, int64_t *span_sum, uint32_t *err,
                hipStream_t s);
void launch_tsearch(const Dev &k, const DevState &m, const Fields &R, const DevNlist &nl,
                    const DevDerived &o, int dens, const int32_t *table, const uint32_t *cpos,
                    float *off, uint16_t *lslot, int32_t *rebin_clear, const VList &v, int vmode,
                    uint32_t *err, hipStream_t s);
void launch_tforce(const Dev &k, const DevState &m, const Fields &R, const Fields &W,
                   const DevNlist &nl, const DevDerived &o, const float *off,
                   const uint32_t *cpos, const int32_t *table, const uint16_t *lslot, int mode,
                   int want_drag, double *dragpart, const double *xbin, int32_t *rebin,
                   uint32_t *err, hipStream_t s);

// reverse pass of one right-hand side
void launch_rhs_adjoint(const Dev &k, const DevState &m, const Fields &R, const DevNlist &nl,
                        const DevDerived &o, const DevAdj &A, const float *off,
                        const uint32_t *cpos, uint32_t *err, hipStream_t s);

// bookkeeping
void launch_end_of_step(const Dev &k, const DevState &st, const DevDerived &o,
                        int32_t *nspawn, uint8_t *sflag, int32_t *stile, int32_t *child,
                        uint8_t *events, int32_t *rebin, uint32_t *err, hipStream_t s);
void launch_finish_spawn(const Dev &k, const DevState &st, int32_t *nspawn, hipStream_t s);

// reverse of one step
void launch_adj_prep(const int64_t *n_src, int64_t *n_dst, int32_t *nspawn, hipStream_t s);
void launch_adj_end(const Dev &k, const DevState &m, const StepAdj &S, const DevAdj &A,
                    hipStream_t s);
void launch_adj_half(const Dev &k, const DevState &m, const StepAdj &S, const DevAdj &A,
                     hipStream_t s);
void launch_adj_finish(const Dev &k, const DevState &m, const DevState &pre,
                       const int32_t *perm, const StepAdj &S, const DevAdj &A, hipStream_t s);
void launch_profile_grad(const Dev &k, const int64_t *n, const DevLam &L, const int32_t *index,
                         int32_t ntheta, double *grad, hipStream_t s);

// entry-point internals shared by the C ABI's source files
int step_on_workspace(const sph_params *prm, sph_state *st, sph_state *alt, sph_nlist *nl,
                      sph_derived *out, int32_t nsteps, double *drag_hist, void *ws,
                      size_t ws_bytes, void *stream);
int api_error(int code, const char *msg);  // sets sph_last_error()'s message, returns code

}  // namespace sph
