// sph_launch.h -- host launchers of the libsph kernels (internal).
#pragma once

#include "sph_dev.h"

namespace sph {

inline int nblocks(int64_t n, int per = kBlock) { return int((n + per - 1) / per); }

// binning
void launch_spread(const Dev &k, uint32_t *spread, hipStream_t s);
void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
void launch_keys(const Dev &k, const DevState &st, const uint32_t *spread, uint32_t *keys,
                 uint32_t *cpos, int32_t *counts, uint32_t *err, hipStream_t s);
void launch_scan(int32_t *data, int64_t n, int32_t *blocksum, hipStream_t s);
int64_t scan_blocksum_len(int64_t n);
void launch_scatter(const Dev &k, const DevState &st, const uint32_t *keys,
                    const int32_t *cell_start, int32_t *cursor, int32_t *tmp, hipStream_t s);
void launch_cellsort(const Dev &k, const DevState &st, const int32_t *cell_start, int32_t *tmp,
                     hipStream_t s);
void launch_gather(const Dev &k, const DevState &src, const DevState &dst, const int32_t *tmp,
                   const int32_t *cell_start, const uint32_t *cpos_in, uint32_t *cpos_out,
                   double *x0, void *u0, void *p0, hipStream_t s);
void launch_set_count(const Dev &k, const DevState &st, const int32_t *cell_start,
                      hipStream_t s);

// pair passes
void launch_neighbors(const Dev &k, const DevState &st, const DevNlist &nl,
                      const uint32_t *spread, const int32_t *cell_start, const uint32_t *cpos,
                      uint32_t *err, hipStream_t s);
void launch_density(const Dev &k, const DevState &st, const DevNlist &nl, const DevDerived &o,
                    uint32_t *err, hipStream_t s);
void launch_boundary(const Dev &k, const DevState &st, const DevNlist &nl, const DevDerived &o,
                     uint32_t *err, hipStream_t s);
void launch_force(const Dev &k, const DevState &st, const DevNlist &nl, const DevDerived &o,
                  double *dragpart, uint32_t *err, hipStream_t s);
void launch_drag_final(const Dev &k, const double *dragpart, double *drag, double *hist,
                       hipStream_t s);

// integration and bookkeeping
void launch_save_start(const Dev &k, const DevState &st, double *x0, void *u0, void *p0,
                       hipStream_t s);
void launch_stage(const Dev &k, const DevState &st, const DevDerived &o, const double *x0,
                  const void *u0, const void *p0, int full, uint32_t *err, hipStream_t s);
void launch_end_of_step(const Dev &k, const DevState &st, const DevDerived &o,
                        int32_t *nspawn, uint32_t *err, hipStream_t s);
void launch_finish_spawn(const Dev &k, const DevState &st, int32_t *nspawn, hipStream_t s);

}  // namespace sph
