/* Bandwidth probe of the population access pattern.
 *
 * A measurement aid beside the method, not a step of it: the FP64 population
 * traffic of one time step of the D2Q9 update (each population pulled from
 * its upstream neighbour, as the streaming of the lattice Boltzmann equation
 * moves it) with none of the collision or force arithmetic.  Timed beside the
 * step kernels, it gives the bandwidth that their access pattern allows on
 * the device: 144 bytes per cell (nine FP64 values read, nine written).
 */
#ifndef LBM_PROBE_H
#define LBM_PROBE_H

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Bytes of one probe buffer for an nx x ny lattice (0 if nx or ny < 3): nine
 * FP64 planes in the library's population layout, row y of population i at
 * element y * pitch + i * plane, plane = nx rounded up to 16 elements (128
 * bytes), pitch = 9 plane. */
size_t lbm_probe_stream_bytes(int32_t nx, int32_t ny);

/* Enqueue one pulled copy on `hip_stream`: dst_i(x, y) = src_i(x - c_ix,
 * y - c_iy) for the nine D2Q9 velocities c_i, periodic in x and y, with
 * non-temporal stores.  Workgroups of 256 threads each walk seg_rows rows of
 * a 256-column strip, in the step kernels' XCD-aware tile order.  d_src and
 * d_dst are distinct device buffers of lbm_probe_stream_bytes(nx, ny) bytes,
 * owned by the caller; their contents are arbitrary FP64 values.  Returns
 * LBM_ERR_INVALID_ARG (nothing enqueued) for NULL or equal buffers, nx or ny
 * < 3, seg_rows < 1 or more workgroups than a launch may have;
 * LBM_ERR_DEVICE if the launch fails.  Asynchronous. */
lbm_status lbm_probe_stream(const double *d_src, double *d_dst, int32_t nx, int32_t ny,
                            int32_t seg_rows, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_PROBE_H */
