/* Phase-profiling hook of libmppi_jump_phases.so: the same library built
 * with MPPI_PHASE_STAMPS, whose wave-specialised rollout kernels record
 * per-workgroup timestamps (100 MHz real-time counter) at the phase
 * boundaries of an iteration.  Not part of the control path; not exported
 * by libmppi_jump.so.
 *
 * Layout of the record: [launch][workgroup][slot], 8 launches (by iteration
 * mod 8) x 256 workgroups x 16 slots of uint64.  Slots: 0 workgroup start,
 * 1 rollout done, 2 partials stored, 3 arrival counted, 4 combine done and
 * 5 epilogue done (the combining workgroup only), 6 one for the combining
 * workgroup, else zero, 7 the consumer's first chunk ready, 8 the combining
 * workgroup's acquire done.  Workgroups from 256 on and grids above 256
 * workgroups are not recorded. */
#ifndef MPPI_JUMP_PHASES_H
#define MPPI_JUMP_PHASES_H
#include <stddef.h>
#ifdef __cplusplus
extern "C" {
#endif

#define MPPI_PHASE_LAUNCHES 8
#define MPPI_PHASE_MAX_WG 256
#define MPPI_PHASE_SLOTS 16

/* Copy the whole record (count >= 8 * 256 * 16 entries) to host memory out;
 * synchronous.  MPPI_EINVAL for a short buffer, MPPI_EDEVICE on a HIP
 * error. */
int mppi_phase_read(unsigned long long* out, size_t count);

/* Batched form: the start and end timestamps of every tile of the last
 * grid-launched batch kernel, [tile][2] for the first 8192 tiles (in the
 * order of the tile list).  count >= 8192 * 2; errors as above. */
#define MPPI_PHASE_TILES 8192
int mppi_phase_read_tiles(unsigned long long* out, size_t count);

#ifdef __cplusplus
}
#endif
#endif
