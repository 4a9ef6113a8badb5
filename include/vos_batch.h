/*
 * vos_batch.h -- C ABI for advancing many independent simulations together.
 *
 * A parameter sweep over micromodels (Section 3.2 of the paper varies the
 * Peclet and Damkohler numbers over several decades, one simulation each)
 * runs many small problems whose individual kernels cannot fill the GPU.  A
 * batch holds n simulations of possibly different grids and parameters,
 * carved from one caller-owned device workspace, each on a stream the batch
 * creates (default priority).  vos_batch_step advances them concurrently:
 * a pool of host worker threads drives the instances, largest first, so the
 * kernels of several instances overlap on the device; every instance runs
 * exactly the kernels of a standalone vos_sim, so its results are
 * bit-identical to a standalone run with the same options.
 *
 * Instances are ordinary vos_sim handles (vos_batch_sim): set geometry,
 * parameters and fields and read results with the vos.h calls.  Calls on
 * one batch are not thread-safe.
 */
#ifndef VOS_BATCH_H
#define VOS_BATCH_H

#include <stddef.h>
#include "vos.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vos_batch vos_batch;

/* Device workspace for n instances (grids[i], opts[i]): the sum of each
 * instance's vos_workspace_bytes, each rounded up to 256 bytes.  1 <= n <= 4096. */
vos_status vos_batch_workspace_bytes(int n, const vos_grid *grids, const vos_opts *opts, size_t *bytes);

/* Create n instances on `workspace` (device, 256-byte aligned, caller-owned,
 * >= vos_batch_workspace_bytes).  workers: host threads of vos_batch_step,
 * 1..64 (0: min(n, 8)).  Each instance starts like vos_create's. */
vos_status vos_batch_create(int n, const vos_grid *grids, const vos_params *params, const vos_opts *opts,
                            void *workspace, size_t workspace_bytes, int workers, vos_batch **out);
vos_status vos_batch_destroy(vos_batch *batch);

/* Borrowed handle of instance i (valid until vos_batch_destroy). */
vos_status vos_batch_sim(vos_batch *batch, int i, vos_sim **sim);

/* Advance every instance nsteps steps of its own dt[i] with vos_step's
 * flags.  last (n entries, may be NULL) receives each instance's final
 * diagnostics and status (n entries, may be NULL) each instance's vos_status;
 * the call returns the first failing status in instance order (its message
 * via vos_last_error), after every instance has finished. */
vos_status vos_batch_step(vos_batch *batch, const double *dt, int nsteps, int flags, vos_diag *last,
                          vos_status *status);

/* Autotuner.  For each candidate worker count (1, 2, 4, ... up to the batch's
 * maximum), each candidate Krylov check interval (2, 4, 8, 16, 32, chosen per
 * grid-size class) and each candidate tile shape of the 2-D tiled V-cycle legs
 * (the level size from which they take 32 x 16 instead of 32 x 2 tiles: 2^16,
 * 2^18, 2^20 cells or never; per grid-size class), time probe_steps
 * solid-frozen steps of the whole batch (VOS_FREEZE_SOLID: flow and transport
 * advance, the geometry does not) and keep the fastest setting.  Results do
 * not depend on it (the check interval only decides how often the host looks
 * at the device convergence flag; every tile shape forms each value by the
 * same expression).  Outputs (may be NULL): the chosen worker count and the
 * best batch step time [ms]. */
vos_status vos_batch_tune(vos_batch *batch, const double *dt, int probe_steps, int *workers, double *best_ms);

/* The tuned settings of instance i (0 <= i < n; errors: VOS_ERR_ARG): its
 * Krylov check interval and the level size from which its 2-D tiled V-cycle
 * legs take the tall tiles (0xffffffff: never).  Outputs may be NULL. */
vos_status vos_batch_tuning(vos_batch *batch, int i, int *check_every, unsigned *tile_big_cells);

#ifdef __cplusplus
}
#endif

#endif /* VOS_BATCH_H */
