// vos_internal.h -- declarations shared by the library's translation units
// (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "vos.h"
#include "vos_unet.h"

namespace vosint {

// Record the calling thread's error message (returned by vos_last_error()).
vos_status fail(vos_status st, const std::string &msg);

// Planned shape of a network.
void unet_dims(const vos_unet *net, int *batch, int *nz, int *ny, int *nx, int *cin);

// Input / output buffers of the network's planned shape (FP32, device).
float *unet_input(vos_unet *net);
float *unet_output(vos_unet *net);

// Forward pass of the network's own input buffer into its output buffer,
// enqueued on `stream`.
vos_status unet_forward_on(vos_unet *net, hipStream_t stream);

// Launch tuning of a simulation (same ranges as vos_opts); drops its
// captured graphs.  Neither value changes the workspace layout.
vos_status set_tuning(vos_sim *s, int check_every, int coarse_cells);
void get_tuning(const vos_sim *s, int *check_every, int *coarse_cells);
// Tile shape of the 2-D tiled V-cycle legs: levels of at least `cells` cells
// take the tall tiles (results do not depend on it).
vos_status set_tile_big(vos_sim *s, unsigned cells);
unsigned get_tile_big(const vos_sim *s);

}  // namespace vosint
