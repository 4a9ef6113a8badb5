/*
 * vos_unet.h -- C ABI of the learned initial guess for the pressure equation.
 *
 * The paper solves the pressure equation obtained from continuity
 * (Eq. contDBSQS) every step and names machine-learned models only as an
 * outlook; this library adds one as an option: a 3-D U-Net that maps the
 * solid fraction and the Jacobi-scaled initial residual of the pressure solve
 * to the pressure increment, used as the solve's starting point.  The solve
 * still runs to the same tolerance, so the result does not depend on the
 * network; only the iteration count does.
 *
 * Network (fixed architecture): 3 levels with 16 / 32 / 64 channels; at each
 * level two 3x3x3 convolutions (zero padding, bias, ReLU); 2x2x2 average
 * pooling down, nearest-neighbour 2x upsampling up, skips concatenated as
 * [upsampled, skip]; a 1x1x1 head 16 -> 1.  Weights are BF16 copies of FP32
 * master weights; activations and their gradients are stored in BF16;
 * every product accumulates in FP32 on the matrix cores.  Loss: mean squared
 * error.  Optimiser: Adam (Kingma & Ba 2015) on the FP32 master weights.
 *
 * Tensors: NDHWC, x fastest among the spatial dims; an input is FP32
 * (batch, nz, ny, nx, cin), an output / target FP32 (batch, nz, ny, nx).
 * Flat parameter vector (FP32), per layer in the order
 * e0a(16->16) e0b(16->16) e1a(16->32) e1b(32->32) ba(32->64) bb(64->64)
 * d1a(96->32) d1b(32->32) d0a(48->16) d0b(16->16): W[27][ci][co] then b[co],
 * with tap = 9 (dz+1) + 3 (dy+1) + (dx+1) reading x[z+dz][y+dy][x+dx];
 * then the head's w[16] and b[1].  The first layer's input channels cin..15
 * are zero padding.
 *
 * Memory and streams follow vos.h: the caller allocates the device
 * workspace (vos_unet_workspace_bytes) and owns it; every call enqueues on
 * the stream given at creation; calls returning data to the host
 * synchronise it.
 */
#ifndef VOS_UNET_H
#define VOS_UNET_H

#include <stddef.h>
#include "vos.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vos_unet vos_unet;

/* Shape the network is planned for.  nx % 64 == 0, ny % 4 == 0,
 * nz % 4 == 0 (three levels of 2x pooling, 16-voxel matrix tiles along x),
 * 1 <= cin <= 16, batch >= 1.  train = 0 plans inference only (no gradient
 * buffers, no optimiser state). */
typedef struct { int batch, nz, ny, nx, cin, train; } vos_unet_shape;

/* Number of FP32 parameters (359761). */
vos_status vos_unet_param_count(size_t *n);

vos_status vos_unet_workspace_bytes(const vos_unet_shape *shape, size_t *bytes);

/* Create a network on `workspace` (device, >= vos_unet_workspace_bytes, 256-byte
 * aligned, caller-owned).  Parameters start at zero: set them with
 * vos_unet_set_params before use. */
vos_status vos_unet_create(const vos_unet_shape *shape, void *workspace, size_t workspace_bytes,
                           void *hip_stream, vos_unet **out);
vos_status vos_unet_destroy(vos_unet *net);

/* Copy the flat FP32 parameter vector in (also clears the Adam moments and
 * step count) or out; host (on_device = 0) or device pointer.  Non-finite
 * values are rejected with VOS_ERR_ARG. */
vos_status vos_unet_set_params(vos_unet *net, const float *theta, int on_device);
vos_status vos_unet_get_params(vos_unet *net, float *theta, int on_device);

/* Parameters to / from a file: 8 bytes "VOSUNET1", the parameter count as a
 * uint64 in the host's byte order, then the flat FP32 vector in the order
 * above.  vos_unet_load checks the header and the length (VOS_ERR_ARG on a
 * mismatch, a missing file or non-finite values) and then behaves as
 * vos_unet_set_params (the Adam state is cleared). */
vos_status vos_unet_save(vos_unet *net, const char *path);
vos_status vos_unet_load(vos_unet *net, const char *path);

/* Gradient of the last vos_unet_loss_grad / vos_unet_train_step, flat order. */
vos_status vos_unet_get_grads(vos_unet *net, float *grad, int on_device);

/* y = network(x); x, y device pointers of the planned shape. */
vos_status vos_unet_forward(vos_unet *net, const float *x, float *y);

/* Forward, loss = mean (y - target)^2 (FP64 sum, returned if loss != NULL)
 * and the gradient with respect to every parameter (kept in the workspace). */
vos_status vos_unet_loss_grad(vos_unet *net, const float *x, const float *target, double *loss);

/* One Adam step with the stored gradient (step count t += 1, bias-corrected
 * moments); lr > 0, 0 <= beta1, beta2 < 1, eps > 0. */
vos_status vos_unet_adam(vos_unet *net, float lr, float beta1, float beta2, float eps);

/* vos_unet_loss_grad followed by vos_unet_adam(lr, 0.9, 0.999, 1e-8). */
vos_status vos_unet_train_step(vos_unet *net, const float *x, const float *target, float lr, double *loss);

/* ---------------------------------------------------------------- warm start
 * With a network attached (planned for batch 1, nz, ny, nx of the simulation,
 * cin = 4), every pressure solve first builds the network input, per cell
 *   [eps_s, (r0 / sqrt(d)) / s0, (i + 1/2) / nx, 1]
 * with r0 = b - A p^n the initial residual, d = diag(A) and
 * s0 = rms(r0 / sqrt(d)) (FP64 reduction): the network works in the space
 * scaled by D^1/2, where the operator has a unit diagonal.  With use_guess = 1
 * its output y gives the search direction v = y / sqrt(d) in cells that carry
 * flow (eps > 2 eps_min; 0 in intact solid), and the solve starts from
 * p^n + alpha v with alpha = (Av . D^-1 r0) / (Av . D^-1 Av), the step that
 * minimises the Jacobi-scaled residual the stopping rule measures, if that
 * residual is then smaller than p^n's; else from p^n.  vos_diag reports
 * which, both residuals and the A-norm error removed.  gain > 0 only scales
 * the training target (vos_warm_start_sample). */
typedef struct { double gain; int use_guess; } vos_warm_start;

/* Attach (net != NULL) or detach (net == NULL).  The network must outlive the
 * attachment. */
vos_status vos_attach_unet(vos_sim *sim, vos_unet *net, const vos_warm_start *ws);

/* Training sample of the last step's pressure solve (attached network
 * required): x_dev receives the network input it was given (nz*ny*nx*4 FP32),
 * target_dev the increment the solve produced in the scaled space,
 * sqrt(d) (p^{n+1} - p^n) / (gain s0) (nz*ny*nx FP32; 0 where s0 = 0).
 * Device pointers; valid until the next step. */
vos_status vos_warm_start_sample(vos_sim *sim, float *x_dev, float *target_dev);

#ifdef __cplusplus
}
#endif

#endif /* VOS_UNET_H */
