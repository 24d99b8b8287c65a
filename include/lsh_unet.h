/*
 * lsh_unet.h -- learned warm start for the Basic Scheme (liblsh.so, gfx950).
 *
 * The Basic Scheme (Sec. 4 of Bergmann & Merkert, arXiv 1701.04685) converges
 * from any start; a good start field saves iterations.  This module predicts
 * the strain fluctuation E_y of eq. (pde_coefficients) from the phase map and
 * the macroscopic strain eps0 with a 3-level 3-D convolutional U-Net.  The
 * fixed point is linear in eps0, so the network maps the phase map to the six
 * unit-load fluctuation fields (36 channels) and the prediction for eps0 is
 * their combination with eps0's Voigt components.  The solver judges the
 * prediction through its Cauchy residual; the caller falls back to the zero
 * start when the residual grows (see lsh_solve's dev_E_init).
 *
 * Network (channels-last activations in bfloat16, float32 accumulation and
 * float32 master weights; 3x3x3 convolutions with periodic padding, ReLU,
 * 2x2x2 average pooling, nearest upsampling, skip connections by channel
 * concatenation): 32-channel input (channel 0 = phase indicator) ->
 * 32,32 | pool | 64,64 | pool | 128,128 | up, concat 64 -> 64,64 | up,
 * concat 32 -> 32,32 | 1x1 -> 64 channels (the first 36 used).
 * Convolutions run as implicit GEMMs on the MFMA bf16 units.
 * The grid side n must be a multiple of 8 (two poolings, 128-voxel tiles).
 *
 * All device memory is allocated by the caller; every call runs on `stream`
 * and synchronises it before returning only where stated.
 */
#ifndef LSH_UNET_H
#define LSH_UNET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lsh_unet lsh_unet;

/* A network with base width 32 (the only width built).  Release with
 * lsh_unet_destroy.  Errors: LSH_EINVAL.                                          */
int lsh_unet_create(int base_channels, lsh_unet **out);
void lsh_unet_destroy(lsh_unet *net);

/* Number of float32 parameters (weights and biases).                              */
int lsh_unet_param_count(const lsh_unet *net, int64_t *count);

/* Device bytes for parameters, gradients, Adam moments and bf16 weight copies.    */
int lsh_unet_param_bytes(const lsh_unet *net, size_t *bytes);

/* Binds the parameter buffer and loads `params` (host float32, param_count
 * entries; the caller draws the initial values).  Resets the Adam state.          */
int lsh_unet_bind(lsh_unet *net, void *dev_params, size_t bytes, const float *params, void *stream);

/* Copies the current float32 parameters to the host (synchronises `stream`).     */
int lsh_unet_get_params(const lsh_unet *net, float *params, void *stream);

/* Device bytes of the activation workspace for an n^3 grid (training needs the
 * gradient buffers too; inference only the forward ones).                         */
int lsh_unet_act_bytes(const lsh_unet *net, int n, int training, size_t *bytes);

/* One training step on one sample: forward, mean squared error against the
 * 36-channel target, backward, and (if lr > 0) an Adam step (beta1 0.9, beta2
 * 0.999, eps 1e-8).  With lr == 0 only the gradients are formed (accumulated
 * into the gradient buffer, which lsh_unet_zero_grad clears).
 *   dev_phase  : uint8 [n^3] phase indices (0/1), grid order (z, y, x).
 *   dev_target : float [n^3][36]: unit-load j, Mandel component c at 6 j + c.
 *   loss_out   : host, the loss of this sample (synchronises `stream`).           */
int lsh_unet_train_step(lsh_unet *net, const uint8_t *dev_phase, const float *dev_target, int n, float lr,
                        void *dev_act, size_t act_bytes, void *stream, double *loss_out);
int lsh_unet_zero_grad(lsh_unet *net, void *stream);
/* Copies the float32 gradient buffer to the host (synchronises `stream`).        */
int lsh_unet_get_grads(const lsh_unet *net, float *grads, void *stream);

/* Prediction for nload macroscopic strains: writes the start fluctuation
 *   dev_E_out : double [nload][6][n^3], Voigt with engineering shear (the layout
 *               lsh_solve takes as dev_E_init).
 *   eps0_voigt: host nload*6.
 * The head and its combination with eps0 run as one kernel, so a prediction
 * leaves no head output behind (lsh_unet_head then returns LSH_ESTATE).          */
int lsh_unet_predict(lsh_unet *net, const uint8_t *dev_phase, int n, const double *eps0_voigt, int nload,
                     double *dev_E_out, void *dev_act, size_t act_bytes, void *stream);

/* Copies the raw 64-channel head output of the last training step's forward
 * pass (float [n^3][64]) into dev_dst, for tests; it lives in that step's
 * activation workspace, which must still be allocated.                            */
int lsh_unet_head(const lsh_unet *net, int n, float *dev_dst, void *stream);

/* Layer table: for layer l < nlayer, input/output channels and kernel size
 * (arrays of at least 16 entries); weights of layer l are [ks^3][cout][cin] in
 * layer order in the parameter vector, followed by all biases.                    */
int lsh_unet_layers(const lsh_unet *net, int *nlayer, int *cin, int *cout, int *ks);

/* Training target from six solved unit-load fields:
 *   dev_E6 : double [6][6][n^3] (load j, Voigt component, point), as lsh_solve's
 *            dev_E_out for the six unit Voigt loads;  dev_target : float [n^3][36].   */
int lsh_unet_pack_target(const double *dev_E6, int n, float *dev_target, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LSH_UNET_H */
