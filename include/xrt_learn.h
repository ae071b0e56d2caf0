/*
 * xrt_learn.h -- regularised reconstruction with the x-ray transform of
 * xrt.h, and a learned (U-Net) preconditioner for it.  C ABI of libxrt.so.
 *
 * Problem (Section IV-A, eq. (opti), with the Tikhonov reading of the
 * regulariser R(c) = 1/2 ||L c||^2):
 *
 *     M c = b,   M = H^T H + lambda L^T L,   b = H^T p,
 *
 * H the forward transform of a plan (xrt_plan_forward), H^T its adjoint, and
 * L the forward differences along both grid axes with a Neumann boundary
 * (no difference across the edge of the grid).  The paper solves this class
 * of problems by conjugate gradients (Section IV-B).
 *
 * The learned preconditioner z = N(r) is a U-Net applied to a residual image:
 * N(r) = gain * rms(r) * U(r / rms(r)), with a fixed positive gain (set
 * before training, e.g. the typical ratio rms(e) / rms(M e)).  U has
 * `levels` resolution levels with c_l = min(base * 2^l, max_channels)
 * channels at level l; encoder level l: two 3x3 convolutions
 * (input -> c_l, c_l -> c_l; the input is the residual at l = 0 and the 2x2
 * average pool of level l-1 otherwise); decoder level l (levels-2 .. 0): a
 * 3x3 convolution c_{l+1} -> c_l at level l+1's resolution followed by
 * nearest 2x upsampling, concatenation [encoder output of level l, that],
 * two 3x3 convolutions 2 c_l -> c_l -> c_l; output: 1x1 convolution c_0 -> 1.
 * Every 3x3 convolution has no bias and is followed by ReLU.  The flat
 * parameter vector concatenates, in this order, enc0a, enc0b, enc1a, enc1b,
 * ..., then dec{l}up, dec{l}a, dec{l}b for l = levels-2 down to 0, then out;
 * a 3x3 weight is [9][c_out][c_in] with tap = 3 ky + kx reading input pixel
 * (h + ky - 1, w + kx - 1); out is [c_0].
 *
 * Arithmetic: the 3x3 convolutions (forward, input gradient and weight
 * gradient) run on bf16 matrix cores with fp32 accumulation; activations and
 * activation gradients are stored in bf16; master weights, Adam state,
 * weight gradients, network input and output are fp32.
 *
 * Conventions are those of xrt.h: device pointers owned by the caller,
 * outputs overwritten, work enqueued on `stream`, argument errors returned
 * before any work is enqueued, XRT_EHIP + xrt_last_error() on HIP failures.
 */
#ifndef XRT_LEARN_H
#define XRT_LEARN_H

#include <stdint.h>

#include "xrt.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------- normal operator */

/* out = lambda L^T L c on an [ny][nx] grid (forward differences along both
 * axes, Neumann boundary).  Errors: EINVAL (null pointer, nx or ny < 1). */
xrt_status xrt_reg_apply(const float* c, int32_t nx, int32_t ny, float lambda, float* out, void* stream);

/* out = (H^T H + lambda L^T L) c for the plan's grid and lines.  `sino_ws`
 * is a device buffer of n_lines floats (NULL: the call allocates one
 * stream-ordered and frees it).  Errors: EPLAN, EINVAL. */
xrt_status xrt_normal_apply(const xrt_plan* plan, float lambda, const float* c, float* out, float* sino_ws,
                            void* stream);

/* --------------------------------------------------------------- U-Net */
typedef struct xrt_unet xrt_unet;

/* A network for images of height x width (both multiples of 2^(levels-1)),
 * batches of up to max_batch images.  2 <= levels <= 8; base is a positive
 * multiple of 32 with 256 % base == 0; max_channels is 0 (cap 512) or a
 * multiple of 32 in [base, 512].
 * Parameters are initialised He-normal (std sqrt(2 / fan_in); the output
 * layer sqrt(1 / c_0)) from `seed`; Adam state is zero.  The network owns
 * its parameters and workspace (allocated here, freed by xrt_unet_destroy).
 * Errors: EINVAL, ESIZE, ENOMEM. */
xrt_status xrt_unet_create(int32_t levels, int32_t base, int32_t max_channels, int32_t height, int32_t width,
                           int32_t max_batch, uint64_t seed, xrt_unet** out);
void xrt_unet_destroy(xrt_unet* net);
xrt_status xrt_unet_num_params(const xrt_unet* net, int64_t* n);

/* Copy the fp32 parameter vector in (device, n floats) and reset Adam; or
 * out.  Errors: EINVAL. */
xrt_status xrt_unet_set_params(xrt_unet* net, const float* params, void* stream);
xrt_status xrt_unet_get_params(const xrt_unet* net, float* params, void* stream);

/* The fixed output gain of N (default 1).  Changing it rescales what the
 * network must learn; set it before training.  Errors: EINVAL (gain <= 0). */
xrt_status xrt_unet_set_gain(xrt_unet* net, float gain);
xrt_status xrt_unet_get_gain(const xrt_unet* net, float* gain);

/* Activation after every 3x3 convolution: ReLU (on != 0, the default) or
 * none (a linear network).  Set it before training.  Errors: EINVAL. */
xrt_status xrt_unet_set_relu(xrt_unet* net, int32_t on);

/* Launch fusion of xrt_unet_apply (on = 1, the default): the 2x2 average
 * pooling before each encoder level and the nearest-neighbour upsampling and
 * concatenation before each decoder level are read inside the convolutions
 * that consume them, and the output unscaling inside the last layer, instead
 * of being written out by kernels of their own (the layers listed at the top
 * of this file).  The values are the same bit for bit; on = 0 restores the separate
 * kernels, as a test hook.  Training always writes the activations out, since
 * the backward pass reads them.  Errors: EINVAL (on not 0 or 1). */
xrt_status xrt_unet_set_fusion(xrt_unet* net, int32_t on);

/* z = N(r) for `batch` images r [batch][height][width] (fp32).  An image of
 * zeros maps to zeros.  Errors: EINVAL (batch out of range, null). */
xrt_status xrt_unet_apply(xrt_unet* net, const float* r, float* z, int32_t batch, void* stream);

/* Training loss for pairs (r_b, e_b):
 *     loss = (1/batch) sum_b ||N(r_b) - e_b||^2 / ||e_b||^2,
 * written to *loss (device float); if grad is not NULL, its gradient with
 * respect to the flat parameters (device, n floats).  Errors: EINVAL. */
xrt_status xrt_unet_loss_grad(xrt_unet* net, const float* r, const float* e, int32_t batch, float* loss,
                              float* grad, void* stream);

/* xrt_unet_loss_grad followed by one Adam step (Kingma and Ba, 2015) on the
 * master parameters with learning rate lr, beta1 = 0.9, beta2 = 0.999,
 * eps = 1e-8; the bf16 copies used by the kernels are refreshed.  *loss is
 * the loss before the step.  Errors: EINVAL. */
xrt_status xrt_unet_train_step(xrt_unet* net, const float* r, const float* e, int32_t batch, float lr,
                               float* loss, void* stream);

/* Residual-space loss for the normal equations of `plan`:
 *     loss = (1/batch) sum_b ||M N(r_b) - r_b||^2 / ||r_b||^2,
 *     M = H^T H + lambda L^T L,
 * the relative residual left by one step x += N(r) (this weights the
 * network's error by M, i.e. by what the solver's residual sees).  Its
 * gradient w.r.t. N(r_b) is 2 M (M N(r_b) - r_b) / (batch ||r_b||^2); two
 * applications of M per image.  The network's image size must equal the
 * plan's grid (ESIZE otherwise).  Temporary device memory is allocated
 * stream-ordered.  Errors: EPLAN, EINVAL, ESIZE. */
xrt_status xrt_unet_loss_grad_normal(xrt_unet* net, const xrt_plan* plan, float lambda, const float* r,
                                     int32_t batch, float* loss, float* grad, void* stream);
/* xrt_unet_loss_grad_normal followed by one Adam step (as xrt_unet_train_step). */
xrt_status xrt_unet_train_step_normal(xrt_unet* net, const xrt_plan* plan, float lambda, const float* r,
                                      int32_t batch, float lr, float* loss, void* stream);

/* Energy-norm loss for the normal equations of `plan`, on pairs (r_b, e_b)
 * with r_b = M e_b:
 *     loss = (1/batch) sum_b (N(r_b) - e_b)^T M (N(r_b) - e_b) / e_b^T M e_b,
 * the squared M-norm of the error left by one step x += N(r), relative to
 * the error's (the norm conjugate gradients minimise, Section IV-B's
 * solver; the residual-space loss above is its M^2-weighted counterpart).
 * The curvature in the network's output is M rather than M^2, and the
 * gradient w.r.t. N(r_b) is 2 (M N(r_b) - r_b) / (batch e_b^T r_b): one
 * application of M per image.  e: [batch][H][W] device floats.  Temporary
 * device memory is allocated stream-ordered.  Errors: EPLAN, EINVAL, ESIZE. */
xrt_status xrt_unet_loss_grad_energy(xrt_unet* net, const xrt_plan* plan, float lambda, const float* r,
                                     const float* e, int32_t batch, float* loss, float* grad, void* stream);
/* xrt_unet_loss_grad_energy followed by one Adam step (as xrt_unet_train_step). */
xrt_status xrt_unet_train_step_energy(xrt_unet* net, const xrt_plan* plan, float lambda, const float* r,
                                      const float* e, int32_t batch, float lr, float* loss, void* stream);

/* Building blocks of the network, exposed for testing.  bf16 arrays are raw
 * 16-bit patterns; x [B][H][W][cin], w [9][cout][cin] (tap = 3 ky + kx),
 * gy [B][H][W][cout], outputs fp32.  cin and cout are multiples of 32.
 *   conv3x3_forward:     y  = conv(x, w) (zero padding; ReLU if relu != 0)
 *   conv3x3_grad_input:  gx = d/dx sum(gy * conv(x, w))
 *   conv3x3_grad_weight: gw = d/dw sum(gy * conv(x, w)), [9][cout][cin]
 * Errors: EINVAL. */
xrt_status xrt_conv3x3_forward(const uint16_t* x, const uint16_t* w, int32_t B, int32_t H, int32_t W,
                               int32_t cin, int32_t cout, int32_t relu, float* y, void* stream);
xrt_status xrt_conv3x3_grad_input(const uint16_t* gy, const uint16_t* w, int32_t B, int32_t H, int32_t W,
                                  int32_t cin, int32_t cout, float* gx, void* stream);
xrt_status xrt_conv3x3_grad_weight(const uint16_t* x, const uint16_t* gy, int32_t B, int32_t H, int32_t W,
                                   int32_t cin, int32_t cout, float* gw, void* stream);

/* ------------------------------------------------------------- solvers */
typedef struct {
    int32_t iterations;         /* accepted steps */
    int32_t operator_applies;   /* applications of M, including rejected steps and residual checks */
    int32_t learned_accepted;   /* steps taken along a network direction */
    int32_t learned_rejected;   /* network steps replaced by a CG step */
    int32_t converged;          /* 1 if the final true residual is <= tol */
    int32_t pad;
    double rel_residual;        /* ||b - M x|| / ||b||, recomputed with the exact operator */
} xrt_solve_info;

/* Solve (H^T H + lambda L^T L) x = b from x = 0 until ||b - M x|| <= tol ||b||
 * or maxit steps.
 *
 * net == NULL: conjugate gradients (Hestenes-Stiefel); window is ignored.
 * net != NULL: flexible CG (Notay's FCG(m), m = window in [1, 16]): with
 *   z_k = N(r_k), the direction p_k = z_k - sum_j (<z_k, M p_j> / <p_j, M p_j>) p_j
 *   over the last m directions, x += alpha p_k, r -= alpha M p_k,
 *   alpha = <r_k, p_k> / <p_k, M p_k>.  m = 1 is the Polak-Ribiere form
 *   beta_k = <z_k, r_k - r_{k-1}> / <z_{k-1}, r_{k-1}> (equal in exact
 *   arithmetic).  The network proposes z_k on every `period`-th step (k = 0,
 *   period, 2 period, ...; period >= 1), the other steps take z_k = r_k.  A
 *   network step is accepted only if the residual it produces,
 *   r - alpha M p with the exact operator, is smaller in norm than r;
 *   otherwise the step is recomputed with z_k = r_k (a CG step).
 * Both stop on the updated residual and then confirm with b - M x computed
 * explicitly; if that check fails they continue from the true residual.
 * history (host, may be NULL) receives the relative residual after each
 * accepted step, up to history_cap entries.  x is overwritten.  The call
 * synchronises with `stream` once per step.  Errors: EPLAN, EINVAL, ESIZE
 * (network image size differs from the plan's grid). */
xrt_status xrt_solve(const xrt_plan* plan, float lambda, const float* b, float* x, float tol, int32_t maxit,
                     xrt_unet* net, int32_t window, int32_t period, xrt_solve_info* info, double* history,
                     int32_t history_cap, void* stream);

/* Options of the flexible CG of xrt_solve_ex. */
typedef struct {
    int32_t window;     /* FCG window m in [1, 16] */
    int32_t period;     /* the network proposes on steps k = 0, period, 2 period, ... (>= 1) */
    int32_t net_steps;  /* ... and only while k < net_steps; 0: on every such step.  After it, the
                           steps take z_k = r_k and keep the M-orthogonalisation against the
                           last m directions (CG-like steps that stay conjugate to the learned
                           ones still in the window) */
    int32_t restart;    /* 1 (needs net_steps > 0): the steps after the first net_steps are plain
                           CG (Hestenes-Stiefel) restarted from the current iterate and residual
                           instead of flexible steps; 0: as described above */
} xrt_solve_opts;

/* xrt_solve with options (opts is required when net != NULL and ignored
 * otherwise); xrt_solve(..., window, period, ...) equals xrt_solve_ex with
 * {window, period, 0, 0}.  Errors: those of xrt_solve; EINVAL for a null
 * opts with a network, net_steps < 0, restart not 0 or 1, or restart with
 * net_steps = 0. */
xrt_status xrt_solve_ex(const xrt_plan* plan, float lambda, const float* b, float* x, float tol, int32_t maxit,
                        xrt_unet* net, const xrt_solve_opts* opts, xrt_solve_info* info, double* history,
                        int32_t history_cap, void* stream);

/* ------------------------------------- sinogram-domain filter preconditioner
 * For line lists made of n_views consecutive runs of n_bins lines (one view
 * each, neighbouring bins neighbouring lines, as parallel- and fan-beam
 * sinograms are), the preconditioner
 *     P r = H^T (f * (H r)) + mu r,
 * f a centred filter of `taps` (odd) coefficients applied along each view.
 * With f a positive combination of second differences and mu >= 0, P is
 * symmetric positive semi-definite (definite if mu > 0).  The filter's
 * coefficients are fitted from training pairs (paper_2503_20907_amd.learn). */

/* out[v][j] = sum_k filter[k] sino[v][j + k - taps/2] for v < n_views,
 * j < n_bins (zero outside a view).  All pointers are device memory; sino
 * and out [n_views][n_bins] must not overlap.  Errors: EINVAL (null pointer,
 * n_views < 0, n_bins < 1, taps even or outside [1, 63]). */
xrt_status xrt_sino_filter(const float* sino, int64_t n_views, int32_t n_bins, const float* filter, int32_t taps,
                           float* out, void* stream);

typedef struct {
    int64_t n_views;       /* the plan's lines: n_views runs of n_bins lines */
    int32_t n_bins;
    int32_t taps;          /* odd, 1..63 */
    const float* filter;   /* device, taps floats, centred */
    float mu;              /* >= 0 */
    int32_t pad;
} xrt_sino_precond;

/* Preconditioned CG (Hestenes-Stiefel with z_k = P r_k, P as above) for
 * (H^T H + lambda L^T L) x = b from x = 0; stopping, confirmation, history
 * and x as for xrt_solve.  info->learned_accepted counts the applications of
 * P (one per step; each costs one forward and one adjoint of the plan).
 * Errors: EPLAN, EINVAL (null pc or filter, taps even or outside [1, 63],
 * mu negative or not finite, n_views * n_bins different from the plan's
 * line count, tol <= 0, maxit < 0). */
xrt_status xrt_solve_sino_pcg(const xrt_plan* plan, float lambda, const float* b, float* x, float tol,
                              int32_t maxit, const xrt_sino_precond* pc, xrt_solve_info* info, double* history,
                              int32_t history_cap, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* XRT_LEARN_H */
