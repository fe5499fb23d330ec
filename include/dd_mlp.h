/*
 * dd_mlp.h -- C-ABI of the warm-start network of the MI355X domain-
 * decomposition library: a 4-layer perceptron (n_in -> width -> width ->
 * width -> n_out, ReLU between layers) whose GEMMs run on BF16 matrix cores
 * with FP32 accumulation, trained with a masked mean-squared error and Adam
 * on FP32 master weights.  It maps features of a composite cell problem
 * (mu_J, nu_J and eps) to an initial X potential for the cell Sinkhorn solve
 * of Algorithm 2; the solve still runs to the same stopping tolerance
 * (Sec. 6.2), so the network only changes where the iteration starts.
 *
 * Parameter layout (flat FP32): for layers l = 0..3, W_l (dims[l] x
 * dims[l+1], row-major, y = x W + b) followed by b_l (dims[l+1]).
 * Device pointers (x_dev, t_dev, mask_dev, y_dev) are HIP device memory of
 * the caller, row-major with n_in / n_out columns; host pointers are plain
 * host memory.  All work runs on the stream given at creation; calls that
 * return host values synchronise it.  Errors: a negative dd_status and a
 * message from dd_mlp_last_error.
 */
#ifndef DD_MLP_H
#define DD_MLP_H
#include <stddef.h>

#include "dd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dd_mlp dd_mlp;

/* n_in, n_out and width multiples of 64; He-initialised from seed */
dd_status dd_mlp_create(int n_in, int n_out, int width, unsigned long long seed, void* stream,
                        dd_mlp** out);
void dd_mlp_free(dd_mlp* net);
const char* dd_mlp_last_error(const dd_mlp* net);
dd_status dd_mlp_shape(const dd_mlp* net, int* n_in, int* n_out, int* width, size_t* n_params);
/* copy all parameters from / to host memory (count must equal n_params); set resets Adam */
dd_status dd_mlp_set_params(dd_mlp* net, const float* host, size_t count);
dd_status dd_mlp_get_params(const dd_mlp* net, float* host, size_t count);
/* y (n_rows x n_out, FP32) = net(x (n_rows x n_in, FP32)); synchronises */
dd_status dd_mlp_forward(dd_mlp* net, const float* x_dev, int n_rows, float* y_dev);
/* same with BF16 inputs already padded to n_rows % 64 == 0; asynchronous */
dd_status dd_mlp_forward_bf16(dd_mlp* net, const unsigned short* xb_dev, int n_rows,
                              float* y_dev);
/* masked MSE L = sum mask (y - t)^2 / sum mask and its gradient (grad_host:
 * n_params floats, nullable); synchronises */
dd_status dd_mlp_loss_grad(dd_mlp* net, const float* x_dev, const float* t_dev,
                           const float* mask_dev, int n_rows, float* loss, float* grad_host);
/* one Adam step (beta 0.9 / 0.999, eps 1e-8) on that loss; loss of the batch before the step */
dd_status dd_mlp_train_step(dd_mlp* net, const float* x_dev, const float* t_dev,
                            const float* mask_dev, int n_rows, float lr, float* loss);
/* the hipStream_t the network's work runs on */
void* dd_mlp_get_stream(const dd_mlp* net);

/* ---- use with a domain-decomposition context (include/dd.h) ----
 *
 * Cell features (768 per cell, the network's input): [0,64) 64 mu_J/|mu_J|
 * on the cell's 8x8 pixel block; [64,640) 576 nu_J/|nu_J| on a 24x24 pixel
 * window around the block moved by the cell's integer shift
 * d_J = round(mean_nu - mean_mu); [640] log(h^2/eps); [641] the nu_J mass
 * outside the window (fraction); [642,644) d_J / 8; [644,708) the potential
 * the solve would start from (the previous sweep's), in units of eps, with
 * the linear part 2 (h^2/eps) (x - x_c).d_J of the shift added, centred over
 * the pixels of positive mass and divided by 16 h^2/eps; [708,768) zero.
 * Output (64): the
 * change of that centred potential which the solve makes, in the same units;
 * a zero output gives back the plain warm start.  Only cells whose Y-support
 * has at most 8192 points (the register and streamed solvers' cells) are
 * eligible; the others keep the plain start.
 *
 * dd_set_warm_start: attach a network (n_in 768, n_out 64) or detach it
 * (net NULL).  policy 1: predict the start of every eligible cell on the
 * first sweep of each partition after dd_init, dd_refine or an eps change;
 * policy 2: on every sweep; policy 3: on the first sweep of each partition
 * after dd_init or dd_refine only; 0: never.  On such a sweep the prediction replaces
 * the start of a cell only if the RMS of its predicted change (output units,
 * over the pixels of positive mass) is at least min_rms.  The network must
 * outlive its use.  The cell solves still run to the stopping tolerance of
 * Sec. 6.2.  dd_warm_start_count: sweeps that ran the network and cells that
 * took its start, since dd_init.
 *
 * dd_collect_cells: training samples of the last half-iteration: for every
 * eligible cell that converged, its features built from the potentials the
 * sweep started from (row of x_dev, 768 floats), the change of the centred
 * potential that its solve made (t_dev, 64 floats) and the mask of pixels
 * with positive mass (mask_dev, 64 floats) and, if cell_dev is not NULL, the
 * cell's index in its partition (int32); at most cap rows in an unspecified
 * order (device buffers of the caller); *n_out = rows written.  Synchronises. */
dd_status dd_set_warm_start(dd_ctx* ctx, dd_mlp* net, int policy, float min_rms);

/* dd_set_warm_prediction: a prediction from elsewhere for the next
 * dd_half_iterate only (then forgotten): y_dev holds one row of 64 floats per
 * cell of that sweep's partition (cells numbered row-major), in the
 * network's output units (the change of the centred potential, units of
 * 16 h^2/eps); it is applied by the same kernel and eligibility rule as the
 * network's output (Y-support of at most 8192 points, RMS of the change at
 * least min_rms), and replaces the network on that sweep.  The device buffer
 * stays the caller's and must live until that sweep has run. */
dd_status dd_set_warm_prediction(dd_ctx* ctx, const float* y_dev, float min_rms);
dd_status dd_warm_start_count(dd_ctx* ctx, int* n_sweeps, long long* n_cells);
dd_status dd_collect_cells(dd_ctx* ctx, float* x_dev, float* t_dev, float* mask_dev,
                           int* cell_dev, int cap, int* n_out);

#ifdef __cplusplus
}
#endif
#endif
