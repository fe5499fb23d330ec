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

#ifdef __cplusplus
}
#endif
#endif
