/*
 * lb_mlp: multilayer perceptron surrogate of the body's restoring-force time series, trained and
 * evaluated by hand-written gfx950 kernels (BF16 matrix-core products with FP32 accumulation,
 * FP32 master weights, Adam).  It maps simulation parameters (stress diffusion, relaxation time,
 * body radius, director angle, polarization magnitude) to the series the lattice Boltzmann method
 * produces for them; the LB run stays the fallback and the reference for its error.
 *
 * Network: widths w[0] -> w[1] -> ... -> w[L]; tanh after every layer but the last.  Parameters
 * are one FP32 array, layer by layer: W_l (w[l+1] x w[l], row major) then b_l (w[l+1]).
 *
 * Conventions: same error codes and thread-local lb_last_error() as lb.h; the handle lives in a
 * caller-owned device arena (lb_mlp_query_bytes); X, Y and outputs passed as device pointers are
 * row-major FP32 (batch rows); calls are asynchronous on the handle's stream unless stated.
 */
#ifndef LB_MLP_H
#define LB_MLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lb_mlp lb_mlp;

typedef struct {
    int32_t n_layers;       /* number of weight layers L, 1 .. 8 */
    int32_t widths[9];      /* w[0] .. w[L], each 1 .. 4096 */
    int32_t max_batch;      /* largest batch passed to forward / train, 1 .. 2^20 */
    float beta1, beta2, eps;/* Adam coefficients (0 selects 0.9, 0.999, 1e-8) */
} lb_mlp_config;

/* Device bytes for the parameters, gradients, Adam moments and activations of max_batch rows. */
int lb_mlp_query_bytes(const lb_mlp_config *cfg, size_t *bytes);

/* Number of FP32 parameters. */
int lb_mlp_n_params(const lb_mlp_config *cfg, size_t *n);

/* Create a network in `device_arena` (256-byte aligned, lb_mlp_query_bytes bytes), bound to
 * `hip_stream` (NULL: own stream).  Parameters start at zero: set them with lb_mlp_set_params. */
int lb_mlp_create(const lb_mlp_config *cfg, void *device_arena, size_t arena_bytes, void *hip_stream,
                  lb_mlp **out);

/* Copy parameters from / to host FP32 arrays of lb_mlp_n_params values (synchronous).
 * Setting parameters clears the Adam moments and the step count. */
int lb_mlp_set_params(lb_mlp *m, const float *host_params);
int lb_mlp_get_params(lb_mlp *m, float *host_params);

/* Y (batch x w[L], device) = network(X (batch x w[0], device)). */
int lb_mlp_forward(lb_mlp *m, const float *X, int32_t batch, float *Y);

/* Loss and gradients without updating: loss = mean over rows of |yhat - y|^2 / |y|^2 (squared
 * relative L2 error of each row).  host_loss may be NULL; host_grads (n_params FP32, may be NULL)
 * receives d loss / d parameters.  Synchronous. */
int lb_mlp_gradients(lb_mlp *m, const float *X, const float *Y, int32_t batch, float *host_loss,
                     float *host_grads);

/* One Adam step on that loss with learning rate lr (asynchronous; the loss of the batch before the
 * update is written to device_loss if not NULL). */
int lb_mlp_train_step(lb_mlp *m, const float *X, const float *Y, int32_t batch, float lr, float *device_loss);

int lb_mlp_destroy(lb_mlp *m);

/* lb_mlp_forward for callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): no handle, no arena, and no device or host allocation
 * in the call.  cfg: the network's widths (n_layers, widths; max_batch and the Adam fields are
 * ignored); params: device FP32 parameters in the layout above; X (batch x w[0]) and Y
 * (batch x w[L]): device FP32, row major.  The hidden activations live in a fixed scratch array of
 * the library in each GPU's memory (2^20 floats, 4 MiB, held until the process ends; its address
 * is looked up on the first call on a device): batch x (widest hidden layer) must not exceed
 * 2^19 (LB_ERANGE otherwise).  Every call on one GPU uses that GPU's array, so calls that may
 * overlap on one GPU (different streams, threads) race; calls in order on one stream are safe.
 * Same products and results as lb_mlp_forward.  Asynchronous on hip_stream. */
int lb_mlp_forward_noalloc(const lb_mlp_config *cfg, const float *params, const float *X, int32_t batch,
                           float *Y, void *hip_stream);

/* D = A B with BF16 operands and FP32 accumulation on the matrix cores (the product the network
 * uses), for testing: A (M x K), B (K x N), D (M x N), all row-major FP32 device arrays; the
 * operands are rounded to BF16 (nearest even).  Asynchronous on hip_stream. */
int lb_mlp_gemm_bf16(const float *A, const float *B, float *D, int32_t M, int32_t N, int32_t K, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
