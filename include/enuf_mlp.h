/*
 * enuf_mlp.h -- C ABI of the small multilayer perceptron that predicts ENUF
 * parameters (alpha, grid per axis, window order, real-space cutoff) from a
 * system description and a target accuracy.  The paper chooses these by the
 * error relations of Eq. 31-32 and an iteration over the reciprocal cutoff
 * (Sec. 2.3.2); the network replaces that search with a regression trained
 * on error/time sweeps of the method itself.
 *
 * Network: n_in inputs -> n_layers hidden layers of n_hidden tanh units ->
 * n_out linear outputs, FP32.  Parameters are one contiguous float array,
 * layer by layer: W_l [out][in] row-major, then b_l [out].
 *
 * Conventions: every pointer argument is device memory (caller owned) unless
 * marked host; work is enqueued on `stream` (hipStream_t, NULL = default)
 * and not synchronised; return codes are enuf_status values from enuf.h.
 * Limits: 1 <= n_in, n_out <= 64; 1 <= n_hidden <= 128; 1 <= n_layers <= 8;
 * batch >= 1.
 */
#ifndef ENUF_MLP_H
#define ENUF_MLP_H

#include <stddef.h>
#include <stdint.h>

#include "enuf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n_in, n_hidden, n_layers, n_out;
} enuf_mlp_shape;

/* Number of floats in the parameter array (host; -1 on a bad shape). */
int64_t enuf_mlp_param_count(const enuf_mlp_shape *shape);

/* Floats of activation cache per sample the forward pass stores for the
 * backward pass (host; -1 on a bad shape). */
int64_t enuf_mlp_cache_count(const enuf_mlp_shape *shape);

/* Forward pass: y[batch][n_out] = net(x[batch][n_in]).  `cache` (may be
 * NULL) receives batch * cache_count floats of hidden activations. */
enuf_status enuf_mlp_forward(const enuf_mlp_shape *shape, const float *params, int64_t batch,
                             const float *x, float *y, float *cache, void *stream);

/* Weighted mean-squared error and its gradient:
 *   loss = sum_{s,o} w_o (y - t)^2 / batch,   dy = 2 w_o (y - t) / batch.
 * `w` holds n_out weights; `loss` is one device double (overwritten). */
enuf_status enuf_mlp_loss(const enuf_mlp_shape *shape, int64_t batch, const float *y,
                          const float *target, const float *w, float *dy, double *loss,
                          void *stream);

/* Bytes of device workspace enuf_mlp_backward needs for `batch` (host). */
size_t enuf_mlp_workspace_bytes(const enuf_mlp_shape *shape, int64_t batch);

/* Backward pass: grad[param_count] = d(sum dy . y)/d(params) for the batch,
 * from the forward cache.  `workspace` must hold enuf_mlp_workspace_bytes. */
enuf_status enuf_mlp_backward(const enuf_mlp_shape *shape, const float *params, int64_t batch,
                              const float *x, const float *cache, const float *dy, float *grad,
                              void *workspace, size_t workspace_bytes, void *stream);

/* One Adam step (Kingma & Ba 2015) on n floats, with bias correction for
 * step number t >= 1:  m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 * p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps). */
enuf_status enuf_mlp_adam(int64_t n, float *params, const float *grad, float *m, float *v,
                          float lr, float beta1, float beta2, float eps, int32_t t, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ENUF_MLP_H */
