/*
 * qw_mlp.h -- C ABI of the surrogate network of the learned form
 * (libqw.so, HIP for gfx950): a multilayer perceptron mapping the
 * parameters of a run -- beam waist w0, field amplitude A0, interaction time,
 * transverse momentum p0y, spin -- to the probabilities the split-operator
 * solver reports (P_0, P_+1, P_-1, P_+2, P_-2, P_flip; see qw_observables),
 * trained on the solver's own batched runs.  The paper has no such network:
 * it runs parameter scans with the solver (beam divergence, i.e. waist, and
 * wavelength in Sec. IV.B, field amplitude in Sec. IV.D); the network is a
 * learned stand-in that interpolates such scans, with the solver as fallback.
 *
 * Network: x -> (x - shift) * scale -> [Linear(width) -> GELU] x depth ->
 * Linear(n_out); an ensemble of n_nets independent nets is evaluated and
 * trained together, their spread serving as the error estimate.
 *   - GELU(z) = z (1 + erf(z / sqrt 2)) / 2;
 *   - loss: mean squared error over the batch and the outputs;
 *   - optimiser: Adam (b1 = 0.9, b2 = 0.999, eps = 1e-8, bias-corrected).
 * Precision: weights, activations and gradients are stored in bfloat16 for
 * the matrix products (v_mfma_f32_32x32x16_bf16, FP32 accumulation); the
 * pre-activations, losses, weight gradients and the Adam state and master
 * parameters are FP32.
 *
 * Parameters of one net, flat FP32: for each linear layer in order, W[out][in]
 * row-major then b[out].  All nets' parameters follow each other.
 *
 * Conventions: device pointers are caller-owned device memory on the
 * workspace's device; calls enqueue on hip_stream and do not wait unless
 * stated; every function returns QW_OK (0) or a negative QW_E_* code (qw.h)
 * and never throws; argument errors come before anything is enqueued;
 * qw_mlp_last_error describes the last failure.  The library allocates no
 * device memory.
 */
#ifndef QW_MLP_H
#define QW_MLP_H

#include <stddef.h>
#include <stdint.h>

#include "qw.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qw_mlp_s *qw_mlp;

/* 1 <= n_in <= 16, width a multiple of 64 in [64, 1024], 1 <= depth <= 16,
 * 1 <= n_out <= 16, 1 <= n_nets <= 16, 1 <= max_batch <= 65536. */
typedef struct {
    int32_t n_in, width, depth, n_out, n_nets, max_batch;
} qw_mlp_shape;

/* FP32 parameters of one net, and workspace bytes (host-only). */
int qw_mlp_param_count(const qw_mlp_shape *s, int64_t *per_net);
int qw_mlp_workspace_bytes(const qw_mlp_shape *s, size_t *bytes);

/* Bind the workspace (256-byte aligned, >= qw_mlp_workspace_bytes) and set
 * the input map (host arrays of n_in floats).  Parameters start at zero
 * until qw_mlp_set_params.  Waits for hip_stream. */
int qw_mlp_init(qw_mlp *out, const qw_mlp_shape *s, const float *shift, const float *scale, void *workspace,
                size_t ws_bytes, void *hip_stream);

/* Load n_nets x per_net FP32 parameters from device memory; resets the Adam
 * moments and step count. */
int qw_mlp_set_params(qw_mlp h, const float *params, void *hip_stream);
/* Copy the current FP32 master parameters to device memory. */
int qw_mlp_get_params(qw_mlp h, float *params, void *hip_stream);

/* Raw outputs of every net (before the output map): x is [B][n_in] FP32,
 * y is [n_nets][B][n_out] FP32 (device), 1 <= B <= max_batch. */
int qw_mlp_forward(qw_mlp h, const float *x, int32_t B, float *y, void *hip_stream);

/* Output map of qw_mlp_predict (host arrays of n_out floats; waits for
 * hip_stream): predictions are y scale + shift of the network outputs y, so
 * a network trained on standardised targets (t - shift) / scale predicts in
 * the targets' own units.  Default: identity. */
int qw_mlp_set_output_map(qw_mlp h, const float *shift, const float *scale, void *hip_stream);

/* Weights of the error estimate (host array of n_out floats >= 0; waits for
 * hip_stream): qw_mlp_predict's spread is the largest over the outputs of
 * weight x standard deviation across the nets.  Default: all one (the
 * deviation in each output's own units).  With weights 1/scale of the
 * output map the estimate is in the units the nets were trained in, which
 * puts outputs of very different magnitudes on one scale. */
int qw_mlp_set_spread_weights(qw_mlp h, const float *w, void *hip_stream);

/* Ensemble prediction: mean [B][n_out] over the nets of the mapped outputs
 * and, per sample, the largest weighted standard deviation over the outputs
 * (the error estimate; qw_mlp_set_spread_weights), spread [B] (both device
 * FP32). */
int qw_mlp_predict(qw_mlp h, const float *x, int32_t B, float *mean, float *spread, void *hip_stream);

/* qw_mlp_predict for callers that cannot allocate or pass scratch memory
 * (code under HIP graph capture, serving loops): the same results, with the
 * inputs and activations of the prediction in a static device array of the
 * library (QW_MLP_STATIC_SCRATCH_BYTES per GPU, held until the process ends,
 * set up by qw_mlp_init) instead of the network's workspace.  Allocates
 * nothing.  B <= QW_MLP_STATIC_MAX_BATCH, and the network's activations for
 * B rows must fit the array (4 nets of depth 4 and width 256: up to 256
 * rows); otherwise QW_E_SIZE before anything is enqueued.  All calls on one
 * GPU share the array: two such calls that overlap on a GPU (other streams,
 * other networks, other host threads) race and must be serialised by the
 * caller. */
#define QW_MLP_STATIC_MAX_BATCH 256
#define QW_MLP_STATIC_SCRATCH_BYTES (4u << 20)
int qw_mlp_predict_static(qw_mlp h, const float *x, int32_t B, float *mean, float *spread, void *hip_stream);

/* Loss and gradients without an update: t is [B][n_out] targets in the
 * units of the raw outputs (standardised, if an output map is used); grads is
 * laid out as the parameters (n_nets x per_net FP32), loss is [n_nets]
 * (device; either may be NULL). */
int qw_mlp_gradients(qw_mlp h, const float *x, const float *t, int32_t B, float *grads, float *loss,
                     void *hip_stream);

/* One Adam step of every net on the batch (x, t) with learning rate lr;
 * loss (device [n_nets], may be NULL) receives the loss before the step. */
int qw_mlp_train_step(qw_mlp h, const float *x, const float *t, int32_t B, float lr, float *loss,
                      void *hip_stream);

/* The building block on its own: C[m][n] = sum_k A[m][k] B[n][k] for
 * bfloat16 A [M][lda] and B [N][ldb] (row-major, K-contiguous), FP32
 * C [M][ldc]; K a multiple of 16, lda and ldb multiples of 8 and >= K,
 * ldc >= N, A and B 16-byte aligned. */
int qw_gemm_bf16_nt(const void *A, int32_t lda, const void *B, int32_t ldb, float *C, int32_t ldc, int32_t M,
                    int32_t N, int32_t K, void *hip_stream);

const char *qw_mlp_last_error(qw_mlp h);
void qw_mlp_destroy(qw_mlp h);

#ifdef __cplusplus
}
#endif
#endif /* QW_MLP_H */
