/*
 * memshield_mlp.h - page-access predictor kernels (bf16 training and
 * inference on gfx950).
 *
 * The paper decrypts a page only when the client touches it (section 4.2,
 * decrypt-on-fault).  This extension learns which pages a client is likely
 * to touch next from its recent fault history, so that the engine can
 * pre-decrypt them; decrypt-on-fault stays the fallback.  The network:
 *   ids[B][C]   the last C fault deltas of a client, as vocabulary ids
 *   x = concat(E[ids])               E: V x D        -> x: B x (C*D)
 *   h1 = relu(x W1 + b1)             W1: (C*D) x H
 *   h2 = relu(h1 W2 + b2)            W2: H x H
 *   logits = h2 W3 + b3              W3: H x V
 *   loss = mean softmax cross-entropy of logits against the next delta id
 * Parameters and the activations x, h1, h2 are stored as bfloat16 (round to
 * nearest even); matrix products run on the matrix cores with float32
 * accumulation; gradients are float32; Adam keeps float32 master weights.
 *
 * Parameter blobs: all seven tensors back to back in the order E, W1, b1,
 * W2, b2, W3, b3, row-major (E[v][d], W1[i][j] maps input i to output j);
 * the bf16 blob, the float32 master weights, Adam's m and v and the
 * gradient blob all share this layout (ms_mlp_offsets).  All pointers are
 * device memory owned by the caller; calls are stream-ordered and return
 * once enqueued.  Shapes: C*D and H multiples of 32, V a multiple of 64,
 * 1 <= batch <= the workspace's max batch.  Errors: MS_EINVAL (shape, null
 * pointer, workspace too small), MS_EDEVICE.
 */
#ifndef MEMSHIELD_MLP_H
#define MEMSHIELD_MLP_H

#include "memshield.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ms_mlp_shape {
    int32_t vocab;     /* V: delta vocabulary incl. the out-of-vocabulary id */
    int32_t context;   /* C: fault deltas per input */
    int32_t embed;     /* D: embedding width */
    int32_t hidden;    /* H: hidden width */
} ms_mlp_shape;

/* Element offsets of E, W1, b1, W2, b2, W3, b3 in a parameter blob; returns
 * the total element count (0 for an invalid shape). */
uint64_t ms_mlp_offsets(const ms_mlp_shape *shape, uint64_t offsets[7]);

/* Bytes of scratch a call needs for batches of up to max_batch rows: the
 * activations and their gradients, plus a fixed 8 MiB for the float32
 * partial products of matrix products that split their K range over
 * several workgroups.  Calls that share a workspace must not overlap on the
 * device (one workspace per stream). */
uint64_t ms_mlp_workspace_bytes(const ms_mlp_shape *shape, int32_t max_batch);

/* Forward pass: logits[batch][V] (float32). */
ms_status ms_mlp_forward(const ms_mlp_shape *shape, const uint16_t *params,
                         const int32_t *ids, int32_t batch, float *logits,
                         void *workspace, uint64_t workspace_bytes,
                         void *stream);

/* Forward + backward: the gradient of the mean loss for every parameter
 * (float32, blob layout) and the mean loss (*loss, device float). */
ms_status ms_mlp_backward(const ms_mlp_shape *shape, const uint16_t *params,
                          const int32_t *ids, const int32_t *targets,
                          int32_t batch, float *grads, float *loss,
                          void *workspace, uint64_t workspace_bytes,
                          void *stream);

/* Adam update of the float32 master weights (step counts from 1), then the
 * bf16 parameter blob is refreshed from them. */
ms_status ms_mlp_adam(const ms_mlp_shape *shape, float *master, float *m,
                      float *v, const float *grads, uint16_t *params,
                      float lr, float beta1, float beta2, float eps,
                      int32_t step, void *stream);

/* Round a float32 blob to bf16 (round to nearest even). */
ms_status ms_mlp_to_bf16(const float *src, uint16_t *dst, uint64_t n,
                         void *stream);

/* Top-k ids of each row of logits[batch][vocab] by value, ties to the lower
 * id, `exclude` (or -1) never chosen; out_ids[batch][k]; k <= 16.  When
 * out_prob is not NULL it receives the softmax probability of each chosen
 * id over the whole row (float32, [batch][k]). */
ms_status ms_mlp_topk(const float *logits, int32_t batch, int32_t vocab,
                      int32_t k, int32_t exclude, int32_t *out_ids,
                      float *out_prob, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MEMSHIELD_MLP_H */
