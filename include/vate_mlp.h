/*
 * vate_mlp.h - C ABI of the learned VATE estimator (part of libvate.so).
 *
 * Not part of the paper: a small network that reads a host's sketch state
 * and stands in for Eq. 11's closed form, which stays as its fallback and as
 * the yardstick of its error.  Features of a host, for a sketch with window k
 * (k + 3 <= 64), all at window k:
 *     x[d]   = hist[d] / g      d < k   (VATs at distance d, Eq. 5)
 *     x[k]   = live / g                 (active VATs)
 *     x[k+1] = 1 - Z_p                  (active fraction of the pool)
 *     x[k+2] = r / 16                   (r below: the log of the closed form,
 *                                        a function of live and Z_p)
 *     x[k+3 .. 63] = 0
 * Network: z1 = W1 x + b1, a1 = GELU(z1), z2 = W2 a1 + b2, a2 = GELU(z2),
 * o = w3 . a2 + b3 + r with r = ln(max(closed-form estimate, 1)); the learned
 * estimate is exp(o).  GELU is 0.5 z (1 + erf(z / sqrt 2)).  Matrix products
 * run on BF16 matrix cores with FP32 accumulation; x, W1, W2, a1, a2 (and in
 * training dz2, dz1) are rounded to BF16 (nearest even) before the products.
 *
 * theta: FP32 parameters, VATE_MLP_PARAMS floats:
 *   W1[64][64] (row = hidden unit), b1[64], W2[64][64], b2[64], w3[64], b3.
 * weights: VATE_MLP_WEIGHT_BYTES bytes (256-byte aligned) of packed BF16
 *   matrices and FP32 vectors, produced from theta by vate_mlp_pack.
 * Feature matrices are bf16 bit patterns, row-major [n][64], 16-byte aligned.
 *
 * Same conventions as vate.h: caller-owned device memory, asynchronous on the
 * given hipStream_t, VATE_* status codes.
 */
#ifndef VATE_MLP_H
#define VATE_MLP_H

#include <stddef.h>
#include <stdint.h>

#include "vate.h"

#ifdef __cplusplus
extern "C" {
#endif

#define VATE_MLP_FEATURES 64
#define VATE_MLP_HIDDEN 64
#define VATE_MLP_PARAMS 8385        /* 64*64 + 64 + 64*64 + 64 + 64 + 1 */
#define VATE_MLP_WEIGHT_BYTES 26368       /* packed network + its training envelope */

/* Pack theta (FP32) into the BF16 inference/training weight layout.  Packing
 * switches the training envelope (below) off. */
int vate_mlp_pack(const float *theta_dev, void *weights_dev, void *stream);

/* The envelope the network was trained in: the sketch geometry of its
 * training states and the range of every feature over them (BF16-rounded
 * values, as the network sees them).  With an envelope set on the weights,
 * the learned estimate entry points return the closed form of Eq. 11
 *   - for every host, when the sketch's k, g, log2_pool or width differs
 *     from the envelope's (the features then mean something else), and
 *   - for a host any of whose features lies outside [lo[f], hi[f]],
 * and count those hosts (plus hosts whose network output is not finite) in
 * device counters kept with the weights (vate_mlp_fallbacks sums them). */
typedef struct vate_mlp_envelope {
    uint32_t k, g, log2_pool, width;
    float lo[VATE_MLP_FEATURES];
    float hi[VATE_MLP_FEATURES];
} vate_mlp_envelope;

/* Set (env non-NULL) or clear (env NULL) the envelope of packed weights and
 * zero their fallback counters.  Synchronises `stream`, then copies; env is
 * read during the call only.  Errors: VATE_E_INVAL, VATE_E_DEVICE. */
int vate_mlp_set_envelope(void *weights_dev, const vate_mlp_envelope *env, void *stream);

/* Hosts given the closed form by the envelope (or a non-finite network
 * output) since the counters were last zeroed; reset != 0 zeroes them.
 * Synchronises `stream`.  Errors: VATE_E_INVAL, VATE_E_DEVICE. */
int vate_mlp_fallbacks(const void *weights_dev, uint64_t *count, int reset, void *stream);

/* o[i] = network(x_i) + r[i] for n feature rows (inference). */
int vate_mlp_forward(const void *weights_dev, const uint16_t *x_dev, const float *r_dev,
                     size_t n, float *o_dev, void *stream);

/* One minibatch of training: forward, loss L = mean_i |exp(o_i - y_i) - 1|
 * (y = ln true cardinality), backward.  Adds dL/dtheta into grad_dev
 * (VATE_MLP_PARAMS floats, zeroed by the caller) and L into *loss_dev. */
int vate_mlp_train_step(const void *weights_dev, const uint16_t *x_dev, const float *r_dev,
                        const float *y_dev, size_t n, float *grad_dev, float *loss_dev,
                        void *stream);

/* Adam update (Kingma & Ba 2015, bias-corrected) of theta with grad; m, v
 * are the moment buffers (VATE_MLP_PARAMS floats each, zero before step 1);
 * step counts from 1. */
int vate_mlp_adam(float *theta_dev, const float *grad_dev, float *m_dev, float *v_dev,
                  uint32_t step, float lr, float beta1, float beta2, float eps, void *stream);

/* dst[0..count) = value (a kernel, so it can sit inside a captured graph). */
int vate_mlp_fill(float *dst_dev, size_t count, float value, void *stream);

/* Features and residual of n hosts from vate_estimate outputs: hist_dev
 * (n x (k+1) uint32, window k), est_dev (closed-form estimates at window k),
 * the pool's active fraction at window k.  Writes x_dev (bf16 [n][64]) and
 * r_dev (n floats).  Requires k + 3 <= 64. */
int vate_mlp_features(const uint32_t *hist_dev, const float *est_dev, size_t n, uint32_t k,
                      uint32_t g, float pool_active_fraction, uint16_t *x_dev, float *r_dev,
                      void *stream);

/* Estimate n_hosts hosts at window k with the learned estimator fused into
 * the gather of vate_estimate (one pass over the VATs): est_cf_dev receives
 * the closed-form estimates, est_dev the learned ones (the closed form where
 * the network's output is not finite, and where the weights' envelope rules
 * the network out).  Requires a closed slice and
 * k + 3 <= 64.  Errors as vate_estimate, VATE_E_UNSUPPORTED for k > 61. */
int vate_estimate_learned(vate_sketch *s, const uint32_t *hosts_dev, size_t n_hosts,
                          const void *weights_dev, float *est_dev, float *est_cf_dev,
                          void *stream);

/* Workspace (bytes) for vate_estimate_learned_ws with n_hosts hosts: the
 * same as vate_estimate_ws needs (the network runs on the histograms while
 * they are in LDS). */
int vate_estimate_learned_workspace_bytes(const vate_sketch *s, size_t n_hosts, size_t *bytes);

/* Same outputs as vate_estimate_learned, with the VAT lookups of
 * vate_estimate_ws (grouped by pool slice, resolved in LDS) and the network
 * applied per 16-host tile in the pass that builds the histograms.  workspace_dev: 256-byte aligned, at
 * least vate_estimate_learned_workspace_bytes; caller-owned scratch. */
int vate_estimate_learned_ws(vate_sketch *s, const uint32_t *hosts_dev, size_t n_hosts,
                             const void *weights_dev, float *est_dev, float *est_cf_dev,
                             void *workspace_dev, size_t workspace_bytes, void *stream);

/* vate_estimate_learned_ws from a host plan made by vate_estimate_plan (vate.h)
 * in a workspace of at least vate_estimate_learned_workspace_bytes: the
 * lookups, histograms and network only.  Errors: as vate_estimate_run. */
int vate_estimate_learned_run(vate_sketch *s, size_t n_hosts, const void *weights_dev,
                              float *est_dev, float *est_cf_dev, void *workspace_dev,
                              size_t workspace_bytes, void *stream);

/* Diagnostic: D = A * B on the matrix cores for one 16x32 (A) by 32x16 (B)
 * tile, A and B row-major bf16, D row-major FP32 - checks the fragment
 * layout the kernels assume. */
int vate_mlp_mfma_selftest(const uint16_t *a_dev, const uint16_t *b_dev, float *d_dev,
                           void *stream);

#ifdef __cplusplus
}
#endif

#endif /* VATE_MLP_H */
