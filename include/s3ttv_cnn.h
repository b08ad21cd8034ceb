/*
 * s3ttv_cnn.h — learned initial estimate for the S3TTV P-PDS solver (gfx950).
 *
 * Alg. 1 leaves the initial values of its iterates free; Prob. (18) is convex, so the start
 * changes how many iterations the stop rule (eq. StopCri_simulated) needs, not the point
 * reached. This library part computes a start u0 = v + f(v) with a small 3-D convolutional network f and
 * trains f on (v, u*) pairs whose targets u* are P-PDS solutions (s3ttv_solve). It is not
 * part of the method of the paper; the cold start (u0 = 0) stays the reference.
 *
 * Network: f = C4 o R o C3 o R o C2 o R o C1 o R o C0, Cl a 3x3x3 convolution with bias and
 * zero padding over (i, j, b), channels 1 -> 32 -> 32 -> 32 -> 32 -> 1, R = ReLU.
 * Arithmetic: weights are rounded to BF16 for each use (the FP32 masters are what the caller
 * holds and what Adam updates); biases stay FP32; activations and their gradients are stored
 * in BF16; all sums are formed in FP32. Results are reproducible run to run.
 *
 * Parameter vector (float32, device, s3ttv_cnn_param_count() entries): layers 0..4 in order,
 * each as its weights [27][cout][cin] followed by its cout biases. The tap index is
 * t = (di+1)*9 + (dj+1)*3 + (db+1) for the input voxel (i+di, j+dj, b+db) of output (i, j, b):
 *     y[i,j,b][co] = bias[co] + sum_t sum_ci W[t][co][ci] x[i+di, j+dj, b+db][ci]
 * (x = 0 outside the volume). Gradients use the same layout.
 *
 * Volumes: nb cubes of n1 x n2 x n3 float32 (band fastest, as in s3ttv.h), stored back to
 * back; no convolution crosses from one volume to the next. nb*n1*n2*n3 < 2^31.
 *
 * Conventions (as in s3ttv.h, except that float alignment suffices): device pointers on the
 * current device, the workspace any address (it is rounded up inside), the caller owns every
 * buffer, the library allocates nothing, stream = hipStream_t as void*,
 * every call returns after its work has completed. Return codes are those of s3ttv.h.
 */
#ifndef S3TTV_CNN_H
#define S3TTV_CNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* n1, n2, n3, nb >= 1. */
typedef struct {
  int32_t n1, n2, n3, nb;
} s3ttv_cnn_shape;

/* Number of float32 parameters (84 801). */
int64_t s3ttv_cnn_param_count(void);

/* Workspace bytes for s3ttv_cnn_forward (training = 0) or for s3ttv_cnn_grad and
 * s3ttv_cnn_train_step (training = 1) on this shape. EINVAL for a bad shape or null bytes,
 * EUNSUPPORTED if nb*n1*n2*n3 >= 2^31. */
int32_t s3ttv_cnn_workspace_bytes(const s3ttv_cnn_shape *shape, int32_t training, size_t *bytes);

/* u0 = v + f(v) for every volume. params: device, s3ttv_cnn_param_count() floats; v, u0:
 * device cubes (may not alias). EINVAL: null pointer or bad shape; EWORKSPACE: workspace
 * smaller than s3ttv_cnn_workspace_bytes(shape, 0). */
int32_t s3ttv_cnn_forward(const s3ttv_cnn_shape *shape, const float *params, const float *v,
                          float *u0, void *workspace, size_t workspace_bytes, void *stream);

/* Loss L = mean over all voxels of all volumes of (v + f(v) - target)^2 and its gradient
 * with respect to the parameters (taken at the BF16-rounded weights). grad: device, param
 * count floats, overwritten. loss: host, nullable. ENONFINITE if L is not finite (grad is
 * then unspecified). */
int32_t s3ttv_cnn_grad(const s3ttv_cnn_shape *shape, const float *params, const float *v,
                       const float *target, float *grad, double *loss, void *workspace,
                       size_t workspace_bytes, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected with the 1-based step
 * number) on the loss of s3ttv_cnn_grad:
 *     m = b1 m + (1-b1) g;  v2 = b2 v2 + (1-b2) g^2;
 *     params -= lr * (m / (1 - b1^step)) / (sqrt(v2 / (1 - b2^step)) + eps)
 * params, adam_m, adam_v: device, param count floats each, updated in place (the moments
 * start at zero). loss (host, nullable) receives L before the update. EINVAL also for
 * step < 1 or lr not positive and finite. ENONFINITE if L is not finite: nothing is updated. */
int32_t s3ttv_cnn_train_step(const s3ttv_cnn_shape *shape, float *params, float *adam_m,
                             float *adam_v, int32_t step, float lr, const float *v,
                             const float *target, double *loss, void *workspace,
                             size_t workspace_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* S3TTV_CNN_H */
