// Internal declarations of the convolutional initial-estimate network (kernels and driver).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace s3ttv {

// nb volumes of n1 x n2 x n3 voxels stacked along the first axis (band fastest); no
// convolution reaches from one volume into the next. N = nb * n1 * n2 * n3 < 2^31.
struct CnnShape {
  int n1, n2, n3, nb;
  int N;
};

// Offsets (in floats) of the parameter vector: per layer its weights [27][cout][cin] (tap
// t = (di+1)*9 + (dj+1)*3 + (db+1) for the neighbour at (i+di, j+dj, b+db)), then its cout
// biases. Channels 1 -> 32 -> 32 -> 32 -> 32 -> 1.
struct CnnLayout {
  static constexpr int kMid = 27 * 32 * 32;  // weights of one 32 -> 32 layer
  static constexpr int kEdge = 27 * 32;      // weights of the 1 -> 32 / 32 -> 1 layer
  static constexpr int w0 = 0, b0 = kEdge;
  static constexpr int mid_w(int l) { return kEdge + 32 + l * (kMid + 32); }
  static constexpr int mid_b(int l) { return mid_w(l) + kMid; }
  static constexpr int out_w = kEdge + 32 + 3 * (kMid + 32);
  static constexpr int out_b = out_w + kEdge;
  static constexpr int total = out_b + 1;
  // The edge-layer working copy holds W0 (BF16-rounded), b0, W4 (BF16-rounded), b4.
  static constexpr int edge_total = 2 * kEdge + 33;
  static constexpr int edge_w4 = kEdge + 32;
  static constexpr int edge_b4 = 2 * kEdge + 32;
};

hipError_t cnn_copies(const float *master, float *edge, uint16_t *fwd, uint16_t *bwd,
                      hipStream_t st);
hipError_t cnn_layer_in(const CnnShape &s, const float *v, const float *edge, uint16_t *out,
                        hipStream_t st);
hipError_t cnn_layer_mid(const CnnShape &s, const uint16_t *in, const uint16_t *W,
                         const float *bias, uint16_t *out, hipStream_t st);
hipError_t cnn_layer_mid_bwd(const CnnShape &s, const uint16_t *gin, const uint16_t *Wt,
                             const uint16_t *act, uint16_t *gout, hipStream_t st);
int cnn_loss_parts(const CnnShape &s);
hipError_t cnn_layer_out(const CnnShape &s, const uint16_t *x, const float *edge,
                         const float *v, float *u, const float *target, float *du, double *part,
                         double *loss, hipStream_t st);
hipError_t cnn_layer_out_bwd(const CnnShape &s, const float *du, const float *edge,
                             const uint16_t *x, uint16_t *dx, hipStream_t st);
size_t cnn_wgrad_part_floats(const CnnShape &s);
hipError_t cnn_wgrad(const CnnShape &s, int cin, int cout, const void *x, const void *g,
                     float *part, float *out, hipStream_t st);
hipError_t cnn_adam(float *w, float *m, float *v, const float *g, int n, float lr, int step,
                    hipStream_t st);

}  // namespace s3ttv
