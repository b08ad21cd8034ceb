// C-ABI driver of the convolutional initial-estimate network: argument checks, workspace
// carving and the launch order of the forward pass, the backward pass and Adam.
#include <math.h>
#include <stdint.h>

#include "../../include/s3ttv.h"
#include "../../include/s3ttv_cnn.h"
#include "s3ttv_cnn_internal.h"

using namespace s3ttv;

namespace {

using L = CnnLayout;
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

#define CK(x)                                \
  do {                                       \
    hipError_t _e = (x);                     \
    if (_e != hipSuccess) return S3TTV_EHIP; \
  } while (0)

int32_t make_shape(const s3ttv_cnn_shape *sh, CnnShape &s) {
  if (!sh || sh->n1 < 1 || sh->n2 < 1 || sh->n3 < 1 || sh->nb < 1) return S3TTV_EINVAL;
  const long long N = (long long)sh->nb * sh->n1 * sh->n2 * sh->n3;
  if (N >= (1ll << 31)) return S3TTV_EUNSUPPORTED;
  s.n1 = sh->n1;
  s.n2 = sh->n2;
  s.n3 = sh->n3;
  s.nb = sh->nb;
  s.N = (int)N;
  return S3TTV_OK;
}

bool float_aligned(const void *p) { return p && ((uintptr_t)p % sizeof(float)) == 0; }

// Workspace regions. Carved from the caller's buffer rounded up to 256 bytes (the query
// includes that slack).
struct Ws {
  float *edge = nullptr;
  uint16_t *wf = nullptr, *wb = nullptr;
  uint16_t *act[4] = {nullptr, nullptr, nullptr, nullptr};
  uint16_t *g[2] = {nullptr, nullptr};
  float *grad = nullptr, *du = nullptr, *wpart = nullptr;
  double *loss = nullptr, *lpart = nullptr;
  size_t bytes = 0;
};

Ws carve(const CnnShape &s, bool training, void *base) {
  Ws w;
  char *b0 = base ? reinterpret_cast<char *>(align_up((uintptr_t)base)) : nullptr;
  size_t off = 0;
  auto take = [&](size_t bytes) -> void * {
    off = align_up(off);
    void *p = b0 ? b0 + off : nullptr;
    off += bytes;
    return p;
  };
  const size_t act = (size_t)s.N * 32 * sizeof(uint16_t);
  w.edge = (float *)take(L::edge_total * sizeof(float));
  w.wf = (uint16_t *)take(3 * L::kMid * sizeof(uint16_t));
  if (training) {
    w.wb = (uint16_t *)take(3 * L::kMid * sizeof(uint16_t));
    w.grad = (float *)take(L::total * sizeof(float));
    w.loss = (double *)take(sizeof(double));
    w.lpart = (double *)take((size_t)cnn_loss_parts(s) * sizeof(double));
    for (int k = 0; k < 4; ++k) w.act[k] = (uint16_t *)take(act);
    for (int k = 0; k < 2; ++k) w.g[k] = (uint16_t *)take(act);
    w.du = (float *)take((size_t)s.N * sizeof(float));
    w.wpart = (float *)take(cnn_wgrad_part_floats(s) * sizeof(float));
  } else {
    for (int k = 0; k < 2; ++k) w.act[k] = (uint16_t *)take(act);
  }
  w.bytes = align_up(off) + kAlign;
  return w;
}

// Forward pass to the last hidden activation: act[0..3] (training) or alternating act[0], act[1]
// (inference, the last one in act[1]).
hipError_t forward_hidden(const CnnShape &s, const Ws &w, const float *params, const float *v,
                          bool training, hipStream_t st) {
  hipError_t e;
  if ((e = cnn_copies(params, w.edge, w.wf, w.wb, st)) != hipSuccess) return e;
  uint16_t *a[4];
  for (int k = 0; k < 4; ++k) a[k] = training ? w.act[k] : w.act[k & 1];
  if ((e = cnn_layer_in(s, v, w.edge, a[0], st)) != hipSuccess) return e;
  for (int l = 0; l < 3; ++l)
    if ((e = cnn_layer_mid(s, a[l], w.wf + (size_t)l * L::kMid, params + L::mid_b(l), a[l + 1],
                           st)) != hipSuccess)
      return e;
  return hipSuccess;
}

// Loss and full parameter gradient into grad (device); the loss to w.loss.
hipError_t loss_and_grad(const CnnShape &s, const Ws &w, const float *params, const float *v,
                         const float *target, float *grad, hipStream_t st) {
  hipError_t e;
  if ((e = forward_hidden(s, w, params, v, true, st)) != hipSuccess) return e;
  if ((e = cnn_layer_out(s, w.act[3], w.edge, v, nullptr, target, w.du, w.lpart, w.loss, st)) !=
      hipSuccess)
    return e;
  // layer 4: weights from (act3, du); data gradient through the ReLU of act3
  if ((e = cnn_wgrad(s, 32, 1, w.act[3], w.du, w.wpart, grad + L::out_w, st)) != hipSuccess)
    return e;
  if ((e = cnn_layer_out_bwd(s, w.du, w.edge, w.act[3], w.g[0], st)) != hipSuccess) return e;
  // layers 3, 2, 1: gradient at the output of layer l + 1 is in g[cur]
  int cur = 0;
  for (int l = 2; l >= 0; --l) {
    if ((e = cnn_wgrad(s, 32, 32, w.act[l], w.g[cur], w.wpart, grad + L::mid_w(l), st)) !=
        hipSuccess)
      return e;
    if ((e = cnn_layer_mid_bwd(s, w.g[cur], w.wb + (size_t)l * L::kMid, w.act[l], w.g[cur ^ 1],
                               st)) != hipSuccess)
      return e;
    cur ^= 1;
  }
  // layer 0: weights from (v, g0)
  return cnn_wgrad(s, 1, 32, v, w.g[cur], w.wpart, grad + L::w0, st);
}

int32_t check_ws(const CnnShape &s, bool training, void *ws, size_t bytes, Ws &w) {
  if (!ws) return S3TTV_EINVAL;
  if (bytes < carve(s, training, nullptr).bytes) return S3TTV_EWORKSPACE;
  w = carve(s, training, ws);
  return S3TTV_OK;
}

int32_t fetch_loss(const Ws &w, double *loss, hipStream_t st) {
  double h = 0;
  CK(hipMemcpyAsync(&h, w.loss, sizeof(double), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  if (loss) *loss = h;
  return isfinite(h) ? S3TTV_OK : S3TTV_ENONFINITE;
}

}  // namespace

extern "C" {

int64_t s3ttv_cnn_param_count(void) { return L::total; }

int32_t s3ttv_cnn_workspace_bytes(const s3ttv_cnn_shape *shape, int32_t training, size_t *bytes) {
  CnnShape s;
  const int32_t r = make_shape(shape, s);
  if (r != S3TTV_OK) return r;
  if (!bytes) return S3TTV_EINVAL;
  *bytes = carve(s, training != 0, nullptr).bytes;
  return S3TTV_OK;
}

int32_t s3ttv_cnn_forward(const s3ttv_cnn_shape *shape, const float *params, const float *v,
                          float *u0, void *workspace, size_t workspace_bytes, void *stream) {
  CnnShape s;
  int32_t r = make_shape(shape, s);
  if (r != S3TTV_OK) return r;
  if (!float_aligned(params) || !float_aligned(v) || !float_aligned(u0) || v == u0)
    return S3TTV_EINVAL;
  Ws w;
  if ((r = check_ws(s, false, workspace, workspace_bytes, w)) != S3TTV_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  CK(forward_hidden(s, w, params, v, false, st));
  CK(cnn_layer_out(s, w.act[1], w.edge, v, u0, nullptr, nullptr, nullptr, nullptr, st));
  CK(hipStreamSynchronize(st));
  return S3TTV_OK;
}

int32_t s3ttv_cnn_grad(const s3ttv_cnn_shape *shape, const float *params, const float *v,
                       const float *target, float *grad, double *loss, void *workspace,
                       size_t workspace_bytes, void *stream) {
  CnnShape s;
  int32_t r = make_shape(shape, s);
  if (r != S3TTV_OK) return r;
  if (!float_aligned(params) || !float_aligned(v) || !float_aligned(target) ||
      !float_aligned(grad))
    return S3TTV_EINVAL;
  Ws w;
  if ((r = check_ws(s, true, workspace, workspace_bytes, w)) != S3TTV_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  CK(loss_and_grad(s, w, params, v, target, grad, st));
  return fetch_loss(w, loss, st);
}

int32_t s3ttv_cnn_train_step(const s3ttv_cnn_shape *shape, float *params, float *adam_m,
                             float *adam_v, int32_t step, float lr, const float *v,
                             const float *target, double *loss, void *workspace,
                             size_t workspace_bytes, void *stream) {
  CnnShape s;
  int32_t r = make_shape(shape, s);
  if (r != S3TTV_OK) return r;
  if (!float_aligned(params) || !float_aligned(adam_m) || !float_aligned(adam_v) ||
      !float_aligned(v) || !float_aligned(target))
    return S3TTV_EINVAL;
  if (step < 1 || !(lr > 0.f) || !isfinite(lr)) return S3TTV_EINVAL;
  Ws w;
  if ((r = check_ws(s, true, workspace, workspace_bytes, w)) != S3TTV_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  CK(loss_and_grad(s, w, params, v, target, w.grad, st));
  if ((r = fetch_loss(w, loss, st)) != S3TTV_OK) return r;
  CK(cnn_adam(params, adam_m, adam_v, w.grad, L::total, lr, step, st));
  CK(hipStreamSynchronize(st));
  return S3TTV_OK;
}

}  // extern "C"
