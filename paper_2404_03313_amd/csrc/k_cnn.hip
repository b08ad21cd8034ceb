// Learned initial estimate u0 for Alg. 1, whose initial values are free (Prob. (18) is convex:
// the start changes the iteration count, not the solution). A five-layer 3-D convolutional
// network computes u0 = v + f(v), f = C4 o R o C3 o R o C2 o R o C1 o R o C0, each C a 3x3x3
// convolution with bias and zero padding (channels 1 -> 32 -> 32 -> 32 -> 32 -> 1), R = ReLU.
// Weights: FP32 masters (Adam), BF16 working copies; biases FP32. Activations and their
// gradients are stored in BF16, channels-last ([voxel][32]); every sum is formed in FP32.
//
// The 32 -> 32 layers are implicit GEMMs on v_mfma_f32_16x16x32_bf16: a wavefront forms 16
// consecutive voxels x 16 output channels, one MFMA per tap with all 32 input channels as the
// K = 32 dimension, so 27 MFMAs (x 2 channel halves) per tile. Lane (i + 16 kb) supplies, as
// the A operand, input channels 8kb..8kb+7 of the neighbour of voxel i (one 16-byte load),
// and as the B operand the weights [tap][co = i][8kb..8kb+7] from LDS. The data gradient of
// the same layers runs through the same kernel with mirrored taps and transposed weights.
// The 1 -> 32 and 32 -> 1 layers and the weight gradients run on FP32 VALU; weight
// gradients are summed per workgroup over a fixed voxel range and then over workgroups in a
// fixed order, so every result is reproducible.
#include "s3ttv_cnn_internal.h"

namespace s3ttv {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kNT = 256;
using L = CnnLayout;

__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// FP32 -> BF16, round to nearest even (the values met here are finite).
__device__ inline uint16_t f2bf(float x) {
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf_round(float x) { return bf2f(f2bf(x)); }

struct Vox {
  int i, il, j, b;  // row over the stacked volumes, row within its volume, column, band
};
__device__ inline Vox vox_of(int e, const CnnShape &s) {
  Vox v;
  const int pix = (int)((unsigned)e / (unsigned)s.n3);
  v.b = e - pix * s.n3;
  v.i = (int)((unsigned)pix / (unsigned)s.n2);
  v.j = pix - v.i * s.n2;
  v.il = (int)((unsigned)v.i % (unsigned)s.n1);
  return v;
}
__device__ inline void vox_next(Vox &v, const CnnShape &s) {
  if (++v.b < s.n3) return;
  v.b = 0;
  if (++v.j < s.n2) return;
  v.j = 0;
  ++v.i;
  if (++v.il == s.n1) v.il = 0;
}
// Voxel index of the neighbour at tap t (mirror: at the opposite offset), -1 outside the
// volume (zero padding).
__device__ inline int neighbour(const Vox &v, int t, const CnnShape &s, bool mirror) {
  int di = t / 9 - 1, dj = (t / 3) % 3 - 1, db = t % 3 - 1;
  if (mirror) {
    di = -di;
    dj = -dj;
    db = -db;
  }
  const int il = v.il + di, j = v.j + dj, b = v.b + db;
  if (il < 0 || il >= s.n1 || j < 0 || j >= s.n2 || b < 0 || b >= s.n3) return -1;
  return ((v.i + di) * s.n2 + j) * s.n3 + b;
}

__device__ inline void store_row32(uint16_t *dst, const float *y) {
  uint4 *o = reinterpret_cast<uint4 *>(dst);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    uint32_t w[4];
#pragma unroll
    for (int h = 0; h < 4; ++h)
      w[h] = (uint32_t)f2bf(y[8 * q + 2 * h]) | ((uint32_t)f2bf(y[8 * q + 2 * h + 1]) << 16);
    o[q] = make_uint4(w[0], w[1], w[2], w[3]);
  }
}
__device__ inline void load_row32(const uint16_t *src, float *x) {
  const uint4 *r = reinterpret_cast<const uint4 *>(src);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint4 a = r[q];
    const uint32_t w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      x[8 * q + 2 * h] = bf2f((uint16_t)(w[h] & 0xffffu));
      x[8 * q + 2 * h + 1] = bf2f((uint16_t)(w[h] >> 16));
    }
  }
}

// ------------------------------------------------------------ layer 0: 1 -> 32, ReLU

__global__ __launch_bounds__(kNT) void k_cnn_in(CnnShape s, const float *v, const float *edge,
                                                uint16_t *out) {
  __shared__ float w[L::kEdge + 32];
  for (int k = threadIdx.x; k < L::kEdge + 32; k += kNT) w[k] = edge[k];
  __syncthreads();
  for (int e = blockIdx.x * kNT + threadIdx.x; e < s.N; e += gridDim.x * kNT) {
    const Vox p = vox_of(e, s);
    float acc[32];
#pragma unroll
    for (int c = 0; c < 32; ++c) acc[c] = w[L::kEdge + c];
    for (int t = 0; t < 27; ++t) {
      const int q = neighbour(p, t, s, false);
      if (q < 0) continue;
      const float x = v[q];
#pragma unroll
      for (int c = 0; c < 32; ++c) acc[c] = fmaf(x, w[t * 32 + c], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < 32; ++c) acc[c] = fmaxf(acc[c], 0.f);
    store_row32(out + (size_t)e * 32, acc);
  }
}

// ------------------------------------------------------------ 32 -> 32 on MFMA

// MODE 0 (forward):       out = relu(conv(in, W) + bias), W as [tap][co][ci]
// MODE 1 (data gradient): out = (act > 0) * conv_mirrored(in, W), W as [tap][ci][co]
template <int MODE>
__global__ __launch_bounds__(kNT) void k_cnn_mid(CnnShape s, const uint16_t *in, const uint16_t *W,
                                                 const float *bias, const uint16_t *act,
                                                 uint16_t *out) {
  __shared__ __align__(16) uint16_t w[L::kMid];
  for (int k = threadIdx.x; k < L::kMid / 8; k += kNT)
    reinterpret_cast<uint4 *>(w)[k] = reinterpret_cast<const uint4 *>(W)[k];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, kb = lane >> 4;
  const int ntiles = (s.N + 15) / 16;
  for (int tile = blockIdx.x * 4 + wave; tile < ntiles; tile += gridDim.x * 4) {
    const int e = tile * 16 + i;  // voxel of this lane's A-operand row
    const bool valid = e < s.N;
    const Vox p = vox_of(valid ? e : 0, s);
    f4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 3
    for (int t = 0; t < 27; ++t) {
      const int q = valid ? neighbour(p, t, s, MODE == 1) : -1;
      bf8 a;
      if (q >= 0) {
        a = *reinterpret_cast<const bf8 *>(in + (size_t)q * 32 + 8 * kb);
      } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] = (__bf16)0.f;
      }
      const bf8 b0 = *reinterpret_cast<const bf8 *>(w + (t * 32 + i) * 32 + 8 * kb);
      const bf8 b1 = *reinterpret_cast<const bf8 *>(w + (t * 32 + 16 + i) * 32 + 8 * kb);
      acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b0, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b1, acc1, 0, 0, 0);
    }
    // result lane (c, g), register r: voxel 4g + r of the tile, output channel c (and 16 + c)
    const int c = lane & 15, g = lane >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int eo = tile * 16 + 4 * g + r;
      if (eo >= s.N) continue;
      float y0 = acc0[r], y1 = acc1[r];
      if (MODE == 0) {
        y0 = fmaxf(y0 + bias[c], 0.f);
        y1 = fmaxf(y1 + bias[16 + c], 0.f);
      } else {
        if (!(bf2f(act[(size_t)eo * 32 + c]) > 0.f)) y0 = 0.f;
        if (!(bf2f(act[(size_t)eo * 32 + 16 + c]) > 0.f)) y1 = 0.f;
      }
      out[(size_t)eo * 32 + c] = f2bf(y0);
      out[(size_t)eo * 32 + 16 + c] = f2bf(y1);
    }
  }
}

// ------------------------------------------------------------ layer 4: 32 -> 1, residual

// u = v + b4 + conv(x, W4). With a target also du = 2 (u - target) / N and, per workgroup, the
// partial sum of (u - target)^2.
__global__ __launch_bounds__(kNT) void k_cnn_out(CnnShape s, const uint16_t *x, const float *edge,
                                                 const float *v, float *u, const float *target,
                                                 float *du, double *part) {
  __shared__ float w[L::kEdge];
  __shared__ double sh[kNT / 64];
  for (int k = threadIdx.x; k < L::kEdge; k += kNT) w[k] = edge[L::edge_w4 + k];
  __syncthreads();
  const float b4 = edge[L::edge_b4];
  double l2 = 0;
  for (int e = blockIdx.x * kNT + threadIdx.x; e < s.N; e += gridDim.x * kNT) {
    const Vox p = vox_of(e, s);
    float acc = 0.f;
    for (int t = 0; t < 27; ++t) {
      const int q = neighbour(p, t, s, false);
      if (q < 0) continue;
      float xr[32];
      load_row32(x + (size_t)q * 32, xr);
#pragma unroll
      for (int c = 0; c < 32; ++c) acc = fmaf(xr[c], w[t * 32 + c], acc);
    }
    const float ue = v[e] + (acc + b4);
    if (u) u[e] = ue;
    if (target) {
      const float d = ue - target[e];
      du[e] = 2.f * d / (float)s.N;
      l2 += (double)d * (double)d;
    }
  }
  if (target) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) l2 += __shfl_xor(l2, m);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = l2;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  }
}

// loss = sum(part) / N, fixed order.
__global__ __launch_bounds__(kNT) void k_cnn_loss(const double *part, int nparts, int N,
                                                  double *loss) {
  __shared__ double sh[kNT];
  double a = 0;
  for (int k = threadIdx.x; k < nparts; k += kNT) a += part[k];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int m = kNT / 2; m >= 1; m >>= 1) {
    if ((int)threadIdx.x < m) sh[threadIdx.x] += sh[threadIdx.x + m];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = sh[0] / (double)N;
}

// Data gradient of layer 4 through the ReLU of its input:
// dx[e][c] = (x[e][c] > 0) * sum_t du[mirrored neighbour t of e] W4[t][c].
__global__ __launch_bounds__(kNT) void k_cnn_out_bwd(CnnShape s, const float *du, const float *edge,
                                                     const uint16_t *x, uint16_t *dx) {
  __shared__ float w[L::kEdge];
  for (int k = threadIdx.x; k < L::kEdge; k += kNT) w[k] = edge[L::edge_w4 + k];
  __syncthreads();
  for (int e = blockIdx.x * kNT + threadIdx.x; e < s.N; e += gridDim.x * kNT) {
    const Vox p = vox_of(e, s);
    float acc[32];
#pragma unroll
    for (int c = 0; c < 32; ++c) acc[c] = 0.f;
    for (int t = 0; t < 27; ++t) {
      const int q = neighbour(p, t, s, true);
      if (q < 0) continue;
      const float g = du[q];
#pragma unroll
      for (int c = 0; c < 32; ++c) acc[c] = fmaf(g, w[t * 32 + c], acc[c]);
    }
    float xr[32];
    load_row32(x + (size_t)e * 32, xr);
#pragma unroll
    for (int c = 0; c < 32; ++c)
      if (!(xr[c] > 0.f)) acc[c] = 0.f;
    store_row32(dx + (size_t)e * 32, acc);
  }
}

// ------------------------------------------------------------ weight gradients

// Partial, over the workgroup's voxel range, of dW[t][co][ci] = sum_e g[e][co] x[nb_t(e)][ci]
// and db[co] = sum_e g[e][co]. CIN, COUT in {1, 32}: one-channel tensors are FP32 cubes,
// 32-channel ones BF16 [voxel][32]. A thread owns output channel co = tid / (256 / COUT) and
// input channels ci0 .. ci0 + CPT - 1, ci0 = (tid % (256 / COUT)) * CPT.
template <int CIN, int COUT>
__global__ __launch_bounds__(kNT) void k_cnn_wgrad(CnnShape s, const void *xin, const void *gout,
                                                   float *part) {
  constexpr int TPC = kNT / COUT;
  constexpr int CPT = CIN >= TPC ? CIN / TPC : 1;
  const int co = threadIdx.x / TPC;
  const int ci0 = (threadIdx.x % TPC) * CPT;
  const bool live = ci0 < CIN;
  float acc[27][CPT];
  float accb = 0.f;
#pragma unroll
  for (int t = 0; t < 27; ++t)
#pragma unroll
    for (int k = 0; k < CPT; ++k) acc[t][k] = 0.f;
  const int chunk = (int)(((long long)s.N + gridDim.x - 1) / gridDim.x);
  const int beg = (int)min((long long)blockIdx.x * chunk, (long long)s.N);
  const int end = (int)min((long long)beg + chunk, (long long)s.N);
  if (beg < end) {
    Vox p = vox_of(beg, s);
    for (int e = beg; e < end; ++e, vox_next(p, s)) {
      float g;
      if constexpr (COUT == 1) g = reinterpret_cast<const float *>(gout)[e];
      else g = bf2f(reinterpret_cast<const uint16_t *>(gout)[(size_t)e * 32 + co]);
      if (g == 0.f) continue;  // masked by the ReLU: contributes nothing
      accb += g;
      if (!live) continue;
#pragma unroll
      for (int t = 0; t < 27; ++t) {
        const int q = neighbour(p, t, s, false);
        if (q < 0) continue;
        if constexpr (CIN == 1) {
          acc[t][0] = fmaf(g, reinterpret_cast<const float *>(xin)[q], acc[t][0]);
        } else if constexpr (CPT == 4) {
          const uint2 r = *reinterpret_cast<const uint2 *>(
              reinterpret_cast<const uint16_t *>(xin) + (size_t)q * 32 + ci0);
          acc[t][0] = fmaf(g, bf2f((uint16_t)(r.x & 0xffffu)), acc[t][0]);
          acc[t][1] = fmaf(g, bf2f((uint16_t)(r.x >> 16)), acc[t][1]);
          acc[t][2] = fmaf(g, bf2f((uint16_t)(r.y & 0xffffu)), acc[t][2]);
          acc[t][3] = fmaf(g, bf2f((uint16_t)(r.y >> 16)), acc[t][3]);
        } else {
#pragma unroll
          for (int k = 0; k < CPT; ++k)
            acc[t][k] = fmaf(
                g, bf2f(reinterpret_cast<const uint16_t *>(xin)[(size_t)q * 32 + ci0 + k]),
                acc[t][k]);
        }
      }
    }
  }
  // partial layout: [27][COUT][CIN] weights, then COUT biases
  float *pw = part + (size_t)blockIdx.x * (27 * COUT * CIN + COUT);
  if (live) {
#pragma unroll
    for (int t = 0; t < 27; ++t)
#pragma unroll
      for (int k = 0; k < CPT; ++k) pw[(t * COUT + co) * CIN + ci0 + k] = acc[t][k];
  }
  if (threadIdx.x % TPC == 0) pw[27 * COUT * CIN + co] = accb;
}

// out[k] = sum over the nparts partials of n floats, fixed order.
__global__ __launch_bounds__(kNT) void k_cnn_sum_parts(const float *part, int nparts, int n,
                                                       float *out) {
  for (int k = blockIdx.x * kNT + threadIdx.x; k < n; k += gridDim.x * kNT) {
    float a = 0.f;
    for (int p = 0; p < nparts; ++p) a += part[(size_t)p * n + k];
    out[k] = a;
  }
}

// ------------------------------------------------------------ Adam and working copies

__global__ __launch_bounds__(kNT) void k_cnn_adam(float *w, float *m, float *v, const float *g,
                                                  int n, float lr, float b1, float b2, float eps,
                                                  float c1, float c2) {
  for (int k = blockIdx.x * kNT + threadIdx.x; k < n; k += gridDim.x * kNT) {
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.f - b1) * gk;
    const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    w[k] -= lr * (mk * c1) / (sqrtf(vk * c2) + eps);
  }
}

// Working copies of the masters: the edge layers as BF16-rounded FP32 weights plus FP32
// biases; the 32 -> 32 weights as BF16 in forward order [t][co][ci] and transposed [t][ci][co]
// for the data gradient (skipped when bwd is null).
__global__ __launch_bounds__(kNT) void k_cnn_copies(const float *master, float *edge,
                                                    uint16_t *fwd, uint16_t *bwd) {
  for (int k = blockIdx.x * kNT + threadIdx.x; k < L::total; k += gridDim.x * kNT) {
    const float x = master[k];
    if (k < L::kEdge) {
      edge[k] = bf_round(x);
    } else if (k < L::kEdge + 32) {
      edge[k] = x;
    } else if (k >= L::out_b) {
      edge[L::edge_b4] = x;
    } else if (k >= L::out_w) {
      edge[L::edge_w4 + k - L::out_w] = bf_round(x);
    } else {
      const int l = (k - L::mid_w(0)) / (L::kMid + 32);
      const int o = k - L::mid_w(l);
      if (o < L::kMid) {
        const int t = o / 1024, co = (o / 32) % 32, ci = o % 32;
        const uint16_t h = f2bf(x);
        fwd[l * L::kMid + o] = h;
        if (bwd) bwd[l * L::kMid + t * 1024 + ci * 32 + co] = h;
      }
    }
  }
}

int grid_for(long long n, long long per_block) {
  long long g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > 65535) g = 65535;
  return (int)g;
}

}  // namespace

// ------------------------------------------------------------ launchers

hipError_t cnn_copies(const float *master, float *edge, uint16_t *fwd, uint16_t *bwd,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_cnn_copies, dim3(grid_for(L::total, kNT)), dim3(kNT), 0, st, master, edge,
                     fwd, bwd);
  return hipGetLastError();
}

hipError_t cnn_layer_in(const CnnShape &s, const float *v, const float *edge, uint16_t *out,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_cnn_in, dim3(grid_for(s.N, kNT)), dim3(kNT), 0, st, s, v, edge, out);
  return hipGetLastError();
}

hipError_t cnn_layer_mid(const CnnShape &s, const uint16_t *in, const uint16_t *W,
                         const float *bias, uint16_t *out, hipStream_t st) {
  hipLaunchKernelGGL(k_cnn_mid<0>, dim3(grid_for((s.N + 15) / 16, 4 * 8)), dim3(kNT), 0, st, s,
                     in, W, bias, (const uint16_t *)nullptr, out);
  return hipGetLastError();
}

hipError_t cnn_layer_mid_bwd(const CnnShape &s, const uint16_t *gin, const uint16_t *Wt,
                             const uint16_t *act, uint16_t *gout, hipStream_t st) {
  hipLaunchKernelGGL(k_cnn_mid<1>, dim3(grid_for((s.N + 15) / 16, 4 * 8)), dim3(kNT), 0, st, s,
                     gin, Wt, (const float *)nullptr, act, gout);
  return hipGetLastError();
}

int cnn_loss_parts(const CnnShape &s) {
  const int g = grid_for(s.N, 4 * kNT);
  return g > 1024 ? 1024 : g;
}

hipError_t cnn_layer_out(const CnnShape &s, const uint16_t *x, const float *edge,
                         const float *v, float *u, const float *target, float *du, double *part,
                         double *loss, hipStream_t st) {
  if (!target) {
    hipLaunchKernelGGL(k_cnn_out, dim3(grid_for(s.N, kNT)), dim3(kNT), 0, st, s, x, edge, v, u,
                       (const float *)nullptr, (float *)nullptr, (double *)nullptr);
    return hipGetLastError();
  }
  const int np = cnn_loss_parts(s);
  hipLaunchKernelGGL(k_cnn_out, dim3(np), dim3(kNT), 0, st, s, x, edge, v, u, target, du, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cnn_loss, dim3(1), dim3(kNT), 0, st, (const double *)part, np, s.N, loss);
  return hipGetLastError();
}

hipError_t cnn_layer_out_bwd(const CnnShape &s, const float *du, const float *edge,
                             const uint16_t *x, uint16_t *dx, hipStream_t st) {
  hipLaunchKernelGGL(k_cnn_out_bwd, dim3(grid_for(s.N, kNT)), dim3(kNT), 0, st, s, du, edge, x,
                     dx);
  return hipGetLastError();
}

int cnn_wgrad_parts(const CnnShape &s) {
  const int g = grid_for(s.N, 1024);
  return g > 1024 ? 1024 : g;
}

hipError_t cnn_wgrad(const CnnShape &s, int cin, int cout, const void *x, const void *g,
                     float *part, float *out, hipStream_t st) {
  const int np = cnn_wgrad_parts(s);
  if (cin == 1 && cout == 32)
    hipLaunchKernelGGL((k_cnn_wgrad<1, 32>), dim3(np), dim3(kNT), 0, st, s, x, g, part);
  else if (cin == 32 && cout == 32)
    hipLaunchKernelGGL((k_cnn_wgrad<32, 32>), dim3(np), dim3(kNT), 0, st, s, x, g, part);
  else if (cin == 32 && cout == 1)
    hipLaunchKernelGGL((k_cnn_wgrad<32, 1>), dim3(np), dim3(kNT), 0, st, s, x, g, part);
  else
    return hipErrorInvalidValue;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int n = 27 * cout * cin + cout;
  hipLaunchKernelGGL(k_cnn_sum_parts, dim3(grid_for(n, kNT)), dim3(kNT), 0, st,
                     (const float *)part, np, n, out);
  return hipGetLastError();
}

hipError_t cnn_adam(float *w, float *m, float *v, const float *g, int n, float lr, int step,
                    hipStream_t st) {
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 / (1.0 - pow(b1, step)));
  const float c2 = (float)(1.0 / (1.0 - pow(b2, step)));
  hipLaunchKernelGGL(k_cnn_adam, dim3(grid_for(n, kNT)), dim3(kNT), 0, st, w, m, v, g, n, lr,
                     (float)b1, (float)b2, 1e-8f, c1, c2);
  return hipGetLastError();
}

}  // namespace s3ttv
