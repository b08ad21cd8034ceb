// Learned initial estimate u0 for Alg. 1, whose initial values are free (Prob. (18) is convex:
// the start changes the iteration count, not the solution). A five-layer 3-D convolutional
// network computes u0 = v + f(v), f = C4 o R o C3 o R o C2 o R o C1 o R o C0, each C a 3x3x3
// convolution with bias and zero padding (channels 1 -> 32 -> 32 -> 32 -> 32 -> 1), R = ReLU.
// Weights: FP32 masters (Adam), BF16 working copies; biases FP32. Activations and their
// gradients are stored in BF16, channels-last ([voxel][32]); every sum is formed in FP32.
//
// The 32 -> 32 layers are implicit GEMMs on v_mfma_f32_16x16x32_bf16 with the 32 input
// channels as K: workgroups stage the 9 neighbour lines of a 32-band chunk in LDS and each
// wave keeps the weights of its taps in registers. The data gradient of these layers runs
// through the same kernel with a mirrored, transposed weight copy; their weight gradient is a
// contraction over voxels on the same MFMA from LDS tiles transposed to [channel][band]. The
// 1 -> 32 and 32 -> 1 layers and their weight gradients run on FP32 VALU. Weight gradients are
// summed per workgroup over a fixed range and then over workgroups in a fixed order, so every
// result is reproducible.
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

constexpr int kCB = 32;       // bands per chunk of the 32 -> 32 convolution
constexpr int kXS = 40;       // LDS row stride (elements) of a staged voxel: 32 channels + 8
constexpr int kRS = 33;       // row stride (floats) of the wave-partial tile

// MODE 0 (forward):       out = relu(conv(in, W) + bias)
// MODE 1 (data gradient): out = (act > 0) * conv(in, W), W the mirrored transposed copy
//                         (tap 26 - t, [ci][co]), which turns the adjoint into a plain
//                         convolution.
// W: BF16 [27][32 (output channel n)][32 (input channel k)]. A workgroup takes a contiguous
// range of chunks (32 bands b0 .. b0 + 31 of one line (i, j)). Per chunk it stages the 9
// neighbour lines, bands b0 - 1 .. b0 + 32, channels-last in LDS; wave w owns the taps
// t = w, w + 4, ... and keeps their weights in registers for the whole range (B operand:
// lane (n, kb) holds W[t][n][8kb .. 8kb + 7]). A tap is then, per 16-band half and 16-channel
// half, one MFMA whose A operand (lane (m, kb): channels 8kb .. 8kb + 7 of band b0 + m + db of
// line t / 3) is one 16-byte LDS read. The four waves' partial tiles are summed in LDS in a
// fixed order and the epilogue (bias + ReLU, or the ReLU mask) writes 8 bytes per thread.
template <int MODE>
__global__ __launch_bounds__(kNT) void k_cnn_conv32(CnnShape s, const uint16_t *in,
                                                    const uint16_t *W, const float *bias,
                                                    const uint16_t *act, uint16_t *out) {
  __shared__ __align__(16) uint16_t xs[9 * (kCB + 2) * kXS];
  __shared__ float red[4][kCB * kRS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, kb = lane >> 4;
  bf8 wb[7][2];
#pragma unroll
  for (int m = 0; m < 7; ++m) {
    const int t = wave + 4 * m < 27 ? wave + 4 * m : 26;
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
      wb[m][nt] = *reinterpret_cast<const bf8 *>(W + (t * 32 + nt * 16 + li) * 32 + 8 * kb);
  }
  // epilogue ownership: voxel ev = tid / 8 of the chunk, channels 4 ec .. 4 ec + 3
  const int ev = tid >> 3, ec = tid & 7;
  float bv[4] = {0.f, 0.f, 0.f, 0.f};
  if (MODE == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) bv[k] = bias[4 * ec + k];
  }
  const int cpl = (s.n3 + kCB - 1) / kCB;
  const long long nchunks = (long long)s.nb * s.n1 * s.n2 * cpl;
  const long long c0 = nchunks * blockIdx.x / gridDim.x;
  const long long c1 = nchunks * (blockIdx.x + 1) / gridDim.x;
  const uint4 zero4 = make_uint4(0u, 0u, 0u, 0u);
  for (long long c = c0; c < c1; ++c) {
    const int line = (int)(c / cpl);
    const int b0 = (int)(c - (long long)line * cpl) * kCB;
    const int i = line / s.n2, j = line - i * s.n2, il = i % s.n1;
    __syncthreads();  // xs and red of the previous chunk are no longer read
    for (int task = tid; task < 9 * (kCB + 2) * 4; task += kNT) {
      const int r = task / ((kCB + 2) * 4), rem = task - r * ((kCB + 2) * 4);
      const int k = rem >> 2, q = rem & 3;
      const int di = r / 3 - 1, dj = r % 3 - 1, bb = b0 - 1 + k;
      const bool ok = il + di >= 0 && il + di < s.n1 && j + dj >= 0 && j + dj < s.n2 &&
                      bb >= 0 && bb < s.n3;
      uint4 val = zero4;
      if (ok)
        val = *reinterpret_cast<const uint4 *>(
            in + ((size_t)((i + di) * s.n2 + (j + dj)) * s.n3 + bb) * 32 + 8 * q);
      *reinterpret_cast<uint4 *>(xs + (r * (kCB + 2) + k) * kXS + 8 * q) = val;
    }
    __syncthreads();
    f4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int m = 0; m < 7; ++m) {
      const int t = wave + 4 * m;
      if (t < 27) {
        const int r = t / 3, d = t % 3;  // band b0 + m' + db sits at staged index m' + d
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
          const bf8 a = *reinterpret_cast<const bf8 *>(
              xs + (r * (kCB + 2) + mt * 16 + li + d) * kXS + 8 * kb);
          acc[mt][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, wb[m][0], acc[mt][0], 0, 0, 0);
          acc[mt][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, wb[m][1], acc[mt][1], 0, 0, 0);
        }
      }
    }
    // result lane (c = li, g = kb), register rr: band mt*16 + 4g + rr, channel nt*16 + c
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
          red[wave][(mt * 16 + 4 * kb + rr) * kRS + nt * 16 + li] = acc[mt][nt][rr];
    __syncthreads();
    const int bb = b0 + ev;
    if (bb < s.n3) {
      const size_t e = (size_t)line * s.n3 + bb;
      float y[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int o = ev * kRS + 4 * ec + k;
        y[k] = ((red[0][o] + red[1][o]) + (red[2][o] + red[3][o])) + bv[k];
      }
      if (MODE == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) y[k] = fmaxf(y[k], 0.f);
      } else {
        const uint2 am = *reinterpret_cast<const uint2 *>(act + e * 32 + 4 * ec);
        if (!(bf2f((uint16_t)(am.x & 0xffffu)) > 0.f)) y[0] = 0.f;
        if (!(bf2f((uint16_t)(am.x >> 16)) > 0.f)) y[1] = 0.f;
        if (!(bf2f((uint16_t)(am.y & 0xffffu)) > 0.f)) y[2] = 0.f;
        if (!(bf2f((uint16_t)(am.y >> 16)) > 0.f)) y[3] = 0.f;
      }
      *reinterpret_cast<uint2 *>(out + e * 32 + 4 * ec) =
          make_uint2((uint32_t)f2bf(y[0]) | ((uint32_t)f2bf(y[1]) << 16),
                     (uint32_t)f2bf(y[2]) | ((uint32_t)f2bf(y[3]) << 16));
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

constexpr int kWC = 32;  // bands per chunk of the 32 -> 32 weight gradient
constexpr int kTS = 40;  // LDS row stride (elements) of its transposed tiles: 32 + 8 padding

__device__ inline uint32_t half_of(const uint4 &a, int h) {
  const uint32_t w = h < 2 ? a.x : h < 4 ? a.y : h < 6 ? a.z : a.w;
  return (h & 1) ? (w >> 16) : (w & 0xffffu);
}
// Channels 8q..8q+7 of two consecutive voxels (k, k+1) -> column pair (k, k+1) of rows
// 8q..8q+7 of a [channel][k] tile (row stride kTS elements). dst points at row 8q, column k.
__device__ inline void put_pair_transposed(uint16_t *dst, const uint4 &va, const uint4 &vb) {
  uint32_t *d = reinterpret_cast<uint32_t *>(dst);
#pragma unroll
  for (int h = 0; h < 8; ++h) d[h * (kTS / 2)] = half_of(va, h) | (half_of(vb, h) << 16);
}

// 32 -> 32 layers, on MFMA: dW[t][co][ci] = sum_e g[e][co] x[e + off_t][ci] and
// db[co] = sum_e g[e][co], partial over the workgroup's chunks. A chunk is 32 consecutive
// bands b' = b0 .. b0 + 31 of one line (i, j); with t = (di, dj, db) its contribution is
//   sum_k g[(i, j), b0 + k - db][co] * x[(i + di, j + dj), b0 + k][ci],
// a 32 x 32 x 32 (co x ci x k) contraction. LDS holds the 9 neighbour lines of x and three
// band-shifted copies of the g line, both transposed to [channel][k] so that every MFMA
// operand is one 16-byte read (g as A with rows co, x as B with columns ci, K = k). Values
// beyond the volume (or the band range) are zero, so each pair (e, e + off_t) inside the
// volume is counted exactly once. Wave w owns the taps t = w, w + 4, ..., so its 7 taps x 4
// output blocks stay in registers for the whole chunk range.
__global__ __launch_bounds__(kNT) void k_cnn_wgrad_mid(CnnShape s, const uint16_t *x,
                                                       const uint16_t *g, float *part) {
  __shared__ __align__(16) uint16_t xs[9 * 32 * kTS];  // [neighbour line r = t / 3][ci][k]
  __shared__ __align__(16) uint16_t gs[3 * 32 * kTS];  // [band shift d = t % 3][co][k]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, kb = lane >> 4;
  const int cpl = (s.n3 + kWC - 1) / kWC;
  const long long nchunks = (long long)s.nb * s.n1 * s.n2 * cpl;
  const long long c0 = nchunks * blockIdx.x / gridDim.x;
  const long long c1 = nchunks * (blockIdx.x + 1) / gridDim.x;
  f4 acc[7][2][2];
#pragma unroll
  for (int m = 0; m < 7; ++m)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[m][a][b] = f4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;
  const uint4 zero4 = make_uint4(0u, 0u, 0u, 0u);
  for (long long c = c0; c < c1; ++c) {
    const int line = (int)(c / cpl);
    const int b0 = (int)(c - (long long)line * cpl) * kWC;
    const int i = line / s.n2, j = line - i * s.n2, il = i % s.n1;
    __syncthreads();  // the previous chunk's operands have been read
    for (int task = tid; task < 9 * 64; task += kNT) {
      const int r = task >> 6, kp = (task >> 2) & 15, q = task & 3;
      const int di = r / 3 - 1, dj = r % 3 - 1;
      const bool ok = il + di >= 0 && il + di < s.n1 && j + dj >= 0 && j + dj < s.n2;
      const int bb = b0 + 2 * kp;
      const size_t base = ok ? (size_t)(((i + di) * s.n2 + (j + dj)) * s.n3) : 0;
      const uint4 va = ok && bb < s.n3 ? *reinterpret_cast<const uint4 *>(x + (base + bb) * 32 + 8 * q)
                                       : zero4;
      const uint4 vb = ok && bb + 1 < s.n3
                           ? *reinterpret_cast<const uint4 *>(x + (base + bb + 1) * 32 + 8 * q)
                           : zero4;
      put_pair_transposed(xs + (r * 32 + 8 * q) * kTS + 2 * kp, va, vb);
    }
    for (int task = tid; task < 3 * 64; task += kNT) {
      const int d = task >> 6, kp = (task >> 2) & 15, q = task & 3;
      const int bb = b0 + 2 * kp - (d - 1);
      const size_t base = (size_t)line * s.n3;
      const uint4 va = bb >= 0 && bb < s.n3
                           ? *reinterpret_cast<const uint4 *>(g + (base + bb) * 32 + 8 * q)
                           : zero4;
      const uint4 vb = bb + 1 >= 0 && bb + 1 < s.n3
                           ? *reinterpret_cast<const uint4 *>(g + (base + bb + 1) * 32 + 8 * q)
                           : zero4;
      put_pair_transposed(gs + (d * 32 + 8 * q) * kTS + 2 * kp, va, vb);
    }
    __syncthreads();
    if (tid < 32) {
#pragma unroll
      for (int k = 0; k < kWC; ++k) bsum += bf2f(gs[(32 + tid) * kTS + k]);
    }
#pragma unroll
    for (int m = 0; m < 7; ++m) {
      const int t = wave + 4 * m;
      if (t < 27) {
        const int r = t / 3, d = t % 3;
        const bf8 a0 = *reinterpret_cast<const bf8 *>(gs + (d * 32 + li) * kTS + 8 * kb);
        const bf8 a1 = *reinterpret_cast<const bf8 *>(gs + (d * 32 + 16 + li) * kTS + 8 * kb);
        const bf8 x0 = *reinterpret_cast<const bf8 *>(xs + (r * 32 + li) * kTS + 8 * kb);
        const bf8 x1 = *reinterpret_cast<const bf8 *>(xs + (r * 32 + 16 + li) * kTS + 8 * kb);
        acc[m][0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, x0, acc[m][0][0], 0, 0, 0);
        acc[m][0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, x1, acc[m][0][1], 0, 0, 0);
        acc[m][1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, x0, acc[m][1][0], 0, 0, 0);
        acc[m][1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, x1, acc[m][1][1], 0, 0, 0);
      }
    }
  }
  // result lane (column li, group kb), register rr: co = 16 coh + 4 kb + rr, ci = 16 cih + li
  float *pw = part + (size_t)blockIdx.x * (L::kMid + 32);
#pragma unroll
  for (int m = 0; m < 7; ++m) {
    const int t = wave + 4 * m;
    if (t < 27) {
#pragma unroll
      for (int coh = 0; coh < 2; ++coh)
#pragma unroll
        for (int cih = 0; cih < 2; ++cih)
#pragma unroll
          for (int rr = 0; rr < 4; ++rr)
            pw[(t * 32 + 16 * coh + 4 * kb + rr) * 32 + 16 * cih + li] = acc[m][coh][cih][rr];
    }
  }
  if (tid < 32) pw[L::kMid + tid] = bsum;
}

// 1 -> 32 (IN1: x = v, FP32; g BF16 [voxel][32]) and 32 -> 1 (x BF16 [voxel][32]; g = du,
// FP32) layers: dW[t][c] = sum_e g[e](c) x[e + off_t](c), the 32-channel side indexed by c,
// and the biases, partial over the workgroup's chunks (32 bands of one line, as in the
// 32 -> 32 kernel). LDS holds the one-channel side with a band halo of one (IN1: v on the 9
// neighbour lines; else du on the line itself) and the 32-channel side channels-last (IN1:
// g on the line; else x on the 9 neighbour lines). Thread (c = tid % 32, sub = tid / 32) owns
// the taps t = sub, sub + 8, ...
template <bool IN1>
__global__ __launch_bounds__(kNT) void k_cnn_wgrad_edge(CnnShape s, const void *xin,
                                                        const void *gin, float *part) {
  __shared__ float one[9][kWC + 2];
  __shared__ __align__(16) uint16_t many[9][kWC][32];
  const int tid = threadIdx.x, c = tid & 31, sub = tid >> 5;
  const int cpl = (s.n3 + kWC - 1) / kWC;
  const long long nchunks = (long long)s.nb * s.n1 * s.n2 * cpl;
  const long long c0 = nchunks * blockIdx.x / gridDim.x;
  const long long c1 = nchunks * (blockIdx.x + 1) / gridDim.x;
  const float *one_src = reinterpret_cast<const float *>(IN1 ? xin : gin);
  const uint16_t *many_src = reinterpret_cast<const uint16_t *>(IN1 ? gin : xin);
  constexpr int kLines1 = IN1 ? 9 : 1;   // lines of the one-channel side
  constexpr int kLinesM = IN1 ? 1 : 9;   // lines of the 32-channel side
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  float accb = 0.f;
  const uint4 zero4 = make_uint4(0u, 0u, 0u, 0u);
  for (long long ch = c0; ch < c1; ++ch) {
    const int line = (int)(ch / cpl);
    const int b0 = (int)(ch - (long long)line * cpl) * kWC;
    const int i = line / s.n2, j = line - i * s.n2, il = i % s.n1;
    __syncthreads();
    for (int task = tid; task < kLines1 * (kWC + 2); task += kNT) {
      const int r = task / (kWC + 2), k = task - r * (kWC + 2);
      const int di = IN1 ? r / 3 - 1 : 0, dj = IN1 ? r % 3 - 1 : 0;
      const int bb = b0 - 1 + k;
      const bool ok = il + di >= 0 && il + di < s.n1 && j + dj >= 0 && j + dj < s.n2 &&
                      bb >= 0 && bb < s.n3;
      one[r][k] = ok ? one_src[((i + di) * s.n2 + (j + dj)) * s.n3 + bb] : 0.f;
    }
    for (int task = tid; task < kLinesM * kWC * 4; task += kNT) {
      const int r = task / (kWC * 4), k = (task >> 2) % kWC, q = task & 3;
      const int di = IN1 ? 0 : r / 3 - 1, dj = IN1 ? 0 : r % 3 - 1;
      const int bb = b0 + k;
      const bool ok = il + di >= 0 && il + di < s.n1 && j + dj >= 0 && j + dj < s.n2 &&
                      bb < s.n3;
      uint4 val = zero4;
      if (ok)
        val = *reinterpret_cast<const uint4 *>(
            many_src + ((size_t)((i + di) * s.n2 + (j + dj)) * s.n3 + bb) * 32 + 8 * q);
      reinterpret_cast<uint4 *>(&many[r][k][0])[q] = val;
    }
    __syncthreads();
    // the 32-channel operand of the line (IN1) stays in registers for all taps; the other
    // operands are read from LDS (the band shift d varies per thread, so it indexes LDS)
    float reg[kWC];
    if constexpr (IN1) {
#pragma unroll
      for (int k = 0; k < kWC; ++k) reg[k] = bf2f(many[0][k][c]);
      if (sub == 0) {
#pragma unroll
        for (int k = 0; k < kWC; ++k) accb += reg[k];
      }
    } else if (tid == 0) {
#pragma unroll
      for (int k = 1; k <= kWC; ++k) accb += one[0][k];
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int t = sub + 8 * m;
      if (t < 27) {
        const int r = t / 3, d = t % 3;  // d = db + 1
        float a = 0.f;
        if constexpr (IN1) {
          // g at band b0 + k of the line, v at band b0 + k + db of neighbour line r
#pragma unroll
          for (int k = 0; k < kWC; ++k) a = fmaf(reg[k], one[r][k + d], a);
        } else {
          // du at band b0 + k - db of the line, x at band b0 + k of neighbour line r
#pragma unroll
          for (int k = 0; k < kWC; ++k) a = fmaf(one[0][k + 2 - d], bf2f(many[r][k][c]), a);
        }
        acc[m] += a;
      }
    }
  }
  // partial layout: 864 weights (index t * 32 + c in both layers), then 32 (IN1) or 1 bias
  float *pw = part + (size_t)blockIdx.x * (IN1 ? L::kEdge + 32 : L::kEdge + 1);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int t = sub + 8 * m;
    if (t < 27) pw[t * 32 + c] = acc[m];
  }
  if (IN1 ? sub == 0 : tid == 0) pw[L::kEdge + (IN1 ? c : 0)] = accb;
}

// out[o] = sum over the nparts partials (each n floats), in a fixed order: 16 slices of the
// parts per output (four interleaved running sums each), combined in LDS.
__global__ __launch_bounds__(1024) void k_cnn_sum_parts(const float *part, int nparts, int n,
                                                        float *out) {
  __shared__ float red[16][64];
  const int lane = threadIdx.x & 63, sl = threadIdx.x >> 6;
  const int o = blockIdx.x * 64 + lane;
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
  if (o < n) {
    int p = sl;
    for (; p + 48 < nparts; p += 64) {
      a0 += part[(size_t)p * n + o];
      a1 += part[(size_t)(p + 16) * n + o];
      a2 += part[(size_t)(p + 32) * n + o];
      a3 += part[(size_t)(p + 48) * n + o];
    }
    for (; p < nparts; p += 16) a0 += part[(size_t)p * n + o];
  }
  red[sl][lane] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  if (sl == 0 && o < n) {
    float a = 0.f;
#pragma unroll
    for (int k = 0; k < 16; ++k) a += red[k][lane];
    out[o] = a;
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
// biases; the 32 -> 32 weights as BF16 in forward order [t][co][ci] and, for the data
// gradient, mirrored and transposed: bwd[26 - t][ci][co] = W[t][co][ci] (skipped when bwd is
// null).
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
        if (bwd) bwd[l * L::kMid + (26 - t) * 1024 + ci * 32 + co] = h;
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

namespace {
int conv32_grid(const CnnShape &s) {
  const long long chunks = (long long)s.nb * s.n1 * s.n2 * ((s.n3 + kCB - 1) / kCB);
  const long long g = (chunks + 3) / 4;
  return (int)(g < 1 ? 1 : g > 4096 ? 4096 : g);
}
}  // namespace

hipError_t cnn_layer_mid(const CnnShape &s, const uint16_t *in, const uint16_t *W,
                         const float *bias, uint16_t *out, hipStream_t st) {
  hipLaunchKernelGGL(k_cnn_conv32<0>, dim3(conv32_grid(s)), dim3(kNT), 0, st, s, in, W, bias,
                     (const uint16_t *)nullptr, out);
  return hipGetLastError();
}

hipError_t cnn_layer_mid_bwd(const CnnShape &s, const uint16_t *gin, const uint16_t *Wt,
                             const uint16_t *act, uint16_t *gout, hipStream_t st) {
  hipLaunchKernelGGL(k_cnn_conv32<1>, dim3(conv32_grid(s)), dim3(kNT), 0, st, s, gin, Wt,
                     (const float *)nullptr, act, gout);
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

namespace {
int mid_parts(const CnnShape &s) {
  const long long chunks = (long long)s.nb * s.n1 * s.n2 * ((s.n3 + kWC - 1) / kWC);
  const long long p = (chunks + 31) / 32;
  return (int)(p < 1 ? 1 : p > 1024 ? 1024 : p);
}
int edge_parts(const CnnShape &s) {
  const long long chunks = (long long)s.nb * s.n1 * s.n2 * ((s.n3 + kWC - 1) / kWC);
  const long long p = (chunks + 15) / 16;
  return (int)(p < 1 ? 1 : p > 4096 ? 4096 : p);
}
}  // namespace

size_t cnn_wgrad_part_floats(const CnnShape &s) {
  const size_t a = (size_t)mid_parts(s) * (L::kMid + 32);
  const size_t b = (size_t)edge_parts(s) * (L::kEdge + 32);
  return a > b ? a : b;
}

hipError_t cnn_wgrad(const CnnShape &s, int cin, int cout, const void *x, const void *g,
                     float *part, float *out, hipStream_t st) {
  int np;
  if (cin == 32 && cout == 32) {
    np = mid_parts(s);
    hipLaunchKernelGGL(k_cnn_wgrad_mid, dim3(np), dim3(kNT), 0, st, s, (const uint16_t *)x,
                       (const uint16_t *)g, part);
  } else if (cin == 1 && cout == 32) {
    np = edge_parts(s);
    hipLaunchKernelGGL(k_cnn_wgrad_edge<true>, dim3(np), dim3(kNT), 0, st, s, x, g, part);
  } else if (cin == 32 && cout == 1) {
    np = edge_parts(s);
    hipLaunchKernelGGL(k_cnn_wgrad_edge<false>, dim3(np), dim3(kNT), 0, st, s, x, g, part);
  } else {
    return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int n = 27 * cout * cin + cout;
  hipLaunchKernelGGL(k_cnn_sum_parts, dim3((n + 63) / 64), dim3(1024), 0, st, (const float *)part,
                     np, n, out);
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
