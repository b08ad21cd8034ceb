// Voxel-wise and stencil kernels of Alg. 1 (arXiv 2404.03313) for gfx950.
//
// Layouts: cubes are (N1, N2, N3) band fastest; the two-component gradient / overlap-add
// fields are [pixel][ncol] with column c = comp*Bp + band (comp 0 = D_v D_s, 1 = D_h D_s),
// padded bands zero. All global sums are accumulated in FP64 per workgroup and reduced in a
// fixed order by one workgroup, so every run is bitwise reproducible.
#include "s3ttv_internal.h"

namespace s3ttv {

namespace {

constexpr int kNT = 256;  // threads per workgroup of the voxel kernels

__device__ inline int wrap_up(int a, int n) { return a >= n ? a - n : a; }
__device__ inline int wrap_dn(int a, int n) { return a < 0 ? a + n : a; }

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over a 256-thread workgroup in a fixed order; result valid in thread 0.
__device__ inline double block_sum(double v, double *sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  return r;
}

__device__ inline double block_max(double v, double *sh) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m));
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0) r = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
  return r;
}

__device__ inline float box(float x, float lo, float hi) { return x < lo ? lo : (x > hi ? hi : x); }

// Soft threshold with an FP64 threshold; the difference is formed in double and rounded once.
__device__ inline float soft(float x, double tau) {
  const double a = fabs((double)x) - tau;
  return a > 0 ? copysignf((float)a, x) : 0.0f;
}

// Histogram key of |x| for the level-1 l1 selection: bin = bits 30..20, significand of the
// value (implicit bit included for normal numbers).
__device__ inline void l1_acc(unsigned long long *h, float x) {
  const uint32_t bits = __float_as_uint(x) & 0x7fffffffu;
  const uint32_t e = bits >> 23;
  const uint32_t sig = e ? ((bits & 0x7fffffu) | 0x800000u) : (bits & 0x7fffffu);
  atomicAdd(&h[bits >> kL1Shift1], (1ull << 40) | (unsigned long long)sig);
}

__device__ inline void l1_flush(const unsigned long long *h, int nb, uint32_t *gcnt,
                                unsigned long long *gsig) {
  for (int k = threadIdx.x; k < nb; k += blockDim.x) {
    const unsigned long long v = h[k];
    if (v) {
      atomicAdd(&gcnt[k], (uint32_t)(v >> 40));
      atomicAdd(&gsig[k], v & ((1ull << 40) - 1));
    }
  }
}

// ---------------------------------------------------------------- primal step

struct PrimalArgs {
  int n1, n2, n3, Bp, ncol;
  long long N;
  float g_u, g_s, g_t, lo, hi;
  const float *u, *s, *t, *y2, *w, *Z;
  const int *zpart, *zslot;  // with zslot: read the overlap-add partials instead of Z
  const float *Z2;           // second dual field (HSSTV), same layout as Z
  float omega;               // its weight
  float *un, *xs, *xt;
  double *red;
  DevScalars *sc;
  L1Hist *hist;
};

// Overlap-add field value at column col of a pixel from its four partial slots, given as
// element offsets into zpart (fixed point; unused entries name an all-zero slot, so the loads
// carry no branches).
__device__ inline float zfold_val(const int *zpart, int4 off, int col) {
  const int acc = (zpart[off.x + col] + zpart[off.y + col]) + (zpart[off.z + col] + zpart[off.w + col]);
  return (float)acc * kZInv;
}

// The same for the four columns col .. col + 3 (col a multiple of 4: 16-byte loads).
__device__ inline float4 zfold_val4(const int *zpart, int4 off, int col) {
  const int4 a = *reinterpret_cast<const int4 *>(zpart + off.x + col);
  const int4 b = *reinterpret_cast<const int4 *>(zpart + off.y + col);
  const int4 c = *reinterpret_cast<const int4 *>(zpart + off.z + col);
  const int4 d = *reinterpret_cast<const int4 *>(zpart + off.w + col);
  return make_float4((float)((a.x + b.x) + (c.x + d.x)) * kZInv, (float)((a.y + b.y) + (c.y + d.y)) * kZInv,
                     (float)((a.z + b.z) + (c.z + d.z)) * kZInv, (float)((a.w + b.w) + (c.w + d.w)) * kZInv);
}

// Alg. 1 steps 2-4 before the l1 projections:
//   u+ = P_box(u - g_u (D_s^T (D_v^T Zv + D_h^T Zh) + y3))        (eq. prox_box_constraint)
//   xs = s - g_s y3,   xt = t - g_t (D_v^T y2 + y3),   y3 = kappa * w.
// MODE 0: the field is adjoined by D_s^T D^T (S3TTV: the overlap-add sum of the blocks; SSTV:
// the dual field itself); MODE 1: by D^T (STV); MODE 2: D_s^T D^T Z + omega D^T Z2 (HSSTV);
// MODE 3: as MODE 0 from the partial slots, four bands per thread; MODE 4: the three-component
// field by D_v^T Zv + D_h^T Zh + D_s^T Zs (SSST).
template <int MODE>
__global__ __launch_bounds__(kNT) void k_primal(PrimalArgs a) {
  __shared__ unsigned long long h[2][kL1Bins1];
  __shared__ double sh[4];
  if (a.sc->done) return;
  for (int k = threadIdx.x; k < 2 * kL1Bins1; k += kNT) (&h[0][0])[k] = 0ull;
  __syncthreads();
  const float kappa = (float)a.sc->kappa;
  double du2 = 0, u2 = 0, bad = 0;
  const int n2 = a.n2, n3 = a.n3, ncol = a.ncol, Bp = a.Bp;
  // MODE 3 (S3TTV with the partial-slot table, N3 divisible by 4, 16-byte aligned arrays): a
  // thread takes four consecutive bands of one pixel, so the partials come in 16-byte loads
  // and column b - 1 of band b is the previous band's column b (one halo column per quad).
  // Same arithmetic per voxel as MODE 0; a separate instance, so that the other modes keep
  // their register budget.
  constexpr bool quads = MODE == 3;
  const long long NQ = quads ? a.N >> 2 : 0;
  // two quads per trip, all of their loads issued before any arithmetic: the slot tables,
  // then the partials and the voxel values (a trip's stores would otherwise hold back the next
  // trip's loads)
  const long long qstride = (long long)gridDim.x * kNT;
  for (long long q0 = (long long)blockIdx.x * kNT + threadIdx.x; q0 < NQ; q0 += 2 * qstride) {
    const int nq = n3 >> 2;
    long long qd[2] = {q0, q0 + qstride};
    const bool on1 = qd[1] < NQ;
    if (!on1) qd[1] = q0;  // loads repeat the first quad; the second is then skipped
    uint32_t pix[2], pim[2], pjm[2];
    int b0[2], bm[2];
    int4 sp[2], si[2], sj[2];
#pragma unroll
    for (int h2 = 0; h2 < 2; ++h2) {
      pix[h2] = (uint32_t)(qd[h2] / nq);
      b0[h2] = (int)(qd[h2] - (long long)pix[h2] * nq) * 4;
      const int i = (int)(pix[h2] / (uint32_t)n2), j = (int)(pix[h2] - (uint32_t)i * n2);
      bm[h2] = wrap_dn(b0[h2] - 1, n3);
      pim[h2] = (uint32_t)(wrap_dn(i - 1, a.n1) * n2 + j);
      pjm[h2] = (uint32_t)(i * n2 + wrap_dn(j - 1, n2));
      sp[h2] = reinterpret_cast<const int4 *>(a.zslot)[pix[h2]];
      si[h2] = reinterpret_cast<const int4 *>(a.zslot)[pim[h2]];
      sj[h2] = reinterpret_cast<const int4 *>(a.zslot)[pjm[h2]];
    }
    float4 vi[2], vp[2], hj[2], hp[2], w4[2], u4[2], s4[2], t4[2], ye[2], ym[2];
    float Q0[2];
    const bool halo[2] = {(threadIdx.x & 63) == 0 || b0[0] == 0, (threadIdx.x & 63) == 0 || b0[1] == 0};
#pragma unroll
    for (int h2 = 0; h2 < 2; ++h2) {
      vi[h2] = zfold_val4(a.zpart, si[h2], b0[h2]);
      vp[h2] = zfold_val4(a.zpart, sp[h2], b0[h2]);
      hj[h2] = zfold_val4(a.zpart, sj[h2], Bp + b0[h2]);
      hp[h2] = zfold_val4(a.zpart, sp[h2], Bp + b0[h2]);
      // Column b0 - 1 is the last column of the previous lane's quad (the same pixel's bands
      // b0 - 4 .. b0 - 1), taken by a shuffle below, except where the quad starts its pixel
      // (the column wraps to band n3 - 1) or the wavefront; only those lanes gather it here,
      // the others all read word 0 (one cache line) and discard it.
      {
        const int4 z0 = make_int4(0, 0, 0, 0);
        const int4 hi_ = halo[h2] ? si[h2] : z0, hp_ = halo[h2] ? sp[h2] : z0,
                   hj_ = halo[h2] ? sj[h2] : z0;
        const int cv = halo[h2] ? bm[h2] : 0, ch = halo[h2] ? Bp + bm[h2] : 0;
        Q0[h2] = (zfold_val(a.zpart, hi_, cv) - zfold_val(a.zpart, hp_, cv)) +
                 (zfold_val(a.zpart, hj_, ch) - zfold_val(a.zpart, hp_, ch));
      }
      const long long e0 = qd[h2] * 4;
      w4[h2] = *reinterpret_cast<const float4 *>(a.w + e0);
      u4[h2] = *reinterpret_cast<const float4 *>(a.u + e0);
      s4[h2] = *reinterpret_cast<const float4 *>(a.s + e0);
      t4[h2] = *reinterpret_cast<const float4 *>(a.t + e0);
      ye[h2] = *reinterpret_cast<const float4 *>(a.y2 + e0);
      ym[h2] = *reinterpret_cast<const float4 *>(a.y2 + (size_t)pim[h2] * n3 + b0[h2]);
    }
    // the last column of every quad, passed one lane up (a lane whose previous quad is in
    // the loop is itself in the loop, also at the tail, so every read is of an active lane)
#pragma unroll
    for (int h2 = 0; h2 < 2; ++h2) {
      const float last = (vi[h2].w - vp[h2].w) + (hj[h2].w - hp[h2].w);
      const float prev = __shfl_up(last, 1, 64);
      if (!halo[h2]) Q0[h2] = prev;
    }
#pragma unroll
    for (int h2 = 0; h2 < 2; ++h2) {
      if (h2 == 1 && !on1) break;
      // Q(c) = (D_v^T Zv + D_h^T Zh)(c) for c = b0 - 1, b0 .. b0 + 3
      const float Q[5] = {Q0[h2], (vi[h2].x - vp[h2].x) + (hj[h2].x - hp[h2].x),
                          (vi[h2].y - vp[h2].y) + (hj[h2].y - hp[h2].y),
                          (vi[h2].z - vp[h2].z) + (hj[h2].z - hp[h2].z),
                          (vi[h2].w - vp[h2].w) + (hj[h2].w - hp[h2].w)};
      const float wv[4] = {w4[h2].x, w4[h2].y, w4[h2].z, w4[h2].w};
      const float uv[4] = {u4[h2].x, u4[h2].y, u4[h2].z, u4[h2].w};
      const float sv[4] = {s4[h2].x, s4[h2].y, s4[h2].z, s4[h2].w};
      const float tv[4] = {t4[h2].x, t4[h2].y, t4[h2].z, t4[h2].w};
      const float yev[4] = {ye[h2].x, ye[h2].y, ye[h2].z, ye[h2].w};
      const float ymv[4] = {ym[h2].x, ym[h2].y, ym[h2].z, ym[h2].w};
      float unv[4], xsv[4], xtv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float adj = Q[k] - Q[k + 1];  // adjoint of D_s: q(b - 1) - q(b)
        const float y3 = kappa * wv[k];
        const float uo = uv[k];
        const float un = box(uo - a.g_u * (adj + y3), a.lo, a.hi);
        const float xs = sv[k] - a.g_s * y3;
        const float xt = tv[k] - a.g_t * ((ymv[k] - yev[k]) + y3);
        unv[k] = un;
        xsv[k] = xs;
        xtv[k] = xt;
        const double d = (double)un - (double)uo;
        du2 += d * d;
        u2 += (double)uo * (double)uo;
        if (!(isfinite(un) && isfinite(xs) && isfinite(xt))) bad = 1;
        l1_acc(h[0], xs);
        l1_acc(h[1], xt);
      }
      const long long e0 = qd[h2] * 4;
      *reinterpret_cast<float4 *>(a.un + e0) = make_float4(unv[0], unv[1], unv[2], unv[3]);
      *reinterpret_cast<float4 *>(a.xs + e0) = make_float4(xsv[0], xsv[1], xsv[2], xsv[3]);
      *reinterpret_cast<float4 *>(a.xt + e0) = make_float4(xtv[0], xtv[1], xtv[2], xtv[3]);
    }
  }
  for (long long e = (long long)blockIdx.x * kNT + threadIdx.x; e < (quads ? 0 : a.N);
       e += (long long)gridDim.x * kNT) {
    const uint32_t pix = (uint32_t)(e / n3);
    const int b = (int)(e - (long long)pix * n3);
    const int i = (int)(pix / (uint32_t)n2), j = (int)(pix - (uint32_t)i * n2);
    const int bm = wrap_dn(b - 1, n3);
    const uint32_t pim = (uint32_t)(wrap_dn(i - 1, a.n1) * n2 + j);
    const uint32_t pjm = (uint32_t)(i * n2 + wrap_dn(j - 1, n2));
    // q(b) = (D_v^T Zv + D_h^T Zh)(b); adjoint of D_s: q(b-1) - q(b)
    float q0, q1, zs = 0.f;
    if (a.zslot) {
      const int4 sp = reinterpret_cast<const int4 *>(a.zslot)[pix];
      const int4 si = reinterpret_cast<const int4 *>(a.zslot)[pim];
      const int4 sj = reinterpret_cast<const int4 *>(a.zslot)[pjm];
      q0 = (zfold_val(a.zpart, si, b) - zfold_val(a.zpart, sp, b)) +
           (zfold_val(a.zpart, sj, Bp + b) - zfold_val(a.zpart, sp, Bp + b));
      if (MODE == 4) {
        // (D_s^T Zs)(b) = Zs(b - 1) - Zs(b)
        zs = zfold_val(a.zpart, sp, 2 * Bp + bm) - zfold_val(a.zpart, sp, 2 * Bp + b);
        q1 = 0.f;
      } else {
        q1 = (zfold_val(a.zpart, si, bm) - zfold_val(a.zpart, sp, bm)) +
             (zfold_val(a.zpart, sj, Bp + bm) - zfold_val(a.zpart, sp, Bp + bm));
      }
    } else {
      const float *Zp = a.Z + (size_t)pix * ncol;
      const float *Zi = a.Z + (size_t)pim * ncol;
      const float *Zj = a.Z + (size_t)pjm * ncol;
      q0 = (Zi[b] - Zp[b]) + (Zj[Bp + b] - Zp[Bp + b]);
      if (MODE == 4) {
        zs = Zp[2 * Bp + bm] - Zp[2 * Bp + b];
        q1 = 0.f;
      } else {
        q1 = (Zi[bm] - Zp[bm]) + (Zj[Bp + bm] - Zp[Bp + bm]);
      }
    }
    float adj = MODE == 1 ? q0 : (MODE == 4 ? q0 + zs : q1 - q0);
    if (MODE == 2) {
      const float *Zp = a.Z2 + (size_t)pix * ncol;
      const float *Zi = a.Z2 + (size_t)pim * ncol;
      const float *Zj = a.Z2 + (size_t)pjm * ncol;
      adj += a.omega * ((Zi[b] - Zp[b]) + (Zj[Bp + b] - Zp[Bp + b]));
    }
    const float y3 = kappa * a.w[e];
    const float uo = a.u[e];
    const float un = box(uo - a.g_u * (adj + y3), a.lo, a.hi);
    const float xs = a.s[e] - a.g_s * y3;
    const size_t em = (size_t)pim * n3 + b;
    const float xt = a.t[e] - a.g_t * ((a.y2[em] - a.y2[e]) + y3);
    a.un[e] = un;
    a.xs[e] = xs;
    a.xt[e] = xt;
    const double d = (double)un - (double)uo;
    du2 += d * d;
    u2 += (double)uo * (double)uo;
    if (!(isfinite(un) && isfinite(xs) && isfinite(xt))) bad = 1;
    l1_acc(h[0], xs);
    l1_acc(h[1], xt);
  }
  du2 = block_sum(du2, sh);
  u2 = block_sum(u2, sh);
  bad = block_sum(bad, sh);
  if (threadIdx.x == 0) {
    a.red[blockIdx.x * 4 + 0] = du2;
    a.red[blockIdx.x * 4 + 1] = u2;
    a.red[blockIdx.x * 4 + 2] = bad;
  }
  __syncthreads();
  l1_flush(h[0], kL1Bins1, a.hist->cnt[0][0], a.hist->sig[0][0]);
  l1_flush(h[1], kL1Bins1, a.hist->cnt[1][0], a.hist->sig[1][0]);
}

// ---------------------------------------------------------------- gradient field

struct GradArgs {
  int n1, n2, n3, Bp, ncol;
  long long P;
  const float *a, *b;
  float ca, cb;
  float *g;
  DevScalars *sc;
};

// u' = ca*a + cb*b;  g[pix][b] = (D_v D_s u')(pix, b),  g[pix][Bp + b] = (D_h D_s u')(pix, b).
__global__ __launch_bounds__(kNT) void k_grad(GradArgs a) {
  if (a.sc && a.sc->done) return;
  const int Bp = a.Bp, n3 = a.n3, n2 = a.n2;
  const long long total = a.P * Bp;
  for (long long idx = (long long)blockIdx.x * kNT + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * kNT) {
    const uint32_t pix = (uint32_t)(idx / Bp);
    const int b = (int)(idx - (long long)pix * Bp);
    float gv = 0.f, gh = 0.f;
    if (b < n3) {
      const int i = (int)(pix / (uint32_t)n2), j = (int)(pix - (uint32_t)i * n2);
      const int b1 = wrap_up(b + 1, n3);
      const size_t o00 = (size_t)pix * n3;
      const size_t o10 = ((size_t)wrap_up(i + 1, a.n1) * n2 + j) * n3;
      const size_t o01 = ((size_t)i * n2 + wrap_up(j + 1, n2)) * n3;
#define UP(o, bb) (a.ca * a.a[(o) + (bb)] + a.cb * a.b[(o) + (bb)])
      const float d00 = UP(o00, b1) - UP(o00, b);
      const float d10 = UP(o10, b1) - UP(o10, b);
      const float d01 = UP(o01, b1) - UP(o01, b);
#undef UP
      gv = d10 - d00;
      gh = d01 - d00;
    }
    a.g[(size_t)pix * a.ncol + b] = gv;
    a.g[(size_t)pix * a.ncol + Bp + b] = gh;
  }
}

// Plain adjoint w = D_s^T (D_v^T Zv + D_h^T Zh) of a [pixel][ncol] field.
__global__ __launch_bounds__(kNT) void k_grad_adj(int n1, int n2, int n3, int Bp, int ncol,
                                                  long long N, const float *Z, float *w) {
  for (long long e = (long long)blockIdx.x * kNT + threadIdx.x; e < N;
       e += (long long)gridDim.x * kNT) {
    const uint32_t pix = (uint32_t)(e / n3);
    const int b = (int)(e - (long long)pix * n3);
    const int i = (int)(pix / (uint32_t)n2), j = (int)(pix - (uint32_t)i * n2);
    const int bm = wrap_dn(b - 1, n3);
    const float *Zp = Z + (size_t)pix * ncol;
    const float *Zi = Z + ((size_t)wrap_dn(i - 1, n1) * n2 + j) * ncol;
    const float *Zj = Z + ((size_t)i * n2 + wrap_dn(j - 1, n2)) * ncol;
    const float q0 = (Zi[b] - Zp[b]) + (Zj[Bp + b] - Zp[Bp + b]);
    const float q1 = (Zi[bm] - Zp[bm]) + (Zj[Bp + bm] - Zp[Bp + bm]);
    w[e] = q1 - q0;
  }
}

// ---------------------------------------------------------------- overlap-add partial sum

struct ZsumArgs {
  int n1, n2, ncol, k1, k2, TA, TB, ntA, ntB, extA, extB;
  const int *zpart;
  float *Z;
  DevScalars *sc;
};

// Overlap-add partials: anchor tile (ta, tb) holds the contributions of its anchors to the
// pixels of its extended region (TA + k1 - 1) x (TB + k2 - 1). Pixel row x receives partials
// from the tiles of the anchors x - a (a < k1, on the torus), at every extended row index
// congruent to x. The anchors x, x-1, ... form one circular run, so a tile repeats only as a
// run of equal neighbours or as the first tile again after the wrap.
__device__ inline int anchor_tile(int x, int off, int n, int TT) { return wrap_dn(x - off, n) / TT; }

__device__ inline bool first_visit(int x, int off, int n, int TT) {
  if (off == 0) return true;
  const int tt = anchor_tile(x, off, n, TT);
  return tt != anchor_tile(x, off - 1, n, TT) && tt != anchor_tile(x, 0, n, TT);
}

// Z[pix][c] = sum over slots of zpart[slot][c] (fixed point, summed exactly), four columns per
// thread.
__global__ __launch_bounds__(kNT) void k_zsum(ZsumArgs a) {
  if (a.sc && a.sc->done) return;
  const int c4n = a.ncol >> 2;
  const long long total = (long long)a.n1 * a.n2 * c4n;
  const size_t tile_stride = (size_t)a.extA * a.extB;
  for (long long idx = (long long)blockIdx.x * kNT + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * kNT) {
    const int pix = (int)(idx / c4n);
    const int c4 = (int)(idx - (long long)pix * c4n);
    const int i = pix / a.n2, j = pix - (pix / a.n2) * a.n2;
    int4 acc = make_int4(0, 0, 0, 0);
    for (int offr = 0; offr < a.k1; ++offr) {
      if (!first_visit(i, offr, a.n1, a.TA)) continue;
      const int ta = anchor_tile(i, offr, a.n1, a.TA);
      int e0 = i - ta * a.TA;
      if (e0 < 0) e0 += a.n1;
      for (int ei = e0; ei < a.extA; ei += a.n1) {
        for (int offc = 0; offc < a.k2; ++offc) {
          if (!first_visit(j, offc, a.n2, a.TB)) continue;
          const int tb = anchor_tile(j, offc, a.n2, a.TB);
          int f0 = j - tb * a.TB;
          if (f0 < 0) f0 += a.n2;
          for (int ej = f0; ej < a.extB; ej += a.n2) {
            const size_t slot = ((size_t)ta * a.ntB + tb) * tile_stride + (size_t)ei * a.extB + ej;
            const int4 v = reinterpret_cast<const int4 *>(a.zpart)[slot * c4n + c4];
            acc.x += v.x;
            acc.y += v.y;
            acc.z += v.z;
            acc.w += v.w;
          }
        }
      }
    }
    reinterpret_cast<float4 *>(a.Z)[(size_t)pix * c4n + c4] =
        make_float4((float)acc.x * kZInv, (float)acc.y * kZInv, (float)acc.z * kZInv,
                    (float)acc.w * kZInv);
  }
}

// Slot table of the same enumeration as k_zsum, as element offsets (slot * ncol) into zpart:
// one thread per pixel.
__global__ __launch_bounds__(kNT) void k_zslots(ZsumArgs a, int *zslot, int zero_slot) {
  const long long P = (long long)a.n1 * a.n2;
  const size_t tile_stride = (size_t)a.extA * a.extB;
  for (long long pix = (long long)blockIdx.x * kNT + threadIdx.x; pix < P;
       pix += (long long)gridDim.x * kNT) {
    const int i = (int)(pix / a.n2), j = (int)(pix - (pix / a.n2) * a.n2);
    const int zero = (int)((long long)zero_slot * a.ncol);  // table unused unless it fits
    int sl[4] = {zero, zero, zero, zero};
    int cnt = 0;
    for (int offr = 0; offr < a.k1; ++offr) {
      if (!first_visit(i, offr, a.n1, a.TA)) continue;
      const int ta = anchor_tile(i, offr, a.n1, a.TA);
      int e0 = i - ta * a.TA;
      if (e0 < 0) e0 += a.n1;
      for (int ei = e0; ei < a.extA; ei += a.n1) {
        for (int offc = 0; offc < a.k2; ++offc) {
          if (!first_visit(j, offc, a.n2, a.TB)) continue;
          const int tb = anchor_tile(j, offc, a.n2, a.TB);
          int f0 = j - tb * a.TB;
          if (f0 < 0) f0 += a.n2;
          for (int ej = f0; ej < a.extB; ej += a.n2) {
            const size_t slot = ((size_t)ta * a.ntB + tb) * tile_stride + (size_t)ei * a.extB + ej;
            if (cnt < 4) sl[cnt] = (int)((long long)slot * a.ncol);
            ++cnt;
          }
        }
      }
    }
    if (cnt > 4) atomicOr(&a.sc->zslot_overflow, 1);
    reinterpret_cast<int4 *>(zslot)[pix] = make_int4(sl[0], sl[1], sl[2], sl[3]);
  }
}

// ---------------------------------------------------------------- dual step

struct DualArgs {
  int n1, n2, n3;
  long long N;
  float g_y2, g_y3;
  const float *un, *uo, *xs, *xt, *to, *v;
  float *s, *tn, *y2, *w;
  double *red;
  DevScalars *sc;
};

// Alg. 1 steps 3-7 (apply the l1 thresholds), 12 (y2) and 13 (y3' kept as w = y3' - g_y3 v).
__global__ __launch_bounds__(kNT) void k_dual(DualArgs a) {
  __shared__ double sh[4];
  if (a.sc->done) return;
  const int act_s = a.sc->active[0], act_t = a.sc->active[1];
  const double tau_s = a.sc->tau[0], tau_t = a.sc->tau[1];
  const float kappa = (float)a.sc->kappa;
  const int n2 = a.n2, n3 = a.n3;
  double w2 = 0;
  for (long long e = (long long)blockIdx.x * kNT + threadIdx.x; e < a.N;
       e += (long long)gridDim.x * kNT) {
    const uint32_t pix = (uint32_t)(e / n3);
    const int b = (int)(e - (long long)pix * n3);
    const int i = (int)(pix / (uint32_t)n2), j = (int)(pix - (uint32_t)i * n2);
    const size_t ep = ((size_t)wrap_up(i + 1, a.n1) * n2 + j) * n3 + b;
    const float xs = a.xs[e];
    const float sn = act_s ? soft(xs, tau_s) : xs;
    const float xt0 = a.xt[e], xt1 = a.xt[ep];
    const float tn0 = act_t ? soft(xt0, tau_t) : xt0;
    const float tn1 = act_t ? soft(xt1, tau_t) : xt1;
    const float tp0 = 2.f * tn0 - a.to[e];
    const float tp1 = 2.f * tn1 - a.to[ep];
    const float sp = 2.f * sn - a.s[e];
    const float up = 2.f * a.un[e] - a.uo[e];
    a.y2[e] = a.y2[e] + a.g_y2 * (tp1 - tp0);
    const float wn = kappa * a.w[e] + a.g_y3 * (((up + sp) + tp0) - a.v[e]);
    a.w[e] = wn;
    a.s[e] = sn;
    a.tn[e] = tn0;
    w2 += (double)wn * (double)wn;
  }
  w2 = block_sum(w2, sh);
  if (threadIdx.x == 0) a.red[blockIdx.x] = w2;
}

// k_dual and k_grad in one sweep (the dual step does not depend on the block pass, which only
// needs the gradient field): one thread per (pixel, padded band); bands >= N3 only write the
// zero padding of the gradient field. The extrapolated u' = 2u+ - u is formed once.
struct DualGradArgs {
  DualArgs d;
  int Bp, ncol;
  float *g;        // gradient field (S3TTV, STV) or the dual field Z updated in place (SSTV, HSSTV)
  float *g2;       // second dual field Z2 (HSSTV)
  float gZ, gZ2, omega;
};

__device__ inline float clip1(float x) { return fminf(1.f, fmaxf(-1.f, x)); }

// REG 0 (S3TTV): g = (D_v D_s u', D_h D_s u') for the block pass. REG 1 (STV): g = (D_v u',
// D_h u'). REG 2 (SSTV): the l1 dual step Z = clip(Z + gZ D D_s u') to [-1, 1] (the Moreau
// form of the prox of ||.||_1), in place. REG 3 (HSSTV): as REG 2 plus
// Z2 = clip(Z2 + gZ2 omega D u'). REG 4 (SSST): g = (D_v u', D_h u', D_s u').
template <int REG>
__global__ __launch_bounds__(kNT) void k_dual_grad(DualGradArgs ag) {
  __shared__ double sh[4];
  const DualArgs &a = ag.d;
  if (a.sc->done) return;
  const int act_s = a.sc->active[0], act_t = a.sc->active[1];
  const double tau_s = a.sc->tau[0], tau_t = a.sc->tau[1];
  const float kappa = (float)a.sc->kappa;
  const int n2 = a.n2, n3 = a.n3, Bp = ag.Bp;
  const long long total = (long long)a.n1 * n2 * Bp;
  double w2 = 0;
  for (long long idx = (long long)blockIdx.x * kNT + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * kNT) {
    const uint32_t pix = (uint32_t)(idx / Bp);
    const int b = (int)(idx - (long long)pix * Bp);
    float gv = 0.f, gh = 0.f, gs = 0.f;
    if (b < n3) {
      const int i = (int)(pix / (uint32_t)n2), j = (int)(pix - (uint32_t)i * n2);
      const size_t e = (size_t)pix * n3 + b;
      const size_t o10 = ((size_t)wrap_up(i + 1, a.n1) * n2 + j) * n3;
      const size_t o01 = ((size_t)i * n2 + wrap_up(j + 1, n2)) * n3;
      const size_t ep = o10 + b;
      // dual step (as k_dual)
      const float xs = a.xs[e];
      const float sn = act_s ? soft(xs, tau_s) : xs;
      const float xt0 = a.xt[e], xt1 = a.xt[ep];
      const float tn0 = act_t ? soft(xt0, tau_t) : xt0;
      const float tn1 = act_t ? soft(xt1, tau_t) : xt1;
      const float tp0 = 2.f * tn0 - a.to[e];
      const float tp1 = 2.f * tn1 - a.to[ep];
      const float sp = 2.f * sn - a.s[e];
      const float up = 2.f * a.un[e] - a.uo[e];
      a.y2[e] = a.y2[e] + a.g_y2 * (tp1 - tp0);
      const float wn = kappa * a.w[e] + a.g_y3 * (((up + sp) + tp0) - a.v[e]);
      a.w[e] = wn;
      a.s[e] = sn;
      a.tn[e] = tn0;
      w2 += (double)wn * (double)wn;
      // gradient field of u' (as k_grad with ca = 2, cb = -1)
      const int b1 = wrap_up(b + 1, n3);
      const size_t o00 = (size_t)pix * n3;
#define UP(o, bb) (2.f * a.un[(o) + (bb)] + -1.f * a.uo[(o) + (bb)])
      const float u10 = UP(o10, b), u01 = UP(o01, b);
      if (REG == 1 || REG == 4) {
        gv = u10 - up;
        gh = u01 - up;
        if (REG == 4) gs = UP(o00, b1) - up;
      } else {
        const float d00 = UP(o00, b1) - up;
        const float d10 = UP(o10, b1) - u10;
        const float d01 = UP(o01, b1) - u01;
        gv = d10 - d00;
        gh = d01 - d00;
      }
#undef UP
      if (REG == 2 || REG == 3) {
        const size_t o = (size_t)pix * ag.ncol + b;
        gv = clip1(ag.g[o] + ag.gZ * gv);
        gh = clip1(ag.g[o + Bp] + ag.gZ * gh);
        if (REG == 3) {
          const float s2 = ag.gZ2 * ag.omega;
          ag.g2[o] = clip1(ag.g2[o] + s2 * (u10 - up));
          ag.g2[o + Bp] = clip1(ag.g2[o + Bp] + s2 * (u01 - up));
        }
      }
    }
    ag.g[(size_t)pix * ag.ncol + b] = gv;
    ag.g[(size_t)pix * ag.ncol + Bp + b] = gh;
    if (REG == 4) ag.g[(size_t)pix * ag.ncol + 2 * Bp + b] = gs;
  }
  w2 = block_sum(w2, sh);
  if (threadIdx.x == 0) a.red[blockIdx.x] = w2;
}

// ---------------------------------------------------------------- scalar finalisation

struct FinalArgs {
  int nblk;
  const double *red_primal, *red_dual;
  double eps_g3;  // eps * gamma_y3
  const int *estat;  // per-workgroup eigen statistics of this iteration (4 ints), or null
  long long nstat;
  DevScalars *sc;
};

__global__ __launch_bounds__(kNT) void k_finalize(FinalArgs a) {
  __shared__ double sh[4];
  if (a.sc->done) return;
  double du2 = 0, u2 = 0, bad = 0, w2 = 0;
  for (int k = threadIdx.x; k < a.nblk; k += kNT) {
    du2 += a.red_primal[k * 4 + 0];
    u2 += a.red_primal[k * 4 + 1];
    bad += a.red_primal[k * 4 + 2];
    w2 += a.red_dual[k];
  }
  du2 = block_sum(du2, sh);
  u2 = block_sum(u2, sh);
  bad = block_sum(bad, sh);
  w2 = block_sum(w2, sh);
  // eigen-solve statistics: rotation steps per block and blocks left to the per-lane Jacobi
  double ssum = 0, nfb = 0, smax = 0, nblk = 0;
  if (a.estat) {
    for (long long k = threadIdx.x; k < a.nstat; k += kNT) {
      const int4 r = *(const int4 *)(a.estat + 4 * k);
      ssum += (double)r.x;
      smax = fmax(smax, (double)r.y);
      nfb += (double)r.z;
      nblk += (double)r.w;
    }
    ssum = block_sum(ssum, sh);
    nfb = block_sum(nfb, sh);
    nblk = block_sum(nblk, sh);
    smax = block_max(smax, sh);
  }
  if (threadIdx.x == 0) {
    DevScalars *sc = a.sc;
    if (a.estat) {
      sc->step_sum += (unsigned long long)ssum;
      sc->step_blocks += (unsigned long long)nblk;
      sc->fallback_blocks += (unsigned long long)nfb;
      if ((int)smax > sc->max_steps) sc->max_steps = (int)smax;
    }
    const double wn = sqrt(w2);
    sc->kappa = wn > a.eps_g3 ? 1.0 - a.eps_g3 / wn : 0.0;
    sc->wnorm2 = w2;
    sc->unorm2 = u2;
    sc->rel_change = u2 > 0 ? sqrt(du2) / sqrt(u2) : INFINITY;
    sc->iters += 1;
    if (bad != 0) {
      sc->nonfinite = 1;
      sc->done = 1;
    }
    if (sc->rel_tol > 0 && sc->iters >= 2 && u2 > 0 && sc->rel_change < sc->rel_tol) {
      sc->converged = 1;
      sc->done = 1;
    }
    if (sc->max_iter > 0 && sc->iters >= sc->max_iter) sc->done = 1;
  }
}

// ---------------------------------------------------------------- small utilities

__global__ void k_fill(float *p, long long n, float val) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    p[e] = val;
}

// Deterministic pseudo-random values in [-scale, scale) (integer hash of the index).
__global__ void k_fill_hash(float *p, long long n, float scale, uint32_t seed) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    uint32_t h = (uint32_t)e * 0x9E3779B1u ^ (uint32_t)(e >> 32) ^ seed * 0x85EBCA77u;
    h ^= h >> 16;
    h *= 0x7FEB352Du;
    h ^= h >> 15;
    h *= 0x846CA68Bu;
    h ^= h >> 16;
    p[e] = scale * ((float)(h >> 8) * (2.f / 16777216.f) - 1.f);
  }
}

__global__ void k_identity16(float *V, long long nblk) {
  const long long n = nblk * 256;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const int w = (int)(e & 255);
    V[e] = (w >> 4) == (w & 15) ? 1.f : 0.f;
  }
}

__global__ void k_copy(float *dst, const float *src, long long n) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

__global__ void k_zero_words(uint32_t *p, long long n) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    p[e] = 0u;
}

__global__ void k_init_scalars(DevScalars *sc, double rel_tol, int max_iter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    DevScalars z = {};
    z.rel_tol = rel_tol;
    z.max_iter = max_iter;
    *sc = z;
  }
}

__global__ void k_mark_state(DevScalars *sc, StateSig sig) {
  if (threadIdx.x < 8 && blockIdx.x == 0) sc->sig[threadIdx.x] = sig.v[threadIdx.x];
}

__global__ void k_resume_scalars(DevScalars *sc, double rel_tol, int budget) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    sc->done = 0;
    sc->converged = 0;
    sc->rel_tol = rel_tol;
    sc->max_iter = sc->iters + budget;
    sc->max_sweeps = 0;
    sc->sweep_sum = 0;
    sc->sweep_waves = 0;
    sc->step_sum = 0;
    sc->step_blocks = 0;
    sc->fallback_blocks = 0;
    sc->max_steps = 0;
  }
}

__global__ void k_check_finite(const float *x, long long n, DevScalars *sc) {
  bool bad = false;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    bad |= !isfinite(x[e]);
  if (bad) atomicOr(&sc->nonfinite, 1);
}

__global__ void k_field_to_cubes(const float *f, float *c0, float *c1, long long P, int n3, int Bp) {
  const long long total = P * n3;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long pix = e / n3;
    const int b = (int)(e - pix * n3);
    c0[e] = f[pix * 2 * Bp + b];
    c1[e] = f[pix * 2 * Bp + Bp + b];
  }
}

__global__ void k_cubes_to_field(const float *c0, const float *c1, float *f, long long P, int n3,
                                 int Bp) {
  const long long total = P * Bp;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long pix = e / Bp;
    const int b = (int)(e - pix * Bp);
    f[pix * 2 * Bp + b] = b < n3 ? c0[pix * n3 + b] : 0.f;
    f[pix * 2 * Bp + Bp + b] = b < n3 ? c1[pix * n3 + b] : 0.f;
  }
}

// Diagnostics: partial sums of |s|, |t|, (u+s+t-v)^2, (D_v t)^2.
__global__ __launch_bounds__(kNT) void k_diag_partial(int n1, int n2, int n3, long long N,
                                                      const float *u, const float *s,
                                                      const float *t, const float *v,
                                                      double *red) {
  __shared__ double sh[4];
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  for (long long e = (long long)blockIdx.x * kNT + threadIdx.x; e < N;
       e += (long long)gridDim.x * kNT) {
    const long long pix = e / n3;
    const int b = (int)(e - pix * n3);
    const int i = (int)(pix / n2), j = (int)(pix - (long long)i * n2);
    const size_t ep = ((size_t)wrap_up(i + 1, n1) * n2 + j) * n3 + b;
    a0 += fabs((double)s[e]);
    a1 += fabs((double)t[e]);
    const double r = (double)u[e] + (double)s[e] + (double)t[e] - (double)v[e];
    a2 += r * r;
    const double dv = (double)t[ep] - (double)t[e];
    a3 += dv * dv;
  }
  a0 = block_sum(a0, sh);
  a1 = block_sum(a1, sh);
  a2 = block_sum(a2, sh);
  a3 = block_sum(a3, sh);
  if (threadIdx.x == 0) {
    red[blockIdx.x * 4 + 0] = a0;
    red[blockIdx.x * 4 + 1] = a1;
    red[blockIdx.x * 4 + 2] = a2;
    red[blockIdx.x * 4 + 3] = a3;
  }
}

__global__ __launch_bounds__(kNT) void k_diag_final(int nblk, const double *red, double *out) {
  __shared__ double sh[4];
  double a[4] = {0, 0, 0, 0};
  for (int k = threadIdx.x; k < nblk; k += kNT)
    for (int c = 0; c < 4; ++c) a[c] += red[k * 4 + c];
  for (int c = 0; c < 4; ++c) {
    const double r = block_sum(a[c], sh);
    if (threadIdx.x == 0) out[c] = r;
  }
}

inline int grid_for(long long n, int per_thread, int nt = kNT) {
  long long g = (n + (long long)nt * per_thread - 1) / ((long long)nt * per_thread);
  if (g < 1) g = 1;
  if (g > 65535) g = 65535;
  return (int)g;
}

}  // namespace

hipError_t launch_fill(float *p, long long n, float val, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 8)), dim3(kNT), 0, st, p, n, val);
  return hipGetLastError();
}

hipError_t launch_fill_hash(float *p, long long n, float scale, uint32_t seed, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_hash, dim3(grid_for(n, 4)), dim3(kNT), 0, st, p, n, scale, seed);
  return hipGetLastError();
}

hipError_t launch_identity16(float *V, long long nblk, hipStream_t st) {
  hipLaunchKernelGGL(k_identity16, dim3(grid_for(nblk * 256, 8)), dim3(kNT), 0, st, V, nblk);
  return hipGetLastError();
}

hipError_t launch_copy(float *dst, const float *src, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_copy, dim3(grid_for(n, 8)), dim3(kNT), 0, st, dst, src, n);
  return hipGetLastError();
}

hipError_t launch_zero_bytes(void *p, size_t bytes, hipStream_t st) {
  const long long n = (long long)(bytes / 4);
  hipLaunchKernelGGL(k_zero_words, dim3(grid_for(n, 8)), dim3(kNT), 0, st, (uint32_t *)p, n);
  return hipGetLastError();
}

hipError_t launch_init_scalars(const Plan &pl, double rel_tol, int max_iter, hipStream_t st) {
  hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(64), 0, st, pl.sc, rel_tol, max_iter);
  return hipGetLastError();
}

hipError_t launch_mark_state(const Plan &pl, const StateSig &sig, hipStream_t st) {
  hipLaunchKernelGGL(k_mark_state, dim3(1), dim3(64), 0, st, pl.sc, sig);
  return hipGetLastError();
}

hipError_t launch_resume_scalars(const Plan &pl, double rel_tol, int budget, hipStream_t st) {
  hipLaunchKernelGGL(k_resume_scalars, dim3(1), dim3(64), 0, st, pl.sc, rel_tol, budget);
  return hipGetLastError();
}

hipError_t launch_check_finite(const float *x, long long n, DevScalars *sc, hipStream_t st) {
  hipLaunchKernelGGL(k_check_finite, dim3(grid_for(n, 16)), dim3(kNT), 0, st, x, n, sc);
  return hipGetLastError();
}

hipError_t launch_primal(const Plan &pl, const float *u_cur, float *u_new, const float *t_cur,
                         hipStream_t st) {
  PrimalArgs a;
  a.n1 = pl.n1; a.n2 = pl.n2; a.n3 = pl.n3; a.Bp = pl.Bp; a.ncol = pl.ncol; a.N = pl.N;
  a.g_u = pl.g_u; a.g_s = pl.g_s; a.g_t = pl.g_t; a.lo = pl.mu_min; a.hi = pl.mu_max;
  a.u = u_cur; a.s = pl.s; a.t = t_cur; a.y2 = pl.y2; a.w = pl.w; a.Z = pl.Z;
  a.zpart = pl.zpart; a.zslot = pl.zfold && !l1_reg(pl.reg) ? pl.zslot : nullptr;
  a.Z2 = pl.gradf; a.omega = pl.omega;
  a.un = u_new; a.xs = pl.xs; a.xt = pl.xt; a.red = pl.red_primal; a.sc = pl.sc; a.hist = pl.hist;
  const uintptr_t align = reinterpret_cast<uintptr_t>(a.u) | reinterpret_cast<uintptr_t>(a.s) |
                          reinterpret_cast<uintptr_t>(a.t) | reinterpret_cast<uintptr_t>(a.w) |
                          reinterpret_cast<uintptr_t>(a.y2) | reinterpret_cast<uintptr_t>(a.un) |
                          reinterpret_cast<uintptr_t>(a.xs) | reinterpret_cast<uintptr_t>(a.xt);
  if (pl.reg == kRegSTV)
    hipLaunchKernelGGL(k_primal<1>, dim3(pl.red_blocks), dim3(kNT), 0, st, a);
  else if (pl.reg == kRegSSST)
    hipLaunchKernelGGL(k_primal<4>, dim3(pl.red_blocks), dim3(kNT), 0, st, a);
  else if (pl.reg == kRegHSSTV)
    hipLaunchKernelGGL(k_primal<2>, dim3(pl.red_blocks), dim3(kNT), 0, st, a);
  else if (a.zslot && (pl.n3 & 3) == 0 && (align & 15) == 0)
    hipLaunchKernelGGL(k_primal<3>, dim3(pl.red_blocks), dim3(kNT), 0, st, a);
  else
    hipLaunchKernelGGL(k_primal<0>, dim3(pl.red_blocks), dim3(kNT), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_grad(const Plan &pl, const float *x, const float *y, float ca, float cb,
                       float *gout, hipStream_t st) {
  GradArgs a;
  a.n1 = pl.n1; a.n2 = pl.n2; a.n3 = pl.n3; a.Bp = pl.Bp; a.ncol = pl.ncol; a.P = pl.P;
  a.a = x; a.b = y; a.ca = ca; a.cb = cb; a.g = gout ? gout : pl.gradf; a.sc = pl.sc;
  hipLaunchKernelGGL(k_grad, dim3(grid_for(pl.P * pl.Bp, 4)), dim3(kNT), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_grad_adj(const Plan &pl, const float *Z, float *w, hipStream_t st) {
  hipLaunchKernelGGL(k_grad_adj, dim3(grid_for(pl.N, 4)), dim3(kNT), 0, st, pl.n1, pl.n2, pl.n3,
                     pl.Bp, pl.ncol, pl.N, Z, w);
  return hipGetLastError();
}

hipError_t launch_zsum(const Plan &pl, hipStream_t st) {
  ZsumArgs a;
  a.n1 = pl.n1; a.n2 = pl.n2; a.ncol = pl.ncol; a.k1 = pl.k1; a.k2 = pl.k2;
  a.TA = pl.TA; a.TB = pl.TB; a.ntA = pl.ntA; a.ntB = pl.ntB; a.extA = pl.extA; a.extB = pl.extB;
  a.zpart = pl.zpart; a.Z = pl.Z; a.sc = pl.sc;
  hipLaunchKernelGGL(k_zsum, dim3(grid_for(pl.P * (pl.ncol / 4), 2)), dim3(kNT), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_zslots(const Plan &pl, hipStream_t st) {
  ZsumArgs a;
  a.n1 = pl.n1; a.n2 = pl.n2; a.ncol = pl.ncol; a.k1 = pl.k1; a.k2 = pl.k2;
  a.TA = pl.TA; a.TB = pl.TB; a.ntA = pl.ntA; a.ntB = pl.ntB; a.extA = pl.extA; a.extB = pl.extB;
  a.zpart = pl.zpart; a.Z = pl.Z; a.sc = pl.sc;
  const int zero_slot = pl.ntA * pl.ntB * pl.extA * pl.extB;  // the extra all-zero slot
  hipLaunchKernelGGL(k_zslots, dim3(grid_for(pl.P, 1)), dim3(kNT), 0, st, a, pl.zslot, zero_slot);
  return hipGetLastError();
}

// The slot table holds 32-bit element offsets: usable while zpart has fewer than 2^31 entries.
bool zslots_fit(const Plan &pl) {
  return ((long long)pl.ntA * pl.ntB * pl.extA * pl.extB + 1) * pl.ncol < (1ll << 31);
}

hipError_t launch_dual(const Plan &pl, const float *u_cur, const float *u_new, const float *t_cur,
                       float *t_new, const float *v, hipStream_t st) {
  DualArgs a;
  a.n1 = pl.n1; a.n2 = pl.n2; a.n3 = pl.n3; a.N = pl.N; a.g_y2 = pl.g_y2; a.g_y3 = pl.g_y3;
  a.un = u_new; a.uo = u_cur; a.xs = pl.xs; a.xt = pl.xt; a.to = t_cur; a.v = v;
  a.s = pl.s; a.tn = t_new; a.y2 = pl.y2; a.w = pl.w; a.red = pl.red_dual; a.sc = pl.sc;
  hipLaunchKernelGGL(k_dual, dim3(pl.red_blocks), dim3(kNT), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_dual_grad(const Plan &pl, const float *u_cur, const float *u_new,
                            const float *t_cur, float *t_new, const float *v, hipStream_t st) {
  DualGradArgs g;
  DualArgs &a = g.d;
  a.n1 = pl.n1; a.n2 = pl.n2; a.n3 = pl.n3; a.N = pl.N; a.g_y2 = pl.g_y2; a.g_y3 = pl.g_y3;
  a.un = u_new; a.uo = u_cur; a.xs = pl.xs; a.xt = pl.xt; a.to = t_cur; a.v = v;
  a.s = pl.s; a.tn = t_new; a.y2 = pl.y2; a.w = pl.w; a.red = pl.red_dual; a.sc = pl.sc;
  g.Bp = pl.Bp; g.ncol = pl.ncol;
  g.g = l1_reg(pl.reg) ? pl.Z : pl.gradf;
  g.g2 = pl.gradf;
  g.gZ = pl.g_Y; g.gZ2 = pl.g_Z2; g.omega = pl.omega;
  switch (pl.reg) {
    case kRegSTV: hipLaunchKernelGGL(k_dual_grad<1>, dim3(pl.red_blocks), dim3(kNT), 0, st, g); break;
    case kRegSSTV: hipLaunchKernelGGL(k_dual_grad<2>, dim3(pl.red_blocks), dim3(kNT), 0, st, g); break;
    case kRegHSSTV: hipLaunchKernelGGL(k_dual_grad<3>, dim3(pl.red_blocks), dim3(kNT), 0, st, g); break;
    case kRegSSST: hipLaunchKernelGGL(k_dual_grad<4>, dim3(pl.red_blocks), dim3(kNT), 0, st, g); break;
    default: hipLaunchKernelGGL(k_dual_grad<0>, dim3(pl.red_blocks), dim3(kNT), 0, st, g); break;
  }
  return hipGetLastError();
}

hipError_t launch_finalize(const Plan &pl, bool eig_stats, hipStream_t st) {
  FinalArgs a;
  a.nblk = pl.red_blocks; a.red_primal = pl.red_primal; a.red_dual = pl.red_dual;
  a.eps_g3 = pl.eps * (double)pl.g_y3; a.sc = pl.sc;
  a.estat = eig_stats ? pl.estat : nullptr;
  a.nstat = (pl.P + 63) / 64;
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kNT), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_field_to_cubes(const float *f, float *c0, float *c1, long long P, int n3, int Bp,
                                 hipStream_t st) {
  hipLaunchKernelGGL(k_field_to_cubes, dim3(grid_for(P * n3, 4)), dim3(kNT), 0, st, f, c0, c1, P,
                     n3, Bp);
  return hipGetLastError();
}

hipError_t launch_cubes_to_field(const float *c0, const float *c1, float *f, long long P, int n3,
                                 int Bp, hipStream_t st) {
  hipLaunchKernelGGL(k_cubes_to_field, dim3(grid_for(P * Bp, 4)), dim3(kNT), 0, st, c0, c1, f, P,
                     n3, Bp);
  return hipGetLastError();
}

hipError_t launch_diagnostics(const Plan &pl, const float *u, const float *s, const float *t,
                              const float *v, double *out4, hipStream_t st) {
  hipLaunchKernelGGL(k_diag_partial, dim3(pl.red_blocks), dim3(kNT), 0, st, pl.n1, pl.n2, pl.n3,
                     pl.N, u, s, t, v, pl.red_primal);
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kNT), 0, st, pl.red_blocks, pl.red_primal, out4);
  return hipGetLastError();
}

}  // namespace s3ttv
