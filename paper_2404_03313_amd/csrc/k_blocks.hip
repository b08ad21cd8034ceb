// Block kernels of Alg. 1 steps 9-10 (arXiv 2404.03313, Sec. III-A and III-C) for gfx950.
//
// For every block l (one torus window per pixel anchor) the dual step is
//   Y'_l = Y_l + g_Y T_l,       T_l = P_l D D_s u'                 (step 9, eq. rewrite_Lu)
//   Y+_l = Y'_l - g_Y prox_{||.||_*/g_Y}(Y'_l / g_Y)               (step 10)
// which by eq. ProxConjugate and eq. prox_nuclear_norm equals U diag(min(sigma, 1)) V^T,
// the projection of Y'_l onto the unit spectral-norm ball. With K <= 2B rows this is
//   Y+_l = W_l Y'_l,   W_l = I - sum_{lambda_k > 1} (1 - lambda_k^{-1/2}) v_k v_k^T,
// where (lambda_k, v_k) are the eigenpairs of the K x K Gram matrix G_l = Y'_l Y'_l^T.
// Three kernels: Gram on MFMA (k_gram), which in the solver also diagonalises the Gram matrix
// on MFMA (simultaneous Jacobi rotations from the previous eigenbasis, the identity before the
// first iteration) and forms W_l; a per-lane cyclic Jacobi eigen-solve (k_eig) for the
// stand-alone block operator and for the blocks the MFMA rotations cannot certify; and
// W_l Y'_l on MFMA with a deterministic overlap-add (k_apply). With at most 24 column tiles
// (S3TTV and STV: N3 <= 192) the solver runs all of it in one pass (k_block_fused).
//
// Block storage ("apply layout", 16 rows x ncol columns per block, ncol = 2*Bp, column
// c = comp*Bp + band): column tile t holds columns 16t..16t+15 as 64 lanes x 4 floats,
// lane L = 16*g + tc, slot s <-> element (row 4g+s, column 16t+tc). This is the B-operand /
// result layout of v_mfma_f32_16x16x4_f32, so k_apply streams it with 16-byte accesses.
#include <atomic>
#include "s3ttv_internal.h"

namespace s3ttv {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

__device__ inline f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// 16 x 16 matrices in the MFMA result layout ("D-form"): lane j + 16g, register v holds
// X[4g+v][j]. Feeding the four registers of two D-form matrices M, N as the A and B operands
// of four consecutive 16x16x4 steps accumulates M^T N.
__device__ inline f4 mtn(f4 M, f4 N) {
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  acc = mfma4(M[0], N[0], acc);
  acc = mfma4(M[1], N[1], acc);
  acc = mfma4(M[2], N[2], acc);
  acc = mfma4(M[3], N[3], acc);
  return acc;
}

__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A non-finite (or out-of-range) overlap-add value: flag the solve and stop it.
__device__ inline void flag_nonfinite(DevScalars *sc, bool bad) {
  if (__any(bad) && sc && (threadIdx.x & 63) == 0) {
    atomicOr(&sc->nonfinite, 1);
    atomicOr(&sc->done, 1);
  }
}

// Sum over the 64 lanes; every lane receives the same (bitwise) value.
__device__ inline float wave_sum(float x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m);
  return x;
}

// Sum over the 16 lanes j of a row group (same value in all 16 lanes).
__device__ inline float row_sum16(float x) {
#pragma unroll
  for (int m = 8; m >= 1; m >>= 1) x += __shfl_xor(x, m);
  return x;
}

// Transpose of a D-form matrix through the wavefront's LDS tile (row stride 20 floats).
__device__ inline f4 dform_transpose(f4 x, float *tb, int j, int g) {
#pragma unroll
  for (int v = 0; v < 4; ++v) tb[(4 * g + v) * 20 + j] = x[v];
  wave_lds_sync();
  const f4 y = *(const f4 *)(tb + j * 20 + 4 * g);
  wave_lds_sync();
  return y;
}

// Pixel offset (into the [pixel][ncol] field) of block row `row` of anchor l, or -1.
__device__ inline int row_pixel(const BlockArgs &a, long long l, int row) {
  if (row >= a.K) return -1;
  const int p = (int)(l / a.n2), q = (int)(l - (long long)(l / a.n2) * a.n2);
  const int ar = row / a.k2, cr = row - (row / a.k2) * a.k2;
  int i = p + ar;
  if (i >= a.n1) i -= a.n1;
  int j = q + cr;
  if (j >= a.n2) j -= a.n2;
  return i * a.n2 + j;
}

// ---------------------------------------------------------------- eigen-solve on MFMA

// Simultaneous Jacobi rotations on the wavefront's 16 x 16 Gram matrix G (D-form), warm
// started from the stored eigenbasis V of the previous iteration:
//   A = V^T G V; repeat: symmetrise A; if certified stop; else K_ij = tan(theta_ij), the
//   tangent of the angle that zeroes A_ij in its own 2 x 2 rotation (|theta| <= pi/4), for all
//   pairs at once (K is exactly skew: it is computed from the symmetrised A), damped to
//   ||K||_F <= kStepCap; J = I + K + K^2/2 with J^T J = I + K^4/4, corrected to first order
//   by J (I - K^4/8); A <- J^T A J, V <- V J.
// Certificate (what W = f(G), f(l) = min(1, l^-1/2), needs): every off-diagonal A_ij with
// A_ii > 1 or A_jj > 1 is at most kJacobiTol ||G||_F, and every row i with A_ii <= 1 has its
// Gershgorin radius over the other such rows within 1 + kGershSlack, so no eigenvalue of that
// sub-block exceeds 1. After a damped (large) step, V is re-orthogonalised by a Newton-Schulz
// step and A recomputed as V^T G V before the certificate may be accepted. Certified blocks get
// W = I - V diag((1 - A_ii^-1/2)_+) V^T; others (rare; cold starts) are left to k_eig with
// A and V stored. V always leaves with one Newton-Schulz step applied.
// The tolerance sits at the rounding level of G itself: an FP32 sum of 2 N3 = 256 products
// carries about 1e-6 relative error, so certifying the rotated matrix further would not make W
// more accurate. Gram products formed from inputs rounded to bfloat16 (8-bit significand) are
// known only to about 4e-3 relative; that mode is certified to 1e-5 of ||G||_F, still far
// below its rounding (binary16 inputs, 5e-4, keep the FP32 tolerance).
constexpr float kJacobiTol = 1e-6f;
constexpr float kJacobiTolBF16 = 1e-5f;
constexpr float kStepCap = 0.5f;
constexpr float kRoughNorm2 = 0.0225f;    // a step with ||K||_F > 0.15 forces the recompute
constexpr float kQuarticNorm2 = 2e-4f;    // below this ||K^4||/8 is under FP32 rounding
constexpr float kGershSlack = 1e-6f;

// Returns true with W (D-form) for a certified block; otherwise stores A (into a.G) for k_eig.
// Always stores the re-orthogonalised V and the block's flag.
// The stored basis of block l in both D-forms (V and V^T), loaded ahead of use.
__device__ inline void load_basis(const BlockArgs &a, long long l, f4 &vd, f4 &vt) {
  const int lane = threadIdx.x & 63;
  const int j = lane & 15, g = lane >> 4;
  const float *Vl = a.V + (size_t)l * 256;
#pragma unroll
  for (int v = 0; v < 4; ++v) vd[v] = Vl[(4 * g + v) * 16 + j];
  vt = *(const f4 *)(Vl + j * 16 + 4 * g);
}

__device__ __forceinline__ bool eigen_mfma(const BlockArgs &a, long long l, f4 G, f4 vd, f4 Vt,
                                           float *tb, f4 &Wout, bool refine = false,
                                           f4 Xres = f4{0.f, 0.f, 0.f, 0.f}) {
  const int lane = threadIdx.x & 63;
  const int j = lane & 15, g = lane >> 4;
  float *Vl = a.V + (size_t)l * 256;
  f4 A = mtn(vd, mtn(G, vd));                   // V^T G V  (G symmetric; Vt = D-form of V^T)
  const float fro = sqrtf(wave_sum(G[0] * G[0] + G[1] * G[1] + G[2] * G[2] + G[3] * G[3]));
  const float thr = (a.gram_prec == 1 ? kJacobiTolBF16 : kJacobiTol) * fro;

  // Newton-Schulz re-orthogonalisation of V (held as Vt); optionally returns D-form V too.
  auto orthonormalise = [&](f4 &Vc) {
    const f4 Vd = dform_transpose(Vt, tb, j, g);
    const f4 X = mtn(Vd, Vd);          // V^T V
    const f4 VX = mtn(Vt, X);          // V X
    const f4 XVt = mtn(X, Vt);         // X V^T
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Vc[v] = fmaf(1.5f, Vd[v], -0.5f * VX[v]);
      Vt[v] = fmaf(1.5f, Vt[v], -0.5f * XVt[v]);
    }
  };

  f4 dI;
  float dJ = 0.f;
  // symmetrise A (exactly) and fetch the diagonal for rows 4g+v and column j
  auto symmetrise = [&]() {
#pragma unroll
    for (int v = 0; v < 4; ++v) tb[(4 * g + v) * 20 + j] = A[v];
    wave_lds_sync();
    const f4 At = *(const f4 *)(tb + j * 20 + 4 * g);
    dJ = tb[j * 20 + j];
#pragma unroll
    for (int v = 0; v < 4; ++v) dI[v] = tb[(4 * g + v) * 20 + 4 * g + v];
    wave_lds_sync();
#pragma unroll
    for (int v = 0; v < 4; ++v) A[v] = 0.5f * (A[v] + At[v]);
  };
  // one damped simultaneous rotation step on the symmetrised A; returns ||K||_F^2
  auto rotate = [&]() -> float {
    f4 K;
    float kf2 = 0.f;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 4 * g + v;
      const float den = dJ - dI[v];
      const float sg = (den > 0.f || (den == 0.f && i < j)) ? 1.f : -1.f;
      const float q = fabsf(den) + sqrtf(fmaf(den, den, 4.f * A[v] * A[v]));
      const float t = (i != j && q > 0.f) ? __fdividef(2.f * A[v] * sg, q) : 0.f;
      K[v] = t;
      kf2 = fmaf(t, t, kf2);
    }
    kf2 = wave_sum(kf2);
    if (kf2 > kStepCap * kStepCap) {
      const float sc = kStepCap * rsqrtf(kf2);
#pragma unroll
      for (int v = 0; v < 4; ++v) K[v] *= sc;
      kf2 = kStepCap * kStepCap;
    }
    const f4 KK = mtn(K, K);  // K^T K = -K^2
    f4 J, Jt;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float id = (4 * g + v) == j ? 1.f : 0.f;
      const float h = -0.5f * KK[v];
      J[v] = id + K[v] + h;
      Jt[v] = id - K[v] + h;
    }
    if (kf2 > kQuarticNorm2) {
      f4 K2;
#pragma unroll
      for (int v = 0; v < 4; ++v) K2[v] = -KK[v];
      const f4 K4 = mtn(K2, K2);   // (K^2)^T K^2 = K^4
      const f4 JK4 = mtn(Jt, K4);  // J K^4
#pragma unroll
      for (int v = 0; v < 4; ++v) J[v] = fmaf(-0.125f, JK4[v], J[v]);
    }
    A = mtn(J, mtn(A, J));  // J^T (A J), A symmetric
    Vt = mtn(J, Vt);        // (V J)^T
    return kf2;
  };

  bool ok = false, rough = false;
  int steps = 0;
  for (;;) {
    symmetrise();
    // certificate
    bool bad = false;
    float gr[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const bool off = (4 * g + v) != j;
      bad |= off && (dI[v] > 1.f || dJ > 1.f) && fabsf(A[v]) > thr;
      gr[v] = (off && !(dJ > 1.f)) ? fabsf(A[v]) : 0.f;
    }
    if (!__any(bad)) {
      bool gbad = false;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float rs = row_sum16(gr[v]);
        gbad |= !(dI[v] > 1.f) && dI[v] + rs > 1.f + kGershSlack;
      }
      if (!__any(gbad)) {
        if (!rough) {
          ok = true;
          break;
        }
        // large steps were taken: restore orthonormality exactly and re-derive A from G
        f4 Vc;
        orthonormalise(Vc);
        A = mtn(Vc, mtn(G, Vc));
        rough = false;
        continue;
      }
    }
    if (steps >= a.eig_steps) break;
    rough |= rotate() > kRoughNorm2;
    ++steps;
  }

  // Reduced-precision Gram (refine): G is the Gram matrix of the rounded block Yh, and Xres
  // holds Yh Dh^T with Dh the rounded residual Y' - Yh, so Gc = G + X + X^T is the Gram matrix
  // of Y' up to the residual's own rounding and Dh Dh^T (relative 2^-16 of G for bfloat16
  // inputs, 2^-22 for binary16).
  // The refinement cannot change W when every eigenvalue of G lies below 1 by more than the
  // spectral norm of X + X^T (Weyl), bounded here by 2 ||X||_F (the omitted Dh Dh^T is far
  // smaller): then W = I either way.
  if (refine && ok) {
    float dmax = fmaxf(fmaxf(dI[0], dI[1]), fmaxf(dI[2], dI[3]));
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) dmax = fmaxf(dmax, __shfl_xor(dmax, m));
    const float xf = sqrtf(wave_sum(Xres[0] * Xres[0] + Xres[1] * Xres[1] + Xres[2] * Xres[2] +
                                    Xres[3] * Xres[3]));
    if (dmax + 2.001f * xf < 1.f) refine = false;
  }
  f4 Gc = G;
  if (refine) {
    const f4 Xt = dform_transpose(Xres, tb, j, g);
#pragma unroll
    for (int v = 0; v < 4; ++v) Gc[v] = G[v] + (Xres[v] + Xt[v]);
  }
  float *Gl = a.G + (size_t)l * 256 + (4 * g) * 16 + j;
  if (ok) {
    f4 Vc;
    orthonormalise(Vc);
    if (refine) {
      // One FP32 refinement step of the eigenvectors against Gc: A = V^T Gc V and one
      // simultaneous rotation (its off-diagonal entries are of the size of the Gram's
      // rounding, so one step leaves a residual of second order), then the clip factors from
      // the refined diagonal. A block whose refined spectrum stays below 1 gets W = I.
      A = mtn(Vc, mtn(Gc, Vc));
      symmetrise();
      if (rotate() > kRoughNorm2) orthonormalise(Vc);
      symmetrise();
    }
    f4 H;
#pragma unroll
    for (int v = 0; v < 4; ++v) H[v] = (dI[v] > 1.f ? 1.f - rsqrtf(dI[v]) : 0.f) * Vt[v];
    const f4 S = mtn(Vt, H);  // V diag(h) V^T
#pragma unroll
    for (int v = 0; v < 4; ++v) Wout[v] = ((4 * g + v) == j ? 1.f : 0.f) - S[v];
  } else {
    // left to the per-lane Jacobi, which solves the rotated (corrected) Gram matrix
    f4 Vc;
    orthonormalise(Vc);
    A = mtn(Vc, mtn(Gc, Vc));
#pragma unroll
    for (int v = 0; v < 4; ++v) Gl[16 * v] = A[v];
  }
  *(f4 *)(Vl + j * 16 + 4 * g) = Vt;
  if (lane == 0) a.eflag[l] = steps | (ok ? 0 : 256);
  return ok;
}

// k_gram's warm mode: W of a certified block goes to a.W (row-major) for k_apply.
__device__ __forceinline__ void block_eigen_mfma(const BlockArgs &a, long long l, f4 G, f4 vd,
                                                 f4 vt, float *tb) {
  f4 W;
  if (eigen_mfma(a, l, G, vd, vt, tb, W)) {
    const int lane = threadIdx.x & 63;
    float *Wl = a.W + (size_t)l * 256 + (4 * (lane >> 4)) * 16 + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) Wl[16 * v] = W[v];
  }
}

// ---------------------------------------------------------------- Gram on MFMA

// One wavefront per block. In MFMA step (t, s) lane (r = lane&15, kk = lane>>4) supplies
// Y'[r][16t + 4kk + s] as both operands, so the 16x16x4 products accumulate
// G = sum_c Y'[:, c] Y'[:, c]^T. Result lane (j, g) register v = G[4g+v][j].
__global__ __launch_bounds__(256) void k_gram(BlockArgs a) {
  // per-wavefront transpose buffer for one 16 x 16 tile, row stride 20 floats (conflict-free
  // for both the 4-byte writes and the 16-byte reads)
  __shared__ __align__(16) float tbuf[4][16 * 20];
  if (a.sc && a.sc->done) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long l = (long long)blockIdx.x * 4 + wave;
  if (l >= a.nblk) return;
  const int r = lane & 15, kk = lane >> 4;
  const int pix = a.gradf ? row_pixel(a, l, r) : -1;
  const f4 *Yl = (const f4 *)(a.Y + (size_t)l * kRows * a.ncol) + lane;
  const float *Tp = pix >= 0 ? a.gradf + (size_t)pix * a.ncol + 4 * kk : nullptr;
  float *tb = tbuf[wave];
  f4 vd = {0.f, 0.f, 0.f, 0.f}, vt = {0.f, 0.f, 0.f, 0.f};
  if (a.V && a.eflag) load_basis(a, l, vd, vt);
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  f4 ycur = Yl[0];
  for (int t = 0; t < a.ntile; ++t) {
    // apply layout: this lane holds rows 4kk+s of column r of tile t (lane = 16*kk + r)
    const f4 ynext = t + 1 < a.ntile ? Yl[64 * (t + 1)] : ycur;
    f4 T = {0.f, 0.f, 0.f, 0.f};
    if (Tp) T = *(const f4 *)(Tp + 16 * t);
#pragma unroll
    for (int s = 0; s < 4; ++s) tb[(4 * kk + s) * 20 + r] = ycur[s];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // Gram layout: row r, columns 4kk..4kk+3 of the tile
    const f4 yg = *(const f4 *)(tb + r * 20 + 4 * kk);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const float y0 = fmaf(a.gY, T[0], yg[0]);
    const float y1 = fmaf(a.gY, T[1], yg[1]);
    const float y2 = fmaf(a.gY, T[2], yg[2]);
    const float y3 = fmaf(a.gY, T[3], yg[3]);
    acc = mfma4(y0, y0, acc);
    acc = mfma4(y1, y1, acc);
    acc = mfma4(y2, y2, acc);
    acc = mfma4(y3, y3, acc);
    ycur = ynext;
  }
  if (a.V && a.eflag) {
    block_eigen_mfma(a, l, acc, vd, vt, tb);
    return;
  }
  if (a.V) {
    // Warm start. With M and N held in the result layout (lane j + 16g, register
    // v = X[4g+v][j]) the four MFMA steps MFMA(M_v, N_v) accumulate M^T N.
    // 1) Re-orthogonalise the stored eigenvector basis V by one Newton-Schulz step,
    //    Vc = V (3I - V^T V) / 2, so rounding in the rotations never accumulates.
    // 2) Rotate the Gram matrix into it: Gt = Vc^T G Vc.
    const int j = lane & 15, g = lane >> 4;
    float *Vl = a.V + (size_t)l * 256;
    const float vd0 = Vl[(4 * g) * 16 + j], vd1 = Vl[(4 * g + 1) * 16 + j];
    const float vd2 = Vl[(4 * g + 2) * 16 + j], vd3 = Vl[(4 * g + 3) * 16 + j];
    const f4 vt = *(const f4 *)(Vl + j * 16 + 4 * g);  // result layout of V^T
    f4 X = {0.f, 0.f, 0.f, 0.f};
    X = mfma4(vd0, vd0, X);  // V^T V
    X = mfma4(vd1, vd1, X);
    X = mfma4(vd2, vd2, X);
    X = mfma4(vd3, vd3, X);
    f4 VX = {0.f, 0.f, 0.f, 0.f};
    VX = mfma4(vt[0], X[0], VX);  // (V^T)^T X = V X
    VX = mfma4(vt[1], X[1], VX);
    VX = mfma4(vt[2], X[2], VX);
    VX = mfma4(vt[3], X[3], VX);
    const float c0 = fmaf(1.5f, vd0, -0.5f * VX[0]), c1 = fmaf(1.5f, vd1, -0.5f * VX[1]);
    const float c2 = fmaf(1.5f, vd2, -0.5f * VX[2]), c3 = fmaf(1.5f, vd3, -0.5f * VX[3]);
    f4 P = {0.f, 0.f, 0.f, 0.f};
    P = mfma4(acc[0], c0, P);  // G^T Vc = G Vc
    P = mfma4(acc[1], c1, P);
    P = mfma4(acc[2], c2, P);
    P = mfma4(acc[3], c3, P);
    f4 Gt = {0.f, 0.f, 0.f, 0.f};
    Gt = mfma4(c0, P[0], Gt);  // Vc^T (G Vc)
    Gt = mfma4(c1, P[1], Gt);
    Gt = mfma4(c2, P[2], Gt);
    Gt = mfma4(c3, P[3], Gt);
    acc = Gt;
    Vl[(4 * g) * 16 + j] = c0;
    Vl[(4 * g + 1) * 16 + j] = c1;
    Vl[(4 * g + 2) * 16 + j] = c2;
    Vl[(4 * g + 3) * 16 + j] = c3;
  }
  float *Gl = a.G + (size_t)l * 256 + (4 * (lane >> 4)) * 16 + (lane & 15);
  Gl[0] = acc[0];
  Gl[16] = acc[1];
  Gl[32] = acc[2];
  Gl[48] = acc[3];
}

// ---------------------------------------------------------------- Jacobi eigen-solve

// One lane per block: the lane holds the upper triangle of its symmetric Gram matrix (136
// floats) and the eigenvector matrix V (256 floats) in registers and runs cyclic Jacobi
// sweeps (row order p < q). All register indices are compile-time constants (the sweep is
// fully unrolled). A rotation whose pivot |G_pq| is at most thr = kJacobiTol * ||G||_F in
// every lane of the wavefront is skipped; the solve stops when no pivot exceeds thr.
// With a stored basis (warm start) the input is V^T G V and the rotations continue V.
// Output: W = I - sum_k (1 - min(1, lambda_k^{-1/2})) v_k v_k^T, row-major.

constexpr int kMaxSweeps = 16;

__host__ __device__ constexpr int tri(int p, int q) { return p * 16 - p * (p - 1) / 2 + (q - p); }

template <int P, int Q>
__device__ __forceinline__ void jrot(float (&A)[136], float (&V)[256], float thr) {
  const float apq = A[tri(P, Q)];
  if (!__any(fabsf(apq) > thr)) return;
  const float app = A[tri(P, P)], aqq = A[tri(Q, Q)];
  float t = 0.f;
  if (fabsf(apq) > thr) {
    const float zeta = __fdividef(aqq - app, 2.f * apq);
    t = copysignf(__frcp_rn(fabsf(zeta) + sqrtf(fmaf(zeta, zeta, 1.f))), zeta);
  }
  const float c = rsqrtf(fmaf(t, t, 1.f)), s = t * c;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    if (k == P || k == Q) continue;
    const int ip = k < P ? tri(k, P) : tri(P, k);
    const int iq = k < Q ? tri(k, Q) : tri(Q, k);
    const float g = A[ip], h = A[iq];
    A[ip] = fmaf(c, g, -s * h);
    A[iq] = fmaf(s, g, c * h);
  }
  A[tri(P, P)] = fmaf(-t, apq, app);
  A[tri(Q, Q)] = fmaf(t, apq, aqq);
  A[tri(P, Q)] = 0.f;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const float g = V[k * 16 + P], h = V[k * 16 + Q];
    V[k * 16 + P] = fmaf(c, g, -s * h);
    V[k * 16 + Q] = fmaf(s, g, c * h);
  }
}

template <int P, int Q>
__device__ __forceinline__ void jsweep(float (&A)[136], float (&V)[256], float thr) {
  if constexpr (P < 15) {
    jrot<P, Q>(A, V, thr);
    if constexpr (Q < 15)
      jsweep<P, Q + 1>(A, V, thr);
    else
      jsweep<P + 1, P + 2>(A, V, thr);
  }
}

__global__ __launch_bounds__(64) void k_eig(BlockArgs a) {
  if (a.sc && a.sc->done) return;
  long long blk = (long long)blockIdx.x * 64 + threadIdx.x;
  bool valid = blk < a.nblk;
  if (a.eflag) {
    // Only the blocks k_gram could not certify. First the workgroup's statistics (summed
    // later by the finalize kernel, no atomics).
    const int f = valid ? a.eflag[blk] : 0;
    const bool mine = valid && (f & 256);
    int st = f & 255, mx = st, nv = valid ? 1 : 0;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      st += __shfl_xor(st, m);
      mx = max(mx, __shfl_xor(mx, m));
      nv += __shfl_xor(nv, m);
    }
    const unsigned long long fb = __ballot(mine);
    if (threadIdx.x == 0) {
      int4 r;
      r.x = st;
      r.y = mx;
      r.z = __popcll(fb);
      r.w = nv;
      *(int4 *)(a.estat + 4 * (size_t)blockIdx.x) = r;
    }
    if (!fb) return;
    // lanes without a flagged block mirror the first flagged one (run the same sweeps, store nothing)
    const long long first = __shfl(blk, __ffsll((long long)fb) - 1);
    if (!mine) blk = first;
    valid = mine;
  } else if (!valid) {
    blk = a.nblk - 1;  // duplicate a real block so every lane runs the same sweeps
  }
  // The Gram matrix from k_gram is symmetric; read its upper triangle.
  const float *Gl = a.G + (size_t)blk * 256;
  float A[136], V[256];
  float fro = 0.f;
#pragma unroll
  for (int p = 0; p < 16; ++p)
#pragma unroll
    for (int q = p; q < 16; ++q) {
      const float x = Gl[p * 16 + q];
      A[tri(p, q)] = x;
      fro = fmaf(p == q ? x : 2.f * x, x, fro);
    }
  if (a.V) {
    const f4 *v4 = (const f4 *)(a.V + (size_t)blk * 256);
#pragma unroll
    for (int k = 0; k < 64; ++k) {
      const f4 x = v4[k];
      V[4 * k] = x[0];
      V[4 * k + 1] = x[1];
      V[4 * k + 2] = x[2];
      V[4 * k + 3] = x[3];
    }
  } else {
#pragma unroll
    for (int k = 0; k < 256; ++k) V[k] = (k / 16 == k % 16) ? 1.f : 0.f;
  }
  const float thr = kJacobiTol * sqrtf(fro);
  int sweeps = 0;
  for (; sweeps < kMaxSweeps; ++sweeps) {
    float off = 0.f;
#pragma unroll
    for (int p = 0; p < 16; ++p)
#pragma unroll
      for (int q = p + 1; q < 16; ++q) off = fmaxf(off, fabsf(A[tri(p, q)]));
    if (!__any(off > thr)) break;
    jsweep<0, 1>(A, V, thr);
  }
  float h[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const float lam = A[tri(k, k)];
    h[k] = lam > 1.f ? 1.f - rsqrtf(lam) : 0.f;
  }
  if (valid) {
    // W row by row (W = I - V diag(h) V^T), written as it is formed
    f4 *w4 = (f4 *)(a.W + (size_t)blk * 256);
#pragma unroll
    for (int p = 0; p < 16; ++p) {
      float hv[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) hv[k] = h[k] * V[p * 16 + k];
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4) {
        f4 o;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int q = 4 * q4 + e;
          float acc = 0.f;
#pragma unroll
          for (int k = 0; k < 16; ++k) acc = fmaf(hv[k], V[q * 16 + k], acc);
          o[e] = (p == q ? 1.f : 0.f) - acc;
        }
        w4[p * 4 + q4] = o;
      }
    }
    if (a.V) {
      f4 *v4 = (f4 *)(a.V + (size_t)blk * 256);
#pragma unroll
      for (int k = 0; k < 64; ++k) v4[k] = (f4){V[4 * k], V[4 * k + 1], V[4 * k + 2], V[4 * k + 3]};
    }
  }
  if (a.sc && threadIdx.x == 0) {
    atomicMax(&a.sc->max_sweeps, sweeps);
    atomicAdd(&a.sc->sweep_sum, (unsigned long long)sweeps);
    atomicAdd(&a.sc->sweep_waves, 1ull);
  }
}

// ---------------------------------------------------------------- apply on MFMA + overlap-add

// Workgroup = one TA x TB tile of anchors, `waves` wavefronts; wavefront w owns column tiles
// t = w, w + waves, ... of every block of the tile, so the fixed-point overlap-add
// accumulators in LDS (extA x extB pixels x ncol columns) are private per column.
// MFMA step s: A = W[r][4g+s] (lane r + 16g), B = Y'[4g+s][tc] (lane tc + 16g);
// result lane (tc, g) register v = (W Y')[4g+v][tc] is written back in place.
__global__ __launch_bounds__(1024) void k_apply(BlockArgs a) {
  extern __shared__ int zacc_i[];  // fixed point: the result does not depend on the tiling
  int *zacc = zacc_i;
  if (a.sc && a.sc->done) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tc = lane & 15, g = lane >> 4;
  const int ta = blockIdx.x / a.ntB, tb = blockIdx.x - (blockIdx.x / a.ntB) * a.ntB;
  const int p0 = ta * a.TA, q0 = tb * a.TB;
  const int np = min(a.TA, a.n1 - p0), nq = min(a.TB, a.n2 - q0);
  const bool doz = a.zpart != nullptr;
  const int next = a.extA * a.extB;
  const int zs = a.ncol + 16;  // padded LDS row stride: the four row groups land in distinct banks
  if (doz) {
    for (int t = wave; t < a.ntile; t += a.waves)
      for (int e = g; e < next; e += 4) zacc[(size_t)e * zs + 16 * t + tc] = 0;
  }
  bool bad = false;
  // Window geometry of this lane's four rows 4g+s (fixed for the whole kernel).
  int ar[4], cr[4];
  bool rv[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int row = 4 * g + s;
    rv[s] = row < a.K && a.gradf != nullptr;
    ar[s] = row / a.k2;
    cr[s] = row - ar[s] * a.k2;
  }
  const bool hasT = a.gradf != nullptr;
  // Anchors are visited in a fixed order (row-major inside the tile); for each group of kU
  // anchors all loads are issued before any result is consumed, so each wavefront keeps
  // several 1 KB tiles in flight. Per column the overlap-add order is the anchor order.
  constexpr int kU = 4;
  const int nanch = np * nq;
  for (int anc0 = 0; anc0 < nanch; anc0 += kU) {
    long long lb[kU];
    int pixo[kU][4], zo[kU][4];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int anc = anc0 + u < nanch ? anc0 + u : nanch - 1;  // tail: repeat, not stored
      const int da = anc / nq, db = anc - (anc / nq) * nq;
      const int p = p0 + da, q = q0 + db;
      lb[u] = (long long)p * a.n2 + q;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        int i = p + ar[s];
        if (i >= a.n1) i -= a.n1;
        int j = q + cr[s];
        if (j >= a.n2) j -= a.n2;
        pixo[u][s] = rv[s] ? (i * a.n2 + j) * a.ncol : -1;
        zo[u][s] = (4 * g + s < a.K) ? ((da + ar[s]) * a.extB + (db + cr[s])) * zs : -1;
      }
    }
    for (int t = wave; t < a.ntile; t += a.waves) {
      const int col = 16 * t + tc;
      f4 wv[kU], y[kU];
      float T[kU][4];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        wv[u] = *(const f4 *)(a.W + (size_t)lb[u] * 256 + tc * 16 + 4 * g);
        y[u] = *(const f4 *)(a.Y + (size_t)lb[u] * kRows * a.ncol + t * 256 + lane * 4);
#pragma unroll
        for (int s = 0; s < 4; ++s) T[u][s] = (hasT && pixo[u][s] >= 0) ? a.gradf[pixo[u][s] + col] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        if (anc0 + u >= nanch) break;
        const float yp0 = fmaf(a.gY, T[u][0], y[u][0]);
        const float yp1 = fmaf(a.gY, T[u][1], y[u][1]);
        const float yp2 = fmaf(a.gY, T[u][2], y[u][2]);
        const float yp3 = fmaf(a.gY, T[u][3], y[u][3]);
        f4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma4(wv[u][0], yp0, acc);
        acc = mfma4(wv[u][1], yp1, acc);
        acc = mfma4(wv[u][2], yp2, acc);
        acc = mfma4(wv[u][3], yp3, acc);
        *(f4 *)(a.Y + (size_t)lb[u] * kRows * a.ncol + t * 256 + lane * 4) = acc;
        if (doz) {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (zo[u][v] >= 0) zacc[zo[u][v] + col] += to_fixed(acc[v], bad);
        }
      }
    }
  }
  if (doz) {
    int *zp = a.zpart + (size_t)blockIdx.x * next * a.ncol;
    for (int t = wave; t < a.ntile; t += a.waves)
      for (int e = g; e < next; e += 4)
        zp[(size_t)e * a.ncol + 16 * t + tc] = zacc[(size_t)e * zs + 16 * t + tc];
    flag_nonfinite(a.sc, bad);
  }
}

// ---------------------------------------------------------------- fused warm-iteration pass

// Steps 9-10 and the overlap-add of the next step 2 in one pass over Y (at most kFusedTiles
// column tiles: N3 <= 192 for the two-component field, N3 <= 128 for SSST's three; beyond 16
// tiles the accumulators of an 8 x 8 anchor tile outgrow the LDS and the tile shrinks to
// 8 x 4). Workgroup = one TA x TB anchor tile with kFW
// wavefronts; each wavefront takes anchors from a shared counter and keeps Y'_l (16 x ncol)
// in registers in the apply layout: loads Y_l and T_l, forms the Gram matrix (column tiles
// transposed in pairs through LDS into the Gram operand layout), diagonalises it on MFMA
// (eigen_mfma), applies W_l on MFMA and stores Y+_l. The overlap-add goes to fixed-point LDS
// accumulators with integer atomics, so the wavefronts never wait for each other and the sum
// does not depend on their order. Blocks eigen_mfma cannot certify keep Y'_l in Y and are
// finished by k_eig and k_fixup.
constexpr int kFW = 8;
constexpr int kFusedTiles = 24;

template <int NT>
__global__ __launch_bounds__(kFW * 64) void k_block_fused(BlockArgs a) {
  extern __shared__ __align__(16) float zacc_f[];
  __shared__ int next_anchor;
  int *zacc = reinterpret_cast<int *>(zacc_f);
  if (a.sc && a.sc->done) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tc = lane & 15, g = lane >> 4;
  const int tile = xcd_block(blockIdx.x, gridDim.x);  // neighbouring tiles share an L2
  const int ta = tile / a.ntB, tb_ = tile - (tile / a.ntB) * a.ntB;
  const int p0 = ta * a.TA, q0 = tb_ * a.TB;
  const int np = min(a.TA, a.n1 - p0), nq = min(a.TB, a.n2 - q0);
  const int next = a.extA * a.extB;
  const int zs = a.ncol + 16;
  // this wavefront's two transpose tiles (row stride 20 floats)
  float *tbw = zacc_f + (size_t)next * zs + wave * 640;
  // zs and ncol are multiples of 4 (ncol of 32), so the accumulators are cleared and copied
  // out 16 bytes per lane
  int4 *zacc4 = reinterpret_cast<int4 *>(zacc_f);
  for (int e = threadIdx.x; e < (next * zs) >> 2; e += kFW * 64) zacc4[e] = int4{0, 0, 0, 0};
  if (threadIdx.x == 0) next_anchor = kFW;
  // rows 4g+s of this lane: window offsets (fixed for the kernel); rows >= K are padding
  int ar[4], cr[4];
  float tw[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int row = 4 * g + s;
    const bool rv = row < a.K;
    ar[s] = rv ? row / a.k2 : 0;
    cr[s] = rv ? row - (row / a.k2) * a.k2 : 0;
    tw[s] = rv ? a.gY : 0.f;
  }
  __syncthreads();
  bool bad = false;
  const int nanch = np * nq;
  // anchors are handed out dynamically (the eigen-solve cost varies a lot between blocks)
  for (int idx = wave; idx < nanch;) {
    const int da = idx / nq, db = idx - (idx / nq) * nq;
    const int p = p0 + da, q = q0 + db;
    const long long lb = (long long)p * a.n2 + q;
    const float *gp[4];
    int zo[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      int i = p + ar[s];
      if (i >= a.n1) i -= a.n1;
      int j = q + cr[s];
      if (j >= a.n2) j -= a.n2;
      gp[s] = a.gradf + (size_t)(i * a.n2 + j) * a.ncol + tc;  // padding rows: a real pixel, weight 0
      zo[s] = ((da + ar[s]) * a.extB + (db + cr[s])) * zs + tc;
    }
    float *Yl = a.Y + (size_t)lb * kRows * a.ncol + lane * 4;
    // all loads of the block first, then Y' = Y + g_Y T in the apply layout
    f4 y[NT];
    float T[NT][4];
    f4 vd, vt;
    load_basis(a, lb, vd, vt);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      // Y is streamed (read and written once per pass): non-temporal, so that the L2 keeps
      // the gradient-field rows that the neighbouring windows of the tile read again
      y[t] = __builtin_nontemporal_load((const f4 *)(Yl + t * 256));
#pragma unroll
      for (int s = 0; s < 4; ++s) T[t][s] = gp[s][16 * t];
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int s = 0; s < 4; ++s) y[t][s] = fmaf(tw[s], T[t][s], y[t][s]);
    // Gram: two column tiles per LDS round trip, transposed into the operand layout
    // (lane r + 16kk: row r, columns 4kk..4kk+3 of the tile), accumulating Y' Y'^T. With
    // reduced-precision inputs one 16x16x32 MFMA takes both tiles' eight columns per lane
    // (A and B are the same registers, so any fixed column-to-slot assignment is a valid
    // order of the sum).
    f4 G = {0.f, 0.f, 0.f, 0.f};
    f4 X = {0.f, 0.f, 0.f, 0.f};  // reduced precision: Yh Dh^T (rounded block x its residual)
    const int prec = a.gram_prec;
#pragma unroll
    for (int t = 0; t < NT; t += 2) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        tbw[(4 * g + s) * 20 + tc] = y[t][s];
        tbw[320 + (4 * g + s) * 20 + tc] = y[t + 1][s];
      }
      wave_lds_sync();
      const f4 y0 = *(const f4 *)(tbw + tc * 20 + 4 * g);
      const f4 y1 = *(const f4 *)(tbw + 320 + tc * 20 + 4 * g);
      wave_lds_sync();
      if (prec == 0) {
        G = mfma4(y0[0], y0[0], G);
        G = mfma4(y0[1], y0[1], G);
        G = mfma4(y0[2], y0[2], G);
        G = mfma4(y0[3], y0[3], G);
        G = mfma4(y1[0], y1[0], G);
        G = mfma4(y1[1], y1[1], G);
        G = mfma4(y1[2], y1[2], G);
        G = mfma4(y1[3], y1[3], G);
      } else if (prec == 1) {
        bf8 v, r;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          v[s] = (__bf16)y0[s];
          v[4 + s] = (__bf16)y1[s];
          r[s] = (__bf16)(y0[s] - (float)v[s]);
          r[4 + s] = (__bf16)(y1[s] - (float)v[4 + s]);
        }
        G = __builtin_amdgcn_mfma_f32_16x16x32_bf16(v, v, G, 0, 0, 0);
        X = __builtin_amdgcn_mfma_f32_16x16x32_bf16(v, r, X, 0, 0, 0);
      } else {
        h8 v, r;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          v[s] = (_Float16)y0[s];
          v[4 + s] = (_Float16)y1[s];
          r[s] = (_Float16)(y0[s] - (float)v[s]);
          r[4 + s] = (_Float16)(y1[s] - (float)v[4 + s]);
        }
        G = __builtin_amdgcn_mfma_f32_16x16x32_f16(v, v, G, 0, 0, 0);
        X = __builtin_amdgcn_mfma_f32_16x16x32_f16(v, r, X, 0, 0, 0);
      }
    }
    // Y+ below is a spectral-norm projection (entries in [-1, 1]) of Y'; a non-finite Y'
    // shows in its Gram matrix, so that is the one check needed before the fixed-point sum.
    const bool fin = isfinite(G[0] + G[1] + G[2] + G[3]);
    bad |= !fin;
    f4 W;
    if (eigen_mfma(a, lb, G, vd, vt, tbw, W, prec != 0, X) && fin) {
      // Y+ = W Y' (W symmetric: its D-form register s of lane (r, g) is W[r][4g+s]),
      // stored in place and added to the tile's overlap-add accumulators
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        f4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma4(W[0], y[t][0], acc);
        acc = mfma4(W[1], y[t][1], acc);
        acc = mfma4(W[2], y[t][2], acc);
        acc = mfma4(W[3], y[t][3], acc);
        __builtin_nontemporal_store(acc, (f4 *)(Yl + t * 256));
        // rows >= K are padding (their zo names the anchor pixel) and add nothing; the test
        // is uniform over the wave when every row is real
        if (a.K == kRows) {
#pragma unroll
          for (int s = 0; s < 4; ++s) atomicAdd(&zacc[zo[s] + 16 * t], to_fixed_bounded(acc[s]));
        } else {
#pragma unroll
          for (int s = 0; s < 4; ++s)
            if (4 * g + s < a.K) atomicAdd(&zacc[zo[s] + 16 * t], to_fixed_bounded(acc[s]));
        }
      }
    } else {
      // left to k_eig / k_fixup: keep Y'
#pragma unroll
      for (int t = 0; t < NT; ++t) *(f4 *)(Yl + t * 256) = y[t];
    }
    int nxt = 0;
    if (lane == 0) nxt = atomicAdd(&next_anchor, 1);
    idx = __shfl(nxt, 0);
  }
  flag_nonfinite(a.sc, bad);
  __syncthreads();
  // the tile's partial: a pixel row per wave and trip (ncol / 4 <= 96 quads: one or two per
  // lane), 16 bytes per lane, four rows in flight
  int4 *zp4 = reinterpret_cast<int4 *>(a.zpart + (size_t)tile * next * a.ncol);
  const int nc4 = a.ncol >> 2, zs4 = zs >> 2;
  for (int c = lane; c < nc4; c += 64) {
    for (int px = wave; px < next; px += 4 * kFW) {
      // rows past the end read row 0 again and are not stored
      const int p1 = px + kFW < next ? px + kFW : 0, p2 = px + 2 * kFW < next ? px + 2 * kFW : 0;
      const int p3 = px + 3 * kFW < next ? px + 3 * kFW : 0;
      const int4 v0 = zacc4[px * zs4 + c], v1 = zacc4[p1 * zs4 + c];
      const int4 v2 = zacc4[p2 * zs4 + c], v3 = zacc4[p3 * zs4 + c];
      zp4[(size_t)px * nc4 + c] = v0;
      if (p1) zp4[(size_t)p1 * nc4 + c] = v1;
      if (p2) zp4[(size_t)p2 * nc4 + c] = v2;
      if (p3) zp4[(size_t)p3 * nc4 + c] = v3;
    }
  }
}

// Finishes the blocks k_block_fused left uncertified once k_eig has written their W: one
// wavefront per anchor tile applies W to Y' and adds the result to the tile's fixed-point
// overlap-add partial.
__global__ __launch_bounds__(64) void k_fixup(BlockArgs a) {
  if (a.sc && a.sc->done) return;
  const int lane = threadIdx.x, tc = lane & 15, g = lane >> 4;
  const int ta = blockIdx.x / a.ntB, tb_ = blockIdx.x - (blockIdx.x / a.ntB) * a.ntB;
  const int p0 = ta * a.TA, q0 = tb_ * a.TB;
  const int np = min(a.TA, a.n1 - p0), nq = min(a.TB, a.n2 - q0);
  const int nanch = np * nq;  // <= 64
  bool mine = false;
  if (lane < nanch) {
    const int da = lane / nq, db = lane - (lane / nq) * nq;
    mine = (a.eflag[(long long)(p0 + da) * a.n2 + (q0 + db)] & 256) != 0;
  }
  unsigned long long todo = __ballot(mine);
  if (!todo) return;
  int *zp = a.zpart + (size_t)blockIdx.x * a.extA * a.extB * a.ncol;
  bool bad = false;
  while (todo) {
    const int anc = __ffsll((long long)todo) - 1;
    todo &= todo - 1;
    const int da = anc / nq, db = anc - (anc / nq) * nq;
    const long long lb = (long long)(p0 + da) * a.n2 + (q0 + db);
    const f4 wv = *(const f4 *)(a.W + (size_t)lb * 256 + tc * 16 + 4 * g);
    float *Yl = a.Y + (size_t)lb * kRows * a.ncol + lane * 4;
    for (int t = 0; t < a.ntile; ++t) {
      const f4 yp = *(const f4 *)(Yl + t * 256);
      f4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = mfma4(wv[0], yp[0], acc);
      acc = mfma4(wv[1], yp[1], acc);
      acc = mfma4(wv[2], yp[2], acc);
      acc = mfma4(wv[3], yp[3], acc);
      *(f4 *)(Yl + t * 256) = acc;
      const int col = 16 * t + tc;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int row = 4 * g + s;
        if (row < a.K) {
          const int ar = row / a.k2, cr = row - (row / a.k2) * a.k2;
          zp[(size_t)((da + ar) * a.extB + (db + cr)) * a.ncol + col] += to_fixed(acc[s], bad);
        }
      }
    }
  }
  flag_nonfinite(a.sc, bad);
}

// ---------------------------------------------------------------- layout converters

// src: nblk blocks of K rows x ncols_src (row-major). paper_cols: column 2b+comp <-> internal
// comp*Bp + b; otherwise column c <-> c. Internal padding (rows >= K, extra columns) is zero.
__global__ void k_pack_blocks(const float *src, float *Y, long long nblk, int K, int ncols_src,
                              int ncol, int paper_cols, int Bp) {
  const long long total = nblk * kRows * ncol;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long l = e / (kRows * ncol);
    const int rem = (int)(e - l * kRows * ncol);
    const int t = rem / 256, w = rem - t * 256;
    const int L = w >> 2, s = w & 3;
    const int row = 4 * (L >> 4) + s, c = 16 * t + (L & 15);
    int cs;
    if (paper_cols) {
      const int comp = c / Bp, b = c - comp * Bp;
      cs = 2 * b + comp;
    } else {
      cs = c;
    }
    float val = 0.f;
    if (row < K && cs < ncols_src) val = src[(l * K + row) * ncols_src + cs];
    Y[e] = val;
  }
}

__global__ void k_unpack_blocks(const float *Y, float *dst, long long nblk, int K, int ncols_src,
                                int ncol, int paper_cols, int Bp) {
  const long long total = nblk * K * ncols_src;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long l = e / ((long long)K * ncols_src);
    const int rem = (int)(e - l * K * ncols_src);
    const int row = rem / ncols_src, cs = rem - row * ncols_src;
    int c;
    if (paper_cols) {
      c = (cs & 1) * Bp + (cs >> 1);
    } else {
      c = cs;
    }
    const int t = c >> 4, tc = c & 15;
    const int L = 16 * (row >> 2) + tc, s = row & 3;
    dst[e] = Y[l * kRows * ncol + t * 256 + L * 4 + s];
  }
}

inline int grid_for(long long n, int nt, int per) {
  long long g = (n + (long long)nt * per - 1) / ((long long)nt * per);
  if (g < 1) g = 1;
  if (g > 65535) g = 65535;
  return (int)g;
}

}  // namespace

hipError_t launch_gram(const BlockArgs &a, hipStream_t st) {
  const long long g = (a.nblk + 3) / 4;
  hipLaunchKernelGGL(k_gram, dim3((unsigned)g), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_eig(const BlockArgs &a, hipStream_t st) {
  const long long g = (a.nblk + 63) / 64;
  hipLaunchKernelGGL(k_eig, dim3((unsigned)g), dim3(64), 0, st, a);
  return hipGetLastError();
}

size_t fused_lds_bytes(const BlockArgs &a) {
  return (size_t)a.extA * a.extB * (a.ncol + 16) * sizeof(float) + (size_t)kFW * 640 * sizeof(float);
}

bool fused_supported(const BlockArgs &a) {
  // ntile = 2 ceil(N3/16) is even
  return a.ntile <= kFusedTiles && a.ntile % 2 == 0 && a.TA * a.TB <= 64 && a.zpart && a.gradf &&
         a.V && a.eflag;
}

template <int NT>
hipError_t launch_fused_nt(const BlockArgs &a, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL(k_block_fused<NT>, dim3((unsigned)(a.ntA * a.ntB)), dim3(kFW * 64), lds, st,
                     a);
  return hipGetLastError();
}

template <int NT>
hipError_t allow_lds_nt(int bytes) {
  return hipFuncSetAttribute((const void *)k_block_fused<NT>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

// Raises the dynamic-LDS limit of the kernels that take it, once per process (a host-side
// attribute, so it is done before any stream work that might be captured into a graph).
hipError_t configure_block_kernels() {
  // once per device (a bit per device id; a repeated call from a racing thread is harmless)
  static std::atomic<unsigned long long> done{0};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const unsigned long long bit = dev < 64 ? 1ull << dev : 0ull;
  if (bit && (done.load(std::memory_order_acquire) & bit)) return hipSuccess;
  const int bytes = (int)kLdsLimit;
  e = hipFuncSetAttribute((const void *)k_apply, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess) e = allow_lds_nt<2>(bytes);
  if (e == hipSuccess) e = allow_lds_nt<4>(bytes);
  if (e == hipSuccess) e = allow_lds_nt<6>(bytes);
  if (e == hipSuccess) e = allow_lds_nt<8>(bytes);
  if (e == hipSuccess) e = allow_lds_nt<10>(bytes);
  if (e == hipSuccess) e = allow_lds_nt<12>(bytes);
  if (e == hipSuccess) e = allow_lds_nt<14>(bytes);
  if (e == hipSuccess) e = allow_lds_nt<16>(bytes);
  if (e == hipSuccess) e = allow_lds_nt<18>(bytes);
  if (e == hipSuccess) e = allow_lds_nt<20>(bytes);
  if (e == hipSuccess) e = allow_lds_nt<22>(bytes);
  if (e == hipSuccess) e = allow_lds_nt<24>(bytes);
  if (e == hipSuccess && bit) done.fetch_or(bit, std::memory_order_release);
  return e;
}

hipError_t launch_block_fused(const BlockArgs &a, hipStream_t st) {
  const size_t lds = fused_lds_bytes(a);
  switch (a.ntile) {
    case 2: return launch_fused_nt<2>(a, lds, st);
    case 4: return launch_fused_nt<4>(a, lds, st);
    case 6: return launch_fused_nt<6>(a, lds, st);
    case 8: return launch_fused_nt<8>(a, lds, st);
    case 10: return launch_fused_nt<10>(a, lds, st);
    case 12: return launch_fused_nt<12>(a, lds, st);
    case 14: return launch_fused_nt<14>(a, lds, st);
    case 16: return launch_fused_nt<16>(a, lds, st);
    case 18: return launch_fused_nt<18>(a, lds, st);
    case 20: return launch_fused_nt<20>(a, lds, st);
    case 22: return launch_fused_nt<22>(a, lds, st);
    case 24: return launch_fused_nt<24>(a, lds, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fixup(const BlockArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(k_fixup, dim3((unsigned)(a.ntA * a.ntB)), dim3(64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_apply(const BlockArgs &a, hipStream_t st) {
  const unsigned g = (unsigned)(a.ntA * a.ntB);
  hipLaunchKernelGGL(k_apply, dim3(g), dim3(64 * a.waves), a.zpart ? a.lds : 0, st, a);
  return hipGetLastError();
}

hipError_t launch_pack_blocks(const float *src, float *Y, long long nblk, int K, int ncols_src,
                              int ncol, int paper_cols, int n3, int Bp, hipStream_t st) {
  (void)n3;
  hipLaunchKernelGGL(k_pack_blocks, dim3(grid_for(nblk * kRows * ncol, 256, 4)), dim3(256), 0, st,
                     src, Y, nblk, K, ncols_src, ncol, paper_cols, Bp);
  return hipGetLastError();
}

hipError_t launch_unpack_blocks(const float *Y, float *dst, long long nblk, int K, int ncols_src,
                                int ncol, int paper_cols, int n3, int Bp, hipStream_t st) {
  (void)n3;
  hipLaunchKernelGGL(k_unpack_blocks, dim3(grid_for(nblk * K * ncols_src, 256, 4)), dim3(256), 0,
                     st, Y, dst, nblk, K, ncols_src, ncol, paper_cols, Bp);
  return hipGetLastError();
}

}  // namespace s3ttv
