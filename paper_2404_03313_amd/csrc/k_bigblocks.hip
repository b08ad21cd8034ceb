// Block pass for blocks of more than 16 rows (K = k1 k2 up to 100; the paper's experiments use
// 10 x 10 windows, Sec. IV-A): Alg. 1 steps 9-10 and the overlap-add of step 2, one workgroup
// per block.
//
// Per block l (rows r = a k2 + c, columns in the comp-major field layout):
//   Y' = Y + g_Y P_l D D_s u'                      (step 9, written back in place)
//   G  = Y' Y'^T                                    (K x K, FP32 sums, 32-column chunks)
//   if every Gershgorin row bound of G is <= 1, no singular value of Y' exceeds 1 and step 10
//   leaves Y' unchanged; otherwise
//   A = V^T G V from the stored (orthonormal) eigenbasis V of the previous iteration; from the
//   second iteration on, up to kSimSteps simultaneous rotation steps on MFMA (all pairs at
//   once, J = I + K + K^2/2, see below) usually reach the certificate; then
//   parallel cyclic Jacobi on A (round-robin pair order, all K/2 rotations of a step at once:
//   a row pass and a column pass, accumulated into V) until a certificate holds: every
//   off-diagonal entry in a row or column whose diagonal exceeds 0.999 is at most
//   1e-6 ||A||_F (about the FP32 rounding level of the rotations), and every other row has a
//   Gershgorin bound <= 1, so no eigenvalue above 1 hides among them (the clip factor
//   1 - lambda^-1/2 is continuous at 1, so eigenvalues next to 1 need no separation). A sweep
//   rotates only pairs with a row that failed this test when the sweep began (a pair of two
//   certified rows needs nothing; from the fifth sweep on, every pair), so with the warm basis
//   a step touches a few rows and columns of A instead of all of them;
//   lambda_i = A_ii, the diagonal of the certified A (the rows with A_ii > 1 are among those
//   whose off-diagonal entries passed the test, so A_ii is their eigenvalue to second order);
//   one Newton-Schulz step V <- V (3 I - V^T V) / 2 restores orthonormality lost to rounding
//   (unless Newton-Schulz steps already followed the last change of V);
//   Y+ = Y' - M Y',  M = V_R diag(1 - lambda^-1/2) V_R^T   over R = {i : lambda_i > 1}
// which is the spectral clip of step 10 (eqs. ProxConjugate, prox_nuclear_norm), formed as
// Y' - U^T (U Y') with U = diag(1 - lambda^-1/2)^1/2 V_R^T when at most 32 directions clip,
// else through M. The basis is kept for the next iteration.
//
// The overlap-add sum_l P_l^T Y_l is a gather (each pixel reads its K windows in a fixed
// order), so results are reproducible.
#include <atomic>
#include "s3ttv_internal.h"

namespace s3ttv {

namespace {

constexpr int kNT = 256;   // overlap-add and fill kernels
constexpr int kBT = 512;   // the block kernel: eight wavefronts per block
constexpr int kNW = kBT / 64;
constexpr int kChunk = 32;
// Row stride of a staged Y' chunk in the Gram: 34 makes the MFMA operand reads of a half-wave
// (rows i = 0..15, columns g = 0..1) hit 32 distinct banks.
constexpr int kGS = kChunk + 2;
// 16 x 16 Gram tiles per wave: ceil(28 / kNW) for K <= 112 (7 x 7 tiles, upper triangle).
constexpr int kGramTiles = (28 + kNW - 1) / kNW;

typedef float f4 __attribute__((ext_vector_type(4)));

// Chunk staging: thread t moves rows t / 32 + kRowStep k, column t mod 32, kStage of them.
constexpr int kRowStep = kBT / kChunk;
constexpr int kStage = (kBigMax * kChunk + kBT - 1) / kBT;
static_assert(kChunk == 32 && kBT % kChunk == 0, "chunk staging");
// Rows whose diagonal exceeds this take part in the off-diagonal test of the certificate.
constexpr float kNearOne = 0.999f;
// Sweeps that rotate only pairs touching a row that failed the certificate; later sweeps
// rotate every pair above the skip threshold.
constexpr int kRestricted = 4;
// Pairs a wave rotates in a rotation pass: a group of pairs has at most
// ceil((kBigMax / 2) / (kNW / 2)) = 13 of them. The K / 2 <= 50 rotations of a step fit the
// lanes of one wavefront.
constexpr int kBatch = 13;
static_assert(kBigMax <= 100 && kBT % 128 == 0 && kBatch * (kNW / 2) >= kBigMax / 2,
              "rotation pass mapping: one batch covers a wave's pairs");
static_assert(4 * kBigMax <= kBT, "certificate: four threads per row");

// Value of x in lane u of the wave (u a compile-time constant).
__device__ inline float lane_value(float x, int u) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), u));
}

__device__ inline int wrapm(int x, int n) { return x < 0 ? x + n : (x >= n ? x - n : x); }

// Round-robin pairing of m (even) indices, step s (0 <= s < m - 1), pair k (0 <= k < m / 2):
// index m - 1 stays, the others rotate.
__device__ inline void rr_pair(int m, int s, int k, int &p, int &q) {
  const int n = m - 1;  // 0 <= s < n, 0 <= k < m / 2
  int x = n, y = s;
  if (k != 0) {
    x = s + k;
    y = s + n - k;
    x = x >= n ? x - n : x;
    y = y >= n ? y - n : y;
  }
  p = min(x, y);
  q = max(x, y);
}

// A band of NJ 16 x 16 tiles (rows 16 I .., columns 16 (J0 + j) ..) of
// C = op(A) B over k < kd on v_mfma_f32_16x16x4_f32, with op(A)[r][k] = TA ? A[k * as + r] :
// A[r * as + k] and B[k][c] = B[k * bs + c]. Lane i + 16 g supplies op(A)[16 I + i][k0 + g]
// (shared by the band) and B[k0 + g][16 (J0 + j) + i]; result lane i + 16 g, register v of
// tile j holds C[16 I + 4 g + v][16 (J0 + j) + i]. Row and column indices are clamped to
// nr - 1, nc - 1 (those outputs are not used) and k >= kd contributes zero, so every load is
// unconditional. The loop is software-pipelined by hand (two register sets): the compiler does
// not unroll loops around MFMA.
template <bool TA, int NJ>
__device__ __forceinline__ void mfma_band(const float *A, int as, const float *B, int bs, int kd,
                                          int nr, int nc, int I, int J0, int i16, int g4,
                                          f4 acc[NJ]) {
#pragma unroll
  for (int j = 0; j < NJ; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
  const int r = min(16 * I + i16, nr - 1);
  int c[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) c[j] = min(16 * (J0 + j) + i16, nc - 1);
  // one MFMA k-step (k0 .. k0 + 3) per load; the next step's operands are loaded while the
  // current step's MFMAs run. k past kd reads row kd - 1 and is zeroed at the MFMA (not at
  // the load, which would make the loads wait)
  const int nk = (kd + 3) >> 2;
  float a0, a1, b0[NJ], b1[NJ];
  auto load = [&](int k4, float &av, float (&bv)[NJ]) {
    const int k = min(4 * k4 + g4, kd - 1);
    av = TA ? A[k * as + r] : A[r * as + k];
#pragma unroll
    for (int j = 0; j < NJ; ++j) bv[j] = B[k * bs + c[j]];
  };
  auto step = [&](int k4, float av, const float (&bv)[NJ]) {
    const float a = 4 * k4 + g4 < kd ? av : 0.f;
#pragma unroll
    for (int j = 0; j < NJ; ++j)
      acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv[j], acc[j], 0, 0, 0);
  };
  load(0, a0, b0);
  for (int k4 = 0; k4 < nk; k4 += 2) {
    const bool more = k4 + 1 < nk;
    if (more) load(k4 + 1, a1, b1);
    step(k4, a0, b0);
    if (k4 + 2 < nk) load(k4 + 2, a0, b0);
    if (more) step(k4 + 1, a1, b1);
  }
}

// K x K products C = op(A) B (K <= 112, so at most kMaxT = 7 tiles of 16 per side), computed
// into registers and written by a separate release call, so that after a barrier the result
// may overwrite one of its operands.
constexpr int kMaxT = 7;
static_assert(kBigMax <= 16 * kMaxT && kMaxT <= kNW, "one row of tiles per wave");

// General product: wave w < nt computes row tile I = w against every column tile (the A
// operand is read once per row).
template <bool TA>
__device__ __forceinline__ void prod_rows(const float *A, int as, const float *B, int bs, int K,
                                          int wave, int i16, int g4, f4 acc[kMaxT]) {
  const int nt = (K + 15) >> 4;
  // tiles past nt (K <= 96) read clamped columns and are not released
  if (wave < nt) mfma_band<TA, kMaxT>(A, as, B, bs, K, K, K, wave, 0, i16, g4, acc);
}

template <typename Out>
__device__ __forceinline__ void release_rows(int K, int wave, int i16, int g4, const f4 acc[kMaxT],
                                    Out out) {
  const int nt = (K + 15) >> 4;
  if (wave >= nt) return;
#pragma unroll
  for (int j = 0; j < kMaxT; ++j) {
    const int cc = 16 * j + i16;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * wave + 4 * g4 + v;
      if (j < nt && r < K && cc < K) out(r, cc, acc[j][v]);
    }
  }
}

// Product with a symmetric result (V^T V, V^T G V, K^T K, U^T U): only the tiles on and
// above the diagonal are formed, dealt round-robin to the waves (at most kSymHold each), and
// each entry above the diagonal is written to both (r, c) and (c, r), so the result is exactly
// symmetric.
constexpr int kSymHold = (kMaxT * (kMaxT + 1) / 2 + kNW - 1) / kNW;

// Upper tile number t (row-major over I <= J) -> (I, J).
__device__ inline void upper_tile(int t, int nt, int &I, int &J) {
  I = 0;
  while (t >= nt - I) {
    t -= nt - I;
    ++I;
  }
  J = I + t;
}

template <bool TA>
__device__ __forceinline__ void prod_sym(const float *A, int as, const float *B, int bs, int K,
                                         int wave, int i16, int g4, f4 acc[kSymHold],
                                         int kd = 0) {
  // K x K result; the contraction runs over kd (K when 0)
  if (kd <= 0) kd = K;
  const int nt = (K + 15) >> 4, nup = nt * (nt + 1) / 2;
  // all of the wave's tiles advance together, so their MFMA chains are independent; a tile
  // past nup repeats tile 0 and is not released
  int r[kSymHold], c[kSymHold];
#pragma unroll
  for (int m = 0; m < kSymHold; ++m) {
    int I, J;
    const int t = wave + kNW * m;
    upper_tile(t < nup ? t : 0, nt, I, J);
    r[m] = min(16 * I + i16, K - 1);
    c[m] = min(16 * J + i16, K - 1);
    acc[m] = f4{0.f, 0.f, 0.f, 0.f};
  }
  const int nk = (kd + 3) >> 2;
  float a0[kSymHold], b0[kSymHold], a1[kSymHold], b1[kSymHold];
  auto load = [&](int k4, float (&av)[kSymHold], float (&bv)[kSymHold]) {
    const int k = min(4 * k4 + g4, kd - 1);
#pragma unroll
    for (int m = 0; m < kSymHold; ++m) {
      av[m] = TA ? A[k * as + r[m]] : A[r[m] * as + k];
      bv[m] = B[k * bs + c[m]];
    }
  };
  auto step = [&](int k4, const float (&av)[kSymHold], const float (&bv)[kSymHold]) {
    const bool in = 4 * k4 + g4 < kd;
#pragma unroll
    for (int m = 0; m < kSymHold; ++m)
      acc[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(in ? av[m] : 0.f, bv[m], acc[m], 0, 0, 0);
  };
  load(0, a0, b0);
  for (int k4 = 0; k4 < nk; k4 += 2) {
    const bool more = k4 + 1 < nk;
    if (more) load(k4 + 1, a1, b1);
    step(k4, a0, b0);
    if (k4 + 2 < nk) load(k4 + 2, a0, b0);
    if (more) step(k4 + 1, a1, b1);
  }
}

template <typename Out>
__device__ __forceinline__ void release_sym(int K, int wave, int i16, int g4,
                                            const f4 acc[kSymHold], Out out) {
  const int nt = (K + 15) >> 4, nup = nt * (nt + 1) / 2;
#pragma unroll
  for (int m = 0; m < kSymHold; ++m) {
    const int t = wave + kNW * m;
    if (t < nup) {
      int I, J;
      upper_tile(t, nt, I, J);
      const int cc = 16 * J + i16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * I + 4 * g4 + v;
        if (r < K && cc < K && r <= cc) {
          out(r, cc, acc[m][v]);
          if (r != cc) out(cc, r, acc[m][v]);
        }
      }
    }
  }
}

// Entries of U (at most 32 x K) a thread gathers in registers before writing them over the basis.
constexpr int kUtRegs = (32 * kBigMax + kBT - 1) / kBT;

// Row stride of the two K x K arrays: odd, and above the Gram chunk stride kGS (the chunks are
// staged in the basis array before the basis is loaded).
__host__ __device__ constexpr int big_stride(int K) { return K + 1 > kGS + 1 ? K + 1 : kGS + 1; }

// A K x K row-major matrix from global memory into LDS rows of stride KS, in two rounds of
// kCopyRegs entries per thread; each round issues all of its loads before its first store.
constexpr int kCopyRegs = (kBigMax * kBigMax + 2 * kBT - 1) / (2 * kBT);
__device__ __forceinline__ void copy_in(const float *src, float *dst, int K, int KS, int tid) {
  int r = tid / K, c = tid - (tid / K) * K;
  const int dr = kBT / K, dc = kBT - (kBT / K) * K;
  for (int j0 = 0; j0 < 2 * kCopyRegs; j0 += kCopyRegs) {
    float x[kCopyRegs];
#pragma unroll
    for (int j = 0; j < kCopyRegs; ++j)
      if ((j0 + j) * kBT < K * K) x[j] = src[min(tid + (j0 + j) * kBT, K * K - 1)];
#pragma unroll
    for (int j = 0; j < kCopyRegs; ++j) {
      if (tid + (j0 + j) * kBT < K * K) dst[r * KS + c] = x[j];
      r += dr;
      c += dc;
      if (c >= K) {
        c -= K;
        ++r;
      }
    }
  }
}

// Simultaneous rotation steps before the cyclic sweeps (warm-started iterations): at most this
// many, each damped to ||K||_F <= kSimCap.
constexpr int kSimSteps = 12;
constexpr float kSimCap = 0.7f;
// Orthonormality defect ||V^T V - I|| the Newton-Schulz steps of a simultaneous step aim below:
// the FP32 products that form V J and V^T V leave defects of this order themselves.
constexpr float kDriftTol = 1e-7f;

// The block's rows of Y (K x ncol, row-major) as a buffer resource: the chunk loops address
// an entry by one per-lane byte offset (row srow, column scol) plus a wave-uniform one (the
// chunk's column and the row step), so the staging needs no per-row address registers.
// 0x00020000: the third descriptor word of a raw 32-bit buffer on gfx9-family chips.
__device__ inline __amdgpu_buffer_rsrc_t y_rsrc(float *Yb, int K, int ncol) {
  return __builtin_amdgcn_make_buffer_rsrc(Yb, (short)0, K * ncol * (int)sizeof(float), 0x00020000);
}

// The K x 32 chunk of Y at column c0 into registers: thread t holds rows srow + kRowStep k,
// column scol (byte offset yo0 of row srow, column scol; rows kRowStep * ncol * 4 bytes apart).
// Loading the next chunk before working on the current one hides the memory latency.
__device__ inline void load_chunk(__amdgpu_buffer_rsrc_t rs, int yo0, int rstep, int c0, int K,
                                  int srow, float y[kStage]) {
#pragma unroll
  for (int k = 0; k < kStage; ++k)
    if (srow + kRowStep * k < K)
      y[k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
          rs, yo0, c0 * (int)sizeof(float) + k * rstep, 0));
}

__device__ inline void store_chunk(const float y[kStage], int K, int srow, int scol, float *T,
                                   int ts) {
#pragma unroll
  for (int k = 0; k < kStage; ++k)
    if (srow + kRowStep * k < K) T[(srow + kRowStep * k) * ts + scol] = y[k];
}

// The block's copy of its Gram matrix (K x K, row-major) in a.Gg.
__device__ inline const float *Ggb_all(const BigArgs &a, long long blk, int K) {
  return a.Gg + blk * (long long)K * K;
}

}  // namespace

// Two workgroups share a CU (four wavefronts per SIMD): the dynamic LDS is two K x KS arrays
// (80 800 bytes at K = 100) and the static part about 1 KB, within half of the 160 KB.
__global__ __launch_bounds__(kBT) __attribute__((amdgpu_waves_per_eu(4, 4)))
void k_big_block(BigArgs a) {
  extern __shared__ float lds[];
  const int K = a.K, KS = big_stride(K);
  // Each product result is held in registers until a barrier, so it may overwrite an operand.
  float *G = lds;       // Gram, A, the rotation generator and J, V^T V, U_R^T, a Y' chunk
  float *V = G + K * KS;  // Gram chunks, then the eigenbasis (column c = vector c), then M
  __shared__ float lam[112];
  __shared__ bool hot[112];
  __shared__ float red[kNW];
  __shared__ int wfail[kNW];
  if (a.sc->done) return;
  const int tid = threadIdx.x;
  const long long blk = blockIdx.x;
  const int p0 = (int)(blk / a.n2), q0 = (int)(blk - (long long)p0 * a.n2);
  const int ncol = a.ncol;
  float *Yb = a.Y + blk * (long long)K * ncol;
  const int CS = kChunk + 1;

  // ---- Gram over column chunks on v_mfma_f32_16x16x4_f32; Y' is written back. The K x K
  // Gram is cut into 16 x 16 tiles; the tiles on and above the diagonal are dealt round-robin
  // to the waves. In a 16x16x4 step, lane 16 g + i supplies row i, column g of the
  // A operand and row g, column i of the B operand, so with both taken from the staged chunk
  // (rows 16 I + i and 16 J + i, column 4 s + g) a tile accumulates Y'_I Y'_J^T.
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int i16 = lane & 15, g4 = lane >> 4;
  const int srow = tid >> 5, scol = tid & 31;  // chunk staging: rows srow + kRowStep k
  const __amdgpu_buffer_rsrc_t yrs = y_rsrc(Yb, K, ncol);
  const int yo0 = (srow * ncol + scol) * (int)sizeof(float);
  const int rstep = kRowStep * ncol * (int)sizeof(float);
  {
    const int nt = (K + 15) >> 4, ntiles = nt * (nt + 1) / 2;
    int tI[kGramTiles], tJ[kGramTiles];
#pragma unroll
    for (int m = 0; m < kGramTiles; ++m) {
      int rem = wave + kNW * m, I = 0;
      while (I < nt && rem >= nt - I) {
        rem -= nt - I;
        ++I;
      }
      tI[m] = I;
      tJ[m] = I + rem;  // valid only if wave + kNW m < ntiles
    }
    f4 gacc[kGramTiles];
#pragma unroll
    for (int m = 0; m < kGramTiles; ++m) gacc[m] = f4{0.f, 0.f, 0.f, 0.f};
    // staging: thread t moves rows t / 32 + kRowStep k, column t mod 32 of each chunk; the field
    // offset of each row's pixel is fixed for the block
    // (no gradient field: the blocks are clipped as they are)
    // (the field has fewer than 2^32 entries, checked at launch; rows past K read the first
    // pixel's, and their sums are neither staged nor stored)
    const bool hasg = a.gradf != nullptr;
    unsigned goff[kStage];
#pragma unroll
    for (int k = 0; k < kStage; ++k) {
      const int r = srow + kRowStep * k;
      const int ra = r / a.k2, rc = r - ra * a.k2;
      goff[k] = hasg && r < K
                    ? ((unsigned)wrapm(p0 + ra, a.n1) * a.n2 + wrapm(q0 + rc, a.n2)) * ncol + scol
                    : 0u;
    }
    // the loads of chunk c0 + 32 are issued before the products of chunk c0
    float yv[kStage], gv[kStage];
    load_chunk(yrs, yo0, rstep, 0, K, srow, yv);
#pragma unroll
    for (int k = 0; k < kStage; ++k) gv[k] = hasg ? a.gradf[goff[k]] : 0.f;
    for (int c0 = 0; c0 < ncol; c0 += kChunk) {
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kStage; ++k)
        if (srow + kRowStep * k < K) {
          const float y = yv[k] + a.gY * gv[k];
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(y), yrs, yo0,
                                                c0 * (int)sizeof(float) + k * rstep, 0);
          V[(srow + kRowStep * k) * kGS + scol] = y;
        }
      if (c0 + kChunk < ncol) {
        load_chunk(yrs, yo0, rstep, c0 + kChunk, K, srow, yv);
#pragma unroll
        for (int k = 0; k < kStage; ++k)
          gv[k] = hasg ? a.gradf[goff[k] + (unsigned)(c0 + kChunk)] : 0.f;
      }
      __syncthreads();
      // every tile slot of the wave runs (a slot past ntiles has rows past K, which read as
      // zero, and is not stored), so the chains of the slots interleave
#pragma unroll
      for (int st = 0; st < kChunk / 4; ++st)
#pragma unroll
        for (int m = 0; m < kGramTiles; ++m) {
          const int ra = 16 * tI[m] + i16, rb = 16 * tJ[m] + i16;
          const float av = V[min(ra, K - 1) * kGS + g4 + 4 * st];
          const float bv = V[min(rb, K - 1) * kGS + g4 + 4 * st];
          gacc[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(ra < K ? av : 0.f, rb < K ? bv : 0.f,
                                                         gacc[m], 0, 0, 0);
        }
    }
    // result layout: lane i + 16 g, register v holds tile entry (4 g + v, i); a copy of the
    // Gram goes to the block's slot of a.Gg (when given) for the re-derivation of A below
    float *Ggb = a.Gg ? a.Gg + blk * (long long)K * K : nullptr;
#pragma unroll
    for (int m = 0; m < kGramTiles; ++m) {
      if (wave + kNW * m < ntiles) {
        const int c = 16 * tJ[m] + i16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * tI[m] + 4 * g4 + v;
          if (r < K && c < K) {
            G[r * KS + c] = gacc[m][v];
            if (tI[m] != tJ[m]) G[c * KS + r] = gacc[m][v];
            if (Ggb) {
              Ggb[r * K + c] = gacc[m][v];
              if (tI[m] != tJ[m]) Ggb[c * K + r] = gacc[m][v];
            }
          }
        }
      }
    }
  }
  __syncthreads();
  // ---- finiteness and the Gershgorin bound: max_i sum_j |G_ij| <= 1 => nothing to clip
  {
    bool over = false, nonfin = false;
    for (int r = tid; r < K; r += kBT) {
      float s = 0.f;
      for (int c = 0; c < K; ++c) s += fabsf(G[r * KS + c]);
      over |= !(s <= 1.f);
      nonfin |= !isfinite(s);
    }
    const bool wo = __any(over), wn = __any(nonfin);
    if ((tid & 63) == 0) wfail[tid >> 6] = (wo ? 1 : 0) | (wn ? 2 : 0);
  }
  __syncthreads();
  int flag = 0;
#pragma unroll
  for (int w = 0; w < kNW; ++w) flag |= wfail[w];
  if (flag & 2) {
    if (tid == 0) atomicExch(&a.sc->nonfinite, 1);
    return;
  }
  if (flag == 0) return;  // Y' already stored; the basis is kept as it is

  // ---- basis: identity on the first use, else the stored one (orthonormal to rounding)
  float *Vg = a.V + blk * (long long)K * K;
  if (a.first) {
    int r = tid / K, c = tid - (tid / K) * K;
    const int dr = kBT / K, dc = kBT - (kBT / K) * K;
#pragma unroll 4
    for (int e = tid; e < K * K; e += kBT) {
      V[r * KS + c] = r == c ? 1.f : 0.f;
      r += dr;
      c += dc;
      if (c >= K) {
        c -= K;
        ++r;
      }
    }
  } else {
    copy_in(Vg, V, K, KS, tid);
  }
  __syncthreads();
  // ---- A = V^T (G V): H = G V over G, then A over H (exactly symmetric). G is symmetric, so
  // its operand is read as G^T (16 consecutive entries of a row per lane group). From the
  // identity basis A = G exactly, and the products are skipped.
  if (!a.first) {
    f4 hr[kMaxT];
    prod_rows<true>(G, KS, V, KS, K, wave, i16, g4, hr);
    __syncthreads();
    release_rows(K, wave, i16, g4, hr, [&](int r, int c, float x) { G[r * KS + c] = x; });
    __syncthreads();
    f4 hs[kSymHold];
    prod_sym<true>(V, KS, G, KS, K, wave, i16, g4, hs);
    __syncthreads();
    release_sym(K, wave, i16, g4, hs, [&](int r, int c, float x) { G[r * KS + c] = x; });
    __syncthreads();
  }

  // ---- parallel cyclic Jacobi
  const int m = (K + 1) & ~1;  // even; index K (if m > K) is a dummy whose rotation is identity
  const int H = m / 2;         // pairs per step
  // row / column passes: ceil(K / 64) waves per group of pairs, each wave covering a run of
  // cpw consecutive indices vi; ngV groups
  const int wpg = (K + 63) >> 6, ngV = kNW / wpg, cpw = (K + wpg - 1) / wpg;
  const int vkg = wave / wpg, vi = (wave - vkg * wpg) * cpw + lane, viK = vi * KS;
  const bool von = lane < cpw && vi < K;  // lanes 0 .. kBatch - 1 are always on (cpw > 16)
  // certificate (see the header): four threads per row; marks the rows that fail it (all rows
  // once `all_hot`) and returns whether any does, with the tolerance in `tol`. The diagonal
  // is copied to lam[] for the rotation generator of a simultaneous step.
  float tol = -1.f;
  auto certify = [&](bool all_hot) -> bool {
    // which diagonal entries exceed kNearOne, as two 64-bit masks every wave forms itself
    const float d0 = G[min(lane, K - 1) * (KS + 1)], d1 = G[min(lane + 64, K - 1) * (KS + 1)];
    const unsigned long long dm0 = __ballot(lane < K && d0 > kNearOne);
    const unsigned long long dm1 = __ballot(lane + 64 < K && d1 > kNearOne);
    const bool first = tol < 0.f;
    __syncthreads();  // the previous call's readers of wfail and red are done
    float sum = 0.f, mx = 0.f, fsq = 0.f, dr = 0.f;
    const int r = tid >> 2, part = tid & 3;
    if (tid < 4 * K) {  // four consecutive lanes per row, columns interleaved
      dr = G[r * KS + r];
      const bool rnear = dr > kNearOne;
#pragma unroll 5
      for (int c = part; c < K; c += 4) {
        const float g = G[r * KS + c];
        const float x = c == r ? 0.f : fabsf(g);
        fsq = fmaf(g, g, fsq);
        sum += x;
        const bool cnear = ((c < 64 ? dm0 >> c : dm1 >> (c - 64)) & 1ull) != 0;
        mx = fmaxf(mx, rnear || cnear ? x : 0.f);
      }
      sum += __shfl_xor(sum, 1);  // fixed order within the group of four
      sum += __shfl_xor(sum, 2);
      mx = fmaxf(mx, __shfl_xor(mx, 1));
      mx = fmaxf(mx, __shfl_xor(mx, 2));
    }
    if (first) {
      // ||A||_F on the first call; rotations and the re-derivation of A from an orthonormal
      // basis keep it (to rounding), so later calls reuse the tolerance
      for (int mm = 32; mm >= 1; mm >>= 1) fsq += __shfl_xor(fsq, mm);
      if (lane == 0) red[wave] = fsq;
      __syncthreads();
      float fs = 0.f;
#pragma unroll
      for (int w = 0; w < kNW; ++w) fs += red[w];  // fixed order
      tol = 1e-6f * sqrtf(fs);
    }
    bool fail = false;
    if (tid < 4 * K && part == 0) {
      fail = mx > tol || (dr <= kNearOne && dr + sum > 1.f);
      hot[r] = fail || all_hot;
      lam[r] = dr;
    }
    // one flag per wave (no atomics on a shared word)
    const bool wf = __any(fail);
    if (lane == 0) wfail[wave] = wf;
    __syncthreads();
    bool notyet = false;
#pragma unroll
    for (int w = 0; w < kNW; ++w) notyet |= wfail[w] != 0;
    return notyet;
  };

  // ---- simultaneous rotations on MFMA (warm-started iterations). With the previous basis
  // the off-diagonal entries of A are small, and one step with the angles of all pairs at
  // once removes them to second order: K_ij = tan(theta_ij) of the 2 x 2 rotation that zeroes
  // A_ij, for the pairs with a row that fails the certificate (K exactly skew), damped to
  // ||K||_F <= kSimCap; J = I + K + K^2 / 2; V <- V J, which drifts from orthonormal by K^4 / 4
  // per step (J^T J = I + K^4 / 4). After a step whose drift bound ||K^T K||_F^2 / 4 exceeds
  // kDriftTol V is re-orthonormalised by Newton-Schulz steps (each maps a drift e to 3 e^2 / 4);
  // after every step A is re-derived from the Gram copy, so the certificate is always judged on
  // V^T G V of an orthonormal V. The cyclic sweeps below finish whatever the certificate still
  // rejects.
  int ssteps = 0;
  bool certified = false;  // by the last certificate of the simultaneous steps
  // V orthonormal to rounding: as stored (or the identity), or re-orthonormalised after its
  // last change
  bool fresh = true;
  if (!a.first && a.Gg) {
    const float *Gb = Ggb_all(a, blk, K);
    for (; ssteps < kSimSteps; ++ssteps) {
      if (!certify(false)) {
        certified = true;
        break;
      }
      // the generator K (tangents) over A: entry (r, c) needs A_rc and the diagonal (copied by
      // the certificate), so each thread overwrites only what it read
      float kf2 = 0.f;
      {
        const unsigned long long hm0 = __ballot(lane < K && hot[min(lane, K - 1)]);
        const unsigned long long hm1 = __ballot(lane + 64 < K && hot[min(lane + 64, K - 1)]);
        // entry e = r K + c of this thread, stepped without divisions
        int r = tid / K, c = tid - (tid / K) * K;
        const int dr = kBT / K, dc = kBT - (kBT / K) * K;
#pragma unroll 4
        for (int e = tid; e < K * K; e += kBT) {
          float t = 0.f;
          const bool hr_ = ((r < 64 ? hm0 >> r : hm1 >> (r - 64)) & 1ull) != 0;
          const bool hc_ = ((c < 64 ? hm0 >> c : hm1 >> (c - 64)) & 1ull) != 0;
          if (r != c && (hr_ || hc_)) {
            // hardware square root and reciprocal: (c, r) gets exactly -t, so K stays skew
            const float arc = G[r * KS + c], den = lam[c] - lam[r];
            const float sg = (den > 0.f || (den == 0.f && r < c)) ? 1.f : -1.f;
            const float q = fabsf(den) + __builtin_sqrtf(fmaf(den, den, 4.f * arc * arc));
            t = q > 0.f ? (2.f * arc * sg) * __builtin_amdgcn_rcpf(q) : 0.f;
          }
          G[r * KS + c] = t;
          kf2 = fmaf(t, t, kf2);
          r += dr;
          c += dc;
          if (c >= K) {
            c -= K;
            ++r;
          }
        }
      }
      for (int mm = 32; mm >= 1; mm >>= 1) kf2 += __shfl_xor(kf2, mm);
      __syncthreads();  // red[] is free again (the certificate has read it)
      if ((tid & 63) == 0) red[tid >> 6] = kf2;
      __syncthreads();
      float ksum = 0.f;
#pragma unroll
      for (int w = 0; w < kNW; ++w) ksum += red[w];
      const float sc = ksum > kSimCap * kSimCap ? kSimCap * rsqrtf(ksum) : 1.f;
      f4 hr[kMaxT], hs[kSymHold];
      // J = I + sc K + (sc^2 / 2) K^2, with K^2 = -K^T K, over K; ||K^T K||_F^2 on the way
      prod_sym<true>(G, KS, G, KS, K, wave, i16, g4, hs);
      __syncthreads();  // every thread has read red[] (ksum) and K
      float kt2 = 0.f;
      release_sym(K, wave, i16, g4, hs, [&](int r, int c, float x) {
        G[r * KS + c] = (r == c ? 1.f : 0.f) + sc * G[r * KS + c] - 0.5f * sc * sc * x;
        kt2 = fmaf(x, x, kt2);
      });
      for (int mm = 32; mm >= 1; mm >>= 1) kt2 += __shfl_xor(kt2, mm);
      if (lane == 0) red[wave] = kt2;
      __syncthreads();
      float kts = 0.f;
#pragma unroll
      for (int w = 0; w < kNW; ++w) kts += red[w];  // fixed order
      // V J drifts from orthonormal by J^T J - I = (sc K)^4 / 4, whose norm is
      // sc^4 ||K^T K||_2^2 / 4 <= sc^4 ||K^T K||_F^2 / 4 (K is skew, so K^4 = (K^T K)^2)
      const float e0 = 0.25f * (sc * sc) * (sc * sc) * kts;
      prod_rows<false>(V, KS, G, KS, K, wave, i16, g4, hr);  // V J
      __syncthreads();
      release_rows(K, wave, i16, g4, hr, [&](int r, int c, float x) { V[r * KS + c] = x; });
      __syncthreads();
      fresh = false;
      if (e0 > kDriftTol) {
        // Newton-Schulz V <- V (3 I - V^T V) / 2 until the drift bound, mapped by e -> 3 e^2 / 4
        // per step, is below kDriftTol
        float drift = 0.75f * e0 * e0;
        int nns = 1;
        while (drift > kDriftTol && nns < 4) {
          drift = 0.75f * drift * drift;
          ++nns;
        }
        for (int ns = 0; ns < nns; ++ns) {
          prod_sym<true>(V, KS, V, KS, K, wave, i16, g4, hs);  // V^T V over J (no longer read)
          release_sym(K, wave, i16, g4, hs, [&](int r, int c, float x) { G[r * KS + c] = x; });
          __syncthreads();
          prod_rows<false>(V, KS, G, KS, K, wave, i16, g4, hr);
          __syncthreads();
          release_rows(K, wave, i16, g4, hr, [&](int r, int c, float x) {
            V[r * KS + c] = 1.5f * V[r * KS + c] - 0.5f * x;
          });
          __syncthreads();
        }
        fresh = true;
      }
      // A = V^T G V from the Gram copy: G back into LDS, H = G V over it (G symmetric, read as
      // G^T), then A over H
      {
        int r = tid / K, c = tid - (tid / K) * K;
        const int dr = kBT / K, dc = kBT - (kBT / K) * K;
        for (int e = tid; e < K * K; e += kBT) {
          G[r * KS + c] = Gb[e];
          r += dr;
          c += dc;
          if (c >= K) {
            c -= K;
            ++r;
          }
        }
      }
      __syncthreads();
      prod_rows<true>(G, KS, V, KS, K, wave, i16, g4, hr);
      __syncthreads();
      release_rows(K, wave, i16, g4, hr, [&](int r, int c, float x) { G[r * KS + c] = x; });
      __syncthreads();
      prod_sym<true>(V, KS, G, KS, K, wave, i16, g4, hs);
      __syncthreads();
      release_sym(K, wave, i16, g4, hs, [&](int r, int c, float x) { G[r * KS + c] = x; });
      __syncthreads();
      // A is exactly symmetric again (written from the upper tiles only)
    }
  }

  int sweeps = 0;
  for (; !certified && sweeps < a.max_sweeps; ++sweeps) {
    if (!certify(sweeps >= kRestricted)) break;
    fresh = false;
    const float skip = 0.1f * tol;
    for (int s = 0; s < m - 1; ++s) {
      // rotation angles; a pair rotates only if a row of it failed the certificate at the
      // start of the sweep (pairs of two certified rows need nothing) and its entry exceeds
      // the skip threshold. Every wave derives the step's rotations itself (lane k: pair k) and
      // permutes the active ones, in pair order, to lanes 0 .. na - 1, so no record passes
      // through LDS. The angles are read before the barrier, the updates come after it.
      int p = 0, q = 0;
      float c = 1.f, sv = 0.f;
      if (lane < H) {
        rr_pair(m, s, lane, p, q);
        const int qq = q < K ? q : p;
        const float apq = G[p * KS + qq], app = G[p * KS + p], aqq = G[qq * KS + qq];
        if (q < K && (hot[p] || hot[q]) && fabsf(apq) > skip) {
          // tan of the rotation angle, |t| <= 1 (hardware reciprocal and square roots: the
          // rotation stays orthogonal to about 1e-7 and the basis is re-orthonormalised)
          const float zeta = (aqq - app) * __builtin_amdgcn_rcpf(2.f * apq);
          const float az = fabsf(zeta);
          const float t =
              az > 1e15f
                  ? 0.5f * __builtin_amdgcn_rcpf(zeta)
                  : copysignf(__builtin_amdgcn_rcpf(az + __builtin_sqrtf(fmaf(zeta, zeta, 1.f))),
                              zeta);
          c = __builtin_amdgcn_rsqf(fmaf(t, t, 1.f));
          sv = t * c;
        }
      }
      const unsigned long long act = __ballot(sv != 0.f);
      const int na = __popcll(act);
      const int before = __popcll(act & ((1ull << lane) - 1ull));
      // a permutation of the 64 lanes: active pairs first, then the rest, each in lane order
      const int to = 4 * (sv != 0.f ? before : na + lane - before);
      const int pc = __builtin_amdgcn_ds_permute(to, __float_as_int(c));
      const int ps = __builtin_amdgcn_ds_permute(to, __float_as_int(sv));
      const int pp0 = __builtin_amdgcn_ds_permute(to, p);
      const int pq0 = __builtin_amdgcn_ds_permute(to, q);
      // this wave's items: active pairs vkg + u ngV (u < kBatch covers them all); lane u
      // fetches item u, and readlane broadcasts it below
      const int from = 4 * min(vkg + lane * ngV, 63);
      const float mc = __int_as_float(__builtin_amdgcn_ds_bpermute(from, pc));
      const float ms = __int_as_float(__builtin_amdgcn_ds_bpermute(from, ps));
      const int mp = __builtin_amdgcn_ds_bpermute(from, pp0);
      const int mq = __builtin_amdgcn_ds_bpermute(from, pq0);
      __syncthreads();
      // rows: A <- J^T A over the active pairs. Each wave serves one group of pairs (every
      // ngV-th active pair) and its lanes cover a run of columns; the rotation is wave-uniform
      // and held in scalar registers
      if (von && vkg < na) {
        float cu[kBatch], sn[kBatch], ap[kBatch], aq[kBatch];
        int pK[kBatch], qK[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
          cu[u] = lane_value(mc, u);
          sn[u] = lane_value(ms, u);
          pK[u] = __builtin_amdgcn_readlane(mp, u) * KS;
          qK[u] = __builtin_amdgcn_readlane(mq, u) * KS;
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u)
          if (vkg + u * ngV < na) {
            ap[u] = G[pK[u] + vi];
            aq[u] = G[qK[u] + vi];
          }
#pragma unroll
        for (int u = 0; u < kBatch; ++u)
          if (vkg + u * ngV < na) {
            G[pK[u] + vi] = cu[u] * ap[u] - sn[u] * aq[u];
            G[qK[u] + vi] = sn[u] * ap[u] + cu[u] * aq[u];
          }
      }
      __syncthreads();
      // columns: A <- A J, V <- V J, lanes over rows (row stride KS is odd, so they hit
      // distinct banks); the entry the rotation annihilates is set to 0
      if (von && vkg < na) {
        float cu[kBatch], sn[kBatch], ap[kBatch], aq[kBatch], vp[kBatch], vq[kBatch];
        int pp[kBatch], qq[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
          cu[u] = lane_value(mc, u);
          sn[u] = lane_value(ms, u);
          pp[u] = __builtin_amdgcn_readlane(mp, u);
          qq[u] = __builtin_amdgcn_readlane(mq, u);
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u)
          if (vkg + u * ngV < na) {
            ap[u] = G[viK + pp[u]];
            aq[u] = G[viK + qq[u]];
            vp[u] = V[viK + pp[u]];
            vq[u] = V[viK + qq[u]];
          }
#pragma unroll
        for (int u = 0; u < kBatch; ++u)
          if (vkg + u * ngV < na) {
            G[viK + pp[u]] = vi == qq[u] ? 0.f : cu[u] * ap[u] - sn[u] * aq[u];
            G[viK + qq[u]] = vi == pp[u] ? 0.f : sn[u] * ap[u] + cu[u] * aq[u];
            V[viK + pp[u]] = cu[u] * vp[u] - sn[u] * vq[u];
            V[viK + qq[u]] = sn[u] * vp[u] + cu[u] * vq[u];
          }
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    atomicMax(&a.sc->max_sweeps, sweeps);
    atomicAdd(&a.sc->step_sum, (unsigned long long)sweeps);  // sweeps per clipped block
    atomicAdd(&a.sc->step_blocks, 1ull);
    atomicAdd(&a.sc->sweep_sum, (unsigned long long)ssteps);  // simultaneous steps
    atomicAdd(&a.sc->sweep_waves, 1ull);
    if (sweeps == a.max_sweeps) atomicAdd(&a.sc->fallback_blocks, 1ull);  // not certified
  }
  __syncthreads();
  // ---- clip factors from the diagonal of the certified A = V^T G V: a row of A whose
  // diagonal exceeds 1 passed the off-diagonal test, so its diagonal is its eigenvalue to
  // second order in the residual; every other row has a Gershgorin bound <= 1 and no clip
  for (int i = tid; i < K; i += kBT) {
    const float d = G[i * KS + i];
    lam[i] = d > 1.f ? 1.f - 1.f / sqrtf(d) : 0.f;  // f_i of the clip
  }
  __syncthreads();
  // ---- Newton-Schulz: V^T V over A, V <- 1.5 V - 0.5 V (V^T V), unless V is orthonormal to
  // rounding already; V is stored for the next iteration unless it is the stored one
  if (!fresh) {
    f4 hr[kMaxT], hs[kSymHold];
    prod_sym<true>(V, KS, V, KS, K, wave, i16, g4, hs);
    release_sym(K, wave, i16, g4, hs, [&](int r, int c, float x) { G[r * KS + c] = x; });
    __syncthreads();
    prod_rows<false>(V, KS, G, KS, K, wave, i16, g4, hr);
    __syncthreads();
    release_rows(K, wave, i16, g4, hr, [&](int r, int c, float x) {
      V[r * KS + c] = 1.5f * V[r * KS + c] - 0.5f * x;
    });
    __syncthreads();
  }
  if (ssteps > 0 || sweeps > 0) {
    int r = tid / K, c = tid - (tid / K) * K;
    const int dr = kBT / K, dc = kBT - (kBT / K) * K;
#pragma unroll 4
    for (int e = tid; e < K * K; e += kBT) {
      Vg[e] = V[r * KS + c];
      r += dr;
      c += dc;
      if (c >= K) {
        c -= K;
        ++r;
      }
    }
  }
  // indices of the clipped directions, in order
  __shared__ int ridx[112];
  __shared__ int nr;
  if (tid == 0) {
    int n = 0;
    for (int i = 0; i < K; ++i)
      if (lam[i] > 0.f) ridx[n++] = i;
    nr = n;
  }
  __syncthreads();
  const int R = nr;
  const int nt = (K + 15) >> 4;
  // byte offset of this lane's first output (row 16 wave + 4 g4, column i16 of a chunk)
  const int co0 = ((16 * wave + 4 * g4) * ncol + i16) * (int)sizeof(float);
  // Y+ = Y' - acc for this wave's row tile of the chunk staged at stg (stride CS)
  auto store_out = [&](int c0, const float *stg, const f4 (&acc)[kChunk / 16]) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rr = 16 * wave + 4 * g4 + v;
      if (rr < K) {
#pragma unroll
        for (int J = 0; J < kChunk / 16; ++J) {
          const int cc = 16 * J + i16;
          __builtin_amdgcn_raw_buffer_store_b32(
              __float_as_uint(stg[rr * CS + cc] - acc[J][v]), yrs, co0,
              (c0 + v * ncol + 16 * J) * (int)sizeof(float), 0);
        }
      }
    }
  };
  if (R > 0 && R <= 32 && K * (KS - CS) >= 32 * CS) {
    // ---- Y+ = Y' - U^T (U Y') with U = diag(sqrt f) V_R^T (R x K, over the basis, which is
    // stored): per column chunk (staged in the first array) P = U Y' (R x 32, after the chunk)
    // by the waves of its 16 x 16 tiles, then each wave its row tile of Y' - U^T P
    {
      float ut[kUtRegs];
#pragma unroll
      for (int j = 0; j < kUtRegs; ++j) {
        const int e = tid + j * kBT;
        if (e < R * K) {
          const int n = e / K, r = e - (e / K) * K;
          const int i = ridx[n];
          ut[j] = V[r * KS + i] * sqrtf(lam[i]);
        }
      }
      __syncthreads();  // every read of the basis is done
#pragma unroll
      for (int j = 0; j < kUtRegs; ++j) {
        const int e = tid + j * kBT;
        if (e < R * K) {
          const int n = e / K, r = e - (e / K) * K;
          V[n * KS + r] = ut[j];
        }
      }
    }
    float *P = G + K * CS;
    const int nR = (R + 15) >> 4;
    float yv[kStage];
    load_chunk(yrs, yo0, rstep, 0, K, srow, yv);
    for (int c0 = 0; c0 < ncol; c0 += kChunk) {
      __syncthreads();  // U complete (first chunk); the previous chunk's products are done
      store_chunk(yv, K, srow, scol, G, CS);
      if (c0 + kChunk < ncol) load_chunk(yrs, yo0, rstep, c0 + kChunk, K, srow, yv);
      __syncthreads();
      if (wave < 2 * nR) {
        f4 acc[1];
        mfma_band<false, 1>(V, KS, G, CS, K, R, kChunk, wave >> 1, wave & 1, i16, g4, acc);
#pragma unroll
        for (int v = 0; v < 4; ++v)
          P[(16 * (wave >> 1) + 4 * g4 + v) * CS + 16 * (wave & 1) + i16] = acc[0][v];
      }
      __syncthreads();
      if (wave < nt) {
        f4 acc[kChunk / 16];
        mfma_band<true, kChunk / 16>(V, KS, P, CS, R, K, kChunk, wave, 0, i16, g4, acc);
        store_out(c0, G, acc);
      }
    }
  } else if (R > 0) {
    // ---- Y+ = Y' - M Y' with M = V_R diag(f) V_R^T (K x K, symmetric), formed once per
    // block: the clipped directions scaled by sqrt(f) are gathered as the rows of U (over
    // V^T V, R x K), so M = U^T U (over the basis, which is stored); then every column chunk of
    // Y' is staged over U and each wave updates its row tile of the chunk (M read as its own
    // transpose)
    for (int e = tid; e < R * K; e += kBT) {
      const int n = e / K, r = e - (e / K) * K;
      const int i = ridx[n];
      G[n * KS + r] = V[r * KS + i] * sqrtf(lam[i]);
    }
    __syncthreads();
    {
      f4 hs[kSymHold];
      prod_sym<true>(G, KS, G, KS, K, wave, i16, g4, hs, R);
      __syncthreads();
      release_sym(K, wave, i16, g4, hs, [&](int r, int c, float x) { V[r * KS + c] = x; });
    }
    // the loads of chunk c0 + 32 (a column range this pass has not written) are issued before
    // the products of chunk c0
    float yv[kStage];
    load_chunk(yrs, yo0, rstep, 0, K, srow, yv);
    for (int c0 = 0; c0 < ncol; c0 += kChunk) {
      __syncthreads();  // M is complete (first chunk); the previous chunk's products are done
      store_chunk(yv, K, srow, scol, G, CS);
      if (c0 + kChunk < ncol) load_chunk(yrs, yo0, rstep, c0 + kChunk, K, srow, yv);
      __syncthreads();
      if (wave < nt) {
        f4 acc[kChunk / 16];
        mfma_band<true, kChunk / 16>(V, KS, G, CS, K, K, kChunk, wave, 0, i16, g4, acc);
        store_out(c0, G, acc);
      }
    }
  }
}

// Z[pix][col] = sum over the K windows containing pix of their row for pix (fixed order).
__global__ __launch_bounds__(kNT) void k_big_overlap(BigArgs a, float *Z) {
  if (a.sc->done) return;
  const int K = a.K, ncol = a.ncol;
  const long long total = (long long)a.n1 * a.n2 * ncol;
  for (long long idx = (long long)blockIdx.x * kNT + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * kNT) {
    const long long pix = idx / ncol;
    const int col = (int)(idx - pix * ncol);
    const int i = (int)(pix / a.n2), j = (int)(pix - (long long)i * a.n2);
    float s = 0.f;
    for (int ra = 0; ra < a.k1; ++ra) {
      const long long rowb = (long long)wrapm(i - ra, a.n1) * a.n2;
      const float *Yr = a.Y + (long long)(ra * a.k2) * ncol + col;
      // five windows' loads in flight, summed in the same order as one at a time
      int rc = 0;
      for (; rc + 5 <= a.k2; rc += 5) {
        float x[5];
#pragma unroll
        for (int u = 0; u < 5; ++u) {
          const long long blk = rowb + wrapm(j - rc - u, a.n2);
          x[u] = Yr[(blk * K + rc + u) * ncol];
        }
#pragma unroll
        for (int u = 0; u < 5; ++u) s += x[u];
      }
      for (; rc < a.k2; ++rc) {
        const long long blk = rowb + wrapm(j - rc, a.n2);
        s += Yr[(blk * K + rc) * ncol];
      }
    }
    Z[idx] = s;
  }
}

__global__ __launch_bounds__(kNT) void k_big_identity(float *V, long long nblk, int K) {
  const long long total = nblk * K * K;
  for (long long e = (long long)blockIdx.x * kNT + threadIdx.x; e < total;
       e += (long long)gridDim.x * kNT) {
    const int rc = (int)(e % ((long long)K * K));
    V[e] = (rc / K == rc % K) ? 1.f : 0.f;
  }
}

// Blocks in the paper's column order (column 2b + comp of a row: band b of the D_v (comp 0)
// or D_h (comp 1) part) <-> the block layout [block][K][ncol] with column comp * Bp + b; the
// columns b >= n3 of each part are zero.
__global__ __launch_bounds__(kNT) void k_big_pack(const float *src, float *Y, long long nblk, int K,
                                                  int n3, int Bp) {
  const int ncol = 2 * Bp;
  const long long total = nblk * K * ncol;
  for (long long e = (long long)blockIdx.x * kNT + threadIdx.x; e < total;
       e += (long long)gridDim.x * kNT) {
    const long long r = e / ncol;  // block * K + row
    const int c = (int)(e - r * ncol);
    const int comp = c >= Bp ? 1 : 0, b = c - comp * Bp;
    Y[e] = b < n3 ? src[r * 2 * n3 + 2 * b + comp] : 0.f;
  }
}

__global__ __launch_bounds__(kNT) void k_big_unpack(const float *Y, float *dst, long long nblk,
                                                    int K, int n3, int Bp) {
  const long long total = nblk * K * 2 * n3;
  for (long long e = (long long)blockIdx.x * kNT + threadIdx.x; e < total;
       e += (long long)gridDim.x * kNT) {
    const long long r = e / (2 * n3);
    const int cs = (int)(e - r * 2 * n3);
    dst[e] = Y[r * 2 * Bp + (cs & 1) * Bp + (cs >> 1)];
  }
}

size_t big_lds_bytes(int K) { return (size_t)(2 * K * big_stride(K)) * sizeof(float); }

hipError_t launch_big_block(const BigArgs &a, hipStream_t st) {
  // the dynamic-LDS limit, raised once per device (a bit per device id)
  static std::atomic<unsigned long long> done{0};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const unsigned long long bit = dev < 64 ? 1ull << dev : 0ull;
  if (!bit || !(done.load(std::memory_order_acquire) & bit)) {
    e = hipFuncSetAttribute((const void *)k_big_block, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)kLdsLimit);
    if (e != hipSuccess) return e;
    if (bit) done.fetch_or(bit, std::memory_order_release);
  }
  hipLaunchKernelGGL(k_big_block, dim3((unsigned)a.nblk), dim3(kBT), big_lds_bytes(a.K), st, a);
  return hipGetLastError();
}

hipError_t launch_big_overlap(const BigArgs &a, float *Z, hipStream_t st) {
  long long g = ((long long)a.n1 * a.n2 * a.ncol + kNT * 4 - 1) / (kNT * 4);
  if (g > 65535) g = 65535;
  hipLaunchKernelGGL(k_big_overlap, dim3((unsigned)g), dim3(kNT), 0, st, a, Z);
  return hipGetLastError();
}

hipError_t launch_big_pack(const float *src, float *Y, long long nblk, int K, int n3, int Bp,
                          hipStream_t st) {
  long long g = (nblk * K * 2 * Bp + kNT * 4 - 1) / (kNT * 4);
  if (g > 65535) g = 65535;
  hipLaunchKernelGGL(k_big_pack, dim3((unsigned)g), dim3(kNT), 0, st, src, Y, nblk, K, n3, Bp);
  return hipGetLastError();
}

hipError_t launch_big_unpack(const float *Y, float *dst, long long nblk, int K, int n3, int Bp,
                            hipStream_t st) {
  long long g = (nblk * K * 2 * n3 + kNT * 4 - 1) / (kNT * 4);
  if (g > 65535) g = 65535;
  hipLaunchKernelGGL(k_big_unpack, dim3((unsigned)g), dim3(kNT), 0, st, Y, dst, nblk, K, n3, Bp);
  return hipGetLastError();
}

hipError_t launch_big_identity(float *V, long long nblk, int K, hipStream_t st) {
  long long g = (nblk * K * K + kNT * 4 - 1) / (kNT * 4);
  if (g > 65535) g = 65535;
  hipLaunchKernelGGL(k_big_identity, dim3((unsigned)g), dim3(kNT), 0, st, V, nblk, K);
  return hipGetLastError();
}

}  // namespace s3ttv
