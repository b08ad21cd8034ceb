// Internal declarations shared by the gfx950 kernels and the C-ABI driver.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace s3ttv {

// Regularisers on the P-PDS skeleton (values of s3ttv_params.regularizer): the S3TTV term of
// Prob. (18), or the terms of the compared P-PDS-applicable methods in its place.
constexpr int kRegS3TTV = 0, kRegSTV = 1, kRegSSTV = 2, kRegHSSTV = 3, kRegSSST = 4;
// Regularisers whose dual is a field clipped entrywise (no block pass).
__host__ __device__ inline bool l1_reg(int reg) { return reg == kRegSSTV || reg == kRegHSSTV; }
// Components of the block columns per band: 3 for SSST (D_v u, D_h u, D_s u), else 2.
__host__ __device__ inline int block_comps(int reg) { return reg == kRegSSST ? 3 : 2; }

// Overlap-add partials (P_l^T of step 2) are accumulated in 32-bit fixed point with this
// scale: every entry of Y+_l lies in [-1, 1] (its spectral norm is at most 1), so a pixel's
// sum over at most 16 windows stays below 2^30. Integer addition is associative, so the
// accumulation order (and thus the run) does not change the result.
constexpr float kZScale = 67108864.f;        // 2^26
constexpr float kZInv = 1.f / 67108864.f;
constexpr float kZMax = 16.f;                // larger magnitudes (or NaN) are flagged

// Fixed-point value of y; sets bad if |y| > kZMax or y is not a number.
__device__ inline int to_fixed(float y, bool &bad) {
  bad |= !(fabsf(y) <= kZMax);
  return __float2int_rn(fminf(fmaxf(y, -kZMax), kZMax) * kZScale);
}
// Same for a value already known to be finite and within [-kZMax, kZMax].
__device__ inline int to_fixed_bounded(float y) { return __float2int_rn(y * kZScale); }

// Workgroups are dispatched to the 8 XCDs (each with its own L2) round-robin. Remapping
// workgroup b to logical index (b % 8) * (G / 8) + b / 8 gives each XCD a contiguous eighth of
// the work, so stencil neighbours are found in the same L2. Identity when G % 8 != 0.
constexpr int kXcds = 8;
__device__ inline int xcd_block(int b, int G) {
  return (G % kXcds) ? b : (b % kXcds) * (G / kXcds) + b / kXcds;
}

// Number of float32 columns per block tile handled by one 16x16 MFMA step group.
constexpr int kTile = 16;
// Rows of the padded block (K <= 16 rows of the structure tensor, zero padded).
constexpr int kRows = 16;
// Blocks of more rows (16 < K <= kBigMax) take the one-workgroup-per-block path.
constexpr int kBigMax = 100;

// l1-ball threshold selection: radix selection on the IEEE bits of |x| in three levels
// (bits 30..20, 19..9, 8..0). All values in one level-1 bin share an exponent, so per-bin
// sums of the 24-bit significands are exact in 64-bit integers.
constexpr int kL1Bins1 = 2048, kL1Shift1 = 20;
constexpr int kL1Bins2 = 2048, kL1Shift2 = 9;
constexpr int kL1Bins3 = 512, kL1Shift3 = 0;
constexpr int kL1MaxBins = 2048;
// Dynamic LDS a block kernel may use (of the 160 KB per CU).
constexpr size_t kLdsLimit = 152 * 1024;
// Level 2 is histogrammed per workgroup over at most this many elements per ball, so the
// packed LDS bins (count << 40 | significand sum) cannot overflow.
constexpr int kL1PartElems = 32768;

// Device-resident scalars of one solve.
struct DevScalars {
  double kappa;          // y3 = kappa * w, kappa in [0, 1)
  double tau[2];         // soft thresholds of the s (0) and t (1) l1 balls
  double S_above[2];     // l1 selection carry: sum of |x| above the current bin
  unsigned long long C_above[2];  // ... and their count
  uint32_t prefix[2];    // selected bit prefix so far
  int32_t active[2];     // 1 if the l1 projection is not the identity
  int32_t done;          // stop: the rule fired, max_iter was reached or a value was not finite
  int32_t iters;         // completed iterations
  int32_t converged;     // the stop rule fired
  int32_t max_iter;      // iteration budget (the finalize kernel sets done when it is used up)
  double rel_change;     // of the last completed iteration
  double unorm2;         // ||u^(k-1)||^2 of the last iteration
  int32_t nonfinite;     // a NaN/Inf was seen
  int32_t max_sweeps;    // largest Jacobi sweep count seen
  double wnorm2;         // ||w||^2 of the last dual step
  double rel_tol;
  unsigned long long sweep_sum;   // Jacobi sweeps summed over wavefronts
  unsigned long long sweep_waves; // wavefronts counted in sweep_sum
  unsigned long long step_sum;    // MFMA rotation steps summed over blocks (warm iterations)
  unsigned long long step_blocks; // blocks counted in step_sum
  unsigned long long fallback_blocks;  // warm-iteration blocks handed to the per-lane Jacobi
  int32_t max_steps;              // largest rotation step count of one block
  int32_t zslot_overflow;         // some pixel has more than 4 overlap-add partial slots
  // Signature of the iterate the workspace holds (a solve may be continued from it):
  // sig[0] = kStateMagic once a single solve has initialised its state, then the shape
  // (n1, n2, n3, k1, k2), the regulariser and the anchor tile (TA * 256 + TB).
  int32_t sig[8];
};

constexpr int32_t kStateMagic = 0x53335456;
struct StateSig {
  int32_t v[8];
};

// l1 histograms: per ball, per level: counts (u32) and significand sums (u64).
struct L1Hist {
  uint32_t cnt[2][3][kL1MaxBins];
  unsigned long long sig[2][3][kL1MaxBins];
};

struct Plan {
  int n1, n2, n3, k1, k2, K;
  int Bp;        // bands padded to a multiple of 16 (of 32 for three components)
  int ncol;      // comps * Bp columns per block (comp-major: c = comp*Bp + band)
  int ntile;     // ncol / 16
  long long N;   // n1*n2*n3
  long long P;   // n1*n2 pixels (= L blocks)
  // apply tiling (anchors per workgroup tile) and overlap-add partial geometry
  int TA, TB, ntA, ntB, extA, extB, apply_waves;
  size_t apply_lds;
  // step sizes and box (float for the vector arithmetic), radii (double)
  float g_u, g_s, g_t, g_Y, g_y2, g_y3, mu_min, mu_max;
  // regulariser (kReg*), HSSTV weight and the step of its second dual field
  int reg;
  float omega, g_Z2;
  double eps, alpha, beta;
  // grids of the reduction kernels
  int red_blocks;
  // workspace carve
  float *u[2], *s, *t[2], *y2, *w, *xs, *xt, *gradf, *Y, *G, *W, *V, *Z;
  int *zpart;          // overlap-add partials per anchor tile, fixed point (kZScale)
  int *zslot;          // per pixel: the (up to 4) partial slots holding its overlap-add terms;
                       // absent ones name the extra all-zero slot at the end of zpart
  bool zfold;          // the primal step sums the partials itself (no separate zsum pass)
  bool big;            // K > kRows: one workgroup per block, overlap-add by gather
  long long zslots_n;  // overlap-add partial slots carved (tiles x extent + the zero slot)
  int *eflag;          // per block: rotation steps | 256 if the per-lane Jacobi must finish it
  int *estat;          // per k_eig workgroup (64 blocks): step sum, max steps, fallbacks, blocks
  unsigned long long *l1part;  // level-2 l1 partial histograms: 2 x l1_part_blocks(N) x 2048
  double *red_primal;  // red_blocks * 4
  double *red_dual;    // red_blocks
  DevScalars *sc;
  L1Hist *hist;
  size_t bytes;
};

// ---------------------------------------------------------------- launchers (return hipError_t)

// Vector / stencil kernels.
hipError_t launch_fill(float *p, long long n, float val, hipStream_t st);
hipError_t launch_identity16(float *V, long long nblk, hipStream_t st);
// Deterministic pseudo-random fill in [-scale, scale) (synthetic data for tile tuning).
hipError_t launch_fill_hash(float *p, long long n, float scale, uint32_t seed, hipStream_t st);
hipError_t launch_copy(float *dst, const float *src, long long n, hipStream_t st);
hipError_t launch_init_scalars(const Plan &pl, double rel_tol, int max_iter, hipStream_t st);
// Records the state signature (after the state has been initialised).
hipError_t launch_mark_state(const Plan &pl, const StateSig &sig, hipStream_t st);
// Continues from the iterate held in the workspace: clears the stop flags and the eigen-solve
// statistics, sets the stop tolerance and a budget of `budget` more iterations.
hipError_t launch_resume_scalars(const Plan &pl, double rel_tol, int budget, hipStream_t st);
hipError_t launch_zero_bytes(void *p, size_t bytes, hipStream_t st);
hipError_t launch_check_finite(const float *x, long long n, DevScalars *sc, hipStream_t st);
// Primal step (Alg. 1 steps 2-4) from (u_cur, s, t_cur, y2, w, Z) into (u_new, xs, xt),
// plus the level-1 l1 histograms and the stop-rule partial sums.
hipError_t launch_primal(const Plan &pl, const float *u_cur, float *u_new, const float *t_cur,
                         hipStream_t st);
// gradient field of u' = ca*a + cb*b into pl.gradf (or gout with the given column stride)
hipError_t launch_grad(const Plan &pl, const float *a, const float *b, float ca, float cb,
                       float *gout, hipStream_t st);
hipError_t launch_zsum(const Plan &pl, hipStream_t st);
// Per-pixel slot table for the primal step's own overlap-add sum; flags pixels with more
// than 4 slots in DevScalars::zslot_overflow.
hipError_t launch_zslots(const Plan &pl, hipStream_t st);
bool zslots_fit(const Plan &pl);
hipError_t launch_dual(const Plan &pl, const float *u_cur, const float *u_new, const float *t_cur,
                       float *t_new, const float *v, hipStream_t st);
// launch_dual and the gradient field of u' = 2 u_new - u_cur (into pl.gradf) in one sweep.
hipError_t launch_dual_grad(const Plan &pl, const float *u_cur, const float *u_new,
                            const float *t_cur, float *t_new, const float *v, hipStream_t st);
// eig_stats: also fold this iteration's eigen-solve statistics (written by k_eig) in.
hipError_t launch_finalize(const Plan &pl, bool eig_stats, hipStream_t st);

// l1 threshold selection for the two balls (ball count 1 or 2): level = 1, 2, 3.
hipError_t launch_l1_hist(const float *x0, const float *x1, long long n, int nballs, int level,
                          L1Hist *hist, DevScalars *sc, hipStream_t st);
hipError_t launch_l1_select(int nballs, int level, double r0, double r1, L1Hist *hist,
                            DevScalars *sc, hipStream_t st);
// Level 2 in two passes: per-workgroup partial histograms (l1_part_blocks(n) per ball, 2048
// u64 each), then their per-bin sum into hist level 2.
int l1_part_blocks(long long n);
hipError_t launch_l1_hist_part(const float *x0, const float *x1, long long n, int nballs,
                               unsigned long long *part, DevScalars *sc, hipStream_t st);
hipError_t launch_l1_part_reduce(int nballs, long long n, const unsigned long long *part,
                                 L1Hist *hist, DevScalars *sc, hipStream_t st);
hipError_t launch_l1_apply(const float *x, float *out, long long n, int ball, DevScalars *sc,
                           hipStream_t st);

// Blocks of more than 16 rows (Alg. 1 steps 9-10 and the overlap-add).
struct BigArgs {
  int n1, n2, k1, k2, K, ncol;
  long long nblk;
  const float *gradf;
  float gY;
  float *Y;   // [block][K][ncol]
  float *V;   // [block][K][K] eigenbasis, kept across iterations
  float *Gg;  // [block][K][K] copy of each block's Gram matrix (nullable: no simultaneous
              // rotation steps before the cyclic sweeps)
  int first;  // V is still the identity
  int max_sweeps;
  DevScalars *sc;
};
hipError_t launch_big_block(const BigArgs &a, hipStream_t st);
hipError_t launch_big_overlap(const BigArgs &a, float *Z, hipStream_t st);
hipError_t launch_big_identity(float *V, long long nblk, int K, hipStream_t st);
// Blocks in the paper's column order (L x K x 2 n3) <-> the block layout [L][K][2 Bp].
hipError_t launch_big_pack(const float *src, float *Y, long long nblk, int K, int n3, int Bp,
                          hipStream_t st);
hipError_t launch_big_unpack(const float *Y, float *dst, long long nblk, int K, int n3, int Bp,
                            hipStream_t st);
size_t big_lds_bytes(int K);

// Block kernels (Alg. 1 steps 9-10).
struct BlockArgs {
  int n1, n2, k1, k2, K, ncol, ntile;
  long long nblk;          // number of blocks (anchors)
  const float *gradf;      // [pixel][ncol] or nullptr (T = 0)
  float gY;
  float *Y;                // apply layout, nblk * 16 * ncol floats
  float *G, *W;            // nblk * 256 floats each
  float *V;                // nblk * 256: eigenvectors of the previous step (warm start) or null
  // Eigen mode. eflag == nullptr: k_gram writes the (rotated) Gram matrix and k_eig solves
  // every block. eflag != nullptr (requires V): k_gram diagonalises each block itself on MFMA
  // starting from V, writes W and V, and flags the blocks it cannot certify; k_eig solves
  // only the flagged ones.
  int *eflag;
  int *estat;              // with eflag: per-workgroup eigen statistics written by k_eig
  int eig_steps;           // with eflag: MFMA rotation steps per block before the fallback
  int gram_prec;           // fused pass: Gram inputs FP32 (0), BF16 (1) or FP16 (2)
  // apply tiling / overlap-add (zpart == nullptr: no overlap-add)
  int TA, TB, ntA, ntB, extA, extB, waves;
  size_t lds;
  int *zpart;              // fixed point (kZScale)
  DevScalars *sc;          // done flag and sweep statistics (nullable)
};
hipError_t launch_gram(const BlockArgs &a, hipStream_t st);
hipError_t launch_eig(const BlockArgs &a, hipStream_t st);
hipError_t launch_apply(const BlockArgs &a, hipStream_t st);
// Warm iterations in one pass over Y (Gram, MFMA eigen-solve, clip, overlap-add), followed by
// launch_eig and launch_fixup for the blocks it could not certify. Requires fused_supported.
bool fused_supported(const BlockArgs &a);
// Sets the dynamic-LDS limit of the block kernels (once per process; call before launching).
hipError_t configure_block_kernels();
size_t fused_lds_bytes(const BlockArgs &a);
hipError_t launch_block_fused(const BlockArgs &a, hipStream_t st);
hipError_t launch_fixup(const BlockArgs &a, hipStream_t st);

// Layout converters for the operator entry points.
// rows x ncols_src row-major blocks <-> apply layout with ncol padded columns. For the
// structure-tensor layout (paper column order 2b+comp) set paper_cols = 1 with n3 bands.
hipError_t launch_pack_blocks(const float *src, float *Y, long long nblk, int K, int ncols_src,
                              int ncol, int paper_cols, int n3, int Bp, hipStream_t st);
hipError_t launch_unpack_blocks(const float *Y, float *dst, long long nblk, int K,
                                int ncols_src, int ncol, int paper_cols, int n3, int Bp,
                                hipStream_t st);
// [pixel][ncol] field <-> two ABI cubes.
hipError_t launch_field_to_cubes(const float *f, float *c0, float *c1, long long P, int n3,
                                 int Bp, hipStream_t st);
hipError_t launch_cubes_to_field(const float *c0, const float *c1, float *f, long long P, int n3,
                                 int Bp, hipStream_t st);
// Plain adjoint D_s^T(D_v^T zv + D_h^T zh) from a [pixel][ncol] field.
hipError_t launch_grad_adj(const Plan &pl, const float *Z, float *w, hipStream_t st);
// Residual diagnostics of the result (host reads): ||s||_1, ||t||_1, ||u+s+t-v||, ||D_v t||.
hipError_t launch_diagnostics(const Plan &pl, const float *u, const float *s, const float *t,
                              const float *v, double *out4, hipStream_t st);

}  // namespace s3ttv
