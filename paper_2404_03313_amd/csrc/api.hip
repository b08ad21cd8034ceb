// C-ABI driver of the gfx950 S3TTV solver (Alg. 1 of arXiv 2404.03313).
//
// Validates arguments, carves the caller's workspace, and enqueues the per-iteration
// kernel chain:
//   primal (steps 2-4, level-1 l1 histograms) -> l1 select / level-2 partial histograms /
//   reduce / select / level-3 histogram / select (tau_s, tau_t) -> dual steps (3-7
//   thresholds, 12, 13) with the gradient field D_v D_s u', D_h D_s u' -> block pass (steps
//   9-10 + overlap-add: fused Gram / MFMA eigen-solve / clip from the second iteration on,
//   else gram -> eig -> apply) -> zsum (P^T for the next step 2) -> finalize (y3 projection
//   scalar of step 14, stop rule).
// The only device->host traffic inside the loop is a 4-byte stop flag every check_every
// iterations when rel_tol > 0.
#include <math.h>
#include <string.h>

#include <map>
#include <mutex>
#include <vector>

#include "../../include/s3ttv.h"
#include "s3ttv_internal.h"

using namespace s3ttv;

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kMaxLds = kLdsLimit;
constexpr int kDefaultEigSteps = 24;
// Jacobi sweeps at most per block on the K > 16 path (from the identity about 8 suffice for
// K = 100; warm started fewer).
constexpr int kBigMaxSweeps = 30;
// Iterations per captured graph of the batched solve (even: the u / t buffer parity of the
// captured launches then holds for every replay).
constexpr int kBatchSpan = 16;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Carver {
  char *base;
  size_t off = 0;
  bool dry;
  template <typename T>
  T *take(size_t count) {
    off = align_up(off);
    T *p = dry ? nullptr : reinterpret_cast<T *>(base + off);
    off += count * sizeof(T);
    return p;
  }
};

bool valid_shape(const s3ttv_shape *sh) {
  if (!sh) return false;
  if (sh->n1 < 2 || sh->n2 < 2 || sh->n3 < 2) return false;
  if (sh->k1 < 1 || sh->k2 < 1 || sh->k1 > sh->n1 || sh->k2 > sh->n2) return false;
  return true;
}

// Bands padded to whole column tiles: 16 per component, and for three components a multiple
// of 32, so that every block has an even number of 16-column tiles (pairs of tiles per LDS
// round trip in the fused pass) and a multiple of 32 columns (the large-block chunks).
int padded_bands(int n3, int reg) {
  const int q = block_comps(reg) == 3 ? 32 : 16;
  return (n3 + q - 1) / q * q;
}

int32_t supported_shape(const s3ttv_shape *sh, int reg) {
  if (sh->k1 * sh->k2 > kBigMax) return S3TTV_EUNSUPPORTED;
  const long long N = (long long)sh->n1 * sh->n2 * sh->n3;
  if (N >= (1ll << 31)) return S3TTV_EUNSUPPORTED;
  if (sh->k1 * sh->k2 <= kRows) {
    // the smallest anchor tile (1 x 1) must hold its overlap-add accumulators in LDS:
    // k1 k2 pixels of comps * Bp + 16 floats (N3 up to 1200 for 4 x 4 blocks of S3TTV)
    const size_t ncol = (size_t)block_comps(reg) * padded_bands(sh->n3, reg);
    if ((size_t)sh->k1 * sh->k2 * (ncol + 16) * sizeof(float) > kMaxLds)
      return S3TTV_EUNSUPPORTED;
  } else {
    // the large-block kernel addresses the gradient field by 32-bit entry offsets
    const long long ncol = (long long)block_comps(reg) * padded_bands(sh->n3, reg);
    if ((long long)sh->n1 * sh->n2 * ncol >= (1ll << 32)) return S3TTV_EUNSUPPORTED;
  }
  return S3TTV_OK;
}

// Regulariser of a call's parameters (null parameters: S3TTV).
int reg_of(const s3ttv_params *pr) { return pr ? pr->regularizer : S3TTV_REG_S3TTV; }

// Anchor-tile candidates (largest first). The arithmetic of a solve does not depend on the
// tile (the overlap-add is exact fixed point), only its speed does.
const int kTileCand[][2] = {{8, 8}, {8, 4}, {4, 8}, {4, 4}, {4, 2}, {2, 4}, {2, 2}, {2, 1}, {1, 1}};

size_t apply_lds_bytes(const Plan &pl, int TA, int TB) {
  return (size_t)(TA + pl.k1 - 1) * (TB + pl.k2 - 1) * (pl.ncol + 16) * sizeof(float);
}

// Anchor tile: the forced one (clipped to the image) or the largest candidate whose
// overlap-add accumulators fit LDS.
void choose_tiles(Plan &pl, int forceTA, int forceTB) {
  if (forceTA > 0 && forceTB > 0) {
    pl.TA = forceTA < pl.n1 ? forceTA : pl.n1;
    pl.TB = forceTB < pl.n2 ? forceTB : pl.n2;
    pl.apply_lds = apply_lds_bytes(pl, pl.TA, pl.TB);
  } else {
    for (auto &c : kTileCand) {
      const int TA = c[0] < pl.n1 ? c[0] : pl.n1, TB = c[1] < pl.n2 ? c[1] : pl.n2;
      pl.TA = TA;
      pl.TB = TB;
      pl.apply_lds = apply_lds_bytes(pl, TA, TB);
      if (pl.apply_lds <= kMaxLds) break;
    }
  }
  pl.extA = pl.TA + pl.k1 - 1;
  pl.extB = pl.TB + pl.k2 - 1;
  pl.ntA = (pl.n1 + pl.TA - 1) / pl.TA;
  pl.ntB = (pl.n2 + pl.TB - 1) / pl.TB;
  pl.apply_waves = pl.ntile < 16 ? pl.ntile : 16;
}

// Geometry + carve. base == nullptr -> size only. forceTA/TB > 0 fix the anchor tile.
void make_plan(Plan &pl, const s3ttv_shape *sh, char *base, int reg, int forceTA = 0,
               int forceTB = 0) {
  memset(&pl, 0, sizeof(pl));
  pl.n1 = sh->n1;
  pl.n2 = sh->n2;
  pl.n3 = sh->n3;
  pl.k1 = sh->k1;
  pl.k2 = sh->k2;
  pl.K = sh->k1 * sh->k2;
  pl.reg = reg;
  pl.Bp = padded_bands(sh->n3, reg);
  pl.ncol = block_comps(reg) * pl.Bp;
  pl.ntile = pl.ncol / 16;
  pl.P = (long long)sh->n1 * sh->n2;
  pl.N = pl.P * sh->n3;
  pl.big = pl.K > kRows;
  if (pl.big) {
    // no anchor tiles: one workgroup per block, the overlap-add is a gather
    pl.TA = pl.TB = 1;
    pl.extA = pl.k1;
    pl.extB = pl.k2;
    pl.ntA = pl.n1;
    pl.ntB = pl.n2;
    pl.apply_waves = 1;
    pl.zslots_n = 1;
  } else {
    choose_tiles(pl, forceTA, forceTB);
    pl.zslots_n = (long long)pl.ntA * pl.ntB * pl.extA * pl.extB + 1;
  }
  long long rb = (pl.N + 8191) / 8192;
  pl.red_blocks = (int)(rb < 1 ? 1 : (rb > 65535 ? 65535 : rb));
  Carver cv{base, 0, base == nullptr};
  const size_t N = (size_t)pl.N;
  pl.u[0] = cv.take<float>(N);
  pl.u[1] = cv.take<float>(N);
  pl.s = cv.take<float>(N);
  pl.t[0] = cv.take<float>(N);
  pl.t[1] = cv.take<float>(N);
  pl.y2 = cv.take<float>(N);
  pl.w = cv.take<float>(N);
  pl.xs = cv.take<float>(N);
  pl.xt = cv.take<float>(N);
  pl.gradf = cv.take<float>((size_t)pl.P * pl.ncol);
  pl.Z = cv.take<float>((size_t)pl.P * pl.ncol);
  // one extra all-zero slot at the end (named by the primal step's slot table for absent terms)
  pl.zpart = cv.take<int>((size_t)pl.zslots_n * pl.ncol);
  pl.zslot = cv.take<int>((size_t)pl.P * 4);
  // K <= 16: the rotated Gram of blocks left to the per-lane Jacobi; K > 16: a copy of every
  // block's Gram (the large-block kernel re-derives V^T G V from it after its rotation steps)
  pl.G = cv.take<float>((size_t)pl.P * (pl.big ? (size_t)pl.K * pl.K : 256));
  pl.W = cv.take<float>((size_t)pl.P * 256);
  pl.V = cv.take<float>((size_t)pl.P * (pl.big ? (size_t)pl.K * pl.K : 256));
  pl.eflag = cv.take<int>((size_t)pl.P);
  pl.estat = cv.take<int>((size_t)(pl.P + 63) / 64 * 4);
  pl.l1part = cv.take<unsigned long long>((size_t)2 * l1_part_blocks(pl.N) * kL1Bins2);
  pl.Y = cv.take<float>((size_t)pl.P * (pl.big ? pl.K : kRows) * pl.ncol);
  pl.red_primal = cv.take<double>((size_t)pl.red_blocks * 4);
  pl.red_dual = cv.take<double>((size_t)(pl.red_blocks > 4 ? pl.red_blocks : 4));
  pl.sc = cv.take<DevScalars>(1);
  pl.hist = cv.take<L1Hist>(1);
  pl.bytes = align_up(cv.off);
}

// Operator l1 projection: scalars, histograms and the level-2 partial histograms.
size_t l1_workspace_bytes(long long n) {
  return align_up(sizeof(DevScalars)) + align_up(sizeof(L1Hist)) +
         align_up((size_t)l1_part_blocks(n) * kL1Bins2 * sizeof(unsigned long long));
}

BlockArgs block_args(const Plan &pl) {
  BlockArgs a;
  memset(&a, 0, sizeof(a));
  a.n1 = pl.n1;
  a.n2 = pl.n2;
  a.k1 = pl.k1;
  a.k2 = pl.k2;
  a.K = pl.K;
  a.ncol = pl.ncol;
  a.ntile = pl.ntile;
  a.nblk = pl.P;
  a.gradf = pl.gradf;
  a.gY = pl.g_Y;
  a.Y = pl.Y;
  a.G = pl.G;
  a.W = pl.W;
  a.V = pl.V;
  a.TA = pl.TA;
  a.TB = pl.TB;
  a.ntA = pl.ntA;
  a.ntB = pl.ntB;
  a.extA = pl.extA;
  a.extB = pl.extB;
  a.waves = pl.apply_waves;
  a.lds = pl.apply_lds;
  a.zpart = pl.zpart;
  a.sc = pl.sc;
  return a;
}

struct Gammas {
  double u, s, t, Y, y2, y3;
};

// HSSTV weight in effect (0 selects the comparison value 0.05).
double hsstv_omega(const s3ttv_params *pr) { return pr->omega > 0 ? pr->omega : 0.05; }

bool resolve_gammas(const s3ttv_shape *sh, const s3ttv_params *pr, Gammas &g) {
  const bool all0 = pr->gamma_u == 0 && pr->gamma_s == 0 && pr->gamma_t == 0 && pr->gamma_Y == 0 &&
                    pr->gamma_y2 == 0 && pr->gamma_y3 == 0;
  if (all0) {
    // Lemma 2 on the stacked operator: column sums 8K+1 (u), 1 (s), 3 (t); row sums 4 (Y),
    // 2 (y2), 3 (y3). Variants: u column sums 4K+1 (STV), 9 (SSTV), 9 + 4 omega (HSSTV);
    // the STV block rows sum to 2.
    const double K = (double)sh->k1 * sh->k2, om = hsstv_omega(pr);
    switch (pr->regularizer) {
      case S3TTV_REG_STV: g.u = 1.0 / (4.0 * K + 1.0); break;
      case S3TTV_REG_SSTV: g.u = 1.0 / 9.0; break;
      case S3TTV_REG_HSSTV: g.u = 1.0 / (9.0 + 4.0 * om); break;
      case S3TTV_REG_SSST: g.u = 1.0 / (6.0 * K + 1.0); break;
      default: g.u = 1.0 / (8.0 * K + 1.0); break;
    }
    g.s = 1.0;
    g.t = 1.0 / 3.0;
    g.Y = (pr->regularizer == S3TTV_REG_STV || pr->regularizer == S3TTV_REG_SSST) ? 0.5 : 0.25;
    g.y2 = 0.5;
    g.y3 = 1.0 / 3.0;
  } else {
    g = {pr->gamma_u, pr->gamma_s, pr->gamma_t, pr->gamma_Y, pr->gamma_y2, pr->gamma_y3};
  }
  const double *v = &g.u;
  for (int k = 0; k < 6; ++k)
    if (!(v[k] > 0 && isfinite(v[k]))) return false;
  return true;
}

bool valid_params(const s3ttv_params *pr) {
  if (!pr) return false;
  const double r[3] = {pr->eps, pr->alpha, pr->beta};
  for (double x : r)
    if (!(x > 0 && isfinite(x))) return false;
  if (!(isfinite(pr->mu_min) && isfinite(pr->mu_max) && pr->mu_min < pr->mu_max)) return false;
  if (pr->max_iter < 1) return false;
  if (!(pr->rel_tol >= 0 && isfinite(pr->rel_tol))) return false;
  if (pr->eig_max_steps > 255) return false;
  if (pr->gram_precision < S3TTV_GRAM_FP32 || pr->gram_precision > S3TTV_GRAM_FP16) return false;
  if (pr->regularizer < S3TTV_REG_S3TTV || pr->regularizer > S3TTV_REG_SSST) return false;
  if (!(pr->omega >= 0 && isfinite(pr->omega))) return false;
  return true;
}

// The HIP device current on the calling thread (streams and events belong to one device).
int current_device() {
  int d = 0;
  (void)hipGetDevice(&d);
  return d;
}

// Reusable HIP events for per-launch timing, per thread and device (kept until the thread
// ends).
struct EventPool {
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  hipEvent_t get() {
    if (used == ev.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      ev.push_back(e);
    }
    return ev[used++];
  }
};

EventPool &event_pool() {
  thread_local std::map<int, EventPool> pools;
  return pools[current_device()];
}

struct Timer {
  int mask;
  hipStream_t st;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> rec;
  hipEvent_t begin(int cls) {
    if (!(mask >> cls & 1)) return nullptr;
    hipEvent_t e = event_pool().get();
    if (e) (void)hipEventRecord(e, st);
    return e;
  }
  void end(int cls, hipEvent_t b) {
    if (!b) return;
    hipEvent_t e = event_pool().get();
    if (!e) return;
    (void)hipEventRecord(e, st);
    rec.push_back({cls, {b, e}});
  }
};

#define CK(x)                        \
  do {                               \
    hipError_t _e = (x);             \
    if (_e != hipSuccess) return S3TTV_EHIP; \
  } while (0)

#define TIMED(cls, call)                   \
  do {                                     \
    hipEvent_t _b = tm.begin(cls);         \
    CK(call);                              \
    tm.end(cls, _b);                       \
  } while (0)

// One problem of a solve: plan, kernel arguments and the caller's buffers.
struct Problem {
  Plan pl;
  BlockArgs bw;  // block-pass arguments (MFMA eigen-solve from the stored basis)
  bool fused = false;
  const s3ttv_params *prm = nullptr;
  const float *v = nullptr, *u0 = nullptr, *s0 = nullptr, *t0 = nullptr;
  float *u = nullptr, *s = nullptr, *t = nullptr;
};

// Validation, plan and parameters; no device work. forceTA/TB > 0 fix the anchor tile.
int32_t prepare(Problem &pr, const s3ttv_shape *shape, const s3ttv_params *params,
                const float *v, const float *u0, float *u, float *s, float *t, void *ws,
                size_t ws_bytes, int forceTA, int forceTB) {
  if (!valid_shape(shape) || !valid_params(params) || !v || !u || !s || !t || !ws)
    return S3TTV_EINVAL;
  const int32_t sup = supported_shape(shape, params->regularizer);
  if (sup != S3TTV_OK) return sup;
  Gammas gm;
  if (!resolve_gammas(shape, params, gm)) return S3TTV_EINVAL;
  Plan &pl = pr.pl;
  make_plan(pl, shape, nullptr, params->regularizer, forceTA, forceTB);
  if (ws_bytes < pl.bytes) return S3TTV_EWORKSPACE;
  make_plan(pl, shape, (char *)ws, params->regularizer, forceTA, forceTB);
  pl.g_u = (float)gm.u;
  pl.g_s = (float)gm.s;
  pl.g_t = (float)gm.t;
  pl.g_Y = (float)gm.Y;
  pl.g_y2 = (float)gm.y2;
  pl.g_y3 = (float)gm.y3;
  pl.mu_min = (float)params->mu_min;
  pl.mu_max = (float)params->mu_max;
  pl.reg = params->regularizer;
  pl.omega = (float)hsstv_omega(params);
  pl.g_Z2 = (float)(1.0 / (2.0 * hsstv_omega(params)));
  pl.eps = params->eps;
  pl.alpha = params->alpha;
  pl.beta = params->beta;
  pr.prm = params;
  pr.v = v;
  pr.u0 = u0;
  pr.u = u;
  pr.s = s;
  pr.t = t;
  // Every iteration diagonalises on MFMA from the stored basis (the identity before the
  // first); blocks the rotations cannot certify go to the per-lane Jacobi.
  pr.bw = block_args(pl);
  pr.bw.eflag = pl.eflag;
  pr.bw.estat = pl.estat;
  pr.bw.gram_prec = params->gram_precision;
  pr.bw.eig_steps = params->eig_max_steps == 0
                        ? kDefaultEigSteps
                        : (params->eig_max_steps < 0 ? 0 : params->eig_max_steps);
  pr.fused = !pl.big && fused_supported(pr.bw) && fused_lds_bytes(pr.bw) <= kMaxLds;
  // the separate Gram kernel sums in FP32 whatever was asked: its certificate takes the FP32
  // tolerance
  if (!pr.fused) pr.bw.gram_prec = 0;
  return S3TTV_OK;
}

// Scalars and block arguments point at sc (the batched solve keeps them side by side).
void set_scalars(Problem &pr, DevScalars *sc) {
  pr.pl.sc = sc;
  pr.bw.sc = sc;
}

// Initial state (all zero except u0) and the input checks.
int32_t enqueue_init(const Problem &pr, hipStream_t st) {
  const Plan &pl = pr.pl;
  CK(launch_init_scalars(pl, pr.prm->rel_tol, pr.prm->max_iter, st));
  CK(launch_zero_bytes(pl.hist, sizeof(L1Hist), st));
  CK(launch_check_finite(pr.v, pl.N, pl.sc, st));
  if (pr.u0) {
    CK(launch_check_finite(pr.u0, pl.N, pl.sc, st));
    CK(launch_copy(pl.u[0], pr.u0, pl.N, st));
  } else {
    CK(launch_fill(pl.u[0], pl.N, 0.f, st));
  }
  if (pr.s0) {
    CK(launch_check_finite(pr.s0, pl.N, pl.sc, st));
    CK(launch_copy(pl.s, pr.s0, pl.N, st));
  } else {
    CK(launch_fill(pl.s, pl.N, 0.f, st));
  }
  if (pr.t0) {
    CK(launch_check_finite(pr.t0, pl.N, pl.sc, st));
    CK(launch_copy(pl.t[0], pr.t0, pl.N, st));
  } else {
    CK(launch_fill(pl.t[0], pl.N, 0.f, st));
  }
  CK(launch_fill(pl.y2, pl.N, 0.f, st));
  CK(launch_fill(pl.w, pl.N, 0.f, st));
  CK(launch_fill(pl.Z, pl.P * pl.ncol, 0.f, st));
  CK(launch_fill(pl.Y, pl.P * (pl.big ? pl.K : kRows) * pl.ncol, 0.f, st));
  if (pl.reg == kRegHSSTV) CK(launch_fill(pl.gradf, pl.P * pl.ncol, 0.f, st));
  if (pl.big) {
    CK(launch_big_identity(pl.V, pl.P, pl.K, st));
    CK(launch_fill(pl.Z, pl.P * pl.ncol, 0.f, st));
    return S3TTV_OK;
  }
  CK(launch_identity16(pl.V, pl.P, st));
  // overlap-add partials start at zero (the first primal step may read them directly)
  CK(launch_fill(reinterpret_cast<float *>(pl.zpart), pl.zslots_n * pl.ncol, 0.f, st));
  CK(launch_zslots(pl, st));
  return S3TTV_OK;
}

// After enqueue_init has completed: the input check and the overlap-add route.
int32_t check_init(Problem &pr, const DevScalars &hs0) {
  if (hs0.nonfinite) return S3TTV_ENONFINITE;
  pr.pl.zfold = !pr.pl.big && hs0.zslot_overflow == 0 && zslots_fit(pr.pl);
  return S3TTV_OK;
}

// Iteration `it` (0-based) of Alg. 1 steps 2-14 for one problem.
int32_t enqueue_iteration(const Problem &pr, int it, Timer &tm, hipStream_t st) {
  const Plan &pl = pr.pl;
  const int c = it & 1, n = c ^ 1;
  TIMED(S3TTV_K_PRIMAL, launch_primal(pl, pl.u[c], pl.u[n], pl.t[c], st));
  TIMED(S3TTV_K_L1, launch_l1_select(2, 1, pl.alpha, pl.beta, pl.hist, pl.sc, st));
  TIMED(S3TTV_K_L1, launch_l1_hist_part(pl.xs, pl.xt, pl.N, 2, pl.l1part, pl.sc, st));
  TIMED(S3TTV_K_L1, launch_l1_part_reduce(2, pl.N, pl.l1part, pl.hist, pl.sc, st));
  TIMED(S3TTV_K_L1, launch_l1_select(2, 2, pl.alpha, pl.beta, pl.hist, pl.sc, st));
  TIMED(S3TTV_K_L1, launch_l1_hist(pl.xs, pl.xt, pl.N, 2, 3, pl.hist, pl.sc, st));
  TIMED(S3TTV_K_L1, launch_l1_select(2, 3, pl.alpha, pl.beta, pl.hist, pl.sc, st));
  // dual steps (3-7 thresholds, 12, 13) together with the gradient field of u' (steps 5, 9):
  // neither depends on the block pass
  TIMED(S3TTV_K_DUAL, launch_dual_grad(pl, pl.u[c], pl.u[n], pl.t[c], pl.t[n], pr.v, st));
  if (l1_reg(pl.reg)) {
    // l1 regulariser: its dual step ran inside the dual sweep; there are no blocks
    TIMED(S3TTV_K_FINAL, launch_finalize(pl, false, st));
    return S3TTV_OK;
  }
  if (pl.big) {
    BigArgs ba;
    ba.n1 = pl.n1; ba.n2 = pl.n2; ba.k1 = pl.k1; ba.k2 = pl.k2; ba.K = pl.K; ba.ncol = pl.ncol;
    ba.nblk = pl.P; ba.gradf = pl.gradf; ba.gY = pl.g_Y; ba.Y = pl.Y; ba.V = pl.V;
    ba.Gg = pl.G; ba.first = it == 0; ba.max_sweeps = kBigMaxSweeps; ba.sc = pl.sc;
    TIMED(S3TTV_K_BLOCK, launch_big_block(ba, st));
    TIMED(S3TTV_K_ZSUM, launch_big_overlap(ba, pl.Z, st));
    TIMED(S3TTV_K_FINAL, launch_finalize(pl, false, st));
    return S3TTV_OK;
  }
  // every iteration diagonalises on MFMA from the stored basis (the identity before the first),
  // the per-lane Jacobi taking only the blocks that rotation cannot certify
  if (pr.fused) {
    TIMED(S3TTV_K_BLOCK, launch_block_fused(pr.bw, st));
    TIMED(S3TTV_K_EIG, launch_eig(pr.bw, st));
    TIMED(S3TTV_K_EIG, launch_fixup(pr.bw, st));
  } else {
    TIMED(S3TTV_K_GRAM, launch_gram(pr.bw, st));
    TIMED(S3TTV_K_EIG, launch_eig(pr.bw, st));
    TIMED(S3TTV_K_APPLY, launch_apply(pr.bw, st));
  }
  if (!pl.zfold) TIMED(S3TTV_K_ZSUM, launch_zsum(pl, st));
  TIMED(S3TTV_K_FINAL, launch_finalize(pl, true, st));
  return S3TTV_OK;
}

// Result copies and statistics from the final scalars hs (tm: timed launches, nullable).
int32_t finish(const Problem &pr, const DevScalars &hs, float ms, Timer *tm, s3ttv_stats *stats,
               hipStream_t st, int iters_before = 0) {
  const Plan &pl = pr.pl;
  int32_t code = S3TTV_OK;
  if (hs.nonfinite) code = S3TTV_ENONFINITE;
  else if (pr.prm->rel_tol > 0 && !hs.converged) code = S3TTV_NOT_CONVERGED;
  if (code >= 0) {
    const int fin = hs.iters & 1;
    CK(launch_copy(pr.u, pl.u[fin], pl.N, st));
    CK(launch_copy(pr.s, pl.s, pl.N, st));
    CK(launch_copy(pr.t, pl.t[fin], pl.N, st));
  }
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    if (code >= 0) {
      double diag[4] = {0, 0, 0, 0};
      double *ddev = pl.red_dual;  // reuse: 4 doubles
      CK(launch_diagnostics(pl, pr.u, pr.s, pr.t, pr.v, ddev, st));
      CK(hipMemcpyAsync(diag, ddev, sizeof(diag), hipMemcpyDeviceToHost, st));
      CK(hipStreamSynchronize(st));
      stats->l1_s = diag[0];
      stats->l1_t = diag[1];
      stats->fid = sqrt(diag[2]);
      stats->dv_t = sqrt(diag[3]);
    }
    stats->iters = hs.iters - iters_before;
    stats->converged = hs.converged && !hs.nonfinite;
    stats->rel_change = hs.rel_change;
    stats->eig_max_sweeps = hs.max_sweeps;
    stats->eig_avg_sweeps =
        hs.sweep_waves ? (float)((double)hs.sweep_sum / (double)hs.sweep_waves) : 0.f;
    stats->eig_avg_steps =
        hs.step_blocks ? (float)((double)hs.step_sum / (double)hs.step_blocks) : 0.f;
    stats->eig_max_steps = hs.max_steps;
    stats->eig_fallback_blocks = (int64_t)hs.fallback_blocks;
    stats->eig_blocks = (int64_t)hs.step_blocks;
    stats->ms = ms;
    stats->tile_a = pl.TA;
    stats->tile_b = pl.TB;
    stats->status = code;
    if (tm) {
      for (auto &r : tm->rec) {
        float k = 0.f;
        if (hipEventElapsedTime(&k, r.second.first, r.second.second) == hipSuccess) {
          stats->kernel_ms[r.first] += k;
          stats->kernel_calls[r.first] += 1;
        }
      }
    }
  } else {
    CK(hipStreamSynchronize(st));
  }
  return code;
}

}  // namespace

// Batched-solve helpers.
namespace {

// Workspace bytes of one problem for any anchor tile the tuner may choose.
size_t plan_bytes_any_tile(const s3ttv_shape *sh, int reg) {
  size_t m = 0;
  for (auto &c : kTileCand) {
    Plan pl;
    make_plan(pl, sh, nullptr, reg, c[0], c[1]);
    if (pl.bytes > m) m = pl.bytes;
  }
  return m;
}

size_t batch_header_bytes(int n) { return align_up((size_t)n * sizeof(DevScalars)); }

// Streams and events of the batched solve, created once per thread and device (default
// priority), so that concurrent batched calls from different threads do not share them.
constexpr int kBatchStreams = 4;
struct BatchStreams {
  hipStream_t main = nullptr, fork[kBatchStreams] = {};
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_fork = nullptr, ev_join[kBatchStreams] = {};
  hipError_t status = hipSuccess;
  BatchStreams() {
    status = hipStreamCreateWithFlags(&main, hipStreamNonBlocking);
    for (int k = 0; k < kBatchStreams && status == hipSuccess; ++k)
      status = hipStreamCreateWithFlags(&fork[k], hipStreamNonBlocking);
    if (status == hipSuccess) status = hipEventCreateWithFlags(&ev_in, hipEventDisableTiming);
    if (status == hipSuccess) status = hipEventCreateWithFlags(&ev_out, hipEventDisableTiming);
    if (status == hipSuccess) status = hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming);
    for (int k = 0; k < kBatchStreams && status == hipSuccess; ++k)
      status = hipEventCreateWithFlags(&ev_join[k], hipEventDisableTiming);
  }
};

BatchStreams &batch_streams() {
  thread_local std::map<int, BatchStreams> m;
  return m[current_device()];
}

// Anchor tile per problem shape: the fastest candidate for the warm block pass, timed on the
// problem's own workspace with synthetic blocks (the arithmetic does not depend on the tile,
// so the choice only changes speed). Results are cached per shape for the process.
struct TileKey {
  int n1, n2, n3, k1, k2, prec, reg;
  bool operator<(const TileKey &o) const {
    const int a[7] = {n1, n2, n3, k1, k2, prec, reg};
    const int b[7] = {o.n1, o.n2, o.n3, o.k1, o.k2, o.prec, o.reg};
    for (int i = 0; i < 7; ++i)
      if (a[i] != b[i]) return a[i] < b[i];
    return false;
  }
};

std::map<TileKey, std::pair<int, int>> &tile_cache() {
  static std::map<TileKey, std::pair<int, int>> m;
  return m;
}

std::mutex &tile_mutex() {
  static std::mutex m;
  return m;
}

int32_t tune_tiles(const s3ttv_shape *shape, const s3ttv_params *params, void *ws, size_t ws_bytes,
                   hipStream_t st, int &TA, int &TB) {
  const TileKey key{shape->n1, shape->n2, shape->n3, shape->k1, shape->k2, params->gram_precision,
                     params->regularizer};
  {
    std::lock_guard<std::mutex> lk(tile_mutex());
    auto it = tile_cache().find(key);
    if (it != tile_cache().end()) {
      TA = it->second.first;
      TB = it->second.second;
      return S3TTV_OK;
    }
  }
  Problem def;
  float *dummy = reinterpret_cast<float *>(ws);
  int32_t r = prepare(def, shape, params, dummy, nullptr, dummy, dummy, dummy, ws, ws_bytes, 0, 0);
  if (r != S3TTV_OK) return r;
  TA = def.pl.TA;
  TB = def.pl.TB;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  float best = 1e30f;
  for (auto &c : kTileCand) {
    if (c[0] * c[1] > 64) continue;
    Problem pr;
    r = prepare(pr, shape, params, dummy, nullptr, dummy, dummy, dummy, ws, ws_bytes, c[0], c[1]);
    if (r != S3TTV_OK) continue;
    // keep the route of the default tile (fused or separate kernels)
    if (pr.fused != def.fused) continue;
    if (!pr.fused && pr.pl.apply_lds > kMaxLds) continue;
    const Plan &pl = pr.pl;
    CK(launch_init_scalars(pl, 0.0, 0, st));
    CK(launch_fill_hash(pl.Y, pl.P * kRows * pl.ncol, 0.01f, 1u, st));
    CK(launch_fill_hash(pl.gradf, pl.P * pl.ncol, 0.01f, 2u, st));
    CK(launch_identity16(pl.V, pl.P, st));
    const BlockArgs &b = pr.bw;
    float t_best = 1e30f;
    for (int rep = 0; rep < 4; ++rep) {
      CK(hipEventRecord(e0, st));
      if (pr.fused) {
        CK(launch_block_fused(b, st));
      } else {
        CK(launch_gram(b, st));
        CK(launch_eig(b, st));
        CK(launch_apply(b, st));
      }
      CK(hipEventRecord(e1, st));
      CK(hipEventSynchronize(e1));
      float ms = 0.f;
      CK(hipEventElapsedTime(&ms, e0, e1));
      if (rep > 0 && ms < t_best) t_best = ms;  // first launch is a warm-up
    }
    if (t_best < best) {
      best = t_best;
      TA = pl.TA;
      TB = pl.TB;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::lock_guard<std::mutex> lk(tile_mutex());
  tile_cache()[key] = {TA, TB};
  return S3TTV_OK;
}

}  // namespace

extern "C" {

const char *s3ttv_strerror(int32_t code) {
  switch (code) {
    case S3TTV_OK: return "ok";
    case S3TTV_NOT_CONVERGED: return "max_iter reached before rel_tol";
    case S3TTV_EINVAL: return "invalid argument";
    case S3TTV_EUNSUPPORTED:
      return "unsupported configuration (block rows k1*k2 > 100, 2^31 or more voxels, or a block "
             "pass that does not fit the LDS)";
    case S3TTV_EWORKSPACE: return "workspace too small";
    case S3TTV_EHIP: return "HIP runtime error";
    case S3TTV_ENONFINITE: return "non-finite value in input or iterates";
    default: return "unknown error";
  }
}

int32_t s3ttv_workspace_bytes(const s3ttv_shape *shape, const s3ttv_params *params, size_t *bytes) {
  if (!bytes || !valid_shape(shape)) return S3TTV_EINVAL;
  const int reg = reg_of(params);
  if (reg < S3TTV_REG_S3TTV || reg > S3TTV_REG_SSST) return S3TTV_EINVAL;
  const int32_t sup = supported_shape(shape, reg);
  if (sup != S3TTV_OK) return sup;
  Plan pl;
  make_plan(pl, shape, nullptr, reg);
  *bytes = pl.bytes;
  return S3TTV_OK;
}

int32_t s3ttv_solve(const s3ttv_shape *shape, const s3ttv_params *params, const float *v,
                    const float *u0, float *u, float *s, float *t, void *workspace,
                    size_t workspace_bytes, void *stream, s3ttv_stats *stats) {
  return s3ttv_solve_from(shape, params, v, u0, nullptr, nullptr, u, s, t, workspace,
                          workspace_bytes, stream, stats);
}

// A non-blocking stream of the calling thread and device on which a solve captures and
// replays its iteration graphs (a capture needs a stream of its own; the caller's stream may
// be the null stream). Joined to the caller's stream with events before and after.
struct SolveStream {
  hipStream_t s = nullptr;
  hipEvent_t in = nullptr, out = nullptr;
  hipError_t status;
  SolveStream() {
    status = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (status == hipSuccess) status = hipEventCreateWithFlags(&in, hipEventDisableTiming);
    if (status == hipSuccess) status = hipEventCreateWithFlags(&out, hipEventDisableTiming);
  }
};

static SolveStream &solve_stream() {
  thread_local std::map<int, SolveStream> m;
  return m[current_device()];
}

// The state signature a single solve records in its workspace (checked by a continuation).
static StateSig state_sig(const Problem &pr) {
  const Plan &pl = pr.pl;
  return StateSig{{kStateMagic, pl.n1, pl.n2, pl.n3, pl.k1, pl.k2, pl.reg, pl.TA * 256 + pl.TB}};
}

// Iterations it0 .. it_end - 1 of one problem whose state is in its workspace (stopping early
// when the rule fires), then the result copies and statistics. Iteration it0 == 0 runs
// directly; then, unless kernel timing is requested, one captured graph of `span` iterations
// (even, so the u / t buffer parity of its launches repeats) is replayed until the budget is
// used or the stop rule has fired on the device (a finished solve's later launches exit at
// once), and the remainder runs directly. The host reads the stop flag between spans.
static int32_t run_iterations(Problem &pr, const s3ttv_params *params, int it0, int it_end,
                              hipStream_t user, Timer &tm, s3ttv_stats *stats) {
  hipStream_t st = user;
  const int check = params->check_every > 0 ? params->check_every : 16;
  const int span = check < 2 ? 2 : (check > 256 ? 256 : (check + 1) & ~1);
  bool use_graph = params->timing_mask == 0 && it_end - it0 > 1 + span;
  if (use_graph) {
    SolveStream &ss = solve_stream();
    if (ss.status == hipSuccess) {
      CK(hipEventRecord(ss.in, user));
      CK(hipStreamWaitEvent(ss.s, ss.in, 0));
      st = ss.s;
    } else {
      use_graph = false;
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  CK(hipEventRecord(e0, st));
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int32_t r = S3TTV_OK;
  int it = it0;
  while (r == S3TTV_OK && it < it_end) {
    if (it >= 1 && use_graph && !exec && it + span <= it_end) {
      // capture once; if the stream cannot be captured, keep launching directly
      if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
      } else {
        for (int j = it; j < it + span && r == S3TTV_OK; ++j) r = enqueue_iteration(pr, j, tm, st);
        const hipError_t ce = hipStreamEndCapture(st, &graph);
        if (r != S3TTV_OK) break;
        if (ce != hipSuccess || hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
          if (graph) (void)hipGraphDestroy(graph);
          graph = nullptr;
          exec = nullptr;
          (void)hipGetLastError();
        }
      }
    }
    int next;
    if (exec && it + span <= it_end) {
      if (hipGraphLaunch(exec, st) != hipSuccess) r = S3TTV_EHIP;
      next = it + span;
    } else {
      // direct launches up to the next check point (or the end)
      next = it == 0 ? 1 : (params->rel_tol > 0 ? it + check : it_end);
      if (next > it_end) next = it_end;
      for (int j = it; j < next && r == S3TTV_OK; ++j) r = enqueue_iteration(pr, j, tm, st);
    }
    it = next;
    if (r == S3TTV_OK && params->rel_tol > 0 && it < it_end && it > 1) {
      int32_t done = 0;
      if (hipMemcpyAsync(&done, &pr.pl.sc->done, sizeof(done), hipMemcpyDeviceToHost, st) !=
              hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        r = S3TTV_EHIP;
      else if (done)
        break;
    }
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (st != user) {  // the caller's stream waits for the solve, also after an error
    if (hipEventRecord(solve_stream().out, st) != hipSuccess ||
        hipStreamWaitEvent(user, solve_stream().out, 0) != hipSuccess)
      r = r == S3TTV_OK ? S3TTV_EHIP : r;
    st = user;
  }
  if (r != S3TTV_OK) return r;
  CK(hipEventRecord(e1, st));
  DevScalars hs;
  CK(hipMemcpyAsync(&hs, pr.pl.sc, sizeof(hs), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  float ms = 0.f;
  CK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return finish(pr, hs, ms, &tm, stats, st, it0);
}

int32_t s3ttv_solve_from(const s3ttv_shape *shape, const s3ttv_params *params, const float *v,
                         const float *u0, const float *s0, const float *t0, float *u, float *s,
                         float *t, void *workspace, size_t workspace_bytes, void *stream,
                         s3ttv_stats *stats) {
  Problem pr;
  const int32_t prep = prepare(pr, shape, params, v, u0, u, s, t, workspace, workspace_bytes, 0, 0);
  if (prep != S3TTV_OK) return prep;
  pr.s0 = s0;
  pr.t0 = t0;
  CK(configure_block_kernels());
  hipStream_t st = (hipStream_t)stream;
  Timer tm{params->timing_mask, st, {}};
  event_pool().used = 0;
  const int32_t ini = enqueue_init(pr, st);
  if (ini != S3TTV_OK) return ini;
  CK(launch_mark_state(pr.pl, state_sig(pr), st));
  {
    DevScalars hs0;
    CK(hipMemcpyAsync(&hs0, pr.pl.sc, sizeof(hs0), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    const int32_t chk = check_init(pr, hs0);
    if (chk != S3TTV_OK) return chk;
  }
  return run_iterations(pr, params, 0, params->max_iter, st, tm, stats);
}

int32_t s3ttv_solve_continue(const s3ttv_shape *shape, const s3ttv_params *params, const float *v,
                             float *u, float *s, float *t, void *workspace,
                             size_t workspace_bytes, void *stream, s3ttv_stats *stats) {
  Problem pr;
  const int32_t prep =
      prepare(pr, shape, params, v, nullptr, u, s, t, workspace, workspace_bytes, 0, 0);
  if (prep != S3TTV_OK) return prep;
  CK(configure_block_kernels());
  hipStream_t st = (hipStream_t)stream;
  Timer tm{params->timing_mask, st, {}};
  event_pool().used = 0;
  DevScalars hs0;
  CK(hipMemcpyAsync(&hs0, pr.pl.sc, sizeof(hs0), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  const StateSig want = state_sig(pr);
  for (int k = 0; k < 8; ++k)
    if (hs0.sig[k] != want.v[k]) return S3TTV_EINVAL;
  if (hs0.nonfinite) return S3TTV_ENONFINITE;
  if (hs0.iters < 1 || hs0.iters > INT32_MAX - params->max_iter) return S3TTV_EINVAL;
  const int32_t chk = check_init(pr, hs0);
  if (chk != S3TTV_OK) return chk;
  CK(launch_resume_scalars(pr.pl, params->rel_tol, params->max_iter, st));
  return run_iterations(pr, params, hs0.iters, hs0.iters + params->max_iter, st, tm, stats);
}

// ---------------------------------------------------------------- batched solve

int32_t s3ttv_batch_workspace_bytes(int32_t n, const s3ttv_shape *shapes,
                                    const s3ttv_params *params, size_t *bytes) {
  if (n < 1 || !shapes || !bytes) return S3TTV_EINVAL;
  size_t total = batch_header_bytes(n);
  for (int i = 0; i < n; ++i) {
    if (!valid_shape(&shapes[i])) return S3TTV_EINVAL;
    const int reg = reg_of(params ? &params[i] : nullptr);
    if (reg < S3TTV_REG_S3TTV || reg > S3TTV_REG_SSST) return S3TTV_EINVAL;
    const int32_t sup = supported_shape(&shapes[i], reg);
    if (sup != S3TTV_OK) return sup;
    total += align_up(plan_bytes_any_tile(&shapes[i], reg));
  }
  *bytes = total;
  return S3TTV_OK;
}

int32_t s3ttv_solve_batched(int32_t n, const s3ttv_shape *shapes, const s3ttv_params *params,
                            const float *const *v, const float *const *u0, float *const *u,
                            float *const *s, float *const *t, void *workspace,
                            size_t workspace_bytes, void *stream, s3ttv_stats *stats) {
  if (n < 1 || !shapes || !params || !v || !u || !s || !t || !workspace) return S3TTV_EINVAL;
  size_t need = 0;
  const int32_t wb = s3ttv_batch_workspace_bytes(n, shapes, params, &need);
  if (wb != S3TTV_OK) return wb;
  if (workspace_bytes < need) return S3TTV_EWORKSPACE;
  for (int i = 0; i < n; ++i)
    if (!valid_params(&params[i]) || !v[i] || !u[i] || !s[i] || !t[i]) return S3TTV_EINVAL;
  CK(configure_block_kernels());
  BatchStreams &bs = batch_streams();
  CK(bs.status);
  hipStream_t user = (hipStream_t)stream, st = bs.main;
  CK(hipEventRecord(bs.ev_in, user));
  CK(hipStreamWaitEvent(st, bs.ev_in, 0));

  // ---- carve: scalars of all problems first (one read gathers every stop flag), then each
  // problem's region with its tuned anchor tile
  char *base = (char *)workspace;
  DevScalars *scs = reinterpret_cast<DevScalars *>(base);
  size_t off = batch_header_bytes(n);
  std::vector<Problem> prs(n);
  std::vector<int32_t> code(n, S3TTV_OK);
  for (int i = 0; i < n; ++i) {
    const size_t region = align_up(plan_bytes_any_tile(&shapes[i], params[i].regularizer));
    int TA = 0, TB = 0;
    // the l1 regularisers and blocks of more than 16 rows have no anchor tiles to tune
    int32_t r = l1_reg(params[i].regularizer) ||
                        shapes[i].k1 * shapes[i].k2 > kRows
                    ? S3TTV_OK
                    : tune_tiles(&shapes[i], &params[i], base + off, region, st, TA, TB);
    if (r == S3TTV_OK)
      r = prepare(prs[i], &shapes[i], &params[i], v[i], u0 ? u0[i] : nullptr, u[i], s[i], t[i],
                  base + off, region, TA, TB);
    if (r != S3TTV_OK) return r;
    set_scalars(prs[i], &scs[i]);
    off += region;
  }
  for (int i = 0; i < n; ++i) {
    const int32_t r = enqueue_init(prs[i], st);
    if (r != S3TTV_OK) return r;
  }
  std::vector<DevScalars> hs(n);
  CK(hipMemcpyAsync(hs.data(), scs, n * sizeof(DevScalars), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  std::vector<int> active;
  int max_iter = 0;
  for (int i = 0; i < n; ++i) {
    code[i] = check_init(prs[i], hs[i]);
    if (code[i] == S3TTV_OK) {
      active.push_back(i);
      if (params[i].max_iter > max_iter) max_iter = params[i].max_iter;
    }
  }
  Timer none{0, st, {}};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  CK(hipEventRecord(e0, st));

  // Enqueues iterations [it0, it1) of every active problem, problem i on fork stream i % K.
  auto enqueue_span = [&](int it0, int it1) -> int32_t {
    CK(hipEventRecord(bs.ev_fork, st));
    for (int k = 0; k < kBatchStreams; ++k) CK(hipStreamWaitEvent(bs.fork[k], bs.ev_fork, 0));
    for (int it = it0; it < it1; ++it)
      for (size_t a = 0; a < active.size(); ++a) {
        Timer tk{0, bs.fork[a % kBatchStreams], {}};
        const int32_t r = enqueue_iteration(prs[active[a]], it, tk, bs.fork[a % kBatchStreams]);
        if (r != S3TTV_OK) return r;
      }
    for (int k = 0; k < kBatchStreams; ++k) {
      CK(hipEventRecord(bs.ev_join[k], bs.fork[k]));
      CK(hipStreamWaitEvent(st, bs.ev_join[k], 0));
    }
    return S3TTV_OK;
  };
  auto all_done = [&]() -> int32_t {
    CK(hipMemcpyAsync(hs.data(), scs, n * sizeof(DevScalars), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    for (int i : active)
      if (!hs[i].done) return 0;
    return 1;
  };

  int32_t r = S3TTV_OK;
  if (!active.empty() && max_iter > 0) {
    // iteration 1 directly, then graphs of kBatchSpan iterations each (an
    // even span keeps the buffer parity of the captured launches); problems stop on the
    // device (stop rule or their own max_iter), their later launches exit at once
    r = enqueue_span(0, 1);
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    int it = 1;
    if (r == S3TTV_OK && max_iter > kBatchSpan) {
      CK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      r = enqueue_span(1, 1 + kBatchSpan);
      hipError_t ce = hipStreamEndCapture(st, &graph);
      if (r == S3TTV_OK && ce != hipSuccess) r = S3TTV_EHIP;
      if (r == S3TTV_OK && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
        r = S3TTV_EHIP;
    }
    while (r == S3TTV_OK && it < max_iter) {
      if (exec && it + kBatchSpan <= max_iter) {
        if (hipGraphLaunch(exec, st) != hipSuccess) r = S3TTV_EHIP;
        it += kBatchSpan;
      } else {
        r = enqueue_span(it, max_iter);
        it = max_iter;
      }
      if (r == S3TTV_OK && it < max_iter) {
        const int32_t d = all_done();
        if (d < 0) r = d;
        if (d == 1) break;
      }
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
  if (r != S3TTV_OK) return r;
  CK(hipEventRecord(e1, st));
  CK(hipMemcpyAsync(hs.data(), scs, n * sizeof(DevScalars), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  float ms = 0.f;
  CK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  int32_t overall = S3TTV_OK;
  for (int i = 0; i < n; ++i) {
    int32_t ci = code[i];
    if (ci == S3TTV_OK) ci = finish(prs[i], hs[i], ms, nullptr, stats ? &stats[i] : nullptr, st);
    else if (stats) {
      memset(&stats[i], 0, sizeof(stats[i]));
      stats[i].status = ci;
    }
    if (ci < 0 && overall >= 0) overall = ci;
    else if (ci == S3TTV_NOT_CONVERGED && overall == S3TTV_OK) overall = ci;
  }
  CK(hipEventRecord(bs.ev_out, st));
  CK(hipStreamWaitEvent(user, bs.ev_out, 0));
  return overall;
}

// ---------------------------------------------------------------- operator entry points

// Workspace of the spectral-clip operator: K <= 16 uses the fused block kernels (blocks of 16
// rows, 16-column tiles, Gram and basis scratch); larger K the large-block kernel (rows
// padded to 32-column chunks and a K x K basis per block).
static size_t clip_workspace_bytes(int64_t nblk, int K, int ncols) {
  if (K > kRows) {
    const size_t ncolp = (size_t)(ncols + 31) / 32 * 32;
    return align_up((size_t)nblk * K * ncolp * 4) + align_up((size_t)nblk * K * K * 4) +
           align_up(sizeof(DevScalars));
  }
  const size_t ncol = (size_t)(ncols + 15) / 16 * 16;
  return align_up((size_t)nblk * kRows * ncol * 4) + 2 * align_up((size_t)nblk * 256 * 4) +
         align_up(sizeof(DevScalars));
}

// The clip for K > 16: the blocks are copied into K x ncolp rows (zero columns appended up to
// a multiple of 32, which leave the singular values and vectors unchanged) and projected by
// the large-block kernel with no gradient term, its eigen-solve starting from the identity.
static int32_t spectral_clip_big(int32_t nblk, int32_t K, int32_t ncols, const float *yin, float *yout,
                          void *workspace, hipStream_t st) {
  const int ncolp = (ncols + 31) / 32 * 32;
  Carver cv{(char *)workspace, 0, false};
  float *Y = cv.take<float>((size_t)nblk * K * ncolp);
  float *V = cv.take<float>((size_t)nblk * K * K);
  DevScalars *sc = cv.take<DevScalars>(1);
  Plan tmp;
  memset(&tmp, 0, sizeof(tmp));
  tmp.sc = sc;
  CK(launch_init_scalars(tmp, 0.0, 0, st));
  CK(launch_fill(Y, (long long)nblk * K * ncolp, 0.f, st));
  CK(hipMemcpy2DAsync(Y, (size_t)ncolp * 4, yin, (size_t)ncols * 4, (size_t)ncols * 4,
                      (size_t)nblk * K, hipMemcpyDeviceToDevice, st));
  BigArgs ba;
  memset(&ba, 0, sizeof(ba));
  ba.n1 = 1;
  ba.n2 = nblk;
  ba.k1 = 1;
  ba.k2 = K;
  ba.K = K;
  ba.ncol = ncolp;
  ba.nblk = nblk;
  ba.gradf = nullptr;
  ba.gY = 0.f;
  ba.Y = Y;
  ba.V = V;
  ba.first = 1;
  ba.max_sweeps = kBigMaxSweeps;
  ba.sc = sc;
  CK(launch_big_block(ba, st));
  CK(hipMemcpy2DAsync(yout, (size_t)ncols * 4, Y, (size_t)ncolp * 4, (size_t)ncols * 4,
                      (size_t)nblk * K, hipMemcpyDeviceToDevice, st));
  CK(hipStreamSynchronize(st));
  return S3TTV_OK;
}

int32_t s3ttv_op_workspace_bytes(int32_t op, const s3ttv_shape *shape, int64_t n, size_t *bytes) {
  if (!bytes) return S3TTV_EINVAL;
  Plan pl;
  switch (op) {
    case S3TTV_OP_GRAD:
    case S3TTV_OP_GRAD_ADJ:
    case S3TTV_OP_DUAL_BLOCKS: {
      if (!valid_shape(shape)) return S3TTV_EINVAL;
      const int32_t sup = supported_shape(shape, kRegS3TTV);
      if (sup != S3TTV_OK) return sup;
      make_plan(pl, shape, nullptr, kRegS3TTV);
      *bytes = pl.bytes;
      return S3TTV_OK;
    }
    case S3TTV_OP_CLIP: {
      if (!shape || n < 1 || shape->k1 < 1 || shape->n3 < 1) return S3TTV_EINVAL;
      if (shape->k1 > kBigMax || n >= (1ll << 31)) return S3TTV_EUNSUPPORTED;
      *bytes = clip_workspace_bytes(n, shape->k1, shape->n3);
      return S3TTV_OK;
    }
    case S3TTV_OP_L1:
      if (n < 1) return S3TTV_EINVAL;
      if (n >= (1ll << 31)) return S3TTV_EUNSUPPORTED;
      *bytes = l1_workspace_bytes(n);
      return S3TTV_OK;
    default:
      return S3TTV_EINVAL;
  }
}

int32_t s3ttv_op_grad(const s3ttv_shape *shape, const float *u, float *gv, float *gh,
                      void *workspace, size_t workspace_bytes, void *stream) {
  if (!valid_shape(shape) || !u || !gv || !gh || !workspace) return S3TTV_EINVAL;
  const int32_t sup = supported_shape(shape, kRegS3TTV);
  if (sup != S3TTV_OK) return sup;
  Plan pl;
  make_plan(pl, shape, nullptr, kRegS3TTV);
  if (workspace_bytes < pl.bytes) return S3TTV_EWORKSPACE;
  make_plan(pl, shape, (char *)workspace, kRegS3TTV);
  hipStream_t st = (hipStream_t)stream;
  CK(launch_init_scalars(pl, 0.0, 0, st));
  CK(launch_grad(pl, u, u, 1.f, 0.f, pl.gradf, st));
  CK(launch_field_to_cubes(pl.gradf, gv, gh, pl.P, pl.n3, pl.Bp, st));
  CK(hipStreamSynchronize(st));
  return S3TTV_OK;
}

int32_t s3ttv_op_grad_adj(const s3ttv_shape *shape, const float *zv, const float *zh, float *w,
                          void *workspace, size_t workspace_bytes, void *stream) {
  if (!valid_shape(shape) || !zv || !zh || !w || !workspace) return S3TTV_EINVAL;
  const int32_t sup = supported_shape(shape, kRegS3TTV);
  if (sup != S3TTV_OK) return sup;
  Plan pl;
  make_plan(pl, shape, nullptr, kRegS3TTV);
  if (workspace_bytes < pl.bytes) return S3TTV_EWORKSPACE;
  make_plan(pl, shape, (char *)workspace, kRegS3TTV);
  hipStream_t st = (hipStream_t)stream;
  CK(launch_cubes_to_field(zv, zh, pl.Z, pl.P, pl.n3, pl.Bp, st));
  CK(launch_grad_adj(pl, pl.Z, w, st));
  CK(hipStreamSynchronize(st));
  return S3TTV_OK;
}

int32_t s3ttv_op_spectral_clip(int32_t nblk, int32_t K, int32_t ncols, const float *yin,
                               float *yout, void *workspace, size_t workspace_bytes, void *stream) {
  if (nblk < 1 || K < 1 || ncols < 1 || !yin || !yout || !workspace) return S3TTV_EINVAL;
  if (K > kBigMax) return S3TTV_EUNSUPPORTED;
  if (workspace_bytes < clip_workspace_bytes(nblk, K, ncols)) return S3TTV_EWORKSPACE;
  if (K > kRows) return spectral_clip_big(nblk, K, ncols, yin, yout, workspace, (hipStream_t)stream);
  const int ncol = (ncols + 15) / 16 * 16;
  Carver cv{(char *)workspace, 0, false};
  float *Y = cv.take<float>((size_t)nblk * kRows * ncol);
  float *G = cv.take<float>((size_t)nblk * 256);
  float *W = cv.take<float>((size_t)nblk * 256);
  DevScalars *sc = cv.take<DevScalars>(1);
  hipStream_t st = (hipStream_t)stream;
  Plan tmp;
  memset(&tmp, 0, sizeof(tmp));
  tmp.sc = sc;
  CK(launch_init_scalars(tmp, 0.0, 0, st));
  CK(launch_pack_blocks(yin, Y, nblk, K, ncols, ncol, 0, 0, 0, st));
  BlockArgs a;
  memset(&a, 0, sizeof(a));
  a.n1 = 1;
  a.n2 = nblk;
  a.k1 = 1;
  a.k2 = K;
  a.K = K;
  a.ncol = ncol;
  a.ntile = ncol / 16;
  a.nblk = nblk;
  a.gradf = nullptr;
  a.gY = 0.f;
  a.Y = Y;
  a.G = G;
  a.W = W;
  a.V = nullptr;
  a.TA = 1;
  a.TB = nblk < 64 ? nblk : 64;
  a.ntA = 1;
  a.ntB = (nblk + a.TB - 1) / a.TB;
  a.extA = 1;
  a.extB = a.TB;
  a.waves = a.ntile < 16 ? a.ntile : 16;
  a.lds = 0;
  a.zpart = nullptr;
  a.sc = sc;
  CK(launch_gram(a, st));
  CK(launch_eig(a, st));
  CK(launch_apply(a, st));
  CK(launch_unpack_blocks(Y, yout, nblk, K, ncols, ncol, 0, 0, 0, st));
  CK(hipStreamSynchronize(st));
  return S3TTV_OK;
}

int32_t s3ttv_op_dual_blocks(const s3ttv_shape *shape, double gamma_Y, const float *up,
                             const float *yin, float *yout, float *zv, float *zh,
                             void *workspace, size_t workspace_bytes, void *stream) {
  if (!valid_shape(shape) || !up || !yin || !yout || !zv || !zh || !workspace) return S3TTV_EINVAL;
  if (!(gamma_Y > 0 && isfinite(gamma_Y))) return S3TTV_EINVAL;
  const int32_t sup = supported_shape(shape, kRegS3TTV);
  if (sup != S3TTV_OK) return sup;
  Plan pl;
  make_plan(pl, shape, nullptr, kRegS3TTV);
  if (workspace_bytes < pl.bytes) return S3TTV_EWORKSPACE;
  make_plan(pl, shape, (char *)workspace, kRegS3TTV);
  pl.g_Y = (float)gamma_Y;
  hipStream_t st = (hipStream_t)stream;
  CK(configure_block_kernels());  // the apply kernel's overlap-add may need more than 64 KB of LDS
  CK(launch_init_scalars(pl, 0.0, 0, st));
  CK(launch_grad(pl, up, up, 1.f, 0.f, pl.gradf, st));
  if (pl.big) {
    // one workgroup per block, its eigen-solve started from the identity; the overlap-add
    // is a gather in a fixed order
    CK(launch_big_pack(yin, pl.Y, pl.P, pl.K, pl.n3, pl.Bp, st));
    BigArgs ba;
    memset(&ba, 0, sizeof(ba));
    ba.n1 = pl.n1; ba.n2 = pl.n2; ba.k1 = pl.k1; ba.k2 = pl.k2; ba.K = pl.K; ba.ncol = pl.ncol;
    ba.nblk = pl.P; ba.gradf = pl.gradf; ba.gY = pl.g_Y; ba.Y = pl.Y; ba.V = pl.V;
    ba.first = 1; ba.max_sweeps = kBigMaxSweeps; ba.sc = pl.sc;
    CK(launch_big_block(ba, st));
    CK(launch_big_overlap(ba, pl.Z, st));
    CK(launch_big_unpack(pl.Y, yout, pl.P, pl.K, pl.n3, pl.Bp, st));
    CK(launch_field_to_cubes(pl.Z, zv, zh, pl.P, pl.n3, pl.Bp, st));
    int32_t bad = 0;
    CK(hipMemcpyAsync(&bad, &pl.sc->nonfinite, sizeof(bad), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    return bad ? S3TTV_ENONFINITE : S3TTV_OK;
  }
  CK(launch_pack_blocks(yin, pl.Y, pl.P, pl.K, 2 * pl.n3, pl.ncol, 1, pl.n3, pl.Bp, st));
  BlockArgs ba = block_args(pl);
  ba.V = nullptr;
  CK(launch_gram(ba, st));
  CK(launch_eig(ba, st));
  CK(launch_apply(ba, st));
  CK(launch_zsum(pl, st));
  CK(launch_unpack_blocks(pl.Y, yout, pl.P, pl.K, 2 * pl.n3, pl.ncol, 1, pl.n3, pl.Bp, st));
  CK(launch_field_to_cubes(pl.Z, zv, zh, pl.P, pl.n3, pl.Bp, st));
  int32_t bad = 0;
  CK(hipMemcpyAsync(&bad, &pl.sc->nonfinite, sizeof(bad), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  return bad ? S3TTV_ENONFINITE : S3TTV_OK;
}

int32_t s3ttv_op_l1_project(int64_t n, const float *x, double radius, float *out, double *tau,
                            void *workspace, size_t workspace_bytes, void *stream) {
  if (n < 1 || !x || !out || !workspace || !(radius > 0 && isfinite(radius))) return S3TTV_EINVAL;
  if (n >= (1ll << 31)) return S3TTV_EUNSUPPORTED;
  const size_t need = l1_workspace_bytes(n);
  if (workspace_bytes < need) return S3TTV_EWORKSPACE;
  Carver cv{(char *)workspace, 0, false};
  DevScalars *sc = cv.take<DevScalars>(1);
  L1Hist *h = cv.take<L1Hist>(1);
  unsigned long long *part = cv.take<unsigned long long>((size_t)l1_part_blocks(n) * kL1Bins2);
  hipStream_t st = (hipStream_t)stream;
  Plan tmp;
  memset(&tmp, 0, sizeof(tmp));
  tmp.sc = sc;
  CK(launch_init_scalars(tmp, 0.0, 0, st));
  CK(launch_zero_bytes(h, sizeof(L1Hist), st));
  for (int level = 1; level <= 3; ++level) {
    if (level == 2) {
      CK(launch_l1_hist_part(x, nullptr, n, 1, part, sc, st));
      CK(launch_l1_part_reduce(1, n, part, h, sc, st));
    } else {
      CK(launch_l1_hist(x, nullptr, n, 1, level, h, sc, st));
    }
    CK(launch_l1_select(1, level, radius, radius, h, sc, st));
  }
  CK(launch_l1_apply(x, out, n, 0, sc, st));
  DevScalars hs;
  CK(hipMemcpyAsync(&hs, sc, sizeof(hs), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  if (tau) *tau = hs.active[0] ? hs.tau[0] : 0.0;
  return S3TTV_OK;
}

// ---------------------------------------------------------------- allocation-free l1 projection

}  // extern "C"

namespace {

// Scratch of s3ttv_op_l1_project_noalloc: the device scalars, the l1 histograms and the
// level-2 partial histograms of one projection of at most kNoAllocMaxN elements. Each GPU the
// library runs on holds one copy until the process ends. In host code the name `scratch` is a
// host-side stand-in: only the device address from hipGetSymbolAddress may reach a kernel.
constexpr long long kNoAllocMaxN = 1ll << 24;
constexpr size_t kNoAllocBytes = ((sizeof(DevScalars) + kAlign - 1) / kAlign * kAlign) +
                                 ((sizeof(L1Hist) + kAlign - 1) / kAlign * kAlign) +
                                 (size_t)((kNoAllocMaxN + kL1PartElems - 1) / kL1PartElems) *
                                     kL1Bins2 * sizeof(unsigned long long);
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// Device address of `scratch` on the current device, looked up once per device. The mutex
// also serialises the calls of this process on one device (they share the array).
struct NoAllocScratch {
  std::mutex mu;
  std::map<int, void *> ptr;
};

NoAllocScratch &noalloc_scratch() {
  static NoAllocScratch s;
  return s;
}

}  // namespace

extern "C" {

int32_t s3ttv_op_l1_project_noalloc(int64_t n, const float *x, double radius, float *out,
                                    double *tau, void *stream) {
  if (n < 1 || !x || !out || !(radius > 0 && isfinite(radius))) return S3TTV_EINVAL;
  if (n > kNoAllocMaxN) return S3TTV_EUNSUPPORTED;
  int dev = 0;
  CK(hipGetDevice(&dev));
  NoAllocScratch &ns = noalloc_scratch();
  std::lock_guard<std::mutex> lk(ns.mu);
  auto it = ns.ptr.find(dev);
  if (it == ns.ptr.end()) {
    void *p = nullptr;
    CK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return S3TTV_EHIP;
    it = ns.ptr.emplace(dev, p).first;
  }
  Carver cv{(char *)it->second, 0, false};
  DevScalars *sc = cv.take<DevScalars>(1);
  L1Hist *h = cv.take<L1Hist>(1);
  unsigned long long *part = cv.take<unsigned long long>((size_t)l1_part_blocks(n) * kL1Bins2);
  if (cv.off > kNoAllocBytes) return S3TTV_EUNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  Plan tmp;
  memset(&tmp, 0, sizeof(tmp));
  tmp.sc = sc;
  // the array keeps the previous call's contents: the scalars and the histograms that are
  // accumulated start from zero (the level-2 partials are written whole by their pass)
  CK(launch_init_scalars(tmp, 0.0, 0, st));
  CK(launch_zero_bytes(h, sizeof(L1Hist), st));
  for (int level = 1; level <= 3; ++level) {
    if (level == 2) {
      CK(launch_l1_hist_part(x, nullptr, n, 1, part, sc, st));
      CK(launch_l1_part_reduce(1, n, part, h, sc, st));
    } else {
      CK(launch_l1_hist(x, nullptr, n, 1, level, h, sc, st));
    }
    CK(launch_l1_select(1, level, radius, radius, h, sc, st));
  }
  CK(launch_l1_apply(x, out, n, 0, sc, st));
  DevScalars hs;
  CK(hipMemcpyAsync(&hs, sc, sizeof(hs), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  if (tau) *tau = hs.active[0] ? hs.tau[0] : 0.0;
  return S3TTV_OK;
}

}  // extern "C"

