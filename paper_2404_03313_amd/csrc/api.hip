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

#include <vector>

#include "../../include/s3ttv.h"
#include "s3ttv_internal.h"

using namespace s3ttv;

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kMaxLds = 152 * 1024;
constexpr int kDefaultEigSteps = 24;

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

int32_t supported_shape(const s3ttv_shape *sh) {
  if (sh->k1 * sh->k2 > kRows) return S3TTV_EUNSUPPORTED;
  const long long N = (long long)sh->n1 * sh->n2 * sh->n3;
  if (N >= (1ll << 31)) return S3TTV_EUNSUPPORTED;
  return S3TTV_OK;
}

// Anchor tile of the apply kernel: the largest tile whose overlap-add accumulators fit LDS.
void choose_tiles(Plan &pl) {
  static const int cand[][2] = {{8, 8}, {8, 4}, {4, 4}, {4, 2}, {2, 2}, {2, 1}, {1, 1}};
  for (auto &c : cand) {
    int TA = c[0] < pl.n1 ? c[0] : pl.n1, TB = c[1] < pl.n2 ? c[1] : pl.n2;
    const size_t lds = (size_t)(TA + pl.k1 - 1) * (TB + pl.k2 - 1) * (pl.ncol + 16) * sizeof(float);
    pl.TA = TA;
    pl.TB = TB;
    pl.apply_lds = lds;
    if (lds <= kMaxLds) break;
  }
  pl.extA = pl.TA + pl.k1 - 1;
  pl.extB = pl.TB + pl.k2 - 1;
  pl.ntA = (pl.n1 + pl.TA - 1) / pl.TA;
  pl.ntB = (pl.n2 + pl.TB - 1) / pl.TB;
  pl.apply_waves = pl.ntile < 16 ? pl.ntile : 16;
}

// Geometry + carve. base == nullptr -> size only.
void make_plan(Plan &pl, const s3ttv_shape *sh, char *base) {
  memset(&pl, 0, sizeof(pl));
  pl.n1 = sh->n1;
  pl.n2 = sh->n2;
  pl.n3 = sh->n3;
  pl.k1 = sh->k1;
  pl.k2 = sh->k2;
  pl.K = sh->k1 * sh->k2;
  pl.Bp = (sh->n3 + 15) / 16 * 16;
  pl.ncol = 2 * pl.Bp;
  pl.ntile = pl.ncol / 16;
  pl.P = (long long)sh->n1 * sh->n2;
  pl.N = pl.P * sh->n3;
  choose_tiles(pl);
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
  pl.zpart = cv.take<int>(((size_t)pl.ntA * pl.ntB * pl.extA * pl.extB + 1) * pl.ncol);
  pl.zslot = cv.take<int>((size_t)pl.P * 4);
  pl.G = cv.take<float>((size_t)pl.P * 256);
  pl.W = cv.take<float>((size_t)pl.P * 256);
  pl.V = cv.take<float>((size_t)pl.P * 256);
  pl.eflag = cv.take<int>((size_t)pl.P);
  pl.estat = cv.take<int>((size_t)(pl.P + 63) / 64 * 4);
  pl.l1part = cv.take<unsigned long long>((size_t)2 * l1_part_blocks(pl.N) * kL1Bins2);
  pl.Y = cv.take<float>((size_t)pl.P * kRows * pl.ncol);
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

bool resolve_gammas(const s3ttv_shape *sh, const s3ttv_params *pr, Gammas &g) {
  const bool all0 = pr->gamma_u == 0 && pr->gamma_s == 0 && pr->gamma_t == 0 && pr->gamma_Y == 0 &&
                    pr->gamma_y2 == 0 && pr->gamma_y3 == 0;
  if (all0) {
    // Lemma 2 on the stacked operator: column sums 8K+1 (u), 1 (s), 3 (t); row sums 4 (Y),
    // 2 (y2), 3 (y3).
    g.u = 1.0 / (8.0 * sh->k1 * sh->k2 + 1.0);
    g.s = 1.0;
    g.t = 1.0 / 3.0;
    g.Y = 0.25;
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
  return true;
}

// Reusable HIP events for per-launch timing (kept for the life of the process).
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
  static EventPool p;
  return p;
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

}  // namespace

extern "C" {

const char *s3ttv_strerror(int32_t code) {
  switch (code) {
    case S3TTV_OK: return "ok";
    case S3TTV_NOT_CONVERGED: return "max_iter reached before rel_tol";
    case S3TTV_EINVAL: return "invalid argument";
    case S3TTV_EUNSUPPORTED: return "unsupported configuration (block rows k1*k2 > 16 or too large)";
    case S3TTV_EWORKSPACE: return "workspace too small";
    case S3TTV_EHIP: return "HIP runtime error";
    case S3TTV_ENONFINITE: return "non-finite value in input or iterates";
    default: return "unknown error";
  }
}

int32_t s3ttv_workspace_bytes(const s3ttv_shape *shape, const s3ttv_params *params, size_t *bytes) {
  (void)params;
  if (!bytes || !valid_shape(shape)) return S3TTV_EINVAL;
  const int32_t sup = supported_shape(shape);
  if (sup != S3TTV_OK) return sup;
  Plan pl;
  make_plan(pl, shape, nullptr);
  *bytes = pl.bytes;
  return S3TTV_OK;
}

int32_t s3ttv_solve(const s3ttv_shape *shape, const s3ttv_params *params, const float *v,
                    const float *u0, float *u, float *s, float *t, void *workspace,
                    size_t workspace_bytes, void *stream, s3ttv_stats *stats) {
  if (!valid_shape(shape) || !valid_params(params) || !v || !u || !s || !t || !workspace)
    return S3TTV_EINVAL;
  const int32_t sup = supported_shape(shape);
  if (sup != S3TTV_OK) return sup;
  Gammas gm;
  if (!resolve_gammas(shape, params, gm)) return S3TTV_EINVAL;
  Plan pl;
  make_plan(pl, shape, nullptr);
  if (workspace_bytes < pl.bytes) return S3TTV_EWORKSPACE;
  make_plan(pl, shape, (char *)workspace);
  pl.g_u = (float)gm.u;
  pl.g_s = (float)gm.s;
  pl.g_t = (float)gm.t;
  pl.g_Y = (float)gm.Y;
  pl.g_y2 = (float)gm.y2;
  pl.g_y3 = (float)gm.y3;
  pl.mu_min = (float)params->mu_min;
  pl.mu_max = (float)params->mu_max;
  pl.eps = params->eps;
  pl.alpha = params->alpha;
  pl.beta = params->beta;
  hipStream_t st = (hipStream_t)stream;
  Timer tm{params->timing_mask, st, {}};
  event_pool().used = 0;

  // ---- initial state (all zero except u0)
  CK(launch_init_scalars(pl, params->rel_tol, st));
  CK(launch_zero_bytes(pl.hist, sizeof(L1Hist), st));
  CK(launch_check_finite(v, pl.N, pl.sc, st));
  if (u0) {
    CK(launch_check_finite(u0, pl.N, pl.sc, st));
    CK(launch_copy(pl.u[0], u0, pl.N, st));
  } else {
    CK(launch_fill(pl.u[0], pl.N, 0.f, st));
  }
  CK(launch_fill(pl.s, pl.N, 0.f, st));
  CK(launch_fill(pl.t[0], pl.N, 0.f, st));
  CK(launch_fill(pl.y2, pl.N, 0.f, st));
  CK(launch_fill(pl.w, pl.N, 0.f, st));
  CK(launch_fill(pl.Z, pl.P * pl.ncol, 0.f, st));
  CK(launch_fill(pl.Y, pl.P * kRows * pl.ncol, 0.f, st));
  CK(launch_identity16(pl.V, pl.P, st));
  // overlap-add partials start at zero (the first primal step may read them directly)
  CK(launch_fill(reinterpret_cast<float *>(pl.zpart),
                 ((long long)pl.ntA * pl.ntB * pl.extA * pl.extB + 1) * pl.ncol, 0.f, st));
  CK(launch_zslots(pl, st));
  {
    DevScalars hs0;
    CK(hipMemcpyAsync(&hs0, pl.sc, sizeof(hs0), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    if (hs0.nonfinite) return S3TTV_ENONFINITE;
    pl.zfold = hs0.zslot_overflow == 0 && zslots_fit(pl);
  }
  // First iteration: the stored basis is the identity, so every block is solved by the
  // per-lane Jacobi (cold). Later iterations diagonalise on MFMA from the previous basis.
  const BlockArgs ba = block_args(pl);
  BlockArgs bw = ba;
  bw.eflag = pl.eflag;
  bw.estat = pl.estat;
  bw.gram_prec = params->gram_precision;
  bw.eig_steps = params->eig_max_steps == 0 ? kDefaultEigSteps
                                            : (params->eig_max_steps < 0 ? 0 : params->eig_max_steps);
  const bool fused = fused_supported(bw) && fused_lds_bytes(bw) <= kMaxLds;
  const int check = params->check_every > 0 ? params->check_every : 16;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  CK(hipEventRecord(e0, st));
  int launched = 0;
  for (int it = 0; it < params->max_iter; ++it) {
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
    TIMED(S3TTV_K_DUAL, launch_dual_grad(pl, pl.u[c], pl.u[n], pl.t[c], pl.t[n], v, st));
    if (it > 0 && fused) {
      TIMED(S3TTV_K_BLOCK, launch_block_fused(bw, st));
      TIMED(S3TTV_K_EIG, launch_eig(bw, st));
      TIMED(S3TTV_K_EIG, launch_fixup(bw, st));
    } else {
      const BlockArgs &bk = it == 0 ? ba : bw;
      TIMED(S3TTV_K_GRAM, launch_gram(bk, st));
      TIMED(S3TTV_K_EIG, launch_eig(bk, st));
      TIMED(S3TTV_K_APPLY, launch_apply(bk, st));
    }
    if (!pl.zfold) TIMED(S3TTV_K_ZSUM, launch_zsum(pl, st));
    TIMED(S3TTV_K_FINAL, launch_finalize(pl, it > 0, st));
    ++launched;
    if (params->rel_tol > 0 && (it + 1) % check == 0 && it + 1 < params->max_iter) {
      int32_t done = 0;
      CK(hipMemcpyAsync(&done, &pl.sc->done, sizeof(done), hipMemcpyDeviceToHost, st));
      CK(hipStreamSynchronize(st));
      if (done) break;
    }
  }
  CK(hipEventRecord(e1, st));
  DevScalars hs;
  CK(hipMemcpyAsync(&hs, pl.sc, sizeof(hs), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  float ms = 0.f;
  CK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)launched;
  if (hs.nonfinite) return S3TTV_ENONFINITE;
  const int fin = hs.iters & 1;
  CK(launch_copy(u, pl.u[fin], pl.N, st));
  CK(launch_copy(s, pl.s, pl.N, st));
  CK(launch_copy(t, pl.t[fin], pl.N, st));
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    double diag[4] = {0, 0, 0, 0};
    double *ddev = pl.red_dual;  // reuse: 4 doubles
    CK(launch_diagnostics(pl, u, s, t, v, ddev, st));
    CK(hipMemcpyAsync(diag, ddev, sizeof(diag), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    stats->iters = hs.iters;
    stats->converged = hs.done && !hs.nonfinite;
    stats->rel_change = hs.rel_change;
    stats->l1_s = diag[0];
    stats->l1_t = diag[1];
    stats->fid = sqrt(diag[2]);
    stats->dv_t = sqrt(diag[3]);
    stats->eig_max_sweeps = hs.max_sweeps;
    stats->eig_avg_sweeps = hs.sweep_waves ? (float)((double)hs.sweep_sum / (double)hs.sweep_waves) : 0.f;
    stats->eig_avg_steps = hs.step_blocks ? (float)((double)hs.step_sum / (double)hs.step_blocks) : 0.f;
    stats->eig_max_steps = hs.max_steps;
    stats->eig_fallback_blocks = (int64_t)hs.fallback_blocks;
    stats->ms = ms;
    for (auto &r : tm.rec) {
      float k = 0.f;
      if (hipEventElapsedTime(&k, r.second.first, r.second.second) == hipSuccess) {
        stats->kernel_ms[r.first] += k;
        stats->kernel_calls[r.first] += 1;
      }
    }
  } else {
    CK(hipStreamSynchronize(st));
  }
  if (params->rel_tol > 0 && !hs.done) return S3TTV_NOT_CONVERGED;
  return S3TTV_OK;
}

// ---------------------------------------------------------------- operator entry points

int32_t s3ttv_op_workspace_bytes(int32_t op, const s3ttv_shape *shape, int64_t n, size_t *bytes) {
  if (!bytes) return S3TTV_EINVAL;
  Plan pl;
  switch (op) {
    case S3TTV_OP_GRAD:
    case S3TTV_OP_GRAD_ADJ:
    case S3TTV_OP_DUAL_BLOCKS: {
      if (!valid_shape(shape)) return S3TTV_EINVAL;
      const int32_t sup = supported_shape(shape);
      if (sup != S3TTV_OK) return sup;
      make_plan(pl, shape, nullptr);
      *bytes = pl.bytes;
      return S3TTV_OK;
    }
    case S3TTV_OP_CLIP: {
      if (!shape || n < 1 || shape->k1 < 1 || shape->k1 > kRows || shape->n3 < 1) return S3TTV_EINVAL;
      const int ncols = shape->n3;
      const int ncol = (ncols + 15) / 16 * 16;
      *bytes = align_up((size_t)n * kRows * ncol * 4) + 2 * align_up((size_t)n * 256 * 4) +
               align_up(sizeof(DevScalars));
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
  const int32_t sup = supported_shape(shape);
  if (sup != S3TTV_OK) return sup;
  Plan pl;
  make_plan(pl, shape, nullptr);
  if (workspace_bytes < pl.bytes) return S3TTV_EWORKSPACE;
  make_plan(pl, shape, (char *)workspace);
  hipStream_t st = (hipStream_t)stream;
  CK(launch_init_scalars(pl, 0.0, st));
  CK(launch_grad(pl, u, u, 1.f, 0.f, pl.gradf, st));
  CK(launch_field_to_cubes(pl.gradf, gv, gh, pl.P, pl.n3, pl.Bp, st));
  CK(hipStreamSynchronize(st));
  return S3TTV_OK;
}

int32_t s3ttv_op_grad_adj(const s3ttv_shape *shape, const float *zv, const float *zh, float *w,
                          void *workspace, size_t workspace_bytes, void *stream) {
  if (!valid_shape(shape) || !zv || !zh || !w || !workspace) return S3TTV_EINVAL;
  const int32_t sup = supported_shape(shape);
  if (sup != S3TTV_OK) return sup;
  Plan pl;
  make_plan(pl, shape, nullptr);
  if (workspace_bytes < pl.bytes) return S3TTV_EWORKSPACE;
  make_plan(pl, shape, (char *)workspace);
  hipStream_t st = (hipStream_t)stream;
  CK(launch_cubes_to_field(zv, zh, pl.Z, pl.P, pl.n3, pl.Bp, st));
  CK(launch_grad_adj(pl, pl.Z, w, st));
  CK(hipStreamSynchronize(st));
  return S3TTV_OK;
}

int32_t s3ttv_op_spectral_clip(int32_t nblk, int32_t K, int32_t ncols, const float *yin,
                               float *yout, void *workspace, size_t workspace_bytes, void *stream) {
  if (nblk < 1 || K < 1 || ncols < 1 || !yin || !yout || !workspace) return S3TTV_EINVAL;
  if (K > kRows) return S3TTV_EUNSUPPORTED;
  const int ncol = (ncols + 15) / 16 * 16;
  const size_t need = align_up((size_t)nblk * kRows * ncol * 4) + 2 * align_up((size_t)nblk * 256 * 4) +
                      align_up(sizeof(DevScalars));
  if (workspace_bytes < need) return S3TTV_EWORKSPACE;
  Carver cv{(char *)workspace, 0, false};
  float *Y = cv.take<float>((size_t)nblk * kRows * ncol);
  float *G = cv.take<float>((size_t)nblk * 256);
  float *W = cv.take<float>((size_t)nblk * 256);
  DevScalars *sc = cv.take<DevScalars>(1);
  hipStream_t st = (hipStream_t)stream;
  Plan tmp;
  memset(&tmp, 0, sizeof(tmp));
  tmp.sc = sc;
  CK(launch_init_scalars(tmp, 0.0, st));
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
  const int32_t sup = supported_shape(shape);
  if (sup != S3TTV_OK) return sup;
  Plan pl;
  make_plan(pl, shape, nullptr);
  if (workspace_bytes < pl.bytes) return S3TTV_EWORKSPACE;
  make_plan(pl, shape, (char *)workspace);
  pl.g_Y = (float)gamma_Y;
  hipStream_t st = (hipStream_t)stream;
  CK(launch_init_scalars(pl, 0.0, st));
  CK(launch_grad(pl, up, up, 1.f, 0.f, pl.gradf, st));
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
  CK(launch_init_scalars(tmp, 0.0, st));
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
