// Exact projection onto the zero-centred l1 ball {||w||_1 <= r} (Alg. 1 steps 3-4,
// eqs. constraint_sparse / constraint_stripe) for gfx950.
//
// The projection is w = sign(x) max(|x| - tau, 0) where tau solves
//   phi(tau) = sum_i max(|x_i| - tau, 0) = r           (phi decreasing, piecewise linear).
// The paper cites a sort-based fast algorithm; here tau is found without sorting by a
// three-level multisection over the IEEE-754 bit pattern of |x| (a non-negative float orders
// like its bit pattern): level 1 bins bits 30..20, level 2 bits 19..9 inside the chosen
// level-1 bin, level 3 bits 8..0, where every bin is a single float value. At each level
// phi is evaluated at every bin edge at once from per-bin counts and sums, and the last
// edge with phi >= r selects the bin that brackets tau. All values of one level-1 bin share
// the exponent, so per-bin sums of the 24-bit significands are exact in 64-bit integers;
// edge sums are formed in FP64 in a fixed order. After level 3 the active set is known
// exactly and tau = (sum of |x| above the bin - r) / (their count).
#include "s3ttv_internal.h"

namespace s3ttv {

namespace {

constexpr int kNT = 256;

__device__ inline int level_shift(int level) {
  return level == 1 ? kL1Shift1 : (level == 2 ? kL1Shift2 : kL1Shift3);
}
__device__ inline int level_bins(int level) {
  return level == 1 ? kL1Bins1 : (level == 2 ? kL1Bins2 : kL1Bins3);
}
// Bits above this level (the parent prefix), as a shift: level 2 -> 20, level 3 -> 9.
__device__ inline int parent_shift(int level) { return level == 2 ? kL1Shift1 : kL1Shift2; }

__global__ __launch_bounds__(kNT) void k_l1_hist(const float *x0, const float *x1, long long n,
                                                 int nballs, int level, int vec, L1Hist *hist,
                                                 DevScalars *sc) {
  __shared__ unsigned long long h[2][kL1MaxBins];
  if (sc->done) return;
  const int shift = level_shift(level), nb = level_bins(level);
  int use[2] = {1, nballs > 1};
  uint32_t pref[2] = {0u, 0u};
  const int ps = level > 1 ? parent_shift(level) : 31;
  for (int k = 0; k < 2; ++k) {
    if (level > 1) use[k] = use[k] && sc->active[k];
    pref[k] = sc->prefix[k] >> ps;
  }
  if (!use[0] && !use[1]) return;
  for (int k = threadIdx.x; k < 2 * kL1MaxBins; k += kNT) (&h[0][0])[k] = 0ull;
  __syncthreads();
  const uint32_t mask = (uint32_t)nb - 1u;
  auto add = [&](int k, float x) {
    const uint32_t bits = __float_as_uint(x) & 0x7fffffffu;
    if (level > 1 && (bits >> ps) != pref[k]) return;
    const uint32_t ex = bits >> 23;
    const uint32_t sig = ex ? ((bits & 0x7fffffu) | 0x800000u) : (bits & 0x7fffffu);
    atomicAdd(&h[k][(bits >> shift) & mask], (1ull << 40) | (unsigned long long)sig);
  };
  // four elements per thread per trip (16-byte loads when aligned), scalar tail
  const long long n4 = vec ? n >> 2 : 0;
  for (long long e = (long long)blockIdx.x * kNT + threadIdx.x; e < n4;
       e += (long long)gridDim.x * kNT) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (!use[k]) continue;
      const float4 x = reinterpret_cast<const float4 *>(k == 0 ? x0 : x1)[e];
      add(k, x.x);
      add(k, x.y);
      add(k, x.z);
      add(k, x.w);
    }
  }
  for (long long e = 4 * n4 + (long long)blockIdx.x * kNT + threadIdx.x; e < n;
       e += (long long)gridDim.x * kNT) {
#pragma unroll
    for (int k = 0; k < 2; ++k)
      if (use[k]) add(k, (k == 0 ? x0 : x1)[e]);
  }
  __syncthreads();
  for (int k = 0; k < 2; ++k) {
    if (!use[k]) continue;
    uint32_t *gc = hist->cnt[k][level - 1];
    unsigned long long *gs = hist->sig[k][level - 1];
    for (int bi = threadIdx.x; bi < nb; bi += kNT) {
      const unsigned long long v = h[k][bi];
      if (v) {
        atomicAdd(&gc[bi], (uint32_t)(v >> 40));
        atomicAdd(&gs[bi], v & ((1ull << 40) - 1));
      }
    }
  }
}

// Level 2 without global atomics. Each workgroup histograms kL1PartElems elements per ball in
// LDS (count << 40 | significand sum: the significand sum of kL1PartElems 24-bit values fits
// in 40 bits) and writes its whole 2048-bin histogram to part[ball][workgroup][bin];
// k_l1_part_reduce then sums the partials per bin into the level-2 histogram. Every thread
// issues its kPartLoads 16-byte loads per ball before it touches the histogram.
constexpr int kPT = 1024;
constexpr int kPartLoads = kL1PartElems / (4 * kPT);  // float4 per thread per ball

__global__ __launch_bounds__(kPT) void k_l1_hist_part(const float *x0, const float *x1,
                                                      long long n, int nballs, int vec,
                                                      unsigned long long *part, DevScalars *sc) {
  __shared__ unsigned long long h[2][kL1Bins2];
  if (sc->done) return;
  const int ps = parent_shift(2);
  const bool use[2] = {sc->active[0] != 0, nballs > 1 && sc->active[1] != 0};
  if (!use[0] && !use[1]) return;
  const uint32_t pref[2] = {sc->prefix[0] >> ps, sc->prefix[1] >> ps};
  for (int k = threadIdx.x; k < 2 * kL1Bins2; k += kPT) (&h[0][0])[k] = 0ull;
  __syncthreads();
  const long long beg = (long long)blockIdx.x * kL1PartElems;
  const long long end = beg + kL1PartElems < n ? beg + kL1PartElems : n;
  auto add = [&](int k, float xv) {
    const uint32_t bits = __float_as_uint(xv) & 0x7fffffffu;
    if ((bits >> ps) != pref[k]) return;
    const uint32_t ex = bits >> 23;
    const uint32_t sig = ex ? ((bits & 0x7fffffu) | 0x800000u) : (bits & 0x7fffffu);
    atomicAdd(&h[k][(bits >> kL1Shift2) & (kL1Bins2 - 1)], (1ull << 40) | (unsigned long long)sig);
  };
  for (int k = 0; k < 2; ++k) {
    if (!use[k]) continue;
    const float *x = k == 0 ? x0 : x1;
    if (vec && end - beg == kL1PartElems) {
      const float4 *x4 = reinterpret_cast<const float4 *>(x + beg);
      float4 r[kPartLoads];
#pragma unroll
      for (int j = 0; j < kPartLoads; ++j) r[j] = x4[j * kPT + threadIdx.x];
#pragma unroll
      for (int j = 0; j < kPartLoads; ++j) {
        add(k, r[j].x);
        add(k, r[j].y);
        add(k, r[j].z);
        add(k, r[j].w);
      }
    } else {
      for (long long e = beg + threadIdx.x; e < end; e += kPT) add(k, x[e]);
    }
  }
  __syncthreads();
  for (int k = 0; k < 2; ++k) {
    if (!use[k]) continue;
    unsigned long long *dst = part + ((size_t)k * gridDim.x + blockIdx.x) * kL1Bins2;
    for (int bi = threadIdx.x; bi < kL1Bins2; bi += kPT) dst[bi] = h[k][bi];
  }
}

// Sums the level-2 partials: workgroup = 32 bins x 32 row groups; writes hist level 2.
__global__ __launch_bounds__(kPT) void k_l1_part_reduce(const unsigned long long *part, int nparts,
                                                        L1Hist *hist, DevScalars *sc) {
  __shared__ unsigned long long sc_[32][33], ss_[32][33];
  if (sc->done) return;
  const int per_ball = kL1Bins2 / 32;
  const int ball = blockIdx.x / per_ball;
  if (!sc->active[ball]) return;
  const int lb = threadIdx.x & 31, rg = threadIdx.x >> 5;
  const int b = (blockIdx.x - ball * per_ball) * 32 + lb;
  const unsigned long long *src = part + (size_t)ball * nparts * kL1Bins2 + b;
  unsigned long long c = 0, g = 0;
  for (int w = rg; w < nparts; w += 32) {
    const unsigned long long v = src[(size_t)w * kL1Bins2];
    c += v >> 40;
    g += v & ((1ull << 40) - 1);
  }
  sc_[rg][lb] = c;
  ss_[rg][lb] = g;
  __syncthreads();
  if (rg == 0) {
    for (int r = 1; r < 32; ++r) {
      c += sc_[r][lb];
      g += ss_[r][lb];
    }
    hist->cnt[ball][1][b] = (uint32_t)c;
    hist->sig[ball][1][b] = g;
  }
}

// One workgroup per ball. Scans the level's bins from the top, finds the bracketing bin and
// updates the carry; after level 3 writes tau. Clears the consumed histogram.
__global__ __launch_bounds__(kNT) void k_l1_select(int level, double r0, double r1, L1Hist *hist,
                                                   DevScalars *sc) {
  __shared__ double sS[kNT];
  __shared__ double sC[kNT];
  __shared__ int best;
  const int ball = blockIdx.x;
  const double radius = ball == 0 ? r0 : r1;
  uint32_t *gc = hist->cnt[ball][level - 1];
  unsigned long long *gs = hist->sig[ball][level - 1];
  const int nb = level_bins(level), shift = level_shift(level);
  const int per = nb / kNT;  // 8 or 2 bins per thread
  // thread t owns bins [nb - per*(t+1), nb - per*t), i.e. thread 0 the highest bins. Every
  // global value the kernel needs is requested first, so their latencies overlap.
  const int hi = nb - per * threadIdx.x;
  unsigned long long sraw[8];
  uint32_t craw[8];
#pragma unroll
  for (int m = 0; m < 8; ++m)
    if (m < per) {
      sraw[m] = gs[hi - 1 - m];
      craw[m] = gc[hi - 1 - m];
    }
  const int done = sc->done, act = sc->active[ball];
  const uint32_t pfx = sc->prefix[ball];
  const double S_carry = level == 1 ? 0.0 : sc->S_above[ball];
  const double C_carry = level == 1 ? 0.0 : (double)sc->C_above[ball];
  const bool skip = done || (level > 1 && !act);
  if (skip) {
    for (int k = threadIdx.x; k < nb; k += kNT) {
      gc[k] = 0u;
      gs[k] = 0ull;
    }
    return;
  }
  const uint32_t parent = level == 1 ? 0u : (pfx >> parent_shift(level)) << parent_shift(level);
  double val[8];
  double cnt[8];
  double lo_edge[8];
  double S = 0, C = 0;
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    if (m >= per) break;
    const int k = hi - 1 - m;  // descending
    const uint32_t bits = parent | ((uint32_t)k << shift);
    const int ex = (int)(bits >> 23);
    const double scale = ldexp(1.0, (ex > 0 ? ex : 1) - 150);
    val[m] = (double)sraw[m] * scale;
    cnt[m] = (double)craw[m];
    lo_edge[m] = (double)__uint_as_float(bits);
    S += val[m];
    C += cnt[m];
  }
  // exclusive prefix over threads (fixed Hillis-Steele order)
  sS[threadIdx.x] = S;
  sC[threadIdx.x] = C;
  __syncthreads();
  for (int off = 1; off < kNT; off <<= 1) {
    double s2 = 0, c2 = 0;
    if (threadIdx.x >= off) {
      s2 = sS[threadIdx.x - off];
      c2 = sC[threadIdx.x - off];
    }
    __syncthreads();
    sS[threadIdx.x] += s2;
    sC[threadIdx.x] += c2;
    __syncthreads();
  }
  double Sx = S_carry + (threadIdx.x ? sS[threadIdx.x - 1] : 0.0);
  double Cx = C_carry + (threadIdx.x ? sC[threadIdx.x - 1] : 0.0);
  const double total = S_carry + sS[kNT - 1];
  if (threadIdx.x == 0) best = -1;
  __syncthreads();
  if (level == 1 && total <= radius) {
    // already inside the ball: the projection is the identity
    if (threadIdx.x == 0) {
      sc->active[ball] = 0;
      sc->tau[ball] = 0.0;
    }
  } else {
    int mine = -1;
    double Sa = 0, Ca = 0;  // sums strictly above the candidate bin
    for (int m = 0; m < per; ++m) {
      const double Sb = Sx, Cb = Cx;
      Sx += val[m];
      Cx += cnt[m];
      if (Sx - Cx * lo_edge[m] >= radius) {
        mine = hi - 1 - m;
        Sa = Sb;
        Ca = Cb;
        break;
      }
    }
    if (mine >= 0) atomicMax(&best, mine);
    __syncthreads();
    int kstar = best;
    const bool owner = (kstar >= 0) ? (mine == kstar) : (threadIdx.x == kNT - 1);
    if (kstar < 0 && owner) {
      // rounding left no edge with phi >= r: take the lowest bin, carry = everything above it
      kstar = 0;
      Sa = Sx - val[per - 1];
      Ca = Cx - cnt[per - 1];
    }
    if (owner) {
      const uint32_t bits = parent | ((uint32_t)kstar << shift);
      if (level == 1) sc->active[ball] = 1;
      if (level < 3) {
        sc->prefix[ball] = bits;
        sc->S_above[ball] = Sa;
        sc->C_above[ball] = (unsigned long long)Ca;
      } else {
        const double vstar = (double)__uint_as_float(bits);
        sc->tau[ball] = Ca > 0 ? (Sa - radius) / Ca : vstar;
      }
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nb; k += kNT) {
    gc[k] = 0u;
    gs[k] = 0ull;
  }
}

__global__ void k_l1_apply(const float *x, float *out, long long n, int ball, DevScalars *sc) {
  const int act = sc->active[ball];
  const double tau = sc->tau[ball];
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const float v = x[e];
    if (!act) {
      out[e] = v;
    } else {
      const double a = fabs((double)v) - tau;
      out[e] = a > 0 ? copysignf((float)a, v) : 0.0f;
    }
  }
}

}  // namespace

int l1_grid(long long n) {
  long long g = (n + 8191) / 8192;
  if (g < 1) g = 1;
  if (g > 65535) g = 65535;
  return (int)g;
}

hipError_t launch_l1_hist(const float *x0, const float *x1, long long n, int nballs, int level,
                          L1Hist *hist, DevScalars *sc, hipStream_t st) {
  if (!x1) x1 = x0;
  const int vec = ((reinterpret_cast<uintptr_t>(x0) | reinterpret_cast<uintptr_t>(x1)) & 15) == 0;
  hipLaunchKernelGGL(k_l1_hist, dim3(l1_grid(n)), dim3(kNT), 0, st, x0, x1, n, nballs, level, vec,
                     hist, sc);
  return hipGetLastError();
}

int l1_part_blocks(long long n) {
  long long g = (n + kL1PartElems - 1) / kL1PartElems;
  return (int)(g < 1 ? 1 : g);
}

hipError_t launch_l1_hist_part(const float *x0, const float *x1, long long n, int nballs,
                               unsigned long long *part, DevScalars *sc, hipStream_t st) {
  if (!x1) x1 = x0;
  // 16-byte loads for the full chunks when both vectors are 16-byte aligned
  const int vec = ((reinterpret_cast<uintptr_t>(x0) | reinterpret_cast<uintptr_t>(x1)) & 15) == 0;
  hipLaunchKernelGGL(k_l1_hist_part, dim3(l1_part_blocks(n)), dim3(kPT), 0, st, x0, x1, n,
                     nballs, vec, part, sc);
  return hipGetLastError();
}

hipError_t launch_l1_part_reduce(int nballs, long long n, const unsigned long long *part,
                                 L1Hist *hist, DevScalars *sc, hipStream_t st) {
  hipLaunchKernelGGL(k_l1_part_reduce, dim3(nballs * (kL1Bins2 / 32)), dim3(kPT), 0, st, part,
                     l1_part_blocks(n), hist, sc);
  return hipGetLastError();
}

hipError_t launch_l1_select(int nballs, int level, double r0, double r1, L1Hist *hist,
                            DevScalars *sc, hipStream_t st) {
  hipLaunchKernelGGL(k_l1_select, dim3(nballs), dim3(kNT), 0, st, level, r0, r1, hist, sc);
  return hipGetLastError();
}

hipError_t launch_l1_apply(const float *x, float *out, long long n, int ball, DevScalars *sc,
                           hipStream_t st) {
  long long g = (n + 2047) / 2048;
  if (g < 1) g = 1;
  if (g > 65535) g = 65535;
  hipLaunchKernelGGL(k_l1_apply, dim3((int)g), dim3(kNT), 0, st, x, out, n, ball, sc);
  return hipGetLastError();
}

}  // namespace s3ttv
