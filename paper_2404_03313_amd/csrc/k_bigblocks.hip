// Block pass for blocks of more than 16 rows (K = k1 k2 up to 100; the paper's experiments use
// 10 x 10 windows, Sec. IV-A): Alg. 1 steps 9-10 and the overlap-add of step 2, one workgroup
// per block.
//
// Per block l (rows r = a k2 + c, columns in the comp-major field layout):
//   Y' = Y + g_Y P_l D D_s u'                      (step 9, written back in place)
//   G  = Y' Y'^T                                    (K x K, FP32 sums, 32-column chunks)
//   if every Gershgorin row bound of G is <= 1, no singular value of Y' exceeds 1 and step 10
//   leaves Y' unchanged; otherwise
//   A = V^T G V from the stored (orthonormal) eigenbasis V of the previous iteration,
//   parallel cyclic Jacobi on A (round-robin pair order, all K/2 rotations of a step at once,
//   accumulated into V) until a certificate holds: every off-diagonal entry in a row or column
//   whose diagonal exceeds 0.999 is at most 1e-6 ||A||_F (about the FP32 rounding level of
//   the rotations), and every other row has a Gershgorin bound <= 1, so no eigenvalue above 1
//   hides among them (the clip factor 1 - lambda^-1/2 is continuous at 1 and uses the
//   Rayleigh quotients below, so eigenvalues next to 1 need no separation);
//   one Newton-Schulz step V <- V (3 I - V^T V) / 2 restores orthonormality lost to rounding;
//   lambda_i = ||v_i^T Y'||^2 (Rayleigh quotients, more accurate than the rotated diagonal);
//   Y+ = Y' - V_R diag(1 - lambda^-1/2) V_R^T Y'   over R = {i : lambda_i > 1}
// which is the spectral clip of step 10 (eqs. ProxConjugate, prox_nuclear_norm), formed as a
// low-rank correction. The basis is kept for the next iteration.
//
// The overlap-add sum_l P_l^T Y_l is a gather (each pixel reads its K windows in a fixed
// order), so results are reproducible.
#include "s3ttv_internal.h"

namespace s3ttv {

namespace {

constexpr int kNT = 256;
constexpr int kChunk = 32;
// Rows whose diagonal exceeds this take part in the off-diagonal test of the certificate.
constexpr float kNearOne = 0.999f;

__device__ inline int wrapm(int x, int n) { return x < 0 ? x + n : (x >= n ? x - n : x); }

// Round-robin pairing of m (even) indices, step s (0 <= s < m - 1), pair k (0 <= k < m / 2):
// index m - 1 stays, the others rotate.
__device__ inline void rr_pair(int m, int s, int k, int &p, int &q) {
  const int n = m - 1;
  int x = k == 0 ? n : (s + k) % n;
  int y = (s + n - k) % n;
  if (k == 0) y = s % n;
  p = min(x, y);
  q = max(x, y);
}

// C (K x K) = op(A) B with A and B in LDS (row stride KS); op(A) = A^T when TA. Thread
// (ti, tj) of a 16 x 16 grid forms the 8 x 8 tile at rows 8 ti, columns 8 tj (K <= 128), so
// each k costs 16 LDS reads for 64 independent FMAs.
template <bool TA>
__device__ inline void mm_tile(const float *A, const float *B, int K, int KS, int ti, int tj,
                               float acc[8][8]) {
#pragma unroll
  for (int x = 0; x < 8; ++x)
#pragma unroll
    for (int y = 0; y < 8; ++y) acc[x][y] = 0.f;
  for (int k = 0; k < K; ++k) {
    float av[8], bv[8];
#pragma unroll
    for (int x = 0; x < 8; ++x) {
      const int r = 8 * ti + x, c = 8 * tj + x;
      av[x] = r < K ? (TA ? A[k * KS + r] : A[r * KS + k]) : 0.f;
      bv[x] = c < K ? B[k * KS + c] : 0.f;
    }
#pragma unroll
    for (int x = 0; x < 8; ++x)
#pragma unroll
      for (int y = 0; y < 8; ++y) acc[x][y] = fmaf(av[x], bv[y], acc[x][y]);
  }
}

// P (K x 32, row stride cs) = V^T Y (Y: K x 32 chunk, row stride cs); thread (ti, tc) of a
// 32 x 8 grid forms rows 4 ti .. 4 ti + 3, columns 4 tc .. 4 tc + 3.
__device__ inline void proj_tile(const float *V, const float *Y, int K, int KS, int cs, int ti,
                                 int tc, float acc[4][4]) {
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = 0.f;
  for (int r = 0; r < K; ++r) {
    float av[4], bv[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      av[x] = 4 * ti + x < K ? V[r * KS + 4 * ti + x] : 0.f;
      bv[x] = Y[r * cs + 4 * tc + x];
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[x][y] = fmaf(av[x], bv[y], acc[x][y]);
  }
}

}  // namespace

__global__ __launch_bounds__(kNT) void k_big_block(BigArgs a) {
  extern __shared__ float lds[];
  const int K = a.K, KS = a.K + 1;
  const int GS = KS > kChunk + 1 ? KS : kChunk + 1;
  float *G = lds;                 // K x GS: Gram, then A, then projections of a chunk
  float *V = G + K * GS;          // K x KS: eigenbasis, column c = vector c
  float *T3 = V + K * KS;         // K x GS: H = G V, V^T V, or a Y' column chunk
  __shared__ float cs[64], sn[64], lam[112];
  __shared__ int pq[64][2];
  __shared__ float red[kNT / 64];
  __shared__ int flag;
  if (a.sc->done) return;
  const int tid = threadIdx.x;
  const long long blk = blockIdx.x;
  const int p0 = (int)(blk / a.n2), q0 = (int)(blk - (long long)p0 * a.n2);
  const int ncol = a.ncol;
  float *Yb = a.Y + blk * (long long)K * ncol;
  const int CS = kChunk + 1;

  // ---- Gram over column chunks; Y' is written back
  // thread (ti, tj) of a 16 x 16 grid owns rows 8 ti .. 8 ti + 7 and columns 8 tj .. 8 tj + 7
  const int ti = tid >> 4, tj = tid & 15;
  float acc[8][8];
#pragma unroll
  for (int x = 0; x < 8; ++x)
#pragma unroll
    for (int y = 0; y < 8; ++y) acc[x][y] = 0.f;
  for (int c0 = 0; c0 < ncol; c0 += kChunk) {
    __syncthreads();
    for (int e = tid; e < K * kChunk; e += kNT) {
      const int r = e / kChunk, cc = e - r * kChunk, col = c0 + cc;
      const int ra = r / a.k2, rc = r - ra * a.k2;
      const long long pix = (long long)wrapm(p0 + ra, a.n1) * a.n2 + wrapm(q0 + rc, a.n2);
      const float y = Yb[(long long)r * ncol + col] + a.gY * a.gradf[pix * ncol + col];
      Yb[(long long)r * ncol + col] = y;
      T3[r * CS + cc] = y;
    }
    __syncthreads();
    for (int cc = 0; cc < kChunk; ++cc) {
      float yr[8], yc[8];
#pragma unroll
      for (int x = 0; x < 8; ++x) {
        const int r = 8 * ti + x, c = 8 * tj + x;
        yr[x] = r < K ? T3[r * CS + cc] : 0.f;
        yc[x] = c < K ? T3[c * CS + cc] : 0.f;
      }
#pragma unroll
      for (int x = 0; x < 8; ++x)
#pragma unroll
        for (int y = 0; y < 8; ++y) acc[x][y] = fmaf(yr[x], yc[y], acc[x][y]);
    }
  }
#pragma unroll
  for (int x = 0; x < 8; ++x)
#pragma unroll
    for (int y = 0; y < 8; ++y) {
      const int r = 8 * ti + x, c = 8 * tj + y;
      if (r < K && c < K) G[r * KS + c] = acc[x][y];
    }
  if (tid == 0) flag = 0;
  __syncthreads();
  // ---- finiteness and the Gershgorin bound: max_i sum_j |G_ij| <= 1 => nothing to clip
  for (int r = tid; r < K; r += kNT) {
    float s = 0.f;
    for (int c = 0; c < K; ++c) s += fabsf(G[r * KS + c]);
    if (!(s <= 1.f)) atomicOr(&flag, isfinite(s) ? 1 : 2);
  }
  __syncthreads();
  if (flag & 2) {
    if (tid == 0) atomicExch(&a.sc->nonfinite, 1);
    return;
  }
  if (flag == 0) return;  // Y' already stored; the basis is kept as it is

  // ---- basis: identity on the first use, else the stored one (orthonormal to rounding)
  float *Vg = a.V + blk * (long long)K * K;
  for (int e = tid; e < K * K; e += kNT) {
    const int r = e / K, c = e - r * K;
    V[r * KS + c] = a.first ? (r == c ? 1.f : 0.f) : Vg[e];
  }
  __syncthreads();
  // ---- A = V^T (G V): H = G V into T3, then A into G
  {
    float acc[8][8];
    mm_tile<false>(G, V, K, KS, ti, tj, acc);
#pragma unroll
    for (int x = 0; x < 8; ++x)
#pragma unroll
      for (int y = 0; y < 8; ++y)
        if (8 * ti + x < K && 8 * tj + y < K) T3[(8 * ti + x) * KS + 8 * tj + y] = acc[x][y];
    __syncthreads();
    mm_tile<true>(V, T3, K, KS, ti, tj, acc);
#pragma unroll
    for (int x = 0; x < 8; ++x)
#pragma unroll
      for (int y = 0; y < 8; ++y)
        if (8 * ti + x < K && 8 * tj + y < K) G[(8 * ti + x) * KS + 8 * tj + y] = acc[x][y];
  }
  __syncthreads();
  // symmetrise exactly
  for (int e = tid; e < K * K; e += kNT) {
    const int r = e / K, c = e - r * K;
    if (r < c) {
      const float m = 0.5f * (G[r * KS + c] + G[c * KS + r]);
      G[r * KS + c] = m;
      G[c * KS + r] = m;
    }
  }
  __syncthreads();

  // ---- parallel cyclic Jacobi
  const int m = (K + 1) & ~1;  // even; index K (if m > K) is a dummy
  const int nsplit = kNT / K;  // threads per column (row) in the rotation phases
  const int part = tid / K;
  int sweeps = 0;
  for (; sweeps < a.max_sweeps; ++sweeps) {
    // certificate (see the header): one thread per row
    float fro = 0.f;
    for (int e = tid; e < K * K; e += kNT) {
      const int r = e / K, c = e - r * K;
      fro = fmaf(G[r * KS + c], G[r * KS + c], fro);
    }
    for (int mm = 32; mm >= 1; mm >>= 1) fro += __shfl_xor(fro, mm);
    if ((tid & 63) == 0) red[tid >> 6] = fro;
    if (tid == 0) flag = 0;
    __syncthreads();
    const float tol = 1e-6f * sqrtf((red[0] + red[1]) + (red[2] + red[3]));
    if (tid < K) {
      const float dr = G[tid * KS + tid];
      float sum = 0.f, mx = 0.f;
      for (int c = 0; c < K; ++c) {
        if (c == tid) continue;
        const float x = fabsf(G[tid * KS + c]);
        sum += x;
        if (dr > kNearOne || G[c * KS + c] > kNearOne) mx = fmaxf(mx, x);
      }
      if (mx > tol || (dr <= kNearOne && dr + sum > 1.f)) atomicOr(&flag, 1);
    }
    __syncthreads();
    const int notyet = flag;
    __syncthreads();
    if (!notyet) break;
    const float skip = 0.1f * tol;
    for (int s = 0; s < m - 1; ++s) {
      if (tid < m / 2) {
        int p, q;
        rr_pair(m, s, tid, p, q);
        float c = 1.f, sv = 0.f;
        if (q < K) {
          const float apq = G[p * KS + q];
          if (fabsf(apq) > skip) {  // threshold Jacobi: pairs already below skip stay
            const float app = G[p * KS + p], aqq = G[q * KS + q];
            const float zeta = (aqq - app) / (2.f * apq);
            const float t = fabsf(zeta) > 1e15f
                                ? 0.5f / zeta
                                : copysignf(1.f, zeta) / (fabsf(zeta) + sqrtf(1.f + zeta * zeta));
            c = 1.f / sqrtf(1.f + t * t);
            sv = t * c;
          }
        }
        cs[tid] = c;
        sn[tid] = sv;
        pq[tid][0] = p;
        pq[tid][1] = q;
      }
      __syncthreads();
      // rows: A <- J^T A. Thread t < nsplit K owns column j = t mod K and every nsplit-th pair,
      // four pairs at a time (their rows are distinct, so the loads overlap)
      if (tid < nsplit * K) {
        const int j = tid - part * K;
        for (int k0 = part; k0 < m / 2; k0 += 4 * nsplit) {
          float c[4], sv[4], ap[4], aq[4];
          int pp[4], qq[4];
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int k = k0 + b * nsplit;
            const bool on = k < m / 2;
            sv[b] = on ? sn[k] : 0.f;
            c[b] = on ? cs[k] : 1.f;
            pp[b] = on ? pq[k][0] : 0;
            qq[b] = on ? pq[k][1] : 0;
          }
#pragma unroll
          for (int b = 0; b < 4; ++b)
            if (sv[b] != 0.f) {
              ap[b] = G[pp[b] * KS + j];
              aq[b] = G[qq[b] * KS + j];
            }
#pragma unroll
          for (int b = 0; b < 4; ++b)
            if (sv[b] != 0.f) {
              G[pp[b] * KS + j] = c[b] * ap[b] - sv[b] * aq[b];
              G[qq[b] * KS + j] = sv[b] * ap[b] + c[b] * aq[b];
            }
        }
      }
      __syncthreads();
      // columns: A <- A J, V <- V J. Thread t owns row i = t mod K and the same pairs
      if (tid < nsplit * K) {
        const int i = tid - part * K;
        for (int k0 = part; k0 < m / 2; k0 += 4 * nsplit) {
          float c[4], sv[4], ap[4], aq[4], vp[4], vq[4];
          int pp[4], qq[4];
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int k = k0 + b * nsplit;
            const bool on = k < m / 2;
            sv[b] = on ? sn[k] : 0.f;
            c[b] = on ? cs[k] : 1.f;
            pp[b] = on ? pq[k][0] : 0;
            qq[b] = on ? pq[k][1] : 0;
          }
#pragma unroll
          for (int b = 0; b < 4; ++b)
            if (sv[b] != 0.f) {
              ap[b] = G[i * KS + pp[b]];
              aq[b] = G[i * KS + qq[b]];
              vp[b] = V[i * KS + pp[b]];
              vq[b] = V[i * KS + qq[b]];
            }
#pragma unroll
          for (int b = 0; b < 4; ++b)
            if (sv[b] != 0.f) {
              G[i * KS + pp[b]] = c[b] * ap[b] - sv[b] * aq[b];
              G[i * KS + qq[b]] = sv[b] * ap[b] + c[b] * aq[b];
              V[i * KS + pp[b]] = c[b] * vp[b] - sv[b] * vq[b];
              V[i * KS + qq[b]] = sv[b] * vp[b] + c[b] * vq[b];
            }
        }
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    atomicMax(&a.sc->max_sweeps, sweeps);
    if (sweeps == a.max_sweeps) atomicAdd(&a.sc->fallback_blocks, 1ull);  // not certified
  }
  __syncthreads();
  // ---- Newton-Schulz: M = V^T V (T3), V <- 1.5 V - 0.5 V M (via G)
  {
    float acc[8][8];
    mm_tile<true>(V, V, K, KS, ti, tj, acc);
#pragma unroll
    for (int x = 0; x < 8; ++x)
#pragma unroll
      for (int y = 0; y < 8; ++y)
        if (8 * ti + x < K && 8 * tj + y < K) T3[(8 * ti + x) * KS + 8 * tj + y] = acc[x][y];
    __syncthreads();
    mm_tile<false>(V, T3, K, KS, ti, tj, acc);
#pragma unroll
    for (int x = 0; x < 8; ++x)
#pragma unroll
      for (int y = 0; y < 8; ++y) {
        const int r = 8 * ti + x, c = 8 * tj + y;
        if (r < K && c < K) G[r * KS + c] = 1.5f * V[r * KS + c] - 0.5f * acc[x][y];
      }
  }
  __syncthreads();
  for (int e = tid; e < K * K; e += kNT) {
    const int r = e / K, c = e - r * K;
    V[r * KS + c] = G[r * KS + c];
    Vg[e] = G[r * KS + c];
  }
  // ---- Rayleigh quotients lambda_i = ||v_i^T Y'||^2 over the column chunks (fixed order)
  const int pi = tid >> 3, pc = tid & 7;  // 32 x 8 grid of 4 x 4 tiles over (i, column)
  float lacc[4] = {0.f, 0.f, 0.f, 0.f};   // kept by the pc == 0 thread of each row group
  for (int c0 = 0; c0 < ncol; c0 += kChunk) {
    __syncthreads();
    for (int e = tid; e < K * kChunk; e += kNT) {
      const int r = e / kChunk, cc = e - r * kChunk;
      T3[r * CS + cc] = Yb[(long long)r * ncol + c0 + cc];
    }
    __syncthreads();
    float acc[4][4];
    proj_tile(V, T3, K, KS, CS, pi, pc, acc);
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      float sq = 0.f;
#pragma unroll
      for (int y = 0; y < 4; ++y) sq = fmaf(acc[x][y], acc[x][y], sq);
      // the 8 threads of a row group are consecutive lanes: fixed-order butterfly sum
      sq += __shfl_xor(sq, 1);
      sq += __shfl_xor(sq, 2);
      sq += __shfl_xor(sq, 4);
      lacc[x] += sq;
    }
  }
  if (pc == 0) {
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      const int i = 4 * pi + x;
      if (i < K) lam[i] = lacc[x] > 1.f ? 1.f - 1.f / sqrtf(lacc[x]) : 0.f;  // f_i of the clip
    }
  }
  __syncthreads();
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
  // ---- Y+ = Y' - V_R diag(f) V_R^T Y', by column chunks (T3: Y' chunk, G: f V_R^T Y')
  for (int c0 = 0; c0 < ncol && R > 0; c0 += kChunk) {
    __syncthreads();
    for (int e = tid; e < K * kChunk; e += kNT) {
      const int r = e / kChunk, cc = e - r * kChunk;
      T3[r * CS + cc] = Yb[(long long)r * ncol + c0 + cc];
    }
    __syncthreads();
    // projections onto the clipped directions: P[n][cc] = f_i v_i^T y'_cc, i = ridx[n]
    for (int e = tid; e < R * (kChunk / 4); e += kNT) {
      const int n = e / (kChunk / 4), c4 = (e - n * (kChunk / 4)) * 4;
      const int i = ridx[n];
      float d0 = 0.f, d1 = 0.f, d2 = 0.f, d3 = 0.f;
      for (int r = 0; r < K; ++r) {
        const float vv = V[r * KS + i];
        d0 = fmaf(vv, T3[r * CS + c4], d0);
        d1 = fmaf(vv, T3[r * CS + c4 + 1], d1);
        d2 = fmaf(vv, T3[r * CS + c4 + 2], d2);
        d3 = fmaf(vv, T3[r * CS + c4 + 3], d3);
      }
      const float f = lam[i];
      G[n * CS + c4] = f * d0;
      G[n * CS + c4 + 1] = f * d1;
      G[n * CS + c4 + 2] = f * d2;
      G[n * CS + c4 + 3] = f * d3;
    }
    __syncthreads();
    // Y+[r][cc] = Y'[r][cc] - sum_n V[r][i_n] P[n][cc]; thread tile 4 rows x 4 columns
    {
      float acc[4][4];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = 0.f;
      for (int n = 0; n < R; ++n) {
        const int i = ridx[n];
        float av[4], bv[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          av[x] = 4 * pi + x < K ? V[(4 * pi + x) * KS + i] : 0.f;
          bv[x] = G[n * CS + 4 * pc + x];
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) acc[x][y] = fmaf(av[x], bv[y], acc[x][y]);
      }
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int r = 4 * pi + x;
        if (r < K) {
#pragma unroll
          for (int y = 0; y < 4; ++y) {
            const int cc = 4 * pc + y;
            Yb[(long long)r * ncol + c0 + cc] = T3[r * CS + cc] - acc[x][y];
          }
        }
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
    for (int ra = 0; ra < a.k1; ++ra)
      for (int rc = 0; rc < a.k2; ++rc) {
        const long long blk = (long long)wrapm(i - ra, a.n1) * a.n2 + wrapm(j - rc, a.n2);
        s += a.Y[(blk * K + ra * a.k2 + rc) * ncol + col];
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

size_t big_lds_bytes(int K) {
  const int KS = K + 1;
  const int GS = KS > kChunk + 1 ? KS : kChunk + 1;
  return (size_t)(2 * K * GS + K * KS) * sizeof(float);
}

hipError_t launch_big_block(const BigArgs &a, hipStream_t st) {
  static bool configured = false;
  if (!configured) {
    hipError_t e = hipFuncSetAttribute((const void *)k_big_block,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);
    if (e != hipSuccess) return e;
    configured = true;
  }
  hipLaunchKernelGGL(k_big_block, dim3((unsigned)a.nblk), dim3(kNT), big_lds_bytes(a.K), st, a);
  return hipGetLastError();
}

hipError_t launch_big_overlap(const BigArgs &a, float *Z, hipStream_t st) {
  long long g = ((long long)a.n1 * a.n2 * a.ncol + kNT * 4 - 1) / (kNT * 4);
  if (g > 65535) g = 65535;
  hipLaunchKernelGGL(k_big_overlap, dim3((unsigned)g), dim3(kNT), 0, st, a, Z);
  return hipGetLastError();
}

hipError_t launch_big_identity(float *V, long long nblk, int K, hipStream_t st) {
  long long g = (nblk * K * K + kNT * 4 - 1) / (kNT * 4);
  if (g > 65535) g = 65535;
  hipLaunchKernelGGL(k_big_identity, dim3((unsigned)g), dim3(kNT), 0, st, V, nblk, K);
  return hipGetLastError();
}

}  // namespace s3ttv
