/*
 * FP64 CPU oracle for S3TTV denoising/destriping solved by P-PDS.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow, literal statement of what the
 * GPU library computes. It is compiled into its own shared library and is called only by
 * the test-suite, by the smoke check and by the benchmark's CPU-baseline leg. It shares
 * no code, header, table or helper with the GPU library.
 *
 * Paper: Takemoto, Naganuma, Ono, "Spatio-Spectral Structure Tensor Total Variation for
 * Hyperspectral Image Denoising and Destriping" (arXiv 2404.03313).
 *
 * Conventions (paper Sec. II-A): a cube x has N1 rows (index i, "vertical"), N2 columns
 * (index j, "horizontal") and N3 bands (index b); it is stored C-contiguous as
 * x[(i*N2 + j)*N3 + b]. D_v, D_h, D_s are periodic forward differences along i, j, b.
 *
 * Readings of the paper taken here (each is listed with its reason in the design notes):
 *  - D_v acts along i and D_h along j (the stripe constraint D_v t = 0 models vertical
 *    stripes, which are constant along i).
 *  - Blocks (Sec. III-A, eq. SSST / rewrite_Lu): one k1 x k2 window per pixel anchor
 *    (p, q), rows (p+a) mod N1, columns (q+c) mod N2, so L = N1*N2. Block row r = a*k2+c,
 *    block column 2b (D_v D_s u) and 2b+1 (D_h D_s u): the band-interleaved order of eq. SSST.
 *  - Alg. 1 dual updates use '+', all initial values are zero except an optional u0.
 *  - Default step sizes follow Lemma 2 applied to the stacked operator:
 *    gamma_u = 1/(8K+1) (K = k1*k2), gamma_s = 1, gamma_t = 1/3, gamma_Y = 1/4,
 *    gamma_y2 = 1/2, gamma_y3 = 1/3 (eq. stepsize_denoising prints 1/(8L+1) for gamma_u).
 *  - Stopping rule (eq. StopCri_simulated): ||u+ - u|| / ||u|| < tol, tested once at least
 *    two iterations are done and ||u|| > 0.
 *
 * Sums of many terms use long double accumulators; everything else is IEEE double with
 * no contraction and no reassociation.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define X3(i, j, b) ((((size_t)(i)) * (size_t)n2 + (size_t)(j)) * (size_t)n3 + (size_t)(b))

static int wrapi(int a, int n) {
  a %= n;
  return a < 0 ? a + n : a;
}

void ora_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int ora_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ---------------- Difference operators (Sec. II-A) ---------------- */

/* (D_v x)(i,j,b) = x(i+1,j,b) - x(i,j,b), periodic in i. */
void ora_dv(int n1, int n2, int n3, const double *x, double *y) {
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n2; ++j)
      for (int b = 0; b < n3; ++b) y[X3(i, j, b)] = x[X3((i + 1) % n1, j, b)] - x[X3(i, j, b)];
}

/* Adjoint: (D_v^T y)(i,j,b) = y(i-1,j,b) - y(i,j,b). */
void ora_dv_t(int n1, int n2, int n3, const double *x, double *y) {
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n2; ++j)
      for (int b = 0; b < n3; ++b) y[X3(i, j, b)] = x[X3(wrapi(i - 1, n1), j, b)] - x[X3(i, j, b)];
}

void ora_dh(int n1, int n2, int n3, const double *x, double *y) {
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n2; ++j)
      for (int b = 0; b < n3; ++b) y[X3(i, j, b)] = x[X3(i, (j + 1) % n2, b)] - x[X3(i, j, b)];
}

void ora_dh_t(int n1, int n2, int n3, const double *x, double *y) {
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n2; ++j)
      for (int b = 0; b < n3; ++b) y[X3(i, j, b)] = x[X3(i, wrapi(j - 1, n2), b)] - x[X3(i, j, b)];
}

void ora_ds(int n1, int n2, int n3, const double *x, double *y) {
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n2; ++j)
      for (int b = 0; b < n3; ++b) y[X3(i, j, b)] = x[X3(i, j, (b + 1) % n3)] - x[X3(i, j, b)];
}

void ora_ds_t(int n1, int n2, int n3, const double *x, double *y) {
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n2; ++j)
      for (int b = 0; b < n3; ++b) y[X3(i, j, b)] = x[X3(i, j, wrapi(b - 1, n3))] - x[X3(i, j, b)];
}

/* ---------------- Block expansion P_l (Sec. III-A, eq. SSST, rewrite_Lu) ---------------- */

/* T[l][r][2b+comp] = g_comp((p+a)%N1, (q+c)%N2, b), l = p*N2+q, r = a*k2+c.
   g_0 = gv, g_1 = gh. T has L*K*2*N3 entries, L = N1*N2, K = k1*k2. */
void ora_blocks_extract(int n1, int n2, int n3, int k1, int k2, const double *gv, const double *gh,
                        double *T) {
  const int K = k1 * k2;
  const size_t C = 2 * (size_t)n3;
#pragma omp parallel for schedule(static)
  for (int p = 0; p < n1; ++p)
    for (int q = 0; q < n2; ++q) {
      double *Tl = T + ((size_t)p * n2 + q) * K * C;
      for (int a = 0; a < k1; ++a)
        for (int c = 0; c < k2; ++c) {
          const int i = (p + a) % n1, j = (q + c) % n2, r = a * k2 + c;
          for (int b = 0; b < n3; ++b) {
            Tl[r * C + 2 * b] = gv[X3(i, j, b)];
            Tl[r * C + 2 * b + 1] = gh[X3(i, j, b)];
          }
        }
    }
}

/* Adjoint P^T: zv, zh = sum_l P_l^T Y_l (scatter with '+='). Parallel over bands so that each
   output entry is accumulated by one thread in a fixed order. */
void ora_blocks_scatter(int n1, int n2, int n3, int k1, int k2, const double *Y, double *zv,
                        double *zh) {
  const int K = k1 * k2;
  const size_t C = 2 * (size_t)n3;
  const size_t N = (size_t)n1 * n2 * n3;
  memset(zv, 0, N * sizeof(double));
  memset(zh, 0, N * sizeof(double));
#pragma omp parallel for schedule(static)
  for (int b = 0; b < n3; ++b)
    for (int p = 0; p < n1; ++p)
      for (int q = 0; q < n2; ++q) {
        const double *Yl = Y + ((size_t)p * n2 + q) * K * C;
        for (int a = 0; a < k1; ++a)
          for (int c = 0; c < k2; ++c) {
            const int i = (p + a) % n1, j = (q + c) % n2, r = a * k2 + c;
            zv[X3(i, j, b)] += Yl[r * C + 2 * b];
            zh[X3(i, j, b)] += Yl[r * C + 2 * b + 1];
          }
      }
}

/* Three-component blocks (the compared SSST regulariser): T[l][r][3b+comp] =
   g_comp((p+a)%N1, (q+c)%N2, b) with g_0 = gv, g_1 = gh, g_2 = gs; T has L*K*3*N3 entries. */
void ora_blocks_extract3(int n1, int n2, int n3, int k1, int k2, const double *gv,
                         const double *gh, const double *gs, double *T) {
  const int K = k1 * k2;
  const size_t C = 3 * (size_t)n3;
#pragma omp parallel for schedule(static)
  for (int p = 0; p < n1; ++p)
    for (int q = 0; q < n2; ++q) {
      double *Tl = T + ((size_t)p * n2 + q) * K * C;
      for (int a = 0; a < k1; ++a)
        for (int c = 0; c < k2; ++c) {
          const int i = (p + a) % n1, j = (q + c) % n2, r = a * k2 + c;
          for (int b = 0; b < n3; ++b) {
            Tl[r * C + 3 * b] = gv[X3(i, j, b)];
            Tl[r * C + 3 * b + 1] = gh[X3(i, j, b)];
            Tl[r * C + 3 * b + 2] = gs[X3(i, j, b)];
          }
        }
    }
}

/* Its adjoint: zv, zh, zs = sum_l P_l^T Y_l for three-component blocks. */
void ora_blocks_scatter3(int n1, int n2, int n3, int k1, int k2, const double *Y, double *zv,
                         double *zh, double *zs) {
  const int K = k1 * k2;
  const size_t C = 3 * (size_t)n3;
  const size_t N = (size_t)n1 * n2 * n3;
  memset(zv, 0, N * sizeof(double));
  memset(zh, 0, N * sizeof(double));
  memset(zs, 0, N * sizeof(double));
#pragma omp parallel for schedule(static)
  for (int b = 0; b < n3; ++b)
    for (int p = 0; p < n1; ++p)
      for (int q = 0; q < n2; ++q) {
        const double *Yl = Y + ((size_t)p * n2 + q) * K * C;
        for (int a = 0; a < k1; ++a)
          for (int c = 0; c < k2; ++c) {
            const int i = (p + a) % n1, j = (q + c) % n2, r = a * k2 + c;
            zv[X3(i, j, b)] += Yl[r * C + 3 * b];
            zh[X3(i, j, b)] += Yl[r * C + 3 * b + 1];
            zs[X3(i, j, b)] += Yl[r * C + 3 * b + 2];
          }
      }
}

/* Composite forward operator of eq. rewrite_Lu: T_l = P_l D D_s u for every l. */
void ora_struct_tensor(int n1, int n2, int n3, int k1, int k2, const double *u, double *T) {
  const size_t N = (size_t)n1 * n2 * n3;
  double *ds = (double *)malloc(N * sizeof(double));
  double *gv = (double *)malloc(N * sizeof(double));
  double *gh = (double *)malloc(N * sizeof(double));
  ora_ds(n1, n2, n3, u, ds);
  ora_dv(n1, n2, n3, ds, gv);
  ora_dh(n1, n2, n3, ds, gh);
  ora_blocks_extract(n1, n2, n3, k1, k2, gv, gh, T);
  free(ds);
  free(gv);
  free(gh);
}

/* Its adjoint: w = sum_l D_s^T D^T P_l^T Y_l = D_s^T (D_v^T zv + D_h^T zh). */
void ora_struct_tensor_adj(int n1, int n2, int n3, int k1, int k2, const double *Y, double *w) {
  const size_t N = (size_t)n1 * n2 * n3;
  double *zv = (double *)malloc(N * sizeof(double));
  double *zh = (double *)malloc(N * sizeof(double));
  double *a = (double *)malloc(N * sizeof(double));
  double *c = (double *)malloc(N * sizeof(double));
  ora_blocks_scatter(n1, n2, n3, k1, k2, Y, zv, zh);
  ora_dv_t(n1, n2, n3, zv, a);
  ora_dh_t(n1, n2, n3, zh, c);
  for (size_t e = 0; e < N; ++e) a[e] += c[e];
  ora_ds_t(n1, n2, n3, a, w);
  free(zv);
  free(zh);
  free(a);
  free(c);
}

/* ---------------- One-sided (Hestenes) Jacobi SVD, hand written ---------------- */

/* Orthogonalise the m rows of B (m x n, row-major) by plane rotations applied from the left,
   accumulating U (m x m) so that the input equals U * B at every step. Stops when every pair
   satisfies |b_p . b_q| <= tol * ||b_p|| ||b_q||. Returns sweeps used, or -1. */
static int jacobi_rows(int m, int n, double *B, double *U, double tol, int max_sweeps) {
  for (int a = 0; a < m; ++a)
    for (int c = 0; c < m; ++c) U[a * m + c] = (a == c) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    int rotated = 0;
    for (int p = 0; p < m - 1; ++p)
      for (int q = p + 1; q < m; ++q) {
        double *bp = B + (size_t)p * n, *bq = B + (size_t)q * n;
        long double al = 0, be = 0, ga = 0;
        for (int k = 0; k < n; ++k) {
          al += (long double)bp[k] * bp[k];
          be += (long double)bq[k] * bq[k];
          ga += (long double)bp[k] * bq[k];
        }
        const double alpha = (double)al, beta = (double)be, gamma = (double)ga;
        if (gamma == 0.0 || fabs(gamma) <= tol * sqrt(alpha) * sqrt(beta)) continue;
        rotated = 1;
        const double zeta = (beta - alpha) / (2.0 * gamma);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
        for (int k = 0; k < n; ++k) {
          const double x = bp[k], y = bq[k];
          bp[k] = cs * x - sn * y;
          bq[k] = sn * x + cs * y;
        }
        for (int k = 0; k < m; ++k) {
          const double x = U[k * m + p], y = U[k * m + q];
          U[k * m + p] = cs * x - sn * y;
          U[k * m + q] = sn * x + cs * y;
        }
      }
    if (!rotated) return sweep + 1;
  }
  return -1;
}

#define ORA_SVD_TOL 1e-14
#define ORA_SVD_SWEEPS 60

/* Full SVD of A (m x n) with m <= n: A = U diag(sig) Vt, U m x m, Vt m x n (rows orthonormal
   where sig > 0, zero rows where sig == 0). Returns sweeps or -1. */
int ora_svd_rows(int m, int n, const double *A, double *sig, double *U, double *Vt) {
  memcpy(Vt, A, (size_t)m * n * sizeof(double));
  const int sw = jacobi_rows(m, n, Vt, U, ORA_SVD_TOL, ORA_SVD_SWEEPS);
  for (int a = 0; a < m; ++a) {
    long double s2 = 0;
    for (int k = 0; k < n; ++k) s2 += (long double)Vt[(size_t)a * n + k] * Vt[(size_t)a * n + k];
    sig[a] = sqrt((double)s2);
    for (int k = 0; k < n; ++k) Vt[(size_t)a * n + k] = sig[a] > 0 ? Vt[(size_t)a * n + k] / sig[a] : 0.0;
  }
  return sw;
}

/* Nuclear-norm prox (eq. prox_nuclear_norm): U diag(max(sig - lam, 0)) V^T.
   Works on whichever side is shorter; the prox commutes with transposition. */
int ora_prox_nuclear(int m, int n, double lam, const double *A, double *out) {
  const int tr = m > n;
  const int r = tr ? n : m, c = tr ? m : n;
  double *B = (double *)malloc((size_t)r * c * sizeof(double));
  double *U = (double *)malloc((size_t)r * r * sizeof(double));
  double *sig = (double *)malloc((size_t)r * sizeof(double));
  double *Vt = (double *)malloc((size_t)r * c * sizeof(double));
  if (tr) {
    for (int a = 0; a < m; ++a)
      for (int k = 0; k < n; ++k) B[(size_t)k * m + a] = A[(size_t)a * n + k];
  } else {
    memcpy(B, A, (size_t)m * n * sizeof(double));
  }
  const int sw = ora_svd_rows(r, c, B, sig, U, Vt);
  /* R = U * diag(max(sig - lam, 0)) * Vt   (r x c) */
  for (int a = 0; a < r; ++a)
    for (int k = 0; k < c; ++k) {
      long double acc = 0;
      for (int e = 0; e < r; ++e) {
        const double d = sig[e] - lam;
        if (d > 0) acc += (long double)U[a * r + e] * d * Vt[(size_t)e * c + k];
      }
      B[(size_t)a * c + k] = (double)acc;
    }
  if (tr) {
    for (int a = 0; a < m; ++a)
      for (int k = 0; k < n; ++k) out[(size_t)a * n + k] = B[(size_t)k * m + a];
  } else {
    memcpy(out, B, (size_t)m * n * sizeof(double));
  }
  free(B);
  free(U);
  free(sig);
  free(Vt);
  return sw;
}

/* Dual nuclear step of Alg. 1 (steps 9-10) through the Moreau identity (eq. ProxConjugate):
   out = Yp - g * prox_{(1/g)||.||_*}(Yp / g). */
int ora_dual_nuclear(int m, int n, double g, const double *Yp, double *out) {
  const size_t mn = (size_t)m * n;
  double *X = (double *)malloc(mn * sizeof(double));
  for (size_t e = 0; e < mn; ++e) X[e] = Yp[e] / g;
  const int sw = ora_prox_nuclear(m, n, 1.0 / g, X, out);
  for (size_t e = 0; e < mn; ++e) out[e] = Yp[e] - g * out[e];
  free(X);
  return sw;
}

/* ---------------- Projections (eqs. prox_box_constraint, prox_l2ball_constraint; l1 ball) --- */

void ora_proj_box(int64_t n, const double *x, double lo, double hi, double *out) {
  for (int64_t e = 0; e < n; ++e) out[e] = x[e] < lo ? lo : (x[e] > hi ? hi : x[e]);
}

/* v-centred l2 ball of radius eps. */
void ora_proj_l2(int64_t n, const double *x, const double *v, double eps, double *out) {
  long double s = 0;
  for (int64_t e = 0; e < n; ++e) s += (long double)(x[e] - v[e]) * (x[e] - v[e]);
  const double d = sqrt((double)s);
  if (d <= eps) {
    memcpy(out, x, (size_t)n * sizeof(double));
    return;
  }
  for (int64_t e = 0; e < n; ++e) out[e] = v[e] + eps * (x[e] - v[e]) / d;
}

static int cmp_desc(const void *pa, const void *pb) {
  const double a = *(const double *)pa, b = *(const double *)pb;
  return (a < b) - (a > b);
}

/* Zero-centred l1 ball of radius alpha, by sorting magnitudes (the exact projection the paper
   obtains with a fast l1-ball algorithm, Sec. III-C). Returns the threshold tau (0 if x is
   already inside the ball). */
double ora_proj_l1(int64_t n, const double *x, double alpha, double *out) {
  long double tot = 0;
  for (int64_t e = 0; e < n; ++e) tot += fabs(x[e]);
  if ((double)tot <= alpha) {
    memcpy(out, x, (size_t)n * sizeof(double));
    return 0.0;
  }
  double *mu = (double *)malloc((size_t)n * sizeof(double));
  for (int64_t e = 0; e < n; ++e) mu[e] = fabs(x[e]);
  qsort(mu, (size_t)n, sizeof(double), cmp_desc);
  long double cum = 0;
  double tau = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    cum += mu[j];
    const double cand = (double)((cum - (long double)alpha) / (long double)(j + 1));
    if (mu[j] - cand > 0) tau = cand;
  }
  free(mu);
  for (int64_t e = 0; e < n; ++e) {
    const double a = fabs(x[e]) - tau;
    out[e] = a > 0 ? (x[e] > 0 ? a : -a) : 0.0;
  }
  return tau;
}

/* ---------------- S3TTV value (eq. S3TTV_Lu) ---------------- */

double ora_s3ttv(int n1, int n2, int n3, int k1, int k2, const double *u) {
  const int K = k1 * k2;
  const int C = 2 * n3;
  const size_t L = (size_t)n1 * n2;
  double *T = (double *)malloc(L * K * C * sizeof(double));
  ora_struct_tensor(n1, n2, n3, k1, k2, u, T);
  const int r = K < C ? K : C, c = K < C ? C : K;
  double *vals = (double *)malloc(L * sizeof(double));
#pragma omp parallel
  {
    double *B = (double *)malloc((size_t)r * c * sizeof(double));
    double *U = (double *)malloc((size_t)r * r * sizeof(double));
    double *sig = (double *)malloc((size_t)r * sizeof(double));
    double *Vt = (double *)malloc((size_t)r * c * sizeof(double));
#pragma omp for schedule(static)
    for (size_t l = 0; l < L; ++l) {
      const double *Tl = T + l * K * C;
      if (K <= C) {
        memcpy(B, Tl, (size_t)K * C * sizeof(double));
      } else {
        for (int a = 0; a < K; ++a)
          for (int k = 0; k < C; ++k) B[(size_t)k * K + a] = Tl[(size_t)a * C + k];
      }
      ora_svd_rows(r, c, B, sig, U, Vt);
      double s = 0;
      for (int e = 0; e < r; ++e) s += sig[e];
      vals[l] = s;
    }
    free(B);
    free(U);
    free(sig);
    free(Vt);
  }
  long double tot = 0;
  for (size_t l = 0; l < L; ++l) tot += vals[l];
  free(vals);
  free(T);
  return (double)tot;
}

/* ---------------- Alg. 1: P-PDS solver for Prob. (18) ---------------- */

/* Regularisers on the P-PDS skeleton of Alg. 1 (Sec. IV-A replaces the S3TTV term of
   Prob. (18) by those of the compared P-PDS-applicable methods and solves each by P-PDS):
     0 S3TTV: sum_l ||P_l D D_s u||_*          (dual: blocks Y_l, step 10 = spectral clip)
     1 STV:   sum_l ||P_l D u||_*              (blocks of first-order spatial differences)
     2 SSTV:  ||D D_s u||_1                    (dual: field Z, step = clip to [-1, 1])
     3 HSSTV: ||D D_s u||_1 + omega ||D u||_1  (two fields, the second with step 1/(2 omega))
     4 SSST:  sum_l ||P_l [D_v u, D_h u, D_s u]||_*  (blocks of first-order spatial and
              spectral differences, three columns per band) */
enum { REG_S3TTV = 0, REG_STV = 1, REG_SSTV = 2, REG_HSSTV = 3, REG_SSST = 4 };

/* gv, gh = D_v x, D_h x, after D_s when spectral != 0. tmp: N scratch doubles. */
static void grad_pair(int n1, int n2, int n3, int spectral, const double *x, double *gv,
                      double *gh, double *tmp) {
  const double *src = x;
  if (spectral) {
    ora_ds(n1, n2, n3, x, tmp);
    src = tmp;
  }
  ora_dv(n1, n2, n3, src, gv);
  ora_dh(n1, n2, n3, src, gh);
}

/* out = D_v^T zv + D_h^T zh, then D_s^T of it when spectral != 0. a, c: N scratch doubles. */
static void grad_pair_adj(int n1, int n2, int n3, int spectral, const double *zv, const double *zh,
                          double *out, double *a, double *c) {
  const size_t N = (size_t)n1 * n2 * n3;
  ora_dv_t(n1, n2, n3, zv, a);
  ora_dh_t(n1, n2, n3, zh, c);
  for (size_t e = 0; e < N; ++e) a[e] += c[e];
  if (spectral) ora_ds_t(n1, n2, n3, a, out);
  else memcpy(out, a, N * sizeof(double));
}

/* prm: [0] eps [1] alpha [2] beta [3] mu_min [4] mu_max
        [5] gamma_u [6] gamma_s [7] gamma_t [8] gamma_Y [9] gamma_y2 [10] gamma_y3 [11] rel_tol
        [12] regulariser (REG_*) [13] omega (HSSTV weight, > 0 for REG_HSSTV)
   Step sizes that are all zero select the Lemma-2 defaults of the regulariser's stacked
   operator: gamma_u = 1/(8K+1) (S3TTV), 1/(4K+1) (STV), 1/9 (SSTV), 1/(9 + 4 omega) (HSSTV),
   1/(6K+1) (SSST); gamma_Y (the step of the regulariser's dual) = 1/4, except 1/2 for STV and
   SSST; gamma_s = 1,
   gamma_t = 1/3, gamma_y2 = 1/2, gamma_y3 = 1/3. The HSSTV second field always steps with
   1/(2 omega).
   Initial values (Alg. 1 leaves them free): u0, s0, t0 (nullable: zero); all duals start at
   zero.
   dims: [0] N1 [1] N2 [2] N3 [3] k1 [4] k2 (blocks; unused by SSTV and HSSTV).
   stats (out, 8 doubles): [0] iterations run [1] last relative change [2] converged flag
        [3] ||D_v t|| [4] ||u+s+t-v|| - eps [5] ||s||_1 - alpha [6] ||t||_1 - beta
        [7] worst SVD sweep count (-1 if some block did not converge).
   trace (nullable, max_iter doubles): relative change after each iteration.
   Y_out (S3TTV, STV, SSST), z_out (SSTV, HSSTV: 4N doubles z1v, z1h, z2v, z2h), y2_out, y3_out
   (nullable): final dual variables (Y in the T layout).
   Returns 0, or -1 for invalid arguments. */
int ora_solve(const int *dims, const double *prm, int max_iter, const double *v, const double *u0,
              const double *s0, const double *t0, double *u, double *s, double *t,
              double *stats, double *trace, double *Y_out, double *z_out, double *y2_out,
              double *y3_out) {
  const int n1 = dims[0], n2 = dims[1], n3 = dims[2], k1 = dims[3], k2 = dims[4];
  if (n1 < 2 || n2 < 2 || n3 < 2 || k1 < 1 || k2 < 1 || k1 > n1 || k2 > n2 || max_iter < 1)
    return -1;
  const double eps = prm[0], alpha = prm[1], beta = prm[2], lo = prm[3], hi = prm[4];
  double g_u = prm[5], g_s = prm[6], g_t = prm[7], g_Y = prm[8], g_y2 = prm[9], g_y3 = prm[10];
  const double tol = prm[11];
  const int reg = (int)prm[12];
  const double omega = prm[13];
  if (reg < REG_S3TTV || reg > REG_SSST) return -1;
  if (reg == REG_HSSTV && !(omega > 0)) return -1;
  const int blocks = reg == REG_S3TTV || reg == REG_STV || reg == REG_SSST;
  const int spectral = reg != REG_STV && reg != REG_SSST;
  const int K = k1 * k2, C = (reg == REG_SSST ? 3 : 2) * n3;
  if (g_u == 0 && g_s == 0 && g_t == 0 && g_Y == 0 && g_y2 == 0 && g_y3 == 0) {
    g_u = reg == REG_S3TTV ? 1.0 / (8.0 * K + 1.0)
          : reg == REG_STV ? 1.0 / (4.0 * K + 1.0)
          : reg == REG_SSST ? 1.0 / (6.0 * K + 1.0)
          : reg == REG_SSTV ? 1.0 / 9.0
                            : 1.0 / (9.0 + 4.0 * omega);
    g_s = 1.0;
    g_t = 1.0 / 3.0;
    g_Y = (reg == REG_STV || reg == REG_SSST) ? 0.5 : 0.25;
    g_y2 = 0.5;
    g_y3 = 1.0 / 3.0;
  }
  const double g_Z2 = reg == REG_HSSTV ? 1.0 / (2.0 * omega) : 0.0;
  if (!(eps > 0 && alpha > 0 && beta > 0 && lo < hi && g_u > 0 && g_s > 0 && g_t > 0 && g_Y > 0 &&
        g_y2 > 0 && g_y3 > 0))
    return -1;
  const size_t N = (size_t)n1 * n2 * n3, L = (size_t)n1 * n2, BL = (size_t)K * C;

  double *Y = blocks ? (double *)calloc(L * BL, sizeof(double)) : NULL;
  double *T = blocks ? (double *)malloc(L * BL * sizeof(double)) : NULL;
  double *Z = !blocks ? (double *)calloc(4 * N, sizeof(double)) : NULL;  /* z1v z1h z2v z2h */
  double *y2 = (double *)calloc(N, sizeof(double));
  double *y3 = (double *)calloc(N, sizeof(double));
  double *un = (double *)malloc(N * sizeof(double));
  double *sn = (double *)malloc(N * sizeof(double));
  double *tn = (double *)malloc(N * sizeof(double));
  double *w = (double *)malloc(N * sizeof(double));
  double *tmp = (double *)malloc(N * sizeof(double));
  double *up = (double *)malloc(N * sizeof(double));
  double *gv = (double *)malloc(N * sizeof(double));
  double *gh = (double *)malloc(N * sizeof(double));
  double *s1 = (double *)malloc(N * sizeof(double));
  double *s2 = (double *)malloc(N * sizeof(double));
  double *gs = reg == REG_SSST ? (double *)malloc(N * sizeof(double)) : NULL;

  for (size_t e = 0; e < N; ++e) {
    u[e] = u0 ? u0[e] : 0.0;
    s[e] = s0 ? s0[e] : 0.0;
    t[e] = t0 ? t0[e] : 0.0;
  }
  int it = 0, converged = 0, worst_sweeps = 0;
  double rel = 0.0;
  for (it = 0; it < max_iter;) {
    /* Step 2: u+ = P_box(u - g_u (A^T(dual of the regulariser) + y3)); for S3TTV
       A^T Y = sum_l D_s^T D^T P_l^T Y_l. */
    if (reg == REG_S3TTV) {
      ora_struct_tensor_adj(n1, n2, n3, k1, k2, Y, w);
    } else if (reg == REG_STV) {
      ora_blocks_scatter(n1, n2, n3, k1, k2, Y, gv, gh);
      grad_pair_adj(n1, n2, n3, 0, gv, gh, w, s1, s2);
    } else if (reg == REG_SSST) {
      /* w = D_v^T zv + D_h^T zh + D_s^T zs */
      ora_blocks_scatter3(n1, n2, n3, k1, k2, Y, gv, gh, gs);
      grad_pair_adj(n1, n2, n3, 0, gv, gh, w, s1, s2);
      ora_ds_t(n1, n2, n3, gs, s1);
      for (size_t e = 0; e < N; ++e) w[e] += s1[e];
    } else {
      grad_pair_adj(n1, n2, n3, 1, Z, Z + N, w, s1, s2);
      if (reg == REG_HSSTV) {
        grad_pair_adj(n1, n2, n3, 0, Z + 2 * N, Z + 3 * N, gv, s1, s2);
        for (size_t e = 0; e < N; ++e) w[e] += omega * gv[e];
      }
    }
    for (size_t e = 0; e < N; ++e) tmp[e] = u[e] - g_u * (w[e] + y3[e]);
    ora_proj_box((int64_t)N, tmp, lo, hi, un);
    /* Step 3: s+ = P_{B1,alpha}(s - g_s y3). */
    for (size_t e = 0; e < N; ++e) tmp[e] = s[e] - g_s * y3[e];
    ora_proj_l1((int64_t)N, tmp, alpha, sn);
    /* Step 4: t+ = P_{B1,beta}(t - g_t (D_v^T y2 + y3)). */
    ora_dv_t(n1, n2, n3, y2, w);
    for (size_t e = 0; e < N; ++e) tmp[e] = t[e] - g_t * (w[e] + y3[e]);
    ora_proj_l1((int64_t)N, tmp, beta, tn);
    /* Steps 5-7: extrapolation (u' kept in up; s', t' formed where used). */
    for (size_t e = 0; e < N; ++e) up[e] = 2.0 * un[e] - u[e];
    /* Steps 8-11 for the regulariser's dual: Y'_l = Y_l + g_Y A_l u',
       Y_l = Y'_l - g_Y prox_{(1/g_Y) R}(Y'_l / g_Y): a spectral clip of each block for the
       nuclear norms, a clip of each entry to [-1, 1] for the l1 norms. */
    if (blocks) {
      grad_pair(n1, n2, n3, spectral, up, gv, gh, s1);
      if (reg == REG_SSST) {
        ora_ds(n1, n2, n3, up, gs);
        ora_blocks_extract3(n1, n2, n3, k1, k2, gv, gh, gs, T);
      } else {
        ora_blocks_extract(n1, n2, n3, k1, k2, gv, gh, T);
      }
      int sweeps_max = 0, failed = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(max : sweeps_max) reduction(| : failed)
      for (size_t l = 0; l < L; ++l) {
        double *Yl = Y + l * BL;
        const double *Tl = T + l * BL;
        double *Yp = (double *)malloc(BL * sizeof(double));
        for (size_t e = 0; e < BL; ++e) Yp[e] = Yl[e] + g_Y * Tl[e];
        const int sw = ora_dual_nuclear(K, C, g_Y, Yp, Yl);
        if (sw < 0) failed = 1;
        if (sw > sweeps_max) sweeps_max = sw;
        free(Yp);
      }
      if (failed) worst_sweeps = -1;
      else if (worst_sweeps >= 0 && sweeps_max > worst_sweeps) worst_sweeps = sweeps_max;
    } else {
      grad_pair(n1, n2, n3, 1, up, gv, gh, s1);
      for (size_t e = 0; e < N; ++e) {
        Z[e] = fmin(1.0, fmax(-1.0, Z[e] + g_Y * gv[e]));
        Z[N + e] = fmin(1.0, fmax(-1.0, Z[N + e] + g_Y * gh[e]));
      }
      if (reg == REG_HSSTV) {
        grad_pair(n1, n2, n3, 0, up, gv, gh, s1);
        for (size_t e = 0; e < N; ++e) {
          Z[2 * N + e] = fmin(1.0, fmax(-1.0, Z[2 * N + e] + g_Z2 * omega * gv[e]));
          Z[3 * N + e] = fmin(1.0, fmax(-1.0, Z[3 * N + e] + g_Z2 * omega * gh[e]));
        }
      }
    }
    /* Step 12: y2 = y2 + g_y2 D_v t'. */
    for (size_t e = 0; e < N; ++e) tmp[e] = 2.0 * tn[e] - t[e];
    ora_dv(n1, n2, n3, tmp, w);
    for (size_t e = 0; e < N; ++e) y2[e] += g_y2 * w[e];
    /* Steps 13-14: y3' = y3 + g_y3 (u' + s' + t');  y3 = y3' - g_y3 P_{B2,eps}^v(y3'/g_y3). */
    for (size_t e = 0; e < N; ++e)
      y3[e] = y3[e] + g_y3 * (up[e] + (2.0 * sn[e] - s[e]) + (2.0 * tn[e] - t[e]));
    for (size_t e = 0; e < N; ++e) tmp[e] = y3[e] / g_y3;
    ora_proj_l2((int64_t)N, tmp, v, eps, w);
    for (size_t e = 0; e < N; ++e) y3[e] = y3[e] - g_y3 * w[e];
    /* Stopping rule (eq. StopCri_simulated), relative to the previous u. */
    long double dn = 0, un2 = 0;
    for (size_t e = 0; e < N; ++e) {
      dn += (long double)(un[e] - u[e]) * (un[e] - u[e]);
      un2 += (long double)u[e] * u[e];
    }
    rel = un2 > 0 ? sqrt((double)dn) / sqrt((double)un2) : INFINITY;
    memcpy(u, un, N * sizeof(double));
    memcpy(s, sn, N * sizeof(double));
    memcpy(t, tn, N * sizeof(double));
    if (trace) trace[it] = rel;
    ++it;
    if (tol > 0 && it >= 2 && un2 > 0 && rel < tol) {
      converged = 1;
      break;
    }
  }
  /* Diagnostics of the final iterate. */
  ora_dv(n1, n2, n3, t, w);
  long double a = 0, f = 0, l1s = 0, l1t = 0;
  for (size_t e = 0; e < N; ++e) {
    a += (long double)w[e] * w[e];
    const double r = u[e] + s[e] + t[e] - v[e];
    f += (long double)r * r;
    l1s += fabs(s[e]);
    l1t += fabs(t[e]);
  }
  stats[0] = it;
  stats[1] = rel;
  stats[2] = converged;
  stats[3] = sqrt((double)a);
  stats[4] = sqrt((double)f) - eps;
  stats[5] = (double)l1s - alpha;
  stats[6] = (double)l1t - beta;
  stats[7] = worst_sweeps;
  if (Y_out && Y) memcpy(Y_out, Y, L * BL * sizeof(double));
  if (z_out && Z) memcpy(z_out, Z, 4 * N * sizeof(double));
  if (y2_out) memcpy(y2_out, y2, N * sizeof(double));
  if (y3_out) memcpy(y3_out, y3, N * sizeof(double));
  free(Y);
  free(T);
  free(Z);
  free(y2);
  free(y3);
  free(un);
  free(sn);
  free(tn);
  free(w);
  free(tmp);
  free(up);
  free(gv);
  free(gh);
  free(s1);
  free(s2);
  free(gs);
  return 0;
}
