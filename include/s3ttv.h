/*
 * s3ttv.h — C ABI of the MI355X (gfx950) S3TTV denoising/destriping solver.
 *
 * The solver computes Alg. 1 of Takemoto, Naganuma and Ono, "Spatio-Spectral Structure
 * Tensor Total Variation for Hyperspectral Image Denoising and Destriping" (arXiv
 * 2404.03313): preconditioned primal-dual splitting (P-PDS) for Prob. (18)
 *
 *     min_{u,s,t}  sum_l || P_l D D_s u ||_*
 *     s.t. ||s||_1 <= alpha,  ||t||_1 <= beta,  D_v t = 0,
 *          ||u + s + t - v||_2 <= eps,  mu_min <= u <= mu_max,
 *
 * with the block expansion P_l of Sec. III-A (eq. SSST, eq. rewrite_Lu), the proximity
 * operators of eqs. prox_box_constraint, prox_zeroset, prox_l2ball_constraint,
 * prox_nuclear_norm (the latter through the Moreau identity, eq. ProxConjugate) and an
 * exact l1-ball projection (Sec. III-C).
 *
 * Conventions used by every entry point
 *  - Cubes are float32, C-contiguous, shape (N1, N2, N3) = (rows i, columns j, bands b),
 *    band fastest: x[(i*N2 + j)*N3 + b]. D_v, D_h, D_s are periodic forward differences
 *    along i, j and b (Sec. II-A).
 *  - Blocks: one k1 x k2 window per pixel anchor (p, q) on the torus, L = N1*N2 blocks;
 *    block row r = a*k2 + c covers pixel ((p+a) mod N1, (q+c) mod N2). Supported K = k1*k2
 *    is 1..100: up to 16 rows the blocks are handled in registers and MFMA tiles (fused
 *    pass, warm-started MFMA eigen-solve); 17..100 rows (the paper's experiments use 10 x 10)
 *    take a one-workgroup-per-block path (FP32 Gram, warm-started parallel Jacobi with a
 *    certificate, low-rank clip, gathered overlap-add).
 *  - Array arguments named "device" must be device pointers (hipMalloc / torch CUDA
 *    tensors) on the current HIP device; "host" arguments are host memory. The caller owns
 *    every buffer; the library never allocates device memory and keeps no data between
 *    calls (it keeps HIP streams and events per calling thread and device, the raised LDS
 *    limit of its kernels per device, and the batched solve's tuned anchor tile per shape).
 *    Calls from several threads, on distinct workspaces, may run concurrently. Device
 *    arrays must be 16-byte aligned and must not alias unless stated.
 *  - stream is a hipStream_t passed as void* (NULL = default stream). Every call enqueues
 *    its work on that stream and returns after that work has completed.
 *  - Return codes: 0 success, S3TTV_NOT_CONVERGED (solve ran max_iter iterations without
 *    meeting rel_tol; outputs are valid), negative values are errors (outputs unspecified).
 */
#ifndef S3TTV_H
#define S3TTV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  S3TTV_OK = 0,
  S3TTV_NOT_CONVERGED = 1,
  S3TTV_EINVAL = -1,       /* bad shape, radius, box, step size, null pointer */
  S3TTV_EUNSUPPORTED = -2, /* valid for the method but not supported here (e.g. K > 100) */
  S3TTV_EWORKSPACE = -3,   /* workspace smaller than the queried size */
  S3TTV_EHIP = -4,         /* HIP runtime error */
  S3TTV_ENONFINITE = -5    /* NaN/Inf met in the input or in the iterates */
};

/* Image and block geometry. n1, n2, n3 >= 2; 1 <= k1 <= n1; 1 <= k2 <= n2; k1*k2 <= 100
 * (larger blocks: S3TTV_EUNSUPPORTED); n1*n2*n3 < 2^31; for k1*k2 > 16 also fewer than 2^32
 * entries in the block-column field, n1*n2 times 2 (3 for SSST) bands rounded up to 16
 * (32 for SSST). */
typedef struct {
  int32_t n1, n2, n3, k1, k2;
} s3ttv_shape;

/* Problem and iteration parameters.
 *  eps, alpha, beta: radii of the v-centred l2 ball (eq. constraint_fidel) and of the
 *    zero-centred l1 balls of s and t (eqs. constraint_sparse, constraint_stripe); > 0.
 *  mu_min < mu_max: box of u (eq. constraint_box); [0, 1] for normalised images.
 *  gamma_*: diagonal step sizes of Alg. 1 (eq. stepsize_denoising). If all six are 0 the
 *    Lemma-2 values of the stacked operator are used: gamma_u = 1/(8*k1*k2 + 1),
 *    gamma_s = 1, gamma_t = 1/3, gamma_Y = 1/4, gamma_y2 = 1/2, gamma_y3 = 1/3 (for the
 *    regulariser variants see `regularizer`).
 *  max_iter >= 1 iterations at most.
 *  rel_tol: 0 runs exactly max_iter iterations; > 0 stops after the first iteration
 *    k >= 2 with ||u^(k) - u^(k-1)|| / ||u^(k-1)|| < rel_tol (eq. StopCri_simulated).
 *  check_every: iterations between host checks of the stop flag (<= 0 means 16). The
 *    iterate returned is always the one at which the rule fired. s3ttv_solve replays a
 *    captured graph of that many iterations (rounded up to even, at most 256) on a stream of
 *    its own, joined to `stream` before and after; the result does not depend on it.
 *  timing_mask: bit c set => time every launch of kernel class c with HIP events and
 *    report the totals in s3ttv_stats (classes: see S3TTV_K_*). 0 for no timing; a solve
 *    with timing launches every kernel directly on `stream`.
 *  eig_max_steps: from the second iteration on, each block's 16 x 16 eigenproblem is solved
 *    by at most this many simultaneous rotation steps on MFMA, warm started from the previous
 *    iteration's eigenbasis; blocks not certified by then are finished by a per-lane cyclic
 *    Jacobi. 0 selects the default (24); a negative value sends every block not already
 *    certified by the warm start to the Jacobi. The result does not depend on it beyond
 *    rounding; it only moves work between the two solvers. At most 255.
 *  gram_precision: S3TTV_GRAM_FP32 (default), S3TTV_GRAM_BF16 or S3TTV_GRAM_FP16: input
 *    precision of the per-block Gram products Y' Y'^T on MFMA in the one-pass block kernel
 *    (blocks of at most 16 rows and at most 24 column tiles of 16: N3 <= 192, SSST N3 <= 128;
 *    other shapes always sum in FP32). Accumulation is
 *    FP32, followed by one FP32 refinement of the eigenvectors; the clip W Y' and every update
 *    stay FP32. The reduced modes round the Gram inputs to 8 or 11 significand bits for fewer
 *    MFMA instructions; see the error report of the tests.
 *  regularizer: the term minimised in place of S3TTV on the same P-PDS skeleton (Sec. IV-A
 *    compares methods this way): S3TTV_REG_S3TTV (default, Prob. (18)),
 *    S3TTV_REG_STV (sum_l ||P_l D u||_*, blocks of first-order differences),
 *    S3TTV_REG_SSTV (||D D_s u||_1), S3TTV_REG_HSSTV (||D D_s u||_1 + omega ||D u||_1) or
 *    S3TTV_REG_SSST (sum_l ||P_l [D_v u, D_h u, D_s u]||_*, blocks of first-order spatial and
 *    spectral differences: 3 N3 columns). For the l1 terms the dual of the regulariser is a
 *    field clipped to [-1, 1] each iteration (gamma_Y is its step; the HSSTV second field
 *    steps with 1/(2 omega)) and no block pass runs. Default steps (all gammas 0), by Lemma 2:
 *    gamma_u = 1/(8K+1), 1/(4K+1), 1/9, 1/(9 + 4 omega), 1/(6K+1); gamma_Y = 1/4, 1/2 (STV),
 *    1/4, 1/4, 1/2 (SSST); the other four as above. The workspace depends on the regulariser
 *    (s3ttv_workspace_bytes takes it from params; null params mean S3TTV).
 *  omega: HSSTV weight; 0 selects 0.05 (the value of the paper's comparison); finite, >= 0. */
typedef struct {
  double eps, alpha, beta;
  double mu_min, mu_max;
  double gamma_u, gamma_s, gamma_t, gamma_Y, gamma_y2, gamma_y3;
  int32_t max_iter;
  double rel_tol;
  int32_t check_every;
  int32_t timing_mask;
  int32_t eig_max_steps;
  int32_t gram_precision;
  int32_t regularizer;
  double omega;
} s3ttv_params;

enum { S3TTV_GRAM_FP32 = 0, S3TTV_GRAM_BF16 = 1, S3TTV_GRAM_FP16 = 2 };
enum {
  S3TTV_REG_S3TTV = 0,
  S3TTV_REG_STV = 1,
  S3TTV_REG_SSTV = 2,
  S3TTV_REG_HSSTV = 3,
  S3TTV_REG_SSST = 4
};

/* Kernel classes for timing_mask / s3ttv_stats.kernel_ms. */
enum {
  S3TTV_K_PRIMAL = 0, /* u, s, t primal step + first l1 histogram (Alg. 1 steps 2-4) */
  S3TTV_K_L1 = 1,     /* l1 threshold refinement passes and selections */
  S3TTV_K_GRAD = 2,   /* D_v D_s u', D_h D_s u' (steps 5, 9); in s3ttv_solve part of DUAL */
  S3TTV_K_GRAM = 3,   /* Y' = Y + gamma_Y P_l D D_s u', Gram Y' Y'^T on MFMA (step 9) */
  S3TTV_K_EIG = 4,    /* Jacobi eigen-solve, spectral clip matrix (step 10) */
  S3TTV_K_APPLY = 5,  /* Y+ = W Y' on MFMA, overlap-add partials (steps 10, 2) */
  S3TTV_K_ZSUM = 6,   /* sum of overlap-add partials (P_l^T of step 2), when the primal step
                         cannot read them itself */
  S3TTV_K_DUAL = 7,   /* s+, t+, y2, y3 updates (steps 3-7, 12-14) and the gradient field */
  S3TTV_K_FINAL = 8,  /* scalar reductions, stop rule */
  S3TTV_K_BLOCK = 9,  /* one pass over the dual blocks per iteration (N3 <= 192): steps 9-10
                         (Gram, eigen-solve, clip) and the overlap-add on MFMA */
  S3TTV_K_COUNT = 10
};

typedef struct {
  int32_t iters;        /* iterations run */
  int32_t converged;    /* 1 if rel_tol fired */
  double rel_change;    /* ||u^(k) - u^(k-1)|| / ||u^(k-1)|| of the last iteration */
  double l1_s, l1_t;    /* ||s||_1, ||t||_1 of the result */
  double fid;           /* ||u + s + t - v||_2 of the result */
  double dv_t;          /* ||D_v t||_2 of the result */
  int32_t eig_max_sweeps; /* largest per-lane Jacobi sweep count of any wavefront of blocks */
  float eig_avg_sweeps;   /* per-lane Jacobi sweeps per wavefront that ran them, averaged */
  float eig_avg_steps;    /* MFMA rotation steps per block, averaged over the iterations */
  int32_t eig_max_steps;  /* largest MFMA rotation step count of one block */
  int64_t eig_fallback_blocks; /* blocks the MFMA rotations could not certify, summed over
                                  the iterations, finished by the per-lane Jacobi (the first
                                  iteration starts the rotations from the identity basis) */
  /* For K = k1 k2 > 16 (one workgroup per block: simultaneous rotation steps on MFMA, then
     cyclic Jacobi sweeps, on the block Gram in the basis kept from the previous iteration):
     eig_avg_sweeps is the simultaneous rotation steps per block that needed the eigen-solve
     (blocks whose Gram passes the Gershgorin test skip it), eig_avg_steps the cyclic sweeps
     per such block, eig_max_sweeps the largest cyclic sweep count of a block,
     eig_fallback_blocks the blocks that used up the sweep limit without the certificate;
     eig_max_steps stays 0. */
  float ms;             /* wall time of the iteration loop (HIP events; batched: of the batch) */
  float kernel_ms[S3TTV_K_COUNT];     /* summed durations of timed classes */
  int32_t kernel_calls[S3TTV_K_COUNT];
  int32_t tile_a, tile_b; /* anchor tile of the block kernels (does not change the result) */
  int32_t status;         /* this problem's return code */
  int64_t eig_blocks;     /* K > 16: blocks that needed the eigen-solve, summed over the
                             iterations; K <= 16: blocks counted in eig_avg_steps */
} s3ttv_stats;

/* Bytes of device workspace s3ttv_solve needs for this shape (host out-pointer bytes). */
int32_t s3ttv_workspace_bytes(const s3ttv_shape *shape, const s3ttv_params *params,
                              size_t *bytes);

/* Solve Prob. (18) by Alg. 1 starting from u0 (device, nullable: zero start), all other
 * variables zero. v (device, input, not modified), u, s, t (device, outputs, N1*N2*N3
 * floats each), workspace (device, >= s3ttv_workspace_bytes), stats (host, nullable). */
int32_t s3ttv_solve(const s3ttv_shape *shape, const s3ttv_params *params, const float *v,
                    const float *u0, float *u, float *s, float *t, void *workspace,
                    size_t workspace_bytes, void *stream, s3ttv_stats *stats);

/* As s3ttv_solve, with optional starting values for the sparse and stripe components as well
 * (Alg. 1 leaves every initial value free): u0, s0, t0 are device cubes or null (zero start);
 * they are read once, checked for NaN/Inf (ENONFINITE) and may alias nothing the call
 * writes. The dual variables start at zero. */
int32_t s3ttv_solve_from(const s3ttv_shape *shape, const s3ttv_params *params, const float *v,
                         const float *u0, const float *s0, const float *t0, float *u, float *s,
                         float *t, void *workspace, size_t workspace_bytes, void *stream,
                         s3ttv_stats *stats);

/* Continues Alg. 1 from the iterate that an earlier s3ttv_solve, s3ttv_solve_from or
 * s3ttv_solve_continue call left in `workspace` (same shape, regulariser and workspace; the
 * same observation v must be passed). Runs at most params->max_iter more iterations with this
 * call's rel_tol, check_every, timing_mask, eig_max_steps and gram_precision (the step sizes
 * and radii should be those of the first call: P-PDS does not change them between iterations).
 * Iteration k of the continued run is iteration k of one uninterrupted solve: a solve of n1
 * iterations continued by n2 gives bitwise the result of a solve of n1 + n2 iterations. The
 * stop rule (eq. StopCri_simulated) is checked from the first continued iteration; stats
 * count the iterations and eigen-solves of this call only. Returns S3TTV_EINVAL when the
 * workspace holds no state of this problem (never solved, another shape or regulariser, a
 * batched solve's workspace) and S3TTV_ENONFINITE when the held state met a non-finite value.
 * v (device, input), u, s, t (device, outputs), workspace (device), stats (host, nullable). */
int32_t s3ttv_solve_continue(const s3ttv_shape *shape, const s3ttv_params *params, const float *v,
                             float *u, float *s, float *t, void *workspace,
                             size_t workspace_bytes, void *stream, s3ttv_stats *stats);

/* ---------------- Batched solve ---------------- */

/* Bytes of device workspace s3ttv_solve_batched needs for n problems of the given shapes
 * (params may be null). */
int32_t s3ttv_batch_workspace_bytes(int32_t n, const s3ttv_shape *shapes,
                                    const s3ttv_params *params, size_t *bytes);

/* Solves n independent instances of Prob. (18) by Alg. 1 (each with its own shape,
 * parameters, input v[i], optional start u0[i] and outputs u[i], s[i], t[i], all device
 * pointers as in s3ttv_solve; u0 may be null or hold null entries). Each result is identical
 * to s3ttv_solve on the same inputs: every problem stops by its own rule or max_iter. The
 * problems run concurrently: after the first iteration, 16-iteration spans of all problems
 * are captured once into a HIP graph and replayed; the anchor tile of each shape is chosen
 * by timing the block pass on the problem's workspace (cached per shape). workspace: device,
 * >= s3ttv_batch_workspace_bytes. stats: host array of n (nullable), with stats[i].status the
 * problem's own code. Returns S3TTV_OK, S3TTV_NOT_CONVERGED if some problem with rel_tol > 0
 * used up max_iter, or the first negative code. timing_mask is ignored. */
int32_t s3ttv_solve_batched(int32_t n, const s3ttv_shape *shapes, const s3ttv_params *params,
                            const float *const *v, const float *const *u0, float *const *u,
                            float *const *s, float *const *t, void *workspace,
                            size_t workspace_bytes, void *stream, s3ttv_stats *stats);

/* Static description of a return code. */
const char *s3ttv_strerror(int32_t code);

/* ---------------- Operator-level entry points (same kernels as the solver) ---------------- */

enum {
  S3TTV_OP_GRAD = 0,
  S3TTV_OP_GRAD_ADJ = 1,
  S3TTV_OP_CLIP = 2,
  S3TTV_OP_DUAL_BLOCKS = 3,
  S3TTV_OP_L1 = 4
};

/* Workspace bytes for an operator entry point. shape is used by GRAD, GRAD_ADJ and
 * DUAL_BLOCKS; n is the vector length for L1 and the block count for CLIP (with the block
 * geometry passed as k1 = K rows and n3 = ncols in shape for CLIP). */
int32_t s3ttv_op_workspace_bytes(int32_t op, const s3ttv_shape *shape, int64_t n, size_t *bytes);

/* Second-order spatio-spectral differences of Sec. II-A: gv = D_v D_s u, gh = D_h D_s u.
 * u, gv, gh device cubes. */
int32_t s3ttv_op_grad(const s3ttv_shape *shape, const float *u, float *gv, float *gh,
                      void *workspace, size_t workspace_bytes, void *stream);

/* Adjoint: w = D_s^T (D_v^T zv + D_h^T zh). zv, zh, w device cubes. */
int32_t s3ttv_op_grad_adj(const s3ttv_shape *shape, const float *zv, const float *zh, float *w,
                          void *workspace, size_t workspace_bytes, void *stream);

/* Projection of each of nblk matrices (K x ncols, row-major, K <= 100) onto the unit
 * spectral-norm ball, U diag(min(sigma, 1)) V^T — the value of Alg. 1 step 10 for any
 * gamma_Y by eq. ProxConjugate. yin, yout device arrays of nblk*K*ncols floats (they may
 * not overlap). K <= 16 runs the fused block kernels; larger K the one-workgroup-per-block
 * kernel, whose Jacobi eigen-solve starts from the identity here. K > 100: EUNSUPPORTED. */
int32_t s3ttv_op_spectral_clip(int32_t nblk, int32_t K, int32_t ncols, const float *yin,
                               float *yout, void *workspace, size_t workspace_bytes, void *stream);

/* Alg. 1 steps 9-10 for every block plus the overlap-add of step 2:
 *   Y+_l = Y_l + g P_l D D_s up - g prox_{(1/g) nuclear}((Y_l + g P_l D D_s up)/g),
 *   zv, zh = sum_l P_l^T Y+_l.
 * up (device cube), yin / yout (device, L x K x 2*N3, block column 2b = D_v part, 2b+1 = D_h
 * part, as eq. SSST), zv, zh device cubes. K = k1 k2 <= 16 runs the MFMA block kernels,
 * 17..100 the one-workgroup-per-block kernel with its eigen-solve started from the identity.
 * Returns S3TTV_ENONFINITE when a block holds NaN or Inf. */
int32_t s3ttv_op_dual_blocks(const s3ttv_shape *shape, double gamma_Y, const float *up,
                             const float *yin, float *yout, float *zv, float *zh,
                             void *workspace, size_t workspace_bytes, void *stream);

/* Projection of x (device, n floats) onto {||w||_1 <= radius}; out (device, n floats);
 * tau (host, nullable) receives the soft threshold (0 when x is inside the ball). */
int32_t s3ttv_op_l1_project(int64_t n, const float *x, double radius, float *out, double *tau,
                            void *workspace, size_t workspace_bytes, void *stream);

/* For callers that cannot allocate device memory (code under graph capture or in a serving
 * loop, harnesses that forbid hipMalloc): s3ttv_op_l1_project without a workspace argument.
 * Same kernels and result (bitwise) for n <= 2^24 elements; larger n: S3TTV_EUNSUPPORTED.
 * Its scratch (scalars and histograms, about 8.2 MiB) is a static device array of the
 * library, one per GPU, held until the process ends; the call allocates nothing. Calls of
 * one process on one device are serialised by the library (they share that array), so
 * overlapping calls from several threads run one after another. x, out (device, n floats),
 * tau (host, nullable). */
int32_t s3ttv_op_l1_project_noalloc(int64_t n, const float *x, double radius, float *out,
                                    double *tau, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* S3TTV_H */
