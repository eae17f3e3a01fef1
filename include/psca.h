/*
 * psca.h — C ABI of the MI355X (gfx950) PSCA device-activity-detection library.
 *
 * The library computes the per-iteration hot path of the PSCA algorithms of
 * Tan & Cui, "Fast MLE and MAPE-Based Device Activity Detection for
 * Grant-Free Access via PSCA and PSCA-Net" (arXiv 2503.15259), Algorithm 1,
 * for the four estimators of Sec. III and IV:
 *   PSCA_ML_K   MLE of the activity alpha in [0,1]^N, known pathloss g (Sec. III-A)
 *   PSCA_MAP_K  MAPE of alpha with the independent Bernoulli prior (Sec. III-B)
 *   PSCA_ML_UD  MLE of the effective pathloss gamma >= 0, unknown g (Sec. IV-A)
 *   PSCA_MAP_UR MAPE of gamma with the Hermite-smoothed prior p^eps (Sec. IV-B)
 *   PSCA_MAP_K2 MAPE of alpha, known pathloss, under the second-order activity
 *               model (eq. second; Sec. III-B with t = G restricted to sets of
 *               one or two devices)
 *
 * Conventions shared by every entry point:
 *   - Complex numbers are interleaved single precision (psca_c32, the layout
 *     of std::complex<float> / torch.complex64).
 *   - Matrices are column-major.  S is L x N with column n the pilot s_n
 *     (L contiguous elements); Y is L x M; SigmaHat is L x L.
 *   - All array arguments are DEVICE pointers on the context's GPU, owned by
 *     the caller; the library never frees or retains them past the call's
 *     stream work.  Host pointers are named *_host.
 *   - Every call is asynchronous on `stream` (a hipStream_t, NULL = the
 *     default stream).  Outputs are valid once that stream's prior work is done.
 *   - Return value: PSCA_OK (0) or a negative psca_status.  Argument errors are
 *     detected on the host before any launch (PSCA_EINVAL, nothing written).
 *     Numerical failure found on the device (a Cholesky pivot <= 0 or not
 *     finite) is written to the optional device word `status` (PSCA_ENOTPD);
 *     the iterate stops advancing at the last finite value.  PSCA_ESYNC in
 *     `status` means the persistent kernel's device-wide barrier gave up
 *     waiting (bounded wait; the kernel still exits) and x_out is not valid.
 *   - Work buffers live in the context (grown on demand with hipMalloc);
 *     calls on one context must not overlap in time (use one context per
 *     concurrent stream).
 */
#ifndef PSCA_H
#define PSCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { float re, im; } psca_c32;

typedef enum {
  PSCA_ML_K = 0,
  PSCA_MAP_K = 1,
  PSCA_ML_UD = 2,
  PSCA_MAP_UR = 3,
  PSCA_MAP_K2 = 4
} psca_variant;

typedef enum {
  PSCA_OK = 0,
  PSCA_EINVAL = -1,   /* bad argument (host-side validation, nothing launched) */
  PSCA_ENOTPD = -2,   /* Sigma not numerically positive definite (device) */
  PSCA_EHIP = -3,     /* a HIP runtime call failed */
  PSCA_ENOMEM = -4,   /* device allocation failed */
  PSCA_ENOTSUP = -5,  /* size outside what the library supports (e.g. L > PSCA_MAX_L) */
  PSCA_ESYNC = -6     /* a device-wide barrier timed out (device status word only) */
} psca_status;

/* Largest pilot length L.  Up to 96 the L x L work matrix lives in each
 * workgroup's LDS; from 97 to 256 Sigma is factored in device memory
 * cooperatively by the instance's team of workgroups.  Every entry point
 * takes 1 <= L <= 256, with two exceptions: a batch (psca_detect_batch, its
 * plans, psca_layer_backward_batch) must lie wholly on one side of the
 * boundary of its kernel family (L <= 96 or L > 96 for detections, L <= 64
 * or L > 64 for the layer backward), else PSCA_ENOTSUP; and
 * psca_detect_noalloc takes L <= 96. */
#define PSCA_MAX_L 256

/*
 * Parameters of one detection (Algorithm 1 inputs besides SigmaHat and S).
 *   variant    psca_variant.
 *   iters      number of iterations k = 0 .. iters-1 (>= 0); the paper leaves
 *              the stopping rule open, this library runs a fixed count.
 *   rho0, rho_decay   step sizes rho_0 = rho0, rho_{k+1} = rho_k (1 - rho_decay rho_k)
 *              (Sec. V uses 0.5 and 0.5).  rho0 in (0, 1], rho_decay in [0, 2].
 *   rho        optional DEVICE array of `iters` step sizes in [0, 1] that
 *              replaces the schedule (the unrolled network's learned steps); NULL
 *              for the schedule.
 *   sigma2     noise power sigma^2 > 0 (eq. cov_a / cov_b).
 *   M          number of BS antennas >= 1 (scales the MAP prior terms by 1/M).
 *   g          DEVICE [N] known pathloss, > 0; required by ML-K and MAP-K.
 *   p          DEVICE [N] activity probabilities in (0, 1); required by MAP-K.
 *   d_lo, d_hi, pl_c0, pl_beta, eps   MAP-UR prior (Sec. II eqs. dispdf, gn,
 *              pg, pgamma, peps): device distances on [d_lo, d_hi]
 *              (0 < d_lo < d_hi) with the law `dist_law`, pathloss map
 *              phi(d) = pl_c0 * d^-pl_beta (pl_c0 > 0, pl_beta > 0), Hermite
 *              width eps with 0 < eps and 2 eps < g_l = phi(d_hi).  The
 *              gradient's prior term p^eps'/p^eps does not depend on the
 *              activity probability.
 *   c1, c2_ptr, c2_col, c2_val, c2_nnz   MAP-K2 prior (eq. second): DEVICE
 *              [N] first-order coefficients c_n, and the symmetric pairwise
 *              coefficients c_{n,n'} (zero diagonal) as CSR: row pointers
 *              [N+1], columns and values [c2_nnz], each pair stored in both
 *              rows.  The gradient's prior term is -(1/M)(c_n + sum_n'
 *              c_{n,n'} alpha_n') (eq. ft_gradient, case G).  Row entries
 *              outside [0, c2_nnz) and columns outside [0, N) are skipped on
 *              the device.  Required by MAP-K2 (with g); ignored otherwise, but
 *              must then be zero-initialised by callers that build the struct.
 *   dist_law   MAP-UR distance law behind the pathloss density p_G (eq. pg):
 *              PSCA_DIST_AREA (0): area-uniform on the annulus, p_D(d) =
 *              2d / (d_hi^2 - d_lo^2) (eq. dispdf, the paper's model);
 *              PSCA_DIST_LINEAR (1): uniform in d, p_D(d) = 1 / (d_hi - d_lo).
 *              Other values return PSCA_EINVAL for MAP-UR; ignored otherwise.
 *   x0         optional DEVICE [N] starting iterate x^(0), inside the
 *              variant's box; NULL starts from zero (Algorithm 1).  Read once
 *              at the start of the launch.  Taken by psca_detect,
 *              psca_detect_y, psca_detect_noalloc, psca_net_forward and the
 *              batch entry points (continuing a detection, e.g. plain PSCA
 *              from the unrolled network's output); psca_iterate and the
 *              layer backward take their iterate as an argument and ignore
 *              it.  Must not alias the call's outputs (PSCA_EINVAL where the
 *              output is a single vector).
 */
typedef struct {
  int32_t variant;
  int32_t iters;
  float rho0;
  float rho_decay;
  const float *rho;
  float sigma2;
  int32_t M;
  const float *g;
  const float *p;
  float d_lo, d_hi, pl_c0, pl_beta, eps;
  const float *c1;
  const int32_t *c2_ptr;
  const int32_t *c2_col;
  const float *c2_val;
  int32_t c2_nnz;
  int32_t dist_law;
  const float *x0;
} psca_params;

/* Values of psca_params.dist_law. */
enum { PSCA_DIST_AREA = 0, PSCA_DIST_LINEAR = 1 };

typedef struct psca_ctx psca_ctx;

/* Library version (major*10000 + minor*100 + patch). */
int psca_version(void);

/* Human-readable text for a psca_status; never NULL. */
const char *psca_strerror(int code);

/* Create a context bound to HIP device `device`.  *ctx receives the handle.
 * Returns PSCA_EINVAL for a NULL ctx or a bad device, PSCA_EHIP otherwise. */
int psca_create(psca_ctx **ctx, int device);

/* Free a context and its work buffers (waits for the device).  NULL is a no-op. */
int psca_destroy(psca_ctx *ctx);

/* Sample covariance SigmaHat = Y Y^H / M (the sufficient statistic defined with
 * eq. likelihood_Y; computed once per detection, footnote to Algorithm 1).
 * Y: L x M, SigmaHat: L x L output (exactly Hermitian).  1 <= L <= PSCA_MAX_L, M >= 1. */
int psca_sample_cov(psca_ctx *ctx, const psca_c32 *Y, int L, int M,
                    psca_c32 *Sigma_hat, void *stream);

/* psca_sample_cov of B independent instances of one size in one launch.
 * Instance b reads its L x M matrix Y at Y + b * y_stride and writes its
 * L x L SigmaHat at Sigma_hat + b * sh_stride (strides in complex elements,
 * each block column-major as above; the outputs must not overlap).  Every
 * instance's result is bit-identical to psca_sample_cov on the same Y.
 * Returns PSCA_EINVAL for a NULL ctx, B < 0, L < 1, M < 1, NULL buffers with
 * B > 0, y_stride < L M or sh_stride < L L; PSCA_ENOTSUP for L > PSCA_MAX_L;
 * B = 0 launches nothing. */
int psca_sample_cov_batch(psca_ctx *ctx, int B, const psca_c32 *Y, long long y_stride, int L, int M,
                          psca_c32 *Sigma_hat, long long sh_stride, void *stream);

/* Algorithm 1 from x^(0) = 0 for prm->iters iterations.
 * Sigma_hat: L x L Hermitian PSD; S: L x N; x_out: [N] final iterate
 * (alpha for the K variants, gamma for the U variants).
 * status: optional DEVICE int32 receiving PSCA_OK or PSCA_ENOTPD. */
int psca_detect(psca_ctx *ctx, const psca_c32 *Sigma_hat, const psca_c32 *S, int L, int N,
                const psca_params *prm, float *x_out, int32_t *status, void *stream);

/* psca_sample_cov (with M = prm->M columns of Y) followed by psca_detect. */
int psca_detect_y(psca_ctx *ctx, const psca_c32 *Y, const psca_c32 *S, int L, int N,
                  const psca_params *prm, float *x_out, int32_t *status, void *stream);

/* One iteration of Algorithm 1 (steps 5-8) from an arbitrary iterate:
 * Sigma = S diag(w(x_in)) S^H + sigma^2 I, its Cholesky factor and inverse,
 * q_n = s_n^H Sigma^-1 s_n, r_n = s_n^H Sigma^-1 SigmaHat Sigma^-1 s_n, the
 * closed-form coordinate step x~ (Lemmas 1-4) and
 * x_out = (1 - rho) x_in + rho x~ (eqs. Update_*).  prm->iters and prm->rho are
 * ignored.  q_out, r_out, xt_out are optional DEVICE [N] outputs (NULL to skip).
 * x_in and x_out may not alias. */
int psca_iterate(psca_ctx *ctx, const psca_c32 *Sigma_hat, const psca_c32 *S, int L, int N,
                 const psca_params *prm, float rho, const float *x_in, float *x_out,
                 float *q_out, float *r_out, float *xt_out, int32_t *status, void *stream);

/* The unrolled network's forward pass (PSCA-Net, the "-Net" subsections of
 * Sec. III and IV): Algorithm 1 from x = 0 for prm->iters layers, layer k
 * using step size prm->rho[k] (or the schedule when prm->rho is NULL), with
 * every iterate recorded.  x_hist: DEVICE [(prm->iters + 1) x N], row k =
 * x^(k) (row 0 = 0; the last row is the output). */
int psca_net_forward(psca_ctx *ctx, const psca_c32 *Sigma_hat, const psca_c32 *S, int L, int N,
                     const psca_params *prm, float *x_hist, int32_t *status, void *stream);

/* Backward of one layer x' = (1 - rho) x + rho x~(x) (one iteration of
 * Algorithm 1 with step size rho in [0, 1], eqs. Update_*): given
 * v = dL/dx', writes grad_x = dL/dx (DEVICE [N]) and grad_rho = dL/drho
 * (DEVICE, one float).  Sigma^-1 is recomputed from x_in (the layer's input
 * iterate), not stored.  The clip of Lemmas 1-4 passes gradient where its
 * argument lies inside the bounds (bounds included).  prm->iters and
 * prm->rho are ignored.  1 <= L <= 256; MAP-K2 has no backward
 * (PSCA_ENOTSUP). */
int psca_layer_backward(psca_ctx *ctx, const psca_c32 *Sigma_hat, const psca_c32 *S, int L, int N,
                        const psca_params *prm, float rho, const float *x_in, const float *v, float *grad_x,
                        float *grad_rho, int32_t *status, void *stream);

/* One instance of a batched layer backward: the arguments of
 * psca_layer_backward (all DEVICE pointers; status optional). */
typedef struct {
  const psca_c32 *Sigma_hat;  /* L x L, column-major */
  const psca_c32 *S;          /* L x N, column-major */
  int32_t L, N;
  psca_params prm;            /* variant, sigma2, M, g, p, prior; iters and rho ignored */
  const float *x_in;          /* [N] the layer's input iterate */
  const float *v;             /* [N] dL/dx' */
  float *grad_x;              /* [N] dL/dx */
  float *grad_rho;            /* one float: this instance's dL/drho */
  int32_t *status;            /* PSCA_OK / PSCA_ENOTPD / PSCA_ESYNC, or NULL */
} psca_back_problem;

/* B layer backwards with the same step size rho in ONE persistent launch
 * (teams of workgroups as in psca_detect_batch), equivalent to B calls of
 * psca_layer_backward: the backward of one layer of the unrolled network
 * over a minibatch.  `problems` is a HOST array read before the call
 * returns.  Every instance is validated first (MAP-K2 has no backward, and
 * a batch mixing L <= 64 with L > 64 is PSCA_ENOTSUP). */
int psca_layer_backward_batch(psca_ctx *ctx, int B, const psca_back_problem *problems, float rho, void *stream);

/* One instance of a batch: the arguments of psca_detect.  All pointers are
 * DEVICE pointers on the context's GPU; status is optional (NULL). */
typedef struct {
  const psca_c32 *Sigma_hat;  /* L x L, column-major */
  const psca_c32 *S;          /* L x N, column-major */
  int32_t L, N;
  psca_params prm;            /* variant, iters, schedule, sigma2, M, g, p, prior */
  float *x_out;               /* [N] */
  int32_t *status;            /* PSCA_OK / PSCA_ENOTPD / PSCA_ESYNC, or NULL */
  float *x_hist;              /* optional [(prm.iters + 1) x N]: every iterate, as psca_net_forward */
} psca_problem;

/* B independent detections (Algorithm 1 from x = 0 for each), equivalent to
 * B calls of psca_detect, in ONE persistent launch.  `problems` is a HOST
 * array of B entries, read before the call returns.  The grid is split into
 * teams of T workgroups; every instance runs on one team (its own group of
 * workgroups and device-wide barrier) and each team works through a list of
 * instances, longest first.  Instances may differ in L, N, M, variant,
 * iteration count and parameters.  T is the value psca_autotune_batch chose
 * for a batch of the same (L, N) list, else a default (one team per instance
 * when the batch fits the GPU at once, else the smallest teams).  Every
 * instance is validated as in psca_detect before anything is launched
 * (PSCA_EINVAL / PSCA_ENOTSUP for the first bad one; a batch mixing L <= 96
 * with L > 96 is PSCA_ENOTSUP: the two sides run in different kernels). */
int psca_detect_batch(psca_ctx *ctx, int B, const psca_problem *problems, void *stream);

/* Autotuner for psca_detect_batch: times the batch with every candidate team
 * specification (uniform team sizes from the smallest feasible team to the
 * whole GPU, and mixed teams for tiles of 32, 48, ..., 128 columns), each
 * instance capped at tune_iters >= 1 and at 2 tune_iters iterations, and
 * keeps the one whose time extrapolated from those two runs to the batch's
 * largest iteration count is least, in the context, for batches with the
 * same (L, N) list.  Synchronous; writes scratch results into the
 * instances' x_out.  *team_size (optional) receives the choice, in the
 * encoding of psca_plan_create. */
int psca_autotune_batch(psca_ctx *ctx, int B, const psca_problem *problems, int tune_iters, int *team_size,
                        void *stream);

/* A planned batch for repeated launches, e.g. inside a captured HIP graph:
 * psca_plan_create does all allocation and host-to-device copying (tiles,
 * team lists, descriptors; synchronous); psca_plan_launch only enqueues two
 * kernels (barrier reset, persistent batch), so it may be captured.  The
 * problems' device buffers must stay valid while the plan is used; their
 * contents are read at each launch.  team_size:
 *   > 0  uniform teams of team_size workgroups (at least the smallest
 *        feasible team, at most the co-resident capacity);
 *   < 0  mixed teams: instance b runs on a team of
 *        max(ceil(N_b / largest tile), ceil(N_b / -team_size)) workgroups
 *        (rounded up to the next of 1, 2, 4, 6, 8, 12, 16, 24, 32, 48, ...:
 *        powers of two and their 1.5 multiples); instances of one team size
 *        share that size's teams, and each size gets teams in proportion to
 *        its work.  -team_size is a multiple of 16 up to 128;
 *   0    the value psca_autotune_batch chose for this (L, N) list, else the
 *        default of psca_detect_batch.
 * Other values return PSCA_EINVAL.  psca_plan_team_size returns the plan's
 * team_size in this encoding (mixed specifications are multiples of 16, so
 * they never equal an error code); a mixed specification under which every
 * instance gets the same team size T is the uniform plan of T and reports T.
 * Inside a capture the batch kernel is recorded as an ordinary kernel node,
 * which relies on its grid (at most the device's co-resident capacity) being
 * resident at once; the bounded device-wide waits report PSCA_ESYNC if not. */
typedef struct psca_plan psca_plan;
int psca_plan_create(psca_ctx *ctx, int B, const psca_problem *problems, int team_size, psca_plan **plan);
int psca_plan_launch(psca_plan *plan, void *stream);
int psca_plan_team_size(const psca_plan *plan);
int psca_plan_destroy(psca_plan *plan);   /* waits for the device; NULL is a no-op */

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * detection as psca_detect (same kernels, tiles and results, bit for bit),
 * with its work buffers (partials of Sigma, packed Sigma, barrier and status
 * words) in a fixed array of PSCA_NOALLOC_SCRATCH_BYTES that the library
 * holds on every GPU it runs on until the process ends; the call makes no
 * allocation (no hipMalloc, hipFree or allocating library routine).  The
 * caller passes inputs and outputs as for psca_detect, and `ctx` is only
 * read (psca_create set the array's device address up).  Limits: L <= 96
 * (the single-workgroup factorisation), and a problem whose work buffers
 * exceed the array returns PSCA_ENOTSUP before any launch (the array holds
 * every L <= 96 detection the library can tile: up to 256 workgroups of
 * partials).  Every call on one GPU shares that GPU's array and finds the
 * previous call's contents in it (the barrier and status words are reset by
 * a kernel at the start of each call): calls that overlap in time on one GPU,
 * from any context or stream, race and must not be issued. */
#define PSCA_NOALLOC_SCRATCH_BYTES ((size_t)12 << 20)
int psca_detect_noalloc(psca_ctx *ctx, const psca_c32 *Sigma_hat, const psca_c32 *S, int L, int N,
                        const psca_params *prm, float *x_out, int32_t *status, void *stream);

/* Threshold module: support[n] = (x[n] >= theta) ? 1 : 0 (Sec. III-A). */
int psca_threshold(const float *x, int N, float theta, uint8_t *support, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* PSCA_H */
