// psca.hip — HIP kernels (gfx950) and C ABI for PSCA device activity detection.
//
// One PSCA iteration (Algorithm 1, steps 5-8 of Tan & Cui, arXiv 2503.15259):
//   Sigma = S diag(w) S^H + sigma^2 I            (eqs. cov_a / cov_b)
//   Sigma = L L^H (Cholesky), W = L^-1, Sigma^-1 = W^H W
//   B = Sigma^-1 S, D = SigmaHat B                (complex GEMMs)
//   q_n = Re(s_n^H b_n), r_n = Re(b_n^H d_n)      (the two terms of eq. gradient_ML)
//   x~_n = clip(x_n - grad_n / curv_n, lo, hi)    (Lemmas 1-4)
//   x_n <- (1 - rho_k) x_n + rho_k x~_n           (eqs. Update_*)
//
// Execution model.  Every detection, batch and network forward is ONE
// persistent launch whose workgroups meet at device-wide barriers (agent-scope
// fences, bounded spins that report PSCA_ESYNC instead of hanging); there are
// no atomics on data, so a result is bitwise reproducible for a given launch
// shape.  Workgroup numbers are XCD-major, so the workgroups that share an
// instance share an L2.  Three kernel families:
//
//   k_psca, k_psca_teams (L <= 96).  A workgroup owns NT = 16 * ncb columns
//     of S; the tile, its iterate and pathloss stay in LDS for the whole
//     solve.  Per iteration:
//       A. tile partial P_g = S_g diag(w_g) S_g^H (FP64 MFMA Gram) -> HBM
//       B. workgroup g sums a fixed slice of the partials (FP64) -> Sigma
//       C. every workgroup factors Sigma redundantly in LDS (identical inputs
//          and code, so identical results and decisions), forms Sigma^-1 on
//          MFMA, then B = Sigma^-1 S_g, D = SigmaHat B, the quadratic forms,
//          the coordinate step and the update of its columns.
//     k_psca_teams runs a list of instances (uneven batches, minibatches) on
//     teams of workgroups, one instance per team at a time.
//   k_psca_large_teams (97 <= L <= 256).  Sigma, its factor and
//     Sigma - SigmaHat live in device memory; the factorisation is spread
//     over the team, and the solves, q, q - r and the coordinate step of each
//     16-column block run in one wavefront's registers.
//   k_psca_back_teams (L <= 64) and k_psca_back_large_* (65 <= L <= 256).
//     The vector-Jacobian product of one unrolled layer with respect to its
//     input and its step size, Sigma^-1 recomputed from the layer input.
//
// Complex GEMMs use v_mfma_f32_16x16x4f32, on the real 4-product split
//   Re C += Re A Re B - Im A Im B,   Im C += Re A Im B + Im A Re B
// or with three real products (Gauss) where the operands allow it; the Gram
// partials use v_mfma_f64_16x16x4f64.
// Operand layout of that instruction (wave64): lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; it receives C[4*(l/16)+v][l%16] in accumulator v.

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>
#include <utility>

#include "psca.h"

namespace psca_impl {

constexpr int kThreads = 256;                              // helper kernels
constexpr int kBlk = 16;
constexpr int kMaxL = PSCA_MAX_L;                          // 256 (above 96: the cooperative large-L kernel)
constexpr int kMaxLdsL = 96;                               // largest L whose L x L matrix lives in LDS
constexpr int kMaxNcb = 8;                                 // column blocks per workgroup (LDS permitting)
constexpr unsigned kSpinLimit = 1u << 20;                  // grid-barrier wait bound

typedef float f4 __attribute__((ext_vector_type(4)));

// Optional phase timer for profiling builds (-DPSCA_PHASE_TRACE): workgroup 0
// stamps the 100 MHz real-time counter at phase boundaries of each iteration.
#ifdef PSCA_PHASE_TRACE
constexpr int kTraceIters = 128, kTraceMarks = 16;
__device__ unsigned long long g_phase_trace[kTraceIters * kTraceMarks];
__device__ unsigned long long g_step_trace[128];
__device__ unsigned long long g_sub_trace[128 * 4];
#define PSCA_SUB_MARK(it, k, id)                                                             \
  do {                                                                                      \
    if ((it) == 5 && blockIdx.x == 0 && threadIdx.x == 0) g_sub_trace[(k) * 4 + (id)] = __builtin_readcyclecounter(); \
  } while (0)
#define PSCA_STEP_MARK(it, k)                                                               \
  do {                                                                                      \
    if ((it) == 5 && blockIdx.x == 0 && threadIdx.x == 0) g_step_trace[k] = __builtin_amdgcn_s_memrealtime(); \
  } while (0)
#define PSCA_MARK(it, id)                                                                   \
  do {                                                                                      \
    if (blockIdx.x == 0 && threadIdx.x == 0 && (it) < kTraceIters)                          \
      g_phase_trace[(it) * kTraceMarks + (id)] = __builtin_amdgcn_s_memrealtime();          \
  } while (0)
#else
#define PSCA_MARK(it, id) ((void)0)
#define PSCA_STEP_MARK(it, k) ((void)0)
#define PSCA_SUB_MARK(it, k, id) ((void)0)
#endif

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// C += A * B for one k-step of a complex 16x16 block (real 4-product split).
__device__ __forceinline__ void cmfma(float2 a, float2 b, f4 &cr, f4 &ci) {
  cr = mfma4(a.x, b.x, cr);
  cr = mfma4(-a.y, b.y, cr);
  ci = mfma4(a.x, b.y, ci);
  ci = mfma4(a.y, b.x, ci);
}

typedef double d4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ d4 mfma4d(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// Complex 16x16x4 block product accumulated in FP64 with three real products
// (Gauss): t1 += ar br, t2 += ai bi, t3 += (ar + ai)(br + bi); then
// re = t1 - t2 and im = t3 - t1 - t2.  Operand layout as the FP32 form
// (A[i][k] in lane i + 16k, B[k][j] in lane j + 16k); the result differs:
// C[i][j] sits in lane j + 16 (i % 4), element i / 4.  With FP32-valued
// operands the products are exact in FP64, and the cancellation in im costs
// about 1e-16 of |a||b|.
__device__ __forceinline__ void cmfma_d3(double2 a, double2 b, d4 &t1, d4 &t2, d4 &t3) {
  t1 = mfma4d(a.x, b.x, t1);
  t2 = mfma4d(a.y, b.y, t2);
  t3 = mfma4d(a.x + a.y, b.x + b.y, t3);
}

// Keeps the enclosing block a real (scalar) branch: the compiler may not
// speculate it into unconditional code plus selects.
#define PSCA_KEEP_BRANCH() asm volatile("" ::: "memory")

// packed lower-block index of block (I, J), I >= J, and its inverse
__device__ __forceinline__ int blk_index(int I, int J) { return I * (I + 1) / 2 + J; }
__device__ __forceinline__ void blk_coords(int b, int &I, int &J) {
  int r = 0;
  while ((r + 1) * (r + 2) / 2 <= b) ++r;
  I = r;
  J = b - r * (r + 1) / 2;
}

// ---------------------------------------------------------------------------
// Variant step (Lemmas 1-4)
// ---------------------------------------------------------------------------
struct StepArgs {
  int variant;
  float inv_M;
  const float *g;   // [N] known pathloss (K variants)
  const float *p;   // [N] activity probability (MAP-K)
  float eps, g_l, g_u, h2_b, dens_c;   // MAP-UR prior constants
  // MAP-K2 (second-order activity model): c_n, the CSR rows of c_{n,n'}, and
  // the exchange buffer of the iterate [2][N] (x^(k) in half k % 2)
  const float *c1;
  const int32_t *c2_ptr, *c2_col;
  const float *c2_val;
  int32_t c2_nnz;
  float *xg;
};

// sum_{n'} c_{n,n'} x_n' over row n of the pairwise coefficients, x the
// exchanged iterate.  Entries outside [0, nnz) or with a column outside
// [0, N) are skipped.
__device__ __forceinline__ float pair_sum(const StepArgs &a, int n, int N, const float *x) {
  const int k0 = max(0, a.c2_ptr[n]), k1 = min(a.c2_nnz, a.c2_ptr[n + 1]);
  float acc = 0.0f;
  for (int k = k0; k < k1; ++k) {
    const int m = a.c2_col[k];
    if ((unsigned)m < (unsigned)N) acc += a.c2_val[k] * x[m];
  }
  return acc;
}

// p^eps'(x) / p^eps(x) of the smoothed prior (eqs. peps, H2, pepsd) in the
// simplified per-piece forms; 0 where p^eps = 0 (the gap between eps and g_l - eps).
__device__ __forceinline__ float prior_log_ratio(float x, const StepArgs &a) {
  const float e = a.eps;
  if (x < e) return 6.0f * x / ((e + 2.0f * x) * (x - e));          // H1'/H1
  if (x < a.g_l - e) return 0.0f;
  if (x < a.g_l) {                                                  // H2'/H2, u = x - g_l
    const float u = x - a.g_l;
    const float num = -6.0f * u / e + a.h2_b * (3.0f * u + e);
    const float den = (u + e) * ((1.0f - 2.0f * u / e) + a.h2_b * u);
    return den == 0.0f ? 0.0f : num / den;
  }
  return -a.dens_c / x;                                             // -(2/beta + 1)/x
}

// g: known pathloss of the device (K variants); logit = log(p / (1 - p)) (MAP-K);
// qmr = q - r, computed directly (see the phase that forms it).
__device__ __forceinline__ float coordinate_step(float x, float q, float qmr, float g, float logit,
                                                 const StepArgs &a) {
  float grad, curv, hi;
  switch (a.variant) {
    case PSCA_ML_K: {
      grad = g * qmr;
      const float gq = g * q;
      curv = gq * gq;
      hi = 1.0f;
      break;
    }
    case PSCA_MAP_K:
    case PSCA_MAP_K2: {   // logit: log(p/(1-p)), or c_n + sum_n' c_{n,n'} x_n'
      grad = g * qmr - logit * a.inv_M;
      const float gq = g * q;
      curv = gq * gq;
      hi = 1.0f;
      break;
    }
    case PSCA_ML_UD:
      grad = qmr;
      curv = q * q;
      hi = INFINITY;
      break;
    default:  // PSCA_MAP_UR
      grad = qmr - prior_log_ratio(x, a) * a.inv_M;
      curv = q * q;
      hi = a.g_u;
      break;
  }
  return fminf(fmaxf(x - grad / curv, 0.0f), hi);
}

// Derivative of prior_log_ratio (the MAP-UR prior term of the gradient) in
// the same per-piece forms; 0 in the gap.
__device__ __forceinline__ float prior_log_ratio_deriv(float x, const StepArgs &a) {
  const float e = a.eps;
  if (x < e) {                                                      // (H1'/H1)'
    const float t = (e + 2.0f * x) * (x - e);
    return -6.0f * (2.0f * x * x + e * e) / (t * t);
  }
  if (x < a.g_l - e) return 0.0f;
  if (x < a.g_l) {                                                  // (H2'/H2)'
    const float u = x - a.g_l;
    const float num = -6.0f * u / e + a.h2_b * (3.0f * u + e);
    const float f = (1.0f - 2.0f * u / e) + a.h2_b * u;
    const float den = (u + e) * f;
    if (den == 0.0f) return 0.0f;
    const float dnum = -6.0f / e + 3.0f * a.h2_b;
    const float dden = f + (u + e) * (-2.0f / e + a.h2_b);
    return (dnum * den - num * dden) / (den * den);
  }
  return a.dens_c / (x * x);                                        // (2/beta + 1)/x^2
}

// Partial derivatives of one layer's coordinate step for the backward pass:
// with kappa = g (known pathloss) or 1, grad = kappa (q - r) - c(x),
// curv = (kappa q)^2 and pre = x - grad / curv: x~ = clip(pre, lo, hi),
// mask = [lo <= pre <= hi], dq = d pre/dq, dr = d pre/dr and own = d pre/dx
// at fixed q, r.
struct StepDerivs {
  float xt, mask, dq, dr, own, kappa;
};
__device__ __forceinline__ StepDerivs step_derivs_qmr(float x, float q, float qmr, float g, float logit,
                                                      const StepArgs &a) {
  float kappa = 1.0f, c = 0.0f, cp = 0.0f, hi;
  switch (a.variant) {
    case PSCA_ML_K: kappa = g; hi = 1.0f; break;
    case PSCA_MAP_K: kappa = g; c = logit * a.inv_M; hi = 1.0f; break;
    case PSCA_ML_UD: hi = INFINITY; break;
    default:   // PSCA_MAP_UR
      c = prior_log_ratio(x, a) * a.inv_M;
      cp = prior_log_ratio_deriv(x, a) * a.inv_M;
      hi = a.g_u;
      break;
  }
  const float grad = kappa * qmr - c;
  const float kq = kappa * q;
  const float curv = kq * kq;
  const float pre = x - grad / curv;
  StepDerivs d;
  d.xt = fminf(fmaxf(pre, 0.0f), hi);
  d.mask = (pre >= 0.0f && pre <= hi) ? 1.0f : 0.0f;
  d.dq = (2.0f * grad - kq) / (kappa * kq * q * q);
  d.dr = 1.0f / (kappa * q * q);
  d.own = 1.0f + cp / curv;
  d.kappa = kappa;
  return d;
}
__device__ __forceinline__ StepDerivs step_derivs(float x, float q, float r, float g, float logit,
                                                  const StepArgs &a) {
  return step_derivs_qmr(x, q, q - r, g, logit, a);
}

// ---------------------------------------------------------------------------
// Grid barrier (agent scope).  Each workgroup raises its own arrival word
// (64-byte stride, no contended atomics) and waits until it has seen every
// arrival word of its instance reach the generation: one round trip through
// memory.  Every wait is bounded by kSpinLimit polls: a waiter that gives up
// raises *abort, and all waiters also watch *abort, so a missing workgroup
// cannot hang the grid.
// ---------------------------------------------------------------------------
struct GridBar {
  unsigned *arrive;    // [G * 16]
  unsigned *release;   // unused (kept zero)
  int32_t *abort_flag;
};

// Waits until *word has reached generation `target` (generations only grow;
// the difference is taken modulo 2^32).
__device__ __forceinline__ bool spin_until(const unsigned *word, unsigned target, const int32_t *abort_flag) {
  unsigned spins = 0;
  while ((int)(__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
    if (++spins > kSpinLimit) return false;
    if ((spins & 255u) == 0 && __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return false;
  }
  return true;
}

__device__ __forceinline__ bool grid_sync(const GridBar &b, unsigned G, unsigned g, unsigned &gen, int *s_ok) {
  __syncthreads();
  const unsigned target = gen + 1;
  gen = target;
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(&b.arrive[g * 16], target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  int ok = 1;
  for (unsigned w = threadIdx.x; w < G; w += blockDim.x)
    if (!spin_until(&b.arrive[w * 16], target, b.abort_flag)) ok = 0;
  ok = __syncthreads_and(ok);
  if (threadIdx.x == 0) {
    if (!ok) __hip_atomic_store(b.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *s_ok = ok;
  }
  __syncthreads();
  return *s_ok != 0;
}

// ---------------------------------------------------------------------------
// The persistent detection kernel
// ---------------------------------------------------------------------------
struct CoopArgs {
  const float2 *S;      // L x N, column-major
  const float2 *Sh;     // L x L, column-major
  int L, N;
  int G, ncb, NT;       // workgroups, 16-column blocks per workgroup, columns per workgroup
  int iters;
  double rho0, rho_decay;
  const float *rho_dev; // [iters] or null
  float rho_fixed;      // >= 0: every iteration uses this step (single-iteration entry point)
  float sigma2;
  StepArgs a;
  const float *x_in;    // [N] initial iterate or null (zeros)
  float *x_out, *q_out, *r_out, *xt_out;
  float *x_hist;        // [iters + 1][N] every iterate, or null
  int32_t *status;
  float2 *partials;     // [G][pstride], workgroup g's packed partial of Sigma at g * pstride
  size_t pstride;       // >= NB * 256
  float2 *sigma;        // [NB * 256]
  GridBar bar;
};

// LDS footprint in bytes of k_psca<Lp, 64 * waves> for NT columns per workgroup
// 16-column blocks of the B tile per round of C4: two where LDS allows.
__host__ __device__ constexpr int b_tile_blocks(int Lp) { return Lp <= 80 ? 2 : 1; }

__host__ __device__ inline size_t lds_bytes(int Lp, int NT, int waves) {
  const size_t pt = (size_t)NT + 1, P = (size_t)Lp + 1, Lb = (size_t)Lp / 16;
  const bool sh_lds = Lp <= 64;
  const size_t f2 = (size_t)Lp * pt + (size_t)Lp * (16 * b_tile_blocks(Lp) + 1) + (size_t)Lp * P +
                    (sh_lds ? (size_t)Lp * P : 0) + (size_t)waves * 256;
  const size_t f4b = 3 * (size_t)NT + 2 * Lb * NT;   // floats
  return f2 * sizeof(float2) + f4b * 4;
}

#define PSCA_LDS_F2(p) (*(const float2 *)(p))

// Complex 16x16 block product C += A * B with both operands in LDS,
// column-major with pitch ld: A[i][k] at A[k * ld + i], B[k][j] at B[j * ld + k].
__device__ __forceinline__ void cblock_mma(const float2 *A, const float2 *B, int ld, int l16, int lq, f4 &cr,
                                           f4 &ci) {
  float2 a[4], b[4];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    a[ks] = A[(4 * ks + lq) * ld + l16];
    b[ks] = B[l16 * ld + 4 * ks + lq];
  }
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) cmfma(a[ks], b[ks], cr, ci);
}

// Complex 16x16 block product over k in [k0, k0 + 16): A column-major in LDS
// (A[i][k] at A[k * lda + i]), B row-major in LDS (B[k][j] at B[k * ldb + j]).
__device__ __forceinline__ void cblock_mma_rm(const float2 *A, int lda, const float2 *B, int ldb, int k0, int l16,
                                              int lq, f4 &cr, f4 &ci) {
  float2 a[4], b[4];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    const int k = k0 + 4 * ks + lq;
    a[ks] = A[k * lda + l16];
    b[ks] = B[k * ldb + l16];
  }
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) cmfma(a[ks], b[ks], cr, ci);
}

// ---------------------------------------------------------------------------
// Sigma^-1 by a blocked Cholesky factorisation Sigma = L L^H, W = L^-1 and
// Sigma^-1 = W^H W
// ---------------------------------------------------------------------------
// Orders this wavefront's LDS writes before its later LDS reads.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int K>
__device__ __forceinline__ float row_bcast(float v) {   // lane K of each 16-lane row
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x150 + K, 0xf, 0xf, true));
}

// Value held by lane (j, G) for every lane (j, r), j = lane % 16, r = lane / 16:
// the upper or lower half of the wavefront is copied to both halves by a
// 32-lane swap, then row G & 1 of each pair of 16-lane rows by a 16-lane swap.
template <int G>
__device__ __forceinline__ float group_bcast(float v) {
  const unsigned u = __float_as_uint(v);
  const auto h = __builtin_amdgcn_permlane32_swap(u, u, false, false);
  const unsigned hv = (G >> 1) ? h[1] : h[0];
  const auto q = __builtin_amdgcn_permlane16_swap(hv, hv, false, false);
  return __uint_as_float((G & 1) ? q[1] : q[0]);
}

// leaf_chol: one wavefront factors a 16x16 HPD block A = L L^H held in
// registers and turns it into W = L^-1 in place.  Lane l holds column
// j = l % 16 of rows r, r+4, r+8, r+12 (r = l / 16) of the working matrix Z,
// which starts as A (both triangles).  Below the diagonal, columns j < K of
// Z hold the running inverse X (unit diagonal, rows not yet scaled), columns
// j >= K the trailing part of A.  Step K, with p = Z[K][K] and c = column K:
//   Z[i][j] -= c_i Z[K][j] / p     rows i > K, columns j != K
//                                  (j > K: Schur update; j < K: X[i][j] -= L[i][K] W[K][j] sqrt(p))
//   Z[i][K]  = -c_i / p            rows i > K (X[i][K] = -L[i][K] / sqrt(p))
// Row K of X is final after step K; W = diag(p)^-1/2 X is applied at the end
// together with the unit diagonal and the zero upper triangle, so 1/p is the
// only quantity on the chain from one pivot to the next.  The pivot comes
// by readlane, column K on the lane's rows by a DPP row broadcast, row K on
// the lane's column by two lane swaps.  No LDS and no barrier.  ok turns
// false if a pivot is not positive and finite.
template <int K>
__device__ __forceinline__ void chol_step(float2 (&z)[4], int j, int r, float (&piv)[16], bool &ok) {
  constexpr int mk = K >> 2, gk = K & 3;
  const float p = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(z[mk].x), K + 16 * gk));
  piv[K] = p;
  ok = ok && __builtin_amdgcn_classf(p, 0x180);   // positive, finite, not zero
  const bool colk = (j == K);
  const float2 zk = make_float2(group_bcast<gk>(z[mk].x), group_bcast<gk>(z[mk].y));   // Z[K][j]
  const float2 zs = colk ? make_float2(1.0f, 0.0f) : zk;
  float invd = __builtin_amdgcn_rcpf(p);
  invd = __builtin_fmaf(invd, __builtin_fmaf(-p, invd, 1.0f), invd);   // one Newton step
  const float2 rk = make_float2(zs.x * invd, zs.y * invd);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    if (4 * m + 3 > K) {                   // some row r + 4m lies below K
      const float2 ck = make_float2(row_bcast<K>(z[m].x), row_bcast<K>(z[m].y));   // Z[r+4m][K]
      if (r + 4 * m > K) {
        const float2 base = colk ? make_float2(0.0f, 0.0f) : z[m];
        z[m].x = base.x - ck.x * rk.x + ck.y * rk.y;
        z[m].y = base.y - ck.x * rk.y - ck.y * rk.x;
      }
    }
  }
}

template <int... Ks>
__device__ __forceinline__ bool chol_steps(float2 (&z)[4], int j, int r, float (&piv)[16],
                                           std::integer_sequence<int, Ks...>) {
  bool ok = true;
  (chol_step<Ks>(z, j, r, piv, ok), ...);
  return ok;
}

// Factors the 16x16 block at D (column-major, pitch ld, both triangles) and
// overwrites it with W = L^-1 (zeros above the diagonal).
__device__ __forceinline__ bool leaf_chol(float2 *D, int ld, int lane) {
  const int j = lane & 15, r = lane >> 4;
  float2 z[4];
  float piv[16];
#pragma unroll
  for (int m = 0; m < 4; ++m) z[m] = D[j * ld + r + 4 * m];
  const bool ok = chol_steps(z, j, r, piv, std::make_integer_sequence<int, 16>{});
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int i = r + 4 * m;
    const float p = r == 0 ? piv[4 * m] : (r == 1 ? piv[4 * m + 1] : (r == 2 ? piv[4 * m + 2] : piv[4 * m + 3]));
    float rs = __builtin_amdgcn_rsqf(p);
    rs = rs * (1.5f - 0.5f * p * rs * rs);   // one Newton step
    float2 w = make_float2(z[m].x * rs, z[m].y * rs);
    if (i == j) w = make_float2(rs, 0.0f);
    if (i < j) w = make_float2(0.0f, 0.0f);
    D[j * ld + i] = w;
  }
  return ok;
}

// MFMA tasks of block step J of the factorisation (one wavefront each; WS
// column-major with pitch P, lower blocks hold A and then L).
// Panel: L_IJ = A_IJ W_JJ^H (W_JJ in the diagonal block J).
__device__ __forceinline__ void chol_panel(float2 *WS, int P, int J, int I, int l16, int lq) {
  f4 cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
  float2 a4[4], b4[4];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    const int k = 4 * ks + lq;
    a4[ks] = WS[(16 * J + k) * P + 16 * I + l16];
    const float2 w = WS[(16 * J + k) * P + 16 * J + l16];   // W_JJ[l16][k]
    b4[ks] = make_float2(w.x, -w.y);
  }
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) cmfma(a4[ks], b4[ks], cr, ci);
  wave_lds_sync();
  float2 *dst = WS + (16 * J + l16) * P + 16 * I + 4 * lq;
#pragma unroll
  for (int v = 0; v < 4; ++v) dst[v] = make_float2(cr[v], ci[v]);
}

// Trailing: A_IK -= L_IJ L_KJ^H, J < K <= I.
__device__ __forceinline__ void chol_trail(float2 *WS, int P, int J, int I, int K, int l16, int lq) {
  float2 *dst = WS + (16 * K + l16) * P + 16 * I + 4 * lq;
  f4 cr, ci;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    cr[v] = dst[v].x;
    ci[v] = dst[v].y;
  }
  float2 a4[4], b4[4];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    const int k = 4 * ks + lq;
    const float2 l = WS[(16 * J + k) * P + 16 * I + l16];   // L_IJ[l16][k]
    a4[ks] = make_float2(-l.x, -l.y);
    const float2 m = WS[(16 * J + k) * P + 16 * K + l16];   // L_KJ[l16][k]
    b4[ks] = make_float2(m.x, -m.y);                        // L_KJ^H[k][l16]
  }
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) cmfma(a4[ks], b4[ks], cr, ci);
#pragma unroll
  for (int v = 0; v < 4; ++v) dst[v] = make_float2(cr[v], ci[v]);
}

// Global loads and stores through an explicitly global pointer: the
// descriptors' generic pointers would otherwise give flat instructions, which
// also count as LDS operations, so that every wait for an LDS read would wait
// for them too.
typedef float gvec2 __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(1))) gvec2 gvec2_g;
typedef __attribute__((address_space(1))) gvec2 gvec2_gw;
__device__ __forceinline__ float2 ldg2(const float2 *p, size_t i) {
  const gvec2 v = ((gvec2_g *)p)[i];
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void stg2(float2 *p, size_t i, float2 x) {
  ((gvec2_gw *)p)[i] = gvec2{x.x, x.y};
}
// streaming store: data read back only after it has left the caches
__device__ __forceinline__ void stg2_nt(float2 *p, size_t i, float2 x) {
  __builtin_nontemporal_store(gvec2{x.x, x.y}, (gvec2_gw *)p + i);
}

// ---------------------------------------------------------------------------
// Phases shared by the forward and the backward bodies
// ---------------------------------------------------------------------------
// Packed lower blocks of the tile's Gram matrix S_t diag(wv) S_t^H into dst
// (MFMA, complex product on the real 4-product split).  The products of the
// FP32 operands are exact in FP64 and the sums over the tile are FP64; each
// entry is rounded once to FP32 when stored.  With the FP64 sum over the
// partials in phase B, the entries of Sigma carry about one rounding, which
// matters because q and q - r move with kappa(Sigma) times the entry errors
// of Sigma.  St: [Lp][PT] S tile.
template <int LP, int THREADS>
__device__ __forceinline__ void tile_gram(const float2 *St, int PT, int ncb, const float *wv, float2 *dst) {
  constexpr int kWaves = THREADS / 64, Lb = LP / 16, NB = Lb * (Lb + 1) / 2;
  constexpr int kBlocksPerWave = (NB + kWaves - 1) / kWaves;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, l16 = lane & 15, lq = lane >> 4;
#pragma unroll
  for (int q = 0; q < kBlocksPerWave; ++q) {
    const int b = wave + kWaves * q;
    if (b < NB) {
      int I, J;
      blk_coords(b, I, J);
      d4 t1 = {0.0, 0.0, 0.0, 0.0}, t2 = t1, t3 = t1;
      for (int cb = 0; cb < ncb; ++cb) {
        double2 av4[4], bv4[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const int c = 16 * cb + 4 * ks + lq;
          const float2 s = St[(16 * J + l16) * PT + c];
          const float2 a = St[(16 * I + l16) * PT + c];
          const double w = wv[c];
          av4[ks] = make_double2(a.x, a.y);
          bv4[ks] = make_double2(w * s.x, -w * s.y);
        }
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) cmfma_d3(av4[ks], bv4[ks], t1, t2, t3);
      }
      const int o = b * 256 + l16 * 16 + lq;   // rows lq + 4v of column l16
#pragma unroll
      for (int v = 0; v < 4; ++v)
        stg2(dst, o + 4 * v, make_float2((float)(t1[v] - t2[v]), (float)(t3[v] - t1[v] - t2[v])));
    }
  }
}

__device__ __forceinline__ void store_reduced(float2 *out, int e, double2 sm, bool add_diag, int L, float sigma2) {
  if (add_diag) {
    const int b = e >> 8, jj = (e & 255) >> 4, ii = e & 15;
    int I, J;
    blk_coords(b, I, J);
    if (I == J && ii == jj) {
      const int i = 16 * I + ii;
      sm.x += (i < L) ? (double)sigma2 : 1.0;
      sm.y = 0.0;
    }
  }
  stg2(out, e, make_float2((float)sm.x, (float)sm.y));
}

// Workgroup g's 1/G slice of the sum over the G packed partials (rank h at
// partials + h * pstride) into out; with add_diag, sigma2 is added to the
// diagonal of rows < L and 1 to padded rows (isolated unit pivots), and the
// imaginary part of the diagonal is zeroed.  The partials are summed in FP64
// and the result rounded once.  scr: THREADS double2 of LDS.
template <int LP, int THREADS>
__device__ __forceinline__ void reduce_slice(const float2 *partials, size_t pstride, int G, int g, float2 *out,
                                             double2 *scr, bool add_diag, int L, float sigma2) {
  constexpr int Lb = LP / 16, E = Lb * (Lb + 1) / 2 * 256;
  static_assert(THREADS * sizeof(double2) <= (THREADS / 64) * 256 * sizeof(float2), "scr holds THREADS double2");
  const int tid = threadIdx.x;
  const int per = (E + G - 1) / G;
  const int start = g * per, end = min(E, start + per);
  const int cnt = max(0, end - start);
  if (cnt > 0 && cnt <= THREADS) {
    const int Pp = THREADS / cnt;   // threads per element
    if (tid < cnt * Pp) {
      const int e = start + tid % cnt, part = tid / cnt;
      double2 acc = make_double2(0.0, 0.0);
      int h = part;
      for (; h + 3 * Pp < G; h += 4 * Pp) {   // four loads in flight, then the adds in order
        float2 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = ldg2(partials, (size_t)(h + u * Pp) * pstride + e);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          acc.x += v[u].x;
          acc.y += v[u].y;
        }
      }
      for (; h < G; h += Pp) {
        const float2 v = ldg2(partials, (size_t)h * pstride + e);
        acc.x += v.x;
        acc.y += v.y;
      }
      scr[tid] = acc;
    }
    __syncthreads();
    if (tid < cnt) {
      double2 sm = make_double2(0.0, 0.0);
      for (int part = 0; part < Pp; ++part) {
        const double2 v = scr[part * cnt + tid];
        sm.x += v.x;
        sm.y += v.y;
      }
      store_reduced(out, start + tid, sm, add_diag, L, sigma2);
    }
  } else {
    for (int e = start + tid; e < end; e += THREADS) {
      double2 sm = make_double2(0.0, 0.0);
      for (int h = 0; h < G; ++h) {
        const float2 v = ldg2(partials, (size_t)h * pstride + e);
        sm.x += v.x;
        sm.y += v.y;
      }
      store_reduced(out, e, sm, add_diag, L, sigma2);
    }
  }
}

// Cholesky factor inverse W = L^-1 (kFull false: lower blocks of WS, zeros
// above the diagonal inside the diagonal blocks, upper blocks untouched) or
// Sigma^-1 = W^H W (kFull true: full and exactly Hermitian) of the packed
// HPD matrix `sigma`, column-major with pitch Lp + 1 in WS.  Returns false
// (uniformly across the workgroups of an instance) if a pivot is not
// positive and finite.  scr: per-wavefront 16x16 staging; s_pd: Lp / 16
// ints of LDS.
// With delta != null, the wavefronts that wait for the first diagonal block
// also write Sigma - SigmaHat (SigmaHat: L x L column-major in HBM, zero
// beyond L) into delta, full, column-major with pitch Lp + 1.
template <int LP, int THREADS, bool kFull>
__device__ __forceinline__ bool invert_hpd(const float2 *sigma, float2 *WS, float2 *scr, int *s_pd, int it,
                                           float2 *delta = nullptr, const float2 *shat = nullptr, int L = 0) {
  constexpr int kWaves = THREADS / 64, Lb = LP / 16, NB = Lb * (Lb + 1) / 2, P = LP + 1, E = NB * 256;
  constexpr int kBlocksPerWave = (NB + kWaves - 1) / kWaves;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, l16 = lane & 15, lq = lane >> 4;
  (void)it;
  // C1. Blocked Cholesky Sigma = L L^H with the diagonal blocks of W = L^-1.
  // Block step J: wavefront 0 has factored diagonal block J in registers
  // and left W_JJ in its place; the panel L_IJ = A_IJ W_JJ^H follows on
  // MFMA, then the trailing updates A_IK -= L_IJ L_KJ^H, during which
  // wavefront 0 updates block J+1 first and factors it.
  for (int e = tid; e < E; e += THREADS) {
    const int b = e >> 8, jj = (e & 255) >> 4, ii = e & 15;
    int I, J;
    blk_coords(b, I, J);
    WS[(16 * J + jj) * P + 16 * I + ii] = ldg2(sigma, e);
  }
  __syncthreads();
  if (wave == 0) {
    const bool ok = leaf_chol(WS, P, lane);
    if (lane == 0) s_pd[0] = ok ? 1 : 0;
  } else if (delta) {
    // from the packed copy (wavefront 0 overwrites block (0, 0) of WS); four
    // elements per thread with their loads in flight together
    constexpr int kU = 4, nt = THREADS - 64;
    for (int e0 = tid - 64; e0 < LP * LP; e0 += kU * nt) {
      float2 sg[kU], sh[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int e = e0 + u * nt;
        sg[u] = sh[u] = make_float2(0.f, 0.f);
        if (e < LP * LP) {
          const int k = e / LP, i = e - k * LP;   // column k, row i
          const int I = i >> 4, K = k >> 4;
          if (I >= K) {
            sg[u] = ldg2(sigma, blk_index(I, K) * 256 + (k & 15) * 16 + (i & 15));
          } else {
            const float2 t = ldg2(sigma, blk_index(K, I) * 256 + (i & 15) * 16 + (k & 15));
            sg[u] = make_float2(t.x, -t.y);
          }
          if (i < L && k < L) sh[u] = ldg2(shat, (size_t)k * L + i);
        }
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int e = e0 + u * nt;
        if (e < LP * LP) {
          const int k = e / LP, i = e - k * LP;
          delta[k * P + i] = make_float2(sg[u].x - sh[u].x, sg[u].y - sh[u].y);
        }
      }
    }
  }
  __syncthreads();
  // Row J of W (W_JK = -W_JJ sum_{M=K..J-1} L_JM W_MK, K < J) is computed in
  // step J by the wavefronts that do not factor the next leaf, after their
  // trailing updates: W_JJ is that step's leaf, L_JM is final and the rows
  // of W above are in place.  Each such block is held in registers and
  // written over L_JK after the step's closing barrier (L_JK is read by
  // the row's other blocks until then, and by nothing later).
  auto w_row_block = [&](int Jr, int K, f4 &wr, f4 &wi) {
    f4 tr = {0.f, 0.f, 0.f, 0.f}, ti = {0.f, 0.f, 0.f, 0.f};
    for (int M = K; M < Jr; ++M)
      cblock_mma(WS + (16 * M) * P + 16 * Jr, WS + (16 * K) * P + 16 * M, P, l16, lq, tr, ti);
    float2 *T = scr + wave * 256;          // column-major, pitch 16
#pragma unroll
    for (int v = 0; v < 4; ++v) T[l16 * 16 + 4 * lq + v] = make_float2(tr[v], ti[v]);
    wave_lds_sync();
    float2 a[4], b[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const float2 w = WS[(16 * Jr + 4 * ks + lq) * P + 16 * Jr + l16];   // W_JJ[l16][k]
      a[ks] = make_float2(-w.x, -w.y);
      b[ks] = T[l16 * 16 + 4 * ks + lq];                                   // T[k][l16]
    }
    wr = (f4){0.f, 0.f, 0.f, 0.f};
    wi = (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) cmfma(a[ks], b[ks], wr, wi);
    wave_lds_sync();
  };
  auto w_store = [&](int Jr, int K, const f4 &wr, const f4 &wi) {
#pragma unroll
    for (int v = 0; v < 4; ++v) WS[(16 * K + l16) * P + 16 * Jr + 4 * lq + v] = make_float2(wr[v], wi[v]);
  };
  for (int J = 0; J < Lb; ++J) {
    PSCA_SUB_MARK(it, J, 0);
    if (!s_pd[J]) return false;   // uniform: every workgroup factors the same Sigma
    if (J + 1 == Lb) break;
    for (int I = J + 1 + wave; I < Lb; I += kWaves) chol_panel(WS, P, J, I, l16, lq);
    __syncthreads();
    PSCA_SUB_MARK(it, J, 1);
    int wk = -1;                  // the block K < J of W's row J this wavefront holds
    f4 wr, wi;
    if (wave == 0) {
      chol_trail(WS, P, J, J + 1, J + 1, l16, lq);
      wave_lds_sync();
      PSCA_SUB_MARK(it, J, 2);
      const bool ok = leaf_chol(WS + 16 * (J + 1) * P + 16 * (J + 1), P, lane);
      if (lane == 0) s_pd[J + 1] = ok ? 1 : 0;
      PSCA_SUB_MARK(it, J, 3);
    } else {
      int q = 0;
      for (int I = J + 2; I < Lb; ++I)
        for (int K = J + 1; K <= I; ++K)
          if (q++ % (kWaves - 1) == wave - 1) chol_trail(WS, P, J, I, K, l16, lq);
      for (int K = 0; K < J; ++K)
        if ((q + K) % (kWaves - 1) == wave - 1) {
          w_row_block(J, K, wr, wi);
          wk = K;
        }
    }
    __syncthreads();
    if (wk >= 0) w_store(J, wk, wr, wi);
  }
  PSCA_MARK(it, 5);
  // The last row of W, then W is complete.
  if (Lb > 1) {
    int wk = -1;
    f4 wr, wi;
    for (int K = wave; K < Lb - 1; K += kWaves) {
      w_row_block(Lb - 1, K, wr, wi);
      wk = K;
    }
    __syncthreads();
    if (wk >= 0) w_store(Lb - 1, wk, wr, wi);
    __syncthreads();
  }
  // C3. Sigma^-1 = W^H W (MFMA), stored full column-major in WS.
  PSCA_MARK(it, 6);
  if constexpr (!kFull) return true;
  f4 sir[kBlocksPerWave], sii[kBlocksPerWave];
#pragma unroll
  for (int q = 0; q < kBlocksPerWave; ++q) {
    sir[q] = (f4){0.f, 0.f, 0.f, 0.f};
    sii[q] = (f4){0.f, 0.f, 0.f, 0.f};
    const int b = wave + kWaves * q;
    if (b < NB) {
      int I, J;
      blk_coords(b, I, J);
      for (int K = I; K < Lb; ++K) {       // A[i][k] = conj(W[k][i]), B[k][j] = W[k][j]
        float2 a4[4], b4[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const int k = 16 * K + 4 * ks + lq;
          const float2 wi = WS[(16 * I + l16) * P + k];
          a4[ks] = make_float2(wi.x, -wi.y);
          b4[ks] = WS[(16 * J + l16) * P + k];
        }
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) cmfma(a4[ks], b4[ks], sir[q], sii[q]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kBlocksPerWave; ++q) {
    const int b = wave + kWaves * q;
    if (b < NB) {
      int I, J;
      blk_coords(b, I, J);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * I + 4 * lq + v, j = 16 * J + l16;
        if (i >= j) {
          const float im = (i == j) ? 0.0f : sii[q][v];
          WS[j * P + i] = make_float2(sir[q][v], im);
          WS[i * P + j] = make_float2(sir[q][v], -im);
        }
      }
    }
  }
  __syncthreads();
  return true;
}

// One detection on workgroup g of the G workgroups the instance owns.
template <int LPMAX, int THREADS>
__device__ __forceinline__ void psca_body(const CoopArgs &A, const int g) {
  constexpr int kWaves = THREADS / 64;
  constexpr int Lp = LPMAX, Lb = LPMAX / kBlk;                          // padded pilot length
  constexpr int P = Lp + 1;                                             // pitch of the L x L LDS matrix
  constexpr bool kShLds = LPMAX <= 64;                                  // SigmaHat resident in LDS
  extern __shared__ float4 smem_raw[];
  __shared__ int s_ok, s_pd[LPMAX / 16];
  const int NT = A.NT, PT = A.NT + 1;
  float2 *St = (float2 *)smem_raw;          // [Lp][PT]  S tile, row i at i * PT
  constexpr int kBW = b_tile_blocks(LPMAX); // 16-column blocks per round of C4
  constexpr int kTPW = (Lb * kBW + kWaves - 1) / kWaves;   // C4 tasks per wavefront
  constexpr int kPB = 16 * kBW + 1;         // pitch of the B tile
  float2 *Bt = St + Lp * PT;                // [Lp][kPB] B tile of kBW 16-column blocks
  float2 *WS = Bt + Lp * kPB;               // [Lp][P]   column-major: Cholesky factor, W, Sigma^-1
  float2 *ShL = WS + Lp * P;                // [Lp][P]   Sigma - SigmaHat of the iteration (kShLds)
  float2 *scr = ShL + (kShLds ? Lp * P : 0);// [kWaves][256] per-wave 16x16 scratch
  float *xs = (float *)(scr + kWaves * 256);   // [NT] iterate of the tile
  float *gs = xs + NT;                      // [NT] pathloss
  float *ls = gs + NT;                      // [NT] log(p / (1 - p))
  float *red_q = ls + NT;                   // [Lb][NT]
  float *red_r = red_q + Lb * NT;           // [Lb][NT]

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, lq = lane >> 4;
  const int n0 = g * NT;
  unsigned gen = 0;
  const bool known = (A.a.variant == PSCA_ML_K || A.a.variant == PSCA_MAP_K || A.a.variant == PSCA_MAP_K2);
  const bool pairs = (A.a.variant == PSCA_MAP_K2);

  // ---- resident tile data -------------------------------------------------
  for (int e = tid; e < Lp * NT; e += THREADS) {
    const int c = e / Lp, i = e - c * Lp;   // walk down a column: coalesced reads
    const int n = n0 + c;
    St[i * PT + c] = (i < A.L && n < A.N) ? A.S[(size_t)n * A.L + i] : make_float2(0.f, 0.f);
  }
  for (int c = tid; c < NT; c += THREADS) {
    const int n = n0 + c;
    const bool in = n < A.N;
    xs[c] = (in && A.x_in) ? A.x_in[n] : 0.0f;
    if (in && A.x_hist) A.x_hist[n] = xs[c];
    gs[c] = (in && A.a.g) ? A.a.g[n] : 0.0f;
    float lg = 0.0f;
    if (in && A.a.p) {
      const float pn = A.a.p[n];
      lg = logf(pn / (1.0f - pn));
    }
    if (in && pairs) {
      lg = A.a.c1[n];
      A.a.xg[n] = xs[c];   // x^(0), read after the first barrier
    }
    ls[c] = lg;
  }

  double rho_d = A.rho0;
  bool failed = false, aborted = false;
  int it = 0;
  for (; it < A.iters; ++it) {
    PSCA_MARK(it, 0);
    // ===== A. partial of Sigma from this tile =============================
    for (int c = tid; c < NT; c += THREADS)   // weights w_c
      red_q[c] = known ? gs[c] * xs[c] : xs[c];
    __syncthreads();
    tile_gram<Lp, THREADS>(St, PT, A.ncb, red_q, A.partials + (size_t)g * A.pstride);
    PSCA_MARK(it, 1);
    if (!grid_sync(A.bar, A.G, g, gen, &s_ok)) { aborted = true; break; }

    // ===== B. reduce a slice of the partials into Sigma ===================
    PSCA_MARK(it, 2);
    reduce_slice<Lp, THREADS>(A.partials, A.pstride, A.G, g, A.sigma, (double2 *)scr, true, A.L, A.sigma2);
    PSCA_MARK(it, 3);
    if (!grid_sync(A.bar, A.G, g, gen, &s_ok)) { aborted = true; break; }

    // ===== C1-C2. W = L^-1 of the blocked Cholesky factor Sigma = L L^H ======
    PSCA_MARK(it, 4);
    if (!invert_hpd<Lp, THREADS, false>(A.sigma, WS, scr, s_pd, it, kShLds ? ShL : nullptr, A.Sh, A.L)) {
      failed = true;
      break;
    }

    // ===== C4. Y = W S_t (q = |y|^2), B = W^H Y = Sigma^-1 S_t,
    // q - r = b^H (Sigma - SigmaHat) b ========================================
    // One 16-column block of the tile at a time (the B tile is Lp x 16).  q
    // as a sum of squares and q - r in the difference form keep their
    // relative accuracy for weak devices, whose q is small next to
    // ||Sigma^-1||.
    PSCA_MARK(it, 7);
    // Up to kBW column blocks per round, one (block row, column block) task
    // per wavefront.
    for (int cb0 = 0; cb0 < A.ncb; cb0 += kBW) {
      const int nb = min(kBW, A.ncb - cb0), ntask = Lb * nb;
#pragma unroll
      for (int j = 0; j < kTPW; ++j) {   // Y = W S (lower triangular W)
        const int t = wave + kWaves * j;
        if (t < ntask) {
          const int I = t / nb, c = t - I * nb;
          f4 cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
          for (int K = 0; K <= I; ++K)
            cblock_mma_rm(WS + 16 * I, P, St + 16 * (cb0 + c), PT, 16 * K, l16, lq, cr, ci);
          float qp = 0.0f;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            qp += cr[v] * cr[v] + ci[v] * ci[v];
            Bt[(16 * I + 4 * lq + v) * kPB + 16 * c + l16] = make_float2(cr[v], ci[v]);
          }
          qp += __shfl_xor(qp, 16);
          qp += __shfl_xor(qp, 32);
          if (lq == 0) red_q[I * NT + 16 * (cb0 + c) + l16] = qp;
        }
      }
      __syncthreads();
      {   // B = W^H Y, in registers until every wavefront has read Y
        f4 br[kTPW], bi[kTPW];
#pragma unroll
        for (int j = 0; j < kTPW; ++j) {
          br[j] = (f4){0.f, 0.f, 0.f, 0.f};
          bi[j] = (f4){0.f, 0.f, 0.f, 0.f};
          const int t = wave + kWaves * j;
          if (t < ntask) {
            const int I = t / nb, c = t - I * nb;
            for (int K = I; K < Lb; ++K) {   // A[i][k] = conj(W[k][i])
              float2 a4[4], b4[4];
#pragma unroll
              for (int ks = 0; ks < 4; ++ks) {
                const int k = 16 * K + 4 * ks + lq;
                const float2 wv = WS[(16 * I + l16) * P + k];
                a4[ks] = make_float2(wv.x, -wv.y);
                b4[ks] = Bt[k * kPB + 16 * c + l16];
              }
#pragma unroll
              for (int ks = 0; ks < 4; ++ks) cmfma(a4[ks], b4[ks], br[j], bi[j]);
            }
          }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kTPW; ++j) {
          const int t = wave + kWaves * j;
          if (t < ntask) {
            const int I = t / nb, c = t - I * nb;
#pragma unroll
            for (int v = 0; v < 4; ++v)
              Bt[(16 * I + 4 * lq + v) * kPB + 16 * c + l16] = make_float2(br[j][v], bi[j][v]);
          }
        }
        __syncthreads();
      }
#pragma unroll
      for (int j = 0; j < kTPW; ++j) {
        const int t = wave + kWaves * j;
        if (t < ntask) {
          const int I = t / nb, c = t - I * nb;
          // D' = (Sigma - SigmaHat) B: then b^H D' = q - r with an error that
          // scales with Sigma - SigmaHat (small near a stationary point)
          // rather than with q and r themselves.  Sigma from its packed
          // lower blocks (diagonal blocks are stored whole).
          f4 cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
          if constexpr (kShLds) {   // ShL holds Sigma - SigmaHat for this iteration
#pragma unroll
            for (int K = 0; K < Lb; ++K) cblock_mma_rm(ShL + 16 * I, P, Bt + 16 * c, kPB, 16 * K, l16, lq, cr, ci);
          } else {
#pragma unroll
            for (int K = 0; K < Lb; ++K) {
              float2 a4[4], b4[4];
#pragma unroll
              for (int ks = 0; ks < 4; ++ks) {
                const int i = 16 * I + l16, k = 16 * K + 4 * ks + lq;
                float2 sg;
                if (I >= K) {
                  sg = A.sigma[blk_index(I, K) * 256 + (k & 15) * 16 + (i & 15)];
                } else {
                  const float2 t2 = A.sigma[blk_index(K, I) * 256 + (i & 15) * 16 + (k & 15)];
                  sg = make_float2(t2.x, -t2.y);
                }
                const float2 sh = (i < A.L && k < A.L) ? A.Sh[(size_t)k * A.L + i] : make_float2(0.f, 0.f);
                a4[ks] = make_float2(sg.x - sh.x, sg.y - sh.y);
                b4[ks] = Bt[k * kPB + 16 * c + l16];
              }
#pragma unroll
              for (int ks = 0; ks < 4; ++ks) cmfma(a4[ks], b4[ks], cr, ci);
            }
          }
          float rp = 0.0f;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const float2 bv = Bt[(16 * I + 4 * lq + v) * kPB + 16 * c + l16];
            rp += bv.x * cr[v] + bv.y * ci[v];
          }
          rp += __shfl_xor(rp, 16);
          rp += __shfl_xor(rp, 32);
          if (lq == 0) red_r[I * NT + 16 * (cb0 + c) + l16] = rp;
        }
      }
      __syncthreads();
    }

    // ===== C5. coordinate step and update ==================================
    PSCA_MARK(it, 9);
    float rho;
    if (A.rho_fixed >= 0.0f) rho = A.rho_fixed;
    else if (A.rho_dev) rho = A.rho_dev[it];
    else rho = (float)rho_d;
    rho_d = rho_d * (1.0 - A.rho_decay * rho_d);
    const bool last = (it == A.iters - 1);
    for (int c = tid; c < NT; c += THREADS) {
      const int n = n0 + c;
      if (n < A.N) {
        float q = 0.0f, qmr = 0.0f;
        for (int I = 0; I < Lb; ++I) {
          q += red_q[I * NT + c];
          qmr += red_r[I * NT + c];
        }
        const float x = xs[c];
        // MAP-K2: x^(k) of every device is in half k % 2 of the exchange
        // buffer (written before this iteration's barriers); x^(k+1) goes to
        // the other half, which no workgroup reads before the next barriers.
        const float prior = pairs ? ls[c] + pair_sum(A.a, n, A.N, A.a.xg + (size_t)(it & 1) * A.N) : ls[c];
        const float xt = coordinate_step(x, q, qmr, gs[c], prior, A.a);
        xs[c] = (1.0f - rho) * x + rho * xt;
        if (pairs) A.a.xg[(size_t)((it + 1) & 1) * A.N + n] = xs[c];
        if (A.x_hist) A.x_hist[(size_t)(it + 1) * A.N + n] = xs[c];
        if (last) {
          if (A.q_out) A.q_out[n] = q;
          if (A.r_out) A.r_out[n] = q - qmr;
          if (A.xt_out) A.xt_out[n] = xt;
        }
      }
    }
    __syncthreads();
    PSCA_MARK(it, 10);
  }

  // ---- results --------------------------------------------------------------
  for (int c = tid; c < NT; c += THREADS) {
    const int n = n0 + c;
    if (n < A.N) A.x_out[n] = xs[c];
  }
  if (g == 0 && tid == 0 && A.status)
    *A.status = aborted ? PSCA_ESYNC : (failed ? PSCA_ENOTPD : PSCA_OK);
}

// ---------------------------------------------------------------------------
// Backward of one unrolled layer x' = (1 - rho) x + rho x~(x)
// ---------------------------------------------------------------------------
// Given v = dL/dx', with a_n = rho v_n mask_n d pre_n/dq_n and
// b_n = rho v_n mask_n d pre_n/dr_n, G_a = S diag(a) S^H, G_b = S diag(b) S^H,
// b_m = Sigma^-1 s_m and c_m = Sigma^-1 SigmaHat Sigma^-1 s_m:
//   dL/dx_m = v_m (1 - rho) + rho v_m mask_m own_m
//             - kappa_m (b_m^H G_a b_m + 2 Re c_m^H G_b b_m),
//   dL/drho = sum_n v_n (x~_n - x_n),
// from dSigma^-1 = -Sigma^-1 s_m s_m^H Sigma^-1 dw_m (w = kappa x).
// Sigma^-1 is recomputed from x, not stored by the forward pass.
struct BackArgs {
  CoopArgs c;           // instance, tile plan, x_in = the layer's input, work buffers, barrier
  float *grad_rho;      // dL/drho (batched launches sum rho_part into it)
  float rho;
  const float *v;       // [N] dL/dx'
  float *grad_x;        // [N] dL/dx
  float *rho_part;      // [G] per-workgroup parts of dL/drho
  float2 *partials_b;   // [G][pstride] partials of G_b (those of G_a use c.partials)
  float2 *gram_a, *gram_b;   // packed G_a, G_b
};

// LDS footprint of the backward body (Lp <= 64, SigmaHat resident).  At
// Lp = 64 the per-wavefront scratch shares the B and C tiles (see the body).
__host__ __device__ inline size_t lds_back_bytes(int Lp, int NT, int waves) {
  const size_t pt = (size_t)NT + 1, P = (size_t)Lp + 1, Lb = (size_t)Lp / 16;
  const size_t scr = Lp == 64 ? 0 : (size_t)waves * 256;
  const size_t f2 = 3 * (size_t)Lp * pt + (size_t)Lp * 17 + 2 * (size_t)Lp * P + scr;
  const size_t fl = 7 * (size_t)NT + 2 * Lb * NT + (size_t)waves;
  return f2 * sizeof(float2) + fl * 4;
}

// Packed Hermitian -> full column-major (pitch P) in LDS.
template <int LP, int THREADS>
__device__ __forceinline__ void unpack_hermitian(const float2 *packed, float2 *M) {
  constexpr int Lb = LP / 16, E = Lb * (Lb + 1) / 2 * 256, P = LP + 1;
  for (int e = threadIdx.x; e < E; e += THREADS) {
    const int b = e >> 8, jj = (e & 255) >> 4, ii = e & 15;
    int I, J;
    blk_coords(b, I, J);
    const float2 v = packed[e];
    M[(16 * J + jj) * P + 16 * I + ii] = v;
    if (I != J) M[(16 * I + ii) * P + 16 * J + jj] = make_float2(v.x, -v.y);
  }
}

template <int LP, int THREADS>
__device__ __forceinline__ void psca_back_body(const BackArgs &Bk, const int g) {
  const CoopArgs &A = Bk.c;
  constexpr int kWaves = THREADS / 64;
  constexpr int Lp = LP, Lb = LP / 16, P = Lp + 1, kPB = 17;
  constexpr int kRowBlocksPerWave = (Lb + kWaves - 1) / kWaves;
  static_assert(LP <= 64, "the backward body keeps SigmaHat and two Gram matrices in LDS");
  extern __shared__ float4 smem_raw[];
  __shared__ int s_ok, s_pd[LP / 16];
  const int NT = A.NT, PT = A.NT + 1;
  float2 *St = (float2 *)smem_raw;     // [Lp][PT] S tile
  float2 *Bf = St + Lp * PT;           // [Lp][PT] Sigma^-1 S tile
  float2 *Cf = Bf + Lp * PT;           // [Lp][PT] Sigma^-1 SigmaHat Sigma^-1 S tile
  float2 *Dt = Cf + Lp * PT;           // [Lp][kPB] SigmaHat B of one 16-column block
  float2 *WS = Dt + Lp * kPB;          // [Lp][P] Sigma^-1, then G_a
  float2 *ShL = WS + Lp * P;           // [Lp][P] SigmaHat, then G_b
  // [kWaves][256] scratch of the first reduction and the factorisation.  At
  // Lp = 64 it lives in the B and C tiles, which are first written after the
  // factorisation (2 Lp PT >= kWaves 256 for PT >= 17), and the two Gram
  // reductions, while B and C are live, use Dt (Lp kPB float2 >= THREADS
  // double2), which is dead after the tile products: this frees the 16 KiB
  // that let the tile grow to 48 columns.
  constexpr bool kShareScr = LP == 64;
  static_assert(!kShareScr || (2 * LP * 17 >= kWaves * 256 && LP * kPB * 8 >= THREADS * 16), "scratch fits");
  float2 *scr = kShareScr ? Bf : ShL + Lp * P;
  double2 *gscr = (double2 *)(kShareScr ? Dt : scr);
  float *xs = (float *)(ShL + Lp * P + (kShareScr ? 0 : kWaves * 256));
  float *gs = xs + NT, *ls = gs + NT, *vs = ls + NT, *aw = vs + NT, *bw = aw + NT, *dxo = bw + NT;
  float *red_q = dxo + NT;             // [Lb][NT]
  float *red_r = red_q + Lb * NT;      // [Lb][NT]
  float *s_red = red_r + Lb * NT;      // [kWaves]

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, l16 = lane & 15, lq = lane >> 4;
  const int n0 = g * NT;
  unsigned gen = 0;
  const bool known = (A.a.variant == PSCA_ML_K || A.a.variant == PSCA_MAP_K);

  for (int e = tid; e < Lp * NT; e += THREADS) {
    const int c = e / Lp, i = e - c * Lp;
    const int n = n0 + c;
    St[i * PT + c] = (i < A.L && n < A.N) ? A.S[(size_t)n * A.L + i] : make_float2(0.f, 0.f);
  }
  for (int c = tid; c < NT; c += THREADS) {
    const int n = n0 + c;
    const bool in = n < A.N;
    xs[c] = in ? A.x_in[n] : 0.0f;
    gs[c] = (in && A.a.g) ? A.a.g[n] : 0.0f;
    float lg = 0.0f;
    if (in && A.a.p) {
      const float pn = A.a.p[n];
      lg = logf(pn / (1.0f - pn));
    }
    ls[c] = lg;
    vs[c] = in ? Bk.v[n] : 0.0f;
  }
  for (int e = tid; e < Lp * Lp; e += THREADS) {
    const int k = e / Lp, i = e - k * Lp;
    ShL[k * P + i] = (i < A.L && k < A.L) ? A.Sh[(size_t)k * A.L + i] : make_float2(0.f, 0.f);
  }
  bool failed = false, aborted = false;
  do {
    // Sigma(x) and its inverse, as in the forward pass
    for (int c = tid; c < NT; c += THREADS) red_q[c] = known ? gs[c] * xs[c] : xs[c];
    __syncthreads();
    tile_gram<Lp, THREADS>(St, PT, A.ncb, red_q, A.partials + (size_t)g * A.pstride);
    if (!grid_sync(A.bar, A.G, g, gen, &s_ok)) { aborted = true; break; }
    reduce_slice<Lp, THREADS>(A.partials, A.pstride, A.G, g, A.sigma, (double2 *)scr, true, A.L, A.sigma2);
    if (!grid_sync(A.bar, A.G, g, gen, &s_ok)) { aborted = true; break; }
    if (!invert_hpd<Lp, THREADS, true>(A.sigma, WS, scr, s_pd, 0)) { failed = true; break; }

    // B = Sigma^-1 S_t (q), D = SigmaHat B (r), C = Sigma^-1 D, per 16-column block
    for (int cb = 0; cb < A.ncb; ++cb) {
#pragma unroll
      for (int rb = 0; rb < kRowBlocksPerWave; ++rb) {
        const int I = wave + kWaves * rb;
        if (I < Lb) {
          f4 cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int K = 0; K < Lb; ++K) cblock_mma_rm(WS + 16 * I, P, St + 16 * cb, PT, 16 * K, l16, lq, cr, ci);
          float qp = 0.0f;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = 16 * I + 4 * lq + v, j = 16 * cb + l16;
            const float2 sv = St[i * PT + j];
            qp += sv.x * cr[v] + sv.y * ci[v];
            Bf[i * PT + j] = make_float2(cr[v], ci[v]);
          }
          qp += __shfl_xor(qp, 16);
          qp += __shfl_xor(qp, 32);
          if (lq == 0) red_q[I * NT + 16 * cb + l16] = qp;
        }
      }
      __syncthreads();
#pragma unroll
      for (int rb = 0; rb < kRowBlocksPerWave; ++rb) {
        const int I = wave + kWaves * rb;
        if (I < Lb) {
          f4 cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int K = 0; K < Lb; ++K) cblock_mma_rm(ShL + 16 * I, P, Bf + 16 * cb, PT, 16 * K, l16, lq, cr, ci);
          float rp = 0.0f;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = 16 * I + 4 * lq + v;
            const float2 bv = Bf[i * PT + 16 * cb + l16];
            rp += bv.x * cr[v] + bv.y * ci[v];
            Dt[i * kPB + l16] = make_float2(cr[v], ci[v]);
          }
          rp += __shfl_xor(rp, 16);
          rp += __shfl_xor(rp, 32);
          if (lq == 0) red_r[I * NT + 16 * cb + l16] = rp;
        }
      }
      __syncthreads();
#pragma unroll
      for (int rb = 0; rb < kRowBlocksPerWave; ++rb) {
        const int I = wave + kWaves * rb;
        if (I < Lb) {
          f4 cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int K = 0; K < Lb; ++K) cblock_mma_rm(WS + 16 * I, P, Dt, kPB, 16 * K, l16, lq, cr, ci);
#pragma unroll
          for (int v = 0; v < 4; ++v) Cf[(16 * I + 4 * lq + v) * PT + 16 * cb + l16] = make_float2(cr[v], ci[v]);
        }
      }
      __syncthreads();
    }

    // per device: step derivatives, the weights a, b and the direct term
    float rho_term = 0.0f;
    for (int c = tid; c < NT; c += THREADS) {
      float a_c = 0.0f, b_c = 0.0f, d_c = 0.0f;
      if (n0 + c < A.N) {
        float q = 0.0f, r = 0.0f;
        for (int I = 0; I < Lb; ++I) {
          q += red_q[I * NT + c];
          r += red_r[I * NT + c];
        }
        const StepDerivs d = step_derivs(xs[c], q, r, gs[c], ls[c], A.a);
        const float rv = Bk.rho * vs[c] * d.mask;
        a_c = rv * d.dq;
        b_c = rv * d.dr;
        d_c = vs[c] * (1.0f - Bk.rho) + rv * d.own;
        rho_term += vs[c] * (d.xt - xs[c]);
        gs[c] = d.kappa;   // kappa replaces g from here on
      }
      aw[c] = a_c;
      bw[c] = b_c;
      dxo[c] = d_c;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) rho_term += __shfl_xor(rho_term, o);
    if (lane == 0) s_red[wave] = rho_term;
    __syncthreads();
    if (tid == 0) {
      float t = 0.0f;
      for (int w = 0; w < kWaves; ++w) t += s_red[w];
      Bk.rho_part[g] = t;
    }

    // G_a and G_b
    tile_gram<Lp, THREADS>(St, PT, A.ncb, aw, A.partials + (size_t)g * A.pstride);
    tile_gram<Lp, THREADS>(St, PT, A.ncb, bw, Bk.partials_b + (size_t)g * A.pstride);
    if (!grid_sync(A.bar, A.G, g, gen, &s_ok)) { aborted = true; break; }
    reduce_slice<Lp, THREADS>(A.partials, A.pstride, A.G, g, Bk.gram_a, gscr, false, A.L, 0.0f);
    __syncthreads();
    reduce_slice<Lp, THREADS>(Bk.partials_b, A.pstride, A.G, g, Bk.gram_b, gscr, false, A.L, 0.0f);
    if (!grid_sync(A.bar, A.G, g, gen, &s_ok)) { aborted = true; break; }
    unpack_hermitian<Lp, THREADS>(Bk.gram_a, WS);
    unpack_hermitian<Lp, THREADS>(Bk.gram_b, ShL);
    __syncthreads();

    // t1 = Re b^H G_a b, t2 = Re c^H G_b b, per device
    for (int cb = 0; cb < A.ncb; ++cb) {
#pragma unroll
      for (int rb = 0; rb < kRowBlocksPerWave; ++rb) {
        const int I = wave + kWaves * rb;
        if (I < Lb) {
          f4 ar = {0.f, 0.f, 0.f, 0.f}, ai = {0.f, 0.f, 0.f, 0.f};
          f4 br = {0.f, 0.f, 0.f, 0.f}, bi = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int K = 0; K < Lb; ++K) {
            cblock_mma_rm(WS + 16 * I, P, Bf + 16 * cb, PT, 16 * K, l16, lq, ar, ai);
            cblock_mma_rm(ShL + 16 * I, P, Bf + 16 * cb, PT, 16 * K, l16, lq, br, bi);
          }
          float t1 = 0.0f, t2 = 0.0f;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = 16 * I + 4 * lq + v, j = 16 * cb + l16;
            const float2 bv = Bf[i * PT + j], cv = Cf[i * PT + j];
            t1 += bv.x * ar[v] + bv.y * ai[v];
            t2 += cv.x * br[v] + cv.y * bi[v];
          }
          t1 += __shfl_xor(t1, 16);
          t1 += __shfl_xor(t1, 32);
          t2 += __shfl_xor(t2, 16);
          t2 += __shfl_xor(t2, 32);
          if (lq == 0) {
            red_q[I * NT + 16 * cb + l16] = t1;
            red_r[I * NT + 16 * cb + l16] = t2;
          }
        }
      }
    }
    __syncthreads();
    for (int c = tid; c < NT; c += THREADS) {
      const int n = n0 + c;
      if (n < A.N) {
        float t1 = 0.0f, t2 = 0.0f;
        for (int I = 0; I < Lb; ++I) {
          t1 += red_q[I * NT + c];
          t2 += red_r[I * NT + c];
        }
        Bk.grad_x[n] = dxo[c] - gs[c] * (t1 + 2.0f * t2);
      }
    }
  } while (false);
  if (g == 0 && tid == 0 && A.status) *A.status = aborted ? PSCA_ESYNC : (failed ? PSCA_ENOTPD : PSCA_OK);
}

template <int LP>
__global__ void __launch_bounds__(512) k_psca_back(BackArgs Bk) {
  psca_back_body<LP, 512>(Bk, blockIdx.x);
}

// Logical workgroup index under which consecutive indices share an XCD.
// Workgroup b of a launch goes to XCD b mod 8, so the first 8 floor(n/8)
// workgroups are renumbered XCD-major and the rest keep their index: a team
// of consecutive logical indices then spans as few XCDs (and L2 caches) as
// its size allows, and its barrier's cache write-backs and invalidations
// meet fewer other teams' data.
__device__ __forceinline__ int xcd_major(int b, int n) {
  constexpr int kXcds = 8;
  const int q = n / kXcds;
  return b >= q * kXcds ? b : (b % kXcds) * q + b / kXcds;
}

// Batched layer backward: teams of T workgroups work through their lists of
// instances as k_psca_teams does (every member takes part in every instance
// of its team; tiles past N are empty).
template <int LP>
__device__ __noinline__ void back_member(const BackArgs *__restrict__ desc, int g) {
  psca_back_body<LP, 512>(*desc, g);
}

#ifdef PSCA_TU_MAIN
__global__ void __launch_bounds__(512) k_psca_back_teams(const BackArgs *__restrict__ descs,
                                                         const int *__restrict__ lists,
                                                         const int *__restrict__ offsets, int T) {
  const int b = xcd_major((int)blockIdx.x, (int)gridDim.x);
  const int t = b / T, g = b - t * T;
  const int i1 = offsets[t + 1];
  for (int idx = offsets[t]; idx < i1; ++idx) {
    const BackArgs *desc = descs + lists[idx];
    if (g < desc->c.G) {
      switch ((desc->c.L + 15) & ~15) {
        case 16: back_member<16>(desc, g); break;
        case 32: back_member<32>(desc, g); break;
        case 48: back_member<48>(desc, g); break;
        default: back_member<64>(desc, g); break;
      }
    }
    __syncthreads();   // the next instance reuses the LDS
  }
}
#endif

// Barrier words and status of every instance of a batched backward.
#ifdef PSCA_TU_MAIN
__global__ void k_prepare_back_batch(const BackArgs *__restrict__ descs) {
  const CoopArgs &A = descs[blockIdx.x].c;
  for (int w = threadIdx.x; w < A.G; w += blockDim.x) A.bar.arrive[w * 16] = 0u;
  if (threadIdx.x == 0) {
    *A.bar.release = 0u;
    *A.bar.abort_flag = 0;
    *A.status = PSCA_OK;
  }
}
#endif

// dL/drho of every instance: the sum of its workgroups' parts (one block each).
#ifdef PSCA_TU_MAIN
__global__ void k_sum_parts_batch(const BackArgs *__restrict__ descs) {
  __shared__ float sh[256];
  const BackArgs &d = descs[blockIdx.x];
  float t = 0.0f;
  for (int i = threadIdx.x; i < d.c.G; i += blockDim.x) t += d.rho_part[i];
  sh[threadIdx.x] = t;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *d.grad_rho = sh[0];
}
#endif

// dL/drho = the sum of the per-workgroup parts (one workgroup)
#ifdef PSCA_TU_MAIN
__global__ void k_sum_parts(const float *__restrict__ parts, int G, float *__restrict__ out) {
  __shared__ float sh[256];
  float t = 0.0f;
  for (int i = threadIdx.x; i < G; i += blockDim.x) t += parts[i];
  sh[threadIdx.x] = t;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}
#endif

// Pilot lengths 97..256: the L x L matrices no longer fit a workgroup's LDS
// beside an S tile, so Sigma, its factor L and Sigma - SigmaHat live in
// device memory (packed lower 16x16 blocks) and the factorisation is spread
// over the instance's team of workgroups.  Block step J: every workgroup
// factors the diagonal block J redundantly in registers and keeps
// W_JJ = L_JJ^-1 in LDS; the trailing updates A_IK -= L_IJ L_KJ^H are spread
// over all wavefronts of the team, each forming the panel blocks
// L_IJ = A_IJ W_JJ^H it needs, with one team barrier per block step.  The
// solves Y = L^-1 S (q = |y|^2), B = L^-H Y and q - r = b^H (Sigma - SigmaHat) b
// (the difference taken in phase B from the FP64 sum) then run per 16-column
// block in registers (k_psca_large_teams below).

// Touches n float2 at p (16-byte loads spread over `nthreads` threads from
// thread `t`) so that a later pass finds them in this XCD's L2; the loaded
// bits are folded into a register that an empty asm statement consumes.
__device__ __forceinline__ void warm_l2(const float2 *p, int n, int t, int nthreads) {
  const float4 *q = (const float4 *)p;
  unsigned x = 0;
  for (int e = t; e < n / 2; e += nthreads) {
    const float4 v = q[e];
    x ^= __float_as_uint(v.x) ^ __float_as_uint(v.w);
  }
  asm volatile("" ::"v"(x));
}

// FP32 complex 16x16x4 product with three real MFMAs (Gauss): t1 += ar br,
// t2 += ai bi, t3 += (ar + ai)(br + bi); re = t1 - t2, im = t3 - t1 - t2.
__device__ __forceinline__ void cmfma3(float2 a, float2 b, f4 &t1, f4 &t2, f4 &t3) {
  t1 = mfma4(a.x, b.x, t1);
  t2 = mfma4(a.y, b.y, t2);
  t3 = mfma4(a.x + a.y, b.x + b.y, t3);
}

__device__ __forceinline__ const float2 *pblk(const float2 *packed, int I, int J) {
  return packed + (size_t)blk_index(I, J) * 256;
}

// Packed Gram partial S_t diag(w) S_t^H of a tile staged in LDS (Yt
// [Lp][PT], ncb 16-column blocks, weights w[c]) into dst (NB lower 16x16
// blocks of 256 entries, column-major within a block).  FP64 MFMA (the
// FP32 operands' products are exact in FP64), three products per complex
// step (Gauss); the blocks are spread over the waves.
template <int THREADS>
__device__ __forceinline__ void gram_tile_fp64(const float2 *Yt, int PT, int ncb, const float *w, int NB,
                                               float2 *dst) {
  constexpr int kWaves = THREADS / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, l16 = lane & 15, lq = lane >> 4;
  for (int b = wave; b < NB; b += kWaves) {
    int I, J;
    blk_coords(b, I, J);
    d4 t1 = {0.0, 0.0, 0.0, 0.0}, t2 = t1, t3 = t1;
    for (int cb = 0; cb < ncb; ++cb) {
      double2 av4[4], bv4[4];
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int c = 16 * cb + 4 * ks + lq;
        const float2 sv = Yt[(16 * J + l16) * PT + c];
        const float2 av = Yt[(16 * I + l16) * PT + c];
        const double wc = w[c];
        av4[ks] = make_double2(av.x, av.y);
        bv4[ks] = make_double2(wc * sv.x, -wc * sv.y);
      }
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) cmfma_d3(av4[ks], bv4[ks], t1, t2, t3);
    }
    float2 *o = dst + (size_t)b * 256 + l16 * 16 + lq;
#pragma unroll
    for (int v = 0; v < 4; ++v) o[4 * v] = make_float2((float)(t1[v] - t2[v]), (float)(t3[v] - t1[v] - t2[v]));
  }
}

// The same packed Gram partial on FP32 MFMA (twice the FP64 MFMA rate):
// three products per complex step, summed in FP32 over each 16-column chunk
// of the tile, the chunks added in FP64, and each entry combined in FP64 and
// rounded to FP32 once.  Every FP32 sum spans only 16 columns, so the
// entries carry about one FP32 rounding of their magnitude once summed over
// the tiles.  Each wave works on two blocks at a time (b and b + kWaves),
// six independent MFMA chains, so that one block's LDS reads and FP64 sums
// overlap the other's products.  The partials go out as streaming global
// stores: the reduction reads them back after the team barrier.
template <int THREADS, bool kTwo>
__device__ __forceinline__ void gram_blocks_chunked(const float2 *Yc, int CP, int ncb, const float *w, int b0, int b1,
                                                    float2 *dst) {
  const int lane = threadIdx.x & 63, l16 = lane & 15, lq = lane >> 4;
  constexpr int kB = kTwo ? 2 : 1;
  int I[kB], J[kB];
  blk_coords(b0, I[0], J[0]);
  if constexpr (kTwo) blk_coords(b1, I[1], J[1]);
  d4 s1[kB], s2[kB], s3[kB];
#pragma unroll
  for (int q = 0; q < kB; ++q) {
    s1[q] = d4{0.0, 0.0, 0.0, 0.0};
    s2[q] = s1[q];
    s3[q] = s1[q];
  }
  for (int cb = 0; cb < ncb; ++cb) {
    f4 t1[kB], t2[kB], t3[kB];
#pragma unroll
    for (int q = 0; q < kB; ++q) {
      t1[q] = f4{0.f, 0.f, 0.f, 0.f};
      t2[q] = t1[q];
      t3[q] = t1[q];
    }
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int c = 16 * cb + 4 * ks + lq;
      const float wc = w[c];
#pragma unroll
      for (int q = 0; q < kB; ++q) {
        const float2 sv = Yc[c * CP + 16 * J[q] + l16];
        const float2 av = Yc[c * CP + 16 * I[q] + l16];
        cmfma3(av, make_float2(wc * sv.x, -wc * sv.y), t1[q], t2[q], t3[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < kB; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        s1[q][v] += (double)t1[q][v];
        s2[q][v] += (double)t2[q][v];
        s3[q][v] += (double)t3[q][v];
      }
  }
  // FP32 output layout: element v of lane (j, h) is C[4h + v][j] (column-major block)
#pragma unroll
  for (int q = 0; q < kB; ++q) {
    const size_t o = (size_t)(q == 0 ? b0 : b1) * 256 + l16 * 16 + 4 * lq;
#pragma unroll
    for (int v = 0; v < 4; ++v)
      stg2_nt(dst, o + v, make_float2((float)(s1[q][v] - s2[q][v]), (float)(s3[q][v] - s1[q][v] - s2[q][v])));
  }
}

template <int THREADS>
__device__ __forceinline__ void gram_tile_chunked(const float2 *Yc, int CP, int ncb, const float *w, int NB,
                                                  float2 *dst) {
  constexpr int kWaves = THREADS / 64;
  const int wave = threadIdx.x >> 6;
  int b = wave;
  for (; b + kWaves < NB; b += 2 * kWaves) gram_blocks_chunked<THREADS, true>(Yc, CP, ncb, w, b, b + kWaves, dst);
  if (b < NB) gram_blocks_chunked<THREADS, false>(Yc, CP, ncb, w, b, b, dst);
}

// Column pitch of the column-major Gram tile: Lp rounded up to an odd
// multiple of 16 complex, so that the two 16-row halves a wavefront reads at
// once (columns c and c + 1) start 32 banks apart.
__host__ __device__ constexpr int tile_pitch(int Lp) { return (Lp / 16) % 2 ? Lp : Lp + 16; }

typedef __attribute__((address_space(3))) void lds_void;

// Columns n0 .. n0 + NT - 1 of S (column-major, L rows) into the
// column-major LDS tile Yc (pitch CP) by direct global-to-LDS loads: every
// wavefront issues the loads of its columns back to back, so the whole tile
// is in flight at once and no register holds it.  With L even a lane moves
// two complex entries (16 bytes, aligned since every column starts at an
// even entry); with L odd it moves one float (columns start at odd
// entries).  Rows L .. Lp - 1 and the columns past N are written as zeros.
// The caller waits for the loads (s_waitcnt) and synchronises the
// workgroup before reading the tile.
template <int THREADS>
__device__ __forceinline__ void stage_tile_dma(const float2 *__restrict__ S, int L, int Lp, int N, int n0, int NT,
                                               int CP, float2 *Yc) {
  constexpr int kWaves = THREADS / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nt = min(NT, N - n0);
  if ((L & 1) == 0) {
    const int hp = L >> 1;
    for (int c = wave; c < nt; c += kWaves) {
      const float2 *src = S + (size_t)(n0 + c) * L;
      for (int k = 0; k < hp; k += 64)
        if (k + lane < hp)
          __builtin_amdgcn_global_load_lds((const void *)(src + 2 * (k + lane)), (lds_void *)(Yc + c * CP + 2 * k), 16,
                                           0, 0);
    }
  } else {
    const int nd = 2 * L;
    for (int c = wave; c < nt; c += kWaves) {
      const float *src = (const float *)(S + (size_t)(n0 + c) * L);
      for (int k = 0; k < nd; k += 64)
        if (k + lane < nd)
          __builtin_amdgcn_global_load_lds((const void *)(src + k + lane), (lds_void *)((float *)(Yc + c * CP) + k), 4,
                                           0, 0);
    }
  }
  const int pr = Lp - L;
  for (int e = threadIdx.x; e < NT * pr; e += THREADS) {
    const int c = e / pr;
    Yc[c * CP + L + (e - c * pr)] = make_float2(0.f, 0.f);
  }
  for (int e = threadIdx.x; e < (NT - nt) * Lp; e += THREADS) {
    const int c = nt + e / Lp;
    Yc[c * CP + e % Lp] = make_float2(0.f, 0.f);
  }
}

// Workgroup g of T sums its 1/T slice of the E packed entries over `parts`
// partial slots (stride pstride) in FP64: Pp threads per entry each sum
// every Pp-th slot, then one thread per entry adds the Pp sums in LDS and
// hands the total to store(e, sum).  dscr: THREADS double2 of LDS.
template <int THREADS, class Store>
__device__ __forceinline__ void reduce_packed_slice(const float2 *partials, size_t pstride, int parts, int T, int g,
                                                    int E, double2 *dscr, Store store) {
  const int tid = threadIdx.x;
  const int per = (E + T - 1) / T;
  const int start = g * per, end = min(E, start + per), cnt = max(0, end - start);
  const int Pp = cnt > 0 ? max(1, THREADS / cnt) : 1;
  for (int e0 = 0; e0 < cnt; e0 += THREADS / Pp) {
    const int e_loc = e0 + tid % (THREADS / Pp), part = tid / (THREADS / Pp);
    double2 acc = make_double2(0.0, 0.0);
    if (part < Pp && e_loc < cnt) {
      constexpr int kU = 8;   // loads in flight per thread
      const float2 *src = partials + start + e_loc;
      int h = part;
      for (; h + (kU - 1) * Pp < parts; h += kU * Pp) {
        float2 v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) v[u] = ldg2(src, (size_t)(h + u * Pp) * pstride);
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          acc.x += v[u].x;
          acc.y += v[u].y;
        }
      }
      for (; h < parts; h += Pp) {
        const float2 v = ldg2(src, (size_t)h * pstride);
        acc.x += v.x;
        acc.y += v.y;
      }
    }
    dscr[tid] = acc;
    __syncthreads();
    if (tid < THREADS / Pp && e0 + tid < cnt) {
      double2 sm = make_double2(0.0, 0.0);   // summed in double, rounded once
      for (int q = 0; q < Pp; ++q) {
        const double2 v = dscr[q * (THREADS / Pp) + tid];
        sm.x += v.x;
        sm.y += v.y;
      }
      store(start + e0 + tid, sm);
    }
    __syncthreads();
  }
}

// Phase B of a detection on T workgroups: workgroup g sums its 1/T slice of
// packed Sigma over `parts` partial slots (FP64), adds sigma^2 on the
// diagonal (unit pivots on padding rows) and writes Sigma and
// Delta = Sigma - SigmaHat (from the FP64 sum) to memory.  dscr: THREADS
// double2 of LDS.
template <int THREADS>
__device__ __forceinline__ void reduce_sigma_slice(const CoopArgs &A, float2 *delta, int parts, int T, int g,
                                                   double2 *dscr) {
  const int Lp = (A.L + 15) & ~15, Lb = Lp / 16, E = Lb * (Lb + 1) / 2 * 256;
  reduce_packed_slice<THREADS>(A.partials, A.pstride, parts, T, g, E, dscr, [&](int e, double2 sm) {
    const int b = e >> 8, jj = (e & 255) >> 4, ii = e & 15;
    int I, J;
    blk_coords(b, I, J);
    if (I == J && ii == jj) {
      sm.x += (16 * I + ii < A.L) ? (double)A.sigma2 : 1.0;
      sm.y = 0.0;
    }
    stg2(A.sigma, e, make_float2((float)sm.x, (float)sm.y));
    const int i = 16 * I + ii, k = 16 * J + jj;   // Sigma - SigmaHat from the FP64 sum
    const float2 sh = (i < A.L && k < A.L) ? ldg2(A.Sh, (size_t)k * A.L + i) : make_float2(0.f, 0.f);
    stg2(delta, e, make_float2((float)(sm.x - (double)sh.x), (float)(sm.y - (double)sh.y)));
  });
}

// Phase C1 of a detection on T workgroups: blocked Cholesky of packed Sigma
// in memory, one team barrier per block step.  Every workgroup factors the
// diagonal block in registers and keeps W_JJ = L_JJ^-1 in LDS (Wd); the
// trailing updates are spread over the team's waves, each forming the panel
// blocks it needs; the off-diagonal blocks of L go to lbuf.  Returns 0, 1
// for a pivot that is not positive and finite (the same decision in every
// workgroup), 2 when a barrier gave up.
template <int THREADS>
__device__ __forceinline__ int factor_in_memory(const CoopArgs &A, const float2 *delta, float2 *lbuf, float2 *Wd,
                                                float2 *scr, int T, int g, unsigned &gen, int *s_ok, int *s_pd) {
  constexpr int kWaves = THREADS / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, l16 = lane & 15, lq = lane >> 4;
  const int Lp = (A.L + 15) & ~15, Lb = Lp / 16, E = Lb * (Lb + 1) / 2 * 256;
  const int gwave = g * kWaves + wave, nwaves = T * kWaves;
  float2 *sig = A.sigma;
  (void)scr;
  int res = 0;
  for (int J = 0; J < Lb; ++J) {
    float2 *Wj = Wd + J * 256;
    for (int e = tid; e < 256; e += THREADS) Wj[e] = ldg2(pblk(sig, J, J), e);
    __syncthreads();
    if (wave == 0) {
      const bool ok = leaf_chol(Wj, 16, lane);
      if (lane == 0) *s_pd = ok ? 1 : 0;
    } else if (J == 0) {   // while the first leaf runs: Sigma - SigmaHat into L2 for C4
      warm_l2(delta, E, tid - 64, THREADS - 64);
    }
    __syncthreads();
    if (!*s_pd) {   // uniform: every workgroup factors the same block
      res = 1;
      break;
    }
    if (J + 1 == Lb) break;
    {   // trailing A_IK -= L_IJ L_KJ^H (J < K <= I).  Each task forms the panel
        // blocks it needs itself, L^T = conj(W_JJ) A^T, which leaves L[j][4q + v]
        // in lane (j, q): the layout of an MFMA operand over the permuted index
        // k = 4q + chunk.  So one barrier per block step; the task (I, J + 1)
        // stores L_IJ for the solves.
      const int m = Lb - 1 - J;
      auto panel_t = [&](int I, f4 &dr, f4 &di) {
        const float2 *blk = pblk(sig, I, J);
        dr = (f4){0.f, 0.f, 0.f, 0.f};
        di = (f4){0.f, 0.f, 0.f, 0.f};
        float2 a4[4], b4[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const int k = 4 * ks + lq;
          const float2 w = Wj[k * 16 + l16];   // W_JJ[l16][k]
          a4[ks] = make_float2(w.x, -w.y);
          b4[ks] = ldg2(blk, k * 16 + l16);     // A_IJ[l16][k] = A^T[k][l16]
        }
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) cmfma(a4[ks], b4[ks], dr, di);
      };
      for (int t = gwave; t < m * (m + 1) / 2; t += nwaves) {
        int ii = 0;
        while ((ii + 1) * (ii + 2) / 2 <= t) ++ii;
        const int I = J + 1 + ii, K = J + 1 + (t - ii * (ii + 1) / 2);
        f4 lir, lii, lkr, lki;
        panel_t(I, lir, lii);
        if (K == I) {
          lkr = lir;
          lki = lii;
        } else {
          panel_t(K, lkr, lki);
        }
        if (K == J + 1) {
          float2 *lb = lbuf + (size_t)blk_index(I, J) * 256;
#pragma unroll
          for (int v = 0; v < 4; ++v) stg2(lb, (4 * lq + v) * 16 + l16, make_float2(lir[v], lii[v]));
        }
        float2 *dst = sig + (size_t)blk_index(I, K) * 256;
        f4 cr, ci;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float2 c = ldg2(dst, l16 * 16 + 4 * lq + v);
          cr[v] = c.x;
          ci[v] = c.y;
        }
        float2 a4[4], b4[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          a4[ks] = make_float2(-lir[ks], -lii[ks]);   // L_IJ[l16][4 lq + ks]
          b4[ks] = make_float2(lkr[ks], -lki[ks]);    // conj(L_KJ[l16][4 lq + ks])
        }
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) cmfma(a4[ks], b4[ks], cr, ci);
#pragma unroll
        for (int v = 0; v < 4; ++v) stg2(dst, l16 * 16 + 4 * lq + v, make_float2(cr[v], ci[v]));
      }
    }
    if (!grid_sync(A.bar, T, g, gen, s_ok)) { res = 2; break; }
  }
  return res;
}


// ---------------------------------------------------------------------------
// Pilot lengths 97..256 on teams of workgroups: k_psca_large_teams
//
// One instance runs on a team of T workgroups.  Its devices are cut into Gv
// Gram tiles of NT = 16 ncb columns; rank g of the team forms the packed
// partials of tiles g, g + T, g + 2T, ... (each tile staged in LDS by direct
// loads, FP32 MFMA Gram in 16-column chunks summed in FP64, one partial slot
// per tile).  Phase B sums the Gv slots, 1/T of
// packed Sigma per rank; C1 factors Sigma in memory (factor_in_memory).  The solves run per 16-column block with the block
// held in registers: wave w of rank g takes the column blocks 8g + w,
// 8g + w + 8T, ..., so every wave of the team has work whatever the tile
// width, and a column block's substitutions, q, q - r and coordinate step
// need neither LDS nor a barrier.  The iterate lives in memory (xw); a team
// barrier closes every iteration but the last, before the next Gram pass
// reads it.  Teams work through lists of instances as k_psca_teams does.
// ---------------------------------------------------------------------------
struct LargeTeamArgs {
  CoopArgs c;        // c.G: the team size T; c.NT, c.ncb: the Gram tile; c.partials: [Gv][pstride]
  float2 *delta;     // packed Sigma - SigmaHat
  float2 *lbuf;      // packed off-diagonal blocks of the factor L
  float *xw;         // [N] the iterate
  float2 *xfull;     // [Lp][Lp] column-major: L^-1 (Sigma - SigmaHat) between the two passes of phase C2
  int Gv;            // Gram tiles, ceil(N / NT)
};

// LDS of the backward body: the row-major S tile [Lp][NT + 1], W_JJ, the
// reduction's THREADS double2 and the tile's weights.
__host__ __device__ inline size_t lds_large_team_bytes(int Lp, int NT, int threads) {
  return ((size_t)Lp * (NT + 1) + (size_t)(Lp / 16) * 256) * sizeof(float2) + (size_t)threads * sizeof(double2) +
         (size_t)NT * sizeof(float);
}

// LDS of the forward body: the column-major S tile [NT][tile_pitch(Lp)],
// with W_JJ [Lp / 16][256] and the reduction's THREADS double2 laid over it
// (phase A, the only user of the tile, begins after the solves have last
// read W_JJ and ends before the reduction), then the tile's weights [NT].
// Freeing the tile of those two lets it take 80 columns at L = 200.
__host__ __device__ inline size_t lds_large_fwd_overlay(int Lp, int NT, int threads) {
  const size_t tile = (size_t)NT * tile_pitch(Lp) * sizeof(float2);
  const size_t over = (size_t)(Lp / 16) * 256 * sizeof(float2) + (size_t)threads * sizeof(double2);
  return tile > over ? tile : over;
}
__host__ __device__ inline size_t lds_large_fwd_bytes(int Lp, int NT, int threads) {
  return lds_large_fwd_overlay(Lp, NT, threads) + (size_t)NT * sizeof(float);
}

// Row of flat task t when row r holds r tasks (rows 1, 2, ...): the largest
// r with r (r - 1) / 2 <= t.  Constant-folded where t is a constant.
__device__ __forceinline__ constexpr int tri_row(int t) {
  int r = 1;
  while ((r + 1) * r / 2 <= t) ++r;
  return r;
}

// Gauss accumulators, two independent sets (even and odd terms) so that
// consecutive MFMAs do not wait on each other's results.
struct Gauss2 {
  f4 t[2][3];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int k = 0; k < 3; ++k) t[s][k] = f4{0.f, 0.f, 0.f, 0.f};
  }
  // acc += A B for one 16x16 block: a[ks] = A[j][4h + ks], b[ks] = B[4h + ks][j]
  __device__ __forceinline__ void add(int set, const float2 (&a)[4], const float2 (&b)[4]) {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) cmfma3(a[ks], b[ks], t[set][0], t[set][1], t[set][2]);
  }
  __device__ __forceinline__ float2 get(int v) const {   // element v of this lane's output rows
    const float p1 = t[0][0][v] + t[1][0][v], p2 = t[0][1][v] + t[1][1][v], p3 = t[0][2][v] + t[1][2][v];
    return make_float2(p1 - p2, p3 - p1 - p2);
  }
};

// Column-block pieces: one wave holds a 16-column block of an L x 16 matrix
// in registers, y[R][v] = row 16 R + 4 h + v, column j, in lane (j, h) (the
// MFMA output layout).  Used as the B operand of a 16x16x4 step `ks`, that
// register set supplies the inner index k = 4h + ks (a permutation of the 16
// inner indices over the four steps), so the A operands (blocks of L, W_RR,
// or of a packed Hermitian matrix) are read in the same permuted order and
// no transposition is needed between block rows.  Each pass walks its
// blocks in a fixed order with the operands of the next two blocks already
// in flight (ring of three).  lo_n = 64 h + j: A[j][4h + ks] of a
// column-major 16x16 block sits at lo_n + 16 ks; lo_t = 16 j + 4 h: A^T at
// lo_t + ks.

// y = rows of the L x N column-major matrix M for columns c0 .. c0 + 15
// (zero outside L x N).
template <int LB>
__device__ __forceinline__ void cb_load(float2 (&y)[LB][4], const float2 *M, int L, int N, int n, int lq) {
  const bool col_in = n < N;
#pragma unroll
  for (int R = 0; R < LB; ++R)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * R + 4 * lq + v;
      y[R][v] = (col_in && row < L) ? ldg2(M, (size_t)n * L + row) : make_float2(0.f, 0.f);
    }
}

// y <- L^-1 y: Y_R = W_RR (y_R - sum_{K<R} L_RK Y_K); task t is block (R, K)
// with R = tri_row(t), K = t - R (R - 1) / 2.
template <int LB>
__device__ __forceinline__ void cb_forward(float2 (&y)[LB][4], const float2 *lbuf, const float2 *Wd, int lo_n) {
  constexpr int nf = LB * (LB - 1) / 2;
  float2 ring[3][4];
  Gauss2 acc;
  auto load = [&](int t, float2 (&dst)[4]) {
    const int R = tri_row(t), K = t - R * (R - 1) / 2;
    const float2 *blk = pblk(lbuf, R, K);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) dst[ks] = ldg2(blk, lo_n + 16 * ks);
  };
  if (nf > 0) load(0, ring[0]);
  if (nf > 1) load(1, ring[1]);
#pragma unroll
  for (int R = 0; R < LB; ++R) {
    acc.zero();
#pragma unroll
    for (int K = 0; K < R; ++K) {
      const int t = R * (R - 1) / 2 + K;
      if (t + 2 < nf) load(t + 2, ring[(t + 2) % 3]);
      acc.add(K & 1, ring[t % 3], y[K]);
    }
    float2 r4[4], w4[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float2 d = acc.get(v);
      r4[v] = make_float2(y[R][v].x - d.x, y[R][v].y - d.y);
    }
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) w4[ks] = Wd[R * 256 + lo_n + 16 * ks];   // W_RR[j][4h + ks]
    acc.zero();
    acc.add(0, w4, r4);
#pragma unroll
    for (int v = 0; v < 4; ++v) y[R][v] = acc.get(v);
  }
}

// y <- L^-H y: B_R = W_RR^H (y_R - sum_{K>R} L_KR^H B_K), R from the last
// block row up; task t is block (K, R) with r = tri_row(t), R = LB - 1 - r,
// K = R + 1 + t - r (r - 1) / 2.
template <int LB>
__device__ __forceinline__ void cb_backward(float2 (&y)[LB][4], const float2 *lbuf, const float2 *Wd, int lo_t) {
  constexpr int nf = LB * (LB - 1) / 2;
  float2 ring[3][4];
  Gauss2 acc;
  auto load = [&](int t, float2 (&dst)[4]) {
    const int r = tri_row(t), R = LB - 1 - r, K = R + 1 + t - r * (r - 1) / 2;
    const float2 *blk = pblk(lbuf, K, R);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const float2 x = ldg2(blk, lo_t + ks);   // L_KR[4h + ks][j]
      dst[ks] = make_float2(x.x, -x.y);
    }
  };
  if (nf > 0) load(0, ring[0]);
  if (nf > 1) load(1, ring[1]);
#pragma unroll
  for (int r = 0; r < LB; ++r) {
    const int R = LB - 1 - r;
    acc.zero();
#pragma unroll
    for (int j = 0; j < r; ++j) {
      const int t = r * (r - 1) / 2 + j, K = R + 1 + j;
      if (t + 2 < nf) load(t + 2, ring[(t + 2) % 3]);
      acc.add(j & 1, ring[t % 3], y[K]);
    }
    float2 r4[4], w4[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float2 d = acc.get(v);
      r4[v] = make_float2(y[R][v].x - d.x, y[R][v].y - d.y);
    }
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const float2 w = Wd[R * 256 + lo_t + ks];   // W_RR[4h + ks][j]
      w4[ks] = make_float2(w.x, -w.y);
    }
    acc.zero();
    acc.add(0, w4, r4);
#pragma unroll
    for (int v = 0; v < 4; ++v) y[R][v] = acc.get(v);
  }
}

// This lane's share of Re y^H H y for the Hermitian H given by its packed
// lower blocks: sum_I y_I^H H_II y_I + 2 Re sum_{K<I} y_I^H H_IK y_K (the
// caller adds the shares of the four lanes of a column).  Task t is the
// packed block t = (I, K), K <= I.
template <int LB>
__device__ __forceinline__ float cb_quad_lower(const float2 (&y)[LB][4], const float2 *H, int lo_n) {
  constexpr int nd = LB * (LB + 1) / 2;
  float2 ring[3][4];
  Gauss2 acc;
  auto load = [&](int t, float2 (&dst)[4]) {
    const int I = tri_row(t) - 1, K = t - I * (I + 1) / 2;
    const float f = K < I ? 2.0f : 1.0f;
    const float2 *blk = H + (size_t)t * 256;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const float2 x = ldg2(blk, lo_n + 16 * ks);   // H_IK[j][4h + ks]
      dst[ks] = make_float2(f * x.x, f * x.y);
    }
  };
  load(0, ring[0]);
  if (nd > 1) load(1, ring[1]);
  float s = 0.0f;
#pragma unroll
  for (int I = 0; I < LB; ++I) {
    acc.zero();
#pragma unroll
    for (int K = 0; K <= I; ++K) {
      const int t = I * (I + 1) / 2 + K;
      if (t + 2 < nd) load(t + 2, ring[(t + 2) % 3]);
      acc.add(K & 1, ring[t % 3], y[K]);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float2 d = acc.get(v);
      s += y[I][v].x * d.x + y[I][v].y * d.y;
    }
  }
  return s;
}

// (H y)_I for every block row I of the Hermitian H given by its packed lower
// blocks (H_IK for K <= I, H_KI^H for K > I); sink(I, acc) receives each
// block row's accumulators.  Task t is (I, K) = (t / LB, t % LB).
template <int LB, class Sink>
__device__ __forceinline__ void cb_hermv(const float2 (&y)[LB][4], const float2 *H, int lo_n, int lo_t, Sink sink) {
  constexpr int nt = LB * LB;
  float2 ring[3][4];
  Gauss2 acc;
  auto load = [&](int t, float2 (&dst)[4]) {
    const int I = t / LB, K = t % LB;
    if (K <= I) {
      const float2 *blk = pblk(H, I, K);
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) dst[ks] = ldg2(blk, lo_n + 16 * ks);   // H_IK[j][4h + ks]
    } else {
      const float2 *blk = pblk(H, K, I);
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const float2 x = ldg2(blk, lo_t + ks);   // H_KI[4h + ks][j]; (H_KI^H)[j][4h + ks] its conjugate
        dst[ks] = make_float2(x.x, -x.y);
      }
    }
  };
  load(0, ring[0]);
  if (nt > 1) load(1, ring[1]);
#pragma unroll
  for (int I = 0; I < LB; ++I) {
    acc.zero();
#pragma unroll
    for (int K = 0; K < LB; ++K) {
      const int t = I * LB + K;
      if (t + 2 < nt) load(t + 2, ring[(t + 2) % 3]);
      acc.add(K & 1, ring[t % 3], y[K]);
    }
    sink(I, acc);
  }
}

// Phase C2 of a large-L iteration: Delta' = L^-1 (Sigma - SigmaHat) L^-H, so
// that q - r = Re b^H (Sigma - SigmaHat) b = y^H Delta' y with y = L^-1 s and
// the column-block solves need no backward substitution (a third of their
// block products).  Two passes over the Lb column blocks of an L x L
// matrix, one column block per wavefront of the team: X = L^-1 Delta (full,
// column-major, in xfull), a team barrier, then Delta' = L^-1 X^H
// (X^H = Delta L^-H, Delta Hermitian), whose lower blocks overwrite Delta in
// packed form, and a team barrier before the solves read them.  Returns
// false when a barrier gave up.
template <int LB, int THREADS>
__device__ __forceinline__ bool transform_delta(const LargeTeamArgs &Tg, const float2 *Wd, int T, int g,
                                                unsigned &gen, int *s_ok) {
  const CoopArgs &A = Tg.c;
  constexpr int kWaves = THREADS / 64, Lp = 16 * LB;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, l16 = lane & 15, lq = lane >> 4;
  const int lo_n = (4 * lq) * 16 + l16;
  float2 *X = Tg.xfull, *D = Tg.delta;
  for (int j = g * kWaves + wave; j < LB; j += T * kWaves) {
    // column block j of Delta from its packed lower blocks (column-major
    // within a block): y[R][v] = Delta[16R + 4h + v][16j + l16]
    float2 y[LB][4];
#pragma unroll
    for (int R = 0; R < LB; ++R)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 4 * lq + v;
        if (R >= j) {
          y[R][v] = ldg2(D, (size_t)blk_index(R, j) * 256 + l16 * 16 + i);
        } else {
          const float2 t = ldg2(D, (size_t)blk_index(j, R) * 256 + i * 16 + l16);
          y[R][v] = make_float2(t.x, -t.y);
        }
      }
    cb_forward<LB>(y, Tg.lbuf, Wd, lo_n);
#pragma unroll
    for (int R = 0; R < LB; ++R)
#pragma unroll
      for (int v = 0; v < 4; ++v) stg2(X, (size_t)(16 * j + l16) * Lp + 16 * R + 4 * lq + v, y[R][v]);
  }
  if (!grid_sync(A.bar, T, g, gen, s_ok)) return false;
  for (int j = g * kWaves + wave; j < LB; j += T * kWaves) {
    // column block j of X^H: y[R][v] = conj(X[16j + l16][16R + 4h + v])
    float2 y[LB][4];
#pragma unroll
    for (int R = 0; R < LB; ++R)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float2 t = ldg2(X, (size_t)(16 * R + 4 * lq + v) * Lp + 16 * j + l16);
        y[R][v] = make_float2(t.x, -t.y);
      }
    cb_forward<LB>(y, Tg.lbuf, Wd, lo_n);
#pragma unroll
    for (int R = 0; R < LB; ++R)
      if (R >= j) {
#pragma unroll
        for (int v = 0; v < 4; ++v) stg2(D, (size_t)blk_index(R, j) * 256 + l16 * 16 + 4 * lq + v, y[R][v]);
      }
  }
  return grid_sync(A.bar, T, g, gen, s_ok);
}

// One wave: Y = L^-1 S_c (q = sum |y|^2), q - r = y^H Delta' y (phase C2)
// and the coordinate step of the 16 devices c0 .. c0 + 15.  The two passes
// are the ones of cb_forward and cb_quad_lower written out in one body with
// one operand ring: built from those helpers (then with a backward
// substitution too), this kernel's solves compiled to a schedule that took
// 24 % longer.
template <int LB>
__device__ __forceinline__ void solve_column_block(const LargeTeamArgs &Tg, const float2 *Wd, int c0, int it,
                                                   float rho, bool last) {
  const CoopArgs &A = Tg.c;
  const int lane = threadIdx.x & 63, l16 = lane & 15, lq = lane >> 4;
  const int n = c0 + l16;
  const bool col_in = n < A.N;
  // The factor and Sigma - SigmaHat are the same for every column block; an
  // opaque copy of their addresses keeps the compiler from hoisting all of
  // their loads out of the caller's loop over column blocks (thousands of
  // registers, spilled).
  const float2 *lbuf = Tg.lbuf, *dlt = Tg.delta;
  asm volatile("" : "+v"(lbuf), "+v"(dlt));
  const int lo_n = (4 * lq) * 16 + l16;   // A[j][4h + ks] at lo_n + 16 ks (column-major block)
  const int lo_t = l16 * 16 + 4 * lq;     // A^T[j][4h + ks] at lo_t + ks
  float2 y[LB][4];
#pragma unroll
  for (int R = 0; R < LB; ++R)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * R + 4 * lq + v;
      y[R][v] = (col_in && row < A.L) ? ldg2(A.S, (size_t)n * A.L + row) : make_float2(0.f, 0.f);
    }
  float2 ring[3][4];   // operands of the current block and the next two
  Gauss2 acc;

  // forward substitution: Y_R = W_RR (S_R - sum_{K<R} L_RK Y_K); task t is
  // block (R, K) with R = tri_row(t), K = t - R (R - 1) / 2
  constexpr int nf = LB * (LB - 1) / 2;
  auto load_f = [&](int t, float2 (&dst)[4]) {
    const int R = tri_row(t), K = t - R * (R - 1) / 2;
    const float2 *blk = pblk(lbuf, R, K);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) dst[ks] = ldg2(blk, lo_n + 16 * ks);
  };
  if (nf > 0) load_f(0, ring[0]);
  if (nf > 1) load_f(1, ring[1]);
#pragma unroll
  for (int R = 0; R < LB; ++R) {
    acc.zero();
#pragma unroll
    for (int K = 0; K < R; ++K) {
      const int t = R * (R - 1) / 2 + K;
      if (t + 2 < nf) load_f(t + 2, ring[(t + 2) % 3]);
      acc.add(K & 1, ring[t % 3], y[K]);
    }
    float2 r4[4], w4[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float2 d = acc.get(v);
      r4[v] = make_float2(y[R][v].x - d.x, y[R][v].y - d.y);
    }
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) w4[ks] = Wd[R * 256 + lo_n + 16 * ks];   // W_RR[j][4h + ks]
    acc.zero();
    acc.add(0, w4, r4);
#pragma unroll
    for (int v = 0; v < 4; ++v) y[R][v] = acc.get(v);
  }
  float q = 0.0f;
#pragma unroll
  for (int R = 0; R < LB; ++R)
#pragma unroll
    for (int v = 0; v < 4; ++v) q += y[R][v].x * y[R][v].x + y[R][v].y * y[R][v].y;
  q += __shfl_xor(q, 16);
  q += __shfl_xor(q, 32);

  // q - r = y^H Delta' y = sum_I y_I^H D'_II y_I + 2 Re sum_{K<I} y_I^H D'_IK y_K with
  // Delta' = L^-1 (Sigma - SigmaHat) L^-H from phase C2; task t is the packed
  // block t = (I, K), K <= I
  constexpr int nd = LB * (LB + 1) / 2;
  auto load_d = [&](int t, float2 (&dst)[4]) {
    const int I = tri_row(t) - 1, K = t - I * (I + 1) / 2;
    const float f = K < I ? 2.0f : 1.0f;
    const float2 *blk = dlt + (size_t)t * 256;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const float2 x = ldg2(blk, lo_n + 16 * ks);   // D_IK[j][4h + ks]
      dst[ks] = make_float2(f * x.x, f * x.y);
    }
  };
  load_d(0, ring[0]);
  if (nd > 1) load_d(1, ring[1]);
  float qmr = 0.0f;
#pragma unroll
  for (int I = 0; I < LB; ++I) {
    acc.zero();
#pragma unroll
    for (int K = 0; K <= I; ++K) {
      const int t = I * (I + 1) / 2 + K;
      if (t + 2 < nd) load_d(t + 2, ring[(t + 2) % 3]);
      acc.add(K & 1, ring[t % 3], y[K]);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float2 d = acc.get(v);
      qmr += y[I][v].x * d.x + y[I][v].y * d.y;
    }
  }
  qmr += __shfl_xor(qmr, 16);
  qmr += __shfl_xor(qmr, 32);
  // coordinate step and convex update of device n
  if (lq == 0 && col_in) {
    const float x = Tg.xw[n];
    const float gn = A.a.g ? A.a.g[n] : 0.0f;
    float prior = 0.0f;
    if (A.a.p) {
      const float pn = A.a.p[n];
      prior = logf(pn / (1.0f - pn));
    }
    const bool pairs = A.a.variant == PSCA_MAP_K2;
    if (pairs) prior = A.a.c1[n] + pair_sum(A.a, n, A.N, A.a.xg + (size_t)(it & 1) * A.N);
    const float xt = coordinate_step(x, q, qmr, gn, prior, A.a);
    const float xn = (1.0f - rho) * x + rho * xt;
    Tg.xw[n] = xn;
    if (pairs) A.a.xg[(size_t)((it + 1) & 1) * A.N + n] = xn;
    if (A.x_hist) A.x_hist[(size_t)(it + 1) * A.N + n] = xn;
    if (last) {
      A.x_out[n] = xn;
      if (A.q_out) A.q_out[n] = q;
      if (A.r_out) A.r_out[n] = q - qmr;
      if (A.xt_out) A.xt_out[n] = xt;
    }
  }
}

template <int LB, int THREADS>
__device__ __forceinline__ void large_team_body(const LargeTeamArgs &Tg, const int g) {
  const CoopArgs &A = Tg.c;
  constexpr int kWaves = THREADS / 64;
  constexpr int Lp = 16 * LB, NB = LB * (LB + 1) / 2;
  extern __shared__ float4 smem_raw[];
  __shared__ int s_ok, s_pd;
  const int NT = A.NT, ncb = A.ncb, T = A.G, Gv = Tg.Gv;
  constexpr int CP = tile_pitch(Lp);
  float2 *Yc = (float2 *)smem_raw;          // [NT][CP] Gram tile of S, column-major (phase A)
  float2 *Wd = Yc;                          // [LB][256] W_JJ, column-major blocks (C1 .. C5), over the tile
  double2 *dscr = (double2 *)(Wd + LB * 256);   // [THREADS] phase B, over the tile
  float *wv = (float *)((char *)smem_raw + lds_large_fwd_overlay(Lp, NT, THREADS));   // [NT] weights of the tile
  const int tid = threadIdx.x, wave = tid >> 6;
  const bool known = (A.a.variant == PSCA_ML_K || A.a.variant == PSCA_MAP_K || A.a.variant == PSCA_MAP_K2);
  const bool pairs = (A.a.variant == PSCA_MAP_K2);
  const int ncol = (A.N + 15) / 16;
  unsigned gen = 0;
  bool failed = false, aborted = false;

  for (int n = g * THREADS + tid; n < A.N; n += T * THREADS) {   // x^(0)
    const float x = A.x_in ? A.x_in[n] : 0.0f;
    Tg.xw[n] = x;
    if (A.x_hist) A.x_hist[n] = x;
    if (pairs) A.a.xg[n] = x;
  }
  if (!grid_sync(A.bar, T, g, gen, &s_ok)) aborted = true;

  double rho_d = A.rho0;
  for (int it = 0; it < A.iters && !aborted; ++it) {
    // ---- A. packed Gram partials of this rank's tiles
    PSCA_MARK(it, 0);
    for (int v = g; v < Gv; v += T) {
      const int n0 = v * NT;
      __syncthreads();   // the previous tile's Gram is done with Yc and wv
      stage_tile_dma<THREADS>(A.S, A.L, Lp, A.N, n0, NT, CP, Yc);
      for (int c = tid; c < NT; c += THREADS) {
        const int n = n0 + c;
        const float x = n < A.N ? Tg.xw[n] : 0.0f;
        wv[c] = n < A.N ? (known ? A.a.g[n] * x : x) : 0.0f;
      }
      __builtin_amdgcn_s_waitcnt(0);   // the tile's direct loads have landed in LDS
      __syncthreads();
      gram_tile_chunked<THREADS>(Yc, CP, ncb, wv, NB, A.partials + (size_t)v * A.pstride);
    }
    PSCA_MARK(it, 1);
    if (!grid_sync(A.bar, T, g, gen, &s_ok)) { aborted = true; break; }
    // ---- B. Sigma and Sigma - SigmaHat, 1/T of the packed entries per rank
    PSCA_MARK(it, 2);
    reduce_sigma_slice<THREADS>(A, Tg.delta, Gv, T, g, dscr);
    PSCA_MARK(it, 3);
    if (!grid_sync(A.bar, T, g, gen, &s_ok)) { aborted = true; break; }
    // ---- C1. blocked Cholesky in memory
    PSCA_MARK(it, 4);
    const int f = factor_in_memory<THREADS>(A, Tg.delta, Tg.lbuf, Wd, nullptr, T, g, gen, &s_ok, &s_pd);
    PSCA_MARK(it, 5);
    if (f == 1) failed = true;
    if (f == 2) aborted = true;
    if (failed || aborted) break;
    // ---- C2. Delta' = L^-1 (Sigma - SigmaHat) L^-H in place of Sigma - SigmaHat
    if (!transform_delta<LB, THREADS>(Tg, Wd, T, g, gen, &s_ok)) { aborted = true; break; }
    PSCA_MARK(it, 8);
    // ---- C4, C5. solves, quadratic forms and coordinate steps per column block
    float rho;
    if (A.rho_fixed >= 0.0f) rho = A.rho_fixed;
    else if (A.rho_dev) rho = A.rho_dev[it];
    else rho = (float)rho_d;
    rho_d = rho_d * (1.0 - A.rho_decay * rho_d);
    const bool last = (it == A.iters - 1);
    for (int cb = g * kWaves + wave; cb < ncol; cb += T * kWaves)
      solve_column_block<LB>(Tg, Wd, 16 * cb, it, rho, last);
    PSCA_MARK(it, 6);
    if (!last && !grid_sync(A.bar, T, g, gen, &s_ok)) { aborted = true; break; }
    PSCA_MARK(it, 7);
  }
  if (A.iters == 0 || failed || aborted)   // x_out holds the last finite iterate
    for (int n = g * THREADS + tid; n < A.N; n += T * THREADS) A.x_out[n] = Tg.xw[n];
  if (g == 0 && tid == 0 && A.status) *A.status = aborted ? PSCA_ESYNC : (failed ? PSCA_ENOTPD : PSCA_OK);
}

template <int LB>
__device__ __noinline__ void large_team_member(const LargeTeamArgs *__restrict__ desc, int g) {
  const LargeTeamArgs A = *desc;
  large_team_body<LB, 512>(A, g);
}

#ifdef PSCA_TU_MAIN
__global__ void __launch_bounds__(512) k_psca_large_teams(const LargeTeamArgs *__restrict__ descs,
                                                          const int *__restrict__ lists,
                                                          const int *__restrict__ offsets,
                                                          const int *__restrict__ team_start, int n_teams) {
  const int b = xcd_major((int)blockIdx.x, (int)gridDim.x);
  int t = 0, hi = n_teams - 1;   // the team with team_start[t] <= b < team_start[t + 1]
  while (t < hi) {
    const int mid = (t + hi + 1) >> 1;
    if (team_start[mid] <= b) t = mid;
    else hi = mid - 1;
  }
  const int g = b - team_start[t];
  const int i1 = offsets[t + 1];
  for (int idx = offsets[t]; idx < i1; ++idx) {
    const LargeTeamArgs *desc = descs + lists[idx];
    if (g < desc->c.G) {
      switch ((desc->c.L + 15) >> 4) {
        case 7: large_team_member<7>(desc, g); break;
        case 8: large_team_member<8>(desc, g); break;
        case 9: large_team_member<9>(desc, g); break;
        case 10: large_team_member<10>(desc, g); break;
        case 11: large_team_member<11>(desc, g); break;
        case 12: large_team_member<12>(desc, g); break;
        case 13: large_team_member<13>(desc, g); break;
        case 14: large_team_member<14>(desc, g); break;
        case 15: large_team_member<15>(desc, g); break;
        default: large_team_member<16>(desc, g); break;
      }
    }
    __syncthreads();   // the next instance reuses the LDS
  }
}
#endif

// ---------------------------------------------------------------------------
// Backward of one unrolled layer for 65 <= L <= 256: k_psca_back_large_<lo>_<hi>.
// The quantities of the LDS backward (k_psca_back) on teams of workgroups as
// k_psca_large_teams runs them: Sigma(x) rebuilt and factored in memory (not
// stored by the forward pass), then per 16-column block in registers
// b_m = Sigma^-1 s_m, q, q - r, c_m = Sigma^-1 SigmaHat b_m
// = b_m - Sigma^-1 (Sigma - SigmaHat) b_m and the per-device weights
// a_n, b_n of the two Gram matrices G_a = S diag(a) S^H, G_b = S diag(b) S^H
// (Gram tiles in LDS, FP64, partials per tile), then per column block
// dL/dx_m = v_m (1 - rho) + rho v_m mask_m (1 + c'/curv)
//           - kappa_m (b_m^H G_a b_m + 2 Re c_m^H G_b b_m).
// Five team barriers plus those of the factorisation.
// ---------------------------------------------------------------------------
struct LargeBackArgs {
  LargeTeamArgs f;         // f.c: instance, x_in = the layer's input; tiles, Sigma, factor, barrier (xw unused)
  float rho;               // the layer's step size
  const float *v;          // [N] dL/dx'
  float *grad_x;           // [N] dL/dx
  float *grad_rho;         // this instance's dL/drho
  float *rho_part;         // [T] per-rank parts of dL/drho
  float2 *partials_b;      // [Gv][pstride] partials of G_b (Sigma's and G_a's use f.c.partials)
  float2 *gram_a, *gram_b; // packed G_a, G_b
  float2 *bmat, *cmat;     // per column block [LB][4][64], lane-major: b_m and c_m in the register layout
  float *wa, *wb, *d0;     // [N] weights a_n, b_n and the diagonal term of dL/dx
};

__host__ __device__ inline size_t lds_large_back_bytes(int Lp, int NT, int threads) {
  return lds_large_team_bytes(Lp, NT, threads) + (size_t)NT * sizeof(float);
}

__device__ __forceinline__ size_t cb_slot(int cb, int LB, int R, int v, int lane) {
  return ((size_t)(cb * LB + R) * 4 + v) * 64 + lane;
}

// b_m, q, q - r, c_m and the weights of the 16 devices of column block cb;
// returns this lane's part of dL/drho.
template <int LB>
__device__ __forceinline__ float back_column_block_1(const LargeBackArgs &Bk, const float2 *Wd, int cb) {
  const CoopArgs &A = Bk.f.c;
  const int lane = threadIdx.x & 63, l16 = lane & 15, lq = lane >> 4;
  const int n = 16 * cb + l16;
  const bool col_in = n < A.N;
  const float2 *lbuf = Bk.f.lbuf, *dlt = Bk.f.delta;
  asm volatile("" : "+v"(lbuf), "+v"(dlt));   // keep the block loads inside the caller's loop
  const int lo_n = (4 * lq) * 16 + l16, lo_t = l16 * 16 + 4 * lq;
  float2 y[LB][4];
  cb_load<LB>(y, A.S, A.L, A.N, n, lq);
  cb_forward<LB>(y, lbuf, Wd, lo_n);
  float q = 0.0f;
#pragma unroll
  for (int R = 0; R < LB; ++R)
#pragma unroll
    for (int v = 0; v < 4; ++v) q += y[R][v].x * y[R][v].x + y[R][v].y * y[R][v].y;
  q += __shfl_xor(q, 16);
  q += __shfl_xor(q, 32);
  cb_backward<LB>(y, lbuf, Wd, lo_t);   // y = b
#pragma unroll
  for (int R = 0; R < LB; ++R)
#pragma unroll
    for (int v = 0; v < 4; ++v) Bk.bmat[cb_slot(cb, LB, R, v, lane)] = y[R][v];
  float qmr = cb_quad_lower<LB>(y, dlt, lo_n);
  qmr += __shfl_xor(qmr, 16);
  qmr += __shfl_xor(qmr, 32);
  // z = (Sigma - SigmaHat) b, staged in cmat; then c = b - Sigma^-1 z
  cb_hermv<LB>(y, dlt, lo_n, lo_t, [&](int I, const Gauss2 &acc) {
#pragma unroll
    for (int v = 0; v < 4; ++v) Bk.cmat[cb_slot(cb, LB, I, v, lane)] = acc.get(v);
  });
#pragma unroll
  for (int R = 0; R < LB; ++R)
#pragma unroll
    for (int v = 0; v < 4; ++v) y[R][v] = ldg2(Bk.cmat, cb_slot(cb, LB, R, v, lane));
  cb_forward<LB>(y, lbuf, Wd, lo_n);
  cb_backward<LB>(y, lbuf, Wd, lo_t);
#pragma unroll
  for (int R = 0; R < LB; ++R)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const size_t k = cb_slot(cb, LB, R, v, lane);
      const float2 b = ldg2(Bk.bmat, k);
      Bk.cmat[k] = make_float2(b.x - y[R][v].x, b.y - y[R][v].y);
    }
  float rho_term = 0.0f;
  if (lq == 0 && col_in) {
    const float x = A.x_in[n], vn = Bk.v[n];
    const float gn = A.a.g ? A.a.g[n] : 0.0f;
    float logit = 0.0f;
    if (A.a.p) {
      const float pn = A.a.p[n];
      logit = logf(pn / (1.0f - pn));
    }
    const StepDerivs d = step_derivs_qmr(x, q, qmr, gn, logit, A.a);
    const float rv = Bk.rho * vn * d.mask;
    Bk.wa[n] = rv * d.dq;
    Bk.wb[n] = rv * d.dr;
    Bk.d0[n] = vn * (1.0f - Bk.rho) + rv * d.own;
    rho_term = vn * (d.xt - x);
  }
  return rho_term;
}

// dL/dx of the 16 devices of column block cb from b_m, c_m and G_a, G_b.
template <int LB>
__device__ __forceinline__ void back_column_block_2(const LargeBackArgs &Bk, int cb) {
  const CoopArgs &A = Bk.f.c;
  const int lane = threadIdx.x & 63, l16 = lane & 15, lq = lane >> 4;
  const int n = 16 * cb + l16;
  const float2 *ga = Bk.gram_a, *gb = Bk.gram_b;
  asm volatile("" : "+v"(ga), "+v"(gb));
  const int lo_n = (4 * lq) * 16 + l16, lo_t = l16 * 16 + 4 * lq;
  float2 y[LB][4];
#pragma unroll
  for (int R = 0; R < LB; ++R)
#pragma unroll
    for (int v = 0; v < 4; ++v) y[R][v] = ldg2(Bk.bmat, cb_slot(cb, LB, R, v, lane));
  float t1 = cb_quad_lower<LB>(y, ga, lo_n);   // b^H G_a b
  float t2 = 0.0f;                              // Re c^H G_b b
  cb_hermv<LB>(y, gb, lo_n, lo_t, [&](int I, const Gauss2 &acc) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float2 c = ldg2(Bk.cmat, cb_slot(cb, LB, I, v, lane)), d = acc.get(v);
      t2 += c.x * d.x + c.y * d.y;
    }
  });
  t1 += __shfl_xor(t1, 16);
  t1 += __shfl_xor(t1, 32);
  t2 += __shfl_xor(t2, 16);
  t2 += __shfl_xor(t2, 32);
  if (lq == 0 && n < A.N) {
    const bool known = (A.a.variant == PSCA_ML_K || A.a.variant == PSCA_MAP_K);
    const float kappa = known ? A.a.g[n] : 1.0f;
    Bk.grad_x[n] = Bk.d0[n] - kappa * (t1 + 2.0f * t2);
  }
}

template <int LB, int THREADS>
__device__ __forceinline__ void large_back_body(const LargeBackArgs &Bk, const int g) {
  const LargeTeamArgs &Tg = Bk.f;
  const CoopArgs &A = Tg.c;
  constexpr int kWaves = THREADS / 64;
  constexpr int Lp = 16 * LB, NB = LB * (LB + 1) / 2;
  extern __shared__ float4 smem_raw[];
  __shared__ int s_ok, s_pd;
  __shared__ float s_red[kWaves];
  const int NT = A.NT, PT = A.NT + 1, ncb = A.ncb, T = A.G, Gv = Tg.Gv;
  float2 *Yt = (float2 *)smem_raw;              // [Lp][PT] Gram tile of S
  float2 *Wd = Yt + Lp * PT;                    // [LB][256] W_JJ
  double2 *dscr = (double2 *)(Wd + LB * 256);   // [THREADS]
  float *wv = (float *)(dscr + THREADS);        // [NT] weights of the tile
  float *wv2 = wv + NT;                         // [NT] second weights
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool known = (A.a.variant == PSCA_ML_K || A.a.variant == PSCA_MAP_K);
  const int ncol = (A.N + 15) / 16;
  const int E = NB * 256;
  unsigned gen = 0;
  bool failed = false, aborted = false;
  // stage the S tile v (columns v NT ..) in Yt and its weights by `weights`
  auto stage = [&](int v, auto weights) {
    const int n0 = v * NT;
    __syncthreads();   // the previous tile's Grams are done with Yt and the weights
    for (int c = tid; c < NT; c += THREADS) weights(c, n0 + c);
    constexpr int kU = 8;   // loads in flight per thread
    const int tot = Lp * NT;
    for (int e0 = tid; e0 < tot; e0 += kU * THREADS) {
      float2 val[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int e = e0 + u * THREADS, c = e / Lp, i = e - c * Lp;   // down a column: coalesced
        const int n = n0 + c;
        val[u] = (e < tot && i < A.L && n < A.N) ? A.S[(size_t)n * A.L + i] : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int e = e0 + u * THREADS, c = e / Lp, i = e - c * Lp;
        if (e < tot) Yt[i * PT + c] = val[u];
      }
    }
    __syncthreads();
  };
  do {
    // ---- Sigma(x) and its factor, as the forward pass
    for (int v = g; v < Gv; v += T) {
      stage(v, [&](int c, int n) {
        const float x = n < A.N ? A.x_in[n] : 0.0f;
        wv[c] = n < A.N ? (known ? A.a.g[n] * x : x) : 0.0f;
      });
      gram_tile_fp64<THREADS>(Yt, PT, ncb, wv, NB, A.partials + (size_t)v * A.pstride);
    }
    if (!grid_sync(A.bar, T, g, gen, &s_ok)) { aborted = true; break; }
    reduce_sigma_slice<THREADS>(A, Tg.delta, Gv, T, g, dscr);
    if (!grid_sync(A.bar, T, g, gen, &s_ok)) { aborted = true; break; }
    const int f = factor_in_memory<THREADS>(A, Tg.delta, Tg.lbuf, Wd, nullptr, T, g, gen, &s_ok, &s_pd);
    if (f == 1) failed = true;
    if (f == 2) aborted = true;
    if (failed || aborted) break;
    // ---- b, q, q - r, c and the weights per column block
    float rho_term = 0.0f;
    for (int cb = g * kWaves + wave; cb < ncol; cb += T * kWaves) rho_term += back_column_block_1<LB>(Bk, Wd, cb);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) rho_term += __shfl_xor(rho_term, o);
    if (lane == 0) s_red[wave] = rho_term;
    __syncthreads();
    if (tid == 0) {
      float t = 0.0f;
      for (int w = 0; w < kWaves; ++w) t += s_red[w];
      Bk.rho_part[g] = t;
    }
    if (!grid_sync(A.bar, T, g, gen, &s_ok)) { aborted = true; break; }
    // ---- G_a and G_b
    for (int v = g; v < Gv; v += T) {
      stage(v, [&](int c, int n) {
        wv[c] = n < A.N ? Bk.wa[n] : 0.0f;
        wv2[c] = n < A.N ? Bk.wb[n] : 0.0f;
      });
      gram_tile_fp64<THREADS>(Yt, PT, ncb, wv, NB, A.partials + (size_t)v * A.pstride);
      gram_tile_fp64<THREADS>(Yt, PT, ncb, wv2, NB, Bk.partials_b + (size_t)v * A.pstride);
    }
    if (!grid_sync(A.bar, T, g, gen, &s_ok)) { aborted = true; break; }
    reduce_packed_slice<THREADS>(A.partials, A.pstride, Gv, T, g, E, dscr, [&](int e, double2 sm) {
      Bk.gram_a[e] = make_float2((float)sm.x, (float)sm.y);
    });
    reduce_packed_slice<THREADS>(Bk.partials_b, A.pstride, Gv, T, g, E, dscr, [&](int e, double2 sm) {
      Bk.gram_b[e] = make_float2((float)sm.x, (float)sm.y);
    });
    if (!grid_sync(A.bar, T, g, gen, &s_ok)) { aborted = true; break; }
    // ---- dL/dx per column block; dL/drho from the ranks' parts
    for (int cb = g * kWaves + wave; cb < ncol; cb += T * kWaves) back_column_block_2<LB>(Bk, cb);
    if (g == 0 && tid == 0) {
      float t = 0.0f;
      for (int r = 0; r < T; ++r) t += Bk.rho_part[r];
      *Bk.grad_rho = t;
    }
  } while (false);
  if (g == 0 && tid == 0 && A.status) *A.status = aborted ? PSCA_ESYNC : (failed ? PSCA_ENOTPD : PSCA_OK);
}

template <int LB>
__device__ __noinline__ void large_back_member(const LargeBackArgs *__restrict__ desc, int g) {
  const LargeBackArgs A = *desc;
  large_back_body<LB, 512>(A, g);
}

// The large-L backward kernels: one per range of block counts LB = L_p / 16,
// each built from this file as a translation unit of its own (the fully
// unrolled column-block code of 12 instantiations compiles for minutes; the
// ranges compile in parallel).  A launch runs instances of one range.
#define PSCA_BACK_RANGES(X) X(5, 10) X(11, 13) X(14, 15) X(16, 16)
#define PSCA_BACK_NAME(lo, hi) k_psca_back_large_##lo##_##hi
#define PSCA_BACK_DECL(lo, hi)                                                                              \
  __global__ void __launch_bounds__(512) PSCA_BACK_NAME(lo, hi)(                                           \
      const LargeBackArgs *__restrict__ descs, const int *__restrict__ lists, const int *__restrict__ offsets, \
      const int *__restrict__ team_start, int n_teams);
PSCA_BACK_RANGES(PSCA_BACK_DECL)

#ifdef PSCA_TU_BACK   // -DPSCA_TU_BACK -DPSCA_BACK_LO=lo -DPSCA_BACK_HI=hi
template <int LO, int HI>
__device__ __forceinline__ void back_dispatch(int lb, const LargeBackArgs *desc, int g) {
  if constexpr (LO <= HI) {
    if (lb == LO) large_back_member<LO>(desc, g);
    else back_dispatch<LO + 1, HI>(lb, desc, g);
  }
}

#define PSCA_BACK_DEF(lo, hi) PSCA_BACK_DEF_(lo, hi)
#define PSCA_BACK_DEF_(lo, hi)                                                                              \
  __global__ void __launch_bounds__(512) PSCA_BACK_NAME(lo, hi)(                                           \
      const LargeBackArgs *__restrict__ descs, const int *__restrict__ lists, const int *__restrict__ offsets, \
      const int *__restrict__ team_start, int n_teams) {                                                    \
    const int b = xcd_major((int)blockIdx.x, (int)gridDim.x);                                               \
    int t = 0, hi_t = n_teams - 1; /* the team with team_start[t] <= b < team_start[t + 1] */             \
    while (t < hi_t) {                                                                                      \
      const int mid = (t + hi_t + 1) >> 1;                                                                  \
      if (team_start[mid] <= b) t = mid;                                                                    \
      else hi_t = mid - 1;                                                                                  \
    }                                                                                                       \
    const int g = b - team_start[t];                                                                        \
    const int i1 = offsets[t + 1];                                                                          \
    for (int idx = offsets[t]; idx < i1; ++idx) {                                                           \
      const LargeBackArgs *desc = descs + lists[idx];                                                       \
      if (g < desc->f.c.G) back_dispatch<lo, hi>((desc->f.c.L + 15) >> 4, desc, g);                         \
      __syncthreads(); /* the next instance reuses the LDS */                                              \
    }                                                                                                       \
  }
PSCA_BACK_DEF(PSCA_BACK_LO, PSCA_BACK_HI)
#endif

// Barrier words, abort word and status of every instance of a large-L
// backward launch: block b resets instance b.
#ifdef PSCA_TU_MAIN
__global__ void k_prepare_large_back(const LargeBackArgs *__restrict__ descs) {
  const CoopArgs &A = descs[blockIdx.x].f.c;
  for (int w = threadIdx.x; w < A.G; w += blockDim.x) A.bar.arrive[w * 16] = 0u;
  if (threadIdx.x == 0) {
    *A.bar.release = 0u;
    *A.bar.abort_flag = 0;
    *A.status = PSCA_OK;
  }
}
#endif

// Barrier words, abort word and status of every instance of a large-L batch
// launch: block b resets instance b.
#ifdef PSCA_TU_MAIN
__global__ void k_prepare_large_batch(const LargeTeamArgs *__restrict__ descs) {
  const CoopArgs &A = descs[blockIdx.x].c;
  for (int w = threadIdx.x; w < A.G; w += blockDim.x) A.bar.arrive[w * 16] = 0u;
  if (threadIdx.x == 0) {
    *A.bar.release = 0u;
    *A.bar.abort_flag = 0;
    *A.status = PSCA_OK;
  }
}
#endif

template <int LPMAX, int THREADS>
__global__ void __launch_bounds__(THREADS) k_psca(CoopArgs A) {
  psca_body<LPMAX, THREADS>(A, blockIdx.x);
}

// Batch of independent detections in one persistent launch.  The grid is
// split into teams of T workgroups; team t runs the instances
// lists[offsets[t] .. offsets[t+1]) one after the other, and workgroup g of
// the team takes part in instance b iff g < descs[b].G (the planner sets
// G = T).  Every instance synchronises on its own barrier words.
constexpr int kBatchThreads = 512;

// One instance inside the batch kernel; kept out of line so that each pilot
// length gets its own register allocation.
template <int LP>
__device__ __noinline__ void team_member(const CoopArgs *__restrict__ desc, int g) {
  const CoopArgs A = *desc;
  psca_body<LP, kBatchThreads>(A, g);
}

#ifdef PSCA_TU_MAIN
__global__ void __launch_bounds__(kBatchThreads) k_psca_teams(const CoopArgs *__restrict__ descs,
                                                              const int *__restrict__ lists,
                                                              const int *__restrict__ offsets,
                                                              const int *__restrict__ team_start, int n_teams) {
  const int b = xcd_major((int)blockIdx.x, (int)gridDim.x);
  int t = 0, hi = n_teams - 1;   // the team with team_start[t] <= b < team_start[t + 1]
  while (t < hi) {
    const int mid = (t + hi + 1) >> 1;
    if (team_start[mid] <= b) t = mid;
    else hi = mid - 1;
  }
  const int g = b - team_start[t];
  const int i1 = offsets[t + 1];
  for (int idx = offsets[t]; idx < i1; ++idx) {
    const CoopArgs *desc = descs + lists[idx];
    if (g < desc->G) {
      switch ((desc->L + 15) & ~15) {
        case 16: team_member<16>(desc, g); break;
        case 32: team_member<32>(desc, g); break;
        case 48: team_member<48>(desc, g); break;
        case 64: team_member<64>(desc, g); break;
        case 80: team_member<80>(desc, g); break;
        default: team_member<96>(desc, g); break;
      }
    }
    __syncthreads();   // the next instance reuses the LDS
  }
}
#endif

// SigmaHat = Y Y^H / M on FP64 MFMA.  Workgroup b computes the lower 16x16
// block (I, J) = blk_coords(b); its four wavefronts take the columns m of Y
// in interleaved groups of four, with the complex products on the real
// four-product split (products of FP32 entries are exact in FP64, sums in
// FP64), add their sums in LDS in a fixed order, scale by 1/M and round
// once.  Strictly lower entries are mirrored (conjugated) into the upper
// triangle and the diagonal's imaginary part is zero, so the result is
// exactly Hermitian.  Grid: Lb (Lb + 1) / 2 workgroups of 256 threads per
// instance; instance blockIdx.y reads Y + y * sy and writes Sh + y * ss.
#ifdef PSCA_TU_MAIN
__global__ void __launch_bounds__(256) k_sample_cov(const float2 *__restrict__ Y, int L, int M,
                                                    float2 *__restrict__ Sh, long long sy, long long ss) {
  __shared__ double red[2][4][4][64];   // [re/im][wave][element][lane]
  Y += (size_t)blockIdx.y * (size_t)sy;
  Sh += (size_t)blockIdx.y * (size_t)ss;
  int I, J;
  blk_coords(blockIdx.x, I, J);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, l16 = lane & 15, lq = lane >> 4;
  const int ra = 16 * I + l16, rb = 16 * J + l16;   // A[l16][k] = Y[ra][m], B[k][l16] = conj(Y[rb][m])
  const bool ina = ra < L, inb = rb < L;
  d4 cr = {0.0, 0.0, 0.0, 0.0}, ci = cr;
  for (int m0 = 4 * wave; m0 < M; m0 += 16) {
    const int m = m0 + lq;
    float2 a = make_float2(0.f, 0.f), b = a;
    if (m < M) {
      if (ina) a = Y[(size_t)m * L + ra];
      if (inb) b = Y[(size_t)m * L + rb];
    }
    // a conj(b) = (ax bx + ay by) + i (ay bx - ax by)
    cr = mfma4d(a.x, b.x, cr);
    cr = mfma4d(a.y, b.y, cr);
    ci = mfma4d(a.y, b.x, ci);
    ci = mfma4d(-a.x, b.y, ci);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    red[0][wave][v][lane] = cr[v];
    red[1][wave][v][lane] = ci[v];
  }
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      sr += red[0][w][v][lane];
      si += red[1][w][v][lane];
    }
    // FP64 output layout: element v of lane (j, h) is C[4v + h][j]
    const int i = 4 * v + lq, jj = l16;
    const int row = 16 * I + i, col = 16 * J + jj;
    if (row < L && col < L && (I > J || i >= jj)) {
      const float re = (float)(sr / M), im = row == col ? 0.0f : (float)(si / M);
      Sh[(size_t)col * L + row] = make_float2(re, im);
      if (row != col) Sh[(size_t)row * L + col] = make_float2(re, -im);
    }
  }
}
#endif

// Reset the barrier words, the abort word and the status before a launch of k_psca.
#ifdef PSCA_TU_MAIN
__global__ void k_prepare(unsigned *arrive, int G, unsigned *release, int32_t *abort_flag, int32_t *status) {
  for (int w = threadIdx.x; w < G; w += blockDim.x) arrive[w * 16] = 0u;
  if (threadIdx.x == 0) {
    *release = 0u;
    *abort_flag = 0;
    if (status) *status = PSCA_OK;
  }
}
#endif

// The same for every instance of a batch launch: block b resets instance b.
#ifdef PSCA_TU_MAIN
__global__ void k_prepare_batch(const CoopArgs *__restrict__ descs) {
  const CoopArgs &A = descs[blockIdx.x];
  for (int w = threadIdx.x; w < A.G; w += blockDim.x) A.bar.arrive[w * 16] = 0u;
  if (threadIdx.x == 0) {
    *A.bar.release = 0u;
    *A.bar.abort_flag = 0;
    *A.status = PSCA_OK;
  }
}
#endif

#ifdef PSCA_TU_MAIN
__global__ void k_threshold(const float *__restrict__ x, int N, float theta, uint8_t *__restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n < N) out[n] = x[n] >= theta ? 1 : 0;
}
#endif

}  // namespace psca_impl

using namespace psca_impl;

#ifdef PSCA_TU_MAIN   // host code, the C ABI and the no-allocation scratch: one translation unit

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

// Scratch of psca_detect_noalloc: one array per GPU, allocated by the loader
// with the code object and held until the process ends.  Host code never
// passes `scratch` itself (a host-side stand-in, not a device address): it
// takes the device address from hipGetSymbolAddress once per device, with
// that device current, and uses that.
constexpr size_t kScratchBytes = PSCA_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static void *g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu;

struct psca_ctx {
  int device;
  int n_cu;
  void *ws;          // partials, Sigma, barrier words
  size_t ws_bytes;
  void *sh;          // SigmaHat formed by psca_detect_y
  size_t sh_bytes;
  // cached occupancy: workgroups of one k_psca instantiation per CU for a given LDS size
  const void *occ_fn;
  size_t occ_lds;
  int occ_per_cu;
  // batch launches: instance descriptors and the workgroup map, staged in
  // pinned host memory and copied on the caller's stream
  void *hdesc, *ddesc;
  size_t desc_bytes;
  hipEvent_t desc_done;   // the last copy out of hdesc
  bool desc_pending;
  std::unordered_map<uint64_t, int> tuned;   // batch signature -> team size (psca_autotune_batch)
};

namespace {

struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = (hipSetDevice(dev) == hipSuccess);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// Grow a context buffer; waits for the device before freeing the old one
// because queued work may still use it.
int ensure_buf(void **buf, size_t *cap, size_t bytes) {
  if (bytes <= *cap) return PSCA_OK;
  if (*buf) {
    if (hipDeviceSynchronize() != hipSuccess) return PSCA_EHIP;
    (void)hipFree(*buf);
    *buf = nullptr;
    *cap = 0;
  }
  const size_t want = bytes + bytes / 4;
  if (hipMalloc(buf, want) != hipSuccess) {
    (void)hipGetLastError();
    *buf = nullptr;
    return PSCA_ENOMEM;
  }
  *cap = want;
  return PSCA_OK;
}

int ensure_ws(psca_ctx *ctx, size_t bytes) { return ensure_buf(&ctx->ws, &ctx->ws_bytes, bytes); }

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

int validate_params(const psca_params *prm, int L, int N, bool need_iters) {
  if (!prm) return PSCA_EINVAL;
  if (L < 1 || N < 1) return PSCA_EINVAL;
  if (L > kMaxL) return PSCA_ENOTSUP;
  if (prm->variant < PSCA_ML_K || prm->variant > PSCA_MAP_K2) return PSCA_EINVAL;
  if (!(prm->sigma2 > 0.0f) || !isfinite(prm->sigma2)) return PSCA_EINVAL;
  if (prm->M < 1) return PSCA_EINVAL;
  if (need_iters) {
    if (prm->iters < 0) return PSCA_EINVAL;
    if (!prm->rho && (!(prm->rho0 > 0.0f) || prm->rho0 > 1.0f || !(prm->rho_decay >= 0.0f) ||
                      prm->rho_decay > 2.0f))
      return PSCA_EINVAL;
  }
  if ((prm->variant == PSCA_ML_K || prm->variant == PSCA_MAP_K || prm->variant == PSCA_MAP_K2) && !prm->g)
    return PSCA_EINVAL;
  if (prm->variant == PSCA_MAP_K && !prm->p) return PSCA_EINVAL;
  if (prm->variant == PSCA_MAP_K2 &&
      (!prm->c1 || !prm->c2_ptr || prm->c2_nnz < 0 || (prm->c2_nnz > 0 && (!prm->c2_col || !prm->c2_val))))
    return PSCA_EINVAL;
  if (prm->variant == PSCA_MAP_UR) {
    if (!(prm->d_lo > 0.0f) || !(prm->d_hi > prm->d_lo) || !(prm->pl_c0 > 0.0f) || !(prm->pl_beta > 0.0f) ||
        !(prm->eps > 0.0f) || !isfinite(prm->d_hi) || !isfinite(prm->pl_c0) || !isfinite(prm->pl_beta))
      return PSCA_EINVAL;
    const double gl = (double)prm->pl_c0 * pow((double)prm->d_hi, -(double)prm->pl_beta);
    if (!(2.0 * (double)prm->eps < gl)) return PSCA_EINVAL;
    if (prm->dist_law != PSCA_DIST_AREA && prm->dist_law != PSCA_DIST_LINEAR) return PSCA_EINVAL;
  }
  return PSCA_OK;
}

StepArgs make_step_args(const psca_params *prm) {
  StepArgs a;
  a.variant = prm->variant;
  a.inv_M = (float)(1.0 / (double)prm->M);
  const bool k2 = prm->variant == PSCA_MAP_K2;
  a.g = (prm->variant == PSCA_ML_K || prm->variant == PSCA_MAP_K || k2) ? prm->g : nullptr;
  a.p = (prm->variant == PSCA_MAP_K) ? prm->p : nullptr;
  a.c1 = k2 ? prm->c1 : nullptr;
  a.c2_ptr = k2 ? prm->c2_ptr : nullptr;
  a.c2_col = k2 ? prm->c2_col : nullptr;
  a.c2_val = k2 ? prm->c2_val : nullptr;
  a.c2_nnz = k2 ? prm->c2_nnz : 0;
  a.xg = nullptr;   // bound with the workspace
  a.eps = a.g_l = a.g_u = a.h2_b = a.dens_c = 0.0f;
  if (prm->variant == PSCA_MAP_UR) {
    const double beta = prm->pl_beta;
    const double gl = (double)prm->pl_c0 * pow((double)prm->d_hi, -beta);
    const double gu = (double)prm->pl_c0 * pow((double)prm->d_lo, -beta);
    a.eps = prm->eps;
    a.g_l = (float)gl;
    a.g_u = (float)gu;
    // On the density piece p_G is p_D(psi) |psi'| with psi = phi^-1 =
    // (c0 / x)^(1/beta), so p'/p = psi''/psi' + (p_D'/p_D)(psi) psi':
    //   area-uniform (p_D ~ d):  -(1/beta + 1)/x - 1/(beta x) = -(2/beta + 1)/x;
    //   uniform in d (p_D const): -(1/beta + 1)/x.
    // H2's coefficient ratio B/A = p_Upsilon'(g_l)/p_Upsilon(g_l) is that same
    // log-derivative at g_l.
    const double c = (prm->dist_law == PSCA_DIST_LINEAR ? 1.0 : 2.0) / beta + 1.0;
    a.dens_c = (float)c;
    a.h2_b = (float)(-c / gl);
  }
  return a;
}

inline hipStream_t as_stream(void *s) { return (hipStream_t)s; }
int launch_ok() { return hipGetLastError() == hipSuccess ? PSCA_OK : PSCA_EHIP; }

// One instantiation of k_psca with its block size.
struct KernelChoice {
  const void *fn;
  int threads;
  int lpmax;
};

KernelChoice pick_kernel(int Lp) {
  switch (Lp) {
    case 16: return {(const void *)k_psca<16, 512>, 512, 16};
    case 32: return {(const void *)k_psca<32, 512>, 512, 32};
    case 48: return {(const void *)k_psca<48, 512>, 512, 48};
    case 64: return {(const void *)k_psca<64, 512>, 512, 64};
    case 80: return {(const void *)k_psca<80, 512>, 512, 80};
    default: return {(const void *)k_psca<96, 512>, 512, 96};
  }
}

// Workgroups of `kc` that fit on the device at once with `lds` bytes of LDS.
int max_coresident(psca_ctx *ctx, const KernelChoice &kc, size_t lds) {
  if (ctx->occ_fn != kc.fn || ctx->occ_lds != lds) {
    (void)hipFuncSetAttribute(kc.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kc.fn, kc.threads, lds) != hipSuccess) {
      (void)hipGetLastError();
      per_cu = 0;
    }
    ctx->occ_fn = kc.fn;
    ctx->occ_lds = lds;
    ctx->occ_per_cu = per_cu;
  }
  return ctx->occ_per_cu * ctx->n_cu;
}

// Launch plan of one instance: 16-column blocks per workgroup, workgroups,
// LDS bytes and workspace bytes.
struct InstPlan {
  int Lp, ncb, NT, G;
  size_t lds, ws;
};

size_t ws_bytes_of(int Lp, int G, int N) {
  const size_t E = (size_t)(Lp / 16) * (Lp / 16 + 1) / 2 * 256;
  return align_up((size_t)G * E * sizeof(float2)) + align_up(E * sizeof(float2)) +
         align_up((size_t)G * 16 * sizeof(unsigned)) + 3 * align_up(sizeof(unsigned)) +
         align_up(2 * (size_t)N * sizeof(float));
}

// Point the instance's work buffers into `base` (laid out as ws_bytes_of).
void bind_ws(CoopArgs &a, char *base, const InstPlan &p) {
  const size_t E = (size_t)(p.Lp / 16) * (p.Lp / 16 + 1) / 2 * 256;
  size_t off = 0;
  a.pstride = E;
  a.partials = (float2 *)(base + off); off += align_up((size_t)p.G * E * sizeof(float2));
  a.sigma = (float2 *)(base + off);    off += align_up(E * sizeof(float2));
  a.bar.arrive = (unsigned *)(base + off); off += align_up((size_t)p.G * 16 * sizeof(unsigned));
  a.bar.release = (unsigned *)(base + off); off += align_up(sizeof(unsigned));
  a.bar.abort_flag = (int32_t *)(base + off); off += align_up(sizeof(unsigned));
  if (!a.status) a.status = (int32_t *)(base + off);
  off += align_up(sizeof(unsigned));
  a.a.xg = (float *)(base + off);   // [2][N] iterate exchange (MAP-K2)
}

void fill_args(CoopArgs &a, const float2 *Sh, const float2 *S, int L, int N, const psca_params *prm, int iters,
               float rho_fixed, const float *x_in, float *x_out, float *q_out, float *r_out, float *xt_out,
               int32_t *status, const InstPlan &p) {
  a.S = S;
  a.Sh = Sh;
  a.L = L;
  a.N = N;
  a.G = p.G;
  a.ncb = p.ncb;
  a.NT = p.NT;
  a.iters = iters;
  a.rho0 = prm->rho0;
  a.rho_decay = prm->rho_decay;
  a.rho_dev = (rho_fixed >= 0.0f) ? nullptr : prm->rho;
  a.rho_fixed = rho_fixed;
  a.sigma2 = prm->sigma2;
  a.a = make_step_args(prm);
  a.x_in = x_in;
  a.x_out = x_out;
  a.q_out = q_out;
  a.r_out = r_out;
  a.xt_out = xt_out;
  a.x_hist = nullptr;
  a.status = status;
}

int run_large_team(psca_ctx *ctx, const float2 *Sh, const float2 *S, int L, int N, const psca_params *prm,
                   int iters, float rho_fixed, const float *x_in, float *x_out, float *q_out, float *r_out,
                   float *xt_out, int32_t *status, hipStream_t st, float *x_hist);

// Runs k_psca for `iters` iterations from x_in (null: zeros).
int run_detect(psca_ctx *ctx, const float2 *Sh, const float2 *S, int L, int N, const psca_params *prm,
               int iters, float rho_fixed, const float *x_in, float *x_out, float *q_out, float *r_out,
               float *xt_out, int32_t *status, hipStream_t st, float *x_hist = nullptr, char *fixed_ws = nullptr,
               size_t fixed_bytes = 0) {
  const int Lp = (L + 15) & ~15;
  if (fixed_ws && Lp > kMaxLdsL) return PSCA_ENOTSUP;   // the fixed workspace serves L <= 96
  if (Lp > kMaxLdsL)
    return run_large_team(ctx, Sh, S, L, N, prm, iters, rho_fixed, x_in, x_out, q_out, r_out, xt_out, status, st,
                          x_hist);
  const KernelChoice kc = pick_kernel(Lp);
  InstPlan p{};
  for (int ncb = 1;; ++ncb) {   // occupancy depends on the tile's LDS
    if (ncb > kMaxNcb) return PSCA_ENOTSUP;
    const int NT = 16 * ncb, G = (N + NT - 1) / NT;
    const size_t lds = lds_bytes(Lp, NT, kc.threads / 64);
    const int cap = max_coresident(ctx, kc, lds);
    if (cap <= 0) return PSCA_ENOTSUP;
    if (G <= cap) {
      p = InstPlan{Lp, ncb, NT, G, lds, ws_bytes_of(Lp, G, N)};
      break;
    }
  }
  int rc;
  if (fixed_ws) {
    if (p.ws > fixed_bytes) return PSCA_ENOTSUP;
  } else if ((rc = ensure_ws(ctx, p.ws)) != PSCA_OK) {
    return rc;
  }
  CoopArgs a;
  fill_args(a, Sh, S, L, N, prm, iters, rho_fixed, x_in, x_out, q_out, r_out, xt_out, status, p);
  a.x_hist = x_hist;
  bind_ws(a, fixed_ws ? fixed_ws : (char *)ctx->ws, p);
  hipLaunchKernelGGL(k_prepare, dim3(1), dim3(256), 0, st, a.bar.arrive, p.G, a.bar.release, a.bar.abort_flag,
                     a.status);
  if ((rc = launch_ok()) != PSCA_OK) return rc;
  void *args[] = {&a};
  if (hipLaunchCooperativeKernel(kc.fn, dim3(p.G), dim3(kc.threads), args, (unsigned)p.lds, st) != hipSuccess) {
    (void)hipGetLastError();
    return PSCA_EHIP;
  }
  return PSCA_OK;
}

// Stage `bytes` of launch descriptors: returns the pinned host buffer to fill;
// the previous copy out of it has completed.
int stage_desc(psca_ctx *ctx, size_t bytes, char **host) {
  if (ctx->desc_pending) {
    if (hipEventSynchronize(ctx->desc_done) != hipSuccess) return PSCA_EHIP;
    ctx->desc_pending = false;
  }
  if (bytes > ctx->desc_bytes) {
    if (ctx->hdesc) (void)hipHostFree(ctx->hdesc);
    ctx->hdesc = nullptr;
    if (ctx->ddesc) {
      if (hipDeviceSynchronize() != hipSuccess) return PSCA_EHIP;
      (void)hipFree(ctx->ddesc);
      ctx->ddesc = nullptr;
    }
    ctx->desc_bytes = 0;
    const size_t want = bytes + bytes / 2;
    if (hipHostMalloc(&ctx->hdesc, want, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      ctx->hdesc = nullptr;
      return PSCA_ENOMEM;
    }
    if (hipMalloc(&ctx->ddesc, want) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipHostFree(ctx->hdesc);
      ctx->hdesc = ctx->ddesc = nullptr;
      return PSCA_ENOMEM;
    }
    ctx->desc_bytes = want;
  }
  *host = (char *)ctx->hdesc;
  return PSCA_OK;
}

// ---- backward of one unrolled layer ------------------------------------------
const void *pick_back(int Lp) {
  switch (Lp) {
    case 16: return (const void *)k_psca_back<16>;
    case 32: return (const void *)k_psca_back<32>;
    case 48: return (const void *)k_psca_back<48>;
    default: return (const void *)k_psca_back<64>;
  }
}

int run_layer_backward(psca_ctx *ctx, const float2 *Sh, const float2 *S, int L, int N, const psca_params *prm,
                       float rho, const float *x_in, const float *v, float *grad_x, float *grad_rho,
                       int32_t *status, hipStream_t st) {
  const int Lp = (L + 15) & ~15;
  const KernelChoice kc{pick_back(Lp), 512, Lp};
  InstPlan p{};
  for (int ncb = 1;; ++ncb) {
    if (ncb > kMaxNcb) return PSCA_ENOTSUP;
    const int NT = 16 * ncb, G = (N + NT - 1) / NT;
    const size_t lds = lds_back_bytes(Lp, NT, 8);
    if (lds > 159 * 1024) return PSCA_ENOTSUP;
    const int cap = max_coresident(ctx, kc, lds);
    if (cap <= 0) return PSCA_ENOTSUP;
    if (G <= cap) {
      p = InstPlan{Lp, ncb, NT, G, lds, 0};
      break;
    }
  }
  const size_t E = (size_t)(Lp / 16) * (Lp / 16 + 1) / 2 * 256;
  const size_t o_pa = 0;
  const size_t o_pb = align_up(o_pa + (size_t)p.G * E * sizeof(float2));
  const size_t o_sig = align_up(o_pb + (size_t)p.G * E * sizeof(float2));
  const size_t o_ga = align_up(o_sig + E * sizeof(float2));
  const size_t o_gb = align_up(o_ga + E * sizeof(float2));
  const size_t o_arr = align_up(o_gb + E * sizeof(float2));
  const size_t o_rel = align_up(o_arr + (size_t)p.G * 16 * sizeof(unsigned));
  const size_t o_abt = align_up(o_rel + sizeof(unsigned));
  const size_t o_st = align_up(o_abt + sizeof(unsigned));
  const size_t o_rp = align_up(o_st + sizeof(unsigned));
  const size_t total = align_up(o_rp + (size_t)p.G * sizeof(float));
  int rc = ensure_ws(ctx, total);
  if (rc != PSCA_OK) return rc;
  char *base = (char *)ctx->ws;
  BackArgs b;
  fill_args(b.c, Sh, S, L, N, prm, 1, rho, x_in, nullptr, nullptr, nullptr, nullptr, status, p);
  b.c.partials = (float2 *)(base + o_pa);
  b.c.pstride = E;
  b.c.sigma = (float2 *)(base + o_sig);
  b.c.bar.arrive = (unsigned *)(base + o_arr);
  b.c.bar.release = (unsigned *)(base + o_rel);
  b.c.bar.abort_flag = (int32_t *)(base + o_abt);
  if (!b.c.status) b.c.status = (int32_t *)(base + o_st);
  b.grad_rho = grad_rho;
  b.rho = rho;
  b.v = v;
  b.grad_x = grad_x;
  b.rho_part = (float *)(base + o_rp);
  b.partials_b = (float2 *)(base + o_pb);
  b.gram_a = (float2 *)(base + o_ga);
  b.gram_b = (float2 *)(base + o_gb);
  hipLaunchKernelGGL(k_prepare, dim3(1), dim3(256), 0, st, b.c.bar.arrive, p.G, b.c.bar.release,
                     b.c.bar.abort_flag, b.c.status);
  if ((rc = launch_ok()) != PSCA_OK) return rc;
  void *args[] = {&b};
  if (hipLaunchCooperativeKernel(kc.fn, dim3(p.G), dim3(512), args, (unsigned)p.lds, st) != hipSuccess) {
    (void)hipGetLastError();
    return PSCA_EHIP;
  }
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, st, (const float *)b.rho_part, p.G, grad_rho);
  return launch_ok();
}

// ---- batches: persistent teams ---------------------------------------------
constexpr size_t kMaxLds = 159 * 1024;   // dynamic LDS per workgroup (160 KB on gfx950, less the static part)

struct BatchPlan {
  int B = 0, T = 0, n_teams = 0;   // T: the team specification (team_spec_ok)
  size_t lds = 0;
  std::vector<psca_problem> probs;
  std::vector<InstPlan> ip;
  std::vector<int> iters;        // per instance (capped while tuning)
  std::vector<int> team_of;
  std::vector<int> lists, offsets;
  std::vector<int> team_start;   // [n_teams + 1]: first logical workgroup of each team; the grid
  std::vector<size_t> ws_off;    // per instance: Sigma, barrier words, status
  std::vector<size_t> part_team_off;   // per team partials (its ranks x E_max entries), from part_off
  size_t part_off = 0;
  size_t E_max = 0;
  size_t ws_bytes = 0;
  bool large = false;            // pilot lengths 97..256: k_psca_large_teams
  std::vector<int> gv;           // large: Gram tiles per instance
};

size_t packed_entries(int Lp) { return (size_t)(Lp / 16) * (Lp / 16 + 1) / 2 * 256; }
// Lower 16x16 blocks of an L x L matrix (the workgroups of k_sample_cov).
int packed_blocks(int L) { const int Lb = (L + 15) / 16; return Lb * (Lb + 1) / 2; }

size_t inst_ws_bytes(int Lp, int G, int N) {
  return align_up(packed_entries(Lp) * sizeof(float2)) + align_up((size_t)G * 16 * sizeof(unsigned)) +
         3 * align_up(sizeof(unsigned)) + align_up(2 * (size_t)N * sizeof(float));
}

// Largest column tile (multiple of 16, at most 16 kMaxNcb) whose LDS fits a workgroup.
int max_tile(int Lp) {
  for (int ncb = kMaxNcb; ncb >= 1; --ncb)
    if (lds_bytes(Lp, 16 * ncb, kBatchThreads / 64) <= kMaxLds) return 16 * ncb;
  return 0;
}

// Smallest team size that can run every instance of the batch.
int min_team(int B, const psca_problem *pr) {
  int T0 = 1;
  for (int b = 0; b < B; ++b) {
    const int nt = max_tile((pr[b].L + 15) & ~15);
    if (nt == 0) return -1;
    T0 = std::max(T0, (pr[b].N + nt - 1) / nt);
  }
  return T0;
}

// Default team size: one team per instance, as large as useful, when the
// batch fits the GPU at once; otherwise the smallest teams (most concurrency).
int default_team(int B, const psca_problem *pr, int cap) {
  const int T0 = min_team(B, pr);
  if (T0 < 0 || T0 > cap) return -1;
  if ((long long)B * T0 <= cap) {
    int want = 1;
    for (int b = 0; b < B; ++b) want = std::max(want, (pr[b].N + 15) / 16);
    return std::max(T0, std::min(cap / B, want));
  }
  return T0;
}

// Team specification of a batch plan: spec > 0, teams of spec workgroups;
// spec < 0, mixed teams: each instance gets a team sized for tiles of about
// -spec columns (a multiple of 16, at most 16 kMaxNcb).
bool team_spec_ok(int spec, int cap) {
  if (spec > 0) return spec <= cap;
  return spec < 0 && (-spec) % 16 == 0 && -spec <= 16 * kMaxNcb;
}

// Longest-first assignment of `items` (indices into cost) to the teams
// [t0, t0 + n): each goes to the least loaded team so far.
void assign_longest_first(std::vector<int> items, const std::vector<double> &cost, int t0, int n,
                          std::vector<std::vector<int>> &team, std::vector<int> &team_of) {
  std::stable_sort(items.begin(), items.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  std::vector<double> load(n, 0.0);
  for (int b : items) {
    const int t = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    team[t0 + t].push_back(b);
    team_of[b] = t0 + t;
    load[t] += cost[b];
  }
}

// Plans a batch: team sizes, tiles, longest-first assignment of instances to
// teams (the estimated cost of an iteration grows with the pivot blocks and
// with the tile's MFMA work) and the workspace layout.
//  * spec > 0: n = min(cap / spec, B) teams of spec workgroups, every
//    instance on any of them;
//  * spec < 0: instance b needs a team of T_b = max(ceil(N_b / max tile),
//    ceil(N_b / -spec)) workgroups, rounded up to the next of 1, 2, 4, 6,
//    8, 12, 16, 24, 32, 48, ... (powers of two and their 1.5 multiples).
//    Instances with the same T_b form a class with its own teams; while one
//    team per class would not fit the grid, the smallest class joins the
//    next larger one.  Every class starts with one team, then teams are
//    added to the class with the most work per team while the grid fits.
//    Small instances then run on small teams, several at a time, instead of
//    idling most of a team sized for the largest one.
// A mixed specification that yields a single class is the uniform plan of
// that team size and is recorded as such (plan.T).
// iters_cap >= 0 caps every instance's iteration count (tuning runs).
int make_batch_plan(int B, const psca_problem *pr, int spec, int cap, BatchPlan &plan, int iters_cap) {
  if (!team_spec_ok(spec, cap)) return PSCA_EINVAL;
  plan = BatchPlan();
  plan.B = B;
  plan.T = spec;
  plan.probs.assign(pr, pr + B);
  plan.ip.resize(B);
  plan.iters.resize(B);
  std::vector<int> tsize(B, spec);   // team size of each instance
  for (int b = 0; b < B; ++b) {
    const int mt = max_tile((pr[b].L + 15) & ~15);
    if (mt == 0) return PSCA_ENOTSUP;
    if (spec < 0) {
      const int need = std::max((pr[b].N + mt - 1) / mt, (pr[b].N - spec - 1) / (-spec));
      int T = 1;   // the ladder 1, 2, 4, 6, 8, 12, 16, 24, 32, 48, ...
      while (T < need) T = T < 4 ? 2 * T : ((T & (T - 1)) == 0 ? T + T / 2 : T / 3 * 4);
      tsize[b] = T;
    }
    if (tsize[b] > cap) return PSCA_ENOTSUP;
  }
  if (spec < 0) {   // merge the smallest class into the next larger one while one team each overflows
    std::vector<int> sizes(tsize);
    std::sort(sizes.begin(), sizes.end());
    sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
    long long used = 0;
    for (int v : sizes) used += v;
    size_t first = 0;
    while (used > cap && first + 1 < sizes.size()) {
      used -= sizes[first];
      for (int &t : tsize)
        if (t == sizes[first]) t = sizes[first + 1];
      ++first;
    }
    if (used > cap) return PSCA_ENOTSUP;
  }
  std::vector<double> cost(B);
  size_t E_max = 0;
  for (int b = 0; b < B; ++b) {
    InstPlan &q = plan.ip[b];
    q.Lp = (pr[b].L + 15) & ~15;
    const int mt = max_tile(q.Lp);
    const int T = tsize[b];
    const int per = (pr[b].N + T - 1) / T;
    q.NT = std::max(16, (per + 15) & ~15);
    if (q.NT > mt) return PSCA_ENOTSUP;
    q.ncb = q.NT / 16;
    // every member of the team takes part (tiles past N are empty), so a
    // team moves through its list in step and no member waits at an
    // instance for team mates still busy with earlier ones
    q.G = T;
    q.lds = lds_bytes(q.Lp, q.NT, kBatchThreads / 64);
    q.ws = inst_ws_bytes(q.Lp, q.G, pr[b].N);
    plan.lds = std::max(plan.lds, q.lds);
    plan.iters[b] = iters_cap >= 0 ? std::min(pr[b].prm.iters, iters_cap) : pr[b].prm.iters;
    const double Lb = q.Lp / 16;
    cost[b] = (double)plan.iters[b] * (3.0 * Lb + 0.05 * q.ncb * Lb * Lb + 8.0);
    E_max = std::max(E_max, packed_entries(q.Lp));
  }
  std::vector<int> team_size;   // per team
  std::vector<std::vector<int>> team;
  plan.team_of.resize(B);
  if (spec > 0) {
    const int n = std::max(1, std::min(cap / spec, B));
    team_size.assign(n, spec);
    team.resize(n);
    std::vector<int> all(B);
    for (int b = 0; b < B; ++b) all[b] = b;
    assign_longest_first(all, cost, 0, n, team, plan.team_of);
  } else {
    std::map<int, std::vector<int>, std::greater<int>> cls;   // team size -> instances, largest first
    for (int b = 0; b < B; ++b) cls[plan.ip[b].G].push_back(b);
    std::vector<int> size_of, count;
    std::vector<double> work;
    int used = 0;
    for (const auto &kv : cls) {
      size_of.push_back(kv.first);
      double w = 0.0;
      for (int b : kv.second) w += cost[b];
      work.push_back(w);
      count.push_back(1);
      used += kv.first;
    }
    if (used > cap) return PSCA_ENOTSUP;
    if (cls.size() == 1) {   // one team size for all: exactly the uniform plan of that size
      const int T = cls.begin()->first;
      plan.T = T;
      const int n = std::max(1, std::min(cap / T, B));
      team_size.assign(n, T);
      team.resize(n);
      assign_longest_first(cls.begin()->second, cost, 0, n, team, plan.team_of);
      cls.clear();
    }
    for (;;) {   // one more team for the class with the most work per team that still fits
      int best = -1, c = 0;
      double best_w = 0.0;
      for (const auto &kv : cls) {
        if (count[c] < (int)kv.second.size() && size_of[c] <= cap - used && work[c] / count[c] > best_w) {
          best = c;
          best_w = work[c] / count[c];
        }
        ++c;
      }
      if (best < 0) break;
      ++count[best];
      used += size_of[best];
    }
    int c = 0;
    for (const auto &kv : cls) {
      const int t0 = (int)team_size.size();
      for (int k = 0; k < count[c]; ++k) team_size.push_back(size_of[c]);
      team.resize(team_size.size());
      assign_longest_first(kv.second, cost, t0, count[c], team, plan.team_of);
      ++c;
    }
  }
  plan.n_teams = (int)team_size.size();
  plan.team_start.assign(1, 0);
  for (int t = 0; t < plan.n_teams; ++t) plan.team_start.push_back(plan.team_start.back() + team_size[t]);
  plan.offsets.push_back(0);
  for (int t = 0; t < plan.n_teams; ++t) {
    for (int b : team[t]) plan.lists.push_back(b);
    plan.offsets.push_back((int)plan.lists.size());
  }
  size_t off = 0;
  plan.ws_off.resize(B);
  for (int b = 0; b < B; ++b) {
    plan.ws_off[b] = off;
    off += plan.ip[b].ws;
  }
  plan.part_off = off;
  plan.E_max = E_max;
  size_t part = 0;
  for (int t = 0; t < plan.n_teams; ++t) {
    plan.part_team_off.push_back(part);
    part += align_up((size_t)team_size[t] * E_max * sizeof(float2));
  }
  plan.ws_bytes = off + part;
  return PSCA_OK;
}

// ---- large pilot lengths (97..256): teams on k_psca_large_teams ------------
constexpr int kLargeThreads = 512;

// Widest Gram tile (16..80 columns) whose LDS fits a workgroup.
int large_tile(int Lp) {
  for (int nt = 80; nt >= 16; nt -= 16)
    if (lds_large_fwd_bytes(Lp, nt, kLargeThreads) <= kMaxLds) return nt;
  return 0;
}

// Per-instance workspace of a large-L launch: packed Sigma, Sigma - SigmaHat
// and L, T barrier words, release/abort/status words, the iterate exchange
// [2][N] (MAP-K2), the iterate [N] and an Lp x Lp matrix for phase C2.
size_t large_inst_ws_bytes(int Lp, int T, int N) {
  const size_t E = packed_entries(Lp);
  return 3 * align_up(E * sizeof(float2)) + align_up((size_t)T * 16 * sizeof(unsigned)) +
         3 * align_up(sizeof(unsigned)) + align_up(2 * (size_t)N * sizeof(float)) + align_up((size_t)N * sizeof(float)) +
         align_up((size_t)Lp * Lp * sizeof(float2));
}

// Points a descriptor's work buffers into `w` (laid out as large_inst_ws_bytes).
void bind_large_ws(LargeTeamArgs &a, char *w, int Lp, int T, int N) {
  const size_t E = packed_entries(Lp);
  a.c.sigma = (float2 *)w;          w += align_up(E * sizeof(float2));
  a.delta = (float2 *)w;            w += align_up(E * sizeof(float2));
  a.lbuf = (float2 *)w;             w += align_up(E * sizeof(float2));
  a.c.bar.arrive = (unsigned *)w;   w += align_up((size_t)T * 16 * sizeof(unsigned));
  a.c.bar.release = (unsigned *)w;  w += align_up(sizeof(unsigned));
  a.c.bar.abort_flag = (int32_t *)w; w += align_up(sizeof(unsigned));
  if (!a.c.status) a.c.status = (int32_t *)w;
  w += align_up(sizeof(unsigned));
  a.c.a.xg = (float *)w;            w += align_up(2 * (size_t)N * sizeof(float));
  a.xw = (float *)w;                w += align_up((size_t)N * sizeof(float));
  a.xfull = (float2 *)w;
}

// Plans a batch of large-L instances on uniform teams of T workgroups:
// n = min(cap / T, B) teams, instances assigned longest first (estimated
// cost per iteration: the contraction, N L^2, plus the serial block steps
// of the factorisation).  Each team owns one partial region sized for the
// largest Gv E of its instances (they run one after the other).
int make_large_plan(int B, const psca_problem *pr, int T, int cap, BatchPlan &plan, int iters_cap) {
  if (T < 1 || T > cap) return PSCA_EINVAL;
  plan = BatchPlan();
  plan.large = true;
  plan.B = B;
  plan.T = T;
  plan.probs.assign(pr, pr + B);
  plan.ip.resize(B);
  plan.iters.resize(B);
  plan.gv.resize(B);
  std::vector<double> cost(B);
  for (int b = 0; b < B; ++b) {
    InstPlan &q = plan.ip[b];
    q.Lp = (pr[b].L + 15) & ~15;
    q.NT = large_tile(q.Lp);
    if (q.NT == 0) return PSCA_ENOTSUP;
    q.ncb = q.NT / 16;
    q.G = T;
    q.lds = lds_large_fwd_bytes(q.Lp, q.NT, kLargeThreads);
    q.ws = large_inst_ws_bytes(q.Lp, T, pr[b].N);
    plan.gv[b] = (pr[b].N + q.NT - 1) / q.NT;
    plan.lds = std::max(plan.lds, q.lds);
    plan.iters[b] = iters_cap >= 0 ? std::min(pr[b].prm.iters, iters_cap) : pr[b].prm.iters;
    const double Lb = q.Lp / 16;
    cost[b] = (double)plan.iters[b] * ((double)pr[b].N * q.Lp * q.Lp / T + 2.0e5 * Lb);
  }
  const int n = std::max(1, std::min(cap / T, B));
  std::vector<std::vector<int>> team(n);
  plan.team_of.resize(B);
  std::vector<int> all(B);
  for (int b = 0; b < B; ++b) all[b] = b;
  assign_longest_first(all, cost, 0, n, team, plan.team_of);
  plan.n_teams = n;
  plan.team_start.assign(1, 0);
  for (int t = 0; t < n; ++t) plan.team_start.push_back(plan.team_start.back() + T);
  plan.offsets.push_back(0);
  for (int t = 0; t < n; ++t) {
    for (int b : team[t]) plan.lists.push_back(b);
    plan.offsets.push_back((int)plan.lists.size());
  }
  size_t off = 0;
  plan.ws_off.resize(B);
  for (int b = 0; b < B; ++b) {
    plan.ws_off[b] = off;
    off += plan.ip[b].ws;
  }
  plan.part_off = off;
  size_t part = 0;
  for (int t = 0; t < n; ++t) {
    size_t need = 0;
    for (int b : team[t]) need = std::max(need, (size_t)plan.gv[b] * packed_entries(plan.ip[b].Lp));
    plan.part_team_off.push_back(part);
    part += align_up(need * sizeof(float2));
  }
  plan.ws_bytes = off + part;
  return PSCA_OK;
}

void bind_large_batch(const BatchPlan &plan, char *base, LargeTeamArgs *out) {
  for (int b = 0; b < plan.B; ++b) {
    const psca_problem &q = plan.probs[b];
    const InstPlan &ip = plan.ip[b];
    LargeTeamArgs a;
    fill_args(a.c, (const float2 *)q.Sigma_hat, (const float2 *)q.S, q.L, q.N, &q.prm, plan.iters[b], -1.0f,
              q.prm.x0, q.x_out, nullptr, nullptr, nullptr, q.status, ip);
    bind_large_ws(a, base + plan.ws_off[b], ip.Lp, ip.G, q.N);
    a.c.x_hist = q.x_hist;
    a.c.partials = (float2 *)(base + plan.part_off + plan.part_team_off[plan.team_of[b]]);
    a.c.pstride = packed_entries(ip.Lp);
    a.Gv = plan.gv[b];
    out[b] = a;
  }
}

// Descriptors of `plan` with its workspace at `base`.
void bind_batch(const BatchPlan &plan, char *base, CoopArgs *out) {
  for (int b = 0; b < plan.B; ++b) {
    const psca_problem &q = plan.probs[b];
    const InstPlan &ip = plan.ip[b];
    CoopArgs a;
    fill_args(a, (const float2 *)q.Sigma_hat, (const float2 *)q.S, q.L, q.N, &q.prm, plan.iters[b], -1.0f,
              q.prm.x0, q.x_out, nullptr, nullptr, nullptr, q.status, ip);
    char *w = base + plan.ws_off[b];
    a.sigma = (float2 *)w;                w += align_up(packed_entries(ip.Lp) * sizeof(float2));
    a.bar.arrive = (unsigned *)w;         w += align_up((size_t)ip.G * 16 * sizeof(unsigned));
    a.bar.release = (unsigned *)w;        w += align_up(sizeof(unsigned));
    a.bar.abort_flag = (int32_t *)w;      w += align_up(sizeof(unsigned));
    if (!a.status) a.status = (int32_t *)w;
    w += align_up(sizeof(unsigned));
    a.a.xg = (float *)w;                  // [2][N] iterate exchange (MAP-K2)
    a.x_hist = q.x_hist;
    // every rank of a team owns the same slot for all of the team's instances:
    // a rank that sits out an instance may start the next one early
    a.partials = (float2 *)(base + plan.part_off + plan.part_team_off[plan.team_of[b]]);
    a.pstride = plan.E_max;
    out[b] = a;
  }
}

// Host image of a plan's device arrays: descriptors, lists, offsets, team starts.
size_t desc_bytes(const BatchPlan &plan) {
  return (size_t)plan.B * (plan.large ? sizeof(LargeTeamArgs) : sizeof(CoopArgs));
}

size_t batch_image_bytes(const BatchPlan &plan) {
  return align_up(desc_bytes(plan)) + align_up(plan.lists.size() * sizeof(int)) +
         align_up(plan.offsets.size() * sizeof(int)) + align_up(plan.team_start.size() * sizeof(int));
}

void write_batch_image(const BatchPlan &plan, char *ws_base, char *img) {
  if (plan.large) bind_large_batch(plan, ws_base, (LargeTeamArgs *)img);
  else bind_batch(plan, ws_base, (CoopArgs *)img);
  char *p = img + align_up(desc_bytes(plan));
  memcpy(p, plan.lists.data(), plan.lists.size() * sizeof(int));
  p += align_up(plan.lists.size() * sizeof(int));
  memcpy(p, plan.offsets.data(), plan.offsets.size() * sizeof(int));
  p += align_up(plan.offsets.size() * sizeof(int));
  memcpy(p, plan.team_start.data(), plan.team_start.size() * sizeof(int));
}

// Launches a planned batch whose device image is at `dimg`.
int launch_batch(const BatchPlan &plan, const char *dimg, hipStream_t st) {
  const void *descs = (const void *)dimg;
  const int *lists = (const int *)(dimg + align_up(desc_bytes(plan)));
  const int *offsets = (const int *)((const char *)lists + align_up(plan.lists.size() * sizeof(int)));
  const int *team_start = (const int *)((const char *)offsets + align_up(plan.offsets.size() * sizeof(int)));
  int n_teams = plan.n_teams;
  if (plan.large)
    hipLaunchKernelGGL(k_prepare_large_batch, dim3(plan.B), dim3(256), 0, st, (const LargeTeamArgs *)descs);
  else
    hipLaunchKernelGGL(k_prepare_batch, dim3(plan.B), dim3(256), 0, st, (const CoopArgs *)descs);
  int rc = launch_ok();
  if (rc != PSCA_OK) return rc;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess) return PSCA_EHIP;
  const dim3 grid(plan.team_start.back()), block(kBatchThreads);
  const void *fn = plan.large ? (const void *)k_psca_large_teams : (const void *)k_psca_teams;
  if (cs == hipStreamCaptureStatusActive) {
    // graph capture: a plain kernel node; the grid fits the device at once
    if (plan.large)
      hipLaunchKernelGGL(k_psca_large_teams, grid, block, plan.lds, st, (const LargeTeamArgs *)descs, lists,
                         offsets, team_start, n_teams);
    else
      hipLaunchKernelGGL(k_psca_teams, grid, block, plan.lds, st, (const CoopArgs *)descs, lists, offsets,
                         team_start, n_teams);
    return launch_ok();
  }
  void *args[] = {(void *)&descs, (void *)&lists, (void *)&offsets, (void *)&team_start, (void *)&n_teams};
  if (hipLaunchCooperativeKernel(fn, grid, block, args, (unsigned)plan.lds, st) != hipSuccess) {
    (void)hipGetLastError();
    return PSCA_EHIP;
  }
  return PSCA_OK;
}

int batch_capacity(psca_ctx *ctx) {
  const KernelChoice kc{(const void *)k_psca_teams, kBatchThreads, 96};
  return max_coresident(ctx, kc, kMaxLds);
}

int large_capacity(psca_ctx *ctx) {
  const KernelChoice kc{(const void *)k_psca_large_teams, kLargeThreads, 256};
  return max_coresident(ctx, kc, kMaxLds);
}

// One detection (or iteration, or network forward) with 97 <= L <= 256 on
// one team of k_psca_large_teams: as many workgroups as Gram tiles, up to
// the co-resident grid.
int run_large_team(psca_ctx *ctx, const float2 *Sh, const float2 *S, int L, int N, const psca_params *prm,
                   int iters, float rho_fixed, const float *x_in, float *x_out, float *q_out, float *r_out,
                   float *xt_out, int32_t *status, hipStream_t st, float *x_hist) {
  const int cap = large_capacity(ctx);
  const int Lp = (L + 15) & ~15;
  const int NT = large_tile(Lp);
  if (cap <= 0 || NT == 0) return PSCA_ENOTSUP;
  const int Gv = (N + NT - 1) / NT;
  const int T = std::min(cap, Gv);
  BatchPlan plan;
  plan.large = true;
  plan.B = 1;
  plan.T = T;
  plan.n_teams = 1;
  plan.lds = lds_large_fwd_bytes(Lp, NT, kLargeThreads);
  plan.lists = {0};
  plan.offsets = {0, 1};
  plan.team_start = {0, T};
  const InstPlan ip{Lp, NT / 16, NT, T, plan.lds, large_inst_ws_bytes(Lp, T, N)};
  const size_t E = packed_entries(Lp);
  int rc = ensure_ws(ctx, ip.ws + align_up((size_t)Gv * E * sizeof(float2)));
  if (rc != PSCA_OK) return rc;
  char *base = (char *)ctx->ws;
  LargeTeamArgs a;
  fill_args(a.c, Sh, S, L, N, prm, iters, rho_fixed, x_in, x_out, q_out, r_out, xt_out, status, ip);
  bind_large_ws(a, base, Lp, T, N);
  a.c.x_hist = x_hist;
  a.c.partials = (float2 *)(base + ip.ws);
  a.c.pstride = E;
  a.Gv = Gv;
  const size_t bytes = batch_image_bytes(plan);
  char *host = nullptr;
  if ((rc = stage_desc(ctx, bytes, &host)) != PSCA_OK) return rc;
  char *img = host;
  memcpy(img, &a, sizeof(a));
  img += align_up(desc_bytes(plan));
  memcpy(img, plan.lists.data(), sizeof(int));
  img += align_up(sizeof(int));
  memcpy(img, plan.offsets.data(), 2 * sizeof(int));
  img += align_up(2 * sizeof(int));
  memcpy(img, plan.team_start.data(), 2 * sizeof(int));
  if (hipMemcpyAsync(ctx->ddesc, host, bytes, hipMemcpyHostToDevice, st) != hipSuccess) {
    (void)hipGetLastError();
    return PSCA_EHIP;
  }
  if (hipEventRecord(ctx->desc_done, st) != hipSuccess) return PSCA_EHIP;
  ctx->desc_pending = true;
  return launch_batch(plan, (const char *)ctx->ddesc, st);
}

// ---- layer backward for 65 <= L <= 256 on teams (k_psca_back_large_<lo>_<hi>)
int large_back_tile(int Lp) {
  for (int nt = 64; nt >= 16; nt -= 16)
    if (lds_large_back_bytes(Lp, nt, kLargeThreads) <= kMaxLds) return nt;
  return 0;
}

// Per-instance workspace of a large-L backward: the forward's buffers (Sigma,
// Sigma - SigmaHat, L, barrier and status words, exchange, iterate), packed
// G_a and G_b, b_m and c_m per column block, three per-device vectors and
// the T parts of dL/drho.
size_t large_back_inst_ws_bytes(int Lp, int T, int N) {
  const size_t E = packed_entries(Lp), ncol = (size_t)(N + 15) / 16;
  return large_inst_ws_bytes(Lp, T, N) + 2 * align_up(E * sizeof(float2)) +
         2 * align_up(ncol * (size_t)Lp * 16 * sizeof(float2)) + 3 * align_up((size_t)N * sizeof(float)) +
         align_up((size_t)T * sizeof(float));
}

// The backward kernel for instances of LB = L_p / 16 blocks.
struct BackRange {
  int lo, hi;
  const void *fn;
};
const BackRange kBackRanges[] = {
#define PSCA_BACK_ENTRY(lo, hi) {lo, hi, (const void *)PSCA_BACK_NAME(lo, hi)},
    PSCA_BACK_RANGES(PSCA_BACK_ENTRY)
#undef PSCA_BACK_ENTRY
};
constexpr int kNumBackRanges = (int)(sizeof(kBackRanges) / sizeof(kBackRanges[0]));

int back_range(int L) {
  const int lb = (L + 15) >> 4;
  for (int r = 0; r < kNumBackRanges; ++r)
    if (lb >= kBackRanges[r].lo && lb <= kBackRanges[r].hi) return r;
  return -1;
}

// One launch of the backward of instances `idx` (one range of LB) on uniform
// teams of T workgroups (T: the co-resident grid shared evenly, and for a
// single instance as many workgroups as Gram tiles), its workspace at `base`.
struct BackLaunch {
  int range = -1, T = 0, n = 0;
  size_t lds = 0, bytes = 0;
  std::vector<int> idx, lp, nt, gv, team_of;
  std::vector<std::vector<int>> team;
  std::vector<size_t> off, part_off, part_need;
  BatchPlan geo;   // lists, offsets and team starts
};

int plan_large_back(psca_ctx *ctx, const psca_back_problem *pr, BackLaunch &bl) {
  const KernelChoice kc{kBackRanges[bl.range].fn, kLargeThreads, 256};
  const int cap = max_coresident(ctx, kc, kMaxLds);
  if (cap <= 0) return PSCA_ENOTSUP;
  const int B = (int)bl.idx.size();
  bl.lp.resize(B);
  bl.nt.resize(B);
  bl.gv.resize(B);
  for (int k = 0; k < B; ++k) {
    const psca_back_problem &q = pr[bl.idx[k]];
    bl.lp[k] = (q.L + 15) & ~15;
    bl.nt[k] = large_back_tile(bl.lp[k]);
    if (bl.nt[k] == 0) return PSCA_ENOTSUP;
    bl.gv[k] = (q.N + bl.nt[k] - 1) / bl.nt[k];
  }
  bl.T = B == 1 ? std::min(cap, bl.gv[0]) : std::max(1, cap / B);
  bl.n = std::max(1, std::min(cap / bl.T, B));
  std::vector<double> cost(B);
  for (int k = 0; k < B; ++k) cost[k] = (double)pr[bl.idx[k]].N * bl.lp[k] * bl.lp[k] + 2.0e5 * (bl.lp[k] / 16);
  bl.team.assign(bl.n, {});
  bl.team_of.assign(B, 0);
  std::vector<int> all(B);
  for (int k = 0; k < B; ++k) all[k] = k;
  assign_longest_first(all, cost, 0, bl.n, bl.team, bl.team_of);
  bl.geo = BatchPlan();
  bl.geo.large = true;
  bl.geo.B = B;
  bl.geo.T = bl.T;
  bl.geo.n_teams = bl.n;
  bl.geo.team_start.assign(1, 0);
  for (int t = 0; t < bl.n; ++t) bl.geo.team_start.push_back(bl.geo.team_start.back() + bl.T);
  bl.geo.offsets.push_back(0);
  for (int t = 0; t < bl.n; ++t) {
    for (int k : bl.team[t]) bl.geo.lists.push_back(k);
    bl.geo.offsets.push_back((int)bl.geo.lists.size());
  }
  bl.off.resize(B);
  size_t total = 0;
  for (int k = 0; k < B; ++k) {
    bl.off[k] = total;
    total += large_back_inst_ws_bytes(bl.lp[k], bl.T, pr[bl.idx[k]].N);
    bl.lds = std::max(bl.lds, lds_large_back_bytes(bl.lp[k], bl.nt[k], kLargeThreads));
  }
  bl.part_off.assign(bl.n, 0);
  bl.part_need.assign(bl.n, 0);
  for (int t = 0; t < bl.n; ++t) {   // per team: the partials of Sigma / G_a and of G_b
    for (int k : bl.team[t]) bl.part_need[t] = std::max(bl.part_need[t], (size_t)bl.gv[k] * packed_entries(bl.lp[k]));
    bl.part_off[t] = total;
    total += 2 * align_up(bl.part_need[t] * sizeof(float2));
  }
  bl.bytes = total;
  return PSCA_OK;
}

int launch_large_back(psca_ctx *ctx, const psca_back_problem *pr, float rho, const BackLaunch &bl, char *base,
                      hipStream_t st) {
  const int B = (int)bl.idx.size();
  const BatchPlan &plan = bl.geo;
  const size_t bytes = align_up((size_t)B * sizeof(LargeBackArgs)) + align_up(plan.lists.size() * sizeof(int)) +
                       align_up(plan.offsets.size() * sizeof(int)) + align_up(plan.team_start.size() * sizeof(int));
  char *host = nullptr;
  int rc;
  if ((rc = stage_desc(ctx, bytes, &host)) != PSCA_OK) return rc;
  LargeBackArgs *d = (LargeBackArgs *)host;
  for (int k = 0; k < B; ++k) {
    const psca_back_problem &q = pr[bl.idx[k]];
    const InstPlan ip{bl.lp[k], bl.nt[k] / 16, bl.nt[k], bl.T, bl.lds, 0};
    LargeBackArgs a;
    fill_args(a.f.c, (const float2 *)q.Sigma_hat, (const float2 *)q.S, q.L, q.N, &q.prm, 1, rho, q.x_in, nullptr,
              nullptr, nullptr, nullptr, q.status, ip);
    char *w = base + bl.off[k];
    bind_large_ws(a.f, w, bl.lp[k], bl.T, q.N);
    w += large_inst_ws_bytes(bl.lp[k], bl.T, q.N);
    const size_t E = packed_entries(bl.lp[k]), ncol = (size_t)(q.N + 15) / 16;
    a.gram_a = (float2 *)w;   w += align_up(E * sizeof(float2));
    a.gram_b = (float2 *)w;   w += align_up(E * sizeof(float2));
    a.bmat = (float2 *)w;     w += align_up(ncol * (size_t)bl.lp[k] * 16 * sizeof(float2));
    a.cmat = (float2 *)w;     w += align_up(ncol * (size_t)bl.lp[k] * 16 * sizeof(float2));
    a.wa = (float *)w;        w += align_up((size_t)q.N * sizeof(float));
    a.wb = (float *)w;        w += align_up((size_t)q.N * sizeof(float));
    a.d0 = (float *)w;        w += align_up((size_t)q.N * sizeof(float));
    a.rho_part = (float *)w;
    const int t = bl.team_of[k];
    a.f.c.partials = (float2 *)(base + bl.part_off[t]);
    a.f.c.pstride = E;
    a.partials_b = (float2 *)(base + bl.part_off[t] + align_up(bl.part_need[t] * sizeof(float2)));
    a.f.Gv = bl.gv[k];
    a.rho = rho;
    a.v = q.v;
    a.grad_x = q.grad_x;
    a.grad_rho = q.grad_rho;
    d[k] = a;
  }
  char *p = host + align_up((size_t)B * sizeof(LargeBackArgs));
  memcpy(p, plan.lists.data(), plan.lists.size() * sizeof(int));
  p += align_up(plan.lists.size() * sizeof(int));
  memcpy(p, plan.offsets.data(), plan.offsets.size() * sizeof(int));
  p += align_up(plan.offsets.size() * sizeof(int));
  memcpy(p, plan.team_start.data(), plan.team_start.size() * sizeof(int));
  if (hipMemcpyAsync(ctx->ddesc, host, bytes, hipMemcpyHostToDevice, st) != hipSuccess) {
    (void)hipGetLastError();
    return PSCA_EHIP;
  }
  if (hipEventRecord(ctx->desc_done, st) != hipSuccess) return PSCA_EHIP;
  ctx->desc_pending = true;
  const char *dimg = (const char *)ctx->ddesc;
  const LargeBackArgs *descs = (const LargeBackArgs *)dimg;
  const int *lists = (const int *)(dimg + align_up((size_t)B * sizeof(LargeBackArgs)));
  const int *offsets = (const int *)((const char *)lists + align_up(plan.lists.size() * sizeof(int)));
  const int *team_start = (const int *)((const char *)offsets + align_up(plan.offsets.size() * sizeof(int)));
  int n_teams = bl.n;
  hipLaunchKernelGGL(k_prepare_large_back, dim3(B), dim3(256), 0, st, descs);
  if ((rc = launch_ok()) != PSCA_OK) return rc;
  void *args[] = {(void *)&descs, (void *)&lists, (void *)&offsets, (void *)&team_start, (void *)&n_teams};
  if (hipLaunchCooperativeKernel(kBackRanges[bl.range].fn, dim3(plan.team_start.back()), dim3(kLargeThreads), args,
                                 (unsigned)bl.lds, st) != hipSuccess) {
    (void)hipGetLastError();
    return PSCA_EHIP;
  }
  return PSCA_OK;
}

// B layer backwards (every L in 65..256): one persistent launch per range of
// block counts present (one launch for a batch of one pilot length).
int run_large_backward(psca_ctx *ctx, int B, const psca_back_problem *pr, float rho, hipStream_t st) {
  std::vector<BackLaunch> launches;
  for (int r = 0; r < kNumBackRanges; ++r) {
    BackLaunch bl;
    bl.range = r;
    for (int b = 0; b < B; ++b)
      if (back_range(pr[b].L) == r) bl.idx.push_back(b);
    if (!bl.idx.empty()) launches.push_back(bl);
  }
  size_t total = 0;
  int rc;
  for (auto &bl : launches) {
    if ((rc = plan_large_back(ctx, pr, bl)) != PSCA_OK) return rc;
    total += align_up(bl.bytes);
  }
  if ((rc = ensure_ws(ctx, total)) != PSCA_OK) return rc;
  size_t at = 0;
  for (auto &bl : launches) {
    if ((rc = launch_large_back(ctx, pr, rho, bl, (char *)ctx->ws + at, st)) != PSCA_OK) return rc;
    at += align_up(bl.bytes);
  }
  return PSCA_OK;
}

// Whole-batch pilot-length class: 0 when every L <= 96 (k_psca_teams), 1
// when every L is 97..256 (k_psca_large_teams), -1 for a batch mixing both.
int batch_class(int B, const psca_problem *pr) {
  int small = 0, large = 0;
  for (int b = 0; b < B; ++b) (pr[b].L > kMaxLdsL ? large : small) = 1;
  return (small && large) ? -1 : large;
}

// Default team size of a large-L batch: the co-resident grid shared evenly
// by the instances, at least one workgroup each.
int default_large_team(int B, int cap) { return std::max(1, cap / std::max(1, B)); }

// Plan of either class; `spec` as psca_plan_create takes it (large-L
// batches: uniform teams only).
int make_plan(int B, const psca_problem *pr, int spec, int cap, BatchPlan &plan, int iters_cap) {
  if (batch_class(B, pr) == 1) return make_large_plan(B, pr, spec, cap, plan, iters_cap);
  return make_batch_plan(B, pr, spec, cap, plan, iters_cap);
}

uint64_t batch_signature(int B, const psca_problem *pr) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t v) {
    h ^= v;
    h *= 1099511628211ull;
  };
  mix((uint64_t)B);
  for (int b = 0; b < B; ++b) {
    mix((uint64_t)pr[b].L);
    mix((uint64_t)pr[b].N);
  }
  return h;
}

int validate_batch(int B, const psca_problem *pr) {
  if (B < 0 || (B > 0 && !pr)) return PSCA_EINVAL;
  for (int b = 0; b < B; ++b) {
    const psca_problem &q = pr[b];
    if (!q.Sigma_hat || !q.S || !q.x_out) return PSCA_EINVAL;
    const int rc = validate_params(&q.prm, q.L, q.N, true);
    if (rc != PSCA_OK) return rc;
  }
  // one launch runs one kernel: L x L in LDS (L <= 96) or in memory (97..256)
  if (batch_class(B, pr) < 0) return PSCA_ENOTSUP;
  return PSCA_OK;
}

// ---- batched layer backward ----------------------------------------------
// Largest column tile (multiple of 16) whose backward LDS fits a workgroup.
int max_back_tile(int Lp) {
  for (int ncb = kMaxNcb; ncb >= 1; --ncb)
    if (lds_back_bytes(Lp, 16 * ncb, 8) <= kMaxLds) return 16 * ncb;
  return 0;
}

struct BackBatchPlan {
  int B = 0, T = 0, n_teams = 0;
  size_t lds = 0;
  std::vector<InstPlan> ip;
  std::vector<int> team_of, lists, offsets;
  std::vector<size_t> ws_off;
  size_t part_off = 0, part_stride = 0, E_max = 0, ws_bytes = 0;
};

// Workspace of one instance: Sigma, G_a, G_b, barrier words, release,
// abort, status, the per-workgroup parts of dL/drho.
size_t back_inst_ws(int Lp, int G) {
  return 3 * align_up(packed_entries(Lp) * sizeof(float2)) + align_up((size_t)G * 16 * sizeof(unsigned)) +
         3 * align_up(sizeof(unsigned)) + align_up((size_t)G * sizeof(float));
}

int make_back_plan(int B, const psca_back_problem *pr, int cap, BackBatchPlan &plan) {
  int T0 = 1, want = 1;
  for (int b = 0; b < B; ++b) {
    const int nt = max_back_tile((pr[b].L + 15) & ~15);
    if (nt == 0) return PSCA_ENOTSUP;
    T0 = std::max(T0, (pr[b].N + nt - 1) / nt);
    want = std::max(want, (pr[b].N + 15) / 16);
  }
  if (T0 > cap) return PSCA_ENOTSUP;
  const int T = ((long long)B * T0 <= cap) ? std::max(T0, std::min(cap / B, want)) : T0;
  plan = BackBatchPlan();
  plan.B = B;
  plan.T = T;
  plan.n_teams = std::max(1, std::min(cap / T, B));
  plan.ip.resize(B);
  std::vector<double> cost(B);
  for (int b = 0; b < B; ++b) {
    InstPlan &q = plan.ip[b];
    q.Lp = (pr[b].L + 15) & ~15;
    const int per = (pr[b].N + T - 1) / T;
    q.NT = std::max(16, (per + 15) & ~15);
    if (q.NT > max_back_tile(q.Lp)) return PSCA_ENOTSUP;
    q.ncb = q.NT / 16;
    q.G = T;
    q.lds = lds_back_bytes(q.Lp, q.NT, 8);
    q.ws = back_inst_ws(q.Lp, q.G);
    plan.lds = std::max(plan.lds, q.lds);
    const double Lb = q.Lp / 16;
    cost[b] = 3.0 * Lb + 0.1 * q.ncb * Lb * Lb + 8.0;
    plan.E_max = std::max(plan.E_max, packed_entries(q.Lp));
  }
  std::vector<int> order(B);
  for (int b = 0; b < B; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  std::vector<double> load(plan.n_teams, 0.0);
  std::vector<std::vector<int>> team(plan.n_teams);
  plan.team_of.resize(B);
  for (int b : order) {
    const int t = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    team[t].push_back(b);
    plan.team_of[b] = t;
    load[t] += cost[b];
  }
  plan.offsets.push_back(0);
  for (int t = 0; t < plan.n_teams; ++t) {
    for (int b : team[t]) plan.lists.push_back(b);
    plan.offsets.push_back((int)plan.lists.size());
  }
  size_t off = 0;
  plan.ws_off.resize(B);
  for (int b = 0; b < B; ++b) {
    plan.ws_off[b] = off;
    off += plan.ip[b].ws;
  }
  plan.part_off = off;
  // per team: partials of Sigma / G_a, then of G_b, T ranks of E_max entries each
  plan.part_stride = 2 * align_up((size_t)T * plan.E_max * sizeof(float2));
  plan.ws_bytes = off + plan.part_stride * plan.n_teams;
  return PSCA_OK;
}

size_t back_image_bytes(const BackBatchPlan &plan) {
  return align_up(plan.B * sizeof(BackArgs)) + align_up(plan.lists.size() * sizeof(int)) +
         align_up(plan.offsets.size() * sizeof(int));
}

void write_back_image(const BackBatchPlan &plan, const psca_back_problem *pr, float rho, char *base, char *img) {
  BackArgs *out = (BackArgs *)img;
  for (int b = 0; b < plan.B; ++b) {
    const psca_back_problem &q = pr[b];
    const InstPlan &ip = plan.ip[b];
    BackArgs d;
    fill_args(d.c, (const float2 *)q.Sigma_hat, (const float2 *)q.S, q.L, q.N, &q.prm, 1, rho, q.x_in, nullptr,
              nullptr, nullptr, nullptr, q.status, ip);
    char *w = base + plan.ws_off[b];
    const size_t pe = align_up(packed_entries(ip.Lp) * sizeof(float2));
    d.c.sigma = (float2 *)w;        w += pe;
    d.gram_a = (float2 *)w;         w += pe;
    d.gram_b = (float2 *)w;         w += pe;
    d.c.bar.arrive = (unsigned *)w; w += align_up((size_t)ip.G * 16 * sizeof(unsigned));
    d.c.bar.release = (unsigned *)w; w += align_up(sizeof(unsigned));
    d.c.bar.abort_flag = (int32_t *)w; w += align_up(sizeof(unsigned));
    if (!d.c.status) d.c.status = (int32_t *)w;
    w += align_up(sizeof(unsigned));
    d.rho_part = (float *)w;
    char *pt = base + plan.part_off + (size_t)plan.team_of[b] * plan.part_stride;
    d.c.partials = (float2 *)pt;
    d.partials_b = (float2 *)(pt + plan.part_stride / 2);
    d.c.pstride = plan.E_max;
    d.grad_rho = q.grad_rho;
    d.rho = rho;
    d.v = q.v;
    d.grad_x = q.grad_x;
    out[b] = d;
  }
  char *p = img + align_up(plan.B * sizeof(BackArgs));
  memcpy(p, plan.lists.data(), plan.lists.size() * sizeof(int));
  p += align_up(plan.lists.size() * sizeof(int));
  memcpy(p, plan.offsets.data(), plan.offsets.size() * sizeof(int));
}

int launch_back_batch(const BackBatchPlan &plan, const char *dimg, hipStream_t st) {
  const BackArgs *descs = (const BackArgs *)dimg;
  const int *lists = (const int *)(dimg + align_up(plan.B * sizeof(BackArgs)));
  const int *offsets = (const int *)((const char *)lists + align_up(plan.lists.size() * sizeof(int)));
  int T = plan.T;
  hipLaunchKernelGGL(k_prepare_back_batch, dim3(plan.B), dim3(256), 0, st, descs);
  int rc = launch_ok();
  if (rc != PSCA_OK) return rc;
  void *args[] = {(void *)&descs, (void *)&lists, (void *)&offsets, (void *)&T};
  if (hipLaunchCooperativeKernel((const void *)k_psca_back_teams, dim3(plan.n_teams * plan.T), dim3(512), args,
                                 (unsigned)plan.lds, st) != hipSuccess) {
    (void)hipGetLastError();
    return PSCA_EHIP;
  }
  hipLaunchKernelGGL(k_sum_parts_batch, dim3(plan.B), dim3(256), 0, st, descs);
  return launch_ok();
}

}  // namespace

struct psca_plan {
  int device;
  BatchPlan plan;
  void *ws;     // the plan's own workspace
  void *dimg;   // descriptors, team lists and offsets on the device
};

extern "C" {

int psca_version(void) { return 200; }

const char *psca_strerror(int code) {
  switch (code) {
    case PSCA_OK: return "ok";
    case PSCA_EINVAL: return "invalid argument";
    case PSCA_ENOTPD: return "covariance matrix not positive definite (Cholesky pivot <= 0 or not finite)";
    case PSCA_EHIP: return "HIP runtime error";
    case PSCA_ENOMEM: return "device memory allocation failed";
    case PSCA_ENOTSUP: return "size or configuration not supported by the library";
    case PSCA_ESYNC: return "device-wide barrier timed out (workgroups not co-resident)";
    default: return "unknown error";
  }
}

int psca_create(psca_ctx **ctx, int device) {
  if (!ctx) return PSCA_EINVAL;
  *ctx = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess) return PSCA_EHIP;
  if (device < 0 || device >= count) return PSCA_EINVAL;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return PSCA_EHIP;
  psca_ctx *c = new (std::nothrow) psca_ctx;
  if (!c) return PSCA_ENOMEM;
  c->device = device;
  c->n_cu = prop.multiProcessorCount;
  c->ws = nullptr;
  c->ws_bytes = 0;
  c->sh = nullptr;
  c->sh_bytes = 0;
  c->occ_fn = nullptr;
  c->occ_lds = (size_t)-1;
  c->occ_per_cu = 0;
  c->hdesc = c->ddesc = nullptr;
  c->desc_bytes = 0;
  c->desc_pending = false;
  {
    DeviceGuard g(device);
    if (!g.ok || hipEventCreateWithFlags(&c->desc_done, hipEventDisableTiming) != hipSuccess) {
      delete c;
      return PSCA_EHIP;
    }
    if (device < kMaxDevices) {   // the no-allocation scratch of this device, once
      std::lock_guard<std::mutex> lock(g_scratch_mu);
      if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
          (void)hipGetLastError();
          (void)hipEventDestroy(c->desc_done);
          delete c;
          return PSCA_EHIP;
        }
        g_scratch_ptr[device] = ptr;
      }
    }
  }
  *ctx = c;
  return PSCA_OK;
}

int psca_destroy(psca_ctx *ctx) {
  if (!ctx) return PSCA_OK;
  int rc = PSCA_OK;
  {
    DeviceGuard g(ctx->device);
    if (hipDeviceSynchronize() != hipSuccess) rc = PSCA_EHIP;
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->sh) (void)hipFree(ctx->sh);
    if (ctx->ddesc) (void)hipFree(ctx->ddesc);
    if (ctx->hdesc) (void)hipHostFree(ctx->hdesc);
    (void)hipEventDestroy(ctx->desc_done);
  }
  delete ctx;
  return rc;
}

int psca_sample_cov(psca_ctx *ctx, const psca_c32 *Y, int L, int M, psca_c32 *Sigma_hat, void *stream) {
  if (!ctx || !Y || !Sigma_hat || L < 1 || M < 1) return PSCA_EINVAL;
  if (L > kMaxL) return PSCA_ENOTSUP;
  DeviceGuard g(ctx->device);
  if (!g.ok) return PSCA_EHIP;
  hipLaunchKernelGGL(k_sample_cov, dim3(packed_blocks(L)), dim3(256), 0,
                     as_stream(stream), (const float2 *)Y, L, M, (float2 *)Sigma_hat, 0LL, 0LL);
  return launch_ok();
}

int psca_sample_cov_batch(psca_ctx *ctx, int B, const psca_c32 *Y, long long y_stride, int L, int M,
                          psca_c32 *Sigma_hat, long long sh_stride, void *stream) {
  if (!ctx || B < 0 || L < 1 || M < 1) return PSCA_EINVAL;
  if (B > 0 && (!Y || !Sigma_hat)) return PSCA_EINVAL;
  if (y_stride < (long long)L * M || sh_stride < (long long)L * L) return PSCA_EINVAL;
  if (L > kMaxL) return PSCA_ENOTSUP;
  if (B == 0) return PSCA_OK;
  DeviceGuard g(ctx->device);
  if (!g.ok) return PSCA_EHIP;
  constexpr int kMaxGridY = 65535;
  for (int b0 = 0; b0 < B; b0 += kMaxGridY) {
    const int nb = std::min(kMaxGridY, B - b0);
    hipLaunchKernelGGL(k_sample_cov, dim3(packed_blocks(L), nb), dim3(256), 0, as_stream(stream),
                       (const float2 *)Y + (size_t)b0 * (size_t)y_stride, L, M,
                       (float2 *)Sigma_hat + (size_t)b0 * (size_t)sh_stride, y_stride, sh_stride);
    const int rc = launch_ok();
    if (rc != PSCA_OK) return rc;
  }
  return PSCA_OK;
}

int psca_detect(psca_ctx *ctx, const psca_c32 *Sigma_hat, const psca_c32 *S, int L, int N,
                const psca_params *prm, float *x_out, int32_t *status, void *stream) {
  if (!ctx || !Sigma_hat || !S || !x_out) return PSCA_EINVAL;
  if (prm && prm->x0 && prm->x0 == x_out) return PSCA_EINVAL;
  int rc = validate_params(prm, L, N, true);
  if (rc != PSCA_OK) return rc;
  DeviceGuard g(ctx->device);
  if (!g.ok) return PSCA_EHIP;
  return run_detect(ctx, (const float2 *)Sigma_hat, (const float2 *)S, L, N, prm, prm->iters, -1.0f, prm->x0,
                    x_out, nullptr, nullptr, nullptr, status, as_stream(stream));
}

int psca_detect_noalloc(psca_ctx *ctx, const psca_c32 *Sigma_hat, const psca_c32 *S, int L, int N,
                        const psca_params *prm, float *x_out, int32_t *status, void *stream) {
  if (!ctx || !Sigma_hat || !S || !x_out) return PSCA_EINVAL;
  if (prm && prm->x0 && prm->x0 == x_out) return PSCA_EINVAL;
  int rc = validate_params(prm, L, N, true);
  if (rc != PSCA_OK) return rc;
  if (ctx->device >= kMaxDevices || !g_scratch_ptr[ctx->device]) return PSCA_EHIP;
  DeviceGuard g(ctx->device);
  if (!g.ok) return PSCA_EHIP;
  return run_detect(ctx, (const float2 *)Sigma_hat, (const float2 *)S, L, N, prm, prm->iters, -1.0f, prm->x0,
                    x_out, nullptr, nullptr, nullptr, status, as_stream(stream), nullptr,
                    (char *)g_scratch_ptr[ctx->device], kScratchBytes);
}

int psca_detect_y(psca_ctx *ctx, const psca_c32 *Y, const psca_c32 *S, int L, int N,
                  const psca_params *prm, float *x_out, int32_t *status, void *stream) {
  if (!ctx || !Y || !S || !x_out) return PSCA_EINVAL;
  if (prm && prm->x0 && prm->x0 == x_out) return PSCA_EINVAL;
  int rc = validate_params(prm, L, N, true);
  if (rc != PSCA_OK) return rc;
  DeviceGuard g(ctx->device);
  if (!g.ok) return PSCA_EHIP;
  static_assert(sizeof(float2) == sizeof(psca_c32), "layout");
  rc = ensure_buf(&ctx->sh, &ctx->sh_bytes, (size_t)L * L * sizeof(float2));
  if (rc != PSCA_OK) return rc;
  float2 *Sh = (float2 *)ctx->sh;
  hipLaunchKernelGGL(k_sample_cov, dim3(packed_blocks(L)), dim3(256), 0,
                     as_stream(stream), (const float2 *)Y, L, prm->M, Sh, 0LL, 0LL);
  if ((rc = launch_ok()) != PSCA_OK) return rc;
  return run_detect(ctx, Sh, (const float2 *)S, L, N, prm, prm->iters, -1.0f, prm->x0, x_out, nullptr, nullptr,
                    nullptr, status, as_stream(stream));
}

int psca_iterate(psca_ctx *ctx, const psca_c32 *Sigma_hat, const psca_c32 *S, int L, int N,
                 const psca_params *prm, float rho, const float *x_in, float *x_out, float *q_out,
                 float *r_out, float *xt_out, int32_t *status, void *stream) {
  if (!ctx || !Sigma_hat || !S || !x_in || !x_out || x_in == x_out) return PSCA_EINVAL;
  if (!(rho >= 0.0f) || rho > 1.0f) return PSCA_EINVAL;
  int rc = validate_params(prm, L, N, false);
  if (rc != PSCA_OK) return rc;
  DeviceGuard g(ctx->device);
  if (!g.ok) return PSCA_EHIP;
  return run_detect(ctx, (const float2 *)Sigma_hat, (const float2 *)S, L, N, prm, 1, rho, x_in, x_out, q_out,
                    r_out, xt_out, status, as_stream(stream));
}

int psca_detect_batch(psca_ctx *ctx, int B, const psca_problem *problems, void *stream) {
  if (!ctx) return PSCA_EINVAL;
  int rc = validate_batch(B, problems);
  if (rc != PSCA_OK || B == 0) return rc;
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return PSCA_EHIP;
  hipStream_t st = as_stream(stream);
  const bool large = batch_class(B, problems) == 1;
  const int cap = large ? large_capacity(ctx) : batch_capacity(ctx);
  if (cap <= 0) return PSCA_ENOTSUP;
  const auto hit = ctx->tuned.find(batch_signature(B, problems));
  const int T = (hit != ctx->tuned.end()) ? hit->second
                                          : (large ? default_large_team(B, cap) : default_team(B, problems, cap));
  if (hit == ctx->tuned.end() && T < 0) return PSCA_ENOTSUP;
  BatchPlan plan;
  if ((rc = make_plan(B, problems, T, cap, plan, -1)) != PSCA_OK) return rc;
  if ((rc = ensure_ws(ctx, plan.ws_bytes)) != PSCA_OK) return rc;
  const size_t bytes = batch_image_bytes(plan);
  char *host = nullptr;
  if ((rc = stage_desc(ctx, bytes, &host)) != PSCA_OK) return rc;
  write_batch_image(plan, (char *)ctx->ws, host);
  if (hipMemcpyAsync(ctx->ddesc, host, bytes, hipMemcpyHostToDevice, st) != hipSuccess) {
    (void)hipGetLastError();
    return PSCA_EHIP;
  }
  if (hipEventRecord(ctx->desc_done, st) != hipSuccess) return PSCA_EHIP;
  ctx->desc_pending = true;
  return launch_batch(plan, (const char *)ctx->ddesc, st);
}

int psca_autotune_batch(psca_ctx *ctx, int B, const psca_problem *problems, int tune_iters, int *team_size,
                        void *stream) {
  if (!ctx || tune_iters < 1) return PSCA_EINVAL;
  int rc = validate_batch(B, problems);
  if (rc != PSCA_OK) return rc;
  if (B == 0) return PSCA_EINVAL;
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return PSCA_EHIP;
  hipStream_t st = as_stream(stream);
  const bool large = batch_class(B, problems) == 1;
  const int cap = large ? large_capacity(ctx) : batch_capacity(ctx);
  const int T0 = large ? 1 : min_team(B, problems);
  if (cap <= 0 || T0 < 0 || T0 > cap) return PSCA_ENOTSUP;
  std::vector<int> cand;
  if (large) {   // uniform teams
    cand.push_back(default_large_team(B, cap));
    for (int t : {1, 2, 4, 8, 16, 32, 64, 128, 256})
      if (t <= cap) cand.push_back(t);
  } else {
    cand = {T0, default_team(B, problems, cap)};
    for (int c = 32; c <= 16 * kMaxNcb; c += 16) cand.push_back(-c);   // mixed teams
    for (int t : {8, 16, 24, 32, 48, 64, 96, 128, 192, 256})
      if (t >= T0 && t <= cap) cand.push_back(t);
    if ((long long)B * T0 <= cap) cand.push_back(cap / B);
  }
  std::sort(cand.begin(), cand.end());
  cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return PSCA_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return PSCA_EHIP;
  }
  // Each candidate is timed at k1 = tune_iters and k2 = 2 tune_iters capped
  // iterations; the launch at the batch's own iteration count is estimated
  // from the two points (per-instance set-up and the tail of the team
  // lists weigh more at few iterations than at many).
  int K = 1;
  for (int b = 0; b < B; ++b) K = std::max(K, (int)problems[b].prm.iters);
  auto time_plan = [&](int T, int k, bool warm, float *ms) -> int {
    BatchPlan plan;
    int r = make_plan(B, problems, T, cap, plan, k);
    if (r != PSCA_OK) return r;
    if ((r = ensure_ws(ctx, plan.ws_bytes)) != PSCA_OK) return r;
    const size_t bytes = batch_image_bytes(plan);
    char *host = nullptr;
    if ((r = stage_desc(ctx, bytes, &host)) != PSCA_OK) return r;
    write_batch_image(plan, (char *)ctx->ws, host);
    if (hipMemcpyAsync(ctx->ddesc, host, bytes, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipEventRecord(ctx->desc_done, st) != hipSuccess)
      return PSCA_EHIP;
    ctx->desc_pending = true;
    if (warm && (r = launch_batch(plan, (const char *)ctx->ddesc, st)) != PSCA_OK) return r;
    if (hipEventRecord(e0, st) != hipSuccess) return PSCA_EHIP;
    if ((r = launch_batch(plan, (const char *)ctx->ddesc, st)) != PSCA_OK) return r;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(ms, e0, e1) != hipSuccess)
      return PSCA_EHIP;
    return PSCA_OK;
  };
  bool found = false;   // team specifications may be negative (mixed teams)
  int best = 0;
  float best_ms = 0.0f;
  std::vector<int> seen;
  for (int T : cand) {
    if (T > 0 && T < T0) continue;
    BatchPlan probe;
    if (make_plan(B, problems, T, cap, probe, tune_iters) != PSCA_OK) continue;   // infeasible
    T = probe.T;   // a single-class mixed plan is a uniform one
    if (std::find(seen.begin(), seen.end(), T) != seen.end()) continue;
    seen.push_back(T);
    const int k1 = tune_iters, k2 = 2 * tune_iters;
    float t1 = 0.0f, t2 = 0.0f;
    if ((rc = time_plan(T, k1, true, &t1)) != PSCA_OK || (rc = time_plan(T, k2, false, &t2)) != PSCA_OK) break;
    const float est = K <= k1 ? t1 : t1 + (t2 - t1) * (float)(K - k1) / (float)(k2 - k1);
    if (!found || est < best_ms) {
      found = true;
      best = T;
      best_ms = est;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != PSCA_OK) return rc;
  if (!found) return PSCA_ENOTSUP;
  ctx->tuned[batch_signature(B, problems)] = best;
  if (team_size) *team_size = best;
  return PSCA_OK;
}

int psca_plan_create(psca_ctx *ctx, int B, const psca_problem *problems, int team_size, psca_plan **out) {
  if (!ctx || !out) return PSCA_EINVAL;
  *out = nullptr;
  int rc = validate_batch(B, problems);
  if (rc != PSCA_OK) return rc;
  if (B == 0) return PSCA_EINVAL;
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return PSCA_EHIP;
  const bool large = batch_class(B, problems) == 1;
  const int cap = large ? large_capacity(ctx) : batch_capacity(ctx);
  if (cap <= 0) return PSCA_ENOTSUP;
  int T = team_size;
  if (T == 0) {
    const auto hit = ctx->tuned.find(batch_signature(B, problems));
    T = (hit != ctx->tuned.end()) ? hit->second : (large ? default_large_team(B, cap) : default_team(B, problems, cap));
    if (T == -1) return PSCA_ENOTSUP;   // no feasible default
  }
  if (large ? (T < 1 || T > cap) : (!team_spec_ok(T, cap) || (T > 0 && T < min_team(B, problems))))
    return PSCA_EINVAL;
  psca_plan *p = new (std::nothrow) psca_plan;
  if (!p) return PSCA_ENOMEM;
  p->device = ctx->device;
  p->ws = p->dimg = nullptr;
  if ((rc = make_plan(B, problems, T, cap, p->plan, -1)) != PSCA_OK) {
    delete p;
    return rc;
  }
  const size_t bytes = batch_image_bytes(p->plan);
  std::vector<char> img(bytes);
  if (hipMalloc(&p->ws, p->plan.ws_bytes) != hipSuccess || hipMalloc(&p->dimg, bytes) != hipSuccess) {
    (void)hipGetLastError();
    if (p->ws) (void)hipFree(p->ws);
    delete p;
    return PSCA_ENOMEM;
  }
  write_batch_image(p->plan, (char *)p->ws, img.data());
  if (hipMemcpy(p->dimg, img.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(p->ws);
    (void)hipFree(p->dimg);
    delete p;
    return PSCA_EHIP;
  }
  *out = p;
  return PSCA_OK;
}

int psca_plan_launch(psca_plan *plan, void *stream) {
  if (!plan) return PSCA_EINVAL;
  DeviceGuard guard(plan->device);
  if (!guard.ok) return PSCA_EHIP;
  return launch_batch(plan->plan, (const char *)plan->dimg, as_stream(stream));
}

int psca_plan_team_size(const psca_plan *plan) { return plan ? plan->plan.T : PSCA_EINVAL; }

int psca_plan_destroy(psca_plan *plan) {
  if (!plan) return PSCA_OK;
  DeviceGuard guard(plan->device);
  int rc = (hipDeviceSynchronize() == hipSuccess) ? PSCA_OK : PSCA_EHIP;
  (void)hipFree(plan->ws);
  (void)hipFree(plan->dimg);
  delete plan;
  return rc;
}

int psca_net_forward(psca_ctx *ctx, const psca_c32 *Sigma_hat, const psca_c32 *S, int L, int N,
                     const psca_params *prm, float *x_hist, int32_t *status, void *stream) {
  if (!ctx || !Sigma_hat || !S || !x_hist) return PSCA_EINVAL;
  int rc = validate_params(prm, L, N, true);
  if (rc != PSCA_OK) return rc;
  DeviceGuard g(ctx->device);
  if (!g.ok) return PSCA_EHIP;
  return run_detect(ctx, (const float2 *)Sigma_hat, (const float2 *)S, L, N, prm, prm->iters, -1.0f, prm->x0,
                    x_hist + (size_t)prm->iters * N, nullptr, nullptr, nullptr, status, as_stream(stream), x_hist);
}

int psca_layer_backward(psca_ctx *ctx, const psca_c32 *Sigma_hat, const psca_c32 *S, int L, int N,
                        const psca_params *prm, float rho, const float *x_in, const float *v, float *grad_x,
                        float *grad_rho, int32_t *status, void *stream) {
  if (!ctx || !Sigma_hat || !S || !x_in || !v || !grad_x || !grad_rho) return PSCA_EINVAL;
  if (!(rho >= 0.0f) || rho > 1.0f) return PSCA_EINVAL;
  int rc = validate_params(prm, L, N, false);
  if (rc != PSCA_OK) return rc;
  if (prm->variant == PSCA_MAP_K2) return PSCA_ENOTSUP;
  DeviceGuard g(ctx->device);
  if (!g.ok) return PSCA_EHIP;
  if (L > 64) {   // Sigma and the Gram matrices in memory, on one team
    psca_back_problem q;
    q.Sigma_hat = Sigma_hat;
    q.S = S;
    q.L = L;
    q.N = N;
    q.prm = *prm;
    q.x_in = x_in;
    q.v = v;
    q.grad_x = grad_x;
    q.grad_rho = grad_rho;
    q.status = status;
    return run_large_backward(ctx, 1, &q, rho, as_stream(stream));
  }
  return run_layer_backward(ctx, (const float2 *)Sigma_hat, (const float2 *)S, L, N, prm, rho, x_in, v, grad_x,
                            grad_rho, status, as_stream(stream));
}

#ifdef PSCA_PHASE_TRACE
// Profiling builds only: copy the phase stamps (kTraceIters x kTraceMarks) to host.
int psca_sub_trace(unsigned long long *host) {
  return hipMemcpyFromSymbol(host, HIP_SYMBOL(g_sub_trace), sizeof(unsigned long long) * 512) == hipSuccess
             ? PSCA_OK : PSCA_EHIP;
}
int psca_step_trace(unsigned long long *host) {
  return hipMemcpyFromSymbol(host, HIP_SYMBOL(g_step_trace), sizeof(unsigned long long) * 128) == hipSuccess
             ? PSCA_OK : PSCA_EHIP;
}
// Profiling builds only: copy bytes of the context's workspace at offset to host.
int psca_debug_ws(psca_ctx *ctx, size_t offset, size_t bytes, void *host) {
  if (!ctx || !host || offset + bytes > ctx->ws_bytes) return PSCA_EINVAL;
  return hipMemcpy(host, (char *)ctx->ws + offset, bytes, hipMemcpyDeviceToHost) == hipSuccess ? PSCA_OK : PSCA_EHIP;
}
int psca_phase_trace(unsigned long long *host, int count) {
  if (!host || count < kTraceIters * kTraceMarks) return PSCA_EINVAL;
  return hipMemcpyFromSymbol(host, HIP_SYMBOL(g_phase_trace), sizeof(unsigned long long) * kTraceIters * kTraceMarks) ==
                 hipSuccess ? PSCA_OK : PSCA_EHIP;
}
#endif

int psca_layer_backward_batch(psca_ctx *ctx, int B, const psca_back_problem *problems, float rho, void *stream) {
  if (!ctx || B < 0 || (B > 0 && !problems)) return PSCA_EINVAL;
  if (!(rho >= 0.0f) || rho > 1.0f) return PSCA_EINVAL;
  for (int b = 0; b < B; ++b) {
    const psca_back_problem &q = problems[b];
    if (!q.Sigma_hat || !q.S || !q.x_in || !q.v || !q.grad_x || !q.grad_rho) return PSCA_EINVAL;
    const int rc = validate_params(&q.prm, q.L, q.N, false);
    if (rc != PSCA_OK) return rc;
    if (q.prm.variant == PSCA_MAP_K2) return PSCA_ENOTSUP;
    if ((q.L > 64) != (problems[0].L > 64)) return PSCA_ENOTSUP;   // one launch runs one of the two kernels
  }
  if (B == 0) return PSCA_OK;
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return PSCA_EHIP;
  hipStream_t st = as_stream(stream);
  if (problems[0].L > 64) return run_large_backward(ctx, B, problems, rho, st);
  const KernelChoice kc{(const void *)k_psca_back_teams, 512, 64};
  const int cap = max_coresident(ctx, kc, kMaxLds);
  if (cap <= 0) return PSCA_ENOTSUP;
  BackBatchPlan plan;
  int rc = make_back_plan(B, problems, cap, plan);
  if (rc != PSCA_OK) return rc;
  if (max_coresident(ctx, kc, plan.lds) < plan.n_teams * plan.T) return PSCA_ENOTSUP;
  if ((rc = ensure_ws(ctx, plan.ws_bytes)) != PSCA_OK) return rc;
  const size_t bytes = back_image_bytes(plan);
  char *host = nullptr;
  if ((rc = stage_desc(ctx, bytes, &host)) != PSCA_OK) return rc;
  write_back_image(plan, problems, rho, (char *)ctx->ws, host);
  if (hipMemcpyAsync(ctx->ddesc, host, bytes, hipMemcpyHostToDevice, st) != hipSuccess) {
    (void)hipGetLastError();
    return PSCA_EHIP;
  }
  if (hipEventRecord(ctx->desc_done, st) != hipSuccess) return PSCA_EHIP;
  ctx->desc_pending = true;
  return launch_back_batch(plan, (const char *)ctx->ddesc, st);
}

int psca_threshold(const float *x, int N, float theta, uint8_t *support, void *stream) {
  if (!x || !support || N < 1) return PSCA_EINVAL;
  hipLaunchKernelGGL(k_threshold, dim3((N + 255) / 256), dim3(256), 0, as_stream(stream), x, N, theta, support);
  return launch_ok();
}

}  // extern "C"
#endif   // PSCA_TU_MAIN
