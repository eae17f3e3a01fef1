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
// Execution model.  One detection is ONE cooperative persistent kernel
// (k_psca) with G workgroups of 256 threads (512 for L > 64).  Workgroup g owns
// NT = 16 * ncb consecutive columns of S; that tile, the tile's iterate and
// its pathloss stay in LDS for the whole solve, and the Sigma^-1-independent
// operand SigmaHat stays in registers.  Per iteration:
//   A. tile partial  P_g = S_g diag(w_g) S_g^H   (FP32 MFMA, lower 16x16 blocks) -> HBM
//      grid barrier
//   B. workgroup g sums a contiguous slice of the G partials (fixed order) -> Sigma
//      grid barrier
//   C. every workgroup factors Sigma redundantly in LDS/registers (identical
//      inputs and code, so all reach identical results and decisions), forms
//      Sigma^-1 = W^H W on MFMA, then B = Sigma^-1 S_g, D = SigmaHat B (MFMA),
//      the quadratic forms, the coordinate step and the update of its columns.
// Two grid barriers per iteration; no atomics on data, so a run is bitwise
// reproducible for a given launch shape.
//
// Complex GEMMs use v_mfma_f32_16x16x4f32 on the real 4-product split:
//   Re C += Re A Re B - Im A Im B,   Im C += Re A Im B + Im A Re B.
// Operand layout of that instruction (wave64): lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; it receives C[4*(l/16)+v][l%16] in accumulator v.

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <new>

#include "psca.h"

namespace {

constexpr int kThreads = 256;                              // helper kernels
constexpr int kBlk = 16;
constexpr int kMaxL = PSCA_MAX_L;                          // 96
constexpr int kMaxNcb = 4;                                 // column blocks per workgroup
constexpr unsigned kSpinLimit = 1u << 20;                  // grid-barrier wait bound

// Register-array sizes of k_psca for a padded pilot length of at most LPMAX
// with THREADS threads per workgroup.
template <int LPMAX, int THREADS>
struct Shape {
  static constexpr int kWaves = THREADS / 64;
  static constexpr int kMaxLb = LPMAX / kBlk;
  static constexpr int kMaxNB = kMaxLb * (kMaxLb + 1) / 2;
  static constexpr int kMaxTri = LPMAX * (LPMAX + 1) / 2;
  static constexpr int kSlots = (kMaxTri + THREADS - 1) / THREADS;     // entries per thread
  static constexpr int kRowBlocksPerWave = (kMaxLb + kWaves - 1) / kWaves;
  static constexpr int kBlocksPerWave = (kMaxNB + kWaves - 1) / kWaves;
  static constexpr int kKSteps = LPMAX / 4;
};

typedef float f4 __attribute__((ext_vector_type(4)));

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

__device__ __forceinline__ float2 cmul_conj(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// packed lower-block index of block (I, J), I >= J, and its inverse
__device__ __forceinline__ int blk_index(int I, int J) { return I * (I + 1) / 2 + J; }
__device__ __forceinline__ void blk_coords(int b, int &I, int &J) {
  int r = 0;
  while ((r + 1) * (r + 2) / 2 <= b) ++r;
  I = r;
  J = b - r * (r + 1) / 2;
}
// offset of element (i, j), i >= j, in the block-packed lower triangle
// (blocks column-major inside: element (ii, jj) at jj * 16 + ii)
__device__ __forceinline__ int bp_offset(int i, int j) {
  return blk_index(i >> 4, j >> 4) * 256 + (j & 15) * 16 + (i & 15);
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
};

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

// g: known pathloss of the device (K variants); logit = log(p / (1 - p)) (MAP-K).
__device__ __forceinline__ float coordinate_step(float x, float q, float r, float g, float logit,
                                                 const StepArgs &a) {
  float grad, curv, hi;
  switch (a.variant) {
    case PSCA_ML_K: {
      grad = g * (q - r);
      const float gq = g * q;
      curv = gq * gq;
      hi = 1.0f;
      break;
    }
    case PSCA_MAP_K: {
      grad = g * (q - r) - logit * a.inv_M;
      const float gq = g * q;
      curv = gq * gq;
      hi = 1.0f;
      break;
    }
    case PSCA_ML_UD:
      grad = q - r;
      curv = q * q;
      hi = INFINITY;
      break;
    default:  // PSCA_MAP_UR
      grad = q - r - prior_log_ratio(x, a) * a.inv_M;
      curv = q * q;
      hi = a.g_u;
      break;
  }
  return fminf(fmaxf(x - grad / curv, 0.0f), hi);
}

// ---------------------------------------------------------------------------
// Grid barrier (agent scope).  bar[0] counts arrivals, bar[1] is the
// generation.  A waiter gives up after kSpinLimit polls and raises *abort,
// which every workgroup checks, so a missing workgroup cannot hang the grid.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool grid_sync(unsigned *bar, unsigned G, unsigned &gen, int32_t *abort_flag,
                                          int *s_ok) {
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    const unsigned target = gen + 1;
    const unsigned old = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (old == G - 1) {
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&bar[1], target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned spins = 0;
      while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != target) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit) { ok = 0; break; }
        if ((spins & 1023u) == 0 &&
            __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { ok = 0; break; }
      }
    }
    __atomic_thread_fence(__ATOMIC_ACQUIRE);
    gen = target;
    if (!ok) __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
  int L, N, Lp, Lb, NB; // Lp = L rounded up to 16, Lb = Lp / 16, NB = Lb (Lb + 1) / 2
  int G, ncb, NT;       // workgroups, 16-column blocks per workgroup, columns per workgroup
  int iters;
  double rho0, rho_decay;
  const float *rho_dev; // [iters] or null
  float rho_fixed;      // >= 0: every iteration uses this step (single-iteration entry point)
  float sigma2;
  StepArgs a;
  const float *x_in;    // [N] initial iterate or null (zeros)
  float *x_out, *q_out, *r_out, *xt_out;
  int32_t *status;
  float2 *partials;     // [G][NB * 256]
  float2 *sigma;        // [NB * 256]
  unsigned *bar;        // [2]
  int32_t *abort_flag;
};

// LDS footprint in bytes for a launch shape
__host__ __device__ inline size_t lds_bytes(int Lp, int NT, int Lb) {
  const size_t pt = (size_t)NT + 1;
  size_t f2 = 2 * (size_t)Lp * pt + (size_t)Lp * Lp + 5 * (size_t)Lp;
  size_t fl = 3 * (size_t)NT + 2 * (size_t)Lb * NT;
  return f2 * sizeof(float2) + fl * sizeof(float);
}

template <int LPMAX, int THREADS>
__global__ void __launch_bounds__(THREADS) k_psca(CoopArgs A) {
  using Sh = Shape<LPMAX, THREADS>;
  constexpr int kWaves = Sh::kWaves;
  constexpr int kMaxSlots = Sh::kSlots;
  constexpr int kMaxRowBlocksPerWave = Sh::kRowBlocksPerWave;
  constexpr int kMaxBlocksPerWave = Sh::kBlocksPerWave;
  constexpr int kMaxKSteps = Sh::kKSteps;
  extern __shared__ float4 smem_raw[];
  __shared__ int s_ok;
  const int Lp = A.Lp, Lb = A.Lb, NB = A.NB, NT = A.NT, PT = A.NT + 1;
  float2 *St = (float2 *)smem_raw;          // [Lp][PT]  S tile, row i at i * PT
  float2 *Bt = St + Lp * PT;                // [Lp][PT]  B tile (also reduction scratch)
  float2 *WS = Bt + Lp * PT;                // [Lp][Lp]  W (row-major) then Sigma^-1 (column-major)
  float2 *colbuf = WS + Lp * Lp;            // [3][Lp]   published pivot columns
  float2 *wbuf = colbuf + 3 * Lp;           // [2][Lp]   published rows of W
  float *xs = (float *)(wbuf + 2 * Lp);     // [NT] iterate of the tile
  float *gs = xs + NT;                      // [NT] pathloss
  float *ls = gs + NT;                      // [NT] log(p / (1 - p))
  float *red_q = ls + NT;                   // [Lb][NT]
  float *red_r = red_q + Lb * NT;           // [Lb][NT]

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, lq = lane >> 4;
  const int g = blockIdx.x;
  const int n0 = g * NT;
  const int E = NB * 256;
  unsigned gen = 0;
  const bool known = (A.a.variant == PSCA_ML_K || A.a.variant == PSCA_MAP_K);

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
    gs[c] = (in && A.a.g) ? A.a.g[n] : 0.0f;
    float lg = 0.0f;
    if (in && A.a.p) {
      const float pn = A.a.p[n];
      lg = logf(pn / (1.0f - pn));
    }
    ls[c] = lg;
  }
  // ---- ownership of lower-triangle entries for the factorisation --------
  // Cholesky entries in column-packed order, W entries in row-packed order;
  // chunk c of 64 consecutive entries belongs to wave c % 4, slot c / 4.
  // Packed per slot: (bound << 16) | (i << 8) | j  with bound = last column
  // (Cholesky) or last row (W) of the chunk; i = 255 marks an empty slot.
  const int Tp = Lp * (Lp + 1) / 2;
  int ch_meta[kMaxSlots], w_meta[kMaxSlots];
#pragma unroll
  for (int s = 0; s < kMaxSlots; ++s) {
    const int chunk = kWaves * s + wave;
    const int e = chunk * 64 + lane;
    const int elast = min(chunk * 64 + 63, Tp - 1);
    int ci = 255, cj = 0, cbound = -1, wi = 255, wc = 0, wbound = -1;
    if (chunk * 64 < Tp) {
      // column-packed: column j holds rows j..Lp-1
      int j = 0, start = 0;
      while (j < Lp && start + (Lp - j) <= elast) { start += Lp - j; ++j; }
      cbound = j;  // column of the chunk's last entry
      if (e < Tp) {
        int jj = 0, st = 0;
        while (st + (Lp - jj) <= e) { st += Lp - jj; ++jj; }
        cj = jj;
        ci = jj + (e - st);
      }
      // row-packed: row i holds columns 0..i
      int r = 0;
      while ((r + 1) * (r + 2) / 2 <= elast) ++r;
      wbound = r;
      if (e < Tp) {
        int rr = 0;
        while ((rr + 1) * (rr + 2) / 2 <= e) ++rr;
        wi = rr;
        wc = e - rr * (rr + 1) / 2;
      }
    }
    ch_meta[s] = ((cbound & 0xff) << 16) | (ci << 8) | cj;
    w_meta[s] = ((wbound & 0xff) << 16) | (wi << 8) | wc;
    if (cbound < 0) ch_meta[s] = (0xff << 8);          // empty chunk: never active
    if (wbound < 0) w_meta[s] = (0xff << 8);
  }

  double rho_d = A.rho0;
  bool failed = false, aborted = false;
  int it = 0;
  for (; it < A.iters; ++it) {
    // ===== A. partial of Sigma from this tile =============================
    for (int c = tid; c < NT; c += THREADS)   // weights w_c
      red_q[c] = known ? gs[c] * xs[c] : xs[c];
    __syncthreads();
    {
      const float *wv = red_q;
      float2 *dst = A.partials + (size_t)g * E;
      for (int b = wave; b < NB; b += kWaves) {
        int I, J;
        blk_coords(b, I, J);
        f4 cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
        for (int c0 = 0; c0 < NT; c0 += 4) {
          const int c = c0 + lq;
          const float2 a = St[(16 * I + l16) * PT + c];
          const float2 s = St[(16 * J + l16) * PT + c];
          const float w = wv[c];
          cmfma(a, make_float2(w * s.x, -w * s.y), cr, ci);
        }
        float4 *o = (float4 *)(dst + b * 256 + l16 * 16 + 4 * lq);
        o[0] = make_float4(cr[0], ci[0], cr[1], ci[1]);
        o[1] = make_float4(cr[2], ci[2], cr[3], ci[3]);
      }
    }
    if (!grid_sync(A.bar, A.G, gen, A.abort_flag, &s_ok)) { aborted = true; break; }

    // ===== B. reduce a slice of the partials into Sigma ===================
    {
      const int per = (E + A.G - 1) / A.G;
      const int start = g * per, end = min(E, start + per);
      const int cnt = max(0, end - start);
      if (cnt > 0 && cnt <= THREADS) {
        const int P = THREADS / cnt;   // threads per element
        float2 acc = make_float2(0.f, 0.f);
        if (tid < cnt * P) {
          const int e = start + tid % cnt, part = tid / cnt;
          for (int h = part; h < A.G; h += P) {
            const float2 v = A.partials[(size_t)h * E + e];
            acc.x += v.x;
            acc.y += v.y;
          }
          Bt[tid] = acc;
        }
        __syncthreads();
        if (tid < cnt) {
          float2 s = make_float2(0.f, 0.f);
          for (int part = 0; part < P; ++part) {
            const float2 v = Bt[part * cnt + tid];
            s.x += v.x;
            s.y += v.y;
          }
          const int e = start + tid;
          const int b = e >> 8, jj = (e & 255) >> 4, ii = e & 15;
          int I, J;
          blk_coords(b, I, J);
          if (I == J && ii == jj) {
            const int i = 16 * I + ii;
            s.x += (i < A.L) ? A.sigma2 : 1.0f;   // padded rows: isolated unit pivots
            s.y = 0.0f;
          }
          A.sigma[e] = s;
        }
      } else {
        for (int e = start + tid; e < end; e += THREADS) {
          float2 s = make_float2(0.f, 0.f);
          for (int h = 0; h < A.G; ++h) {
            const float2 v = A.partials[(size_t)h * E + e];
            s.x += v.x;
            s.y += v.y;
          }
          const int b = e >> 8, jj = (e & 255) >> 4, ii = e & 15;
          int I, J;
          blk_coords(b, I, J);
          if (I == J && ii == jj) {
            const int i = 16 * I + ii;
            s.x += (i < A.L) ? A.sigma2 : 1.0f;
            s.y = 0.0f;
          }
          A.sigma[e] = s;
        }
      }
    }
    if (!grid_sync(A.bar, A.G, gen, A.abort_flag, &s_ok)) { aborted = true; break; }

    // ===== C1. Cholesky Sigma = L L^H fused with W = L^-1 ===================
    float2 av[kMaxSlots], wx[kMaxSlots];
#pragma unroll
    for (int s = 0; s < kMaxSlots; ++s) {
      const int i = (ch_meta[s] >> 8) & 0xff, j = ch_meta[s] & 0xff;
      av[s] = (i != 0xff) ? A.sigma[bp_offset(i, j)] : make_float2(0.f, 0.f);
      const int wi = (w_meta[s] >> 8) & 0xff, wc = w_meta[s] & 0xff;
      wx[s] = make_float2((wi != 0xff && wi == wc) ? 1.0f : 0.0f, 0.0f);
    }
    for (int e = tid; e < Lp * Lp; e += THREADS) WS[e] = make_float2(0.f, 0.f);
#pragma unroll
    for (int s = 0; s < kMaxSlots; ++s) {        // publish column 0
      const int i = (ch_meta[s] >> 8) & 0xff, j = ch_meta[s] & 0xff;
      if (i != 0xff && j == 0) colbuf[i] = av[s];
    }
    float rs_prev = 0.0f;
    for (int k = 0; k < Lp; ++k) {
      __syncthreads();
      const float2 *cbk = colbuf + (k % 3) * Lp;
      const float d = cbk[k].x;
      if (!(d > 0.0f) || !(d < INFINITY)) { failed = true; break; }   // uniform
      const float rs = 1.0f / sqrtf(d);
      const float invd = rs * rs;
      if (k > 0) {   // W rows >= k receive row k-1:  X[i][c] -= L[i][k-1] W[k-1][c]
        const float2 *colp = colbuf + ((k + 2) % 3) * Lp;
        const float2 *wrow = wbuf + ((k - 1) & 1) * Lp;
#pragma unroll
        for (int s = 0; s < kMaxSlots; ++s) {
          if (((w_meta[s] >> 16) & 0xff) >= k) {
            const int i = (w_meta[s] >> 8) & 0xff, c = w_meta[s] & 0xff;
            if (i != 0xff && i >= k && c < k) {
              const float2 lv = colp[i];
              const float2 wv = wrow[c];
              const float2 t = cmul(make_float2(lv.x * rs_prev, lv.y * rs_prev), wv);
              wx[s].x -= t.x;
              wx[s].y -= t.y;
            }
          }
        }
      }
      {  // finalise row k of W: W[k][c] = X[k][c] / L[k][k]
        float2 *wnew = wbuf + (k & 1) * Lp;
#pragma unroll
        for (int s = 0; s < kMaxSlots; ++s) {
          const int i = (w_meta[s] >> 8) & 0xff, c = w_meta[s] & 0xff;
          if (i == k) {
            wx[s].x *= rs;
            wx[s].y *= rs;
            wnew[c] = wx[s];
          }
        }
      }
      {  // trailing update A[i][j] -= A[i][k] conj(A[j][k]) / A[k][k]; publish column k+1
        float2 *cbn = colbuf + ((k + 1) % 3) * Lp;
#pragma unroll
        for (int s = 0; s < kMaxSlots; ++s) {
          if (((ch_meta[s] >> 16) & 0xff) > k) {
            const int i = (ch_meta[s] >> 8) & 0xff, j = ch_meta[s] & 0xff;
            if (i != 0xff && j > k) {
              const float2 t = cmul_conj(cbk[i], cbk[j]);
              av[s].x -= t.x * invd;
              av[s].y -= t.y * invd;
              if (j == k + 1) cbn[i] = av[s];
            }
          }
        }
      }
      rs_prev = rs;
    }
    if (failed) break;   // uniform: every workgroup factors the same Sigma

    // ===== C2. Sigma^-1 = W^H W (MFMA), stored full column-major in WS ======
#pragma unroll
    for (int s = 0; s < kMaxSlots; ++s) {
      const int i = (w_meta[s] >> 8) & 0xff, c = w_meta[s] & 0xff;
      if (i != 0xff) WS[i * Lp + c] = wx[s];
    }
    __syncthreads();
    f4 sir[kMaxBlocksPerWave], sii[kMaxBlocksPerWave];
#pragma unroll
    for (int q = 0; q < kMaxBlocksPerWave; ++q) {
      sir[q] = (f4){0.f, 0.f, 0.f, 0.f};
      sii[q] = (f4){0.f, 0.f, 0.f, 0.f};
      const int b = wave + kWaves * q;
      if (b < NB) {
        int I, J;
        blk_coords(b, I, J);
        for (int k0 = 16 * I; k0 < Lp; k0 += 4) {
          const int k = k0 + lq;
          const float2 wi = WS[k * Lp + 16 * I + l16];   // A[i][k] = conj(W[k][i])
          const float2 wj = WS[k * Lp + 16 * J + l16];   // B[k][j] = W[k][j]
          cmfma(make_float2(wi.x, -wi.y), wj, sir[q], sii[q]);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kMaxBlocksPerWave; ++q) {
      const int b = wave + kWaves * q;
      if (b < NB) {
        int I, J;
        blk_coords(b, I, J);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * I + 4 * lq + v, j = 16 * J + l16;
          if (i >= j) {
            const float im = (i == j) ? 0.0f : sii[q][v];
            WS[j * Lp + i] = make_float2(sir[q][v], im);
            WS[i * Lp + j] = make_float2(sir[q][v], -im);
          }
        }
      }
    }
    __syncthreads();

    // ===== C3. B = Sigma^-1 S_g and q ======================================
    // SigmaHat fragments (A operand of D = SigmaHat B) for this wave's row
    // blocks; the loads are issued here and consumed after GEMM 1.
    float2 shf[kMaxRowBlocksPerWave][kMaxKSteps];
#pragma unroll
    for (int rb = 0; rb < kMaxRowBlocksPerWave; ++rb) {
      const int I = wave + kWaves * rb;
#pragma unroll
      for (int ks = 0; ks < kMaxKSteps; ++ks) {
        const int i = 16 * I + l16, k = 4 * ks + lq;
        shf[rb][ks] = (I < Lb && i < A.L && k < A.L) ? A.Sh[(size_t)k * A.L + i] : make_float2(0.f, 0.f);
      }
    }
#pragma unroll
    for (int rb = 0; rb < kMaxRowBlocksPerWave; ++rb) {
      const int I = wave + kWaves * rb;
      if (I < Lb) {
        for (int cb = 0; cb < A.ncb; ++cb) {
          f4 cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
          for (int k0 = 0; k0 < Lp; k0 += 4) {
            const int k = k0 + lq;
            cmfma(WS[k * Lp + 16 * I + l16], St[k * PT + 16 * cb + l16], cr, ci);
          }
          float qp = 0.0f;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = 16 * I + 4 * lq + v, j = 16 * cb + l16;
            const float2 s = St[i * PT + j];
            qp += s.x * cr[v] + s.y * ci[v];
            Bt[i * PT + j] = make_float2(cr[v], ci[v]);
          }
          qp += __shfl_xor(qp, 16);
          qp += __shfl_xor(qp, 32);
          if (lq == 0) red_q[I * NT + 16 * cb + l16] = qp;
        }
      }
    }
    __syncthreads();

    // ===== C4. D = SigmaHat B and r ========================================
#pragma unroll
    for (int rb = 0; rb < kMaxRowBlocksPerWave; ++rb) {
      const int I = wave + kWaves * rb;
      if (I < Lb) {
        for (int cb = 0; cb < A.ncb; ++cb) {
          f4 cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int ks = 0; ks < kMaxKSteps; ++ks) {
            if (4 * ks < Lp) {
              const int k = 4 * ks + lq;
              cmfma(shf[rb][ks], Bt[k * PT + 16 * cb + l16], cr, ci);
            }
          }
          float rp = 0.0f;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = 16 * I + 4 * lq + v, j = 16 * cb + l16;
            const float2 bv = Bt[i * PT + j];
            rp += bv.x * cr[v] + bv.y * ci[v];
          }
          rp += __shfl_xor(rp, 16);
          rp += __shfl_xor(rp, 32);
          if (lq == 0) red_r[I * NT + 16 * cb + l16] = rp;
        }
      }
    }
    __syncthreads();

    // ===== C5. coordinate step and update ==================================
    float rho;
    if (A.rho_fixed >= 0.0f) rho = A.rho_fixed;
    else if (A.rho_dev) rho = A.rho_dev[it];
    else rho = (float)rho_d;
    rho_d = rho_d * (1.0 - A.rho_decay * rho_d);
    const bool last = (it == A.iters - 1);
    for (int c = tid; c < NT; c += THREADS) {
      const int n = n0 + c;
      if (n < A.N) {
        float q = 0.0f, r = 0.0f;
        for (int I = 0; I < Lb; ++I) {
          q += red_q[I * NT + c];
          r += red_r[I * NT + c];
        }
        const float x = xs[c];
        const float xt = coordinate_step(x, q, r, gs[c], ls[c], A.a);
        xs[c] = (1.0f - rho) * x + rho * xt;
        if (last) {
          if (A.q_out) A.q_out[n] = q;
          if (A.r_out) A.r_out[n] = r;
          if (A.xt_out) A.xt_out[n] = xt;
        }
      }
    }
    __syncthreads();
  }

  // ---- results --------------------------------------------------------------
  for (int c = tid; c < NT; c += THREADS) {
    const int n = n0 + c;
    if (n < A.N) A.x_out[n] = xs[c];
  }
  if (g == 0 && tid == 0 && A.status)
    *A.status = aborted ? PSCA_ESYNC : (failed ? PSCA_ENOTPD : PSCA_OK);
}

// SigmaHat = Y Y^H / M; one thread per lower-triangle entry, mirrored so the
// result is exactly Hermitian.
__global__ void __launch_bounds__(kThreads) k_sample_cov(const float2 *__restrict__ Y, int L, int M,
                                                         float2 *__restrict__ Sh) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= L * (L + 1) / 2) return;
  int i = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
  while (i * (i + 1) / 2 > e) --i;
  while ((i + 1) * (i + 2) / 2 <= e) ++i;
  const int j = e - i * (i + 1) / 2;
  float2 acc = make_float2(0.f, 0.f);
  for (int m = 0; m < M; ++m) {
    const float2 t = cmul_conj(Y[i + (size_t)m * L], Y[j + (size_t)m * L]);
    acc.x += t.x;
    acc.y += t.y;
  }
  const float s = 1.0f / (float)M;
  acc.x *= s;
  acc.y *= s;
  if (i == j) acc.y = 0.0f;
  Sh[i + (size_t)j * L] = acc;
  Sh[j + (size_t)i * L] = make_float2(acc.x, -acc.y);
}

// Reset the barrier and abort words before a launch of k_psca.
__global__ void k_prepare(unsigned *bar, int32_t *abort_flag, int32_t *status) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    bar[0] = 0u;
    bar[1] = 0u;
    *abort_flag = 0;
    if (status) *status = PSCA_OK;
  }
}

__global__ void k_threshold(const float *__restrict__ x, int N, float theta, uint8_t *__restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n < N) out[n] = x[n] >= theta ? 1 : 0;
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

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
  if (prm->variant < PSCA_ML_K || prm->variant > PSCA_MAP_UR) return PSCA_EINVAL;
  if (!(prm->sigma2 > 0.0f) || !isfinite(prm->sigma2)) return PSCA_EINVAL;
  if (prm->M < 1) return PSCA_EINVAL;
  if (need_iters) {
    if (prm->iters < 0) return PSCA_EINVAL;
    if (!prm->rho && (!(prm->rho0 > 0.0f) || prm->rho0 > 1.0f || !(prm->rho_decay >= 0.0f) ||
                      prm->rho_decay > 2.0f))
      return PSCA_EINVAL;
  }
  if ((prm->variant == PSCA_ML_K || prm->variant == PSCA_MAP_K) && !prm->g) return PSCA_EINVAL;
  if (prm->variant == PSCA_MAP_K && !prm->p) return PSCA_EINVAL;
  if (prm->variant == PSCA_MAP_UR) {
    if (!(prm->d_lo > 0.0f) || !(prm->d_hi > prm->d_lo) || !(prm->pl_c0 > 0.0f) || !(prm->pl_beta > 0.0f) ||
        !(prm->eps > 0.0f) || !isfinite(prm->d_hi) || !isfinite(prm->pl_c0) || !isfinite(prm->pl_beta))
      return PSCA_EINVAL;
    const double gl = (double)prm->pl_c0 * pow((double)prm->d_hi, -(double)prm->pl_beta);
    if (!(2.0 * (double)prm->eps < gl)) return PSCA_EINVAL;
  }
  return PSCA_OK;
}

StepArgs make_step_args(const psca_params *prm) {
  StepArgs a;
  a.variant = prm->variant;
  a.inv_M = (float)(1.0 / (double)prm->M);
  a.g = (prm->variant == PSCA_ML_K || prm->variant == PSCA_MAP_K) ? prm->g : nullptr;
  a.p = (prm->variant == PSCA_MAP_K) ? prm->p : nullptr;
  a.eps = a.g_l = a.g_u = a.h2_b = a.dens_c = 0.0f;
  if (prm->variant == PSCA_MAP_UR) {
    const double beta = prm->pl_beta;
    const double gl = (double)prm->pl_c0 * pow((double)prm->d_hi, -beta);
    const double gu = (double)prm->pl_c0 * pow((double)prm->d_lo, -beta);
    a.eps = prm->eps;
    a.g_l = (float)gl;
    a.g_u = (float)gu;
    a.dens_c = (float)(2.0 / beta + 1.0);
    a.h2_b = (float)(-(2.0 / beta + 1.0) / gl);
  }
  return a;
}

inline hipStream_t as_stream(void *s) { return (hipStream_t)s; }
int launch_ok() { return hipGetLastError() == hipSuccess ? PSCA_OK : PSCA_EHIP; }

// One instantiation of k_psca with its block size.
struct KernelChoice {
  const void *fn;
  int threads;
};

KernelChoice pick_kernel(int Lp) {
  if (Lp <= 32) return {(const void *)k_psca<32, 256>, 256};
  if (Lp <= 64) return {(const void *)k_psca<64, 256>, 256};
  return {(const void *)k_psca<96, 512>, 512};
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

// Runs k_psca for `iters` iterations from x_in (null: zeros).
int run_detect(psca_ctx *ctx, const float2 *Sh, const float2 *S, int L, int N, const psca_params *prm,
               int iters, float rho_fixed, const float *x_in, float *x_out, float *q_out, float *r_out,
               float *xt_out, int32_t *status, hipStream_t st) {
  const int Lp = (L + 15) & ~15, Lb = Lp / 16, NB = Lb * (Lb + 1) / 2;
  const int E = NB * 256;
  const KernelChoice kc = pick_kernel(Lp);
  int ncb = 1, G = 0;
  size_t lds = 0;
  for (;; ++ncb) {
    if (ncb > kMaxNcb) return PSCA_ENOTSUP;
    const int NT = 16 * ncb;
    G = (N + NT - 1) / NT;
    lds = lds_bytes(Lp, NT, Lb);
    const int cap = max_coresident(ctx, kc, lds);
    if (cap <= 0) return PSCA_ENOTSUP;
    if (G <= cap) break;
  }
  const int NT = 16 * ncb;
  // workspace: partials, Sigma, barrier words
  size_t off = 0;
  const size_t o_part = off; off = align_up(off + (size_t)G * E * sizeof(float2));
  const size_t o_sig = off;  off = align_up(off + (size_t)E * sizeof(float2));
  const size_t o_bar = off;  off = align_up(off + 4 * sizeof(unsigned));
  const size_t o_abt = off;  off = align_up(off + sizeof(int32_t));
  const size_t o_st = off;   off = align_up(off + sizeof(int32_t));
  int rc = ensure_ws(ctx, off);
  if (rc != PSCA_OK) return rc;
  char *base = (char *)ctx->ws;

  CoopArgs a;
  a.S = S;
  a.Sh = Sh;
  a.L = L;
  a.N = N;
  a.Lp = Lp;
  a.Lb = Lb;
  a.NB = NB;
  a.G = G;
  a.ncb = ncb;
  a.NT = NT;
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
  a.status = status ? status : (int32_t *)(base + o_st);
  a.partials = (float2 *)(base + o_part);
  a.sigma = (float2 *)(base + o_sig);
  a.bar = (unsigned *)(base + o_bar);
  a.abort_flag = (int32_t *)(base + o_abt);

  hipLaunchKernelGGL(k_prepare, dim3(1), dim3(64), 0, st, a.bar, a.abort_flag, a.status);
  if ((rc = launch_ok()) != PSCA_OK) return rc;
  void *args[] = {&a};
  if (hipLaunchCooperativeKernel(kc.fn, dim3(G), dim3(kc.threads), args, (unsigned)lds, st) !=
      hipSuccess) {
    (void)hipGetLastError();
    return PSCA_EHIP;
  }
  return PSCA_OK;
}

}  // namespace

extern "C" {

int psca_version(void) { return 200; }

const char *psca_strerror(int code) {
  switch (code) {
    case PSCA_OK: return "ok";
    case PSCA_EINVAL: return "invalid argument";
    case PSCA_ENOTPD: return "covariance matrix not positive definite (Cholesky pivot <= 0 or not finite)";
    case PSCA_EHIP: return "HIP runtime error";
    case PSCA_ENOMEM: return "device memory allocation failed";
    case PSCA_ENOTSUP: return "size not supported by this build";
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
  *ctx = c;
  return PSCA_OK;
}

int psca_destroy(psca_ctx *ctx) {
  if (!ctx) return PSCA_OK;
  int rc = PSCA_OK;
  if (ctx->ws || ctx->sh) {
    DeviceGuard g(ctx->device);
    if (hipDeviceSynchronize() != hipSuccess) rc = PSCA_EHIP;
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->sh) (void)hipFree(ctx->sh);
  }
  delete ctx;
  return rc;
}

int psca_sample_cov(psca_ctx *ctx, const psca_c32 *Y, int L, int M, psca_c32 *Sigma_hat, void *stream) {
  if (!ctx || !Y || !Sigma_hat || L < 1 || M < 1) return PSCA_EINVAL;
  if (L > kMaxL) return PSCA_ENOTSUP;
  DeviceGuard g(ctx->device);
  if (!g.ok) return PSCA_EHIP;
  const int T = L * (L + 1) / 2;
  hipLaunchKernelGGL(k_sample_cov, dim3((T + kThreads - 1) / kThreads), dim3(kThreads), 0, as_stream(stream),
                     (const float2 *)Y, L, M, (float2 *)Sigma_hat);
  return launch_ok();
}

int psca_detect(psca_ctx *ctx, const psca_c32 *Sigma_hat, const psca_c32 *S, int L, int N,
                const psca_params *prm, float *x_out, int32_t *status, void *stream) {
  if (!ctx || !Sigma_hat || !S || !x_out) return PSCA_EINVAL;
  int rc = validate_params(prm, L, N, true);
  if (rc != PSCA_OK) return rc;
  DeviceGuard g(ctx->device);
  if (!g.ok) return PSCA_EHIP;
  return run_detect(ctx, (const float2 *)Sigma_hat, (const float2 *)S, L, N, prm, prm->iters, -1.0f, nullptr,
                    x_out, nullptr, nullptr, nullptr, status, as_stream(stream));
}

int psca_detect_y(psca_ctx *ctx, const psca_c32 *Y, const psca_c32 *S, int L, int N,
                  const psca_params *prm, float *x_out, int32_t *status, void *stream) {
  if (!ctx || !Y || !S || !x_out) return PSCA_EINVAL;
  int rc = validate_params(prm, L, N, true);
  if (rc != PSCA_OK) return rc;
  DeviceGuard g(ctx->device);
  if (!g.ok) return PSCA_EHIP;
  static_assert(sizeof(float2) == sizeof(psca_c32), "layout");
  rc = ensure_buf(&ctx->sh, &ctx->sh_bytes, (size_t)L * L * sizeof(float2));
  if (rc != PSCA_OK) return rc;
  float2 *Sh = (float2 *)ctx->sh;
  const int T = L * (L + 1) / 2;
  hipLaunchKernelGGL(k_sample_cov, dim3((T + kThreads - 1) / kThreads), dim3(kThreads), 0, as_stream(stream),
                     (const float2 *)Y, L, prm->M, Sh);
  if ((rc = launch_ok()) != PSCA_OK) return rc;
  return run_detect(ctx, Sh, (const float2 *)S, L, N, prm, prm->iters, -1.0f, nullptr, x_out, nullptr, nullptr,
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

int psca_threshold(const float *x, int N, float theta, uint8_t *support, void *stream) {
  if (!x || !support || N < 1) return PSCA_EINVAL;
  hipLaunchKernelGGL(k_threshold, dim3((N + 255) / 256), dim3(256), 0, as_stream(stream), x, N, theta, support);
  return launch_ok();
}

}  // extern "C"
