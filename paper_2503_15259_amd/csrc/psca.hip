// psca.hip — HIP kernels (gfx950) and C ABI for PSCA device activity detection.
//
// One PSCA iteration (Algorithm 1, steps 5-8 of Tan & Cui, arXiv 2503.15259):
//   Sigma = S diag(w) S^H + sigma^2 I            (eq. cov_a / cov_b)
//   Sigma = L L^H (Cholesky), W = L^-1, Sigma^-1 = W^H W
//   B = Sigma^-1 S, D = SigmaHat B                (complex GEMMs)
//   q_n = Re(s_n^H b_n), r_n = Re(b_n^H D_n)      (quadratic forms of eq. gradient_ML)
//   x~_n = clip(x_n - grad_n / curv_n, lo, hi)    (Lemmas 1-4)
//   x_n <- (1 - rho_k) x_n + rho_k x~_n           (eqs. Update_*)
//
// Launch structure per iteration (all on the caller's stream):
//   k_factor  : 1 workgroup. Sums the per-tile partials of Sigma, factors it in
//               LDS and writes Sigma^-1 (full, column-major) to the workspace.
//   k_step    : one workgroup per 64-column tile of S.  Both GEMMs, the
//               quadratic forms, the variant's step and the update; then the
//               tile's partial S_t diag(w^(k+1)) S_t^H of the next Sigma
//               (packed lower triangle) so the next k_factor needs no pass
//               over S.
//
// Numerics: complex single precision, FP32 accumulation in a fixed order (no
// atomics), so a run is bitwise reproducible.

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <new>

#include "psca.h"

namespace {

constexpr int kThreads = 256;       // threads per workgroup (4 wave64)
constexpr int kTileN = 64;          // columns of S per k_step workgroup
constexpr int kMaxL = PSCA_MAX_L;
constexpr int kLdsPitch = kMaxL + 1;  // row pitch of the LDS L x L matrices
constexpr int kMaxRowsPerThread = (kMaxL + 3) / 4;

// ---------------------------------------------------------------------------
// complex helpers (float2 = re, im)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// a * b
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmul_conj(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// acc += a * b
__device__ __forceinline__ void cfma(float2 &acc, float2 a, float2 b) {
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(-a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(a.y, b.x, acc.y);
}

__device__ __forceinline__ int tri_size(int L) { return L * (L + 1) / 2; }

// (i, j) with j <= i of packed lower-triangle index e = i (i + 1) / 2 + j
__device__ __forceinline__ void tri_index(int e, int &i, int &j) {
  int r = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
  while (r * (r + 1) / 2 > e) --r;
  while ((r + 1) * (r + 2) / 2 <= e) ++r;
  i = r;
  j = e - r * (r + 1) / 2;
}

// ---------------------------------------------------------------------------
// Variant step (Lemmas 1-4)
// ---------------------------------------------------------------------------
struct StepArgs {
  int variant;
  float inv_M;          // 1 / M
  const float *g;       // [N] known pathloss (K variants)
  const float *p;       // [N] activity probability (MAP-K)
  // MAP-UR prior constants (power-law pathloss map, area-uniform distance)
  float eps, g_l, g_u, h2_b, dens_c;
};

// p^eps'(x) / p^eps(x) of the smoothed prior (eqs. peps, H2, pepsd), in the
// simplified per-piece forms; 0 where p^eps = 0 (the gap).
__device__ __forceinline__ float prior_log_ratio(float x, const StepArgs &a) {
  const float e = a.eps;
  if (x < e) {
    // H1'/H1 = 6 x / ((eps + 2x)(x - eps))
    return 6.0f * x / ((e + 2.0f * x) * (x - e));
  }
  if (x < a.g_l - e) return 0.0f;
  if (x < a.g_l) {
    // H2'/H2 with u = x - g_l and b = B/A:
    //   [-6u/eps + b(3u + eps)] / ((u + eps)[(1 - 2u/eps) + b u])
    const float u = x - a.g_l;
    const float num = -6.0f * u / e + a.h2_b * (3.0f * u + e);
    const float den = (u + e) * ((1.0f - 2.0f * u / e) + a.h2_b * u);
    return den == 0.0f ? 0.0f : num / den;
  }
  // density piece, phi(d) = c0 d^-beta: -(2/beta + 1) / x
  return -a.dens_c / x;
}

// Returns x~; writes nothing else.
__device__ __forceinline__ float coordinate_step(float x, float q, float r, int n, const StepArgs &a) {
  float grad, curv, lo = 0.0f, hi;
  switch (a.variant) {
    case PSCA_ML_K: {
      const float g = a.g[n];
      grad = g * (q - r);
      const float gq = g * q;
      curv = gq * gq;
      hi = 1.0f;
      break;
    }
    case PSCA_MAP_K: {
      const float g = a.g[n];
      const float pn = a.p[n];
      grad = g * (q - r) - logf(pn / (1.0f - pn)) * a.inv_M;
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
  return fminf(fmaxf(x - grad / curv, lo), hi);
}

__device__ __forceinline__ float weight_of(float x, int n, const StepArgs &a) {
  return (a.variant == PSCA_ML_K || a.variant == PSCA_MAP_K) ? a.g[n] * x : x;
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// SigmaHat = Y Y^H / M; one thread per lower-triangle entry, mirrored.
__global__ void __launch_bounds__(kThreads) k_sample_cov(const float2 *__restrict__ Y, int L, int M,
                                                         float2 *__restrict__ Sh) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= tri_size(L)) return;
  int i, j;
  tri_index(e, i, j);
  float2 acc = make_float2(0.f, 0.f);
  for (int m = 0; m < M; ++m) {
    const float2 yi = Y[i + (size_t)m * L];
    const float2 yj = Y[j + (size_t)m * L];
    const float2 t = cmul_conj(yi, yj);
    acc = cadd(acc, t);
  }
  const float s = 1.0f / (float)M;
  acc.x *= s;
  acc.y *= s;
  if (i == j) acc.y = 0.0f;
  Sh[i + (size_t)j * L] = acc;
  Sh[j + (size_t)i * L] = make_float2(acc.x, -acc.y);
}

// x = 0 (or copy), clear the failure flag and the caller's status word.
__global__ void k_init(float *__restrict__ x, const float *__restrict__ x_src, int N,
                       int32_t *__restrict__ flag, int32_t *__restrict__ status) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n < N) x[n] = x_src ? x_src[n] : 0.0f;
  if (n == 0) {
    *flag = 0;
    if (status) *status = PSCA_OK;
  }
}

__global__ void k_copy(float *__restrict__ dst, const float *__restrict__ src, int N) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n < N) dst[n] = src[n];
}

__global__ void k_finish(const int32_t *__restrict__ flag, int32_t *__restrict__ status) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && status) *status = *flag ? PSCA_ENOTPD : PSCA_OK;
}

// Load the 64-column tile t of S (L x N, column-major) into LDS St[j * kTileN + c];
// columns past N are zero.
__device__ __forceinline__ void load_tile(const float2 *__restrict__ S, int L, int N, int tile,
                                          float2 *St) {
  const int n0 = tile * kTileN;
  for (int e = threadIdx.x; e < L * kTileN; e += blockDim.x) {
    const int c = e / L;        // consecutive threads walk down a column: coalesced reads
    const int j = e - c * L;
    const int n = n0 + c;
    St[j * kTileN + c] = (n < N) ? S[(size_t)n * L + j] : make_float2(0.f, 0.f);
  }
}

// Partial S_t diag(w) S_t^H of one tile (packed lower triangle) from LDS.
__device__ __forceinline__ void tile_partial(const float2 *St, const float *w, int L,
                                             float2 *__restrict__ out) {
  const int T = tri_size(L);
  for (int e = threadIdx.x; e < T; e += blockDim.x) {
    int i, j;
    tri_index(e, i, j);
    float2 acc = make_float2(0.f, 0.f);
    const float2 *si = St + i * kTileN;
    const float2 *sj = St + j * kTileN;
    for (int c = 0; c < kTileN; ++c) {
      const float2 t = cmul_conj(si[c], sj[c]);
      acc.x = fmaf(w[c], t.x, acc.x);
      acc.y = fmaf(w[c], t.y, acc.y);
    }
    out[e] = acc;
  }
}

// Partials of Sigma(x) for every tile (used before the first iteration).
__global__ void __launch_bounds__(kThreads) k_partial(const float2 *__restrict__ S, int L, int N,
                                                      const float *__restrict__ x, StepArgs a,
                                                      float2 *__restrict__ partials) {
  __shared__ float2 St[kMaxL * kTileN];
  __shared__ float w[kTileN];
  const int tile = blockIdx.x;
  load_tile(S, L, N, tile, St);
  if (threadIdx.x < kTileN) {
    const int n = tile * kTileN + threadIdx.x;
    w[threadIdx.x] = (n < N) ? weight_of(x[n], n, a) : 0.0f;
  }
  __syncthreads();
  tile_partial(St, w, L, partials + (size_t)tile * tri_size(L));
}

// Sigma = sigma^2 I + sum_t partial_t; Cholesky Sigma = L L^H; W = L^-1;
// Sigma^-1 = W^H W written full, column-major, to Sinv.  A pivot that is not
// finite and positive raises *flag and leaves Sinv untouched.
__global__ void __launch_bounds__(kThreads) k_factor(const float2 *__restrict__ partials, int n_tiles,
                                                     int L, float sigma2, float2 *__restrict__ Sinv,
                                                     int32_t *__restrict__ flag) {
  __shared__ float2 A[kMaxL * kLdsPitch];   // row-major, lower triangle used
  __shared__ float2 W[kMaxL * kLdsPitch];   // row-major, lower triangle
  __shared__ float dg[kMaxL];               // diagonal of the Cholesky factor
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int T = tri_size(L);
  if (*flag) return;  // an earlier iteration already failed

  for (int e = tid; e < T; e += blockDim.x) {
    int i, j;
    tri_index(e, i, j);
    float2 acc = make_float2(i == j ? sigma2 : 0.f, 0.f);
    for (int t = 0; t < n_tiles; ++t) acc = cadd(acc, partials[(size_t)t * T + e]);
    if (i == j) acc.y = 0.0f;
    A[i * kLdsPitch + j] = acc;
  }
  if (tid == 0) bad = 0;
  __syncthreads();

  // Right-looking Cholesky, column k per step.
  for (int k = 0; k < L; ++k) {
    const float d = A[k * kLdsPitch + k].x;
    if (!(d > 0.0f) || !isfinite(d)) {  // uniform across the block
      if (tid == 0) bad = 1;
      break;
    }
    const float sd = sqrtf(d);
    const float inv = 1.0f / sd;
    if (tid == 0) dg[k] = sd;
    for (int i = k + 1 + tid; i < L; i += blockDim.x) {
      float2 v = A[i * kLdsPitch + k];
      A[i * kLdsPitch + k] = make_float2(v.x * inv, v.y * inv);
    }
    __syncthreads();
    const int m = L - k - 1;
    for (int e = tid; e < m * m; e += blockDim.x) {
      const int ii = e / m, jj = e - ii * m;
      if (jj > ii) continue;
      const int i = k + 1 + ii, j = k + 1 + jj;
      const float2 lik = A[i * kLdsPitch + k];
      const float2 ljk = A[j * kLdsPitch + k];
      A[i * kLdsPitch + j] = csub(A[i * kLdsPitch + j], cmul_conj(lik, ljk));
    }
    __syncthreads();
  }
  __syncthreads();
  if (bad) {
    if (tid == 0) *flag = 1;
    return;
  }

  // W = L^-1 by forward substitution on the identity, row k per step.
  for (int e = tid; e < L * L; e += blockDim.x) {
    const int i = e / L, j = e - (e / L) * L;
    W[i * kLdsPitch + j] = make_float2(i == j ? 1.0f : 0.0f, 0.0f);
  }
  __syncthreads();
  for (int k = 0; k < L; ++k) {
    const float inv = 1.0f / dg[k];
    for (int c = tid; c <= k; c += blockDim.x) {
      const float2 v = W[k * kLdsPitch + c];
      W[k * kLdsPitch + c] = make_float2(v.x * inv, v.y * inv);
    }
    __syncthreads();
    const int rows = L - k - 1, cols = k + 1;
    for (int e = tid; e < rows * cols; e += blockDim.x) {
      const int ii = e / cols, c = e - ii * cols;
      const int i = k + 1 + ii;
      const float2 lik = A[i * kLdsPitch + k];
      W[i * kLdsPitch + c] = csub(W[i * kLdsPitch + c], cmul(lik, W[k * kLdsPitch + c]));
    }
    __syncthreads();
  }

  // Sigma^-1[i][j] = sum_{k >= max(i,j)} conj(W[k][i]) W[k][j]
  for (int e = tid; e < T; e += blockDim.x) {
    int i, j;
    tri_index(e, i, j);  // j <= i
    float2 acc = make_float2(0.f, 0.f);
    for (int k = i; k < L; ++k) {
      const float2 wki = W[k * kLdsPitch + i];
      const float2 wkj = W[k * kLdsPitch + j];
      // conj(wki) * wkj
      acc.x = fmaf(wki.x, wkj.x, acc.x);
      acc.x = fmaf(wki.y, wkj.y, acc.x);
      acc.y = fmaf(wki.x, wkj.y, acc.y);
      acc.y = fmaf(-wki.y, wkj.x, acc.y);
    }
    if (i == j) acc.y = 0.0f;
    Sinv[i + (size_t)j * L] = acc;
    Sinv[j + (size_t)i * L] = make_float2(acc.x, -acc.y);
  }
}

// acc[r] = sum_j A[rows_r, j] * X[j, c] for the thread's rows i0 + 4 r and
// column c; A is L x L column-major in global memory, X lives in LDS.
__device__ __forceinline__ void tile_gemm(const float2 *__restrict__ A, const float2 *X, int L,
                                          int i0, int c, float2 (&acc)[kMaxRowsPerThread]) {
#pragma unroll
  for (int r = 0; r < kMaxRowsPerThread; ++r) acc[r] = make_float2(0.f, 0.f);
  for (int j = 0; j < L; ++j) {
    const float2 xv = X[j * kTileN + c];
    const float2 *Acol = A + (size_t)j * L;
#pragma unroll
    for (int r = 0; r < kMaxRowsPerThread; ++r) {
      const int i = i0 + 4 * r;
      if (i < L) cfma(acc[r], Acol[i], xv);
    }
  }
}

// One tile of steps 7-8 plus the next iteration's partial of Sigma.
__global__ void __launch_bounds__(kThreads) k_step(const float2 *__restrict__ S, const float2 *__restrict__ Sh,
                                                   const float2 *__restrict__ Sinv, int L, int N,
                                                   StepArgs a, float rho, const float *__restrict__ rho_dev,
                                                   int rho_index, const float *__restrict__ x_in,
                                                   float *__restrict__ x_out, float *__restrict__ q_out,
                                                   float *__restrict__ r_out, float *__restrict__ xt_out,
                                                   float2 *__restrict__ partials,
                                                   const int32_t *__restrict__ flag) {
  __shared__ float2 St[kMaxL * kTileN];
  __shared__ float2 Bt[kMaxL * kTileN];
  __shared__ float red_q[4][kTileN];
  __shared__ float red_r[4][kTileN];
  __shared__ float w[kTileN];
  const int tid = threadIdx.x;
  const int tile = blockIdx.x;
  const int c = tid % kTileN;
  const int i0 = tid / kTileN;
  const int n = tile * kTileN + c;

  if (*flag) {  // Sigma of this iterate was not positive definite: hold x
    if (i0 == 0 && n < N) x_out[n] = x_in[n];
    return;
  }
  if (rho_dev) rho = rho_dev[rho_index];

  load_tile(S, L, N, tile, St);
  __syncthreads();

  float2 acc[kMaxRowsPerThread];
  // B = Sigma^-1 S_t
  tile_gemm(Sinv, St, L, i0, c, acc);
  float qp = 0.0f;
#pragma unroll
  for (int r = 0; r < kMaxRowsPerThread; ++r) {
    const int i = i0 + 4 * r;
    if (i < L) {
      const float2 s = St[i * kTileN + c];
      qp = fmaf(s.x, acc[r].x, qp);
      qp = fmaf(s.y, acc[r].y, qp);
      Bt[i * kTileN + c] = acc[r];
    }
  }
  red_q[i0][c] = qp;
  __syncthreads();
  // D = SigmaHat B
  tile_gemm(Sh, Bt, L, i0, c, acc);
  float rp = 0.0f;
#pragma unroll
  for (int r = 0; r < kMaxRowsPerThread; ++r) {
    const int i = i0 + 4 * r;
    if (i < L) {
      const float2 b = Bt[i * kTileN + c];
      rp = fmaf(b.x, acc[r].x, rp);
      rp = fmaf(b.y, acc[r].y, rp);
    }
  }
  red_r[i0][c] = rp;
  __syncthreads();

  if (tid < kTileN) {
    float wn = 0.0f;
    if (n < N) {
      const float q = (red_q[0][c] + red_q[1][c]) + (red_q[2][c] + red_q[3][c]);
      const float r = (red_r[0][c] + red_r[1][c]) + (red_r[2][c] + red_r[3][c]);
      const float x = x_in[n];
      const float xt = coordinate_step(x, q, r, n, a);
      const float xn = (1.0f - rho) * x + rho * xt;
      x_out[n] = xn;
      if (q_out) q_out[n] = q;
      if (r_out) r_out[n] = r;
      if (xt_out) xt_out[n] = xt;
      wn = weight_of(xn, n, a);
    }
    w[c] = wn;
  }
  if (partials == nullptr) return;  // uniform: no next iteration
  __syncthreads();
  tile_partial(St, w, L, partials + (size_t)tile * tri_size(L));
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
  void *ws;
  size_t ws_bytes;
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

int ensure_ws(psca_ctx *ctx, size_t bytes) {
  if (bytes <= ctx->ws_bytes) return PSCA_OK;
  if (ctx->ws) {
    if (hipDeviceSynchronize() != hipSuccess) return PSCA_EHIP;
    (void)hipFree(ctx->ws);
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  size_t want = bytes + bytes / 4;
  if (hipMalloc(&ctx->ws, want) != hipSuccess) {
    (void)hipGetLastError();
    ctx->ws = nullptr;
    return PSCA_ENOMEM;
  }
  ctx->ws_bytes = want;
  return PSCA_OK;
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

struct Workspace {
  float2 *partials;
  float2 *Sinv;
  float2 *Sh;     // sample covariance for psca_detect_y
  float *x0, *x1;
  int32_t *flag;
};

int layout_ws(psca_ctx *ctx, int L, int N, bool need_sh, Workspace &w) {
  const int tiles = (N + kTileN - 1) / kTileN;
  const size_t tri = (size_t)L * (L + 1) / 2;
  size_t off = 0;
  const size_t o_part = off; off = align_up(off + (size_t)tiles * tri * sizeof(float2));
  const size_t o_sinv = off; off = align_up(off + (size_t)L * L * sizeof(float2));
  const size_t o_sh = off;   off = align_up(off + (need_sh ? (size_t)L * L * sizeof(float2) : 0));
  const size_t o_x0 = off;   off = align_up(off + (size_t)N * sizeof(float));
  const size_t o_x1 = off;   off = align_up(off + (size_t)N * sizeof(float));
  const size_t o_flag = off; off = align_up(off + 256);
  const int rc = ensure_ws(ctx, off);
  if (rc != PSCA_OK) return rc;
  char *base = (char *)ctx->ws;
  w.partials = (float2 *)(base + o_part);
  w.Sinv = (float2 *)(base + o_sinv);
  w.Sh = need_sh ? (float2 *)(base + o_sh) : nullptr;
  w.x0 = (float *)(base + o_x0);
  w.x1 = (float *)(base + o_x1);
  w.flag = (int32_t *)(base + o_flag);
  return PSCA_OK;
}

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
  a.g = prm->g;
  a.p = prm->p;
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

// Runs `iters` iterations from x0 (already initialised in w.x0); the final
// iterate is copied to x_out.  Optional per-iteration outputs are written
// by the last iteration only.
int run_iterations(const float2 *Sh, const float2 *S, int L, int N, const psca_params *prm,
                   const Workspace &w, int iters, const float *rho_host_single, float *x_out,
                   float *q_out, float *r_out, float *xt_out, hipStream_t st) {
  const StepArgs a = make_step_args(prm);
  const int tiles = (N + kTileN - 1) / kTileN;
  hipLaunchKernelGGL(k_partial, dim3(tiles), dim3(kThreads), 0, st, S, L, N, w.x0, a, w.partials);
  float *xa = w.x0, *xb = w.x1;
  double rho = prm->rho0;
  for (int k = 0; k < iters; ++k) {
    const bool last = (k == iters - 1);
    hipLaunchKernelGGL(k_factor, dim3(1), dim3(kThreads), 0, st, w.partials, tiles, L, prm->sigma2, w.Sinv,
                       w.flag);
    const float rk = rho_host_single ? *rho_host_single : (float)rho;
    float *dst = last ? x_out : xb;
    hipLaunchKernelGGL(k_step, dim3(tiles), dim3(kThreads), 0, st, S, Sh, w.Sinv, L, N, a, rk,
                       rho_host_single ? nullptr : prm->rho, k, xa, dst, last ? q_out : nullptr,
                       last ? r_out : nullptr, last ? xt_out : nullptr, last ? nullptr : w.partials, w.flag);
    rho = rho * (1.0 - (double)prm->rho_decay * rho);
    float *t = xa;
    xa = xb;
    xb = t;
  }
  if (iters == 0) {
    hipLaunchKernelGGL(k_copy, dim3((N + 255) / 256), dim3(256), 0, st, x_out, w.x0, N);
  }
  return launch_ok();
}

}  // namespace

extern "C" {

int psca_version(void) { return 100; }

const char *psca_strerror(int code) {
  switch (code) {
    case PSCA_OK: return "ok";
    case PSCA_EINVAL: return "invalid argument";
    case PSCA_ENOTPD: return "covariance matrix not positive definite (Cholesky pivot <= 0 or not finite)";
    case PSCA_EHIP: return "HIP runtime error";
    case PSCA_ENOMEM: return "device memory allocation failed";
    case PSCA_ENOTSUP: return "size not supported by this build";
    default: return "unknown error";
  }
}

int psca_create(psca_ctx **ctx, int device) {
  if (!ctx) return PSCA_EINVAL;
  *ctx = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess) return PSCA_EHIP;
  if (device < 0 || device >= count) return PSCA_EINVAL;
  psca_ctx *c = new (std::nothrow) psca_ctx;
  if (!c) return PSCA_ENOMEM;
  c->device = device;
  c->ws = nullptr;
  c->ws_bytes = 0;
  *ctx = c;
  return PSCA_OK;
}

int psca_destroy(psca_ctx *ctx) {
  if (!ctx) return PSCA_OK;
  int rc = PSCA_OK;
  if (ctx->ws) {
    DeviceGuard g(ctx->device);
    if (hipDeviceSynchronize() != hipSuccess) rc = PSCA_EHIP;
    (void)hipFree(ctx->ws);
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
  Workspace w;
  rc = layout_ws(ctx, L, N, false, w);
  if (rc != PSCA_OK) return rc;
  hipStream_t st = as_stream(stream);
  hipLaunchKernelGGL(k_init, dim3((N + 255) / 256), dim3(256), 0, st, w.x0, (const float *)nullptr, N, w.flag,
                     status);
  rc = run_iterations((const float2 *)Sigma_hat, (const float2 *)S, L, N, prm, w, prm->iters, nullptr, x_out,
                      nullptr, nullptr, nullptr, st);
  if (rc != PSCA_OK) return rc;
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, st, w.flag, status);
  return launch_ok();
}

int psca_detect_y(psca_ctx *ctx, const psca_c32 *Y, const psca_c32 *S, int L, int N,
                  const psca_params *prm, float *x_out, int32_t *status, void *stream) {
  if (!ctx || !Y || !S || !x_out) return PSCA_EINVAL;
  int rc = validate_params(prm, L, N, true);
  if (rc != PSCA_OK) return rc;
  DeviceGuard g(ctx->device);
  if (!g.ok) return PSCA_EHIP;
  Workspace w;
  rc = layout_ws(ctx, L, N, true, w);
  if (rc != PSCA_OK) return rc;
  hipStream_t st = as_stream(stream);
  const int T = L * (L + 1) / 2;
  hipLaunchKernelGGL(k_sample_cov, dim3((T + kThreads - 1) / kThreads), dim3(kThreads), 0, st, (const float2 *)Y,
                     L, prm->M, w.Sh);
  hipLaunchKernelGGL(k_init, dim3((N + 255) / 256), dim3(256), 0, st, w.x0, (const float *)nullptr, N, w.flag,
                     status);
  rc = run_iterations(w.Sh, (const float2 *)S, L, N, prm, w, prm->iters, nullptr, x_out, nullptr, nullptr,
                      nullptr, st);
  if (rc != PSCA_OK) return rc;
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, st, w.flag, status);
  return launch_ok();
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
  Workspace w;
  rc = layout_ws(ctx, L, N, false, w);
  if (rc != PSCA_OK) return rc;
  hipStream_t st = as_stream(stream);
  hipLaunchKernelGGL(k_init, dim3((N + 255) / 256), dim3(256), 0, st, w.x0, x_in, N, w.flag, status);
  rc = run_iterations((const float2 *)Sigma_hat, (const float2 *)S, L, N, prm, w, 1, &rho, x_out, q_out, r_out,
                      xt_out, st);
  if (rc != PSCA_OK) return rc;
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, st, w.flag, status);
  return launch_ok();
}

int psca_threshold(const float *x, int N, float theta, uint8_t *support, void *stream) {
  if (!x || !support || N < 1) return PSCA_EINVAL;
  hipLaunchKernelGGL(k_threshold, dim3((N + 255) / 256), dim3(256), 0, as_stream(stream), x, N, theta, support);
  return launch_ok();
}

}  // extern "C"
