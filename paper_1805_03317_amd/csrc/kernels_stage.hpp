// Device kernels of the per-stage steps around the move (gfx950, wave64):
// initial particles, the tempering exponent search and reweighting, the
// weighted moments and Cholesky factor of the mass matrix, resampling with
// its gathers, and the control-variate build. Each step has a single-dataset
// entry point and a batched one (one workgroup range per batch member).
#pragma once

#include "kernels.hpp"

namespace subsmc {

// --------------------------------------------------------------------------
// initial particles (Algorithm 2 step 1)
// --------------------------------------------------------------------------

struct InitArgs {
  Prob P;
  const double* L0inv;  // inverse of the lower Cholesky factor of the prior precision
  double* theta;
  int32_t* u;
  double* logw;
};

__global__ void __launch_bounds__(kWave) init_kernel(InitArgs A) {
  const int i = blockIdx.x;
  const int lane = threadIdx.x;
  const Prob& P = A.P;
  if (i >= P.M) return;
  const int d = P.d;
  const uint64_t c0 = stream_ctr0(kPriorNormal, 0, 0, P.dataset);
  const double z = lane < d ? stream_normal(P.seed, c0, (uint64_t)i, (uint32_t)lane) : 0.0;
  double x = 0.0;  // theta - mu0 = L0^{-T} z
  for (int e = 0; e < d; ++e) {
    const double ze = readlane_d(z, e);
    x += (lane < d && e >= lane ? A.L0inv[e * d + lane] : 0.0) * ze;
  }
  if (lane < d) A.theta[(int64_t)i * d + lane] = P.mu0[lane] + x;
  const uint64_t c1 = stream_ctr0(kInitIndex, 0, 0, P.dataset);
  int32_t* urow = A.u + (int64_t)i * P.m;
  for (int j = lane; j < P.m; j += kWave)
    urow[j] = (int32_t)word_to_index(stream_word(P.seed, c1, (uint64_t)i, (uint64_t)j), (uint64_t)P.n);
  if (lane == 0) A.logw[i] = -log((double)P.M);
}

// --------------------------------------------------------------------------
// block-level helpers (multi-wave kernels)
// --------------------------------------------------------------------------

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int k = 0; k < NT / kWave; ++k) t += sh[k];
  return t;
}

template <int NT>
__device__ __forceinline__ double block_max(double v, double* sh) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double t = -INFINITY;
#pragma unroll
  for (int k = 0; k < NT / kWave; ++k) t = fmax(t, sh[k]);
  return t;
}

// --------------------------------------------------------------------------
// tempering: ESS bisection, reweighting and evidence increment
// (sections 2.2, 3.3 and 3.5; Algorithm 2 steps b-c)
// --------------------------------------------------------------------------

constexpr int kTemperThreads = 1024;
constexpr int kTemperWaves = kTemperThreads / kWave;
constexpr int kTemperPer = 8;        // particles per thread: M <= 8192

struct TemperArgs {
  int M;
  double a_prev, ess_frac;
  const double* lhat;
  const double* sig2;
  double* logw;     // in/out
  double* out;      // [a, dlogz, ess, status, evaluations]
  const double* grid_ess;  // null: the exponent search's result; else the ESS at grid_n grid points
  int grid_n;
  struct SearchSlot* search;  // two slots of the exponent search
};

// Grid of candidate exponents of the paper's grid rule (section 2.2):
// a_j = a_prev + (1 - a_prev) 2^(-j/4), a_0 = 1 (2^(-1/4), 2^(-1/2) and
// 2^(-3/4) correctly rounded), with the product and the sum rounded
// separately (no fused multiply-add), so every grid point is a fixed function
// of a_prev and j.
__device__ inline double grid_exponent(double a_prev, int j) {
#pragma clang fp contract(off)
  if (j == 0) return 1.0;
  const int r = j & 3;
  const double f = r == 0 ? 1.0 : r == 1 ? 0x1.ae89f995ad3adp-1 : r == 2 ? 0x1.6a09e667f3bcdp-1 : 0x1.306fe0a31b715p-1;
  return a_prev + (1.0 - a_prev) * ldexp(f, -(j >> 2));
}

constexpr int kGridMax = 256;
constexpr int kGridThreads = 256;

struct GridArgs {
  int M;
  double a_prev;
  const double* lhat;
  const double* sig2;
  const double* logw;
  double* ess;  // grid_n
};

__device__ __forceinline__ double incr_weight(double a, double a_prev, double lh, double s2) {
  const double v = (a - a_prev) * (lh - 0.5 * (a + a_prev) * s2);
  return isfinite(v) ? v : -INFINITY;
}

// Block reductions with one barrier each: every call writes the wave partials
// into its own slice of `sh` (the caller rotates `buf` over 4 slices), so a
// write never races the previous call's reads. Fixed order: butterfly, then
// waves 0..15.
constexpr int kTemperSlice = 5 * kTemperWaves;

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}

__device__ __forceinline__ double block_max_1(double v, double* sh, int buf) {
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  v = wave_max(v);
  double* b = sh + buf * kTemperSlice;
  if (l == 0) b[w] = v;
  __syncthreads();
  double t = -INFINITY;
#pragma unroll
  for (int q = 0; q < kTemperWaves; ++q) t = fmax(t, b[q]);
  return t;
}

template <int N>
__device__ __forceinline__ void block_sum_n(double* v, double* sh, int buf) {
  static_assert(N <= 5, "slice holds 5 values per wave");
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = wave_sum(v[k]);
  double* b = sh + buf * kTemperSlice;
  if (l == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) b[k * kTemperWaves + w] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < N; ++k) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kTemperWaves; ++q) t += b[k * kTemperWaves + q];
    v[k] = t;
  }
}

__device__ __forceinline__ void block_sum_2(double& v1, double& v2, double* sh, int buf) {
  double v[2] = {v1, v2};
  block_sum_n<2>(v, sh, buf);
  v1 = v[0];
  v2 = v[1];
}

// ESS at grid point j = blockIdx.x (block_max over 256 threads, then the two
// sums in fixed order).
__global__ void __launch_bounds__(kGridThreads) grid_ess_kernel(GridArgs A) {
  __shared__ double sh[3 * (kGridThreads / kWave)];
  const int t = threadIdx.x, w = t / kWave, l = t % kWave;
  const double a = grid_exponent(A.a_prev, blockIdx.x);
  double mx = -INFINITY;
  for (int i = t; i < A.M; i += kGridThreads) mx = fmax(mx, A.logw[i] + incr_weight(a, A.a_prev, A.lhat[i], A.sig2[i]));
  mx = wave_max(mx);
  if (l == 0) sh[w] = mx;
  __syncthreads();
  mx = -INFINITY;
#pragma unroll
  for (int q = 0; q < kGridThreads / kWave; ++q) mx = fmax(mx, sh[q]);
  double s1 = 0.0, s2 = 0.0;
  if (isfinite(mx)) {
    for (int i = t; i < A.M; i += kGridThreads) {
      const double e = exp(A.logw[i] + incr_weight(a, A.a_prev, A.lhat[i], A.sig2[i]) - mx);
      s1 += e;
      s2 += e * e;
    }
  }
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if (l == 0) {
    sh[kGridThreads / kWave + w] = s1;
    sh[2 * (kGridThreads / kWave) + w] = s2;
  }
  __syncthreads();
  if (t == 0) {
    double t1 = 0.0, t2 = 0.0;
    for (int q = 0; q < kGridThreads / kWave; ++q) {
      t1 += sh[kGridThreads / kWave + q];
      t2 += sh[2 * (kGridThreads / kWave) + q];
    }
    A.ess[blockIdx.x] = isfinite(mx) ? t1 * t1 / t2 : 0.0;
  }
}

// --------------------------------------------------------------------------
// Exponent search (section 2.2; Algorithm 2 step b): a in (a_prev, 1] with
// ESS(a) = ess_frac M. a = 1 when ESS(1) meets the target; otherwise 60
// halvings of [a_prev, 1], each keeping the half whose lower end has ESS at
// least the target (the midpoint becomes lo when its ESS >= target, else hi),
// and a = lo (hi if lo never moved). The ESS need not be monotone in a, so the
// crossing is the one this sequence of halvings selects.
//
// The halvings are spread over the chip: a pass evaluates, one workgroup per
// point, the ESS at the 2^K - 1 midpoints the next K halvings can visit (the
// same 0.5 (lo + hi) values a one-by-one halving forms, in tree order: node n
// has children 2n and 2n + 1), and the next pass first follows the path
// through them. 60 halvings take 8 passes (7 of 8 levels, then 4); pass 0
// also evaluates ESS(1). The state travels between passes through two
// alternating slots in device memory, so the passes run back to back on the
// stream without the host.
// --------------------------------------------------------------------------

constexpr int kBisectLevels = 60;                   // halvings of (a_prev, 1]
constexpr int kPassLevels = 8;                      // halvings resolved per pass
constexpr int kPassPoints = (1 << kPassLevels) - 1;
constexpr int kSearchPasses = (kBisectLevels + kPassLevels - 1) / kPassLevels;
constexpr int kSearchThreads = 1024;       // workgroup of one search point (one dataset)
constexpr int kSearchThreadsBatch = 256;   // (batches: many more workgroups per pass)

__host__ __device__ inline int pass_levels(int pass) {
  const int left = kBisectLevels - pass * kPassLevels;
  return left < kPassLevels ? left : kPassLevels;
}

// workgroups of a pass: its trial points, and ESS(1) on pass 0
__host__ __device__ inline int pass_groups(int pass) { return (1 << pass_levels(pass)) - 1 + (pass == 0 ? 1 : 0); }

struct SearchSlot {
  double lo, hi;                 // the bracket the pass split
  double ess[kPassPoints + 1];   // ESS at its trial points in tree order; [kPassPoints]: ESS(1)
  int levels;                    // halvings of the pass
  int done;                      // ESS(1) met the target
};

// The trial point of node n (1-based, tree order) over [lo, hi]: the
// midpoints along the path from the root, each formed as 0.5 (lo + hi).
__device__ __forceinline__ double tree_point(double lo, double hi, int n) {
  int top = 31 - __clz(n);
  for (int b = top - 1; b >= 0; --b) {
    const double mid = 0.5 * (lo + hi);
    if ((n >> b) & 1) lo = mid;
    else hi = mid;
  }
  return 0.5 * (lo + hi);
}

// Follow `levels` halvings through the ESS values of a pass.
__device__ __forceinline__ void search_descend(const double* ess, int levels, double target, double& lo,
                                               double& hi) {
  int n = 1;
  for (int k = 0; k < levels; ++k) {
    const double mid = 0.5 * (lo + hi);
    const bool up = ess[n - 1] >= target;
    if (up) lo = mid;
    else hi = mid;
    n = 2 * n + (up ? 1 : 0);
  }
}

// ESS(a) = (sum w)^2 / sum w^2 over the M particles, w_i = exp(x_i - max x),
// x_i = log W_i + nu_i(a); 0 when every x_i is -inf. One workgroup of
// NT threads, sums in a fixed order.
template <int NT>
__device__ __forceinline__ double ess_block(const TemperArgs& A, double a, double* sh) {
  const int t = threadIdx.x, w = t / kWave, l = t % kWave;
  constexpr int NW = NT / kWave;
  double mx = -INFINITY;
  for (int i = t; i < A.M; i += NT)
    mx = fmax(mx, A.logw[i] + incr_weight(a, A.a_prev, A.lhat[i], A.sig2[i]));
  mx = xl::wave_allmax(mx);
  if (l == 0) sh[w] = mx;
  __syncthreads();
  mx = sh[0];
#pragma unroll
  for (int q = 1; q < NW; ++q) mx = fmax(mx, sh[q]);
  if (!isfinite(mx)) return 0.0;
  double s1 = 0.0, s2 = 0.0;
  for (int i = t; i < A.M; i += NT) {
    const double e = exp(A.logw[i] + incr_weight(a, A.a_prev, A.lhat[i], A.sig2[i]) - mx);
    s1 += e;
    s2 += e * e;
  }
  s1 = xl::wave_allsum(s1);
  s2 = xl::wave_allsum(s2);
  if (l == 0) {
    sh[NW + w] = s1;
    sh[2 * NW + w] = s2;
  }
  __syncthreads();
  double t1 = 0.0, t2 = 0.0;
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    t1 += sh[NW + q];
    t2 += sh[2 * NW + q];
  }
  return t1 * t1 / t2;
}

// Pass `pass`, workgroup j: follow the previous pass's halvings, then the ESS
// at trial point j of this pass (j = 2^K - 1 on pass 0: a = 1).
template <int NT>
__device__ __forceinline__ void search_pass_body(const TemperArgs& A, int pass, int j) {
  __shared__ double sh[3 * (NT / kWave)];
  __shared__ double br[2];
  __shared__ int dn;
  const int t = threadIdx.x;
  const int K = pass_levels(pass);
  const double target = A.ess_frac * (double)A.M;
  SearchSlot* cur = A.search + (pass & 1);
  if (t == 0) {
    double lo = A.a_prev, hi = 1.0;
    int done = 0;
    if (pass > 0) {
      const SearchSlot* prev = A.search + ((pass - 1) & 1);
      lo = prev->lo;
      hi = prev->hi;
      done = pass == 1 ? (prev->ess[kPassPoints] >= target ? 1 : 0) : prev->done;
      if (!done) search_descend(prev->ess, prev->levels, target, lo, hi);
    }
    br[0] = lo;
    br[1] = hi;
    dn = done;
    if (j == 0) {
      cur->lo = lo;
      cur->hi = hi;
      cur->levels = K;
      cur->done = done;
    }
  }
  __syncthreads();
  if (dn) return;
  const int np = (1 << K) - 1;
  const double a = j < np ? tree_point(br[0], br[1], j + 1) : 1.0;
  const double e = ess_block<NT>(A, a, sh);
  if (t == 0) cur->ess[j < np ? j : kPassPoints] = e;
}

// Then the exponent (the search's result, or the paper's grid rule), the
// reweighting, normalisation and the evidence increment
// log sum_i W_i exp(nu_i) (sections 3.3, 3.5; Algorithm 2 step c).
template <int NQ>
__device__ __forceinline__ void temper_run(const TemperArgs& A) {
  __shared__ double sh[4 * kTemperSlice];
  const int t = threadIdx.x;
  double lw[NQ], lh[NQ], s2[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = t + q * kTemperThreads;
    const bool ok = i < A.M;
    lw[q] = ok ? A.logw[i] : -INFINITY;
    lh[q] = ok ? A.lhat[i] : 0.0;
    s2[q] = ok ? A.sig2[i] : 0.0;
  }
  const double target = A.ess_frac * (double)A.M;
  int evals = 0;
  double a = 1.0;
  if (A.grid_ess) {
    // the paper's grid rule: the grid point above a_prev whose ESS is closest
    // to the target, the first on ties
    int best = 0;
    double bestd = INFINITY;
    for (int j = 0; j < A.grid_n; ++j) {
      const double dist = fabs(A.grid_ess[j] - target);
      if (grid_exponent(A.a_prev, j) > A.a_prev && dist < bestd) {
        bestd = dist;
        best = j;
      }
    }
    a = grid_exponent(A.a_prev, best);
    evals = A.grid_n;
  } else {
    const SearchSlot* last = A.search + ((kSearchPasses - 1) & 1);
    evals = 1;
    if (!last->done) {
      double lo = last->lo, hi = last->hi;
      search_descend(last->ess, last->levels, target, lo, hi);
      a = (lo > A.a_prev) ? lo : hi;
      evals += kBisectLevels;
    }
  }
  __syncthreads();
  // reweight, normalise and the evidence increment
  double nw[NQ];
  double mo = -INFINITY, mn = -INFINITY;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = t + q * kTemperThreads;
    nw[q] = i < A.M ? lw[q] + incr_weight(a, A.a_prev, lh[q], s2[q]) : -INFINITY;
    mo = fmax(mo, lw[q]);
    mn = fmax(mn, nw[q]);
  }
  mo = block_max_1(mo, sh, 0);
  mn = block_max_1(mn, sh, 1);
  double so = 0.0, sn = 0.0, sn2 = 0.0;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    so += exp(lw[q] - mo);
    const double e = exp(nw[q] - mn);
    sn += e;
    sn2 += e * e;
  }
  block_sum_2(sn, sn2, sh, 2);
  double dummy = 0.0;
  block_sum_2(so, dummy, sh, 3);
  const double lse_old = mo + log(so);
  const double lse_new = mn + log(sn);
  const bool ok = isfinite(lse_new);
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = t + q * kTemperThreads;
    if (i < A.M && ok) A.logw[i] = nw[q] - lse_new;
  }
  if (t == 0) {
    A.out[0] = a;
    A.out[1] = lse_new - lse_old;
    A.out[2] = sn * sn / sn2;
    A.out[3] = ok ? 0.0 : 1.0;
    A.out[4] = (double)evals;
  }
}

// particles per thread: the smallest power of two that covers M
__device__ __forceinline__ void temper_body(const TemperArgs& A) {
  if (A.M <= kTemperThreads) temper_run<1>(A);
  else if (A.M <= 2 * kTemperThreads) temper_run<2>(A);
  else if (A.M <= 4 * kTemperThreads) temper_run<4>(A);
  else temper_run<kTemperPer>(A);
}

// --------------------------------------------------------------------------
// mass matrix: weighted particle covariance, Cholesky factor and its inverse
// (Algorithm 2 step d). One workgroup; the matrix lives in global scratch.
// --------------------------------------------------------------------------

constexpr int kMomThreads = 256;

struct FactorArgs {
  int d;
  double* S;      // d*d in: symmetric positive definite (jitter may be added in place)
  double* L;      // d*d out: lower Cholesky factor
  double* Linv;   // d*d out: inverse of L (lower)
  double* status; // 1: 0 ok, 1 not positive definite
};

// Cholesky with a jitter ladder (1e-10 * mean diagonal * 10^t, t = 0..9) and
// the inverse factor by column-wise forward substitution.
__device__ void factor_spd(const FactorArgs& F, double* sh) {
  const int d = F.d;
  const int t = threadIdx.x;
  double tr = 0.0;
  for (int r = 0; r < d; ++r) tr += F.S[r * d + r];
  bool ok = false;
  for (int att = 0; att <= 10 && !ok; ++att) {
    if (att > 0) {
      const double jit = 1e-10 * (tr / d) * pow(10.0, (double)(att - 1));
      // restart from S + jit*I: S is kept pristine, jitter accumulates only in L's input copy
      for (int e = t; e < d * d; e += kMomThreads) {
        const int r = e / d, c = e % d;
        F.L[e] = F.S[e] + (r == c ? jit : 0.0);
      }
    } else {
      for (int e = t; e < d * d; e += kMomThreads) F.L[e] = F.S[e];
    }
    __syncthreads();
    // right-looking Cholesky in place on F.L (lower part)
    bool good = true;
    for (int j = 0; j < d; ++j) {
      const double ljj2 = F.L[j * d + j];
      good = good && (ljj2 > 0.0);
      if (!good) break;
      const double ljj = sqrt(ljj2);
      __syncthreads();
      for (int i2 = j + 1 + t; i2 < d; i2 += kMomThreads) F.L[i2 * d + j] /= ljj;
      __syncthreads();
      for (int e = t; e < (d - j - 1) * (d - j - 1); e += kMomThreads) {
        const int r = j + 1 + e / (d - j - 1), c = j + 1 + e % (d - j - 1);
        if (c <= r) F.L[r * d + c] -= F.L[r * d + j] * F.L[c * d + j];
      }
      __syncthreads();
      if (t == 0) F.L[j * d + j] = ljj;
      __syncthreads();
    }
    ok = good;
    __syncthreads();
    if (ok && att > 0) {
      const double jit = 1e-10 * (tr / d) * pow(10.0, (double)(att - 1));
      for (int r = t; r < d; r += kMomThreads) F.S[r * d + r] += jit;
    }
    __syncthreads();
  }
  // zero the strict upper triangle
  for (int e = t; e < d * d; e += kMomThreads) {
    const int r = e / d, c = e % d;
    if (c > r) F.L[e] = 0.0;
  }
  __syncthreads();
  // inverse: column c of L^{-1} solves L x = e_c
  for (int c = t; c < d; c += kMomThreads) {
    for (int r = 0; r < d; ++r) {
      double s = (r == c) ? 1.0 : 0.0;
      if (r < c) { F.Linv[r * d + c] = 0.0; continue; }
      for (int k = c; k < r; ++k) s -= F.L[r * d + k] * F.Linv[k * d + c];
      F.Linv[r * d + c] = s / F.L[r * d + r];
    }
  }
  if (t == 0) F.status[0] = ok ? 0.0 : 1.0;
  (void)sh;
}

// The same factorisation with the factor in LDS (d <= kFactorLdsLMaxD):
// left-looking by columns, L[r][j] = (S[r][j] - sum_{k<j} L[r][k] L[j][k]) /
// L[j][j] with the subtractions in the order of the right-looking update
// above, so the factor is the same; then the inverse by the same column-wise
// forward substitution. Ls is d*d doubles of LDS; Li is d*d doubles of LDS
// (d <= kFactorLdsMaxD) or F.Linv itself (the inverse written in place).
constexpr int kFactorLdsMaxD = 64;    // factor and inverse in LDS
constexpr int kFactorLdsLMaxD = 128;  // the factor in LDS, the inverse in global memory

__device__ void factor_spd_lds(const FactorArgs& F, double* Ls, double* Li) {
  __shared__ int good_flag;
  const int d = F.d;
  const int t = threadIdx.x;
  double tr = 0.0;  // trace, needed once a factorisation has failed
  bool ok = false;
  for (int att = 0; att <= 10 && !ok; ++att) {
    if (att == 1)
      for (int r = 0; r < d; ++r) tr += F.S[r * d + r];
    const double jit = att > 0 ? 1e-10 * (tr / d) * pow(10.0, (double)(att - 1)) : 0.0;
    for (int e = t; e < d * d; e += kMomThreads) {
      const int r = e / d, c = e % d;
      Ls[e] = F.S[e] + (r == c ? jit : 0.0);
    }
    __syncthreads();
    // the columns by wavefront 0 alone (rows t and t + 64 in lane t, d <=
    // 128), so the steps of a column synchronise one wavefront only
    if (t < kWave) {
      bool good = true;
      for (int j = 0; j < d; ++j) {
        double sj0 = 0.0, sj1 = 0.0;
        const int r1 = t + kWave;
        if (t >= j && t < d) {
          sj0 = Ls[t * d + j];
#pragma unroll 8
          for (int k = 0; k < j; ++k) sj0 -= Ls[t * d + k] * Ls[j * d + k];
        }
        if (r1 >= j && r1 < d) {
          sj1 = Ls[r1 * d + j];
#pragma unroll 8
          for (int k = 0; k < j; ++k) sj1 -= Ls[r1 * d + k] * Ls[j * d + k];
        }
        // row j's entries left of the diagonal are final; nobody reads (j, j) now
        if (t == j) Ls[j * d + j] = sj0;
        if (r1 == j) Ls[j * d + j] = sj1;
        wave_lds_sync();
        const double p = Ls[j * d + j];
        good = p > 0.0;
        if (!good) break;  // the same value in every lane
        const double ljj = sqrt(p);
        if (t > j && t < d) Ls[t * d + j] = sj0 / ljj;
        if (r1 > j && r1 < d) Ls[r1 * d + j] = sj1 / ljj;
        wave_lds_sync();
        // (j, j) is read again only after the loop
        if (t == j || r1 == j) Ls[j * d + j] = ljj;
      }
      if (t == 0) good_flag = good ? 1 : 0;
    }
    __syncthreads();
    ok = good_flag != 0;
    if (ok && att > 0) {
      for (int r = t; r < d; r += kMomThreads) F.S[r * d + r] += jit;
    }
    __syncthreads();
  }
  // inverse: column c of L^{-1} solves L x = e_c
  for (int c = t; c < d; c += kMomThreads) {
    for (int r = 0; r < d; ++r) {
      if (r < c) { Li[r * d + c] = 0.0; continue; }
      double s = (r == c) ? 1.0 : 0.0;
#pragma unroll 8
      for (int k = c; k < r; ++k) s -= Ls[r * d + k] * Li[k * d + c];
      Li[r * d + c] = s / Ls[r * d + r];
    }
  }
  __syncthreads();
  for (int e = t; e < d * d; e += kMomThreads) {
    const int r = e / d, c = e % d;
    F.L[e] = c > r ? 0.0 : Ls[e];
    if (Li != F.Linv) F.Linv[e] = Li[e];
  }
  if (t == 0) F.status[0] = ok ? 0.0 : 1.0;
}

// dynamic LDS bytes of factor_kernel for dimension d (host side too)
__host__ __device__ inline size_t factor_lds_bytes(int d) {
  return d <= kFactorLdsMaxD ? (size_t)2 * d * d * 8 : (d <= kFactorLdsLMaxD ? (size_t)d * d * 8 : 0);
}

__global__ void __launch_bounds__(kMomThreads) factor_kernel(FactorArgs F) {
  __shared__ double sh[kMomThreads / kWave];
  extern __shared__ double fl[];  // factor_lds_bytes(d)
  if (F.d <= kFactorLdsMaxD) factor_spd_lds(F, fl, fl + F.d * F.d);
  else if (F.d <= kFactorLdsLMaxD) factor_spd_lds(F, fl, F.Linv);
  else factor_spd(F, sh);
}

// Weighted mean and covariance, accumulated about theta_bar (close to the
// particle mean, so the one-pass second moment does not cancel): block b sums
// W_i (theta_i - theta_bar) and W_i (theta_i - theta_bar)(theta_i - theta_bar)'
// over its particles into partials; the final kernel adds the partials in block
// order, forms mean and covariance and factors the covariance.
constexpr int kMomTile = 128;  // particles per block

struct MomentArgs {
  int M, d;
  const double* theta;
  const double* logw;
  const double* centre;   // d: the shift of the one-pass sums (a point inside the cloud)
  double* partials;       // nblocks * (d + d(d+1)/2)
  int nblocks;
  double* mean;           // d
  FactorArgs F;           // F.S receives the covariance
};

__device__ __forceinline__ void tri_index(int f, int& r, int& c) {
  r = (int)((sqrt(8.0 * f + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= f) ++r;
  while (r * (r + 1) / 2 > f) --r;
  c = f - r * (r + 1) / 2;
}

__device__ __forceinline__ void moments_partial_body(const MomentArgs& A, const int tile) {
  __shared__ double sh[kMomThreads / kWave];
  __shared__ double wt[kMomTile];
  extern __shared__ double xs[];  // kMomTile * d
  const int t = threadIdx.x;
  const int M = A.M, d = A.d;
  // log-sum-exp of all weights (each block redundantly)
  double mx = -INFINITY;
  for (int i = t; i < M; i += kMomThreads) mx = fmax(mx, A.logw[i]);
  mx = block_max<kMomThreads>(mx, sh);
  double s = 0.0;
  for (int i = t; i < M; i += kMomThreads) s += exp(A.logw[i] - mx);
  s = block_sum<kMomThreads>(s, sh);
  const double lse = mx + log(s);
  const int i0 = tile * kMomTile;
  const int cnt = min(kMomTile, M - i0);
  for (int q = t; q < kMomTile; q += kMomThreads) wt[q] = q < cnt ? exp(A.logw[i0 + q] - lse) : 0.0;
  for (int e = t; e < kMomTile * d; e += kMomThreads) {
    const int q = e / d, c = e % d;
    xs[e] = q < cnt ? A.theta[(int64_t)(i0 + q) * d + c] - A.centre[c] : 0.0;
  }
  __syncthreads();
  const int ne = d + d * (d + 1) / 2;
  for (int e = t; e < ne; e += kMomThreads) {
    double acc = 0.0;
    if (e < d) {
      for (int q = 0; q < cnt; ++q) acc += wt[q] * xs[q * d + e];
    } else {
      int r, c;
      tri_index(e - d, r, c);
      for (int q = 0; q < cnt; ++q) acc += wt[q] * xs[q * d + r] * xs[q * d + c];
    }
    A.partials[(int64_t)tile * ne + e] = acc;
  }
}

__device__ __forceinline__ void moments_final_body(const MomentArgs& A) {
  __shared__ double sh[kMomThreads / kWave];
  extern __shared__ double tot[];  // d + d(d+1)/2 (moments_final_lds), then the factor's LDS
  const int t = threadIdx.x;
  const int d = A.d;
  const int ne = d + d * (d + 1) / 2;
  for (int e = t; e < ne; e += kMomThreads) {
    double acc = 0.0;
    for (int b = 0; b < A.nblocks; ++b) acc += A.partials[(int64_t)b * ne + e];
    tot[e] = acc;
  }
  __syncthreads();
  for (int r = t; r < d; r += kMomThreads) A.mean[r] = A.centre[r] + tot[r];
  for (int f = t; f < d * (d + 1) / 2; f += kMomThreads) {
    int r, c;
    tri_index(f, r, c);
    const double v = tot[d + f] - tot[r] * tot[c];
    A.F.S[r * d + c] = v;
    A.F.S[c * d + r] = v;
  }
  __syncthreads();
  if (d <= kFactorLdsMaxD) {
    double* Ls = tot + ne;
    factor_spd_lds(A.F, Ls, Ls + d * d);
  } else if (d <= kFactorLdsLMaxD) {
    // the moments are in A.F.S now: the factor takes their LDS
    factor_spd_lds(A.F, tot, A.F.Linv);
  } else {
    factor_spd(A.F, sh);
  }
}

// --------------------------------------------------------------------------
// systematic resampling in exact integer arithmetic
// --------------------------------------------------------------------------

constexpr int kResThreads = 1024;
constexpr int kResPer = 8;  // M <= 8192

struct ResampleArgs {
  int M;
  int multinomial;  // 0: systematic, 1: multinomial
  uint64_t seed;
  uint32_t stage, dataset;
  const double* logw;
  int32_t* anc;
};

// floor(X / M) for X = hi:lo (X < 2^72 after the 2^32 split), M < 2^31
__device__ __forceinline__ uint64_t div_u96_by_u32(uint64_t hi32, uint64_t lo64, uint32_t M) {
  // X = hi32 * 2^64 + lo64 with hi32 < 2^32
  uint64_t r = 0, q2, q1, q0;
  uint64_t cur = hi32;
  q2 = cur / M; r = cur % M;
  cur = (r << 32) | (lo64 >> 32);
  q1 = cur / M; r = cur % M;
  cur = (r << 32) | (lo64 & 0xffffffffull);
  q0 = cur / M;
  (void)q2;  // zero by construction (quotient < 2^64)
  return (q1 << 32) + q0;
}

__device__ __forceinline__ void resample_body(const ResampleArgs& A) {
  __shared__ double sh[kResThreads / kWave];
  __shared__ unsigned long long cum[kResThreads * kResPer];
  __shared__ unsigned long long wsum[kResThreads / kWave];
  const int t = threadIdx.x;
  const int M = A.M;
  double mx = -INFINITY;
  for (int i = t; i < M; i += kResThreads) mx = fmax(mx, A.logw[i]);
  mx = block_max<kResThreads>(mx, sh);
  // each thread owns a contiguous run of kResPer particles
  unsigned long long c[kResPer];
  unsigned long long run = 0;
#pragma unroll
  for (int q = 0; q < kResPer; ++q) {
    const int i = t * kResPer + q;
    unsigned long long ci = 0;
    if (i < M) {
      const double w = exp(A.logw[i] - mx);
      ci = (unsigned long long)floor(ldexp(w, 48));
    }
    run += ci;
    c[q] = run;
  }
  // exclusive scan of per-thread totals: wave scan then across waves
  const int l = t % kWave, w = t / kWave;
  unsigned long long incl = run;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const unsigned long long y = __shfl_up(incl, o, kWave);
    if (l >= o) incl += y;
  }
  if (l == kWave - 1) wsum[w] = incl;
  __syncthreads();
  unsigned long long base = 0;
  for (int k = 0; k < w; ++k) base += wsum[k];
  const unsigned long long excl = base + incl - run;
#pragma unroll
  for (int q = 0; q < kResPer; ++q) cum[t * kResPer + q] = excl + c[q];
  __syncthreads();
  const unsigned long long S = cum[M - 1];
  const uint64_t c0 = stream_ctr0(kResampleOffset, A.stage, 0, A.dataset);
  const uint32_t U32 = (uint32_t)(stream_word(A.seed, c0, 0, 0) >> 32);
  for (int k = t; k < M; k += kResThreads) {
    uint64_t tk;
    if (A.multinomial) {
      // slot k's own uniform word (particle k, draw 1): t_k = floor(r_k S / 2^64)
      tk = __umul64hi(stream_word(A.seed, c0, (uint64_t)k, 1), (uint64_t)S);
    } else {
      // t_k = floor((k 2^32 + U32) S / (M 2^32)) = floor(floor(P / 2^32) / M)
      const uint64_t a = ((uint64_t)k << 32) + U32;
      const uint64_t plo = a * (uint64_t)S, phi = __umul64hi(a, (uint64_t)S);
      const uint64_t shi = phi >> 32;
      const uint64_t slo = (phi << 32) | (plo >> 32);
      tk = div_u96_by_u32(shi, slo, (uint32_t)M);
    }
    // smallest j with cum[j] > tk
    int lo = 0, hi = M - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (cum[mid] > tk) hi = mid;
      else lo = mid + 1;
    }
    A.anc[k] = lo;
  }
}

struct GatherArgs {
  int M, d, m;
  const int32_t* anc;
  const double* theta; const int32_t* u; const double* lhat; const double* sig2;
  const double* gl; const double* gs;
  double* theta2; int32_t* u2; double* lhat2; double* sig22; double* gl2; double* gs2;
};

// dst row k <- src row anc[k]; one workgroup per row k, the u row copied with 16-byte moves
__device__ __forceinline__ void gather_body(const GatherArgs& A, const int k) {
  const int t = threadIdx.x;
  const int s = A.anc[k];
  const int d = A.d, m = A.m;
  for (int c = t; c < d; c += 256) {
    A.theta2[(int64_t)k * d + c] = A.theta[(int64_t)s * d + c];
    A.gl2[(int64_t)k * d + c] = A.gl[(int64_t)s * d + c];
    A.gs2[(int64_t)k * d + c] = A.gs[(int64_t)s * d + c];
  }
  if (t == 0) {
    A.lhat2[k] = A.lhat[s];
    A.sig22[k] = A.sig2[s];
  }
  const int32_t* src = A.u + (int64_t)s * m;
  int32_t* dst = A.u2 + (int64_t)k * m;
  if ((m & 3) == 0) {
    const int4* s4 = reinterpret_cast<const int4*>(src);
    int4* d4 = reinterpret_cast<int4*>(dst);
    for (int j = t; j < m / 4; j += 256) d4[j] = s4[j];
  } else {
    for (int j = t; j < m; j += 256) dst[j] = src[j];
  }
}

struct CopyBackArgs {
  int M, d, m;
  const double* theta2; const int32_t* u2; const double* lhat2; const double* sig22;
  const double* gl2; const double* gs2;
  double* theta; int32_t* u; double* lhat; double* sig2; double* gl; double* gs; double* logw;
};

__device__ __forceinline__ void copyback_body(const CopyBackArgs& A, const int k) {
  const int t = threadIdx.x;
  const int d = A.d, m = A.m;
  for (int c = t; c < d; c += 256) {
    A.theta[(int64_t)k * d + c] = A.theta2[(int64_t)k * d + c];
    A.gl[(int64_t)k * d + c] = A.gl2[(int64_t)k * d + c];
    A.gs[(int64_t)k * d + c] = A.gs2[(int64_t)k * d + c];
  }
  if (t == 0) {
    A.lhat[k] = A.lhat2[k];
    A.sig2[k] = A.sig22[k];
    A.logw[k] = -log((double)A.M);
  }
  const int32_t* src = A.u2 + (int64_t)k * m;
  int32_t* dst = A.u + (int64_t)k * m;
  if ((m & 3) == 0) {
    const int4* s4 = reinterpret_cast<const int4*>(src);
    int4* d4 = reinterpret_cast<int4*>(dst);
    for (int j = t; j < m / 4; j += 256) d4[j] = s4[j];
  } else {
    for (int j = t; j < m; j += 256) dst[j] = src[j];
  }
}

// --------------------------------------------------------------------------
// full-data control-variate summaries A, B, C at theta (section 3.2) and the
// packed rows; FP64 throughout. A block takes tiles of up to 256 rows: in
// phase 1 one thread per row forms eta, l_k, l_k', l_k'' and writes the packed
// row, keeping x and the derivatives in LDS; in phase 2 each thread sums its
// entries of [A, B, C upper triangle] over the tile (the row being read is the
// same for every thread, so LDS reads broadcast). Per-block partials are then
// summed by a reduction with one workgroup per entry, in fixed order. The
// eta-free part of A (sum of log y!) is summed once by cv_const_kernel.
// --------------------------------------------------------------------------

constexpr int kCvThreads = 256;
constexpr int kCvMaxD = 128;

struct CvArgs {
  int family, d, ld_in, ld_out, in_fp32, out_fp32;
  int tile_rows;        // rows per tile (<= kCvThreads)
  int64_t n;
  double inv_s2, log2pis2;
  const void* Xin;      // caller rows [x (d) | y | ...], pitch ld_in
  const double* theta;  // d
  void* Xout;           // packed rows or nullptr
  double* partials;     // gridDim.x * (1 + d + d(d+1)/2)
};

// LDS of cv_kernel: theta (d, padded to even), the per-thread accumulators
// (ceil(ne / 256) * 256) and a tile of `rows` rows of (l, l', l'', x)
__host__ __device__ inline int cv_acc_per(int d) { return (1 + d + d * (d + 1) / 2 + kCvThreads - 1) / kCvThreads; }
__host__ __device__ inline size_t cv_lds_bytes(int d, int rows) {
  return (size_t)(((d + 1) & ~1) + cv_acc_per(d) * kCvThreads + rows * (d + 3)) * sizeof(double);
}

// entry f of the upper triangle (row-major over r >= c) -> (r, c)
__device__ __forceinline__ void tri_entry(int f, int& r, int& c) {
  r = (int)((sqrt(8.0 * f + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= f) ++r;
  while (r * (r + 1) / 2 > f) --r;
  c = f - r * (r + 1) / 2;
}

__global__ void __launch_bounds__(kCvThreads) cv_kernel(CvArgs A) {
  extern __shared__ double cvsm[];
  const int t = threadIdx.x;
  const int d = A.d;
  const int stride = d + 3;
  const int ne = 1 + d + d * (d + 1) / 2;
  const int per = cv_acc_per(d);
  double* th = cvsm;
  double* acc = cvsm + ((d + 1) & ~1);    // entry t + q*256 at acc[q*256 + t]
  double* tile = acc + per * kCvThreads;
  for (int c = t; c < d; c += kCvThreads) th[c] = A.theta[c];
  for (int q = 0; q < per; ++q) acc[q * kCvThreads + t] = 0.0;
  __syncthreads();
  const int TR = A.tile_rows;
  const int64_t ntiles = (A.n + TR - 1) / TR;
  for (int64_t tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
    const int64_t r0 = tl * TR;
    const int rows = (int)((A.n - r0) < TR ? (A.n - r0) : TR);
    if (t < rows) {
      const int64_t k = r0 + t;
      double* trow = tile + t * stride;
      double eta = 0.0, y;
      if (A.in_fp32) {
        const float* row = static_cast<const float*>(A.Xin) + k * A.ld_in;
        for (int c = 0; c < d; ++c) { const double x = row[c]; trow[3 + c] = x; eta += x * th[c]; }
        y = row[d];
      } else {
        const double* row = static_cast<const double*>(A.Xin) + k * A.ld_in;
        for (int c = 0; c < d; ++c) { const double x = row[c]; trow[3 + c] = x; eta += x * th[c]; }
        y = row[d];
      }
      double f0, f1, f2;
      loglik_derivs(A.family, y, eta, A.inv_s2, f0, f1, f2);
      trow[0] = f0; trow[1] = f1; trow[2] = f2;
      if (A.Xout) {
        double aux = 0.0;
        if (A.family == kLogistic) aux = sigmoid<double>(-fabs(eta));
        else if (A.family == kPoisson) aux = exp(eta);
        else if (A.family == kStudentT) aux = y - eta;
        if (A.out_fp32) {
          float* o = static_cast<float*>(A.Xout) + k * A.ld_out;
          o[0] = (float)eta; o[1] = (float)aux; o[2] = (float)y; o[3] = 0.f;
          for (int c = 0; c < d; ++c) o[kHeader + c] = (float)trow[3 + c];
          for (int c = kHeader + d; c < A.ld_out; ++c) o[c] = 0.f;
        } else {
          double* o = static_cast<double*>(A.Xout) + k * A.ld_out;
          o[0] = eta; o[1] = aux; o[2] = y; o[3] = 0.0;
          for (int c = 0; c < d; ++c) o[kHeader + c] = trow[3 + c];
          for (int c = kHeader + d; c < A.ld_out; ++c) o[c] = 0.0;
        }
      }
    }
    __syncthreads();
#pragma unroll 1
    for (int q = 0; q < per; ++q) {
      const int e = t + q * kCvThreads;
      if (e >= ne) break;
      double s = 0.0;
      if (e == 0) {
        for (int rr = 0; rr < rows; ++rr) s += tile[rr * stride];
      } else if (e <= d) {
        const int ib = 3 + (e - 1);
        for (int rr = 0; rr < rows; ++rr) s += tile[rr * stride + 1] * tile[rr * stride + ib];
      } else {
        int r, c;
        tri_entry(e - 1 - d, r, c);
        const int ia = 3 + r, ib = 3 + c;
        for (int rr = 0; rr < rows; ++rr) {
          const double* tr = tile + rr * stride;
          s += tr[2] * tr[ia] * tr[ib];
        }
      }
      acc[q * kCvThreads + t] += s;
    }
    __syncthreads();
  }
  for (int q = 0; q < per; ++q) {
    const int e = t + q * kCvThreads;
    if (e < ne) A.partials[(int64_t)blockIdx.x * ne + e] = acc[q * kCvThreads + t];
  }
}

// Sum over all rows of the eta-free part of l_k (per-block partials).
struct CvConstArgs {
  int family, ld_in, in_fp32, d;
  int64_t n;
  double log2pis2;
  const void* Xin;
  double* partials;  // gridDim.x
};

__global__ void __launch_bounds__(kCvThreads) cv_const_kernel(CvConstArgs A) {
  __shared__ double sh[kCvThreads / kWave];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * kCvThreads + t; k < A.n; k += (int64_t)gridDim.x * kCvThreads) {
    const double y = A.in_fp32 ? (double)static_cast<const float*>(A.Xin)[k * A.ld_in + A.d]
                               : static_cast<const double*>(A.Xin)[k * A.ld_in + A.d];
    s += loglik_const(A.family, y, A.log2pis2);
  }
  s = wave_sum(s);
  if (t % kWave == 0) sh[t / kWave] = s;
  __syncthreads();
  if (t == 0) {
    double tot = 0.0;
    for (int q = 0; q < kCvThreads / kWave; ++q) tot += sh[q];
    A.partials[blockIdx.x] = tot;
  }
}

struct CvReduceArgs {
  int nblocks, d;
  const double* partials;
  const double* aconst;  // 1: added to A
  double* A;  // 1
  double* B;  // d
  double* C;  // d*d
};

// One workgroup per entry e: the nblocks partials of e in fixed order (strided
// per thread, then the wavefront butterflies and the 4 wavefronts in order).
__global__ void __launch_bounds__(256) cv_reduce_kernel(CvReduceArgs R) {
  __shared__ double sh[4];
  const int d = R.d;
  const int ne = 1 + d + d * (d + 1) / 2;
  const int e = blockIdx.x;
  const int t = threadIdx.x;
  double s = 0.0;
  for (int b = t; b < R.nblocks; b += 256) s += R.partials[(int64_t)b * ne + e];
  s = wave_sum(s);
  if (t % kWave == 0) sh[t / kWave] = s;
  __syncthreads();
  if (t != 0 || e >= ne) return;
  s = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  if (e == 0) {
    R.A[0] = s + (R.aconst ? R.aconst[0] : 0.0);
  } else if (e <= d) {
    R.B[e - 1] = s;
  } else {
    int r, c;
    tri_entry(e - 1 - d, r, c);
    R.C[r * d + c] = s;
    R.C[c * d + r] = s;
  }
}

// sum of the const-kernel partials into one value
__global__ void __launch_bounds__(256) cv_const_reduce_kernel(const double* partials, int nblocks, double* out) {
  __shared__ double sh[4];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int b = t; b < nblocks; b += 256) s += partials[b];
  s = wave_sum(s);
  if (t % kWave == 0) sh[t / kWave] = s;
  __syncthreads();
  if (t == 0) out[0] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// --------------------------------------------------------------------------
// Entry points: one dataset per launch, and the batched forms.
// --------------------------------------------------------------------------

__global__ void __launch_bounds__(kSearchThreads) search_pass_kernel(TemperArgs A, int pass) {
  search_pass_body<kSearchThreads>(A, pass, blockIdx.x);
}

// members own pass_groups(pass) consecutive workgroups each
__global__ void __launch_bounds__(kSearchThreadsBatch) search_pass_kernel_batch(Batch<TemperArgs> B, int pass) {
  const int per = pass_groups(pass);
  const int k = blockIdx.x / per;
  const TemperArgs A = B.args[k];
  search_pass_body<kSearchThreadsBatch>(A, pass, blockIdx.x - k * per);
}

__global__ void __launch_bounds__(kTemperThreads) temper_kernel(TemperArgs A) { temper_body(A); }

__global__ void __launch_bounds__(kTemperThreads) temper_kernel_batch(Batch<TemperArgs> B) {
  const TemperArgs A = B.args[blockIdx.x];
  temper_body(A);
}

__global__ void __launch_bounds__(kMomThreads) moments_partial_kernel(MomentArgs A) {
  moments_partial_body(A, blockIdx.x);
}

__global__ void __launch_bounds__(kMomThreads) moments_partial_kernel_batch(Batch<MomentArgs> B) {
  const int k = batch_member(B.first, B.count, blockIdx.x);
  const MomentArgs A = B.args[k];
  moments_partial_body(A, blockIdx.x - B.first[k]);
}

__global__ void __launch_bounds__(kMomThreads) moments_final_kernel(MomentArgs A) { moments_final_body(A); }

__global__ void __launch_bounds__(kMomThreads) moments_final_kernel_batch(Batch<MomentArgs> B) {
  const MomentArgs A = B.args[blockIdx.x];
  moments_final_body(A);
}

__global__ void __launch_bounds__(kResThreads) resample_kernel(ResampleArgs A) { resample_body(A); }

__global__ void __launch_bounds__(kResThreads) resample_kernel_batch(Batch<ResampleArgs> B) {
  const ResampleArgs A = B.args[blockIdx.x];
  resample_body(A);
}

__global__ void __launch_bounds__(256) gather_kernel(GatherArgs A) { gather_body(A, blockIdx.x); }

__global__ void __launch_bounds__(256) gather_kernel_batch(Batch<GatherArgs> B) {
  const int k = batch_member(B.first, B.count, blockIdx.x);
  const GatherArgs A = B.args[k];
  gather_body(A, blockIdx.x - B.first[k]);
}

__global__ void __launch_bounds__(256) copyback_kernel(CopyBackArgs A) { copyback_body(A, blockIdx.x); }

__global__ void __launch_bounds__(256) copyback_kernel_batch(Batch<CopyBackArgs> B) {
  const int k = batch_member(B.first, B.count, blockIdx.x);
  const CopyBackArgs A = B.args[k];
  copyback_body(A, blockIdx.x - B.first[k]);
}

}  // namespace subsmc
