// Device kernels of the Subsampling SMC hot path (gfx950, wave64).
//
// Particle work maps one wavefront to one particle: the wave owns the
// particle's theta, momentum and caches (component c in lane c, d <= 64) and
// streams its m subsample rows, 64 rows at a time, one row per lane. Every
// reduction is a fixed-order butterfly across the 64 lanes (all lanes end
// with bitwise-identical sums), so decisions are wave-uniform and runs are
// bitwise reproducible.
//
// Packed data row (Real = double for the FP64 path, float for mixed):
//   [eta_bar, aux, y, 0, x_0 .. x_{d-1}, 0 ...], pitch ld (a multiple of 64 B)
// with eta_bar = x' theta_bar and aux = sigmoid(-|eta_bar|) (logistic),
// exp(eta_bar) (Poisson) or y - eta_bar (Student-t), all computed in FP64
// whenever the control-variate centre is set.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "glm.hpp"
#include "rng.hpp"
#include "xlane.hpp"

namespace subsmc {

constexpr int kWave = 64;
constexpr int kHeader = 4;  // eta_bar, aux, y, pad

// --------------------------------------------------------------------------
// wave-level helpers
// --------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) { return xl::wave_allsum(v); }

__device__ __forceinline__ double readlane_d(double v, int l) {
  const unsigned long long b = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)(b & 0xffffffffu), l);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), l);
  return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}

template <int DC>
__device__ __forceinline__ double pick_lane(const double (&a)[DC], int lane) {
  double r = 0.0;
#pragma unroll
  for (int c = 0; c < DC; ++c) r = (lane == c) ? a[c] : r;
  return r;
}

// --------------------------------------------------------------------------
// problem description handed to kernels
// --------------------------------------------------------------------------

struct Prob {
  int family, cv_order, d, ld;
  int64_t n;
  int M, m, G;
  uint64_t seed;
  double inv_s2, log2pis2;
  double n_over_m;
  const void* X;            // packed rows
  const double* theta_bar;  // d
  const double* cvA;        // 1
  const double* cvB;        // d
  const double* cvC;        // d*d
  const double* mu0;        // d
  const double* Q0;         // d*d
  const double* Sigma;      // d*d
  const double* Linv;       // d*d, inverse of the lower Cholesky factor of Sigma
};

template <typename Real, int DC>
struct RowLoad {
  Real eb, aux;
  Real x[DC];
};

template <typename Real, int DC>
__device__ __forceinline__ void load_row(const Real* __restrict__ row, RowLoad<Real, DC>& r) {
  if constexpr (sizeof(Real) == 4) {
    const float2 h = *reinterpret_cast<const float2*>(row);
    r.eb = h.x;
    r.aux = h.y;
    const float4* xv = reinterpret_cast<const float4*>(row + kHeader);
#pragma unroll
    for (int q = 0; q < DC / 4; ++q) {
      const float4 t = xv[q];
      r.x[4 * q + 0] = t.x; r.x[4 * q + 1] = t.y; r.x[4 * q + 2] = t.z; r.x[4 * q + 3] = t.w;
    }
  } else {
    const double2 h = *reinterpret_cast<const double2*>(row);
    r.eb = h.x;
    r.aux = h.y;
    const double2* xv = reinterpret_cast<const double2*>(row + kHeader);
#pragma unroll
    for (int q = 0; q < DC / 2; ++q) {
      const double2 t = xv[q];
      r.x[2 * q + 0] = t.x; r.x[2 * q + 1] = t.y;
    }
  }
}

// Result of one estimator pass for one particle (wave-uniform scalars; the
// gradient components live in lane c).
struct PassResult {
  double lhat, sig2, dhat;
  double gl, gs;  // lane c: component c of grad l_hat and grad sigma2_hat
};

// Sum over the 64 lanes of v[c], returned in lane c (0 elsewhere), through
// 64*DC elements of LDS; the adds run in FP64 in lane order.
template <typename Real, int DC>
__device__ __forceinline__ double lds_column_sum(const Real (&v)[DC], Real* red, int lane) {
  __syncthreads();
#pragma unroll
  for (int c = 0; c < DC; ++c) red[lane * DC + c] = v[c];
  __syncthreads();
  double s = 0.0;
  if (lane < DC) {
    for (int r = 0; r < kWave; ++r) s += (double)red[r * DC + lane];
  }
  return s;
}

// One pass of the difference estimator (eq. difference_estimator_logl), its
// variance estimate (section 3.2) and both gradients at theta = theta_bar + delta,
// for the subsample urow; slots [b0, b1) take their indices from `blk` (the
// freshly drawn block of a pseudo-marginal refresh, staged in LDS).
//   l_hat   = A + B'delta + delta'C delta/2 + (n/m) sum_j d_j
//   s2_hat  = (n/m)^2 sum_j (d_j - dbar)^2
//   grad l  = B + C delta + (n/m) sum_j d'_j x_j
//   grad s2 = 2 (n/m)^2 sum_j (d_j - dbar) d'_j x_j
// The d_j sums are taken about the shift d_{u_0} (evaluated first by every
// lane) to keep the single-pass variance accurate. Each lane streams slots
// lane, lane+64, ...; the next row and the index after it are loaded before
// the current row is used, so two gathers per lane are in flight.
// A caller index outside [0, n) is never dereferenced: it poisons the pass
// with NaN.
template <typename Real, int DC, int FAM, bool BLK>
__device__ __forceinline__ PassResult estimator_pass(const Prob& P, const int32_t* __restrict__ urow,
                                                     int b0, int b1, const int32_t* blk, Real* red,
                                                     double delta64, int lane) {
  const Real* __restrict__ X = static_cast<const Real*>(P.X);
  const int m = P.m;
  const int ld = P.ld;
  const uint32_t n = (uint32_t)P.n;
  const Real inv_s2 = (Real)P.inv_s2;
  // both sources are read unconditionally and the value selected, so the
  // LDS and global accesses keep their own address spaces
  auto index_of = [&](int j) -> int32_t {
    const int32_t g = urow[j];
    if constexpr (BLK) {
      const bool in = (unsigned)(j - b0) < (unsigned)(b1 - b0);
      const int32_t l = blk[in ? j - b0 : 0];
      return in ? l : g;
    } else {
      return g;
    }
  };

  Real dl[DC];
#pragma unroll
  for (int c = 0; c < DC; ++c) dl[c] = (Real)readlane_d(delta64, c);

  // shift: the remainder at slot 0, evaluated redundantly by every lane
  double shift;
  {
    const int32_t k0 = index_of(0);
    const bool bad = (uint32_t)k0 >= n;
    RowLoad<Real, DC> r;
    load_row<Real, DC>(X + (int64_t)(bad ? 0 : k0) * ld, r);
    Real D = Real(0);
#pragma unroll
    for (int c = 0; c < DC; ++c) D += r.x[c] * dl[c];
    Real dd, dp;
    cv_remainder<Real, FAM>(P.cv_order, r.eb, r.aux, D, inv_s2, dd, dp);
    shift = bad ? __builtin_nan("") : (double)dd;
  }

  double se = 0.0, se2 = 0.0;
  Real S1[DC], T1[DC];
#pragma unroll
  for (int c = 0; c < DC; ++c) { S1[c] = Real(0); T1[c] = Real(0); }

  // rows are prefetched one iteration ahead (measured: for FP64 d = 20 one
  // resident wave with the prefetch beats two without it)
  constexpr bool kPrefetchRow = true;
  int j = lane;
  int32_t k_cur = j < m ? index_of(j) : 0;
  int32_t k_nxt = j + kWave < m ? index_of(j + kWave) : 0;
  RowLoad<Real, DC> r_nxt;
  if constexpr (kPrefetchRow) {
    if (j < m) load_row<Real, DC>(X + (int64_t)((uint32_t)k_cur < n ? k_cur : 0) * ld, r_nxt);
  }
  for (; j < m; j += kWave) {
    RowLoad<Real, DC> r;
    const bool bad = (uint32_t)k_cur >= n;
    if constexpr (kPrefetchRow) {
      r = r_nxt;
      if (j + kWave < m) load_row<Real, DC>(X + (int64_t)((uint32_t)k_nxt < n ? k_nxt : 0) * ld, r_nxt);
    } else {
      load_row<Real, DC>(X + (int64_t)(bad ? 0 : k_cur) * ld, r);
    }
    k_cur = k_nxt;
    k_nxt = j + 2 * kWave < m ? index_of(j + 2 * kWave) : 0;

    Real D = Real(0);
#pragma unroll
    for (int c = 0; c < DC; ++c) D += r.x[c] * dl[c];
    Real dd, dp;
    cv_remainder<Real, FAM>(P.cv_order, r.eb, r.aux, D, inv_s2, dd, dp);
    if (bad) dd = dp = Real(__builtin_nan(""));
    const double e = (double)dd - shift;
    se += e;
    se2 += e * e;
    const Real edp = (Real)e * dp;
#pragma unroll
    for (int c = 0; c < DC; ++c) {
      S1[c] += dp * r.x[c];
      T1[c] += edp * r.x[c];
    }
  }

  // fixed-order reductions: scalars by butterfly; the vectors S1, T1 by an LDS
  // transpose (lane c adds column c over lanes 0..63 in FP64)
  se = wave_sum(se);
  se2 = wave_sum(se2);
  const double s1c = lds_column_sum<Real, DC>(S1, red, lane);
  const double t1c = lds_column_sum<Real, DC>(T1, red, lane);

  const double md = (double)m;
  const double nm = P.n_over_m;
  const double dsum = se + md * shift;
  const double dbar_minus_shift = se / md;
  const double m2 = se2 - se * dbar_minus_shift;  // sum (d - dbar)^2
  PassResult out;
  out.dhat = nm * dsum;
  out.sig2 = nm * nm * (m2 < 0.0 ? 0.0 : m2);  // NaN propagates

  // control-variate quadratic and its gradient, FP64
  const int d = P.d;
  double cdel = 0.0;
  for (int e = 0; e < d; ++e) {
    const double de = readlane_d(delta64, e);
    cdel += (lane < d ? P.cvC[lane * d + e] : 0.0) * de;
  }
  const double bl = lane < d ? P.cvB[lane] : 0.0;
  const double qpart = (P.cv_order == 2) ? (bl * delta64 + 0.5 * delta64 * cdel) : bl * delta64;
  const double qsum = wave_sum(qpart);
  out.lhat = P.cvA[0] + qsum + out.dhat;
  out.gl = lane < d ? bl + (P.cv_order == 2 ? cdel : 0.0) + nm * s1c : 0.0;
  out.gs = lane < d ? 2.0 * nm * nm * (t1c - dbar_minus_shift * s1c) : 0.0;
  return out;
}

// --------------------------------------------------------------------------
// estimator kernels (loglik_est / loglik_grad / cache refresh)
// --------------------------------------------------------------------------

struct EstArgs {
  Prob P;
  int count;
  const double* theta;   // count*d
  const int32_t* u;      // count*m
  double* lhat;          // count (nullable)
  double* sig2;          // count (nullable)
  double* dhat;          // count (nullable)
  double* grad_l;        // count*d (nullable)
  double* grad_s;        // count*d (nullable)
  const double* g_lhat;  // count (nullable): combined gradient g_l * grad l + g_s * grad s2
  const double* g_sig2;  // count (nullable)
  double* grad;          // count*d (nullable)
};

template <typename Real, int DC, int FAM>
__global__ void __launch_bounds__(kWave) estimator_kernel(EstArgs A) {
  __shared__ Real red[kWave * DC];
  const int i = blockIdx.x;
  const int lane = threadIdx.x;
  if (i >= A.count) return;
  const Prob& P = A.P;
  const int d = P.d;
  const double th = lane < d ? A.theta[(int64_t)i * d + lane] : 0.0;
  const double tb = lane < d ? P.theta_bar[lane] : 0.0;
  const PassResult r = estimator_pass<Real, DC, FAM, false>(P, A.u + (int64_t)i * P.m, 0, 0, nullptr, red, th - tb, lane);
  if (lane == 0) {
    if (A.lhat) A.lhat[i] = r.lhat;
    if (A.sig2) A.sig2[i] = r.sig2;
    if (A.dhat) A.dhat[i] = r.dhat;
  }
  if (lane < d) {
    if (A.grad_l) A.grad_l[(int64_t)i * d + lane] = r.gl;
    if (A.grad_s) A.grad_s[(int64_t)i * d + lane] = r.gs;
    if (A.grad) {
      const double gl = A.g_lhat ? A.g_lhat[i] : 0.0;
      const double gs = A.g_sig2 ? A.g_sig2[i] : 0.0;
      A.grad[(int64_t)i * d + lane] = gl * r.gl + gs * r.gs;
    }
  }
}

// --------------------------------------------------------------------------
// fused Markov move (Algorithm 1): block pseudo-marginal refresh of u, then
// HMC on theta given u with inverse mass matrix Sigma; R = 1 per launch.
// Dynamic LDS: ceil(m/G) int32 for the refreshed block's indices.
// --------------------------------------------------------------------------

struct MoveArgs {
  Prob P;
  double a, eps;
  int L;
  uint32_t stage, move;
  double* theta;   // M*d
  int32_t* u;      // M*m
  double* lhat;    // M   cache at the current state
  double* sig2;    // M
  double* grad_l;  // M*d
  double* grad_s;  // M*d
  int32_t* accept; // M*2
};

template <int DC>
__device__ __forceinline__ void prior_terms(const Prob& P, double th, int lane, double& r, double& lp) {
  // r = (Q0 (theta - mu0))_lane, lp = -(theta-mu0)' Q0 (theta-mu0) / 2
  const int d = P.d;
  const double dm = lane < d ? th - P.mu0[lane] : 0.0;
  double acc = 0.0;
  for (int e = 0; e < d; ++e) {
    const double x = readlane_d(dm, e);
    acc += (lane < d ? P.Q0[lane * d + e] : 0.0) * x;
  }
  r = acc;
  lp = wave_sum(-0.5 * dm * acc);
}

__device__ __forceinline__ double sigma_times(const Prob& P, double p, int lane) {
  const int d = P.d;
  double acc = 0.0;
  for (int e = 0; e < d; ++e) {
    const double x = readlane_d(p, e);
    acc += (lane < d ? P.Sigma[lane * d + e] : 0.0) * x;
  }
  return acc;
}

template <typename Real, int DC, int FAM>
__global__ void __launch_bounds__(kWave) move_kernel(MoveArgs A) {
  __shared__ Real red[kWave * DC];
  extern __shared__ int32_t blk[];
  const int i = blockIdx.x;
  const int lane = threadIdx.x;
  const Prob& P = A.P;
  if (i >= P.M) return;
  const int d = P.d;
  const int m = P.m;
  const double a = A.a;
  const double eps = A.eps;
  int32_t* urow = A.u + (int64_t)i * m;

  const double tb = lane < d ? P.theta_bar[lane] : 0.0;
  double th = lane < d ? A.theta[(int64_t)i * d + lane] : 0.0;
  double lh0 = A.lhat[i], sg0 = A.sig2[i];
  double gl0 = lane < d ? A.grad_l[(int64_t)i * d + lane] : 0.0;
  double gs0 = lane < d ? A.grad_s[(int64_t)i * d + lane] : 0.0;

  // ---- 1. u | theta: one block, chosen uniformly, replaced by fresh indices
  const uint64_t cg = stream_ctr0(kBlockChoice, A.stage, A.move, 0);
  const int g = (int)word_to_index(stream_word(P.seed, cg, (uint64_t)i, 0), (uint64_t)P.G);
  const int b0 = (int)((int64_t)g * m / P.G);
  const int b1 = (int)((int64_t)(g + 1) * m / P.G);
  const uint64_t cb = stream_ctr0(kBlockIndex, A.stage, A.move, 0);
  for (int t = lane; t < b1 - b0; t += kWave)
    blk[t] = (int32_t)word_to_index(stream_word(P.seed, cb, (uint64_t)i, (uint64_t)t), (uint64_t)P.n);
  __syncthreads();
  int ob0 = 0, ob1 = 0;  // block override seen by the leapfrog passes
  {
    const PassResult r = estimator_pass<Real, DC, FAM, true>(P, urow, b0, b1, blk, red, th - tb, lane);
    const double lam0 = a * lh0 - 0.5 * a * a * sg0;
    const double lam1 = a * r.lhat - 0.5 * a * a * r.sig2;
    const double logr = lam1 - lam0;
    const double logU = log(word_to_uniform(stream_word(P.seed, stream_ctr0(kUAccept, A.stage, A.move, 0), (uint64_t)i, 0)));
    const bool acc = isfinite(logr) && (logU < logr);
    if (acc) {
      for (int t = lane; t < b1 - b0; t += kWave) urow[b0 + t] = blk[t];
      lh0 = r.lhat; sg0 = r.sig2; gl0 = r.gl; gs0 = r.gs;
      ob0 = b0; ob1 = b1;
    }
    if (lane == 0) A.accept[2 * i] = acc ? 1 : 0;
  }

  // ---- 2. theta | u: HMC
  const uint64_t cm = stream_ctr0(kMomentum, A.stage, A.move, 0);
  const double z = lane < d ? stream_normal(P.seed, cm, (uint64_t)i, (uint32_t)lane) : 0.0;
  double p = 0.0;  // p = Linv' z, so p ~ N(0, Sigma^{-1})
  for (int e = 0; e < d; ++e) {
    const double ze = readlane_d(z, e);
    p += (lane < d && e >= lane ? P.Linv[e * d + lane] : 0.0) * ze;
  }
  double v = sigma_times(P, p, lane);
  const double K0 = 0.5 * wave_sum(p * v);
  double rq, lp;
  prior_terms<DC>(P, th, lane, rq, lp);
  const double logpi0 = (a * lh0 - 0.5 * a * a * sg0) + lp;
  const double H0 = -logpi0 + K0;
  double grad = a * gl0 - 0.5 * a * a * gs0 - rq;
  p += 0.5 * eps * grad;
  double th1 = th;
  PassResult r1;
  r1.lhat = lh0; r1.sig2 = sg0; r1.gl = gl0; r1.gs = gs0; r1.dhat = 0.0;
  double lp1 = lp;
  for (int l = 1; l <= A.L; ++l) {
    v = sigma_times(P, p, lane);
    th1 += eps * v;
    r1 = estimator_pass<Real, DC, FAM, true>(P, urow, ob0, ob1, blk, red, th1 - tb, lane);
    prior_terms<DC>(P, th1, lane, rq, lp1);
    grad = a * r1.gl - 0.5 * a * a * r1.gs - rq;
    p += ((l < A.L) ? eps : 0.5 * eps) * grad;
  }
  v = sigma_times(P, p, lane);
  const double K1 = 0.5 * wave_sum(p * v);
  const double logpi1 = (a * r1.lhat - 0.5 * a * a * r1.sig2) + lp1;
  const double H1 = -logpi1 + K1;
  const double logr = H0 - H1;
  const double logU = log(word_to_uniform(stream_word(P.seed, stream_ctr0(kThetaAccept, A.stage, A.move, 0), (uint64_t)i, 0)));
  const bool acc = isfinite(logr) && (logU < logr);
  if (acc) {
    th = th1; lh0 = r1.lhat; sg0 = r1.sig2; gl0 = r1.gl; gs0 = r1.gs;
  }
  if (lane < d) {
    A.theta[(int64_t)i * d + lane] = th;
    A.grad_l[(int64_t)i * d + lane] = gl0;
    A.grad_s[(int64_t)i * d + lane] = gs0;
  }
  if (lane == 0) {
    A.lhat[i] = lh0;
    A.sig2[i] = sg0;
    A.accept[2 * i + 1] = acc ? 1 : 0;
  }
}

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
  const uint64_t c0 = stream_ctr0(kPriorNormal, 0, 0, 0);
  const double z = lane < d ? stream_normal(P.seed, c0, (uint64_t)i, (uint32_t)lane) : 0.0;
  double x = 0.0;  // theta - mu0 = L0^{-T} z
  for (int e = 0; e < d; ++e) {
    const double ze = readlane_d(z, e);
    x += (lane < d && e >= lane ? A.L0inv[e * d + lane] : 0.0) * ze;
  }
  if (lane < d) A.theta[(int64_t)i * d + lane] = P.mu0[lane] + x;
  const uint64_t c1 = stream_ctr0(kInitIndex, 0, 0, 0);
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
constexpr int kTemperMaxIter = 100;  // root-finding iterations (each one ESS evaluation)

struct TemperArgs {
  int M;
  double a_prev, ess_frac;
  const double* lhat;
  const double* sig2;
  double* logw;     // in/out
  double* out;      // [a, dlogz, ess, status, evaluations]
  const double* grid_ess;  // null: root search; else the ESS at grid_n grid points
  int grid_n;
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

// Tempering exponent (section 2.2; Algorithm 2 step b): the root in
// (a_prev, 1] of g(a) = log ESS(a) - log(ess_frac M). a = 1 when ESS(1)
// meets the target. Otherwise a safeguarded Newton iteration on g, whose
// derivative comes with the same sums: with x_i(a) = log W_i + nu_i(a) and
// nu_i' = lhat_i - a sig2_i,
//   g'(a) = 2 sum w nu' / sum w - 2 sum w^2 nu' / sum w^2.
// The bracket [lo, hi] keeps g(lo) >= 0 > g(hi); a step that leaves it, or a
// non-negative slope, is replaced by bisection. The first trial point treats
// the log weights as Gaussian in a: g(a) ~ g(a_prev) - (a - a_prev)^2 V with
// V the weighted variance of nu' at a_prev. The iteration stops when a step
// or the bracket is below 1e-15 (1 - a_prev); a = lo (the largest point found
// with ESS >= target), or hi if lo never moved.
// Then the reweighting, normalisation and the evidence increment
// log sum_i W_i exp(nu_i) (sections 3.3, 3.5; Algorithm 2 step c).
__global__ void __launch_bounds__(kTemperThreads) temper_kernel(TemperArgs A) {
  __shared__ double sh[4 * kTemperSlice];
  const int t = threadIdx.x;
  double lw[kTemperPer], lh[kTemperPer], s2[kTemperPer];
#pragma unroll
  for (int q = 0; q < kTemperPer; ++q) {
    const int i = t + q * kTemperThreads;
    const bool ok = i < A.M;
    lw[q] = ok ? A.logw[i] : -INFINITY;
    lh[q] = ok ? A.lhat[i] : 0.0;
    s2[q] = ok ? A.sig2[i] : 0.0;
  }
  const double log_target = log(A.ess_frac * (double)A.M);
  int buf = 0, evals = 0;
  // g(a), g'(a) and (with var) the weighted variance of nu' at a
  auto eval = [&](double a, double& g, double& dg, double* var) {
    double mx = -INFINITY;
#pragma unroll
    for (int q = 0; q < kTemperPer; ++q) mx = fmax(mx, lw[q] + incr_weight(a, A.a_prev, lh[q], s2[q]));
    mx = block_max_1(mx, sh, buf);
    buf = (buf + 1) & 3;
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (isfinite(mx)) {
#pragma unroll
      for (int q = 0; q < kTemperPer; ++q) {
        const double x = lw[q] + incr_weight(a, A.a_prev, lh[q], s2[q]);
        const double w = exp(x - mx);
        const double nd = (w > 0.0) ? lh[q] - a * s2[q] : 0.0;
        v[0] += w;
        v[1] += w * w;
        v[2] += w * nd;
        v[3] += w * w * nd;
        v[4] += w * nd * nd;
      }
    }
    if (var) block_sum_n<5>(v, sh, buf);
    else block_sum_n<4>(v, sh, buf);
    buf = (buf + 1) & 3;
    ++evals;
    if (!isfinite(mx)) {
      g = -INFINITY;
      dg = 0.0;
      if (var) *var = 0.0;
      return;
    }
    g = 2.0 * log(v[0]) - log(v[1]) - log_target;
    dg = 2.0 * v[2] / v[0] - 2.0 * v[3] / v[1];
    if (var) {
      const double mu = v[2] / v[0];
      *var = v[4] / v[0] - mu * mu;
    }
  };
  double a = 1.0;
  double ghi = 0.0, dghi;
  if (A.grid_ess) {
    // the paper's grid rule: the grid point above a_prev whose ESS is closest
    // to the target, the first on ties
    const double target = A.ess_frac * (double)A.M;
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
  } else {
    eval(1.0, ghi, dghi, nullptr);
  }
  if (!A.grid_ess && !(ghi >= 0.0)) {
    double lo = A.a_prev, hi = 1.0;
    double glo, dglo, var;
    eval(lo, glo, dglo, &var);
    const double tol = 1e-15 * (1.0 - A.a_prev);
    if (glo >= 0.0) {
      double c = (var > 0.0 && isfinite(var)) ? lo + sqrt(glo / var) : 0.5 * (lo + hi);
      for (int it = 0; it < kTemperMaxIter && (hi - lo) > tol; ++it) {
        if (!(c > lo && c < hi)) c = 0.5 * (lo + hi);
        if (!(c > lo && c < hi)) break;  // no representable point inside the bracket
        double gc, dgc;
        eval(c, gc, dgc, nullptr);
        if (gc >= 0.0) lo = c; else hi = c;
        // Newton from c, or bisection when the step is unusable
        double nxt = (dgc < 0.0 && isfinite(gc)) ? c - gc / dgc : 0.5 * (lo + hi);
        if (!(nxt > lo && nxt < hi)) nxt = 0.5 * (lo + hi);
        if (fabs(nxt - c) <= tol) {
          // converged: settle on the side of the root with ESS >= target
          if (gc < 0.0 && nxt > lo && nxt < hi) {
            double gn, dgn;
            eval(nxt, gn, dgn, nullptr);
            if (gn >= 0.0) lo = nxt; else hi = nxt;
          }
          break;
        }
        c = nxt;
      }
    } else {
      // ESS already below the target at a_prev: the smallest step a 60-step
      // bisection of (a_prev, 1] can take
      hi = A.a_prev + (1.0 - A.a_prev) * 0x1.0p-60;
    }
    a = (lo > A.a_prev) ? lo : hi;
  }
  __syncthreads();
  // reweight, normalise and the evidence increment
  double nw[kTemperPer];
  double mo = -INFINITY, mn = -INFINITY;
#pragma unroll
  for (int q = 0; q < kTemperPer; ++q) {
    const int i = t + q * kTemperThreads;
    nw[q] = i < A.M ? lw[q] + incr_weight(a, A.a_prev, lh[q], s2[q]) : -INFINITY;
    mo = fmax(mo, lw[q]);
    mn = fmax(mn, nw[q]);
  }
  mo = block_max_1(mo, sh, 0);
  mn = block_max_1(mn, sh, 1);
  double so = 0.0, sn = 0.0, sn2 = 0.0;
#pragma unroll
  for (int q = 0; q < kTemperPer; ++q) {
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
  for (int q = 0; q < kTemperPer; ++q) {
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

// The same factorisation with the matrices in LDS (d <= kFactorLdsMaxD):
// left-looking by columns, L[r][j] = (S[r][j] - sum_{k<j} L[r][k] L[j][k]) /
// L[j][j] with the subtractions in the order of the right-looking update
// above, so the factor is the same; then the inverse by the same column-wise
// forward substitution. Ls and Li are d*d doubles of LDS each.
constexpr int kFactorLdsMaxD = 64;

__device__ void factor_spd_lds(const FactorArgs& F, double* Ls, double* Li) {
  const int d = F.d;
  const int t = threadIdx.x;
  double tr = 0.0;
  for (int r = 0; r < d; ++r) tr += F.S[r * d + r];
  bool ok = false;
  for (int att = 0; att <= 10 && !ok; ++att) {
    const double jit = att > 0 ? 1e-10 * (tr / d) * pow(10.0, (double)(att - 1)) : 0.0;
    for (int e = t; e < d * d; e += kMomThreads) {
      const int r = e / d, c = e % d;
      Ls[e] = F.S[e] + (r == c ? jit : 0.0);
    }
    __syncthreads();
    bool good = true;
    for (int j = 0; j < d; ++j) {
      double sj = 0.0;
      if (t >= j && t < d) {
        sj = Ls[t * d + j];
        for (int k = 0; k < j; ++k) sj -= Ls[t * d + k] * Ls[j * d + k];
      }
      // row j's entries left of the diagonal are final; nobody reads (j, j) now
      if (t == j) Ls[j * d + j] = sj;
      __syncthreads();
      const double p = Ls[j * d + j];
      good = p > 0.0;
      if (!good) break;  // the same value in every thread
      const double ljj = sqrt(p);
      if (t > j && t < d) Ls[t * d + j] = sj / ljj;
      __syncthreads();
      // (j, j) is read again only after the loop
      if (t == j) Ls[j * d + j] = ljj;
    }
    ok = good;
    __syncthreads();
    if (ok && att > 0) {
      for (int r = t; r < d; r += kMomThreads) F.S[r * d + r] += jit;
    }
  }
  // inverse: column c of L^{-1} solves L x = e_c
  for (int c = t; c < d; c += kMomThreads) {
    for (int r = 0; r < d; ++r) {
      if (r < c) { Li[r * d + c] = 0.0; continue; }
      double s = (r == c) ? 1.0 : 0.0;
      for (int k = c; k < r; ++k) s -= Ls[r * d + k] * Li[k * d + c];
      Li[r * d + c] = s / Ls[r * d + r];
    }
  }
  __syncthreads();
  for (int e = t; e < d * d; e += kMomThreads) {
    const int r = e / d, c = e % d;
    F.L[e] = c > r ? 0.0 : Ls[e];
    F.Linv[e] = Li[e];
  }
  if (t == 0) F.status[0] = ok ? 0.0 : 1.0;
}

__global__ void __launch_bounds__(kMomThreads) factor_kernel(FactorArgs F) {
  __shared__ double sh[kMomThreads / kWave];
  extern __shared__ double fl[];  // 2 d*d when d <= kFactorLdsMaxD
  if (F.d <= kFactorLdsMaxD) factor_spd_lds(F, fl, fl + F.d * F.d);
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
  const double* centre;   // d
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

__global__ void __launch_bounds__(kMomThreads) moments_partial_kernel(MomentArgs A) {
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
  const int i0 = blockIdx.x * kMomTile;
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
    A.partials[(int64_t)blockIdx.x * ne + e] = acc;
  }
}

__global__ void __launch_bounds__(kMomThreads) moments_final_kernel(MomentArgs A) {
  __shared__ double sh[kMomThreads / kWave];
  extern __shared__ double tot[];  // d + d(d+1)/2, then 2 d*d when d <= kFactorLdsMaxD
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
  uint32_t stage;
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

__global__ void __launch_bounds__(kResThreads) resample_kernel(ResampleArgs A) {
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
  const uint64_t c0 = stream_ctr0(kResampleOffset, A.stage, 0, 0);
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

// dst row k <- src row anc[k]; blockIdx.x = k, the u row copied with 16-byte moves
__global__ void __launch_bounds__(256) gather_kernel(GatherArgs A) {
  const int k = blockIdx.x;
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

__global__ void __launch_bounds__(256) copyback_kernel(CopyBackArgs A) {
  const int k = blockIdx.x;
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

}  // namespace subsmc
