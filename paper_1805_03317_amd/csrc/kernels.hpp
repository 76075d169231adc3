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

// The streaming moves exchange data between the lanes of one wavefront through
// LDS. A wavefront's LDS instructions execute in program order, so such an
// exchange needs no workgroup barrier, only a fence that keeps the compiler
// from moving the accesses across it. With this, several wavefronts of one
// workgroup can each run a particle of their own, none waiting for another.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// lane of the calling thread within its wavefront
__device__ __forceinline__ int wave_lane() { return (int)__lane_id(); }

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
  uint32_t dataset;  // dataset field of every random-number counter
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

// --------------------------------------------------------------------------
// Batched launches: one grid serves several datasets. Workgroup b belongs to
// member k with first[k] <= b < first[k + 1] and runs as workgroup
// b - first[k] of that member's own launch, with the member's argument block.
// --------------------------------------------------------------------------
template <typename Args>
struct Batch {
  const Args* args;  // device, count argument blocks
  const int* first;  // device, count + 1 prefix sums of workgroup counts, first[0] = 0
  int count;
};

// Workgroups are dispatched to the chip's 8 XCDs in turn (workgroup b to XCD b mod 8), each XCD
// with its own L2. The moves run particle xcd_particle(b, count) in workgroup b, which gives
// every XCD a contiguous range of particles: systematic resampling leaves the copies of a
// particle at adjacent indices with the same subsample u, so the copies run behind one L2 at
// about the same time and share their row fetches there. (A bijection of [0, count); for a
// batch member, b and count are local to the member, whose workgroups with equal b mod 8 also
// share an XCD.)
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_particle(int b, int count) {
  const int x = b % kXcds, k = b / kXcds, q = count / kXcds, r = count % kXcds;
  return x * q + (x < r ? x : r) + k;
}

// the member owning workgroup b: the largest k with first[k] <= b
__device__ __forceinline__ int batch_member(const int* __restrict__ first, int count, int b) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

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
  wave_lds_sync();
#pragma unroll
  for (int c = 0; c < DC; ++c) red[lane * DC + c] = v[c];
  wave_lds_sync();
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
  auto resolve = [&](int j, int32_t g) -> int32_t {
    if constexpr (BLK) {
      const bool in = (unsigned)(j - b0) < (unsigned)(b1 - b0);
      const int32_t l = blk[in ? j - b0 : 0];
      return in ? l : g;
    } else {
      return g;
    }
  };
  auto index_of = [&](int j) -> int32_t { return resolve(j, urow[j]); };

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

  // urow of slot j clamped to the last slot, loaded without a branch; it is
  // resolved an iteration later (the vector-memory counter retires loads in
  // order, so a wait for an index loaded after a row waits for that row too)
  auto fetch = [&](int j) -> int32_t { return urow[j < m ? j : m - 1]; };
  // rows are prefetched one iteration ahead (measured: for FP64 d = 20 one
  // resident wave with the prefetch beats two without it), their indices two
  // ahead: each iteration loads urow of slot j + 128, then resolves the index
  // of slot j + 64 (loaded before the current row) and requests that row, so
  // no wait is ever for a load younger than the row it needs
  int j = lane;
  int32_t k_cur = j < m ? index_of(j) : 0;
  int32_t g_nxt = fetch(j + kWave);
  RowLoad<Real, DC> r_nxt;
  if (j < m) load_row<Real, DC>(X + (int64_t)((uint32_t)k_cur < n ? k_cur : 0) * ld, r_nxt);
  for (; j < m; j += kWave) {
    const int32_t g_far = fetch(j + 2 * kWave);
    const RowLoad<Real, DC> r = r_nxt;
    const bool bad = (uint32_t)k_cur >= n;
    const int32_t k_nxt = resolve(j + kWave < m ? j + kWave : m - 1, g_nxt);
    if (j + kWave < m) load_row<Real, DC>(X + (int64_t)((uint32_t)k_nxt < n ? k_nxt : 0) * ld, r_nxt);
    k_cur = k_nxt;
    g_nxt = g_far;

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
  double a;              // exponent of lam
  double* lam;           // count (nullable): a l_hat - a^2 sigma2_hat / 2
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
    if (A.lam) A.lam[i] = A.a * r.lhat - 0.5 * A.a * A.a * r.sig2;
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
  int32_t* ties;   // M*2 (nullable): 1 where the decision was a near tie
  double tie_tol;  // near tie: |log U - log r| <= tie_tol (1 + |log r|)
  double* diag;    // M*4 (nullable): log r and log U of the u refresh, then of the HMC step
};

// A Metropolis-Hastings decision that rounding could change.
__device__ __forceinline__ int32_t near_tie(double logU, double logr, double tol) {
  return (isfinite(logr) && fabs(logU - logr) <= tol * (1.0 + fabs(logr))) ? 1 : 0;
}

// the move's record of one Metropolis-Hastings decision (k = 0: u refresh, 1: HMC)
__device__ __forceinline__ void record_decision(const MoveArgs& A, int i, int k, double logU, double logr) {
  if (A.ties) A.ties[2 * i + k] = near_tie(logU, logr, A.tie_tol);
  if (A.diag) {
    A.diag[4 * i + 2 * k] = logr;
    A.diag[4 * i + 2 * k + 1] = logU;
  }
}


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

// One particle's move on one wavefront. red (kWave * DC values) and blk (the
// refreshed block's indices, ceil(m / G) values) are LDS of this wavefront's own.
template <typename Real, int DC, int FAM>
__device__ __forceinline__ void move_body(const MoveArgs& A, const int i, Real* red, int32_t* blk) {
  const int lane = wave_lane();
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
  const uint64_t cg = stream_ctr0(kBlockChoice, A.stage, A.move, P.dataset);
  const int g = (int)word_to_index(stream_word(P.seed, cg, (uint64_t)i, 0), (uint64_t)P.G);
  const int b0 = (int)((int64_t)g * m / P.G);
  const int b1 = (int)((int64_t)(g + 1) * m / P.G);
  const uint64_t cb = stream_ctr0(kBlockIndex, A.stage, A.move, P.dataset);
  for (int t = lane; t < b1 - b0; t += kWave)
    blk[t] = (int32_t)word_to_index(stream_word(P.seed, cb, (uint64_t)i, (uint64_t)t), (uint64_t)P.n);
  wave_lds_sync();
  int ob0 = 0, ob1 = 0;  // block override seen by the leapfrog passes
  {
    const PassResult r = estimator_pass<Real, DC, FAM, true>(P, urow, b0, b1, blk, red, th - tb, lane);
    const double lam0 = a * lh0 - 0.5 * a * a * sg0;
    const double lam1 = a * r.lhat - 0.5 * a * a * r.sig2;
    const double logr = lam1 - lam0;
    const double logU = log(word_to_uniform(stream_word(P.seed, stream_ctr0(kUAccept, A.stage, A.move, P.dataset), (uint64_t)i, 0)));
    const bool acc = isfinite(logr) && (logU < logr);
    if (acc) {
      for (int t = lane; t < b1 - b0; t += kWave) urow[b0 + t] = blk[t];
      lh0 = r.lhat; sg0 = r.sig2; gl0 = r.gl; gs0 = r.gs;
      ob0 = b0; ob1 = b1;
    }
    if (lane == 0) {
      A.accept[2 * i] = acc ? 1 : 0;
      record_decision(A, i, 0, logU, logr);
    }
  }

  // ---- 2. theta | u: HMC
  const uint64_t cm = stream_ctr0(kMomentum, A.stage, A.move, P.dataset);
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
  const double logU = log(word_to_uniform(stream_word(P.seed, stream_ctr0(kThetaAccept, A.stage, A.move, P.dataset), (uint64_t)i, 0)));
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
    record_decision(A, i, 1, logU, logr);
  }
}

// --------------------------------------------------------------------------
// Move entry points: one dataset per launch, and the batched form (one launch
// for every member of a batch, the member's argument block copied in first).
// --------------------------------------------------------------------------

// Wavefronts per SIMD the streaming moves are compiled for. With float rows
// two fit (at most 256 registers per lane, a few spilled for the widest
// logistic shapes), which hides more of the random row reads: measured 27%
// faster at d = 50, 8% at d = 30. The double-row kernels stay at one: their
// rows need the whole register file and spilling them halves their speed.
template <typename Real>
constexpr int kMoveWaves = sizeof(Real) == 4 ? 2 : 1;

template <typename Real, int DC, int FAM>
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(kMoveWaves<Real>))) move_kernel(MoveArgs A) {
  __shared__ Real red[kWave * DC];
  extern __shared__ int32_t blk[];
  move_body<Real, DC, FAM>(A, xcd_particle((int)blockIdx.x, (int)gridDim.x), red, blk);
}

template <typename Real, int DC, int FAM>
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(kMoveWaves<Real>))) move_kernel_batch(Batch<MoveArgs> B) {
  __shared__ Real red[kWave * DC];
  extern __shared__ int32_t blk[];
  const int k = batch_member(B.first, B.count, blockIdx.x);
  const MoveArgs A = B.args[k];
  move_body<Real, DC, FAM>(A, xcd_particle((int)blockIdx.x - B.first[k], B.first[k + 1] - B.first[k]), red, blk);
}

}  // namespace subsmc
