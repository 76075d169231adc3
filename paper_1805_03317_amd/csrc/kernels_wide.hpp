// Wide-row variants of the estimator pass and the fused move for
// 32 < d <= 128. A group of G lanes (G = 4 or 8) shares one packed row, each
// lane holding a contiguous chunk of CH elements of it, so a wavefront streams
// 64/G rows per iteration with 16-byte loads. Parameter component c lives in
// lane c % 64, slot c / 64 (NC slots per lane: 1 for 4-lane rows, 2 for
// 8-lane rows). Vectors that every lane
// needs at arbitrary positions (delta, momentum, theta) are broadcast through
// LDS. Everything else (remainders, fixed-order reductions, RNG streams, the
// structure of Algorithm 1) is as in the narrow kernels.
#pragma once
#include "kernels.hpp"

namespace subsmc {

// parameter components per lane: one for 4-lane rows (d <= 60), two for
// 8-lane rows (d <= 128)
template <int G>
constexpr int wide_nc() { return G == 4 ? 1 : 2; }

template <int NC>
struct PassResultW {
  double lhat, sig2, dhat;
  double gl[NC], gs[NC];
};

template <typename Real, int CH>
__device__ __forceinline__ void load_chunk(const Real* __restrict__ p, Real (&x)[CH]) {
  if constexpr (sizeof(Real) == 4) {
    static_assert(CH % 4 == 0, "float chunk must be a multiple of 4");
    const float4* v = reinterpret_cast<const float4*>(p);
#pragma unroll
    for (int q = 0; q < CH / 4; ++q) {
      const float4 t = v[q];
      x[4 * q] = t.x; x[4 * q + 1] = t.y; x[4 * q + 2] = t.z; x[4 * q + 3] = t.w;
    }
  } else {
    static_assert(CH % 2 == 0, "double chunk must be even");
    const double2* v = reinterpret_cast<const double2*>(p);
#pragma unroll
    for (int q = 0; q < CH / 2; ++q) {
      const double2 t = v[q];
      x[2 * q] = t.x; x[2 * q + 1] = t.y;
    }
  }
}

// Pass of the difference estimator for one particle (see estimator_pass);
// `vec` (LDS) holds delta = theta - theta_bar. Each lane gathers the CH
// elements of delta aligned with its chunk of the row (zero at the header and
// padding positions).
// Tile forms of the row loop (TL): 0, the default, evaluates each row's
// remainder once per row for FP32 logistic rows (one lane of the group per
// row, four row iterations per step); 1 evaluates it in every lane of the
// row's group (the only form for the other shapes). The autotuner measures
// both where both exist.
template <typename Real, int FAM, int G, int TL>
constexpr bool wide_one_remainder_per_lane() {
  return sizeof(Real) == 4 && FAM == kLogistic && (G == 4 || G == 8) && TL == 0;
}

// SYNC: the caller runs several particles in one workgroup (one per wavefront)
// and the wavefronts meet at a workgroup barrier once every kSyncIters
// iterations of the row loop (every wavefront of the workgroup takes the same
// number of steps: same m), so that the copies of a resampled particle, which
// read the same rows, read them at nearly the same time (the second read then
// hits the L2 or merges with the first). A barrier at every step holds each
// wavefront to the slowest one's remainders; with none the copies drift apart.
constexpr int kSyncIters = 32;
template <typename Real, int G, int CH, int FAM, bool BLK, int TL = 0, bool SYNC = false>
__device__ __forceinline__ PassResultW<wide_nc<G>()> estimator_pass_wide(const Prob& P, const int32_t* __restrict__ urow,
                                                           int b0, int b1, const int32_t* blk, Real* red,
                                                           const double* vec /* LDS: delta, d values */,
                                                           int lane) {
  const Real* __restrict__ X = static_cast<const Real*>(P.X);
  const int m = P.m;
  const int ld = P.ld;
  const int d = P.d;
  const uint32_t n = (uint32_t)P.n;
  const Real inv_s2 = (Real)P.inv_s2;
  constexpr int kRows = kWave / G;  // rows per wave iteration
  const int q = lane % G;           // chunk index within the row
  const int grp = lane / G;         // row group

  Real dl[CH];
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    const int c = q * CH + k - kHeader;
    dl[k] = (c >= 0 && c < d) ? (Real)vec[c] : Real(0);
  }
  // the index of slot j, given g = urow[j]: the refreshed block's (staged in
  // LDS) inside [b0, b1), else the particle's own
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
  auto eval_row = [&](const Real (&x)[CH], Real& dd, Real& dp) {
    Real part = Real(0);
#pragma unroll
    for (int k = 0; k < CH; ++k) part += x[k] * dl[k];
    part = xl::group_sum<G>(part);
    const Real eb = xl::group_lead<G>(x[0], lane);
    const Real aux = xl::group_lead<G>(x[1], lane);
    cv_remainder<Real, FAM>(P.cv_order, eb, aux, part, inv_s2, dd, dp);
  };

  double shift;
  {
    const int32_t k0 = index_of(0);
    const bool bad = (uint32_t)k0 >= n;
    Real x[CH];
    load_chunk<Real, CH>(X + (int64_t)(bad ? 0 : k0) * ld + q * CH, x);
    Real dd, dp;
    eval_row(x, dd, dp);
    shift = bad ? __builtin_nan("") : (double)dd;
  }

  double se = 0.0, se2 = 0.0;
  Real S1[CH], T1[CH];
#pragma unroll
  for (int k = 0; k < CH; ++k) { S1[k] = Real(0); T1[k] = Real(0); }

  const int nit = (m + kRows - 1) / kRows;  // row iterations t (rows grp + kRows t)
  // slot of iteration t's row in this group, clamped to the last slot:
  // iterations past the group's last row read a real row and add nothing, and
  // all groups run the same number of steps
  auto slot_at = [&](int t) -> int {
    const int jj = grp + kRows * t;
    return jj < m ? jj : m - 1;
  };
  // urow of iteration t, loaded without a branch and not used until
  // resolve_at a step later: the vector-memory counter retires loads in
  // order, so a wait for an index loaded after rows would wait for those rows
  auto fetch_at = [&](int t) -> int32_t { return urow[slot_at(t)]; };
  auto resolve_at = [&](int t, int32_t g) -> int32_t { return resolve(slot_at(t), g); };
  auto index_at = [&](int t) -> int32_t { return resolve_at(t, fetch_at(t)); };
  auto load_row = [&](int32_t k, Real (&x)[CH]) {
    load_chunk<Real, CH>(X + (int64_t)((uint32_t)k < n ? k : 0) * ld + q * CH, x);
  };
  // Row indices are loaded a step ahead of their rows and resolved only when
  // their rows are requested, so a row load never waits behind the load of its
  // own index, and every wait is for the oldest rows in flight.
  if constexpr (wide_one_remainder_per_lane<Real, FAM, G, TL>()) {
    // (the logistic remainder is the costly one; for the other families the
    // register cost of two buffered steps outweighs it)
    // PT = 4 iterations per step, two steps of rows in flight (buffers xa, xb).
    // Each group forms the PT dot products of a step; lane q then evaluates
    // the remainder of iteration q % PT only (one remainder per lane of a
    // quad, not one per row and lane; with 8-lane rows each quad of the group
    // evaluates the same four), and the PT pairs (d, d') go back to every lane
    // of the quad by quad broadcasts for the accumulation.
    constexpr int PT = 4;
    static_assert(PT <= 4 && PT <= G, "one quad holds the step's remainders");
    const int nsteps = (nit + PT - 1) / PT;
    const int mine = q % PT;
    Real xa[PT][CH], xb[PT][CH];
    int32_t ka[PT], kb[PT], kf[PT];
#pragma unroll
    for (int s = 0; s < PT; ++s) ka[s] = index_at(s);
#pragma unroll
    for (int s = 0; s < PT; ++s) load_row(ka[s], xa[s]);
#pragma unroll
    for (int s = 0; s < PT; ++s) kb[s] = index_at(PT + s);
#pragma unroll
    for (int s = 0; s < PT; ++s) load_row(kb[s], xb[s]);
#pragma unroll
    for (int s = 0; s < PT; ++s) kf[s] = fetch_at(2 * PT + s);
    // one step on buffer x (rows of step `step`, indices kx); refills x with
    // the rows of step + 2 (urow of those in kf, not yet resolved)
    auto step_on = [&](Real (&x)[PT][CH], int32_t (&kx)[PT], int step) {
      int32_t kg[PT];
#pragma unroll
      for (int s = 0; s < PT; ++s) kg[s] = fetch_at(PT * (step + 3) + s);
      Real Dm = Real(0), ebm = Real(0), auxm = Real(0);
      int32_t km = 0;
#pragma unroll
      for (int s = 0; s < PT; ++s) {
        Real part = Real(0);
#pragma unroll
        for (int k = 0; k < CH; ++k) part += x[s][k] * dl[k];
        part = xl::group_sum<G>(part);
        const Real eb = xl::group_lead<G>(x[s][0], lane);
        const Real aux = xl::group_lead<G>(x[s][1], lane);
        Dm = (mine == s) ? part : Dm;
        ebm = (mine == s) ? eb : ebm;
        auxm = (mine == s) ? aux : auxm;
        km = (mine == s) ? kx[s] : km;
      }
      Real dd, dp;
      cv_remainder<Real, FAM>(P.cv_order, ebm, auxm, Dm, inv_s2, dd, dp);
      const bool valid = grp + kRows * (PT * step + mine) < m;
      if ((uint32_t)km >= n) dd = dp = Real(__builtin_nan(""));
      if (!valid) dp = Real(0);
      const double e = valid ? (double)dd - shift : 0.0;
      if (q < PT) {
        se += e;
        se2 += e * e;
      }
      const Real edp = (Real)e * dp;
#pragma unroll
      for (int s = 0; s < PT; ++s) {
        // (s is a constant once the loop is unrolled)
        Real dps, edps;
        switch (s) {
          case 0: dps = xl::quad_pick<0>(dp); edps = xl::quad_pick<0>(edp); break;
          case 1: dps = xl::quad_pick<1>(dp); edps = xl::quad_pick<1>(edp); break;
          case 2: dps = xl::quad_pick<2>(dp); edps = xl::quad_pick<2>(edp); break;
          default: dps = xl::quad_pick<3>(dp); edps = xl::quad_pick<3>(edp); break;
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          S1[k] += dps * x[s][k];
          T1[k] += edps * x[s][k];
        }
        const int32_t kr = resolve_at(PT * (step + 2) + s, kf[s]);
        load_row(kr, x[s]);
        kx[s] = kr;
      }
#pragma unroll
      for (int s = 0; s < PT; ++s) kf[s] = kg[s];
    };
    for (int step = 0; step < nsteps; step += 2) {
      if constexpr (SYNC) {
        if (step % (kSyncIters / PT) == 0) __builtin_amdgcn_s_barrier();
      }
      step_on(xa, ka, step);
      if (step + 1 < nsteps) step_on(xb, kb, step + 1);
    }
  } else {
    // PD iterations per step, their chunks in xb, each refilled with the next
    // step's row as soon as it has been used.
    constexpr int PD = 2;
    const int nsteps = (nit + PD - 1) / PD;
    Real xb[PD][CH];
    int32_t kc[PD], kn[PD];
#pragma unroll
    for (int s = 0; s < PD; ++s) kc[s] = index_at(s);
#pragma unroll
    for (int s = 0; s < PD; ++s) load_row(kc[s], xb[s]);
#pragma unroll
    for (int s = 0; s < PD; ++s) kn[s] = fetch_at(PD + s);
    for (int step = 0; step < nsteps; ++step) {
      if constexpr (SYNC) {
        if (step % (kSyncIters / PD) == 0) __builtin_amdgcn_s_barrier();
      }
      int32_t kf[PD];
#pragma unroll
      for (int s = 0; s < PD; ++s) kf[s] = fetch_at(PD * (step + 2) + s);
#pragma unroll
      for (int s = 0; s < PD; ++s) {
        const bool valid = grp + kRows * (PD * step + s) < m;
        const bool bad = (uint32_t)kc[s] >= n;
        Real dd, dp;
        eval_row(xb[s], dd, dp);
        if (bad) dd = dp = Real(__builtin_nan(""));
        if (!valid) dp = Real(0);
        const double e = valid ? (double)dd - shift : 0.0;
        if (q == 0) {
          se += e;
          se2 += e * e;
        }
        const Real edp = (Real)e * dp;
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          S1[k] += dp * xb[s][k];
          T1[k] += edp * xb[s][k];
        }
        const int32_t kr = resolve_at(PD * (step + 1) + s, kn[s]);
        load_row(kr, xb[s]);
        kc[s] = kr;
      }
#pragma unroll
      for (int s = 0; s < PD; ++s) kn[s] = kf[s];
    }
  }

  se = wave_sum(se);
  se2 = wave_sum(se2);
  // column sums: position p = c + header lives in chunk p / CH, element p % CH
  constexpr int NC = wide_nc<G>();
  auto column = [&](const Real (&v)[CH], double (&out)[NC]) {
    wave_lds_sync();
#pragma unroll
    for (int k = 0; k < CH; ++k) red[lane * CH + k] = v[k];
    wave_lds_sync();
#pragma unroll
    for (int s = 0; s < NC; ++s) {
      const int c = lane + kWave * s;
      double acc = 0.0;
      if (c < d) {
        const int p = c + kHeader;
        const int qq = p / CH, kk = p % CH;
        for (int g = 0; g < kRows; ++g) acc += (double)red[(g * G + qq) * CH + kk];
      }
      out[s] = acc;
    }
  };
  double s1[NC], t1[NC];
  column(S1, s1);
  column(T1, t1);

  const double md = (double)m;
  const double nm = P.n_over_m;
  const double dsum = se + md * shift;
  const double dbar_minus_shift = se / md;
  const double m2 = se2 - se * dbar_minus_shift;
  PassResultW<NC> out;
  out.dhat = nm * dsum;
  out.sig2 = nm * nm * (m2 < 0.0 ? 0.0 : m2);
  double qpart = 0.0;
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    const int c = lane + kWave * s;
    double cdel = 0.0, bl = 0.0, dc = 0.0;
    if (c < d) {
      for (int e = 0; e < d; ++e) cdel += P.cvC[c * d + e] * vec[e];
      bl = P.cvB[c];
      dc = vec[c];
    }
    qpart += (P.cv_order == 2) ? (bl * dc + 0.5 * dc * cdel) : bl * dc;
    out.gl[s] = c < d ? bl + (P.cv_order == 2 ? cdel : 0.0) + nm * s1[s] : 0.0;
    out.gs[s] = c < d ? 2.0 * nm * nm * (t1[s] - dbar_minus_shift * s1[s]) : 0.0;
  }
  out.lhat = P.cvA[0] + wave_sum(qpart) + out.dhat;
  return out;
}

// vec <- x (component slots of every lane), with the fences around it
template <int NC>
__device__ __forceinline__ void to_lds(double* vec, const double (&x)[NC], int lane, int d) {
  wave_lds_sync();
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    const int c = lane + kWave * s;
    if (c < d) vec[c] = x[s];
  }
  wave_lds_sync();
}

template <typename Real, int G, int CH, int FAM>
__global__ void __launch_bounds__(kWave) estimator_kernel_wide(EstArgs A) {
  __shared__ Real red[kWave * CH];
  __shared__ double vec[128];
  const int i = blockIdx.x;
  const int lane = threadIdx.x;
  if (i >= A.count) return;
  const Prob& P = A.P;
  const int d = P.d;
  constexpr int NC = wide_nc<G>();
  double dl[NC];
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    const int c = lane + kWave * s;
    dl[s] = c < d ? A.theta[(int64_t)i * d + c] - P.theta_bar[c] : 0.0;
  }
  to_lds(vec, dl, lane, d);
  const auto r = estimator_pass_wide<Real, G, CH, FAM, false>(P, A.u + (int64_t)i * P.m, 0, 0, nullptr,
                                                                     red, vec, lane);
  if (lane == 0) {
    if (A.lhat) A.lhat[i] = r.lhat;
    if (A.sig2) A.sig2[i] = r.sig2;
    if (A.dhat) A.dhat[i] = r.dhat;
    if (A.lam) A.lam[i] = A.a * r.lhat - 0.5 * A.a * A.a * r.sig2;
  }
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    const int c = lane + kWave * s;
    if (c < d) {
      if (A.grad_l) A.grad_l[(int64_t)i * d + c] = r.gl[s];
      if (A.grad_s) A.grad_s[(int64_t)i * d + c] = r.gs[s];
      if (A.grad) {
        const double gl = A.g_lhat ? A.g_lhat[i] : 0.0;
        const double gs = A.g_sig2 ? A.g_sig2[i] : 0.0;
        A.grad[(int64_t)i * d + c] = gl * r.gl[s] + gs * r.gs[s];
      }
    }
  }
}

// y = M x for a d x d row-major matrix; x broadcast through LDS
template <int NC>
__device__ __forceinline__ void matvec_wide(const double* __restrict__ Mx, const double* vec, int d, int lane,
                                            double (&y)[NC]) {
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    const int c = lane + kWave * s;
    double acc = 0.0;
    if (c < d)
      for (int e = 0; e < d; ++e) acc += Mx[c * d + e] * vec[e];
    y[s] = acc;
  }
}

// Fused Markov move (Algorithm 1) for wide rows; same steps, draws and
// decisions as move_kernel.
// One particle's move on one wavefront. red (kWave * CH values), vec (128
// doubles) and blk (the refreshed block's indices, ceil(m / G) values) are LDS of
// this wavefront's own.
template <typename Real, int G, int CH, int FAM, int TL, bool SYNC = false>
__device__ __forceinline__ void move_wide_body(const MoveArgs& A, const int i, Real* red, double* vec,
                                               int32_t* blk) {
  const int lane = wave_lane();
  const Prob& P = A.P;
  if (i >= P.M) return;
  const int d = P.d;
  const int m = P.m;
  const double a = A.a;
  const double eps = A.eps;
  int32_t* urow = A.u + (int64_t)i * m;
  constexpr int NC = wide_nc<G>();

  double tb[NC], th[NC], gl0[NC], gs0[NC];
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    const int c = lane + kWave * s;
    tb[s] = c < d ? P.theta_bar[c] : 0.0;
    th[s] = c < d ? A.theta[(int64_t)i * d + c] : 0.0;
    gl0[s] = c < d ? A.grad_l[(int64_t)i * d + c] : 0.0;
    gs0[s] = c < d ? A.grad_s[(int64_t)i * d + c] : 0.0;
  }
  double lh0 = A.lhat[i], sg0 = A.sig2[i];

  // ---- 1. u | theta
  const uint64_t cg = stream_ctr0(kBlockChoice, A.stage, A.move, P.dataset);
  const int g = (int)word_to_index(stream_word(P.seed, cg, (uint64_t)i, 0), (uint64_t)P.G);
  const int b0 = (int)((int64_t)g * m / P.G);
  const int b1 = (int)((int64_t)(g + 1) * m / P.G);
  const uint64_t cb = stream_ctr0(kBlockIndex, A.stage, A.move, P.dataset);
  for (int t = lane; t < b1 - b0; t += kWave)
    blk[t] = (int32_t)word_to_index(stream_word(P.seed, cb, (uint64_t)i, (uint64_t)t), (uint64_t)P.n);
  int ob0 = 0, ob1 = 0;
  {
    double dl[NC];
#pragma unroll
    for (int s = 0; s < NC; ++s) dl[s] = th[s] - tb[s];
    to_lds(vec, dl, lane, d);  // also fences the block indices
    const auto r = estimator_pass_wide<Real, G, CH, FAM, true, TL, SYNC>(P, urow, b0, b1, blk, red, vec, lane);
    const double lam0 = a * lh0 - 0.5 * a * a * sg0;
    const double lam1 = a * r.lhat - 0.5 * a * a * r.sig2;
    const double logr = lam1 - lam0;
    const double logU = log(word_to_uniform(stream_word(P.seed, stream_ctr0(kUAccept, A.stage, A.move, P.dataset), (uint64_t)i, 0)));
    const bool acc = isfinite(logr) && (logU < logr);
    if (acc) {
      for (int t = lane; t < b1 - b0; t += kWave) urow[b0 + t] = blk[t];
      lh0 = r.lhat; sg0 = r.sig2;
#pragma unroll
      for (int s = 0; s < NC; ++s) { gl0[s] = r.gl[s]; gs0[s] = r.gs[s]; }
      ob0 = b0; ob1 = b1;
    }
    if (lane == 0) {
      A.accept[2 * i] = acc ? 1 : 0;
      record_decision(A, i, 0, logU, logr);
    }
  }

  // ---- 2. theta | u: HMC
  const uint64_t cm = stream_ctr0(kMomentum, A.stage, A.move, P.dataset);
  double z[NC];
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    const int c = lane + kWave * s;
    z[s] = c < d ? stream_normal(P.seed, cm, (uint64_t)i, (uint32_t)c) : 0.0;
  }
  to_lds(vec, z, lane, d);
  double p[NC];  // p = Linv' z
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    const int c = lane + kWave * s;
    double acc = 0.0;
    if (c < d)
      for (int e = c; e < d; ++e) acc += P.Linv[e * d + c] * vec[e];
    p[s] = acc;
  }
  auto kinetic_and_velocity = [&](double (&v)[NC]) -> double {
    to_lds(vec, p, lane, d);
    matvec_wide(P.Sigma, vec, d, lane, v);
    double k = 0.0;
#pragma unroll
    for (int s = 0; s < NC; ++s) k += p[s] * v[s];
    return 0.5 * wave_sum(k);
  };
  auto prior = [&](const double (&t)[NC], double (&r)[NC]) -> double {
    double dm[NC];
#pragma unroll
    for (int s = 0; s < NC; ++s) {
      const int c = lane + kWave * s;
      dm[s] = c < d ? t[s] - P.mu0[c] : 0.0;
    }
    to_lds(vec, dm, lane, d);
    matvec_wide(P.Q0, vec, d, lane, r);
    double lp = 0.0;
#pragma unroll
    for (int s = 0; s < NC; ++s) lp += -0.5 * dm[s] * r[s];
    return wave_sum(lp);
  };
  double v[NC], rq[NC];
  const double K0 = kinetic_and_velocity(v);
  const double lp0 = prior(th, rq);
  const double logpi0 = (a * lh0 - 0.5 * a * a * sg0) + lp0;
  const double H0 = -logpi0 + K0;
  double th1[NC];
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    p[s] += 0.5 * eps * (a * gl0[s] - 0.5 * a * a * gs0[s] - rq[s]);
    th1[s] = th[s];
  }
  double lh1 = lh0, sg1 = sg0, gl1[NC], gs1[NC], lp1 = lp0;
#pragma unroll
  for (int s = 0; s < NC; ++s) { gl1[s] = gl0[s]; gs1[s] = gs0[s]; }
  for (int l = 1; l <= A.L; ++l) {
    to_lds(vec, p, lane, d);
    matvec_wide(P.Sigma, vec, d, lane, v);
    double dl[NC];
#pragma unroll
    for (int s = 0; s < NC; ++s) {
      th1[s] += eps * v[s];
      dl[s] = th1[s] - tb[s];
    }
    to_lds(vec, dl, lane, d);
    const auto r = estimator_pass_wide<Real, G, CH, FAM, true, TL, SYNC>(P, urow, ob0, ob1, blk, red, vec, lane);
    lh1 = r.lhat;
    sg1 = r.sig2;
    lp1 = prior(th1, rq);
    const double h = (l < A.L) ? eps : 0.5 * eps;
#pragma unroll
    for (int s = 0; s < NC; ++s) {
      gl1[s] = r.gl[s];
      gs1[s] = r.gs[s];
      p[s] += h * (a * gl1[s] - 0.5 * a * a * gs1[s] - rq[s]);
    }
  }
  const double K1 = kinetic_and_velocity(v);
  const double logpi1 = (a * lh1 - 0.5 * a * a * sg1) + lp1;
  const double H1 = -logpi1 + K1;
  const double logr = H0 - H1;
  const double logU = log(word_to_uniform(stream_word(P.seed, stream_ctr0(kThetaAccept, A.stage, A.move, P.dataset), (uint64_t)i, 0)));
  const bool acc = isfinite(logr) && (logU < logr);
  if (acc) {
    lh0 = lh1; sg0 = sg1;
#pragma unroll
    for (int s = 0; s < NC; ++s) { th[s] = th1[s]; gl0[s] = gl1[s]; gs0[s] = gs1[s]; }
  }
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    const int c = lane + kWave * s;
    if (c < d) {
      A.theta[(int64_t)i * d + c] = th[s];
      A.grad_l[(int64_t)i * d + c] = gl0[s];
      A.grad_s[(int64_t)i * d + c] = gs0[s];
    }
  }
  if (lane == 0) {
    A.lhat[i] = lh0;
    A.sig2[i] = sg0;
    A.accept[2 * i + 1] = acc ? 1 : 0;
    record_decision(A, i, 1, logU, logr);
  }
}

template <typename Real, int G, int CH, int FAM, int TL>
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(kMoveWaves<Real>))) move_kernel_wide(MoveArgs A) {
  __shared__ Real red[kWave * CH];
  __shared__ double vec[128];
  extern __shared__ int32_t blk[];
  move_wide_body<Real, G, CH, FAM, TL>(A, xcd_particle((int)blockIdx.x, (int)gridDim.x), red, vec, blk);
}

// The lane-group move (tile form 2: form 0's row loop) with kWideGroup
// consecutive particles per workgroup, one per wavefront, each
// with an LDS slice of its own of wide_group_wave_lds bytes, their row steps
// held close together by a barrier every kSyncIters row iterations
// (estimator_pass_wide, SYNC). The launch covers
// the particles exactly (gridDim.x * kWideGroup == M), so every wavefront has a
// particle and takes the same number of barriers.
constexpr int kWideGroup = 4;

__host__ __device__ inline int wide_group_wave_lds(int ch, int real_bytes, int block_bytes) {
  return ((kWave * ch * real_bytes + 15) & ~15) + 128 * 8 + ((block_bytes + 15) & ~15);
}

template <typename Real, int G, int CH, int FAM, int TL>
__global__ void __launch_bounds__(kWave * kWideGroup) __attribute__((amdgpu_waves_per_eu(kMoveWaves<Real>)))
move_kernel_wide_group(MoveArgs A, int wave_lds) {
  extern __shared__ __attribute__((aligned(16))) char gsm[];
  const int wave = (int)threadIdx.x / kWave;
  char* base = gsm + wave * wave_lds;
  constexpr int kRed = (kWave * CH * (int)sizeof(Real) + 15) & ~15;
  const int i = kWideGroup * xcd_particle((int)blockIdx.x, (int)gridDim.x) + wave;
  move_wide_body<Real, G, CH, FAM, TL, true>(A, i, reinterpret_cast<Real*>(base), reinterpret_cast<double*>(base + kRed),
                                             reinterpret_cast<int32_t*>(base + kRed + 128 * 8));
}

template <typename Real, int G, int CH, int FAM, int TL>
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(kMoveWaves<Real>))) move_kernel_wide_batch(Batch<MoveArgs> B) {
  __shared__ Real red[kWave * CH];
  __shared__ double vec[128];
  extern __shared__ int32_t blk[];
  const int k = batch_member(B.first, B.count, blockIdx.x);
  const MoveArgs A = B.args[k];
  move_wide_body<Real, G, CH, FAM, TL>(A, xcd_particle((int)blockIdx.x - B.first[k], B.first[k + 1] - B.first[k]),
                                       red, vec, blk);
}

}  // namespace subsmc

