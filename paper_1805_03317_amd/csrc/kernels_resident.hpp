// Fused Markov move with the particle's subsample rows resident on chip.
//
// One workgroup of 4 wavefronts (256 lanes, one wavefront per SIMD, so each
// lane may use the whole 512-entry VGPR + AGPR file) owns one particle for the
// whole move. The m packed rows selected by u are gathered from HBM once per
// move and kept for all L + 1 estimator passes of Algorithm 1: slot
// j < 256*RPL in registers of lane j % 256 (RPL rows per lane), the remaining
// slots in LDS. A pass then reads no global memory. Partial sums are reduced
// inside each wavefront by a VALU-only reduce-scatter and across the 4
// wavefronts through LDS in fixed order; wavefront 0 does the leapfrog and MH
// arithmetic (component c of theta, p and the gradient in its lane c) and
// broadcasts delta = theta - theta_bar through LDS.
//
// The leapfrog passes between the first and the last need the gradient of the
// extended target only (section 3.3). With K = a C - Q0 (K = -Q0 for a
// first-order control variate) and
// g0 = a B - Q0 (theta_bar - mu0) it is
//   g0 + K delta + a (n/m) S1 - a^2 (n/m)^2 (T1 - dbar S1),
// S1 = sum_j d'_j x_j and T1 = sum_j (d_j - shift) d'_j x_j; the estimator
// value, sigma^2 and the prior density are formed at the u-refresh pass and at
// the last pass only. K delta is carried along the trajectory: after
// p <- p + eps grad, delta <- delta + eps Sigma p and
// K delta <- K delta + eps (K Sigma) p, where Sigma p and (K Sigma) p come
// out of one sweep (lanes 0..d-1 and 32..32+d-1). Draws, decisions and the
// order of the steps are those of move_kernel.
#pragma once
#include "kernels.hpp"
#include "xlane.hpp"

namespace subsmc {

constexpr int kResWaves = 4;
constexpr int kResLanes = kResWaves * kWave;  // 256: one wavefront per SIMD

// LDS carve of the resident kernel (all offsets in bytes, 16-byte aligned).
//
// Rows kept in LDS are stored by groups of 256 (LDS slot t = 256 k + lane is
// row k of lane `lane`), each group lane-major so that a wavefront's reads of
// one field are consecutive words and free of bank conflicts: the header
// (FP32: 256 eta_bar then 256 aux; FP64: 256 (eta_bar, aux) pairs), then
// DC / (16 / sizeof(Real)) slabs of 256 16-byte chunks of x. The last group
// is allocated whole. This is also the layout in which gfx950's
// global_load_lds (4 or 16 bytes per lane, lane-major at a wavefront base)
// deposits rows, so rows reach LDS without passing through registers.
constexpr int kResMaxLdsGroups = 16;
struct ResLayout {
  int nlds;       // rows held in LDS
  int row_bytes;  // (2 + DC) reals
  int off_rows, off_row0, off_blk, off_redv, off_reds, off_dl, off_flag, off_mat, total;
};

__host__ __device__ inline int res_align16(int x) { return (x + 15) & ~15; }

__host__ __device__ inline ResLayout res_layout(int m, int G, int dc, int rpl, int real_bytes, int d) {
  ResLayout L;
  L.row_bytes = (2 + dc) * real_bytes;
  L.nlds = m - kResLanes * rpl;
  if (L.nlds < 0) L.nlds = 0;
  const int rows_bytes = (L.nlds + kResLanes - 1) / kResLanes * kResLanes * L.row_bytes;
  int off = 0;
  L.off_rows = off; off = res_align16(off + rows_bytes);
  L.off_row0 = off; off = res_align16(off + (kHeader + dc) * real_bytes);
  L.off_blk = off; off = res_align16(off + ((m + G - 1) / G) * 4);
  L.off_redv = off; off = res_align16(off + kResWaves * kWave * 8);
  L.off_reds = off; off = res_align16(off + kResWaves * 2 * 8);
  L.off_dl = off; off = res_align16(off + dc * real_bytes);
  L.off_flag = off; off = res_align16(off + 16);
  L.off_mat = off; off = res_align16(off + 5 * dc * dc * 8);  // C, Q0, Sigma, K Sigma, Linv
  L.total = off;
  return L;
}

// y_c = sum_e M_ce x_e for a d x d matrix stored transposed in LDS with
// column stride DC and zero padding to DC x DC (M_ce at MT[e*DC + c]), x_e
// held by lane e of the wavefront (zero for e >= d); lanes c >= d get 0. The
// reads are unconditional, so they issue together.
template <int DC>
__device__ __forceinline__ double lds_matvec(const double* MT, int d, double x, int lane) {
  double acc = 0.0;
  const int r = lane < DC ? lane : 0;
#pragma unroll
  for (int e = 0; e < DC; ++e) acc += MT[e * DC + r] * readlane_d(x, e);
  return lane < d ? acc : 0.0;
}

// Two products of one vector in one sweep: AT (transposed A) is followed by
// BT (transposed B), both padded as above; lane c < d returns (A x)_c, lane
// 32 + c returns (B x)_c.
template <int DC>
__device__ __forceinline__ double lds_matvec2(const double* AT, int d, double x, int lane) {
  const int c = lane & 31;
  const double* base = AT + (lane >> 5) * DC * DC;
  const int r = c < DC ? c : 0;
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < DC; ++e) acc += base[e * DC + r] * readlane_d(x, e);
  return c < d ? acc : 0.0;
}

// Lane l < 32 receives the value of lane l + 32.
__device__ __forceinline__ double from_upper_half(double y) {
  uint32_t a0, b0, a1, b1;
  xl::swap_words<0>(xl::lo_word(y), xl::lo_word(y), a0, b0);
  xl::swap_words<0>(xl::hi_word(y), xl::hi_word(y), a1, b1);
  return xl::make_double(b0, b1);
}

template <typename Real, int DC>
struct ResRow {
  Real eb, aux;
  Real x[DC];
};

// Lane `lane`'s slots in the LDS row groups (see ResLayout).
template <typename Real, int DC>
struct LdsSlots {
  static constexpr int kPer = 16 / (int)sizeof(Real);  // reals per 16-byte chunk
  static constexpr int kChunks = DC / kPer;
  static constexpr int kHdrBytes = kResLanes * 2 * (int)sizeof(Real);
  static constexpr int kGroupBytes = kResLanes * (2 + DC) * (int)sizeof(Real);
  char* hdr0;  // group 0 header of this lane
  char* x0;    // group 0 chunk 0 of this lane
  __device__ __forceinline__ LdsSlots(char* rows, int lane)
      : hdr0(rows + lane * (sizeof(Real) == 4 ? 4 : 16)), x0(rows + kHdrBytes + lane * 16) {}
  __device__ __forceinline__ Real eb(int k) const { return *reinterpret_cast<const Real*>(hdr0 + k * kGroupBytes); }
  __device__ __forceinline__ Real aux(int k) const {
    return *reinterpret_cast<const Real*>(hdr0 + k * kGroupBytes + (sizeof(Real) == 4 ? kResLanes * 4 : 8));
  }
  __device__ __forceinline__ const uint4* chunk(int k, int q) const {
    return reinterpret_cast<const uint4*>(x0 + k * kGroupBytes + q * kResLanes * 16);
  }
};

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;

// Asynchronous copy of this lane's packed row g into LDS group k (waited for
// with vmcnt). The LDS base of each transfer is the wavefront's: group k +
// field offset + 64 * wave * size.
template <typename Real, int DC>
__device__ __forceinline__ void dma_row_to_lds(const Real* g, char* rows, int k, int wave) {
  using S = LdsSlots<Real, DC>;
  char* grp = rows + k * S::kGroupBytes;
  if constexpr (sizeof(Real) == 4) {
    const int o_eb = __builtin_amdgcn_readfirstlane(k * S::kGroupBytes + wave * kWave * 4);
    const int o_aux = __builtin_amdgcn_readfirstlane(k * S::kGroupBytes + kResLanes * 4 + wave * kWave * 4);
    __builtin_amdgcn_global_load_lds((glb_void_t*)g, (lds_void_t*)(rows + o_eb), 4, 0, 0);
    __builtin_amdgcn_global_load_lds((glb_void_t*)(g + 1), (lds_void_t*)(rows + o_aux), 4, 0, 0);
  } else {
    const int o_h = __builtin_amdgcn_readfirstlane(k * S::kGroupBytes + wave * kWave * 16);
    __builtin_amdgcn_global_load_lds((glb_void_t*)g, (lds_void_t*)(rows + o_h), 16, 0, 0);
  }
  (void)grp;
#pragma unroll
  for (int q = 0; q < S::kChunks; ++q) {
    const int o = __builtin_amdgcn_readfirstlane(k * S::kGroupBytes + S::kHdrBytes + q * kResLanes * 16 +
                                                 wave * kWave * 16);
    __builtin_amdgcn_global_load_lds((glb_void_t*)(g + kHeader + q * S::kPer), (lds_void_t*)(rows + o), 16, 0, 0);
  }
}

// Wait for all of this wavefront's outstanding global loads (LDS transfers
// included): s_waitcnt with vmcnt 0 and the expcnt / lgkmcnt fields at their
// maxima (gfx9 encoding), emitted as the instruction the compiler's own
// wait-count tracking knows.
__device__ __forceinline__ void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// the shift row (read by every lane): plain packed layout
template <typename Real, int DC>
__device__ __forceinline__ void copy_row_plain(const Real* __restrict__ g, Real* s) {
  const uint4* a = reinterpret_cast<const uint4*>(g);
  uint4* b = reinterpret_cast<uint4*>(s);
#pragma unroll
  for (int q = 0; q < (kHeader + DC) * (int)sizeof(Real) / 16; ++q) b[q] = a[q];
}

// Per-lane accumulation of one pass over the resident rows; CV is the order
// of the control variate.
template <typename Real, int DC, int FAM, int RPL, int CV>
__device__ __forceinline__ void resident_accumulate(const Prob& P, const ResRow<Real, DC> (&rr)[RPL > 0 ? RPL : 1],
                                                    char* lrows, int nlds, const Real* row0,
                                                    const Real* dsh, int tid, double& se, double& se2,
                                                    Real (&S1)[DC], Real (&T1)[DC], double& shift) {
  const int m = P.m;
  const Real inv_s2 = (Real)P.inv_s2;
  Real dl[DC];
#pragma unroll
  for (int c = 0; c < DC; ++c) dl[c] = dsh[c];
  auto eval = [&](Real eb, Real aux, const Real (&x)[DC], Real& dd, Real& dp) {
    Real D = Real(0);
#pragma unroll
    for (int c = 0; c < DC; ++c) D += x[c] * dl[c];
    cv_remainder<Real, FAM>(CV, eb, aux, D, inv_s2, dd, dp);
  };
  {
    Real x[DC];
#pragma unroll
    for (int c = 0; c < DC; ++c) x[c] = row0[kHeader + c];
    Real dd, dp;
    eval(row0[0], row0[1], x, dd, dp);
    shift = (double)dd;
  }
  se = 0.0;
  se2 = 0.0;
#pragma unroll
  for (int c = 0; c < DC; ++c) { S1[c] = Real(0); T1[c] = Real(0); }
  auto add = [&](const Real (&x)[DC], Real dd, Real dp) {
    const double e = (double)dd - shift;
    se += e;
    se2 += e * e;
    const Real edp = (Real)e * dp;
#pragma unroll
    for (int c = 0; c < DC; ++c) {
      S1[c] += dp * x[c];
      T1[c] += edp * x[c];
    }
  };
  // every register slot holds a row (the host launches RPL > 0 only when
  // m >= 256 RPL), so the rows need no lane predication; the uniform test
  // (always true) only keeps each row in a block of its own, so that rows are
  // not interleaved beyond what the register file holds
  const int nfull = (m / kResLanes < RPL) ? m / kResLanes : RPL;
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    if (r < nfull) {
      // one copy of the row into vector registers serves both contractions
      // (the empty asm marks the copy as a new value, so that it is not
      // re-read from the accumulation registers for the second)
      Real x[DC];
#pragma unroll
      for (int c = 0; c < DC; ++c) {
        x[c] = rr[r].x[c];
        asm("" : "+v"(x[c]));
      }
      Real dd, dp;
      eval(rr[r].eb, rr[r].aux, x, dd, dp);
      add(x, dd, dp);
    }
  }
  const LdsSlots<Real, DC> S(lrows, tid);
#pragma unroll 1
  for (int k = 0; k * kResLanes + tid < nlds; ++k) {
    Real x[DC];
#pragma unroll
    for (int q = 0; q < LdsSlots<Real, DC>::kChunks; ++q) {
      if constexpr (sizeof(Real) == 4) {
        const float4 v = *reinterpret_cast<const float4*>(S.chunk(k, q));
        x[4 * q] = v.x; x[4 * q + 1] = v.y; x[4 * q + 2] = v.z; x[4 * q + 3] = v.w;
      } else {
        const double2 v = *reinterpret_cast<const double2*>(S.chunk(k, q));
        x[2 * q] = v.x; x[2 * q + 1] = v.y;
      }
    }
    Real dd, dp;
    eval(S.eb(k), S.aux(k), x, dd, dp);
    add(x, dd, dp);
  }
}

// x'delta of this lane's row on the matrix core. v_mfma_f32_4x4x1f32 works
// on 16 blocks of 4 lanes: lane 4b + t receives D[i] += A(lane 4b + i) *
// B(lane 4b + t) for i = 0..3. With delta_c as A in every lane and the row's
// x_c as B (each lane its own row), every element of lane 4b + t's
// accumulator is sum_c delta_c x_t[c]: the row's linear predictor, with no
// exchange between lanes. Two accumulators (even and odd c) halve the chain
// of dependent products. The row stays in the registers it lives in (the
// matrix core reads VGPRs and AGPRs alike).
typedef float mfma_f4 __attribute__((ext_vector_type(4)));

template <int DC>
__device__ __forceinline__ float mfma_row_dot(const float (&dl)[DC], const float (&x)[DC]) {
  mfma_f4 a0 = {0.f, 0.f, 0.f, 0.f}, a1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < DC; c += 2) {
    a0 = __builtin_amdgcn_mfma_f32_4x4x1f32(dl[c], x[c], a0, 0, 0, 0);
    if (c + 1 < DC) a1 = __builtin_amdgcn_mfma_f32_4x4x1f32(dl[c + 1], x[c + 1], a1, 0, 0, 0);
  }
  return a0[0] + a1[0];
}

// resident_accumulate with x'delta formed on the matrix core (FP32 rows).
// Each row's product is issued one row ahead of the vector work on the row
// before it (remainder, S1, T1, the FP64 sums), so the matrix pipe runs beside
// the vector ALU. LDS rows are taken in whole groups of 256 (the last group
// is allocated whole; lanes past the LDS rows zero their row and add
// nothing), so every product runs with the full wavefront.
template <int DC, int FAM, int RPL, int CV>
__device__ __forceinline__ void resident_accumulate_mfma(const Prob& P, const ResRow<float, DC> (&rr)[RPL > 0 ? RPL : 1],
                                                         char* lrows, int nlds, const float* row0, const float* dsh,
                                                         int tid, double& se, double& se2, float (&S1)[DC],
                                                         float (&T1)[DC], double& shift) {
  const float inv_s2 = (float)P.inv_s2;
  float dl[DC];
#pragma unroll
  for (int c = 0; c < DC; ++c) dl[c] = dsh[c];
  {
    float x[DC];
#pragma unroll
    for (int c = 0; c < DC; ++c) x[c] = row0[kHeader + c];
    float D = 0.f;
#pragma unroll
    for (int c = 0; c < DC; ++c) D += x[c] * dl[c];
    float dd, dp;
    cv_remainder<float, FAM>(CV, row0[0], row0[1], D, inv_s2, dd, dp);
    shift = (double)dd;
  }
  se = 0.0;
  se2 = 0.0;
#pragma unroll
  for (int c = 0; c < DC; ++c) { S1[c] = 0.f; T1[c] = 0.f; }
  auto add = [&](const float (&x)[DC], float dd, float dp) {
    const double e = (double)dd - shift;
    se += e;
    se2 += e * e;
    const float edp = (float)e * dp;
#pragma unroll
    for (int c = 0; c < DC; ++c) {
      S1[c] += dp * x[c];
      T1[c] += edp * x[c];
    }
  };
  // register rows: every slot holds a row (the host launches RPL > 0 only
  // when m >= 256 RPL), so the rows need no test and run as one block, in
  // which the scheduler can overlap a row's product with the row before
  if constexpr (RPL > 0) {
    float Dn = mfma_row_dot<DC>(dl, rr[0].x);
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const float Dc = Dn;
      if (r + 1 < RPL) Dn = mfma_row_dot<DC>(dl, rr[r + 1 < RPL ? r + 1 : r].x);
      float x[DC];
#pragma unroll
      for (int c = 0; c < DC; ++c) {
        x[c] = rr[r].x[c];
        asm("" : "+v"(x[c]));
      }
      float dd, dp;
      cv_remainder<float, FAM, true>(CV, rr[r].eb, rr[r].aux, Dc, inv_s2, dd, dp);
      add(x, dd, dp);
    }
  }
  // LDS rows, whole groups, the next group's row and product one step ahead
  const LdsSlots<float, DC> S(lrows, tid);
  const int ngroups = (nlds + kResLanes - 1) / kResLanes;
  auto load = [&](int k, float (&x)[DC], float& eb, float& aux) {
    const bool ok = k * kResLanes + tid < nlds;
#pragma unroll
    for (int q = 0; q < LdsSlots<float, DC>::kChunks; ++q) {
      const float4 v = *reinterpret_cast<const float4*>(S.chunk(k, q));
      x[4 * q] = ok ? v.x : 0.f; x[4 * q + 1] = ok ? v.y : 0.f;
      x[4 * q + 2] = ok ? v.z : 0.f; x[4 * q + 3] = ok ? v.w : 0.f;
    }
    eb = ok ? S.eb(k) : 0.f;
    aux = ok ? S.aux(k) : 0.f;
  };
  if (ngroups > 0) {
    float xn[DC], ebn, auxn;
    load(0, xn, ebn, auxn);
    float Dn = mfma_row_dot<DC>(dl, xn);
#pragma unroll 1
    for (int k = 0; k < ngroups; ++k) {
      float x[DC];
#pragma unroll
      for (int c = 0; c < DC; ++c) x[c] = xn[c];
      const float eb = ebn, aux = auxn, Dc = Dn;
      if (k + 1 < ngroups) {
        load(k + 1, xn, ebn, auxn);
        Dn = mfma_row_dot<DC>(dl, xn);
      }
      if (k * kResLanes + tid < nlds) {
        float dd, dp;
        cv_remainder<float, FAM, true>(CV, eb, aux, Dc, inv_s2, dd, dp);
        add(x, dd, dp);
      }
    }
  }
}

template <typename Real, int DC, int FAM, int RPL, int MF>
__device__ __forceinline__ void move_res_body(const MoveArgs& A, const ResLayout& Ly, const int i) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  char* lrows = smem + Ly.off_rows;
  Real* row0 = reinterpret_cast<Real*>(smem + Ly.off_row0);
  int32_t* blk = reinterpret_cast<int32_t*>(smem + Ly.off_blk);
  double* redv = reinterpret_cast<double*>(smem + Ly.off_redv);
  double* reds = reinterpret_cast<double*>(smem + Ly.off_reds);
  Real* dsh = reinterpret_cast<Real*>(smem + Ly.off_dl);
  int* flag = reinterpret_cast<int*>(smem + Ly.off_flag);

  const Prob& P = A.P;
  if (i >= P.M) return;
  const int tid = threadIdx.x;
  const int w = tid / kWave, lane = tid % kWave;
  const int d = P.d;
  const int m = P.m;
  const int ld = P.ld;
  const double a = A.a;
  const double eps = A.eps;
  const Real* __restrict__ X = static_cast<const Real*>(P.X);
  int32_t* urow = A.u + (int64_t)i * m;
  const bool lead = (w == 0);

  // the small matrices of the move, stored transposed with column stride DC
  // (element (r, c) at c*DC + r) so that lanes c = 0..d-1 read consecutive
  // words at compile-time offsets: C, Q0, Sigma and, below, (a C - Q0)
  // Sigma; then Linv' (the momentum draw p = Linv' z)
  constexpr int kM = DC * DC;
  double* Cm = reinterpret_cast<double*>(smem + Ly.off_mat);
  double* Qm = Cm + kM;
  double* Sm = Qm + kM;   // Sigma, then K Sigma right below it
  double* KSm = Sm + kM;
  double* LTm = KSm + kM;
  for (int o = tid; o < kM; o += kResLanes) {
    const int r = o / DC, c = o - r * DC;  // element (r, c) of the padded matrices
    const bool in = r < d && c < d;
    const int g = in ? r * d + c : 0;
    Cm[c * DC + r] = in ? P.cvC[g] : 0.0;
    Qm[c * DC + r] = in ? P.Q0[g] : 0.0;
    Sm[c * DC + r] = in ? P.Sigma[g] : 0.0;
    LTm[r * DC + c] = in ? P.Linv[g] : 0.0;
  }

  // wave 0 state (component c in lane c)
  double tb = 0.0, th = 0.0, gl0 = 0.0, gs0 = 0.0, mu0l = 0.0, bl = 0.0;
  if (lead && lane < d) {
    tb = P.theta_bar[lane];
    mu0l = P.mu0[lane];
    bl = P.cvB[lane];
    th = A.theta[(int64_t)i * d + lane];
    gl0 = A.grad_l[(int64_t)i * d + lane];
    gs0 = A.grad_s[(int64_t)i * d + lane];
  }
  double lh0 = A.lhat[i], sg0 = A.sig2[i];

  // ---- the proposed block of the pseudo-marginal refresh
  const uint64_t cg = stream_ctr0(kBlockChoice, A.stage, A.move, P.dataset);
  const int g = (int)word_to_index(stream_word(P.seed, cg, (uint64_t)i, 0), (uint64_t)P.G);
  const int b0 = (int)((int64_t)g * m / P.G);
  const int b1 = (int)((int64_t)(g + 1) * m / P.G);
  const uint64_t cb = stream_ctr0(kBlockIndex, A.stage, A.move, P.dataset);
  for (int t = tid; t < b1 - b0; t += kResLanes)
    blk[t] = (int32_t)word_to_index(stream_word(P.seed, cb, (uint64_t)i, (uint64_t)t), (uint64_t)P.n);
  __syncthreads();
  // K = a C - Q0 (a first-order control variate has no C delta term)
  const double ac = (P.cv_order == 2) ? a : 0.0;
  for (int o = tid; o < kM; o += kResLanes) {
    const int r = o / DC, c = o - r * DC;
    double acc = 0.0;
    for (int f = 0; f < d; ++f) acc += (ac * Cm[f * DC + r] - Qm[f * DC + r]) * Sm[c * DC + f];
    KSm[c * DC + r] = acc;  // zero outside d x d: the padded entries of C, Q0, Sigma are 0
  }
  const uint32_t n = (uint32_t)P.n;
  // indices of u* (refreshed block) or of u; a caller index outside [0, n)
  // reads row 0 and poisons the estimator
  auto index_star = [&](int j) -> int32_t {
    const bool in = (unsigned)(j - b0) < (unsigned)(b1 - b0);
    const int32_t gk = urow[j];
    const int32_t lk = blk[in ? j - b0 : 0];
    return in ? lk : gk;
  };
  bool poisoned = false;
  auto load_reg = [&](ResRow<Real, DC>& r, int32_t k) {
    const bool bad = (uint32_t)k >= n;
    poisoned |= bad;
    RowLoad<Real, DC> t;
    load_row<Real, DC>(X + (int64_t)(bad ? 0 : k) * ld, t);
    r.eb = t.eb;
    r.aux = t.aux;
#pragma unroll
    for (int c = 0; c < DC; ++c) r.x[c] = t.x[c];
  };
  auto load_lds = [&](int grp, int32_t k) {
    const bool bad = (uint32_t)k >= n;
    poisoned |= bad;
    dma_row_to_lds<Real, DC>(X + (int64_t)(bad ? 0 : k) * ld, lrows, grp, w);
  };
  auto load_row0 = [&](int32_t k) {
    const bool bad = (uint32_t)k >= n;
    poisoned |= bad;
    copy_row_plain<Real, DC>(X + (int64_t)(bad ? 0 : k) * ld, row0);
  };

  // gather: every subsample index first (slots past m read a valid entry
  // and are never used), then the rows (LDS slots by direct transfers,
  // register slots by loads), then one wait
  const int ngroups = (Ly.nlds + kResLanes - 1) / kResLanes;
  auto u_at = [&](int j) -> int32_t { return urow[j < m ? j : m - 1]; };
  auto refreshed = [&](int j, int32_t gk) -> int32_t {
    const bool in = (unsigned)(j - b0) < (unsigned)(b1 - b0);
    const int32_t lk = blk[in ? j - b0 : 0];
    return in ? lk : gk;
  };
  int32_t kx_lds[kResMaxLdsGroups];
#pragma unroll
  for (int k = 0; k < kResMaxLdsGroups; ++k)
    if (k < ngroups) kx_lds[k] = u_at(kResLanes * (RPL + k) + tid);
  int32_t kx_reg[RPL > 0 ? RPL : 1];
#pragma unroll
  for (int r = 0; r < RPL; ++r) kx_reg[r] = u_at(kResLanes * r + tid);
  wait_vm();
#pragma unroll
  for (int k = 0; k < kResMaxLdsGroups; ++k)
    if (k < ngroups) kx_lds[k] = refreshed(kResLanes * (RPL + k) + tid, kx_lds[k]);
#pragma unroll
  for (int r = 0; r < RPL; ++r) kx_reg[r] = refreshed(kResLanes * r + tid, kx_reg[r]);
#pragma unroll
  for (int k = 0; k < kResMaxLdsGroups; ++k) {
    if (k < ngroups) {
      if (k * kResLanes + tid < Ly.nlds) load_lds(k, kx_lds[k]);
    }
  }
  ResRow<Real, DC> rr[RPL > 0 ? RPL : 1];
#pragma unroll
  for (int r = 0; r < RPL; ++r) load_reg(rr[r], kx_reg[r]);
  if (tid == 0) load_row0(index_star(0));
  wait_vm();
  // poisoned rows (caller index out of range) make every pass NaN; the
  // barrier also publishes the LDS rows
  int bad = __syncthreads_or(poisoned ? 1 : 0);

  const double nm = P.n_over_m;
  const double md = (double)m;
  const int L = A.L;
  // wave 0 leapfrog state
  double delta = th - tb;   // theta - theta_bar of the current pass
  double th1 = th;          // theta of the current pass
  double p = 0.0, kd = 0.0, g0 = 0.0, H0 = 0.0, cdel0 = 0.0, lp1 = 0.0;
  double lhat_r = 0.0, sig2_r = 0.0, gl_r = 0.0, gs_r = 0.0;
  // theta <- theta + eps Sigma p, K delta <- K delta + eps K Sigma p
  auto drift = [&]() {
    const double y = lds_matvec2<DC>(Sm, d, p, lane);
    const double ky = from_upper_half(y);
    if (lane < d) {
      delta += eps * y;
      th1 += eps * y;
      kd += eps * ky;
    }
  };

  // pass 0: the u-refresh at theta; passes 1..L: the leapfrog positions
  for (int l = 0; l <= L; ++l) {
    if (lead && lane < DC) dsh[lane] = (Real)delta;
    __syncthreads();
    double se, se2, shift;
    Real S1[DC], T1[DC];
    if constexpr (MF != 0 && sizeof(Real) == 4) {
      if (P.cv_order == 2)
        resident_accumulate_mfma<DC, FAM, RPL, 2>(P, rr, lrows, Ly.nlds, row0, dsh, tid, se, se2, S1, T1, shift);
      else
        resident_accumulate_mfma<DC, FAM, RPL, 1>(P, rr, lrows, Ly.nlds, row0, dsh, tid, se, se2, S1, T1, shift);
    } else {
      if (P.cv_order == 2)
        resident_accumulate<Real, DC, FAM, RPL, 2>(P, rr, lrows, Ly.nlds, row0, dsh, tid, se, se2, S1, T1, shift);
      else
        resident_accumulate<Real, DC, FAM, RPL, 1>(P, rr, lrows, Ly.nlds, row0, dsh, tid, se, se2, S1, T1, shift);
    }
    const bool full = (l == 0 || l == L);  // estimator value needed (not only the gradient)
    se = xl::wave_allsum(se);
    if (full) se2 = xl::wave_allsum(se2);
    Real v[2 * DC];
#pragma unroll
    for (int c = 0; c < DC; ++c) {
      v[c] = S1[c];
      v[DC + c] = T1[c];
    }
    xl::reduce_scatter<Real, 2 * DC, 0>(v, lane);
    const int comp = xl::scatter_index<2 * DC>(lane);
    if (comp >= 0) redv[w * kWave + comp] = (double)v[0];
    if (lane == 0) {
      reds[2 * w] = se;
      reds[2 * w + 1] = se2;
    }
    __syncthreads();
    if (lead) {
      double tse = 0.0, tse2 = 0.0, s1c = 0.0, t1c = 0.0;
#pragma unroll
      for (int q = 0; q < kResWaves; ++q) {
        tse += reds[2 * q];
        tse2 += reds[2 * q + 1];
        const int c = lane < DC ? lane : 0;
        s1c += redv[q * kWave + c];
        t1c += redv[q * kWave + DC + c];
      }
      if (bad) tse = tse2 = __builtin_nan("");
      const double dbms = tse / md;
      if (full) {
        // the estimator and both gradients at delta
        const double m2 = tse2 - tse * dbms;
        const double dhat = nm * (tse + md * shift);
        sig2_r = nm * nm * (m2 < 0.0 ? 0.0 : m2);
        const double cdel = lds_matvec<DC>(Cm, d, delta, lane);
        const double qpart = (P.cv_order == 2) ? (bl * delta + 0.5 * delta * cdel) : bl * delta;
        lhat_r = P.cvA[0] + xl::wave_allsum(qpart) + dhat;
        gl_r = lane < d ? bl + (P.cv_order == 2 ? cdel : 0.0) + nm * s1c : 0.0;
        gs_r = lane < d ? 2.0 * nm * nm * (t1c - dbms * s1c) : 0.0;
        if (l == 0) {
          cdel0 = cdel;
        } else {
          // closing half step at theta_L
          const double dm = lane < d ? th1 - mu0l : 0.0;
          const double rq = lds_matvec<DC>(Qm, d, dm, lane);
          lp1 = xl::wave_allsum(-0.5 * dm * rq);
          p += 0.5 * eps * (a * gl_r - 0.5 * a * a * gs_r - rq);
        }
      } else {
        const double grad = lane < d ? g0 + kd + a * nm * s1c - a * a * nm * nm * (t1c - dbms * s1c) : 0.0;
        p += eps * grad;
        drift();
      }
    }
    if (l == 0) {
      // ---- 1. u | theta
      if (lead) {
        const double lam0 = a * lh0 - 0.5 * a * a * sg0;
        const double lam1 = a * lhat_r - 0.5 * a * a * sig2_r;
        const double logr = lam1 - lam0;
        const double logU =
            log(word_to_uniform(stream_word(P.seed, stream_ctr0(kUAccept, A.stage, A.move, P.dataset), (uint64_t)i, 0)));
        const bool acc = isfinite(logr) && (logU < logr);
        if (lane == 0) {
          flag[0] = acc ? 1 : 0;
          A.accept[2 * i] = acc ? 1 : 0;
          record_decision(A, i, 0, logU, logr);
        }
        if (acc) {
          lh0 = lhat_r; sg0 = sig2_r; gl0 = gl_r; gs0 = gs_r;
        }
      }
      __syncthreads();
      const bool acc_u = flag[0] != 0;
      if (acc_u) {
        for (int t = tid; t < b1 - b0; t += kResLanes) urow[b0 + t] = blk[t];
      } else {
        // restore the rows of the current block from u
        poisoned = false;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
          const int j = tid + kResLanes * r;
          if (j >= b0 && j < b1) load_reg(rr[r], urow[j]);
          else poisoned |= (uint32_t)urow[j] >= n;
        }
        for (int k = 0; k < ngroups; ++k) {
          const int j = kResLanes * (RPL + k) + tid;
          if (j < kResLanes * RPL + Ly.nlds) {
            if (j >= b0 && j < b1) load_lds(k, urow[j]);
            else poisoned |= (uint32_t)urow[j] >= n;
          }
        }
        if (tid == 0 && b0 == 0 && b1 > 0) load_row0(urow[0]);
        wait_vm();
        bad = __syncthreads_or(poisoned ? 1 : 0);
      }
      // ---- 2. theta | u: HMC from (theta, u), opening half step and drift
      if (lead) {
        const uint64_t cm = stream_ctr0(kMomentum, A.stage, A.move, P.dataset);
        const double z = lane < d ? stream_normal(P.seed, cm, (uint64_t)i, (uint32_t)lane) : 0.0;
        p = lds_matvec<DC>(LTm, d, z, lane);  // Linv is lower triangular
        const double sp = lds_matvec<DC>(Sm, d, p, lane);
        const double K0 = 0.5 * xl::wave_allsum(p * sp);
        const double dm = lane < d ? th - mu0l : 0.0;
        const double rq = lds_matvec<DC>(Qm, d, dm, lane);
        const double lp = xl::wave_allsum(-0.5 * dm * rq);
        H0 = -((a * lh0 - 0.5 * a * a * sg0) + lp) + K0;
        p += 0.5 * eps * (a * gl0 - 0.5 * a * a * gs0 - rq);
        lp1 = lp;
        lhat_r = lh0; sig2_r = sg0; gl_r = gl0; gs_r = gs0;
        // constant and linear parts of the gradient along the trajectory
        const double qb = lds_matvec<DC>(Qm, d, tb - mu0l, lane);
        g0 = lane < d ? a * bl - qb : 0.0;
        kd = lane < d ? ac * cdel0 - (rq - qb) : 0.0;
        drift();
      }
      // (the next pass starts with a barrier)
    }
  }
  if (lead) {
    const double sp = lds_matvec<DC>(Sm, d, p, lane);
    const double K1 = 0.5 * xl::wave_allsum(p * sp);
    const double logpi1 = (a * lhat_r - 0.5 * a * a * sig2_r) + lp1;
    const double H1 = -logpi1 + K1;
    const double logr = H0 - H1;
    const double logU =
        log(word_to_uniform(stream_word(P.seed, stream_ctr0(kThetaAccept, A.stage, A.move, P.dataset), (uint64_t)i, 0)));
    const bool acc = isfinite(logr) && (logU < logr);
    if (acc) {
      th = th1; lh0 = lhat_r; sg0 = sig2_r; gl0 = gl_r; gs0 = gs_r;
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
}

template <typename Real, int DC, int FAM, int RPL, int MF>
__global__ void __launch_bounds__(kResLanes) move_kernel_res(MoveArgs A, ResLayout Ly) {
  move_res_body<Real, DC, FAM, RPL, MF>(A, Ly, xcd_particle((int)blockIdx.x, (int)gridDim.x));
}

// a batch member of the resident move: its arguments and its on-chip layout
// (the launch reserves the largest member's LDS)
struct ResMoveArgs {
  MoveArgs A;
  ResLayout Ly;
};

template <typename Real, int DC, int FAM, int RPL, int MF>
__global__ void __launch_bounds__(kResLanes) move_kernel_res_batch(Batch<ResMoveArgs> B) {
  const int k = batch_member(B.first, B.count, blockIdx.x);
  const ResMoveArgs R = B.args[k];
  move_res_body<Real, DC, FAM, RPL, MF>(R.A, R.Ly, xcd_particle((int)blockIdx.x - B.first[k], B.first[k + 1] - B.first[k]));
}

}  // namespace subsmc

