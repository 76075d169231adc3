// Host side of the C ABI declared in include/subsmc.h: workspace layout,
// argument checks, kernel dispatch and the Newton iteration for the
// control-variate centre.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/subsmc.h"
#include "kernels.hpp"
#include "kernels_wide.hpp"
#include "kernels_resident.hpp"

using namespace subsmc;

namespace {

constexpr int kMaxNarrowD = 32;   // one lane per row up to here
constexpr int kMaxD = 128;        // lane groups per row beyond
constexpr int kMaxM = kTemperThreads * kTemperPer;
constexpr int kCvMaxBlocks = 768;   // 3 workgroups per CU

// rows per CV tile: up to one per thread, the whole LDS carve within 56 KB
// (d = 128 needs 32 rows and 102 KB)
int cv_tile_rows(int d) {
  int r = kCvThreads;
  while (r > 32 && cv_lds_bytes(d, r) > 56 * 1024) r -= 32;
  return r;
}
constexpr int kMaxBlock = 16384;  // slots per refreshed block (LDS)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int pad_dc(int d) { return (d + 3) & ~3; }

// Lanes per row and elements per lane for d > 32 (see kernels_wide.hpp).
struct WideShape { int G, CH; };
WideShape wide_shape(int d, bool fp32) {
  const int vw = fp32 ? 4 : 2;
  const int G = (d + kHeader <= 4 * 16) ? 4 : 8;
  int ch = (d + kHeader + G - 1) / G;
  ch = (ch + vw - 1) / vw * vw;
  return {G, ch};
}

int packed_ld(int d, bool fp32) {
  const int per64 = fp32 ? 16 : 8;
  int need = kHeader + pad_dc(d);
  if (d > kMaxNarrowD) {
    const WideShape w = wide_shape(d, fp32);
    need = w.G * w.CH;
  }
  return (need + per64 - 1) / per64 * per64;
}

// Workspace regions, in carve order.
struct Layout {
  size_t Xp, theta_bar, cvA, cvB, cvC, mu0, Q0, Qw, L0, L0inv, Sigma, Lchol, Linv, mean, status,
      tout, grid, aconst, scratch_theta, grad_l, grad_s, anc, th2, u2, lh2, sg2, gl2, gs2, partials, mpartials, total;
  int ld;
  int cv_blocks, cv_rows;
  int mom_blocks;
};

bool compute_layout(const smc_problem* pb, Layout& L) {
  const bool fp32 = pb->precision == SMC_MIXED;
  const size_t es = fp32 ? 4 : 8;
  const int d = pb->d;
  const size_t M = pb->M, m = pb->m, n = (size_t)pb->n;
  L.ld = packed_ld(d, fp32);
  L.cv_rows = cv_tile_rows(d);
  const int64_t ntiles = (pb->n + L.cv_rows - 1) / L.cv_rows;
  L.cv_blocks = (int)(ntiles < kCvMaxBlocks ? ntiles : kCvMaxBlocks);
  const size_t ne = 1 + d + (size_t)d * (d + 1) / 2;
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off = align256(off + bytes); return o; };
  const size_t dd = (size_t)d * d * 8;
  L.Xp = take(n * L.ld * es);
  L.theta_bar = take(d * 8);
  L.cvA = take(8);
  L.cvB = take(d * 8);
  L.cvC = take(dd);
  L.mu0 = take(d * 8);
  L.Q0 = take(dd);
  L.Qw = take(dd);
  L.L0 = take(dd);
  L.L0inv = take(dd);
  L.Sigma = take(dd);
  L.Lchol = take(dd);
  L.Linv = take(dd);
  L.mean = take(d * 8);
  L.status = take(4 * 8);
  L.tout = take(8 * 8);
  L.grid = take((size_t)kGridMax * 8);
  L.aconst = take(8);
  L.scratch_theta = take(d * 8);
  L.grad_l = take(M * d * 8);
  L.grad_s = take(M * d * 8);
  L.anc = take(M * 4);
  L.th2 = take(M * d * 8);
  L.u2 = take(M * m * 4);
  L.lh2 = take(M * 8);
  L.sg2 = take(M * 8);
  L.gl2 = take(M * d * 8);
  L.gs2 = take(M * d * 8);
  L.partials = take((size_t)L.cv_blocks * ne * 8);
  L.mom_blocks = (pb->M + kMomTile - 1) / kMomTile;
  L.mpartials = take((size_t)L.mom_blocks * (d + (size_t)d * (d + 1) / 2) * 8);
  L.total = off;
  return true;
}

}  // namespace

struct smc_ctx_s {
  smc_problem pb;
  hipStream_t stream = nullptr;
  Layout lay;
  char* ws = nullptr;
  Prob prob;
  double a = 0.0, logz = 0.0;
  int stage = 0, move = 0, have_mass = 0, newton_iters = 0;
  int res_rpl = -1;  // register rows per lane of the resident move kernel; -1: streaming
  ResLayout res_ly{};
  std::vector<double> mu0, Q0;
  char err[512] = {0};

  template <typename T> T* at(size_t off) { return reinterpret_cast<T*>(ws + off); }
};

namespace {

smc_status fail(smc_ctx c, smc_status s, const char* fmt, ...) {
  if (c) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->err, sizeof(c->err), fmt, ap);
    va_end(ap);
  }
  return s;
}

#define HIP_TRY(ctx, expr)                                                                      \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return fail(ctx, SMC_ERR_DEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),   \
                  __FILE__, __LINE__);                                                          \
  } while (0)

#define LAUNCH_CHECK(ctx) HIP_TRY(ctx, hipGetLastError())

smc_status validate(const smc_problem* pb) {
  if (!pb) return SMC_ERR_INVALID_ARG;
  if (pb->family < 0 || pb->family > 3) return SMC_ERR_INVALID_ARG;
  if (pb->precision != SMC_FP64 && pb->precision != SMC_MIXED) return SMC_ERR_INVALID_ARG;
  if (pb->cv_order != 1 && pb->cv_order != 2) return SMC_ERR_INVALID_ARG;
  if (pb->d < 1 || pb->n < 1 || pb->n >= (int64_t(1) << 31)) return SMC_ERR_INVALID_ARG;
  if (pb->ld < pb->d + 1 || !pb->Xy) return SMC_ERR_INVALID_ARG;
  if (pb->M < 1 || pb->M > kMaxM || pb->m < 1 || pb->G < 1 || pb->G > pb->m) return SMC_ERR_INVALID_ARG;
  if (!(pb->ess_frac > 0.0 && pb->ess_frac <= 1.0)) return SMC_ERR_INVALID_ARG;
  if (pb->move_path < SMC_MOVE_AUTO || pb->move_path > SMC_MOVE_RESIDENT) return SMC_ERR_INVALID_ARG;
  if ((pb->m + pb->G - 1) / pb->G > kMaxBlock) return SMC_ERR_UNSUPPORTED;
  if (!pb->prior_mean || !pb->prior_prec) return SMC_ERR_INVALID_ARG;
  if (!pb->theta || !pb->u || !pb->logw || !pb->lhat || !pb->sig2 || !pb->accept || !pb->workspace)
    return SMC_ERR_INVALID_ARG;
  if (pb->family == SMC_GAUSSIAN && !(pb->gauss_s2 > 0.0)) return SMC_ERR_INVALID_ARG;
  if (pb->d > kMaxD) return SMC_ERR_UNSUPPORTED;
  if (pb->d > kMaxNarrowD && pb->family == SMC_GAUSSIAN) return SMC_ERR_UNSUPPORTED;
  return SMC_OK;
}

// ------------------------------------------------------------------------
// kernel dispatch on (precision, padded d)
// ------------------------------------------------------------------------

template <typename Real, int FAM>
hipError_t launch_estimator_t(int dc, int count, const EstArgs& a, hipStream_t s) {
  switch (dc) {
#define CASE(DC) case DC: hipLaunchKernelGGL((estimator_kernel<Real, DC, FAM>), dim3(count), dim3(kWave), 0, s, a); break;
    CASE(4) CASE(8) CASE(12) CASE(16) CASE(20) CASE(24) CASE(28) CASE(32)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename Real, int FAM>
hipError_t launch_move_t(int dc, int M, size_t lds, const MoveArgs& a, hipStream_t s) {
  switch (dc) {
#define CASE(DC) case DC: hipLaunchKernelGGL((move_kernel<Real, DC, FAM>), dim3(M), dim3(kWave), lds, s, a); break;
    CASE(4) CASE(8) CASE(12) CASE(16) CASE(20) CASE(24) CASE(28) CASE(32)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_estimator_p(int fam, int dc, int count, const EstArgs& a, hipStream_t s) {
  switch (fam) {
    case kLogistic: return launch_estimator_t<Real, kLogistic>(dc, count, a, s);
    case kPoisson: return launch_estimator_t<Real, kPoisson>(dc, count, a, s);
    case kStudentT: return launch_estimator_t<Real, kStudentT>(dc, count, a, s);
    default: return launch_estimator_t<Real, kGaussian>(dc, count, a, s);
  }
}

template <typename Real>
hipError_t launch_move_p(int fam, int dc, int M, size_t lds, const MoveArgs& a, hipStream_t s) {
  switch (fam) {
    case kLogistic: return launch_move_t<Real, kLogistic>(dc, M, lds, a, s);
    case kPoisson: return launch_move_t<Real, kPoisson>(dc, M, lds, a, s);
    case kStudentT: return launch_move_t<Real, kStudentT>(dc, M, lds, a, s);
    default: return launch_move_t<Real, kGaussian>(dc, M, lds, a, s);
  }
}

// wide kernels: (precision, G, CH) instantiated for the shapes wide_shape() produces
#define WIDE_SHAPES(X)                                                      \
  X(float, 4, 12) X(float, 4, 16) X(float, 8, 12) X(float, 8, 16) X(float, 8, 20) \
  X(double, 4, 10) X(double, 4, 12) X(double, 4, 14) X(double, 4, 16)             \
  X(double, 8, 10) X(double, 8, 12) X(double, 8, 14) X(double, 8, 16) X(double, 8, 18)

template <typename Real, int G, int CH>
hipError_t launch_wide_est_fam(int fam, int count, const EstArgs& a, hipStream_t s) {
  if (fam == kLogistic)
    hipLaunchKernelGGL((estimator_kernel_wide<Real, G, CH, kLogistic>), dim3(count), dim3(kWave), 0, s, a);
  else if (fam == kPoisson)
    hipLaunchKernelGGL((estimator_kernel_wide<Real, G, CH, kPoisson>), dim3(count), dim3(kWave), 0, s, a);
  else if (fam == kStudentT)
    hipLaunchKernelGGL((estimator_kernel_wide<Real, G, CH, kStudentT>), dim3(count), dim3(kWave), 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename Real, int G, int CH>
hipError_t launch_wide_move_fam(int fam, int M, size_t lds, const MoveArgs& a, hipStream_t s) {
  if (fam == kLogistic)
    hipLaunchKernelGGL((move_kernel_wide<Real, G, CH, kLogistic>), dim3(M), dim3(kWave), lds, s, a);
  else if (fam == kPoisson)
    hipLaunchKernelGGL((move_kernel_wide<Real, G, CH, kPoisson>), dim3(M), dim3(kWave), lds, s, a);
  else if (fam == kStudentT)
    hipLaunchKernelGGL((move_kernel_wide<Real, G, CH, kStudentT>), dim3(M), dim3(kWave), lds, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_wide_estimator(smc_ctx c, int count, const EstArgs& a) {
  const bool fp32 = c->pb.precision == SMC_MIXED;
  const WideShape w = wide_shape(c->pb.d, fp32);
#define X(T, G_, CH_) \
  if ((sizeof(T) == 4) == fp32 && w.G == G_ && w.CH == CH_) return launch_wide_est_fam<T, G_, CH_>(c->pb.family, count, a, c->stream);
  WIDE_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_wide_move(smc_ctx c, size_t lds, const MoveArgs& a) {
  const bool fp32 = c->pb.precision == SMC_MIXED;
  const WideShape w = wide_shape(c->pb.d, fp32);
#define X(T, G_, CH_) \
  if ((sizeof(T) == 4) == fp32 && w.G == G_ && w.CH == CH_) return launch_wide_move_fam<T, G_, CH_>(c->pb.family, c->pb.M, lds, a, c->stream);
  WIDE_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

// resident move kernels: (precision, padded d, family, register rows per lane)
#define RES_SHAPES(X)                                                                                  \
  X(float, 4, 1, 0) X(float, 4, 1, 14) X(float, 8, 1, 0) X(float, 8, 1, 14) X(float, 12, 1, 0)          \
  X(float, 12, 1, 14) X(float, 16, 1, 0) X(float, 16, 1, 14) X(float, 20, 1, 0) X(float, 20, 1, 14)     \
  X(float, 24, 1, 0) X(float, 4, 0, 0) X(float, 8, 0, 0) X(float, 12, 0, 0) X(float, 16, 0, 0)          \
  X(float, 20, 0, 0) X(float, 24, 0, 0)                                                                 \
  X(double, 4, 0, 0) X(double, 8, 0, 0) X(double, 12, 0, 0) X(double, 16, 0, 0) X(double, 20, 0, 0)     \
  X(double, 24, 0, 0) X(double, 4, 1, 0) X(double, 8, 1, 0) X(double, 12, 1, 0) X(double, 16, 1, 0)     \
  X(double, 20, 1, 0) X(double, 24, 1, 0)

template <typename Real, int DC, int FAM, int RPL>
hipError_t launch_res(int M, const ResLayout& ly, const MoveArgs& a, hipStream_t s) {
  auto k = move_kernel_res<Real, DC, FAM, RPL>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                     ly.total);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(M), dim3(kResLanes), ly.total, s, a, ly);
  return hipGetLastError();
}

// register-row candidates for (precision, padded d, family): the ones
// instantiated above (the logistic remainder needs the registers the row
// cache would use, so logistic keeps all rows in LDS)
int res_candidates(bool fp32, int dc, int family, int out[2]) {
  if (dc > 24) return 0;
  out[0] = 0;
  if (fp32 && family == SMC_POISSON && dc <= 20) { out[1] = 14; return 2; }
  return 1;
}

// Smallest register-row count whose LDS part fits; -1 if the resident kernel
// does not apply.
int choose_resident(const smc_problem& pb, int max_lds, ResLayout& ly) {
  if (pb.d > kMaxNarrowD || (pb.family != SMC_LOGISTIC && pb.family != SMC_POISSON)) return -1;
  const bool fp32 = pb.precision == SMC_MIXED;
  const int dc = pad_dc(pb.d);
  int cand[2];
  const int nc = res_candidates(fp32, dc, pb.family, cand);
  for (int q = 0; q < nc; ++q) {
    const ResLayout l = res_layout(pb.m, pb.G, dc, cand[q], fp32 ? 4 : 8, pb.d);
    // register rows are unpredicated in the kernel: every slot must hold a row
    const bool regs_full = pb.m >= kResLanes * cand[q];
    if (regs_full && l.total <= max_lds && (l.nlds + kResLanes - 1) / kResLanes <= kResMaxLdsGroups) {
      ly = l;
      return cand[q];
    }
  }
  return -1;
}

hipError_t launch_resident(smc_ctx c, const MoveArgs& a) {
  const bool fp32 = c->pb.precision == SMC_MIXED;
  const int dc = pad_dc(c->pb.d);
#define X(T, DC_, FAM_, RPL_)                                                                    \
  if ((sizeof(T) == 4) == fp32 && dc == DC_ && c->pb.family == FAM_ && c->res_rpl == RPL_)        \
    return launch_res<T, DC_, FAM_, RPL_>(c->pb.M, c->res_ly, a, c->stream);
  RES_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_estimator(smc_ctx c, int count, const EstArgs& a) {
  if (count <= 0) return hipSuccess;
  if (c->pb.d > kMaxNarrowD) return launch_wide_estimator(c, count, a);
  const int dc = pad_dc(c->pb.d);
  return c->pb.precision == SMC_MIXED ? launch_estimator_p<float>(c->pb.family, dc, count, a, c->stream)
                                      : launch_estimator_p<double>(c->pb.family, dc, count, a, c->stream);
}

size_t block_lds_bytes(const smc_problem& pb) {
  return (size_t)((pb.m + pb.G - 1) / pb.G) * sizeof(int32_t);
}

hipError_t launch_move(smc_ctx c, const MoveArgs& a) {
  if (c->res_rpl >= 0) return launch_resident(c, a);
  const int dc = pad_dc(c->pb.d);
  const size_t lds = block_lds_bytes(c->pb);
  if (c->pb.d > kMaxNarrowD) return launch_wide_move(c, lds, a);
  return c->pb.precision == SMC_MIXED ? launch_move_p<float>(c->pb.family, dc, c->pb.M, lds, a, c->stream)
                                      : launch_move_p<double>(c->pb.family, dc, c->pb.M, lds, a, c->stream);
}

// Full-data A, B, C at device theta; packs rows when pack != 0.
smc_status run_cv(smc_ctx c, const double* dtheta, bool pack, double* dA, double* dB, double* dC) {
  const smc_problem& pb = c->pb;
  CvArgs a;
  a.family = pb.family;
  a.d = pb.d;
  a.ld_in = pb.ld;
  a.ld_out = c->lay.ld;
  a.in_fp32 = pb.xy_fp32;
  a.out_fp32 = pb.precision == SMC_MIXED;
  a.n = pb.n;
  a.inv_s2 = c->prob.inv_s2;
  a.log2pis2 = c->prob.log2pis2;
  a.Xin = pb.Xy;
  a.theta = dtheta;
  a.Xout = pack ? c->ws + c->lay.Xp : nullptr;
  a.partials = c->at<double>(c->lay.partials);
  a.tile_rows = c->lay.cv_rows;
  const size_t shmem = cv_lds_bytes(pb.d, c->lay.cv_rows);
  HIP_TRY(c, hipFuncSetAttribute(reinterpret_cast<const void*>(cv_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)shmem));
  hipLaunchKernelGGL(cv_kernel, dim3(c->lay.cv_blocks), dim3(kCvThreads), shmem, c->stream, a);
  LAUNCH_CHECK(c);
  CvReduceArgs r;
  r.nblocks = c->lay.cv_blocks;
  r.d = pb.d;
  r.partials = a.partials;
  r.aconst = c->at<double>(c->lay.aconst);
  r.A = dA;
  r.B = dB;
  r.C = dC;
  const int ne = 1 + pb.d + pb.d * (pb.d + 1) / 2;
  hipLaunchKernelGGL(cv_reduce_kernel, dim3(ne), dim3(256), 0, c->stream, r);
  LAUNCH_CHECK(c);
  return SMC_OK;
}

// The eta-free part of A (sum of log y!), once per context.
smc_status run_cv_const(smc_ctx c) {
  const smc_problem& pb = c->pb;
  const int ne = 1 + pb.d + pb.d * (pb.d + 1) / 2;
  int64_t nb = (pb.n + kCvThreads - 1) / kCvThreads;
  const int64_t cap = (int64_t)c->lay.cv_blocks * ne;
  if (nb > 1024) nb = 1024;
  if (nb > cap) nb = cap;
  CvConstArgs a;
  a.family = pb.family;
  a.ld_in = pb.ld;
  a.in_fp32 = pb.xy_fp32;
  a.d = pb.d;
  a.n = pb.n;
  a.log2pis2 = c->prob.log2pis2;
  a.Xin = pb.Xy;
  a.partials = c->at<double>(c->lay.partials);
  hipLaunchKernelGGL(cv_const_kernel, dim3((int)nb), dim3(kCvThreads), 0, c->stream, a);
  LAUNCH_CHECK(c);
  hipLaunchKernelGGL(cv_const_reduce_kernel, dim3(1), dim3(256), 0, c->stream, a.partials, (int)nb,
                     c->at<double>(c->lay.aconst));
  LAUNCH_CHECK(c);
  return SMC_OK;
}

// host FP64 Cholesky solve of H s = g (H SPD), false if not PD
bool host_spd_solve(int d, const std::vector<double>& H, const std::vector<double>& g, std::vector<double>& s) {
  std::vector<double> L(d * d, 0.0);
  for (int j = 0; j < d; ++j) {
    double t = H[j * d + j];
    for (int k = 0; k < j; ++k) t -= L[j * d + k] * L[j * d + k];
    if (!(t > 0.0)) return false;
    L[j * d + j] = std::sqrt(t);
    for (int i = j + 1; i < d; ++i) {
      double u = H[i * d + j];
      for (int k = 0; k < j; ++k) u -= L[i * d + k] * L[j * d + k];
      L[i * d + j] = u / L[j * d + j];
    }
  }
  std::vector<double> y(d);
  for (int k = 0; k < d; ++k) {
    double t = g[k];
    for (int j = 0; j < k; ++j) t -= L[k * d + j] * y[j];
    y[k] = t / L[k * d + k];
  }
  s.assign(d, 0.0);
  for (int k = d - 1; k >= 0; --k) {
    double t = y[k];
    for (int j = k + 1; j < d; ++j) t -= L[j * d + k] * s[j];
    s[k] = t / L[k * d + k];
  }
  return true;
}

double host_log_prior(const smc_ctx c, const std::vector<double>& th) {
  const int d = c->pb.d;
  double s = 0.0;
  for (int r = 0; r < d; ++r)
    for (int q = 0; q < d; ++q) s += (th[r] - c->mu0[r]) * c->Q0[r * d + q] * (th[q] - c->mu0[q]);
  return -0.5 * s;
}

smc_status full_eval(smc_ctx c, const std::vector<double>& th, double& A, std::vector<double>& B,
                     std::vector<double>& C) {
  const int d = c->pb.d;
  double* dth = c->at<double>(c->lay.scratch_theta);
  HIP_TRY(c, hipMemcpyAsync(dth, th.data(), d * 8, hipMemcpyHostToDevice, c->stream));
  double* dA = c->at<double>(c->lay.tout);
  double* dB = c->at<double>(c->lay.mean);
  double* dC = c->at<double>(c->lay.Qw);
  smc_status st = run_cv(c, dth, false, dA, dB, dC);
  if (st != SMC_OK) return st;
  B.resize(d);
  C.resize(d * d);
  HIP_TRY(c, hipMemcpyAsync(&A, dA, 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(B.data(), dB, d * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(C.data(), dC, d * d * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return SMC_OK;
}

// Posterior mode by Newton's method with step halving (same stopping rule as
// a plain textbook Newton: step below 1e-12 in max norm, or no ascent).
smc_status newton_mode(smc_ctx c, std::vector<double>& th) {
  const int d = c->pb.d;
  th = c->mu0;
  double A;
  std::vector<double> B, C, H(d * d), g(d), s, tn(d);
  smc_status st = full_eval(c, th, A, B, C);
  if (st != SMC_OK) return st;
  double obj = A + host_log_prior(c, th);
  int it;
  for (it = 0; it < 100; ++it) {
    for (int r = 0; r < d; ++r) {
      double q = 0.0;
      for (int k = 0; k < d; ++k) q += c->Q0[r * d + k] * (th[k] - c->mu0[k]);
      g[r] = B[r] - q;
      for (int k = 0; k < d; ++k) H[r * d + k] = -C[r * d + k] + c->Q0[r * d + k];
    }
    if (!host_spd_solve(d, H, g, s)) {
      // not concave here (e.g. Student-t far from the mode): damp the step
      // with a diagonal shift 1e-6 (1 + max |H_rr|) 10^k until H is PD
      double hmax = 0.0;
      for (int r = 0; r < d; ++r) hmax = std::fmax(hmax, std::fabs(H[r * d + r]));
      int k = 0;
      for (; k < 24; ++k) {
        std::vector<double> Hs = H;
        const double lam = 1e-6 * (1.0 + hmax) * std::pow(10.0, k);
        for (int r = 0; r < d; ++r) Hs[r * d + r] += lam;
        if (host_spd_solve(d, Hs, g, s)) break;
      }
      if (k == 24) return fail(c, SMC_ERR_NOT_PD, "Newton: no positive definite damped Hessian");
    }
    double t = 1.0, newobj = 0.0;
    bool ok = false;
    std::vector<double> Bn, Cn;
    double An = 0.0;
    for (int h = 0; h < 60; ++h) {
      for (int r = 0; r < d; ++r) tn[r] = th[r] + t * s[r];
      st = full_eval(c, tn, An, Bn, Cn);
      if (st != SMC_OK) return st;
      newobj = An + host_log_prior(c, tn);
      if (newobj >= obj || std::isnan(obj)) { ok = true; break; }
      t *= 0.5;
    }
    if (!ok) { ++it; break; }
    double stepmax = 0.0;
    for (int r = 0; r < d; ++r) stepmax = std::fmax(stepmax, std::fabs(tn[r] - th[r]));
    th = tn;
    obj = newobj;
    B = Bn;
    C = Cn;
    if (stepmax < 1e-12) { ++it; break; }
  }
  c->newton_iters = it;
  return SMC_OK;
}

smc_status factor_device(smc_ctx c, double* S, double* L, double* Linv) {
  FactorArgs f;
  f.d = c->pb.d;
  f.S = S;
  f.L = L;
  f.Linv = Linv;
  f.status = c->at<double>(c->lay.status);
  const size_t flds = (c->pb.d <= kFactorLdsMaxD) ? (size_t)2 * c->pb.d * c->pb.d * 8 : 0;
  HIP_TRY(c, hipFuncSetAttribute(reinterpret_cast<const void*>(factor_kernel),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)flds));
  hipLaunchKernelGGL(factor_kernel, dim3(1), dim3(kMomThreads), flds, c->stream, f);
  LAUNCH_CHECK(c);
  double stv = 0.0;
  HIP_TRY(c, hipMemcpyAsync(&stv, f.status, 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (stv != 0.0) return fail(c, SMC_ERR_NOT_PD, "matrix not positive definite");
  return SMC_OK;
}

smc_status refresh(smc_ctx c) {
  EstArgs a;
  std::memset(&a, 0, sizeof(a));
  a.P = c->prob;
  a.count = c->pb.M;
  a.theta = c->pb.theta;
  a.u = c->pb.u;
  a.lhat = c->pb.lhat;
  a.sig2 = c->pb.sig2;
  a.grad_l = c->at<double>(c->lay.grad_l);
  a.grad_s = c->at<double>(c->lay.grad_s);
  HIP_TRY(c, launch_estimator(c, c->pb.M, a));
  return SMC_OK;
}

}  // namespace

extern "C" {

size_t smc_workspace_size(const smc_problem* pb) {
  smc_problem tmp;
  if (!pb) return 0;
  tmp = *pb;
  // workspace itself is what is being sized
  if (!tmp.workspace) tmp.workspace = reinterpret_cast<void*>(1);
  if (validate(&tmp) != SMC_OK) return 0;
  Layout L;
  compute_layout(pb, L);
  return L.total;
}

smc_status smc_init(const smc_problem* pb, void* stream, smc_ctx* out) {
  if (!out) return SMC_ERR_INVALID_ARG;
  *out = nullptr;
  smc_status st = validate(pb);
  if (st != SMC_OK) return st;
  Layout lay;
  compute_layout(pb, lay);
  if (pb->workspace_bytes < lay.total || (reinterpret_cast<uintptr_t>(pb->workspace) & 255))
    return SMC_ERR_INVALID_ARG;
  smc_ctx c = new (std::nothrow) smc_ctx_s;
  if (!c) return SMC_ERR_DEVICE;
  c->pb = *pb;
  c->stream = reinterpret_cast<hipStream_t>(stream);
  c->lay = lay;
  c->ws = static_cast<char*>(pb->workspace);
  const int d = pb->d;
  if (pb->move_path != SMC_MOVE_STREAMING) {
    int dev = 0, max_lds = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess)
      c->res_rpl = choose_resident(*pb, max_lds, c->res_ly);
    if (pb->move_path == SMC_MOVE_RESIDENT && c->res_rpl < 0) {
      *out = c;
      return fail(c, SMC_ERR_UNSUPPORTED, "resident move kernel does not apply to this problem");
    }
  }
  c->mu0.assign(pb->prior_mean, pb->prior_mean + d);
  c->Q0.assign(pb->prior_prec, pb->prior_prec + (size_t)d * d);
  c->pb.theta_bar = nullptr;  // host pointer not kept

  Prob& P = c->prob;
  P.family = pb->family;
  P.cv_order = pb->cv_order;
  P.d = d;
  P.ld = lay.ld;
  P.n = pb->n;
  P.M = pb->M;
  P.m = pb->m;
  P.G = pb->G;
  P.seed = pb->seed;
  P.inv_s2 = pb->family == SMC_GAUSSIAN ? 1.0 / pb->gauss_s2 : 0.0;
  P.log2pis2 = pb->family == SMC_GAUSSIAN ? std::log(2.0 * M_PI * pb->gauss_s2) : 0.0;
  P.n_over_m = (double)pb->n / (double)pb->m;
  P.X = c->ws + lay.Xp;
  P.theta_bar = c->at<double>(lay.theta_bar);
  P.cvA = c->at<double>(lay.cvA);
  P.cvB = c->at<double>(lay.cvB);
  P.cvC = c->at<double>(lay.cvC);
  P.mu0 = c->at<double>(lay.mu0);
  P.Q0 = c->at<double>(lay.Q0);
  P.Sigma = c->at<double>(lay.Sigma);
  P.Linv = c->at<double>(lay.Linv);

#define TRY(expr)                                 \
  do {                                            \
    smc_status s_ = (expr);                       \
    if (s_ != SMC_OK) { *out = c; return s_; }    \
  } while (0)
#define HTRY(expr)                                                                                 \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess) {                                                                        \
      *out = c;                                                                                    \
      return fail(c, SMC_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));              \
    }                                                                                              \
  } while (0)

  HTRY(hipMemcpyAsync((void*)P.mu0, pb->prior_mean, d * 8, hipMemcpyHostToDevice, c->stream));
  HTRY(hipMemcpyAsync((void*)P.Q0, pb->prior_prec, (size_t)d * d * 8, hipMemcpyHostToDevice, c->stream));
  HTRY(hipMemcpyAsync(c->at<double>(lay.Qw), pb->prior_prec, (size_t)d * d * 8, hipMemcpyHostToDevice, c->stream));
  TRY(factor_device(c, c->at<double>(lay.Qw), c->at<double>(lay.L0), c->at<double>(lay.L0inv)));

  TRY(run_cv_const(c));
  std::vector<double> tb(d);
  if (pb->theta_bar) {
    tb.assign(pb->theta_bar, pb->theta_bar + d);
  } else {
    TRY(newton_mode(c, tb));
  }
  HTRY(hipMemcpyAsync((void*)P.theta_bar, tb.data(), d * 8, hipMemcpyHostToDevice, c->stream));
  TRY(run_cv(c, P.theta_bar, true, (double*)P.cvA, (double*)P.cvB, (double*)P.cvC));

  InitArgs ia;
  ia.P = P;
  ia.L0inv = c->at<double>(lay.L0inv);
  ia.theta = pb->theta;
  ia.u = pb->u;
  ia.logw = pb->logw;
  hipLaunchKernelGGL(init_kernel, dim3(pb->M), dim3(kWave), 0, c->stream, ia);
  HTRY(hipGetLastError());
  TRY(refresh(c));
  HTRY(hipStreamSynchronize(c->stream));
  c->a = 0.0;
  c->logz = 0.0;
  c->stage = 0;
  c->move = 0;
  *out = c;
  return SMC_OK;
#undef TRY
#undef HTRY
}

static smc_status temper_impl(smc_ctx c, int grid_points, double ess_frac, double* a_out, double* dlogz_out,
                              double* ess_out, double* ess_grid_out) {
  if (c->a >= 1.0) return fail(c, SMC_ERR_STATE, "tempering already reached a = 1");
  TemperArgs t;
  t.M = c->pb.M;
  t.a_prev = c->a;
  t.ess_frac = ess_frac;
  t.lhat = c->pb.lhat;
  t.sig2 = c->pb.sig2;
  t.logw = c->pb.logw;
  t.out = c->at<double>(c->lay.tout);
  t.grid_ess = nullptr;
  t.grid_n = 0;
  if (grid_points > 0) {
    GridArgs g;
    g.M = c->pb.M;
    g.a_prev = c->a;
    g.lhat = c->pb.lhat;
    g.sig2 = c->pb.sig2;
    g.logw = c->pb.logw;
    g.ess = c->at<double>(c->lay.grid);
    hipLaunchKernelGGL(grid_ess_kernel, dim3(grid_points), dim3(kGridThreads), 0, c->stream, g);
    LAUNCH_CHECK(c);
    t.grid_ess = g.ess;
    t.grid_n = grid_points;
    if (ess_grid_out)
      HIP_TRY(c, hipMemcpyAsync(ess_grid_out, g.ess, (size_t)grid_points * 8, hipMemcpyDeviceToHost, c->stream));
  }
  hipLaunchKernelGGL(temper_kernel, dim3(1), dim3(kTemperThreads), 0, c->stream, t);
  LAUNCH_CHECK(c);
  double o[5];
  HIP_TRY(c, hipMemcpyAsync(o, t.out, sizeof(o), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (o[3] != 0.0) return fail(c, SMC_ERR_NONFINITE, "all incremental weights non-finite");
  c->stage += 1;
  c->move = 0;
  c->a = o[0];
  c->logz += o[1];
  c->have_mass = 0;
  if (a_out) *a_out = o[0];
  if (dlogz_out) *dlogz_out = o[1];
  if (ess_out) *ess_out = o[2];
  return SMC_OK;
}

smc_status smc_temper(smc_ctx c, double* a_out, double* dlogz_out, double* ess_out) {
  if (!c) return SMC_ERR_INVALID_ARG;
  return temper_impl(c, 0, c->pb.ess_frac, a_out, dlogz_out, ess_out, nullptr);
}

smc_status smc_temper_grid(smc_ctx c, int32_t grid_points, double ess_frac, double* a_out, double* dlogz_out,
                           double* ess_out, double* ess_grid_out) {
  if (!c) return SMC_ERR_INVALID_ARG;
  if (grid_points < 1 || grid_points > kGridMax) return fail(c, SMC_ERR_INVALID_ARG, "grid_points must be in [1, 256]");
  if (!(ess_frac > 0.0 && ess_frac <= 1.0)) return fail(c, SMC_ERR_INVALID_ARG, "ess_frac must be in (0, 1]");
  return temper_impl(c, grid_points, ess_frac, a_out, dlogz_out, ess_out, ess_grid_out);
}

smc_status smc_mass(smc_ctx c) {
  if (!c) return SMC_ERR_INVALID_ARG;
  const int d = c->pb.d;
  MomentArgs a;
  a.M = c->pb.M;
  a.d = d;
  a.theta = c->pb.theta;
  a.logw = c->pb.logw;
  a.centre = c->prob.theta_bar;
  a.partials = c->at<double>(c->lay.mpartials);
  a.nblocks = c->lay.mom_blocks;
  a.mean = c->at<double>(c->lay.mean);
  a.F.d = d;
  a.F.S = c->at<double>(c->lay.Sigma);
  a.F.L = c->at<double>(c->lay.Lchol);
  a.F.Linv = c->at<double>(c->lay.Linv);
  a.F.status = c->at<double>(c->lay.status);
  hipLaunchKernelGGL(moments_partial_kernel, dim3(a.nblocks), dim3(kMomThreads), (size_t)kMomTile * d * 8,
                     c->stream, a);
  LAUNCH_CHECK(c);
  const size_t mlds = (size_t)(d + d * (d + 1) / 2) * 8 + (d <= kFactorLdsMaxD ? (size_t)2 * d * d * 8 : 0);
  HIP_TRY(c, hipFuncSetAttribute(reinterpret_cast<const void*>(moments_final_kernel),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)mlds));
  hipLaunchKernelGGL(moments_final_kernel, dim3(1), dim3(kMomThreads), mlds, c->stream, a);
  LAUNCH_CHECK(c);
  double stv = 0.0;
  HIP_TRY(c, hipMemcpyAsync(&stv, a.F.status, 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (stv != 0.0) return fail(c, SMC_ERR_NOT_PD, "particle covariance not positive definite");
  c->have_mass = 1;
  return SMC_OK;
}

static smc_status resample_impl(smc_ctx c, int multinomial) {
  const smc_problem& pb = c->pb;
  ResampleArgs r;
  r.M = pb.M;
  r.multinomial = multinomial;
  r.seed = pb.seed;
  r.stage = (uint32_t)c->stage;
  r.logw = pb.logw;
  r.anc = c->at<int32_t>(c->lay.anc);
  hipLaunchKernelGGL(resample_kernel, dim3(1), dim3(kResThreads), 0, c->stream, r);
  LAUNCH_CHECK(c);
  GatherArgs g;
  g.M = pb.M; g.d = pb.d; g.m = pb.m;
  g.anc = r.anc;
  g.theta = pb.theta; g.u = pb.u; g.lhat = pb.lhat; g.sig2 = pb.sig2;
  g.gl = c->at<double>(c->lay.grad_l); g.gs = c->at<double>(c->lay.grad_s);
  g.theta2 = c->at<double>(c->lay.th2); g.u2 = c->at<int32_t>(c->lay.u2);
  g.lhat2 = c->at<double>(c->lay.lh2); g.sig22 = c->at<double>(c->lay.sg2);
  g.gl2 = c->at<double>(c->lay.gl2); g.gs2 = c->at<double>(c->lay.gs2);
  hipLaunchKernelGGL(gather_kernel, dim3(pb.M), dim3(256), 0, c->stream, g);
  LAUNCH_CHECK(c);
  CopyBackArgs b;
  b.M = pb.M; b.d = pb.d; b.m = pb.m;
  b.theta2 = g.theta2; b.u2 = g.u2; b.lhat2 = g.lhat2; b.sig22 = g.sig22; b.gl2 = g.gl2; b.gs2 = g.gs2;
  b.theta = pb.theta; b.u = pb.u; b.lhat = pb.lhat; b.sig2 = pb.sig2;
  b.gl = const_cast<double*>(g.gl); b.gs = const_cast<double*>(g.gs); b.logw = pb.logw;
  hipLaunchKernelGGL(copyback_kernel, dim3(pb.M), dim3(256), 0, c->stream, b);
  LAUNCH_CHECK(c);
  return SMC_OK;
}

smc_status smc_resample(smc_ctx c) {
  if (!c) return SMC_ERR_INVALID_ARG;
  return resample_impl(c, 0);
}

smc_status smc_resample_multinomial(smc_ctx c) {
  if (!c) return SMC_ERR_INVALID_ARG;
  return resample_impl(c, 1);
}

smc_status smc_move(smc_ctx c, double eps, int32_t L, int32_t R) {
  if (!c) return SMC_ERR_INVALID_ARG;
  if (!(eps > 0.0) || L < 1 || R < 0) return fail(c, SMC_ERR_INVALID_ARG, "bad eps/L/R");
  if (!c->have_mass) return fail(c, SMC_ERR_STATE, "no mass matrix for this stage");
  if (c->move + R > 0xFFFF) return fail(c, SMC_ERR_INVALID_ARG, "too many moves in one stage");
  for (int r = 0; r < R; ++r) {
    MoveArgs a;
    a.P = c->prob;
    a.a = c->a;
    a.eps = eps;
    a.L = L;
    a.stage = (uint32_t)c->stage;
    a.move = (uint32_t)c->move;
    a.theta = c->pb.theta;
    a.u = c->pb.u;
    a.lhat = c->pb.lhat;
    a.sig2 = c->pb.sig2;
    a.grad_l = c->at<double>(c->lay.grad_l);
    a.grad_s = c->at<double>(c->lay.grad_s);
    a.accept = c->pb.accept;
    HIP_TRY(c, launch_move(c, a));
    c->move += 1;
  }
  return SMC_OK;
}

smc_status loglik_est(smc_ctx c, int32_t count, const double* theta, const int32_t* u, double* lhat,
                      double* sig2, double* dhat) {
  if (!c || count < 0 || (count > 0 && (!theta || !u))) return SMC_ERR_INVALID_ARG;
  EstArgs a;
  std::memset(&a, 0, sizeof(a));
  a.P = c->prob;
  a.count = count;
  a.theta = theta;
  a.u = u;
  a.lhat = lhat;
  a.sig2 = sig2;
  a.dhat = dhat;
  HIP_TRY(c, launch_estimator(c, count, a));
  return SMC_OK;
}

smc_status loglik_grad(smc_ctx c, int32_t count, const double* theta, const int32_t* u, const double* g_lhat,
                       const double* g_sig2, double* grad, double* grad_l, double* grad_s) {
  if (!c || count < 0 || (count > 0 && (!theta || !u))) return SMC_ERR_INVALID_ARG;
  EstArgs a;
  std::memset(&a, 0, sizeof(a));
  a.P = c->prob;
  a.count = count;
  a.theta = theta;
  a.u = u;
  a.g_lhat = g_lhat;
  a.g_sig2 = g_sig2;
  a.grad = grad;
  a.grad_l = grad_l;
  a.grad_s = grad_s;
  HIP_TRY(c, launch_estimator(c, count, a));
  return SMC_OK;
}

smc_status smc_refresh(smc_ctx c) {
  if (!c) return SMC_ERR_INVALID_ARG;
  return refresh(c);
}

smc_status smc_recentre(smc_ctx c, const double* theta_bar_host) {
  if (!c) return SMC_ERR_INVALID_ARG;
  const int d = c->pb.d;
  double* tb = const_cast<double*>(c->prob.theta_bar);
  if (theta_bar_host) {
    for (int r = 0; r < d; ++r)
      if (!std::isfinite(theta_bar_host[r])) return fail(c, SMC_ERR_INVALID_ARG, "theta_bar is not finite");
    HIP_TRY(c, hipMemcpyAsync(tb, theta_bar_host, (size_t)d * 8, hipMemcpyHostToDevice, c->stream));
  } else {
    if (!c->have_mass) return fail(c, SMC_ERR_STATE, "no weighted mean for this stage (call smc_mass first)");
    HIP_TRY(c, hipMemcpyAsync(tb, c->at<double>(c->lay.mean), (size_t)d * 8, hipMemcpyDeviceToDevice, c->stream));
  }
  smc_status st = run_cv(c, tb, true, const_cast<double*>(c->prob.cvA), const_cast<double*>(c->prob.cvB),
                         const_cast<double*>(c->prob.cvC));
  if (st != SMC_OK) return st;
  st = refresh(c);
  if (st != SMC_OK) return st;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return SMC_OK;
}

smc_status smc_get_info(smc_ctx c, smc_info* o) {
  if (!c || !o) return SMC_ERR_INVALID_ARG;
  o->a = c->a;
  o->logz = c->logz;
  o->stage = c->stage;
  o->move = c->move;
  o->have_mass = c->have_mass;
  o->newton_iters = c->newton_iters;
  o->move_path = c->res_rpl >= 0 ? SMC_MOVE_RESIDENT : SMC_MOVE_STREAMING;
  return SMC_OK;
}

smc_status smc_set_stage(smc_ctx c, int32_t stage, int32_t move, double a, double logz) {
  if (!c || stage < 0 || stage > 0xFFFFFF || move < 0 || move > 0xFFFF || !(a >= 0.0 && a <= 1.0))
    return SMC_ERR_INVALID_ARG;
  c->stage = stage;
  c->move = move;
  c->a = a;
  c->logz = logz;
  return SMC_OK;
}

smc_status smc_set_mass(smc_ctx c, const double* sigma_host) {
  if (!c || !sigma_host) return SMC_ERR_INVALID_ARG;
  const int d = c->pb.d;
  double* S = c->at<double>(c->lay.Sigma);
  HIP_TRY(c, hipMemcpyAsync(S, sigma_host, (size_t)d * d * 8, hipMemcpyHostToDevice, c->stream));
  smc_status st = factor_device(c, S, c->at<double>(c->lay.Lchol), c->at<double>(c->lay.Linv));
  if (st != SMC_OK) return st;
  c->have_mass = 1;
  return SMC_OK;
}

smc_status smc_get_mass(smc_ctx c, double* sigma, double* chol, double* chol_inv) {
  if (!c) return SMC_ERR_INVALID_ARG;
  const size_t b = (size_t)c->pb.d * c->pb.d * 8;
  if (sigma) HIP_TRY(c, hipMemcpyAsync(sigma, c->at<double>(c->lay.Sigma), b, hipMemcpyDeviceToHost, c->stream));
  if (chol) HIP_TRY(c, hipMemcpyAsync(chol, c->at<double>(c->lay.Lchol), b, hipMemcpyDeviceToHost, c->stream));
  if (chol_inv) HIP_TRY(c, hipMemcpyAsync(chol_inv, c->at<double>(c->lay.Linv), b, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return SMC_OK;
}

smc_status smc_get_cv(smc_ctx c, double* theta_bar, double* A, double* B, double* C) {
  if (!c) return SMC_ERR_INVALID_ARG;
  const int d = c->pb.d;
  if (theta_bar) HIP_TRY(c, hipMemcpyAsync(theta_bar, c->prob.theta_bar, d * 8, hipMemcpyDeviceToHost, c->stream));
  if (A) HIP_TRY(c, hipMemcpyAsync(A, c->prob.cvA, 8, hipMemcpyDeviceToHost, c->stream));
  if (B) HIP_TRY(c, hipMemcpyAsync(B, c->prob.cvB, d * 8, hipMemcpyDeviceToHost, c->stream));
  if (C) HIP_TRY(c, hipMemcpyAsync(C, c->prob.cvC, (size_t)d * d * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return SMC_OK;
}

smc_status smc_full_loglik(smc_ctx c, const double* theta, double* A, double* B, double* C) {
  if (!c || !theta) return SMC_ERR_INVALID_ARG;
  const int d = c->pb.d;
  std::vector<double> th(theta, theta + d), Bv, Cv;
  double Av = 0.0;
  smc_status st = full_eval(c, th, Av, Bv, Cv);
  if (st != SMC_OK) return st;
  if (A) *A = Av;
  if (B) std::memcpy(B, Bv.data(), d * 8);
  if (C) std::memcpy(C, Cv.data(), (size_t)d * d * 8);
  return SMC_OK;
}

void smc_destroy(smc_ctx c) { delete c; }

const char* smc_status_string(smc_status s) {
  switch (s) {
    case SMC_OK: return "ok";
    case SMC_ERR_INVALID_ARG: return "invalid argument";
    case SMC_ERR_STATE: return "call out of order";
    case SMC_ERR_DEVICE: return "device error";
    case SMC_ERR_NOT_PD: return "matrix not positive definite";
    case SMC_ERR_NONFINITE: return "non-finite weights";
    case SMC_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* smc_last_error(smc_ctx c) { return c ? c->err : "no context"; }

}  // extern "C"
