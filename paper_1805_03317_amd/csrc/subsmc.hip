// Host side of the C ABI declared in include/subsmc.h: workspace layout,
// argument checks, kernel dispatch and the Newton iteration for the
// control-variate centre.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/subsmc.h"
#include "dispatch.hpp"
#include "kernels_stage.hpp"

using namespace subsmc;

namespace {

constexpr int kMaxNarrowD = 32;   // one lane per row up to here
constexpr int kMaxD = 128;        // lane groups per row beyond
constexpr int kMaxM = kTemperThreads * kTemperPer;
constexpr int kMaxBatch = 65536;  // the dataset field of the random-number counter
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
      tout, grid, search, aconst, scratch_theta, grad_l, grad_s, ties, diag, anc, th2, u2, lh2, sg2, gl2, gs2, partials, mpartials,
      total;
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
  L.search = take(2 * sizeof(SearchSlot));
  L.aconst = take(8);
  L.scratch_theta = take(d * 8);
  L.grad_l = take(M * d * 8);
  L.grad_s = take(M * d * 8);
  L.ties = take(M * 2 * 4);
  L.diag = take(M * 4 * 8);
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
  int stage = 0, move = 0, newton_iters = 0;
  // mass matrix of this stage: 0 none, 1 ready, 2 computed with its
  // positive-definiteness flag still on its way to the host (mass_ev, hstatus)
  int have_mass = 0;
  double* hstatus = nullptr;  // pinned: [0] the mass flag, [1..5] smc_stage's tempering results
  hipEvent_t mass_ev = nullptr;
  hipEvent_t temper_ev = nullptr;
  // optional timing of move launches: a ring of event pairs
  std::vector<hipEvent_t> mev;
  int mev_next = 0, mev_count = 0;
  int moved = 0;     // a move has written the accept and near-tie flags
  int res_rpl = -1;  // register rows per lane of the resident move kernel; -1: streaming
  int res_mf = 0;    // the resident move forms x'delta on the matrix cores
  int wide_tile = 0; // tile form of the lane-group streaming move's row loop
  ResLayout res_ly{};
  std::vector<double> mu0, Q0;
  char err[512] = {0};

  template <typename T> T* at(size_t off) { return reinterpret_cast<T*>(ws + off); }
};

// A batch: member contexts on one stream whose per-stage steps run as one
// launch per kernel (the move: one launch per kernel shape among the members).
struct smc_batch_s {
  std::vector<smc_ctx> ctx;
  hipStream_t stream = nullptr;
  char* dev = nullptr;          // caller's workspace: argument tables, then results
  char* host = nullptr;         // pinned mirror of the workspace
  size_t table_bytes = 0;       // capacity of the table region
  hipEvent_t staged = nullptr;  // recorded after the last upload from `host`
  std::vector<int> active;      // members tempered in the current stage
  int have_stage = 0;
  // optional timing of the move launches: an event pair per launch and move
  int timing = 0;
  std::vector<hipEvent_t> ev;          // 2 per (move, launch) of the last smc_batch_move
  std::vector<int> launch_kind;        // per launch of the last smc_batch_move
  std::vector<int> member_launch;      // per member: its launch, -1 if inactive
  int timed_moves = 0;
  // optional replay of the move's launches as one HIP graph, captured again
  // whenever the launch structure changes
  int use_graph = 0;
  hipStream_t capture = nullptr;  // private stream the graph is captured on
  hipGraphExec_t gexec = nullptr;
  std::vector<long long> graph_key;
  int graph_captures = 0;
  // the move's launches spread over `lanes` streams (the batch's stream and
  // lanes - 1 private ones), forked from and joined back to the batch's
  // stream, so that launches too small to fill the chip overlap
  int lanes = 8;
  std::vector<hipStream_t> side;  // lanes - 1 private streams
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  // optional persistent move: one launch per (row type, family) with a device
  // work queue over every member's particles (smc_batch_set_persistent)
  int persistent = 0;
  int cus = 0;                   // compute units of the batch's device
  std::vector<int> member_kind;  // per member: the kernel kind of its last move, -1 if not moved
  char err[512] = {0};
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
  if (pb->move_path < SMC_MOVE_AUTO || pb->move_path > SMC_MOVE_RESIDENT_MFMA) return SMC_ERR_INVALID_ARG;
  if (pb->dataset > 0xFFFFu) return SMC_ERR_INVALID_ARG;
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
// kernel selection (the launchers live in launch_*.hip)
// ------------------------------------------------------------------------

// register-row candidates for (precision, padded d, family) of the resident
// move, smallest first: the shapes instantiated in launch_resident.hip. All
// rows in LDS always; 4 or 14 register rows per lane for FP32 rows whose
// remainder leaves the register file room for them (the logistic remainder
// needs more registers than the Poisson one: at d = 20 its rows would spill).
// 4 covers the subsamples just too large for LDS alone, 14 the largest.
constexpr int kResMaxRows = 3;
// each FP32 layout in both forms of the x'delta product (vector ALU, matrix cores)
constexpr int kResMaxOptions = 2 * kResMaxRows;
// the form smc_init picks for FP32 rows (smc_autotune_move measures both)
constexpr int kResMfmaDefault = 0;

int res_candidates(bool fp32, int dc, int family, int out[kResMaxRows]) {
  if (dc > 24) return 0;
  out[0] = 0;
  if (fp32 && ((family == SMC_POISSON && dc <= 20) || (family == SMC_LOGISTIC && dc <= 16))) {
    out[1] = 4;
    out[2] = 14;
    return 3;
  }
  return 1;
}

struct ResOption {
  int rpl, mf;
  ResLayout ly;
  int tile;  // streaming options (rpl = -1): the lane-group row loop's tile form
};

// tile forms of the lane-group streaming move for a problem (see launch_wide.hip)
// Tile forms of the lane-group move for this problem, as bits: form 0 always;
// form 1 (the remainder in every lane) for FP32 logistic rows; form 2 (form 0
// with kWideGroup particles per workgroup whose row loops meet at a barrier
// every kSyncIters iterations) when
// kWideGroup divides the particle count. The narrow move has form 0 only.
int wide_forms(const smc_problem& pb) {
  if (pb.d <= kMaxNarrowD) return 1;
  const WideShape w = wide_shape(pb.d, pb.precision == SMC_MIXED);
  int f = 1;
  if (pb.precision == SMC_MIXED && pb.family == SMC_LOGISTIC && (w.G == 4 || w.G == 8)) f |= 2;
  if (pb.M % kWideGroup == 0) f |= 4;
  return f;
}

bool wide_form_ok(const smc_problem& pb, int t) { return t >= 0 && t <= 2 && ((wide_forms(pb) >> t) & 1); }

// The default tile form: 2 for FP32 logistic rows of 8-lane groups (d > 60; measured on
// the d = 116 configuration's live stages 288 -> 228 ms, where resampled copies
// share their rows), else 0 (d = 50: 34.8 ms against 36.9 with form 2).
int default_wide_tile(const smc_problem& pb) {
  const WideShape w = wide_shape(pb.d, pb.precision == SMC_MIXED);
  return (wide_form_ok(pb, 2) && w.G == 8 && pb.precision == SMC_MIXED && pb.family == SMC_LOGISTIC) ? 2 : 0;
}

// Every register-row count whose layout fits, smallest first, each FP32 one
// with the x'delta product on the vector ALU and on the matrix cores.
int resident_options(const smc_problem& pb, int max_lds, ResOption opt[kResMaxOptions]) {
  if (pb.d > kMaxNarrowD || (pb.family != SMC_LOGISTIC && pb.family != SMC_POISSON)) return 0;
  const bool fp32 = pb.precision == SMC_MIXED;
  const int dc = pad_dc(pb.d);
  int cand[kResMaxRows];
  const int nc = res_candidates(fp32, dc, pb.family, cand);
  int n = 0;
  for (int q = 0; q < nc; ++q) {
    const ResLayout l = res_layout(pb.m, pb.G, dc, cand[q], fp32 ? 4 : 8, pb.d);
    // register rows are unpredicated in the kernel: every slot must hold a row
    const bool regs_full = pb.m >= kResLanes * cand[q];
    if (regs_full && l.total <= max_lds && (l.nlds + kResLanes - 1) / kResLanes <= kResMaxLdsGroups) {
      for (int mf = 0; mf <= (fp32 ? 1 : 0); ++mf) opt[n++] = ResOption{cand[q], mf, l, 0};
    }
  }
  return n;
}

// Smallest register-row count whose LDS part fits, with the product in the
// form the move path asks for (the default form on the automatic path);
// false if the resident kernel does not apply.
bool choose_resident(const smc_problem& pb, int max_lds, ResOption& o) {
  ResOption opt[kResMaxOptions];
  const int n = resident_options(pb, max_lds, opt);
  const int want = pb.move_path == SMC_MOVE_RESIDENT_MFMA ? 1
                   : pb.move_path == SMC_MOVE_RESIDENT    ? 0
                                                           : kResMfmaDefault;
  int best = -1;
  for (int q = 0; q < n && best < 0; ++q)  // the options come by register rows, ascending
    if (opt[q].mf == want) best = q;
  if (best < 0 && pb.move_path == SMC_MOVE_AUTO && n > 0) best = 0;  // FP64 rows: the vector form only
  if (best < 0) return false;
  o = opt[best];
  return true;
}

// The move kernel of a context (the estimator kernels use the narrow or wide
// shape of the same d).
KernelShape move_shape(smc_ctx c) {
  KernelShape s{};
  s.fp32 = c->pb.precision == SMC_MIXED ? 1 : 0;
  s.fam = c->pb.family;
  s.dc = pad_dc(c->pb.d);
  const WideShape w = wide_shape(c->pb.d, s.fp32 != 0);
  s.lanes = w.G;
  s.ch = w.CH;
  s.rpl = c->res_rpl;
  s.mf = c->res_rpl >= 0 ? c->res_mf : 0;
  s.kind = c->res_rpl >= 0 ? kMoveResident : (c->pb.d > kMaxNarrowD ? kMoveWide : kMoveNarrow);
  s.tile = s.kind == kMoveWide ? c->wide_tile : 0;
  return s;
}

// A batch member's shape: tile form 2 (grouped particles) is form 0 in batch launches
KernelShape member_shape(smc_ctx c) {
  KernelShape s = move_shape(c);
  if (s.tile == 2) s.tile = 0;
  return s;
}

hipError_t launch_estimator(smc_ctx c, int count, const EstArgs& a) {
  if (count <= 0) return hipSuccess;
  const KernelShape s = move_shape(c);
  return s.kind == kMoveWide ? launch_estimator_wide(s, count, a, c->stream)
                             : launch_estimator_narrow(s, count, a, c->stream);
}

// dynamic LDS of the streaming moves: one refreshed block of indices
size_t block_lds_bytes(const smc_problem& pb) {
  return (size_t)((pb.m + pb.G - 1) / pb.G) * sizeof(int32_t);
}

hipError_t launch_move(smc_ctx c, const MoveArgs& a) {
  const KernelShape s = move_shape(c);
  switch (s.kind) {
    case kMoveResident: return launch_move_resident(s, c->pb.M, c->res_ly, a, c->stream);
    case kMoveWide: return launch_move_wide(s, c->pb.M, block_lds_bytes(c->pb), a, c->stream);
    default: return launch_move_narrow(s, c->pb.M, block_lds_bytes(c->pb), a, c->stream);
  }
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
  const size_t flds = factor_lds_bytes(c->pb.d);
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

// Settles a mass matrix computed by smc_mass: waits for its
// positive-definiteness flag and reports SMC_ERR_NOT_PD (dropping the matrix)
// if the factorisation failed.
smc_status mass_ready(smc_ctx c) {
  if (c->have_mass != 2) return SMC_OK;
  HIP_TRY(c, hipEventSynchronize(c->mass_ev));
  if (c->hstatus[0] != 0.0) {
    c->have_mass = 0;
    return fail(c, SMC_ERR_NOT_PD, "particle covariance not positive definite");
  }
  c->have_mass = 1;
  return SMC_OK;
}

// ------------------------------------------------------------------------
// argument blocks of the per-stage kernels, shared by the single-context
// calls and the batched ones
// ------------------------------------------------------------------------

TemperArgs temper_args(smc_ctx c, double ess_frac, double* out) {
  TemperArgs t;
  t.M = c->pb.M;
  t.a_prev = c->a;
  t.ess_frac = ess_frac;
  t.lhat = c->pb.lhat;
  t.sig2 = c->pb.sig2;
  t.logw = c->pb.logw;
  t.out = out;
  t.grid_ess = nullptr;
  t.grid_n = 0;
  t.search = c->at<SearchSlot>(c->lay.search);
  return t;
}

// the passes of the exponent search (they end in the context's search slots)
hipError_t launch_search(const TemperArgs& t, hipStream_t s) {
  for (int pass = 0; pass < kSearchPasses; ++pass) {
    hipLaunchKernelGGL(search_pass_kernel, dim3(pass_groups(pass)), dim3(kSearchThreads), 0, s, t, pass);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// state after a successful exponent search with outputs o = [a, dlogz, ess, ...]
void temper_commit(smc_ctx c, const double* o) {
  c->stage += 1;
  c->move = 0;
  c->a = o[0];
  c->logz += o[1];
  c->have_mass = 0;
}

MomentArgs moment_args(smc_ctx c, double* status) {
  const int d = c->pb.d;
  MomentArgs a;
  a.M = c->pb.M;
  a.d = d;
  a.theta = c->pb.theta;
  a.logw = c->pb.logw;
  // the one-pass sums are taken about particle 0's theta: a point inside the
  // cloud, so E[(theta - c)(theta - c)'] - (mean - c)(mean - c)' loses no more
  // than the cloud's own spread to cancellation (about the control-variate
  // centre, a cloud far from it would lose up to (distance / spread)^2)
  a.centre = c->pb.theta;
  a.partials = c->at<double>(c->lay.mpartials);
  a.nblocks = c->lay.mom_blocks;
  a.mean = c->at<double>(c->lay.mean);
  a.F.d = d;
  a.F.S = c->at<double>(c->lay.Sigma);
  a.F.L = c->at<double>(c->lay.Lchol);
  a.F.Linv = c->at<double>(c->lay.Linv);
  a.F.status = status;
  return a;
}

size_t moments_partial_lds(int d) { return (size_t)kMomTile * d * 8; }
size_t moments_final_lds(int d) {
  const size_t mom = (size_t)(d + d * (d + 1) / 2) * 8;
  // d <= kFactorLdsMaxD: the factor after the moments; up to kFactorLdsLMaxD: over them
  return d <= kFactorLdsMaxD ? mom + factor_lds_bytes(d) : std::max(mom, factor_lds_bytes(d));
}

ResampleArgs resample_args(smc_ctx c, int multinomial) {
  ResampleArgs r;
  r.M = c->pb.M;
  r.multinomial = multinomial;
  r.seed = c->pb.seed;
  r.dataset = c->pb.dataset;
  r.stage = (uint32_t)c->stage;
  r.logw = c->pb.logw;
  r.anc = c->at<int32_t>(c->lay.anc);
  return r;
}

GatherArgs gather_args(smc_ctx c) {
  const smc_problem& pb = c->pb;
  GatherArgs g;
  g.M = pb.M; g.d = pb.d; g.m = pb.m;
  g.anc = c->at<int32_t>(c->lay.anc);
  g.theta = pb.theta; g.u = pb.u; g.lhat = pb.lhat; g.sig2 = pb.sig2;
  g.gl = c->at<double>(c->lay.grad_l); g.gs = c->at<double>(c->lay.grad_s);
  g.theta2 = c->at<double>(c->lay.th2); g.u2 = c->at<int32_t>(c->lay.u2);
  g.lhat2 = c->at<double>(c->lay.lh2); g.sig22 = c->at<double>(c->lay.sg2);
  g.gl2 = c->at<double>(c->lay.gl2); g.gs2 = c->at<double>(c->lay.gs2);
  return g;
}

CopyBackArgs copyback_args(smc_ctx c) {
  const smc_problem& pb = c->pb;
  CopyBackArgs b;
  b.M = pb.M; b.d = pb.d; b.m = pb.m;
  b.theta2 = c->at<double>(c->lay.th2); b.u2 = c->at<int32_t>(c->lay.u2);
  b.lhat2 = c->at<double>(c->lay.lh2); b.sig22 = c->at<double>(c->lay.sg2);
  b.gl2 = c->at<double>(c->lay.gl2); b.gs2 = c->at<double>(c->lay.gs2);
  b.theta = pb.theta; b.u = pb.u; b.lhat = pb.lhat; b.sig2 = pb.sig2;
  b.gl = c->at<double>(c->lay.grad_l); b.gs = c->at<double>(c->lay.grad_s); b.logw = pb.logw;
  return b;
}

MoveArgs move_args(smc_ctx c, double eps, int L) {
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
  a.ties = c->at<int32_t>(c->lay.ties);
  a.tie_tol = c->pb.precision == SMC_MIXED ? 1e-5 : 1e-9;
  a.diag = c->at<double>(c->lay.diag);
  return a;
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
  if (hipHostMalloc(reinterpret_cast<void**>(&c->hstatus), 64, hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&c->mass_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->temper_ev, hipEventDisableTiming) != hipSuccess) {
    smc_destroy(c);
    return SMC_ERR_DEVICE;
  }
  c->pb = *pb;
  c->stream = reinterpret_cast<hipStream_t>(stream);
  c->lay = lay;
  c->ws = static_cast<char*>(pb->workspace);
  const int d = pb->d;
  if (pb->move_path != SMC_MOVE_STREAMING) {
    int dev = 0, max_lds = 0;
    ResOption o;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        choose_resident(*pb, max_lds, o)) {
      c->res_rpl = o.rpl;
      c->res_mf = o.mf;
      c->res_ly = o.ly;
    }
    if ((pb->move_path == SMC_MOVE_RESIDENT || pb->move_path == SMC_MOVE_RESIDENT_MFMA) && c->res_rpl < 0) {
      *out = c;
      return fail(c, SMC_ERR_UNSUPPORTED, "resident move kernel does not apply to this problem");
    }
  }
  c->wide_tile = default_wide_tile(*pb);
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
  P.dataset = pb->dataset;
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
  TemperArgs t = temper_args(c, ess_frac, c->at<double>(c->lay.tout));
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
  } else {
    HIP_TRY(c, launch_search(t, c->stream));
  }
  hipLaunchKernelGGL(temper_kernel, dim3(1), dim3(kTemperThreads), 0, c->stream, t);
  LAUNCH_CHECK(c);
  double o[5];
  HIP_TRY(c, hipMemcpyAsync(o, t.out, sizeof(o), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (o[3] != 0.0) return fail(c, SMC_ERR_NONFINITE, "all incremental weights non-finite");
  temper_commit(c, o);
  if (a_out) *a_out = o[0];
  if (dlogz_out) *dlogz_out = o[1];
  if (ess_out) *ess_out = o[2];
  return SMC_OK;
}

}  // extern "C"

namespace {

// Scratch of smc_temper_noalloc: the two alternating slots of the exponent
// search, in device memory the library owns for the life of the process (one
// copy per GPU). Host code never uses this name as an address: the device
// address of each GPU's copy is looked up once per device and kept below.
constexpr size_t kNoAllocScratchBytes = 2 * sizeof(SearchSlot);
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {nullptr};

// The current device's copy of `scratch` (nullptr on failure, with the HIP error in *err).
char* scratch_for_current_device(hipError_t* err) {
  int dev = 0;
  *err = hipGetDevice(&dev);
  if (*err != hipSuccess) return nullptr;
  if (dev < 0 || dev >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

smc_status smc_temper_noalloc(int32_t M, const double* lhat, const double* sig2, double* logw, double a_prev,
                              double ess_frac, double* out, void* stream) {
  if (M < 1 || M > kMaxM || !lhat || !sig2 || !logw || !out) return SMC_ERR_INVALID_ARG;
  if (!(a_prev >= 0.0 && a_prev < 1.0) || !(ess_frac > 0.0 && ess_frac <= 1.0)) return SMC_ERR_INVALID_ARG;
  hipError_t e = hipSuccess;
  char* ptr = scratch_for_current_device(&e);
  if (!ptr) return SMC_ERR_DEVICE;
  TemperArgs t;
  t.M = M;
  t.a_prev = a_prev;
  t.ess_frac = ess_frac;
  t.lhat = lhat;
  t.sig2 = sig2;
  t.logw = logw;
  t.out = out;
  t.grid_ess = nullptr;
  t.grid_n = 0;
  // every slot entry a pass reads is written by the pass before it in the
  // same call, so the scratch needs no clearing between calls
  t.search = reinterpret_cast<SearchSlot*>(ptr);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (launch_search(t, st) != hipSuccess) return SMC_ERR_DEVICE;
  hipLaunchKernelGGL(temper_kernel, dim3(1), dim3(kTemperThreads), 0, st, t);
  if (hipGetLastError() != hipSuccess) return SMC_ERR_DEVICE;
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
  const MomentArgs a = moment_args(c, c->at<double>(c->lay.status));
  hipLaunchKernelGGL(moments_partial_kernel, dim3(a.nblocks), dim3(kMomThreads), moments_partial_lds(d),
                     c->stream, a);
  LAUNCH_CHECK(c);
  const size_t mlds = moments_final_lds(d);
  HIP_TRY(c, hipFuncSetAttribute(reinterpret_cast<const void*>(moments_final_kernel),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)mlds));
  hipLaunchKernelGGL(moments_final_kernel, dim3(1), dim3(kMomThreads), mlds, c->stream, a);
  LAUNCH_CHECK(c);
  // the positive-definiteness flag travels to the host behind the kernels;
  // the first call that uses the mass matrix waits for it (mass_ready)
  HIP_TRY(c, hipMemcpyAsync(c->hstatus, a.F.status, 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipEventRecord(c->mass_ev, c->stream));
  c->have_mass = 2;
  return SMC_OK;
}

static smc_status resample_impl(smc_ctx c, int multinomial) {
  const smc_problem& pb = c->pb;
  const ResampleArgs r = resample_args(c, multinomial);
  hipLaunchKernelGGL(resample_kernel, dim3(1), dim3(kResThreads), 0, c->stream, r);
  LAUNCH_CHECK(c);
  const GatherArgs g = gather_args(c);
  hipLaunchKernelGGL(gather_kernel, dim3(pb.M), dim3(256), 0, c->stream, g);
  LAUNCH_CHECK(c);
  const CopyBackArgs b = copyback_args(c);
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

smc_status smc_stage(smc_ctx c, double eps, int32_t L, int32_t R, double* a_out, double* dlogz_out,
                     double* ess_out) {
  if (!c) return SMC_ERR_INVALID_ARG;
  if (!(eps > 0.0) || L < 1 || R < 0) return fail(c, SMC_ERR_INVALID_ARG, "bad eps/L/R");
  const bool tempering = c->a < 1.0;
  double o[5] = {c->a, 0.0, 0.0, 0.0, 0.0};
  if (tempering) {
    const TemperArgs t = temper_args(c, c->pb.ess_frac, c->at<double>(c->lay.tout));
    HIP_TRY(c, launch_search(t, c->stream));
    hipLaunchKernelGGL(temper_kernel, dim3(1), dim3(kTemperThreads), 0, c->stream, t);
    LAUNCH_CHECK(c);
    HIP_TRY(c, hipMemcpyAsync(c->hstatus + 1, t.out, 5 * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipEventRecord(c->temper_ev, c->stream));
    // the mass matrix and the resampling need the new weights and the stage
    // number, not the exponent on the host: they are queued while it travels
    c->stage += 1;
    c->move = 0;
  }
  smc_status st = smc_mass(c);
  if (st != SMC_OK) return st;
  st = resample_impl(c, 0);
  if (st != SMC_OK) return st;
  if (tempering) {
    HIP_TRY(c, hipEventSynchronize(c->temper_ev));
    std::memcpy(o, c->hstatus + 1, sizeof(o));
    if (o[3] != 0.0) return fail(c, SMC_ERR_NONFINITE, "all incremental weights non-finite");
    c->a = o[0];
    c->logz += o[1];
  }
  st = smc_move(c, eps, L, R);
  if (st != SMC_OK) return st;
  if (a_out) *a_out = o[0];
  if (dlogz_out) *dlogz_out = o[1];
  if (ess_out) *ess_out = o[2];
  return SMC_OK;
}

smc_status smc_move(smc_ctx c, double eps, int32_t L, int32_t R) {
  if (!c) return SMC_ERR_INVALID_ARG;
  if (!(eps > 0.0) || L < 1 || R < 0) return fail(c, SMC_ERR_INVALID_ARG, "bad eps/L/R");
  {
    const smc_status ms = mass_ready(c);
    if (ms != SMC_OK) return ms;
  }
  if (!c->have_mass) return fail(c, SMC_ERR_STATE, "no mass matrix for this stage");
  if (c->move + R > 0xFFFF) return fail(c, SMC_ERR_INVALID_ARG, "too many moves in one stage");
  const int ring = (int)c->mev.size() / 2;
  for (int r = 0; r < R; ++r) {
    hipEvent_t* ev = ring > 0 ? &c->mev[2 * (c->mev_next % ring)] : nullptr;
    if (ev) HIP_TRY(c, hipEventRecord(ev[0], c->stream));
    HIP_TRY(c, launch_move(c, move_args(c, eps, L)));
    c->moved = 1;
    if (ev) {
      HIP_TRY(c, hipEventRecord(ev[1], c->stream));
      c->mev_next += 1;
      c->mev_count = std::min(c->mev_count + 1, ring);
    }
    c->move += 1;
  }
  return SMC_OK;
}

smc_status smc_autotune_move(smc_ctx c, double eps, int32_t L, int32_t* rpl_out, float* ms_out) {
  if (!c || !(eps > 0.0) || L < 1) return SMC_ERR_INVALID_ARG;
  {
    const smc_status ms = mass_ready(c);
    if (ms != SMC_OK) return ms;
  }
  if (!c->have_mass) return fail(c, SMC_ERR_STATE, "no mass matrix for this stage");
  const smc_problem& pb = c->pb;
  // the options: the streaming kernel and every resident layout that fits,
  // within the path the problem asked for
  std::vector<ResOption> opts;
  if (pb.move_path == SMC_MOVE_AUTO || pb.move_path == SMC_MOVE_STREAMING)
    for (int t = 0; t <= 2; ++t)
      if (wide_form_ok(pb, t)) opts.push_back(ResOption{-1, 0, ResLayout{}, t});
  if (pb.move_path != SMC_MOVE_STREAMING) {
    int dev = 0, max_lds = 0;
    HIP_TRY(c, hipGetDevice(&dev));
    HIP_TRY(c, hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    ResOption o[kResMaxOptions];
    const int n = resident_options(pb, max_lds, o);
    for (int q = 0; q < n; ++q) opts.push_back(o[q]);
  }
  const size_t M = pb.M, d = pb.d, m = pb.m;
  struct Buf { void* live; void* saved; size_t bytes; };
  const Buf bufs[6] = {{pb.theta, c->at<double>(c->lay.th2), M * d * 8}, {pb.u, c->at<int32_t>(c->lay.u2), M * m * 4},
                       {pb.lhat, c->at<double>(c->lay.lh2), M * 8}, {pb.sig2, c->at<double>(c->lay.sg2), M * 8},
                       {c->at<double>(c->lay.grad_l), c->at<double>(c->lay.gl2), M * d * 8},
                       {c->at<double>(c->lay.grad_s), c->at<double>(c->lay.gs2), M * d * 8}};
  // the accept flags go through host memory (no spare device buffer of their
  // size); plain synchronous copies after the stream has drained
  std::vector<int32_t> acc(M * 2);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, hipMemcpy(acc.data(), pb.accept, M * 2 * 4, hipMemcpyDeviceToHost));
  for (const Buf& b : bufs) HIP_TRY(c, hipMemcpyAsync(b.saved, b.live, b.bytes, hipMemcpyDeviceToDevice, c->stream));
  auto restore = [&]() -> hipError_t {
    for (const Buf& b : bufs) {
      const hipError_t e = hipMemcpyAsync(b.live, b.saved, b.bytes, hipMemcpyDeviceToDevice, c->stream);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  const int move0 = c->move, rpl0 = c->res_rpl, mf0 = c->res_mf, tile0 = c->wide_tile;
  const ResLayout ly0 = c->res_ly;
  std::vector<hipEvent_t> ev(2 * opts.size(), nullptr);
  for (hipEvent_t& e : ev) HIP_TRY(c, hipEventCreate(&e));
  hipError_t err = hipSuccess;
  for (size_t q = 0; q < opts.size() && err == hipSuccess; ++q) {
    c->res_rpl = opts[q].rpl;
    c->res_mf = opts[q].mf;
    c->res_ly = opts[q].ly;
    c->wide_tile = opts[q].rpl < 0 ? opts[q].tile : tile0;
    // a first launch absorbs one-time costs, the second is timed; both
    // start from the saved state
    for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) {
      if ((err = restore()) != hipSuccess) break;
      if (rep == 1 && (err = hipEventRecord(ev[2 * q], c->stream)) != hipSuccess) break;
      err = launch_move(c, move_args(c, eps, L));
      if (err == hipSuccess && rep == 1) err = hipEventRecord(ev[2 * q + 1], c->stream);
    }
  }
  if (err == hipSuccess) err = restore();
  if (err == hipSuccess) err = hipStreamSynchronize(c->stream);
  if (err == hipSuccess) err = hipMemcpy(pb.accept, acc.data(), M * 2 * 4, hipMemcpyHostToDevice);
  c->move = move0;
  int best = -1;
  float best_ms = 0.f;
  for (size_t q = 0; q < opts.size() && err == hipSuccess; ++q) {
    float t = 0.f;
    err = hipEventElapsedTime(&t, ev[2 * q], ev[2 * q + 1]);
    if (ms_out) ms_out[q] = t;
    if (best < 0 || t < best_ms) {
      best = (int)q;
      best_ms = t;
    }
  }
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  if (err != hipSuccess || best < 0) {
    c->res_rpl = rpl0;
    c->res_mf = mf0;
    c->res_ly = ly0;
    c->wide_tile = tile0;
    HIP_TRY(c, err);
    return fail(c, SMC_ERR_STATE, "no move kernel to tune");
  }
  c->res_rpl = opts[best].rpl;
  c->res_mf = opts[best].mf;
  c->res_ly = opts[best].ly;
  c->wide_tile = opts[best].rpl < 0 ? opts[best].tile : tile0;
  if (rpl_out) *rpl_out = opts[best].rpl;
  return SMC_OK;
}

smc_status smc_set_move_option(smc_ctx c, int32_t res_rows, int32_t res_mfma, int32_t stream_tile) {
  if (!c) return SMC_ERR_INVALID_ARG;
  const smc_problem& pb = c->pb;
  if (res_rows < 0) {
    if (pb.move_path == SMC_MOVE_RESIDENT || pb.move_path == SMC_MOVE_RESIDENT_MFMA)
      return fail(c, SMC_ERR_UNSUPPORTED, "the problem asks for the resident move");
    if (!wide_form_ok(pb, stream_tile))
      return fail(c, SMC_ERR_UNSUPPORTED, "no tile form %d for this problem", stream_tile);
    c->res_rpl = -1;
    c->res_mf = 0;
    c->wide_tile = stream_tile;
    return SMC_OK;
  }
  if (pb.move_path == SMC_MOVE_STREAMING) return fail(c, SMC_ERR_UNSUPPORTED, "the problem asks for the streaming move");
  int dev = 0, max_lds = 0;
  HIP_TRY(c, hipGetDevice(&dev));
  HIP_TRY(c, hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  ResOption o[kResMaxOptions];
  const int n = resident_options(pb, max_lds, o);
  for (int q = 0; q < n; ++q) {
    if (o[q].rpl == res_rows && o[q].mf == res_mfma) {
      c->res_rpl = o[q].rpl;
      c->res_mf = o[q].mf;
      c->res_ly = o[q].ly;
      return SMC_OK;
    }
  }
  return fail(c, SMC_ERR_UNSUPPORTED, "no resident layout with %d register rows (matrix cores %d) fits", res_rows,
              res_mfma);
}

smc_status smc_set_move_timing(smc_ctx c, int32_t n) {
  if (!c || n < 0 || n > 4096) return SMC_ERR_INVALID_ARG;
  for (hipEvent_t e : c->mev) (void)hipEventDestroy(e);
  c->mev.clear();
  c->mev_next = c->mev_count = 0;
  for (int k = 0; k < 2 * n; ++k) {
    hipEvent_t e;
    HIP_TRY(c, hipEventCreate(&e));
    c->mev.push_back(e);
  }
  return SMC_OK;
}

smc_status smc_move_times(smc_ctx c, int32_t cap, float* ms, int32_t* count) {
  if (!c || !count || (cap > 0 && !ms)) return SMC_ERR_INVALID_ARG;
  const int ring = (int)c->mev.size() / 2;
  const int n = std::min(c->mev_count, cap);
  *count = n;
  for (int k = 0; k < n; ++k) {
    const int slot = (c->mev_next - n + k) % ring;
    const hipEvent_t* ev = &c->mev[2 * slot];
    HIP_TRY(c, hipEventSynchronize(ev[1]));
    HIP_TRY(c, hipEventElapsedTime(&ms[k], ev[0], ev[1]));
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

smc_status loglik_lambda(smc_ctx c, int32_t count, const double* theta, const int32_t* u, double a, double* lam,
                         double* lhat, double* sig2) {
  if (!c || count < 0 || (count > 0 && (!theta || !u || !lam))) return SMC_ERR_INVALID_ARG;
  if (!(a >= 0.0 && a <= 1.0)) return fail(c, SMC_ERR_INVALID_ARG, "exponent must be in [0, 1]");
  EstArgs e;
  std::memset(&e, 0, sizeof(e));
  e.P = c->prob;
  e.count = count;
  e.theta = theta;
  e.u = u;
  e.lhat = lhat;
  e.sig2 = sig2;
  e.a = a;
  e.lam = lam;
  HIP_TRY(c, launch_estimator(c, count, e));
  return SMC_OK;
}

smc_status smc_move_diag(smc_ctx c, double* diag) {
  if (!c || !diag) return SMC_ERR_INVALID_ARG;
  if (!c->moved) return fail(c, SMC_ERR_STATE, "no move has run on this context");
  HIP_TRY(c, hipMemcpyAsync(diag, c->at<double>(c->lay.diag), (size_t)c->pb.M * 32, hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return SMC_OK;
}

smc_status smc_move_stats(smc_ctx c, double* accept_u, double* accept_theta, int64_t* near_ties_u,
                          int64_t* near_ties_theta) {
  if (!c) return SMC_ERR_INVALID_ARG;
  if (!c->moved) return fail(c, SMC_ERR_STATE, "no move has run on this context");
  const size_t M = c->pb.M;
  std::vector<int32_t> acc(M * 2), tie(M * 2);
  HIP_TRY(c, hipMemcpyAsync(acc.data(), c->pb.accept, M * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(tie.data(), c->at<int32_t>(c->lay.ties), M * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  int64_t au = 0, at = 0, tu = 0, tt = 0;
  for (size_t i = 0; i < M; ++i) {
    au += acc[2 * i] != 0;
    at += acc[2 * i + 1] != 0;
    tu += tie[2 * i] != 0;
    tt += tie[2 * i + 1] != 0;
  }
  if (accept_u) *accept_u = (double)au / (double)M;
  if (accept_theta) *accept_theta = (double)at / (double)M;
  if (near_ties_u) *near_ties_u = tu;
  if (near_ties_theta) *near_ties_theta = tt;
  return SMC_OK;
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
    const smc_status ms = mass_ready(c);
    if (ms != SMC_OK) return ms;
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
  (void)mass_ready(c);  // a failed factorisation shows as have_mass = 0
  o->have_mass = c->have_mass;
  o->newton_iters = c->newton_iters;
  o->move_path = c->res_rpl >= 0 ? SMC_MOVE_RESIDENT : SMC_MOVE_STREAMING;
  o->res_rows = c->res_rpl;
  o->res_mfma = c->res_rpl >= 0 ? c->res_mf : 0;
  o->stream_tile = c->wide_tile;
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

// ------------------------------------------------------------------------
// checkpoint and resume
// ------------------------------------------------------------------------

}  // extern "C"

namespace {

constexpr uint64_t kStateMagic = 0x5453434D53425553ull;  // "SUBSMCST"
constexpr uint32_t kStateVersion = 3;

struct StateHeader {
  uint64_t magic;
  uint32_t version;
  int32_t family, precision, cv_order, d, M, m, G;
  uint32_t dataset;
  int64_t n;
  uint64_t seed;
  int32_t stage, move, have_mass, res_rpl, res_mf, wide_tile, newton_iters, moved;
  double a, logz;
  uint64_t bytes;
};

// the arrays of a state blob, in blob order: (device pointer, bytes)
std::vector<std::pair<char*, size_t>> state_arrays(smc_ctx c) {
  const size_t M = c->pb.M, d = c->pb.d, m = c->pb.m, dd = d * d * 8;
  return {{const_cast<char*>(reinterpret_cast<const char*>(c->prob.theta_bar)), d * 8},
          {c->at<char>(c->lay.Sigma), dd},
          {c->at<char>(c->lay.Lchol), dd},
          {c->at<char>(c->lay.Linv), dd},
          {c->at<char>(c->lay.mean), d * 8},
          {reinterpret_cast<char*>(c->pb.theta), M * d * 8},
          {reinterpret_cast<char*>(c->pb.u), M * m * 4},
          {reinterpret_cast<char*>(c->pb.logw), M * 8},
          {reinterpret_cast<char*>(c->pb.lhat), M * 8},
          {reinterpret_cast<char*>(c->pb.sig2), M * 8},
          {c->at<char>(c->lay.grad_l), M * d * 8},
          {c->at<char>(c->lay.grad_s), M * d * 8},
          {reinterpret_cast<char*>(c->pb.accept), M * 8},
          {c->at<char>(c->lay.ties), M * 8},
          {c->at<char>(c->lay.diag), M * 32}};
}

size_t state_bytes(smc_ctx c) {
  size_t total = sizeof(StateHeader);
  for (const auto& a : state_arrays(c)) total += a.second;
  return total;
}

StateHeader state_identity(smc_ctx c) {
  StateHeader h;
  std::memset(&h, 0, sizeof(h));
  h.magic = kStateMagic;
  h.version = kStateVersion;
  h.family = c->pb.family;
  h.precision = c->pb.precision;
  h.cv_order = c->pb.cv_order;
  h.d = c->pb.d;
  h.M = c->pb.M;
  h.m = c->pb.m;
  h.G = c->pb.G;
  h.dataset = c->pb.dataset;
  h.n = c->pb.n;
  h.seed = c->pb.seed;
  h.bytes = state_bytes(c);
  return h;
}

}  // namespace

extern "C" {

smc_status smc_get_state(smc_ctx c, void* blob, size_t* bytes) {
  if (!c || !bytes) return SMC_ERR_INVALID_ARG;
  const size_t need = state_bytes(c);
  if (!blob) {
    *bytes = need;
    return SMC_OK;
  }
  if (*bytes < need) return fail(c, SMC_ERR_INVALID_ARG, "state blob needs %zu bytes", need);
  (void)mass_ready(c);  // a failed factorisation is saved as no mass matrix
  StateHeader h = state_identity(c);
  h.stage = c->stage;
  h.move = c->move;
  h.have_mass = c->have_mass;
  h.res_rpl = c->res_rpl;
  h.res_mf = c->res_mf;
  h.wide_tile = c->wide_tile;
  h.newton_iters = c->newton_iters;
  h.moved = c->moved;
  h.a = c->a;
  h.logz = c->logz;
  char* out = static_cast<char*>(blob);
  std::memcpy(out, &h, sizeof(h));
  size_t off = sizeof(h);
  for (const auto& a : state_arrays(c)) {
    HIP_TRY(c, hipMemcpyAsync(out + off, a.first, a.second, hipMemcpyDeviceToHost, c->stream));
    off += a.second;
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  *bytes = need;
  return SMC_OK;
}

smc_status smc_set_state(smc_ctx c, const void* blob, size_t bytes) {
  if (!c || !blob) return SMC_ERR_INVALID_ARG;
  StateHeader h;
  if (bytes < sizeof(h)) return fail(c, SMC_ERR_INVALID_ARG, "state blob too short");
  std::memcpy(&h, blob, sizeof(h));
  const StateHeader id = state_identity(c);
  if (h.magic != id.magic || h.version != id.version)
    return fail(c, SMC_ERR_INVALID_ARG, "not a state blob of this library version");
  if (h.family != id.family || h.precision != id.precision || h.cv_order != id.cv_order || h.d != id.d ||
      h.M != id.M || h.m != id.m || h.G != id.G || h.dataset != id.dataset || h.n != id.n || h.seed != id.seed)
    return fail(c, SMC_ERR_INVALID_ARG, "state blob belongs to a different problem");
  if (h.bytes != id.bytes || bytes < h.bytes) return fail(c, SMC_ERR_INVALID_ARG, "state blob size mismatch");
  if (h.stage < 0 || h.move < 0 || !(h.a >= 0.0 && h.a <= 1.0) || h.have_mass < 0 || h.have_mass > 1)
    return fail(c, SMC_ERR_INVALID_ARG, "state blob holds invalid counters");
  if (!wide_form_ok(c->pb, h.wide_tile))
    return fail(c, SMC_ERR_INVALID_ARG, "state blob holds an unknown tile form");
  // the move kernel: streaming, or a resident layout that fits this device
  ResLayout ly{};
  if (h.res_rpl >= 0) {
    if (c->pb.move_path == SMC_MOVE_STREAMING) return fail(c, SMC_ERR_INVALID_ARG, "state uses the resident move");
    int dev = 0, max_lds = 0;
    HIP_TRY(c, hipGetDevice(&dev));
    HIP_TRY(c, hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    ResOption o[kResMaxOptions];
    const int n = resident_options(c->pb, max_lds, o);
    int q = 0;
    while (q < n && !(o[q].rpl == h.res_rpl && o[q].mf == h.res_mf)) ++q;
    if (q == n) return fail(c, SMC_ERR_INVALID_ARG, "state's resident layout does not fit this device");
    ly = o[q].ly;
  } else if (c->pb.move_path == SMC_MOVE_RESIDENT || c->pb.move_path == SMC_MOVE_RESIDENT_MFMA) {
    return fail(c, SMC_ERR_INVALID_ARG, "state uses the streaming move");
  }
  // settle anything in flight on the stream before overwriting its buffers
  if (c->have_mass == 2) HIP_TRY(c, hipEventSynchronize(c->mass_ev));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int d = c->pb.d;
  const char* in = static_cast<const char*>(blob) + sizeof(h);
  // control-variate centre: rebuild A, B, C and the packed rows when it moved
  std::vector<double> tb_now(d);
  HIP_TRY(c, hipMemcpy(tb_now.data(), c->prob.theta_bar, (size_t)d * 8, hipMemcpyDeviceToHost));
  const bool recentre = std::memcmp(tb_now.data(), in, (size_t)d * 8) != 0;
  size_t off = 0;
  for (const auto& a : state_arrays(c)) {
    HIP_TRY(c, hipMemcpyAsync(a.first, in + off, a.second, hipMemcpyHostToDevice, c->stream));
    off += a.second;
  }
  if (recentre) {
    double* tb = const_cast<double*>(c->prob.theta_bar);
    smc_status st = run_cv(c, tb, true, const_cast<double*>(c->prob.cvA), const_cast<double*>(c->prob.cvB),
                           const_cast<double*>(c->prob.cvC));
    if (st != SMC_OK) return st;
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->stage = h.stage;
  c->move = h.move;
  c->a = h.a;
  c->logz = h.logz;
  c->have_mass = h.have_mass;
  c->res_rpl = h.res_rpl;
  c->res_mf = h.res_rpl >= 0 ? h.res_mf : 0;
  c->res_ly = ly;
  c->wide_tile = h.wide_tile;
  c->newton_iters = h.newton_iters;
  c->moved = h.moved;
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

// ------------------------------------------------------------------------
// batches
// ------------------------------------------------------------------------

}  // extern "C"

namespace {

constexpr size_t kBatchArgBytes = 512;  // bound on every argument block
static_assert(sizeof(ResMoveArgs) <= kBatchArgBytes && sizeof(MoveArgs) <= kBatchArgBytes &&
                  sizeof(TemperArgs) <= kBatchArgBytes && sizeof(MomentArgs) <= kBatchArgBytes &&
                  sizeof(ResampleArgs) <= kBatchArgBytes && sizeof(GatherArgs) <= kBatchArgBytes &&
                  sizeof(CopyBackArgs) <= kBatchArgBytes,
              "argument block larger than its table slot");
constexpr size_t kBatchResultDoubles = 8;  // per member

// the most any step stages: three tables of count blocks, a prefix array
// per table and per move group, each placement 256-byte aligned
size_t batch_table_bytes(int count) { return (size_t)count * (3 * kBatchArgBytes + 1024) + 4096; }

smc_status bfail(smc_batch b, smc_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(b->err, sizeof(b->err), fmt, ap);
  va_end(ap);
  return s;
}

#define BATCH_TRY(b, expr)                                                                     \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return bfail(b, SMC_ERR_DEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),    \
                   __FILE__, __LINE__);                                                        \
  } while (0)

// Argument tables of one step, laid out on the host and uploaded in one copy
// on the batch's stream (kernels launched earlier on that stream have read
// the previous tables by the time it lands).
class Tables {
 public:
  explicit Tables(smc_batch b) : b_(b) {}
  template <typename T>
  size_t put(const std::vector<T>& v) {
    const size_t off = align256(buf_.size());
    buf_.resize(off + v.size() * sizeof(T));
    std::memcpy(buf_.data() + off, v.data(), v.size() * sizeof(T));
    return off;
  }
  template <typename T>
  const T* at(size_t off) const { return reinterpret_cast<const T*>(b_->dev + off); }
  smc_status upload() {
    if (buf_.size() > b_->table_bytes) return bfail(b_, SMC_ERR_UNSUPPORTED, "argument tables exceed the workspace");
    // the staging buffer is reused: wait until the previous upload has read it
    BATCH_TRY(b_, hipEventSynchronize(b_->staged));
    std::memcpy(b_->host, buf_.data(), buf_.size());
    BATCH_TRY(b_, hipMemcpyAsync(b_->dev, b_->host, buf_.size(), hipMemcpyHostToDevice, b_->stream));
    BATCH_TRY(b_, hipEventRecord(b_->staged, b_->stream));
    return SMC_OK;
  }

 private:
  smc_batch b_;
  std::vector<char> buf_;
};

double* batch_results_dev(smc_batch b) { return reinterpret_cast<double*>(b->dev + b->table_bytes); }

// the persistent move's queues (two counters per launch) after the results
constexpr int kPersistQueues = 8;
size_t batch_results_bytes(int count) { return align256((size_t)count * kBatchResultDoubles * 8); }
int32_t* batch_queue_dev(smc_batch b) {
  return reinterpret_cast<int32_t*>(b->dev + b->table_bytes + batch_results_bytes((int)b->ctx.size()));
}
double* batch_results_host(smc_batch b) { return reinterpret_cast<double*>(b->host + b->table_bytes); }

// results of the active members (kBatchResultDoubles each) to the host; synchronises
smc_status batch_fetch(smc_batch b) {
  const size_t bytes = b->active.size() * kBatchResultDoubles * 8;
  BATCH_TRY(b, hipMemcpyAsync(batch_results_host(b), batch_results_dev(b), bytes, hipMemcpyDeviceToHost, b->stream));
  BATCH_TRY(b, hipStreamSynchronize(b->stream));
  return SMC_OK;
}

template <typename T>
Batch<T> batch_of(const Tables& t, size_t args_off, size_t first_off, int count) {
  Batch<T> r;
  r.args = t.at<T>(args_off);
  r.first = t.at<int>(first_off);
  r.count = count;
  return r;
}

// LDS a workgroup of the persistent move may take: with float rows two
// workgroups share a CU (the streaming kernels' two wavefronts per SIMD), with
// double rows one does; 2 KB of each share stays for static LDS
constexpr size_t kPersistLdsF32 = 78 * 1024;
constexpr size_t kPersistLdsF64 = 156 * 1024;

// the streaming form of a member's move (its kernel when the resident layout
// does not apply)
KernelShape stream_shape(smc_ctx c) {
  KernelShape s = member_shape(c);
  s.kind = c->pb.d > kMaxNarrowD ? kMoveWide : kMoveNarrow;
  s.rpl = -1;
  s.mf = 0;
  s.tile = s.kind == kMoveWide && c->wide_tile != 2 ? c->wide_tile : 0;
  return s;
}

// One move of every active member in one persistent launch per (row type,
// family): members costliest first, items numbered in that order.
smc_status batch_move_persistent(smc_batch b, const double* eps, int32_t L, int32_t R) {
  struct Mem {
    int k;
    KernelShape s;
    int body;
    bool res;
    double cost;  // of one item
  };
  std::map<std::pair<int, int>, std::vector<Mem>> groups;
  b->member_kind.assign(b->ctx.size(), -1);
  b->member_launch.assign(b->ctx.size(), -1);
  for (int k : b->active) {
    smc_ctx c = b->ctx[k];
    KernelShape s = member_shape(c);
    const size_t cap = s.fp32 ? kPersistLdsF32 : kPersistLdsF64;
    int body = -1;
    if (s.kind == kMoveResident && (size_t)c->res_ly.total <= cap) body = persist_body(s);
    if (body < 0) {
      s = stream_shape(c);
      body = persist_body(s);
    }
    if (body < 0) return bfail(b, SMC_ERR_UNSUPPORTED, "member %d: no body in the persistent move", k);
    const bool res = s.kind == kMoveResident;
    // bytes a particle's move streams; a resident item spreads them over the workgroup
    const double rows = (double)c->pb.m * (L + 1) * (c->pb.d + 4) * (s.fp32 ? 4.0 : 8.0);
    groups[{s.fp32, s.fam}].push_back(Mem{k, s, body, res, res ? rows / kPersistWaves : rows});
    b->member_kind[k] = s.kind;
  }
  if (!b->cus) {
    int dev = 0;
    BATCH_TRY(b, hipGetDevice(&dev));
    BATCH_TRY(b, hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev));
  }
  const int ng = (int)groups.size();
  if (ng > kPersistQueues) return bfail(b, SMC_ERR_UNSUPPORTED, "%d persistent launches, at most %d", ng, kPersistQueues);
  b->launch_kind.assign(ng, kMovePersistent);
  b->timed_moves = 0;
  if (b->timing) {
    const size_t need = (size_t)2 * ng * R;
    while (b->ev.size() < need) {
      hipEvent_t e;
      BATCH_TRY(b, hipEventCreate(&e));
      b->ev.push_back(e);
    }
  }
  for (int r = 0; r < R; ++r) {
    Tables T(b);
    struct Launch {
      int fp32, fam, grid, count, n_items;
      size_t lds, off, foff;
    };
    std::vector<Launch> launches;
    int gi = 0;
    for (auto& g : groups) {
      std::vector<Mem>& mem = g.second;
      std::stable_sort(mem.begin(), mem.end(), [](const Mem& x, const Mem& y) { return x.cost > y.cost; });
      std::vector<PersistMember> pm(mem.size());
      std::vector<int32_t> first(mem.size() + 1, 0);
      size_t lds = 0;
      for (size_t q = 0; q < mem.size(); ++q) {
        smc_ctx c = b->ctx[mem[q].k];
        const KernelShape& s = mem[q].s;
        PersistMember& p = pm[q];
        std::memset(&p, 0, sizeof(p));
        p.A = move_args(c, eps[mem[q].k], L);
        p.body = mem[q].body;
        p.resident = mem[q].res ? 1 : 0;
        int items;
        if (mem[q].res) {
          p.Ly = c->res_ly;
          lds = std::max(lds, (size_t)c->res_ly.total);
          items = c->pb.M;
        } else {
          const bool wide = s.kind == kMoveWide;
          p.wave_lds = persist_wave_lds(wide, wide ? s.ch : s.dc, s.fp32 ? 4 : 8,
                                        (c->pb.m + c->pb.G - 1) / c->pb.G);
          lds = std::max(lds, (size_t)kPersistWaves * p.wave_lds);
          items = (c->pb.M + kPersistWaves - 1) / kPersistWaves;
        }
        first[q + 1] = first[q] + items;
        b->member_launch[mem[q].k] = gi;
      }
      int per_cu = 0;
      BATCH_TRY(b, persist_occupancy(g.first.first, g.first.second, lds, &per_cu));
      if (per_cu < 1) return bfail(b, SMC_ERR_UNSUPPORTED, "persistent move: %zu bytes of LDS do not fit", lds);
      Launch l;
      l.fp32 = g.first.first;
      l.fam = g.first.second;
      l.count = (int)mem.size();
      l.n_items = first.back();
      l.grid = std::min(per_cu * b->cus, l.n_items);
      l.lds = lds;
      l.off = T.put(pm);
      l.foff = T.put(first);
      launches.push_back(l);
      ++gi;
    }
    smc_status st = T.upload();
    if (st != SMC_OK) return st;
    auto issue = [&](size_t li, hipStream_t s) -> hipError_t {
      const Launch& l = launches[li];
      PersistArgs a;
      a.mem = T.at<PersistMember>(l.off);
      a.first = T.at<int32_t>(l.foff);
      a.count = l.count;
      a.n_items = l.n_items;
      a.queue = batch_queue_dev(b) + 2 * li;
      return launch_move_persist(l.fp32, l.fam, l.grid, l.lds, a, s);
    };
    if (b->use_graph && !b->timing) {
      std::vector<long long> key{-1};
      for (const Launch& l : launches) {
        const long long v[8] = {l.fp32, l.fam, l.grid, l.count, l.n_items, (long long)l.lds, (long long)l.off,
                                (long long)l.foff};
        key.insert(key.end(), v, v + 8);
      }
      if (!b->gexec || key != b->graph_key) {
        if (b->gexec) {
          BATCH_TRY(b, hipGraphExecDestroy(b->gexec));
          b->gexec = nullptr;
        }
        if (!b->capture) BATCH_TRY(b, hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
        BATCH_TRY(b, hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
        hipError_t le = hipSuccess;
        for (size_t li = 0; li < launches.size() && le == hipSuccess; ++li) le = issue(li, b->capture);
        hipGraph_t gr = nullptr;
        const hipError_t ce = hipStreamEndCapture(b->capture, &gr);
        BATCH_TRY(b, le);
        BATCH_TRY(b, ce);
        const hipError_t ie = hipGraphInstantiate(&b->gexec, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        BATCH_TRY(b, ie);
        b->graph_key = key;
        b->graph_captures += 1;
      }
      BATCH_TRY(b, hipGraphLaunch(b->gexec, b->stream));
    } else {
      for (size_t li = 0; li < launches.size(); ++li) {
        hipEvent_t* ev = b->timing ? &b->ev[2 * ((size_t)r * ng + li)] : nullptr;
        if (ev) BATCH_TRY(b, hipEventRecord(ev[0], b->stream));
        BATCH_TRY(b, issue(li, b->stream));
        if (ev) BATCH_TRY(b, hipEventRecord(ev[1], b->stream));
      }
    }
    for (int k : b->active) {
      b->ctx[k]->move += 1;
      b->ctx[k]->moved = 1;
    }
    if (b->timing) b->timed_moves += 1;
  }
  return SMC_OK;
}

}  // namespace

extern "C" {

size_t smc_batch_workspace_size(int32_t count) {
  if (count < 1 || count > kMaxBatch) return 0;
  return align256(batch_table_bytes(count)) + batch_results_bytes(count) + 256;
}

smc_status smc_batch_create(const smc_ctx* ctxs, int32_t count, void* workspace, size_t workspace_bytes,
                            smc_batch* out) {
  if (!out) return SMC_ERR_INVALID_ARG;
  *out = nullptr;
  if (!ctxs || count < 1 || count > kMaxBatch || !workspace) return SMC_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return SMC_ERR_INVALID_ARG;
  const size_t need = smc_batch_workspace_size(count);
  if (workspace_bytes < need) return SMC_ERR_INVALID_ARG;
  for (int k = 0; k < count; ++k) {
    if (!ctxs[k] || ctxs[k]->stream != ctxs[0]->stream) return SMC_ERR_INVALID_ARG;
    for (int q = 0; q < k; ++q)
      if (ctxs[q] == ctxs[k]) return SMC_ERR_INVALID_ARG;
  }
  smc_batch b = new (std::nothrow) smc_batch_s;
  if (!b) return SMC_ERR_DEVICE;
  b->ctx.assign(ctxs, ctxs + count);
  b->stream = ctxs[0]->stream;
  b->dev = static_cast<char*>(workspace);
  b->table_bytes = align256(batch_table_bytes(count));
  if (hipHostMalloc(reinterpret_cast<void**>(&b->host), need, hipHostMallocDefault) != hipSuccess) {
    delete b;
    return SMC_ERR_DEVICE;
  }
  // the persistent move's queues start at zero (each launch leaves them so)
  if (hipMemsetAsync(batch_queue_dev(b), 0, 2 * kPersistQueues * sizeof(int32_t), b->stream) != hipSuccess ||
      hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(b->staged, b->stream) != hipSuccess) {
    if (b->staged) (void)hipEventDestroy(b->staged);
    (void)hipHostFree(b->host);
    delete b;
    return SMC_ERR_DEVICE;
  }
  *out = b;
  return SMC_OK;
}

smc_status smc_batch_temper(smc_batch b, double* a_out, double* dlogz_out, double* ess_out, int32_t* active_out) {
  if (!b) return SMC_ERR_INVALID_ARG;
  const int count = (int)b->ctx.size();
  b->active.clear();
  b->have_stage = 0;
  for (int k = 0; k < count; ++k)
    if (b->ctx[k]->a < 1.0) b->active.push_back(k);
  for (int k = 0; k < count; ++k) {
    if (a_out) a_out[k] = b->ctx[k]->a;
    if (dlogz_out) dlogz_out[k] = 0.0;
    if (ess_out) ess_out[k] = 0.0;
    if (active_out) active_out[k] = 0;
  }
  if (b->active.empty()) return bfail(b, SMC_ERR_STATE, "every member has reached a = 1");
  const int na = (int)b->active.size();
  std::vector<TemperArgs> ta(na);
  for (int q = 0; q < na; ++q) {
    smc_ctx c = b->ctx[b->active[q]];
    ta[q] = temper_args(c, c->pb.ess_frac, batch_results_dev(b) + (size_t)q * kBatchResultDoubles);
  }
  Tables T(b);
  const size_t off = T.put(ta);
  smc_status st = T.upload();
  if (st != SMC_OK) return st;
  Batch<TemperArgs> bt;
  bt.args = T.at<TemperArgs>(off);
  bt.first = nullptr;
  bt.count = na;
  for (int pass = 0; pass < kSearchPasses; ++pass) {
    hipLaunchKernelGGL(search_pass_kernel_batch, dim3(na * pass_groups(pass)), dim3(kSearchThreadsBatch), 0, b->stream,
                       bt, pass);
    BATCH_TRY(b, hipGetLastError());
  }
  hipLaunchKernelGGL(temper_kernel_batch, dim3(na), dim3(kTemperThreads), 0, b->stream, bt);
  BATCH_TRY(b, hipGetLastError());
  if ((st = batch_fetch(b)) != SMC_OK) return st;
  int bad = -1;
  for (int q = 0; q < na; ++q) {
    const int k = b->active[q];
    const double* o = batch_results_host(b) + (size_t)q * kBatchResultDoubles;
    if (o[3] != 0.0) {
      if (bad < 0) bad = k;
      continue;
    }
    temper_commit(b->ctx[k], o);
    if (a_out) a_out[k] = o[0];
    if (dlogz_out) dlogz_out[k] = o[1];
    if (ess_out) ess_out[k] = o[2];
    if (active_out) active_out[k] = 1;
  }
  if (bad >= 0) return bfail(b, SMC_ERR_NONFINITE, "member %d: all incremental weights non-finite", bad);
  b->have_stage = 1;
  return SMC_OK;
}

smc_status smc_batch_mass(smc_batch b) {
  if (!b) return SMC_ERR_INVALID_ARG;
  if (!b->have_stage) return bfail(b, SMC_ERR_STATE, "no tempered stage");
  const int na = (int)b->active.size();
  std::vector<MomentArgs> ma(na);
  std::vector<int> first(na + 1, 0);
  size_t lds_p = 0, lds_f = 0;
  for (int q = 0; q < na; ++q) {
    smc_ctx c = b->ctx[b->active[q]];
    ma[q] = moment_args(c, batch_results_dev(b) + (size_t)q * kBatchResultDoubles);
    first[q + 1] = first[q] + ma[q].nblocks;
    lds_p = std::max(lds_p, moments_partial_lds(c->pb.d));
    lds_f = std::max(lds_f, moments_final_lds(c->pb.d));
  }
  Tables T(b);
  const size_t off = T.put(ma), foff = T.put(first);
  smc_status st = T.upload();
  if (st != SMC_OK) return st;
  const Batch<MomentArgs> bm = batch_of<MomentArgs>(T, off, foff, na);
  BATCH_TRY(b, hipFuncSetAttribute(reinterpret_cast<const void*>(moments_partial_kernel_batch),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_p));
  hipLaunchKernelGGL(moments_partial_kernel_batch, dim3(first[na]), dim3(kMomThreads), lds_p, b->stream, bm);
  BATCH_TRY(b, hipGetLastError());
  BATCH_TRY(b, hipFuncSetAttribute(reinterpret_cast<const void*>(moments_final_kernel_batch),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_f));
  hipLaunchKernelGGL(moments_final_kernel_batch, dim3(na), dim3(kMomThreads), lds_f, b->stream, bm);
  BATCH_TRY(b, hipGetLastError());
  if ((st = batch_fetch(b)) != SMC_OK) return st;
  int bad = -1;
  for (int q = 0; q < na; ++q) {
    if (batch_results_host(b)[(size_t)q * kBatchResultDoubles] != 0.0) {
      if (bad < 0) bad = b->active[q];
      continue;
    }
    b->ctx[b->active[q]]->have_mass = 1;
  }
  if (bad >= 0) return bfail(b, SMC_ERR_NOT_PD, "member %d: particle covariance not positive definite", bad);
  return SMC_OK;
}

smc_status smc_batch_resample(smc_batch b, int32_t multinomial) {
  if (!b || (multinomial != 0 && multinomial != 1)) return SMC_ERR_INVALID_ARG;
  if (!b->have_stage) return bfail(b, SMC_ERR_STATE, "no tempered stage");
  const int na = (int)b->active.size();
  std::vector<ResampleArgs> ra(na);
  std::vector<GatherArgs> ga(na);
  std::vector<CopyBackArgs> ca(na);
  std::vector<int> first(na + 1, 0);
  for (int q = 0; q < na; ++q) {
    smc_ctx c = b->ctx[b->active[q]];
    ra[q] = resample_args(c, multinomial);
    ga[q] = gather_args(c);
    ca[q] = copyback_args(c);
    first[q + 1] = first[q] + c->pb.M;
  }
  Tables T(b);
  const size_t roff = T.put(ra), goff = T.put(ga), coff = T.put(ca), foff = T.put(first);
  smc_status st = T.upload();
  if (st != SMC_OK) return st;
  const Batch<ResampleArgs> br = batch_of<ResampleArgs>(T, roff, foff, na);
  hipLaunchKernelGGL(resample_kernel_batch, dim3(na), dim3(kResThreads), 0, b->stream, br);
  BATCH_TRY(b, hipGetLastError());
  const Batch<GatherArgs> bg = batch_of<GatherArgs>(T, goff, foff, na);
  hipLaunchKernelGGL(gather_kernel_batch, dim3(first[na]), dim3(256), 0, b->stream, bg);
  BATCH_TRY(b, hipGetLastError());
  const Batch<CopyBackArgs> bc = batch_of<CopyBackArgs>(T, coff, foff, na);
  hipLaunchKernelGGL(copyback_kernel_batch, dim3(first[na]), dim3(256), 0, b->stream, bc);
  BATCH_TRY(b, hipGetLastError());
  return SMC_OK;
}

smc_status smc_batch_move(smc_batch b, const double* eps, int32_t L, int32_t R) {
  if (!b || !eps || L < 1 || R < 0) return SMC_ERR_INVALID_ARG;
  if (!b->have_stage) return bfail(b, SMC_ERR_STATE, "no tempered stage");
  for (int k : b->active) {
    smc_ctx c = b->ctx[k];
    if (!(eps[k] > 0.0)) return bfail(b, SMC_ERR_INVALID_ARG, "member %d: eps must be positive", k);
    if (mass_ready(c) != SMC_OK) return bfail(b, SMC_ERR_NOT_PD, "member %d: particle covariance not positive definite", k);
    if (!c->have_mass) return bfail(b, SMC_ERR_STATE, "member %d: no mass matrix for this stage", k);
    if (c->move + R > 0xFFFF) return bfail(b, SMC_ERR_INVALID_ARG, "member %d: too many moves in one stage", k);
  }
  if (b->persistent) return batch_move_persistent(b, eps, L, R);
  // members grouped by kernel shape: one launch per group
  std::map<KernelShape, std::vector<int>> groups;
  b->member_kind.assign(b->ctx.size(), -1);
  for (int k : b->active) {
    const KernelShape s = member_shape(b->ctx[k]);
    groups[s].push_back(k);
    b->member_kind[k] = s.kind;
  }
  const int ng = (int)groups.size();
  b->launch_kind.clear();
  b->member_launch.assign(b->ctx.size(), -1);
  {
    int gi = 0;
    for (const auto& g : groups) {
      b->launch_kind.push_back(g.first.kind);
      for (int k : g.second) b->member_launch[k] = gi;
      ++gi;
    }
  }
  b->timed_moves = 0;
  if (b->timing) {
    const size_t need = (size_t)2 * ng * R;
    while (b->ev.size() < need) {
      hipEvent_t e;
      BATCH_TRY(b, hipEventCreate(&e));
      b->ev.push_back(e);
    }
  }
  for (int r = 0; r < R; ++r) {
    Tables T(b);
    struct Launch { KernelShape s; size_t off, foff; int n, grid; size_t lds; double cost; };
    std::vector<Launch> launches;
    for (const auto& g : groups) {
      const KernelShape& s = g.first;
      const std::vector<int>& mem = g.second;
      std::vector<int> first(mem.size() + 1, 0);
      size_t lds = 0;
      std::vector<MoveArgs> ma;
      std::vector<ResMoveArgs> rma;
      double cost = 0.0;
      for (size_t q = 0; q < mem.size(); ++q) {
        smc_ctx c = b->ctx[mem[q]];
        // rough work of the member: its row bytes over the move's passes
        cost += (double)c->pb.M * c->pb.m * (L + 1) * (c->pb.d + 2) * (s.fp32 ? 4.0 : 8.0);
        const MoveArgs a = move_args(c, eps[mem[q]], L);
        if (s.kind == kMoveResident) {
          rma.push_back(ResMoveArgs{a, c->res_ly});
          lds = std::max(lds, (size_t)c->res_ly.total);
        } else {
          ma.push_back(a);
          lds = std::max(lds, block_lds_bytes(c->pb));
        }
        first[q + 1] = first[q] + c->pb.M;
      }
      Launch l;
      l.s = s;
      l.off = s.kind == kMoveResident ? T.put(rma) : T.put(ma);
      l.foff = T.put(first);
      l.n = (int)mem.size();
      l.grid = first.back();
      l.lds = lds;
      l.cost = cost;
      launches.push_back(l);
    }
    // launch -> stream: the costliest first, each onto the least loaded
    // stream (lane 0 is the stream the move is issued on)
    const int nl = b->timing ? 1 : std::min<int>(b->lanes, (int)launches.size());
    std::vector<int> lane_of(launches.size(), 0);
    {
      std::vector<size_t> order(launches.size());
      std::iota(order.begin(), order.end(), (size_t)0);
      std::stable_sort(order.begin(), order.end(),
                       [&](size_t x, size_t y) { return launches[x].cost > launches[y].cost; });
      std::vector<double> load((size_t)std::max(nl, 1), 0.0);
      for (size_t q : order) {
        const int j = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        lane_of[q] = j;
        load[j] += launches[q].cost;
      }
    }
    while ((int)b->side.size() < nl - 1) {
      hipStream_t sd;
      BATCH_TRY(b, hipStreamCreateWithFlags(&sd, hipStreamNonBlocking));
      b->side.push_back(sd);
    }
    if (nl > 1 && !b->fork) BATCH_TRY(b, hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
    while ((int)b->join.size() < nl - 1) {
      hipEvent_t e;
      BATCH_TRY(b, hipEventCreateWithFlags(&e, hipEventDisableTiming));
      b->join.push_back(e);
    }
    smc_status st = T.upload();
    if (st != SMC_OK) return st;
    auto issue = [&](const Launch& l, hipStream_t st) -> hipError_t {
      if (l.s.kind == kMoveResident)
        return launch_move_resident_batch(l.s, l.grid, l.lds, batch_of<ResMoveArgs>(T, l.off, l.foff, l.n), st);
      if (l.s.kind == kMoveWide)
        return launch_move_wide_batch(l.s, l.grid, l.lds, batch_of<MoveArgs>(T, l.off, l.foff, l.n), st);
      return launch_move_narrow_batch(l.s, l.grid, l.lds, batch_of<MoveArgs>(T, l.off, l.foff, l.n), st);
    };
    // every launch, forked from and joined back to `main`
    auto issue_all = [&](hipStream_t main) -> hipError_t {
      hipError_t e = hipSuccess;
      if (nl > 1) {
        if ((e = hipEventRecord(b->fork, main)) != hipSuccess) return e;
        for (int j = 1; j < nl; ++j)
          if ((e = hipStreamWaitEvent(b->side[j - 1], b->fork, 0)) != hipSuccess) return e;
      }
      for (size_t li = 0; li < launches.size(); ++li) {
        const hipStream_t st = lane_of[li] == 0 ? main : b->side[lane_of[li] - 1];
        if ((e = issue(launches[li], st)) != hipSuccess) return e;
      }
      for (int j = 1; j < nl; ++j) {
        if ((e = hipEventRecord(b->join[j - 1], b->side[j - 1])) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(main, b->join[j - 1], 0)) != hipSuccess) return e;
      }
      return hipSuccess;
    };
    if (b->use_graph && !b->timing) {
      // the launches read their arguments from the uploaded tables, so a graph
      // captured once replays any move with the same launch structure
      std::vector<long long> key;
      for (size_t li = 0; li < launches.size(); ++li) {
        const Launch& l = launches[li];
        const long long v[13] = {l.s.kind, l.s.fp32, l.s.fam, l.s.dc, l.s.lanes, l.s.ch, l.s.rpl,
                                 l.grid, (long long)l.lds, l.n, (long long)l.off, (long long)l.foff, lane_of[li]};
        key.insert(key.end(), v, v + 13);
      }
      if (!b->gexec || key != b->graph_key) {
        if (b->gexec) {
          BATCH_TRY(b, hipGraphExecDestroy(b->gexec));
          b->gexec = nullptr;
        }
        // captured on a stream of the batch's own (the caller's stream may be
        // the null stream, which cannot capture); nothing runs during capture
        if (!b->capture) BATCH_TRY(b, hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
        BATCH_TRY(b, hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
        const hipError_t le = issue_all(b->capture);
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(b->capture, &g);
        BATCH_TRY(b, le);
        BATCH_TRY(b, ce);
        const hipError_t ie = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        BATCH_TRY(b, ie);
        b->graph_key = key;
        b->graph_captures += 1;
      }
      BATCH_TRY(b, hipGraphLaunch(b->gexec, b->stream));
    } else if (b->timing) {
      // one after another, each between its own event pair
      for (size_t li = 0; li < launches.size(); ++li) {
        hipEvent_t* ev = &b->ev[2 * ((size_t)r * ng + li)];
        BATCH_TRY(b, hipEventRecord(ev[0], b->stream));
        BATCH_TRY(b, issue(launches[li], b->stream));
        BATCH_TRY(b, hipEventRecord(ev[1], b->stream));
      }
    } else {
      BATCH_TRY(b, issue_all(b->stream));
    }
    for (int k : b->active) {
      b->ctx[k]->move += 1;
      b->ctx[k]->moved = 1;
    }
    if (b->timing) b->timed_moves += 1;
  }
  return SMC_OK;
}

smc_status smc_batch_set_streams(smc_batch b, int32_t n) {
  if (!b || n < 1 || n > 8) return SMC_ERR_INVALID_ARG;
  b->lanes = n;
  return SMC_OK;
}

smc_status smc_batch_set_persistent(smc_batch b, int32_t on) {
  if (!b || (on != 0 && on != 1)) return SMC_ERR_INVALID_ARG;
  b->persistent = on;
  return SMC_OK;
}

smc_status smc_batch_member_kernels(smc_batch b, int32_t* kind) {
  if (!b || !kind) return SMC_ERR_INVALID_ARG;
  for (size_t k = 0; k < b->ctx.size(); ++k) kind[k] = b->member_kind.empty() ? -1 : b->member_kind[k];
  return SMC_OK;
}

smc_status smc_batch_set_graph(smc_batch b, int32_t on) {
  if (!b || (on != 0 && on != 1)) return SMC_ERR_INVALID_ARG;
  b->use_graph = on;
  return SMC_OK;
}

int32_t smc_batch_graph_captures(smc_batch b) { return b ? b->graph_captures : 0; }

smc_status smc_batch_set_timing(smc_batch b, int32_t on) {
  if (!b || (on != 0 && on != 1)) return SMC_ERR_INVALID_ARG;
  b->timing = on;
  return SMC_OK;
}

smc_status smc_batch_move_timing(smc_batch b, int32_t cap, int32_t* launches, int32_t* kind, double* ms,
                                 int32_t* member_launch) {
  if (!b || !launches) return SMC_ERR_INVALID_ARG;
  const int ng = (int)b->launch_kind.size();
  *launches = ng;
  if (member_launch)
    for (size_t k = 0; k < b->ctx.size(); ++k) member_launch[k] = b->member_launch.empty() ? -1 : b->member_launch[k];
  if (ng > cap) return bfail(b, SMC_ERR_INVALID_ARG, "%d launches, capacity %d", ng, cap);
  for (int g = 0; g < ng; ++g) {
    if (kind) kind[g] = b->launch_kind[g];
    if (!ms) continue;
    ms[g] = 0.0;
    for (int r = 0; r < b->timed_moves; ++r) {
      const hipEvent_t* ev = &b->ev[2 * ((size_t)r * ng + g)];
      BATCH_TRY(b, hipEventSynchronize(ev[1]));
      float t = 0.f;
      BATCH_TRY(b, hipEventElapsedTime(&t, ev[0], ev[1]));
      ms[g] += t;
    }
  }
  return SMC_OK;
}

int32_t smc_batch_launches(smc_batch b) {
  if (!b || !b->have_stage) return 0;
  std::map<KernelShape, int> groups;
  for (int k : b->active) {
    KernelShape s = member_shape(b->ctx[k]);
    if (b->persistent) s = KernelShape{kMovePersistent, s.fp32, s.fam, 0, 0, 0, 0, 0, 0};
    groups[s] += 1;
  }
  return (int32_t)groups.size();
}

void smc_batch_destroy(smc_batch b) {
  if (!b) return;
  if (b->staged) {
    (void)hipEventSynchronize(b->staged);
    (void)hipEventDestroy(b->staged);
  }
  for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  for (hipStream_t sd : b->side) {
    (void)hipStreamSynchronize(sd);
    (void)hipStreamDestroy(sd);
  }
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (hipEvent_t e : b->join) (void)hipEventDestroy(e);
  if (b->host) (void)hipHostFree(b->host);
  delete b;
}

const char* smc_batch_last_error(smc_batch b) { return b ? b->err : "no batch"; }

void smc_destroy(smc_ctx c) {
  if (!c) return;
  if (c->mass_ev) {
    (void)hipEventSynchronize(c->mass_ev);
    (void)hipEventDestroy(c->mass_ev);
  }
  if (c->temper_ev) {
    (void)hipEventSynchronize(c->temper_ev);
    (void)hipEventDestroy(c->temper_ev);
  }
  for (hipEvent_t e : c->mev) (void)hipEventDestroy(e);
  if (c->hstatus) (void)hipHostFree(c->hstatus);
  delete c;
}

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
