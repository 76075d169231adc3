// Body lists of the persistent batched move and its launcher, one launch per
// (row type, family). A list holds every narrow and lane-group shape of that
// row type and family and the resident shapes whose register rows leave the
// launch's occupancy intact: with float rows the launch keeps two wavefronts
// per SIMD (at most 256 registers per lane, the streaming kernels' own
// occupancy), so the resident layouts with 14 register rows per lane, and the
// x'delta-on-the-matrix-cores form, are not in it; members that would use them
// move with their streaming body instead.
#pragma once

#include "kernels_persist.hpp"
#include "launch_common.hpp"

namespace subsmc {

template <typename Real, int FAM>
struct PersistList;

using NarrowAll = BodyList<NarrowBody<4>, NarrowBody<8>, NarrowBody<12>, NarrowBody<16>, NarrowBody<20>,
                           NarrowBody<24>, NarrowBody<28>, NarrowBody<32>>;

template <typename... A, typename... B>
constexpr BodyList<A..., B...> cat(BodyList<A...>, BodyList<B...>) {
  return {};
}

using WideF32 = BodyList<WideBody<4, 12, 0>, WideBody<4, 16, 0>, WideBody<8, 12, 0>, WideBody<8, 16, 0>,
                         WideBody<8, 20, 0>>;
using WideF32Tiles = BodyList<WideBody<4, 12, 1>, WideBody<4, 16, 1>, WideBody<8, 12, 1>, WideBody<8, 16, 1>,
                              WideBody<8, 20, 1>>;
using WideF64 = BodyList<WideBody<4, 10, 0>, WideBody<4, 12, 0>, WideBody<4, 14, 0>, WideBody<4, 16, 0>,
                         WideBody<8, 10, 0>, WideBody<8, 12, 0>, WideBody<8, 14, 0>, WideBody<8, 16, 0>,
                         WideBody<8, 18, 0>>;
using ResRpl0 = BodyList<ResBody<4, 0>, ResBody<8, 0>, ResBody<12, 0>, ResBody<16, 0>, ResBody<20, 0>,
                         ResBody<24, 0>>;
using ResRpl4Logistic = BodyList<ResBody<4, 4>, ResBody<8, 4>, ResBody<12, 4>, ResBody<16, 4>>;
using ResRpl4Poisson = BodyList<ResBody<4, 4>, ResBody<8, 4>, ResBody<12, 4>, ResBody<16, 4>, ResBody<20, 4>>;

template <>
struct PersistList<float, kLogistic> {
  using type = decltype(cat(cat(NarrowAll{}, WideF32{}), cat(WideF32Tiles{}, cat(ResRpl0{}, ResRpl4Logistic{}))));
};
template <>
struct PersistList<float, kPoisson> {
  using type = decltype(cat(cat(NarrowAll{}, WideF32{}), cat(ResRpl0{}, ResRpl4Poisson{})));
};
template <>
struct PersistList<float, kStudentT> {
  using type = decltype(cat(NarrowAll{}, WideF32{}));
};
template <>
struct PersistList<float, kGaussian> {
  using type = NarrowAll;
};
template <>
struct PersistList<double, kLogistic> {
  using type = decltype(cat(cat(NarrowAll{}, WideF64{}), ResRpl0{}));
};
template <>
struct PersistList<double, kPoisson> {
  using type = decltype(cat(cat(NarrowAll{}, WideF64{}), ResRpl0{}));
};
template <>
struct PersistList<double, kStudentT> {
  using type = decltype(cat(NarrowAll{}, WideF64{}));
};
template <>
struct PersistList<double, kGaussian> {
  using type = NarrowAll;
};

// host: does body B serve shape s
template <int DC>
bool persist_matches(NarrowBody<DC>, const KernelShape& s) {
  return s.kind == kMoveNarrow && s.dc == DC;
}
template <int G, int CH, int TL>
bool persist_matches(WideBody<G, CH, TL>, const KernelShape& s) {
  return s.kind == kMoveWide && s.lanes == G && s.ch == CH && s.tile == TL;
}
template <int DC, int RPL>
bool persist_matches(ResBody<DC, RPL>, const KernelShape& s) {
  return s.kind == kMoveResident && s.dc == DC && s.rpl == RPL && s.mf == 0;
}

template <typename... B>
int persist_index(BodyList<B...>, const KernelShape& s) {
  int k = 0, found = -1;
  ((found < 0 && persist_matches(B{}, s) ? (found = k) : 0, ++k), ...);
  return found;
}

// The row type's three entry points, defined in launch_persist_f32.hip and
// launch_persist_f64.hip.
template <typename Real>
struct PersistLauncher {
  static int body(const KernelShape& s) {
    switch (s.fam) {
      case kLogistic: return persist_index(typename PersistList<Real, kLogistic>::type{}, s);
      case kPoisson: return persist_index(typename PersistList<Real, kPoisson>::type{}, s);
      case kStudentT: return persist_index(typename PersistList<Real, kStudentT>::type{}, s);
      case kGaussian: return persist_index(typename PersistList<Real, kGaussian>::type{}, s);
      default: return -1;
    }
  }

  template <int FAM>
  static const void* kernel() {
    return reinterpret_cast<const void*>(
        move_kernel_persist<Real, FAM, typename PersistList<Real, FAM>::type>);
  }

  static const void* kernel_of(int fam) {
    switch (fam) {
      case kLogistic: return kernel<kLogistic>();
      case kPoisson: return kernel<kPoisson>();
      case kStudentT: return kernel<kStudentT>();
      case kGaussian: return kernel<kGaussian>();
      default: return nullptr;
    }
  }

  // workgroups of the launch that fit on one CU at once with `lds` bytes
  static hipError_t occupancy(int fam, size_t lds, int* per_cu) {
    const void* k = kernel_of(fam);
    if (!k) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k, kPersistThreads, lds);
  }

  static hipError_t launch(int fam, int grid, size_t lds, const PersistArgs& a, hipStream_t st) {
    const void* k = kernel_of(fam);
    if (!k) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    PersistArgs arg = a;
    void* params[] = {&arg};
    return hipLaunchKernel(k, dim3(grid), dim3(kPersistThreads), params, lds, st);
  }
};

}  // namespace subsmc
