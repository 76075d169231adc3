// Instantiation and launch of the wide particle kernels (32 < d <= 128: a
// group of `lanes` lanes per row, `ch` elements per lane). The shapes are
// those the host's packing rule produces for d in (32, 128]; the Gaussian
// test family is narrow only. The move of FP32 logistic rows comes in both
// tile forms of its row loop (one remainder per row or per lane); the other
// moves and the estimator kernels in form 0.
#include "kernels_wide.hpp"
#include "launch_common.hpp"

namespace subsmc {
namespace {

#define WIDE_SHAPES(X)                                                                \
  X(float, 4, 12) X(float, 4, 16) X(float, 8, 12) X(float, 8, 16) X(float, 8, 20)       \
  X(double, 4, 10) X(double, 4, 12) X(double, 4, 14) X(double, 4, 16)                   \
  X(double, 8, 10) X(double, 8, 12) X(double, 8, 14) X(double, 8, 16) X(double, 8, 18)

// f(IntC<lanes>{}, IntC<ch>{}) for an instantiated (Real, lanes, ch)
template <typename Real, typename F>
hipError_t by_wide(const KernelShape& s, F&& f) {
#define X(T, G_, CH_)                                                           \
  if constexpr (std::is_same<Real, T>::value) {                                 \
    if (s.lanes == G_ && s.ch == CH_) return f(IntC<G_>{}, IntC<CH_>{});         \
  }
  WIDE_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

// f(real, family, lanes, ch, tile) for an instantiated shape; `tiles` allows
// tile forms 1 (FP32 logistic rows) and 2 (form 0 with kWideGroup particles
// per workgroup, every shape)
template <typename F>
hipError_t wide_dispatch(const KernelShape& s, bool tiles, F&& f) {
  auto go = [&](auto real) -> hipError_t {
    using Real = decltype(real);
    auto fam_go = [&](auto fam) {
      return by_wide<Real>(s, [&](auto g, auto ch) -> hipError_t {
        constexpr bool two = wide_one_remainder_per_lane<Real, decltype(fam)::value, decltype(g)::value, 0>();
        if (s.tile == 0) return f(real, fam, g, ch, IntC<0>{});
        if (tiles && s.tile == 2) return f(real, fam, g, ch, IntC<2>{});
        if constexpr (two) {
          if (tiles && s.tile == 1) return f(real, fam, g, ch, IntC<1>{});
        }
        return hipErrorInvalidValue;
      });
    };
    switch (s.fam) {
      case kLogistic: return fam_go(IntC<kLogistic>{});
      case kPoisson: return fam_go(IntC<kPoisson>{});
      case kStudentT: return fam_go(IntC<kStudentT>{});
      default: return hipErrorInvalidValue;
    }
  };
  return s.fp32 ? go(float{}) : go(double{});
}

}  // namespace

hipError_t launch_estimator_wide(const KernelShape& s, int grid, const EstArgs& a, hipStream_t st) {
  KernelShape s0 = s;
  s0.tile = 0;
  return wide_dispatch(s0, false, [&](auto real, auto fam, auto g, auto ch, auto) {
    using Real = decltype(real);
    hipLaunchKernelGGL((estimator_kernel_wide<Real, decltype(g)::value, decltype(ch)::value, decltype(fam)::value>),
                       dim3(grid), dim3(kWave), 0, st, a);
    return hipGetLastError();
  });
}

hipError_t launch_move_wide(const KernelShape& s, int grid, size_t lds, const MoveArgs& a, hipStream_t st) {
  return wide_dispatch(s, true, [&](auto real, auto fam, auto g, auto ch, auto tl) {
    using Real = decltype(real);
    constexpr int G = decltype(g)::value, CH = decltype(ch)::value, FAM = decltype(fam)::value;
    if constexpr (decltype(tl)::value == 2) {
      // grid particles, kWideGroup to a workgroup (the host offers form 2 only
      // when they divide the particle count)
      if (grid % kWideGroup != 0) return hipErrorInvalidValue;
      const int wave_lds = wide_group_wave_lds(CH, (int)sizeof(Real), (int)lds);
      hipLaunchKernelGGL((move_kernel_wide_group<Real, G, CH, FAM, 0>), dim3(grid / kWideGroup),
                         dim3(kWave * kWideGroup), (size_t)wave_lds * kWideGroup, st, a, wave_lds);
    } else {
      hipLaunchKernelGGL((move_kernel_wide<Real, G, CH, FAM, decltype(tl)::value>), dim3(grid), dim3(kWave), lds, st,
                         a);
    }
    return hipGetLastError();
  });
}

hipError_t launch_move_wide_batch(const KernelShape& s, int grid, size_t lds, const Batch<MoveArgs>& b,
                                  hipStream_t st) {
  return wide_dispatch(s, true, [&](auto real, auto fam, auto g, auto ch, auto tl) {
    using Real = decltype(real);
    // (form 2 is form 0 with grouped particles; batch launches take form 0)
    constexpr int TL = decltype(tl)::value == 2 ? 0 : decltype(tl)::value;
    hipLaunchKernelGGL(
        (move_kernel_wide_batch<Real, decltype(g)::value, decltype(ch)::value, decltype(fam)::value, TL>),
        dim3(grid), dim3(kWave), lds, st, b);
    return hipGetLastError();
  });
}

}  // namespace subsmc
