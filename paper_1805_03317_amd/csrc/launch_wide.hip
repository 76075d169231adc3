// Instantiation and launch of the wide particle kernels (32 < d <= 128: a
// group of `lanes` lanes per row, `ch` elements per lane). The shapes are
// those the host's packing rule produces for d in (32, 128]; the Gaussian
// test family is narrow only.
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

template <typename F>
hipError_t wide_dispatch(const KernelShape& s, F&& f) {
  auto go = [&](auto real) -> hipError_t {
    using Real = decltype(real);
    auto fam_go = [&](auto fam) { return by_wide<Real>(s, [&](auto g, auto ch) { return f(real, fam, g, ch); }); };
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
  return wide_dispatch(s, [&](auto real, auto fam, auto g, auto ch) {
    using Real = decltype(real);
    hipLaunchKernelGGL((estimator_kernel_wide<Real, decltype(g)::value, decltype(ch)::value, decltype(fam)::value>),
                       dim3(grid), dim3(kWave), 0, st, a);
    return hipGetLastError();
  });
}

hipError_t launch_move_wide(const KernelShape& s, int grid, size_t lds, const MoveArgs& a, hipStream_t st) {
  return wide_dispatch(s, [&](auto real, auto fam, auto g, auto ch) {
    using Real = decltype(real);
    hipLaunchKernelGGL((move_kernel_wide<Real, decltype(g)::value, decltype(ch)::value, decltype(fam)::value>),
                       dim3(grid), dim3(kWave), lds, st, a);
    return hipGetLastError();
  });
}

hipError_t launch_move_wide_batch(const KernelShape& s, int grid, size_t lds, const Batch<MoveArgs>& b,
                                  hipStream_t st) {
  return wide_dispatch(s, [&](auto real, auto fam, auto g, auto ch) {
    using Real = decltype(real);
    hipLaunchKernelGGL(
        (move_kernel_wide_batch<Real, decltype(g)::value, decltype(ch)::value, decltype(fam)::value>),
        dim3(grid), dim3(kWave), lds, st, b);
    return hipGetLastError();
  });
}

}  // namespace subsmc
