// Instantiation and launch of the narrow particle kernels (d <= 32: one lane
// per row, padded d in steps of 4).
#include "launch_common.hpp"

namespace subsmc {
namespace {

template <typename F>
hipError_t by_dc(int dc, F&& f) {
  switch (dc) {
    case 4: return f(IntC<4>{});
    case 8: return f(IntC<8>{});
    case 12: return f(IntC<12>{});
    case 16: return f(IntC<16>{});
    case 20: return f(IntC<20>{});
    case 24: return f(IntC<24>{});
    case 28: return f(IntC<28>{});
    case 32: return f(IntC<32>{});
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_estimator_narrow(const KernelShape& s, int grid, const EstArgs& a, hipStream_t st) {
  return by_real_family(s.fp32, s.fam, [&](auto real, auto fam) {
    return by_dc(s.dc, [&](auto dc) {
      using Real = decltype(real);
      hipLaunchKernelGGL((estimator_kernel<Real, decltype(dc)::value, decltype(fam)::value>), dim3(grid),
                         dim3(kWave), 0, st, a);
      return hipGetLastError();
    });
  });
}

hipError_t launch_move_narrow(const KernelShape& s, int grid, size_t lds, const MoveArgs& a, hipStream_t st) {
  return by_real_family(s.fp32, s.fam, [&](auto real, auto fam) {
    return by_dc(s.dc, [&](auto dc) {
      using Real = decltype(real);
      hipLaunchKernelGGL((move_kernel<Real, decltype(dc)::value, decltype(fam)::value>), dim3(grid), dim3(kWave),
                         lds, st, a);
      return hipGetLastError();
    });
  });
}

hipError_t launch_move_narrow_batch(const KernelShape& s, int grid, size_t lds, const Batch<MoveArgs>& b,
                                    hipStream_t st) {
  return by_real_family(s.fp32, s.fam, [&](auto real, auto fam) {
    return by_dc(s.dc, [&](auto dc) {
      using Real = decltype(real);
      hipLaunchKernelGGL((move_kernel_batch<Real, decltype(dc)::value, decltype(fam)::value>), dim3(grid),
                         dim3(kWave), lds, st, b);
      return hipGetLastError();
    });
  });
}

}  // namespace subsmc
