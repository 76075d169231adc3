// Compile-time dispatch helpers shared by the launcher translation units.
#pragma once

#include <type_traits>

#include "dispatch.hpp"

namespace subsmc {

template <int V>
using IntC = std::integral_constant<int, V>;

// f(Real{}, IntC<FAM>{}) for the row type and likelihood family of a shape
template <typename F>
hipError_t by_real_family(int fp32, int fam, F&& f) {
  auto go = [&](auto real) -> hipError_t {
    switch (fam) {
      case kLogistic: return f(real, IntC<kLogistic>{});
      case kPoisson: return f(real, IntC<kPoisson>{});
      case kGaussian: return f(real, IntC<kGaussian>{});
      case kStudentT: return f(real, IntC<kStudentT>{});
      default: return hipErrorInvalidValue;
    }
  };
  return fp32 ? go(float{}) : go(double{});
}

}  // namespace subsmc
