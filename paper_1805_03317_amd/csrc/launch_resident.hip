// Instantiation and launch of the resident move (subsample rows on chip):
// (row type, padded d, family, register rows per lane, x'delta on the matrix
// cores). The host chooses among these shapes only; every FP32 shape comes in
// both forms of the x'delta product.
#include "launch_common.hpp"

namespace subsmc {
namespace {

#define RES_SHAPES(X)                                                                                   \
  X(float, 4, 1, 0, 0) X(float, 4, 1, 0, 1) X(float, 4, 1, 14, 0) X(float, 4, 1, 14, 1)                 \
  X(float, 8, 1, 0, 0) X(float, 8, 1, 0, 1) X(float, 8, 1, 14, 0) X(float, 8, 1, 14, 1)                 \
  X(float, 12, 1, 0, 0) X(float, 12, 1, 0, 1) X(float, 12, 1, 14, 0) X(float, 12, 1, 14, 1)             \
  X(float, 16, 1, 0, 0) X(float, 16, 1, 0, 1) X(float, 16, 1, 14, 0) X(float, 16, 1, 14, 1)             \
  X(float, 20, 1, 0, 0) X(float, 20, 1, 0, 1) X(float, 20, 1, 14, 0) X(float, 20, 1, 14, 1)             \
  X(float, 24, 1, 0, 0) X(float, 24, 1, 0, 1) X(float, 4, 0, 0, 0) X(float, 4, 0, 0, 1)                 \
  X(float, 8, 0, 0, 0) X(float, 8, 0, 0, 1) X(float, 12, 0, 0, 0) X(float, 12, 0, 0, 1)                 \
  X(float, 16, 0, 0, 0) X(float, 16, 0, 0, 1) X(float, 20, 0, 0, 0) X(float, 20, 0, 0, 1)               \
  X(float, 24, 0, 0, 0) X(float, 24, 0, 0, 1) X(float, 4, 0, 14, 0) X(float, 4, 0, 14, 1)               \
  X(float, 8, 0, 14, 0) X(float, 8, 0, 14, 1) X(float, 12, 0, 14, 0) X(float, 12, 0, 14, 1)             \
  X(float, 16, 0, 14, 0) X(float, 16, 0, 14, 1) X(float, 4, 1, 4, 0) X(float, 4, 1, 4, 1)               \
  X(float, 8, 1, 4, 0) X(float, 8, 1, 4, 1) X(float, 12, 1, 4, 0) X(float, 12, 1, 4, 1)                 \
  X(float, 16, 1, 4, 0) X(float, 16, 1, 4, 1) X(float, 20, 1, 4, 0) X(float, 20, 1, 4, 1)               \
  X(float, 4, 0, 4, 0) X(float, 4, 0, 4, 1) X(float, 8, 0, 4, 0) X(float, 8, 0, 4, 1)                   \
  X(float, 12, 0, 4, 0) X(float, 12, 0, 4, 1) X(float, 16, 0, 4, 0) X(float, 16, 0, 4, 1)               \
  X(double, 4, 0, 0, 0) X(double, 8, 0, 0, 0) X(double, 12, 0, 0, 0) X(double, 16, 0, 0, 0)             \
  X(double, 20, 0, 0, 0) X(double, 24, 0, 0, 0) X(double, 4, 1, 0, 0) X(double, 8, 1, 0, 0)             \
  X(double, 12, 1, 0, 0) X(double, 16, 1, 0, 0) X(double, 20, 1, 0, 0) X(double, 24, 1, 0, 0)

template <typename K>
hipError_t allow_lds(K kernel, size_t lds) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds);
}

}  // namespace

hipError_t launch_move_resident(const KernelShape& s, int grid, const ResLayout& ly, const MoveArgs& a,
                                hipStream_t st) {
#define X(T, DC_, FAM_, RPL_, MF_)                                                                \
  if ((sizeof(T) == 4) == (s.fp32 != 0) && s.dc == DC_ && s.fam == FAM_ && s.rpl == RPL_ &&       \
      s.mf == MF_) {                                                                              \
    auto k = move_kernel_res<T, DC_, FAM_, RPL_, MF_>;                                            \
    const hipError_t e = allow_lds(k, ly.total);                                                  \
    if (e != hipSuccess) return e;                                                                \
    hipLaunchKernelGGL(k, dim3(grid), dim3(kResLanes), ly.total, st, a, ly);                      \
    return hipGetLastError();                                                                     \
  }
  RES_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_move_resident_batch(const KernelShape& s, int grid, size_t lds, const Batch<ResMoveArgs>& b,
                                      hipStream_t st) {
#define X(T, DC_, FAM_, RPL_, MF_)                                                                \
  if ((sizeof(T) == 4) == (s.fp32 != 0) && s.dc == DC_ && s.fam == FAM_ && s.rpl == RPL_ &&       \
      s.mf == MF_) {                                                                              \
    auto k = move_kernel_res_batch<T, DC_, FAM_, RPL_, MF_>;                                      \
    const hipError_t e = allow_lds(k, lds);                                                       \
    if (e != hipSuccess) return e;                                                                \
    hipLaunchKernelGGL(k, dim3(grid), dim3(kResLanes), lds, st, b);                               \
    return hipGetLastError();                                                                     \
  }
  RES_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace subsmc
