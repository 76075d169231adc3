// The persistent batched move for float rows (mixed precision).
#include "launch_persist.hpp"

namespace subsmc {

int persist_body_f32(const KernelShape& s) { return PersistLauncher<float>::body(s); }

hipError_t persist_occupancy_f32(int fam, size_t lds, int* per_cu) {
  return PersistLauncher<float>::occupancy(fam, lds, per_cu);
}

hipError_t launch_move_persist_f32(int fam, int grid, size_t lds, const PersistArgs& a, hipStream_t st) {
  return PersistLauncher<float>::launch(fam, grid, lds, a, st);
}

}  // namespace subsmc
