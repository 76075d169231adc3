// The persistent batched move for double rows (FP64 path).
#include "launch_persist.hpp"

namespace subsmc {

int persist_body_f64(const KernelShape& s) { return PersistLauncher<double>::body(s); }

hipError_t persist_occupancy_f64(int fam, size_t lds, int* per_cu) {
  return PersistLauncher<double>::occupancy(fam, lds, per_cu);
}

hipError_t launch_move_persist_f64(int fam, int grid, size_t lds, const PersistArgs& a, hipStream_t st) {
  return PersistLauncher<double>::launch(fam, grid, lds, a, st);
}

}  // namespace subsmc
