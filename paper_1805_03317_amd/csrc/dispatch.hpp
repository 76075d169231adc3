// Launchers of the templated particle kernels (estimator and move), one
// translation unit per kernel family so that they compile in parallel:
// launch_narrow.hip (d <= 32, one lane per row), launch_wide.hip
// (32 < d <= 128, lane groups per row) and launch_resident.hip (the move with
// the subsample held on chip). Each returns hipErrorInvalidValue for a shape
// that has no instantiation.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "kernels_persist.hpp"
#include "kernels_resident.hpp"

namespace subsmc {

enum MoveKind : int { kMoveNarrow = 0, kMoveWide = 1, kMoveResident = 2, kMovePersistent = 3 };

// The instantiation of the particle kernels that serves one dataset.
struct KernelShape {
  int kind;       // MoveKind
  int fp32;       // 1: float rows (mixed precision), 0: double rows
  int fam;        // likelihood family
  int dc;         // padded d (narrow and resident kernels)
  int lanes, ch;  // lanes per row and elements per lane (wide kernels)
  int rpl;        // register rows per lane (resident kernel)
  int mf;         // 1: the resident kernel forms x'delta on the matrix cores
  int tile;       // lane-group streaming move: the tile form of its row loop
};

inline bool operator<(const KernelShape& a, const KernelShape& b) {
  const int x[9] = {a.kind, a.fp32, a.fam, a.dc, a.lanes, a.ch, a.rpl, a.mf, a.tile};
  const int y[9] = {b.kind, b.fp32, b.fam, b.dc, b.lanes, b.ch, b.rpl, b.mf, b.tile};
  for (int k = 0; k < 9; ++k)
    if (x[k] != y[k]) return x[k] < y[k];
  return false;
}

// one dataset: `grid` workgroups (count particles / M)
hipError_t launch_estimator_narrow(const KernelShape& s, int grid, const EstArgs& a, hipStream_t st);
hipError_t launch_estimator_wide(const KernelShape& s, int grid, const EstArgs& a, hipStream_t st);
hipError_t launch_move_narrow(const KernelShape& s, int grid, size_t lds, const MoveArgs& a, hipStream_t st);
hipError_t launch_move_wide(const KernelShape& s, int grid, size_t lds, const MoveArgs& a, hipStream_t st);
hipError_t launch_move_resident(const KernelShape& s, int grid, const ResLayout& ly, const MoveArgs& a,
                                hipStream_t st);

// batched: `grid` = the members' workgroups together, `lds` = the largest
// member's dynamic LDS; the argument blocks are on the device
hipError_t launch_move_narrow_batch(const KernelShape& s, int grid, size_t lds, const Batch<MoveArgs>& b,
                                    hipStream_t st);
hipError_t launch_move_wide_batch(const KernelShape& s, int grid, size_t lds, const Batch<MoveArgs>& b,
                                  hipStream_t st);
hipError_t launch_move_resident_batch(const KernelShape& s, int grid, size_t lds, const Batch<ResMoveArgs>& b,
                                      hipStream_t st);

// persistent batched move (launch_persist_f32.hip, launch_persist_f64.hip): the
// body of shape s in the launch for its row type and family (-1: none), the
// launch's workgroups per CU with `lds` bytes of dynamic LDS, and the launch
int persist_body_f32(const KernelShape& s);
int persist_body_f64(const KernelShape& s);
hipError_t persist_occupancy_f32(int fam, size_t lds, int* per_cu);
hipError_t persist_occupancy_f64(int fam, size_t lds, int* per_cu);
hipError_t launch_move_persist_f32(int fam, int grid, size_t lds, const PersistArgs& a, hipStream_t st);
hipError_t launch_move_persist_f64(int fam, int grid, size_t lds, const PersistArgs& a, hipStream_t st);

inline int persist_body(const KernelShape& s) { return s.fp32 ? persist_body_f32(s) : persist_body_f64(s); }
inline hipError_t persist_occupancy(int fp32, int fam, size_t lds, int* per_cu) {
  return fp32 ? persist_occupancy_f32(fam, lds, per_cu) : persist_occupancy_f64(fam, lds, per_cu);
}
inline hipError_t launch_move_persist(int fp32, int fam, int grid, size_t lds, const PersistArgs& a,
                                      hipStream_t st) {
  return fp32 ? launch_move_persist_f32(fam, grid, lds, a, st) : launch_move_persist_f64(fam, grid, lds, a, st);
}

}  // namespace subsmc
