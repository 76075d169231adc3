// Persistent batched move: one launch moves every particle of every member of
// a batch (Algorithm 1 for each dataset's particles, section 2.1: the particles
// move independently). A grid of as many workgroups as the chip holds at once
// takes work items from a device queue until it is empty. An item is either
// one particle of a member moved by the resident kernel (the whole workgroup
// of four wavefronts, its subsample on chip) or four consecutive particles of
// a member moved by a streaming kernel (one per wavefront, each with an LDS
// slice of its own and no barrier shared with the others). Items are numbered
// costliest member first, so the long moves start first and the short ones
// fill the tail. Each particle runs the same body, with the same arguments, as
// in that member's own launch, so results are bit for bit those of the
// per-shape launches.
#pragma once

#include "kernels.hpp"
#include "kernels_resident.hpp"
#include "kernels_wide.hpp"

namespace subsmc {

constexpr int kPersistThreads = kResLanes;             // four wavefronts
constexpr int kPersistWaves = kPersistThreads / kWave;  // streaming particles per item

// One member of the launch.
struct PersistMember {
  MoveArgs A;
  ResLayout Ly;      // resident members: the on-chip layout
  int32_t body;      // the member's body in the launch's list
  int32_t resident;  // 1: an item is one particle (the workgroup); 0: kPersistWaves particles
  int32_t wave_lds;  // streaming members: bytes of each wavefront's LDS slice
  int32_t pad;
};

struct PersistArgs {
  const PersistMember* mem;  // count members, costliest first
  const int32_t* first;      // count + 1 prefix sums of the members' item counts
  int32_t count;
  int32_t n_items;
  int32_t* queue;  // [0] next item, [1] workgroups finished; both zero between launches
};

// Body kinds of the launch's list: narrow (padded d), lane-group (lanes, chunk,
// tile form) and resident (padded d, register rows per lane). Each body is a
// function of its own (not inlined into the kernel), so that its registers are
// allocated as in its own kernel: inlined together, the bodies' live ranges
// made the allocator spill some 1,800 values per lane.
template <int DC>
struct NarrowBody {};
template <int G, int CH, int TL>
struct WideBody {};
template <int DC, int RPL>
struct ResBody {};
template <typename... B>
struct BodyList {};

template <typename Real, int FAM, int DC>
__device__ __noinline__ void run_body(NarrowBody<DC>, const PersistMember& Mb, int j, char* smem) {
  const int wave = (int)threadIdx.x / kWave;
  const MoveArgs A = Mb.A;
  char* base = smem + wave * Mb.wave_lds;
  constexpr int kRed = (kWave * DC * (int)sizeof(Real) + 15) & ~15;
  move_body<Real, DC, FAM>(A, j * kPersistWaves + wave, reinterpret_cast<Real*>(base),
                           reinterpret_cast<int32_t*>(base + kRed));
}

template <typename Real, int FAM, int G, int CH, int TL>
__device__ __noinline__ void run_body(WideBody<G, CH, TL>, const PersistMember& Mb, int j, char* smem) {
  const int wave = (int)threadIdx.x / kWave;
  const MoveArgs A = Mb.A;
  char* base = smem + wave * Mb.wave_lds;
  constexpr int kRed = (kWave * CH * (int)sizeof(Real) + 15) & ~15;
  move_wide_body<Real, G, CH, FAM, TL>(A, j * kPersistWaves + wave, reinterpret_cast<Real*>(base),
                                       reinterpret_cast<double*>(base + kRed),
                                       reinterpret_cast<int32_t*>(base + kRed + 128 * 8));
}

template <typename Real, int FAM, int DC, int RPL>
__device__ __noinline__ void run_body(ResBody<DC, RPL>, const PersistMember& Mb, int j, char*) {
  const MoveArgs A = Mb.A;
  const ResLayout Ly = Mb.Ly;
  move_res_body<Real, DC, FAM, RPL, 0>(A, Ly, j);
}

// LDS bytes of one wavefront's slice for a streaming body (host side too)
__host__ __device__ inline int persist_wave_lds(bool wide, int dc_or_ch, int real_bytes, int block_ints) {
  return res_align16(kWave * dc_or_ch * real_bytes) + (wide ? 128 * 8 : 0) + res_align16(block_ints * 4);
}

template <typename Real, int FAM, typename... B>
__device__ __forceinline__ void run_listed(BodyList<B...>, const PersistMember& Mb, int j, char* smem) {
  const int body = Mb.body;
  int k = 0;
  ((body == k++ ? (run_body<Real, FAM>(B{}, Mb, j, smem), 0) : 0), ...);
}

// Every workgroup: take the next item, run it, until the queue is empty. The
// last workgroup to leave puts the queue back to zero for the next launch
// (every other workgroup has taken its last, failing, ticket before it counts
// itself out).
template <typename Real, int FAM, typename List>
__global__ void __launch_bounds__(kPersistThreads) __attribute__((amdgpu_waves_per_eu(kMoveWaves<Real>)))
move_kernel_persist(PersistArgs P) {
  extern __shared__ __attribute__((aligned(16))) char psm[];
  __shared__ int32_t s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(&P.queue[0], 1);
    __syncthreads();
    const int it = s_item;
    __syncthreads();
    if (it >= P.n_items) break;
    const int q = batch_member(P.first, P.count, it);
    run_listed<Real, FAM>(List{}, P.mem[q], it - P.first[q], psm);
  }
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&P.queue[1], 1) == (int)gridDim.x - 1) {
      atomicExch(&P.queue[0], 0);
      atomicExch(&P.queue[1], 0);
    }
  }
}

}  // namespace subsmc
