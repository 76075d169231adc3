// Cross-lane exchanges inside one 64-lane wavefront that stay in the VALU.
//
// A butterfly over the 64 lanes takes six pairing steps. Step s pairs each
// lane with a partner that differs from it in "role bit" 5 - s and agrees
// with it in every higher role bit, which is all a butterfly needs (the
// partner does not have to be lane ^ (1 << bit)):
//   step 0: lanes 32 apart      v_permlane32_swap   (role bit 5)
//   step 1: lanes 16 apart      v_permlane16_swap   (role bit 4)
//   step 2: i <-> 15 - i        DPP row_mirror      (role bit 3)
//   step 3: i <-> 7 - i         DPP row_half_mirror (role bit 2)
//   step 4: i <-> i ^ 2         DPP quad_perm       (role bit 1)
//   step 5: i <-> i ^ 1         DPP quad_perm       (role bit 0)
// ds_bpermute (the LDS crossbar) is avoided: its latency is exposed when a
// SIMD runs a single wavefront.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace subsmc {
namespace xl {

constexpr int kRowMirror = 0x140;
constexpr int kRowHalfMirror = 0x141;
constexpr int kQuadXor2 = 0x4E;  // quad_perm [2,3,0,1]
constexpr int kQuadXor1 = 0xB1;  // quad_perm [1,0,3,2]

template <int S>
__device__ __forceinline__ uint32_t dpp_word(uint32_t x) {
  constexpr int ctrl = S == 2 ? kRowMirror : S == 3 ? kRowHalfMirror : S == 4 ? kQuadXor2 : kQuadXor1;
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, ctrl, 0xf, 0xf, false);
}

// permlane swap of steps 0 and 1: with (a, b) in, lanes whose role bit is 0
// get (a, partner's a) and lanes whose role bit is 1 get (partner's b, b).
template <int S>
__device__ __forceinline__ void swap_words(uint32_t a, uint32_t b, uint32_t& ra, uint32_t& rb) {
  if constexpr (S == 0) {
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    ra = r[0];
    rb = r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
    ra = r[0];
    rb = r[1];
  }
}

__device__ __forceinline__ uint32_t lo_word(double x) { return (uint32_t)((uint64_t)__double_as_longlong(x)); }
__device__ __forceinline__ uint32_t hi_word(double x) { return (uint32_t)((uint64_t)__double_as_longlong(x) >> 32); }
__device__ __forceinline__ double make_double(uint32_t lo, uint32_t hi) {
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// x of this lane plus x of its partner at step S (bitwise the same in both).
template <int S>
__device__ __forceinline__ float pair_all(float x) {
  if constexpr (S < 2) {
    uint32_t a, b;
    swap_words<S>(__float_as_uint(x), __float_as_uint(x), a, b);
    return __uint_as_float(a) + __uint_as_float(b);
  } else {
    return x + __uint_as_float(dpp_word<S>(__float_as_uint(x)));
  }
}

template <int S>
__device__ __forceinline__ double pair_all(double x) {
  if constexpr (S < 2) {
    uint32_t a0, b0, a1, b1;
    swap_words<S>(lo_word(x), lo_word(x), a0, b0);
    swap_words<S>(hi_word(x), hi_word(x), a1, b1);
    return make_double(a0, a1) + make_double(b0, b1);
  } else {
    return x + make_double(dpp_word<S>(lo_word(x)), dpp_word<S>(hi_word(x)));
  }
}

// Reduce-scatter step: lanes with role bit 1 keep `hi` and send `lo`, the
// others keep `lo` and send `hi`; returns kept + received.
template <int S>
__device__ __forceinline__ float pair_rs(float lo, float hi, int lane) {
  if constexpr (S < 2) {
    uint32_t a, b;
    swap_words<S>(__float_as_uint(lo), __float_as_uint(hi), a, b);
    return __uint_as_float(a) + __uint_as_float(b);
  } else {
    const bool up = (lane >> (5 - S)) & 1;
    const float send = up ? lo : hi;
    const float keep = up ? hi : lo;
    return keep + __uint_as_float(dpp_word<S>(__float_as_uint(send)));
  }
}

template <int S>
__device__ __forceinline__ double pair_rs(double lo, double hi, int lane) {
  if constexpr (S < 2) {
    uint32_t a0, b0, a1, b1;
    swap_words<S>(lo_word(lo), lo_word(hi), a0, b0);
    swap_words<S>(hi_word(lo), hi_word(hi), a1, b1);
    return make_double(a0, a1) + make_double(b0, b1);
  } else {
    const bool up = (lane >> (5 - S)) & 1;
    const double send = up ? lo : hi;
    const double keep = up ? hi : lo;
    return keep + make_double(dpp_word<S>(lo_word(send)), dpp_word<S>(hi_word(send)));
  }
}

// Sum over the 64 lanes, the same value in every lane.
template <typename T>
__device__ __forceinline__ T wave_allsum(T x) {
  x = pair_all<0>(x);
  x = pair_all<1>(x);
  x = pair_all<2>(x);
  x = pair_all<3>(x);
  x = pair_all<4>(x);
  return pair_all<5>(x);
}

// max(x of this lane, x of its partner at step S).
template <int S>
__device__ __forceinline__ double pair_max(double x) {
  if constexpr (S < 2) {
    uint32_t a0, b0, a1, b1;
    swap_words<S>(lo_word(x), lo_word(x), a0, b0);
    swap_words<S>(hi_word(x), hi_word(x), a1, b1);
    return fmax(make_double(a0, a1), make_double(b0, b1));
  } else {
    return fmax(x, make_double(dpp_word<S>(lo_word(x)), dpp_word<S>(hi_word(x))));
  }
}

// Maximum over the 64 lanes, the same value in every lane.
__device__ __forceinline__ double wave_allmax(double x) {
  x = pair_max<0>(x);
  x = pair_max<1>(x);
  x = pair_max<2>(x);
  x = pair_max<3>(x);
  x = pair_max<4>(x);
  return pair_max<5>(x);
}

// Sum and maximum over each row of 16 lanes (steps 2..5), the same value in
// every lane of the row.
__device__ __forceinline__ double row_allsum(double x) {
  x = pair_all<2>(x);
  x = pair_all<3>(x);
  x = pair_all<4>(x);
  return pair_all<5>(x);
}

__device__ __forceinline__ double row_allmax(double x) {
  x = pair_max<2>(x);
  x = pair_max<3>(x);
  x = pair_max<4>(x);
  return pair_max<5>(x);
}

// Row groups of G = 4 or 8 consecutive lanes (a row shared by G lanes).
// Sum over the group, the same bits in every lane of the group: pairs i ^ 1,
// i ^ 2, then (G = 8) i <-> 7 - i, which pairs the two quads.
template <int G, typename T>
__device__ __forceinline__ T group_sum(T x) {
  static_assert(G == 4 || G == 8, "groups of 4 or 8 lanes");
  x = pair_all<5>(x);
  x = pair_all<4>(x);
  if constexpr (G == 8) x = pair_all<3>(x);
  return x;
}

constexpr int kQuadLead = 0x00;  // quad_perm [0,0,0,0]

__device__ __forceinline__ uint32_t quad_lead_word(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, kQuadLead, 0xf, 0xf, false);
}

// The value of the group's first lane in every lane of the group: the quad's
// first lane, and for G = 8 the upper quad takes the lower quad's through
// i <-> 7 - i.
template <int G>
__device__ __forceinline__ float group_lead(float x, int lane) {
  static_assert(G == 4 || G == 8, "groups of 4 or 8 lanes");
  uint32_t w = quad_lead_word(__float_as_uint(x));
  if constexpr (G == 8) {
    const uint32_t m = dpp_word<3>(w);
    w = (lane & 4) ? m : w;
  }
  return __uint_as_float(w);
}

template <int G>
__device__ __forceinline__ double group_lead(double x, int lane) {
  static_assert(G == 4 || G == 8, "groups of 4 or 8 lanes");
  uint32_t lo = quad_lead_word(lo_word(x)), hi = quad_lead_word(hi_word(x));
  if constexpr (G == 8) {
    const uint32_t ml = dpp_word<3>(lo), mh = dpp_word<3>(hi);
    lo = (lane & 4) ? ml : lo;
    hi = (lane & 4) ? mh : hi;
  }
  return make_double(lo, hi);
}

// The value of lane S of each quad, in every lane of the quad.
template <int S>
__device__ __forceinline__ float quad_pick(float x) {
  static_assert(S >= 0 && S < 4, "lane of a quad");
  constexpr int ctrl = S | (S << 2) | (S << 4) | (S << 6);
  return __uint_as_float((uint32_t)__builtin_amdgcn_mov_dpp((int)__float_as_uint(x), ctrl, 0xf, 0xf, false));
}

// Reduce-scatter of N values held by every lane: afterwards v[0] of a lane is
// the wavefront total of one value (or zero padding). The value a lane ends
// with depends only on its role bits: the lane keeps the upper half of its
// remaining (zero padded) values at each step whose role bit is set.
template <typename T, int N, int S>
__device__ __forceinline__ void reduce_scatter(T* v, int lane) {
  if constexpr (S < 6) {
    constexpr int H = (N + 1) / 2;
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const T hi = (H + k < N) ? v[H + k] : T(0);
      v[k] = pair_rs<S>(v[k], hi, lane);
    }
    reduce_scatter<T, H, S + 1>(v, lane);
  }
}

// Index of the value that lane holds after reduce_scatter<T, N, 0>, or -1
// for zero padding: the step-s array length is N_s (N_0 = N, N_{s+1} =
// ceil(N_s / 2)); walking back from position 0 after the last step, a lane
// whose role bit is set came from position ceil(N_s / 2) + pos.
template <int N>
__device__ __forceinline__ int scatter_index(int lane) {
  int ns[6];
  int n = N;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    ns[s] = n;
    n = (n + 1) / 2;
  }
  int pos = 0;
  bool valid = true;
#pragma unroll
  for (int s = 5; s >= 0; --s) {
    if ((lane >> (5 - s)) & 1) pos += (ns[s] + 1) / 2;
    valid = valid && (pos < ns[s]);
  }
  return valid ? pos : -1;
}

}  // namespace xl
}  // namespace subsmc
