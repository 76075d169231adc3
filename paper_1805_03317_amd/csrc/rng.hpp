// Counter-based random numbers for the device path: Philox4x64-10
// (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
// SC'11), keyed by (seed, 0).
//
// Stream layout (one 64-bit word per draw):
//   counter word0 = purpose<<56 | stage<<32 | move<<16 | dataset
//   counter word1 = particle, word2 = draw>>2, word3 = 0; output word draw&3.
// Purposes: 0 prior normals, 1 initial subsample, 2 resampling offset,
// 3 block choice, 4 block indices, 5 u-accept, 6 momentum, 7 theta-accept.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace subsmc {

enum Purpose : uint32_t {
  kPriorNormal = 0, kInitIndex = 1, kResampleOffset = 2, kBlockChoice = 3,
  kBlockIndex = 4, kUAccept = 5, kMomentum = 6, kThetaAccept = 7
};

struct Block4 { uint64_t w[4]; };

__device__ __forceinline__ Block4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
    const uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += W0; k1 += W1;
  }
  Block4 b;
  b.w[0] = c0; b.w[1] = c1; b.w[2] = c2; b.w[3] = c3;
  return b;
}

__device__ __forceinline__ uint64_t stream_ctr0(uint32_t purpose, uint32_t stage, uint32_t move,
                                                uint32_t dataset) {
  return ((uint64_t)(purpose & 0xFFu) << 56) | ((uint64_t)(stage & 0xFFFFFFu) << 32) |
         ((uint64_t)(move & 0xFFFFu) << 16) | (uint64_t)(dataset & 0xFFFFu);
}

// The four consecutive words draw&~3 .. draw|3 of one stream.
__device__ __forceinline__ Block4 stream_block(uint64_t seed, uint64_t ctr0, uint64_t particle,
                                               uint64_t draw) {
  return philox4x64_10(ctr0, particle, draw >> 2, 0, seed, 0);
}

__device__ __forceinline__ uint64_t pick(const Block4& b, uint32_t i) {
  // select without dynamic register indexing
  uint64_t r = b.w[0];
  r = (i == 1) ? b.w[1] : r;
  r = (i == 2) ? b.w[2] : r;
  r = (i == 3) ? b.w[3] : r;
  return r;
}

__device__ __forceinline__ uint64_t stream_word(uint64_t seed, uint64_t ctr0, uint64_t particle,
                                                uint64_t draw) {
  return pick(stream_block(seed, ctr0, particle, draw), (uint32_t)(draw & 3));
}

// uniform integer in [0, n): high 64 bits of the 128-bit product w*n
__device__ __forceinline__ int64_t word_to_index(uint64_t w, uint64_t n) {
  return (int64_t)__umul64hi(w, n);
}

// uniform double in (0, 1]
__device__ __forceinline__ double word_to_uniform(uint64_t w) {
  return ((double)(w >> 11) + 1.0) * 0x1.0p-53;
}

// k-th standard normal of a stream: Box-Muller on the word pair (2*(k/2), 2*(k/2)+1);
// even k takes the cosine branch, odd k the sine branch.
__device__ __forceinline__ double stream_normal(uint64_t seed, uint64_t ctr0, uint64_t particle,
                                                uint32_t k) {
  const uint64_t base = 2ull * (k >> 1);
  const Block4 b = stream_block(seed, ctr0, particle, base);  // base and base+1 share a block
  const uint32_t o = (uint32_t)(base & 3);
  const uint64_t wa = pick(b, o), wb = pick(b, o + 1);
  const double u1 = word_to_uniform(wa);
  const double u2 = (double)(wb >> 11) * 0x1.0p-53;
  const double r = sqrt(-2.0 * log(u1));
  const double ang = 6.283185307179586476925286766559 * u2;
  return (k & 1) ? r * sin(ang) : r * cos(ang);
}

}  // namespace subsmc
