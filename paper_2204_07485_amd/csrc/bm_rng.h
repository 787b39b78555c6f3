// bm_rng.h -- counter-based random stream of the GPU library (host + device).
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11) keyed by the 64-bit seed.  The stream layout, fixed by
// this library because the paper names no generator:
//   counter word 2 = sample index t, counter word 3 = stream tag
//   (kTagSample = 0 for the sampler, kTagSeed = 1 for K-means++ draws);
//   sampler: one block per pair of points, block b = i >> 1 at counter
//     (lo32(b), hi32(b), t, 0); the even point takes words 0-1, the odd point
//     words 2-3, as the 64-bit key (hi << 32) | lo;
//   K-means++: draw q at counter (lo32(q), hi32(q), t, 1) gives the word
//     (out0 << 32) | out1.
// A unit double is (w >> 11) * 2^-53; a bounded integer in [0, N) is the high
// half of the 128-bit product w * N.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bm {

constexpr uint32_t kTagSample = 0u;
constexpr uint32_t kTagSeed = 1u;

struct Block4 {
  uint32_t v[4];
};

__host__ __device__ __forceinline__ Block4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                         uint32_t c3, uint64_t seed) {
  constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
  constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
  uint32_t ka = static_cast<uint32_t>(seed);
  uint32_t kb = static_cast<uint32_t>(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t pa = static_cast<uint64_t>(kMulA) * c0;
    const uint64_t pb = static_cast<uint64_t>(kMulB) * c2;
    const uint32_t y0 = static_cast<uint32_t>(pb >> 32) ^ c1 ^ ka;
    const uint32_t y1 = static_cast<uint32_t>(pb);
    const uint32_t y2 = static_cast<uint32_t>(pa >> 32) ^ c3 ^ kb;
    const uint32_t y3 = static_cast<uint32_t>(pa);
    c0 = y0; c1 = y1; c2 = y2; c3 = y3;
    ka += kWeylA;
    kb += kWeylB;
  }
  return Block4{{c0, c1, c2, c3}};
}

// Keys of the point pair (2b, 2b+1) for sample t.
__host__ __device__ __forceinline__ void sample_key_pair(uint64_t seed, uint32_t t, uint64_t b,
                                                         uint64_t& even, uint64_t& odd) {
  const Block4 o = philox4x32_10(static_cast<uint32_t>(b), static_cast<uint32_t>(b >> 32), t,
                                 kTagSample, seed);
  even = (static_cast<uint64_t>(o.v[0]) << 32) | o.v[1];
  odd = (static_cast<uint64_t>(o.v[2]) << 32) | o.v[3];
}

__host__ __device__ __forceinline__ uint64_t seed_draw(uint64_t seed, uint32_t t, uint64_t q) {
  const Block4 o = philox4x32_10(static_cast<uint32_t>(q), static_cast<uint32_t>(q >> 32), t,
                                 kTagSeed, seed);
  return (static_cast<uint64_t>(o.v[0]) << 32) | o.v[1];
}

__host__ __device__ __forceinline__ double unit_from_word(uint64_t w) {
  return static_cast<double>(w >> 11) * 0x1.0p-53;
}

// High 64 bits of the 128-bit product a * b, from 32-bit limbs.
__host__ __device__ __forceinline__ uint64_t mul_high64(uint64_t a, uint64_t b) {
  const uint64_t al = static_cast<uint32_t>(a), ah = a >> 32;
  const uint64_t bl = static_cast<uint32_t>(b), bh = b >> 32;
  const uint64_t ll = al * bl, lh = al * bh, hl = ah * bl, hh = ah * bh;
  const uint64_t mid = (ll >> 32) + static_cast<uint32_t>(lh) + static_cast<uint32_t>(hl);
  return hh + (lh >> 32) + (hl >> 32) + (mid >> 32);
}

__host__ __device__ __forceinline__ uint64_t below_from_word(uint64_t w, uint64_t n) {
  return mul_high64(w, n);
}

}  // namespace bm
