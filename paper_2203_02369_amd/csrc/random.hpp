// Counter-based random numbers of the chains: Philox4x32-10 words, uniform
// doubles and Box-Muller normal pairs.  Every draw is a function of (seed,
// iteration, purpose, index) alone, so a chain draws the same numbers in
// whatever launch, kernel or order they are computed.
#pragma once

#include "common.hpp"

namespace hamlet {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11), counter (idx lo, idx hi, iteration,
// purpose), key (seed lo, seed hi).
// ---------------------------------------------------------------------------
struct Philox4 { uint32_t v[4]; };

__host__ __device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c0 = hi1 ^ c1 ^ k0; c1 = lo1; c2 = hi0 ^ c3 ^ k1; c3 = lo0;
  }
  Philox4 o; o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3; return o;
}

// Purposes of the draws.  The No-U-Turn sampler's: the direction of doubling
// j (index j), the merge of a subtree's halves (index ((j * 16 + height) <<
// 32) | position), the move to a new subtree's sample (index j).
enum Purpose : uint32_t {
  kPurposeModes = 0, kPurposeDist = 1, kPurposeSnl = 2, kPurposeAccept = 3, kPurposeJitter = 4,
  kPurposeNutsDir = 5, kPurposeNutsMerge = 6, kPurposeNutsTop = 7,
  kPurposeCosmo = 8   // momenta of u8 and phi (index 0: the pair), eta (index 1: its first)
};

__host__ __device__ __forceinline__ Philox4 draw_words(uint64_t seed, uint32_t iteration, uint32_t purpose, uint64_t index) {
  return philox4x32_10((uint32_t)index, (uint32_t)(index >> 32), iteration, purpose,
                       (uint32_t)seed, (uint32_t)(seed >> 32));
}

// ((x >> 11) + 1) 2^-53 in (0, 1], x = (hi << 32) | lo.
__host__ __device__ __forceinline__ double uniform53(uint32_t lo, uint32_t hi) {
  const uint64_t x = ((uint64_t)hi << 32) | lo;
  return ((double)(x >> 11) + 1.0) * 0x1.0p-53;
}

// Box-Muller on the two uniforms of one Philox output.
__device__ __forceinline__ double2 normal_pair(const Philox4& w) {
  const double u1 = uniform53(w.v[0], w.v[1]);
  const double u2 = uniform53(w.v[2], w.v[3]);
  const double rad = sqrt(-2.0 * log(u1));
  const double ang = 2.0 * M_PI * u2;
  double sn, cs;
  sincos(ang, &sn, &cs);
  return make_double2(rad * cs, rad * sn);
}

}  // namespace hamlet
