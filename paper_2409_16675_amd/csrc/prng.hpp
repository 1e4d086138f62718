// Regeneration of the uniform ciphertext component c1 from a seed (Section 7, Discussion:
// the client sends a seed instead of c1 and the server expands it).
//
// Coefficient k of component 1 of ciphertext j at prime i is
//   (w0 * 2^64 + w1) mod q_i,  (w0, w1, w2, w3) = Philox4x64-10(counter (k, j, i, 0), key seed),
// Philox4x64-10 being the counter-based generator of Salmon, Moraes, Dror and
// Shaw (SC 2011): ten rounds, each forming the 128-bit products of two counter
// words with fixed odd multipliers and mixing their halves with the two other
// words and the key, the key stepping by two Weyl constants per round.  The
// 128-bit value keeps each residue within 2^-78 of uniform.  Every coefficient
// is an independent function of its indices, so any thread layout regenerates
// the same component.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "arith.hpp"

namespace he {

struct Seed {
  uint64_t k0, k1;
};

// words w0, w1 of the Philox4x64-10 block of counter (c0, c1, c2, 0)
__device__ __forceinline__ void philox_w01(uint64_t c0, uint64_t c1, uint64_t c2, Seed s, uint64_t &w0, uint64_t &w1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t c3 = 0, k0 = s.k0, k1 = s.k1;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  w0 = c0;
  w1 = c1;
}

// (w0 * 2^64 + w1) mod q: w0 * (2^64 mod q) + w1 * 1 through two Shoup
// products, each in [0, 2q), then two conditional subtractions.
__device__ __forceinline__ uint64_t c1_residue(Seed s, uint32_t j, uint32_t i, uint32_t k, const PrimeK &pk) {
  uint64_t w0, w1;
  philox_w01(k, j, i, s, w0, w1);
  const ArU64 ar(pk);
  uint64_t x = ar.mul(w0, pk.r64, pk.r64s) + ar.mul(w1, 1, pk.one_s);
  x = x >= ar.two_q ? x - ar.two_q : x;
  return x >= ar.q ? x - ar.q : x;
}

}  // namespace he
