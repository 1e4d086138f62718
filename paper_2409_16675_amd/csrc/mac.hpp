// Slot-wise multiply-accumulate in the transformed domain (the CPMul products of
// ciphertext and plaintext slots summed into an output ciphertext, Sec. 3.2 and
// Sec. 3.3): acc[k] = sum_t ct_t[k] * pt_t[k] mod q, shared by the fused
// multiply-accumulate + inverse-transform kernel and the persistent kernel.
#pragma once
#include <type_traits>
#include <utility>

#include "arith.hpp"
#include "ntt.hpp"

namespace he {

template <class A>
struct MacAcc;

// fp64: each product of two canonical residues has |p| <= mulv_out(1) = 0.604 q;
// after a fold |acc| <= 0.51 q, so a chunk of 48 products keeps |acc| <= 29.5 q < 31 q.
template <>
struct MacAcc<ArF64> {
  static constexpr int kChunk = 48;
  static constexpr int kLoadBatch = 32;   // coefficients whose operands are loaded together
  static constexpr bool kLoneReduced = true;   // one product, unfolded, has |p| <= 0.604 q
  static constexpr int kOutBoundX100 = 61;     // bound of value(): a lone product or a fold
  static_assert(ArF64::kReduced + kChunk * ArF64::mulv_out(1.0) <= ArF64::kLimit, "chunk exceeds the fp64 bound");
  static_assert(kOutBoundX100 >= 100.0 * ArF64::mulv_out(1.0) && kOutBoundX100 >= 100.0 * ArF64::kReduced,
                "value() bound understated");
  double acc = 0.0;
  __device__ __forceinline__ void set(const ArF64 &ar, uint64_t a, uint64_t b) { acc = ar.mulv(ar.load(a), ar.load(b)); }
  __device__ __forceinline__ void add(const ArF64 &ar, uint64_t a, uint64_t b) { acc += ar.mulv(ar.load(a), ar.load(b)); }
  __device__ __forceinline__ void fold(const ArF64 &ar, const PrimeK &) { acc = ar.reduce(acc); }
  __device__ __forceinline__ double value() const { return acc; }
};

// integer: 128-bit sums of products < 2^124; a folded value (< q) plus 15
// products stays below 2^128.  fold: hi * (2^64 mod q) + lo, canonical.
template <>
struct MacAcc<ArU64> {
  static constexpr int kChunk = 15;
  static constexpr int kLoadBatch = 8;    // the 128-bit accumulators leave fewer registers
  static constexpr bool kLoneReduced = false;  // a 128-bit product needs its fold
  static constexpr int kOutBoundX100 = 100;    // canonical
  uint64_t lo = 0, hi = 0;
  __device__ __forceinline__ void set(const ArU64 &, uint64_t a, uint64_t b) {
    lo = a * b;
    hi = __umul64hi(a, b);
  }
  __device__ __forceinline__ void add(const ArU64 &, uint64_t a, uint64_t b) {
    const uint64_t pl = a * b, ph = __umul64hi(a, b);
    const uint64_t nl = lo + pl;
    hi += ph + (nl < lo ? 1u : 0u);
    lo = nl;
  }
  __device__ __forceinline__ void fold(const ArU64 &ar, const PrimeK &pk) {
    uint64_t x = ar.mul(hi, pk.r64, pk.r64s) + ar.mul(lo, 1, pk.one_s);   // < 4q
    x = x >= ar.two_q ? x - ar.two_q : x;
    x = x >= ar.q ? x - ar.q : x;
    lo = x;
    hi = 0;
  }
  __device__ __forceinline__ uint64_t value() const { return lo; }
};

// One term for the E coefficients ix(0) .. ix(E-1) of a thread (the slot
// layout of the consumer): the operand loads of a batch of coefficients are
// all issued before its first product, so they are in flight together instead
// of one memory round trip per coefficient.  FIRST: the accumulators take the
// products (no zero start).
template <class A, int E, bool FIRST, class P, class Ix>
__device__ __forceinline__ void mac_term(const A &ar, MacAcc<A> *acc, P a, P b, Ix ix) {
  constexpr int B = E < MacAcc<A>::kLoadBatch ? E : MacAcc<A>::kLoadBatch;
#pragma unroll
  for (int j0 = 0; j0 < E; j0 += B) {
    uint64_t va[B], vb[B];
#pragma unroll
    for (int j = 0; j < B; ++j) {
      // unsigned 32-bit offsets: a scalar base plus a lane offset, no 64-bit adds
      const uint32_t k = ix(j0 + j);
      va[j] = a[k];
      vb[j] = b[k];
    }
#pragma unroll
    for (int j = 0; j < B; ++j) {
      if constexpr (FIRST) acc[j0 + j].set(ar, va[j], vb[j]);
      else acc[j0 + j].add(ar, va[j], vb[j]);
    }
  }
}

// The terms t0 .. t1-1 of one output plane; operands(t, a, b) yields the two
// operand planes of term t.  Folds after every kChunk products; a last run of a
// single product is left unfolded where that is within kOutBoundX100.  An empty
// term list leaves the accumulators at zero.
template <class A, int E, class Ops, class Ix>
__device__ __forceinline__ void mac_terms(const A &ar, const PrimeK &pk, MacAcc<A> *acc, int t0, int t1, Ops operands,
                                          Ix ix) {
  if (t0 >= t1) return;
  {
    auto [a, b] = operands(t0);
    mac_term<A, E, true>(ar, acc, a, b, ix);
  }
  int run = 1;   // products since the start or the last fold
  for (int t = t0 + 1; t < t1; ++t) {
    if (run == MacAcc<A>::kChunk) {
#pragma unroll
      for (int j = 0; j < E; ++j) acc[j].fold(ar, pk);
      run = 0;
    }
    auto [a, b] = operands(t);
    mac_term<A, E, false>(ar, acc, a, b, ix);
    ++run;
  }
  if (run > 1 || !MacAcc<A>::kLoneReduced) {
#pragma unroll
    for (int j = 0; j < E; ++j) acc[j].fold(ar, pk);
  }
}

// Multiply-accumulate over fp64 operands that a batch keeps in its own format:
// a from a plane of doubles reduced to |a| <= 0.51 q (A_U64: canonical
// residues instead, for inputs the caller transformed), b from a plane of
// doubles reduced to |b| <= 0.51 q.  A product is then 7 instructions (its
// quotient companion fl(b fl(1/q)) formed in place) with no conversions; the
// quotient estimate carries three roundings of |a b / q| <= 0.51 q < 0.51 2^48,
// so |p| <= (1/2 + 3 * 0.51 / 32) q + slack.
struct MacWsF64 {
  static constexpr double kProdOut = 0.5 + 3.0 * 0.51 / 32.0 + 0.01;
  static constexpr int kChunk = 48;        // products between folds
  static constexpr int kLoadBatch = 32;    // coefficients whose operands are loaded together
  static constexpr int kOutBoundX100 = 61;
  static_assert(ArF64::kReduced + kChunk * kProdOut <= ArF64::kLimit, "chunk exceeds the fp64 bound");
  static_assert(kOutBoundX100 >= 100.0 * kProdOut && kOutBoundX100 >= 100.0 * ArF64::kReduced, "bound understated");
};

// acc[e] = sum over terms t0 .. t1-1 of a_t[ix(e)] * b_t[ix(e)] (zero for an
// empty range), folded every kChunk products and at the end unless a lone
// product; operands(t) yields the two planes of term t.
template <bool A_U64, int E, class Ops, class Ix>
__device__ __forceinline__ void mac_terms_ws(const ArF64 &ar, double (&acc)[E], int t0, int t1, Ops operands, Ix ix) {
  constexpr int B = E < MacWsF64::kLoadBatch ? E : MacWsF64::kLoadBatch;
  // one term; the first sets the accumulators (no zero start, no add)
  auto term = [&](auto first, int t) {
    const auto [a, b] = operands(t);
#pragma unroll
    for (int j0 = 0; j0 < E; j0 += B) {
      uint64_t va[B], vb[B];
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const uint32_t k = ix(j0 + j);
        va[j] = a[k];
        vb[j] = b[k];
      }
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const double x = A_U64 ? ar.load(va[j]) : __builtin_bit_cast(double, va[j]);
        const double p = ar.mulv(x, __builtin_bit_cast(double, vb[j]));
        if constexpr (decltype(first)::value) acc[j0 + j] = p;
        else acc[j0 + j] += p;
      }
    }
  };
  if (__builtin_expect(t0 >= t1, 0)) {
#pragma unroll
    for (int j = 0; j < E; ++j) acc[j] = 0.0;
    return;
  }
  term(std::true_type{}, t0);
  int run = 1;   // products since the start or the last fold
  for (int t = t0 + 1; t < t1; ++t) {
    if (run == MacWsF64::kChunk) {
#pragma unroll
      for (int j = 0; j < E; ++j) acc[j] = ar.reduce(acc[j]);
      run = 0;
    }
    term(std::false_type{}, t);
    ++run;
  }
  if (run > 1) {
#pragma unroll
    for (int j = 0; j < E; ++j) acc[j] = ar.reduce(acc[j]);
  }
}

}  // namespace he
