// Exact modular arithmetic for gfx950 kernels.
//
// Two interchangeable policies give bit-identical canonical results:
//
//  ArF64  residues held as doubles.  A product y*w mod q is formed exactly
//         with two FMAs: h = fl(y*w), l = y*w - h (exact, one FMA), a quotient
//         estimate k = rint(y * (w/q)), and r = (h - k*q) + l, where the FMA
//         h - k*q is exact because the true difference is an integer below
//         2^53.  With q < 2^48 and |y| <= B*q the estimate y*fl(w/q) carries
//         two roundings of |y w / q| < B 2^48, so the quotient is off by at
//         most 1/2 + B/16 and |r| <= (1/2 + B/16) q.  Values stay signed and
//         lazily reduced; every caller keeps |v| <= 31q < 2^53 (checked at
//         compile time by the bound bookkeeping in ntt.hpp) so every integer
//         is exact in fp64.  (Primes below 2^48 rather than 2^50 give 31q of
//         headroom instead of 7q: the transforms reduce a quarter as often.)
//         gfx950 issues v_fma_f64 / v_mul_f64 / v_rndne_f64 at full rate.
//
//  ArU64  residues held as uint64 in Harvey's lazy ranges, products by
//         Shoup's method with the precomputed companion w' = floor(w 2^64 / q):
//         Q = hi64(y * w'), r = y*w - Q*q in [0, 2q) for any y < 2^64.  The
//         64-bit products are built by the compiler from v_mad_u64_u32 and
//         v_mul_hi_u32 (full rate on gfx950).  Needs q < 2^62.
//
// Both policies expose the same interface so the transform kernels are
// written once.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace he {

struct TwF64 {
  double w, wq;   // twiddle and fl(w / q)
};
struct TwU64 {
  uint64_t w, ws; // twiddle and floor(w * 2^64 / q)
};

// Per-prime constants, one entry per RNS prime, in device memory.
struct PrimeK {
  uint64_t q;
  uint64_t two_q;
  double qd;        // q as double (F64)
  double qinv;      // fl(1/q)
  uint64_t r64;     // 2^64 mod q (U64 128-bit reduction)
  uint64_t r64s;    // Shoup companion of r64
  uint64_t one_s;   // floor(2^64 / q): Shoup companion of 1
  uint64_t pad;
};

struct ArF64 {
  using V = double;
  using Tw = TwF64;
  double q, qinv;

  // Bound bookkeeping, in units of q (compile time).
  static constexpr double kLimit = 31.0;
  static constexpr double kCanon = 1.0;                 // canonical load
  static constexpr double kReduced = 0.51;              // after reduce()
  static constexpr double mul_out(double b_in) { return 0.5 + 0.0625 * b_in + 0.01; }
  // mulv forms the quotient companion in the kernel, fl(b * fl(1/q)), so the
  // quotient estimate carries three roundings of |y b / q| <= b_in q < b_in 2^48:
  // at most 3 * 2^-53 * b_in * 2^48 = 0.094 b_in, plus 1/2 from rint
  static constexpr double mulv_out(double b_in) { return 0.5 + 0.09375 * b_in + 0.01; }

  __device__ __forceinline__ explicit ArF64(const PrimeK &p) : q(p.qd), qinv(p.qinv) {}

  // x < 2^52: the bits of x under the exponent of 2^52 are the double 2^52 + x
  // (exact), so one OR and one subtraction convert it
  __device__ __forceinline__ V load(uint64_t x) const {
    return __builtin_bit_cast(double, x | 0x4330000000000000ull) - 4503599627370496.0;
  }
  __device__ __forceinline__ V load_signed(int64_t x) const {
    // |x| < 2^53 here (plaintext integers); reduce into (-q, q)
    double d = (double)x;
    return __builtin_fma(-__builtin_rint(d * qinv), q, d);
  }
  __device__ __forceinline__ V reduce(V x) const { return __builtin_fma(-__builtin_rint(x * qinv), q, x); }
  // canonical residue of x as an integer: 0 <= r < q < 2^52, so 2^52 + r is
  // exact and its mantissa bits are r
  __device__ __forceinline__ uint64_t store(V x) const {
    double r = reduce(x);          // |r| <= q/2 + 2
    r = r < 0.0 ? r + q : r;
    return __builtin_bit_cast(uint64_t, r + 4503599627370496.0) & 0x000FFFFFFFFFFFFFull;
  }
  // Bound (in units of q) under which store_out applies: the inverse
  // transform's planner keeps its last stage's products below it.
  static constexpr double kStoreIn = 0.99;
  // canonical residue of an inverse transform's output x, |x| < q: floor(x / q)
  // is -1 or 0, and one FMA gives x/q - 1/2 to within 2^-53 (fl(1/q) is within
  // 2^-53 relative, then one rounding), while for integers 0 < |x| < q it is at
  // least 2^-48 away from the ties -1/2 and -3/2 (x = 0 gives -1/2 exactly,
  // which rint takes to -0): so rint finds floor(x / q) and the second FMA adds
  // q back, exactly, when x < 0
  __device__ __forceinline__ uint64_t store_out(V x) const {
    const double t = __builtin_rint(__builtin_fma(x, qinv, -0.5));
    const double r = __builtin_fma(-t, q, x);
    return __builtin_bit_cast(uint64_t, r + 4503599627370496.0) & 0x000FFFFFFFFFFFFFull;
  }
  __device__ __forceinline__ V mul(V y, double w, double wq) const {
    double h = y * w;
    double l = __builtin_fma(y, w, -h);
    double k = __builtin_rint(y * wq);
    double r = __builtin_fma(-k, q, h);
    return r + l;
  }
  __device__ __forceinline__ V mul(V y, Tw w) const { return mul(y, w.w, w.wq); }
  // product of |a| <= kLimit q and a canonical 0 <= b < q (b's quotient
  // companion formed here; bound mulv_out)
  __device__ __forceinline__ V mulv(V a, V b) const { return mul(a, b, b * qinv); }
  __device__ __forceinline__ void ct(V &x, V &y, Tw w) const {
    V t = mul(y, w);
    y = x - t;
    x = x + t;
  }
  __device__ __forceinline__ V add(V a, V b) const { return a + b; }
  __device__ __forceinline__ V sub(V a, V b) const { return a - b; }
  __device__ __forceinline__ V neg(V a) const { return -a; }
};

__device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

struct ArU64 {
  using V = uint64_t;
  using Tw = TwU64;
  uint64_t q, two_q;

  static constexpr double kLimit = 1e9;   // ranges are fixed by construction
  static constexpr double kCanon = 1.0;
  static constexpr double kReduced = 1.0;
  static constexpr double mul_out(double) { return 1.0; }
  static constexpr double mulv_out(double) { return 1.0; }   // (no companions formed in this policy)

  __device__ __forceinline__ explicit ArU64(const PrimeK &p) : q(p.q), two_q(p.two_q) {}

  __device__ __forceinline__ V load(uint64_t x) const { return x; }
  __device__ __forceinline__ V load_signed(int64_t x) const {
    // |x| < 2^62: residue in [0, q)
    int64_t r = x % (int64_t)q;
    return (uint64_t)(r < 0 ? r + (int64_t)q : r);
  }
  __device__ __forceinline__ V reduce(V x) const {   // [0, 4q) -> [0, 2q)
    return x >= two_q ? x - two_q : x;
  }
  __device__ __forceinline__ uint64_t store(V x) const {   // [0, 4q) -> [0, q)
    x = x >= two_q ? x - two_q : x;
    return x >= q ? x - q : x;
  }
  // an inverse transform's outputs are Shoup products in [0, 2q): the full store
  static constexpr double kStoreIn = 1e9;
  __device__ __forceinline__ uint64_t store_out(V x) const { return store(x); }
  // Shoup: y*w mod q in [0, 2q) for any y < 2^64
  __device__ __forceinline__ V mul(V y, uint64_t w, uint64_t ws) const {
    uint64_t Q = mulhi64(y, ws);
    return y * w - Q * q;
  }
  __device__ __forceinline__ V mul(V y, Tw w) const { return mul(y, w.w, w.ws); }
  // Harvey forward butterfly: x, y in [0, 4q) -> x + w y, x - w y in [0, 4q)
  __device__ __forceinline__ void ct(V &x, V &y, Tw w) const {
    V xr = x >= two_q ? x - two_q : x;
    V t = mul(y, w);
    x = xr + t;
    y = xr - t + two_q;
  }
};

}  // namespace he
