// Exact conversions between the RNS base Q = q_0 ... q_{L-1} of a context and an
// auxiliary base P = p_0 ... p_{K-1}, for the ciphertext-ciphertext product
// (Section 3.2, the CCMul of the preprocessing phase).
//
// A value x in [0, Q) is taken apart into mixed-radix digits
//   x = v_0 + v_1 q_0 + v_2 q_0 q_1 + ... ,  v_i in [0, q_i),
// with v_i = (((x_i - v_0) q_0^-1 - v_1) q_1^-1 - ... - v_{i-1}) q_{i-1}^-1 mod q_i.
// The digits give x mod any other modulus m exactly (sum of v_i times
// prod_{j<i} q_j mod m) and compare x with (Q + 1) / 2 exactly (digit by digit
// from the most significant), which is how a value is read as centred:
// x >= (Q + 1) / 2 stands for x - Q.  No floating point is involved, so every
// conversion is exact.
#pragma once
#include <stdint.h>

namespace he {

constexpr int kRnsMax = 8;   // primes per base

struct RnsConv {
  uint32_t L, K, pad0, pad1;
  uint64_t q[kRnsMax], q_one[kRnsMax];        // primes of Q; floor(2^64 / q_i)
  uint64_t p[kRnsMax], p_one[kRnsMax];        // primes of P; floor(2^64 / p_k)
  uint64_t t_q[kRnsMax], t_qs[kRnsMax];       // t mod q_i, Shoup companion
  uint64_t t_p[kRnsMax], t_ps[kRnsMax];       // t mod p_k
  uint64_t qinv_p[kRnsMax], qinv_ps[kRnsMax]; // Q^-1 mod p_k
  uint64_t q_mod_p[kRnsMax];                  // Q mod p_k
  uint64_t p_mod_q[kRnsMax];                  // P mod q_i
  uint64_t hq[kRnsMax], hp[kRnsMax];          // mixed-radix digits of (Q + 1) / 2 and (P + 1) / 2
  uint64_t iqq[kRnsMax][kRnsMax], iqqs[kRnsMax][kRnsMax];   // [j][i]: q_j^-1 mod q_i (j < i)
  uint64_t ipp[kRnsMax][kRnsMax], ipps[kRnsMax][kRnsMax];   // [j][k]: p_j^-1 mod p_k (j < k)
  uint64_t wq[kRnsMax][kRnsMax], wqs[kRnsMax][kRnsMax];     // [i][k]: prod_{j<i} q_j mod p_k
  uint64_t wp[kRnsMax][kRnsMax], wps[kRnsMax][kRnsMax];     // [k][i]: prod_{j<k} p_j mod q_i
  // the same values as doubles (exact when every prime is below 2^50, the
  // condition under which the fp64 products are used), and 1 / prime
  double dq[kRnsMax], dqinv[kRnsMax], dp[kRnsMax], dpinv[kRnsMax];
  double dt_q[kRnsMax], dt_p[kRnsMax], dqinv_p[kRnsMax], dq_mod_p[kRnsMax], dp_mod_q[kRnsMax];
  double dhq[kRnsMax], dhp[kRnsMax];
  double diqq[kRnsMax][kRnsMax], dipp[kRnsMax][kRnsMax], dwq[kRnsMax][kRnsMax], dwp[kRnsMax][kRnsMax];
};

}  // namespace he
