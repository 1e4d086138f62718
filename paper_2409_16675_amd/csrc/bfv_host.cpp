// Client-side decryption step on the host: exact CRT composition and rounding
//   m = round(t * x / Q) mod t,  x = CRT(x_0 .. x_{L-1}) in [0, Q),
// computed as floor((2 t x + Q) / (2 Q)) with fixed-width multiword integers.
// (The ring products before it run on the device.)
#include <cmath>
#include <cstring>

#include "he_internal.hpp"
#include "plan.hpp"

namespace he {

namespace {
typedef unsigned __int128 u128;
constexpr int W = 12;   // limbs: Q < 2^(62*8), with headroom for 2 t Q

struct Big {
  uint64_t w[W];
  Big() { std::memset(w, 0, sizeof(w)); }
  explicit Big(uint64_t v) : Big() { w[0] = v; }
};

int cmp(const Big &a, const Big &b) {
  for (int i = W - 1; i >= 0; --i)
    if (a.w[i] != b.w[i]) return a.w[i] < b.w[i] ? -1 : 1;
  return 0;
}
void add_to(Big &a, const Big &b) {
  u128 c = 0;
  for (int i = 0; i < W; ++i) {
    c += (u128)a.w[i] + b.w[i];
    a.w[i] = (uint64_t)c;
    c >>= 64;
  }
}
void sub_from(Big &a, const Big &b) {   // a >= b
  uint64_t br = 0;
  for (int i = 0; i < W; ++i) {
    const uint64_t bi = b.w[i] + br;
    const uint64_t nb = (bi < br) || (a.w[i] < bi) ? 1u : 0u;
    a.w[i] -= bi;
    br = nb;
  }
}
Big mul_small(const Big &a, uint64_t k) {
  Big r;
  u128 c = 0;
  for (int i = 0; i < W; ++i) {
    c += (u128)a.w[i] * k;
    r.w[i] = (uint64_t)c;
    c >>= 64;
  }
  return r;
}
long double approx(const Big &a) {
  long double v = 0;
  for (int i = W - 1; i >= 0; --i) v = v * 18446744073709551616.0L + (long double)a.w[i];
  return v;
}
uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }
uint64_t powmod(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1;
  for (a %= m; e; e >>= 1, a = mulmod(a, a, m))
    if (e & 1) r = mulmod(r, a, m);
  return r;
}
}  // namespace

he_status client_decrypt_crt(const Ctx &c, const uint64_t *x, uint32_t n_ct, int64_t *m) {
  const uint32_t L = c.L, N = c.N;
  Big Q(1);
  for (uint32_t i = 0; i < L; ++i) Q = mul_small(Q, c.q[i]);
  std::vector<Big> Qhat(L);
  std::vector<uint64_t> Qhat_inv(L);
  for (uint32_t i = 0; i < L; ++i) {
    Big h(1);
    uint64_t hm = 1;
    for (uint32_t j = 0; j < L; ++j)
      if (j != i) {
        h = mul_small(h, c.q[j]);
        hm = mulmod(hm, c.q[j] % c.q[i], c.q[i]);
      }
    Qhat[i] = h;
    Qhat_inv[i] = powmod(hm, c.q[i] - 2, c.q[i]);
  }
  const Big Q2 = mul_small(Q, 2);
  const long double Qd = approx(Q);
  const uint64_t t = c.t;
  for (uint32_t k = 0; k < n_ct; ++k) {
    const uint64_t *xk = x + (size_t)k * L * N;
    for (uint32_t j = 0; j < N; ++j) {
      Big S;
      for (uint32_t i = 0; i < L; ++i) {
        const uint64_t y = mulmod(xk[(size_t)i * N + j], Qhat_inv[i], c.q[i]);
        add_to(S, mul_small(Qhat[i], y));
      }
      while (cmp(S, Q) >= 0) sub_from(S, Q);
      Big U = mul_small(S, 2 * t);
      add_to(U, Q);
      long double est = std::floor((approx(S) * (long double)(2 * t) + Qd) / (2.0L * Qd));
      uint64_t m0 = est < 0 ? 0 : (uint64_t)est;
      if (m0 > t) m0 = t;
      Big V = mul_small(Q2, m0);
      while (cmp(V, U) > 0) {
        sub_from(V, Q2);
        --m0;
      }
      for (;;) {
        Big V2 = V;
        add_to(V2, Q2);
        if (cmp(V2, U) > 0) break;
        V = V2;
        ++m0;
      }
      m[(size_t)k * N + j] = (int64_t)(m0 % t);
    }
  }
  return HE_OK;
}

}  // namespace he

namespace {
// Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC 2011) on the host: ten
// rounds of two 64x64 -> 128-bit products of counter words with fixed odd
// multipliers, the halves mixed with the other two words and the key, the key
// stepping by two Weyl constants per round.
void philox4x64_host(uint64_t c[4], uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  for (int r = 0; r < 10; ++r) {
    const unsigned __int128 p0 = (unsigned __int128)M0 * c[0], p1 = (unsigned __int128)M1 * c[2];
    const uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0, hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    c[0] = hi1 ^ c[1] ^ k0;
    c[1] = lo1;
    c[2] = hi0 ^ c[3] ^ k1;
    c[3] = lo0;
    k0 += W0;
    k1 += W1;
  }
}
}  // namespace

extern "C" he_status he_keygen(const he_ctx *ctx, uint64_t seed, int8_t *sk) {
  if (!ctx || !sk) return he::fail(HE_EINVAL, "null argument");
  const uint32_t N = ctx->c->N;
  for (uint32_t k = 0; k < N; ++k) {
    uint64_t c[4] = {k, 0, 0, ~0ull};
    philox4x64_host(c, seed, 0);
    // floor(3 w / 2^64) in {0, 1, 2}: within 2^-63 of uniform
    sk[k] = (int8_t)((int)(((unsigned __int128)c[0] * 3u) >> 64) - 1);
  }
  return HE_OK;
}
