// Context set-up: RNS primes, roots, twiddle tables and per-prime constants.
#include <cstring>
#include <mutex>
#include <string>

#include "he_internal.hpp"

namespace he {

namespace {
typedef unsigned __int128 u128;

uint64_t mmul(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }
uint64_t mpow(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  for (; e; e >>= 1, a = mmul(a, a, m))
    if (e & 1) r = mmul(r, a, m);
  return r;
}

// Strong-probable-prime test with a witness set proven sufficient below 2^64.
bool prime64(uint64_t n) {
  if (n < 4) return n >= 2;
  if (!(n & 1)) return false;
  uint64_t d = n - 1;
  int s = __builtin_ctzll(d);
  d >>= s;
  static const uint64_t wit[7] = {2, 325, 9375, 28178, 450775, 9780504, 1795265022};
  for (uint64_t a : wit) {
    a %= n;
    if (a == 0) continue;
    uint64_t x = mpow(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool ok = false;
    for (int r = 1; r < s && !ok; ++r) {
      x = mmul(x, x, n);
      ok = (x == n - 1);
    }
    if (!ok) return false;
  }
  return true;
}

uint32_t rev_bits(uint32_t v, uint32_t bits) {
  uint32_t r = 0;
  for (uint32_t k = 0; k < bits; ++k, v >>= 1) r = (r << 1) | (v & 1u);
  return r;
}

// Smallest element of order exactly 2N (N a power of two): the least x with
// x^N = -1.  The set of such x is {g^k : k odd} for any one of them g, found
// from a quadratic non-residue z as z^((q-1)/2N).
uint64_t least_root(uint64_t q, uint32_t N) {
  uint64_t z = 2;
  while (mpow(z, (q - 1) >> 1, q) != q - 1) ++z;
  const uint64_t g = mpow(z, (q - 1) / (2ull * N), q);
  const uint64_t g2 = mmul(g, g, q);
  uint64_t best = g, cur = g;
  for (uint32_t k = 1; k < N; ++k) {
    cur = mmul(cur, g2, q);
    if (cur < best) best = cur;
  }
  return best;
}
}  // namespace

bool is_prime64(uint64_t n) { return prime64(n); }

// max_L: 8 for contexts of the API; internal rings (the extended base of the
// ciphertext-ciphertext product) allow up to 16 primes
he_status build_context(const he_params *p, Ctx **out, uint32_t max_L) {
  if (!p || !out) return fail(HE_EINVAL, "null argument");
  const uint32_t N = p->N, L = p->L;
  if (N < 1024 || N > 16384 || (N & (N - 1))) return fail(HE_EINVAL, "N must be a power of two in [1024, 16384]");
  if (L < 1 || L > max_L) return fail(HE_EINVAL, "L must be in [1, " + std::to_string(max_L) + "]");
  if (p->t < 2 || p->t >= (1ull << 32)) return fail(HE_EINVAL, "t must be in [2, 2^32)");
  Ctx *c = new Ctx();
  c->N = N;
  c->L = L;
  c->logN = (uint32_t)__builtin_ctz(N);
  c->t = p->t;
  c->device = p->device;
  const uint64_t m = 2ull * N;
  if (p->q) {
    for (uint32_t i = 0; i < L; ++i) {
      const uint64_t q = p->q[i];
      if (q >= (1ull << 62) || q % m != 1 || !prime64(q)) {
        delete c;
        return fail(HE_EINVAL, "explicit modulus is not a prime = 1 mod 2N below 2^62");
      }
      c->q.push_back(q);
    }
  } else {
    const uint32_t bits = p->prime_bits;
    if (bits < 20 || bits > 62) {
      delete c;
      return fail(HE_EINVAL, "prime_bits must be in [20, 62]");
    }
    uint64_t cand = ((1ull << bits) - 1) / m * m + 1;
    if (cand >= (1ull << bits)) cand -= m;
    while (c->q.size() < L && cand > m) {
      if (prime64(cand)) c->q.push_back(cand);
      cand -= m;
    }
    if (c->q.size() < L) {
      delete c;
      return fail(HE_EINVAL, "not enough primes");
    }
  }
  for (uint32_t i = 0; i < L; ++i) {
    for (uint32_t j = 0; j < i; ++j)
      if (c->q[i] == c->q[j]) {
        delete c;
        return fail(HE_EINVAL, "primes must be distinct");
      }
    if (c->q[i] % p->t == 0) {
      delete c;
      return fail(HE_EINVAL, "t must be coprime to every prime");
    }
  }
  c->f64_ok = true;
  for (uint64_t q : c->q) c->f64_ok = c->f64_ok && q < (1ull << 48);
  if (p->arith == HE_ARITH_F64 && !c->f64_ok) {
    delete c;
    return fail(HE_EUNSUPPORTED, "fp64 arithmetic needs every prime below 2^48");
  }
  c->arith = p->arith == HE_ARITH_AUTO ? (c->f64_ok ? HE_ARITH_F64 : HE_ARITH_U64) : (int)p->arith;
  const int loge = 4;
  c->s_fwd = c->s_inv = c->s_mac = Sched{c->arith, loge};

  // Delta = floor(Q / t) mod q_i = -(Q mod t) * t^-1 mod q_i
  uint64_t Qmod_t = 1;
  for (uint64_t q : c->q) Qmod_t = (uint64_t)((u128)Qmod_t * (q % p->t) % p->t);
  for (uint64_t q : c->q) {
    const uint64_t tinv = mpow(p->t % q, q - 2, q);
    c->delta_mod.push_back((q - mmul(Qmod_t % q, tinv, q)) % q);
  }

  // host tables
  std::vector<PrimeK> pk(L);
  std::vector<TwF64> ff((size_t)L * N), fi((size_t)L * N);
  std::vector<TwU64> uf((size_t)L * N), ui((size_t)L * N);
  for (uint32_t i = 0; i < L; ++i) {
    const uint64_t q = c->q[i];
    const uint64_t psi = least_root(q, N);
    c->psi.push_back(psi);
    const uint64_t psi_inv = mpow(psi, q - 2, q);
    const uint64_t n_inv = mpow(N, q - 2, q);
    PrimeK &k = pk[i];
    k.q = q;
    k.two_q = 2 * q;
    k.qd = (double)q;
    k.qinv = 1.0 / (double)q;
    k.r64 = (uint64_t)(((u128)1 << 64) % q);
    k.r64s = (uint64_t)(((u128)k.r64 << 64) / q);
    k.one_s = (uint64_t)(((u128)1 << 64) / q);
    k.pad = 0;
    auto put = [&](size_t idx, uint64_t w, bool inv) {
      TwF64 f{(double)w, (double)w / (double)q};
      TwU64 u{w, (uint64_t)(((u128)w << 64) / q)};
      if (inv) {
        fi[idx] = f;
        ui[idx] = u;
      } else {
        ff[idx] = f;
        uf[idx] = u;
      }
    };
    for (uint32_t j = 0; j < N; ++j) {
      const uint32_t r = rev_bits(j, c->logN);
      put((size_t)i * N + j, mpow(psi, r, q), false);
      put((size_t)i * N + j, mpow(psi_inv, r, q), true);
    }
    // inverse entries 0 and 1 carry N^-1 for the last stage
    put((size_t)i * N + 0, n_inv, true);
    put((size_t)i * N + 1, mmul(mpow(psi_inv, rev_bits(1, c->logN), q), n_inv, q), true);
  }

  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "hipSetDevice");
  }
  const size_t tb = (size_t)L * N * 16;
  // the fp64 inverse table is followed by its twiddles alone (8 bytes each),
  // for transform passes whose lanes read different entries: half the bytes
  // and registers, the quotient companion formed at the product
  std::vector<unsigned char> fiw(tb + (size_t)L * N * 8);
  std::memcpy(fiw.data(), fi.data(), tb);
  for (size_t j = 0; j < fi.size(); ++j) std::memcpy(fiw.data() + tb + j * 8, &fi[j].w, 8);
  void *mem[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  const size_t sz[5] = {sizeof(PrimeK) * L, tb, tb + (size_t)L * N * 8, tb, tb};
  const void *src[5] = {pk.data(), ff.data(), fiw.data(), uf.data(), ui.data()};
  for (int j = 0; j < 5; ++j) {
    if ((e = hipMalloc(&mem[j], sz[j])) != hipSuccess || (e = hipMemcpy(mem[j], src[j], sz[j], hipMemcpyHostToDevice)) != hipSuccess) {
      for (int k = 0; k <= j; ++k)
        if (mem[k]) (void)hipFree(mem[k]);
      delete c;
      return hip_fail(e, "context tables");
    }
  }
  c->d_primes = (PrimeK *)mem[0];
  c->d_tw_f64_fwd = mem[1];
  c->d_tw_f64_inv = mem[2];
  c->d_tw_f64_inv_w = (const double *)((const char *)mem[2] + tb);
  c->d_tw_u64_fwd = mem[3];
  c->d_tw_u64_inv = mem[4];
  *out = c;
  return HE_OK;
}

void free_context(Ctx *c) {
  if (!c) return;
  if (c->tctx) free_context(c->tctx);
  if (c->ectx) free_context(c->ectx);
  if (c->d_conv) {
    (void)hipSetDevice(c->device);
    (void)hipFree(c->d_conv);
  }
  for (int k = 0; k < 2; ++k) {
    (void)hipSetDevice(c->device);
    if (c->cc_ev[k]) {
      (void)hipEventSynchronize(c->cc_ev[k]);
      (void)hipEventDestroy(c->cc_ev[k]);
    }
    if (c->cc_pin[k]) (void)hipHostFree(c->cc_pin[k]);
  }
  (void)hipSetDevice(c->device);
  for (void *p : {(void *)c->d_primes, c->d_tw_f64_fwd, c->d_tw_f64_inv, c->d_tw_u64_fwd, c->d_tw_u64_inv})
    if (p) (void)hipFree(p);
  delete c;
}

}  // namespace he
