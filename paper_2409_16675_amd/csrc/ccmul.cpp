// Ciphertext-ciphertext product with relinearization: the CCMul of the
// preprocessing phase of Section 3.2 (CryptoTrain-P), [r_x][r_w] -> [r_x r_w].
//
// BFV product (Fan and Vercauteren) on an extended RNS base Q u P:
//   1. lift both operands exactly from Q to Q u P as centred integers;
//   2. transform them and form the tensor slots x0 = a0 b0, x1 = a0 b1 + a1 b0,
//      x2 = a1 b1, summed over an output's terms, with the term-list multiply
//      and fused inverse transform of the layer path (one component per
//      operand; the three slots are term lists of their own);
//   3. d = round(t x / Q) mod Q exactly (mixed-radix conversions, no floating
//      point); the residue of d2 mod q_j is the digit D_j;
//   4. relinearize: transform every digit at every prime (the forward
//      transform that lifts integer polynomials on load, reading D_j and
//      reducing it mod q_i) and multiply-accumulate them against the key,
//      accumulating into (d0, d1), with the same fused kernel.
// P is sized so that every tensor value and every quotient z = (t x - r) / Q
// is exact in it: log2 P >= log2 t + log2 N + 16 + log2 Q + 2 (up to 2^16
// products per output).
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "he_internal.hpp"
#include "plan.hpp"
#include "rns.hpp"

namespace he {
hipError_t launch_rns_extend(const RnsConv *d_conv, int L, int K, bool f64, uint64_t *out, const uint64_t *in,
                             uint32_t n_polys, uint32_t N, hipStream_t st);
hipError_t launch_rns_scale_round(const RnsConv *d_conv, int L, int K, bool f64, uint64_t *out, uint64_t *dig,
                                  const uint64_t *X, uint32_t n_out, uint32_t N, hipStream_t st);

namespace {
typedef unsigned __int128 u128;
constexpr uint32_t kMaxTermsPerOutput = 1u << 16;
constexpr uint32_t kMaxExtPrimes = 16;

uint64_t mm(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }
uint64_t mp(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  for (; e; e >>= 1, a = mm(a, a, m))
    if (e & 1) r = mm(r, a, m);
  return r;
}
uint64_t inv(uint64_t a, uint64_t m) { return mp(a % m, m - 2, m); }
uint64_t shoup(uint64_t w, uint64_t m) { return (uint64_t)(((u128)w << 64) / m); }

// mixed-radix digits of the residues x over the primes mod[0..n)
void host_mrc(const uint64_t *x, uint64_t *v, int n, const uint64_t *mod) {
  for (int i = 0; i < n; ++i) {
    uint64_t u = x[i];
    for (int j = 0; j < i; ++j) u = mm((u + mod[i] - v[j] % mod[i]) % mod[i], inv(mod[j], mod[i]), mod[i]);
    v[i] = u;
  }
}

void fill_conv(RnsConv &cv, const std::vector<uint64_t> &q, const std::vector<uint64_t> &p, uint64_t t) {
  std::memset(&cv, 0, sizeof(cv));
  const int L = (int)q.size(), K = (int)p.size();
  cv.L = L;
  cv.K = K;
  for (int i = 0; i < L; ++i) {
    cv.q[i] = q[i];
    cv.q_one[i] = (uint64_t)(((u128)1 << 64) / q[i]);
    cv.t_q[i] = t % q[i];
    cv.t_qs[i] = shoup(cv.t_q[i], q[i]);
  }
  for (int k = 0; k < K; ++k) {
    cv.p[k] = p[k];
    cv.p_one[k] = (uint64_t)(((u128)1 << 64) / p[k]);
    cv.t_p[k] = t % p[k];
    cv.t_ps[k] = shoup(cv.t_p[k], p[k]);
    uint64_t Qm = 1;
    for (int i = 0; i < L; ++i) Qm = mm(Qm, q[i], p[k]);
    cv.q_mod_p[k] = Qm;
    cv.qinv_p[k] = inv(Qm, p[k]);
    cv.qinv_ps[k] = shoup(cv.qinv_p[k], p[k]);
  }
  for (int i = 0; i < L; ++i) {
    uint64_t Pm = 1;
    for (int k = 0; k < K; ++k) Pm = mm(Pm, p[k], q[i]);
    cv.p_mod_q[i] = Pm;
  }
  for (int i = 0; i < L; ++i)
    for (int j = 0; j < i; ++j) {
      cv.iqq[j][i] = inv(q[j], q[i]);
      cv.iqqs[j][i] = shoup(cv.iqq[j][i], q[i]);
    }
  for (int k = 0; k < K; ++k)
    for (int j = 0; j < k; ++j) {
      cv.ipp[j][k] = inv(p[j], p[k]);
      cv.ipps[j][k] = shoup(cv.ipp[j][k], p[k]);
    }
  for (int k = 0; k < K; ++k) {
    uint64_t w = 1 % p[k];
    for (int i = 0; i < L; ++i) {
      cv.wq[i][k] = w;
      cv.wqs[i][k] = shoup(w, p[k]);
      w = mm(w, q[i], p[k]);
    }
  }
  for (int i = 0; i < L; ++i) {
    uint64_t w = 1 % q[i];
    for (int k = 0; k < K; ++k) {
      cv.wp[k][i] = w;
      cv.wps[k][i] = shoup(w, q[i]);
      w = mm(w, p[k], q[i]);
    }
  }
  // (Q + 1) / 2 is 2^-1 mod every q_i (Q = 0 there); likewise for P
  uint64_t h[kRnsMax];
  for (int i = 0; i < L; ++i) h[i] = (q[i] + 1) / 2;
  host_mrc(h, cv.hq, L, q.data());
  for (int k = 0; k < K; ++k) h[k] = (p[k] + 1) / 2;
  host_mrc(h, cv.hp, K, p.data());
  for (int i = 0; i < kRnsMax; ++i) {
    cv.dq[i] = (double)cv.q[i];
    cv.dqinv[i] = i < L ? 1.0 / (double)q[i] : 0.0;
    cv.dp[i] = (double)cv.p[i];
    cv.dpinv[i] = i < K ? 1.0 / (double)p[i] : 0.0;
    cv.dt_q[i] = (double)cv.t_q[i];
    cv.dt_p[i] = (double)cv.t_p[i];
    cv.dqinv_p[i] = (double)cv.qinv_p[i];
    cv.dq_mod_p[i] = (double)cv.q_mod_p[i];
    cv.dp_mod_q[i] = (double)cv.p_mod_q[i];
    cv.dhq[i] = (double)cv.hq[i];
    cv.dhp[i] = (double)cv.hp[i];
    for (int j = 0; j < kRnsMax; ++j) {
      cv.diqq[i][j] = (double)cv.iqq[i][j];
      cv.dipp[i][j] = (double)cv.ipp[i][j];
      cv.dwq[i][j] = (double)cv.wq[i][j];
      cv.dwp[i][j] = (double)cv.wp[i][j];
    }
  }
}

// Build the extended base (once; later calls return it).
he_status ext_ring_build(Ctx &c, Ctx **ec, const RnsConv **conv) {
  std::lock_guard<std::mutex> g(c.ectx_mu);
  if (!c.ectx) {
    if (c.L > (uint32_t)kRnsMax) return fail(HE_EUNSUPPORTED, "the ciphertext product supports at most 8 primes");
    uint64_t qmax = 0;
    double need = std::log2((double)c.t) + (double)c.logN + 16.0 + 2.0;
    for (uint64_t q : c.q) {
      need += std::log2((double)q);
      qmax = q > qmax ? q : qmax;
    }
    need += 1.0;   // margin for the double sums
    // auxiliary primes: below 2^48 when the context runs the fp64 path, else as
    // wide as the widest prime of Q; 1 mod 2N, distinct from Q and from t
    const uint32_t bits = c.f64_ok ? 48 : (uint32_t)(64 - __builtin_clzll(qmax));
    const uint64_t m = 2ull * c.N;
    uint64_t cand = ((1ull << bits) - 1) / m * m + 1;
    if (cand >= (1ull << bits)) cand -= m;
    std::vector<uint64_t> P;
    double have = 0.0;
    while (have < need && cand > m) {
      bool clash = cand == c.t;
      for (uint64_t q : c.q) clash = clash || q == cand;
      if (!clash && is_prime64(cand)) {
        P.push_back(cand);
        have += std::log2((double)cand);
      }
      cand -= m;
    }
    if (have < need || P.size() > (size_t)kRnsMax || c.L + P.size() > kMaxExtPrimes)
      return fail(HE_EUNSUPPORTED, "the extended base of the ciphertext product needs too many primes");
    std::vector<uint64_t> all(c.q);
    all.insert(all.end(), P.begin(), P.end());
    he_params prm{};
    prm.N = c.N;
    prm.L = (uint32_t)all.size();
    prm.q = all.data();
    prm.t = c.t;
    prm.arith = c.f64_ok ? HE_ARITH_F64 : HE_ARITH_U64;
    prm.device = c.device;
    Ctx *e = nullptr;
    he_status s = build_context(&prm, &e, kMaxExtPrimes);
    if (s != HE_OK) return s;
    RnsConv cv;
    fill_conv(cv, c.q, P, c.t);
    void *d = nullptr;
    hipError_t err = hipSetDevice(c.device);
    if (err == hipSuccess) err = hipMalloc(&d, sizeof(RnsConv));
    if (err == hipSuccess) err = hipMemcpy(d, &cv, sizeof(RnsConv), hipMemcpyHostToDevice);
    if (err != hipSuccess) {
      if (d) (void)hipFree(d);
      free_context(e);
      return hip_fail(err, "ciphertext product constants");
    }
    c.ectx = e;
    c.d_conv = d;
  }
  *ec = c.ectx;
  *conv = (const RnsConv *)c.d_conv;
  return HE_OK;
}

// The extended base if he_ctx_prepare built it, else HE_EINVAL (hot calls never build it).
he_status ext_ring(Ctx &c, Ctx **ec, const RnsConv **conv) {
  std::lock_guard<std::mutex> g(c.ectx_mu);
  if (!c.ectx) return fail(HE_EINVAL, "ciphertext product not prepared: call he_ctx_prepare with HE_PREPARE_CCMUL");
  *ec = c.ectx;
  *conv = (const RnsConv *)c.d_conv;
  return HE_OK;
}

// int32 words of the device term lists of one call: tensor rows and pairs,
// then the relinearization rows and pairs
size_t cc_list_words(uint32_t n_out, uint32_t n_terms, uint32_t L) {
  return 3 * (size_t)n_out + 1 + 8 * (size_t)n_terms + (size_t)n_out + 1 + 2 * (size_t)n_out * L;
}

size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

struct CcLayout {
  size_t stage, a_hat, b_hat, x, dig, terms, flag, total;
};

CcLayout layout(const Ctx &c, uint32_t E, uint32_t n_a, uint32_t n_b, uint32_t n_out, uint32_t n_terms,
                uint32_t flags) {
  const size_t plane = (size_t)c.N * 8, L = c.L;
  CcLayout l{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += al(bytes);
    return at;
  };
  l.stage = take((size_t)(n_a + n_b) * 2 * E * plane);   // both lifted operands, transformed in one launch
  l.a_hat = take((size_t)n_a * 2 * E * plane);
  l.b_hat = take((size_t)n_b * 2 * E * plane);
  const size_t xb = (size_t)n_out * 3 * E * plane, db = (size_t)n_out * L * L * plane;
  l.x = take(xb > db ? xb : db);                       // tensor slots, then the transformed digits
  l.dig = take((size_t)n_out * L * plane);             // d2: digit j is its residue mod q_j
  l.terms = take(4 * cc_list_words(n_out, n_terms, (uint32_t)L));
  l.flag = take((flags & HE_VALIDATE) ? 256 : 0);
  l.total = off;
  return l;
}
}  // namespace

// The extended base, its constants, and the two pinned staging buffers of the
// term lists sized for calls of up to max_out outputs and max_terms products.
he_status ccmul_prepare(Ctx &c, uint32_t max_out, uint32_t max_terms) {
  Ctx *ec = nullptr;
  const RnsConv *cv = nullptr;
  he_status s = ext_ring_build(c, &ec, &cv);
  if (s != HE_OK) return s;
  std::lock_guard<std::mutex> lk(c.cc_mu);
  const size_t bytes = 4 * cc_list_words(max_out, max_terms, c.L);
  for (int k = 0; k < 2; ++k) {
    hipError_t e = hipSuccess;
    if (!c.cc_ev[k]) e = hipEventCreateWithFlags(&c.cc_ev[k], hipEventDisableTiming);
    else e = hipEventSynchronize(c.cc_ev[k]);
    if (e != hipSuccess) return hip_fail(e, "ccmul staging event");
    if (c.cc_pin_bytes[k] < bytes) {
      if (c.cc_pin[k] && (e = hipHostFree(c.cc_pin[k])) != hipSuccess) return hip_fail(e, "ccmul staging");
      c.cc_pin[k] = nullptr;
      c.cc_pin_bytes[k] = 0;
      if ((e = hipHostMalloc(&c.cc_pin[k], bytes, hipHostMallocDefault)) != hipSuccess)
        return hip_fail(e, "ccmul staging");
      c.cc_pin_bytes[k] = bytes;
    }
  }
  return HE_OK;
}
}  // namespace he

using namespace he;

#define HIPCHK(expr, what)                               \
  do {                                                   \
    hipError_t e_ = (expr);                              \
    if (e_ != hipSuccess) return hip_fail(e_, what);     \
  } while (0)

extern "C" {

he_status he_ccmul_ws_size(he_ctx *ctx, uint32_t n_a, uint32_t n_b, uint32_t n_out, uint32_t n_terms,
                           uint32_t flags, size_t *bytes) {
  if (!ctx || !bytes) return fail(HE_EINVAL, "null argument");
  Ctx &c = *ctx->c;
  Ctx *ec = nullptr;
  const RnsConv *cv = nullptr;
  he_status s = ext_ring(c, &ec, &cv);
  if (s != HE_OK) return s;
  *bytes = layout(c, ec->L, n_a, n_b, n_out, n_terms, flags).total;
  return HE_OK;
}

he_status he_ccmul(he_ctx *ctx, const uint64_t *a, uint32_t n_a, const uint64_t *b, uint32_t n_b, const int32_t *row,
                   const int32_t *a_idx, const int32_t *b_idx, uint32_t n_out, const uint64_t *rlk_hat, uint64_t *out,
                   uint32_t flags, void *ws, size_t ws_bytes, void *stream) {
  if (!ctx || !a || !b || !rlk_hat || !out) return fail(HE_EINVAL, "null argument");
  if (flags & ~HE_VALIDATE) return fail(HE_EINVAL, "flags: only HE_VALIDATE applies");
  Ctx &c = *ctx->c;
  // term lists (host): identity pairs when row is NULL
  std::vector<int32_t> r0, ai, bi;
  if (!row) {
    if (n_a != n_b || n_out != n_a) return fail(HE_EINVAL, "pairwise products need n_a == n_b == n_out");
    for (uint32_t k = 0; k <= n_out; ++k) r0.push_back((int32_t)k);
    for (uint32_t k = 0; k < n_out; ++k) {
      ai.push_back((int32_t)k);
      bi.push_back((int32_t)k);
    }
  } else {
    if (!a_idx || !b_idx) return fail(HE_EINVAL, "null term list");
    if (row[0] != 0) return fail(HE_EINVAL, "row[0] must be 0");
    for (uint32_t o = 0; o < n_out; ++o)
      if (row[o + 1] < row[o] || (uint32_t)(row[o + 1] - row[o]) > kMaxTermsPerOutput)
        return fail(row[o + 1] < row[o] ? HE_EINVAL : HE_EUNSUPPORTED,
                    "row must be non-decreasing with at most 65536 terms per output");
    r0.assign(row, row + n_out + 1);
    ai.assign(a_idx, a_idx + row[n_out]);
    bi.assign(b_idx, b_idx + row[n_out]);
    for (size_t k = 0; k < ai.size(); ++k)
      if (ai[k] < 0 || (uint32_t)ai[k] >= n_a || bi[k] < 0 || (uint32_t)bi[k] >= n_b)
        return fail(HE_EINVAL, "term index out of range");
  }
  const uint32_t n_terms = (uint32_t)ai.size();
  Ctx *ec = nullptr;
  const RnsConv *cv = nullptr;
  he_status rs = ext_ring(c, &ec, &cv);
  if (rs != HE_OK) return rs;
  const uint32_t E = ec->L, L = c.L, N = c.N;
  const CcLayout l = layout(c, E, n_a, n_b, n_out, n_terms, flags);
  if (ws_bytes < l.total || !ws) return fail(HE_ENOMEM, "workspace too small");
  hipStream_t st = (hipStream_t)stream;
  char *w = (char *)ws;
  if (flags & HE_VALIDATE) {
    he_status s = validate(c, a, (size_t)n_a * 2 * L, w + l.flag, st);
    if (s == HE_OK) s = validate(c, b, (size_t)n_b * 2 * L, w + l.flag, st);
    if (s == HE_OK) s = validate(c, rlk_hat, (size_t)L * 2 * L, w + l.flag, st);
    if (s != HE_OK) return s;
  }
  // tensor lists: output (o, slot) over one-component operands a[2 j + c], b[2 j + c]
  std::vector<int32_t> tl;
  tl.reserve(3 * (size_t)n_out + 1 + 8 * (size_t)n_terms + n_out + 1 + 2 * (size_t)n_out * L);
  std::vector<int32_t> tc, tp;
  tl.push_back(0);
  for (uint32_t o = 0; o < n_out; ++o) {
    for (int slot = 0; slot < 3; ++slot) {
      for (int32_t k = r0[o]; k < r0[o + 1]; ++k) {
        const int32_t ja = 2 * ai[k], jb = 2 * bi[k];
        if (slot == 0) {
          tc.push_back(ja);
          tp.push_back(jb);
        } else if (slot == 1) {
          tc.push_back(ja);
          tp.push_back(jb + 1);
          tc.push_back(ja + 1);
          tp.push_back(jb);
        } else {
          tc.push_back(ja + 1);
          tp.push_back(jb + 1);
        }
      }
      tl.push_back((int32_t)tc.size());
    }
  }
  const size_t t_row = 0, t_ct = tl.size(), t_pt = t_ct + tc.size();
  tl.insert(tl.end(), tc.begin(), tc.end());
  tl.insert(tl.end(), tp.begin(), tp.end());
  // relinearization lists: output o = sum_j rlk_j (x) digit (o, j)
  const size_t r_row = tl.size();
  for (uint32_t o = 0; o <= n_out; ++o) tl.push_back((int32_t)(o * L));
  const size_t r_ct = tl.size();
  for (uint32_t o = 0; o < n_out; ++o)
    for (uint32_t j = 0; j < L; ++j) tl.push_back((int32_t)j);
  const size_t r_pt = tl.size();
  for (uint32_t o = 0; o < n_out; ++o)
    for (uint32_t j = 0; j < L; ++j) tl.push_back((int32_t)(o * L + j));
  int32_t *d_tl = (int32_t *)(w + l.terms);
  {
    // through one of the context's two pinned staging buffers: wait only for
    // the copy that last read it (two calls back), so the host prepares this
    // call while the previous one still runs
    std::lock_guard<std::mutex> lk(c.cc_mu);
    const int k = c.cc_next;
    const size_t bytes = tl.size() * 4;
    if (!c.cc_ev[k] || c.cc_pin_bytes[k] < bytes)
      return fail(HE_EINVAL, "term lists larger than he_ctx_prepare sized the staging for");
    HIPCHK(hipEventSynchronize(c.cc_ev[k]), "ccmul staging");
    std::memcpy(c.cc_pin[k], tl.data(), bytes);
    HIPCHK(hipMemcpyAsync(d_tl, c.cc_pin[k], bytes, hipMemcpyHostToDevice, st), "ccmul term lists");
    HIPCHK(hipEventRecord(c.cc_ev[k], st), "ccmul staging");
    c.cc_next = k ^ 1;
  }
  if (!n_out) return HE_OK;

  uint64_t *stage = (uint64_t *)(w + l.stage), *a_hat = (uint64_t *)(w + l.a_hat), *b_hat = (uint64_t *)(w + l.b_hat);
  uint64_t *X = (uint64_t *)(w + l.x), *dig = (uint64_t *)(w + l.dig);
  const Sched sf{ec->f64_ok ? HE_ARITH_F64 : HE_ARITH_U64, c.s_fwd.loge};
  const Sched sm{ec->f64_ok ? HE_ARITH_F64 : HE_ARITH_U64, c.s_mac.loge};
  uint64_t *stage_b = stage + (size_t)n_a * 2 * E * N;
  HIPCHK(timed(c, st, KK_RNS, [&] { return launch_rns_extend(cv, (int)L, (int)(E - L), ec->f64_ok, stage, a, n_a * 2, N, st); }), "ccmul extend a");
  HIPCHK(timed(c, st, KK_RNS, [&] { return launch_rns_extend(cv, (int)L, (int)(E - L), ec->f64_ok, stage_b, b, n_b * 2, N, st); }), "ccmul extend b");
  HIPCHK(timed(c, st, KK_FWD,
               [&] { return launch_ntt_fwd2(*ec, sf, a_hat, stage, n_a * 2 * E, b_hat, stage_b, n_b * 2 * E, st); }),
         "ccmul fwd a, b");
  Terms tt;
  tt.row = d_tl + t_row;
  tt.cti = d_tl + t_ct;
  tt.pti = d_tl + t_pt;
  tt.n_out = n_out * 3;
  HIPCHK(timed(c, st, KK_MAC_INV, [&] { return launch_mac(*ec, sm, X, a_hat, b_hat, tt, false, false, st, 1); }),
         "ccmul tensor");
  HIPCHK(timed(c, st, KK_RNS, [&] { return launch_rns_scale_round(cv, (int)L, (int)(E - L), ec->f64_ok, out, dig, X, n_out, N, st); }),
         "ccmul scale and round");
  // plane (o * L + j) * L + i of the transformed digits: d2[o][j] lifted mod q_i
  HIPCHK(timed(c, st, KK_FWD_LIFT,
               [&] { return launch_ntt_fwd_lift(c, c.s_fwd, X, (const int64_t *)dig, n_out * L, st); }),
         "ccmul fwd digits");
  Terms tr;
  tr.row = d_tl + r_row;
  tr.cti = d_tl + r_ct;
  tr.pti = d_tl + r_pt;
  tr.n_out = n_out;
  HIPCHK(timed(c, st, KK_MAC_INV, [&] { return launch_mac(c, c.s_mac, out, rlk_hat, X, tr, true, false, st, 2); }),
         "ccmul relinearize");
  return HE_OK;
}

}  // extern "C"
