// Internal declarations shared by the host sources of libhe.so.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/he.h"
#include "arith.hpp"

namespace he {

// A transform / fused-kernel schedule: arithmetic policy and threads per plane.
struct Sched {
  int arith;   // HE_ARITH_F64 or HE_ARITH_U64
  int loge;    // log2 of coefficients per thread (3, 4 or 5)
};

struct Ctx {
  uint32_t N = 0, L = 0, logN = 0;
  uint64_t t = 0;
  int device = 0;
  int arith = HE_ARITH_U64;      // default policy
  bool f64_ok = false;           // every q_i < 2^48
  std::vector<uint64_t> q, psi;
  std::vector<uint64_t> delta_mod;   // floor(Q / t) mod q_i
  // device tables
  PrimeK *d_primes = nullptr;        // [L]
  void *d_tw_f64_fwd = nullptr;      // TwF64 [L][N]
  void *d_tw_f64_inv = nullptr;     // TwF64 [L][N], then the twiddles alone:
  const double *d_tw_f64_inv_w = nullptr;   // double [L][N] (same allocation)
  void *d_tw_u64_fwd = nullptr;      // TwU64 [L][N]
  void *d_tw_u64_inv = nullptr;
  // per-kernel timing (he_ctx_profile)
  struct ProfRec {
    int kind;
    hipEvent_t a, b;
  };
  mutable std::mutex prof_mu;
  mutable bool prof_on = false;
  mutable std::vector<ProfRec> prof;
  // schedules chosen per operation (autotuner may change them)
  Sched s_fwd{HE_ARITH_U64, 4}, s_inv{HE_ARITH_U64, 4}, s_mac{HE_ARITH_U64, 4};
  // ring of the plaintext modulus (one prime, q = t), built on first use by
  // the plaintext product; owned by this context
  Ctx *tctx = nullptr;
  std::mutex tctx_mu;
  // extended base Q u P of the ciphertext-ciphertext product (primes of this
  // context first) and its exact conversion constants (device RnsConv),
  // built on first use; owned by this context
  Ctx *ectx = nullptr;
  void *d_conv = nullptr;
  std::mutex ectx_mu;
  // pinned staging of the ciphertext product's term lists, two buffers used
  // in turn; event k completes when the copy that last read buffer k has
  // (so a call waits for the copy two calls back, not for the previous call)
  void *cc_pin[2] = {nullptr, nullptr};
  size_t cc_pin_bytes[2] = {0, 0};
  hipEvent_t cc_ev[2] = {nullptr, nullptr};
  int cc_next = 0;
  std::mutex cc_mu;
};

he_status build_context(const he_params *p, Ctx **out, uint32_t max_L = 8);
void free_context(Ctx *c);
bool is_prime64(uint64_t n);
// HE_ERANGE unless every coefficient of the [n][L][N] planes is below its prime
he_status validate(const Ctx &c, const uint64_t *planes, size_t n_planes, void *flag_mem, hipStream_t st);

enum KernelKind { KK_FWD = 0, KK_FWD_LIFT = 1, KK_INV = 2, KK_MAC_INV = 3, KK_MAC = 4, KK_PACK = 5, KK_PERSIST = 6, KK_RNS = 7 };

// Bracket one launch with events when profiling is on: returns the launch's error.
// Set on a thread while a call that must not allocate runs: kernel timing
// (which creates events) is skipped for its launches.
extern thread_local bool g_untimed;

template <class F>
hipError_t timed(const Ctx &c, hipStream_t st, int kind, F &&launch) {
  if (!c.prof_on || g_untimed) return launch();
  Ctx::ProfRec r{kind, nullptr, nullptr};
  hipError_t e = hipEventCreate(&r.a);
  if (e == hipSuccess) e = hipEventCreate(&r.b);
  if (e == hipSuccess) e = hipEventRecord(r.a, st);
  if (e != hipSuccess) return e;
  e = launch();
  hipError_t e2 = hipEventRecord(r.b, st);
  {
    std::lock_guard<std::mutex> g(c.prof_mu);
    c.prof.push_back(r);
  }
  return e != hipSuccess ? e : e2;
}

// thread-local error text
void set_error(const std::string &msg);
he_status fail(he_status st, const std::string &msg);
he_status hip_fail(hipError_t e, const char *what);

// ------------------------------------------------------------------ launchers
// All return hipSuccess or the launch error.  Planes [n][L][N]; prime of plane p is p % L.
hipError_t launch_ntt_fwd(const Ctx &c, const Sched &s, uint64_t *out, const uint64_t *in, uint32_t n_planes,
                          hipStream_t st);
hipError_t launch_ntt_fwd_lift(const Ctx &c, const Sched &s, uint64_t *out, const int64_t *polys, uint32_t n_polys,
                               hipStream_t st);
hipError_t launch_ntt_inv(const Ctx &c, const Sched &s, uint64_t *out, const uint64_t *in, uint32_t n_planes,
                          hipStream_t st);
// Layout of raw weights packed into plaintext polynomials (pack.hpp scatters them).
enum WPackKind : uint32_t { WP_CONV = 0, WP_CONV_DX = 1, WP_FC = 2 };
struct WPack {
  uint32_t kind;                               // WP_*
  uint32_t M, C, h, O, S, Cw, cb;              // conv (DX: of the equivalent forward conv)
  uint32_t n_out, n_in, n_iw, n_ow, in_ct;     // FC
};
// forward transform of n_polys plaintext polynomials packed from raw int32
// weights in LDS (layout wp): out [n_polys][L][N]
hipError_t launch_ntt_fwd_pack(const Ctx &c, const Sched &s, uint64_t *out, const int32_t *w, const WPack &wp,
                               uint32_t n_polys, hipStream_t st);
// forward transforms of two plane arrays in one launch (in1 -> out1, in2 -> out2)
hipError_t launch_ntt_fwd2(const Ctx &c, const Sched &s, uint64_t *out1, const uint64_t *in1, uint32_t n1_planes,
                           uint64_t *out2, const uint64_t *in2, uint32_t n2_planes, hipStream_t st);
// both in one launch: n_ct_planes ciphertext planes ct_in -> ct_out, and
// n_polys plaintext polynomials packed from w -> pt_out.  With a seed
// (2 words), ct_in holds component 0 only ([n][L][N]) and component 1 is
// regenerated from the seed.
hipError_t launch_ntt_fwd_ct_pack(const Ctx &c, const Sched &s, uint64_t *ct_out, const uint64_t *ct_in,
                                  uint32_t n_ct_planes, uint64_t *pt_out, const int32_t *w, const WPack &wp,
                                  uint32_t n_polys, hipStream_t st, const uint64_t *seed = nullptr);
// forward transform of n_ct ciphertexts [n_ct][2][L][N] whose component 0 is ct0
// [n_ct][L][N] and whose component 1 is regenerated from the seed
hipError_t launch_ntt_fwd_seeded(const Ctx &c, const Sched &s, uint64_t *out, const uint64_t *ct0, uint64_t seed0,
                                 uint64_t seed1, uint32_t n_ct, hipStream_t st);
// component 1 of ciphertexts first .. first+n_ct-1 -> out [n_ct][L][N]
hipError_t launch_expand_c1(const Ctx &c, uint64_t *out, uint64_t seed0, uint64_t seed1, uint32_t first, uint32_t n_ct,
                            hipStream_t st);
// Term-list multiply-accumulate in the transformed domain followed by the
// inverse transform (fused), or left transformed (out_ntt).  Output plane
// (o, comp, i) = sum_t ct_hat[cti[t]][comp][i] * pt_hat[pti[t]][i].
// With row == nullptr there is one output and terms t = 0..K-1 (identity lists).
struct Terms {
  const int32_t *row = nullptr, *cti = nullptr, *pti = nullptr;
  uint32_t n_out = 1;
  uint32_t K = 0;   // identity mode only
};
// ncomp: components per operand (2: ciphertext x plaintext; 1: plaintext x
// plaintext, fused inverse only, no accumulate).
hipError_t launch_mac(const Ctx &c, const Sched &s, uint64_t *out, const uint64_t *ct_hat, const uint64_t *pt_hat,
                      const Terms &tm, bool accumulate, bool out_ntt, hipStream_t st, int ncomp = 2);

hipError_t launch_zero_i64(int64_t *p, size_t n, hipStream_t st);
// dx: read the kernel of an input gradient from forward weights [C][M][h][h]
// (transposed channels, rotated by 180 degrees)
hipError_t launch_pack_conv_w(int64_t *polys, const int32_t *w, uint32_t M, uint32_t C, uint32_t h, uint32_t O,
                              uint32_t S, uint32_t Cw, uint32_t cb, uint32_t N, bool dx, hipStream_t st);
hipError_t launch_pack_fc_w(int64_t *polys, const int32_t *W, uint32_t n_out, uint32_t n_in, uint32_t n_iw,
                            uint32_t n_ow, uint32_t in_ct, uint32_t N, hipStream_t st);
// validation: count of coefficients >= q_i in [n][L][N] planes, written to *bad (device)
hipError_t launch_check_canonical(const Ctx &c, const uint64_t *planes, size_t n_planes, uint32_t *bad,
                                  hipStream_t st);

// encryption helpers
template <class T>
hipError_t launch_lift(const Ctx &c, uint64_t *out, const T *v, hipStream_t st);   // [N] -> [L][N]
hipError_t launch_pmul_bcast(const Ctx &c, uint64_t *out, const uint64_t *x, const uint64_t *y, uint32_t n_planes,
                             hipStream_t st);   // out[p] = x[p] * y[p % L]
hipError_t launch_add_planes(const Ctx &c, uint64_t *out, const uint64_t *a, const uint64_t *b, uint32_t n_planes,
                             hipStream_t st);
hipError_t launch_enc_combine(const Ctx &c, uint64_t *c0, const uint64_t *prod, const int32_t *e, const int64_t *m,
                              const uint64_t *delta_w /*device [2L]: w, w'*/, hipStream_t st);
hipError_t launch_copy_u64(uint64_t *dst, const uint64_t *src, size_t n, hipStream_t st);

// Schedules compiled into the library for a ring degree (used by the autotuner and tests).
std::vector<Sched> schedules_for(uint32_t logN, bool f64_ok);
bool sched_valid(uint32_t logN, const Sched &s);

}  // namespace he
