// C ABI of libhe.so (declared in include/he.h).
#include <cstring>
#include <string>

#include "plan.hpp"

namespace he {
he_status client_decrypt_crt(const Ctx &c, const uint64_t *x, uint32_t n_ct, int64_t *m);
he_status ccmul_prepare(Ctx &c, uint32_t max_out, uint32_t max_terms);

static thread_local std::string g_err;
thread_local bool g_untimed = false;
void set_error(const std::string &msg) { g_err = msg; }
he_status fail(he_status st, const std::string &msg) {
  g_err = msg;
  return st;
}
he_status hip_fail(hipError_t e, const char *what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return HE_EDEVICE;
}
}  // namespace he

using namespace he;

#define HIPCHK(expr, what)                      \
  do {                                          \
    hipError_t e_ = (expr);                     \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

static inline size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

extern "C" {

const char *he_status_str(he_status s) {
  switch (s) {
    case HE_OK: return "ok";
    case HE_EINVAL: return "invalid argument";
    case HE_EUNSUPPORTED: return "unsupported";
    case HE_ENOMEM: return "out of memory or workspace too small";
    case HE_EDEVICE: return "device error";
    case HE_ERANGE: return "coefficient out of range";
    case HE_EBUSY: return "admission refused";
    case HE_ETIMEOUT: return "timeout";
    default: return "unknown status";
  }
}

const char *he_last_error(void) { return g_err.c_str(); }

he_status he_ctx_create(const he_params *params, he_ctx **out) {
  if (!out) return fail(HE_EINVAL, "null output");
  *out = nullptr;
  Ctx *c = nullptr;
  he_status st = build_context(params, &c);
  if (st != HE_OK) return st;
  *out = new he_ctx{c};
  return HE_OK;
}

static void prof_clear(const Ctx &c);

he_status he_ctx_destroy(he_ctx *ctx) {
  if (!ctx) return HE_OK;
  prof_clear(*ctx->c);
  free_context(ctx->c);
  delete ctx;
  return HE_OK;
}

he_status he_ctx_moduli(const he_ctx *ctx, uint64_t *q_out, uint64_t *psi_out) {
  if (!ctx) return fail(HE_EINVAL, "null context");
  for (uint32_t i = 0; i < ctx->c->L; ++i) {
    if (q_out) q_out[i] = ctx->c->q[i];
    if (psi_out) psi_out[i] = ctx->c->psi[i];
  }
  return HE_OK;
}

he_status he_ctx_info(const he_ctx *ctx, uint32_t *N, uint32_t *L, uint64_t *t, uint32_t *arith) {
  if (!ctx) return fail(HE_EINVAL, "null context");
  if (N) *N = ctx->c->N;
  if (L) *L = ctx->c->L;
  if (t) *t = ctx->c->t;
  if (arith) *arith = (uint32_t)ctx->c->arith;
  return HE_OK;
}

static Sched *sched_slot(Ctx &c, uint32_t op) {
  return op == HE_OP_FWD ? &c.s_fwd : op == HE_OP_INV ? &c.s_inv : op == HE_OP_MAC ? &c.s_mac : nullptr;
}

he_status he_ctx_set_schedule(he_ctx *ctx, uint32_t op, uint32_t arith, uint32_t loge) {
  if (!ctx) return fail(HE_EINVAL, "null context");
  Sched *s = sched_slot(*ctx->c, op);
  if (!s) return fail(HE_EINVAL, "unknown operation");
  Sched n{(int)arith, (int)loge};
  if ((arith != HE_ARITH_F64 && arith != HE_ARITH_U64) || !sched_valid(ctx->c->logN, n))
    return fail(HE_EUNSUPPORTED, "schedule not compiled for this ring degree");
  if (arith == HE_ARITH_F64 && !ctx->c->f64_ok) return fail(HE_EUNSUPPORTED, "fp64 arithmetic needs primes below 2^48");
  *s = n;
  return HE_OK;
}

he_status he_ctx_get_schedule(const he_ctx *ctx, uint32_t op, uint32_t *arith, uint32_t *loge) {
  if (!ctx) return fail(HE_EINVAL, "null context");
  Sched *s = sched_slot(*ctx->c, op);
  if (!s) return fail(HE_EINVAL, "unknown operation");
  if (arith) *arith = (uint32_t)s->arith;
  if (loge) *loge = (uint32_t)s->loge;
  return HE_OK;
}

static void prof_clear(const Ctx &c) {
  std::lock_guard<std::mutex> g(c.prof_mu);
  for (auto &r : c.prof) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  c.prof.clear();
}

he_status he_ctx_profile(he_ctx *ctx, int enable) {
  if (!ctx) return fail(HE_EINVAL, "null context");
  if (enable) prof_clear(*ctx->c);
  ctx->c->prof_on = enable != 0;
  return HE_OK;
}

he_status he_ctx_profile_read(he_ctx *ctx, he_kernel_stat *out, uint32_t cap, uint32_t *n) {
  if (!ctx || !n) return fail(HE_EINVAL, "null argument");
  const Ctx &c = *ctx->c;
  he_kernel_stat acc[8];
  for (uint32_t k = 0; k < 8; ++k) acc[k] = he_kernel_stat{k, 0, 0.0, 0.0};
  {
    std::lock_guard<std::mutex> g(c.prof_mu);
    for (auto &r : c.prof) {
      hipError_t e = hipEventSynchronize(r.b);
      if (e != hipSuccess) return hip_fail(e, "profile sync");
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, r.a, r.b);
      if (e != hipSuccess) return hip_fail(e, "profile elapsed");
      he_kernel_stat &s = acc[r.kind & 7];
      s.launches++;
      s.total_ms += ms;
      if (ms > s.max_ms) s.max_ms = ms;
    }
  }
  uint32_t m = 0;
  for (uint32_t k = 0; k < 8; ++k)
    if (acc[k].launches) {
      if (out && m < cap) out[m] = acc[k];
      ++m;
    }
  *n = m < cap ? m : cap;
  return HE_OK;
}

he_status he_ntt_fwd(he_ctx *ctx, uint64_t *planes, uint32_t n_polys, void *stream) {
  if (!ctx || (!planes && n_polys)) return fail(HE_EINVAL, "null argument");
  const Ctx &c = *ctx->c;
  HIPCHK(timed(c, (hipStream_t)stream, KK_FWD, [&] { return launch_ntt_fwd(c, c.s_fwd, planes, planes, n_polys * c.L, (hipStream_t)stream); }), "ntt_fwd launch");
  return HE_OK;
}

he_status he_ntt_inv(he_ctx *ctx, uint64_t *planes, uint32_t n_polys, void *stream) {
  if (!ctx || (!planes && n_polys)) return fail(HE_EINVAL, "null argument");
  const Ctx &c = *ctx->c;
  HIPCHK(timed(c, (hipStream_t)stream, KK_INV, [&] { return launch_ntt_inv(c, c.s_inv, planes, planes, n_polys * c.L, (hipStream_t)stream); }), "ntt_inv launch");
  return HE_OK;
}

he_status he_cpmul_acc_ws(const he_ctx *ctx, uint32_t K, uint32_t flags, size_t *bytes) {
  if (!ctx || !bytes) return fail(HE_EINVAL, "null argument");
  const Ctx &c = *ctx->c;
  size_t b = 0;
  if (!(flags & HE_IN_NTT)) b = al256((size_t)K * 2 * c.L * c.N * 8) + al256((size_t)K * c.L * c.N * 8);
  if (flags & HE_VALIDATE) b += 256;
  *bytes = b;
  return HE_OK;
}

}  // extern "C"

namespace he {
he_status validate(const Ctx &c, const uint64_t *planes, size_t n_planes, void *flag_mem, hipStream_t st) {
  uint32_t *bad = (uint32_t *)flag_mem;
  HIPCHK(hipMemsetAsync(bad, 0, 4, st), "validate memset");
  HIPCHK(launch_check_canonical(c, planes, n_planes, bad, st), "validate launch");
  uint32_t h = 0;
  HIPCHK(hipMemcpyAsync(&h, bad, 4, hipMemcpyDeviceToHost, st), "validate copy");
  HIPCHK(hipStreamSynchronize(st), "validate sync");
  if (h) return fail(HE_ERANGE, std::to_string(h) + " coefficients outside [0, q_i)");
  return HE_OK;
}
}  // namespace he

extern "C" {

// ---------------------------------------------------------------- plaintext product
// The ring of the plaintext modulus: one prime q = t (an NTT-friendly t such
// as 65537 = 2^16 + 1 is 1 mod 2N for every N <= 2^15), built by he_ctx_prepare.
static he_status t_ring(Ctx &c, Ctx **out) {
  std::lock_guard<std::mutex> g(c.tctx_mu);
  if (!c.tctx) return fail(HE_EINVAL, "plaintext product not prepared: call he_ctx_prepare with HE_PREPARE_PPMUL");
  *out = c.tctx;
  return HE_OK;
}

static he_status t_ring_build(Ctx &c) {
  std::lock_guard<std::mutex> g(c.tctx_mu);
  if (!c.tctx) {
    const uint64_t q = c.t;
    he_params p{};
    p.N = c.N;
    p.L = 1;
    p.arith = HE_ARITH_F64;
    p.q = &q;
    p.t = 3;          // unused by the plaintext ring; any value coprime to q
    p.device = c.device;
    Ctx *tc = nullptr;
    if (build_context(&p, &tc) != HE_OK)
      return fail(HE_EUNSUPPORTED, "the plaintext product needs t prime with t = 1 mod 2N");
    c.tctx = tc;
  }
  return HE_OK;
}

he_status he_ctx_prepare(he_ctx *ctx, uint32_t ops, uint32_t ccmul_max_out, uint32_t ccmul_max_terms) {
  if (!ctx) return fail(HE_EINVAL, "null context");
  if (ops & ~(uint32_t)(HE_PREPARE_PPMUL | HE_PREPARE_CCMUL)) return fail(HE_EINVAL, "unknown HE_PREPARE_* bits");
  Ctx &c = *ctx->c;
  hipError_t e = hipSetDevice(c.device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  if (ops & HE_PREPARE_PPMUL) {
    he_status s = t_ring_build(c);
    if (s != HE_OK) return s;
  }
  if (ops & HE_PREPARE_CCMUL) return ccmul_prepare(c, ccmul_max_out, ccmul_max_terms);
  return HE_OK;
}

static size_t al256p(size_t b) { return (b + 255) & ~(size_t)255; }

he_status he_ppmul_ws_size(const he_plan *plan, uint32_t flags, size_t *bytes) {
  if (!plan || !bytes) return fail(HE_EINVAL, "null argument");
  const he_plan_info &in = plan->p.info;
  const size_t plane = (size_t)in.N * 8;
  *bytes = al256p((size_t)in.n_ct_in * plane) + al256p((size_t)in.n_pt * plane) + ((flags & HE_VALIDATE) ? 256 : 0);
  return HE_OK;
}

he_status he_ppmul(he_ctx *ctx, const he_plan *plan, const uint64_t *a, const uint64_t *b, uint64_t *out,
                   uint32_t flags, void *ws, size_t ws_bytes, void *stream) {
  if (!ctx || !plan || !out || !a || !b) return fail(HE_EINVAL, "null argument");
  if (plan->ctx != ctx->c) return fail(HE_EINVAL, "plan belongs to another context");
  if (flags & ~HE_VALIDATE) return fail(HE_EINVAL, "flags: only HE_VALIDATE applies");
  Ctx &c = *ctx->c;
  const Plan &p = plan->p;
  const he_plan_info &in = p.info;
  size_t need = 0;
  he_ppmul_ws_size(plan, flags, &need);
  if (ws_bytes < need || (need && !ws)) return fail(HE_ENOMEM, "workspace too small");
  Ctx *tc = nullptr;
  he_status rs = t_ring(c, &tc);
  if (rs != HE_OK) return rs;
  hipStream_t st = (hipStream_t)stream;
  char *w = (char *)ws;
  uint64_t *a_hat = (uint64_t *)w;
  uint64_t *b_hat = (uint64_t *)(w + al256p((size_t)in.n_ct_in * c.N * 8));
  if (flags & HE_VALIDATE) {
    he_status s = validate(*tc, a, in.n_ct_in, w + need - 256, st);
    if (s == HE_OK) s = validate(*tc, b, in.n_pt, w + need - 256, st);
    if (s != HE_OK) return s;
  }
  // the context's tuned thread counts, fp64 arithmetic (t < 2^32)
  const Sched sf{HE_ARITH_F64, c.s_fwd.loge}, sm{HE_ARITH_F64, c.s_mac.loge};
  Terms tm;
  tm.row = p.d_row();
  tm.cti = p.d_cti();
  tm.pti = p.d_pti();
  tm.n_out = in.n_ct_out;
  HIPCHK(timed(c, st, KK_FWD, [&] { return launch_ntt_fwd2(*tc, sf, a_hat, a, in.n_ct_in, b_hat, b, in.n_pt, st); }),
         "ppmul forward a, b");
  HIPCHK(timed(c, st, KK_MAC_INV, [&] { return launch_mac(*tc, sm, out, a_hat, b_hat, tm, false, false, st, 1); }),
         "ppmul multiply + inverse");
  return HE_OK;
}

he_status he_cpmul_acc(he_ctx *ctx, const uint64_t *ct, const uint64_t *pt, uint32_t K, uint64_t *acc, uint32_t flags,
                       void *ws, size_t ws_bytes, void *stream) {
  if (!ctx || !acc || (K && (!ct || !pt))) return fail(HE_EINVAL, "null argument");
  const Ctx &c = *ctx->c;
  hipStream_t st = (hipStream_t)stream;
  size_t need = 0;
  he_cpmul_acc_ws(ctx, K, flags, &need);
  if (ws_bytes < need || (need && !ws)) return fail(HE_ENOMEM, "workspace too small");
  char *w = (char *)ws;
  if (flags & HE_VALIDATE) {
    he_status s = validate(c, ct, (size_t)K * 2 * c.L, w + need - 256, st);
    if (s == HE_OK) s = validate(c, pt, (size_t)K * c.L, w + need - 256, st);
    if (s == HE_OK && (flags & HE_ACCUMULATE)) s = validate(c, acc, 2 * c.L, w + need - 256, st);
    if (s != HE_OK) return s;
  }
  const uint64_t *ct_hat = ct, *pt_hat = pt;
  if (!(flags & HE_IN_NTT)) {
    uint64_t *a = (uint64_t *)w;
    uint64_t *b = (uint64_t *)(w + al256((size_t)K * 2 * c.L * c.N * 8));
    HIPCHK(timed(c, st, KK_FWD, [&] { return launch_ntt_fwd2(c, c.s_fwd, a, ct, K * 2 * c.L, b, pt, K * c.L, st); }),
           "cpmul fwd ct, pt");
    ct_hat = a;
    pt_hat = b;
  }
  Terms tm;
  tm.n_out = 1;
  tm.K = K;
  HIPCHK(timed(c, st, (flags & HE_OUT_NTT) ? KK_MAC : KK_MAC_INV, [&] { return launch_mac(c, c.s_mac, acc, ct_hat, pt_hat, tm, (flags & HE_ACCUMULATE) != 0, (flags & HE_OUT_NTT) != 0, st); }),
         "cpmul mac");
  return HE_OK;
}

he_status he_plan_create(const he_ctx *ctx, const he_conv_shape *shape, he_plan **out) {
  if (!ctx || !shape || !out) return fail(HE_EINVAL, "null argument");
  *out = nullptr;
  he_plan *p = new he_plan{ctx->c, Plan{}};
  he_status s = make_plan(*ctx->c, *shape, p->p);
  if (s != HE_OK) {
    delete p;
    return s;
  }
  p->p.device = ctx->c->device;
  const size_t n = p->p.row.size() + 2 * p->p.cti.size();
  std::vector<int32_t> all;
  all.reserve(n);
  all.insert(all.end(), p->p.row.begin(), p->p.row.end());
  all.insert(all.end(), p->p.cti.begin(), p->p.cti.end());
  all.insert(all.end(), p->p.pti.begin(), p->p.pti.end());
  hipError_t e = hipSetDevice(p->p.device);
  if (e == hipSuccess) e = hipMalloc(&p->p.d_terms, n * 4);
  if (e == hipSuccess) e = hipMemcpy(p->p.d_terms, all.data(), n * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (p->p.d_terms) (void)hipFree(p->p.d_terms);
    delete p;
    return hip_fail(e, "plan term lists");
  }
  *out = p;
  return HE_OK;
}

he_status he_plan_query(uint32_t N, const he_conv_shape *shape, he_plan_info *info) {
  if (!shape || !info) return fail(HE_EINVAL, "null argument");
  if (N < 16 || N > 32768 || (N & (N - 1))) return fail(HE_EINVAL, "N must be a power of two in [16, 2^15]");
  Ctx c;
  c.N = N;
  Plan p;
  he_status s = make_plan(c, *shape, p);
  if (s == HE_OK) *info = p.info;
  return s;
}

he_status he_plan_destroy(he_plan *plan) {
  if (!plan) return HE_OK;
  if (plan->p.d_terms) (void)hipFree(plan->p.d_terms);
  delete plan;
  return HE_OK;
}

he_status he_plan_get_info(const he_plan *plan, he_plan_info *info) {
  if (!plan || !info) return fail(HE_EINVAL, "null argument");
  *info = plan->p.info;
  return HE_OK;
}

he_status he_plan_terms(const he_plan *plan, int32_t *row, int32_t *ct_idx, int32_t *pt_idx) {
  if (!plan) return fail(HE_EINVAL, "null argument");
  if (row) std::memcpy(row, plan->p.row.data(), plan->p.row.size() * 4);
  if (ct_idx) std::memcpy(ct_idx, plan->p.cti.data(), plan->p.cti.size() * 4);
  if (pt_idx) std::memcpy(pt_idx, plan->p.pti.data(), plan->p.pti.size() * 4);
  return HE_OK;
}

struct WsLayout {
  size_t ct_hat = 0, pt_poly = 0, pt_hat = 0, acc = 0, flag = 0, total = 0;
};

// Host setup of one layer call (no device work): the workspace layout, where
// raw weights are packed, and the planes each stage covers.  he_corr_conv2d
// (and its seeded and allocation-free forms) runs exactly this before its first
// launch; he_layer_query reports it for a host plan.
struct LayerSetup {
  WsLayout ws;
  uint32_t pack = HE_PACK_NONE;
  WPack wp{};
  uint32_t fwd_ct = 0, fwd_pt = 0, mac = 0, inv = 0;
};

static he_status layer_setup(uint32_t N, uint32_t L, const Plan &p, uint32_t flags, LayerSetup &ls) {
  const he_plan_info &in = p.info;
  ls = LayerSetup{};
  if (!L) return fail(HE_EINVAL, "no primes");
  if (in.kind == HE_KIND_DW && !(flags & HE_PLAIN_POLY))
    return fail(HE_EUNSUPPORTED, "weight-gradient plaintexts are passed as packed polynomials (HE_PLAIN_POLY)");
  ls.pack = (flags & HE_PLAIN_POLY) ? HE_PACK_NONE : ((flags & HE_UNFUSED) ? HE_PACK_MEMORY : HE_PACK_FUSED);
  if (ls.pack != HE_PACK_NONE) {
    he_status s = weight_pack(p, ls.wp);
    if (s != HE_OK) return s;
  }
  WsLayout &w = ls.ws;
  size_t off = 0;
  const size_t plane = (size_t)L * N * 8;
  if (!(flags & HE_IN_NTT)) {
    w.ct_hat = off;
    off += al256((size_t)in.n_ct_in * 2 * plane);
  }
  if (ls.pack == HE_PACK_MEMORY) {
    w.pt_poly = off;
    off += al256((size_t)in.n_pt * N * 8);
  }
  w.pt_hat = off;
  off += al256((size_t)in.n_pt * plane);
  if ((flags & HE_UNFUSED) && !(flags & HE_OUT_NTT)) {
    w.acc = off;
    off += al256((size_t)in.n_ct_out * 2 * plane);
  }
  if (flags & HE_VALIDATE) {
    w.flag = off;
    off += 256;
  }
  w.total = off;
  ls.fwd_ct = (flags & HE_IN_NTT) ? 0u : in.n_ct_in * 2 * L;
  ls.fwd_pt = in.n_pt * L;
  ls.mac = in.n_ct_out * 2 * L;
  ls.inv = (flags & HE_OUT_NTT) ? 0u : in.n_ct_out * 2 * L;
  return HE_OK;
}

he_status he_workspace_size(const he_plan *plan, uint32_t flags, size_t *bytes) {
  if (!plan || !bytes) return fail(HE_EINVAL, "null argument");
  if (!plan->ctx) return fail(HE_EINVAL, "a host plan has no context: he_layer_query takes the prime count");
  LayerSetup ls;
  he_status s = layer_setup(plan->ctx->N, plan->ctx->L, plan->p, flags, ls);
  if (s != HE_OK) return s;
  *bytes = ls.ws.total;
  return HE_OK;
}

he_status he_plan_create_host(uint32_t N, const he_conv_shape *shape, he_plan **out) {
  if (!shape || !out) return fail(HE_EINVAL, "null argument");
  *out = nullptr;
  if (N < 16 || N > 32768 || (N & (N - 1))) return fail(HE_EINVAL, "N must be a power of two in [16, 2^15]");
  Ctx c;
  c.N = N;
  he_plan *p = new he_plan{nullptr, Plan{}};
  he_status s = make_plan(c, *shape, p->p);
  if (s != HE_OK) {
    delete p;
    return s;
  }
  p->p.device = -1;
  *out = p;
  return HE_OK;
}

he_status he_layer_query(const he_plan *plan, uint32_t L, uint32_t flags, he_layer_info *info) {
  if (!plan || !info) return fail(HE_EINVAL, "null argument");
  if (plan->ctx && L && L != plan->ctx->L) return fail(HE_EINVAL, "prime count differs from the plan's context");
  if (plan->ctx) L = plan->ctx->L;
  LayerSetup ls;
  he_status s = layer_setup(plan->p.info.N, L, plan->p, flags, ls);
  if (s != HE_OK) return s;
  const uint64_t none = ~0ull;
  const bool ct = !(flags & HE_IN_NTT), acc = (flags & HE_UNFUSED) && !(flags & HE_OUT_NTT);
  *info = he_layer_info{ls.ws.total,
                        ct ? ls.ws.ct_hat : none,
                        ls.pack == HE_PACK_MEMORY ? ls.ws.pt_poly : none,
                        ls.ws.pt_hat,
                        acc ? ls.ws.acc : none,
                        (flags & HE_VALIDATE) ? ls.ws.flag : none,
                        ls.fwd_ct, ls.fwd_pt, ls.mac, ls.inv, ls.pack, 0u};
  return HE_OK;
}

}  // extern "C"

namespace he {
size_t layer_ws_bytes(const Ctx &c, const Plan &p, uint32_t flags) {
  LayerSetup ls;
  return layer_setup(c.N, c.L, p, flags, ls) == HE_OK ? ls.ws.total : 0;
}
he_status run_layer(const Ctx &c, const Plan &p, const uint64_t *ct_in, const void *plain, uint64_t *ct_out,
                    uint32_t flags, void *ws, size_t ws_bytes, hipStream_t st, const uint64_t *seed = nullptr);
}  // namespace he

extern "C" {

he_status he_corr_conv2d(he_ctx *ctx, const he_plan *plan, const uint64_t *ct_in, const void *plain, uint64_t *ct_out,
                         uint32_t flags, void *ws, size_t ws_bytes, void *stream) {
  if (!ctx || !plan || !ct_in || !plain || !ct_out) return fail(HE_EINVAL, "null argument");
  if (plan->ctx != ctx->c) return fail(HE_EINVAL, "plan belongs to another context");
  return run_layer(*ctx->c, plan->p, ct_in, plain, ct_out, flags, ws, ws_bytes, (hipStream_t)stream);
}

he_status he_corr_conv2d_seeded(he_ctx *ctx, const he_plan *plan, const uint64_t *ct0, const uint64_t *seed,
                                const void *plain, uint64_t *ct_out, uint32_t flags, void *ws, size_t ws_bytes,
                                void *stream) {
  if (!ctx || !plan || !ct0 || !seed || !plain || !ct_out) return fail(HE_EINVAL, "null argument");
  if (plan->ctx != ctx->c) return fail(HE_EINVAL, "plan belongs to another context");
  if (flags & HE_IN_NTT) return fail(HE_EINVAL, "a seeded component is regenerated in coefficient form (no HE_IN_NTT)");
  return run_layer(*ctx->c, plan->p, ct0, plain, ct_out, flags, ws, ws_bytes, (hipStream_t)stream, seed);
}

he_status he_expand_c1(he_ctx *ctx, const uint64_t *seed, uint32_t first_ct, uint32_t n_ct, uint64_t *out,
                       void *stream) {
  if (!ctx || !seed || (n_ct && !out)) return fail(HE_EINVAL, "null argument");
  HIPCHK(launch_expand_c1(*ctx->c, out, seed[0], seed[1], first_ct, n_ct, (hipStream_t)stream), "expand c1");
  return HE_OK;
}

}  // extern "C"

he_status he::run_layer(const Ctx &c, const Plan &p, const uint64_t *ct_in, const void *plain, uint64_t *ct_out,
                        uint32_t flags, void *ws, size_t ws_bytes, hipStream_t st, const uint64_t *seed) {
  const he_plan_info &in = p.info;
  LayerSetup ls;
  he_status s0 = layer_setup(c.N, c.L, p, flags, ls);
  if (s0 != HE_OK) return s0;
  const WsLayout &L = ls.ws;
  if (ws_bytes < L.total || (L.total && !ws)) return fail(HE_ENOMEM, "workspace too small");
  char *w = (char *)ws;
  if (flags & HE_VALIDATE) {
    // with a seed, ct_in holds component 0 only
    he_status s = validate(c, ct_in, (size_t)in.n_ct_in * (seed ? 1 : 2) * c.L, w + L.flag, st);
    if (s != HE_OK) return s;
  }
  // weights packed in LDS inside the plaintext transform (fused path), or
  // packed to memory first (unfused baseline), or polynomials given
  uint64_t *pt_hat = (uint64_t *)(w + L.pt_hat);
  const bool pack_fused = ls.pack == HE_PACK_FUSED;
  const WPack &wp = ls.wp;
  // 1. transform the input ciphertexts (2. and the packed plaintexts, in the
  // same launch when both are transformed here)
  const uint64_t *ct_hat = ct_in;
  bool pt_done = false;
  if (seed) {
    uint64_t *d = (uint64_t *)(w + L.ct_hat);
    if (pack_fused) {
      HIPCHK(timed(c, st, KK_FWD, [&] {
               return launch_ntt_fwd_ct_pack(c, c.s_fwd, d, ct_in, in.n_ct_in * 2 * c.L, pt_hat, (const int32_t *)plain,
                                             wp, in.n_pt, st, seed);
             }),
             "conv fwd ct (seeded) + pack fwd pt");
      pt_done = true;
    } else {
      HIPCHK(timed(c, st, KK_FWD,
                   [&] { return launch_ntt_fwd_seeded(c, c.s_fwd, d, ct_in, seed[0], seed[1], in.n_ct_in, st); }),
             "conv fwd ct (seeded)");
    }
    ct_hat = d;
  } else if (!(flags & HE_IN_NTT)) {
    uint64_t *d = (uint64_t *)(w + L.ct_hat);
    if (pack_fused) {
      HIPCHK(timed(c, st, KK_FWD, [&] {
               return launch_ntt_fwd_ct_pack(c, c.s_fwd, d, ct_in, in.n_ct_in * 2 * c.L, pt_hat, (const int32_t *)plain,
                                             wp, in.n_pt, st);
             }),
             "conv fwd ct + pack fwd pt");
      pt_done = true;
    } else {
      HIPCHK(timed(c, st, KK_FWD, [&] { return launch_ntt_fwd(c, c.s_fwd, d, ct_in, in.n_ct_in * 2 * c.L, st); }),
             "conv fwd ct");
    }
    ct_hat = d;
  }
  // 2. pack (raw weights) and transform the plaintexts
  if (pack_fused && !pt_done)
    HIPCHK(timed(c, st, KK_FWD_LIFT,
                 [&] { return launch_ntt_fwd_pack(c, c.s_fwd, pt_hat, (const int32_t *)plain, wp, in.n_pt, st); }),
           "conv pack + fwd pt");
  const int64_t *polys = (const int64_t *)plain;
  if (ls.pack == HE_PACK_MEMORY) {
    int64_t *pp = (int64_t *)(w + L.pt_poly);
    HIPCHK(timed(c, st, KK_PACK, [&] {
             hipError_t e = launch_zero_i64(pp, (size_t)in.n_pt * c.N, st);
             if (e != hipSuccess) return e;
             if (wp.kind != WP_FC)
               return launch_pack_conv_w(pp, (const int32_t *)plain, wp.M, wp.C, wp.h, wp.O, wp.S, wp.Cw, wp.cb, c.N,
                                         wp.kind == WP_CONV_DX, st);
             return launch_pack_fc_w(pp, (const int32_t *)plain, wp.n_out, wp.n_in, wp.n_iw, wp.n_ow, wp.in_ct, c.N,
                                     st);
           }),
           "pack");
    polys = pp;
  }
  if (!pack_fused)
    HIPCHK(timed(c, st, KK_FWD_LIFT, [&] { return launch_ntt_fwd_lift(c, c.s_fwd, pt_hat, polys, in.n_pt, st); }),
           "conv fwd pt");
  // 3. multiply-accumulate + inverse transform
  Terms tm;
  tm.row = p.d_row();
  tm.cti = p.d_cti();
  tm.pti = p.d_pti();
  tm.n_out = in.n_ct_out;
  const bool accum = (flags & HE_ACCUMULATE) != 0;
  if (flags & HE_OUT_NTT) {
    HIPCHK(timed(c, st, KK_MAC, [&] { return launch_mac(c, c.s_mac, ct_out, ct_hat, pt_hat, tm, accum, true, st); }), "conv mac");
  } else if (flags & HE_UNFUSED) {
    uint64_t *acc = (uint64_t *)(w + L.acc);
    HIPCHK(timed(c, st, KK_MAC, [&] { return launch_mac(c, c.s_mac, acc, ct_hat, pt_hat, tm, false, true, st); }), "conv mac");
    if (accum) {
      HIPCHK(timed(c, st, KK_INV, [&] { return launch_ntt_inv(c, c.s_inv, acc, acc, in.n_ct_out * 2 * c.L, st); }), "conv inv");
      HIPCHK(launch_add_planes(c, ct_out, ct_out, acc, in.n_ct_out * 2 * c.L, st), "conv add");
    } else {
      HIPCHK(timed(c, st, KK_INV, [&] { return launch_ntt_inv(c, c.s_inv, ct_out, acc, in.n_ct_out * 2 * c.L, st); }), "conv inv");
    }
  } else {
    HIPCHK(timed(c, st, KK_MAC_INV, [&] { return launch_mac(c, c.s_mac, ct_out, ct_hat, pt_hat, tm, accum, false, st); }), "conv mac+inv");
  }
  return HE_OK;
}

extern "C" {

he_status he_pack_input(const he_plan *plan, const int32_t *x, int64_t *polys) {
  if (!plan || !x || !polys) return fail(HE_EINVAL, "null argument");
  const Plan &p = plan->p;
  const he_plan_info &in = p.info;
  const he_conv_shape &s = p.eq;   // DX: dY packed as the input of the equivalent conv
  const uint32_t N = in.N;
  if (s.kind == HE_KIND_FC) {
    const uint32_t ict = (s.n_in + in.n_iw - 1) / in.n_iw;
    std::memset(polys, 0, sizeof(int64_t) * (size_t)s.B * ict * N);
    for (uint32_t b = 0; b < s.B; ++b)
      for (uint32_t j = 0; j < s.n_in; ++j)
        polys[((size_t)b * ict + j / in.n_iw) * N + j % in.n_iw] = x[(size_t)b * s.n_in + j];
    return HE_OK;
  }
  // CONV, DX and DW inputs: per (image, window) cb polynomials; a window covers
  // rows r*Hw.. and columns s*Ww.. of the map (the whole map when unsplit)
  const uint32_t T = in.tiles ? in.tiles : 1, tw = (s.W + in.Ww - 1) / in.Ww;
  std::memset(polys, 0, sizeof(int64_t) * (size_t)s.B * T * in.cb * N);
  for (uint32_t b = 0; b < s.B; ++b)
    for (uint32_t t = 0; t < T; ++t) {
      const uint32_t r0 = (t / tw) * in.Hw, c0 = (t % tw) * in.Ww;
      for (uint32_t c = 0; c < s.C; ++c) {
        int64_t *poly = polys + (((size_t)b * T + t) * in.cb + c / in.Cw) * N + (size_t)(c % in.Cw) * in.S;
        for (uint32_t i = 0; i < in.Hw && r0 + i < s.H; ++i)
          for (uint32_t j = 0; j < in.Ww && c0 + j < s.W; ++j)
            poly[i * in.O + j] = x[(((size_t)b * s.C + c) * s.H + r0 + i) * s.W + c0 + j];
      }
    }
  return HE_OK;
}

he_status he_extract_output(const he_plan *plan, const int64_t *polys, int64_t *y) {
  if (!plan || !polys || !y) return fail(HE_EINVAL, "null argument");
  const Plan &p = plan->p;
  const he_plan_info &in = p.info;
  const he_conv_shape &s = p.eq;   // DX: dX is the output of the equivalent conv
  const uint32_t N = in.N;
  if (s.kind == HE_KIND_FC) {
    const uint32_t oct = (s.n_out + in.n_ow - 1) / in.n_ow;
    for (uint32_t b = 0; b < s.B; ++b)
      for (uint32_t i = 0; i < s.n_out; ++i)
        y[(size_t)b * s.n_out + i] = polys[((size_t)b * oct + i / in.n_ow) * N + (i % in.n_ow) * in.n_iw + in.n_iw - 1];
    return HE_OK;
  }
  if (s.kind == HE_KIND_CONV) {
    const uint32_t T = in.tiles ? in.tiles : 1, tw = (s.W + in.Ww - 1) / in.Ww, th = T / tw, h = s.h;
    const uint32_t sd = s.stride > 1 ? s.stride : 1;   // a stride subsamples the full correlation
    if (T == 1) {
      for (uint32_t b = 0; b < s.B; ++b)
        for (uint32_t m = 0; m < s.M; ++m) {
          const int64_t *poly = polys + ((size_t)b * s.M + m) * N;
          for (uint32_t yy = 0; yy < in.Hout; ++yy)
            for (uint32_t zz = 0; zz < in.Wout; ++zz)
              y[(((size_t)b * s.M + m) * in.Hout + yy) * in.Wout + zz] =
                  poly[(yy * sd + h - 1 - s.P) * in.O + (zz * sd + h - 1 - s.P)];
        }
      return HE_OK;
    }
    // windows: overlap-add each tile's full correlation at (r*Hw, s*Ww), then crop
    const uint32_t FH = th * in.Hw + h - 1, FW = tw * in.Ww + h - 1;
    std::vector<int64_t> F((size_t)FH * FW);
    for (uint32_t b = 0; b < s.B; ++b)
      for (uint32_t m = 0; m < s.M; ++m) {
        std::fill(F.begin(), F.end(), 0);
        for (uint32_t t = 0; t < T; ++t) {
          const int64_t *poly = polys + (((size_t)b * T + t) * s.M + m) * N;
          const uint32_t r0 = (t / tw) * in.Hw, c0 = (t % tw) * in.Ww;
          for (uint32_t u = 0; u < in.Hw + h - 1; ++u)
            for (uint32_t v = 0; v < in.Ww + h - 1; ++v) F[(size_t)(r0 + u) * FW + c0 + v] += poly[u * in.O + v];
        }
        for (uint32_t yy = 0; yy < in.Hout; ++yy)
          for (uint32_t zz = 0; zz < in.Wout; ++zz)
            y[(((size_t)b * s.M + m) * in.Hout + yy) * in.Wout + zz] =
                F[(size_t)(yy * sd + h - 1 - s.P) * FW + (zz * sd + h - 1 - s.P)];
      }
    return HE_OK;
  }
  // DW: out [M][cb][N] -> dW [M][C][h][h]
  const uint32_t h = s.h, hk = p.hk;
  for (uint32_t m = 0; m < s.M; ++m)
    for (uint32_t c = 0; c < s.C; ++c) {
      const int64_t *poly = polys + ((size_t)m * in.cb + c / in.Cw) * N + (size_t)(c % in.Cw) * in.S;
      for (uint32_t a = 0; a < h; ++a)
        for (uint32_t bb = 0; bb < h; ++bb)
          y[(((size_t)m * s.C + c) * h + a) * h + bb] = poly[(a + hk - 1 - s.P) * in.O + (bb + hk - 1 - s.P)];
    }
  return HE_OK;
}

// ------------------------------------------------------------------ encryption
he_status he_encrypt(he_ctx *ctx, const int8_t *s, const int64_t *m, const uint64_t *a, const int32_t *e, uint64_t *ct,
                     void *stream) {
  if (!ctx || !s || !m || !a || !e || !ct) return fail(HE_EINVAL, "null argument");
  const Ctx &c = *ctx->c;
  hipStream_t st = (hipStream_t)stream;
  const size_t pb = (size_t)c.L * c.N * 8;
  uint64_t *tmp = nullptr;
  HIPCHK(hipMalloc(&tmp, 3 * pb + 256), "encrypt scratch");
  uint64_t *s_hat = tmp, *a_hat = tmp + (size_t)c.L * c.N, *prod = tmp + 2 * (size_t)c.L * c.N;
  uint64_t *dw = tmp + 3 * (size_t)c.L * c.N;
  std::vector<uint64_t> delta_w(2 * c.L);
  for (uint32_t i = 0; i < c.L; ++i) {
    delta_w[i] = c.delta_mod[i];
    delta_w[c.L + i] = (uint64_t)(((unsigned __int128)c.delta_mod[i] << 64) / c.q[i]);
  }
  hipError_t err = hipMemcpyAsync(dw, delta_w.data(), 16 * c.L, hipMemcpyHostToDevice, st);
  if (err == hipSuccess) err = launch_lift<int8_t>(c, s_hat, s, st);
  if (err == hipSuccess) err = launch_ntt_fwd(c, c.s_fwd, s_hat, s_hat, c.L, st);
  if (err == hipSuccess) err = launch_ntt_fwd(c, c.s_fwd, a_hat, a, c.L, st);
  if (err == hipSuccess) err = launch_pmul_bcast(c, prod, a_hat, s_hat, c.L, st);
  if (err == hipSuccess) err = launch_ntt_inv(c, c.s_inv, prod, prod, c.L, st);
  if (err == hipSuccess) err = launch_enc_combine(c, ct, prod, e, m, dw, st);
  if (err == hipSuccess) err = launch_copy_u64(ct + (size_t)c.L * c.N, a, (size_t)c.L * c.N, st);
  hipError_t e2 = hipStreamSynchronize(st);
  (void)hipFree(tmp);
  if (err != hipSuccess) return hip_fail(err, "encrypt");
  if (e2 != hipSuccess) return hip_fail(e2, "encrypt sync");
  return HE_OK;
}

he_status he_decrypt(he_ctx *ctx, const int8_t *s, const uint64_t *ct, uint32_t n_ct, int64_t *m, void *stream) {
  if (!ctx || !s || !ct || !m) return fail(HE_EINVAL, "null argument");
  if (n_ct == 0) return HE_OK;
  const Ctx &c = *ctx->c;
  hipStream_t st = (hipStream_t)stream;
  const size_t pl = (size_t)c.L * c.N;
  uint64_t *tmp = nullptr;
  HIPCHK(hipMalloc(&tmp, (1 + (size_t)n_ct) * pl * 8), "decrypt scratch");
  uint64_t *s_hat = tmp, *x = tmp + pl;
  hipError_t err = launch_lift<int8_t>(c, s_hat, s, st);
  if (err == hipSuccess) err = launch_ntt_fwd(c, c.s_fwd, s_hat, s_hat, c.L, st);
  for (uint32_t k = 0; k < n_ct && err == hipSuccess; ++k) {
    const uint64_t *c0 = ct + (size_t)k * 2 * pl, *c1 = c0 + pl;
    uint64_t *xk = x + (size_t)k * pl;
    err = launch_ntt_fwd(c, c.s_fwd, xk, c1, c.L, st);
    if (err == hipSuccess) err = launch_pmul_bcast(c, xk, xk, s_hat, c.L, st);
    if (err == hipSuccess) err = launch_ntt_inv(c, c.s_inv, xk, xk, c.L, st);
    if (err == hipSuccess) err = launch_add_planes(c, xk, xk, c0, c.L, st);
  }
  std::vector<uint64_t> hx((size_t)n_ct * pl);
  if (err == hipSuccess) err = hipMemcpyAsync(hx.data(), x, hx.size() * 8, hipMemcpyDeviceToHost, st);
  hipError_t e2 = hipStreamSynchronize(st);
  (void)hipFree(tmp);
  if (err != hipSuccess) return hip_fail(err, "decrypt");
  if (e2 != hipSuccess) return hip_fail(e2, "decrypt sync");
  return client_decrypt_crt(c, hx.data(), n_ct, m);
}

}  // extern "C"
