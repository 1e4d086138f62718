// Batch runtime: task-table planning, workspace, graph capture and replay for
// the persistent fused kernel.
#include <algorithm>

#include "batch.hpp"
#include "plan.hpp"


struct he_batch {
  int device = 0;
  std::vector<he::JobRef> jobs;
  bool built = false;
  int arith = HE_ARITH_F64;
  void *d_ws = nullptr;
  size_t ws_bytes = 0;
  he::PTask *d_tasks = nullptr;
  he::PJob *d_jobs = nullptr;
  uint32_t *d_ctl = nullptr;
  uint32_t n_tasks = 0, ctl_words = 0, grid = 0;
  he::PVariant var{};
  he::XQ xq{};
  uint32_t strict = 0;
  std::vector<he::PJob> h_jobs;
  std::vector<char *> ws_ptrs;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  he_batch_info info{};
  uint32_t spin_limit = he::kSpinLimit;
  // HE_BATCH_PROFILE: a ring of event pairs, read back at sync
  static constexpr uint32_t kProfRing = 64;
  std::vector<hipEvent_t> ev;          // 2 * kProfRing when profiling
  uint32_t ev_next = 0, ev_pending = 0;
};

using namespace he;


static void release(he_batch *b) {
  for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
  b->ev.clear();
  b->ev_next = b->ev_pending = 0;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (void *p : {b->d_ws, (void *)b->d_tasks, (void *)b->d_jobs, (void *)b->d_ctl})
    if (p) (void)hipFree(p);
  b->exec = nullptr;
  b->graph = nullptr;
  b->cap = nullptr;
  b->d_ws = nullptr;
  b->d_tasks = nullptr;
  b->d_jobs = nullptr;
  b->d_ctl = nullptr;
  b->built = false;
}

namespace he {

static inline size_t al256b(size_t b) { return (b + 255) & ~(size_t)255; }

// bytes of the transformed inputs of a job (none when already transformed)
static size_t ct_hat_bytes(const JobRef &j) {
  const size_t plane = (size_t)j.ctx->L * j.ctx->N * 8;
  return (j.job.flags & HE_IN_NTT) ? 0 : al256b((size_t)j.plan->info.n_ct_in * 2 * plane);
}

size_t job_ws_bytes(const JobRef &j) {
  const size_t plane = (size_t)j.ctx->L * j.ctx->N * 8;
  return ct_hat_bytes(j) + al256b((size_t)j.plan->info.n_pt * plane);
}

static he_status fill_job(const JobRef &bj, char *ws, int arith, PJob &pj) {
  const Ctx &c = *bj.ctx;
  const Plan &p = *bj.plan;
  const he_plan_info &in = p.info;
  const uint32_t f = bj.job.flags;
  const size_t plane = (size_t)c.L * c.N * 8;
  pj = PJob{};
  pj.primes = c.d_primes;
  pj.tw_fwd = arith == HE_ARITH_F64 ? c.d_tw_f64_fwd : c.d_tw_u64_fwd;
  pj.tw_inv = arith == HE_ARITH_F64 ? c.d_tw_f64_inv : c.d_tw_u64_inv;
  pj.tw_inv_w = arith == HE_ARITH_F64 ? c.d_tw_f64_inv_w : nullptr;
  pj.ct_in = bj.job.ct_in;
  pj.ct_hat = (f & HE_IN_NTT) ? const_cast<uint64_t *>(bj.job.ct_in) : (uint64_t *)ws;
  pj.pt_hat = (uint64_t *)(ws + ct_hat_bytes(bj));
  pj.ct_f64 = (arith == HE_ARITH_F64 && !(f & HE_IN_NTT) && !bj.canon_ct) ? 1u : 0u;
  pj.plain = bj.job.plain;
  pj.ct_out = bj.job.ct_out;
  pj.row = p.d_row();
  pj.cti = p.d_cti();
  pj.pti = p.d_pti();
  pj.logN = c.logN;
  pj.L = c.L;
  pj.accumulate = (f & HE_ACCUMULATE) ? 1u : 0u;
  pj.pkind = (f & HE_PLAIN_POLY) ? PK_POLY
                                 : (in.kind == HE_KIND_FC ? PK_FC : (in.kind == HE_KIND_DX ? PK_CONV_DX : PK_CONV));
  if (in.kind == HE_KIND_DW && pj.pkind != PK_POLY) return fail(HE_EUNSUPPORTED, "weight-gradient jobs need HE_PLAIN_POLY");
  if (pj.pkind != PK_POLY) {
    // the layout the in-LDS scatter follows, its positions checked on the host
    WPack wp;
    he_status s = weight_pack(p, wp);
    if (s != HE_OK) return s;
    pj.M = wp.M;
    pj.C = wp.C;
    pj.h = wp.h;
    pj.O = wp.O;
    pj.S = wp.S;
    pj.Cw = wp.Cw;
    pj.cb = wp.cb;
    pj.n_in = wp.n_in;
    pj.n_out = wp.n_out;
    pj.n_iw = wp.n_iw;
    pj.n_ow = wp.n_ow;
    pj.in_ct = wp.in_ct;
  }
  return HE_OK;
}

he_status build_tables(const std::vector<JobRef> &jobs, const std::vector<char *> &ws, int arith, int slab,
                       std::vector<PTask> &tasks, std::vector<PJob> &pjobs, he_batch_info &info,
                       uint32_t xq[kXcds + 1]) {
  const size_t nj = jobs.size();
  const uint32_t slab_n = 1u << slab;
  tasks.clear();
  pjobs.assign(nj, PJob{});
  info = he_batch_info{};
  std::vector<std::vector<PTask>> pre(nj);
  std::vector<uint32_t> n_dep_job(nj, 0);
  for (size_t j = 0; j < nj; ++j) {
    he_status s = fill_job(jobs[j], ws[j], arith, pjobs[j]);
    if (s != HE_OK) return s;
    const JobRef &bj = jobs[j];
    const he_plan_info &in = bj.plan->info;
    if ((uint32_t)bj.ctx->logN > (uint32_t)slab) return fail(HE_EUNSUPPORTED, "ring degree above the kernel slab");
    const uint32_t G = slab_n >> bj.ctx->logN, L = bj.ctx->L;
    if (!(bj.job.flags & HE_IN_NTT)) {
      const uint32_t planes = in.n_ct_in * 2 * L;
      for (uint32_t p = 0; p < planes; p += G)
        pre[j].push_back(PTask{PT_FWD_CT, (uint32_t)j, p, std::min(G, planes - p), 0, -1, 0, 0});
      info.fwd_planes += planes;
    }
    const uint32_t pplanes = in.n_pt * L;
    for (uint32_t p = 0; p < pplanes; p += G)
      pre[j].push_back(PTask{PT_PT, (uint32_t)j, p, std::min(G, pplanes - p), 0, -1, 0, 0});
    info.fwd_planes += pplanes;
    pjobs[j].n_pre = (uint32_t)pre[j].size();
    info.cpmul += in.n_terms;
    const uint32_t oplanes = in.n_ct_out * 2 * L;
    n_dep_job[j] = G == 1 ? oplanes : (oplanes + G - 1) / G;
  }
  // Pre tasks go first, ordered by how soon an XCD's queue of dependent tasks
  // (below: the job-ordered dependent tasks cut into kXcds contiguous runs)
  // reaches the job: each queue's first jobs get their inputs transformed
  // first, so no XCD starts by waiting for a job whose transforms come last.
  {
    uint64_t n_dep_all = 0;
    for (uint32_t d : n_dep_job) n_dep_all += d;
    std::vector<std::pair<uint64_t, size_t>> order;
    uint64_t s = 0;
    for (size_t j = 0; j < nj; ++j) {
      const uint64_t e = s + n_dep_job[j];
      uint64_t soon = UINT64_MAX;
      for (int x = 0; x < kXcds; ++x) {
        const uint64_t a = n_dep_all * x / kXcds, b = n_dep_all * (x + 1) / kXcds;
        if (s < b && e > a) soon = std::min(soon, std::max(s, a) - a);
      }
      order.emplace_back(soon, j);
      s = e;
    }
    std::stable_sort(order.begin(), order.end(),
                     [](const auto &u, const auto &v) { return u.first < v.first; });
    for (const auto &oj : order) tasks.insert(tasks.end(), pre[oj.second].begin(), pre[oj.second].end());
  }
  const uint32_t n_pre = (uint32_t)tasks.size();
  for (size_t j = 0; j < nj; ++j) {
    const JobRef &bj = jobs[j];
    const uint32_t G = slab_n >> bj.ctx->logN, L = bj.ctx->L;
    const uint32_t planes = bj.plan->info.n_ct_out * 2 * L;
    const uint32_t kind = PT_MAC_INV | (pjobs[j].n_pre ? PT_WAIT : 0u);
    if (G == 1) {
      // one plane per task: prime-major order (plane (o * 2 + comp) * L + i
      // for i, then o, then comp), so that the operands and twiddles an XCD
      // works on at a time are those of one prime and stay in its L2
      const Plan &pl = *bj.plan;
      for (uint32_t i = 0; i < L; ++i)
        for (uint32_t oc = 0; oc < planes / L; ++oc) {
          const uint32_t o = oc / 2, comp = oc % 2;
          const int32_t t0 = pl.row[o], t1 = pl.row[o + 1];
          const uint32_t a0 = t1 > t0 ? ((uint32_t)pl.cti[t0] * 2 + comp) * L + i : 0u;
          const uint32_t b0 = t1 > t0 ? (uint32_t)pl.pti[t0] * L + i : 0u;
          tasks.push_back(PTask{kind, (uint32_t)j, oc * L + i, 1u, t0, t1, a0, b0});
        }
    } else {
      for (uint32_t p = 0; p < planes; p += G)
        tasks.push_back(PTask{kind, (uint32_t)j, p, std::min(G, planes - p), 0, -1, 0, 0});
    }
    info.inv_planes += planes;
  }
  // dependent tasks, in output order, cut into kXcds contiguous queues: outputs
  // that share inputs land on one XCD and share its L2
  const uint32_t n_dep = (uint32_t)tasks.size() - n_pre;
  for (int x = 0; x <= kXcds; ++x) xq[x] = n_pre + (uint32_t)(((uint64_t)n_dep * x) / kXcds);
  info.n_jobs = (uint32_t)nj;
  info.n_tasks = (uint32_t)tasks.size();
  info.arith = (uint32_t)arith;
  return HE_OK;
}

}  // namespace he

extern "C" {

he_status he_batch_create(int32_t device, he_batch **out) {
  if (!out) return fail(HE_EINVAL, "null output");
  *out = new he_batch();
  (*out)->device = device;
  return HE_OK;
}

he_status he_batch_add(he_batch *b, he_ctx *ctx, const he_job *job, uint32_t *index) {
  if (!b || !ctx || !job || !job->plan) return fail(HE_EINVAL, "null argument");
  if (b->built) return fail(HE_EINVAL, "batch already built");
  if (job->plan->ctx != ctx->c) return fail(HE_EINVAL, "plan belongs to another context");
  if (!job->ct_in || !job->plain || !job->ct_out) return fail(HE_EINVAL, "null job buffer");
  if (ctx->c->device != b->device) return fail(HE_EINVAL, "context on another device");
  if (ctx->c->logN < 10 || ctx->c->logN > 14) return fail(HE_EUNSUPPORTED, "ring degree");
  b->jobs.push_back(JobRef{ctx->c, &job->plan->p, *job});
  if (index) *index = (uint32_t)(b->jobs.size() - 1);
  return HE_OK;
}

he_status he_batch_build(he_batch *b, uint32_t flags) {
  if (!b) return fail(HE_EINVAL, "null batch");
  release(b);
  hipError_t e = hipSetDevice(b->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  b->strict = (flags & HE_BATCH_STRICT_SYNC) ? 1u : 0u;
  bool all_f64 = true;
  uint32_t max_logn = 10, min_logn = 14;
  for (auto &j : b->jobs) {
    all_f64 = all_f64 && j.ctx->f64_ok;
    max_logn = std::max(max_logn, j.ctx->logN);
    min_logn = std::min(min_logn, j.ctx->logN);
  }
  if (b->jobs.empty()) min_logn = max_logn;
  b->arith = all_f64 ? HE_ARITH_F64 : HE_ARITH_U64;
  // the first job's autotuned multiply-accumulate schedule picks the thread count
  const int pref = (!b->jobs.empty() && b->jobs[0].ctx->s_mac.arith == b->arith) ? b->jobs[0].ctx->s_mac.loge : 5;
  persistent_variant(b->arith, min_logn, max_logn, pref, b->var);
  const uint32_t slab_n = 1u << b->var.slab;
  // workspace: transformed inputs and plaintexts per job
  const size_t nj = b->jobs.size();
  std::vector<size_t> offs(nj, 0);
  size_t off = 0;
  for (size_t j = 0; j < nj; ++j) {
    offs[j] = off;
    off += job_ws_bytes(b->jobs[j]);
  }
  b->ws_bytes = off;
  if (off && (e = hipMalloc(&b->d_ws, off)) != hipSuccess) {
    release(b);
    return hip_fail(e, "batch workspace");
  }
  std::vector<char *> wsp(nj);
  for (size_t j = 0; j < nj; ++j) wsp[j] = (char *)b->d_ws + offs[j];
  b->ws_ptrs = wsp;
  std::vector<PTask> tasks;
  std::vector<PJob> pjobs;
  he_batch_info info{};
  he_status bs = build_tables(b->jobs, wsp, b->arith, b->var.slab, tasks, pjobs, info, b->xq.b);
  if (bs != HE_OK) {
    release(b);
    return bs;
  }
  b->h_jobs = pjobs;
  b->n_tasks = (uint32_t)tasks.size();
  b->ctl_words = CTL_DONE + (uint32_t)nj;
  int cus = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
  if (e != hipSuccess) {
    release(b);
    return hip_fail(e, "device attribute");
  }
  const int per_cu = b->var.wg_per_cu;
  b->grid = (uint32_t)std::max(1, std::min<int>(cus * per_cu, (int)std::max<uint32_t>(1u, b->n_tasks)));
  if ((e = hipMalloc(&b->d_tasks, std::max<size_t>(1, tasks.size()) * sizeof(PTask))) != hipSuccess ||
      (e = hipMalloc(&b->d_jobs, std::max<size_t>(1, nj) * sizeof(PJob))) != hipSuccess ||
      (e = hipMalloc(&b->d_ctl, b->ctl_words * 4)) != hipSuccess ||
      (e = hipMemset(b->d_ctl, 0, b->ctl_words * 4)) != hipSuccess ||
      (tasks.size() && (e = hipMemcpy(b->d_tasks, tasks.data(), tasks.size() * sizeof(PTask), hipMemcpyHostToDevice)) != hipSuccess) ||
      (nj && (e = hipMemcpy(b->d_jobs, pjobs.data(), nj * sizeof(PJob), hipMemcpyHostToDevice)) != hipSuccess)) {
    release(b);
    return hip_fail(e, "batch tables");
  }
  info.n_jobs = (uint32_t)nj;
  info.n_tasks = b->n_tasks;
  info.grid = b->grid;
  info.arith = (uint32_t)b->arith;
  info.ws_bytes = b->ws_bytes;
  b->info = info;
  if ((flags & HE_BATCH_PROFILE) && !(flags & HE_BATCH_GRAPH)) {
    b->ev.resize(2 * he_batch::kProfRing, nullptr);
    for (hipEvent_t &ev : b->ev)
      if ((e = hipEventCreate(&ev)) != hipSuccess) {
        release(b);
        return hip_fail(e, "profiling events");
      }
  }
  if (flags & HE_BATCH_GRAPH) {
    if ((e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
      release(b);
      return hip_fail(e, "graph capture");
    }
    hipError_t le = launch_persistent(b->var, b->d_tasks, b->n_tasks, b->xq, b->d_jobs, (uint32_t)nj, b->d_ctl,
                                      b->ctl_words, b->grid, b->spin_limit, b->strict, b->cap);
    e = hipStreamEndCapture(b->cap, &b->graph);
    if (le != hipSuccess || e != hipSuccess ||
        (e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess) {
      release(b);
      return hip_fail(le != hipSuccess ? le : e, "graph build");
    }
  }
  b->built = true;
  return HE_OK;
}

he_status he_batch_rebind(he_batch *b, uint32_t index, const he_job *job) {
  if (!b || !job) return fail(HE_EINVAL, "null argument");
  if (index >= b->jobs.size()) return fail(HE_EINVAL, "job index");
  JobRef &bj = b->jobs[index];
  if (job->plan != nullptr && &job->plan->p != bj.plan) return fail(HE_EINVAL, "rebind must keep the plan");
  const uint32_t keep = HE_IN_NTT | HE_PLAIN_POLY;
  if ((job->flags & keep) != (bj.job.flags & keep)) return fail(HE_EINVAL, "rebind must keep the input flags");
  he_job nj = *job;
  nj.plan = bj.job.plan;
  bj.job = nj;
  if (!b->built) return HE_OK;
  PJob pj;
  std::vector<JobRef> one{bj};
  std::vector<char *> w{b->ws_ptrs[index]};
  std::vector<PTask> t;
  std::vector<PJob> pjs;
  he_batch_info tmp;
  uint32_t xq_tmp[kXcds + 1];
  he_status s = build_tables(one, w, b->arith, b->var.slab, t, pjs, tmp, xq_tmp);
  if (s != HE_OK) return s;
  pj = pjs[0];
  pj.n_pre = b->h_jobs[index].n_pre;
  b->h_jobs[index] = pj;
  hipError_t e = hipMemcpy(b->d_jobs + index, &pj, sizeof(PJob), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "rebind");
  return HE_OK;
}

he_status he_batch_run(he_batch *b, void *stream) {
  if (!b || !b->built) return fail(HE_EINVAL, "batch not built");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!b->ev.empty()) {
    if (b->ev_pending >= he_batch::kProfRing) return fail(HE_EINVAL, "profiled batch: sync at least every 64 runs");
    const uint32_t k = (b->ev_next + b->ev_pending) % he_batch::kProfRing;
    e0 = b->ev[2 * k];
    e1 = b->ev[2 * k + 1];
  }
  if (b->exec) e = hipGraphLaunch(b->exec, st);
  else e = launch_persistent(b->var, b->d_tasks, b->n_tasks, b->xq, b->d_jobs, (uint32_t)b->jobs.size(), b->d_ctl,
                             b->ctl_words, b->grid, b->spin_limit, b->strict, st, e0, e1);
  if (e != hipSuccess) return hip_fail(e, "batch launch");
  if (e0) b->ev_pending++;
  return HE_OK;
}

he_status he_batch_sync(he_batch *b, void *stream) {
  if (!b || !b->built) return fail(HE_EINVAL, "batch not built");
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "batch sync");
  for (; b->ev_pending; --b->ev_pending) {
    const uint32_t k = b->ev_next;
    float ms = 0.f;
    if ((e = hipEventElapsedTime(&ms, b->ev[2 * k], b->ev[2 * k + 1])) != hipSuccess) return hip_fail(e, "profiling events");
    b->info.kernel_ms += ms;
    b->info.kernel_launches++;
    b->ev_next = (k + 1) % he_batch::kProfRing;
  }
  // the flag is sticky over the runs since the last sync (the launches leave it
  // alone): read it, and clear it once reported
  uint32_t err = 0;
  e = hipMemcpy(&err, b->d_ctl + CTL_ERR, 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "batch status");
  if (err) {
    if ((e = hipMemset(b->d_ctl + CTL_ERR, 0, 4)) != hipSuccess) return hip_fail(e, "batch status reset");
    return fail(HE_ETIMEOUT, "a dependency wait in the persistent kernel hit its bound");
  }
  return HE_OK;
}

he_status he_batch_set_spin_limit(he_batch *b, uint32_t polls) {
  if (!b) return fail(HE_EINVAL, "null batch");
  b->spin_limit = polls;
  return HE_OK;
}

he_status he_batch_get_info(const he_batch *b, he_batch_info *info) {
  if (!b || !info) return fail(HE_EINVAL, "null argument");
  *info = b->info;
  info->n_jobs = (uint32_t)b->jobs.size();
  return HE_OK;
}

he_status he_batch_destroy(he_batch *b) {
  if (!b) return HE_OK;
  (void)hipSetDevice(b->device);
  release(b);
  delete b;
  return HE_OK;
}

}  // extern "C"
