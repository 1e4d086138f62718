// Serving loop: continuous batching of homomorphic linear-layer jobs.
//
// Submitted jobs wait in a FIFO.  A server thread admits jobs while the device
// footprint of admitted-but-unfinished work (workspace + the job's own buffers
// + transformed inputs kept resident for sessions) stays within the cap, and
// launches every admitted job that is not yet running as one persistent-
// kernel epoch on a free stream slot.  With several slots, jobs that arrive
// while an epoch runs go into the next epoch on another stream and overlap on
// the device.  A finished epoch releases its jobs' workspace and records
// per-job latency (arrival to completion observed on the host).
//
// Residency.  The forward transform of a job's input ciphertexts depends only
// on the ciphertexts and the ring, not on the layer, so a job of a session
// that consumes the same input buffer as an earlier job of that session can
// read its transform instead of computing it again (the layers of a training
// step reuse their inputs, Section 2 "Neural Network Training").  A job
// submitted with HE_SERVE_KEEP_RESIDENT keeps its workspace block, whose first
// part holds its transformed inputs as canonical residues; a later job of the
// same session with HE_IN_RESIDENT and the same context and input buffer then
// runs on that block as an already-transformed input.  Kept blocks are freed
// when their session closes, and evicted (oldest first, when no job reads
// them) when the queue head does not fit while no epoch is running, so kept
// data never blocks admission for good; a job whose resident transform is
// gone transforms its input as usual.
//
// Mode SEQUENTIAL serves one job at a time through the per-layer entry point
// (separate transform / multiply-accumulate / inverse kernels), the plain
// baseline the continuous mode is compared with.
//
// Locking: submissions, waits and statistics take the server mutex; the server
// thread holds it only to move jobs between queue, slots and completion, never
// across a HIP call.  Each slot's task, job and control tables are allocated
// at creation for max_batch_jobs jobs.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <thread>

#include "batch.hpp"

namespace he {
size_t layer_ws_bytes(const Ctx &c, const Plan &p, uint32_t flags);
he_status run_layer(const Ctx &c, const Plan &p, const uint64_t *ct_in, const void *plain, uint64_t *ct_out,
                    uint32_t flags, void *ws, size_t ws_bytes, hipStream_t st, const uint64_t *seed = nullptr);

using Clock = std::chrono::steady_clock;
static double now_s() { return std::chrono::duration<double>(Clock::now().time_since_epoch()).count(); }
static inline size_t al4k(size_t b) { return (b + 4095) & ~(size_t)4095; }

// First-fit allocator over one device arena (offsets only).
class Arena {
 public:
  size_t size = 0;
  char *base = nullptr;
  bool alloc(size_t n, size_t &off) {
    n = al4k(std::max<size_t>(n, 1));
    size_t prev = 0;
    for (auto it = used_.begin(); it != used_.end(); ++it) {
      if (it->first - prev >= n) {
        off = prev;
        used_[off] = n;
        return true;
      }
      prev = it->first + it->second;
    }
    if (size - prev >= n) {
      off = prev;
      used_[off] = n;
      return true;
    }
    return false;
  }
  void release(size_t off) { used_.erase(off); }

 private:
  std::map<size_t, size_t> used_;   // offset -> size, ordered
};

// The kept transform of one job's inputs: canonical residues at the start of
// its workspace block.
struct Resident {
  uint64_t session = 0;
  const Ctx *ctx = nullptr;
  const uint64_t *src = nullptr;   // the caller's input buffer it is the transform of
  uint32_t n_ct = 0;
  size_t off = 0, bytes = 0;       // the arena block
  uint32_t readers = 0;            // running jobs that read it
  bool closed = false;             // session closed while read: freed by the last reader
};

struct SJob {
  uint64_t ticket = 0, session = 0;
  JobRef ref{};                    // as launched (a resident hit runs as HE_IN_NTT on the block)
  const uint64_t *src = nullptr;   // the caller's input buffer
  size_t footprint = 0, ws_bytes = 0, ws_off = 0;
  bool has_ws = false, keep = false, want_resident = false;
  Resident *res = nullptr;         // the resident transform this job reads
  double t_arrive = 0, t_launch = 0, t_done = 0;
  int state = 0;   // 0 queued, 1 running, 2 done
  he_status status = HE_OK;
};

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  PTask *d_tasks = nullptr;
  PJob *d_jobs = nullptr;
  uint32_t *d_ctl = nullptr;
  size_t cap_tasks = 0, cap_jobs = 0;
  PTask *h_tasks = nullptr;   // pinned staging
  PJob *h_jobs = nullptr;
  uint32_t *h_err = nullptr;   // pinned copy of the launch's error flag
  std::vector<SJob *> jobs;
  bool busy = false;
};

}  // namespace he

struct he_server {
  he_server_params p{};
  int cus = 256;
  std::mutex mu;
  std::condition_variable cv_done, cv_work;
  std::deque<he::SJob *> queue;
  std::map<uint64_t, he::SJob *> all;
  std::list<he::Resident> resident;                 // oldest first
  std::map<uint64_t, uint32_t> session_count;
  he::Arena arena;
  std::vector<he::Slot> slots;
  std::thread th;
  bool stop = false;
  uint64_t next_ticket = 1;
  size_t in_use = 0, peak_in_use = 0;
  uint64_t epochs = 0, epoch_jobs = 0, rejected = 0, single_epochs = 0;
  uint64_t hits = 0, misses = 0, evictions = 0, fwd_planes = 0, failed = 0;
  std::vector<double> lat;
  double first_arrive = 0, last_done = 0;
};

using namespace he;

// Grow a slot's tables (only for an epoch larger than the sizes of creation).
static he_status slot_reserve(Slot &s, size_t n_tasks, size_t n_jobs) {
  hipError_t e;
  if (n_tasks > s.cap_tasks) {
    size_t c = std::max(n_tasks, 2 * s.cap_tasks);
    if (s.d_tasks) (void)hipFree(s.d_tasks);
    if (s.h_tasks) (void)hipHostFree(s.h_tasks);
    s.d_tasks = nullptr;
    s.h_tasks = nullptr;
    s.cap_tasks = 0;
    if ((e = hipMalloc(&s.d_tasks, c * sizeof(PTask))) != hipSuccess ||
        (e = hipHostMalloc(&s.h_tasks, c * sizeof(PTask), 0)) != hipSuccess)
      return hip_fail(e, "server task table");
    s.cap_tasks = c;
  }
  if (n_jobs > s.cap_jobs) {
    size_t c = std::max(n_jobs, 2 * s.cap_jobs);
    if (s.d_jobs) (void)hipFree(s.d_jobs);
    if (s.h_jobs) (void)hipHostFree(s.h_jobs);
    if (s.d_ctl) (void)hipFree(s.d_ctl);
    s.d_jobs = nullptr;
    s.h_jobs = nullptr;
    s.d_ctl = nullptr;
    s.cap_jobs = 0;
    if ((e = hipMalloc(&s.d_jobs, c * sizeof(PJob))) != hipSuccess ||
        (e = hipHostMalloc(&s.h_jobs, c * sizeof(PJob), 0)) != hipSuccess ||
        (e = hipMalloc(&s.d_ctl, (CTL_DONE + c) * 4)) != hipSuccess)
      return hip_fail(e, "server job table");
    s.cap_jobs = c;
  }
  return HE_OK;
}

static size_t job_buffers_bytes(const JobRef &j) {
  const he_plan_info &in = j.plan->info;
  const size_t ct = (size_t)2 * j.ctx->L * j.ctx->N * 8;
  return (size_t)in.n_ct_in * ct + (size_t)in.n_ct_out * ct;
}

// Lock held.  Free a kept block (unless read: then its last reader frees it).
static void drop_resident(he_server *S, std::list<Resident>::iterator it) {
  if (it->readers) {
    it->closed = true;
    return;
  }
  S->arena.release(it->off);
  S->in_use -= al4k(it->bytes);
  S->resident.erase(it);
}

static void close_session(he_server *S, uint64_t session) {
  for (auto it = S->resident.begin(); it != S->resident.end();) {
    auto nx = std::next(it);
    if (it->session == session) drop_resident(S, it);
    it = nx;
  }
  S->session_count.erase(session);
}

// Lock held.  Free kept blocks, oldest first, that no job reads; true if any was freed.
static bool evict_one(he_server *S) {
  for (auto it = S->resident.begin(); it != S->resident.end(); ++it)
    if (!it->readers && !it->closed) {
      S->arena.release(it->off);
      S->in_use -= al4k(it->bytes);
      S->resident.erase(it);
      S->evictions++;
      return true;
    }
  return false;
}

// Lock held: a finished (or failed) job leaves; its block is kept for its session or freed.
static void finish_job(he_server *S, SJob *j, double t) {
  j->t_done = t;
  j->state = 2;
  if (j->status != HE_OK) S->failed++;
  if (j->res) {
    Resident *r = j->res;
    j->res = nullptr;
    if (--r->readers == 0 && r->closed)
      for (auto it = S->resident.begin(); it != S->resident.end(); ++it)
        if (&*it == r) {
          drop_resident(S, it);
          break;
        }
  }
  const bool kept = j->has_ws && j->keep && j->status == HE_OK && !(j->ref.job.flags & HE_IN_NTT);
  if (kept) {
    Resident r;
    r.session = j->session;
    r.ctx = j->ref.ctx;
    r.src = j->src;
    r.n_ct = j->ref.plan->info.n_ct_in;
    r.off = j->ws_off;
    r.bytes = j->ws_bytes;
    S->resident.push_back(r);
    S->in_use -= j->footprint - al4k(j->ws_bytes);   // buffers leave, the kept block stays
  } else {
    if (j->has_ws) S->arena.release(j->ws_off);
    S->in_use -= j->footprint;
  }
  j->has_ws = false;
  S->lat.push_back(j->t_done - j->t_arrive);
  S->last_done = std::max(S->last_done, t);
  if (j->session && S->p.session_jobs) {
    uint32_t &n = S->session_count[j->session];
    if (++n >= S->p.session_jobs) close_session(S, j->session);
  }
}

// Lock held.  Admit the queue head if it fits (evicting kept blocks when
// nothing runs that could free memory); resolve its resident input.
static SJob *admit_head(he_server *S, bool any_busy) {
  SJob *j = S->queue.front();
  for (;;) {
    size_t off = 0;
    if (S->in_use + j->footprint <= S->p.mem_cap_bytes && (!j->ws_bytes || S->arena.alloc(j->ws_bytes, off))) {
      j->ws_off = off;
      j->has_ws = j->ws_bytes != 0;
      break;
    }
    if (any_busy || !evict_one(S)) return nullptr;   // wait for running epochs to free memory
  }
  S->in_use += j->footprint;
  S->peak_in_use = std::max(S->peak_in_use, S->in_use);
  S->queue.pop_front();
  if (j->want_resident) {
    for (auto &r : S->resident)
      if (!r.closed && r.session == j->session && r.ctx == j->ref.ctx && r.src == j->src &&
          r.n_ct >= j->ref.plan->info.n_ct_in) {
        j->res = &r;
        break;
      }
    if (j->res) {
      j->res->readers++;
      j->ref.job.ct_in = (const uint64_t *)(S->arena.base + j->res->off);
      j->ref.job.flags |= HE_IN_NTT;
      S->hits++;
    } else {
      S->misses++;
    }
  }
  return j;
}

static uint64_t fwd_planes_of(const JobRef &r) {
  const he_plan_info &in = r.plan->info;
  return (uint64_t)in.n_pt * r.ctx->L + ((r.job.flags & HE_IN_NTT) ? 0 : (uint64_t)in.n_ct_in * 2 * r.ctx->L);
}

// Server thread, no lock held: validate the jobs that ask for it (each alone,
// so a malformed job fails by itself), then launch the rest on the slot.
// Jobs that fail are returned in `failed` with their status set.
static hipError_t launch_epoch(he_server *S, Slot &sl, std::vector<SJob *> &take, std::vector<SJob *> &failed,
                               he_status &st) {
  st = HE_OK;
  std::vector<SJob *> ok;
  for (SJob *j : take) {
    if (j->ref.job.flags & HE_VALIDATE) {
      const Ctx &c = *j->ref.ctx;
      const size_t n = (size_t)j->ref.plan->info.n_ct_in * 2 * c.L;
      he_status v = validate(c, j->ref.job.ct_in, n, S->arena.base + j->ws_off + j->ws_bytes - 256, sl.st);
      if (v != HE_OK) {
        j->status = v;
        failed.push_back(j);
        continue;
      }
    }
    ok.push_back(j);
  }
  take.swap(ok);
  if (take.empty()) return hipSuccess;
  hipError_t e = hipSuccess;
  const uint32_t strip = ~(uint32_t)(HE_VALIDATE | HE_IN_RESIDENT);
  if (S->p.mode == HE_SERVE_SEQUENTIAL) {
    SJob *j = take[0];
    st = run_layer(*j->ref.ctx, *j->ref.plan, j->ref.job.ct_in, j->ref.job.plain, j->ref.job.ct_out,
                   (j->ref.job.flags & strip) | HE_UNFUSED, S->arena.base + j->ws_off, j->ws_bytes, sl.st);
  } else if (take.size() == 1) {
    // a lone job: the fused per-layer kernels have less fixed cost than a
    // persistent launch (no dependency waits, no cache-maintenance kernels)
    SJob *j = take[0];
    *sl.h_err = 0u;
    st = run_layer(*j->ref.ctx, *j->ref.plan, j->ref.job.ct_in, j->ref.job.plain, j->ref.job.ct_out,
                   j->ref.job.flags & strip & ~HE_UNFUSED, S->arena.base + j->ws_off, j->ws_bytes, sl.st);
  } else {
    std::vector<JobRef> refs;
    std::vector<char *> ws;
    bool all_f64 = true;
    uint32_t mn = 14, mx = 10;
    for (SJob *j : take) {
      JobRef r = j->ref;
      r.job.flags &= strip;
      r.canon_ct = j->keep;   // a kept transform is read later as canonical residues
      refs.push_back(r);
      ws.push_back(S->arena.base + j->ws_off);
      all_f64 = all_f64 && j->ref.ctx->f64_ok;
      mn = std::min(mn, j->ref.ctx->logN);
      mx = std::max(mx, j->ref.ctx->logN);
    }
    const int arith = all_f64 ? HE_ARITH_F64 : HE_ARITH_U64;
    PVariant v{};
    const Ctx *c0 = take[0]->ref.ctx;
    persistent_variant(arith, mn, mx, c0->s_mac.arith == arith ? c0->s_mac.loge : 5, v);
    std::vector<PTask> tasks;
    std::vector<PJob> pjobs;
    he_batch_info info;
    XQ xq{};
    st = build_tables(refs, ws, arith, v.slab, tasks, pjobs, info, xq.b);
    if (st == HE_OK) st = slot_reserve(sl, tasks.size(), pjobs.size());
    if (st == HE_OK) {
      std::copy(tasks.begin(), tasks.end(), sl.h_tasks);
      std::copy(pjobs.begin(), pjobs.end(), sl.h_jobs);
      e = hipMemcpyAsync(sl.d_tasks, sl.h_tasks, tasks.size() * sizeof(PTask), hipMemcpyHostToDevice, sl.st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(sl.d_jobs, sl.h_jobs, pjobs.size() * sizeof(PJob), hipMemcpyHostToDevice, sl.st);
      const uint32_t grid = (uint32_t)std::max<size_t>(1, std::min<size_t>((size_t)S->cus * v.wg_per_cu, tasks.size()));
      if (e == hipSuccess)
        e = launch_persistent(v, sl.d_tasks, (uint32_t)tasks.size(), xq, sl.d_jobs, (uint32_t)pjobs.size(), sl.d_ctl,
                              CTL_DONE + (uint32_t)pjobs.size(), grid, kSpinLimit, 0, sl.st, nullptr, nullptr, true);
      if (e == hipSuccess) e = hipMemcpyAsync(sl.h_err, sl.d_ctl + CTL_ERR, 4, hipMemcpyDeviceToHost, sl.st);
    }
  }
  if (e == hipSuccess && st == HE_OK) e = hipEventRecord(sl.ev, sl.st);
  return e;
}

static void server_loop(he_server *S) {
  (void)hipSetDevice(S->p.device);
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    bool progressed = false;
    // 1. completions (the event queries without the lock)
    std::vector<Slot *> done;
    lk.unlock();
    for (Slot &sl : S->slots)
      if (sl.busy && hipEventQuery(sl.ev) == hipSuccess) done.push_back(&sl);
    lk.lock();
    for (Slot *sl : done) {
      const double t = now_s();
      const uint32_t err = S->p.mode == HE_SERVE_CONTINUOUS ? *sl->h_err : 0u;
      for (SJob *j : sl->jobs) {
        if (err) j->status = HE_ETIMEOUT;
        finish_job(S, j, t);
      }
      sl->jobs.clear();
      sl->busy = false;
      progressed = true;
    }
    if (!done.empty()) S->cv_done.notify_all();
    // 2. launches: admit under the lock, build and launch without it
    for (Slot &sl : S->slots) {
      if (sl.busy || S->queue.empty()) continue;
      bool any_busy = false;
      for (Slot &o : S->slots) any_busy = any_busy || o.busy;
      std::vector<SJob *> take;
      const uint32_t max_jobs = S->p.mode == HE_SERVE_SEQUENTIAL ? 1u : S->p.max_batch_jobs;
      while (!S->queue.empty() && take.size() < max_jobs) {
        SJob *j = admit_head(S, any_busy || !take.empty());
        if (!j) break;
        take.push_back(j);
      }
      if (take.empty()) continue;
      const double tl = now_s();
      for (SJob *j : take) {
        j->state = 1;
        j->t_launch = tl;
      }
      sl.busy = true;   // reserved: nobody else touches this slot
      lk.unlock();
      std::vector<SJob *> failed;
      he_status st = HE_OK;
      hipError_t e = launch_epoch(S, sl, take, failed, st);
      lk.lock();
      for (SJob *j : failed) finish_job(S, j, now_s());
      if (e != hipSuccess || st != HE_OK) {
        // failed launch: only these jobs fail
        if (e != hipSuccess) hip_fail(e, "server launch");
        for (SJob *j : take) {
          j->status = st != HE_OK ? st : HE_EDEVICE;
          finish_job(S, j, now_s());
        }
        take.clear();
      }
      if (!failed.empty() || take.empty()) S->cv_done.notify_all();
      if (take.empty()) {
        sl.busy = false;
        progressed = true;
        continue;
      }
      for (SJob *j : take) S->fwd_planes += fwd_planes_of(j->ref);
      sl.jobs = take;
      S->epochs++;
      S->epoch_jobs += take.size();
      if (take.size() == 1 && S->p.mode == HE_SERVE_CONTINUOUS) S->single_epochs++;
      progressed = true;
    }
    bool any_busy = false;
    for (Slot &sl : S->slots) any_busy = any_busy || sl.busy;
    if (S->stop && S->queue.empty() && !any_busy) break;
    if (!progressed) {
      if (any_busy) {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(S->p.poll_us));
        lk.lock();
      } else {
        S->cv_work.wait_for(lk, std::chrono::milliseconds(2));
      }
    }
  }
}

extern "C" {

he_status he_server_create(const he_server_params *p, he_server **out) {
  if (!p || !out) return fail(HE_EINVAL, "null argument");
  if (p->mode != HE_SERVE_CONTINUOUS && p->mode != HE_SERVE_SEQUENTIAL) return fail(HE_EINVAL, "mode");
  he_server *S = new he_server();
  S->p = *p;
  if (!S->p.max_batch_jobs) S->p.max_batch_jobs = 64;
  if (!S->p.slots) S->p.slots = 2;
  if (S->p.slots > 8) S->p.slots = 8;
  if (!S->p.poll_us) S->p.poll_us = 20;
  if (S->p.mode == HE_SERVE_SEQUENTIAL) S->p.slots = 1;
  size_t arena = S->p.arena_bytes ? S->p.arena_bytes : std::min<uint64_t>(S->p.mem_cap_bytes, 8ull << 30);
  hipError_t e = hipSetDevice(S->p.device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&S->cus, hipDeviceAttributeMultiprocessorCount, S->p.device);
  if (e == hipSuccess) e = hipMalloc(&S->arena.base, arena);
  if (e != hipSuccess) {
    delete S;
    return hip_fail(e, "server arena");
  }
  S->arena.size = arena;
  S->slots.resize(S->p.slots);
  for (Slot &sl : S->slots) {
    if ((e = hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming)) != hipSuccess ||
        (e = hipHostMalloc(&sl.h_err, 4, 0)) != hipSuccess) {
      he_server_destroy(S);
      return hip_fail(e, "server streams");
    }
    // tables for max_batch_jobs jobs of up to 1024 tasks each (larger epochs grow them)
    he_status st = slot_reserve(sl, (size_t)S->p.max_batch_jobs * 1024, S->p.max_batch_jobs);
    if (st != HE_OK) {
      he_server_destroy(S);
      return st;
    }
  }
  S->th = std::thread(server_loop, S);
  *out = S;
  return HE_OK;
}

static he_status submit_at(he_server *S, he_ctx *ctx, const he_job *job, uint64_t session, uint32_t flags,
                           uint64_t *ticket, double t_arrive);

he_status he_server_submit(he_server *S, he_ctx *ctx, const he_job *job, uint64_t session, uint32_t flags,
                           uint64_t *ticket) {
  return submit_at(S, ctx, job, session, flags, ticket, now_s());
}

}  // extern "C"

static he_status submit_at(he_server *S, he_ctx *ctx, const he_job *job, uint64_t session, uint32_t flags,
                           uint64_t *ticket, double t_arrive) {
  if (!S || !ctx || !job || !job->plan || !ticket) return fail(HE_EINVAL, "null argument");
  if (job->plan->ctx != ctx->c) return fail(HE_EINVAL, "plan belongs to another context");
  if (!job->ct_in || !job->plain || !job->ct_out) return fail(HE_EINVAL, "null job buffer");
  if (job->plan->p.info.kind == HE_KIND_DW && !(job->flags & HE_PLAIN_POLY))
    return fail(HE_EUNSUPPORTED, "weight-gradient jobs need HE_PLAIN_POLY");
  if ((job->flags & HE_IN_RESIDENT) && ((job->flags & HE_IN_NTT) || !session))
    return fail(HE_EINVAL, "HE_IN_RESIDENT needs a session and coefficient-form inputs");
  SJob *j = new SJob();
  j->ref = JobRef{ctx->c, &job->plan->p, *job};
  j->src = job->ct_in;
  j->session = session;
  j->keep = session != 0 && (flags & HE_SERVE_KEEP_RESIDENT);
  j->want_resident = (job->flags & HE_IN_RESIDENT) != 0;
  // continuous mode runs a job alone in an epoch through the fused per-layer
  // path and with others through the batch kernel: room for either (the
  // transformed inputs sit at the start in both)
  const uint32_t lf = job->flags & ~(uint32_t)HE_IN_RESIDENT;
  j->ws_bytes = S->p.mode == HE_SERVE_SEQUENTIAL
                    ? layer_ws_bytes(*ctx->c, job->plan->p, lf | HE_UNFUSED)
                    : std::max(job_ws_bytes(j->ref), layer_ws_bytes(*ctx->c, job->plan->p, lf & ~HE_UNFUSED));
  if (job->flags & HE_VALIDATE) j->ws_bytes += 256;   // the validation flag, at the end
  j->footprint = al4k(j->ws_bytes) + job_buffers_bytes(j->ref);
  std::lock_guard<std::mutex> g(S->mu);
  if (j->footprint > S->p.mem_cap_bytes || j->ws_bytes > S->arena.size) {
    S->rejected++;
    delete j;
    return fail(HE_EBUSY, "job footprint exceeds the memory cap");
  }
  j->ticket = S->next_ticket++;
  j->t_arrive = t_arrive;
  if (S->first_arrive == 0) S->first_arrive = j->t_arrive;
  S->all[j->ticket] = j;
  S->queue.push_back(j);
  *ticket = j->ticket;
  S->cv_work.notify_one();
  return HE_OK;
}

extern "C" {

he_status he_server_wait(he_server *S, uint64_t ticket, int64_t timeout_us, he_job_result *res) {
  if (!S) return fail(HE_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return fail(HE_EINVAL, "unknown ticket");
  SJob *j = it->second;
  auto done = [&] { return j->state == 2; };
  if (timeout_us < 0) S->cv_done.wait(lk, done);
  else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done))
    return fail(HE_ETIMEOUT, "job not finished");
  if (res) {
    res->status = j->status;
    res->latency_s = j->t_done - j->t_arrive;
    res->queue_s = j->t_launch - j->t_arrive;
  }
  if (j->status != HE_OK) return fail(j->status, "job failed");
  return HE_OK;
}

he_status he_server_close_session(he_server *S, uint64_t session) {
  if (!S) return fail(HE_EINVAL, "null server");
  std::lock_guard<std::mutex> g(S->mu);
  close_session(S, session);
  S->cv_work.notify_one();
  return HE_OK;
}

he_status he_server_stats(he_server *S, he_server_info *out) {
  if (!S || !out) return fail(HE_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(S->mu);
  *out = he_server_info{};
  std::vector<double> l = S->lat;
  std::sort(l.begin(), l.end());
  auto pct = [&](double q) { return l.empty() ? 0.0 : l[std::min(l.size() - 1, (size_t)(q * (l.size() - 1) + 0.5))]; };
  out->completed = l.size();
  out->rejected = S->rejected;
  out->epochs = S->epochs;
  out->single_epochs = S->single_epochs;
  out->mean_jobs_per_epoch = S->epochs ? (double)S->epoch_jobs / S->epochs : 0.0;
  out->p50_s = pct(0.50);
  out->p99_s = pct(0.99);
  double sum = 0;
  for (double v : l) sum += v;
  out->mean_s = l.empty() ? 0 : sum / l.size();
  out->max_s = l.empty() ? 0 : l.back();
  out->span_s = S->last_done > S->first_arrive ? S->last_done - S->first_arrive : 0;
  out->peak_bytes = S->peak_in_use;
  out->in_use_bytes = S->in_use;
  out->resident_hits = S->hits;
  out->resident_misses = S->misses;
  out->evictions = S->evictions;
  out->fwd_planes = S->fwd_planes;
  out->failed = S->failed;
  out->resident_blocks = S->resident.size();
  return HE_OK;
}

he_status he_server_drain(he_server *S) {
  if (!S) return fail(HE_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(S->mu);
  S->cv_done.wait(lk, [&] {
    if (!S->queue.empty()) return false;
    for (Slot &sl : S->slots)
      if (sl.busy) return false;
    return true;
  });
  return HE_OK;
}

he_status he_server_replay(he_server *S, uint32_t n, he_ctx *const *ctxs, const he_job *jobs, const double *arrival_s,
                           const uint64_t *sessions, uint32_t flags, double *latency_s) {
  if (!S || (n && (!ctxs || !jobs || !arrival_s))) return fail(HE_EINVAL, "null argument");
  std::vector<uint64_t> tickets(n, 0);
  std::vector<he_status> sub(n, HE_OK);
  const double t0 = now_s();
  for (uint32_t i = 0; i < n; ++i) {
    while (now_s() - t0 < arrival_s[i]) {
    }
    sub[i] = submit_at(S, ctxs[i], &jobs[i], sessions ? sessions[i] : 0, flags, &tickets[i], t0 + arrival_s[i]);
  }
  he_status worst = HE_OK;
  for (uint32_t i = 0; i < n; ++i) {
    if (sub[i] != HE_OK) {
      if (latency_s) latency_s[i] = -1.0;
      worst = sub[i];
      continue;
    }
    he_job_result r{};
    he_status s = he_server_wait(S, tickets[i], -1, &r);
    if (latency_s) latency_s[i] = r.latency_s;
    if (s != HE_OK) worst = s;
  }
  return worst;
}

he_status he_server_destroy(he_server *S) {
  if (!S) return HE_OK;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
    S->cv_work.notify_all();
  }
  if (S->th.joinable()) S->th.join();
  (void)hipSetDevice(S->p.device);
  for (Slot &sl : S->slots) {
    if (sl.st) (void)hipStreamSynchronize(sl.st);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.st) (void)hipStreamDestroy(sl.st);
    if (sl.d_tasks) (void)hipFree(sl.d_tasks);
    if (sl.d_jobs) (void)hipFree(sl.d_jobs);
    if (sl.d_ctl) (void)hipFree(sl.d_ctl);
    if (sl.h_tasks) (void)hipHostFree(sl.h_tasks);
    if (sl.h_jobs) (void)hipHostFree(sl.h_jobs);
    if (sl.h_err) (void)hipHostFree(sl.h_err);
  }
  if (S->arena.base) (void)hipFree(S->arena.base);
  for (auto &kv : S->all) delete kv.second;
  delete S;
  return HE_OK;
}

}  // extern "C"
