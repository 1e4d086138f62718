// Persistent fused batch kernel: many layers (jobs) of different ring degrees
// and shapes in one launch.
//
// The host builds a task table: for every job, forward-transform tasks for its
// input ciphertext planes and pack-lift-transform tasks for its plaintext
// planes ("pre" tasks), then, after all pre tasks of all jobs, one
// multiply-accumulate + inverse-transform task per output plane group.  The
// grid holds as many workgroups as fit on the chip at once (LDS-limited), and
// they drain the table through atomic counters: one shared queue for the pre
// tasks, then one queue of dependent tasks per XCD (contiguous runs of output
// planes, so outputs sharing inputs share an L2), stolen from other XCDs once a
// workgroup's own queue is empty.  A workgroup owns 2^SLAB coefficients of LDS
// per task: one plane at the largest ring degree of the variant, several
// planes of smaller degrees side by side; every thread holds 2^LOGE
// coefficients whatever the degree, so the register budget does not depend on N.
//
// A multiply-accumulate task of job j waits until every pre task of job j has
// finished: pre tasks write their outputs with device-coherent stores, wait for
// them, and count themselves done in a per-job counter; the waiting workgroup
// acquires the job once (an L2 invalidate).  Every pre task precedes every
// multiply-accumulate task in the table and a workgroup's claims move forward
// through the queues only, so no workgroup waits while holding a pre task: a
// waiting task only waits on tasks that running workgroups will finish, and
// the wait always ends; it is also bounded by a spin limit that raises an
// error flag.
#include "batch.hpp"
#include "ntt.hpp"
#include "mac.hpp"
#include "pack.hpp"

namespace he {

// s_waitcnt immediate for gfx9-family: vmcnt = 0, expcnt and lgkmcnt left at their maxima
constexpr int kWaitVmcnt0 = 0x0F70;

// A pre task's outputs are written with device-coherent stores (agent-scope
// relaxed atomic stores: written through this XCD's L2), so that once a wave's
// stores have completed they are visible to every XCD without writing back the
// whole L2, which a release would do after every task.  Written through, a
// partly filled line costs a partial write: the transforms feeding these
// stores end with a pass through LDS and store whole lines in linear order.
__device__ __forceinline__ void publish(HE_GLOBAL uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A workgroup barrier that orders LDS only: each wave's LDS accesses before it
// have completed, while its global loads and stores may still be in flight
// (__syncthreads would also wait for every outstanding global access, here
// the previous task's output stores).  The compiler fences keep LDS accesses
// from moving across it; global ordering in the task loop comes from the
// explicit waits, counters and acquires around it.
__device__ __forceinline__ void lds_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0); vmcnt and expcnt left at their maxima
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Record idx of a table that no kernel writes during the launch, at an index
// that is the same in every lane: read through the constant address space as
// 32-byte words (records are copied out as vectors, then cast back), so the
// compiler uses scalar loads.
template <class T>
__device__ __forceinline__ T load_const(const T *p, uint32_t idx) {
  typedef uint32_t w8 __attribute__((ext_vector_type(8)));
  static_assert(sizeof(T) % sizeof(w8) == 0, "records of whole 32-byte words");
  constexpr int n = sizeof(T) / sizeof(w8);
  const HE_CONST w8 *c = (const HE_CONST w8 *)(uintptr_t)p + (size_t)idx * n;
  struct Words {
    w8 v[n];
  } r;
#pragma unroll
  for (int k = 0; k < n; ++k) r.v[k] = c[k];
  return __builtin_bit_cast(T, r);
}

// An int32 table that no kernel writes during the launch, read at indices the
// same in every lane (scalar loads).
#define CONST_I32(p) ((const HE_CONST int32_t *)(uintptr_t)(p))

template <class A>
struct PTw {
  using T = typename A::Tw;
  __device__ static const HE_GLOBAL T *fwd(const PJob &j) { return as_global((const T *)j.tw_fwd); }
  __device__ static const HE_GLOBAL T *inv(const PJob &j) { return as_global((const T *)j.tw_inv); }
};

// One task on one plane group member.  G: geometry with E = 16.  `valid` is
// false for a group member past the end of the task's plane range: it runs
// the same barriers but reads zeros and stores nothing.
template <class A, int LOGN, int LOGE, class Hook>
__device__ __forceinline__ void run_task(const PTask &tk, const PJob &jb, int tid_g, int group,
                                         typename A::V *lds_g, Hook hook) {
  using G = Geo<LOGN, LOGN - LOGE>;
  using V = typename A::V;
  const uint32_t plane = tk.first + (uint32_t)group;
  const bool valid = plane < tk.first + tk.count;
  const uint32_t L = jb.L;
  const uint32_t i = valid ? plane % L : 0;
  // (a plane group holds whole waves: the prime index is the same in every lane of a wave)
  const PrimeK pk = load_const(jb.primes, __builtin_amdgcn_readfirstlane(i));
  const A ar(pk);
  const uint32_t kind = tk.kind & PT_KIND_MASK;
  // The batch's own transformed operands (inputs and plaintexts) stay in the
  // policy's format: with fp64, doubles reduced to |v| <= 0.51 q (MacWsF64),
  // so the multiply-accumulate reads them without conversions; with 64-bit
  // integers, canonical residues.
  constexpr bool kF64 = std::is_same<A, ArF64>::value;
  if (kind == PT_FWD_CT) {
    hook();
    // (a member past the task's planes transforms the task's first plane,
    // always a valid input, and stores nothing: no per-coefficient selects)
    const HE_GLOBAL uint64_t *src = as_global(jb.ct_in) + (size_t)(valid ? plane : tk.first) * G::N;
    HE_GLOBAL uint64_t *dst = as_global(jb.ct_hat) + (size_t)plane * G::N;
    auto ld = [&](int k) { return ar.load(src[(uint32_t)k]); };
    // the output format is uniform over the task (inputs kept for later jobs
    // are stored as canonical residues: ct_f64 = 0), so each format has its own
    // transform and the stores carry no per-coefficient branch on it
    auto run = [&](auto f64_out) {
      auto st = [&](int k, V v) {
        if constexpr (decltype(f64_out)::value) {
          if (valid) publish(dst + (uint32_t)k, __builtin_bit_cast(uint64_t, ar.reduce(v)));
        } else {
          if (valid) publish(dst + (uint32_t)k, ar.store(v));
        }
      };
      ntt_forward<A, G, true, false, true>(ar, PTw<A>::fwd(jb) + (size_t)i * G::N, tid_g, lds_g, ld, st);
    };
    if constexpr (kF64) {
      if (jb.ct_f64) run(std::true_type{});
      else run(std::false_type{});
    } else {
      run(std::false_type{});
    }
  } else if (kind == PT_PT) {
    hook();
    const uint32_t pp = valid ? plane / L : 0;
    HE_GLOBAL uint64_t *dst = as_global(jb.pt_hat) + (size_t)plane * G::N;
    auto st = [&](int k, V v) {
      if constexpr (kF64) {
        if (valid) publish(dst + (uint32_t)k, __builtin_bit_cast(uint64_t, ar.reduce(v)));
      } else {
        if (valid) publish(dst + (uint32_t)k, ar.store(v));
      }
    };
    if (jb.pkind == PK_POLY) {
      const HE_GLOBAL int64_t *src = as_global((const int64_t *)jb.plain) + (size_t)pp * G::N;
      auto ld = [&](int k) { return ar.load_signed(src[(uint32_t)k]); };   // (pp = 0 past the planes: a valid row)
      ntt_forward<A, G, true, false, true>(ar, PTw<A>::fwd(jb) + (size_t)i * G::N, tid_g, lds_g, ld, st);
    } else {
      // pack in LDS: zero, scatter this polynomial's weights, then transform from LDS
#pragma unroll
      for (int j = 0; j < G::E; ++j) lds_g[lin_lds<G>(tid_g, j)] = ar.load(0ull);
      __syncthreads();
      if (valid) {
        const WPack wp{jb.pkind == PK_CONV ? (uint32_t)WP_CONV : (jb.pkind == PK_CONV_DX ? (uint32_t)WP_CONV_DX : (uint32_t)WP_FC),
                       jb.M, jb.C, jb.h, jb.O, jb.S, jb.Cw, jb.cb, jb.n_out, jb.n_in, jb.n_iw, jb.n_ow, jb.in_ct};
        scatter_weights<A, G>(ar, lds_g, tid_g, wp, pp, as_global((const int32_t *)jb.plain));
      }
      __syncthreads();
      ntt_forward_tc<A, G, true, false, true>(ar, PTw<A>::fwd(jb) + (size_t)i * G::N, tid_g, lds_g,
                                         LdsAt<typename A::V>{lds_g}, st);
    }
  } else {   // PT_MAC_INV: output plane (o, comp, i)
    const uint32_t comp = (plane / L) & 1, o = plane / (2 * L);
    // a one-plane task carries its term range and its first term's operand
    // planes: the operand loads start without a read of the term lists
    const bool listed = tk.t1 >= 0;
    int t0 = 0, t1 = 0;
    if (listed) {
      t0 = tk.t0;
      t1 = tk.t1;
    } else if (valid) {
      t0 = CONST_I32(jb.row)[o];
      t1 = CONST_I32(jb.row)[o + 1];
    }
    // (term lists: indices the same in every lane, read with scalar loads)
    const HE_CONST int32_t *cti = CONST_I32(jb.cti), *pti = CONST_I32(jb.pti);
    const HE_GLOBAL uint64_t *ct_hat = as_global((const uint64_t *)jb.ct_hat), *pt_hat = as_global((const uint64_t *)jb.pt_hat);
    auto planes = [&](int t) {
      if (listed && t == t0) return std::pair<uint32_t, uint32_t>(tk.a0, tk.b0);
      return std::pair<uint32_t, uint32_t>(((uint32_t)cti[t] * 2 + comp) * L + i, (uint32_t)pti[t] * L + i);
    };
    auto ix = [&](int e) { return slot_index<G, G::NPASS - 1>(tid_g, e); };
    V v[G::E];
    if constexpr (kF64) {
      auto operands = [&](int t) {
        const auto [pa, pb] = planes(t);
        return std::pair<const HE_GLOBAL uint64_t *, const HE_GLOBAL uint64_t *>(ct_hat + (size_t)pa * G::N,
                                                                                 pt_hat + (size_t)pb * G::N);
      };
      // the inputs are the batch's own doubles unless the caller transformed them
      if (jb.ct_f64) mac_terms_ws<false, G::E>(ar, v, t0, t1, operands, ix);
      else mac_terms_ws<true, G::E>(ar, v, t0, t1, operands, ix);
    } else {
      MacAcc<A> acc[G::E];
      auto operands = [&](int t) {
        const auto [pa, pb] = planes(t);
        return std::pair<const HE_GLOBAL uint64_t *, const HE_GLOBAL uint64_t *>(ct_hat + (size_t)pa * G::N,
                                                                                 pt_hat + (size_t)pb * G::N);
      };
      mac_terms<A, G::E>(ar, pk, acc, t0, t1, operands, ix);
#pragma unroll
      for (int e = 0; e < G::E; ++e) v[e] = acc[e].value();
    }
    hook();   // the operands are consumed: the next claim has long returned
    // (the first pass's twiddles are loaded here, not with the operands: held
    // across the products they would push the kernel past its register budget;
    // each later pass's twiddles are loaded during the pass before it)
    const auto twi = PTw<A>::inv(jb) + (size_t)i * G::N;
    // fp64: the passes whose lanes read different twiddles take them alone
    // (8 bytes, the quotient companion formed at the product)
    constexpr int kWM = kF64 ? lane_passes<G>() : 0;
    const double *twi_w = kF64 ? jb.tw_inv_w + (size_t)i * G::N : nullptr;
    PassTw<A, G, G::NPASS - 1, true, wbit<kWM, G::NPASS - 1>()> first;
    first.load2(twi, twi_w, tid_g);
    HE_GLOBAL uint64_t *dst = as_global(jb.ct_out) + (size_t)plane * G::N;
    const uint64_t q = pk.q;
    constexpr int kMacOut = kF64 ? MacWsF64::kOutBoundX100 : MacAcc<A>::kOutBoundX100;
    // the accumulate choice is uniform over the task: one inverse transform per
    // store kind keeps the per-coefficient stores free of branches
    if (jb.accumulate) {
      auto st = [&](int k, uint64_t x) {
        if (valid) {
          const uint64_t s = dst[(uint32_t)k] + x;
          dst[(uint32_t)k] = s >= q ? s - q : s;
        }
      };
      ntt_inverse_regs<A, G, kMacOut, true, kWM>(ar, twi, tid_g, lds_g, first, v, st, twi_w);
    } else {
      // streaming stores: output planes are not read again by this launch
      // (addressed as the thread's part plus a compile-time part; the resource
      // is formed at the stores, not held across the transform)
      auto st = [&](int t, int c, uint64_t x) {
        if (valid) buf_store_u64_nt(buf_rsrc((const void *)dst, G::N * 8u), (uint32_t)t * 8u, (uint32_t)c * 8u, x);
      };
      ntt_inverse_regs<A, G, kMacOut, true, kWM>(ar, twi, tid_g, lds_g, first, v, st, twi_w);
    }
  }
}

// SLAB = log2 of the coefficients one workgroup holds per task, LOGE = log2 of
// the coefficients each thread holds (so a workgroup has 2^(SLAB-LOGE)
// threads), LOGN_MIN..LOGN_MAX = the ring degrees compiled in.  A batch whose
// jobs share one ring degree gets a variant with that degree only (smaller
// code, the register budget of the stand-alone kernels); mixed batches get a
// variant with every degree.  A job's readiness is acquired once per
// workgroup: after the first acquire (which invalidates this CU's caches after
// the producers' release) later tasks of the same job read the finished data.
template <class A, int SLAB, int LOGE, int LOGN_MIN, int LOGN_MAX>
struct PCfg {
  static_assert(LOGN_MIN - LOGE >= 6, "a plane group must hold whole waves");
  static constexpr int NT = 1 << (SLAB - LOGE);
  static constexpr int LDS_BYTES = ((1 << SLAB) + (1 << (SLAB - kLdsPadShift))) * 8;
  static constexpr int WG_PER_CU = (163840 / (LDS_BYTES + 512)) < 1 ? 1 : (163840 / (LDS_BYTES + 512));
  static constexpr int MINW = (WG_PER_CU * NT / 256) < 1 ? 1 : (WG_PER_CU * NT / 256 > 8 ? 8 : WG_PER_CU * NT / 256);
};

template <class A, int SLAB, int LOGE, int LOGN_MIN, int LOGN_MAX>
__global__ __launch_bounds__((PCfg<A, SLAB, LOGE, LOGN_MIN, LOGN_MAX>::NT),
                             (PCfg<A, SLAB, LOGE, LOGN_MIN, LOGN_MAX>::MINW)) void k_persistent(
    const PTask *__restrict__ tasks, uint32_t n_tasks, XQ xq, const PJob *__restrict__ jobs, uint32_t n_jobs,
    uint32_t *__restrict__ ctl, uint32_t spin_limit, uint32_t strict) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t s_task[2];     // the next task, used in turn by consecutive iterations
  __shared__ uint32_t s_ready[64];   // acquired jobs (bitmap, jobs < 2048); written by thread 0 only
  typename A::V *lds = reinterpret_cast<typename A::V *>(smem);
  const int tid = threadIdx.x;
  uint32_t *head = ctl + CTL_HEAD, *err = ctl + CTL_ERR, *done = ctl + CTL_DONE;
  (void)n_tasks;
  if (tid == 0)
    for (int k = 0; k < 64; ++k) s_ready[k] = 0u;
  // (The caches are invalidated before the launch and written back after it by
  // k_edge_fence, see launch_persistent.)
  // Task source: the shared queue of pre tasks [0, xq.b[0]) first; then this
  // XCD's queue of dependent tasks (workgroups are dealt round-robin over the
  // XCDs, so blockIdx % 8 is the XCD), then the other XCDs' queues in turn.
  // Thread 0 claims the next task from a queue's counter at the start of the
  // current one and reads the claim back inside it, before the task's stores
  // (run_task's hook), so the claim's latency hides behind the task and no
  // global access is outstanding across the loop's barrier: that barrier
  // orders LDS only and leaves the previous task's stores in flight.
  const uint32_t my_xcd = blockIdx.x % kXcds;
  constexpr uint32_t kNone = 0xFFFFFFFFu;   // no task left
  uint32_t q = 0;   // thread 0: the queue claimed from (0 pre; 1..8 dependent queue (my_xcd + q - 1) % 8)
  auto queue = [&](uint32_t qq, uint32_t &lo, uint32_t &hi) -> uint32_t * {
    if (qq == 0) {
      lo = 0, hi = xq.b[0];
      return head;
    }
    const uint32_t x = (my_xcd + qq - 1) % kXcds;
    lo = xq.b[x], hi = xq.b[x + 1];
    return ctl + CTL_XQ + 32 * x;
  };
  auto issue = [&]() -> uint32_t {   // thread 0: start a claim on the current queue
    uint32_t lo, hi;
    return q <= (uint32_t)kXcds ? atomicAdd(queue(q, lo, hi), 1u) : 0u;
  };
  auto finish = [&](uint32_t pos) -> uint32_t {   // thread 0: the claimed task, or the next queue's
    while (q <= (uint32_t)kXcds) {
      uint32_t lo, hi;
      queue(q, lo, hi);
      if (lo + pos < hi) return lo + pos;
      if (++q > (uint32_t)kXcds) break;
      pos = atomicAdd(queue(q, lo, hi), 1u);
    }
    return kNone;
  };
  uint32_t ready_job = 0xFFFFFFFFu;   // job of the last dependent task (acquired); workgroup-uniform
  if (tid == 0) s_task[0] = finish(issue());
  for (uint32_t it = 0;; it ^= 1u) {
    // (the slot of iteration it was written by thread 0 during the previous
    // task; it is written again during the next one, after the barrier below
    // that every thread passes only after reading it)
    lds_barrier();
    const uint32_t t = __builtin_amdgcn_readfirstlane(s_task[it]);
    if (t == kNone) break;
    uint32_t pending = 0;
    if (tid == 0) pending = issue();
    auto hook = [&]() {
      if (tid == 0) s_task[it ^ 1u] = finish(pending);
    };
    const PTask tk = load_const(tasks, t);
    const PJob &jb = jobs[tk.job];
    // wait for the job's pre tasks unless this workgroup has acquired them
    // already (the strict mode acquires for every task): the job of the
    // previous dependent task is known in every wave, others are looked up in
    // the bitmap, which changes only after the wait's barrier, so the decision
    // is the same in all waves
    bool must_wait = false;
    if (tk.kind & PT_WAIT) {
      if (strict & 1u) must_wait = true;
      else if (tk.job != ready_job)
        must_wait = tk.job >= 2048 || !((s_ready[tk.job >> 5] >> (tk.job & 31)) & 1u);
      ready_job = tk.job;
    }
    if (must_wait) {
      if (tid == 0) {
        // every waiting workgroup polls the same counter, so back off (up to
        // about 1 us between polls) to keep the polls from crowding the memory
        // channel that the producers are using
        uint32_t spins = 0, backoff = 1;
        while (__hip_atomic_load(done + tk.job, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < jb.n_pre) {
          for (uint32_t k = 0; k < backoff; ++k) __builtin_amdgcn_s_sleep(8);
          backoff = backoff < 6 ? backoff + 1 : 6;
          if (++spins > spin_limit) {
            atomicOr(err, 1u);
            break;
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      __syncthreads();
      // every wave read the bitmap for this task before the barrier above: the
      // bit is set only now, so all waves took the same branch (the next read
      // follows the next loop-top barrier)
      if (tid == 0 && tk.job < 2048) s_ready[tk.job >> 5] |= 1u << (tk.job & 31);
      if (strict & 1u) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    const int logn = (int)jb.logN;
    const int logt = logn - LOGE;
    // a plane group has at least one whole wave (2^logt >= 64 threads), so the
    // group index is wave-uniform
    const int group = __builtin_amdgcn_readfirstlane(tid >> logt);
    const int tid_g = tid & ((1 << logt) - 1);
    const int words = (1 << logn) + (1 << (logn - kLdsPadShift));
    typename A::V *lds_g = lds + (size_t)group * words;
    // (every path calls the hook once: a degree not compiled in runs nothing)
    if constexpr (LOGN_MIN == LOGN_MAX) {
      run_task<A, LOGN_MIN, LOGE>(tk, jb, tid_g, group, lds_g, hook);
    } else {
      switch (logn) {
        case 10:
          if constexpr (LOGN_MIN <= 10) run_task<A, 10, LOGE>(tk, jb, tid_g, group, lds_g, hook);
          else hook();
          break;
        case 11:
          if constexpr (LOGN_MIN <= 11) run_task<A, 11, LOGE>(tk, jb, tid_g, group, lds_g, hook);
          else hook();
          break;
        case 12: run_task<A, 12, LOGE>(tk, jb, tid_g, group, lds_g, hook); break;
        case 13: run_task<A, 13, LOGE>(tk, jb, tid_g, group, lds_g, hook); break;
        default:
          if constexpr (LOGN_MAX >= 14) run_task<A, 14, LOGE>(tk, jb, tid_g, group, lds_g, hook);
          else hook();
          break;
      }
    }
    if ((tk.kind & PT_KIND_MASK) != PT_MAC_INV) {
      // every wave waits until its own device-coherent stores have completed
      // (the barrier alone orders LDS only): the task's outputs are then visible
      // on every XCD, and thread 0 counts the task done.  The strict mode adds
      // a full release (an L2 writeback) before the count.
      __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
      if (strict & 1u) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __syncthreads();
      if (tid == 0) {
        if (strict & 1u) __hip_atomic_fetch_add(done + tk.job, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        else __hip_atomic_fetch_add(done + tk.job, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    // (a dependent task needs no barrier here: the next task touches the plane
    // in LDS only after the next iteration's barrier)
  }
}

// Zero the queue heads and the per-job counters (a kernel, not a memset, so
// that the launch can be captured into a graph and replayed).  The error flag
// is cleared only with clear_err: a batch keeps it set across runs until its
// sync reports it, so a failed wait of any queued run is not lost.
__global__ void k_reset_ctl(uint32_t *ctl, uint32_t n_words, uint32_t clear_err) {
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n_words; k += gridDim.x * blockDim.x)
    if (k != CTL_ERR || clear_err) ctl[k] = 0u;
}

// Cache maintenance around a persistent launch, which may be a graph replay whose
// dispatch neither invalidates nor writes back the XCD L2 caches: before it,
// every XCD drops lines cached earlier (inputs rewritten by copies or by kernels
// on other XCDs); after it, every XCD writes its dirty lines back.  Workgroups
// are dealt round-robin over the XCDs, so 64 of them reach all eight.
__global__ void k_edge_fence(int release) {
  if (threadIdx.x == 0) {
    if (release) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    else __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
  }
}

template <class A, int SLAB, int LOGE, int LOGN_MIN, int LOGN_MAX>
static hipError_t launch_p(const PTask *tasks, uint32_t n_tasks, const XQ &xq, const PJob *jobs, uint32_t n_jobs,
                           uint32_t *ctl, uint32_t grid, uint32_t spin_limit, uint32_t strict, hipStream_t st) {
  using C = PCfg<A, SLAB, LOGE, LOGN_MIN, LOGN_MAX>;
  static bool set = false;
  if (!set) {
    hipError_t e = hipFuncSetAttribute((const void *)k_persistent<A, SLAB, LOGE, LOGN_MIN, LOGN_MAX>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, C::LDS_BYTES);
    if (e != hipSuccess) return e;
    set = true;
  }
  hipLaunchKernelGGL((k_persistent<A, SLAB, LOGE, LOGN_MIN, LOGN_MAX>), dim3(grid), dim3(C::NT), C::LDS_BYTES, st,
                     tasks, n_tasks, xq, jobs, n_jobs, ctl, spin_limit, strict);
  return hipGetLastError();
}

// Variants compiled: F64 single-degree 4096/8192/16384 with 16 or 32
// coefficients per thread (the preferred count -- normally the autotuned
// multiply-accumulate schedule -- clamped to that range), and mixed-degree
// variants (16 per thread) for both arithmetics.
bool persistent_variant(int arith, uint32_t logn_min, uint32_t logn_max, int pref_loge, PVariant &v) {
  if (arith == HE_ARITH_F64 && logn_min == logn_max && logn_min >= 12 && logn_min <= 14) {
    // 16 or 32 per thread: with 8, the task loop's own state leaves the
    // 64-register budget short and the kernel spills
    int loge = pref_loge < 4 ? 4 : (pref_loge > 5 ? 5 : pref_loge);
    if ((int)logn_min - loge > 10) loge = (int)logn_min - 10;
    v = PVariant{arith, (int)logn_min, loge, (int)logn_min, (int)logn_min};
  } else if (logn_max <= 13) {
    v = PVariant{arith, 13, 4, 10, 13};
  } else {
    v = PVariant{arith, 14, 4, 10, 14};
  }
  v.threads = 1 << (v.slab - v.loge);
  v.lds_bytes = ((1 << v.slab) + (1 << (v.slab - kLdsPadShift))) * 8;
  v.wg_per_cu = 163840 / (v.lds_bytes + 512);
  if (v.wg_per_cu < 1) v.wg_per_cu = 1;
  return true;
}

hipError_t launch_persistent(const PVariant &v, const PTask *tasks, uint32_t n_tasks, const XQ &xq, const PJob *jobs,
                             uint32_t n_jobs, uint32_t *ctl, uint32_t ctl_words, uint32_t grid, uint32_t spin_limit,
                             uint32_t strict, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1, bool clear_err) {
  hipLaunchKernelGGL(k_reset_ctl, dim3(1), dim3(256), 0, st, ctl, ctl_words, clear_err ? 1u : 0u);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_edge_fence, dim3(64), dim3(64), 0, st, 0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (ev0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return e;
#define HE_P(A, S, E, MN, MX) \
  launch_p<A, S, E, MN, MX>(tasks, n_tasks, xq, jobs, n_jobs, ctl, grid, spin_limit, strict, st)
  if (v.arith == HE_ARITH_F64) {
    if (v.slab == 12 && v.logn_min == 12 && v.loge == 4) e = HE_P(ArF64, 12, 4, 12, 12);
    else if (v.slab == 12 && v.logn_min == 12) e = HE_P(ArF64, 12, 5, 12, 12);
    else if (v.slab == 13 && v.logn_min == 13 && v.loge == 4) e = HE_P(ArF64, 13, 4, 13, 13);
    else if (v.slab == 13 && v.logn_min == 13) e = HE_P(ArF64, 13, 5, 13, 13);
    else if (v.slab == 14 && v.logn_min == 14 && v.loge == 4) e = HE_P(ArF64, 14, 4, 14, 14);
    else if (v.slab == 14 && v.logn_min == 14) e = HE_P(ArF64, 14, 5, 14, 14);
    else if (v.slab == 13) e = HE_P(ArF64, 13, 4, 10, 13);
    else e = HE_P(ArF64, 14, 4, 10, 14);
  } else {
    e = v.slab == 13 ? HE_P(ArU64, 13, 4, 10, 13) : HE_P(ArU64, 14, 4, 10, 14);
  }
#undef HE_P
  if (e != hipSuccess) return e;
  if (ev1 && (e = hipEventRecord(ev1, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_edge_fence, dim3(64), dim3(64), 0, st, 1);
  return hipGetLastError();
}

}  // namespace he
