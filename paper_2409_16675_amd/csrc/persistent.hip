// Persistent fused batch kernel: many layers (jobs) of different ring degrees
// and shapes in one launch.
//
// The host builds a task table: for every job, forward-transform tasks for its
// input ciphertext planes and pack-lift-transform tasks for its plaintext
// planes ("pre" tasks), then, after all pre tasks of all jobs, one
// multiply-accumulate + inverse-transform task per output plane group.  A grid
// of one 1024-thread workgroup per compute unit drains the table through an
// atomic counter.  Each workgroup owns 16384 coefficients of LDS per task: one
// plane at N = 16384, two at N = 8192, four at N = 4096 (every thread always
// holds 16 coefficients, so the register budget does not depend on N).
//
// A multiply-accumulate task of job j waits until every pre task of job j has
// finished (per-job counter, release/acquire at agent scope).  Because every
// pre task precedes every multiply-accumulate task in the table, a waiting
// task only waits on tasks already taken by running workgroups, so the wait
// always ends; it is also bounded by a spin limit that raises an error flag.
#include "batch.hpp"
#include "ntt.hpp"

namespace he {

// s_waitcnt immediate for gfx9-family: vmcnt = 0, expcnt and lgkmcnt left at their maxima
constexpr int kWaitVmcnt0 = 0x0F70;

template <class A>
struct PTw;
template <>
struct PTw<ArF64> {
  __device__ static const TwF64 *fwd(const PJob &j) { return (const TwF64 *)j.tw_fwd; }
  __device__ static const TwF64 *inv(const PJob &j) { return (const TwF64 *)j.tw_inv; }
};
template <>
struct PTw<ArU64> {
  __device__ static const TwU64 *fwd(const PJob &j) { return (const TwU64 *)j.tw_fwd; }
  __device__ static const TwU64 *inv(const PJob &j) { return (const TwU64 *)j.tw_inv; }
};

template <class A>
struct PMac;
template <>
struct PMac<ArF64> {
  static constexpr int kChunk = 8;
  double acc = 0.0;
  __device__ __forceinline__ void add(const ArF64 &ar, uint64_t a, uint64_t b) { acc += ar.mulv((double)a, (double)b); }
  __device__ __forceinline__ void fold(const ArF64 &ar, const PrimeK &) { acc = ar.reduce(acc); }
  __device__ __forceinline__ double value() const { return acc; }
};
template <>
struct PMac<ArU64> {
  static constexpr int kChunk = 15;
  uint64_t lo = 0, hi = 0;
  __device__ __forceinline__ void add(const ArU64 &, uint64_t a, uint64_t b) {
    const uint64_t pl = a * b, ph = __umul64hi(a, b);
    const uint64_t nl = lo + pl;
    hi += ph + (nl < lo ? 1u : 0u);
    lo = nl;
  }
  __device__ __forceinline__ void fold(const ArU64 &ar, const PrimeK &pk) {
    uint64_t x = ar.mul(hi, pk.r64, pk.r64s) + ar.mul(lo, 1, pk.one_s);
    x = x >= ar.two_q ? x - ar.two_q : x;
    x = x >= ar.q ? x - ar.q : x;
    lo = x;
    hi = 0;
  }
  __device__ __forceinline__ uint64_t value() const { return lo; }
};

// One task on one plane group member.  G: geometry with E = 16.  `valid` is
// false for a group member past the end of the task's plane range: it runs
// the same barriers but reads zeros and stores nothing.
template <class A, int LOGN, int LOGE>
__device__ __forceinline__ void run_task(const PTask &tk, const PJob &jb, int tid_g, int group,
                                         typename A::V *lds_g) {
  using G = Geo<LOGN, LOGN - LOGE>;
  using V = typename A::V;
  const uint32_t plane = tk.first + (uint32_t)group;
  const bool valid = plane < tk.first + tk.count;
  const uint32_t L = jb.L;
  const uint32_t i = valid ? plane % L : 0;
  const PrimeK pk = jb.primes[i];
  const A ar(pk);
  if (tk.kind == PT_FWD_CT) {
    const uint64_t *src = jb.ct_in + (size_t)plane * G::N;
    uint64_t *dst = jb.ct_hat + (size_t)plane * G::N;
    auto ld = [&](int k) { return ar.load(valid ? src[k] : 0ull); };
    auto st = [&](int k, uint64_t v) {
      if (valid) dst[k] = v;
    };
    ntt_forward<A, G>(ar, PTw<A>::fwd(jb) + (size_t)i * G::N, tid_g, lds_g, ld, st);
  } else if (tk.kind == PT_PT) {
    const uint32_t pp = valid ? plane / L : 0;
    uint64_t *dst = jb.pt_hat + (size_t)plane * G::N;
    auto st = [&](int k, uint64_t v) {
      if (valid) dst[k] = v;
    };
    if (jb.pkind == PK_POLY) {
      const int64_t *src = (const int64_t *)jb.plain + (size_t)pp * G::N;
      auto ld = [&](int k) { return ar.load_signed(valid ? src[k] : 0ll); };
      ntt_forward<A, G>(ar, PTw<A>::fwd(jb) + (size_t)i * G::N, tid_g, lds_g, ld, st);
    } else {
      // pack in LDS: zero, scatter this polynomial's weights, then transform from LDS
#pragma unroll
      for (int j = 0; j < G::E; ++j) lds_g[lpad(j * G::NT + tid_g)] = ar.load(0ull);
      __syncthreads();
      const int32_t *w = (const int32_t *)jb.plain;
      if (valid) {
        if (jb.pkind == PK_CONV) {
          const uint32_t m = pp / jb.cb, blk = pp % jb.cb, hh = jb.h * jb.h;
          const uint32_t c0 = blk * jb.Cw, c1 = min(jb.C, c0 + jb.Cw);
          const uint32_t n = (c1 - c0) * hh;
          for (uint32_t id = tid_g; id < n; id += G::NT) {
            const uint32_t cc = id / hh, ab = id % hh, a = ab / jb.h, b = ab % jb.h;
            const int64_t v = w[((size_t)m * jb.C + c0 + cc) * hh + ab];
            const uint32_t pos = (jb.h - 1 - a) * jb.O + (jb.h - 1 - b);
            if (cc == 0) lds_g[lpad(pos)] = ar.load_signed(v);
            else lds_g[lpad(G::N - cc * jb.S + pos)] = ar.load_signed(-v);
          }
        } else {   // PK_FC: poly (ko, ki) holds W[ko*n_ow + ii][ki*n_iw + jj] at ii*n_iw + n_iw-1-jj
          const uint32_t ko = pp / jb.in_ct, ki = pp % jb.in_ct;
          const uint32_t i0 = ko * jb.n_ow, i1 = min(jb.n_out, i0 + jb.n_ow);
          const uint32_t j0 = ki * jb.n_iw, j1 = min(jb.n_in, j0 + jb.n_iw);
          const uint32_t wi = j1 - j0, n = (i1 - i0) * wi;
          for (uint32_t id = tid_g; id < n; id += G::NT) {
            const uint32_t ii = id / wi, jj = id % wi;
            const int64_t v = w[(size_t)(i0 + ii) * jb.n_in + j0 + jj];
            lds_g[lpad(ii * jb.n_iw + jb.n_iw - 1 - jj)] = ar.load_signed(v);
          }
        }
      }
      __syncthreads();
      auto ld = [&](int k) { return lds_g[lpad(k)]; };
      ntt_forward<A, G>(ar, PTw<A>::fwd(jb) + (size_t)i * G::N, tid_g, lds_g, ld, st);
    }
  } else {   // PT_MAC_INV: output plane (o, comp, i)
    const uint32_t comp = (plane / L) & 1, o = plane / (2 * L);
    int t0 = 0, t1 = 0;
    if (valid) {
      t0 = jb.row[o];
      t1 = jb.row[o + 1];
    }
    PMac<A> acc[G::E];
    for (int t = t0; t < t1; t += PMac<A>::kChunk) {
      const int te = min(t + PMac<A>::kChunk, t1);
      for (int tt = t; tt < te; ++tt) {
        const uint64_t *a = jb.ct_hat + ((size_t)(jb.cti[tt] * 2 + comp) * L + i) * G::N;
        const uint64_t *b = jb.pt_hat + ((size_t)jb.pti[tt] * L + i) * G::N;
#pragma unroll
        for (int j = 0; j < G::E; ++j) {
          const int k = j * G::NT + tid_g;
          acc[j].add(ar, a[k], b[k]);
        }
      }
#pragma unroll
      for (int j = 0; j < G::E; ++j) acc[j].fold(ar, pk);
    }
#pragma unroll
    for (int j = 0; j < G::E; ++j) lds_g[lpad(j * G::NT + tid_g)] = acc[j].value();
    uint64_t *dst = jb.ct_out + (size_t)plane * G::N;
    const uint64_t q = pk.q;
    const bool accum = jb.accumulate != 0;
    auto st = [&](int k, uint64_t v) {
      if (!valid) return;
      if (accum) {
        const uint64_t s = dst[k] + v;
        dst[k] = s >= q ? s - q : s;
      } else {
        dst[k] = v;
      }
    };
    ntt_inverse_from_lds<A, G, 51>(ar, PTw<A>::inv(jb) + (size_t)i * G::N, tid_g, lds_g, st);
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
  static constexpr int NT = 1 << (SLAB - LOGE);
  static constexpr int LDS_BYTES = ((1 << SLAB) + (1 << (SLAB - 5))) * 8;
  static constexpr int WG_PER_CU = (163840 / (LDS_BYTES + 512)) < 1 ? 1 : (163840 / (LDS_BYTES + 512));
  static constexpr int MINW = (WG_PER_CU * NT / 256) < 1 ? 1 : (WG_PER_CU * NT / 256 > 8 ? 8 : WG_PER_CU * NT / 256);
};

template <class A, int SLAB, int LOGE, int LOGN_MIN, int LOGN_MAX>
__global__ __launch_bounds__((PCfg<A, SLAB, LOGE, LOGN_MIN, LOGN_MAX>::NT),
                             (PCfg<A, SLAB, LOGE, LOGN_MIN, LOGN_MAX>::MINW)) void k_persistent(
    const PTask *__restrict__ tasks, uint32_t n_tasks, const PJob *__restrict__ jobs, uint32_t n_jobs,
    uint32_t *__restrict__ ctl, uint32_t spin_limit, uint32_t strict) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t s_task, s_wait;
  __shared__ uint32_t s_ready[64];   // acquired jobs (bitmap, jobs < 2048); touched by thread 0 only
  typename A::V *lds = reinterpret_cast<typename A::V *>(smem);
  const int tid = threadIdx.x;
  uint32_t *head = ctl + CTL_HEAD, *err = ctl + CTL_ERR, *done = ctl + CTL_DONE;
  if (tid == 0)
    for (int k = 0; k < 64; ++k) s_ready[k] = 0u;
  // (The caches are invalidated before the launch and written back after it by
  // k_edge_fence, see launch_persistent.)
  // thread 0 keeps the index of the following task in flight while the current
  // one runs, so the queue atomic's latency is hidden
  uint32_t next = 0;
  if (tid == 0) next = atomicAdd(head, 1u);
  for (;;) {
    // thread 0 takes the next task and decides, for the whole workgroup, whether
    // it must wait for the job's pre tasks (so every thread takes the same branch)
    if (tid == 0) {
      const uint32_t t0 = next;
      if (t0 < n_tasks) next = atomicAdd(head, 1u);
      uint32_t w = 0;
      if (t0 < n_tasks) {
        const PTask k0 = tasks[t0];
        if (k0.kind == PT_MAC_INV && jobs[k0.job].n_pre)
          w = (!(strict & 1u) && k0.job < 2048 && ((s_ready[k0.job >> 5] >> (k0.job & 31)) & 1u)) ? 0u : 1u;
      }
      s_task = t0;
      s_wait = w;
    }
    __syncthreads();
    const uint32_t t = s_task;
    const uint32_t must_wait = s_wait;
    __syncthreads();
    if (t >= n_tasks) break;
    const PTask tk = tasks[t];
    const PJob &jb = jobs[tk.job];
    if (must_wait) {
      if (tid == 0) {
        uint32_t spins = 0;
        while (__hip_atomic_load(done + tk.job, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < jb.n_pre) {
          __builtin_amdgcn_s_sleep(2);
          if (++spins > spin_limit) {
            atomicOr(err, 1u);
            break;
          }
        }
        if (strict & 4u) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        else __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (tk.job < 2048) s_ready[tk.job >> 5] |= 1u << (tk.job & 31);
      }
      __syncthreads();
      if (strict & 1u) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    const int logn = (int)jb.logN;
    const int logt = logn - LOGE;
    const int group = tid >> logt;
    const int tid_g = tid & ((1 << logt) - 1);
    const int words = (1 << logn) + (1 << (logn - 5));
    typename A::V *lds_g = lds + (size_t)group * words;
    if constexpr (LOGN_MIN == LOGN_MAX) {
      run_task<A, LOGN_MIN, LOGE>(tk, jb, tid_g, group, lds_g);
    } else {
      switch (logn) {
        case 10: if constexpr (LOGN_MIN <= 10) run_task<A, 10, LOGE>(tk, jb, tid_g, group, lds_g); break;
        case 11: if constexpr (LOGN_MIN <= 11) run_task<A, 11, LOGE>(tk, jb, tid_g, group, lds_g); break;
        case 12: run_task<A, 12, LOGE>(tk, jb, tid_g, group, lds_g); break;
        case 13: run_task<A, 13, LOGE>(tk, jb, tid_g, group, lds_g); break;
        default:
          if constexpr (LOGN_MAX >= 14) run_task<A, 14, LOGE>(tk, jb, tid_g, group, lds_g);
          break;
      }
    }
    if (tk.kind != PT_MAC_INV) {
      // every wave waits until its own global stores have reached L2 (the barrier
      // alone orders LDS only); thread 0's release then writes L2 back and publishes
      __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
      if (strict & 1u) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    }
    __syncthreads();
    if (tk.kind != PT_MAC_INV && tid == 0)
      __hip_atomic_fetch_add(done + tk.job, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Zero the queue head, the error flag and the per-job counters (a kernel, not a
// memset, so that the launch can be captured into a graph and replayed).
__global__ void k_reset_ctl(uint32_t *ctl, uint32_t n_words) {
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n_words; k += gridDim.x * blockDim.x) ctl[k] = 0u;
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
static hipError_t launch_p(const PTask *tasks, uint32_t n_tasks, const PJob *jobs, uint32_t n_jobs, uint32_t *ctl,
                           uint32_t grid, uint32_t spin_limit, uint32_t strict, hipStream_t st) {
  using C = PCfg<A, SLAB, LOGE, LOGN_MIN, LOGN_MAX>;
  static bool set = false;
  if (!set) {
    hipError_t e = hipFuncSetAttribute((const void *)k_persistent<A, SLAB, LOGE, LOGN_MIN, LOGN_MAX>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, C::LDS_BYTES);
    if (e != hipSuccess) return e;
    set = true;
  }
  hipLaunchKernelGGL((k_persistent<A, SLAB, LOGE, LOGN_MIN, LOGN_MAX>), dim3(grid), dim3(C::NT), C::LDS_BYTES, st,
                     tasks, n_tasks, jobs, n_jobs, ctl, spin_limit, strict);
  return hipGetLastError();
}

// Variants compiled: F64 single-degree 4096/8192/16384 with 32 coefficients per
// thread, and mixed-degree variants (16 per thread) for both arithmetics.
bool persistent_variant(int arith, uint32_t logn_min, uint32_t logn_max, PVariant &v) {
  if (arith == HE_ARITH_F64 && logn_min == logn_max && logn_min >= 12 && logn_min <= 14) {
    v = PVariant{arith, (int)logn_min, 5, (int)logn_min, (int)logn_min};
  } else if (logn_max <= 13) {
    v = PVariant{arith, 13, 4, 10, 13};
  } else {
    v = PVariant{arith, 14, 4, 10, 14};
  }
  v.threads = 1 << (v.slab - v.loge);
  v.lds_bytes = ((1 << v.slab) + (1 << (v.slab - 5))) * 8;
  v.wg_per_cu = 163840 / (v.lds_bytes + 512);
  if (v.wg_per_cu < 1) v.wg_per_cu = 1;
  return true;
}

hipError_t launch_persistent(const PVariant &v, const PTask *tasks, uint32_t n_tasks, const PJob *jobs,
                             uint32_t n_jobs, uint32_t *ctl, uint32_t ctl_words, uint32_t grid, uint32_t spin_limit,
                             uint32_t strict, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_ctl, dim3(1), dim3(256), 0, st, ctl, ctl_words);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (!(strict & 8u)) {
    hipLaunchKernelGGL(k_edge_fence, dim3(64), dim3(64), 0, st, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
#define HE_P(A, S, E, MN, MX) launch_p<A, S, E, MN, MX>(tasks, n_tasks, jobs, n_jobs, ctl, grid, spin_limit, strict, st)
  if (v.arith == HE_ARITH_F64) {
    if (v.slab == 12 && v.loge == 5) e = HE_P(ArF64, 12, 5, 12, 12);
    else if (v.slab == 13 && v.loge == 5) e = HE_P(ArF64, 13, 5, 13, 13);
    else if (v.slab == 14 && v.loge == 5) e = HE_P(ArF64, 14, 5, 14, 14);
    else if (v.slab == 13) e = HE_P(ArF64, 13, 4, 10, 13);
    else e = HE_P(ArF64, 14, 4, 10, 14);
  } else {
    e = v.slab == 13 ? HE_P(ArU64, 13, 4, 10, 13) : HE_P(ArU64, 14, 4, 10, 14);
  }
#undef HE_P
  if (e != hipSuccess) return e;
  if (!(strict & 8u)) {
    hipLaunchKernelGGL(k_edge_fence, dim3(64), dim3(64), 0, st, 1);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace he
