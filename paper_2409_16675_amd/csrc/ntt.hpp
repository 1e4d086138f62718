// Negacyclic number-theoretic transform of one plane per workgroup, gfx950.
//
// Forward: Cooley-Tukey butterflies with the powers of psi merged into the
// twiddles (table entry k = psi^brv(k)), natural-order input, bit-reversed
// output, so slot k holds a(psi^(2 brv(k) + 1)).  Inverse: Gentleman-Sande
// butterflies with psi^-1 powers in the same order, N^-1 folded into the last
// stage (table entries 0 and 1), bit-reversed input, natural output.
//
// Work split: a plane of N = 2^LOGN coefficients is held by NT = 2^LOGT
// threads, E = N / NT coefficients each in registers.  The LOGN stages are
// cut into passes of at most LOGE = log2 E stages (PassSplit).  In a pass with first
// stage S0 and R stages the index bits are [S0 high bits | R pass bits | rest]
// and each thread owns whole radix-2^R groups (the pass bits live in the
// register index), so a pass needs no communication; between passes the
// plane goes through LDS (padded by one word every 16 to spread banks).  The
// first and last passes touch HBM (or the producer's registers) directly: the
// first forward and last inverse pass map the thread index to the low index
// bits, and the last forward and first inverse pass have no low index bits
// (each thread holds runs of 2^R consecutive coefficients, adjacent across
// threads), so all four are coalesced and only the passes in between
// exchange through LDS (the last forward pass stores directly only for runs
// of at most 4, see ntt_forward_tc).
#pragma once
#include <type_traits>
#include "arith.hpp"

namespace he {

constexpr int kLdsPadShift = 4;

// Stage counts of the passes.  The first pass takes LOGE stages (it reads or
// writes HBM directly); the rest, with the fewest passes, are sized so that as
// few twiddle entries as possible go through vector memory.  A pass of R stages
// needs E - E / 2^R entries per thread, and they are the same across a wave
// (scalar loads, see PassTw) when its low index bits cover the lane bits:
// LOGN - S0 - R >= 6 (or >= LOGT when a plane has fewer than 64 threads).  Of
// the splits with the fewest vector entries the one with the larger passes
// first is taken.
struct PassSplit {
  int n;
  int r[8];
};
constexpr void split_search(int logn, int loge, int logt, int k, int s0, int vec, PassSplit &cur, PassSplit &best,
                            int &best_vec) {
  if (k == cur.n) {
    if (s0 == logn && vec < best_vec) {
      best_vec = vec;
      best = cur;
    }
    return;
  }
  for (int r = loge; r >= 1; --r) {
    if (s0 + r > logn) continue;
    const int e = 1 << loge;
    const bool uniform = logn - s0 - r >= (logt < 6 ? logt : 6);
    cur.r[k] = r;
    split_search(logn, loge, logt, k + 1, s0 + r, vec + (uniform ? 0 : e - (e >> r)), cur, best, best_vec);
  }
}
constexpr PassSplit choose_split(int logn, int loge) {
  PassSplit cur{(logn + loge - 1) / loge, {}}, best = cur;
  cur.r[0] = loge;
  int best_vec = 1 << 30;
  split_search(logn, loge, logn - loge, 1, loge, 0, cur, best, best_vec);
  return best;
}

template <int LOGN_, int LOGT_>
struct Geo {
  static constexpr int LOGN = LOGN_, LOGT = LOGT_;
  static constexpr int N = 1 << LOGN, NT = 1 << LOGT, LOGE = LOGN - LOGT, E = 1 << LOGE;
  static constexpr int NPASS = (LOGN + LOGE - 1) / LOGE;
  static_assert(NPASS <= 8, "pass table size");
  static constexpr PassSplit split = choose_split(LOGN, LOGE);
  static constexpr int r(int k) { return split.r[k]; }
  static constexpr int s0(int k) {
    int s = 0;
    for (int j = 0; j < k; ++j) s += split.r[j];
    return s;
  }
  static_assert(s0(NPASS) == LOGN && split.r[0] == LOGE, "pass split covers the stages");
  static constexpr int LDS_WORDS = N + (N >> kLdsPadShift);
};

// LDS words of a plane are padded by one word after every 2^kLdsPadShift.
// LDS serves 16 lanes of a 64-bit access per clock over 32 four-byte banks;
// with 16 coefficients per thread every pass's pattern (for N = 2^12 .. 2^14
// and the pass splits chosen below) then spreads over all 32 banks, where a
// pad every 32 words left two of the four passes 2-way conflicted (the
// measured conflict cycles of the transforms match that count exactly).
__device__ __forceinline__ int lpad(int i) { return i + (i >> kLdsPadShift); }
__host__ __device__ constexpr int lpad_c(int i) { return i + (i >> kLdsPadShift); }
// LDS word of linear index j * NT + tid (tid < NT): the two parts have
// disjoint bits, so the padding splits (see pass_index).
template <class G>
__device__ __forceinline__ int lin_lds(int tid, int j) {
  return lpad(tid) + lpad_c(j * G::NT);
}

// Pointers read from memory (job tables) are generic; qualifying them as global
// lets the compiler use global (not flat) loads and stores, which do not tie the
// memory counters to LDS traffic.
#define HE_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ HE_GLOBAL T *as_global(T *p) {
  return (HE_GLOBAL T *)p;
}

// One twiddle entry (16 bytes) through a generic or a global pointer.  The
// byte offset is formed in 32 bits (tables are far below 4 GiB), so the load
// is a scalar base plus a lane offset.
template <class Tw>
__device__ __forceinline__ Tw load_tw(const Tw *tw, uint32_t idx) {
  return *(const Tw *)((const char *)tw + (size_t)(idx * (uint32_t)sizeof(Tw)));
}
template <class Tw>
__device__ __forceinline__ Tw load_tw(const HE_GLOBAL Tw *tw, uint32_t idx) {
  typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
  static_assert(sizeof(Tw) == sizeof(u64x2), "twiddle entries are 16 bytes");
  const u64x2 v = *(const HE_GLOBAL u64x2 *)((const HE_GLOBAL char *)tw + (size_t)(idx * (uint32_t)sizeof(Tw)));
  return __builtin_bit_cast(Tw, v);
}

// Raw buffer access: the resource holds a base address and a bound of
// `bytes`; an access adds a per-lane byte offset (a VGPR) and a scalar one (an
// SGPR or constant), so an index's compile-time part costs no vector address
// arithmetic.  The base must be the same in every lane: it is read from the
// first lane, so that the compiler, which cannot always prove it uniform, does
// not wrap each access in a loop over distinct bases.  Word 3 selects raw
// 32-bit data (gfx950).  Offsets stay below the bound here; past it the
// hardware would read zeros and drop stores.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *p, uint32_t bytes) {
  const uint64_t a = (uint64_t)(uintptr_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  void *u = (void *)(uintptr_t)(((uint64_t)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(u, (short)0, (int)bytes, 0x00020000);
}
template <class Tw>
__device__ __forceinline__ Tw load_tw_buf(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
  static_assert(sizeof(Tw) == 16, "twiddle entries are 16 bytes");
  return __builtin_bit_cast(Tw, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)voff, (int)soff, 0));
}
typedef unsigned int he_u32x2 __attribute__((ext_vector_type(2)));
typedef double he_f64x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint64_t buf_load_u64(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ he_f64x2 buf_load_f64x2(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(he_f64x2, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)voff, (int)soff, 0));
}
// a streaming store (nt: the line is not kept for reuse)
__device__ __forceinline__ void buf_store_u64_nt(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff, uint64_t x) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(he_u32x2, x), rs, (int)voff, (int)soff, 2);
}

// One twiddle entry at an index that every lane of the wave shares: the table
// base is read from the first lane and the table addressed through the
// constant address space, so the compiler reads the entry with a scalar load
// into SGPRs (no vector memory instruction and no VGPRs for it).  A wave never
// holds threads of two planes (a plane has at least 64 threads, or is the
// whole workgroup), so the base is the same in every lane.  The tables are
// written before any kernel that reads them runs.
#define HE_CONST __attribute__((address_space(4)))
template <class Tw, class TwP>
__device__ __forceinline__ Tw load_tw_uniform(TwP tw, uint32_t idx) {
  const uint64_t a = (uint64_t)(uintptr_t)tw;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
  static_assert(sizeof(Tw) == sizeof(u64x2), "twiddle entries are 16 bytes");
  const HE_CONST u64x2 *c = (const HE_CONST u64x2 *)(((uint64_t)hi << 32) | lo);
  return __builtin_bit_cast(Tw, c[idx]);
}

// Waves per SIMD two (or more) resident workgroups need, given the LDS a plane
// takes: passed as the second __launch_bounds__ argument so that the compiler
// keeps the register count low enough for that occupancy.
template <int LOGN, int LOGT>
struct MinWaves {
  static constexpr int lds = ((1 << LOGN) + (1 << (LOGN - kLdsPadShift))) * 8 + 256;
  static constexpr int wg = (163840 / lds) < 1 ? 1 : (163840 / lds);
  static constexpr int w = wg * (1 << LOGT) / 64 / 4;
  static constexpr int value = w < 1 ? 1 : (w > 8 ? 8 : w);
};

// Index of register slot (g, p) of thread tid in a pass starting at stage S0
// with R stages.  The pass's R stage bits hold the register slot p; the other
// index bits take, from the lowest up, the lane bits of tid (tid & 63), the
// group bits g, then the wave bits (tid >> 6).  So the lanes of a wave cover
// the lowest free index bits (coalesced accesses at both ends of a transform)
// and the wave bits sit on the highest free bits: every pass but the first
// leaves the top LOGE bits free (they are the first pass's stage bits), so
// when the wave bits fit there they hold the same index bits in all those
// passes, and the exchanges between them stay inside each wave (no barrier).
template <int LOGN, int LOGT, int S0, int R>
__host__ __device__ constexpr int pass_index(int tid, int g, int p) {
  constexpr int NLOW = LOGN - S0 - R;
  constexpr int LOGNG = (LOGN - LOGT) - R;   // log2 of the radix-2^R groups per thread
  int f = 0;
  if constexpr (LOGT > 6) f = (tid & 63) | (g << 6) | ((tid >> 6) << (6 + LOGNG));
  else f = (g << LOGT) | tid;
  const int low = f & ((1 << NLOW) - 1);
  const int high = f >> NLOW;
  return (high << (LOGN - S0)) | (p << NLOW) | low;
}
// pass_index only moves bits, so it splits into a per-thread part and a
// compile-time part with disjoint bits:
//   pass_index(tid, g, p) = pass_index(tid, 0, 0) + pass_index(0, g, p),
// and so does the LDS padding, lpad(a + b) = lpad(a) + lpad(b) for disjoint
// a and b (a shift distributes over a disjoint union of bits).  Loads and
// stores therefore take (t, c) = (thread part, constant part); an LDS address
// is a per-thread base plus an immediate offset.

// ---------------------------------------------------------------- bound bookkeeping
// For the lazily reduced fp64 policy: worst-case |value| / q through a pass,
// and the stages before which every register is reduced.  Integer policy
// bounds are fixed by construction (kLimit is huge), so no reduction is placed.
struct PassPlan {
  unsigned mask;   // bit u: reduce all registers before stage u
  double b_out;
};

template <class A>
constexpr PassPlan plan_ct(int R, double b_in) {
  PassPlan p{0u, b_in};
  double b = b_in;
  for (int u = 0; u < R; ++u) {
    double nb = b + A::mul_out(b);
    if (nb > A::kLimit) {
      p.mask |= 1u << u;
      b = A::kReduced;
      nb = b + A::mul_out(b);
    }
    b = nb;
  }
  p.b_out = b;
  return p;
}

template <class A>
constexpr PassPlan plan_gs(int R, double b_in) {
  PassPlan p{0u, b_in};
  double b = b_in;
  for (int u = 0; u < R; ++u) {
    double s = 2.0 * b;
    double nb = s > A::mul_out(s) ? s : A::mul_out(s);
    if (s > A::kLimit || nb > A::kLimit) {
      p.mask |= 1u << u;
      b = A::kReduced;
      s = 2.0 * b;
      nb = s > A::mul_out(s) ? s : A::mul_out(s);
    }
    b = nb;
  }
  p.b_out = b;
  return p;
}

// Inverse passes track the bound of every register slot p of a radix-2^R group:
// the Gentleman-Sande sum x + y doubles the bound of the slots whose lower pass
// bits are zero while the product side stays below mul_out, so only the
// growing slots are reduced (before a stage whose sum would leave the limit,
// and at the end of the pass when above end_red).  In the last pass (LAST,
// stages down to 0) stage 0 multiplies both outputs (N^-1 folded in), its
// sums are kept small enough that both products stay below kStoreIn (so the
// store needs no reduction, see store_out), and no slot is reduced at the end.
struct GsPlan {
  uint32_t red[6];   // red[uu]: slots reduced before stage uu; red[R]: slots reduced at the end
  double b_out;
};

template <class A>
constexpr GsPlan plan_gs_slots(int R, double b_in, bool last, double end_red, bool formed = false) {
  GsPlan pl{{0u, 0u, 0u, 0u, 0u, 0u}, b_in};
  // (formed: the pass's twiddles come without their quotient companions,
  // formed at the product, whose bound is then mulv_out)
  auto pout = [formed](double x) { return formed ? A::mulv_out(x) : A::mul_out(x); };
  double b[32] = {};
  const int n = 1 << R;
  for (int p = 0; p < n; ++p) b[p] = b_in;
  for (int uu = 0; uu < R; ++uu) {
    uint32_t m = 0;
    for (int p = 0; p < n; ++p) {
      if (p & (1 << uu)) continue;
      const int p2 = p | (1 << uu);
      double s = b[p] + b[p2];
      const bool final_stage = last && uu == R - 1;
      if (s > A::kLimit || pout(s) > A::kLimit || (final_stage && pout(s) > A::kStoreIn)) {
        m |= (1u << p) | (1u << p2);
        s = 2.0 * A::kReduced;
      }
      b[p] = final_stage ? pout(s) : s;
      b[p2] = pout(s);
    }
    pl.red[uu] = m;
  }
  uint32_t e = 0;
  double mx = 0.0;
  for (int p = 0; p < n; ++p) {
    if (!last && b[p] > end_red && A::kLimit < 100.0) {
      e |= 1u << p;
      b[p] = A::kReduced;
    }
    mx = b[p] > mx ? b[p] : mx;
  }
  pl.red[R] = e;
  pl.b_out = mx;
  return pl;
}

// Bound entering forward pass k (passes run 0, 1, ..., each starting from the previous output).
template <class A, class G>
constexpr double fwd_bound_in(int k) {
  double b = A::kCanon;
  for (int j = 0; j < k; ++j) b = plan_ct<A>(G::r(j), b).b_out;
  return b;
}
// Inverse passes run k = NPASS-1 down to 0; the input is canonical (or a reduced accumulator).
// WMASK: bit k set when pass k forms its twiddles' quotient companions.
template <class A, class G, int WMASK = 0>
constexpr double inv_bound_in(int k, double b0, double end_red) {
  double b = b0;
  for (int j = G::NPASS - 1; j > k; --j) b = plan_gs_slots<A>(G::r(j), b, j == 0, end_red, (WMASK >> j) & 1).b_out;
  return b;
}
// Reductions per thread over a whole inverse transform, and the end-of-pass
// threshold (in units of q) that needs the fewest for this geometry and input
// bound: a low threshold reduces more at pass ends, a high one more inside
// the next pass.
template <class A, class G, int WMASK = 0>
constexpr int inv_reductions(double b0, double end_red) {
  int tot = 0;
  double b = b0;
  for (int j = G::NPASS - 1; j >= 0; --j) {
    const GsPlan p = plan_gs_slots<A>(G::r(j), b, j == 0, end_red, (WMASK >> j) & 1);
    int c = 0;
    for (int u = 0; u <= G::r(j); ++u) c += __builtin_popcount(p.red[u]);
    tot += c * (G::E >> G::r(j));
    b = p.b_out;
  }
  return tot;
}
template <class A, class G, int WMASK = 0>
constexpr double inv_end_red(double b0) {
  constexpr double cands[] = {2.0, 2.5, 3.0, 3.5, 4.0};
  double best = cands[0];
  int best_n = inv_reductions<A, G, WMASK>(b0, cands[0]);
  for (double c : cands) {
    const int n = inv_reductions<A, G, WMASK>(b0, c);
    if (n < best_n) {
      best_n = n;
      best = c;
    }
  }
  return best;
}

// ------------------------------------------------------------------- butterflies
template <class A>
__device__ __forceinline__ void gs_bfly(const A &ar, typename A::V &x, typename A::V &y, typename A::Tw w);

template <>
__device__ __forceinline__ void gs_bfly<ArF64>(const ArF64 &ar, double &x, double &y, TwF64 w) {
  double d = x - y;
  x = x + y;
  y = ar.mul(d, w);
}
template <>
__device__ __forceinline__ void gs_bfly<ArU64>(const ArU64 &ar, uint64_t &x, uint64_t &y, TwU64 w) {
  // x, y in [0, 2q) -> x + y in [0, 2q), (x - y) w in [0, 2q)
  uint64_t s = x + y;
  s = s >= ar.two_q ? s - ar.two_q : s;
  uint64_t d = x - y + ar.two_q;
  y = ar.mul(d, w);
  x = s;
}
// Last inverse stage with N^-1 folded in: x' = (x + y) n, y' = (x - y) (w n).
template <class A>
__device__ __forceinline__ void gs_last(const A &ar, typename A::V &x, typename A::V &y, typename A::Tw n,
                                        typename A::Tw wn);
template <>
__device__ __forceinline__ void gs_last<ArF64>(const ArF64 &ar, double &x, double &y, TwF64 n, TwF64 wn) {
  double d = x - y;
  double s = x + y;
  x = ar.mul(s, n);
  y = ar.mul(d, wn);
}
template <>
__device__ __forceinline__ void gs_last<ArU64>(const ArU64 &ar, uint64_t &x, uint64_t &y, TwU64 n, TwU64 wn) {
  uint64_t s = x + y;               // < 4q < 2^64
  uint64_t d = x - y + ar.two_q;    // < 4q
  x = ar.mul(s, n);
  y = ar.mul(d, wn);
}

// The same with the twiddle alone (fp64): its quotient companion is formed
// at the product (mulv), whose bound is mulv_out.
__device__ __forceinline__ void gs_bfly_formed(const ArF64 &ar, double &x, double &y, double w) {
  double d = x - y;
  x = x + y;
  y = ar.mulv(d, w);
}

template <class A>
__device__ __forceinline__ typename A::V reduce_gs_in(const A &ar, typename A::V v) {
  return ar.reduce(v);
}

// ------------------------------------------------------------------------ passes
// Twiddles of pass K held in registers.  Stage u (of R) of the pass needs the
// 2^u entries (1 << (S0 + u)) + (high << u) + j, j < 2^u, kept in slot
// (1 << u) - 1 + j; an inverse pass starting at stage 0 also needs entries 0
// and 1 (N^-1 folded in).  A pass's twiddles are loaded while the previous pass
// is still running (between its arithmetic and its stores), so their latency
// overlaps the stores, the barrier and the data loads.
// Bits of tid (below `limit`) that pass K places above its stage bits.
template <class G, int K>
constexpr int thread_bits_above(int limit) {
  constexpr int S0 = G::s0(K), R = G::r(K), NLOW = G::LOGN - S0 - R;
  int m = 0;
  for (int b = 0; b < limit && b < G::LOGT; ++b)
    m |= pass_index<G::LOGN, G::LOGT, S0, R>(1 << b, 0, 0) >> (NLOW + R);
  return m;
}

// W: the entries are the twiddles alone (8 bytes, from a table without the
// quotient companions; only for passes whose lanes read different entries,
// fp64): half the bytes and registers, the companion formed at the product.
template <class A, class G, int K, bool INV, bool W = false>
struct PassTw {
  static constexpr int S0 = G::s0(K), R = G::r(K), NG = G::E >> R, NLOW = G::LOGN - S0 - R;
  static constexpr bool kW = W;
  std::conditional_t<W, double, typename A::Tw> w[NG][(1 << R) - 1];
  typename A::Tw n0, n1;
  // the index bits above the stage bits ("high") select a group's entries
  static constexpr bool kPlaneUniform = thread_bits_above<G, K>(G::LOGT) == 0;
  static constexpr bool kWaveUniform = thread_bits_above<G, K>(6) == 0;
  static_assert(!W || (!kWaveUniform && std::is_same<A, ArF64>::value), "twiddles alone: per-lane fp64 passes only");
  // the entries of this pass from the paired table tw, or from the table of
  // twiddles alone tww when W
  template <class TwP>
  __device__ __forceinline__ void load2(TwP tw, const double *tww, int tid) {
    if constexpr (W) {
      const auto rs = buf_rsrc((const void *)tww, (uint32_t)(G::N * 8));
      const uint32_t high_t = (uint32_t)pass_index<G::LOGN, G::LOGT, S0, R>(tid, 0, 0) >> (NLOW + R);
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        const uint32_t high_g = (uint32_t)pass_index<G::LOGN, G::LOGT, S0, R>(0, g, 0) >> (NLOW + R);
        // stage S0: one entry; a later stage's entries of one group are
        // consecutive, two to a 16-byte load (fewer vector memory
        // instructions, which measured faster than one load per entry)
        w[g][0] = __builtin_bit_cast(double, buf_load_u64(rs, high_t * 8u, ((1u << S0) + high_g) * 8u));
#pragma unroll
        for (int u = 1; u < R; ++u) {
          const uint32_t vo = (high_t << u) * 8u;
#pragma unroll
          for (int j = 0; j < (1 << u); j += 2) {
            const he_f64x2 x = buf_load_f64x2(rs, vo, ((1u << (S0 + u)) + (high_g << u) + (uint32_t)j) * 8u);
            w[g][(1 << u) - 1 + j] = x.x;
            w[g][(1 << u) + j] = x.y;
          }
        }
      }
    } else {
      load(tw, tid);
    }
  }
  template <class TwP>
  __device__ __forceinline__ void load(TwP tw, int tid) {
    static_assert(!W, "use load2");
    using Tw = typename A::Tw;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const uint32_t high_g = (uint32_t)pass_index<G::LOGN, G::LOGT, S0, R>(0, g, 0) >> (NLOW + R);
      if constexpr (kPlaneUniform) {
        // the high index bits hold no thread bits: the same entries for the whole plane
        const uint32_t high = high_g;
#pragma unroll
        for (int u = 0; u < R; ++u)
#pragma unroll
          for (int j = 0; j < (1 << u); ++j)
            w[g][(1 << u) - 1 + j] = load_tw_uniform<Tw>(tw, (1u << (S0 + u)) + (high << u) + (uint32_t)j);
      } else if constexpr (kWaveUniform) {
        // the thread bits in the high index bits are wave bits (tid >> 6):
        // the same entries across each wave
        const uint32_t high =
            __builtin_amdgcn_readfirstlane((uint32_t)pass_index<G::LOGN, G::LOGT, S0, R>(tid, 0, 0) >> (NLOW + R)) |
            high_g;
#pragma unroll
        for (int u = 0; u < R; ++u)
#pragma unroll
          for (int j = 0; j < (1 << u); ++j)
            w[g][(1 << u) - 1 + j] = load_tw_uniform<Tw>(tw, (1u << (S0 + u)) + (high << u) + (uint32_t)j);
      } else {
        // entries differ across the lanes: the thread's part of the index
        // (shifted per stage) is the lane offset, the compile-time part (stage,
        // group, entry) the scalar offset of a buffer load, so the addresses
        // cost no per-entry vector arithmetic (the two parts have disjoint
        // bits, see pass_index)
        const auto rs = buf_rsrc((const void *)tw, (uint32_t)(G::N * sizeof(Tw)));
        const uint32_t high_t = (uint32_t)pass_index<G::LOGN, G::LOGT, S0, R>(tid, 0, 0) >> (NLOW + R);
#pragma unroll
        for (int u = 0; u < R; ++u) {
          const uint32_t vo = (high_t << u) * (uint32_t)sizeof(Tw);
#pragma unroll
          for (int j = 0; j < (1 << u); ++j)
            w[g][(1 << u) - 1 + j] =
                load_tw_buf<Tw>(rs, vo, ((1u << (S0 + u)) + (high_g << u) + (uint32_t)j) * (uint32_t)sizeof(Tw));
        }
      }
    }
    if constexpr (INV && S0 == 0) {
      n0 = load_tw_uniform<Tw>(tw, 0);
      n1 = load_tw_uniform<Tw>(tw, 1);
    }
  }
};

// Forward pass K.  ld(t, c) yields the value at plane index t + c, st(t, c, v)
// stores it (t: thread part, c: compile-time part, see pass_index); mid() runs
// after the arithmetic and before the stores.
template <class A, class G, int K, class Ld, class St, class Mid>
__device__ __forceinline__ void fwd_pass(const A &ar, const PassTw<A, G, K, false> &twr, int tid, Ld ld, St st,
                                         Mid mid) {
  using V = typename A::V;
  constexpr int S0 = G::s0(K), R = G::r(K), NG = G::E >> R;
  constexpr PassPlan pp = plan_ct<A>(R, fwd_bound_in<A, G>(K));
  static_assert(pp.b_out <= A::kLimit + 1e-9, "fp64 bound exceeded");
  const int t = pass_index<G::LOGN, G::LOGT, S0, R>(tid, 0, 0);
  V v[G::E];
#pragma unroll
  for (int g = 0; g < NG; ++g)
#pragma unroll
    for (int p = 0; p < (1 << R); ++p) v[(g << R) | p] = ld(t, pass_index<G::LOGN, G::LOGT, S0, R>(0, g, p));
#pragma unroll
  for (int u = 0; u < R; ++u) {
    if ((pp.mask >> u) & 1u) {
#pragma unroll
      for (int e = 0; e < G::E; ++e) v[e] = ar.reduce(v[e]);
    }
#pragma unroll
    for (int g = 0; g < NG; ++g) {
#pragma unroll
      for (int p = 0; p < (1 << R); ++p) {
        if (p & (1 << (R - 1 - u))) continue;
        const int p2 = p | (1 << (R - 1 - u));
        ar.ct(v[(g << R) | p], v[(g << R) | p2], twr.w[g][(1 << u) - 1 + (p >> (R - u))]);
      }
    }
  }
  mid();
#pragma unroll
  for (int g = 0; g < NG; ++g)
#pragma unroll
    for (int p = 0; p < (1 << R); ++p) st(t, pass_index<G::LOGN, G::LOGT, S0, R>(0, g, p), v[(g << R) | p]);
}

// Coefficient index of register slot e = (g << R) | p of thread tid in pass K.
template <class G, int K>
__device__ __forceinline__ uint32_t slot_index(int tid, int e) {
  constexpr int S0 = G::s0(K), R = G::r(K);
  return (uint32_t)pass_index<G::LOGN, G::LOGT, S0, R>(tid, 0, 0) +
         (uint32_t)pass_index<G::LOGN, G::LOGT, S0, R>(0, e >> R, e & ((1 << R) - 1));
}

// Inverse pass K (stages S0+R-1 down to S0) on values already in registers
// (slot e holds coefficient slot_index<G, K>(tid, e)).  B0 is the bound of the
// transform's input; WMASK bit k marks the passes with twiddles alone.
template <int WMASK, int K>
constexpr bool wbit() {
  return ((WMASK >> K) & 1) != 0;
}
template <class A, class G, int K, int B0X100, int WMASK = 0, class St, class Mid>
__device__ __forceinline__ void inv_pass_v(const A &ar, const PassTw<A, G, K, true, wbit<WMASK, K>()> &twr, int tid,
                                           typename A::V (&v)[G::E], St st, Mid mid) {
  constexpr int S0 = G::s0(K), R = G::r(K), NG = G::E >> R;
  constexpr double end_red = inv_end_red<A, G, WMASK>(B0X100 / 100.0);
  constexpr GsPlan pp = plan_gs_slots<A>(R, inv_bound_in<A, G, WMASK>(K, B0X100 / 100.0, end_red), K == 0, end_red,
                                         wbit<WMASK, K>());
  static_assert(pp.b_out <= A::kLimit + 1e-9, "fp64 bound exceeded");
  const int t = pass_index<G::LOGN, G::LOGT, S0, R>(tid, 0, 0);
#pragma unroll
  for (int uu = 0; uu < R; ++uu) {
    const int u = R - 1 - uu;   // stage S0 + u, processed from the highest down
#pragma unroll
    for (int e = 0; e < G::E; ++e)
      if ((pp.red[uu] >> (e & ((1 << R) - 1))) & 1u) v[e] = ar.reduce(v[e]);
    const int s = S0 + u;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
#pragma unroll
      for (int p = 0; p < (1 << R); ++p) {
        if (p & (1 << (R - 1 - u))) continue;
        const int p2 = p | (1 << (R - 1 - u));
        if (s == 0) {
          gs_last<A>(ar, v[(g << R) | p], v[(g << R) | p2], twr.n0, twr.n1);
        } else if constexpr (wbit<WMASK, K>()) {
          gs_bfly_formed(ar, v[(g << R) | p], v[(g << R) | p2], twr.w[g][(1 << u) - 1 + (p >> (R - u))]);
        } else {
          gs_bfly<A>(ar, v[(g << R) | p], v[(g << R) | p2], twr.w[g][(1 << u) - 1 + (p >> (R - u))]);
        }
      }
    }
  }
#pragma unroll
  for (int e = 0; e < G::E; ++e)
    if ((pp.red[R] >> (e & ((1 << R) - 1))) & 1u) v[e] = ar.reduce(v[e]);
  mid();
#pragma unroll
  for (int g = 0; g < NG; ++g)
#pragma unroll
    for (int p = 0; p < (1 << R); ++p) st(t, pass_index<G::LOGN, G::LOGT, S0, R>(0, g, p), v[(g << R) | p]);
}

// Inverse pass K reading its input through ld(t, c).
template <class A, class G, int K, int B0X100, int WMASK = 0, class Ld, class St, class Mid>
__device__ __forceinline__ void inv_pass(const A &ar, const PassTw<A, G, K, true, wbit<WMASK, K>()> &twr, int tid, Ld ld,
                                         St st, Mid mid) {
  constexpr int S0 = G::s0(K), R = G::r(K), NG = G::E >> R;
  const int t = pass_index<G::LOGN, G::LOGT, S0, R>(tid, 0, 0);
  typename A::V v[G::E];
#pragma unroll
  for (int g = 0; g < NG; ++g)
#pragma unroll
    for (int p = 0; p < (1 << R); ++p) v[(g << R) | p] = ld(t, pass_index<G::LOGN, G::LOGT, S0, R>(0, g, p));
  inv_pass_v<A, G, K, B0X100, WMASK>(ar, twr, tid, v, st, mid);
}

// A pass loads and stores the same thread-private set of indices, so passes
// sharing LDS need only one barrier between them.

// LDS access through the split index: per-thread base lpad(t), constant lpad(c).
template <class V>
struct LdsAt {
  V *lds;
  __device__ __forceinline__ V operator()(int t, int c) const { return lds[lpad(t) + lpad_c(c)]; }
};
template <class V>
struct LdsPut {
  V *lds;
  __device__ __forceinline__ void operator()(int t, int c, V v) const { lds[lpad(t) + lpad_c(c)] = v; }
};

// Index bits that hold the wave bits of tid in pass K (none when a plane
// fits in one wave).
template <class G, int K>
constexpr int wave_bits_at() {
  int m = 0;
  for (int b = 6; b < G::LOGT; ++b) m |= pass_index<G::LOGN, G::LOGT, G::s0(K), G::r(K)>(1 << b, 0, 0);
  return m;
}

// Between pass KA's LDS stores and pass KB's LDS loads.  When the wave bits sit
// on the same index bits in both passes, each wave reads back only slots it
// wrote itself: a wave's LDS requests are served in order, so waiting for its
// own stores to complete (lgkmcnt 0) suffices and the other waves run on.
// Otherwise the whole workgroup meets at a barrier.
template <class G, int KA, int KB>
__device__ __forceinline__ void xchg_sync() {
  if constexpr (wave_bits_at<G, KA>() == wave_bits_at<G, KB>()) {
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0); vmcnt and expcnt left at their maxima
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

// Forward passes K..NPASS-2, LDS to LDS; `cur` holds pass K's twiddles and
// `last` receives pass NPASS-1's (the last pass is run by the caller, to the
// destination).  PF: load the next pass's twiddles before this pass's stores
// (more registers live across the barrier); otherwise after the barrier.
template <class A, class G, int K, bool PF, class TwP>
__device__ __forceinline__ void fwd_lds_passes(const A &ar, TwP tw, int tid, typename A::V *lds,
                                               PassTw<A, G, K, false> &cur, PassTw<A, G, G::NPASS - 1, false> &last) {
  xchg_sync<G, K - 1, K>();
  if constexpr (!PF) cur.load(tw, tid);
  if constexpr (K + 2 < G::NPASS) {
    PassTw<A, G, K + 1, false> nxt;
    fwd_pass<A, G, K>(ar, cur, tid, LdsAt<typename A::V>{lds}, LdsPut<typename A::V>{lds}, [&] {
      if constexpr (PF) nxt.load(tw, tid);
    });
    fwd_lds_passes<A, G, K + 1, PF>(ar, tw, tid, lds, nxt, last);
  } else {
    fwd_pass<A, G, K>(ar, cur, tid, LdsAt<typename A::V>{lds}, LdsPut<typename A::V>{lds}, [&] {
      if constexpr (PF) last.load(tw, tid);
    });
  }
}

// Inverse passes K down to 1, LDS to LDS; `cur` holds pass K's twiddles and
// `last` receives pass 0's (pass 0 is run by the caller, to HBM).  tww: the
// table of twiddles alone, for the passes WMASK marks.
template <class A, class G, int K, int B0X100, bool PF, int WMASK, class TwP>
__device__ __forceinline__ void inv_lds_passes(const A &ar, TwP tw, const double *tww, int tid, typename A::V *lds,
                                               PassTw<A, G, K, true, wbit<WMASK, K>()> &cur,
                                               PassTw<A, G, 0, true> &last) {
  xchg_sync<G, K + 1, K>();
  if constexpr (!PF) cur.load2(tw, tww, tid);
  if constexpr (K > 1) {
    PassTw<A, G, K - 1, true, wbit<WMASK, K - 1>()> nxt;
    inv_pass<A, G, K, B0X100, WMASK>(ar, cur, tid, LdsAt<typename A::V>{lds}, LdsPut<typename A::V>{lds}, [&] {
      if constexpr (PF) nxt.load2(tw, tww, tid);
    });
    inv_lds_passes<A, G, K - 1, B0X100, PF, WMASK>(ar, tw, tww, tid, lds, nxt, last);
  } else {
    inv_pass<A, G, K, B0X100, WMASK>(ar, cur, tid, LdsAt<typename A::V>{lds}, LdsPut<typename A::V>{lds}, [&] {
      if constexpr (PF) last.load(tw, tid);
    });
  }
}

// Whole forward transform: ld2(t, c) reads coefficient t + c of the input
// (coalesced pass-0 order), the result is written through st(i, canonical)
// (CANON) or st(i, v) with v the policy's value (bounded by the last pass's
// b_out, not reduced: for a caller that stores its own format).
// The last pass has no low index bits: a thread's 2^R slots of a group are
// consecutive coefficients and consecutive threads hold adjacent runs.  With
// R <= 2 it writes the destination directly (no final round trip through
// LDS; a store instruction then fills at least half of each line it touches).
// With longer runs a store instruction would touch four times the lines of a
// linear store, each a quarter filled, which measured slower than the round
// trip: the pass goes to LDS and the plane is written in linear order.
// LINEAR takes that round trip at any R: for callers whose stores are written
// through to memory, where a partly filled line costs a partial write.
template <class A, class G, bool PF = true, bool CANON = true, bool LINEAR = false, class TwP, class Ld2, class St>
__device__ __forceinline__ void ntt_forward_tc(const A &ar, TwP tw, int tid, typename A::V *lds, Ld2 ld2, St st) {
  static_assert(G::NPASS >= 2, "at least two passes");
  using V = typename A::V;
  PassTw<A, G, 0, false> t0;
  t0.load(tw, tid);
  PassTw<A, G, G::NPASS - 1, false> last;
  if constexpr (G::NPASS > 2) {
    PassTw<A, G, 1, false> t1;
    fwd_pass<A, G, 0>(ar, t0, tid, ld2, LdsPut<V>{lds}, [&] {
      if constexpr (PF) t1.load(tw, tid);
    });
    fwd_lds_passes<A, G, 1, PF>(ar, tw, tid, lds, t1, last);
  } else {
    fwd_pass<A, G, 0>(ar, t0, tid, ld2, LdsPut<V>{lds}, [&] {
      if constexpr (PF) last.load(tw, tid);
    });
  }
  xchg_sync<G, G::NPASS - 2, G::NPASS - 1>();
  if constexpr (!PF) last.load(tw, tid);
  auto out = [&](int i, V v) {
    if constexpr (CANON) st(i, ar.store(v));
    else st(i, v);
  };
  if constexpr (!LINEAR && G::r(G::NPASS - 1) <= 2) {
    auto st_out = [&](int t, int c, V v) { out(t + c, v); };
    fwd_pass<A, G, G::NPASS - 1>(ar, last, tid, LdsAt<V>{lds}, st_out, [] {});
  } else {
    fwd_pass<A, G, G::NPASS - 1>(ar, last, tid, LdsAt<V>{lds}, LdsPut<V>{lds}, [] {});
    __syncthreads();
#pragma unroll
    for (int j = 0; j < G::E; ++j) out(j * G::NT + tid, lds[lin_lds<G>(tid, j)]);
  }
}
// The same with ld(i) reading coefficient i.
template <class A, class G, bool PF = true, bool CANON = true, bool LINEAR = false, class TwP, class Ld, class St>
__device__ __forceinline__ void ntt_forward(const A &ar, TwP tw, int tid, typename A::V *lds, Ld ld, St st) {
  ntt_forward_tc<A, G, PF, CANON, LINEAR>(ar, tw, tid, lds, [&](int t, int c) { return ld(t + c); }, st);
}

// The inverse passes (above pass 0) whose lanes read different twiddle
// entries: bit k for pass k, the passes that can take twiddles alone.
template <class G, int K = 1>
constexpr int lane_passes() {
  if constexpr (K >= G::NPASS) {
    return 0;
  } else {
    return (thread_bits_above<G, K>(6) != 0 ? (1 << K) : 0) | lane_passes<G, K + 1>();
  }
}

// Whole inverse transform of values v already in registers in the layout of
// its first pass (slot e holds coefficient slot_index<G, NPASS-1>(tid, e), bound
// B0X100/100 q): that pass has no low index bits, so a producer reading or
// computing the values pointwise fills it without a round trip through LDS.
// Pass 0 writes st(i, canonical) in coalesced order.  `first` holds the first
// pass's twiddles (loaded by the caller, ahead of the values).  WMASK marks
// the passes (never pass 0) whose twiddles come alone from tww.
template <class A, class G, int B0X100, bool PF = true, int WMASK = 0, class TwP, class St>
__device__ __forceinline__ void ntt_inverse_regs(const A &ar, TwP tw, int tid, typename A::V *lds,
                                                 const PassTw<A, G, G::NPASS - 1, true, wbit<WMASK, G::NPASS - 1>()> &first,
                                                 typename A::V (&v)[G::E], St st, const double *tww = nullptr) {
  static_assert(G::NPASS >= 2, "at least two passes");
  static_assert((WMASK & 1) == 0, "the last pass reads its twiddles with their companions");
  using V = typename A::V;
  PassTw<A, G, 0, true> last;
  if constexpr (G::NPASS > 2) {
    PassTw<A, G, G::NPASS - 2, true, wbit<WMASK, G::NPASS - 2>()> nxt;
    inv_pass_v<A, G, G::NPASS - 1, B0X100, WMASK>(ar, first, tid, v, LdsPut<V>{lds}, [&] {
      if constexpr (PF) nxt.load2(tw, tww, tid);
    });
    inv_lds_passes<A, G, G::NPASS - 2, B0X100, PF, WMASK>(ar, tw, tww, tid, lds, nxt, last);
  } else {
    inv_pass_v<A, G, 1, B0X100, WMASK>(ar, first, tid, v, LdsPut<V>{lds}, [&] {
      if constexpr (PF) last.load(tw, tid);
    });
  }
  xchg_sync<G, 1, 0>();
  if constexpr (!PF) last.load(tw, tid);
  constexpr double end_red = inv_end_red<A, G, WMASK>(B0X100 / 100.0);
  static_assert(plan_gs_slots<A>(G::r(0), inv_bound_in<A, G, WMASK>(0, B0X100 / 100.0, end_red), true, end_red).b_out <=
                    A::kStoreIn,
                "the last stage's products exceed the bound store_out needs");
  // (a store taking the index's two parts, thread and compile-time, can
  // address with a lane offset and a scalar one)
  auto st_out = [&](int t, int c, V x) {
    if constexpr (std::is_invocable_v<St &, int, int, uint64_t>) st(t, c, ar.store_out(x));
    else st(t + c, ar.store_out(x));
  };
  inv_pass<A, G, 0, B0X100, WMASK>(ar, last, tid, LdsAt<V>{lds}, st_out, [] {});
}

}  // namespace he
