// Templates of the per-plane ring kernels (transforms and the fused
// multiply-accumulate + inverse transform) and their launch logic, shared by
// the translation units that instantiate them: ring_<log2 N>.hip compiles
// every kernel of one ring degree, so the degrees build in parallel.
#pragma once
#include <type_traits>

#include "he_internal.hpp"
#include "ntt.hpp"
#include "mac.hpp"
#include "prng.hpp"
#include "pack.hpp"

namespace he {

// ------------------------------------------------------------------ policies
template <class A> struct TwOf;
template <> struct TwOf<ArF64> { using T = TwF64; };
template <> struct TwOf<ArU64> { using T = TwU64; };

template <class A>
__device__ __forceinline__ uint64_t canon_add(const A &, uint64_t a, uint64_t b, uint64_t q) {
  uint64_t s = a + b;
  return s >= q ? s - q : s;
}

// -------------------------------------------------------------- transforms
template <class A, int LOGN, int LOGT>
__global__ __launch_bounds__(1 << LOGT, (MinWaves<LOGN, LOGT>::value)) void k_ntt_fwd(uint64_t *__restrict__ out, const uint64_t *__restrict__ in,
                                                       const PrimeK *__restrict__ primes,
                                                       const typename A::Tw *__restrict__ tw, int L) {
  using G = Geo<LOGN, LOGT>;
  extern __shared__ __align__(16) unsigned char smem[];
  typename A::V *lds = reinterpret_cast<typename A::V *>(smem);
  const int plane = blockIdx.x;
  const int i = plane % L;
  const A ar(primes[i]);
  const uint64_t *src = in + (size_t)plane * G::N;
  uint64_t *dst = out + (size_t)plane * G::N;
  const int tid = threadIdx.x;
  auto ld = [&](int k) { return ar.load(src[(uint32_t)k]); };
  auto st = [&](int k, uint64_t v) { dst[(uint32_t)k] = v; };
  ntt_forward<A, G>(ar, tw + (size_t)i * G::N, tid, lds, ld, st);
}

// Forward transforms of two plane arrays in one launch: workgroups below n1
// take in1 -> out1, the others in2 -> out2 (two small sets run side by side).
template <class A, int LOGN, int LOGT>
__global__ __launch_bounds__(1 << LOGT, (MinWaves<LOGN, LOGT>::value)) void k_ntt_fwd2(
    uint64_t *__restrict__ out1, const uint64_t *__restrict__ in1, int n1, uint64_t *__restrict__ out2,
    const uint64_t *__restrict__ in2, const PrimeK *__restrict__ primes, const typename A::Tw *__restrict__ tw, int L) {
  using G = Geo<LOGN, LOGT>;
  extern __shared__ __align__(16) unsigned char smem[];
  typename A::V *lds = reinterpret_cast<typename A::V *>(smem);
  const bool first = (int)blockIdx.x < n1;
  const int plane = first ? (int)blockIdx.x : (int)blockIdx.x - n1;
  const int i = plane % L;
  const A ar(primes[i]);
  const uint64_t *src = (first ? in1 : in2) + (size_t)plane * G::N;
  uint64_t *dst = (first ? out1 : out2) + (size_t)plane * G::N;
  auto ld = [&](int k) { return ar.load(src[(uint32_t)k]); };
  auto st = [&](int k, uint64_t v) { dst[(uint32_t)k] = v; };
  ntt_forward<A, G>(ar, tw + (size_t)i * G::N, threadIdx.x, lds, ld, st);
}

// Forward transform of ciphertext planes whose component 1 is regenerated from
// a seed: plane (j, comp, i) reads component 0 from ct0 [n][L][N] or forms
// component 1 in registers (no HBM read of c1).
template <class A, int LOGN, int LOGT>
__global__ __launch_bounds__(1 << LOGT, (MinWaves<LOGN, LOGT>::value)) void k_ntt_fwd_seeded(
    uint64_t *__restrict__ out, const uint64_t *__restrict__ ct0, const PrimeK *__restrict__ primes,
    const typename A::Tw *__restrict__ tw, int L, Seed seed) {
  using G = Geo<LOGN, LOGT>;
  extern __shared__ __align__(16) unsigned char smem[];
  typename A::V *lds = reinterpret_cast<typename A::V *>(smem);
  const int plane = blockIdx.x;   // (j * 2 + comp) * L + i
  const int i = plane % L;
  const int comp = (plane / L) & 1;
  const int j = plane / (2 * L);
  const PrimeK pk = primes[i];
  const A ar(pk);
  uint64_t *dst = out + (size_t)plane * G::N;
  const int tid = threadIdx.x;
  auto st = [&](int k, uint64_t v) { dst[(uint32_t)k] = v; };
  if (comp == 0) {
    const uint64_t *src = ct0 + ((size_t)j * L + i) * G::N;
    auto ld = [&](int k) { return ar.load(src[(uint32_t)k]); };
    ntt_forward<A, G>(ar, tw + (size_t)i * G::N, tid, lds, ld, st);
  } else {
    auto ld = [&](int k) { return ar.load(c1_residue(seed, (uint32_t)j, (uint32_t)i, (uint32_t)k, pk)); };
    ntt_forward<A, G>(ar, tw + (size_t)i * G::N, tid, lds, ld, st);
  }
}

// Forward transform of signed integer polynomials lifted to every prime:
// plane p reads polynomial p / L and lifts it modulo q_{p % L}.
template <class A, int LOGN, int LOGT>
__global__ __launch_bounds__(1 << LOGT, (MinWaves<LOGN, LOGT>::value)) void k_ntt_fwd_lift(uint64_t *__restrict__ out,
                                                            const int64_t *__restrict__ polys,
                                                            const PrimeK *__restrict__ primes,
                                                            const typename A::Tw *__restrict__ tw, int L) {
  using G = Geo<LOGN, LOGT>;
  extern __shared__ __align__(16) unsigned char smem[];
  typename A::V *lds = reinterpret_cast<typename A::V *>(smem);
  const int plane = blockIdx.x;
  const int i = plane % L;
  const A ar(primes[i]);
  const int64_t *src = polys + (size_t)(plane / L) * G::N;
  uint64_t *dst = out + (size_t)plane * G::N;
  const int tid = threadIdx.x;
  auto ld = [&](int k) { return ar.load_signed(src[(uint32_t)k]); };
  auto st = [&](int k, uint64_t v) { dst[(uint32_t)k] = v; };
  ntt_forward<A, G>(ar, tw + (size_t)i * G::N, tid, lds, ld, st);
}

// Forward transform of plaintext polynomials packed from raw weights in LDS:
// plane p is polynomial p / L at prime p % L; the workgroup zeroes the plane,
// scatters the polynomial's weights and transforms it from LDS (no packed
// polynomial in HBM).
template <class A, int LOGN, int LOGT>
__global__ __launch_bounds__(1 << LOGT, (MinWaves<LOGN, LOGT>::value)) void k_ntt_fwd_pack(
    uint64_t *__restrict__ out, WPack wp, const int32_t *__restrict__ w, const PrimeK *__restrict__ primes,
    const typename A::Tw *__restrict__ tw, int L) {
  using G = Geo<LOGN, LOGT>;
  extern __shared__ __align__(16) unsigned char smem[];
  typename A::V *lds = reinterpret_cast<typename A::V *>(smem);
  const int plane = blockIdx.x;
  const int i = plane % L;
  const A ar(primes[i]);
  uint64_t *dst = out + (size_t)plane * G::N;
  const int tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j < G::E; ++j) lds[lin_lds<G>(tid, j)] = ar.load(0ull);
  __syncthreads();
  scatter_weights<A, G>(ar, lds, tid, wp, (uint32_t)(plane / L), w);
  __syncthreads();
  auto st = [&](int k, uint64_t v) { dst[(uint32_t)k] = v; };
  ntt_forward_tc<A, G>(ar, tw + (size_t)i * G::N, tid, lds, LdsAt<typename A::V>{lds}, st);
}

// One launch for both operand sets of a layer: workgroups below n_ct_planes
// transform input ciphertext planes (as k_ntt_fwd), the others pack and
// transform plaintext planes from raw weights (as k_ntt_fwd_pack), so the two
// small sets run concurrently instead of one after the other.
// SEEDED: the ciphertexts' component 1 is regenerated from the seed (plane
// (j, comp, i): component 0 read from ct_in [n][L][N], as k_ntt_fwd_seeded).
template <class A, int LOGN, int LOGT, bool SEEDED>
__global__ __launch_bounds__(1 << LOGT, (MinWaves<LOGN, LOGT>::value)) void k_ntt_fwd_ct_pack(
    uint64_t *__restrict__ ct_out, const uint64_t *__restrict__ ct_in, int n_ct_planes, uint64_t *__restrict__ pt_out,
    WPack wp, const int32_t *__restrict__ w, const PrimeK *__restrict__ primes, const typename A::Tw *__restrict__ tw,
    int L, Seed seed) {
  using G = Geo<LOGN, LOGT>;
  extern __shared__ __align__(16) unsigned char smem[];
  typename A::V *lds = reinterpret_cast<typename A::V *>(smem);
  const int tid = threadIdx.x;
  if ((int)blockIdx.x < n_ct_planes) {
    const int plane = blockIdx.x;
    const int i = plane % L;
    const PrimeK pk = primes[i];
    const A ar(pk);
    uint64_t *dst = ct_out + (size_t)plane * G::N;
    auto st = [&](int k, uint64_t v) { dst[(uint32_t)k] = v; };
    if constexpr (SEEDED) {
      const int comp = (plane / L) & 1, j = plane / (2 * L);
      if (comp == 0) {
        const uint64_t *src = ct_in + ((size_t)j * L + i) * G::N;
        auto ld = [&](int k) { return ar.load(src[(uint32_t)k]); };
        ntt_forward<A, G>(ar, tw + (size_t)i * G::N, tid, lds, ld, st);
      } else {
        auto ld = [&](int k) { return ar.load(c1_residue(seed, (uint32_t)j, (uint32_t)i, (uint32_t)k, pk)); };
        ntt_forward<A, G>(ar, tw + (size_t)i * G::N, tid, lds, ld, st);
      }
    } else {
      const uint64_t *src = ct_in + (size_t)plane * G::N;
      auto ld = [&](int k) { return ar.load(src[(uint32_t)k]); };
      ntt_forward<A, G>(ar, tw + (size_t)i * G::N, tid, lds, ld, st);
    }
  } else {
    const int plane = (int)blockIdx.x - n_ct_planes;
    const int i = plane % L;
    const A ar(primes[i]);
    uint64_t *dst = pt_out + (size_t)plane * G::N;
#pragma unroll
    for (int j = 0; j < G::E; ++j) lds[lin_lds<G>(tid, j)] = ar.load(0ull);
    __syncthreads();
    scatter_weights<A, G>(ar, lds, tid, wp, (uint32_t)(plane / L), w);
    __syncthreads();
    auto st = [&](int k, uint64_t v) { dst[(uint32_t)k] = v; };
    ntt_forward_tc<A, G>(ar, tw + (size_t)i * G::N, tid, lds, LdsAt<typename A::V>{lds}, st);
  }
}

template <class A, int LOGN, int LOGT>
__global__ __launch_bounds__(1 << LOGT, (MinWaves<LOGN, LOGT>::value)) void k_ntt_inv(uint64_t *__restrict__ out, const uint64_t *__restrict__ in,
                                                       const PrimeK *__restrict__ primes,
                                                       const typename A::Tw *__restrict__ tw, int L) {
  using G = Geo<LOGN, LOGT>;
  extern __shared__ __align__(16) unsigned char smem[];
  typename A::V *lds = reinterpret_cast<typename A::V *>(smem);
  const int plane = blockIdx.x;
  const int i = plane % L;
  const A ar(primes[i]);
  const uint64_t *src = in + (size_t)plane * G::N;
  uint64_t *dst = out + (size_t)plane * G::N;
  const int tid = threadIdx.x;
  const typename A::Tw *twi = tw + (size_t)i * G::N;
  PassTw<A, G, G::NPASS - 1, true> first;
  first.load(twi, tid);
  typename A::V v[G::E];
#pragma unroll
  for (int e = 0; e < G::E; ++e) v[e] = ar.load(src[slot_index<G, G::NPASS - 1>(tid, e)]);
  auto st = [&](int k, uint64_t x) { dst[(uint32_t)k] = x; };
  ntt_inverse_regs<A, G, 100>(ar, twi, tid, lds, first, v, st);
}

// ------------------------------------------------- multiply-accumulate (slots)
// Term lists: output o sums the terms row[o] .. row[o+1]-1, term t pairing
// ciphertext cti[t] with plaintext pti[t]; with row == nullptr there is one
// output whose terms pair ciphertext t with plaintext t, t < K.
struct TermArgs {
  const int32_t *row, *cti, *pti;
  uint32_t K;     // identity mode (row == nullptr): one output, terms 0..K-1
};

__device__ __forceinline__ void term_range(const TermArgs &ta, int o, int &t0, int &t1) {
  if (ta.row) {
    t0 = ta.row[o];
    t1 = ta.row[o + 1];
  } else {
    t0 = 0;
    t1 = (int)ta.K;
  }
}
__device__ __forceinline__ int term_ct(const TermArgs &ta, int t) { return ta.row ? ta.cti[t] : t; }
__device__ __forceinline__ int term_pt(const TermArgs &ta, int t) { return ta.row ? ta.pti[t] : t; }

// One workgroup per output plane (o, comp, i): multiply-accumulate the slots in
// the layout of the inverse transform's first pass, then the inverse
// transform, then store (or add).
// NCOMP: components per operand and output (2 for ciphertexts; 1 for products
// of plaintext polynomials).
template <class A, int LOGN, int LOGT, bool ACC, int NCOMP = 2>
__global__ __launch_bounds__(1 << LOGT, (MinWaves<LOGN, LOGT>::value)) void k_mac_inv(
    uint64_t *__restrict__ out, const uint64_t *__restrict__ ct_hat, const uint64_t *__restrict__ pt_hat, TermArgs ta,
    const PrimeK *__restrict__ primes, const typename A::Tw *__restrict__ tw, const double *__restrict__ tww, int L,
    uint32_t xcd_chunk, int n_planes) {
  using G = Geo<LOGN, LOGT>;
  extern __shared__ __align__(16) unsigned char smem[];
  typename A::V *lds = reinterpret_cast<typename A::V *>(smem);
  // Workgroups are dealt round-robin over the 8 XCDs; give XCD x a contiguous
  // run of output planes so that outputs sharing inputs share that XCD's L2.
  const int plane = (int)((blockIdx.x & 7u) * xcd_chunk + (blockIdx.x >> 3));   // (o * NCOMP + comp) * L + i
  if (plane >= n_planes) return;
  const int i = plane % L;
  const int comp = NCOMP == 1 ? 0 : (plane / L) % NCOMP;
  const int o = plane / (NCOMP * L);
  const PrimeK *pk = primes + i;
  const A ar(*pk);
  const int tid = threadIdx.x;
  int t0, t1;
  term_range(ta, o, t0, t1);
  MacAcc<A> acc[G::E];
  auto operands = [&](int t) {
    const uint64_t *a = ct_hat + ((size_t)(term_ct(ta, t) * NCOMP + comp) * L + i) * G::N;
    const uint64_t *b = pt_hat + ((size_t)term_pt(ta, t) * L + i) * G::N;
    return std::pair<const uint64_t *, const uint64_t *>(a, b);
  };
  mac_terms<A, G::E>(ar, *pk, acc, t0, t1, operands, [&](int e) { return slot_index<G, G::NPASS - 1>(tid, e); });
  typename A::V v[G::E];
#pragma unroll
  for (int e = 0; e < G::E; ++e) v[e] = acc[e].value();
  const typename A::Tw *twi = tw + (size_t)i * G::N;
  // fp64: the passes whose lanes read different twiddles take them alone
  // (tww: the inverse twiddles without companions, formed at the product)
  constexpr int kWM = std::is_same<A, ArF64>::value ? lane_passes<G>() : 0;
  const double *twi_w = kWM ? tww + (size_t)i * G::N : nullptr;
  PassTw<A, G, G::NPASS - 1, true, wbit<kWM, G::NPASS - 1>()> first;
  first.load2(twi, twi_w, tid);
  uint64_t *dst = out + (size_t)plane * G::N;
  const uint64_t q = pk->q;
  if constexpr (ACC) {
    auto st = [&](int k, uint64_t x) { dst[(uint32_t)k] = canon_add(ar, dst[(uint32_t)k], x, q); };
    ntt_inverse_regs<A, G, MacAcc<A>::kOutBoundX100, true, kWM>(ar, twi, tid, lds, first, v, st, twi_w);
  } else {
    // output planes are not read again here: streaming stores keep them from
    // evicting the operands and twiddles that later planes reuse from L2
    auto st = [&](int k, uint64_t x) { __builtin_nontemporal_store(x, &dst[(uint32_t)k]); };
    ntt_inverse_regs<A, G, MacAcc<A>::kOutBoundX100, true, kWM>(ar, twi, tid, lds, first, v, st, twi_w);
  }
}

// Set the dynamic-LDS limit once per kernel instantiation.
template <class Kern>
static hipError_t prep(Kern k, size_t lds) {
  static thread_local const void *done[512];
  static thread_local int nd = 0;
  for (int j = 0; j < nd; ++j)
    if (done[j] == (const void *)k) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess && nd < 512) done[nd++] = (const void *)k;
  return e;
}

template <class A>
static const typename A::Tw *tw_ptr(const Ctx &c, bool inverse);
template <>
inline const TwF64 *tw_ptr<ArF64>(const Ctx &c, bool inverse) {
  return (const TwF64 *)(inverse ? c.d_tw_f64_inv : c.d_tw_f64_fwd);
}
template <>
inline const TwU64 *tw_ptr<ArU64>(const Ctx &c, bool inverse) {
  return (const TwU64 *)(inverse ? c.d_tw_u64_inv : c.d_tw_u64_fwd);
}

// the inverse twiddles alone (fp64 only: the integer policy forms no companions)
template <class A>
static const double *tww_inv(const Ctx &c) {
  return std::is_same<A, ArF64>::value ? c.d_tw_f64_inv_w : nullptr;
}

enum Op { OP_FWD, OP_FWD_LIFT, OP_INV, OP_MAC_INV, OP_FWD_SEEDED, OP_FWD_PACK, OP_FWD_CT_PACK, OP_FWD2 };

struct LaunchArgs {
  uint64_t *out;
  const uint64_t *in;
  const int64_t *polys;
  const uint64_t *pt;
  TermArgs ta;
  int accumulate;
  int ncomp;
  Seed seed;
  WPack wp;       // OP_FWD_PACK, OP_FWD_CT_PACK: layout of the weights (polys: the int32 weights)
  uint64_t *out2; // OP_FWD_CT_PACK: transformed plaintexts (out, in: the ciphertext planes);
                  // OP_FWD2: second output (out, in: the first array; pt: the second input)
  int n_first;    // OP_FWD_CT_PACK, OP_FWD2: planes of the first array (the first workgroups)
  int seeded;     // OP_FWD_CT_PACK: ciphertext component 1 from `seed`
  unsigned grid;
};

template <class A, int LOGN, int LOGT>
static hipError_t run_op(const Ctx &c, Op op, const LaunchArgs &la, hipStream_t st) {
  using G = Geo<LOGN, LOGT>;
  const size_t lds = (size_t)G::LDS_WORDS * 8;
  hipError_t e;
  switch (op) {
    case OP_FWD:
      if ((e = prep(k_ntt_fwd<A, LOGN, LOGT>, lds)) != hipSuccess) return e;
      hipLaunchKernelGGL((k_ntt_fwd<A, LOGN, LOGT>), dim3(la.grid), dim3(G::NT), lds, st, la.out, la.in, c.d_primes,
                         tw_ptr<A>(c, false), (int)c.L);
      break;
    case OP_FWD_LIFT:
      if ((e = prep(k_ntt_fwd_lift<A, LOGN, LOGT>, lds)) != hipSuccess) return e;
      hipLaunchKernelGGL((k_ntt_fwd_lift<A, LOGN, LOGT>), dim3(la.grid), dim3(G::NT), lds, st, la.out, la.polys,
                         c.d_primes, tw_ptr<A>(c, false), (int)c.L);
      break;
    case OP_FWD_SEEDED:
      if ((e = prep(k_ntt_fwd_seeded<A, LOGN, LOGT>, lds)) != hipSuccess) return e;
      hipLaunchKernelGGL((k_ntt_fwd_seeded<A, LOGN, LOGT>), dim3(la.grid), dim3(G::NT), lds, st, la.out, la.in,
                         c.d_primes, tw_ptr<A>(c, false), (int)c.L, la.seed);
      break;
    case OP_FWD_PACK:
      if ((e = prep(k_ntt_fwd_pack<A, LOGN, LOGT>, lds)) != hipSuccess) return e;
      hipLaunchKernelGGL((k_ntt_fwd_pack<A, LOGN, LOGT>), dim3(la.grid), dim3(G::NT), lds, st, la.out, la.wp,
                         (const int32_t *)la.polys, c.d_primes, tw_ptr<A>(c, false), (int)c.L);
      break;
    case OP_FWD2:
      if ((e = prep(k_ntt_fwd2<A, LOGN, LOGT>, lds)) != hipSuccess) return e;
      hipLaunchKernelGGL((k_ntt_fwd2<A, LOGN, LOGT>), dim3(la.grid), dim3(G::NT), lds, st, la.out, la.in, la.n_first,
                         la.out2, la.pt, c.d_primes, tw_ptr<A>(c, false), (int)c.L);
      break;
    case OP_FWD_CT_PACK:
      if (la.seeded) {
        if ((e = prep(k_ntt_fwd_ct_pack<A, LOGN, LOGT, true>, lds)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_ntt_fwd_ct_pack<A, LOGN, LOGT, true>), dim3(la.grid), dim3(G::NT), lds, st, la.out,
                           la.in, la.n_first, la.out2, la.wp, (const int32_t *)la.polys, c.d_primes,
                           tw_ptr<A>(c, false), (int)c.L, la.seed);
      } else {
        if ((e = prep(k_ntt_fwd_ct_pack<A, LOGN, LOGT, false>, lds)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_ntt_fwd_ct_pack<A, LOGN, LOGT, false>), dim3(la.grid), dim3(G::NT), lds, st, la.out,
                           la.in, la.n_first, la.out2, la.wp, (const int32_t *)la.polys, c.d_primes,
                           tw_ptr<A>(c, false), (int)c.L, la.seed);
      }
      break;
    case OP_INV:
      if ((e = prep(k_ntt_inv<A, LOGN, LOGT>, lds)) != hipSuccess) return e;
      hipLaunchKernelGGL((k_ntt_inv<A, LOGN, LOGT>), dim3(la.grid), dim3(G::NT), lds, st, la.out, la.in, c.d_primes,
                         tw_ptr<A>(c, true), (int)c.L);
      break;
    case OP_MAC_INV: {
      const uint32_t chunk = (la.grid + 7) / 8;
      const unsigned grid = chunk * 8;
      if (la.ncomp == 1) {
        // single-component products (plaintext polynomials, tensor slots)
        if ((e = prep(k_mac_inv<A, LOGN, LOGT, false, 1>, lds)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_mac_inv<A, LOGN, LOGT, false, 1>), dim3(grid), dim3(G::NT), lds, st, la.out, la.in,
                           la.pt, la.ta, c.d_primes, tw_ptr<A>(c, true), tww_inv<A>(c), (int)c.L, chunk, (int)la.grid);
      } else if (la.accumulate) {
        if ((e = prep(k_mac_inv<A, LOGN, LOGT, true>, lds)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_mac_inv<A, LOGN, LOGT, true>), dim3(grid), dim3(G::NT), lds, st, la.out, la.in, la.pt,
                           la.ta, c.d_primes, tw_ptr<A>(c, true), tww_inv<A>(c), (int)c.L, chunk, (int)la.grid);
      } else {
        if ((e = prep(k_mac_inv<A, LOGN, LOGT, false>, lds)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_mac_inv<A, LOGN, LOGT, false>), dim3(grid), dim3(G::NT), lds, st, la.out, la.in, la.pt,
                           la.ta, c.d_primes, tw_ptr<A>(c, true), tww_inv<A>(c), (int)c.L, chunk, (int)la.grid);
      }
      break;
    }
  }
  return hipGetLastError();
}

template <class A, int LOGN>
static hipError_t run_loge(const Ctx &c, int loge, Op op, const LaunchArgs &la, hipStream_t st) {
  if constexpr (LOGN - 3 <= 10) {
    if (loge == 3) return run_op<A, LOGN, LOGN - 3>(c, op, la, st);
  }
  if constexpr (LOGN - 4 >= 6 && LOGN - 4 <= 10) {
    if (loge == 4) return run_op<A, LOGN, LOGN - 4>(c, op, la, st);
  }
  if constexpr (LOGN - 5 >= 6 && LOGN - 5 <= 10) {
    if (loge == 5) return run_op<A, LOGN, LOGN - 5>(c, op, la, st);
  }
  return hipErrorInvalidValue;
}


// every kernel of ring degree 2^LOGN, one translation unit each (ring_<LOGN>.hip)
hipError_t run_ring_10(const Ctx &c, bool f64, int loge, Op op, const LaunchArgs &la, hipStream_t st);
hipError_t run_ring_11(const Ctx &c, bool f64, int loge, Op op, const LaunchArgs &la, hipStream_t st);
hipError_t run_ring_12(const Ctx &c, bool f64, int loge, Op op, const LaunchArgs &la, hipStream_t st);
hipError_t run_ring_13(const Ctx &c, bool f64, int loge, Op op, const LaunchArgs &la, hipStream_t st);
hipError_t run_ring_14(const Ctx &c, bool f64, int loge, Op op, const LaunchArgs &la, hipStream_t st);

}  // namespace he
