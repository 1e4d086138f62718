// Kernels of the ciphertext-ciphertext product (Section 3.2, CCMul in the
// preprocessing phase) that are not transforms or term-list products: the exact
// lift of ciphertexts from base Q to Q u P, and the exact scale-and-round
// round(t x / Q) from Q u P back to Q with the relinearization digits.
//
// Both are one thread per coefficient (256-thread blocks, rows of N
// coefficients along the grid's x dimension) with a few modular products per
// prime, compiled for each pair of base sizes (L, K) so that every loop has
// its exact trip count, in fp64 when every prime of Q u P is below 2^50 and
// in 64-bit integers otherwise.  The conversion constants sit in device
// memory and are read uniformly by all lanes.
#include <hip/hip_runtime.h>

#include "he_internal.hpp"
#include "rns.hpp"

namespace he {
namespace {

struct Mod {
  uint64_t m, one;   // prime, floor(2^64 / m)
  double md, minv;   // prime, 1 / prime
};
struct Cst {
  uint64_t w, ws;    // constant below the prime, floor(w 2^64 / m)
  double wd;
};
__device__ __forceinline__ Mod mod_q(const RnsConv *cv, int i) { return Mod{cv->q[i], cv->q_one[i], cv->dq[i], cv->dqinv[i]}; }
__device__ __forceinline__ Mod mod_p(const RnsConv *cv, int k) { return Mod{cv->p[k], cv->p_one[k], cv->dp[k], cv->dpinv[k]}; }

// 64-bit integer products (Shoup), any primes below 2^62
struct RnsInt {
  using V = uint64_t;
  static __device__ __forceinline__ V ld(uint64_t x) { return x; }
  static __device__ __forceinline__ uint64_t st(V x) { return x; }
  // x w mod m for any x < 2^64
  static __device__ __forceinline__ V mul(V x, const Cst &c, const Mod &m) {
    const uint64_t r = x * c.w - __umul64hi(x, c.ws) * m.m;
    return r >= m.m ? r - m.m : r;
  }
  // x mod m for any x < 2^64
  static __device__ __forceinline__ V red(V x, const Mod &m) {
    const uint64_t r = x - __umul64hi(x, m.one) * m.m;
    return r >= m.m ? r - m.m : r;
  }
  static __device__ __forceinline__ V sub(V a, V b, const Mod &m) { return a >= b ? a - b : a + m.m - b; }
  static __device__ __forceinline__ V add(V a, V b, const Mod &m) {
    const V s = a + b;
    return s >= m.m ? s - m.m : s;
  }
};

// fp64 products, every prime below 2^50; values are integers held exactly in
// doubles.  For x < 2^50 and w < m: x w = h + l exactly (h rounded, l from an
// FMA, |l| <= m / 8); floor(h / m) computed in doubles is within one of the
// true quotient (x w / m < 2^50, relative error below 2^-51), so
// r = (h - qt m) + l is an integer in [-m, 2m) computed without rounding.
struct RnsF64 {
  using V = double;
  static __device__ __forceinline__ V ld(uint64_t x) {
    return __builtin_bit_cast(double, x | 0x4330000000000000ull) - 4503599627370496.0;
  }
  static __device__ __forceinline__ uint64_t st(V x) {
    return __builtin_bit_cast(uint64_t, x + 4503599627370496.0) & 0x000FFFFFFFFFFFFFull;
  }
  static __device__ __forceinline__ V mul(V x, const Cst &c, const Mod &m) {
    const double h = x * c.wd;
    const double l = __builtin_fma(x, c.wd, -h);
    const double qt = __builtin_floor(h * m.minv);
    double r = __builtin_fma(-qt, m.md, h) + l;
    r = r < 0.0 ? r + m.md : r;
    return r >= m.md ? r - m.md : r;
  }
  // x mod m for x < 2^52 (quotient estimate within one, remainder exact)
  static __device__ __forceinline__ V red(V x, const Mod &m) {
    const double qt = __builtin_floor(x * m.minv);
    double r = __builtin_fma(-qt, m.md, x);
    r = r < 0.0 ? r + m.md : r;
    return r >= m.md ? r - m.md : r;
  }
  static __device__ __forceinline__ V sub(V a, V b, const Mod &m) { return a >= b ? a - b : a + m.md - b; }
  static __device__ __forceinline__ V add(V a, V b, const Mod &m) {
    const V s = a + b;
    return s >= m.md ? s - m.md : s;
  }
};

// mixed-radix digits v of the residues x over n primes (of Q when P_ is false)
template <class R, int n, bool P_>
__device__ __forceinline__ void mrc(const typename R::V *x, typename R::V *v, const RnsConv *cv) {
#pragma unroll
  for (int i = 0; i < n; ++i) {
    const Mod mi = P_ ? mod_p(cv, i) : mod_q(cv, i);
    typename R::V u = x[i];
#pragma unroll
    for (int j = 0; j < i; ++j) {
      const Cst c = P_ ? Cst{cv->ipp[j][i], cv->ipps[j][i], cv->dipp[j][i]} : Cst{cv->iqq[j][i], cv->iqqs[j][i], cv->diqq[j][i]};
      u = R::mul(R::sub(u, R::red(v[j], mi), mi), c, mi);
    }
    v[i] = u;
  }
}

// digits v >= digits h (most significant first)
template <class R, int n>
__device__ __forceinline__ bool ge_digits(const typename R::V *v, const typename R::V *h) {
  int c = 0;
#pragma unroll
  for (int i = n - 1; i >= 0; --i) c = c != 0 ? c : (v[i] > h[i] ? 1 : (v[i] < h[i] ? -1 : 0));
  return c >= 0;
}

// the value of the n digits v (of Q when P_ is false) modulo the target prime
// tm: sum_i v_i prod_{j<i} (digit moduli) mod tm, col = the target's index
template <class R, int n, bool P_>
__device__ __forceinline__ typename R::V eval_digits(const typename R::V *v, const RnsConv *cv, int col, const Mod &tm) {
  typename R::V s = 0;
#pragma unroll
  for (int i = 0; i < n; ++i) {
    const Cst c = P_ ? Cst{cv->wp[i][col], cv->wps[i][col], cv->dwp[i][col]} : Cst{cv->wq[i][col], cv->wqs[i][col], cv->dwq[i][col]};
    s = R::add(s, R::mul(v[i], c, tm), tm);
  }
  return s;
}

template <class R, int n>
__device__ __forceinline__ void half_digits(typename R::V *h, const uint64_t *src) {
#pragma unroll
  for (int i = 0; i < n; ++i) h[i] = R::ld(src[i]);
}

// in [n][L][N] (base Q, canonical) -> out [n][L+K][N]: the L residues copied and
// the K residues mod p_k of the centred integer (x - Q when x >= (Q + 1) / 2)
template <class R, int L, int K>
__global__ __launch_bounds__(256) void k_rns_extend(uint64_t *__restrict__ out, const uint64_t *__restrict__ in,
                                                    const RnsConv *__restrict__ cv, uint32_t N, uint32_t sh) {
  using V = typename R::V;
  constexpr int E = L + K;
  const uint32_t k = ((blockIdx.x & ((1u << sh) - 1u)) << 8) + threadIdx.x;
  const uint32_t poly = blockIdx.x >> sh;
  const uint64_t *src = in + (size_t)poly * L * N + k;
  uint64_t *dst = out + (size_t)poly * E * N + k;
  V x[L], v[L], hq[L];
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const uint64_t xi = src[(size_t)i * N];
    dst[(size_t)i * N] = xi;
    x[i] = R::ld(xi);
  }
  mrc<R, L, false>(x, v, cv);
  half_digits<R, L>(hq, cv->hq);
  const bool neg = ge_digits<R, L>(v, hq);
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const Mod pj = mod_p(cv, j);
    V s = eval_digits<R, L, false>(v, cv, j, pj);
    if (neg) s = R::sub(s, R::ld(cv->q_mod_p[j]), pj);
    dst[(size_t)(L + j) * N] = R::st(s);
  }
}

// X [n][3][L+K][N]: the tensor slots as integers |x| < QP / 2 (centred in Q u P).
// For each slot d = round(t x / Q) mod Q: with y = t x and r = y mod Q in [0, Q),
// z = (y - r) / Q is exact in P (|z| < P / 2), and d = z + [r >= (Q + 1) / 2].
// Slots 0 and 1 go to out [n][2][L][N], slot 2 to dig [n][L][N]: its residue
// mod q_j is the relinearization digit D_j (an integer in [0, q_j)).
template <class R, int L, int K>
__global__ __launch_bounds__(256) void k_rns_scale_round(uint64_t *__restrict__ out, uint64_t *__restrict__ dig,
                                                         const uint64_t *__restrict__ X,
                                                         const RnsConv *__restrict__ cv, uint32_t N, uint32_t sh) {
  using V = typename R::V;
  constexpr int E = L + K;
  const uint32_t k = ((blockIdx.x & ((1u << sh) - 1u)) << 8) + threadIdx.x;
  const uint32_t row = blockIdx.x >> sh;   // o * 3 + slot
  const uint32_t o = row / 3, slot = row % 3;
  const uint64_t *src = X + (size_t)row * E * N + k;
  V r[L], v[L], z[K], w[K], hq[L], hp[K];
#pragma unroll
  for (int i = 0; i < L; ++i)   // (t x) mod q_i
    r[i] = R::mul(R::ld(src[(size_t)i * N]), Cst{cv->t_q[i], cv->t_qs[i], cv->dt_q[i]}, mod_q(cv, i));
  mrc<R, L, false>(r, v, cv);
  half_digits<R, L>(hq, cv->hq);
  const bool up = ge_digits<R, L>(v, hq);
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const Mod pj = mod_p(cv, j);
    const V y = R::mul(R::ld(src[(size_t)(L + j) * N]), Cst{cv->t_p[j], cv->t_ps[j], cv->dt_p[j]}, pj);
    const V rp = eval_digits<R, L, false>(v, cv, j, pj);
    z[j] = R::mul(R::sub(y, rp, pj), Cst{cv->qinv_p[j], cv->qinv_ps[j], cv->dqinv_p[j]}, pj);
  }
  mrc<R, K, true>(z, w, cv);
  half_digits<R, K>(hp, cv->hp);
  const bool neg = ge_digits<R, K>(w, hp);
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const Mod qi = mod_q(cv, i);
    V d = eval_digits<R, K, true>(w, cv, i, qi);
    if (neg) d = R::sub(d, R::ld(cv->p_mod_q[i]), qi);
    if (up) d = R::add(d, V(1), qi);
    if (slot < 2) out[((size_t)(o * 2 + slot) * L + i) * N + k] = R::st(d);
    else dig[((size_t)o * L + i) * N + k] = R::st(d);
  }
}

// the kernels for the base sizes (L, K) of a call
template <int L, int K>
hipError_t launch_lk(bool f64, const RnsConv *d_conv, uint64_t *out, uint64_t *dig, const uint64_t *in, uint32_t rows,
                     uint32_t N, bool extend, hipStream_t st) {
  // 256 coefficients per block, rows along x (N is a power of two >= 1024)
  const uint32_t sh = (uint32_t)__builtin_ctz(N) - 8;
  const dim3 grid(rows << sh);
  if (extend && f64)
    hipLaunchKernelGGL((k_rns_extend<RnsF64, L, K>), grid, dim3(256), 0, st, out, in, d_conv, N, sh);
  else if (extend)
    hipLaunchKernelGGL((k_rns_extend<RnsInt, L, K>), grid, dim3(256), 0, st, out, in, d_conv, N, sh);
  else if (f64)
    hipLaunchKernelGGL((k_rns_scale_round<RnsF64, L, K>), grid, dim3(256), 0, st, out, dig, in, d_conv, N, sh);
  else
    hipLaunchKernelGGL((k_rns_scale_round<RnsInt, L, K>), grid, dim3(256), 0, st, out, dig, in, d_conv, N, sh);
  return hipGetLastError();
}

template <int L>
hipError_t launch_l(int K, bool f64, const RnsConv *d_conv, uint64_t *out, uint64_t *dig, const uint64_t *in,
                    uint32_t rows, uint32_t N, bool extend, hipStream_t st) {
  switch (K) {
    case 1: return launch_lk<L, 1>(f64, d_conv, out, dig, in, rows, N, extend, st);
    case 2: return launch_lk<L, 2>(f64, d_conv, out, dig, in, rows, N, extend, st);
    case 3: return launch_lk<L, 3>(f64, d_conv, out, dig, in, rows, N, extend, st);
    case 4: return launch_lk<L, 4>(f64, d_conv, out, dig, in, rows, N, extend, st);
    case 5: return launch_lk<L, 5>(f64, d_conv, out, dig, in, rows, N, extend, st);
    case 6: return launch_lk<L, 6>(f64, d_conv, out, dig, in, rows, N, extend, st);
    case 7: return launch_lk<L, 7>(f64, d_conv, out, dig, in, rows, N, extend, st);
    case 8: return launch_lk<L, 8>(f64, d_conv, out, dig, in, rows, N, extend, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_any(int L, int K, bool f64, const RnsConv *d_conv, uint64_t *out, uint64_t *dig, const uint64_t *in,
                      uint32_t rows, uint32_t N, bool extend, hipStream_t st) {
  switch (L) {
    case 1: return launch_l<1>(K, f64, d_conv, out, dig, in, rows, N, extend, st);
    case 2: return launch_l<2>(K, f64, d_conv, out, dig, in, rows, N, extend, st);
    case 3: return launch_l<3>(K, f64, d_conv, out, dig, in, rows, N, extend, st);
    case 4: return launch_l<4>(K, f64, d_conv, out, dig, in, rows, N, extend, st);
    case 5: return launch_l<5>(K, f64, d_conv, out, dig, in, rows, N, extend, st);
    case 6: return launch_l<6>(K, f64, d_conv, out, dig, in, rows, N, extend, st);
    case 7: return launch_l<7>(K, f64, d_conv, out, dig, in, rows, N, extend, st);
    case 8: return launch_l<8>(K, f64, d_conv, out, dig, in, rows, N, extend, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_rns_extend(const RnsConv *d_conv, int L, int K, bool f64, uint64_t *out, const uint64_t *in,
                             uint32_t n_polys, uint32_t N, hipStream_t st) {
  if (!n_polys) return hipSuccess;
  return launch_any(L, K, f64, d_conv, out, nullptr, in, n_polys, N, true, st);
}

hipError_t launch_rns_scale_round(const RnsConv *d_conv, int L, int K, bool f64, uint64_t *out, uint64_t *dig,
                                  const uint64_t *X, uint32_t n_out, uint32_t N, hipStream_t st) {
  if (!n_out) return hipSuccess;
  return launch_any(L, K, f64, d_conv, out, dig, X, n_out * 3, N, false, st);
}

}  // namespace he
