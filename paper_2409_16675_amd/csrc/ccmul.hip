// Kernels of the ciphertext-ciphertext product (Section 3.2, CCMul in the
// preprocessing phase) that are not transforms or term-list products: the exact
// lift of ciphertexts from base Q to Q u P, and the exact scale-and-round
// round(t x / Q) from Q u P back to Q with the relinearization digits.
//
// Both are one thread per coefficient (256-thread blocks, rows of N
// coefficients along the grid's x dimension) with a few 64-bit modular products per
// prime, compiled for each pair of base sizes (L, K) so that every loop has
// its exact trip count.  The conversion constants sit in device memory and
// are read uniformly by all lanes.
#include <hip/hip_runtime.h>

#include "he_internal.hpp"
#include "rns.hpp"

namespace he {
namespace {

// x * w mod m for any x < 2^64, w < m < 2^63, ws = floor(w 2^64 / m)
__device__ __forceinline__ uint64_t mulc(uint64_t x, uint64_t w, uint64_t ws, uint64_t m) {
  const uint64_t r = x * w - __umul64hi(x, ws) * m;
  return r >= m ? r - m : r;
}
// x mod m for any x < 2^64 (one_s = floor(2^64 / m))
__device__ __forceinline__ uint64_t redc(uint64_t x, uint64_t m, uint64_t one_s) {
  const uint64_t r = x - __umul64hi(x, one_s) * m;
  return r >= m ? r - m : r;
}
__device__ __forceinline__ uint64_t subm(uint64_t a, uint64_t b, uint64_t m) { return a >= b ? a - b : a + m - b; }
__device__ __forceinline__ uint64_t addm(uint64_t a, uint64_t b, uint64_t m) {
  const uint64_t s = a + b;
  return s >= m ? s - m : s;
}

// mixed-radix digits v of the residues x over moduli mod[0..n)
template <int n>
__device__ __forceinline__ void mrc(const uint64_t *x, uint64_t *v, const uint64_t *mod, const uint64_t *one,
                                    const uint64_t (*inv)[kRnsMax], const uint64_t (*invs)[kRnsMax]) {
#pragma unroll
  for (int i = 0; i < n; ++i) {
    uint64_t u = x[i];
#pragma unroll
    for (int j = 0; j < i; ++j) u = mulc(subm(u, redc(v[j], mod[i], one[i]), mod[i]), inv[j][i], invs[j][i], mod[i]);
    v[i] = u;
  }
}

// digits v >= digits h (most significant first)
template <int n>
__device__ __forceinline__ bool ge_digits(const uint64_t *v, const uint64_t *h) {
  int c = 0;
#pragma unroll
  for (int i = n - 1; i >= 0; --i) c = c != 0 ? c : (v[i] > h[i] ? 1 : (v[i] < h[i] ? -1 : 0));
  return c >= 0;
}

// the value of digits v modulo m: sum_i v_i W[i][col] (W[i] = prod_{j<i} of the digit moduli, mod m)
template <int n>
__device__ __forceinline__ uint64_t eval_digits(const uint64_t *v, const uint64_t (*w)[kRnsMax],
                                                const uint64_t (*ws)[kRnsMax], int col, uint64_t m) {
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < n; ++i) s = addm(s, mulc(v[i], w[i][col], ws[i][col], m), m);
  return s;
}

// in [n][L][N] (base Q, canonical) -> out [n][L+K][N]: the L residues copied and
// the K residues mod p_k of the centred integer (x - Q when x >= (Q + 1) / 2)
template <int L, int K>
__global__ __launch_bounds__(256) void k_rns_extend(uint64_t *__restrict__ out, const uint64_t *__restrict__ in,
                                                    const RnsConv *__restrict__ cv, uint32_t N, uint32_t sh) {
  constexpr int E = L + K;
  const uint32_t k = ((blockIdx.x & ((1u << sh) - 1u)) << 8) + threadIdx.x;
  const uint32_t poly = blockIdx.x >> sh;
  const uint64_t *src = in + (size_t)poly * L * N + k;
  uint64_t *dst = out + (size_t)poly * E * N + k;
  uint64_t x[L], v[L];
#pragma unroll
  for (int i = 0; i < L; ++i) {
    x[i] = src[(size_t)i * N];
    dst[(size_t)i * N] = x[i];
  }
  mrc<L>(x, v, cv->q, cv->q_one, cv->iqq, cv->iqqs);
  const bool neg = ge_digits<L>(v, cv->hq);
#pragma unroll
  for (int j = 0; j < K; ++j) {
    uint64_t s = eval_digits<L>(v, cv->wq, cv->wqs, j, cv->p[j]);
    if (neg) s = subm(s, cv->q_mod_p[j], cv->p[j]);
    dst[(size_t)(L + j) * N] = s;
  }
}

// X [n][3][L+K][N]: the tensor slots as integers |x| < QP / 2 (centred in Q u P).
// For each slot d = round(t x / Q) mod Q: with y = t x and r = y mod Q in [0, Q),
// z = (y - r) / Q is exact in P (|z| < P / 2), and d = z + [r >= (Q + 1) / 2].
// Slots 0 and 1 go to out [n][2][L][N]; slot 2 to the digits
// dig [n][L][L][N], dig[o][j][i] = (d mod q_j) mod q_i.
template <int L, int K>
__global__ __launch_bounds__(256) void k_rns_scale_round(uint64_t *__restrict__ out, uint64_t *__restrict__ dig,
                                                         const uint64_t *__restrict__ X,
                                                         const RnsConv *__restrict__ cv, uint32_t N, uint32_t sh) {
  constexpr int E = L + K;
  const uint32_t k = ((blockIdx.x & ((1u << sh) - 1u)) << 8) + threadIdx.x;
  const uint32_t row = blockIdx.x >> sh;   // o * 3 + slot
  const uint32_t o = row / 3, slot = row % 3;
  const uint64_t *src = X + (size_t)row * E * N + k;
  uint64_t r[L], v[L], z[K], w[K];
#pragma unroll
  for (int i = 0; i < L; ++i) r[i] = mulc(src[(size_t)i * N], cv->t_q[i], cv->t_qs[i], cv->q[i]);   // (t x) mod q_i
  mrc<L>(r, v, cv->q, cv->q_one, cv->iqq, cv->iqqs);
  const uint64_t up = ge_digits<L>(v, cv->hq) ? 1 : 0;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const uint64_t pj = cv->p[j];
    const uint64_t y = mulc(src[(size_t)(L + j) * N], cv->t_p[j], cv->t_ps[j], pj);
    const uint64_t rp = eval_digits<L>(v, cv->wq, cv->wqs, j, pj);
    z[j] = mulc(subm(y, rp, pj), cv->qinv_p[j], cv->qinv_ps[j], pj);
  }
  mrc<K>(z, w, cv->p, cv->p_one, cv->ipp, cv->ipps);
  const bool neg = ge_digits<K>(w, cv->hp);
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const uint64_t qi = cv->q[i];
    uint64_t d = eval_digits<K>(w, cv->wp, cv->wps, i, qi);
    if (neg) d = subm(d, cv->p_mod_q[i], qi);
    d = addm(d, up, qi);
    if (slot < 2) {
      out[((size_t)(o * 2 + slot) * L + i) * N + k] = d;
    } else {
      uint64_t *dd = dig + ((size_t)(o * L + i) * L) * N + k;
#pragma unroll
      for (int i2 = 0; i2 < L; ++i2) dd[(size_t)i2 * N] = redc(d, cv->q[i2], cv->q_one[i2]);
    }
  }
}

// the kernels for the base sizes (L, K) of a call
template <int L, int K>
hipError_t launch_lk(const RnsConv *d_conv, uint64_t *out, uint64_t *dig, const uint64_t *in, uint32_t rows, uint32_t N,
                     bool extend, hipStream_t st) {
  // 256 coefficients per block, rows along x (N is a power of two >= 1024)
  const uint32_t sh = (uint32_t)__builtin_ctz(N) - 8;
  const dim3 grid(rows << sh);
  if (extend)
    hipLaunchKernelGGL((k_rns_extend<L, K>), grid, dim3(256), 0, st, out, in, d_conv, N, sh);
  else
    hipLaunchKernelGGL((k_rns_scale_round<L, K>), grid, dim3(256), 0, st, out, dig, in, d_conv, N, sh);
  return hipGetLastError();
}

template <int L>
hipError_t launch_l(int K, const RnsConv *d_conv, uint64_t *out, uint64_t *dig, const uint64_t *in, uint32_t rows,
                    uint32_t N, bool extend, hipStream_t st) {
  switch (K) {
    case 1: return launch_lk<L, 1>(d_conv, out, dig, in, rows, N, extend, st);
    case 2: return launch_lk<L, 2>(d_conv, out, dig, in, rows, N, extend, st);
    case 3: return launch_lk<L, 3>(d_conv, out, dig, in, rows, N, extend, st);
    case 4: return launch_lk<L, 4>(d_conv, out, dig, in, rows, N, extend, st);
    case 5: return launch_lk<L, 5>(d_conv, out, dig, in, rows, N, extend, st);
    case 6: return launch_lk<L, 6>(d_conv, out, dig, in, rows, N, extend, st);
    case 7: return launch_lk<L, 7>(d_conv, out, dig, in, rows, N, extend, st);
    case 8: return launch_lk<L, 8>(d_conv, out, dig, in, rows, N, extend, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_any(int L, int K, const RnsConv *d_conv, uint64_t *out, uint64_t *dig, const uint64_t *in,
                      uint32_t rows, uint32_t N, bool extend, hipStream_t st) {
  switch (L) {
    case 1: return launch_l<1>(K, d_conv, out, dig, in, rows, N, extend, st);
    case 2: return launch_l<2>(K, d_conv, out, dig, in, rows, N, extend, st);
    case 3: return launch_l<3>(K, d_conv, out, dig, in, rows, N, extend, st);
    case 4: return launch_l<4>(K, d_conv, out, dig, in, rows, N, extend, st);
    case 5: return launch_l<5>(K, d_conv, out, dig, in, rows, N, extend, st);
    case 6: return launch_l<6>(K, d_conv, out, dig, in, rows, N, extend, st);
    case 7: return launch_l<7>(K, d_conv, out, dig, in, rows, N, extend, st);
    case 8: return launch_l<8>(K, d_conv, out, dig, in, rows, N, extend, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_rns_extend(const RnsConv *d_conv, int L, int K, uint64_t *out, const uint64_t *in,
                             uint32_t n_polys, uint32_t N, hipStream_t st) {
  if (!n_polys) return hipSuccess;
  return launch_any(L, K, d_conv, out, nullptr, in, n_polys, N, true, st);
}

hipError_t launch_rns_scale_round(const RnsConv *d_conv, int L, int K, uint64_t *out, uint64_t *dig,
                                  const uint64_t *X, uint32_t n_out, uint32_t N, hipStream_t st) {
  if (!n_out) return hipSuccess;
  return launch_any(L, K, d_conv, out, dig, X, n_out * 3, N, false, st);
}

}  // namespace he
