// gfx950 kernels of libhe.so outside the per-degree ring kernels: their launch
// dispatch (the templates are in ring_kernels.hpp, instantiated by
// ring_<log2 N>.hip), the multiply-accumulate left in the transformed domain,
// plaintext packing, and the small helpers used by encryption.
#include "ring_kernels.hpp"

namespace he {

// Component 1 of ciphertexts first .. first+n-1 regenerated from the seed,
// written [n][L][N] (coefficient form).
// one 256-thread block per 256 coefficients of a plane: block b covers plane
// b >> sh, coefficients ((b & (2^sh - 1)) << 8) + threadIdx.x (sh = log2 N - 8)
__global__ void k_expand_c1(uint64_t *__restrict__ out, const PrimeK *__restrict__ primes, int L, int N, Seed seed,
                            uint32_t first, uint32_t sh) {
  const uint32_t k = ((blockIdx.x & ((1u << sh) - 1u)) << 8) + threadIdx.x;
  const uint32_t p = blockIdx.x >> sh;   // jj * L + i
  const uint32_t i = p % (uint32_t)L, jj = p / (uint32_t)L;
  out[(size_t)p * N + k] = c1_residue(seed, first + jj, i, k, primes[i]);
}

// Multiply-accumulate left in the transformed domain: one thread per slot.
template <class A>
__global__ __launch_bounds__(256) void k_mac_slots(uint64_t *__restrict__ out, const uint64_t *__restrict__ ct_hat,
                                                   const uint64_t *__restrict__ pt_hat, TermArgs ta,
                                                   const PrimeK *__restrict__ primes, int L, int N, int accumulate) {
  const int sh = __builtin_ctz((unsigned)N) - 8;           // blocks of 256 per plane: 2^sh
  const int plane = (int)(blockIdx.x >> sh);
  const int k = (int)(((blockIdx.x & ((1u << sh) - 1u)) << 8) + threadIdx.x);
  const int i = plane % L;
  const int comp = (plane / L) & 1;
  const int o = plane / (2 * L);
  const PrimeK *pk = primes + i;
  const A ar(*pk);
  int t0, t1;
  term_range(ta, o, t0, t1);
  MacAcc<A> acc;
  for (int t = t0; t < t1; t += MacAcc<A>::kChunk) {
    const int te = min(t + MacAcc<A>::kChunk, t1);
    for (int tt = t; tt < te; ++tt) {
      const uint64_t a = ct_hat[((size_t)(term_ct(ta, tt) * 2 + comp) * L + i) * N + k];
      const uint64_t b = pt_hat[((size_t)term_pt(ta, tt) * L + i) * N + k];
      acc.add(ar, a, b);
    }
    acc.fold(ar, *pk);
  }
  uint64_t v = ar.store(acc.value());
  uint64_t *dst = out + (size_t)plane * N + k;
  *dst = accumulate ? canon_add(ar, *dst, v, pk->q) : v;
}

// ---------------------------------------------------------------- packing
__global__ void k_zero_i64(int64_t *p, size_t n) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) p[k] = 0;
}

// Weights w[M][C][h][h] -> polynomials [M][cb][N]: channel c of block c / Cw at
// offset -(c mod Cw) * S (stored at N - cc*S + p with the sign flipped, X^N = -1),
// within a channel w[a][b] at (h-1-a)*O + (h-1-b)  (pi_w, Eq. 2).
// dx: the kernel of an input gradient, w'[m][c][a][b] = w[c][m][h-1-a][h-1-b]
// read from the forward weights w [C][M][h][h] (M, C: the equivalent conv's).
__global__ void k_pack_conv_w(int64_t *__restrict__ polys, const int32_t *__restrict__ w, uint32_t M, uint32_t C,
                              uint32_t h, uint32_t O, uint32_t S, uint32_t Cw, uint32_t cb, uint32_t N, int dx) {
  const size_t total = (size_t)M * C * h * h;
  for (size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x; id < total; id += (size_t)gridDim.x * blockDim.x) {
    const uint32_t b = id % h, a = (id / h) % h, c = (id / ((size_t)h * h)) % C, m = id / ((size_t)h * h * C);
    const uint32_t blk = c / Cw, cc = c % Cw;
    const uint32_t p = (h - 1 - a) * O + (h - 1 - b);
    int64_t *poly = polys + ((size_t)m * cb + blk) * N;
    const size_t src = dx ? (((size_t)c * M + m) * h + (h - 1 - a)) * h + (h - 1 - b) : id;
    const int64_t v = w[src];
    if (cc == 0) poly[p] = v;
    else poly[N - cc * S + p] = -v;
  }
}

// FC weights W[n_out][n_in] -> [out_ct][in_ct][N]: W[i][j] at ii*n_iw + n_iw-1-jj.
__global__ void k_pack_fc_w(int64_t *__restrict__ polys, const int32_t *__restrict__ W, uint32_t n_out, uint32_t n_in,
                            uint32_t n_iw, uint32_t n_ow, uint32_t in_ct, uint32_t N) {
  const size_t total = (size_t)n_out * n_in;
  for (size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x; id < total; id += (size_t)gridDim.x * blockDim.x) {
    const uint32_t j = id % n_in, i = id / n_in;
    const uint32_t ko = i / n_ow, ii = i % n_ow, ki = j / n_iw, jj = j % n_iw;
    polys[((size_t)ko * in_ct + ki) * N + ii * n_iw + n_iw - 1 - jj] = W[id];
  }
}

__global__ void k_check_canonical(const uint64_t *__restrict__ planes, size_t n_planes, const PrimeK *primes, int L,
                                  int N, uint32_t *bad) {
  const size_t total = n_planes * (size_t)N;
  uint32_t cnt = 0;
  for (size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x; id < total; id += (size_t)gridDim.x * blockDim.x)
    cnt += planes[id] >= primes[(id / N) % L].q ? 1u : 0u;
  if (cnt) atomicAdd(bad, cnt);
}

// ---------------------------------------------------------- encryption helpers
template <class T>
__global__ void k_lift(uint64_t *__restrict__ out, const T *__restrict__ v, const PrimeK *primes, int L, int N) {
  const int total = L * N;
  for (int id = blockIdx.x * blockDim.x + threadIdx.x; id < total; id += gridDim.x * blockDim.x) {
    const int i = id / N, k = id % N;
    const int64_t x = (int64_t)v[k];
    const int64_t q = (int64_t)primes[i].q;
    int64_t r = x % q;
    out[id] = (uint64_t)(r < 0 ? r + q : r);
  }
}

__device__ __forceinline__ uint64_t mulmod_u128(uint64_t a, uint64_t b, const PrimeK &pk) {
  // a, b < q < 2^62: 128-bit product folded as in MacAcc<ArU64>
  const ArU64 ar(pk);
  const uint64_t lo = a * b, hi = __umul64hi(a, b);
  uint64_t x = ar.mul(hi, pk.r64, pk.r64s) + ar.mul(lo, 1, pk.one_s);
  x = x >= ar.two_q ? x - ar.two_q : x;
  return x >= pk.q ? x - pk.q : x;
}

__global__ void k_pmul_bcast(uint64_t *__restrict__ out, const uint64_t *__restrict__ x, const uint64_t *__restrict__ y,
                             const PrimeK *primes, int L, int N, size_t n_planes) {
  const size_t total = n_planes * N;
  for (size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x; id < total; id += (size_t)gridDim.x * blockDim.x) {
    const int i = (id / N) % L, k = id % N;
    out[id] = mulmod_u128(x[id], y[(size_t)i * N + k], primes[i]);
  }
}

__global__ void k_add_planes(uint64_t *__restrict__ out, const uint64_t *__restrict__ a, const uint64_t *__restrict__ b,
                             const PrimeK *primes, int L, int N, size_t n_planes) {
  const size_t total = n_planes * N;
  for (size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x; id < total; id += (size_t)gridDim.x * blockDim.x) {
    const uint64_t q = primes[(id / N) % L].q;
    const uint64_t s = a[id] + b[id];
    out[id] = s >= q ? s - q : s;
  }
}

// c0 = -prod + e + (Delta mod q_i) * m  (mod q_i); delta_w = [w_0..w_{L-1}, w'_0..w'_{L-1}] (Shoup)
__global__ void k_enc_combine(uint64_t *__restrict__ c0, const uint64_t *__restrict__ prod, const int32_t *__restrict__ e,
                              const int64_t *__restrict__ m, const uint64_t *__restrict__ delta_w, const PrimeK *primes,
                              int L, int N) {
  const int total = L * N;
  for (int id = blockIdx.x * blockDim.x + threadIdx.x; id < total; id += gridDim.x * blockDim.x) {
    const int i = id / N, k = id % N;
    const PrimeK &pk = primes[i];
    const ArU64 ar(pk);
    const uint64_t q = pk.q;
    uint64_t dm = ar.mul((uint64_t)m[k], delta_w[i], delta_w[L + i]);   // [0, 2q)
    dm = dm >= q ? dm - q : dm;
    const int64_t ev = e[k];
    const uint64_t er = ev < 0 ? q - (uint64_t)(-ev) : (uint64_t)ev;
    uint64_t s = dm + er;
    s = s >= q ? s - q : s;
    const uint64_t p = prod[id];
    s = s >= p ? s - p : s + q - p;
    c0[id] = s;
  }
}

__global__ void k_copy_u64(uint64_t *__restrict__ dst, const uint64_t *__restrict__ src, size_t n) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
    dst[k] = src[k];
}

// --------------------------------------------------------------- dispatch
static inline unsigned grid_for(size_t n, unsigned block) {
  size_t g = (n + block - 1) / block;
  if (g > 65535u * 4u) g = 65535u * 4u;
  return (unsigned)(g ? g : 1);
}

static hipError_t dispatch(const Ctx &c, const Sched &s, Op op, const LaunchArgs &la, hipStream_t st) {
  if (la.grid == 0) return hipSuccess;
  const bool f64 = s.arith == HE_ARITH_F64;
  if (f64 && !c.f64_ok) return hipErrorInvalidValue;
  switch (c.logN) {
    case 10: return run_ring_10(c, f64, s.loge, op, la, st);
    case 11: return run_ring_11(c, f64, s.loge, op, la, st);
    case 12: return run_ring_12(c, f64, s.loge, op, la, st);
    case 13: return run_ring_13(c, f64, s.loge, op, la, st);
    case 14: return run_ring_14(c, f64, s.loge, op, la, st);
    default: return hipErrorInvalidValue;
  }
}

bool sched_valid(uint32_t logN, const Sched &s) {
  const int logt = (int)logN - s.loge;
  if (logN < 10 || logN > 14) return false;
  if (s.loge < 3 || s.loge > 5) return false;
  return logt >= 6 && logt <= 10;
}

std::vector<Sched> schedules_for(uint32_t logN, bool f64_ok) {
  std::vector<Sched> v;
  for (int a : {HE_ARITH_F64, HE_ARITH_U64}) {
    if (a == HE_ARITH_F64 && !f64_ok) continue;
    for (int le = 3; le <= 5; ++le) {
      Sched s{a, le};
      if (sched_valid(logN, s)) v.push_back(s);
    }
  }
  return v;
}

hipError_t launch_ntt_fwd(const Ctx &c, const Sched &s, uint64_t *out, const uint64_t *in, uint32_t n_planes,
                          hipStream_t st) {
  LaunchArgs la{};
  la.out = out;
  la.in = in;
  la.grid = n_planes;
  return dispatch(c, s, OP_FWD, la, st);
}

hipError_t launch_ntt_fwd_seeded(const Ctx &c, const Sched &s, uint64_t *out, const uint64_t *ct0, uint64_t seed0,
                                 uint64_t seed1, uint32_t n_ct, hipStream_t st) {
  LaunchArgs la{};
  la.out = out;
  la.in = ct0;
  la.seed = Seed{seed0, seed1};
  la.grid = n_ct * 2 * c.L;
  return dispatch(c, s, OP_FWD_SEEDED, la, st);
}

hipError_t launch_expand_c1(const Ctx &c, uint64_t *out, uint64_t seed0, uint64_t seed1, uint32_t first, uint32_t n_ct,
                            hipStream_t st) {
  if (!n_ct) return hipSuccess;
  const uint32_t sh = c.logN - 8;
  hipLaunchKernelGGL(k_expand_c1, dim3((n_ct * c.L) << sh), dim3(256), 0, st, out, c.d_primes, (int)c.L, (int)c.N,
                     Seed{seed0, seed1}, first, sh);
  return hipGetLastError();
}

hipError_t launch_ntt_fwd_lift(const Ctx &c, const Sched &s, uint64_t *out, const int64_t *polys, uint32_t n_polys,
                               hipStream_t st) {
  LaunchArgs la{};
  la.out = out;
  la.polys = polys;
  la.grid = n_polys * c.L;
  return dispatch(c, s, OP_FWD_LIFT, la, st);
}

hipError_t launch_ntt_fwd_pack(const Ctx &c, const Sched &s, uint64_t *out, const int32_t *w, const WPack &wp,
                               uint32_t n_polys, hipStream_t st) {
  LaunchArgs la{};
  la.out = out;
  la.polys = (const int64_t *)w;
  la.wp = wp;
  la.grid = n_polys * c.L;
  return dispatch(c, s, OP_FWD_PACK, la, st);
}

hipError_t launch_ntt_fwd2(const Ctx &c, const Sched &s, uint64_t *out1, const uint64_t *in1, uint32_t n1_planes,
                           uint64_t *out2, const uint64_t *in2, uint32_t n2_planes, hipStream_t st) {
  LaunchArgs la{};
  la.out = out1;
  la.in = in1;
  la.n_first = (int)n1_planes;
  la.out2 = out2;
  la.pt = in2;
  la.grid = n1_planes + n2_planes;
  return dispatch(c, s, OP_FWD2, la, st);
}

hipError_t launch_ntt_fwd_ct_pack(const Ctx &c, const Sched &s, uint64_t *ct_out, const uint64_t *ct_in,
                                  uint32_t n_ct_planes, uint64_t *pt_out, const int32_t *w, const WPack &wp,
                                  uint32_t n_polys, hipStream_t st, const uint64_t *seed) {
  LaunchArgs la{};
  if (seed) {
    la.seeded = 1;
    la.seed = Seed{seed[0], seed[1]};
  }
  la.out = ct_out;
  la.in = ct_in;
  la.n_first = (int)n_ct_planes;
  la.out2 = pt_out;
  la.polys = (const int64_t *)w;
  la.wp = wp;
  la.grid = n_ct_planes + n_polys * c.L;
  return dispatch(c, s, OP_FWD_CT_PACK, la, st);
}

hipError_t launch_ntt_inv(const Ctx &c, const Sched &s, uint64_t *out, const uint64_t *in, uint32_t n_planes,
                          hipStream_t st) {
  LaunchArgs la{};
  la.out = out;
  la.in = in;
  la.grid = n_planes;
  return dispatch(c, s, OP_INV, la, st);
}

hipError_t launch_mac(const Ctx &c, const Sched &s, uint64_t *out, const uint64_t *ct_hat, const uint64_t *pt_hat,
                      const Terms &tm, bool accumulate, bool out_ntt, hipStream_t st, int ncomp) {
  TermArgs ta{tm.row, tm.cti, tm.pti, tm.K};
  const uint32_t n_planes = tm.n_out * (uint32_t)ncomp * c.L;
  if (ncomp != 1 && ncomp != 2) return hipErrorInvalidValue;
  if (ncomp == 1 && (out_ntt || accumulate)) return hipErrorInvalidValue;
  if (n_planes == 0) return hipSuccess;
  if (out_ntt) {
    const dim3 grid(n_planes << (c.logN - 8));   // 256 coefficients per block, planes along x
    if (s.arith == HE_ARITH_F64 && c.f64_ok)
      hipLaunchKernelGGL(k_mac_slots<ArF64>, grid, dim3(256), 0, st, out, ct_hat, pt_hat, ta, c.d_primes, (int)c.L,
                         (int)c.N, accumulate ? 1 : 0);
    else
      hipLaunchKernelGGL(k_mac_slots<ArU64>, grid, dim3(256), 0, st, out, ct_hat, pt_hat, ta, c.d_primes, (int)c.L,
                         (int)c.N, accumulate ? 1 : 0);
    return hipGetLastError();
  }
  LaunchArgs la{};
  la.out = out;
  la.in = ct_hat;
  la.pt = pt_hat;
  la.ta = ta;
  la.accumulate = accumulate ? 1 : 0;
  la.ncomp = ncomp;
  la.grid = n_planes;
  return dispatch(c, s, OP_MAC_INV, la, st);
}

hipError_t launch_zero_i64(int64_t *p, size_t n, hipStream_t st) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_zero_i64, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_pack_conv_w(int64_t *polys, const int32_t *w, uint32_t M, uint32_t C, uint32_t h, uint32_t O,
                              uint32_t S, uint32_t Cw, uint32_t cb, uint32_t N, bool dx, hipStream_t st) {
  const size_t total = (size_t)M * C * h * h;
  if (!total) return hipSuccess;
  hipLaunchKernelGGL(k_pack_conv_w, dim3(grid_for(total, 256)), dim3(256), 0, st, polys, w, M, C, h, O, S, Cw, cb, N,
                     dx ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_pack_fc_w(int64_t *polys, const int32_t *W, uint32_t n_out, uint32_t n_in, uint32_t n_iw,
                            uint32_t n_ow, uint32_t in_ct, uint32_t N, hipStream_t st) {
  const size_t total = (size_t)n_out * n_in;
  if (!total) return hipSuccess;
  hipLaunchKernelGGL(k_pack_fc_w, dim3(grid_for(total, 256)), dim3(256), 0, st, polys, W, n_out, n_in, n_iw, n_ow,
                     in_ct, N);
  return hipGetLastError();
}

hipError_t launch_check_canonical(const Ctx &c, const uint64_t *planes, size_t n_planes, uint32_t *bad,
                                  hipStream_t st) {
  const size_t total = n_planes * c.N;
  if (!total) return hipSuccess;
  hipLaunchKernelGGL(k_check_canonical, dim3(grid_for(total, 256)), dim3(256), 0, st, planes, n_planes, c.d_primes,
                     (int)c.L, (int)c.N, bad);
  return hipGetLastError();
}

template <class T>
hipError_t launch_lift(const Ctx &c, uint64_t *out, const T *v, hipStream_t st) {
  const size_t total = (size_t)c.L * c.N;
  hipLaunchKernelGGL(k_lift<T>, dim3(grid_for(total, 256)), dim3(256), 0, st, out, v, c.d_primes, (int)c.L, (int)c.N);
  return hipGetLastError();
}
template hipError_t launch_lift<int8_t>(const Ctx &, uint64_t *, const int8_t *, hipStream_t);
template hipError_t launch_lift<int32_t>(const Ctx &, uint64_t *, const int32_t *, hipStream_t);
template hipError_t launch_lift<int64_t>(const Ctx &, uint64_t *, const int64_t *, hipStream_t);

hipError_t launch_pmul_bcast(const Ctx &c, uint64_t *out, const uint64_t *x, const uint64_t *y, uint32_t n_planes,
                             hipStream_t st) {
  const size_t total = (size_t)n_planes * c.N;
  hipLaunchKernelGGL(k_pmul_bcast, dim3(grid_for(total, 256)), dim3(256), 0, st, out, x, y, c.d_primes, (int)c.L,
                     (int)c.N, (size_t)n_planes);
  return hipGetLastError();
}

hipError_t launch_add_planes(const Ctx &c, uint64_t *out, const uint64_t *a, const uint64_t *b, uint32_t n_planes,
                             hipStream_t st) {
  const size_t total = (size_t)n_planes * c.N;
  hipLaunchKernelGGL(k_add_planes, dim3(grid_for(total, 256)), dim3(256), 0, st, out, a, b, c.d_primes, (int)c.L,
                     (int)c.N, (size_t)n_planes);
  return hipGetLastError();
}

hipError_t launch_enc_combine(const Ctx &c, uint64_t *c0, const uint64_t *prod, const int32_t *e, const int64_t *m,
                              const uint64_t *delta_w, hipStream_t st) {
  const size_t total = (size_t)c.L * c.N;
  hipLaunchKernelGGL(k_enc_combine, dim3(grid_for(total, 256)), dim3(256), 0, st, c0, prod, e, m, delta_w, c.d_primes,
                     (int)c.L, (int)c.N);
  return hipGetLastError();
}

hipError_t launch_copy_u64(uint64_t *dst, const uint64_t *src, size_t n, hipStream_t st) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_copy_u64, dim3(grid_for(n, 256)), dim3(256), 0, st, dst, src, n);
  return hipGetLastError();
}

}  // namespace he
