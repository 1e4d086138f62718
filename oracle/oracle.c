/*
 * CPU oracle for the homomorphic linear-layer path of CryptoTrain
 * (arXiv 2409.16675).  TEST INFRASTRUCTURE ONLY: nothing in the product
 * library links, loads or calls this file; only the tests, the smoke entry
 * point and the benchmark's CPU-baseline leg do.
 *
 * Everything here is the plain definition of an exact integer result:
 *   - arithmetic in Z_q via 128-bit products and the C '%' operator;
 *   - the ring A_{N,q} = Z_q[X]/(X^N+1) of Section 2 ("Notations"), whose
 *     product is written out as the schoolbook negacyclic convolution;
 *   - the number-theoretic transform at the library boundary, defined as the
 *     evaluation of a polynomial at the odd powers of a primitive 2N-th root
 *     psi, listed in bit-reversed order (the paper never names the NTT; this
 *     order is a reading, stated where it is used);
 *   - CPMul (ciphertext x plaintext: each of the two ciphertext components is
 *     multiplied by the plaintext polynomial, Section 2 "Motivation") and
 *     CCAdd (component-wise sum), giving the multiply-accumulate that the
 *     online phase of CryptoTrain-P evaluates (Section 3.2).
 *
 * A faster transform (twist by psi^j, then a recursive radix-2 cyclic
 * transform, then a bit-reversal permutation) is provided only so that the
 * tests can compute full expected outputs at N = 8192; it is checked in the
 * test suite against the direct O(N^2) definition below.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

uint64_t orc_mulmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a * b) % q); }
uint64_t orc_addmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a + b) % q); }
uint64_t orc_submod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a + q - (b % q)) % q); }

uint64_t orc_powmod(uint64_t a, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  a %= q;
  while (e) {
    if (e & 1) r = orc_mulmod(r, a, q);
    a = orc_mulmod(a, a, q);
    e >>= 1;
  }
  return r;
}

/* Deterministic Miller-Rabin for n < 2^64 (the first 12 primes as bases are
 * a known sufficient witness set for 64-bit integers). */
int orc_is_prime(uint64_t n) {
  static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return 0;
  for (int i = 0; i < 12; ++i) {
    if (n == bases[i]) return 1;
    if (n % bases[i] == 0) return 0;
  }
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  for (int i = 0; i < 12; ++i) {
    uint64_t x = orc_powmod(bases[i], d, n);
    if (x == 1 || x == n - 1) continue;
    int composite = 1;
    for (int r = 1; r < s; ++r) {
      x = orc_mulmod(x, x, n);
      if (x == n - 1) { composite = 0; break; }
    }
    if (composite) return 0;
  }
  return 1;
}

/* The L largest primes q < 2^bits with q == 1 (mod 2N), in decreasing order.
 * Returns the number found (L on success). */
int orc_find_primes(uint32_t N, uint32_t bits, uint32_t L, uint64_t *out) {
  uint64_t m = 2ull * N;
  uint64_t top = (bits >= 64) ? UINT64_MAX : ((1ull << bits) - 1);
  uint64_t c = top - ((top - 1) % m);   /* largest value <= top that is 1 mod m */
  uint32_t found = 0;
  while (found < L && c > m) {
    if (orc_is_prime(c)) out[found++] = c;
    c -= m;
  }
  return (int)found;
}

/* Smallest x in [2, q) with x^N == -1 (mod q).  For N a power of two these x
 * are exactly the primitive 2N-th roots of unity, i.e. the odd powers of any
 * one of them, so the set is enumerated instead of scanning [2, q):
 *   z   = least quadratic non-residue (z^((q-1)/2) == -1),
 *   r   = z^((q-1)/(2N))  has r^N == -1, hence order 2N,
 *   psi = min over odd k < 2N of r^k.
 * Returns 0 if 2N does not divide q-1. */
uint64_t orc_min_psi(uint32_t N, uint64_t q) {
  uint64_t m = 2ull * N;
  if ((q - 1) % m != 0) return 0;
  uint64_t z = 2;
  while (orc_powmod(z, (q - 1) / 2, q) != q - 1) ++z;
  uint64_t r = orc_powmod(z, (q - 1) / m, q);
  uint64_t r2 = orc_mulmod(r, r, q), x = r, best = r;
  for (uint64_t k = 3; k < m; k += 2) {
    x = orc_mulmod(x, r2, q);
    if (x < best) best = x;
  }
  return best;
}

/* Linear-scan definition of the same value, usable for small q only (pins the above). */
uint64_t orc_min_psi_scan(uint32_t N, uint64_t q) {
  for (uint64_t x = 2; x < q; ++x)
    if (orc_powmod(x, N, q) == q - 1) return x;
  return 0;
}

static uint32_t bitrev(uint32_t v, uint32_t logn) {
  uint32_t r = 0;
  for (uint32_t i = 0; i < logn; ++i) { r = (r << 1) | (v & 1); v >>= 1; }
  return r;
}
static uint32_t ilog2(uint32_t n) { uint32_t l = 0; while ((1u << l) < n) ++l; return l; }

/* Schoolbook product in Z_q[X]/(X^N+1):
 *   c_k = sum_{i+j=k} a_i b_j  -  sum_{i+j=k+N} a_i b_j   (mod q). */
void orc_negacyclic_mul(const uint64_t *a, const uint64_t *b, uint32_t N, uint64_t q, uint64_t *c) {
  for (uint32_t k = 0; k < N; ++k) c[k] = 0;
  for (uint32_t i = 0; i < N; ++i) {
    if (a[i] == 0) continue;
    for (uint32_t j = 0; j < N; ++j) {
      uint64_t p = orc_mulmod(a[i], b[j], q);
      uint32_t k = i + j;
      if (k < N) c[k] = orc_addmod(c[k], p, q);
      else c[k - N] = orc_submod(c[k - N], p, q);
    }
  }
}

/* One coefficient k of the schoolbook product above (O(N)). */
uint64_t orc_negacyclic_coeff(const uint64_t *a, const uint64_t *b, uint32_t N, uint64_t q, uint32_t k) {
  uint64_t acc = 0;
  for (uint32_t i = 0; i < N; ++i) {
    uint64_t p;
    if (i <= k) {
      p = orc_mulmod(a[i], b[k - i], q);
      acc = orc_addmod(acc, p, q);
    } else {
      p = orc_mulmod(a[i], b[k + N - i], q);
      acc = orc_submod(acc, p, q);
    }
  }
  return acc;
}

/* Transform definition: out[k] = a(psi^(2*brv(k)+1)) = sum_j a_j psi^((2 brv(k)+1) j). */
uint64_t orc_ntt_coeff(const uint64_t *a, uint32_t N, uint64_t q, uint64_t psi, uint32_t k) {
  uint32_t logn = ilog2(N);
  uint64_t x = orc_powmod(psi, 2ull * bitrev(k, logn) + 1, q);
  /* Horner evaluation of a at x */
  uint64_t acc = 0;
  for (uint32_t j = N; j-- > 0;) acc = orc_addmod(orc_mulmod(acc, x, q), a[j] % q, q);
  return acc;
}

void orc_ntt_direct(const uint64_t *a, uint32_t N, uint64_t q, uint64_t psi, uint64_t *out) {
  for (uint32_t k = 0; k < N; ++k) out[k] = orc_ntt_coeff(a, N, q, psi, k);
}

/* Inverse of the definition: a_j = N^{-1} sum_k A[k] psi^{-(2 brv(k)+1) j}. */
void orc_intt_direct(const uint64_t *A, uint32_t N, uint64_t q, uint64_t psi, uint64_t *out) {
  uint32_t logn = ilog2(N);
  uint64_t psi_inv = orc_powmod(psi, q - 2, q);
  uint64_t n_inv = orc_powmod(N, q - 2, q);
  for (uint32_t j = 0; j < N; ++j) {
    uint64_t acc = 0;
    for (uint32_t k = 0; k < N; ++k) {
      uint64_t e = ((2ull * bitrev(k, logn) + 1) * j) % (2ull * N);
      acc = orc_addmod(acc, orc_mulmod(A[k], orc_powmod(psi_inv, e, q), q), q);
    }
    out[j] = orc_mulmod(acc, n_inv, q);
  }
}

/* Recursive radix-2 cyclic transform: X[k] = sum_j x_j w^(j k), k < n (natural order). */
static void cyclic_fft(uint64_t *x, uint32_t n, uint64_t w, uint64_t q, uint64_t *tmp) {
  if (n == 1) return;
  uint32_t h = n / 2;
  uint64_t *ev = tmp, *od = tmp + h;
  for (uint32_t j = 0; j < h; ++j) { ev[j] = x[2 * j]; od[j] = x[2 * j + 1]; }
  uint64_t w2 = orc_mulmod(w, w, q);
  cyclic_fft(ev, h, w2, q, x);          /* x is free scratch of size n here */
  cyclic_fft(od, h, w2, q, x);
  uint64_t wk = 1;
  for (uint32_t k = 0; k < h; ++k) {
    uint64_t t = orc_mulmod(wk, od[k], q);
    x[k] = orc_addmod(ev[k], t, q);
    x[k + h] = orc_submod(ev[k], t, q);
    wk = orc_mulmod(wk, w, q);
  }
}

/* Same result as orc_ntt_direct, O(N log N): a(psi^(2m+1)) = sum_j (a_j psi^j) (psi^2)^(j m),
 * then slot k holds m = brv(k). */
void orc_ntt_fast(const uint64_t *a, uint32_t N, uint64_t q, uint64_t psi, uint64_t *out) {
  uint32_t logn = ilog2(N);
  uint64_t *x = (uint64_t *)malloc(sizeof(uint64_t) * N);
  uint64_t *tmp = (uint64_t *)malloc(sizeof(uint64_t) * N);
  uint64_t pj = 1;
  for (uint32_t j = 0; j < N; ++j) { x[j] = orc_mulmod(a[j] % q, pj, q); pj = orc_mulmod(pj, psi, q); }
  cyclic_fft(x, N, orc_mulmod(psi, psi, q), q, tmp);
  for (uint32_t k = 0; k < N; ++k) out[k] = x[bitrev(k, logn)];
  free(x);
  free(tmp);
}

/* Inverse of orc_ntt_fast: undo the permutation, inverse cyclic transform
 * (with w^-1 and a factor N^-1), then untwist by psi^-j. */
void orc_intt_fast(const uint64_t *A, uint32_t N, uint64_t q, uint64_t psi, uint64_t *out) {
  uint32_t logn = ilog2(N);
  uint64_t *x = (uint64_t *)malloc(sizeof(uint64_t) * N);
  uint64_t *tmp = (uint64_t *)malloc(sizeof(uint64_t) * N);
  for (uint32_t k = 0; k < N; ++k) x[bitrev(k, logn)] = A[k] % q;
  uint64_t psi_inv = orc_powmod(psi, q - 2, q);
  cyclic_fft(x, N, orc_mulmod(psi_inv, psi_inv, q), q, tmp);
  uint64_t n_inv = orc_powmod(N, q - 2, q);
  uint64_t pj = n_inv;
  for (uint32_t j = 0; j < N; ++j) { out[j] = orc_mulmod(x[j], pj, q); pj = orc_mulmod(pj, psi_inv, q); }
  free(x);
  free(tmp);
}

/*
 * Multiply-accumulate over a term list (CPMul followed by CCAdd).
 *   ct  : [n_ct][2][L][N]  ciphertexts, residues in [0, q_i)
 *   pt  : [n_pt][L][N]     plaintext polynomials, residues in [0, q_i)
 *   out : [n_out][2][L][N]
 * Output o is  sum_{t in [row[o], row[o+1])}  ct[ct_idx[t]] (x) pt[pt_idx[t]]
 * component by component and prime by prime, where (x) is the ring product.
 * method 0: every ring product by the schoolbook definition;
 * method 1: ring products through orc_ntt_fast / pointwise / orc_intt_fast.
 * Planes are independent, so they are spread over OpenMP threads.
 */
void orc_csr_cpmul(const uint64_t *ct, const uint64_t *pt, const int32_t *row, const int32_t *ct_idx,
                   const int32_t *pt_idx, uint32_t n_out, uint32_t N, uint32_t L, const uint64_t *q,
                   const uint64_t *psi, uint64_t *out, int method) {
  long total = (long)n_out * 2 * L;
#pragma omp parallel
  {
    uint64_t *prod = (uint64_t *)malloc(sizeof(uint64_t) * N);
    uint64_t *fa = (uint64_t *)malloc(sizeof(uint64_t) * N);
    uint64_t *fb = (uint64_t *)malloc(sizeof(uint64_t) * N);
    uint64_t *facc = (uint64_t *)malloc(sizeof(uint64_t) * N);
#pragma omp for schedule(dynamic)
    for (long w = 0; w < total; ++w) {
      uint32_t o = (uint32_t)(w / (2 * L));
      uint32_t c = (uint32_t)((w / L) % 2);
      uint32_t i = (uint32_t)(w % L);
      uint64_t *dst = out + (((size_t)o * 2 + c) * L + i) * N;
      for (uint32_t k = 0; k < N; ++k) dst[k] = 0;
      if (method == 1)
        for (uint32_t k = 0; k < N; ++k) facc[k] = 0;
      for (int32_t t = row[o]; t < row[o + 1]; ++t) {
        const uint64_t *a = ct + (((size_t)ct_idx[t] * 2 + c) * L + i) * N;
        const uint64_t *b = pt + ((size_t)pt_idx[t] * L + i) * N;
        if (method == 0) {
          orc_negacyclic_mul(a, b, N, q[i], prod);
          for (uint32_t k = 0; k < N; ++k) dst[k] = orc_addmod(dst[k], prod[k], q[i]);
        } else {
          orc_ntt_fast(a, N, q[i], psi[i], fa);
          orc_ntt_fast(b, N, q[i], psi[i], fb);
          for (uint32_t k = 0; k < N; ++k) facc[k] = orc_addmod(facc[k], orc_mulmod(fa[k], fb[k], q[i]), q[i]);
        }
      }
      if (method == 1) orc_intt_fast(facc, N, q[i], psi[i], dst);
    }
    free(prod);
    free(fa);
    free(fb);
    free(facc);
  }
}

/* Same result as orc_csr_cpmul, with every input plane transformed once
 * (orc_ntt_fast) and cached: out = INTT( sum_t NTT(ct) * NTT(pt) ).  Needs
 * n_ct*2*L + n_pt*L planes of scratch, allocated here. */
void orc_csr_cpmul_cached(const uint64_t *ct, const uint64_t *pt, uint32_t n_ct, uint32_t n_pt, const int32_t *row,
                          const int32_t *ct_idx, const int32_t *pt_idx, uint32_t n_out, uint32_t N, uint32_t L,
                          const uint64_t *q, const uint64_t *psi, uint64_t *out) {
  size_t nct = (size_t)n_ct * 2 * L, npt = (size_t)n_pt * L;
  uint64_t *fct = (uint64_t *)malloc(sizeof(uint64_t) * N * nct);
  uint64_t *fpt = (uint64_t *)malloc(sizeof(uint64_t) * N * npt);
#pragma omp parallel for schedule(dynamic)
  for (long w = 0; w < (long)(nct + npt); ++w) {
    if ((size_t)w < nct) orc_ntt_fast(ct + (size_t)w * N, N, q[w % L], psi[w % L], fct + (size_t)w * N);
    else {
      size_t v = (size_t)w - nct;
      orc_ntt_fast(pt + v * N, N, q[v % L], psi[v % L], fpt + v * N);
    }
  }
  long total = (long)n_out * 2 * L;
#pragma omp parallel
  {
    uint64_t *facc = (uint64_t *)malloc(sizeof(uint64_t) * N);
#pragma omp for schedule(dynamic)
    for (long w = 0; w < total; ++w) {
      uint32_t o = (uint32_t)(w / (2 * L));
      uint32_t c = (uint32_t)((w / L) % 2);
      uint32_t i = (uint32_t)(w % L);
      for (uint32_t k = 0; k < N; ++k) facc[k] = 0;
      for (int32_t t = row[o]; t < row[o + 1]; ++t) {
        const uint64_t *a = fct + (((size_t)ct_idx[t] * 2 + c) * L + i) * N;
        const uint64_t *b = fpt + ((size_t)pt_idx[t] * L + i) * N;
        for (uint32_t k = 0; k < N; ++k) facc[k] = orc_addmod(facc[k], orc_mulmod(a[k], b[k], q[i]), q[i]);
      }
      orc_intt_fast(facc, N, q[i], psi[i], out + (((size_t)o * 2 + c) * L + i) * N);
    }
    free(facc);
  }
  free(fct);
  free(fpt);
}

/* One output coefficient of orc_csr_cpmul, by the schoolbook definition (O(N * terms)). */
uint64_t orc_csr_cpmul_coeff(const uint64_t *ct, const uint64_t *pt, const int32_t *row, const int32_t *ct_idx,
                             const int32_t *pt_idx, uint32_t N, uint32_t L, const uint64_t *q, uint32_t o,
                             uint32_t c, uint32_t i, uint32_t k) {
  uint64_t acc = 0;
  for (int32_t t = row[o]; t < row[o + 1]; ++t) {
    const uint64_t *a = ct + (((size_t)ct_idx[t] * 2 + c) * L + i) * N;
    const uint64_t *b = pt + ((size_t)pt_idx[t] * L + i) * N;
    acc = orc_addmod(acc, orc_negacyclic_coeff(a, b, N, q[i], k), q[i]);
  }
  return acc;
}

/* Batched transforms over [n][L][N] planes (OpenMP over planes); direction 0 forward, 1 inverse. */
void orc_ntt_planes(const uint64_t *in, uint32_t n, uint32_t N, uint32_t L, const uint64_t *q,
                    const uint64_t *psi, uint64_t *out, int inverse) {
  long total = (long)n * L;
#pragma omp parallel for schedule(dynamic)
  for (long w = 0; w < total; ++w) {
    uint32_t i = (uint32_t)(w % L);
    if (inverse) orc_intt_fast(in + (size_t)w * N, N, q[i], psi[i], out + (size_t)w * N);
    else orc_ntt_fast(in + (size_t)w * N, N, q[i], psi[i], out + (size_t)w * N);
  }
}

/* Ring product of many plane pairs: out[p] = a[p] (x) b[p] mod q[p % L] (schoolbook, OpenMP). */
void orc_negacyclic_mul_planes(const uint64_t *a, const uint64_t *b, uint32_t n, uint32_t N, uint32_t L,
                               const uint64_t *q, uint64_t *out) {
  long total = (long)n * L;
#pragma omp parallel for schedule(dynamic)
  for (long w = 0; w < total; ++w)
    orc_negacyclic_mul(a + (size_t)w * N, b + (size_t)w * N, N, q[w % L], out + (size_t)w * N);
}

/* ---------------------------------------------------------------- seeded c1
 * The client may send a seed instead of the uniform ciphertext component c1,
 * the server regenerating c1 from it (Section 7, Discussion, on the upload cost).
 * Generator: Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC 2011), a counter-based bijection of a
 * 256-bit counter under a 128-bit key: ten rounds, each multiplying two
 * counter words by fixed odd constants into 128-bit products and mixing their
 * halves with the other two words and the key, the key stepping by two Weyl
 * constants between rounds.
 * Reading (not in the paper): coefficient k of component 1 of ciphertext j at
 * prime i is (w0 * 2^64 + w1) mod q_i with (w0, w1, w2, w3) =
 * Philox4x64-10(counter (k, j, i, 0), key (seed0, seed1)); 128 random bits
 * per residue keep the distance from uniform below 2^-78. */
void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3], k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    const u128 p0 = (u128)M0 * c0, p1 = (u128)M1 * c2;
    const uint64_t n0 = (uint64_t)(p1 >> 64) ^ c1 ^ k0, n1 = (uint64_t)p1;
    const uint64_t n2 = (uint64_t)(p0 >> 64) ^ c3 ^ k1, n3 = (uint64_t)p0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
    k0 += W0;
    k1 += W1;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* out [L][N]: component 1 of ciphertext j regenerated from the seed */
void orc_expand_c1(uint64_t seed0, uint64_t seed1, uint64_t j, const uint64_t *q, uint32_t L, uint32_t N,
                   uint64_t *out) {
  const uint64_t key[2] = {seed0, seed1};
  for (uint32_t i = 0; i < L; ++i)
    for (uint32_t k = 0; k < N; ++k) {
      const uint64_t ctr[4] = {k, j, i, 0};
      uint64_t w[4];
      orc_philox4x64(ctr, key, w);
      out[(size_t)i * N + k] = (uint64_t)((((u128)w[0] << 64) | w[1]) % q[i]);
    }
}

int orc_num_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}
