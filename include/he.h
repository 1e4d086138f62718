/*
 * he.h -- C ABI of the MI355X homomorphic linear-layer library (libhe.so).
 *
 * The operations are those of CryptoTrain (arXiv 2409.16675):
 *   - the ring A_{N,q} = Z_q[X]/(X^N+1) of Section 2 ("Notations"), held in
 *     residue-number-system form: one plane of N coefficients per prime q_i;
 *   - CPMul, the ciphertext x plaintext product (c0*p, c1*p) of Section 2
 *     ("Motivation"), and CCAdd, the component-wise sum; together they form
 *     the multiply-accumulate that the online phase of CryptoTrain-P runs on
 *     the server (Section 3.2, c = [x](w - r_w) + [w](x - r_x) + [r_x r_w]);
 *   - the correlation-aware packings pi_x and pi_w of Section 3.3 (Eq. 1 and
 *     Eq. 2), extended to channels, weight gradients and FC layers;
 *   - test-only encryption and decryption (Section 2, "HE": the homomorphic
 *     property sigma(eps(x) o eps(y)) = sigma(eps(x (x) y))).
 *
 * Conventions
 *   Layout     A plane is N contiguous uint64 coefficients; a plaintext is
 *              [L][N]; a ciphertext is [2][L][N] (component, prime, coefficient).
 *              Arrays of polynomials are packed back to back.
 *   Values     Every uint64 coefficient crossing this boundary is canonical,
 *              in [0, q_i).  Inputs outside that range give undefined results
 *              unless HE_VALIDATE is set, in which case HE_ERANGE is returned.
 *   Transform  he_ntt_fwd maps coefficients a_j to slots
 *                A[k] = sum_j a_j psi^((2*brv(k)+1)*j)   (mod q_i),
 *              brv = bit reversal over log2 N bits, psi the primitive 2N-th
 *              root reported by he_ctx_moduli.  he_ntt_inv is its inverse.
 *   Memory     Pointers marked "device" are device memory on the context's
 *              device (for example the data pointer of a torch tensor); "host"
 *              pointers are ordinary host memory.  The caller owns every buffer
 *              and workspace it passes; the library owns only what its create
 *              calls return.  Device calls are asynchronous on `stream` (a
 *              hipStream_t passed as void*; NULL is the null stream) and do not
 *              allocate device memory unless stated.
 *   Errors     Every call returns HE_OK (0) or a negative he_status and never
 *              aborts.  he_last_error() gives a thread-local description of the
 *              most recent failure; HIP failures map to HE_EDEVICE.
 *   Threads    Calls on different contexts are independent; calls that share a
 *              context may run concurrently on different streams.
 */
#ifndef HE_H
#define HE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t he_status;
#define HE_OK 0
#define HE_EINVAL (-1)        /* bad argument, shape or size */
#define HE_EUNSUPPORTED (-2)  /* valid request this build does not handle */
#define HE_ENOMEM (-3)        /* an allocation failed, or a workspace is too small */
#define HE_EDEVICE (-4)       /* a HIP runtime call failed */
#define HE_ERANGE (-5)        /* a coefficient outside [0, q_i) (only with HE_VALIDATE) */
#define HE_EBUSY (-6)         /* admission refused: the job does not fit the memory cap */
#define HE_ETIMEOUT (-7)      /* a wait ended before the job finished */

typedef struct he_ctx he_ctx;
typedef struct he_plan he_plan;
typedef struct he_batch he_batch;
typedef struct he_server he_server;

/* Arithmetic used inside the kernels.  Results are identical (canonical
 * residues); only speed and the admissible primes differ. */
#define HE_ARITH_AUTO 0   /* F64 when every q_i < 2^48, else U64 */
#define HE_ARITH_F64 1    /* exact products through fp64 FMA; needs q_i < 2^48 */
#define HE_ARITH_U64 2    /* Shoup products through 32-bit integer multiplies; q_i < 2^62 */

typedef struct {
  uint32_t N;            /* ring degree, a power of two in [1024, 16384] */
  uint32_t L;            /* number of primes, 1..8 */
  uint32_t prime_bits;   /* when q == NULL: the L largest primes below 2^prime_bits with q_i = 1 mod 2N */
  uint32_t arith;        /* HE_ARITH_* */
  const uint64_t *q;     /* host, optional [L] explicit primes (each = 1 mod 2N, < 2^62) */
  uint64_t t;            /* plaintext modulus, coprime to every q_i, 2 <= t < 2^32 */
  int32_t device;        /* HIP device ordinal */
  int32_t reserved;
} he_params;

/* Create a context: primes, roots psi_i (the smallest x with x^N = -1 mod q_i),
 * twiddle tables and constants, uploaded to `device`.  Allocates device memory. */
he_status he_ctx_create(const he_params *params, he_ctx **out);
he_status he_ctx_destroy(he_ctx *ctx);
/* Host outputs, each [L]: the primes and the roots psi_i.  Either may be NULL. */
he_status he_ctx_moduli(const he_ctx *ctx, uint64_t *q_out, uint64_t *psi_out);
/* Ring degree, prime count, plaintext modulus and arithmetic in use (any may be NULL). */
he_status he_ctx_info(const he_ctx *ctx, uint32_t *N, uint32_t *L, uint64_t *t, uint32_t *arith);

/* Device resources of the protocol steps beside the layer path, built ahead
 * of time so that the hot calls allocate nothing:
 *   HE_PREPARE_PPMUL  the ring of the plaintext modulus, Z_t[X]/(X^N+1), for
 *                     he_ppmul (HE_EUNSUPPORTED unless t is prime and 1 mod 2N);
 *   HE_PREPARE_CCMUL  the extended base Q u P of he_ccmul with its conversion
 *                     constants, and two pinned staging buffers for term lists
 *                     of up to ccmul_max_out outputs and ccmul_max_terms
 *                     products (a later call with larger values grows them).
 * Allocates device and pinned host memory owned by the context; not to be
 * called while calls on the same context run.  he_ppmul, he_ccmul and
 * he_ccmul_ws_size return HE_EINVAL until their resources are prepared. */
#define HE_PREPARE_PPMUL 0x1u
#define HE_PREPARE_CCMUL 0x2u
he_status he_ctx_prepare(he_ctx *ctx, uint32_t ops, uint32_t ccmul_max_out, uint32_t ccmul_max_terms);

/* Kernel schedule used for one operation: arithmetic (HE_ARITH_F64 / HE_ARITH_U64)
 * and log2 of the coefficients each thread holds (3, 4 or 5; the plane is split
 * over N >> loge threads, which must be 64..1024).  Every schedule returns the
 * same bytes; the autotuner picks the fastest.  HE_EUNSUPPORTED if not compiled
 * for this N or if F64 is asked with a prime >= 2^48. */
#define HE_OP_FWD 0   /* forward transforms (inputs and plaintexts) */
#define HE_OP_INV 1   /* stand-alone inverse transforms */
#define HE_OP_MAC 2   /* fused multiply-accumulate + inverse transform */
he_status he_ctx_set_schedule(he_ctx *ctx, uint32_t op, uint32_t arith, uint32_t loge);
he_status he_ctx_get_schedule(const he_ctx *ctx, uint32_t op, uint32_t *arith, uint32_t *loge);

/* Autotuner: times every compiled schedule of the forward transform, the inverse
 * transform and the fused multiply-accumulate + inverse kernel on n_polys
 * polynomials of seeded data, keeps only candidates whose output is identical
 * to the reference schedule's, and installs the fastest in the context
 * (candidates within 5% of the fastest count as a tie, broken in a fixed order:
 * fp64 arithmetic first, then 16, 32, 8 coefficients per thread).  With
 * cache_path, a matching entry (device architecture, N, L, first prime) is read
 * instead of timing, and a new result is appended as one JSON line.  `report`
 * (optional, host) receives up to report_cap entries.  Allocates and frees
 * device memory; synchronises `stream`. */
typedef struct {
  uint32_t op, arith, loge, exact;
  double us;               /* average time per launch */
} he_tune_entry;
he_status he_autotune(he_ctx *ctx, uint32_t n_polys, const char *cache_path, void *stream, he_tune_entry *report,
                      uint32_t report_cap, uint32_t *report_n);

/* ---------------------------------------------------------------- transforms */

/* In-place forward transform of n_polys polynomials, device planes [n_polys][L][N]. */
he_status he_ntt_fwd(he_ctx *ctx, uint64_t *planes, uint32_t n_polys, void *stream);
/* In-place inverse transform (exact inverse of he_ntt_fwd), same layout. */
he_status he_ntt_inv(he_ctx *ctx, uint64_t *planes, uint32_t n_polys, void *stream);

/* ------------------------------------------------------- CPMul + accumulate */

/* Flags for he_cpmul_acc and he_corr_conv2d. */
#define HE_IN_COEFF 0x0u       /* inputs in coefficient form (default) */
#define HE_IN_NTT 0x1u         /* inputs already transformed by he_ntt_fwd */
#define HE_OUT_COEFF 0x0u      /* output in coefficient form (default) */
#define HE_OUT_NTT 0x2u        /* output left in transformed form */
#define HE_OVERWRITE 0x0u      /* acc = sum (default) */
#define HE_ACCUMULATE 0x4u     /* acc += sum; acc is read in the output form */
#define HE_VALIDATE 0x8u       /* check that inputs are canonical (extra pass) */
#define HE_PLAIN_RAW 0x0u      /* he_corr_conv2d: `plain` holds raw int32 weights (default) */
#define HE_PLAIN_POLY 0x10u    /* he_corr_conv2d: `plain` holds packed int64 polynomials */
#define HE_FUSED 0x0u          /* one fused multiply-accumulate + inverse-transform kernel (default) */
#define HE_UNFUSED 0x20u       /* separate transform, multiply-accumulate and inverse kernels */
#define HE_IN_RESIDENT 0x40u   /* he_server_submit only: read the transform of ct_in kept by an earlier
                                  HE_SERVE_KEEP_RESIDENT job of the same session (see the serving section) */

/* CPMul + CCAdd (Section 2 "Motivation", Section 3.2):
 *   acc_c = sum_{k<K} ct[k]_c (x) pt[k]   (ring product per prime), c = 0, 1.
 * ct   device [K][2][L][N]     pt  device [K][L][N]     acc  device [2][L][N]
 * ws   device workspace of at least he_cpmul_acc_ws() bytes (may be NULL if 0). */
he_status he_cpmul_acc(he_ctx *ctx, const uint64_t *ct, const uint64_t *pt, uint32_t K, uint64_t *acc,
                       uint32_t flags, void *ws, size_t ws_bytes, void *stream);
he_status he_cpmul_acc_ws(const he_ctx *ctx, uint32_t K, uint32_t flags, size_t *bytes);

/* --------------------------------------------- correlation-aware convolution */

#define HE_KIND_CONV 0   /* forward conv: out[b][m] = sum_k ct_in[b][k] (x) W[m][k] */
#define HE_KIND_DW 1     /* weight gradient (CryptoTrain-P terms):
                            out[m][k] = sum_b [X_b,k] (x) (dY_b,m - r) + [dY_b,m] (x) (X_b,k - r) */
#define HE_KIND_FC 2     /* fully connected: out[b][o] = sum_j ct_in[b][j] (x) W[o][j] */
#define HE_KIND_DX 3     /* input gradient of a conv layer (Section 2, training):
                            dX[b][c] = sum_m [dY_b,m] (x) rot180(W[m][c]) with padding h-1-P,
                            i.e. the forward conv of dY with the kernel transposed in its
                            channels and rotated by 180 degrees; the shape fields are the
                            forward layer's (C, M, H, W, h, P), the input is dY
                            [B][M][H_out][W_out], the weights the forward W [M][C][h][h],
                            the output dX [B][C][H][W] */

typedef struct {
  int32_t kind;          /* HE_KIND_* */
  uint32_t B;            /* batch */
  uint32_t C, M;         /* input / output channels (CONV, DW; DX: of the forward layer) */
  uint32_t H, W;         /* input map (CONV, DW; DX: of the forward layer) */
  uint32_t h;            /* kernel side (CONV, DW, DX: the forward kernel) */
  uint32_t P;            /* zero padding */
  uint32_t n_in, n_out;  /* FC sizes */
  uint32_t stride;       /* CONV: output stride (0 or 1: none); the packed product holds every
                            position, so a stride only subsamples the extraction; DW, DX: 0 or 1 */
} he_conv_shape;

typedef struct {
  int32_t kind;
  uint32_t N;
  uint32_t O;            /* row pitch of pi_x / pi_w (Eq. 1-2): max(W,H) + h - 1 (DW: h' = H_out) */
  uint32_t span;         /* highest product degree of one channel: (H+h-2)*O + W+h-2 */
  uint32_t S;            /* channel stride span + 1 */
  uint32_t Cw;           /* channels per polynomial, floor(N / S) */
  uint32_t cb;           /* channel blocks, ceil(C / Cw) */
  uint32_t Hout, Wout;   /* conv output map ((H + 2P - h) / stride + 1) */
  uint32_t n_iw, n_ow;   /* FC: input chunk width, outputs per polynomial */
  uint32_t n_ct_in;      /* ciphertexts read  (CONV: B*cb; DW: B*(cb+M); FC: B*in_ct; DX: B*cb over M) */
  uint32_t n_pt;         /* plaintext polynomials (CONV: M*cb; DW: B*(M+cb); FC: out_ct*in_ct; DX: C*cb) */
  uint32_t n_ct_out;     /* ciphertexts written (CONV: B*M; DW: M*cb; FC: B*out_ct; DX: B*C) */
  uint32_t n_terms;      /* CPMul count */
  uint32_t Hw, Ww;       /* CONV, DX: input window (the whole map unless tiles are cheaper or it does not fit) */
  uint32_t tiles;        /* CONV, DX: windows per input map; inputs and outputs are per (b, tile): the
                            counts above are then B*tiles*cb and B*tiles*M (DX: B*tiles*C) */
} he_plan_info;

/* Plan a layer on a context.  Allocates host memory and a small device copy of
 * the term lists on the context's device.  A CONV or DX map is packed in
 * windows (Section 3.3): disjoint H_w x W_w tiles of the unpadded input with
 * pitch O = max(W_w, H_w) + h - 1, chosen among all windows that fit one
 * polynomial (the whole map is one) to minimise the CPMul count (ties: fewer
 * input ciphertexts, then larger H_w, then larger W_w); a map whose channel
 * does not fit is always split, one that fits only when tiles lower the count.
 * he_extract_output overlap-adds the tiles' products.  HE_EUNSUPPORTED when no
 * window fits, or when a weight-gradient (DW) channel does not fit. */
he_status he_plan_create(const he_ctx *ctx, const he_conv_shape *shape, he_plan **out);
he_status he_plan_destroy(he_plan *plan);
/* Host-only planning (Section 3.3): the geometry and counts he_plan_create would
 * give on a context of ring degree N, without a context, device or allocation.
 * N a power of two in [16, 2^15], else HE_EINVAL; shape errors as he_plan_create.
 * For sizing and for multiplication-count studies (n_terms is the CPMul count). */
he_status he_plan_query(uint32_t N, const he_conv_shape *shape, he_plan_info *info);
he_status he_plan_get_info(const he_plan *plan, he_plan_info *info);
/* Host copies of the term lists: output o sums terms [row[o], row[o+1]) of
 * ct_in[ct_idx[t]] (x) pt[pt_idx[t]].  row [n_ct_out+1], ct_idx/pt_idx [n_terms]. */
he_status he_plan_terms(const he_plan *plan, int32_t *row, int32_t *ct_idx, int32_t *pt_idx);
/* Device workspace he_corr_conv2d needs with these flags (HE_EINVAL for a host
 * plan, which has no prime count: use he_layer_query). */
he_status he_workspace_size(const he_plan *plan, uint32_t flags, size_t *bytes);

/* Client-side plan (Section 3.3: the client packs its inputs into pi_x and
 * reads the outputs back): the plan he_plan_create would give on a ring of
 * degree N, with no context and no device memory.  he_plan_get_info,
 * he_plan_terms, he_pack_input, he_extract_output, he_ppmul_ws_size and
 * he_layer_query accept it; calls that run on a device refuse it (HE_EINVAL,
 * "plan belongs to another context").  Free with he_plan_destroy.  Errors as
 * he_plan_query. */
he_status he_plan_create_host(uint32_t N, const he_conv_shape *shape, he_plan **out);

/* Where a layer call packs raw weights into plaintext polynomials. */
#define HE_PACK_NONE 0u   /* HE_PLAIN_POLY: the caller passes packed polynomials */
#define HE_PACK_FUSED 1u  /* scattered in LDS inside the plaintext transform */
#define HE_PACK_MEMORY 2u /* HE_UNFUSED: packed to workspace polynomials first */
typedef struct {
  uint64_t workspace_bytes; /* = he_workspace_size for these flags */
  /* byte offsets of the workspace regions, UINT64_MAX where a region is absent */
  uint64_t off_ct_hat;      /* transformed input ciphertexts (absent with HE_IN_NTT) */
  uint64_t off_pt_poly;     /* packed plaintext polynomials (HE_PACK_MEMORY only) */
  uint64_t off_pt_hat;      /* transformed plaintexts */
  uint64_t off_acc;         /* accumulators of the unfused path (HE_UNFUSED without HE_OUT_NTT) */
  uint64_t off_flag;        /* range-check flag (HE_VALIDATE) */
  uint32_t fwd_ct_planes;   /* ciphertext planes forward transformed: n_ct_in*2*L (0 with HE_IN_NTT) */
  uint32_t fwd_pt_planes;   /* plaintext planes forward transformed: n_pt*L */
  uint32_t mac_planes;      /* output planes multiply-accumulated: n_ct_out*2*L */
  uint32_t inv_planes;      /* output planes inverse transformed (0 with HE_OUT_NTT) */
  uint32_t pack;            /* HE_PACK_* */
  uint32_t reserved;
} he_layer_info;
/* Host-only setup of one he_corr_conv2d call with these flags on L primes (no
 * device work): the same code runs inside the call before its first launch,
 * so this returns the errors the call would return before launching --
 * HE_EUNSUPPORTED for a weight-gradient plan without HE_PLAIN_POLY, HE_EINVAL
 * when the plan's weight layout would place a packed weight outside the
 * N-coefficient plane (every position is checked here, on the host).  L = 0
 * takes a device plan's own prime count; a host plan needs L > 0. */
he_status he_layer_query(const he_plan *plan, uint32_t L, uint32_t flags, he_layer_info *info);

/* Server side of one layer (Section 3.2 online phase with the packing of Section 3.3):
 * transform the input ciphertexts, pack and transform the plaintexts, multiply-
 * accumulate per the plan's term lists, inverse-transform the outputs.
 * ct_in   device [n_ct_in][2][L][N]
 * plain   device; HE_PLAIN_RAW: int32 weights (CONV [M][C][h][h], FC [n_out][n_in]);
 *                 HE_PLAIN_POLY: int64 packed polynomials [n_pt][N] (signed integers,
 *                 lifted to v mod q_i)
 * ct_out  device [n_ct_out][2][L][N]
 * ws      device, at least he_workspace_size() bytes. */
he_status he_corr_conv2d(he_ctx *ctx, const he_plan *plan, const uint64_t *ct_in, const void *plain,
                         uint64_t *ct_out, uint32_t flags, void *ws, size_t ws_bytes, void *stream);

/* he_corr_conv2d for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and results, with the workspace taken from a fixed device array of
 * the library, HE_NOALLOC_SCRATCH_MB MiB per GPU, held from the library's
 * first use of that GPU until the process ends.  No hipMalloc, hipFree or
 * other allocating call; kernel timing (he_ctx_profile) is skipped for it.
 * Arguments as he_corr_conv2d without ws/ws_bytes.  HE_ENOMEM if the layer's
 * he_workspace_size(flags) exceeds the array; HE_EINVAL for HE_VALIDATE
 * (it synchronises the stream).  Every call on one GPU shares that GPU's
 * array (nothing in it needs to start at zero: each call writes what it
 * reads), so calls that overlap on one GPU -- on different streams or from
 * different threads -- race and must be serialised by the caller. */
#define HE_NOALLOC_SCRATCH_MB 64
he_status he_corr_conv2d_noalloc(he_ctx *ctx, const he_plan *plan, const uint64_t *ct_in, const void *plain,
                                 uint64_t *ct_out, uint32_t flags, void *stream);

/* Seeded component c1 (Section 7, Discussion: the client sends a seed instead of the
 * uniform c1; about half the upload).  Coefficient k of component 1 of
 * ciphertext j at prime i is (w0 2^64 + w1) mod q_i, where (w0, w1, w2, w3) is
 * the Philox4x64-10 block (Salmon et al., SC 2011) of counter (k, j, i, 0)
 * under key (seed[0], seed[1]).
 * he_corr_conv2d_seeded: as he_corr_conv2d, with ct0 device [n_ct_in][L][N]
 * (component 0 of each input ciphertext) and seed host [2]; component 1 of
 * input j is regenerated inside the forward transform (never stored or read).
 * HE_IN_NTT is refused (HE_EINVAL); HE_VALIDATE checks ct0.
 * he_expand_c1: writes component 1 of ciphertexts first_ct .. first_ct+n_ct-1
 * to out, device [n_ct][L][N] (the client uses it to encrypt). */
he_status he_corr_conv2d_seeded(he_ctx *ctx, const he_plan *plan, const uint64_t *ct0, const uint64_t *seed,
                                const void *plain, uint64_t *ct_out, uint32_t flags, void *ws, size_t ws_bytes,
                                void *stream);
he_status he_expand_c1(he_ctx *ctx, const uint64_t *seed, uint32_t first_ct, uint32_t n_ct, uint64_t *out,
                       void *stream);

/* Client-side packing (host): CONV x [B][C][H][W] -> [B][tiles][cb][N]; DW is packed as
 * CONV with the plan's geometry; FC x [B][n_in] -> [B][in_ct][N]. */
he_status he_pack_input(const he_plan *plan, const int32_t *x, int64_t *polys);
/* Client-side extraction (host): CONV [B][tiles][M][N] -> y [B][M][Hout][Wout]
 * (windowed plans: the tiles' coefficients summed, so values are sums of the
 * given residues -- reduce mod t after extraction; with a stride s, output
 * (y, z) is the correlation coefficient at (y s, z s) of the padded map);
 * FC [B][out_ct][N] -> y [B][n_out]; DW [M][cb][N] -> dW [M][C][Hk][Hk] with
 * Hk = H + 2P - Hout + 1.  Values are taken as given (mod t after decryption). */
he_status he_extract_output(const he_plan *plan, const int64_t *polys, int64_t *y);

/* ------------------------------- ciphertext-ciphertext product (CCMul) */
/* The server's preprocessing step of Section 3.2 (CryptoTrain-P): products of
 * ciphertexts, [r_x][r_w] -> [r_x r_w], in the BFV scheme of the layer
 * ciphertexts, relinearized back to two components:
 *   out[o] = Relin( round(t/Q * sum over terms k of o of a[a_idx[k]] (x) b[b_idx[k]]) )  mod Q
 * where (x) is the tensor product (c0 d0, c0 d1 + c1 d0, c1 d1) of the
 * ciphertexts' coefficients read as centred integers in (-Q/2, Q/2], exact
 * over the integers, and round is to the nearest integer; one rounding and one
 * relinearization per output.  Relinearization is RNS-digit key switching:
 *   Relin(d0, d1, d2) = (d0, d1) + sum_j [d2]_{q_j} rlk_j,
 *   rlk_j = ([-(a_j s + e_j) + g_j s^2]_Q, a_j),  g_j = (Q/q_j) [(Q/q_j)^-1]_{q_j}
 * with [d2]_{q_j} the residue of d2 mod q_j taken as an integer in [0, q_j).
 * a      device [n_a][2][L][N] and b device [n_b][2][L][N], canonical residues;
 * row    host int32 [n_out + 1], a_idx and b_idx host int32 [row[n_out]]: output
 *        o sums terms row[o] .. row[o+1]-1 (at most 65536; HE_EUNSUPPORTED
 *        beyond); row NULL: pairwise products out[k] = a[k] (x) b[k] with
 *        n_out = n_a = n_b (HE_EINVAL otherwise); indexes out of range: HE_EINVAL;
 * rlk_hat device [L][2][L][N]: the key in the transformed domain (he_ntt_fwd
 *        of its L*2*L planes), read only;
 * out    device [n_out][2][L][N], written (must not alias the inputs).
 * flags: HE_VALIDATE (HE_ERANGE if a, b or rlk_hat is not canonical).
 * ws: device, he_ccmul_ws_size() bytes for the same sizes and flags.
 * The exact rounding runs on an extended base Q u P of auxiliary primes with
 * log2 P >= log2 t + log2 N + log2 Q + 18, built with its conversion constants
 * by he_ctx_prepare(HE_PREPARE_CCMUL) (device memory owned by the context;
 * HE_EUNSUPPORTED there if that base would need more than 16 primes in all or
 * more than 8 auxiliary ones; HE_EINVAL here before it).  The term lists are
 * read during the call (the caller may reuse them on return) and reach the
 * workspace through the context's two pinned staging buffers (HE_EINVAL if
 * they are larger than he_ctx_prepare sized them for); the call waits at most
 * for the staging copy of the call two back, and the rest is asynchronous on
 * stream.  Allocates nothing.  Calls on one context from several host threads
 * are serialized around the staging. */
he_status he_ccmul_ws_size(he_ctx *ctx, uint32_t n_a, uint32_t n_b, uint32_t n_out, uint32_t n_terms,
                           uint32_t flags, size_t *bytes);
he_status he_ccmul(he_ctx *ctx, const uint64_t *a, uint32_t n_a, const uint64_t *b, uint32_t n_b,
                   const int32_t *row, const int32_t *a_idx, const int32_t *b_idx, uint32_t n_out,
                   const uint64_t *rlk_hat, uint64_t *out, uint32_t flags, void *ws, size_t ws_bytes,
                   void *stream);

/* -------------------------------------------- plaintext product (PPMul) */
/* The server's plaintext product of the online linear-layer protocol (Section
 * 3.2): with the client's masked operands (x - r_x) and (w - r_w) it returns
 * p = (x - r_x)(w - r_w), which the client subtracts from Dec(c) to obtain x w.
 * Computed over the ring of the plaintext modulus, Z_t[X]/(X^N + 1), with the
 * plan's term lists:
 *   out[o] = sum over terms k of output o of a[cti[k]] * b[pti[k]]   (mod t)
 * a    device [n_ct_in][N] residues in [0, t) (the input-side polynomials, e.g.
 *      pi_x of the masked input block);
 * b    device [n_pt][N] residues in [0, t) (the weight-side polynomials);
 * out  device [n_ct_out][N], written, residues in [0, t).
 * The transforms of that ring are built by he_ctx_prepare(HE_PREPARE_PPMUL),
 * which needs t prime with t = 1 mod 2N (65537 serves every N <= 2^15);
 * HE_EINVAL before it.  flags: HE_VALIDATE (HE_ERANGE if an input is not
 * below t).  ws: device, he_ppmul_ws_size() bytes.  Allocates nothing;
 * asynchronous on `stream` unless validating. */
he_status he_ppmul_ws_size(const he_plan *plan, uint32_t flags, size_t *bytes);
he_status he_ppmul(he_ctx *ctx, const he_plan *plan, const uint64_t *a, const uint64_t *b, uint64_t *out,
                   uint32_t flags, void *ws, size_t ws_bytes, void *stream);

/* ----------------------------------------------- test-only encryption (client) */

/* Secret key of the test-only client (Section 2 "HE": the client holds the
 * key; ternary secret as in BFV): sk[k] = floor(3 w / 2^64) - 1 in {-1, 0, 1},
 * with w the first 64-bit word of the Philox4x64-10 block (Salmon et al.,
 * SC 2011) of counter (k, 0, 0, 2^64 - 1) under key (seed, 0) -- the last
 * counter word keeps these blocks apart from those of the seeded component 1.
 * sk host int8 [N].  Host only: no device work, no allocation. */
he_status he_keygen(const he_ctx *ctx, uint64_t seed, int8_t *sk);

/* BFV-style secret-key encryption (a reading of Section 2 "HE", which encrypts
 * with a public key; secret-key encryption decrypts identically):
 *   c1 = a,  c0 = -a*s + e + Delta*m  (mod q_i),  Delta = floor(Q / t).
 * s device int8 [N] in {-1,0,1};  m device int64 [N] in [0,t);
 * a device [L][N] canonical;  e device int32 [N];  ct device [2][L][N].
 * Allocates and frees temporary device memory (not a hot-path call). */
he_status he_encrypt(he_ctx *ctx, const int8_t *s, const int64_t *m, const uint64_t *a, const int32_t *e,
                     uint64_t *ct, void *stream);
/* Decryption m = round(t * [c0 + c1*s]_Q / Q) mod t of n_ct ciphertexts.
 * s device int8 [N];  ct device [n_ct][2][L][N];  m host int64 [n_ct][N].
 * The ring products run on the device, the exact CRT rounding on the host.
 * Synchronises `stream`.  Allocates temporary device memory. */
he_status he_decrypt(he_ctx *ctx, const int8_t *s, const uint64_t *ct, uint32_t n_ct, int64_t *m, void *stream);

/* ------------------------------------------------------------------ batching */
/* Many layers (of possibly different ring degrees and shapes) in one persistent
 * fused kernel: forward transforms of every job's inputs and packed plaintexts,
 * then per output the multiply-accumulate and inverse transform, drained from a
 * device task table by one workgroup per compute unit, with per-job completion
 * counters ordering each job's phases.  The launch is captured into a HIP graph
 * at build time and replayed by he_batch_run.  Results are byte-identical to
 * running each job alone with he_corr_conv2d. */
typedef struct {
  const he_plan *plan;     /* the job's layer plan (its context fixes N, L) */
  const uint64_t *ct_in;   /* device [n_ct_in][2][L][N], coefficient form (transformed if HE_IN_NTT) */
  const void *plain;       /* device: raw int32 weights (CONV, FC) or int64 polynomials (HE_PLAIN_POLY) */
  uint64_t *ct_out;        /* device [n_ct_out][2][L][N], coefficient form */
  uint32_t flags;          /* HE_IN_NTT, HE_PLAIN_POLY, HE_ACCUMULATE */
  uint32_t reserved;
} he_job;

typedef struct {
  uint32_t n_jobs, n_tasks, grid, arith;
  uint64_t cpmul;          /* CPMul-accumulates per run */
  uint64_t fwd_planes;     /* forward plane transforms per run */
  uint64_t inv_planes;     /* inverse plane transforms per run */
  uint64_t ws_bytes;       /* device workspace owned by the batch */
  uint64_t kernel_launches;   /* HE_BATCH_PROFILE: persistent-kernel launches timed so far */
  double kernel_ms;           /* HE_BATCH_PROFILE: their total duration (HIP events around the kernel alone) */
} he_batch_info;

#define HE_BATCH_GRAPH 0x1u        /* capture the launch into a HIP graph (default on) */
#define HE_BATCH_STRICT_SYNC 0x2u  /* every wave fences at every dependency (slower; for checking) */
#define HE_BATCH_PROFILE 0x4u      /* direct launches only (not with HE_BATCH_GRAPH): HIP events on the run
                                    * stream around the persistent kernel itself (not the control-word reset
                                    * and cache-fence kernels beside it); he_batch_sync adds their durations
                                    * to he_batch_info.kernel_ms.  At most 64 runs between two syncs. */

/* Create an empty batch for `device` (host memory only). */
he_status he_batch_create(int32_t device, he_batch **out);
/* Append a job; the plan and every buffer must stay valid while the batch is used.
 * All jobs of a batch must use the same arithmetic (all primes < 2^48, or not). */
he_status he_batch_add(he_batch *b, he_ctx *ctx, const he_job *job, uint32_t *index);
/* Plan the task table, allocate the batch workspace and device tables, and
 * (with HE_BATCH_GRAPH) capture the launch into a graph.  Allocates device memory. */
he_status he_batch_build(he_batch *b, uint32_t flags);
/* Point job `index` at new buffers (same plan); no re-capture is needed. */
he_status he_batch_rebind(he_batch *b, uint32_t index, const he_job *job);
/* Launch the whole batch on `stream` (asynchronous).  HE_EINVAL with
 * HE_BATCH_PROFILE after 64 runs without a sync. */
he_status he_batch_run(he_batch *b, void *stream);
/* Wait for `stream` and report HE_ETIMEOUT if a dependency wait of any run
 * since the previous sync hit its bound (the flag stays set over later runs and
 * is cleared once reported; the outputs of such runs are not to be trusted). */
he_status he_batch_sync(he_batch *b, void *stream);
/* Bound on the polls of one dependency wait inside the persistent kernel
 * (default about 2^20, about a second at the longest back-off); a wait that
 * reaches it gives up, the run carries on and he_batch_sync reports
 * HE_ETIMEOUT.  Applies to direct launches and to graphs captured by a later
 * he_batch_build.  A watchdog knob, and the host-side way to test that path:
 * every workgroup still finishes its tasks. */
he_status he_batch_set_spin_limit(he_batch *b, uint32_t polls);
he_status he_batch_get_info(const he_batch *b, he_batch_info *info);
he_status he_batch_destroy(he_batch *b);

/* ------------------------------------------------------------------- serving */
/* A request loop for homomorphic linear-layer jobs.  Jobs (he_job: plan and
 * device buffers owned by the caller) are queued FIFO and admitted while the
 * device footprint of admitted, unfinished work stays within mem_cap_bytes;
 * footprint = the job's workspace + its input and output ciphertexts + the
 * transformed inputs that jobs of open sessions keep resident.  In CONTINUOUS
 * mode every admitted job not yet running is launched as one persistent-kernel
 * epoch on a free stream slot, so jobs that arrive while an epoch runs go into
 * the next epoch on another stream and overlap on the device; SEQUENTIAL mode
 * serves one job at a time through the per-layer path (the plain baseline).
 * Latency is measured from arrival (submission, or the scheduled arrival in
 * he_server_replay) to completion observed by the server thread.
 *
 * Residency (the layers of a training step reuse their inputs, Section 2
 * "Neural Network Training"): the forward transform of a job's input
 * ciphertexts depends only on the ciphertexts and the context.  A job
 * submitted with HE_SERVE_KEEP_RESIDENT and a session keeps, after it
 * finishes, its workspace block holding that transform (canonical residues).
 * A later job of the same session whose he_job.flags has HE_IN_RESIDENT and
 * whose ct_in is the same buffer (same context, at most as many ciphertexts)
 * reads that transform instead of computing it; if none is kept (the
 * producer has not finished, was evicted, or never kept), it transforms ct_in
 * as usual.  Results are identical either way.  Kept blocks count towards the
 * cap; they are freed when the session closes (after session_jobs jobs, or by
 * he_server_close_session) and evicted, oldest first and only when no running
 * job reads them, when the queue head does not fit while no epoch runs.
 * A job with HE_VALIDATE is checked by itself before its epoch is built: a
 * job with a coefficient outside [0, q_i) fails alone with HE_ERANGE. */
#define HE_SERVE_CONTINUOUS 0
#define HE_SERVE_SEQUENTIAL 1
#define HE_SERVE_KEEP_RESIDENT 0x1u   /* he_server_submit flag: keep the job's transformed inputs until its session closes */

typedef struct {
  int32_t device;
  uint32_t mode;              /* HE_SERVE_* */
  uint64_t mem_cap_bytes;     /* admission cap on the device footprint */
  uint64_t arena_bytes;       /* device arena for workspaces (0: min(cap, 8 GiB)); allocated at creation */
  uint32_t max_batch_jobs;    /* jobs per epoch (0: 64) */
  uint32_t slots;             /* concurrent epochs on separate streams (0: 2, at most 8) */
  uint32_t session_jobs;      /* a session closes after this many jobs (0: never, resident data is kept) */
  uint32_t poll_us;           /* completion polling period of the server thread (0: 20) */
} he_server_params;

typedef struct {
  he_status status;
  double latency_s;           /* arrival to completion */
  double queue_s;             /* arrival to launch */
} he_job_result;

typedef struct {
  uint64_t completed, rejected, epochs;
  double mean_jobs_per_epoch;
  double p50_s, p99_s, mean_s, max_s;
  double span_s;              /* first arrival to last completion */
  uint64_t peak_bytes, in_use_bytes;
  uint64_t single_epochs;     /* continuous mode: epochs of one job, run by the per-layer kernels */
  uint64_t resident_hits;     /* HE_IN_RESIDENT jobs that read a kept transform */
  uint64_t resident_misses;   /* HE_IN_RESIDENT jobs that found none and transformed their inputs */
  uint64_t evictions;         /* kept blocks freed to admit the queue head */
  uint64_t fwd_planes;        /* plane forward transforms the served jobs ran */
  uint64_t failed;            /* jobs that finished with an error status */
  uint64_t resident_blocks;   /* kept blocks now on the device */
} he_server_info;

/* Start a server (device arena, stream slots and the server thread). */
he_status he_server_create(const he_server_params *params, he_server **out);
/* Queue a job; HE_EBUSY if its footprint alone exceeds the cap.  `session` (0 =
 * none) groups the jobs of one training step; with HE_SERVE_KEEP_RESIDENT the
 * job's transformed inputs stay on the device until the session closes. */
he_status he_server_submit(he_server *s, he_ctx *ctx, const he_job *job, uint64_t session, uint32_t flags,
                           uint64_t *ticket);
/* Wait for a job (timeout_us < 0: no limit); returns the job's status (result->status
 * too) or HE_ETIMEOUT if it has not finished. */
he_status he_server_wait(he_server *s, uint64_t ticket, int64_t timeout_us, he_job_result *result);
/* Wait until every queued job has finished. */
he_status he_server_drain(he_server *s);
/* Free the blocks a session keeps (a block a running job reads is freed when it finishes). */
he_status he_server_close_session(he_server *s, uint64_t session);
/* Submit n jobs at arrival_s[i] seconds after the call (busy-waiting on the host
 * clock), wait for all, and write each latency (from its scheduled arrival) to
 * latency_s[i] (host, may be NULL; -1 for a rejected job). */
he_status he_server_replay(he_server *s, uint32_t n, he_ctx *const *ctxs, const he_job *jobs, const double *arrival_s,
                           const uint64_t *sessions, uint32_t flags, double *latency_s);
he_status he_server_stats(he_server *s, he_server_info *out);
he_status he_server_destroy(he_server *s);

/* ------------------------------------------------------------ kernel timing */
/* Per-kernel timing on the launch stream: while enabled, every kernel the
 * context's calls launch is bracketed by two HIP events on the stream it is
 * launched on.  he_ctx_profile(ctx, 1) clears and starts, (ctx, 0) stops;
 * he_ctx_profile_read waits for the recorded events and returns one entry per
 * kernel kind (at most cap entries).  Kinds: 0 forward transform, 1 forward
 * transform of packed plaintexts, 2 inverse transform, 3 fused multiply-
 * accumulate + inverse transform, 4 multiply-accumulate in the transformed
 * domain, 5 packing, 6 persistent batch kernel, 7 exact RNS base conversion
 * (the lift and the scale-and-round of the ciphertext product). */
typedef struct {
  uint32_t kind;
  uint32_t launches;
  double total_ms;
  double max_ms;
} he_kernel_stat;
he_status he_ctx_profile(he_ctx *ctx, int enable);
he_status he_ctx_profile_read(he_ctx *ctx, he_kernel_stat *out, uint32_t cap, uint32_t *n);

/* ------------------------------------------------------------------ errors */
const char *he_status_str(he_status status);
const char *he_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HE_H */
