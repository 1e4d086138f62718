"""GPU parity of the ciphertext-ciphertext product with relinearization
(Section 3.2, the CCMul of the preprocessing phase) against the oracle, bit for
bit, and through decryption: pairwise products with coefficients on the
centring boundary, accumulated products over term lists, both arithmetic paths
(fp64 below 2^48 and 64-bit integers for 60-bit primes), the conv layer's mask
products at the benchmark ring, and the error paths."""
import numpy as np
import pytest
import torch

from oracle import bfv, ccmul, core
from paper_2409_16675_amd import synth
from tests.helpers import assert_equal_u64

T = synth.T_PLAIN


def _keys(ctx, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    s = g.integers(-1, 2, size=ctx.N)
    L, N = ctx.L, ctx.N
    a = np.stack([np.stack([g.integers(0, qi, size=N, dtype=np.uint64) for qi in ctx.q]) for _ in range(L)])
    e = np.clip(np.rint(g.normal(0, 3.2, size=(L, N))), -19, 19).astype(np.int64)
    return g, s, ccmul.relin_key(s, a, e, ctx.q, ctx.psi)


def _rlk_hat(he, ctx, rlk):
    d = he.to_device_u64(rlk)
    he.he_ntt_fwd(ctx.h, d, 2 * ctx.L)
    return d


def _boundary(ctx, ct):
    # coefficients at the centring boundary of Q and at the ends of every prime
    Q = bfv.modulus(ctx.q)
    vals = [0, 1, Q - 1, (Q - 1) // 2, (Q + 1) // 2, (Q + 3) // 2]
    for k, v in enumerate(vals):
        for i, qi in enumerate(ctx.q):
            ct[0, 0, i, k] = v % qi
            ct[0, 1, i, k + 8] = v % qi
    for i, qi in enumerate(ctx.q):
        ct[0, 0, i, 16] = qi - 1
        ct[0, 1, i, 17] = (qi - 1) // 2
    return ct


def _run(he, ctx, a, b, row, ai, bi, n_out, rlk_hat, flags=0):
    n_terms = len(ai) if row is not None else a.shape[0]
    he.he_ctx_prepare(ctx.h, he.HE_PREPARE_CCMUL, n_out, n_terms)
    ws = he.workspace(he.he_ccmul_ws_size(ctx.h, a.shape[0], b.shape[0], n_out, n_terms, flags))
    out = he.empty_u64((n_out, 2, ctx.L, ctx.N))
    he.he_ccmul(ctx.h, he.to_device_u64(a), a.shape[0], he.to_device_u64(b), b.shape[0], row, ai, bi, n_out, rlk_hat,
                out, flags, ws, ws.numel())
    torch.cuda.synchronize()
    return he.to_numpy_u64(out)


@pytest.mark.gpu
@pytest.mark.parametrize("N,L,bits", [(1024, 2, 48), (1024, 3, 48), (2048, 2, 60), (4096, 4, 48), (1024, 7, 48),
                                      (1024, 1, 62)])
def test_pairwise_products_match_oracle(gpu_lib, N, L, bits):
    he = gpu_lib
    ctx = he.Context(N, L, prime_bits=bits)
    g, s, rlk = _keys(ctx, 80 + L + bits)
    n = 3
    a = _boundary(ctx, synth.uniform_residues(synth.rng(81, synth.STREAM_CT, N + L), (n, 2), ctx.q, N))
    b = synth.uniform_residues(synth.rng(82, synth.STREAM_CT, N + L), (n, 2), ctx.q, N)
    b[1] = a[0]                                             # a product with itself on the boundary values
    print("case ccmul pairwise N=%d L=%d bits=%d" % (N, L, bits), flush=True)
    got = _run(he, ctx, a, b, None, None, None, n, _rlk_hat(he, ctx, rlk))
    want = ccmul.ccmul_acc(a, b, list(range(n + 1)), list(range(n)), list(range(n)), rlk, ctx.q, ctx.psi, T)
    assert_equal_u64(got, want, "ccmul pairwise")


@pytest.mark.gpu
@pytest.mark.parametrize("N,L,bits", [(2048, 3, 48), (1024, 2, 60)])
def test_accumulated_products_match_oracle_and_decrypt(gpu_lib, N, L, bits):
    he = gpu_lib
    ctx = he.Context(N, L, prime_bits=bits)
    g, s, rlk = _keys(ctx, 83 + N)
    ms = [g.integers(0, T, size=N) for _ in range(5)]

    def enc(m):
        return bfv.encrypt(m, s, synth.uniform_residues(g, (), ctx.q, N), synth.small_error(g, N), ctx.q, ctx.psi, T)

    cts = np.stack([enc(m) for m in ms])
    row, ai, bi = [0, 3, 3, 7], [0, 1, 2, 4, 3, 2, 1], [4, 4, 0, 4, 3, 2, 0]    # an empty output in the middle
    print("case ccmul accumulate N=%d L=%d bits=%d" % (N, L, bits), flush=True)
    got = _run(he, ctx, cts, cts, row, ai, bi, 3, _rlk_hat(he, ctx, rlk), he.HE_VALIDATE)
    want = ccmul.ccmul_acc(cts, cts, row, ai, bi, rlk, ctx.q, ctx.psi, T)
    assert_equal_u64(got, want, "ccmul accumulate")
    for o in range(3):
        m = np.zeros(N, dtype=np.int64)
        for k in range(row[o], row[o + 1]):
            m = (m + core.negacyclic_mul(ms[ai[k]], ms[bi[k]], T).astype(np.int64)) % T
        assert np.array_equal(bfv.decrypt(got[o], s, ctx.q, ctx.psi, T), m), o


@pytest.mark.gpu
def test_back_to_back_calls_with_different_term_lists(gpu_lib):
    # four calls on one context and stream with no synchronization between
    # them, each with its own term lists, workspace and output: the lists pass
    # through the context's two staging buffers in turn (the third and fourth
    # calls reuse the buffers of the first and second), so every output must
    # still be its own product
    he = gpu_lib
    N, L = 1024, 2
    ctx = he.Context(N, L)
    g, s, rlk = _keys(ctx, 97)
    rlk_hat = _rlk_hat(he, ctx, rlk)
    cts = synth.uniform_residues(g, (4, 2), ctx.q, N)
    d_cts = he.to_device_u64(cts)
    lists = [([0, 2, 3], [0, 1, 2], [3, 2, 1]),
             ([0, 1, 4], [3, 0, 1, 2], [3, 0, 0, 1]),
             ([0, 3], [2, 2, 1], [0, 1, 3]),
             ([0, 1, 2, 3, 5], [1, 0, 3, 2, 2], [1, 2, 0, 3, 0])]
    runs = []
    he.he_ctx_prepare(ctx.h, he.HE_PREPARE_CCMUL, 4, 5)
    print("case ccmul back-to-back N=%d L=%d" % (N, L), flush=True)
    for row, ai, bi in lists:
        n_out = len(row) - 1
        ws = he.workspace(he.he_ccmul_ws_size(ctx.h, 4, 4, n_out, len(ai), 0))
        out = he.empty_u64((n_out, 2, L, N))
        he.he_ccmul(ctx.h, d_cts, 4, d_cts, 4, np.array(row, np.int32), np.array(ai, np.int32),
                    np.array(bi, np.int32), n_out, rlk_hat, out, 0, ws, ws.numel())
        runs.append((row, ai, bi, out, ws))
    torch.cuda.synchronize()
    for k, (row, ai, bi, out, _) in enumerate(runs):
        want = ccmul.ccmul_acc(cts, cts, row, ai, bi, rlk, ctx.q, ctx.psi, T)
        assert_equal_u64(he.to_numpy_u64(out), want, "call %d" % k)


@pytest.mark.gpu
def test_conv_mask_products_at_the_benchmark_ring(gpu_lib):
    # [r_x r_w] for the conv-forward workload (batch 16, 3 -> 16 channels,
    # N = 8192, L = 3): 256 outputs of one product each over the plan's term
    # lists; sampled outputs against the oracle, one through decryption
    he = gpu_lib
    ctx = he.Context(8192, 3, prime_bits=48)
    plan = he.Plan(ctx, he.HE_KIND_CONV, B=16, C=3, M=16, H=32, W=32, h=3, P=1)
    row, cti, pti = he.he_plan_terms(plan.h)
    g, s, rlk = _keys(ctx, 84)
    N = ctx.N
    rx = g.integers(0, T, size=(16, N))
    rw = g.integers(0, T, size=(16, N))

    def enc(m):
        return bfv.encrypt(m, s, synth.uniform_residues(g, (), ctx.q, N), synth.small_error(g, N), ctx.q, ctx.psi, T)

    ct_rx = np.stack([enc(m) for m in rx])
    ct_rw = np.stack([enc(m) for m in rw])
    print("case ccmul conv masks N=8192 L=3", flush=True)
    got = _run(he, ctx, ct_rx, ct_rw, row, cti, pti, 256, _rlk_hat(he, ctx, rlk))
    for o in (0, 17, 255):
        want = ccmul.ccmul_acc(ct_rx, ct_rw, [0, 1], [int(cti[row[o]])], [int(pti[row[o]])], rlk, ctx.q, ctx.psi, T)
        assert_equal_u64(got[o], want[0], "conv mask product %d" % o)
    o = 37
    assert np.array_equal(bfv.decrypt(got[o], s, ctx.q, ctx.psi, T),
                          core.negacyclic_mul(rx[cti[row[o]]], rw[pti[row[o]]], T).astype(np.int64))


@pytest.mark.gpu
def test_ccmul_errors(gpu_lib):
    he = gpu_lib
    ctx = he.Context(1024, 2)
    g, s, rlk = _keys(ctx, 85)
    rlk_hat = _rlk_hat(he, ctx, rlk)
    a = synth.uniform_residues(synth.rng(86, synth.STREAM_CT), (2, 2), ctx.q, 1024)
    with pytest.raises(he.HeError) as ei:                  # index out of range
        _run(he, ctx, a, a, [0, 1], [2], [0], 1, rlk_hat)
    assert ei.value.status == he.HE_EINVAL
    with pytest.raises(he.HeError) as ei:                  # pairwise with mismatched counts
        _run(he, ctx, a, a[:1], None, None, None, 2, rlk_hat)
    assert ei.value.status == he.HE_EINVAL
    big = np.zeros(65537, np.int32)
    with pytest.raises(he.HeError) as ei:                  # too many products for one output
        _run(he, ctx, a, a, [0, 65537], big, big, 1, rlk_hat)
    assert ei.value.status == he.HE_EUNSUPPORTED
    # eight 48-bit primes would need nine auxiliary ones: refused
    ctx8 = he.Context(1024, 8)
    with pytest.raises(he.HeError) as ei:
        he.he_ctx_prepare(ctx8.h, he.HE_PREPARE_CCMUL, 1, 1)
    assert ei.value.status == he.HE_EUNSUPPORTED
    # a context whose product was never prepared: refused, nothing built by the call
    ctx_np = he.Context(1024, 2)
    with pytest.raises(he.HeError) as ei:
        he.he_ccmul_ws_size(ctx_np.h, 1, 1, 1, 1)
    assert ei.value.status == he.HE_EINVAL
    # term lists larger than the staging was prepared for: refused
    he.he_ctx_prepare(ctx_np.h, he.HE_PREPARE_CCMUL, 1, 1)
    ap = synth.uniform_residues(synth.rng(96, synth.STREAM_CT), (2, 2), ctx_np.q, 1024)
    wsz = he.he_ccmul_ws_size(ctx_np.h, 2, 2, 2, 2)
    ws = he.workspace(wsz)
    out = he.empty_u64((2, 2, 2, 1024))
    with pytest.raises(he.HeError) as ei:
        he.he_ccmul(ctx_np.h, he.to_device_u64(ap), 2, he.to_device_u64(ap), 2, None, None, None, 2, rlk_hat, out, 0,
                    ws, ws.numel())
    assert ei.value.status == he.HE_EINVAL
    bad = a.copy()
    bad[1, 0, 0, 3] = ctx.q[0]                             # not canonical
    with pytest.raises(he.HeError) as ei:
        _run(he, ctx, bad, a, None, None, None, 2, rlk_hat, he.HE_VALIDATE)
    assert ei.value.status == he.HE_ERANGE
