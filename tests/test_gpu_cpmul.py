"""GPU parity of CPMul + accumulate (Section 2 "Motivation", Section 3.2) and of
the test-only encryption, against the oracle, bit for bit."""
import numpy as np
import pytest
import torch

from oracle import bfv, core
from paper_2409_16675_amd import synth
from tests.helpers import assert_equal_u64


def c1_inputs(ctx, K=8):
    """Plain CPMul-accumulate workload: N = 2048, 2 primes, 8 ciphertexts uniform mod q_i,
    8 plaintexts uniform in [0, t)."""
    N = ctx.N
    ct = synth.uniform_residues(synth.rng(1, synth.STREAM_CT), (K, 2), ctx.q, N)
    ptv = synth.uniform_mod_t(synth.rng(1, synth.STREAM_PT), (K, N))
    pt = core.lift(ptv, ctx.q)
    return ct, pt


@pytest.mark.gpu
@pytest.mark.parametrize("bits,arith", [(48, 1), (48, 2), (50, 2), (54, 2)])
def test_cpmul_acc_plain_workload_schoolbook(gpu_lib, bits, arith):
    he = gpu_lib
    ctx = he.Context(2048, 2, prime_bits=bits, arith=arith)
    ct, pt = c1_inputs(ctx)
    K = 8
    row = np.array([0, K], np.int32)
    idx = np.arange(K, dtype=np.int32)
    expect = core.csr_cpmul(ct, pt, row, idx, idx, ctx.q, ctx.psi, method=0)[0]   # schoolbook definition
    ws = he.workspace(he.he_cpmul_acc_ws(ctx.h, K))
    acc = he.empty_u64((2, 2, 2048))
    dct, dpt = he.to_device_u64(ct), he.to_device_u64(pt)
    for arith2, loge in he.compiled_schedules(2048, f64_ok=bits <= he.F64_MAX_BITS):
        print("case cpmul bits=%d arith=%d loge=%d" % (bits, arith2, loge), flush=True)
        for op in (he.HE_OP_FWD, he.HE_OP_INV, he.HE_OP_MAC):
            he.he_ctx_set_schedule(ctx.h, op, arith2, loge)
        he.he_cpmul_acc(ctx.h, dct, dpt, K, acc, 0, ws, ws.numel())
        torch.cuda.synchronize()
        assert_equal_u64(he.to_numpy_u64(acc), expect, "cpmul")


@pytest.mark.gpu
def test_cpmul_acc_flags(gpu_lib):
    he = gpu_lib
    N, L = 4096, 2
    ctx = he.Context(N, L)
    g = synth.rng(92, 1)
    K = 5
    ct = synth.uniform_residues(g, (K, 2), ctx.q, N)
    pt = synth.uniform_residues(g, (K,), ctx.q, N)
    row = np.array([0, K], np.int32)
    idx = np.arange(K, dtype=np.int32)
    expect = core.csr_cpmul(ct, pt, row, idx, idx, ctx.q, ctx.psi, method=1)[0]
    dct, dpt = he.to_device_u64(ct), he.to_device_u64(pt)
    ws = he.workspace(he.he_cpmul_acc_ws(ctx.h, K))
    # overwrite
    acc = he.empty_u64((2, L, N))
    he.he_cpmul_acc(ctx.h, dct, dpt, K, acc, 0, ws, ws.numel())
    torch.cuda.synchronize()
    assert_equal_u64(he.to_numpy_u64(acc), expect, "overwrite")
    # accumulate on top of a previous value: result is 2x
    he.he_cpmul_acc(ctx.h, dct, dpt, K, acc, he.HE_ACCUMULATE, ws, ws.numel())
    torch.cuda.synchronize()
    twice = np.stack([np.stack([(expect[c, i] * np.uint64(2)) % np.uint64(ctx.q[i]) for i in range(L)])
                      for c in range(2)])
    assert_equal_u64(he.to_numpy_u64(acc), twice, "accumulate")
    # transformed inputs and outputs
    ct_hat = core.ntt_planes(ct, ctx.q, ctx.psi)
    pt_hat = core.ntt_planes(pt, ctx.q, ctx.psi)
    acc2 = he.empty_u64((2, L, N))
    he.he_cpmul_acc(ctx.h, he.to_device_u64(ct_hat), he.to_device_u64(pt_hat), K, acc2, he.HE_IN_NTT | he.HE_OUT_NTT,
                    None, 0)
    torch.cuda.synchronize()
    assert_equal_u64(he.to_numpy_u64(acc2), core.ntt_planes(expect, ctx.q, ctx.psi), "ntt in/out")
    # K = 0 gives zero
    acc3 = he.to_device_u64(np.ones((2, L, N), np.uint64))
    he.he_cpmul_acc(ctx.h, dct, dpt, 0, acc3, 0, ws, ws.numel())
    torch.cuda.synchronize()
    assert not he.to_numpy_u64(acc3).any()


@pytest.mark.gpu
def test_cpmul_validate_rejects_out_of_range(gpu_lib):
    he = gpu_lib
    N, L = 2048, 2
    ctx = he.Context(N, L)
    ct = np.zeros((1, 2, L, N), np.uint64)
    ct[0, 1, 1, 7] = ctx.q[1]          # not canonical
    pt = np.zeros((1, L, N), np.uint64)
    ws = he.workspace(he.he_cpmul_acc_ws(ctx.h, 1, he.HE_VALIDATE))
    acc = he.empty_u64((2, L, N))
    with pytest.raises(he.HeError) as ei:
        he.he_cpmul_acc(ctx.h, he.to_device_u64(ct), he.to_device_u64(pt), 1, acc, he.HE_VALIDATE, ws, ws.numel())
    assert ei.value.status == he.HE_ERANGE
    with pytest.raises(he.HeError) as ei:
        he.he_cpmul_acc(ctx.h, he.to_device_u64(ct), he.to_device_u64(pt), 1, acc, 0, ws, 16)
    assert ei.value.status == he.HE_ENOMEM


@pytest.mark.gpu
@pytest.mark.parametrize("N,L,bits", [(2048, 2, 48), (8192, 3, 48), (2048, 2, 50), (4096, 3, 60), (1024, 8, 48), (1024, 2, 62)])
def test_encrypt_decrypt_match_oracle(gpu_lib, N, L, bits):
    he = gpu_lib
    ctx = he.Context(N, L, prime_bits=bits)
    t = ctx.t
    g = synth.rng(93, N + bits)
    s = synth.ternary(g, N)
    m = synth.uniform_mod_t(g, N)
    a = synth.uniform_residues(g, (), ctx.q, N)
    e = synth.small_error(g, N)
    expect = bfv.encrypt(m, s, a, e, ctx.q, ctx.psi, t)
    ds = torch.from_numpy(s.astype(np.int8)).cuda()
    dm = torch.from_numpy(m.astype(np.int64)).cuda()
    de = torch.from_numpy(e.astype(np.int32)).cuda()
    ct = he.empty_u64((2, L, N))
    he.he_encrypt(ctx.h, ds, dm, he.to_device_u64(a), de, ct)
    assert_equal_u64(he.to_numpy_u64(ct), expect, "encrypt")
    got = he.he_decrypt(ctx.h, ds, ct, 1, N)[0]
    assert np.array_equal(got, m)
    # decryption of arbitrary (uniform) ciphertexts: exact rounding agrees with the oracle
    junk = synth.uniform_residues(g, (2,), ctx.q, N)
    got = he.he_decrypt(ctx.h, ds, he.to_device_u64(junk[None]), 1, N)[0]
    exp = bfv.decrypt(junk, s, ctx.q, ctx.psi, t)
    assert np.array_equal(got, exp)
