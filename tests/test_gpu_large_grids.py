"""Launches with more than 65535 rows of coefficients (the limit of a grid's
second dimension): the component-1 expansion, the multiply-accumulate left in
the transformed domain, and the ciphertext product's conversion kernels lay
their rows along the first dimension.  Sampled rows against the oracle."""
import numpy as np
import pytest
import torch

from oracle import ccmul, core
from paper_2409_16675_amd import synth
from tests.helpers import assert_equal_u64

T = synth.T_PLAIN


@pytest.mark.gpu
def test_expand_c1_past_65535_planes(gpu_lib):
    he = gpu_lib
    ctx = he.Context(1024, 3)
    n = 22000                                               # 66000 planes
    seed = (5, 6)
    out = he.empty_u64((n, 3, 1024))
    he.he_expand_c1(ctx.h, seed, 0, n, out)
    torch.cuda.synchronize()
    for j in (0, 21845, n - 1):
        assert_equal_u64(he.to_numpy_u64(out[j]), core.expand_c1(seed, j, ctx.q, 1024), "c1 %d" % j)


@pytest.mark.gpu
def test_transformed_domain_accumulate_past_65535_planes(gpu_lib):
    # a conv layer left in the transformed domain with 10928 outputs
    # (65568 output planes): sampled outputs against the oracle's term sums
    he = gpu_lib
    N, L, B, M = 1024, 3, 1366, 8
    ctx = he.Context(N, L)
    plan = he.Plan(ctx, he.HE_KIND_CONV, B=B, C=1, M=M, H=4, W=4, h=3, P=1)
    info = plan.info
    assert info["n_ct_out"] * 2 * L > 65535
    ct = synth.uniform_residues(synth.rng(87, synth.STREAM_CT), (info["n_ct_in"], 2), ctx.q, N)
    w = synth.int8_uniform(synth.rng(87, synth.STREAM_PT), (M, 1, 3, 3))
    d_w = torch.from_numpy(w.astype(np.int32).reshape(-1)).cuda()
    out = he.empty_u64((info["n_ct_out"], 2, L, N))
    ws = he.workspace(plan.workspace_size(he.HE_OUT_NTT))
    he.he_corr_conv2d(ctx.h, plan.h, he.to_device_u64(ct), d_w, out, he.HE_OUT_NTT, ws, ws.numel())
    torch.cuda.synchronize()
    # the same layer to the coefficient domain, then transformed: equal planes
    out2 = he.empty_u64((info["n_ct_out"], 2, L, N))
    ws2 = he.workspace(plan.workspace_size(0))
    he.he_corr_conv2d(ctx.h, plan.h, he.to_device_u64(ct), d_w, out2, 0, ws2, ws2.numel())
    torch.cuda.synchronize()
    for o in (0, 5461, info["n_ct_out"] - 1):
        got = he.to_numpy_u64(out[o])
        coeff = he.to_numpy_u64(out2[o])
        assert_equal_u64(got, core.ntt_planes(coeff, ctx.q, ctx.psi), "output %d" % o)
    from oracle import packing
    geo = packing.ConvGeometry(1, 4, 4, 3, 1, N)
    pt = core.lift(packing.pack_conv_weight(w, geo).reshape(-1, N), ctx.q)
    row, cti, pti = packing.conv_terms(B, M, geo.cb)
    o = info["n_ct_out"] - 1
    want = core.csr_cpmul(ct, pt, np.array([0, row[o + 1] - row[o]], np.int32), cti[row[o]:row[o + 1]],
                          pti[row[o]:row[o + 1]], ctx.q, ctx.psi, method=2)[0]
    assert_equal_u64(he.to_numpy_u64(out2[o]), want, "last output against the oracle")


@pytest.mark.gpu
def test_ccmul_conversions_past_65535_rows(gpu_lib):
    # 21846 outputs (65538 tensor rows), each one product of two fixed ciphertexts
    he = gpu_lib
    N, L = 1024, 2
    ctx = he.Context(N, L)
    g = np.random.Generator(np.random.PCG64(88))
    s = g.integers(-1, 2, size=N)
    a_k = np.stack([np.stack([g.integers(0, qi, size=N, dtype=np.uint64) for qi in ctx.q]) for _ in range(L)])
    e_k = np.clip(np.rint(g.normal(0, 3.2, size=(L, N))), -19, 19).astype(np.int64)
    rlk = ccmul.relin_key(s, a_k, e_k, ctx.q, ctx.psi)
    rlk_hat = he.to_device_u64(rlk)
    he.he_ntt_fwd(ctx.h, rlk_hat, 2 * L)
    a = synth.uniform_residues(synth.rng(88, synth.STREAM_CT), (2, 2), ctx.q, N)
    n_out = 21846
    row = np.arange(n_out + 1, dtype=np.int32)
    ai = (np.arange(n_out) % 2).astype(np.int32)
    bi = ((np.arange(n_out) // 2) % 2).astype(np.int32)
    he.he_ctx_prepare(ctx.h, he.HE_PREPARE_CCMUL, n_out, n_out)
    ws = he.workspace(he.he_ccmul_ws_size(ctx.h, 2, 2, n_out, n_out, 0))
    out = he.empty_u64((n_out, 2, L, N))
    he.he_ccmul(ctx.h, he.to_device_u64(a), 2, he.to_device_u64(a), 2, row, ai, bi, n_out, rlk_hat, out, 0, ws,
                ws.numel())
    torch.cuda.synchronize()
    for o in (0, 1, 2, 3):
        want = ccmul.ccmul_acc(a, a, [0, 1], [int(ai[o])], [int(bi[o])], rlk, ctx.q, ctx.psi, T)[0]
        assert_equal_u64(he.to_numpy_u64(out[o]), want, "output %d" % o)
        for o2 in (o + 4 * 5000, n_out - 4 + (o - (n_out - 4) % 4) % 4):
            assert_equal_u64(he.to_numpy_u64(out[o2]), want, "output %d" % o2)
