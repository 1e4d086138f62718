"""GPU parity of the seeded ciphertext component c1 (Section 7, Discussion: the client sends
a seed instead of c1, the server regenerates it): the expansion against the
oracle, and the conv layer with regenerated c1 against the same layer on the
full ciphertexts, against the oracle, and through decryption."""
import numpy as np
import pytest
import torch

from oracle import bfv, core, packing, plain
from paper_2409_16675_amd import synth
from tests.helpers import assert_equal_u64

T = synth.T_PLAIN


@pytest.mark.gpu
@pytest.mark.parametrize("N,L,first,n", [(1024, 2, 0, 3), (8192, 3, 5, 2), (16384, 4, 1, 1)])
def test_expand_c1_matches_oracle(gpu_lib, N, L, first, n):
    he = gpu_lib
    ctx = he.Context(N, L)
    seed = (0x0123456789ABCDEF, 0xFEDCBA9876543210 + N)
    out = he.empty_u64((n, L, N))
    he.he_expand_c1(ctx.h, seed, first, n, out)
    torch.cuda.synchronize()
    got = he.to_numpy_u64(out)
    for jj in range(n):
        assert_equal_u64(got[jj], core.expand_c1(seed, first + jj, ctx.q, N), "c1 of ciphertext %d" % (first + jj))


def _layer(he, ctx, plan, flags=0):
    info = plan.info
    out = he.empty_u64((info["n_ct_out"], 2, ctx.L, ctx.N))
    ws = he.workspace(plan.workspace_size(flags))
    return out, ws


@pytest.mark.gpu
@pytest.mark.parametrize("N,L,B,C,M,H,h,P", [(1024, 2, 2, 3, 2, 6, 3, 1), (8192, 3, 16, 3, 16, 32, 3, 1)])
def test_seeded_layer_equals_full_ciphertext_layer(gpu_lib, N, L, B, C, M, H, h, P):
    he = gpu_lib
    ctx = he.Context(N, L, prime_bits=48)
    plan = he.Plan(ctx, he.HE_KIND_CONV, B=B, C=C, M=M, H=H, W=H, h=h, P=P)
    info = plan.info
    seed = (77, 2 ** 63 + 5)
    g = synth.rng(60, synth.STREAM_CT, N)
    c0 = synth.uniform_residues(g, (info["n_ct_in"],), ctx.q, N)           # [n][L][N]
    w = synth.int8_uniform(synth.rng(60, synth.STREAM_PT), (M, C, h, h))
    d_w = torch.from_numpy(w.astype(np.int32).reshape(-1)).cuda()
    # the full ciphertexts: component 1 expanded on the device
    c1 = he.empty_u64((info["n_ct_in"], L, N))
    he.he_expand_c1(ctx.h, seed, 0, info["n_ct_in"], c1)
    full = torch.stack([he.to_device_u64(c0), c1], dim=1).contiguous()    # [n][2][L][N]
    out_full, ws = _layer(he, ctx, plan)
    he.he_corr_conv2d(ctx.h, plan.h, full, d_w, out_full, 0, ws, ws.numel())
    out_seed, ws2 = _layer(he, ctx, plan)
    he.he_corr_conv2d_seeded(ctx.h, plan.h, he.to_device_u64(c0), seed, d_w, out_seed, 0, ws2, ws2.numel())
    torch.cuda.synchronize()
    got = he.to_numpy_u64(out_seed)
    assert_equal_u64(got, he.to_numpy_u64(out_full), "seeded vs full")
    if N == 1024:
        geo = packing.ConvGeometry(C, H, H, h, P, N)
        ct = np.stack([c0, np.stack([core.expand_c1(seed, j, ctx.q, N) for j in range(info["n_ct_in"])])], axis=1)
        pt = core.lift(packing.pack_conv_weight(w, geo).reshape(-1, N), ctx.q)
        row, cti, pti = packing.conv_terms(B, M, geo.cb)
        assert_equal_u64(got, core.csr_cpmul(ct, pt, row, cti, pti, ctx.q, ctx.psi, method=2), "seeded vs oracle")


@pytest.mark.gpu
def test_seeded_encryption_end_to_end(gpu_lib):
    # client: encrypt with c1 taken from the seed, send c0 and the seed;
    # server: seeded layer; client: decrypt and extract = plaintext conv mod t
    he = gpu_lib
    N, L, B, C, M, H, h, P = 2048, 2, 2, 3, 4, 8, 3, 1
    ctx = he.Context(N, L)
    plan = he.Plan(ctx, he.HE_KIND_CONV, B=B, C=C, M=M, H=H, W=H, h=h, P=P)
    info = plan.info
    seed = (2024, 11)
    x = synth.int8_uniform(synth.rng(62, synth.STREAM_ACT), (B, C, H, H))
    w = synth.int8_uniform(synth.rng(62, synth.STREAM_PT), (M, C, h, h))
    polys = he.he_pack_input(plan.h, x.reshape(-1), B * info["cb"] * N).reshape(-1, N)
    s = synth.ternary(synth.rng(62, synth.STREAM_SK), N)
    ge = synth.rng(62, synth.STREAM_E)
    c0 = np.stack([bfv.encrypt(np.remainder(p, T), s, core.expand_c1(seed, j, ctx.q, N), synth.small_error(ge, N),
                               ctx.q, ctx.psi, T)[0] for j, p in enumerate(polys)])
    out, ws = _layer(he, ctx, plan, he.HE_VALIDATE)
    he.he_corr_conv2d_seeded(ctx.h, plan.h, he.to_device_u64(c0), seed, torch.from_numpy(w.astype(np.int32).reshape(-1)).cuda(),
                             out, he.HE_VALIDATE, ws, ws.numel())
    torch.cuda.synchronize()
    got = he.to_numpy_u64(out)
    dec = np.stack([bfv.decrypt(got[o], s, ctx.q, ctx.psi, T) for o in range(got.shape[0])])
    Ho = H + 2 * P - h + 1
    y = he.he_extract_output(plan.h, dec, B * M * Ho * Ho).reshape(B, M, Ho, Ho)
    for b in range(B):
        assert np.array_equal(y[b], plain.mod_t(plain.conv2d(x[b], w, P), T)), b
    # a transformed-input flag is refused
    with pytest.raises(he.HeError) as ei:
        he.he_corr_conv2d_seeded(ctx.h, plan.h, he.to_device_u64(c0), seed, torch.zeros(1, dtype=torch.int32).cuda(),
                                 out, he.HE_IN_NTT, ws, ws.numel())
    assert ei.value.status == he.HE_EINVAL
