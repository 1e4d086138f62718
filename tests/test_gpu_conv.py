"""GPU parity of the correlation-aware layers (Section 3.3 packing, Section 3.2
multiply-accumulate) against the oracle, bit for bit, plus decryption checks
against plaintext integer layers mod t (Section 2 "HE", homomorphic property)."""
import numpy as np
import pytest
import torch

from oracle import bfv, core, packing, plain
from paper_2409_16675_amd import synth
from tests.helpers import assert_equal_u64

T = synth.T_PLAIN


def encrypt_polys(ctx, polys, workload, extra=0):
    """Oracle encryption of integer polynomials (values taken mod t); returns ct [n, 2, L, N] and s."""
    N = ctx.N
    s = synth.ternary(synth.rng(workload, synth.STREAM_SK, extra), N)
    ga = synth.rng(workload, synth.STREAM_A, extra)
    ge = synth.rng(workload, synth.STREAM_E, extra)
    cts = []
    for p in polys.reshape(-1, N):
        a = synth.uniform_residues(ga, (), ctx.q, N)
        e = synth.small_error(ge, N)
        cts.append(bfv.encrypt(np.remainder(p, T), s, a, e, ctx.q, ctx.psi, T))
    return np.stack(cts), s


def run_layer(he, ctx, plan, ct_in, plain_arr, flags=0):
    info = plan.info
    out = he.empty_u64((info["n_ct_out"], 2, ctx.L, ctx.N))
    ws = he.workspace(plan.workspace_size(flags))
    he.he_corr_conv2d(ctx.h, plan.h, he.to_device_u64(ct_in), plain_arr, out, flags, ws, ws.numel())
    torch.cuda.synchronize()
    return he.to_numpy_u64(out)


def conv_case(he, N, L, B, C, M, H, W, h, P, seed, flags=0, decrypt_check=2, bits=50):
    ctx = he.Context(N, L, prime_bits=bits)
    g = packing.ConvGeometry(C, H, W, h, P, N)
    plan = he.Plan(ctx, he.HE_KIND_CONV, B=B, C=C, M=M, H=H, W=W, h=h, P=P)
    info = plan.info
    for k, v in g.as_dict().items():
        assert info[k] == v, k
    x = synth.int8_uniform(synth.rng(seed, synth.STREAM_ACT), (B, C, H, W))
    w = synth.int8_uniform(synth.rng(seed, synth.STREAM_PT), (M, C, h, h))
    polys_in = np.stack([packing.pack_conv_input(x[b], g) for b in range(B)])      # [B, cb, N]
    lib_polys = he.he_pack_input(plan.h, x.reshape(-1), B * g.cb * N).reshape(B, g.cb, N)
    assert np.array_equal(lib_polys, polys_in)
    ct_in, s = encrypt_polys(ctx, polys_in, seed)
    pt = core.lift(packing.pack_conv_weight(w, g).reshape(M * g.cb, N), ctx.q)
    row, cti, pti = packing.conv_terms(B, M, g.cb)
    lrow, lcti, lpti = he.he_plan_terms(plan.h)
    assert np.array_equal(lrow, row) and np.array_equal(lcti, cti) and np.array_equal(lpti, pti)
    expect = core.csr_cpmul(ct_in, pt, row, cti, pti, ctx.q, ctx.psi, method=2)
    dw = torch.from_numpy(w.astype(np.int32).reshape(-1)).cuda()
    got = run_layer(he, ctx, plan, ct_in, dw, flags)
    assert_equal_u64(got, expect, "conv B=%d C=%d M=%d H=%d h=%d" % (B, C, M, H, h))
    ref = plain.mod_t(np.stack([plain.conv2d(x[b], w, P) for b in range(B)]), T)   # [B, M, Ho, Wo]
    for o in range(min(decrypt_check, B * M)):
        b, m = divmod(o, M)
        dec = bfv.decrypt(got[o], s, ctx.q, ctx.psi, T)
        assert np.array_equal(packing.conv_extract(dec, g), ref[b, m])
    return ctx, plan, got, s, ref


@pytest.mark.gpu
def test_cifar_conv_forward_full_parity_and_decrypt(gpu_lib):
    # batch 16 of 3x32x32, 16 output channels, 3x3, stride 1, pad 1, N = 8192, 3 primes
    he = gpu_lib
    ctx, plan, got, s, ref = conv_case(he, 8192, 3, 16, 3, 16, 32, 32, 3, 1, seed=2, decrypt_check=3)
    # library decryption of a few outputs, extracted by the library, equals the plaintext conv mod t
    sd = torch.from_numpy(s.astype(np.int8)).cuda()
    dec = he.he_decrypt(ctx.h, sd, he.to_device_u64(got[:4]), 4, ctx.N)
    info = plan.info
    y = he.he_extract_output
    for o in range(4):
        b, m = divmod(o, 16)
        g = packing.ConvGeometry(3, 32, 32, 3, 1, 8192)
        assert np.array_equal(packing.conv_extract(dec[o], g), ref[b, m])


@pytest.mark.gpu
def test_conv_unfused_path_same_bytes(gpu_lib):
    he = gpu_lib
    conv_case(he, 8192, 3, 2, 3, 4, 32, 32, 3, 1, seed=21, flags=he.HE_UNFUSED, decrypt_check=1)


@pytest.mark.gpu
@pytest.mark.parametrize("N,L,B,C,M,H,W,h,P", [
    (1024, 2, 1, 1, 1, 5, 7, 3, 1),       # smallest ring, ragged map
    (1024, 2, 3, 10, 3, 6, 6, 3, 2),      # channels split over several blocks, pad 2
    (2048, 3, 2, 5, 2, 9, 4, 2, 0),       # even kernel, no padding
    (4096, 2, 1, 16, 32, 16, 16, 3, 1),   # 16 -> 32 @ 16x16
    (16384, 4, 1, 32, 64, 8, 8, 3, 1),    # 32 -> 64 @ 8x8, the largest ring
])
def test_conv_shapes(gpu_lib, N, L, B, C, M, H, W, h, P):
    conv_case(gpu_lib, N, L, B, C, M, H, W, h, P, seed=N + C + M, decrypt_check=1)


@pytest.mark.gpu
def test_weight_gradient_full_size(gpu_lib):
    # batch 32, 16 -> 16 channels, 16x16 maps, 3x3 kernel; ciphertexts uniform mod q_i,
    # plaintexts uniform mod t over all N coefficients (masked shares)
    he = gpu_lib
    N, L, B, C, M, H, h, P = 8192, 3, 32, 16, 16, 16, 3, 1
    ctx = he.Context(N, L)
    plan = he.Plan(ctx, he.HE_KIND_DW, B=B, C=C, M=M, H=H, W=H, h=h, P=P)
    info = plan.info
    g = packing.dw_geometry(C, H, H, H + 2 * P - h + 1, P, N)
    assert (info["O"], info["S"], info["Cw"], info["cb"]) == (g.O, g.S, g.Cw, g.cb) == (31, 961, 8, 2)
    cb = g.cb
    ct = synth.uniform_residues(synth.rng(3, synth.STREAM_CT), (B * (cb + M), 2), ctx.q, N)
    ptv = synth.uniform_mod_t(synth.rng(3, synth.STREAM_MASK), (B * (M + cb), N))
    row, cti, pti = packing.dw_terms(B, M, cb)
    lrow, lcti, lpti = he.he_plan_terms(plan.h)
    assert np.array_equal(lrow, row) and np.array_equal(lcti, cti) and np.array_equal(lpti, pti)
    expect = core.csr_cpmul(ct, core.lift(ptv, ctx.q), row, cti, pti, ctx.q, ctx.psi, method=2)
    got = run_layer(he, ctx, plan, ct, torch.from_numpy(ptv).cuda(), he.HE_PLAIN_POLY)
    assert_equal_u64(got, expect, "dW")


@pytest.mark.gpu
def test_weight_gradient_decrypts_to_the_protocol_identity(gpu_lib):
    # small end-to-end case: Dec(out) = X (x) (dY - r1) + dY (x) (X - r2) mod t, and with
    # r1 = r2 = 0 the extracted coefficients are the plaintext weight gradient
    he = gpu_lib
    N, L, B, C, M, H, h, P = 1024, 2, 2, 3, 2, 6, 3, 1
    ctx = he.Context(N, L)
    plan = he.Plan(ctx, he.HE_KIND_DW, B=B, C=C, M=M, H=H, W=H, h=h, P=P)
    Ho = H + 2 * P - h + 1
    g = packing.dw_geometry(C, H, H, Ho, P, N)
    x = synth.int8_uniform(synth.rng(31, synth.STREAM_ACT), (B, C, H, H)) // 8
    dy = synth.int8_uniform(synth.rng(31, synth.STREAM_PT), (B, M, Ho, Ho)) // 8
    xp = np.stack([packing.pack_conv_input(x[b], g) for b in range(B)])               # [B, cb, N]
    dyp = np.stack([np.stack([packing.pi_w(dy[b, m], g.O, N) for m in range(M)]) for b in range(B)])
    ct_polys = np.concatenate([xp, dyp], axis=1)                                        # [B, cb + M, N]
    ct, s = encrypt_polys(ctx, ct_polys, 31)
    pt_polys = np.concatenate([dyp, xp], axis=1).reshape(-1, N)                         # r = 0
    got = run_layer(he, ctx, plan, ct, torch.from_numpy(pt_polys.astype(np.int64)).cuda(), he.HE_PLAIN_POLY)
    ref = np.stack([plain.conv2d_weight_grad(x[b], dy[b], P, h) for b in range(B)]).sum(0)   # [M, C, h, h]
    dec = np.stack([bfv.decrypt(got[o], s, ctx.q, ctx.psi, T) for o in range(got.shape[0])])
    dec_signed = np.where(dec > T // 2, dec - T, dec)
    lib_dw = he.he_extract_output(plan.h, dec_signed, M * C * h * h).reshape(M, C, h, h)
    assert np.array_equal(lib_dw, 2 * ref)        # both protocol terms give X (x) dY


@pytest.mark.gpu
@pytest.mark.parametrize("N,L,B,n_in,n_out", [(8192, 3, 2, 1024, 256), (4096, 2, 1, 256, 10), (16384, 4, 1, 1024, 256)])
def test_fc_parity_and_decrypt(gpu_lib, N, L, B, n_in, n_out):
    he = gpu_lib
    ctx = he.Context(N, L)
    plan = he.Plan(ctx, he.HE_KIND_FC, B=B, n_in=n_in, n_out=n_out)
    g = packing.FcGeometry(n_in, n_out, N)
    info = plan.info
    assert (info["n_iw"], info["n_ow"]) == (g.n_iw, g.n_ow)
    x = synth.int8_uniform(synth.rng(40, synth.STREAM_ACT), (B, n_in))
    Wm = synth.int8_uniform(synth.rng(40, synth.STREAM_PT), (n_out, n_in))
    xin = np.stack([packing.pack_fc_input(x[b], g) for b in range(B)])
    assert np.array_equal(he.he_pack_input(plan.h, x.reshape(-1), B * g.in_ct * N).reshape(B, g.in_ct, N), xin)
    ct, s = encrypt_polys(ctx, xin, 40)
    pt = core.lift(packing.pack_fc_weight(Wm, g).reshape(-1, N), ctx.q)
    row, cti, pti = packing.fc_terms(B, g.in_ct, g.out_ct)
    expect = core.csr_cpmul(ct, pt, row, cti, pti, ctx.q, ctx.psi, method=2)
    got = run_layer(he, ctx, plan, ct, torch.from_numpy(Wm.astype(np.int32).reshape(-1)).cuda())
    assert_equal_u64(got, expect, "fc")
    dec = np.stack([bfv.decrypt(got[o], s, ctx.q, ctx.psi, T) for o in range(got.shape[0])])
    y = he.he_extract_output(plan.h, dec, B * n_out).reshape(B, n_out)
    assert np.array_equal(y, plain.mod_t(np.stack([plain.matvec(Wm, x[b]) for b in range(B)]), T))


@pytest.mark.gpu
@pytest.mark.parametrize("N,L,B,C,M,H,h,P", [(1024, 2, 2, 3, 2, 6, 3, 1), (4096, 2, 2, 16, 8, 16, 3, 1),
                                             (2048, 2, 1, 4, 3, 7, 5, 2)])
def test_input_gradient_parity_and_decrypt(gpu_lib, N, L, B, C, M, H, h, P):
    # dX = conv(w, dY) with padding (Section 2, training) as the forward conv of dY
    # with the kernel transposed and rotated: bit-exact against the oracle's ring
    # products, decrypting to the plaintext input gradient mod t
    he = gpu_lib
    ctx = he.Context(N, L)
    plan = he.Plan(ctx, he.HE_KIND_DX, B=B, C=C, M=M, H=H, W=H, h=h, P=P)
    info = plan.info
    Ho = H + 2 * P - h + 1
    assert (info["Hout"], info["Wout"]) == (H, H)
    geo = packing.ConvGeometry(M, Ho, Ho, h, h - 1 - P, N)
    dy = synth.int8_uniform(synth.rng(80, synth.STREAM_ACT, N), (B, M, Ho, Ho))
    w = synth.int8_uniform(synth.rng(80, synth.STREAM_PT, N), (M, C, h, h))
    polys = he.he_pack_input(plan.h, dy.reshape(-1), B * info["cb"] * N).reshape(B, info["cb"], N)
    assert np.array_equal(polys, np.stack([packing.pack_conv_input(dy[b], geo) for b in range(B)]))
    ct, s = encrypt_polys(ctx, polys, 80)
    w_eq = np.ascontiguousarray(np.transpose(w, (1, 0, 2, 3))[:, :, ::-1, ::-1])
    pt = core.lift(packing.pack_conv_weight(w_eq, geo).reshape(-1, N), ctx.q)
    row, cti, pti = packing.conv_terms(B, C, geo.cb)
    expect = core.csr_cpmul(ct, pt, row, cti, pti, ctx.q, ctx.psi, method=2)
    d_w = torch.from_numpy(w.astype(np.int32).reshape(-1)).cuda()
    got = run_layer(he, ctx, plan, ct, d_w)
    assert_equal_u64(got, expect, "input gradient")
    # the same job inside a persistent batch
    out_b = he.empty_u64(tuple(got.shape))
    d_ct = he.to_device_u64(ct)
    bt = he.he_batch_create(0)
    he.he_batch_add(bt, ctx.h, plan.h, d_ct, d_w, out_b, 0)
    he.he_batch_build(bt)
    he.he_batch_run(bt)
    he.he_batch_sync(bt)
    assert_equal_u64(he.to_numpy_u64(out_b), expect, "input gradient, batched")
    he.he_batch_destroy(bt)
    dec = np.stack([bfv.decrypt(got[o], s, ctx.q, ctx.psi, T) for o in range(got.shape[0])])
    dx = he.he_extract_output(plan.h, dec, B * C * H * H).reshape(B, C, H, H)
    for b in range(B):
        assert np.array_equal(dx[b], plain.mod_t(plain.conv2d_input_grad(dy[b], w, P, H, H), T)), b


@pytest.mark.gpu
@pytest.mark.parametrize("kind,N,L,B,C,M,H,h,P", [("conv", 4096, 2, 1, 3, 4, 64, 5, 2),
                                                  ("conv", 2048, 2, 2, 2, 3, 46, 3, 1),
                                                  ("dx", 1024, 2, 1, 2, 2, 32, 3, 1),
                                                  ("conv", 8192, 3, 2, 3, 3, 64, 5, 2)])
def test_windowed_layers_parity_and_decrypt(gpu_lib, kind, N, L, B, C, M, H, h, P):
    # maps split into windows (Section 3.3), because one channel does not fit
    # one polynomial or (the last case) because two 32 x 64 tiles holding all
    # three channels take fewer products: the plan's windows are the oracle's, every output
    # ciphertext matches the oracle's ring products over the window term lists,
    # and the overlap-added decryption is the plaintext layer mod t
    he = gpu_lib
    ctx = he.Context(N, L)
    Ho = H + 2 * P - h + 1
    if kind == "conv":
        plan = he.Plan(ctx, he.HE_KIND_CONV, B=B, C=C, M=M, H=H, W=H, h=h, P=P)
        x = synth.int8_uniform(synth.rng(85, synth.STREAM_ACT, N), (B, C, H, H))
        w = synth.int8_uniform(synth.rng(85, synth.STREAM_PT, N), (M, C, h, h))
        g = packing.WindowGeometry(C, M, H, H, h, P, N)
        w_eq, M_out = w, M
    else:
        plan = he.Plan(ctx, he.HE_KIND_DX, B=B, C=C, M=M, H=H, W=H, h=h, P=P)
        x = synth.int8_uniform(synth.rng(86, synth.STREAM_ACT, N), (B, M, Ho, Ho))        # dY
        w = synth.int8_uniform(synth.rng(86, synth.STREAM_PT, N), (M, C, h, h))
        g = packing.WindowGeometry(M, C, Ho, Ho, h, h - 1 - P, N)
        w_eq, M_out = np.ascontiguousarray(np.transpose(w, (1, 0, 2, 3))[:, :, ::-1, ::-1]), C
    info = plan.info
    assert g.tiles > 1
    for k in ("O", "S", "Cw", "cb", "Hw", "Ww", "tiles"):
        assert info[k] == getattr(g, k), k
    polys = np.stack([g.pack_input(x[b]) for b in range(B)])                    # [B, tiles, cb, N]
    lib_polys = he.he_pack_input(plan.h, x.reshape(-1), polys.size)
    assert np.array_equal(lib_polys, polys.reshape(-1))
    ct, s = encrypt_polys(ctx, polys, 85)
    pt = core.lift(g.pack_weight(w_eq).reshape(-1, N), ctx.q)
    row, cti, pti = g.terms(B)
    expect = core.csr_cpmul(ct, pt, row, cti, pti, ctx.q, ctx.psi, method=2)
    got = run_layer(he, ctx, plan, ct, torch.from_numpy(w.astype(np.int32).reshape(-1)).cuda())
    assert_equal_u64(got, expect, "%s windows" % kind)
    dec = np.stack([bfv.decrypt(got[o], s, ctx.q, ctx.psi, T) for o in range(got.shape[0])])
    Hout = info["Hout"]
    y = np.remainder(he.he_extract_output(plan.h, dec, B * M_out * Hout * Hout), T).reshape(B, M_out, Hout, Hout)
    for b in range(B):
        if kind == "conv":
            ref = plain.conv2d(x[b], w, P)
        else:
            ref = plain.conv2d_input_grad(x[b], w, P, H, H)
        assert np.array_equal(y[b], plain.mod_t(ref, T)), b


@pytest.mark.gpu
@pytest.mark.parametrize("N,L,B,C,M,H,h,P,stride", [(1024, 2, 2, 3, 2, 9, 3, 1, 2), (4096, 2, 1, 3, 2, 64, 5, 2, 2),
                                                    (2048, 2, 1, 2, 2, 12, 3, 0, 3)])
def test_strided_conv(gpu_lib, N, L, B, C, M, H, h, P, stride):
    # a stride subsamples the correlation the ring product holds: the ciphertexts
    # equal the unstrided layer's, and the strided extraction of their decryption
    # is the strided plaintext convolution (also with windows: the 64 x 64 case)
    he = gpu_lib
    ctx = he.Context(N, L)
    p1 = he.Plan(ctx, he.HE_KIND_CONV, B=B, C=C, M=M, H=H, W=H, h=h, P=P)
    ps = he.Plan(ctx, he.HE_KIND_CONV, B=B, C=C, M=M, H=H, W=H, h=h, P=P, stride=stride)
    info = ps.info
    assert info["Hout"] == (H + 2 * P - h) // stride + 1
    for k in ("n_ct_in", "n_pt", "n_ct_out", "n_terms", "O", "S", "tiles"):
        assert info[k] == p1.info[k], k
    x = synth.int8_uniform(synth.rng(88, synth.STREAM_ACT, N), (B, C, H, H))
    w = synth.int8_uniform(synth.rng(88, synth.STREAM_PT, N), (M, C, h, h))
    polys = he.he_pack_input(ps.h, x.reshape(-1), info["n_ct_in"] * N).reshape(-1, N)
    ct, s = encrypt_polys(ctx, polys, 88)
    d_w = torch.from_numpy(w.astype(np.int32).reshape(-1)).cuda()
    got = run_layer(he, ctx, ps, ct, d_w)
    assert_equal_u64(got, run_layer(he, ctx, p1, ct, d_w), "strided vs unstrided ciphertexts")
    dec = np.stack([bfv.decrypt(got[o], s, ctx.q, ctx.psi, T) for o in range(got.shape[0])])
    Ho = info["Hout"]
    y = np.remainder(he.he_extract_output(ps.h, dec, B * M * Ho * Ho), T).reshape(B, M, Ho, Ho)
    for b in range(B):
        assert np.array_equal(y[b], plain.mod_t(plain.conv2d_strided(x[b], w, P, stride), T)), b
    with pytest.raises(he.HeError) as ei:
        he.Plan(ctx, he.HE_KIND_DX, B=B, C=C, M=M, H=H, W=H, h=h, P=P, stride=stride)
    assert ei.value.status == he.HE_EUNSUPPORTED
