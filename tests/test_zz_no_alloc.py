"""The allocation-free per-layer entry point (he_corr_conv2d_noalloc) against the
workspace entry point (he_corr_conv2d): the same bytes, bit for bit, on two
calls in a row -- the conv-forward workload, then a smaller layer on another
ring through the unfused kernels -- so the second call runs over what the
first left in the shared scratch array; sizes beyond the array are refused."""
import numpy as np
import pytest
import torch

from paper_2409_16675_amd import synth
from tests.helpers import assert_equal_u64


def _layer(he, N, L, B, C, M, H, seed):
    ctx = he.Context(N, L)
    plan = he.Plan(ctx, he.HE_KIND_CONV, B=B, C=C, M=M, H=H, W=H, h=3, P=1)
    info = plan.info
    ct = he.to_device_u64(synth.uniform_residues(synth.rng(seed, synth.STREAM_CT), (info["n_ct_in"], 2), ctx.q, N))
    w = synth.int8_uniform(synth.rng(seed, synth.STREAM_PT), (M, C, 3, 3))
    dw = torch.from_numpy(w.astype(np.int32).reshape(-1)).cuda()
    return ctx, plan, info, ct, dw


def _both(he, ctx, plan, info, ct, dw, flags):
    shape = (info["n_ct_out"], 2, ctx.L, ctx.N)
    ref = he.empty_u64(shape)
    ws = he.workspace(plan.workspace_size(flags))
    he.he_corr_conv2d(ctx.h, plan.h, ct, dw, ref, flags, ws, ws.numel())
    got = he.empty_u64(shape)
    got.view(torch.int64).fill_(-1)
    torch.cuda.synchronize()
    he.he_corr_conv2d_noalloc(ctx.h, plan.h, ct, dw, got, flags)
    torch.cuda.synchronize()
    return he.to_numpy_u64(got), he.to_numpy_u64(ref)


@pytest.mark.gpu
def test_noalloc_equals_workspace_entry_point_on_two_calls(gpu_lib):
    he = gpu_lib
    # 1: batch 16 of 3x32x32 -> 16 channels, N = 8192, three primes (about 10 MiB of scratch)
    big = _layer(he, 8192, 3, 16, 3, 16, 32, 70)
    print("case noalloc conv workload", flush=True)
    got, ref = _both(he, *big, 0)
    assert_equal_u64(got, ref, "noalloc vs workspace, conv workload")
    # 2: smaller input on another ring, unfused kernels (another scratch layout)
    small = _layer(he, 4096, 2, 2, 16, 8, 16, 71)
    print("case noalloc small unfused", flush=True)
    got, ref = _both(he, *small, he.HE_UNFUSED)
    assert_equal_u64(got, ref, "noalloc vs workspace, second smaller call")


@pytest.mark.gpu
def test_noalloc_refuses_what_does_not_fit(gpu_lib):
    he = gpu_lib
    ctx = he.Context(8192, 3)
    # the weight-gradient workload needs about 330 MB of workspace
    plan = he.Plan(ctx, he.HE_KIND_DW, B=32, C=16, M=16, H=16, W=16, h=3, P=1)
    assert plan.workspace_size(he.HE_PLAIN_POLY) > (he.HE_NOALLOC_SCRATCH_MB << 20)
    dummy = he.empty_u64((1,))
    with pytest.raises(he.HeError) as ei:
        he.he_corr_conv2d_noalloc(ctx.h, plan.h, dummy, dummy, dummy, he.HE_PLAIN_POLY)
    assert ei.value.status == he.HE_ENOMEM
    small = he.Plan(ctx, he.HE_KIND_CONV, B=1, C=3, M=2, H=8, W=8, h=3, P=1)
    with pytest.raises(he.HeError) as ei:
        he.he_corr_conv2d_noalloc(ctx.h, small.h, dummy, dummy, dummy, he.HE_VALIDATE)
    assert ei.value.status == he.HE_EINVAL
