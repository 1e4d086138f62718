"""GPU parity of the persistent batch kernel: an uneven mix of 64 layer jobs over
three ring degrees, each job bit-identical to the oracle and to its own
stand-alone run; graph replays, rebinding and accumulation."""
import numpy as np
import pytest
import torch

from oracle import core, packing
from paper_2409_16675_amd import synth
from tests.helpers import assert_equal_u64


def make_job(he, ctxs, layer, ring, seed):
    """Synthetic job: ciphertexts uniform mod q_i, int8 weights, batch 1."""
    N, L = synth.MIX_RINGS[ring]
    ctx = ctxs[(N, L)]
    spec = synth.MIX_LAYERS[layer]
    g = synth.rng(4, synth.STREAM_CT, seed)
    gw = synth.rng(4, synth.STREAM_PT, seed)
    if spec[0] == "conv":
        _, C, M, H, W, h, P = spec
        plan = he.Plan(ctx, he.HE_KIND_CONV, B=1, C=C, M=M, H=H, W=W, h=h, P=P)
        geo = packing.ConvGeometry(C, H, W, h, P, N)
        w = synth.int8_uniform(gw, (M, C, h, h))
        pt = core.lift(packing.pack_conv_weight(w, geo).reshape(-1, N), ctx.q)
        row, cti, pti = packing.conv_terms(1, M, geo.cb)
    else:
        _, n_in, n_out = spec
        plan = he.Plan(ctx, he.HE_KIND_FC, B=1, n_in=n_in, n_out=n_out)
        geo = packing.FcGeometry(n_in, n_out, N)
        w = synth.int8_uniform(gw, (n_out, n_in))
        pt = core.lift(packing.pack_fc_weight(w, geo).reshape(-1, N), ctx.q)
        row, cti, pti = packing.fc_terms(1, geo.in_ct, geo.out_ct)
    info = plan.info
    ct = synth.uniform_residues(g, (info["n_ct_in"], 2), ctx.q, N)
    return dict(ctx=ctx, plan=plan, info=info, ct=ct, w=w, pt=pt, terms=(row, cti, pti),
                d_ct=he.to_device_u64(ct), d_w=torch.from_numpy(w.astype(np.int32).reshape(-1)).cuda(),
                out=he.empty_u64((info["n_ct_out"], 2, L, N)))


def oracle_out(job):
    row, cti, pti = job["terms"]
    ctx = job["ctx"]
    return core.csr_cpmul(job["ct"], job["pt"], row, cti, pti, ctx.q, ctx.psi, method=2)


@pytest.fixture(scope="module")
def ctxs(gpu_lib):
    return {(N, L): gpu_lib.Context(N, L) for N, L in synth.MIX_RINGS}


@pytest.mark.gpu
def test_uneven_mix_of_64_jobs_matches_oracle_and_alone(gpu_lib, ctxs):
    he = gpu_lib
    mix = synth.job_mix(64)
    jobs = [make_job(he, ctxs, lay, ring, k) for k, (lay, ring) in enumerate(mix)]
    b = he.he_batch_create(0)
    for j in jobs:
        he.he_batch_add(b, j["ctx"].h, j["plan"].h, j["d_ct"], j["d_w"], j["out"], 0)
    he.he_batch_build(b)
    info = he.he_batch_get_info(b)
    assert info["n_jobs"] == 64 and info["cpmul"] == sum(j["info"]["n_terms"] for j in jobs)
    he.he_batch_run(b)
    he.he_batch_sync(b)
    for k, j in enumerate(jobs):
        print("case mix job %d layer=%s ring=%s" % (k, mix[k][0], mix[k][1]), flush=True)
        got = he.to_numpy_u64(j["out"])
        assert_equal_u64(got, oracle_out(j), "job %d vs oracle" % k)
        # the same job alone through the per-layer entry point
        alone = he.empty_u64(tuple(j["out"].shape))
        ws = he.workspace(j["plan"].workspace_size())
        he.he_corr_conv2d(j["ctx"].h, j["plan"].h, j["d_ct"], j["d_w"], alone, 0, ws, ws.numel())
        torch.cuda.synchronize()
        assert_equal_u64(he.to_numpy_u64(alone), got, "job %d alone vs mix" % k)
    he.he_batch_destroy(b)


@pytest.mark.gpu
def test_graph_replays_with_eager_work_between(gpu_lib, ctxs):
    he = gpu_lib
    jobs = [make_job(he, ctxs, lay, ring, 100 + k) for k, (lay, ring) in enumerate([(0, 1), (3, 0), (1, 2), (4, 1)])]
    expect = [oracle_out(j) for j in jobs]
    b = he.he_batch_create(0)
    for j in jobs:
        he.he_batch_add(b, j["ctx"].h, j["plan"].h, j["d_ct"], j["d_w"], j["out"], 0)
    he.he_batch_build(b, he.HE_BATCH_GRAPH)
    for rep in range(4):
        for j in jobs:
            j["out"].view(torch.int64).zero_()          # eager work between replays
        torch.cuda.synchronize()
        he.he_batch_run(b)
        he.he_batch_sync(b)
        for k, j in enumerate(jobs):
            assert_equal_u64(he.to_numpy_u64(j["out"]), expect[k], "replay %d job %d" % (rep, k))
    he.he_batch_destroy(b)


@pytest.mark.gpu
def test_rebind_accumulate_and_no_graph(gpu_lib, ctxs):
    he = gpu_lib
    j1 = make_job(he, ctxs, 1, 1, 200)
    j2 = make_job(he, ctxs, 1, 1, 201)       # same layer shape, other data
    b = he.he_batch_create(0)
    idx = he.he_batch_add(b, j1["ctx"].h, j1["plan"].h, j1["d_ct"], j1["d_w"], j1["out"], 0)
    he.he_batch_build(b, 0)                     # direct launches, no graph
    he.he_batch_run(b)
    he.he_batch_sync(b)
    e1 = oracle_out(j1)
    assert_equal_u64(he.to_numpy_u64(j1["out"]), e1, "first")
    # point the job at the second data set (same plan)
    he.he_batch_rebind(b, idx, j1["plan"].h, j2["d_ct"], j2["d_w"], j2["out"], 0)
    he.he_batch_run(b)
    he.he_batch_sync(b)
    e2 = oracle_out(j2)
    assert_equal_u64(he.to_numpy_u64(j2["out"]), e2, "rebound")
    # accumulate into the previous result: 2x
    he.he_batch_rebind(b, idx, j1["plan"].h, j2["d_ct"], j2["d_w"], j2["out"], he.HE_ACCUMULATE)
    he.he_batch_run(b)
    he.he_batch_sync(b)
    q = np.array(j2["ctx"].q, dtype=np.uint64)[None, None, :, None]
    assert_equal_u64(he.to_numpy_u64(j2["out"]), (e2 * np.uint64(2)) % q, "accumulate")
    he.he_batch_destroy(b)


@pytest.mark.gpu
def test_batched_conv_workload_and_transformed_inputs(gpu_lib, ctxs):
    # the conv forward workload (batch 16 of 3x32x32, 16 channels) as one batched job,
    # and a job whose inputs are already transformed (HE_IN_NTT)
    he = gpu_lib
    ctx = ctxs[(8192, 3)]
    plan = he.Plan(ctx, he.HE_KIND_CONV, B=16, C=3, M=16, H=32, W=32, h=3, P=1)
    geo = packing.ConvGeometry(3, 32, 32, 3, 1, 8192)
    ct = synth.uniform_residues(synth.rng(2, synth.STREAM_CT), (16, 2), ctx.q, 8192)
    w = synth.int8_uniform(synth.rng(2, synth.STREAM_PT), (16, 3, 3, 3))
    pt = core.lift(packing.pack_conv_weight(w, geo).reshape(-1, 8192), ctx.q)
    row, cti, pti = packing.conv_terms(16, 16, 1)
    expect = core.csr_cpmul(ct, pt, row, cti, pti, ctx.q, ctx.psi, method=2)
    d_w = torch.from_numpy(w.astype(np.int32).reshape(-1)).cuda()
    out = he.empty_u64((256, 2, 3, 8192))
    out2 = he.empty_u64((256, 2, 3, 8192))
    ct_hat = core.ntt_planes(ct, ctx.q, ctx.psi)
    # the batch keeps raw device pointers: the input tensors must outlive it
    d_ct, d_ct_hat = he.to_device_u64(ct), he.to_device_u64(ct_hat)
    b = he.he_batch_create(0)
    he.he_batch_add(b, ctx.h, plan.h, d_ct, d_w, out, 0)
    he.he_batch_add(b, ctx.h, plan.h, d_ct_hat, d_w, out2, he.HE_IN_NTT)
    he.he_batch_build(b)
    he.he_batch_run(b)
    he.he_batch_sync(b)
    assert_equal_u64(he.to_numpy_u64(out), expect, "batched conv")
    assert_equal_u64(he.to_numpy_u64(out2), expect, "batched conv, transformed inputs")
    he.he_batch_destroy(b)


@pytest.mark.gpu
@pytest.mark.parametrize("loge", [3, 4, 5])
def test_single_degree_variants(gpu_lib, ctxs, loge):
    # a batch of one ring degree runs the single-degree persistent variant with the
    # coefficients-per-thread of the context's multiply-accumulate schedule, clamped
    # to the compiled 16 and 32 (a schedule of 8 runs the 16 variant): every case
    # against the oracle, with a layer job and a multi-ciphertext FC job per ring
    he = gpu_lib
    for ring, (N, L) in enumerate(synth.MIX_RINGS):
        ctx = ctxs[(N, L)]
        if (he.HE_ARITH_F64, loge) not in he.compiled_schedules(N):
            continue                       # more than 1024 threads per plane
        saved = he.he_ctx_get_schedule(ctx.h, he.HE_OP_MAC)
        he.he_ctx_set_schedule(ctx.h, he.HE_OP_MAC, he.HE_ARITH_F64, loge)
        try:
            jobs = [make_job(he, ctxs, lay, ring, 300 + 10 * loge + k) for k, lay in enumerate([0, 4])]
            expect = [oracle_out(j) for j in jobs]
            b = he.he_batch_create(0)
            for j in jobs:
                he.he_batch_add(b, j["ctx"].h, j["plan"].h, j["d_ct"], j["d_w"], j["out"], 0)
            he.he_batch_build(b, he.HE_BATCH_GRAPH)
            print("case variant N=%d loge=%d" % (N, loge), flush=True)
            for rep in range(2):
                he.he_batch_run(b)
                he.he_batch_sync(b)
                for k, j in enumerate(jobs):
                    assert_equal_u64(he.to_numpy_u64(j["out"]), expect[k], "N=%d loge=%d job %d rep %d" % (N, loge, k, rep))
            he.he_batch_destroy(b)
        finally:
            he.he_ctx_set_schedule(ctx.h, he.HE_OP_MAC, *saved)


@pytest.mark.gpu
def test_profiled_direct_launches(gpu_lib, ctxs):
    # HE_BATCH_PROFILE times the persistent kernel with HIP events; results unchanged
    he = gpu_lib
    jobs = [make_job(he, ctxs, lay, 1, 400 + k) for k, lay in enumerate([0, 3])]
    expect = [oracle_out(j) for j in jobs]
    b = he.he_batch_create(0)
    for j in jobs:
        he.he_batch_add(b, j["ctx"].h, j["plan"].h, j["d_ct"], j["d_w"], j["out"], 0)
    he.he_batch_build(b, he.HE_BATCH_PROFILE)
    for _ in range(3):
        he.he_batch_run(b)
    he.he_batch_sync(b)
    info = he.he_batch_get_info(b)
    assert info["kernel_launches"] == 3 and info["kernel_ms"] > 0.0
    for k, j in enumerate(jobs):
        assert_equal_u64(he.to_numpy_u64(j["out"]), expect[k], "profiled job %d" % k)
    he.he_batch_destroy(b)


@pytest.mark.gpu
def test_timed_out_wait_is_reported_after_a_later_run(gpu_lib, ctxs):
    # a spin limit of 0 makes every dependency wait give up at its first poll
    # (forced from the host: the kernel still finishes every task); the error
    # flag must survive the next, normal run and be reported by the sync, once
    he = gpu_lib
    jobs = [make_job(he, ctxs, 0, 1, 450 + k) for k in range(2)]   # conv 3->16 @32x32, N = 8192
    expect = [oracle_out(j) for j in jobs]
    b = he.he_batch_create(0)
    for j in jobs:
        he.he_batch_add(b, j["ctx"].h, j["plan"].h, j["d_ct"], j["d_w"], j["out"], 0)
    he.he_batch_build(b, 0)                     # direct launches read the limit at each run
    he.he_batch_set_spin_limit(b, 0)
    he.he_batch_run(b)
    he.he_batch_set_spin_limit(b, 1 << 20)
    he.he_batch_run(b)
    with pytest.raises(he.HeError) as ei:
        he.he_batch_sync(b)
    assert ei.value.status == he.HE_ETIMEOUT
    # reported once: the second run's outputs are right and the next sync is clean
    for k, j in enumerate(jobs):
        assert_equal_u64(he.to_numpy_u64(j["out"]), expect[k], "job %d after the normal run" % k)
    he.he_batch_run(b)
    he.he_batch_sync(b)
    he.he_batch_destroy(b)


@pytest.mark.gpu
def test_batched_weight_gradient_full_size(gpu_lib, ctxs):
    # the weight-gradient layer (batch 32, 16 -> 16 channels, 16x16 maps, 3x3
    # kernel; CryptoTrain-P terms, 64 products per output, so the accumulators
    # fold mid-sum) inside a persistent launch next to a conv job, twice
    he = gpu_lib
    N, L, B, C, M, H, h, P = 8192, 3, 32, 16, 16, 16, 3, 1
    ctx = ctxs[(N, L)]
    plan = he.Plan(ctx, he.HE_KIND_DW, B=B, C=C, M=M, H=H, W=H, h=h, P=P)
    cb = plan.info["cb"]
    ct = synth.uniform_residues(synth.rng(3, synth.STREAM_CT, 9), (B * (cb + M), 2), ctx.q, N)
    ptv = synth.uniform_mod_t(synth.rng(3, synth.STREAM_MASK, 9), (B * (M + cb), N))
    row, cti, pti = packing.dw_terms(B, M, cb)
    assert max(np.diff(row)) == 2 * B
    expect = core.csr_cpmul(ct, core.lift(ptv, ctx.q), row, cti, pti, ctx.q, ctx.psi, method=2)
    d_ct, d_pt = he.to_device_u64(ct), torch.from_numpy(ptv).cuda()
    out = he.empty_u64((plan.info["n_ct_out"], 2, L, N))
    conv = make_job(he, ctxs, 0, 1, 460)
    b = he.he_batch_create(0)
    he.he_batch_add(b, ctx.h, plan.h, d_ct, d_pt, out, he.HE_PLAIN_POLY)
    he.he_batch_add(b, conv["ctx"].h, conv["plan"].h, conv["d_ct"], conv["d_w"], conv["out"], 0)
    he.he_batch_build(b)
    print("case batched dW full size", flush=True)
    for rep in range(2):
        out.view(torch.int64).zero_()
        torch.cuda.synchronize()
        he.he_batch_run(b)
        he.he_batch_sync(b)
        assert_equal_u64(he.to_numpy_u64(out), expect, "batched dW rep %d" % rep)
        assert_equal_u64(he.to_numpy_u64(conv["out"]), oracle_out(conv), "conv beside dW rep %d" % rep)
    he.he_batch_destroy(b)


@pytest.mark.gpu
def test_strict_sync_batch_of_long_and_short_sums(gpu_lib, ctxs):
    # the strict mode (a fence at every dependency, for checking) gives the same
    # bytes: a 64-term weight gradient accumulated onto its output next to conv
    # jobs, two replays
    he = gpu_lib
    ctx = ctxs[(8192, 3)]
    N, L, B, C, M, H, h, P = 8192, 3, 32, 16, 16, 16, 3, 1
    plan = he.Plan(ctx, he.HE_KIND_DW, B=B, C=C, M=M, H=H, W=H, h=h, P=P)
    cb = plan.info["cb"]
    ct = synth.uniform_residues(synth.rng(3, synth.STREAM_CT, 21), (B * (cb + M), 2), ctx.q, N)
    ptv = synth.uniform_mod_t(synth.rng(3, synth.STREAM_MASK, 21), (B * (M + cb), N))
    row, cti, pti = packing.dw_terms(B, M, cb)
    expect = core.csr_cpmul(ct, core.lift(ptv, ctx.q), row, cti, pti, ctx.q, ctx.psi, method=2)
    out = he.empty_u64((plan.info["n_ct_out"], 2, L, N))
    base = synth.uniform_residues(synth.rng(3, synth.STREAM_A, 23), (plan.info["n_ct_out"], 2), ctx.q, N)
    q = np.array(ctx.q, dtype=np.uint64).reshape(1, 1, -1, 1)
    convs = [make_job(he, ctxs, 0, 1, 470 + k) for k in range(2)]
    b = he.he_batch_create(0)
    he.he_batch_add(b, convs[0]["ctx"].h, convs[0]["plan"].h, convs[0]["d_ct"], convs[0]["d_w"], convs[0]["out"], 0)
    he.he_batch_add(b, ctx.h, plan.h, he.to_device_u64(ct), torch.from_numpy(ptv).cuda(), out,
                    he.HE_PLAIN_POLY | he.HE_ACCUMULATE)
    he.he_batch_add(b, convs[1]["ctx"].h, convs[1]["plan"].h, convs[1]["d_ct"], convs[1]["d_w"], convs[1]["out"], 0)
    he.he_batch_build(b, he.HE_BATCH_GRAPH | he.HE_BATCH_STRICT_SYNC)
    print("case strict sync batch", flush=True)
    for rep in range(2):
        out.copy_(he.to_device_u64(base))
        torch.cuda.synchronize()
        he.he_batch_run(b)
        he.he_batch_sync(b)
        assert_equal_u64(he.to_numpy_u64(out), (base + expect) % q, "dW accumulated, strict, rep %d" % rep)
        for k, c in enumerate(convs):
            assert_equal_u64(he.to_numpy_u64(c["out"]), oracle_out(c), "conv %d strict rep %d" % (k, rep))
    he.he_batch_destroy(b)
