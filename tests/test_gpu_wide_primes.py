"""GPU parity with 60-bit primes: every kernel that the 48-bit default contexts
never reach runs here through the 64-bit integer arithmetic (Shoup products,
128-bit multiply-accumulate, signed lifts through a 64-bit remainder).

Covered, bit for bit against the oracle (tolerance 0: exact integers):
  - the conv-forward layer (batch 16 of 3x32x32, 16 output channels, 3x3,
    pad 1, N = 8192, three 60-bit primes), all 256 outputs, fused and unfused;
  - the weight-gradient layer at full size (batch 32, 16 -> 16 channels,
    16x16 maps, CryptoTrain-P terms of Section 3.2, plaintexts given as
    packed polynomials uniform mod t);
  - an uneven mix over N = 4096 / 8192 / 16384 in one persistent launch
    (the mixed-degree 64-bit variant), each job also equal to its own
    per-layer run;
  - served jobs (continuous batching) equal to the oracle.
The primes are the L largest below 2^60 with q = 1 mod 2N."""
import numpy as np
import pytest
import torch

from oracle import core, packing
from paper_2409_16675_amd import synth
from tests.helpers import assert_equal_u64
from tests.test_gpu_batch import make_job, oracle_out
from tests.test_gpu_conv import conv_case, run_layer

BITS = 60


@pytest.fixture(scope="module")
def wide_ctxs(gpu_lib):
    return {(N, L): gpu_lib.Context(N, L, prime_bits=BITS) for N, L in synth.MIX_RINGS}


@pytest.mark.gpu
def test_wide_contexts_use_integer_arithmetic(gpu_lib, wide_ctxs):
    he = gpu_lib
    for (N, L), ctx in wide_ctxs.items():
        assert ctx.arith == he.HE_ARITH_U64
        assert all((1 << 59) < q < (1 << 60) and q % (2 * N) == 1 for q in ctx.q)
        assert list(ctx.q) == list(core.find_primes(N, BITS, L))


@pytest.mark.gpu
@pytest.mark.parametrize("unfused", [False, True])
def test_conv_forward_workload_60bit(gpu_lib, unfused):
    he = gpu_lib
    print("case conv forward 60-bit unfused=%s" % unfused, flush=True)
    flags = he.HE_UNFUSED if unfused else 0
    ctx, plan, got, s, ref = conv_case(he, 8192, 3, 16, 3, 16, 32, 32, 3, 1, seed=2, flags=flags,
                                       decrypt_check=2, bits=BITS)
    assert ctx.arith == he.HE_ARITH_U64 and got.shape == (256, 2, 3, 8192)


@pytest.mark.gpu
def test_conv_shapes_60bit(gpu_lib):
    # signed weight lifts at every ring degree, several channel blocks
    for args in [(1024, 2, 3, 10, 3, 6, 6, 3, 2), (4096, 2, 1, 16, 32, 16, 16, 3, 1),
                 (16384, 4, 1, 32, 64, 8, 8, 3, 1)]:
        print("case conv 60-bit %s" % (args,), flush=True)
        conv_case(gpu_lib, *args, seed=args[0] + 7, decrypt_check=1, bits=BITS)


@pytest.mark.gpu
def test_weight_gradient_full_size_60bit(gpu_lib):
    he = gpu_lib
    N, L, B, C, M, H, h, P = 8192, 3, 32, 16, 16, 16, 3, 1
    ctx = he.Context(N, L, prime_bits=BITS)
    plan = he.Plan(ctx, he.HE_KIND_DW, B=B, C=C, M=M, H=H, W=H, h=h, P=P)
    g = packing.dw_geometry(C, H, H, H + 2 * P - h + 1, P, N)
    cb = g.cb
    ct = synth.uniform_residues(synth.rng(3, synth.STREAM_CT, 60), (B * (cb + M), 2), ctx.q, N)
    ptv = synth.uniform_mod_t(synth.rng(3, synth.STREAM_MASK, 60), (B * (M + cb), N))
    row, cti, pti = packing.dw_terms(B, M, cb)
    expect = core.csr_cpmul(ct, core.lift(ptv, ctx.q), row, cti, pti, ctx.q, ctx.psi, method=2)
    print("case dW full size 60-bit", flush=True)
    got = run_layer(he, ctx, plan, ct, torch.from_numpy(ptv).cuda(), he.HE_PLAIN_POLY)
    assert_equal_u64(got, expect, "dW 60-bit")
    # the same layer with the plaintexts' signed representatives (v - t): the lift
    # v mod q_i of a negative integer goes through the signed remainder
    neg = ptv - np.int64(synth.T_PLAIN)
    expect_n = core.csr_cpmul(ct, core.lift(neg, ctx.q), row, cti, pti, ctx.q, ctx.psi, method=2)
    got_n = run_layer(he, ctx, plan, ct, torch.from_numpy(neg).cuda(), he.HE_PLAIN_POLY)
    assert_equal_u64(got_n, expect_n, "dW 60-bit, negative plaintexts")


@pytest.mark.gpu
def test_uneven_mix_60bit_matches_oracle_and_alone(gpu_lib, wide_ctxs):
    he = gpu_lib
    mix = synth.job_mix(24, workload=40)
    jobs = [make_job(he, wide_ctxs, lay, ring, 6000 + k) for k, (lay, ring) in enumerate(mix)]
    b = he.he_batch_create(0)
    for j in jobs:
        he.he_batch_add(b, j["ctx"].h, j["plan"].h, j["d_ct"], j["d_w"], j["out"], 0)
    he.he_batch_build(b)
    info = he.he_batch_get_info(b)
    assert info["arith"] == he.HE_ARITH_U64 and info["n_jobs"] == len(jobs)
    print("case 60-bit mix of %d jobs, rings %s" % (len(jobs), sorted({r for _, r in mix})), flush=True)
    for rep in range(2):
        for j in jobs:
            j["out"].view(torch.int64).zero_()
        torch.cuda.synchronize()
        he.he_batch_run(b)
        he.he_batch_sync(b)
        for k, j in enumerate(jobs):
            assert_equal_u64(he.to_numpy_u64(j["out"]), oracle_out(j), "60-bit job %d rep %d" % (k, rep))
    he.he_batch_destroy(b)
    for k, j in enumerate(jobs):
        alone = he.empty_u64(tuple(j["out"].shape))
        ws = he.workspace(j["plan"].workspace_size())
        he.he_corr_conv2d(j["ctx"].h, j["plan"].h, j["d_ct"], j["d_w"], alone, 0, ws, ws.numel())
        torch.cuda.synchronize()
        assert_equal_u64(he.to_numpy_u64(alone), he.to_numpy_u64(j["out"]), "60-bit job %d alone vs mix" % k)


@pytest.mark.gpu
def test_single_degree_batch_60bit(gpu_lib, wide_ctxs):
    # a batch of one ring degree with 60-bit primes (the 64-bit arithmetic has
    # one persistent variant per largest degree); conv and FC jobs at N = 8192
    he = gpu_lib
    jobs = [make_job(he, wide_ctxs, lay, 1, 6100 + lay) for lay in range(5)]
    b = he.he_batch_create(0)
    for j in jobs:
        he.he_batch_add(b, j["ctx"].h, j["plan"].h, j["d_ct"], j["d_w"], j["out"], 0)
    he.he_batch_build(b)
    he.he_batch_run(b)
    he.he_batch_sync(b)
    for k, j in enumerate(jobs):
        assert_equal_u64(he.to_numpy_u64(j["out"]), oracle_out(j), "60-bit single-degree job %d" % k)
    he.he_batch_destroy(b)


@pytest.mark.gpu
def test_served_jobs_60bit(gpu_lib, wide_ctxs):
    he = gpu_lib
    mix = synth.job_mix(12, workload=41)
    jobs = [make_job(he, wide_ctxs, lay, ring, 6200 + k) for k, (lay, ring) in enumerate(mix)]
    srv = he.he_server_create(mem_cap_bytes=8 << 30, slots=2, max_batch_jobs=8)
    arr = synth.poisson_arrivals(len(jobs), 20000.0, workload=41)
    arr -= arr[0]
    print("case served 60-bit jobs", flush=True)
    lat = he.he_server_replay(srv, [j["ctx"].h for j in jobs],
                              [(j["plan"].h, j["d_ct"], j["d_w"], j["out"], 0) for j in jobs], arr)
    st = he.he_server_stats(srv)
    he.he_server_destroy(srv)
    assert st["completed"] == len(jobs) and (lat > 0).all()
    for k, j in enumerate(jobs):
        assert_equal_u64(he.to_numpy_u64(j["out"]), oracle_out(j), "served 60-bit job %d" % k)
