"""GPU tests of the serving loop: every job's output is byte-identical whether it
runs alone or among concurrent arrivals, admission respects the memory cap,
oversize jobs are refused, and sessions keep their transformed inputs resident."""
import numpy as np
import pytest
import torch

from paper_2409_16675_amd import synth
from tests.helpers import assert_equal_u64
from tests.test_gpu_batch import make_job, oracle_out


@pytest.fixture(scope="module")
def ctxs(gpu_lib):
    return {(N, L): gpu_lib.Context(N, L) for N, L in synth.MIX_RINGS}


def _mix_jobs(he, ctxs, n, seed0):
    mix = synth.job_mix(n)
    return mix, [make_job(he, ctxs, lay, ring, seed0 + k) for k, (lay, ring) in enumerate(mix)]


@pytest.mark.gpu
def test_served_results_equal_alone_results(gpu_lib, ctxs):
    he = gpu_lib
    mix, jobs = _mix_jobs(he, ctxs, 48, 500)
    # alone: each job through the per-layer entry point
    alone = []
    for j in jobs:
        out = he.empty_u64(tuple(j["out"].shape))
        ws = he.workspace(j["plan"].workspace_size())
        he.he_corr_conv2d(j["ctx"].h, j["plan"].h, j["d_ct"], j["d_w"], out, 0, ws, ws.numel())
        alone.append(out)
    torch.cuda.synchronize()
    srv = he.he_server_create(mem_cap_bytes=8 << 30, slots=2, max_batch_jobs=16)
    # Poisson arrivals at 20000 jobs/s so that jobs overlap on the device
    arr = synth.poisson_arrivals(len(jobs), 20000.0)
    arr -= arr[0]
    lat = he.he_server_replay(srv, [j["ctx"].h for j in jobs],
                              [(j["plan"].h, j["d_ct"], j["d_w"], j["out"], 0) for j in jobs], arr)
    st = he.he_server_stats(srv)
    he.he_server_destroy(srv)
    assert st["completed"] == len(jobs) and (lat > 0).all()
    assert st["epochs"] < len(jobs)          # several jobs shared an epoch (continuous batching)
    for k, j in enumerate(jobs):
        got = he.to_numpy_u64(j["out"])
        assert_equal_u64(got, he.to_numpy_u64(alone[k]), "job %d served vs alone" % k)
    # and the alone results are the oracle's (checked on a few jobs)
    for k in (0, 1, 2):
        assert_equal_u64(he.to_numpy_u64(alone[k]), oracle_out(jobs[k]), "job %d vs oracle" % k)


@pytest.mark.gpu
def test_sequential_mode_matches(gpu_lib, ctxs):
    he = gpu_lib
    mix, jobs = _mix_jobs(he, ctxs, 8, 600)
    srv = he.he_server_create(mem_cap_bytes=8 << 30, mode=he.HE_SERVE_SEQUENTIAL)
    tickets = [he.he_server_submit(srv, j["ctx"].h, j["plan"].h, j["d_ct"], j["d_w"], j["out"]) for j in jobs]
    for t in tickets:
        assert he.he_server_wait(srv, t)["status"] == 0
    st = he.he_server_stats(srv)
    he.he_server_destroy(srv)
    assert st["epochs"] == len(jobs)
    for k, j in enumerate(jobs):
        assert_equal_u64(he.to_numpy_u64(j["out"]), oracle_out(j), "sequential job %d" % k)


@pytest.mark.gpu
def test_admission_cap_queues_and_refuses(gpu_lib, ctxs):
    he = gpu_lib
    j_small = make_job(he, ctxs, 3, 0, 700)     # FC 256->10 at N=4096: tiny footprint
    j_big = make_job(he, ctxs, 2, 2, 701)       # conv 32->64 @8x8 at N=16384
    # a cap that fits the big job alone (about 106 MB: its output and input
    # buffers plus a workspace that either path can use) but not two at once
    cap = 150 << 20
    srv = he.he_server_create(mem_cap_bytes=cap, slots=2, arena_bytes=256 << 20)
    outs = [he.empty_u64(tuple(j_big["out"].shape)) for _ in range(3)]
    tickets = [he.he_server_submit(srv, j_big["ctx"].h, j_big["plan"].h, j_big["d_ct"], j_big["d_w"], o) for o in outs]
    for t in tickets:
        he.he_server_wait(srv, t)
    st = he.he_server_stats(srv)
    assert st["peak_bytes"] <= cap
    assert st["epochs"] == 3                 # the cap forced one big job at a time
    e_big = oracle_out(j_big)
    for o in outs:
        assert_equal_u64(he.to_numpy_u64(o), e_big, "capped big job")
    # a job larger than the cap is refused at submission
    srv2 = he.he_server_create(mem_cap_bytes=1 << 20, slots=1, arena_bytes=64 << 20)
    with pytest.raises(he.HeError) as ei:
        he.he_server_submit(srv2, j_big["ctx"].h, j_big["plan"].h, j_big["d_ct"], j_big["d_w"], outs[0])
    assert ei.value.status == he.HE_EBUSY
    t = he.he_server_submit(srv2, j_small["ctx"].h, j_small["plan"].h, j_small["d_ct"], j_small["d_w"], j_small["out"])
    he.he_server_wait(srv2, t)
    assert_equal_u64(he.to_numpy_u64(j_small["out"]), oracle_out(j_small), "small job under a tiny cap")
    assert he.he_server_stats(srv2)["rejected"] == 1
    he.he_server_destroy(srv)
    he.he_server_destroy(srv2)


@pytest.mark.gpu
def test_session_residency_accounting(gpu_lib, ctxs):
    he = gpu_lib
    mix, jobs = _mix_jobs(he, ctxs, 12, 800)
    srv = he.he_server_create(mem_cap_bytes=8 << 30, slots=2, session_jobs=6)
    tickets = []
    for k, j in enumerate(jobs[:6]):            # one 6-layer step: transformed inputs stay resident
        tickets.append(he.he_server_submit(srv, j["ctx"].h, j["plan"].h, j["d_ct"], j["d_w"], j["out"],
                                           session=1, submit_flags=he.HE_SERVE_KEEP_RESIDENT))
    for t in tickets[:5]:
        he.he_server_wait(srv, t)
    he.he_server_wait(srv, tickets[5])
    he.he_server_drain(srv)
    # the session closed after its sixth job: nothing is left resident
    assert he.he_server_stats(srv)["in_use_bytes"] == 0
    # a session still open keeps its blocks
    for j in jobs[6:9]:
        t = he.he_server_submit(srv, j["ctx"].h, j["plan"].h, j["d_ct"], j["d_w"], j["out"], session=2,
                                submit_flags=he.HE_SERVE_KEEP_RESIDENT)
        he.he_server_wait(srv, t)
    assert he.he_server_stats(srv)["in_use_bytes"] > 0
    for k, j in enumerate(jobs[:9]):
        assert_equal_u64(he.to_numpy_u64(j["out"]), oracle_out(j), "session job %d" % k)
    he.he_server_destroy(srv)
