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


def _twin(he, ctxs, layer, ring, seed):
    """A second job on the same input ciphertexts with other weights (the
    masked-weight term of the online protocol reuses [x], Section 3.2)."""
    j = make_job(he, ctxs, layer, ring, seed)
    k = make_job(he, ctxs, layer, ring, seed + 1)
    k["ct"], k["d_ct"] = j["ct"], j["d_ct"]
    return j, k


@pytest.mark.gpu
def test_resident_inputs_are_reused_and_results_unchanged(gpu_lib, ctxs):
    # a session of producer/consumer pairs: the consumer reads the producer's
    # kept transform of the same input buffer; outputs equal the oracle, the
    # consumers transform nothing, and a run without residency agrees byte for byte
    he = gpu_lib
    pairs = [_twin(he, ctxs, lay, ring, 900 + 10 * k) for k, (lay, ring) in enumerate([(0, 1), (4, 0), (1, 2), (2, 1)])]
    srv = he.he_server_create(mem_cap_bytes=8 << 30, slots=2, max_batch_jobs=8)
    # producers together (one persistent epoch), then consumers together
    tickets = [he.he_server_submit(srv, p["ctx"].h, p["plan"].h, p["d_ct"], p["d_w"], p["out"], session=7,
                                   submit_flags=he.HE_SERVE_KEEP_RESIDENT) for p, _ in pairs]
    for t in tickets:
        he.he_server_wait(srv, t)
    st0 = he.he_server_stats(srv)
    tickets = [he.he_server_submit(srv, c["ctx"].h, c["plan"].h, c["d_ct"], c["d_w"], c["out"], flags=he.HE_IN_RESIDENT,
                                   session=7) for _, c in pairs]
    for t in tickets:
        he.he_server_wait(srv, t)
    st = he.he_server_stats(srv)
    assert st["resident_hits"] == len(pairs) and st["resident_misses"] == 0
    # consumers transformed only their plaintexts
    pt_planes = sum(c["info"]["n_pt"] * c["ctx"].L for _, c in pairs)
    assert st["fwd_planes"] - st0["fwd_planes"] == pt_planes
    assert st0["resident_blocks"] == len(pairs)
    he.he_server_close_session(srv, 7)
    he.he_server_drain(srv)
    assert he.he_server_stats(srv)["resident_blocks"] == 0 and he.he_server_stats(srv)["in_use_bytes"] == 0
    he.he_server_destroy(srv)
    for k, (p, c) in enumerate(pairs):
        assert_equal_u64(he.to_numpy_u64(p["out"]), oracle_out(p), "producer %d" % k)
        assert_equal_u64(he.to_numpy_u64(c["out"]), oracle_out(c), "consumer %d (resident input)" % k)
    # the same consumers with no kept transforms (misses) give the same bytes
    srv = he.he_server_create(mem_cap_bytes=8 << 30, slots=2, max_batch_jobs=8)
    outs = [he.empty_u64(tuple(c["out"].shape)) for _, c in pairs]
    tickets = [he.he_server_submit(srv, c["ctx"].h, c["plan"].h, c["d_ct"], c["d_w"], o, flags=he.HE_IN_RESIDENT,
                                   session=8) for (_, c), o in zip(pairs, outs)]
    for t in tickets:
        he.he_server_wait(srv, t)
    st = he.he_server_stats(srv)
    he.he_server_destroy(srv)
    assert st["resident_hits"] == 0 and st["resident_misses"] == len(pairs)
    for k, ((_, c), o) in enumerate(zip(pairs, outs)):
        assert_equal_u64(he.to_numpy_u64(o), he.to_numpy_u64(c["out"]), "consumer %d without residency" % k)


@pytest.mark.gpu
def test_resident_reuse_in_sequential_mode_and_lone_epochs(gpu_lib, ctxs):
    # the per-layer path (sequential server; a lone job in continuous mode) keeps
    # and reads resident transforms too
    he = gpu_lib
    for mode in (he.HE_SERVE_SEQUENTIAL, he.HE_SERVE_CONTINUOUS):
        p, c = _twin(he, ctxs, 1, 1, 950 + mode)
        srv = he.he_server_create(mem_cap_bytes=8 << 30, mode=mode, session_jobs=2)
        he.he_server_wait(srv, he.he_server_submit(srv, p["ctx"].h, p["plan"].h, p["d_ct"], p["d_w"], p["out"],
                                                   session=3, submit_flags=he.HE_SERVE_KEEP_RESIDENT))
        he.he_server_wait(srv, he.he_server_submit(srv, c["ctx"].h, c["plan"].h, c["d_ct"], c["d_w"], c["out"],
                                                   flags=he.HE_IN_RESIDENT, session=3))
        st = he.he_server_stats(srv)
        he.he_server_destroy(srv)
        assert st["resident_hits"] == 1 and st["resident_blocks"] == 0   # the session closed after 2 jobs
        assert_equal_u64(he.to_numpy_u64(p["out"]), oracle_out(p), "mode %d producer" % mode)
        assert_equal_u64(he.to_numpy_u64(c["out"]), oracle_out(c), "mode %d consumer" % mode)


@pytest.mark.gpu
def test_malformed_job_fails_alone(gpu_lib, ctxs):
    # one job of an epoch carries a coefficient equal to its prime (not a
    # residue) and asks for validation: it fails with HE_ERANGE, the others
    # of the same burst complete with the right bytes
    he = gpu_lib
    jobs = [make_job(he, ctxs, lay, 1, 980 + lay) for lay in range(4)]
    bad = make_job(he, ctxs, 0, 1, 990)
    ct = bad["ct"].copy()
    ct[0, 1, 2, 17] = np.uint64(bad["ctx"].q[2])
    d_bad = he.to_device_u64(ct)
    srv = he.he_server_create(mem_cap_bytes=8 << 30, slots=1, max_batch_jobs=8)
    tickets = [he.he_server_submit(srv, j["ctx"].h, j["plan"].h, j["d_ct"], j["d_w"], j["out"], flags=he.HE_VALIDATE)
               for j in jobs[:2]]
    t_bad = he.he_server_submit(srv, bad["ctx"].h, bad["plan"].h, d_bad, bad["d_w"], bad["out"], flags=he.HE_VALIDATE)
    tickets += [he.he_server_submit(srv, j["ctx"].h, j["plan"].h, j["d_ct"], j["d_w"], j["out"]) for j in jobs[2:]]
    with pytest.raises(he.HeError) as ei:
        he.he_server_wait(srv, t_bad)
    assert ei.value.status == he.HE_ERANGE
    for t in tickets:
        he.he_server_wait(srv, t)
    st = he.he_server_stats(srv)
    he.he_server_destroy(srv)
    assert st["failed"] == 1 and st["completed"] == len(jobs) + 1
    for k, j in enumerate(jobs):
        assert_equal_u64(he.to_numpy_u64(j["out"]), oracle_out(j), "job %d beside the malformed one" % k)


@pytest.mark.gpu
def test_kept_blocks_are_evicted_rather_than_blocking_admission(gpu_lib, ctxs):
    # sessions that never close keep their blocks; under a cap that holds one
    # big job at a time the queue still drains, by evicting kept blocks that
    # no running job reads (waits are bounded so a stuck server fails the test)
    he = gpu_lib
    big = [make_job(he, ctxs, 2, 2, 1000 + k) for k in range(4)]   # conv 32 -> 64 @ 8x8 at N = 16384
    # footprint 98 MB (33 MB workspace, kept afterwards, + 1 MB in + 64 MB out):
    # a kept block and the next job (131 MB) exceed the cap
    cap = 128 << 20
    srv = he.he_server_create(mem_cap_bytes=cap, slots=2, arena_bytes=256 << 20, session_jobs=0)
    tickets = [he.he_server_submit(srv, j["ctx"].h, j["plan"].h, j["d_ct"], j["d_w"], j["out"], session=20 + k,
                                   submit_flags=he.HE_SERVE_KEEP_RESIDENT) for k, j in enumerate(big)]
    for t in tickets:
        he.he_server_wait(srv, t, timeout_us=60_000_000)
    st = he.he_server_stats(srv)
    assert st["evictions"] == len(big) - 1 and st["peak_bytes"] <= cap
    for k, j in enumerate(big):
        assert_equal_u64(he.to_numpy_u64(j["out"]), oracle_out(j), "big job %d" % k)
    for k in range(len(big)):
        he.he_server_close_session(srv, 20 + k)
    assert he.he_server_stats(srv)["resident_blocks"] == 0
    he.he_server_destroy(srv)
