#!/usr/bin/env python3
"""Benchmark: CPMul-accumulates per second of the correlation-aware conv layer on one MI355X.

Workload (one step): the server side of one conv2d forward layer -- batch 16 of
3x32x32 integer activations packed with pi_x and encrypted, 16 output channels,
3x3 kernel, stride 1, pad 1, int8 weights packed with pi_w; ring degree 8192,
3 primes (48-bit); 256 CPMul-accumulates producing 256 output ciphertexts.
Every step transforms the 16 input ciphertexts, packs and transforms the 16
weight polynomials, multiply-accumulates and inverse-transforms the outputs.

Prints one JSON line.  `value` is the whole-job CPMul-accumulate rate of the
batched path -- the persistent fused kernel replayed from a HIP graph, running
several independent instances of the layer (each its own encrypted input batch
and weights, all resident in HBM) per launch, exactly --steps layer steps in
the timed region -- next to the plain per-layer path (separate transform,
multiply-accumulate and inverse kernels) and the fused per-layer path on the
same MI355X.  Also reported: transforms per second, the roofline of the
dominant kernel (timed with HIP events the library records on its launch
stream around the kernel, on direct launches of the same jobs right after the
timed region), serving latency, and the CPU oracle timed on the host cores.
The default of 1024 steps (64 launches, about 60 ms) times the path at the
clocks it holds under sustained load; the first tens of milliseconds run
slower.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CPMul-accumulates/s at N=8192,L=3 (batched vs plain); p50/p99 job latency"
PEAK_HBM_GBS = 8000.0
# fp64 and 32-bit integer VALU issue rate: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12
# minimal VALU instruction counts of the exact fp64 arithmetic: 6 per modular
# product, 2 more per butterfly (sum and difference), 8 per multiply-accumulate
# term (product with its quotient companion formed, plus the add)
OPS_MODMUL = 6          # mul, fma, mul, rndne, fma, add
OPS_BFLY = OPS_MODMUL + 2
OPS_MAC_TERM = OPS_MODMUL + 2   # quotient companion mul + accumulate add


def kernel_src_sha(d=None):
    """Digest of the sources that decide the persistent launch's memory traffic:
    the device code (the .hip kernels and the .hpp headers they include) and
    batch.cpp, which lays out the launch's task queues, with comments and
    blank lines left out (an edit of a comment changes no kernel).  Hardware
    byte counts below are reported only for the code they were taken on."""
    import hashlib
    import re
    d = d or os.path.join(ROOT, "paper_2409_16675_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(x for x in os.listdir(d) if x.endswith((".hip", ".hpp")) or x == "batch.cpp"):
        h.update(f.encode())
        with open(os.path.join(d, f), encoding="utf-8") as fh:
            code = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        code = "\n".join(ln.rstrip() for ln in (re.sub(r"//.*", "", x) for x in code.split("\n")) if ln.strip())
        h.update(code.encode())
    return h.hexdigest()[:16]


# HBM bytes per persistent launch from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE
# passes over this benchmark (summaries under profiles/), each counter scaled by
# what it reads for a plain 512 MiB device copy in the same run; keyed by the
# digest of the sources the counters were taken on.
TRAFFIC = {
    # (source digest, layer jobs per launch): bytes per launch, with the counter readings
    ("d7a3e8df84b35f2d", 20): {"bytes": 2544792941, "fetch_kib": 166697.5, "fetch_scale": 1.9999,
                               "write_kib": 2151773.8, "write_scale": 1.0000,
                               "summary": "profiles/k_persistent_conv2d_fwd_b16_n8192_L3_x20_hbm_bytes.md"},
    ("d7a3e8df84b35f2d", 16): {"bytes": 2032754129, "fetch_kib": 131821.4, "fetch_scale": 1.9999,
                               "write_kib": 1721484.3, "write_scale": 1.0000,
                               "summary": "profiles/k_persistent_conv2d_fwd_b16_n8192_L3_x16_hbm_bytes.md"},
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1024)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--jobs-per-launch", type=int, default=16,
                    help="preferred layer jobs (steps) per persistent launch of the batched path (see launch_sizes)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the weight-gradient, uneven-mix and 60-bit legs")
    ap.add_argument("--preheat-ms", type=float, default=150.0,
                    help="untimed launches before a timed region continue until the GPU has run this long")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 512 MiB device copy (reference for hardware byte counters)")
    ap.add_argument("--cpu-only", action="store_true", help=argparse.SUPPRESS)
    return ap.parse_args()


def workload(he, synth, torch, n_layers=1, bits=48):
    """The conv layer, `n_layers` independent instances of it (input batch and
    weights drawn from their own seeded streams), inputs encrypted on the device."""
    N, L, B, C, M, H, W, h, P = 8192, 3, 16, 3, 16, 32, 32, 3, 1
    import numpy as np
    ctx = he.Context(N, L, prime_bits=bits)
    plan = he.Plan(ctx, he.HE_KIND_CONV, B=B, C=C, M=M, H=H, W=W, h=h, P=P)
    info = plan.info
    s = synth.ternary(synth.rng(2, synth.STREAM_SK), N)
    ds = torch.from_numpy(s.astype(np.int8)).cuda()
    layers = []
    for j in range(n_layers):
        x = synth.int8_uniform(synth.rng(2, synth.STREAM_ACT, j), (B, C, H, W))
        w = synth.int8_uniform(synth.rng(2, synth.STREAM_PT, j), (M, C, h, h))
        polys = he.he_pack_input(plan.h, x.reshape(-1), B * info["cb"] * N).reshape(-1, N)
        # encrypt on the device with the library (client side, outside the timed region)
        ga, ge = synth.rng(2, synth.STREAM_A, j), synth.rng(2, synth.STREAM_E, j)
        ct_in = he.empty_u64((polys.shape[0], 2, L, N))
        for k in range(polys.shape[0]):
            a = he.to_device_u64(synth.uniform_residues(ga, (), ctx.q, N))
            e = torch.from_numpy(synth.small_error(ge, N).astype(np.int32)).cuda()
            m = torch.from_numpy(np.remainder(polys[k], synth.T_PLAIN).astype(np.int64)).cuda()
            he.he_encrypt(ctx.h, ds, m, a, e, ct_in[k])
        dw = torch.from_numpy(w.astype(np.int32).reshape(-1)).cuda()
        layers.append(dict(ct_in=ct_in, w=dw, x=x, wh=w))
    return dict(ctx=ctx, plan=plan, info=info, ct_in=layers[0]["ct_in"], w=layers[0]["w"], x=layers[0]["x"],
                wh=layers[0]["wh"], layers=layers, N=N, L=L,
                config=dict(workload="conv2d forward, batch 16 x 3x32x32 -> 16 channels, 3x3 kernel, stride 1, pad 1; "
                                     "N=8192, 3 primes of %d bits, t=65537; 256 CPMul-accumulates per step" % bits,
                            batch=B, in_channels=C, out_channels=M, map=[H, W], kernel=h, pad=P, N=N, L=L,
                            cpmul_per_step=info["n_terms"]))


def time_path(he, torch, wl, flags, steps, warmup, profile=False, preheat_ms=0.0):
    """The per-layer path (fused kernels, or with HE_UNFUSED separate ones),
    one layer per step; untimed steps first as for the batched path."""
    ctx, plan = wl["ctx"], wl["plan"]
    out = he.empty_u64((wl["info"]["n_ct_out"], 2, wl["L"], wl["N"]))
    ws = he.workspace(plan.workspace_size(flags))
    stream = torch.cuda.current_stream()

    def step():
        he.he_corr_conv2d(ctx.h, plan.h, wl["ct_in"], wl["w"], out, flags, ws, ws.numel(), stream)

    t0, n = time.perf_counter(), 0
    while n < warmup or (time.perf_counter() - t0) * 1e3 < preheat_ms:
        step()
        n += 1
        if n % 16 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    if profile:
        he.he_ctx_profile(ctx.h, True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = None
    if profile:
        he.he_ctx_profile(ctx.h, False)
        stats = he.he_ctx_profile_read(ctx.h)
    return (t1 - t0) / steps, stats, out


MOST_JOBS_PER_LAUNCH = 24


def launch_sizes(steps, per_launch):
    """Launches covering `steps` steps, their sizes within one of each other: as
    many as steps / per_launch rounds to (at least one), and more only where a
    launch would exceed MOST_JOBS_PER_LAUNCH jobs (at 16 per launch: 20 steps
    run as one launch of 20, 64 as four of 16).  Per job the persistent kernel
    is fastest near 16 jobs a launch and slower both well below and well above
    (one box: 48.9 / 47.3 / 46.4 / 45.9 / 47.0 us per job at 8 / 10 / 12 / 16 / 20)."""
    n = max(1, int(steps / max(1, per_launch) + 0.5), -(-steps // MOST_JOBS_PER_LAUNCH))
    base, extra = divmod(steps, n)
    return [base + 1] * extra + [base] * (n - extra)


def kernel_us(he, b, stream, launches):
    """Average duration of the persistent kernel alone over `launches` direct
    launches of batch `b` (built with HE_BATCH_PROFILE): HIP events the library
    records on the launch stream around the kernel, read at most 64 runs apart."""
    he.he_batch_run(b, stream)                 # first launch untimed
    he.he_batch_sync(b, stream)
    k0 = he.he_batch_get_info(b)
    left = launches
    while left > 0:
        c = min(64, left)
        for _ in range(c):
            he.he_batch_run(b, stream)
        he.he_batch_sync(b, stream)
        left -= c
    k1 = he.he_batch_get_info(b)
    return (k1["kernel_ms"] - k0["kernel_ms"]) / (k1["kernel_launches"] - k0["kernel_launches"]) * 1e3


def preheat(he, b, stream, warmup, min_ms):
    """`warmup` untimed launches, then more until the GPU has run the batch for
    at least `min_ms` (its clocks settle over the first tens of milliseconds of
    sustained load).  Returns the number of launches."""
    t0, n = time.perf_counter(), 0
    while n < warmup or (time.perf_counter() - t0) * 1e3 < min_ms:
        he.he_batch_run(b, stream)
        n += 1
        if n % 16 == 0:
            he.he_batch_sync(b, stream)
    he.he_batch_sync(b, stream)
    return n


def time_batched(he, torch, wl, steps, warmup, per_launch, preheat_ms):
    """The persistent fused kernel, replayed from a HIP graph, over exactly
    `steps` layer jobs (steps) split into launches by launch_sizes.  Returns seconds per
    step, the kernel's average duration per full-size launch, the outputs of
    the first launch's jobs, the batch and its info."""
    ctx, plan = wl["ctx"], wl["plan"]
    stream = torch.cuda.current_stream()

    def make(n, flags=he.HE_BATCH_GRAPH):
        b = he.he_batch_create(0)
        outs = []
        for j in range(n):
            lay = wl["layers"][j % len(wl["layers"])]
            out = he.empty_u64((wl["info"]["n_ct_out"], 2, wl["L"], wl["N"]))
            he.he_batch_add(b, ctx.h, plan.h, lay["ct_in"], lay["w"], out, 0)
            outs.append(out)
        he.he_batch_build(b, flags)
        return b, outs

    sizes = launch_sizes(steps, per_launch)
    b, outs = make(sizes[0])
    small = make(sizes[-1])[0] if sizes[-1] != sizes[0] else None
    prof, _ = make(sizes[0], he.HE_BATCH_PROFILE)
    n_pre = preheat(he, b, stream, warmup, preheat_ms)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in sizes]
    t0 = time.perf_counter()
    for n, (a, z) in zip(sizes, ev):
        a.record(stream)
        he.he_batch_run(b if n == sizes[0] else small, stream)
        z.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    he.he_batch_sync(b, stream)
    launch_ms = [a.elapsed_time(z) for (a, z), n in zip(ev, sizes) if n == sizes[0]]
    info = he.he_batch_get_info(b)
    if small:
        he.he_batch_sync(small, stream)
        he.he_batch_destroy(small)
    # the persistent kernel alone, on direct launches of the same jobs
    kern = kernel_us(he, prof, stream, max(16, len(sizes)))
    he.he_batch_destroy(prof)
    info["graph_launch_ms"] = sum(launch_ms) / len(launch_ms)
    info["launch_sizes"] = sizes
    info["preheat_launches"] = n_pre
    return (t1 - t0) / steps, kern / 1e3, outs, b, info


def alg_work(specs):
    """Algorithmic VALU operations and HBM bytes of a set of layer jobs run
    once: forward transforms of inputs and plaintexts, the multiply-accumulate
    terms and the inverse transforms of outputs (8 per butterfly, 8 per term
    and coefficient, 6 per folded N^-1 product), and bytes of the inputs,
    plaintexts and outputs read or written once.  specs: dicts with N, L, the
    plan info, whether inputs come transformed, and the plaintext bytes."""
    ops = bytes_ = 0
    for sp in specs:
        N, L, inf = sp["N"], sp["L"], sp["info"]
        bfly = (N // 2) * (N.bit_length() - 1)
        fwd = inf["n_pt"] * L + (0 if sp.get("in_ntt") else inf["n_ct_in"] * 2 * L)
        inv = inf["n_ct_out"] * 2 * L
        ops += fwd * bfly * OPS_BFLY + inv * (bfly * OPS_BFLY + (N // 2) * OPS_MODMUL) \
            + inf["n_terms"] * 2 * L * N * OPS_MAC_TERM
        bytes_ += 8 * N * (inf["n_ct_in"] * 2 * L + inf["n_ct_out"] * 2 * L) + sp["plain_bytes"]
    return ops, bytes_


def roofline_of(ops, bytes_, kern_s, what):
    alu = ops / kern_s / 1e12
    hbm = bytes_ / kern_s / 1e9
    return {"bound": "alu", "achieved": round(alu, 3), "peak": round(PEAK_VALU_TOPS, 3), "unit": "T VALU-op/s",
            "frac": round(alu / PEAK_VALU_TOPS, 4), "kernel": what, "kernel_avg_us": round(kern_s * 1e6, 2),
            "ops_per_launch": int(ops), "alg_bytes_per_launch": int(bytes_), "hbm_achieved_GBs": round(hbm, 1),
            "hbm_frac": round(hbm / PEAK_HBM_GBS, 4)}


def time_job_set(he, torch, jobs, reps, warmup, preheat_ms, per_layer=True):
    """A set of layer jobs (ctx, plan, ct_in, plain, out, flags, spec): one
    persistent launch per step, replayed from a HIP graph (`reps` steps timed
    after a pre-heat), the kernel alone on direct launches, and -- with
    per_layer -- the same jobs one after another through the fused and the
    plain (unfused) per-layer kernels.  Outputs of all three paths are
    compared byte for byte."""
    stream = torch.cuda.current_stream()

    def make(flags):
        b = he.he_batch_create(0)
        for ctx, plan, ct, pl, out, f, _ in jobs:
            he.he_batch_add(b, ctx.h, plan.h, ct, pl, out, f)
        he.he_batch_build(b, flags)
        return b

    b, prof = make(he.HE_BATCH_GRAPH), make(he.HE_BATCH_PROFILE)
    n_pre = preheat(he, b, stream, warmup, preheat_ms)
    t0 = time.perf_counter()
    for _ in range(reps):
        he.he_batch_run(b, stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    he.he_batch_sync(b, stream)
    info = he.he_batch_get_info(b)
    kern = kernel_us(he, prof, stream, max(16, reps))
    batched_out = [j[4].clone() for j in jobs]
    he.he_batch_destroy(prof)
    he.he_batch_destroy(b)
    res = {"batched_ms_per_step": round(dt * 1e3, 4), "kernel_us": round(kern, 2), "jobs": len(jobs),
           "cpmul_per_step": int(info["cpmul"]), "batched_cpmul_per_s": round(info["cpmul"] / dt, 1),
           "fwd_planes": int(info["fwd_planes"]), "inv_planes": int(info["inv_planes"]), "preheat_launches": n_pre}
    if per_layer:
        wss = [he.workspace(plan.workspace_size(f | he.HE_UNFUSED)) for _, plan, _, _, _, f, _ in jobs]
        same = True
        for name, extra in (("fused", 0), ("plain", he.HE_UNFUSED)):
            def step():
                for (ctx, plan, ct, pl, out, f, _), ws in zip(jobs, wss):
                    he.he_corr_conv2d(ctx.h, plan.h, ct, pl, out, f | extra, ws, ws.numel(), stream)
            for _ in range(warmup):
                step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                step()
            torch.cuda.synchronize()
            d = (time.perf_counter() - t0) / reps
            res[name + "_ms_per_step"] = round(d * 1e3, 4)
            res[name + "_cpmul_per_s"] = round(info["cpmul"] / d, 1)
            same = same and all(torch.equal(j[4].view(torch.int64), o.view(torch.int64)) for j, o in zip(jobs, batched_out))
        res["batched_equals_fused_equals_plain"] = bool(same)
    ops, bytes_ = alg_work([j[6] for j in jobs])
    res["roofline"] = roofline_of(ops, bytes_, kern * 1e-6, "k_persistent (%d jobs per launch)" % len(jobs))
    return res


def weight_gradient_leg(he, torch, synth, reps, warmup, preheat_ms):
    """The weight-gradient workload: batch 32, 16 -> 16 channels, 16x16 maps,
    3x3 kernel, pad 1, N = 8192, 3 primes; ciphertexts uniform mod q_i and
    plaintext polynomials uniform mod t (the masked shares of Section 3.2),
    CryptoTrain-P terms [X](dY - r) + [dY](X - r): 2048 CPMul into 32 outputs."""
    import numpy as np
    N, L, B, C, M, H, h, P = 8192, 3, 32, 16, 16, 16, 3, 1
    ctx = he.Context(N, L)
    plan = he.Plan(ctx, he.HE_KIND_DW, B=B, C=C, M=M, H=H, W=H, h=h, P=P)
    info = plan.info
    ct = he.to_device_u64(synth.uniform_residues(synth.rng(3, synth.STREAM_CT), (info["n_ct_in"], 2), ctx.q, N))
    pt = torch.from_numpy(synth.uniform_mod_t(synth.rng(3, synth.STREAM_MASK), (info["n_pt"], N))).cuda()
    out = he.empty_u64((info["n_ct_out"], 2, L, N))
    spec = dict(N=N, L=L, info=info, plain_bytes=info["n_pt"] * N * 8)
    res = time_job_set(he, torch, [(ctx, plan, ct, pt, out, he.HE_PLAIN_POLY, spec)], reps, warmup, preheat_ms)
    res["workload"] = ("conv2d weight gradient, batch 32, 16 -> 16 channels, 16x16 maps, 3x3 kernel, pad 1; "
                       "N=8192, 3 primes of 48 bits; CryptoTrain-P terms, %d CPMul-accumulates" % info["n_terms"])
    return res


def mix_leg(he, torch, synth, reps, warmup, preheat_ms, n_jobs=64):
    """The uneven mix: 64 jobs drawn over {conv 3->16 @32x32, 16->32 @16x16,
    32->64 @8x8, FC 256->10, FC 1024->256} x {(4096, 2), (8192, 3), (16384, 4)},
    batch 1, ciphertexts uniform mod q_i, int8 weights, all in one persistent
    launch (the mixed-degree variant) replayed from a HIP graph."""
    import numpy as np
    ctxs = {(N, L): he.Context(N, L) for N, L in synth.MIX_RINGS}
    jobs = []
    for k, (lay, ring) in enumerate(synth.job_mix(n_jobs)):
        N, L = synth.MIX_RINGS[ring]
        ctx = ctxs[(N, L)]
        spec = synth.MIX_LAYERS[lay]
        gw = synth.rng(4, synth.STREAM_PT, k)
        if spec[0] == "conv":
            _, C, M, H, W, h, P = spec
            plan = he.Plan(ctx, he.HE_KIND_CONV, B=1, C=C, M=M, H=H, W=W, h=h, P=P)
            w = synth.int8_uniform(gw, (M, C, h, h))
        else:
            _, n_in, n_out = spec
            plan = he.Plan(ctx, he.HE_KIND_FC, B=1, n_in=n_in, n_out=n_out)
            w = synth.int8_uniform(gw, (n_out, n_in))
        info = plan.info
        ct = he.to_device_u64(synth.uniform_residues(synth.rng(4, synth.STREAM_CT, k), (info["n_ct_in"], 2), ctx.q, N))
        out = he.empty_u64((info["n_ct_out"], 2, L, N))
        jobs.append((ctx, plan, ct, torch.from_numpy(w.astype(np.int32).reshape(-1)).cuda(), out, 0,
                     dict(N=N, L=L, info=info, plain_bytes=w.size * 4)))
    res = time_job_set(he, torch, jobs, reps, warmup, preheat_ms)
    res["workload"] = "uneven mix of %d layer jobs over N = 4096 / 8192 / 16384 (2 / 3 / 4 primes of 48 bits)" % n_jobs
    return res


def wide_prime_leg(he, torch, synth, reps, warmup, preheat_ms, jobs_per_launch=16):
    """The conv-forward workload with three 60-bit primes (64-bit integer
    arithmetic throughout): `jobs_per_launch` instances in one persistent launch."""
    wl = workload(he, synth, torch, n_layers=jobs_per_launch, bits=60)
    jobs = [(wl["ctx"], wl["plan"], lay["ct_in"], lay["w"], he.empty_u64((wl["info"]["n_ct_out"], 2, wl["L"], wl["N"])),
             0, dict(N=wl["N"], L=wl["L"], info=wl["info"], plain_bytes=lay["w"].numel() * 4)) for lay in wl["layers"]]
    res = time_job_set(he, torch, jobs, reps, warmup, preheat_ms)
    res["workload"] = wl["config"]["workload"]
    res["arith"] = "u64" if wl["ctx"].arith == he.HE_ARITH_U64 else "f64"
    return res


def time_seeded(he, torch, wl, steps, warmup):
    """The fused per-layer path with input component 1 regenerated from a seed
    (only c0 resident; Section 7, Discussion).  Returns seconds per step and whether the
    output equals the same layer on the expanded ciphertexts."""
    ctx, plan, info = wl["ctx"], wl["plan"], wl["info"]
    seed = (0x5EED, 0xC1)
    c0 = wl["ct_in"][:, 0].contiguous()
    c1 = he.empty_u64((info["n_ct_in"], wl["L"], wl["N"]))
    he.he_expand_c1(ctx.h, seed, 0, info["n_ct_in"], c1)
    full = torch.stack([c0, c1], dim=1).contiguous()
    out = he.empty_u64((info["n_ct_out"], 2, wl["L"], wl["N"]))
    ref = he.empty_u64(tuple(out.shape))
    ws = he.workspace(plan.workspace_size(0))
    stream = torch.cuda.current_stream()
    he.he_corr_conv2d(ctx.h, plan.h, full, wl["w"], ref, 0, ws, ws.numel(), stream)
    for _ in range(warmup):
        he.he_corr_conv2d_seeded(ctx.h, plan.h, c0, seed, wl["w"], out, 0, ws, ws.numel(), stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        he.he_corr_conv2d_seeded(ctx.h, plan.h, c0, seed, wl["w"], out, 0, ws, ws.numel(), stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return dt, bool(torch.equal(out.view(torch.int64), ref.view(torch.int64)))


def time_ppmul(he, torch, wl, steps, warmup):
    """The server's plaintext product of the online protocol (Section 3.2) for the
    same layer: masked input polynomials (16) times masked weight polynomials (16)
    over Z_t[X]/(X^N+1), 256 outputs.  Returns seconds per layer."""
    import numpy as np
    ctx, plan, info, N = wl["ctx"], wl["plan"], wl["info"], wl["N"]
    from paper_2409_16675_amd import synth
    g = synth.rng(2, synth.STREAM_MASK)
    t = ctx.t
    a = he.to_device_u64(g.integers(0, t, size=(info["n_ct_in"], N), dtype=np.uint64))
    b = he.to_device_u64(g.integers(0, t, size=(info["n_pt"], N), dtype=np.uint64))
    out = he.empty_u64((info["n_ct_out"], N))
    he.he_ctx_prepare(ctx.h, he.HE_PREPARE_PPMUL)
    ws = he.workspace(he.he_ppmul_ws_size(plan.h, 0))
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        he.he_ppmul(ctx.h, plan.h, a, b, out, 0, ws, ws.numel(), stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        he.he_ppmul(ctx.h, plan.h, a, b, out, 0, ws, ws.numel(), stream)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def time_ccmul(he, torch, wl, steps, warmup):
    """The preprocessing product of CryptoTrain-P (Section 3.2) for the same layer:
    [r_x r_w] for its 256 outputs, each the relinearized product of one of the 16
    input-side by one of the 16 weight-side mask ciphertexts (the plan's term
    lists).  Ciphertexts and key are uniform residues of the right shapes (the
    work does not depend on their values; the tests check the arithmetic).
    Returns seconds per layer and the per-kernel-kind profile of one call."""
    import numpy as np
    from paper_2409_16675_amd import synth
    ctx, plan, info, N, L = wl["ctx"], wl["plan"], wl["info"], wl["N"], wl["L"]
    row, cti, pti = he.he_plan_terms(plan.h)
    g = synth.rng(2, synth.STREAM_MASK, 1)
    a = he.to_device_u64(synth.uniform_residues(g, (info["n_ct_in"], 2), ctx.q, N))
    b = he.to_device_u64(synth.uniform_residues(g, (info["n_pt"], 2), ctx.q, N))
    rlk = he.to_device_u64(synth.uniform_residues(g, (L, 2), ctx.q, N))
    n_out = info["n_ct_out"]
    out = he.empty_u64((n_out, 2, L, N))
    he.he_ctx_prepare(ctx.h, he.HE_PREPARE_CCMUL, n_out, len(cti))
    ws = he.workspace(he.he_ccmul_ws_size(ctx.h, info["n_ct_in"], info["n_pt"], n_out, len(cti), 0))
    stream = torch.cuda.current_stream()

    def call():
        he.he_ccmul(ctx.h, a, info["n_ct_in"], b, info["n_pt"], row, cti, pti, n_out, rlk, out, 0, ws, ws.numel(),
                    stream)

    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    he.he_ctx_profile(ctx.h, True)
    call()
    torch.cuda.synchronize()
    he.he_ctx_profile(ctx.h, False)
    prof = he.he_ctx_profile_read(ctx.h)
    return dt, n_out, {k: dict(launches=v["launches"], total_us=round(v["total_ms"] * 1e3, 1)) for k, v in prof.items()}


def ntt_rate(he, torch, wl, iters=20):
    ctx = wl["ctx"]
    n_polys = 512
    d = he.empty_u64((n_polys, wl["L"], wl["N"]))
    d.view(torch.int64).zero_()
    for _ in range(3):
        he.he_ntt_fwd(ctx.h, d, n_polys)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        he.he_ntt_fwd(ctx.h, d, n_polys)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / iters
    return n_polys * wl["L"] / dt


def roofline(wl, stats):
    """Roofline of the dominant kernel: the fused multiply-accumulate + inverse transform."""
    info, N, L = wl["info"], wl["N"], wl["L"]
    k = stats["mac_inv"]
    avg_s = k["total_ms"] / k["launches"] / 1e3
    planes = info["n_ct_out"] * 2 * L
    terms_per_plane = info["n_terms"] / info["n_ct_out"]
    logn = N.bit_length() - 1
    ops = planes * (terms_per_plane * N * OPS_MAC_TERM + (N // 2) * logn * OPS_BFLY + (N // 2) * OPS_MODMUL)
    bytes_ = 8 * N * (info["n_ct_in"] * 2 * L + info["n_pt"] * L + planes)
    alu = ops / avg_s / 1e12
    hbm = bytes_ / avg_s / 1e9
    return {"bound": "alu", "achieved": round(alu, 3), "peak": round(PEAK_VALU_TOPS, 3), "unit": "T VALU-op/s",
            "frac": round(alu / PEAK_VALU_TOPS, 4), "traffic": None, "kernel": "k_mac_inv (fused MAC + inverse NTT)",
            "kernel_avg_us": round(avg_s * 1e6, 2), "ops_per_launch": int(ops), "alg_bytes_per_launch": int(bytes_),
            "hbm_achieved_GBs": round(hbm, 1), "hbm_frac": round(hbm / PEAK_HBM_GBS, 4)}


def roofline_persistent(wl, kern_ms, binfo):
    """Roofline of the persistent kernel, which runs whole steps: forward transforms of
    inputs and packed plaintexts, multiply-accumulate, inverse transforms, for every
    job of the launch."""
    info, N, L = wl["info"], wl["N"], wl["L"]
    nj = binfo["n_jobs"]
    logn = N.bit_length() - 1
    avg_s = kern_ms / 1e3
    bfly = (N // 2) * logn
    ops = (binfo["fwd_planes"] * bfly * OPS_BFLY
           + binfo["inv_planes"] * (bfly * OPS_BFLY + (N // 2) * OPS_MODMUL)
           + nj * info["n_terms"] * 2 * L * N * OPS_MAC_TERM)
    bytes_ = nj * (8 * N * (info["n_ct_in"] * 2 * L + info["n_ct_out"] * 2 * L) + 4 * 16 * 3 * 9)
    alu = ops / avg_s / 1e12
    hbm = bytes_ / avg_s / 1e9
    tr = TRAFFIC.get((kernel_src_sha(), nj))
    return {"bound": "alu", "achieved": round(alu, 3), "peak": round(PEAK_VALU_TOPS, 3), "unit": "T VALU-op/s",
            "frac": round(alu / PEAK_VALU_TOPS, 4), "traffic": tr["bytes"] if tr else None,
            "traffic_detail": tr,
            "kernel": "k_persistent (%d whole steps per launch: transforms, packing, MAC, inverse transforms)" % nj,
            "kernel_avg_us": round(avg_s * 1e6, 2), "ops_per_launch": int(ops), "alg_bytes_per_launch": int(bytes_),
            "hbm_achieved_GBs": round(hbm, 1), "hbm_frac": round(hbm / PEAK_HBM_GBS, 4),
            "graph_replay_avg_us": round(binfo["graph_launch_ms"] * 1e3, 2)}


def serving(he, torch, synth, n_jobs=20000, rate=2000.0, copies=4, sweep=(20000.0, 100000.0), sweep_jobs=4000,
            reuse_jobs=6000):
    """Poisson arrivals (mean `rate` jobs/s) of jobs drawn from the uneven layer
    mix, sessions of 6 jobs keeping their transformed inputs resident, 64 GB
    admission cap, continuous batching against the sequential per-layer server
    on the same trace; each server is warmed by a burst of jobs and then
    measured on the trace (latency from each job's scheduled arrival to its
    completion seen by the server).  Then the same at the higher arrival rates
    of `sweep`, and a training-step trace whose sessions are three pairs of
    jobs on the same input ciphertexts (the second of each pair with other
    weights, HE_IN_RESIDENT), with and without reuse of the kept transforms."""
    import numpy as np
    ctxs = {(N, L): he.Context(N, L) for N, L in synth.MIX_RINGS}
    kinds = {}
    for li, spec in enumerate(synth.MIX_LAYERS):
        for ri, (N, L) in enumerate(synth.MIX_RINGS):
            ctx = ctxs[(N, L)]
            if spec[0] == "conv":
                _, C, M, H, W, h, P = spec
                plan = he.Plan(ctx, he.HE_KIND_CONV, B=1, C=C, M=M, H=H, W=W, h=h, P=P)
                ws = [synth.int8_uniform(synth.rng(5, synth.STREAM_PT, 10 * li + k), (M, C, h, h)) for k in range(2)]
            else:
                _, n_in, n_out = spec
                plan = he.Plan(ctx, he.HE_KIND_FC, B=1, n_in=n_in, n_out=n_out)
                ws = [synth.int8_uniform(synth.rng(5, synth.STREAM_PT, 10 * li + k), (n_out, n_in)) for k in range(2)]
            info = plan.info
            g = synth.rng(5, synth.STREAM_CT, 10 * li + ri)
            bufs = [(he.to_device_u64(synth.uniform_residues(g, (info["n_ct_in"], 2), ctx.q, N)),
                     he.empty_u64((info["n_ct_out"], 2, L, N)), he.empty_u64((info["n_ct_out"], 2, L, N)))
                    for _ in range(copies)]
            kinds[(li, ri)] = dict(ctx=ctx, plan=plan, bufs=bufs, cpmul=info["n_terms"],
                                   w=[torch.from_numpy(w.astype(np.int32).reshape(-1)).cuda() for w in ws])
    mix = synth.job_mix(max(n_jobs, reuse_jobs, sweep_jobs), workload=5)
    jobs, twins, ctx_list, cpmul = [], [], [], []
    for k, (li, ri) in enumerate(mix):
        kd = kinds[(li, ri)]
        ct, out, out2 = kd["bufs"][k % copies]
        jobs.append((kd["plan"].h, ct, kd["w"][0], out, 0))
        twins.append((kd["plan"].h, ct, kd["w"][1], out2, he.HE_IN_RESIDENT))
        ctx_list.append(kd["ctx"].h)
        cpmul.append(kd["cpmul"])

    def run(r, n, modes, job_list, ctx_l, cp_l, flags):
        arr = synth.poisson_arrivals(n, r)
        arr = arr - arr[0]
        sessions = np.arange(n, dtype=np.uint64) // 6 + 1
        out = {}
        for name, mode in modes:
            srv = he.he_server_create(mem_cap_bytes=64 << 30, mode=mode, arena_bytes=8 << 30, slots=2,
                                      max_batch_jobs=64, session_jobs=6)
            # warm the kernels, arena and tables of this server with a burst, then measure
            he.he_server_replay(srv, ctx_list[:64], jobs[:64], np.zeros(64))
            st0 = he.he_server_stats(srv)
            t0 = time.perf_counter()
            lat = he.he_server_replay(srv, ctx_l[:n], job_list[:n], arr, sessions, flags)
            wall = time.perf_counter() - t0
            st = he.he_server_stats(srv)
            he.he_server_destroy(srv)
            span = float((arr + lat).max())
            out[name] = {"p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                         "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                         "mean_ms": round(float(lat.mean()) * 1e3, 3),
                         "throughput_jobs_per_s": round(n / span, 1),
                         "cpmul_per_s": round(sum(cp_l[:n]) / span, 1),
                         "epochs": st["epochs"] - st0["epochs"],
                         "single_job_epochs": st["single_epochs"] - st0["single_epochs"],
                         "fwd_planes": st["fwd_planes"] - st0["fwd_planes"],
                         "resident_hits": st["resident_hits"] - st0["resident_hits"],
                         "peak_footprint_GB": round(st["peak_bytes"] / 2 ** 30, 3), "wall_s": round(wall, 3)}
            e = out[name]["epochs"]
            out[name]["mean_jobs_per_epoch"] = round(n / e, 2) if e else 0.0
        return out

    both = (("continuous", he.HE_SERVE_CONTINUOUS), ("sequential", he.HE_SERVE_SEQUENTIAL))
    res = {"rate_jobs_per_s": rate, "jobs": n_jobs, "mix": "uneven 5-layer x 3-ring mix, batch 1",
           "session_jobs": 6, "cap_GB": 64, "server": "warmed by a 64-job burst before each measured trace"}
    res.update(run(rate, n_jobs, both, jobs, ctx_list, cpmul, he.HE_SERVE_KEEP_RESIDENT))
    res["sweep"] = [dict(rate_jobs_per_s=r, jobs=sweep_jobs,
                         **run(r, sweep_jobs, both, jobs, ctx_list, cpmul, he.HE_SERVE_KEEP_RESIDENT)) for r in sweep]
    # training-step sessions: pairs of jobs on the same inputs
    half = reuse_jobs // 2
    step = [j for k in range(half) for j in (jobs[k], twins[k])]
    step_ctx = [c for k in range(half) for c in (ctx_list[k], ctx_list[k])]
    step_cp = [c for k in range(half) for c in (cpmul[k], cpmul[k])]
    no_reuse = [(p, c, w, o, 0) for p, c, w, o, _ in step]
    res["training_step"] = {
        "what": "sessions of 6 = 3 pairs of jobs on the same input ciphertexts, the second with other weights",
        "jobs": reuse_jobs, "rate_jobs_per_s": rate,
        "with_reuse": run(rate, reuse_jobs, both[:1], step, step_ctx, step_cp, he.HE_SERVE_KEEP_RESIDENT)["continuous"],
        "without_reuse": run(rate, reuse_jobs, both[:1], no_reuse, step_ctx, step_cp, 0)["continuous"]}
    return res


def cpu_baseline(wl, he):
    """The oracle (C, one transform per input plane, OpenMP over planes) on the same batch."""
    import numpy as np
    from oracle import core, packing
    ctx, info = wl["ctx"], wl["info"]
    g = packing.ConvGeometry(3, 32, 32, 3, 1, wl["N"])
    ct = he.to_numpy_u64(wl["ct_in"])
    pt = core.lift(packing.pack_conv_weight(wl["wh"], g).reshape(-1, wl["N"]), ctx.q)
    row, cti, pti = packing.conv_terms(16, 16, g.cb)
    reps, t0 = 0, time.perf_counter()
    while True:
        core.csr_cpmul(ct, pt, row, cti, pti, ctx.q, ctx.psi, method=2)
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= 10.0 or reps >= 200:
            break
    return {"value": round(reps * info["n_terms"] / dt, 2), "unit": "CPMul-acc/s", "cores": core.num_threads(),
            "kind": "oracle", "sample": "the full step (256 CPMul-accumulates, batch 16) repeated %d times, %.1f s"
            % (reps, dt)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (--gpus %d refused)" % args.gpus,
              file=sys.stderr)
        return 2
    import torch
    from paper_2409_16675_amd import he, synth
    # as many distinct layers as the largest launch holds jobs: no two jobs of a
    # launch share inputs
    wl = workload(he, synth, torch, n_layers=max(launch_sizes(args.steps, args.jobs_per_launch)))
    n_cpmul = wl["info"]["n_terms"]
    tune = he.he_autotune(wl["ctx"].h, 512)      # set-up: picks the fastest bit-exact schedules
    chosen = {name: he.he_ctx_get_schedule(wl["ctx"].h, op) for name, op in
              (("fwd", he.HE_OP_FWD), ("inv", he.HE_OP_INV), ("mac", he.HE_OP_MAC))}
    plain_dt, _, out_plain = time_path(he, torch, wl, he.HE_UNFUSED, max(5, args.steps // 2), args.warmup,
                                       preheat_ms=args.preheat_ms)
    fused_dt, stats, out_fused = time_path(he, torch, wl, 0, max(5, args.steps // 2), args.warmup, profile=True,
                                           preheat_ms=args.preheat_ms)
    dt, kern_ms, outs, batch, binfo = time_batched(he, torch, wl, args.steps, args.warmup, args.jobs_per_launch,
                                                   args.preheat_ms)
    same = bool(torch.equal(outs[0].view(torch.int64), out_plain.view(torch.int64)) and
                torch.equal(out_fused.view(torch.int64), out_plain.view(torch.int64)))
    # every other job of the launch against the fused per-layer path on its own layer
    ws = he.workspace(wl["plan"].workspace_size(0))
    ref = he.empty_u64(tuple(outs[0].shape))
    for j in range(1, len(outs)):
        lay = wl["layers"][j]
        he.he_corr_conv2d(wl["ctx"].h, wl["plan"].h, lay["ct_in"], lay["w"], ref, 0, ws, ws.numel(),
                          torch.cuda.current_stream())
        torch.cuda.synchronize()
        same = same and bool(torch.equal(outs[j].view(torch.int64), ref.view(torch.int64)))
    seeded_dt, seeded_same = time_seeded(he, torch, wl, max(5, args.steps // 2), args.warmup)
    cc_dt, cc_n, cc_prof = time_ccmul(he, torch, wl, max(5, args.steps // 5), min(args.warmup, 3))
    res = {
        "metric": METRIC, "value": round(n_cpmul / dt, 1), "unit": "CPMul-acc/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic", "config": wl["config"],
        "path": "batched (persistent fused kernel, graph replay, launches of about %d layer jobs)" % args.jobs_per_launch,
        "jobs_per_launch": args.jobs_per_launch, "launch_sizes": binfo["launch_sizes"],
        "preheat": {"launches": binfo["preheat_launches"], "min_ms": args.preheat_ms,
                    "what": "untimed launches of the batch before the timed region (at least --warmup, then until "
                            "the GPU has run for min_ms)"},
        "kernel_src_sha": kernel_src_sha(),
        "plain_value": round(n_cpmul / plain_dt, 1), "plain_ms_per_step": round(plain_dt * 1e3, 4),
        "fused_value": round(n_cpmul / fused_dt, 1), "fused_ms_per_step": round(fused_dt * 1e3, 4),
        "batched_equals_fused_equals_plain": same,
        "ntt_per_s": round(ntt_rate(he, torch, wl), 1),
        "ppmul_ms_per_layer": round(time_ppmul(he, torch, wl, max(5, args.steps // 2), args.warmup) * 1e3, 4),
        "seeded_c1": {"fused_ms_per_step": round(seeded_dt * 1e3, 4), "equals_full_ciphertext_layer": seeded_same,
                      "input_bytes_per_step": wl["info"]["n_ct_in"] * wl["L"] * wl["N"] * 8,
                      "input_bytes_per_step_unseeded": wl["info"]["n_ct_in"] * 2 * wl["L"] * wl["N"] * 8},
        "ccmul": {"what": "relinearized ciphertext products [r_x r_w] of the layer's 256 outputs (preprocessing)",
                  "ms_per_layer": round(cc_dt * 1e3, 4), "us_per_product": round(cc_dt * 1e6 / cc_n, 3),
                  "cpmul_us_fused": round(fused_dt * 1e6 / n_cpmul, 3), "cpmul_us_batched": round(dt * 1e6 / n_cpmul, 3),
                  "ratio_to_cpmul_fused": round(cc_dt / fused_dt, 2), "ratio_to_cpmul_batched": round(cc_dt / dt, 2),
                  "kernels_one_call": cc_prof},
        "kernels_fused_path": {k: dict(v, avg_us=round(v["total_ms"] * 1e3 / v["launches"], 2))
                               for k, v in stats.items()},
        "schedules": {k: {"arith": "f64" if v[0] == 1 else "u64", "coeffs_per_thread": 1 << v[1]}
                      for k, v in chosen.items()},
        "autotune_us": ["%s/%s/%d: %.1f%s" % (("fwd", "inv", "mac")[t["op"]], "f64" if t["arith"] == 1 else "u64",
                                              1 << t["loge"], t["us"], "" if t["exact"] else " (mismatch)")
                        for t in tune],
        "roofline": roofline_persistent(wl, kern_ms, binfo),
        "roofline_fused_mac_inv": roofline(wl, stats),
    }
    he.he_batch_destroy(batch)
    if args.calib_copy:
        src = torch.empty(64 << 20, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        res["calib_copy_bytes"] = src.numel() * 8
    if not args.no_legs:
        reps = max(8, min(64, args.steps // 4))
        res["weight_gradient"] = weight_gradient_leg(he, torch, synth, reps, args.warmup, args.preheat_ms)
        res["uneven_mix"] = mix_leg(he, torch, synth, reps, args.warmup, args.preheat_ms)
        res["wide_primes_60bit"] = wide_prime_leg(he, torch, synth, reps, args.warmup, args.preheat_ms,
                                                  args.jobs_per_launch)
    if not args.no_serve:
        res["serving"] = serving(he, torch, synth)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(wl, he)
    print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
