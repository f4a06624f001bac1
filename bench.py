#!/usr/bin/env python3
"""Benchmark of the LDGM XOR path on one MI355X.

Headline workload: one large stripe, k = 4096 input blocks x 64 KiB (256 MiB),
n = 4506 coded blocks (10 % overhead), finite max-degree-16 table
(w_1 = 0.02, w_d = 1/(d(d-1))), 225 coded blocks erased (5 %).  A step is
encode (fs_encode) and peeling decode of the result, on resident device
buffers: the decode plan (fs_decode_plan: peeling schedule and replay
program; it reads no payload) runs on a second stream while the encode runs,
then fs_decode_apply replays it on the fresh coded blocks.

value = user bytes per second = (k t encoded + |R| t recovered) / step time.
The JSON line also carries the roofline of the step's longest kernel, the
decode replay (algorithmic bytes (|R| + k) t per launch over its
HIP-event-timed duration, against the 8 TB/s HBM peak), the same for the
encode kernel ((k_touched + n) t), HBM traffic from rocprofv3 counters when
they were taken on the current kernel source, and the CPU oracle timed on
the host.  By default (--workload all) the line also carries the rest of the
metric: 512 batched stripes against the plain loop over them ("batched"),
batched repair and update on 256 resident stripes ("resident"), and the
serving loop's p50/p99 latency on a Poisson mix ("serve"), each workload
run by this script in a child process of its own, the headline first;
--workload large_stripe gives the headline alone.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--workload W]
"""

import argparse
import gc
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
PROFILE_COUNTERS = os.path.join(ROOT, "profiles", "large_stripe_counters.json")
CSRC = os.path.join(ROOT, "paper_1702_07409_amd", "csrc")
# what the traffic counters count: requests that leave the L2 for the data
# fabric, which the Infinity Cache (MALL) may serve without touching HBM
TRAFFIC_KIND = "L2-to-fabric bytes per launch from rocprofv3 request counters (128/64/32-byte reads, " \
               "64/32-byte writes); includes Infinity Cache hits, so it bounds HBM traffic from above"


def kernel_source_hash():
    """Hash of every library source (kernels, launch choices, graph layout):
    counters taken on other sources are not reported."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--workload", default="all",
                    choices=["large_stripe", "batch512", "resident256", "serve", "extend", "simdisk", "precode", "checks",
                             "all"],
                    help="large_stripe: plain one-stripe path alone (the headline line); batch512 / "
                         "resident256: batched plans vs the plain loop; serve: the request loop "
                         "on a Poisson mix; extend: code extension of the large stripe; simdisk: "
                         "disk-failure sweeps; precode: Table 2's set-up with the precode; checks: check "
                         "generation and local-group repair of a lost disk; all: the "
                         "headline line with the others attached")
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-seconds", type=float, default=1.0)
    ap.add_argument("--batch-stripes", type=int, default=512)
    ap.add_argument("--resident-stripes", type=int, default=256)
    ap.add_argument("--reps", type=int, default=20,
                    help="timed repetitions of each batched plan and plain loop (batch512, resident256)")
    ap.add_argument("--mode", choices=["step", "counters"], default="step",
                    help="counters: only K encode launches plus one plain copy of the same "
                         "output size, for rocprofv3 --pmc runs")
    return ap.parse_args()


def counters_run(args, fs, torch, g, x, c, t, decode):
    """Encode and decode launches, then a plain device copy of known size
    (the scale of the traffic counters)."""
    stream = torch.cuda.current_stream()
    for _ in range(max(1, args.steps)):
        fs.fs_encode(g, x, c, t, stream)
    for _ in range(max(1, args.steps)):
        decode()
    src = torch.empty(c.numel(), dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "counters", "encode_launches": max(1, args.steps),
                      "decode_launches": max(1, args.steps),
                      "copy_bytes_each_way": int(src.numel())}), flush=True)


# state the forked oracle workers read: the graph, the schedule and the
# payload arrays (c and the decoded x in shared anonymous maps, so each
# worker writes its own byte columns of the parent's arrays)
_POOL = {}


def _shared_u8(shape):
    import mmap
    import numpy as np
    buf = mmap.mmap(-1, int(shape[0]) * int(shape[1]))
    return np.frombuffer(buf, dtype=np.uint8).reshape(shape)


def _slice_encode(ab):
    from oracle import codec
    a, b = ab
    _POOL["c"][:, a:b] = codec.encode(_POOL["G"], _POOL["x"][:, a:b])
    return b - a


def _slice_replay(ab):
    from oracle import codec
    a, b = ab
    _POOL["xd"][:, a:b] = codec.replay(_POOL["G"], _POOL["c"][:, a:b], _POOL["sched"])
    return b - a


def cpu_baseline(spec, seconds):
    """The oracle on the same stripe, timed on the host's cores.

    Only the payload phases are timed, encode (codec.encode) and the decode's
    XOR replay (codec.replay), as the paper times its compute stage; the
    symbolic peel (codec.peel_schedule) is timed on its own and reported
    beside them.  Two legs of about ``seconds`` each: the oracle as one numpy
    process, and one forked process per core, each running the same oracle
    calls on its own byte columns of every block (the code is bytewise, so
    the columns are independent).  Must run before the GPU is initialised:
    the workers are forked."""
    import multiprocessing as mp
    import numpy as np
    from oracle import codec, graph
    G = graph.build(graph.GraphParams(**spec.graph_kwargs()))
    x = spec.x()
    er = spec.erased_mask()
    k, t = spec.k, spec.t
    tp = time.perf_counter()
    sched = codec.peel_schedule(G, er)
    peel_s = time.perf_counter() - tp
    nR = int(sched.recovered_mask().sum())
    user = (k + nR) * t

    # one core: encode XOR then replay XOR of the whole stripe
    reps, enc_s, rep_s = 0, 0.0, 0.0
    while reps == 0 or enc_s + rep_s < seconds:
        t0 = time.perf_counter()
        c = codec.encode(G, x)
        t1 = time.perf_counter()
        codec.replay(G, c, sched)
        t2 = time.perf_counter()
        enc_s += t1 - t0
        rep_s += t2 - t1
        reps += 1
    one = {"value": round(user * reps / (enc_s + rep_s) / 1e9, 4), "unit": "GB/s", "cores": 1,
           "encode_s_per_rep": round(enc_s / reps, 4), "replay_s_per_rep": round(rep_s / reps, 4),
           "reps": reps}

    # all cores: byte columns of every block, one forked worker per core
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    parts = cores
    step = max(8, (t // parts + 7) // 8 * 8)
    slices = [(a, min(t, a + step)) for a in range(0, t, step)]
    _POOL.update(G=G, x=x, sched=sched, c=_shared_u8((spec.n, t)), xd=_shared_u8((k, t)))
    ctx = mp.get_context("fork")
    reps_p, enc_p, rep_p = 0, 0.0, 0.0
    with ctx.Pool(cores) as pool:
        pool.map(_slice_encode, slices)          # workers started and warm
        while reps_p == 0 or enc_p + rep_p < seconds:
            t0 = time.perf_counter()
            pool.map(_slice_encode, slices)
            t1 = time.perf_counter()
            pool.map(_slice_replay, slices)
            t2 = time.perf_counter()
            enc_p += t1 - t0
            rep_p += t2 - t1
            reps_p += 1
    # the forked workers' output is the oracle's: check it against the one-core run
    x_ref = codec.replay(G, c, sched)
    assert np.array_equal(_POOL["c"], c) and np.array_equal(_POOL["xd"], x_ref)
    _POOL.clear()
    return {"value": round(user * reps_p / (enc_p + rep_p) / 1e9, 4), "unit": "GB/s", "cores": cores,
            "kind": "oracle",
            "sample": "full stripe (k=%d, n=%d, t=%d, %d erased): oracle encode + decode replay, %d "
                      "forked numpy processes over %d byte columns of every block, repeated %d times "
                      "(%.1f s); symbolic peel timed apart" % (spec.k, spec.n, spec.t, spec.n_erased, cores,
                                                               len(slices), reps_p, enc_p + rep_p),
            "encode_s_per_rep": round(enc_p / reps_p, 4), "replay_s_per_rep": round(rep_p / reps_p, 4),
            "peel_s": round(peel_s, 4), "recovered": nR,
            "one_core": one}


def _child_workload(args, workload):
    """One workload of the full line, run as ``bench.py --workload <workload>``
    in a child process; returns its JSON line, or the failure as a field."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--workload", workload, "--no-cpu",
           "--steps", str(args.steps), "--warmup", str(args.warmup),
           "--serve-rate", str(args.serve_rate), "--serve-seconds", str(args.serve_seconds),
           "--batch-stripes", str(args.batch_stripes), "--resident-stripes", str(args.resident_stripes),
           "--reps", str(args.reps)]
    _progress_line("%s: in a process of its own" % workload)
    try:
        p = subprocess.run(cmd, stdout=subprocess.PIPE, text=True, timeout=900)
    except subprocess.TimeoutExpired:
        return {"error": "%s timed out after 900 s" % workload}
    lines = [ln for ln in p.stdout.splitlines() if ln.startswith("{")]
    if p.returncode != 0 or not lines:
        return {"error": "%s ended with exit status %d" % (workload, p.returncode)}
    return json.loads(lines[-1])


def _progress_line(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (--gpus %d refused)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    from synth import workloads

    cpu = None
    if args.workload in ("large_stripe", "all") and args.mode == "step" and not args.no_cpu:
        # the oracle's pool is forked, so it runs before anything touches the GPU
        cpu = cpu_baseline(workloads.large_stripe(), args.cpu_seconds)
        _progress_line("cpu_baseline: %.3f GB/s on %d cores (one core %.3f GB/s)"
                       % (cpu["value"], cpu["cores"], cpu["one_core"]["value"]))
    if args.workload == "all" and args.mode == "step":
        # every workload of the full line runs in a process of its own, the
        # headline first, so that each begins from a clean device (allocator,
        # queues, caches) as it would alone; this process never touches the GPU
        out = _child_workload(args, "large_stripe")
        if "error" in out:
            print(json.dumps(out), flush=True)
            sys.exit(1)
        for key, wl in (("serve", "serve"), ("batched", "batch512"), ("resident", "resident256")):
            out[key] = _child_workload(args, wl)   # a failure there is in its field
        if cpu is not None:
            out["cpu_baseline"] = cpu
        print(json.dumps(out), flush=True)
        return
    import torch
    import paper_1702_07409_amd as fs

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.workload in ("batch512", "resident256", "serve", "extend", "simdisk", "precode", "checks"):
        import bench_batch
        if args.workload == "checks":
            res = bench_batch.run_checks()
        elif args.workload == "precode":
            res = bench_batch.run_precode()
        elif args.workload == "extend":
            res = bench_batch.run_extend()
        elif args.workload == "simdisk":
            res = bench_batch.run_simdisk()
        elif args.workload == "batch512":
            res = bench_batch.run_batch512(args.batch_stripes, reps=args.reps, counters=args.mode == "counters")
        elif args.workload == "resident256":
            res = bench_batch.run_resident256(args.resident_stripes, reps=args.reps)
        else:
            res = bench_batch.run_serve(args.serve_rate, args.serve_seconds)
        print(json.dumps(res), flush=True)
        return
    spec = workloads.large_stripe()
    k, n, t = spec.k, spec.n, spec.t
    g = fs.fs_graph_build(**spec.graph_kwargs())
    x = torch.from_numpy(spec.x()).to("cuda")
    c = torch.empty((n, t), dtype=torch.uint8, device="cuda")
    er = torch.from_numpy(spec.erased_mask()).to("cuda")
    xd = torch.empty((k, t), dtype=torch.uint8, device="cuda")
    rec = torch.empty(k, dtype=torch.uint8, device="cuda")
    st = torch.empty(3, dtype=torch.int32, device="cuda")
    ws = fs.workspace(g, fs.FS_OP_DECODE, t)
    stream = torch.cuda.current_stream()
    if args.mode == "counters":
        counters_run(args, fs, torch, g, x, c, t,
                     lambda: fs.fs_decode(g, c, er, 0, xd, rec, st, t, ws, stream))
        return

    side = torch.cuda.Stream()
    # The plans run on a second stream beside the encodes, and the two streams
    # synchronise once per pair of steps (each cross-stream wait and event
    # costs the main stream a few microseconds between kernels).  Four decode
    # workspaces: step i plans into and applies from wss[i % 4], so a pair's
    # plans write two of them while the previous pair's applies read the other
    # two; a pair waits only for the applies of the pair before that.
    wss = [ws] + [fs.workspace(g, fs.FS_OP_DECODE, t) for _ in range(3)]
    applied = [torch.cuda.Event(), torch.cuda.Event()]
    planned = [torch.cuda.Event(), torch.cuda.Event()]
    for e_ in applied:
        e_.record(stream)

    def pair(p, m, end, ev=None):
        """Steps 2p .. 2p+m-1 (m is 1 or 2); ``end`` is recorded after the last
        apply.  ``ev`` (the instrumented pass only) takes timing events around
        the plans and around each encode and apply."""
        steps = [2 * p + j for j in range(m)]
        side.wait_event(applied[p % 2])
        if ev is not None:
            ev["plan"][0].record(side)
        for i in steps:
            fs.fs_decode_plan(g, er, 0, rec, st, wss[i % 4], side)
        planned[p % 2].record(side)
        if ev is not None:
            ev["plan"][1].record(side)
        for j, i in enumerate(steps):
            if ev is not None:
                ev["enc"][j][0].record(stream)
            fs.fs_encode(g, x, c, t, stream)
            if ev is not None:
                ev["enc"][j][1].record(stream)
            if j == 0:
                stream.wait_event(planned[p % 2])
            if ev is not None:
                ev["app"][j][0].record(stream)
            fs.fs_decode_apply(g, c, xd, t, wss[i % 4], stream)
            if ev is not None:
                ev["app"][j][1].record(stream)
        end.record(stream)
        applied[p % 2] = end

    def run_steps(count, ends, evs=None):
        for p in range((count + 1) // 2):
            pair(p, min(2, count - 2 * p), ends[p], None if evs is None else evs[p])

    run_steps(args.warmup, [torch.cuda.Event() for _ in range((args.warmup + 1) // 2)])
    torch.cuda.synchronize()
    # timed region: exactly K steps, inputs resident in HBM, one event per pair
    npairs = (args.steps + 1) // 2
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(npairs)]
    begin = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    begin.record(stream)
    run_steps(args.steps, ends)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # per-step time: each pair's interval (from the previous pair's end) over its steps
    bounds = [begin] + ends
    step_ms = [bounds[q].elapsed_time(bounds[q + 1]) / min(2, args.steps - 2 * q) for q in range(npairs)]

    # instrumented pass (outside the timed steps): the same pairs with timing
    # events around every kernel, for the per-kernel durations in the step
    ipairs = max(1, min(npairs, 25))
    T = lambda: torch.cuda.Event(enable_timing=True)
    ievs = [{"plan": [T(), T()], "enc": [[T(), T()], [T(), T()]], "app": [[T(), T()], [T(), T()]]}
            for _ in range(ipairs)]
    run_steps(2 * ipairs, [torch.cuda.Event() for _ in range(ipairs)], ievs)
    torch.cuda.synchronize()
    enc_ms = [e_["enc"][j][0].elapsed_time(e_["enc"][j][1]) for e_ in ievs for j in range(2)]
    apply_ms = [e_["app"][j][0].elapsed_time(e_["app"][j][1]) for e_ in ievs for j in range(2)]
    plan_ms = [e_["plan"][0].elapsed_time(e_["plan"][1]) / 2 for e_ in ievs]
    status = st.cpu().tolist()
    nR = k - status[1]
    # correctness guard on the last steps' outputs: recovered blocks equal the inputs
    recovered = rec.cpu().numpy().astype(bool)
    rows = np.flatnonzero(recovered)[:: max(1, int(recovered.sum()) // 64)]
    assert torch.equal(xd[torch.from_numpy(rows).cuda()], x[torch.from_numpy(rows).cuda()])

    # one-stream decode and its schedule / replay split (same kernels, outside the timed steps)
    lp = torch.empty(k + 1, dtype=torch.int32, device="cuda")
    df = torch.empty(k, dtype=torch.int32, device="cuda")
    dg = torch.empty(k, dtype=torch.int32, device="cuda")
    pws = fs.workspace(g, fs.FS_OP_PEEL)
    rws = fs.workspace(g, fs.FS_OP_REPLAY, t)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    peel_ms, rep_ms, dec_ms = [], [], []
    for _ in range(5):
        e[0].record(stream)
        fs.fs_peel(g, er, 0, rec, st, lp, df, dg, pws, stream)
        e[1].record(stream)
        fs.fs_replay(g, c, st, lp, df, dg, xd, t, rws, stream)
        e[2].record(stream)
        fs.fs_decode(g, c, er, 0, xd, rec, st, t, ws, stream)
        e[3].record(stream)
        torch.cuda.synchronize()
        peel_ms.append(e[0].elapsed_time(e[1]))
        rep_ms.append(e[1].elapsed_time(e[2]))
        dec_ms.append(e[2].elapsed_time(e[3]))

    # measured streaming ceiling: a plain device copy of 512 MiB (read + write bytes)
    cp_src = torch.empty(1 << 29, dtype=torch.uint8, device="cuda")
    cp_dst = torch.empty_like(cp_src)
    cp_src.fill_(1)
    cp_ms = []
    for r in range(23):
        e[0].record(stream)
        cp_dst.copy_(cp_src)
        e[1].record(stream)
        torch.cuda.synchronize()
        if r >= 3:
            cp_ms.append(e[0].elapsed_time(e[1]))
    copy_GBps = 2 * cp_src.numel() / (float(np.median(cp_ms)) * 1e-3) / 1e9
    del cp_src, cp_dst

    ms_per_step = elapsed * 1e3 / args.steps
    user_bytes = (k + nR) * t
    value = user_bytes / (ms_per_step * 1e-3) / 1e9
    rp, col, _, _ = g.export()
    k_touched = int(len(np.unique(col)))
    enc_alg = (k_touched + n) * t
    enc_avg_ms = float(np.mean(enc_ms))
    enc_achieved = enc_alg / (enc_avg_ms * 1e-3) / 1e9
    # the replay (fs_decode_apply launches only the replay kernel) is the
    # longest kernel of the step: it carries the roofline.  Algorithmic
    # bytes: the |R| coded blocks it reads and the k input blocks it writes
    # (the unrecovered ones as zeros).
    rep_alg = (nR + k) * t
    rep_avg_ms = float(np.mean(apply_ms))
    rep_achieved = rep_alg / (rep_avg_ms * 1e-3) / 1e9
    traffic = {"replay": None, "encode": None}
    if os.path.exists(PROFILE_COUNTERS):
        with open(PROFILE_COUNTERS) as f:
            prof = json.load(f)
        # counters taken on other kernel sources are not reported
        if prof.get("kernel_source_sha256_16") == kernel_source_hash():
            for key, pat in (("encode", "gather_kernel"), ("replay", "replay_wide_kernel")):
                for name, rec in prof.get("kernels", {}).items():
                    d = rec.get("derived", {})
                    if pat in name and "read_bytes" in d and "write_bytes" in d:
                        traffic[key] = int(d["read_bytes"] + d["write_bytes"])
    dec_avg_ms = float(np.median(dec_ms))
    out = {
        "metric": "encode+decode GB/s user data (% HBM peak), plain one-stripe path",
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic (seeded uniform bytes)",
        "config": {"workload": "large_stripe", "k": k, "n": n, "t": t,
                   "dist": "finite max-degree 16 (w1=0.02, wd=1/(d(d-1)))", "erased": spec.n_erased,
                   "step": "fs_decode_plan on a second stream alongside fs_encode, then fs_decode_apply; "
                           "the streams synchronise once per pair of steps",
                   "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": round(rep_achieved, 2), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(rep_achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic["replay"], "traffic_kind": TRAFFIC_KIND,
                     "kernel": "replay_wide_kernel (fs_decode_apply)",
                     "algorithmic_bytes_per_launch": rep_alg},
        "encode_roofline": {"bound": "hbm", "achieved": round(enc_achieved, 2), "peak": HBM_PEAK_GBPS,
                            "unit": "GB/s", "frac": round(enc_achieved / HBM_PEAK_GBPS, 4),
                            "traffic": traffic["encode"], "traffic_kind": TRAFFIC_KIND,
                            "kernel": "gather_kernel (fs_encode)",
                            "algorithmic_bytes_per_launch": enc_alg},
        "step_timing": "timed steps carry one event per pair of steps; the encode, apply and plan "
                       "durations come from a separate pass with events around every kernel",
        "step_ms_median": round(float(np.median(step_ms)), 4),
        "step_ms_p99": round(float(np.percentile(step_ms, 99)), 4),
        "copy_ceiling": {"GBps": round(copy_GBps, 1), "frac_of_peak": round(copy_GBps / HBM_PEAK_GBPS, 4),
                         "what": "plain device copy of 512 MiB, read + write bytes over its median time"},
        "encode_ms": round(enc_avg_ms, 4),
        "encode_ms_median": round(float(np.median(enc_ms)), 4),
        "encode_ms_p99": round(float(np.percentile(enc_ms, 99)), 4),
        "apply_ms_median": round(float(np.median(apply_ms)), 4),
        "apply_ms_p99": round(float(np.percentile(apply_ms, 99)), 4),
        "plan_ms": round(float(np.mean(plan_ms)), 4),
        "apply_ms": round(float(np.mean(apply_ms)), 4),
        "decode_one_stream_ms": round(dec_avg_ms, 4),
        "peel_ms": round(float(np.median(peel_ms)), 4),
        "replay_ms": round(float(np.median(rep_ms)), 4),
        "encode_GBps_user": round(k * t / (enc_avg_ms * 1e-3) / 1e9, 2),
        "decode_GBps_user": round(nR * t / (dec_avg_ms * 1e-3) / 1e9, 2),
        "decode_status": status,
        "recovered_fraction": round(nR / k, 5),
        "hbm_frac_effective_step": round(((k_touched + n) * t + (nR + k) * t) / (ms_per_step * 1e-3)
                                         / 1e9 / HBM_PEAK_GBPS, 4),
        "paper_cpu_context": "Table 2: encode 2722 MB/s, decode 3291/2852/2340 MB/s (2-4 disks lost), "
                             "k=1036 n=2180 t=1024, 2x Xeon E5-2620 with 12 threads",
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
