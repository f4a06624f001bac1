"""Batched workloads for bench.py: many stripes per captured launch (fs_plan)
against the plain path (one fs_encode / fs_decode / fs_repair / fs_update
call per stripe) on the same stripes.

batch512     512 stripes, k log-uniform in [64, 8192), blocks 4 KiB..1 MiB,
             RSD (c=0.05, delta=0.01), 8 % overhead, 4 % erasures.  Processed
             in waves that fit HBM; a wave is an encode plan then a decode plan.
resident256  256 stripes k=1024 x 256 KiB, n=1126, RSD (c=0.1, delta=0.05),
             resident in HBM: repair of 1-4 lost coded blocks per stripe from
             the inputs, and an update of 10 inputs per stripe.
extend       the large stripe (k=4096 x 64 KiB, finite16, n=1.1 k) grown to
             n=1.2 k: 409 new coded blocks from the resident inputs, and from
             the existing blocks with 5 % of them erased.
simdisk      disk-failure sweeps of the larger code of the paper's measurements
             (k=10246, n=21800, finite Raptor table): every combination of 4
             failed disks out of 24, and every failure count on 10 disks.
precode      the paper's Table 2 set-up with its array-LDPC precode: a 64 MiB
             object, b data blocks precoded to k and encoded to n coded blocks
             on 10 disks, decoded with 2, 3 and 4 disks lost.  Partitions of
             one object share one graph, so the object is one stripe whose
             block holds every partition's t bytes side by side.
"""

import sys
import time

import numpy as np


def _progress(msg):
    print(msg, file=sys.stderr, flush=True)

HBM_PEAK_GBPS = 8000.0


def _ev():
    import torch
    return torch.cuda.Event(enable_timing=True)


def _time(fn, reps):
    import torch
    e0, e1 = _ev(), _ev()
    fn()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _time_reps(fn, reps, warm=2):
    """Per-repetition times (ms) of fn, each bracketed by its own events,
    run back to back after ``warm`` untimed calls."""
    import torch
    evs = [(_ev(), _ev()) for _ in range(reps)]
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in evs]


def _stats(ms):
    return {"median_ms": round(float(np.median(ms)), 4), "p99_ms": round(float(np.percentile(ms, 99)), 4),
            "reps": len(ms)}


def _compulsory_encode(g, t):
    _, col, _, _ = g.export()
    return (len(np.unique(col)) + g.n) * t


def run_batch512(count=512, reps=20, tune_cache="/tmp/fs_tune_cache.txt", counters=False):
    """counters: the first wave only, one launch of its encode plan and one of
    its decode plan (tuned from the cache, else by the default rule), for
    rocprofv3 --pmc runs."""
    import torch
    import paper_1702_07409_amd as fs
    import synth.gpu as sg
    from synth import workloads

    specs = workloads.batch512(count)
    free, _ = torch.cuda.mem_get_info()
    budget = int(free * 0.55)
    waves, cur, used = [], [], 0
    for sp in specs:
        need = (2 * sp.k + sp.n) * sp.t
        if cur and used + need > budget:
            waves.append(cur)
            cur, used = [], 0
        cur.append(sp)
        used += need
    if cur:
        waves.append(cur)
    tot = dict(enc_user=0, dec_user=0, comp=0, t_batch=0.0, t_plain=0.0, t_enc=0.0, t_dec=0.0, recovered=0, k=0)
    tune = None
    t_setup = time.perf_counter()
    for wave in waves:
        bufs = []
        for sp in wave:
            g = fs.fs_graph_build(**sp.graph_kwargs())
            x = torch.empty((sp.k, sp.t), dtype=torch.uint8, device="cuda")
            sg.fill(x, sp.data_seed, sp.stripe, sp.t)
            c = torch.empty((sp.n, sp.t), dtype=torch.uint8, device="cuda")
            xd = torch.empty((sp.k, sp.t), dtype=torch.uint8, device="cuda")
            er = torch.from_numpy(sp.erased_mask()).cuda()
            rec = torch.empty(sp.k, dtype=torch.uint8, device="cuda")
            st = torch.empty(3, dtype=torch.int32, device="cuda")
            bufs.append((sp, g, x, c, xd, er, rec, st))
        enc = fs.Plan([fs.work("encode", g, sp.t, x=x, c=c) for sp, g, x, c, xd, er, rec, st in bufs],
                      tune_cache=tune_cache, autotune=not counters)
        dec = fs.Plan([fs.work("decode", g, sp.t, x=xd, c=c, erased=er, recovered=rec, status=st)
                       for sp, g, x, c, xd, er, rec, st in bufs])
        if counters:
            torch.cuda.synchronize()
            enc.launch()
            torch.cuda.synchronize()
            dec.launch()
            torch.cuda.synchronize()
            return {"mode": "counters", "workload": "batch512", "stripes": len(wave),
                    "input_bytes": sum(sp.k * sp.t for sp, *_ in bufs),
                    "compulsory_encode_bytes": sum(_compulsory_encode(g, sp.t) for sp, g, *_ in bufs),
                    "tune": enc.info()["tune"], "gather_jobs": enc.info()["gather_jobs"]}
        tune = enc.info()["tune"]
        enc_ms = _time_reps(enc.launch, reps)
        dec_ms = _time_reps(dec.launch, reps)
        t_enc = float(np.median(enc_ms))
        t_dec = float(np.median(dec_ms))
        # check: the batched coded blocks equal the plain path's, stripe by stripe
        for sp, g, x, c, xd, er, rec, st in bufs:
            cref = torch.empty_like(c)
            fs.fs_encode(g, x, cref, sp.t)
            assert torch.equal(cref, c), "batched encode differs from the plain encode"
            del cref
        # check: every recovered block equals its input (sampled rows)
        nrec = 0
        for sp, g, x, c, xd, er, rec, st in bufs:
            r = rec.cpu().numpy().astype(bool)
            nrec += int(r.sum())
            rows = np.flatnonzero(r)[:: max(1, int(r.sum()) // 8)]
            if len(rows):
                ix = torch.from_numpy(rows).cuda()
                assert torch.equal(xd[ix], x[ix]), "decoded blocks differ from the inputs"
        wss = {id(b[1]): fs.workspace(b[1], fs.FS_OP_DECODE, b[0].t) for b in bufs}

        def plain():
            for sp, g, x, c, xd, er, rec, st in bufs:
                fs.fs_encode(g, x, c, sp.t)
                fs.fs_decode(g, c, er, 0, xd, rec, st, sp.t, wss[id(g)])

        plain_ms = _time_reps(plain, reps, warm=1)
        t_plain = float(np.median(plain_ms))
        for key, v in (("enc", enc_ms), ("dec", dec_ms), ("plain", plain_ms)):
            tot.setdefault("p99_" + key, 0.0)
            tot["p99_" + key] += float(np.percentile(v, 99))
        tot["enc_user"] += sum(sp.k * sp.t for sp, *_ in bufs)
        tot["dec_user"] += sum(int(b[6].sum().item()) * b[0].t for b in bufs)
        tot["comp"] += sum(_compulsory_encode(g, sp.t) + (int(rec.sum().item()) + sp.k) * sp.t
                           for sp, g, x, c, xd, er, rec, st in bufs)
        tot["t_enc"] += t_enc
        tot["t_dec"] += t_dec
        tot["t_batch"] += t_enc + t_dec
        tot["t_plain"] += t_plain
        tot["recovered"] += nrec
        tot["k"] += sum(sp.k for sp in wave)
        del enc, dec, bufs, wss
        torch.cuda.empty_cache()
        _progress("batch512: wave of %d stripes done (enc %.2f ms, dec %.2f ms, plain %.2f ms)"
                  % (len(wave), t_enc, t_dec, t_plain))
    user = tot["enc_user"] + tot["dec_user"]
    return {
        "workload": "batch512", "stripes": count, "waves": len(waves),
        "input_GB": round(tot["enc_user"] / 1e9, 2),
        "batched_GBps_user": round(user / (tot["t_batch"] * 1e-3) / 1e9, 1),
        "plain_loop_GBps_user": round(user / (tot["t_plain"] * 1e-3) / 1e9, 1),
        "batched_encode_GBps_user": round(tot["enc_user"] / (tot["t_enc"] * 1e-3) / 1e9, 1),
        "batched_decode_GBps_user": round(tot["dec_user"] / (tot["t_dec"] * 1e-3) / 1e9, 1),
        "batched_hbm_frac_effective": round(tot["comp"] / (tot["t_batch"] * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "recovered_fraction": round(tot["recovered"] / tot["k"], 4),
        "batched_ms": round(tot["t_batch"], 3), "plain_ms": round(tot["t_plain"], 3),
        "timing": "per wave: %d timed launches of the encode plan, the decode plan and the plain loop, each "
                  "bracketed by its own events; *_ms sum the per-wave medians, *_p99_ms the per-wave p99s" % reps,
        "batched_p99_ms": round(tot["p99_enc"] + tot["p99_dec"], 3), "plain_p99_ms": round(tot["p99_plain"], 3),
        "tune": tune, "setup_s": round(time.perf_counter() - t_setup, 1),
    }


def run_resident256(count=256, reps=20, tune_cache="/tmp/fs_tune_cache.txt"):
    import torch
    import paper_1702_07409_amd as fs
    import synth.gpu as sg
    from synth import gen, workloads

    specs = workloads.resident256(count)
    t0 = time.perf_counter()
    st_ = []
    for sp in specs:
        g = fs.fs_graph_build(**sp.graph_kwargs())
        x = torch.empty((sp.k, sp.t), dtype=torch.uint8, device="cuda")
        sg.fill(x, sp.data_seed, sp.stripe, sp.t)
        c = torch.empty((sp.n, sp.t), dtype=torch.uint8, device="cuda")
        lost = sp.extra["lost"]
        ids = sp.extra["update_ids"]
        new = torch.empty((len(ids), sp.t), dtype=torch.uint8, device="cuda")
        for u, i in enumerate(ids):
            sg.fill(new[u:u + 1], workloads.UPDATE_DATA_SEED, sp.stripe, sp.t, first_block=i,
                    purpose=sg.UPDATE_DATA)
        st_.append(dict(sp=sp, g=g, x=x, c=c, lost=torch.from_numpy(np.array(lost, np.uint32)).cuda(),
                        nl=len(lost), ids=torch.from_numpy(np.array(ids, np.uint32)).cuda(), nu=len(ids),
                        new=new, rep=torch.empty(len(lost), dtype=torch.uint8, device="cuda"),
                        rst=torch.empty(3, dtype=torch.int32, device="cuda"),
                        ust=torch.empty(3, dtype=torch.int32, device="cuda")))
    _progress("resident256: %d stripes resident" % len(st_))
    enc = fs.Plan([fs.work("encode", d["g"], d["sp"].t, x=d["x"], c=d["c"]) for d in st_])
    enc.launch()
    torch.cuda.synchronize()
    rep = fs.Plan([fs.work("repair", d["g"], d["sp"].t, x=d["x"], c=d["c"], ids=d["lost"], n_ids=d["nl"],
                           repaired=d["rep"], status=d["rst"]) for d in st_],
                  tune_cache=tune_cache, autotune=True)
    upd = fs.Plan([fs.work("update", d["g"], d["sp"].t, x=d["x"], c=d["c"], ids=d["ids"], n_ids=d["nu"],
                           new_blocks=d["new"], status=d["ust"]) for d in st_])
    rep_ms = _time_reps(rep.launch, reps)
    # the first update applies the new blocks; repeats carry zero deltas but the same traffic
    upd_ms = _time_reps(upd.launch, reps)
    t_rep, t_upd = float(np.median(rep_ms)), float(np.median(upd_ms))
    assert all(d["rst"].cpu().tolist() == [1, 0, 0] for d in st_)
    ws = {}
    for d in st_:
        ws[id(d)] = (fs.workspace(d["g"], fs.FS_OP_REPAIR, d["sp"].t, d["nl"]),
                     fs.workspace(d["g"], fs.FS_OP_UPDATE, d["sp"].t, d["nu"]))

    def plain_rep():
        for d in st_:
            fs.fs_repair(d["g"], d["x"], d["c"], None, d["lost"], d["nl"], d["rep"], d["rst"], d["sp"].t,
                         ws[id(d)][0])

    def plain_upd():
        for d in st_:
            fs.fs_update(d["g"], d["x"], d["c"], d["ids"], d["nu"], d["new"], d["ust"], d["sp"].t, ws[id(d)][1])

    prep_ms = _time_reps(plain_rep, reps)
    pupd_ms = _time_reps(plain_upd, reps)
    tp_rep, tp_upd = float(np.median(prep_ms)), float(np.median(pupd_ms))
    # bytes: repair rebuilds |lost| blocks; update rewrites |U| inputs
    t = specs[0].t
    rep_user = sum(d["nl"] for d in st_) * t
    upd_user = sum(d["nu"] for d in st_) * t
    rep_comp = 0
    upd_comp = 0
    for d in st_:
        rp, col, cp, ri = d["g"].export()
        lost = d["sp"].extra["lost"]
        nb = set()
        for j in lost:
            nb.update(col[rp[j]:rp[j + 1]].tolist())
        rep_comp += (len(nb) + len(lost)) * t
        aff = set()
        for i in d["sp"].extra["update_ids"]:
            aff.update(ri[cp[i]:cp[i + 1]].tolist())
        upd_comp += (3 * d["nu"] + 2 * len(aff)) * t
    return {
        "workload": "resident256", "stripes": count,
        "resident_GB": round(sum((d["sp"].k + d["sp"].n) * d["sp"].t for d in st_) / 1e9, 1),
        "repair_batched_ms": round(t_rep, 3), "repair_plain_ms": round(tp_rep, 3),
        "repair_batched_GBps_user": round(rep_user / (t_rep * 1e-3) / 1e9, 1),
        "repair_hbm_frac_effective": round(rep_comp / (t_rep * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "update_batched_ms": round(t_upd, 3), "update_plain_ms": round(tp_upd, 3),
        "update_batched_GBps_user": round(upd_user / (t_upd * 1e-3) / 1e9, 1),
        "update_hbm_frac_effective": round(upd_comp / (t_upd * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "repair_batched": _stats(rep_ms), "repair_plain": _stats(prep_ms),
        "update_batched": _stats(upd_ms), "update_plain": _stats(pupd_ms),
        "repair_tune": rep.info()["tune"], "setup_s": round(time.perf_counter() - t0, 1),
    }


def run_extend(reps=20):
    import torch
    import paper_1702_07409_amd as fs
    import synth.gpu as sg
    from dataclasses import replace
    from synth import gen, workloads

    base = workloads.large_stripe()
    sp = replace(base, n=gen.overhead_n(base.k, 0.20))
    k, n_old, n, t = sp.k, base.n, sp.n, sp.t
    g = fs.fs_graph_build(**sp.graph_kwargs())
    x = torch.empty((k, t), dtype=torch.uint8, device="cuda")
    sg.fill(x, sp.data_seed, sp.stripe, t)
    c = torch.empty((n, t), dtype=torch.uint8, device="cuda")
    fs.fs_encode(g, x, c, t)
    er = torch.from_numpy(gen.erasure_mask(sp.erase_seed, sp.stripe, n_old, base.n_erased)).cuda()
    made = torch.empty(n - n_old, dtype=torch.uint8, device="cuda")
    st = torch.empty(3, dtype=torch.int32, device="cuda")
    wa = fs.workspace(g, fs.FS_OP_EXTEND, t)
    wb = fs.workspace(g, fs.FS_OP_EXTEND_CONVENTIONAL, t)
    t_a = _time(lambda: fs.fs_extend(g, n_old, x, c, None, made, st, t, wa), reps)
    made_a = int(made.sum())
    t_b = _time(lambda: fs.fs_extend(g, n_old, None, c, er, made, st, t, wb), reps)
    made_b = int(made.sum())
    rp, col, _, _ = g.export()
    touched = len(np.unique(col[rp[n_old]:rp[n]]))
    new_bytes = (n - n_old) * t
    return {
        "workload": "extend", "k": k, "n_old": n_old, "n": n, "t": t, "erased_old": base.n_erased,
        "from_inputs_ms": round(t_a, 3), "from_inputs_made": made_a,
        "from_inputs_GBps_new": round(new_bytes / (t_a * 1e-3) / 1e9, 1),
        "from_inputs_hbm_frac_effective": round((touched + n - n_old) * t / (t_a * 1e-3) / 1e9
                                                / HBM_PEAK_GBPS, 4),
        "conventional_ms": round(t_b, 3), "conventional_made": made_b,
        "conventional_GBps_new": round(made_b * t / (t_b * 1e-3) / 1e9, 1),
    }


def run_simdisk(reps=5):
    import math
    import torch
    import paper_1702_07409_amd as fs

    g = fs.fs_graph_build(k=10246, n=21800, dist="raptor", seed=1)
    ws = fs.workspace(g, fs.FS_OP_SIM_DISKS)
    out = {"workload": "simdisk", "k": 10246, "n": 21800, "dist": "raptor", "graph_seed": 1, "nnz": int(g.nnz)}
    s, f = 24, 4
    total = math.comb(s, f)
    res = torch.empty((total, 3), dtype=torch.int32, device="cuda")
    ms = _time(lambda: fs.fs_sim_disks(g, s, f, 0, total, 0, res, ws), reps)
    r = res.cpu().numpy()
    out.update({"s": s, "f": f, "combinations": total, "ms": round(ms, 3),
                "combinations_per_s": round(total / (ms * 1e-3)),
                "tolerable": int(r[:, 0].sum()), "mean_levels": round(float(r[:, 2].mean()), 1)})
    per_f = []
    t_all = 0.0
    for f10 in range(0, 11):
        c = math.comb(10, f10)
        res10 = torch.empty((c, 3), dtype=torch.int32, device="cuda")
        m = _time(lambda: fs.fs_sim_disks(g, 10, f10, 0, c, 0, res10, ws), reps)
        t_all += m
        per_f.append(int(res10[:, 0].sum().item()))
    out.update({"ten_disks_tolerable_by_f": per_f, "ten_disks_all_ms": round(t_all, 3)})
    # the same code with its array-LDPC precode (b = 9919, j' = 3): a pattern
    # is tolerable when the two-stage decode recovers every data block
    pc = fs.fs_precode_build(9919, 10246)
    wsp = fs.workspace(g, fs.FS_OP_SIM_DISKS, 16, pc.k - pc.b)
    resp = torch.empty((total, 4), dtype=torch.int32, device="cuda")
    msp = _time(lambda: fs.fs_sim_disks_precoded(g, pc, s, f, 0, total, 0, resp, wsp), reps)
    per_fp = []
    for f10 in range(0, 11):
        c = math.comb(10, f10)
        r10 = torch.empty((c, 4), dtype=torch.int32, device="cuda")
        fs.fs_sim_disks_precoded(g, pc, 10, f10, 0, c, 0, r10, wsp)
        per_fp.append(int(r10[:, 0].sum().item()))
    out["precoded"] = {"b": 9919, "ms": round(msp, 3), "combinations_per_s": round(total / (msp * 1e-3)),
                       "tolerable": int(resp[:, 0].sum().item()), "ten_disks_tolerable_by_f": per_fp}
    # The sweep is bound by instruction issue, not HBM: the roofline is the
    # VALU issue rate (256 CUs x 2.4 GHz x one wave64 VALU instruction per CU
    # per cycle) against the VALU instructions per pattern that the committed
    # counter profile recorded for this kernel source (null once it changed).
    peak = 256 * 2.4e9
    valu = None
    try:
        import json, os
        import bench
        prof = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                                           "simdisk_counters.json")))
        if prof.get("kernel_source_sha256_16") == bench.kernel_source_hash():
            valu = prof["valu_per_pattern"]
    except (OSError, ValueError, KeyError):
        valu = None
    achieved = valu * total / (ms * 1e-3) if valu else None
    out["roofline"] = {"bound": "alu", "unit": "wave64 VALU instructions/s", "peak": peak,
                       "achieved": achieved, "frac": round(achieved / peak, 4) if achieved else None,
                       "valu_per_pattern": valu, "kernel": "simdisk_kernel"}
    return out


PAPER_TABLE2 = {1036: {"encode": 2722, "decode": {2: 3291, 3: 2852, 4: 2340}, "t": 1024},
                10246: {"encode": 1691, "decode": {2: 2668, 3: 2496, 4: 2356}, "t": 512}}


def _largest_prime_factor(k):
    best, x, d = 1, k, 2
    while d * d <= x:
        while x % d == 0:
            best, x = d, x // d
        d += 1
    return max(best, x) if x > 1 else best


def run_precode(reps=10):
    import torch
    import paper_1702_07409_amd as fs
    import synth.gpu as sg

    out = {"workload": "precode", "object_MiB": 64, "disks": 10, "codes": []}
    size = 64 << 20
    for k, n in ((1036, 2180), (10246, 21800)):
        # array code with j' = 3: b = (k' - 3) p
        lp = _largest_prime_factor(k)
        b = (k // lp - 3) * lp
        t_part = PAPER_TABLE2[k]["t"]
        parts = -(-size // (b * t_part))
        t = parts * t_part
        g = fs.fs_graph_build(k=k, n=n, dist="raptor", seed=1)
        pcode = fs.fs_precode_build(b, k)
        x = torch.empty((k, t), dtype=torch.uint8, device="cuda")
        sg.fill(x[:b], 0, 0, t)
        c = torch.empty((n, t), dtype=torch.uint8, device="cuda")

        def enc():
            fs.fs_precode_encode(pcode, x, t)
            fs.fs_encode(g, x, c, t)
        t_enc = _time(enc, reps)
        row = {"k": k, "b": b, "n": n, "p": pcode.p, "k'": pcode.kp, "j'": pcode.jp, "partitions": parts,
               "t_partition": t_part, "stripe_t": t, "encode_ms": round(t_enc, 3),
               "encode_MBps": round(size / (t_enc * 1e-3) / 1e6), "paper_encode_MBps": PAPER_TABLE2[k]["encode"],
               "decode": []}
        xd = torch.empty_like(x)
        rec = torch.empty(k, dtype=torch.uint8, device="cuda")
        st = torch.empty(4, dtype=torch.int32, device="cuda")
        ws = fs.workspace(g, fs.FS_OP_DECODE_PRECODED, t)
        for f in (2, 3, 4):
            er_h = np.zeros(n, np.uint8)
            for d in range(f):
                er_h[d * n // 10:(d + 1) * n // 10] = 1
            er = torch.from_numpy(er_h).cuda()
            t_dec = _time(lambda: fs.fs_decode_precoded(g, pcode, c, er, 0, xd, rec, st, t, ws), reps)
            s_ = st.cpu().tolist()
            ok = bool(s_[0]) and bool(torch.equal(xd[:b], x[:b]))
            row["decode"].append({"disks_lost": f, "ms": round(t_dec, 3), "MBps": round(size / (t_dec * 1e-3) / 1e6),
                                  "status": s_, "data_intact": ok,
                                  "paper_MBps": PAPER_TABLE2[k]["decode"][f]})
        out["codes"].append(row)
        del x, c, xd
        torch.cuda.empty_cache()
    out["paper_context"] = ("Table 2: 2x Xeon E5-2620 (12 cores, 12 threads), 64 MiB file over 10 disks, "
                            "MB/s of the compute stage; precode parameters not given")
    return out


def _local_reads(groups, lost):
    """Coded blocks read by local repair (BP over the groups, the rule the
    library applies): (blocks rebuilt, block reads, distinct surviving blocks
    read, levels).  Bandwidth accounting for the report; the rebuilt count
    and levels are checked against the library's status."""
    down = set(lost)
    lost_set = set(lost)
    by_block = {}
    for q, grp in enumerate(groups):
        for m in grp:
            by_block.setdefault(m, []).append(q)
    todo = list(lost)
    rebuilt = reads = levels = 0
    fetched = set()
    while todo:
        picks = []
        for s in todo:
            for q in by_block.get(s, ()):
                if not any(m in down for m in groups[q] if m != s):
                    picks.append((s, q))
                    break
        if not picks:
            break
        for s, q in picks:
            reads += len(groups[q]) - 1
            fetched.update(m for m in groups[q] if m not in lost_set)
        for s, _ in picks:
            down.discard(s)
        rebuilt += len(picks)
        done = {s for s, _ in picks}
        todo = [s for s in todo if s not in done]
        levels += 1
    return rebuilt, reads, len(fetched), levels


def run_checks(reps=10):
    """Check #2/#3 generation (Algorithm 4) and repair of lost disks by local
    groups (BP over the check #3 groups) against the conventional repair
    (decode, then re-encode), before and after adding §2.5's groups from
    degree-one blocks and from the precode's check #1 sets.

    Codes, Raptor Omega graphs over precoded objects (array code with j' = 3)
    striped over 10 disks: the paper's illustrative one (k=500, n=1000,
    t=512; §4) and Table 2's smaller one (k=1036, n=2180, a 64 MiB object)
    with disk 0 (rows 0 .. n/10-1) lost; the §5 repair case (k=10246,
    n=21800, 10240-byte blocks: 100 MiB) with disks 0 and 1 lost.  Repair
    bandwidth is the bytes of coded blocks read: for local repair the other
    members of each block's group, for the conventional repair the coded
    blocks the decode uses (one per recovered input).  bytes_read counts every
    source of every XOR; bytes_transferred counts each surviving block once
    (what a repair would fetch over the network, the paper's measure)."""
    import torch
    import paper_1702_07409_amd as fs
    import synth.gpu as sg

    out = {"workload": "checks", "disks": 10, "codes": []}
    for k, n, t, disks in ((500, 1000, 512, 1), (1036, 2180, 65536, 1), (10246, 21800, 10240, 2)):
        lp = _largest_prime_factor(k)
        b = (k // lp - 3) * lp
        g = fs.fs_graph_build(k=k, n=n, dist="raptor", seed=1)
        pc = fs.fs_precode_build(b, k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ch = fs.fs_checks_generate(g)
        torch.cuda.synchronize()
        gen_ms = (time.perf_counter() - t0) * 1e3
        x = torch.empty((k, t), dtype=torch.uint8, device="cuda")
        sg.fill(x[:b], 0, 0, t)
        fs.fs_precode_encode(pc, x, t)
        c = torch.empty((n, t), dtype=torch.uint8, device="cuda")
        fs.fs_encode(g, x, c, t)
        lost_h = np.arange(0, disks * n // 10, dtype=np.uint32)
        m = len(lost_h)
        lost = torch.from_numpy(lost_h).cuda()
        c_ref = c[:m].clone()
        rep = torch.empty(m, dtype=torch.uint8, device="cuda")
        st = torch.empty(3, dtype=torch.int32, device="cuda")
        ws_l = fs.workspace(g, fs.FS_OP_REPAIR_LOCAL, t, m)

        def local(tag):
            t_loc = _time(lambda: fs.fs_repair_local(g, ch, c, None, lost, m, rep, st, t, ws_l), reps)
            n_loc = int(rep.sum().item())
            ok = bool(torch.equal(c[:m][rep.bool()], c_ref[rep.bool()]))
            _, c3 = ch.export()
            n_acc, reads, fetched, levels = _local_reads(c3, lost_h.tolist())
            assert n_acc == n_loc and levels == st.cpu().tolist()[2]
            _progress("checks: k=%d n=%d %s: local repair %d/%d in %.3f ms" % (k, n, tag, n_loc, m, t_loc))
            # rates: every source read with repetition (what the rebuild issues),
            # and the compulsory bytes (each surviving source once, each rebuilt block
            # written once), against the 8 TB/s HBM peak
            src_gbps = reads * t / (t_loc * 1e6)
            comp_gbps = (fetched + n_loc) * t / (t_loc * 1e6)
            return {"groups": ch.n_check3, "ms": round(t_loc, 4), "repaired": n_loc, "levels": levels, "exact": ok,
                    "bytes_read": reads * t, "bytes_transferred": fetched * t,
                    "mean_group_read": round(reads / max(n_loc, 1), 2),
                    "source_reads_GBps": round(src_gbps, 1), "source_reads_hbm_frac": round(src_gbps / 8000.0, 4),
                    "compulsory_GBps": round(comp_gbps, 1)}

        row = {"k": k, "n": n, "t": t, "b": b, "object_bytes": b * t, "generate_ms": round(gen_ms, 2),
               "sweeps": ch.sweeps, "check2": ch.n_check2, "check3": ch.n_check3, "disks_lost": disks,
               "lost_blocks": m}
        row["local"] = local("generated groups")
        t0 = time.perf_counter()
        row["added_groups"] = ch.add_groups(g, pc)
        row["add_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
        row["local_with_added"] = local("with added groups")
        # conventional repair of the same disks: decode from the other rows, re-encode
        rep2 = torch.empty(m, dtype=torch.uint8, device="cuda")
        st2 = torch.empty(3, dtype=torch.int32, device="cuda")
        ws_c = fs.workspace(g, fs.FS_OP_REPAIR_CONVENTIONAL, t, m)
        t_conv = _time(lambda: fs.fs_repair(g, None, c, None, lost, m, rep2, st2, t, ws_c), reps)
        n_conv = int(rep2.sum().item())
        conv_ok = bool(torch.equal(c[:m][rep2.bool()], c_ref[rep2.bool()]))
        er = torch.zeros(n, dtype=torch.uint8, device="cuda")
        er[:m] = 1
        xd = torch.empty_like(x)
        rec = torch.empty(k, dtype=torch.uint8, device="cuda")
        st3 = torch.empty(3, dtype=torch.int32, device="cuda")
        fs.fs_decode(g, c, er, 0, xd, rec, st3, t, fs.workspace(g, fs.FS_OP_DECODE, t))
        n_rec = int(rec.sum().item())
        row["conventional"] = {"ms": round(t_conv, 4), "repaired": n_conv, "exact": conv_ok,
                               "decode_recovered": n_rec, "bytes_read": n_rec * t, "bytes_transferred": n_rec * t}
        # the same with the two-stage decode (the precode's BP after the LDGM one)
        ws_p = fs.workspace(g, fs.FS_OP_REPAIR_PRECODED, t, m)
        t_pre = _time(lambda: fs.fs_repair_precoded(g, pc, c, None, lost, m, rep2, st2, t, ws_p), reps)
        n_pre = int(rep2.sum().item())
        row["conventional_precoded"] = {"ms": round(t_pre, 4), "repaired": n_pre,
                                        "exact": bool(torch.equal(c[:m][rep2.bool()], c_ref[rep2.bool()]))}
        out["codes"].append(row)
        del x, c, xd, c_ref
        torch.cuda.empty_cache()
    out["paper_context"] = ("§5: k=10246, n=21800, 100 MiB, two disks lost: conventional repair 108,267,520 "
                            "bytes, local groups at most 65,952,320 bytes (2x Xeon E5-2620)")
    return out


def _fresh(reqs, Request):
    """New request objects with the same inputs (results cleared)."""
    out = []
    for r in reqs:
        out.append(Request(r.kind, arrival=r.arrival, params=r.params, t=r.t, x=r.x, stripe=r.stripe,
                           erased=r.erased, maxit=r.maxit, ids=r.ids, new_blocks=r.new_blocks, rid=r.rid))
    return out


def run_serve(rate=2000.0, duration=1.0, pool_size=256, sweep=(8000.0, 32000.0, 0.0), budget_gib=48):
    """Poisson mix of requests served by the continuous-batching loop.

    The pool of resident stripes and every request's device inputs are made
    before the clock starts (inputs resident in HBM).  The headline run
    replays the trace at `rate`; the sweep replays the same requests with
    arrival times scaled to higher rates (0: all at once), with the graph
    cache already warm.  Busy time is the union of the ticks' device
    intervals (HIP events); user bytes: k t per encode, |recovered| t per
    decode, m t per repair and update.
    """
    import torch
    from paper_1702_07409_amd.serve import Request, Server
    from synth import serving, workloads

    srv = Server(budget=budget_gib << 30, streams=3, max_inflight=4, max_items=64, workers=12)
    t0 = time.perf_counter()
    pool = serving.build_pool(srv, pool_size)
    torch.cuda.synchronize()
    _progress("serve: pool of %d stripes ready (%.1f s)" % (pool_size, time.perf_counter() - t0))
    # warm the allocator and the launch path on a trace of another seed
    warm = serving.build_requests(workloads.serving_trace(rate=20000.0, duration=0.002, seed=99,
                                                          pool_size=pool_size, hi=8 << 20),
                                  pool, Request)
    srv.run(warm)
    trace = workloads.serving_trace(rate=rate, duration=duration, pool_size=pool_size)
    reqs = serving.build_requests(trace, pool, Request)
    torch.cuda.synchronize()
    _progress("serve: %d requests staged (%.1f s)" % (len(reqs), time.perf_counter() - t0))
    b0, h0 = srv.cache.builds, srv.cache.hits
    head = srv.run(reqs)
    head["graph_builds"] -= b0
    head["graph_hits"] -= h0
    head["rate_offered"] = rate
    head["hbm_frac_busy"] = (round(head["user_GBps_busy"] / HBM_PEAK_GBPS, 4)
                             if head["user_GBps_busy"] else None)
    _progress("serve: rate %.0f p50 %.3f ms p99 %.3f ms" % (rate, head["p50_ms"], head["p99_ms"]))
    runs = []
    for r2 in sweep:
        scale = rate / r2 if r2 > 0 else 0.0
        b0, h0 = srv.cache.builds, srv.cache.hits
        st = srv.run(_fresh(reqs, Request), time_scale=scale)
        st["graph_builds"] -= b0
        st["graph_hits"] -= h0
        st["rate_offered"] = r2 if r2 > 0 else "all_at_once"
        st.pop("by_kind", None)
        runs.append(st)
        _progress("serve: rate %s p50 %.3f ms p99 %.3f ms busy %.1f GB/s"
                  % (st["rate_offered"], st["p50_ms"], st["p99_ms"], st["user_GBps_busy"] or 0))
    srv.close()
    mix = {}
    for r in reqs:
        mix[r.kind] = mix.get(r.kind, 0) + 1
    return {
        "workload": "serving",
        "trace": {"rate_per_s": rate, "duration_s": duration, "requests": len(reqs), "mix": mix,
                  "pool_stripes": pool_size,
                  "encode_input_GB": round(sum(r.x.numel() for r in reqs if r.kind == "encode") / 1e9, 2)},
        "headline": head,
        "saturation_sweep": runs,
    }
