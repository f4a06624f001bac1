"""Device inputs of the serving workload: the resident pool and the requests
of a trace, as tensors ready before the clock starts.

  pool stripe s    x = payload of stripe 1_000_000 + s (seeded uniform
                   bytes, the tail of the last block zeroed), c = its
                   encoding by the library under test
  encode r         x = payload of stripe 2_000_000 + r, zero-padded likewise
  decode r         erased = 5 % of the target's coded rows, erasure stream of
                   stripe 3_000_000 + r
  repair r         1-4 lost coded rows, repair stream of stripe 3_000_000 + r
  update r         1 % (at least 1) of the target's inputs, update-id stream
                   of stripe 3_000_000 + r; new contents = blocks 0.. of the
                   update-data stream of that stripe

Graphs of serving stripes are shared per (k, n): stripe key 0, graph seed 1.
Nothing here does coding arithmetic.
"""

import numpy as np

from . import gen, workloads


def graph_params(sp):
    return dict(k=sp.k, n=sp.n, dist="rsd", rsd_c=sp.rsd_c, rsd_delta=sp.rsd_delta, finite_w=(),
                seed=sp.graph_seed, stripe_key=0)


def payload_tensor(sp, device="cuda"):
    """x[k][t] holding sp.extra['payload'] seeded bytes, the rest zero."""
    import torch
    from . import gpu as synth_gpu
    x = torch.empty((sp.k, sp.t), dtype=torch.uint8, device=device)
    synth_gpu.fill(x, workloads.DATA_SEED, sp.stripe, sp.t)
    P = sp.extra.get("payload", sp.k * sp.t)
    if P < sp.k * sp.t:
        x.view(-1)[P:].zero_()
    return x


def build_pool(server, count, hi=256 << 20, device="cuda"):
    """Resident stripes 0..count-1 registered with `server`; returns their specs."""
    specs = workloads.serving_pool(count, hi=hi)
    for i, sp in enumerate(specs):
        x = payload_tensor(sp, device)
        p = graph_params(sp)
        c = server.encode_now(p, x, sp.t)
        server.add_stripe(i, p, x, c, sp.t)
    return specs


def build_requests(trace, pool_specs, Request, device="cuda", hi=256 << 20):
    """Request objects (class `Request` of the server) for a trace."""
    import torch
    from . import gpu as synth_gpu
    out = []
    for tr in trace:
        rid, kind = tr["id"], tr["type"]
        key = 3_000_000 + rid
        if kind == "encode":
            sp = workloads.serve_stripe(2_000_000 + rid, tr["payload"], tr["block"])
            out.append(Request("encode", arrival=tr["t"], params=graph_params(sp), t=sp.t,
                               x=payload_tensor(sp, device), rid=rid))
            continue
        sp = pool_specs[tr["target"]]
        if kind == "decode":
            m = gen.erasure_mask(workloads.ERASE_SEED, key, sp.n, gen.round_half_up(0.05 * sp.n))
            out.append(Request("decode", arrival=tr["t"], t=sp.t, stripe=tr["target"],
                               erased=torch.from_numpy(m).to(device), rid=rid))
        elif kind == "repair":
            lost = np.array(gen.repair_lost(workloads.REPAIR_SEED, key, sp.n), np.uint32)
            out.append(Request("repair", arrival=tr["t"], t=sp.t, stripe=tr["target"],
                               ids=torch.from_numpy(lost).to(device), rid=rid))
        else:
            nu = max(1, gen.round_half_up(0.01 * sp.k))
            ids = np.array(gen.update_ids(workloads.UPDATE_IDS_SEED, key, sp.k, nu), np.uint32)
            new = torch.empty((len(ids), sp.t), dtype=torch.uint8, device=device)
            synth_gpu.fill(new, workloads.UPDATE_DATA_SEED, key, sp.t, purpose=synth_gpu.UPDATE_DATA)
            out.append(Request("update", arrival=tr["t"], t=sp.t, stripe=tr["target"],
                               ids=torch.from_numpy(ids).to(device), new_blocks=new, rid=rid))
    return out
