"""Named synthetic workloads (shapes, distributions, seeds).

Each workload is described by plain parameters; the coding itself is done
elsewhere.  Payloads are uniform random bytes: XOR cost does not depend on
content, so seeded uniform bytes stand in for the paper's unspecified files.

  tiny          1 stripe, k=64 x 4 KiB, n=96, Robust Soliton (c=0.1, delta=0.05),
                16 coded rows erased
  large_stripe  1 stripe, k=4096 x 64 KiB (256 MiB), n=4506 (10 % overhead),
                finite max-degree 16 table w_1 = 0.02, w_d = 1/(d(d-1)),
                225 coded rows erased (5 %)
  batch512      512 stripes, k log-uniform in [64, 8192), block size 4 KiB..1 MiB
                (powers of two), RSD (c=0.05, delta=0.01), 8 % overhead,
                4 % erasures
  resident256   256 stripes, k=1024 x 256 KiB, n=1126, RSD (c=0.1, delta=0.05);
                1-4 lost coded rows per stripe, 10 updated inputs per stripe
  serving       Poisson arrivals of encode / decode / repair / update requests
                (50/30/15/5 %), payloads log-uniform in [64 KiB, 256 MiB),
                blocks of 16, 64 or 256 KiB, k = ceil(P / B), n = max(k+1,
                round(1.1 k)), RSD (c=0.1, delta=0.05); decode, repair and
                update target a resident pool of 256 such stripes
"""

from dataclasses import dataclass, field, replace
import math

from . import gen

DATA_SEED = 0
GRAPH_SEED = 1
ERASE_SEED = 2
BATCH_MANIFEST_SEED = 3
REPAIR_SEED = 4
UPDATE_IDS_SEED = 5
UPDATE_DATA_SEED = 6
SERVE_SEED = 7

BATCH_WORKLOAD_ID = 3


def finite16_weights():
    """w_1 = 0.02, w_d = 1/(d(d-1)) for 2 <= d <= 16 (normalised together on use)."""
    return tuple([0.02] + [1.0 / (d * (d - 1)) for d in range(2, 17)])


@dataclass
class StripeSpec:
    stripe: int              # stripe id: selects the data / erasure streams
    k: int
    n: int
    t: int                   # block bytes
    dist: str = "rsd"        # "rsd" | "finite" | "raptor"
    rsd_c: float = 0.1
    rsd_delta: float = 0.05
    finite_w: tuple = ()
    graph_seed: int = GRAPH_SEED
    stripe_key: int = 0
    data_seed: int = DATA_SEED
    erase_seed: int = ERASE_SEED
    n_erased: int = 0
    extra: dict = field(default_factory=dict)

    def graph_kwargs(self):
        return dict(k=self.k, n=self.n, dist=self.dist, rsd_c=self.rsd_c,
                    rsd_delta=self.rsd_delta, finite_w=tuple(self.finite_w),
                    seed=self.graph_seed, stripe_key=self.stripe_key)

    def x(self):
        return gen.payload(self.data_seed, self.stripe, self.k, self.t)

    def x_slice(self, blocks, lo, hi):
        return gen.payload_slice(self.data_seed, self.stripe, blocks, lo, hi)

    def erased_ids(self):
        return gen.erasure_ids(self.erase_seed, self.stripe, self.n, self.n_erased)

    def erased_mask(self):
        return gen.erasure_mask(self.erase_seed, self.stripe, self.n, self.n_erased)

    @property
    def input_bytes(self):
        return self.k * self.t

    @property
    def coded_bytes(self):
        return self.n * self.t


def tiny():
    return StripeSpec(stripe=0, k=64, n=96, t=4096, dist="rsd", rsd_c=0.1, rsd_delta=0.05,
                      n_erased=16)


def large_stripe():
    n = gen.overhead_n(4096, 0.10)
    return StripeSpec(stripe=0, k=4096, n=n, t=65536, dist="finite",
                      finite_w=finite16_weights(), n_erased=gen.round_half_up(0.05 * n))


def scaled(spec, t):
    """Same code and erasures with a different block size (for CPU-sized parity runs)."""
    return replace(spec, t=t)


def batch512(count=512):
    """Manifest of the heterogeneous batch: per stripe k, n, t, erasures.

    Stripe s draws U, U' from key(3, WORKLOAD, 3, s):
      k = floor(64 * 2**(7 U)),  t = 4096 * 2**floor(9 U'),
      n = round(1.08 k),         erased = round(0.04 n).
    Each stripe has its own graph (stripe key = s).
    """
    out = []
    for s in range(count):
        key = gen.stream_key(BATCH_MANIFEST_SEED, gen.WORKLOAD, BATCH_WORKLOAD_ID, s)
        U = gen.uniform01(gen.draw(key, 0))
        U2 = gen.uniform01(gen.draw(key, 1))
        k = int(math.floor(64.0 * 2.0 ** (7.0 * U)))
        t = 4096 * (1 << int(math.floor(9.0 * U2)))
        n = gen.overhead_n(k, 0.08)
        out.append(StripeSpec(stripe=s, k=k, n=n, t=t, dist="rsd", rsd_c=0.05,
                              rsd_delta=0.01, stripe_key=s,
                              n_erased=gen.round_half_up(0.04 * n)))
    return out


def resident256(count=256):
    """Resident batch for repair and update: identical shapes, one graph per stripe."""
    out = []
    for s in range(count):
        sp = StripeSpec(stripe=s, k=1024, n=1126, t=262144, dist="rsd", rsd_c=0.1,
                        rsd_delta=0.05, stripe_key=s)
        sp.extra["lost"] = gen.repair_lost(REPAIR_SEED, s, sp.n)
        sp.extra["update_ids"] = gen.update_ids(UPDATE_IDS_SEED, s, sp.k,
                                                max(1, gen.round_half_up(0.01 * sp.k)))
        out.append(sp)
    return out


# ---------------------------------------------------------------- serving

SERVE_MIX = (("encode", 0.50), ("decode", 0.30), ("repair", 0.15), ("update", 0.05))
SERVE_BLOCKS = (16 << 10, 64 << 10, 256 << 10)


def serve_stripe(stripe, payload, block):
    """A stripe holding `payload` bytes in blocks of `block` bytes (the last
    block zero-padded): k = ceil(P / B), n = max(k + 1, round(1.1 k)),
    Robust Soliton (c = 0.1, delta = 0.05); stripes of equal (k, n) share
    one graph (stripe key 0)."""
    k = max(1, -(-payload // block))
    n = max(k + 1, gen.overhead_n(k, 0.10))
    return StripeSpec(stripe=stripe, k=k, n=n, t=block, dist="rsd", rsd_c=0.1, rsd_delta=0.05,
                      stripe_key=0, n_erased=gen.round_half_up(0.05 * n),
                      extra={"payload": payload})


def serve_payload(u, lo=64 << 10, hi=256 << 20):
    """Log-uniform payload size in [lo, hi)."""
    return int(math.floor(lo * (hi / lo) ** u))


def serving_pool(count=256, seed=SERVE_SEED, hi=256 << 20):
    """Resident stripes targeted by decode, repair and update requests."""
    out = []
    for s in range(count):
        key = gen.stream_key(seed, gen.WORKLOAD, 5, s)
        P = serve_payload(gen.uniform01(gen.draw(key, 0)), hi=hi)
        B = SERVE_BLOCKS[int(gen.uniform01(gen.draw(key, 1)) * len(SERVE_BLOCKS))]
        out.append(serve_stripe(1_000_000 + s, P, B))
    return out


def serving_trace(rate=2000.0, duration=1.0, seed=SERVE_SEED, pool_size=256, hi=256 << 20):
    """Requests with Poisson arrivals at `rate` per second over `duration` s.

    Request r draws from key(seed, ARRIVAL, 0, r): u0 the exponential gap,
    u1 the type (50/30/15/5 % encode/decode/repair/update), u2 the payload
    (encode) or the target stripe of the pool (others), u3 the block size.
    Decode erases 5 % of the target's coded blocks; repair loses 1-4 coded
    blocks; update rewrites 1 % (at least one) of the target's inputs.
    """
    reqs, t, r = [], 0.0, 0
    while True:
        key = gen.stream_key(seed, gen.ARRIVAL, 0, r)
        u = [gen.uniform01(gen.draw(key, i)) for i in range(4)]
        t += -math.log(1.0 - u[0]) / rate
        if t >= duration:
            break
        acc, kind = 0.0, SERVE_MIX[-1][0]
        for name, p in SERVE_MIX:
            acc += p
            if u[1] < acc:
                kind = name
                break
        req = {"id": r, "t": t, "type": kind}
        if kind == "encode":
            req["payload"] = serve_payload(u[2], hi=hi)
            req["block"] = SERVE_BLOCKS[int(u[3] * len(SERVE_BLOCKS))]
        else:
            req["target"] = int(u[2] * pool_size)
        reqs.append(req)
        r += 1
    return reqs
