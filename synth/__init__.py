"""Seeded synthetic inputs shared by the tests, the oracle runs and the benchmark.

This module generates INPUTS only: payload bytes, erasure patterns, lost-row
lists, update ids and blocks, and workload manifests.  It holds none of the
coding arithmetic (no degree sampling, no graph, no XOR of blocks) and imports
neither the oracle nor the library, so both sides can consume the same inputs
without sharing code.

Streams follow one counter-based definition (SplitMix64's output mixer,
Steele, Lea & Flood 2014; constants of Stafford's "Mix13"):
  key(seed, purpose, a, b) = mix(mix(mix(mix(seed + G) ^ purpose) ^ a) ^ b)
  draw i = mix(key + (i + 1) G),  G = 0x9E3779B97F4A7C15
with purposes
  2 DATA (stripe, block)     3 ERASE (stripe, 0)     4 REPAIR (stripe, 0)
  5 UPDATE_IDS (stripe, 0)   6 UPDATE_DATA (stripe, block)
  7 WORKLOAD (workload id, item)   8 ARRIVAL (0, request)
(purpose 1 belongs to the code's graph and is not generated here).
"""

from .gen import (  # noqa: F401
    mix64, stream_key, draw, draws_np, payload, payload_slice, sample_distinct,
    erasure_ids, erasure_mask, repair_lost, update_ids, update_blocks,
    overhead_n, round_half_up, uniform01,
)
from . import workloads  # noqa: F401
