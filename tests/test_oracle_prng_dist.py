"""Pins of the oracle's random streams and degree distributions (CPU only)."""

import math

import numpy as np
import pytest
from scipy import stats

from oracle import dist, prng


def test_splitmix64_published_sequence(golden):
    g = golden("splitmix64_seed0.json")
    state = 0
    got = []
    for _ in range(3):
        state = (state + prng.GOLDEN) & prng.MASK64
        got.append(prng.mix64(state))
    assert got == [int(h, 16) for h in g["outputs_hex"]]


def test_stream_numpy_matches_int_path():
    for seed, purpose, a, b in [(0, 1, 0, 0), (1389488782, 1, 7, 123), (2**63 + 5, 1, 2**40, 99)]:
        key = prng.stream_key(seed, purpose, a, b)
        want = [prng.draw(key, i) for i in range(50)]
        got = prng.draws_np(key, 0, 50)
        assert [int(v) for v in got] == want
        got2 = prng.draws_np(key, 17, 10)
        assert [int(v) for v in got2] == want[17:27]


def test_streams_distinct_per_coordinate():
    base = prng.stream_key(1, 1, 0, 0)
    for other in [prng.stream_key(2, 1, 0, 0), prng.stream_key(1, 2, 0, 0),
                  prng.stream_key(1, 1, 1, 0), prng.stream_key(1, 1, 0, 1)]:
        assert other != base


def harmonic(m):
    return sum(1.0 / i for i in range(1, m + 1))


@pytest.mark.parametrize("k,c,delta", [(1, 0.1, 0.05), (2, 0.1, 0.05), (64, 0.1, 0.05),
                                       (500, 0.1, 0.05), (1024, 0.1, 0.05), (4096, 0.1, 0.05),
                                       (724, 0.05, 0.01), (8192, 0.05, 0.01), (100, 0.5, 0.5)])
def test_rsd_beta_closed_form(k, c, delta):
    # sum of rho telescopes to exactly 1, so beta = 1 + sum(tau)
    w, R, M = dist.rsd_weights(k, c, delta)
    beta = math.fsum(w[1:])
    closed = 1.0 + (R / k) * (harmonic(M - 1) + math.log(R / delta))
    assert abs(beta - closed) < 1e-12 * closed
    rho_sum = math.fsum([1.0 / k] + [1.0 / (i * (i - 1)) for i in range(2, k + 1)])
    assert abs(rho_sum - 1.0) < 1e-13
    p = dist.probabilities(w)
    assert abs(math.fsum(p[1:]) - 1.0) < 1e-12
    assert M == max(1, min(k, int(k // R)))


@pytest.mark.parametrize("k,c,delta,M,beta,dbar", [
    (64, 0.1, 0.05, 11, 1.68589, 6.110),
    (1024, 0.1, 0.05, 32, 1.32516, 11.227),
    (4096, 0.1, 0.05, 56, 1.20986, 14.111),
    (64, 0.05, 0.01, 18, 1.50936, 7.588),
    (8192, 0.05, 0.01, 132, 1.10668, 17.383),
])
def test_rsd_known_values(k, c, delta, M, beta, dbar):
    w, R, M_got = dist.rsd_weights(k, c, delta)
    assert M_got == M
    assert abs(sum(w[1:]) - beta) < 6e-6
    assert abs(dist.mean_degree(w) - dbar) < 6e-4


def test_rsd_rejects_bad_parameters():
    for args in [(0, 0.1, 0.05), (10, 0.0, 0.05), (10, 0.1, 0.0), (10, 0.1, 1.0)]:
        with pytest.raises(dist.DistError):
            dist.rsd_weights(*args)
    with pytest.raises(dist.DistError):      # R/delta <= 1: non-positive spike
        dist.rsd_weights(1, 0.001, 0.9)


def test_finite16_table():
    w_in = [0.02] + [1.0 / (d * (d - 1)) for d in range(2, 17)]
    w = dist.finite_weights(w_in, 4096)
    W = sum(w[1:])
    assert abs(W - (0.02 + 1.0 - 1.0 / 16)) < 1e-15          # telescoping: 0.9575
    p = dist.probabilities(w)
    assert abs(p[1] - 0.0208877) < 5e-8
    assert abs(p[2] - 0.522193) < 5e-7
    assert abs(p[16] - 0.0043516) < 5e-8
    assert abs(dist.mean_degree(w) - 3.48640) < 5e-6
    # truncation to k renormalises over the kept degrees
    w4 = dist.finite_weights(w_in, 4)
    assert len(w4) == 5 and abs(sum(dist.probabilities(w4)[1:]) - 1.0) < 1e-15


def test_raptor_omega_as_printed():
    assert abs(sum(dist.RAPTOR_OMEGA.values()) - 0.999998) < 1e-12
    w = dist.raptor_weights(1000)
    assert len(w) == 66 and w[65] == 0.003135 and w[6] == 0.0
    assert abs(dist.mean_degree(w) - 5.842) < 5e-4
    # degrees above k are dropped
    assert len(dist.raptor_weights(20)) == 21


def test_thresholds_and_sampling_boundaries():
    w, _, _ = dist.rsd_weights(64, 0.1, 0.05)
    T = dist.thresholds(w)
    assert len(T) == 64 and T[-1] == 2**53
    assert all(a <= b for a, b in zip(T, T[1:]))
    for d in [1, 2, 11, 12, 64]:
        lo = T[d - 2] if d > 1 else 0
        if T[d - 1] > lo:
            assert dist.sample_degree(lo << 11, T) == d
            assert dist.sample_degree(((T[d - 1] - 1) << 11) | 0x7FF, T) == d
    # zero-weight degrees are never drawn
    wf = dist.finite_weights([0.5, 0.0, 0.5], 10)
    Tf = dist.thresholds(wf)
    assert Tf[0] == Tf[1]
    rng = np.random.default_rng(0)
    for u in rng.integers(0, 2**63, size=2000, dtype=np.uint64):
        assert dist.sample_degree(int(u) * 2, Tf) in (1, 3)


def test_degree_sampler_chi_square():
    w, _, _ = dist.rsd_weights(64, 0.1, 0.05)
    T = dist.thresholds(w)
    p = np.array(dist.probabilities(w)[1:])
    key = prng.stream_key(99, 1, 0, 0)
    u = prng.draws_np(key, 0, 200000)
    # vectorised inverse CDF, checked against the scalar scan on a prefix
    d = np.searchsorted(np.array(T, dtype=np.uint64), u >> np.uint64(11), side="right") + 1
    for i in range(500):
        assert d[i] == dist.sample_degree(int(u[i]), T)
    counts = np.bincount(d, minlength=65)[1:]
    exp = p * len(u)
    keep = exp >= 5
    obs, ex = counts[keep], exp[keep]
    if (~keep).any():
        obs = np.append(obs, counts[~keep].sum())
        ex = np.append(ex, exp[~keep].sum())
    chi2 = float(((obs - ex) ** 2 / ex).sum())
    assert stats.chi2.sf(chi2, len(obs) - 1) > 1e-4
