"""Degree distributions of the LDGM base code (oracle copy).

§1 of the paper: the code supports the Robust Soliton Distribution of Luby's
LT codes and any finite max-degree distribution, by default the Raptor
distribution Omega(x) printed in §2.2.  A coded symbol's degree d is drawn from
the distribution and d distinct input symbols are then chosen (§2.2).

The paper only cites the Robust Soliton Distribution, so its definition here
is Luby's (FOCS 2002), with k inputs, constants c > 0 and 0 < delta < 1:

  R      = c * ln(k / delta) * sqrt(k)
  M      = floor(k / R), clamped to [1, k]           (the spike position)
  rho(1) = 1/k,   rho(i) = 1 / (i (i - 1))           for 2 <= i <= k
  tau(i) = R / (i k)                                 for 1 <= i < M
  tau(M) = R ln(R / delta) / k,  tau(i) = 0          for i > M
  beta   = sum_i (rho(i) + tau(i)),  mu(i) = (rho(i) + tau(i)) / beta

Reading taken (the paper prints no formula): the spike sits at floor(k/R); a
parameter set with R/delta <= 1 (a non-positive spike) is rejected.

Sampling uses integer thresholds so that the oracle and the library agree bit
for bit: weights are summed in float64 in order d = 1..D into W, p_d = w_d / W,
C_d is the running sum of the p_d, T_d = min(2**53, floor(C_d * 2**53)) for
d < D and T_D = 2**53.  A draw u picks d = min{d : (u >> 11) < T_d}.  Degrees
above k are impossible for RSD and are cut from finite tables (renormalising).

Scalar ``math.log`` / ``math.sqrt`` are used on purpose (libm, like the C side).

Pinned by: the telescoping closed form beta = 1 + (R/k)(H_{M-1} + ln(R/delta)),
the printed Omega coefficients (their sum is 0.999998), and a chi-square test
of sampled degrees against mu.
"""

import math

TWO53 = 1 << 53

# Raptor degree distribution printed in §2.2 (Omega_i for the listed i).
RAPTOR_OMEGA = {
    1: 0.007969, 2: 0.49357, 3: 0.16622, 4: 0.072646, 5: 0.082558,
    8: 0.056058, 9: 0.037229, 19: 0.05559, 64: 0.025023, 65: 0.003135,
}


class DistError(ValueError):
    pass


def rsd_weights(k, c, delta):
    """Unnormalised Robust Soliton weights w_1..w_k (index 0 unused).

    Returns (w, R, M) with w[d] = rho(d) + tau(d); beta = sum(w[1:]).
    """
    if k < 1 or not (c > 0.0) or not (0.0 < delta < 1.0):
        raise DistError("RSD needs k >= 1, c > 0, 0 < delta < 1")
    R = c * math.log(k / delta) * math.sqrt(k)
    if not (R / delta > 1.0):
        raise DistError("RSD needs R/delta > 1")
    M = int(math.floor(k / R))
    M = max(1, min(k, M))
    w = [0.0] * (k + 1)
    for i in range(1, k + 1):
        rho = 1.0 / k if i == 1 else 1.0 / (i * (i - 1))
        if i < M:
            tau = R / (i * k)
        elif i == M:
            tau = R * math.log(R / delta) / k
        else:
            tau = 0.0
        w[i] = rho + tau
    return w, R, M


def finite_weights(weights, k):
    """Finite max-degree table: weights[d-1] is w_d for d = 1..D.

    Degrees above k are dropped (a coded symbol cannot have more than k
    distinct neighbours).  Returns w with w[d] for d = 1..min(D, k).
    """
    if len(weights) < 1:
        raise DistError("empty finite table")
    if any((not (x >= 0.0)) or math.isinf(x) for x in weights):
        raise DistError("finite weights must be finite and >= 0")
    D = min(len(weights), k)
    w = [0.0] + [float(x) for x in weights[:D]]
    if not (sum(w) > 0.0):
        raise DistError("finite table has no mass at degrees <= k")
    return w


def raptor_weights(k):
    """The Raptor Omega of §2.2 as a finite table (renormalised on use)."""
    D = max(RAPTOR_OMEGA)
    tab = [RAPTOR_OMEGA.get(d, 0.0) for d in range(1, D + 1)]
    return finite_weights(tab, k)


def probabilities(w):
    """p_d = w_d / W with W summed in order d = 1..D (index 0 unused)."""
    W = 0.0
    for d in range(1, len(w)):
        W += w[d]
    return [0.0] + [w[d] / W for d in range(1, len(w))]


def thresholds(w):
    """Integer CDF thresholds T_1..T_D (list index d-1 holds T_d)."""
    p = probabilities(w)
    D = len(w) - 1
    T = []
    C = 0.0
    for d in range(1, D + 1):
        C += p[d]
        if d < D:
            T.append(min(TWO53, int(math.floor(C * TWO53))))
        else:
            T.append(TWO53)
    return T


def sample_degree(u0, T):
    """Smallest d with (u0 >> 11) < T_d, by a plain linear scan."""
    v = u0 >> 11
    for d, td in enumerate(T, start=1):
        if v < td:
            return d
    raise AssertionError("last threshold is 2**53; unreachable")


def mean_degree(w):
    p = probabilities(w)
    return sum(d * p[d] for d in range(1, len(p)))
