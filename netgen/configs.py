"""Named workload recipes.

* ``small_net``      - 1,000 neurons in 2 regions (80/20 E/I), in-degree 100
                       (70 own-region + 30 other-region), delays 1-5 steps.
* ``partition_net``  - one GPU's partition: 90 regions with log-normal sizes,
                       a seeded region-to-region matrix with ~10 % non-zeros
                       and heavy-tailed row sums, in-degree 100, delays 1-20.
                       Full size is 20,000,000 neurons / 2e9 synapses; any
                       smaller ``n`` gives the same construction scaled down.
* ``ensemble_member`` - one member of the 64-network batched ensemble
                       (20 regions, 50k-400k neurons, same construction).

The LIF constants are the ones of the model of Sec. III-B with the values of
the workload description (C=1, gL=0.03, EL=-75, Vth=-50, Vreset=-65 mV,
2 ms refractory, tau = 2/40/10/50 ms, E = 0/0/-70/-100 mV, dt = 1 ms).
The channel conductances are not printed in the paper (it tunes g_AMPA and
g_NMDA to set the rate, Sec. VII-A); the values below were fixed once by
bisecting a common scale on g_AMPA and g_NMDA with the FP64 reference on the
1,000-neuron net until its mean rate fell in 5-10 Hz, then frozen.
"""
from __future__ import annotations

import numpy as np

from . import NetSpec, make_network

# conductances (AMPA, NMDA, GABAa, GABAb); see module docstring
G_DEFAULT = (0.023125, 0.00115625, 0.32, 0.008)

# background drive (mean Poisson count per neuron-step) giving ~7/15/30 Hz on
# the partition network; fixed by bisection on the mean rate, then frozen
PARTITION_LAMBDA = {7: 0.27346, 15: 0.56492, 30: 1.52745}

FULL_PARTITION_N = 20_000_000


def lognormal_region_sizes(n: int, n_regions: int, sigma: float, floor: int, seed: int) -> np.ndarray:
    """Region sizes proportional to LogNormal(0, sigma) draws, each at least
    ``floor``, rounded by largest remainder so that they sum exactly to n."""
    rng = np.random.default_rng(seed)
    x = rng.lognormal(0.0, sigma, n_regions)
    rest = n - floor * n_regions
    if rest < 0:
        raise ValueError("n too small for the region floor")
    share = x / x.sum() * rest
    base = np.floor(share).astype(np.int64)
    rem = int(rest - base.sum())
    order = np.argsort(-(share - base), kind="stable")
    base[order[:rem]] += 1
    return base + floor


def region_matrix(n_regions: int, p_offdiag: float, src_sigma: float, seed: int) -> np.ndarray:
    """M[s, t] = weight of source region s onto target region t: off-diagonal
    entries present with probability p, value LogNormal(0, 1) times a
    per-source multiplier LogNormal(0, src_sigma) (heavy-tailed out-strength).
    The diagonal is marked present; in-region synapses are drawn separately."""
    rng = np.random.default_rng(seed)
    present = rng.random((n_regions, n_regions)) < p_offdiag
    np.fill_diagonal(present, True)
    vals = rng.lognormal(0.0, 1.0, (n_regions, n_regions))
    rho = rng.lognormal(0.0, src_sigma, n_regions)
    return present * vals * rho[:, None]


def small_net(seed_offset: int = 0, n: int = 1000, bg_lambda: float = 0.25,
              g=G_DEFAULT, max_delay: int = 5, k_in: int = 70, k_cross: int = 30):
    """The 1,000-neuron, 2-region net (sizes can be shrunk for brute-force
    tests; n must be even).  seed_offset > 0 gives the pooled-test seeds."""
    if n % 2:
        raise ValueError("n must be even")
    half = n // 2
    s = 0 if seed_offset == 0 else 10_000 + seed_offset
    spec = NetSpec(n=n, region_sizes=np.array([half, half], dtype=np.int64),
                   cross_w=np.array([[0.0, 1.0], [1.0, 0.0]]), k_in=k_in, k_cross=k_cross,
                   max_delay=max_delay, net_seed=1 + 3 * s, v0_seed=2 + 3 * s, bg_seed=3 + 3 * s,
                   bg_lambda=bg_lambda, g=tuple(g), name=f"small_net(n={n},seed={seed_offset})")
    return spec


def partition_spec(n: int = FULL_PARTITION_N, rate_hz: int = 7, n_regions: int = 90,
                   seeds=(11, 12, 13), bg_lambda=None, max_delay: int = 20, g=G_DEFAULT,
                   member: int = 0, name: str = "") -> NetSpec:
    floor = max(10, int(round(1000 * n / FULL_PARTITION_N)))
    sizes = lognormal_region_sizes(n, n_regions, 1.0, floor, seed=seeds[0] * 7919 + 1)
    p = 720.0 / (n_regions * n_regions - n_regions) if n_regions > 1 else 0.0
    M = region_matrix(n_regions, p, 0.74, seed=seeds[0] * 7919 + 2)
    lam = PARTITION_LAMBDA[rate_hz] if bg_lambda is None else bg_lambda
    return NetSpec(n=n, region_sizes=sizes, cross_w=M, k_in=70, k_cross=30, max_delay=max_delay,
                   net_seed=seeds[0], v0_seed=seeds[1], bg_seed=seeds[2], bg_lambda=lam,
                   g=tuple(g), member=member,
                   name=name or f"partition_net(n={n},R={n_regions},rate={rate_hz}Hz)")


def slice_spec(rate_hz: int = 7, n: int = 200_000, **kw) -> NetSpec:
    """The independent 200k-neuron slice built by the partition generator."""
    return partition_spec(n=n, rate_hz=rate_hz, seeds=(21, 22, 23), **kw)


def ensemble_sizes(n_members: int = 64, lo: int = 50_000, hi: int = 400_000, seed: int = 31) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, n_members).astype(np.int64)


def ensemble_gains(n_members: int = 64, n_regions: int = 20, seed: int = 32, sd: float = 0.2) -> np.ndarray:
    """Per-(member, region, channel) conductance gains ~ N(1, sd^2), clipped at 0."""
    rng = np.random.default_rng(seed)
    return np.clip(rng.normal(1.0, sd, (n_members, n_regions, 4)), 0.0, None).astype(np.float32)


def ensemble_member_spec(m: int, n_m: int, rate_hz: int = 7, n_regions: int = 20) -> NetSpec:
    return partition_spec(n=int(n_m), rate_hz=rate_hz, n_regions=n_regions,
                          seeds=(3100 + m, 3100 + m, 3100 + m), member=m,
                          name=f"ensemble_member({m},n={n_m})")


__all__ = ["G_DEFAULT", "PARTITION_LAMBDA", "FULL_PARTITION_N", "lognormal_region_sizes",
           "region_matrix", "small_net", "partition_spec", "slice_spec", "ensemble_sizes",
           "ensemble_gains", "ensemble_member_spec"]
