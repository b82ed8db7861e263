"""Pins of the reference's Ornstein-Uhlenbeck background (the paper's own
input model, Sec. III-B: uncorrelated OU currents I_ou on every neuron).

* the Gaussian draws are normal (moments, Kolmogorov-Smirnov against scipy)
  and their Philox words are numpy's Philox at counter (t, i, member, 1);
* the process has the closed-form moments of the exact discretisation:
  E[I_ou^t] = mu, Var[I_ou^t] = sigma^2 (1 - a^(2t)) from I_ou^0 = mu, and
  lag-one correlation a = exp(-dt/tau) in the stationary regime;
* with sigma = 0 it is a constant current mu, i.e. the same network with
  Iext + mu and no background.
"""
import dataclasses

import numpy as np
import pytest
import scipy.stats

import netgen
import oracle


def test_ou_normals_are_box_muller_on_numpy_philox_stream_1():
    seed = 12345
    for t, i, m in [(0, 0, 0), (5, 17, 0), (999, 123456, 3), (2**33, 7, 1)]:
        ctr = [t, i, m, 1]
        c = sum(int(x) << (64 * k) for k, x in enumerate(ctr)) - 1
        prev = [(c >> (64 * k)) & (2**64 - 1) for k in range(4)]
        raw = np.random.Philox(key=np.array([seed, 0], dtype=np.uint64),
                               counter=np.array(prev, dtype=np.uint64)).random_raw(4)
        u1 = (float(int(raw[0]) >> 32) + 1.0) / 2**32
        u2 = float(int(raw[1]) >> 32) / 2**32
        assert oracle.ou_normal(seed, t, i, m) == pytest.approx(
            np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2), rel=1e-14, abs=1e-14)


def test_ou_normals_are_standard_normal():
    x = np.array([oracle.ou_normal(77, t, i, 0) for t in range(40) for i in range(2500)])
    n = len(x)
    assert abs(x.mean()) < 5.0 / np.sqrt(n)
    assert abs(x.var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
    assert scipy.stats.kstest(x, "norm").pvalue > 1e-4
    # draws of different neurons, steps and members are not the same numbers
    assert oracle.ou_normal(77, 3, 4, 0) != oracle.ou_normal(77, 3, 4, 1)
    assert oracle.ou_normal(77, 3, 4, 0) != oracle.ou_normal(77, 4, 3, 0)


def test_ou_moments_follow_the_exact_discretisation():
    net = netgen.make_network(netgen.small_net(n=2000, bg_lambda=0.0))
    mu, sigma, tau = 0.3, 0.25, 10.0
    a = np.exp(-net.dt_ms / tau)
    o = oracle.OracleNet(net)
    o.set_ou(mu, sigma, tau)
    np.testing.assert_array_equal(o.get("I_ou"), mu)
    hist = []
    for t in range(1, 401):
        o.step()
        x = o.get("I_ou")
        hist.append(x)
        if t in (1, 5, 20, 200, 400):
            var = sigma**2 * (1.0 - a ** (2 * t))
            se = var * np.sqrt(2.0 / net.n)
            assert abs(x.var() - var) < 6 * se, (t, x.var(), var)
            assert abs(x.mean() - mu) < 6 * np.sqrt(var / net.n), (t, x.mean())
    H = np.array(hist[200:]) - mu
    lag1 = np.sum(H[1:] * H[:-1]) / np.sum(H[:-1] * H[:-1])
    assert abs(lag1 - a) < 0.01, (lag1, a)


def test_ou_with_zero_sigma_is_a_constant_current():
    base = netgen.make_network(netgen.small_net(bg_lambda=0.0))
    mu = 0.875                           # V_inf = EL + mu / gL = -45.8 mV: tonic firing
    o1 = oracle.OracleNet(base)
    o1.set_ou(mu, 0.0, 5.0)
    pt = base.ptypes.copy()
    pt[:, 6] += mu                       # Iext + mu, exact in float32 (Iext = 0)
    assert np.all(pt[:, 6] == np.float32(mu))
    o2 = oracle.OracleNet(dataclasses.replace(base, ptypes=pt))
    r1 = o1.run(150, want_state=True)
    r2 = o2.run(150, want_state=True)
    np.testing.assert_array_equal(r1["raster"], r2["raster"])
    assert r1["raster"].sum() > 0
    np.testing.assert_array_equal(o1.get("V"), o2.get("V"))
    np.testing.assert_array_equal(o1.get("I_ou"), mu)
    assert np.all(r1["ev_bg"] == 0)
