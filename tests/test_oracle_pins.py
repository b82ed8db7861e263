"""Pins of the FP64 reference against things other than itself: library
routines (numpy's Philox, scipy's Poisson CDF), closed forms of the model of
Sec. III-B Eq. (1) under forward Euler (Sec. VI-A), integer invariants of the
spike delivery, and a dense brute-force formulation on tiny nets."""
import json
import math
import os

import numpy as np
import pytest
import scipy.stats

import netgen
import oracle
from oracle import brute
from nethelpers import hand_net

GOLDEN = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "worked_examples.json")))


# ---------------------------------------------------------------- RNG / Poisson

@pytest.mark.parametrize("ctr,key", [
    ((1, 0, 0, 0), (5, 0)),
    ((7, 123456, 3, 0), (13, 0)),
    ((0, 1, 0, 0), (2**64 - 1, 0)),          # 256-bit borrow into word 0
    ((2**40 + 3, 2**33, 2**20, 5), (0xDEADBEEF, 77)),
])
def test_philox_matches_numpy(ctr, key):
    c = sum(int(x) << (64 * k) for k, x in enumerate(ctr)) - 1
    prev = [(c >> (64 * k)) & (2**64 - 1) for k in range(4)]
    ref = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(prev, dtype=np.uint64)).random_raw(4)
    got = oracle.philox4x64_10(ctr, key)
    assert [int(x) for x in got] == [int(x) for x in ref]


@pytest.mark.parametrize("lam", [0.0, 0.25, 0.5, 1.7, 10.0, 60.0])
def test_poisson_table_matches_scipy(lam):
    T = oracle.poisson_table(lam)
    k = np.arange(len(T) + 1)
    ref = np.floor(scipy.stats.poisson.cdf(k, lam) * 4294967296.0)
    # entries agree to within one unit of the last place of the CDF
    assert np.all(np.abs(T.astype(np.float64) - ref[:-1]) <= 1.0)
    # the table ends exactly where the CDF saturates the uint32 range
    assert ref[-1] >= 4294967295.0 - 1.0
    if len(T):
        assert ref[len(T) - 1] < 4294967295.0
    assert np.all(np.diff(T.astype(np.int64)) >= 0)


def test_background_uniforms_are_numpy_philox_values():
    """Neuron i's background value at step t is value i mod 8 of the Philox
    block of counter (t, i // 8, member, 0) - word (i mod 8) // 2, high half
    for even i, low half for odd - computed here with numpy's Philox."""
    from oracle.brute import _numpy_philox_u32
    for seed, t, member in ((99, 0, 0), (7, 13, 0), (123456789, 4, 3)):
        for i in list(range(0, 20)) + [63, 64, 65, 1_000_003]:
            assert oracle.bg_uniform(seed, t, i, member) == _numpy_philox_u32(seed, t, i, member), (seed, t, i)
    # eight neurons share one block: neighbours in a group draw different values
    vals = {oracle.bg_uniform(5, 2, i) for i in range(8)}
    assert len(vals) == 8


def test_background_counts_are_poisson():
    lam = 0.7
    T = oracle.poisson_table(lam)
    u = np.array([oracle.bg_uniform(99, t, i) for t in range(40) for i in range(500)], dtype=np.uint64)
    c = (u[:, None] >= T[None, :].astype(np.uint64)).sum(axis=1)
    n = len(c)
    assert abs(c.mean() - lam) < 5 * math.sqrt(lam / n)
    obs = np.bincount(c, minlength=6)[:6].astype(float)
    exp = scipy.stats.poisson.pmf(np.arange(6), lam) * n
    exp[-1] = n - exp[:-1].sum()
    obs[-1] = n - obs[:-1].sum()
    chi2 = ((obs - exp) ** 2 / exp).sum()
    assert chi2 < scipy.stats.chi2.ppf(0.999, 5)


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("inh,d", [(0, 1), (0, 3), (1, 2), (1, 5)])
def test_single_spike_impulse_and_exact_decay(inh, d):
    """One presynaptic spike at step e through delay d raises the post gates
    by exactly w in gather step e+d-1 (so in state t = e+d), then the gates
    decay as w exp(-n dt / tau) (jump + exponential decay, Sec. III-B)."""
    e, w, T = 4, 1.0, 30
    net = hand_net(2, [(1, 0, d, w)], is_inh=[inh, 0])
    o = oracle.OracleNet(net)
    forced = np.zeros((T, 2), dtype=np.uint8)
    forced[e, 0] = 1
    js = []
    for t in range(T):
        o.step(forced=forced[t])
        js.append([o.get(f)[1] for f in ("j_AMPA", "j_NMDA", "j_GABAa", "j_GABAb")])
    js = np.array(js)  # js[t] = gates after step t, i.e. state t+1
    arrive = e + d - 1
    on = (2, 3) if inh else (0, 1)
    off = (0, 1) if inh else (2, 3)
    assert np.all(js[:arrive] == 0.0)
    assert np.all(js[:, off] == 0.0)
    tau = np.array([2.0, 40.0, 10.0, 50.0])
    for u in on:
        n = np.arange(T - arrive)
        expect = w * np.exp(-n * 1.0 / tau[u])
        np.testing.assert_allclose(js[arrive:, u], expect, rtol=1e-13, atol=0)
    # tau = 2 ms, 10 steps: e^-5
    if not inh:
        assert abs(js[arrive + 10, 0] - 6.737946999085467e-03) < 1e-15
        assert abs(js[arrive + 10, 0] - GOLDEN["gate_decay"]["value"]) < 1e-9


def test_isi_discrete_closed_form():
    """No synaptic input, constant Iext: V_n - Vinf = rho^n (Vreset - Vinf),
    rho = 1 - dt gL / C.  With gL = 0.03, Iext = 1.05 (Vinf = -40 mV) the
    threshold -50 mV is reached after n* = ceil(ln(0.4)/ln(0.97)) = 31
    integration steps; the ISI is n_ref + n* = 33 steps."""
    net = hand_net(1, [], V0=[-65.0], Iext=1.05)
    o = oracle.OracleNet(net)
    r = o.run(200, want_state=True, want_margin=True)
    spikes = np.nonzero(r["raster"][:, 0])[0]
    # the network carries float32 parameters: use exactly those values
    gL, Iext = float(np.float32(0.03)), float(np.float32(1.05))
    rho, Vinf = 1.0 - gL, -75.0 + Iext / gL
    nstar = math.ceil(math.log((Vinf + 50.0) / (Vinf + 65.0)) / math.log(rho))
    ex = GOLDEN["isi_discrete"]
    assert nstar == ex["n_star"]
    assert spikes[0] == nstar - 1          # integrates from step 0
    assert np.all(np.diff(spikes) == ex["isi_steps"])
    V = np.array([s["V"][0] for s in r["states"]])  # V after step t
    # after 30 integration steps from Vreset (state after step 29)
    np.testing.assert_allclose(V[29], Vinf + rho**30 * (-65.0 - Vinf), rtol=1e-14)
    assert abs(V[29] - ex["V_after_30_steps_mV"]) < 1e-3
    # the step that crosses: Vt = -49.724 mV, margin 0.276 mV
    assert abs(r["margins"][30, 0] - abs(Vinf + rho**31 * (-65.0 - Vinf) + 50.0)) < 1e-12
    assert abs(r["margins"][30, 0] - ex["crossing_margin_mV"]) < 1e-3
    # refractory: held at Vreset for the 2 steps after a spike
    s0 = spikes[0]
    assert V[s0] == -65.0 and V[s0 + 1] == -65.0 and V[s0 + 2] == -65.0
    assert r["raster"][s0 + 1, 0] == 0 and r["raster"][s0 + 2, 0] == 0


def test_isi_converges_to_continuous_limit():
    """dt -> 0: ISI -> T_ref + tau_m ln((Vinf - Vreset)/(Vinf - Vth)) = 32.543 ms."""
    dt = 0.002
    net = hand_net(1, [], V0=[-65.0], Iext=1.05, dt_ms=dt)
    o = oracle.OracleNet(net)
    n_steps = int(80.0 / dt)
    r = o.run(n_steps)
    spikes = np.nonzero(r["raster"][:, 0])[0]
    isi_ms = np.diff(spikes)[0] * dt
    limit = 2.0 + (1.0 / 0.03) * math.log(25.0 / 10.0)
    assert abs(limit - GOLDEN["isi_continuous_limit_ms"]["value"]) < 1e-3
    assert abs(isi_ms - limit) < 3 * dt


# ---------------------------------------------------------------- invariants

def _run_small(seed=0, steps=200, lam=0.25):
    net = netgen.make_network(netgen.small_net(seed_offset=seed, bg_lambda=lam))
    return net, oracle.OracleNet(net).run(steps)


def test_event_count_equals_spikes_times_outdegree():
    """Sum over steps of delivered recurrent events = sum over spikes (m, e)
    of the out-synapses of m whose arrival step e + d - 1 is inside the run:
    a count over out-edges (push view) against the oracle's pull."""
    net, r = _run_small(steps=300)
    T = r["raster"].shape[0]
    cum = np.cumsum(r["raster"].astype(np.int64), axis=0)          # spikes of m in [0, t]
    d = net.delay.astype(np.int64)
    last = T - d                                                   # e <= T - d
    ok = last >= 0
    per_syn = np.where(ok, cum[np.clip(last, 0, T - 1), net.col], 0)
    assert int(per_syn.sum()) == int(r["ev_rec"].sum())
    # per step: events of step t = spikes (m, t - d + 1) over out-edges
    post = np.repeat(np.arange(net.n), np.diff(net.row_ptr))
    for t in (0, 7, 150, T - 1):
        te = t - d + 1
        v = np.where(te >= 0, r["raster"][np.clip(te, 0, T - 1), net.col], 0)
        assert int(v.sum()) == int(r["ev_rec"][t])
    assert len(post) == net.nnz


def test_region_counts_equal_raster_rows():
    net, r = _run_small(steps=100)
    for t in range(100):
        np.testing.assert_array_equal(r["counts"][t],
                                      np.bincount(net.region, weights=r["raster"][t], minlength=2))


def test_forced_replay_reproduces_free_run():
    net, r = _run_small(steps=120)
    o = oracle.OracleNet(net)
    r2 = o.run(120, forced=r["raster"])
    np.testing.assert_array_equal(r2["raster"], r["raster"])
    np.testing.assert_array_equal(r2["ev_rec"], r["ev_rec"])
    o1 = oracle.OracleNet(net)
    o1.run(120)
    np.testing.assert_array_equal(o.get("V"), o1.get("V"))


def test_row_subset_matches_full_step():
    net, r = _run_small(steps=60)
    rows = np.array([0, 5, 399, 400, 777, 999])
    full = oracle.OracleNet(net)
    part = oracle.OracleNet(net)
    for t in range(60):
        full.step(forced=r["raster"][t])
        part.step(forced=r["raster"][t], rows=rows)
    for f in ("V", "j_AMPA", "j_NMDA", "j_GABAa", "j_GABAb", "ref"):
        np.testing.assert_array_equal(full.get(f)[rows], part.get(f)[rows])


def test_thread_count_does_not_change_results():
    net = netgen.make_network(netgen.small_net())
    nt = oracle.max_threads()
    oracle.set_threads(1)
    try:
        a = oracle.OracleNet(net).run(80)
    finally:
        oracle.set_threads(nt)
    b = oracle.OracleNet(net).run(80)
    np.testing.assert_array_equal(a["raster"], b["raster"])


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("seed,lam,forced", [(0, 3.0, False), (1, 2.0, False), (2, 3.0, True)])
def test_sparse_ring_gather_matches_dense_brute_force(seed, lam, forced):
    """The CSR walk through the delay ring equals the dense delay-indexed
    contraction over the full history (numpy Philox + scipy CDF for the
    background), on 40-neuron nets with multi-edges and mixed delays."""
    spec = netgen.small_net(seed_offset=seed + 1, n=40, bg_lambda=lam, k_in=7, k_cross=3)
    net = netgen.make_network(spec)
    T = 100
    f = None
    if forced:
        rng = np.random.default_rng(seed)
        f = (rng.random((T, net.n)) < 0.05).astype(np.uint8)
    ref = brute.run(net, T, forced=f)
    o = oracle.OracleNet(net)
    r = o.run(T, forced=f, want_state=True)
    assert ref["raster"].sum() > 20, "test net must be active"
    np.testing.assert_array_equal(r["raster"], ref["raster"])
    np.testing.assert_array_equal(r["ev_rec"], ref["ev_rec"])
    np.testing.assert_array_equal(r["ev_bg"], ref["ev_bg"])
    V = np.array([s["V"] for s in r["states"]])
    np.testing.assert_allclose(V, ref["V"][1:], rtol=1e-12, atol=1e-10)
    for u, f_ in enumerate(("j_AMPA", "j_NMDA", "j_GABAa", "j_GABAb")):
        J = np.array([s[f_] for s in r["states"]])
        np.testing.assert_allclose(J, ref["j"][1:, :, u], rtol=1e-12, atol=1e-12)


def test_gain_scales_conductances():
    """Per-(region, channel) gains multiply g_u: gain 2 on a channel equals
    doubling that channel's conductance in the parameter table."""
    spec = netgen.small_net(n=40, bg_lambda=3.0, k_in=7, k_cross=3)
    net = netgen.make_network(spec)
    gain = np.ones((2, 4))
    gain[:, 0] = 2.0
    a = oracle.OracleNet(net, gain=gain).run(60)
    net2 = netgen.make_network(spec)
    net2.ptypes[0, 7] *= 2.0
    b = oracle.OracleNet(net2).run(60)
    ref = brute.run(net, 60, gain=gain)
    np.testing.assert_array_equal(a["raster"], b["raster"])
    np.testing.assert_array_equal(a["raster"], ref["raster"])


def test_bf16_round_matches_torch():
    import torch
    rng = np.random.default_rng(3)
    w = np.concatenate([rng.lognormal(-1, 0.5, 10000).astype(np.float32),
                        np.array([1.0, 1.00390625, 1.005859375, 3.0e-39, 0.0], dtype=np.float32)])
    ref = torch.from_numpy(w).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(oracle.bf16_round(w), ref)
