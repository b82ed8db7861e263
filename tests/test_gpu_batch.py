"""GPU checks of the batched ensemble, the captured-graph stepping and the
Balloon-Windkessel readout (the assimilation side of Sec. V-E)."""
import numpy as np
import pytest

import netgen
import oracle
from oracle import bold as bold_ref
from parity import lockstep, report

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dtb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2308_01241_amd as m
    m.load()
    return m


def _stream():
    import torch
    return torch.cuda.current_stream()


def _members(sizes, rate=15):
    out = []
    for m, n in enumerate(sizes):
        out.append(netgen.make_network(netgen.ensemble_member_spec(m, n, rate_hz=rate, n_regions=4)))
    return out


def test_batch_equals_members_run_alone(dtb):
    """Each member of a batch computes bit for bit what it computes alone,
    with its own per-population gains (block-diagonal partition, own
    background counter)."""
    sizes = [3000, 5200, 4100]
    mem = _members(sizes)
    gains = netgen.ensemble_gains(len(sizes), 4, seed=7)
    b = dtb.Net.batch(mem, record_steps=300, stream=_stream())
    assert b.n_members == 3 and b.n == sum(sizes) and b.n_regions == 12
    b.set_gains(gains.reshape(-1, 4))
    b.run(300)
    ras = b.raster(0, 300)
    for m, nw in enumerate(mem):
        g = dtb.Net(nw, record_steps=300, stream=_stream())
        g.set_gains(gains[m])
        g.step(300)
        lo, hi = b.neuron_offset[m], b.neuron_offset[m + 1]
        np.testing.assert_array_equal(ras[:, lo:hi], g.raster(0, 300))
        r0, r1 = b.region_offset[m], b.region_offset[m + 1]
        np.testing.assert_array_equal(b.region_counts(0, 300)[:, r0:r1], g.region_counts(0, 300))


def test_batch_equals_members_run_alone_with_ou_background(dtb):
    """The OU background draws are keyed by (step, neuron inside the member,
    member): a member in a batch gets the same I_ou sequence, hence the same
    raster, as alone, under graph replay too."""
    sizes = [2500, 3300]
    mem = _members(sizes)
    b = dtb.Net.batch(mem, record_steps=200, stream=_stream())
    b.set_background_ou(0.6, 0.4, 8.0)
    b.run(200)
    ras = b.raster(0, 200)
    ou_b = b.state("I_ou")
    assert ras.sum() > 0
    for m, nw in enumerate(mem):
        g = dtb.Net(nw, record_steps=200, stream=_stream())
        g.set_background_ou(0.6, 0.4, 8.0)
        g.step(200)
        lo, hi = b.neuron_offset[m], b.neuron_offset[m + 1]
        np.testing.assert_array_equal(ras[:, lo:hi], g.raster(0, 200))
        np.testing.assert_array_equal(ou_b[lo:hi], g.state("I_ou"))


def test_batch_member_with_gains_matches_reference(dtb):
    mem = _members([2000, 2600])
    gains = netgen.ensemble_gains(2, 4, seed=9)
    b = dtb.Net.batch(mem, record_steps=120, stream=_stream())
    b.set_gains(gains.reshape(-1, 4))
    b.step(120)
    counts = b.region_counts(0, 120)
    for m, nw in enumerate(mem):
        ref = oracle.OracleNet(nw, gain=gains[m].astype(np.float64)).run(120)
        lo, hi = b.neuron_offset[m], b.neuron_offset[m + 1]
        ras = b.raster(0, 120)[:, lo:hi]
        ls = lockstep(oracle.OracleNet(nw, gain=gains[m].astype(np.float64)), ras)
        if not ls["ties"]:
            np.testing.assert_array_equal(ras, ref["raster"])
        r0, r1 = b.region_offset[m], b.region_offset[m + 1]
        np.testing.assert_array_equal(counts[:, r0:r1], ls["counts"])
        report("batch_member_gains_120", member=m, ties=len(ls["ties"]))


def test_graph_replays_equal_eager_steps(dtb):
    """dtb_run (captured graph, replayed several times with eager reads in
    between) gives the same raster, state and counters as dtb_step."""
    net = netgen.make_network(netgen.small_net(seed_offset=6))
    a = dtb.Net(net, record_steps=200, stream=_stream())
    e = dtb.Net(net, record_steps=200, stream=_stream())
    for r in range(4):
        a.run(50)
        e.step(50)
        np.testing.assert_array_equal(a.raster(50 * r, 50 * (r + 1)), e.raster(50 * r, 50 * (r + 1)))
        np.testing.assert_array_equal(a.state("V"), e.state("V"))
        assert a.counters() == e.counters()
    np.testing.assert_array_equal(a.bold(), e.bold())


def test_bold_matches_reference_on_the_reference_raster(dtb):
    """FP32 Balloon-Windkessel on the GPU (deviation form) against the FP64
    reference, both driven by the population rates of the reference's own
    raster (forced on the GPU, so the counts are identical)."""
    net = netgen.make_network(netgen.small_net(seed_offset=7, bg_lambda=0.6))
    T = 1000
    free = oracle.OracleNet(net).run(T)
    g = dtb.Net(net, record_steps=T, stream=_stream())
    g.force(free["raster"])
    g.step(T)
    np.testing.assert_array_equal(g.region_counts(0, T), free["counts"])
    sizes = np.bincount(net.region, minlength=net.n_regions)
    rates = free["counts"] / (sizes[None, :] * net.dt_ms * 1e-3)
    st, ys = bold_ref.run(rates, dt_s=net.dt_ms * 1e-3)
    y, sfvq = g.bold(state=True)
    assert np.abs(ys[-1]).max() > 1e-4, "BOLD signal should have moved"
    np.testing.assert_allclose(y, ys[-1], rtol=0, atol=1e-3 * np.abs(ys[-1]).max())
    np.testing.assert_allclose(sfvq, st, rtol=0, atol=2e-5)
