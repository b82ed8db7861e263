"""Spike-driven delivery (gather_events = 2) against the pull sweep
(gather_events = 1): the last D steps' spikes each deliver through their
out-synapses of the matching delay, bucketed per bundle, and set the same
hit bits the sweep finds, so rasters, states and counters are identical bit
for bit - across drives, row-sum placements, weight types, graph replay,
teacher forcing, the OU background, a batch, a remote block, checkpoint
resume (the spike-id lists are rebuilt from the restored bitmaps) and reset.
The sweep itself is checked against the FP64 reference elsewhere; one run
here is checked against it directly too."""
import numpy as np
import pytest

import netgen
import oracle
from parity import lockstep

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


def _run(dtb, net, T, graph=False, **kw):
    g = dtb.Net(net, record_steps=T, stream=_stream(), **kw)
    if graph:
        g.run(T // 2)
        g.step(T - T // 2)
    else:
        g.step(T)
    out = (g.spikes_bits(0, T), g.state("V"), g.state("j_AMPA"), g.state("j_GABAb"), g.counters(),
           g.step_events(0, T))
    ids = g.spike_ids(T - 1)
    g.close()
    return out, ids


def _same(a, b):
    for x, y in zip(a[:4], b[:4]):
        np.testing.assert_array_equal(x, y)
    assert a[4] == b[4]
    np.testing.assert_array_equal(a[5][0], b[5][0])
    np.testing.assert_array_equal(a[5][1], b[5][1])


@pytest.mark.parametrize("lam", [0.27346, 1.52745])
def test_spike_driven_equals_sweep_on_a_partition_net(dtb, lam):
    """60,000 neurons, 90 populations, delays 1-20: the 7 Hz and 30 Hz
    drives, both row-sum placements, FP32 and BF16, with and without graph
    replay.  With the row sums fused, three bundle sizes: 20,000 synapses
    (hundreds of bundles, every bucket's weights fit the LDS at once),
    880,000 (seven bundles with LDS room for about 6,300 carried weights
    each: at 7 Hz the buckets hold about that many, so a launch mixes
    bundles that order their weights in LDS and bundles that order them in
    the free part of their bucket; at 30 Hz every bundle does the latter)
    and 1,048,575 (the LDS cannot hold the bitmap's prefix counts: every
    weight from the CSR)."""
    net = netgen.make_network(netgen.partition_spec(n=60_000, bg_lambda=lam))
    T = 120
    print(f"partition n={net.n} lambda={lam}", flush=True)
    for wt in ("f32", "bf16"):
        ref, ids_ref = _run(dtb, net, T, wtype=wt, bundle_syn=20_000, events=1)
        assert ref[4]["spikes"] > 0 and ref[4]["ev_rec"] > 0
        for bs, fuse in ((20_000, 1), (20_000, 2), (880_000, 1), (1_048_575, 1)):
            for graph in (False, True):
                print(f"  {wt} bundle_syn={bs} fuse={fuse} graph={graph}", flush=True)
                got, ids = _run(dtb, net, T, graph=graph, wtype=wt, bundle_syn=bs, fuse=fuse, events=2)
                _same(got, ref)
                np.testing.assert_array_equal(ids, ids_ref)


def test_spike_driven_matches_the_reference(dtb):
    """The 1,000-neuron net free-run 100 steps with spike-driven delivery, in
    lockstep with the FP64 reference (no tie expected for this seed)."""
    net = netgen.make_network(netgen.small_net(seed_offset=2))
    T = 100
    g = dtb.Net(net, record_steps=T, stream=_stream(), events=2)
    g.step(T)
    ras = g.raster(0, T)
    er, eb = g.step_events(0, T)
    g.close()
    ls = lockstep(oracle.OracleNet(net), ras)
    assert not ls["ties"]
    np.testing.assert_array_equal(er, ls["ev_rec"])
    np.testing.assert_array_equal(eb, ls["ev_bg"])
    assert ras.sum() > 0


def test_spike_driven_teacher_forcing_and_ou(dtb):
    net = netgen.make_network(netgen.small_net(seed_offset=3, bg_lambda=0.0))
    T = 80
    forced = (np.random.default_rng(9).random((40, net.n)) < 0.03).astype(np.uint8)
    outs = []
    for ev in (1, 2):
        g = dtb.Net(net, record_steps=T, stream=_stream(), events=ev)
        g.set_background_ou(0.6, 0.4, 8.0)
        g.force(forced)
        g.step(T)
        outs.append((g.spikes_bits(0, T), g.state("V"), g.state("I_ou"), g.state("j_NMDA"), g.counters(),
                     g.step_events(0, T)))
        g.close()
    _same(outs[1], outs[0])


def test_spike_driven_batch_and_resume(dtb):
    """A three-member batch under graph replay; a state saved by a sweep
    handle resumes in a spike-driven one (its spike-id lists rebuilt from the
    restored bitmaps) and continues exactly as the sweep handle does; reset
    reproduces the first run."""
    members = [netgen.make_network(netgen.ensemble_member_spec(m, 20_000 + 3_000 * m, rate_hz=15, n_regions=5))
               for m in range(3)]
    gains = np.random.default_rng(1).uniform(0.8, 1.2, (15, 4)).astype(np.float32)
    hs = []
    for ev in (1, 2):
        g = dtb.Net.batch(members, record_steps=64, stream=_stream(), events=ev)
        g.set_gains(gains)
        hs.append(g)
    a, b = hs
    a.run(30)
    state = a.save()
    a.run(40)
    b.load(state)
    b.run(40)
    np.testing.assert_array_equal(b.spikes_bits(30, 70), a.spikes_bits(30, 70))
    np.testing.assert_array_equal(b.state("V"), a.state("V"))
    assert b.counters() == a.counters()
    np.testing.assert_array_equal(b.spike_ids(69), a.spike_ids(69))
    first = b.spikes_bits(30, 70)
    b.reset()
    b.set_gains(gains)
    b.run(30)
    b.run(40)
    a.reset()
    a.set_gains(gains)
    a.run(70)
    np.testing.assert_array_equal(b.spikes_bits(30, 70), a.spikes_bits(30, 70))
    np.testing.assert_array_equal(b.spikes_bits(30, 70), first)
    for g in hs:
        g.close()


def test_spike_driven_local_block_with_a_remote_block(dtb):
    net = netgen.make_network(netgen.small_net(seed_offset=7))
    blk = netgen.make_remote_block(net.n, 400, 12, max_delay=net.max_delay, seed=3)
    rem = netgen.remote_raster(60, 400, rate_hz=30.0, seed=4)
    outs = []
    for ev in (1, 2):
        g = dtb.Net(net, record_steps=60, stream=_stream(), events=ev)
        g.set_remote_block(blk)
        g.push_remote(rem)
        g.step(60)
        outs.append((g.spikes_bits(0, 60), g.state("V"), g.state("j_AMPA"), g.state("j_GABAa"), g.counters(),
                     g.step_events(0, 60)))
        g.close()
    _same(outs[1], outs[0])


def test_too_many_bundles_for_spike_driven_delivery(dtb):
    from paper_2308_01241_amd import DtbError
    net = netgen.make_network(netgen.partition_spec(n=200_000))  # 2e7 synapses / 4,096 > 4,096 bundles
    with pytest.raises(DtbError, match="4096"):
        dtb.Net(net, record_steps=16, stream=_stream(), bundle_syn=4096, events=2)
