"""GPU parity of the J_inter path (Sec. V-B): a partition with a remote
in-edge block whose sources' spikes are replayed, against the FP64 reference
given the same remote raster.  Bars as in test_gpu_parity: every spike
decision equal to the FP64 threshold test's except at counted near-threshold
ties (lockstep), teacher-forced state within 1e-5 relative, event counts
exact."""
import numpy as np
import pytest

import netgen
import oracle
from parity import DELTA, FIELDS, lockstep, report

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dtb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2308_01241_amd as m
    m.load()
    return m


def _gpu(dtb, net, blk=None, **kw):
    import torch
    g = dtb.Net(net, stream=torch.cuda.current_stream(), **kw)
    if blk is not None:
        g.set_remote_block(blk)
    return g


def _state_close(x_gpu, x_ref, floor):
    tol = 1e-5 * np.maximum(np.abs(x_ref), floor)
    return np.abs(x_gpu.astype(np.float64) - x_ref) <= tol


def _case(seed=0, n_remote=300, k=9, rate=40.0, T=100, **kw):
    net = netgen.make_network(netgen.small_net(seed_offset=seed, **kw))
    blk = netgen.make_remote_block(net.n, n_remote, k, max_delay=net.max_delay, seed=30 + seed)
    rem = netgen.remote_raster(T, n_remote, rate_hz=rate, seed=40 + seed)
    return net, blk, rem


@pytest.mark.parametrize("seed", [0, 1])
def test_remote_raster_matches_reference_100_steps(dtb, seed):
    net, blk, rem = _case(seed)
    T = rem.shape[0]
    o = oracle.OracleNet(net)
    o.set_remote(blk)
    ref = o.run(T, want_margin=True, remote=rem)
    print(f"remote raster parity seed={seed} n={net.n} n_remote={blk.n_remote}", flush=True)
    g = _gpu(dtb, net, blk)
    g.push_remote(rem)
    g.step(T)
    ras = g.raster(0, T)
    assert ref["raster"].sum() > 0
    o_ls = oracle.OracleNet(net)
    o_ls.set_remote(blk)
    ls = lockstep(o_ls, ras, remote=rem)
    if not ls["ties"]:
        np.testing.assert_array_equal(ras, ref["raster"])
    er, eb = g.step_events(0, T)
    assert len(er) == T
    np.testing.assert_array_equal(er, ls["ev_rec"])
    np.testing.assert_array_equal(eb, ls["ev_bg"])
    np.testing.assert_array_equal(g.region_counts(0, T), ls["counts"])
    report("remote_raster_100", seed=seed, ties=len(ls["ties"]))


@pytest.mark.parametrize("wtype", ["f32", "bf16"])
def test_remote_teacher_forced_state_many_bundles_ragged(dtb, wtype):
    """60,000 rows (hundreds of bundles in each block), ragged remote rows
    (0 .. 40 in-edges), 20,000 remote sources at 10 Hz, own raster forced at
    10 Hz: exact per-step events, state within tolerance.  BF16 runs against
    the reference on BF16-rounded weights of both blocks.  (The forced drive
    keeps V in its physical range: far stronger forcing pushes the total
    conductance past the forward-Euler stability bound 2 C / dt, where V
    leaves [E_GABA, E_AMPA] and rounding differences grow step by step.)"""
    net = netgen.make_network(netgen.partition_spec(n=60_000, bg_lambda=0.5))
    T, R = 30, 20_000
    k = np.random.default_rng(3).integers(0, 41, net.n)
    blk = netgen.make_remote_block(net.n, R, k, max_delay=net.max_delay, seed=8)
    rem = netgen.remote_raster(T, R, rate_hz=10.0, seed=9)
    rng = np.random.default_rng(11)
    forced = (rng.random((T, net.n)) < 0.01).astype(np.uint8)
    ref_net, ref_blk = net, blk
    if wtype == "bf16":
        import dataclasses
        ref_net = dataclasses.replace(net, w=oracle.bf16_round(net.w))
        ref_blk = dataclasses.replace(blk, w=oracle.bf16_round(blk.w))
    o = oracle.OracleNet(ref_net)
    o.set_remote(ref_blk)
    print(f"remote teacher-forced {wtype} n={net.n} n_remote={R}", flush=True)
    g = _gpu(dtb, net, blk, wtype=wtype)
    g.force(forced)
    g.push_remote(rem)
    for t in range(T):
        o.give_remote(rem[t])
        out = o.step(forced=forced[t])
        g.step(1)
        er, eb = g.step_events(t, t + 1)
        assert int(er[0]) == out["ev_rec"] and int(eb[0]) == out["ev_bg"], f"step {t}"
    jmax = max(np.abs(o.get(f)).max() for f in FIELDS[1:])
    for f in FIELDS:
        floor = 0.0 if f == "V" else 1e-3 * jmax
        x, ref = g.state(f), o.get(f)
        ok = _state_close(x, ref, floor)
        i = int(np.argmax(np.abs(x - ref)))
        assert ok.all(), f"{f}: {np.count_nonzero(~ok)} neurons out of tolerance (worst {i}: {x[i]} vs {ref[i]})"
    assert -90.0 < o.get("V").min() and o.get("V").max() < 0.0


def test_silent_remote_block_is_bit_identical_to_no_block(dtb):
    net, blk, _ = _case(2)
    T = 80
    a = _gpu(dtb, net, blk)
    a.push_remote(np.zeros((T, blk.n_remote), np.uint8))
    a.step(T)
    b = _gpu(dtb, net)
    b.step(T)
    np.testing.assert_array_equal(a.raster(0, T), b.raster(0, T))
    for f in FIELDS:
        np.testing.assert_array_equal(a.state(f), b.state(f))
    assert a.counters() == b.counters()


def test_remote_launch_shapes_reset_and_timing(dtb):
    """Tiles per round only change the schedule; a reset with the same
    pushes reproduces the run; the remote gather is timed once per step."""
    net, blk, rem = _case(3, T=60)
    T = rem.shape[0]
    runs = []
    for u in (1, 2, 3):
        g = _gpu(dtb, net, blk, unroll=u)
        g.set_timing(True)
        g.push_remote(rem)
        g.step(T)
        kt = g.read_timing()
        assert kt["remote_gather"]["launches"] == T and kt["gather"]["launches"] == T
        runs.append((g.raster(0, T), g.state("V"), g.counters()))
        g.reset()
        g.push_remote(rem)
        g.step(T)
        np.testing.assert_array_equal(g.raster(0, T), runs[-1][0])
        np.testing.assert_array_equal(g.state("V"), runs[-1][1])
        g.close()
    for r in runs[1:]:
        np.testing.assert_array_equal(r[0], runs[0][0])
        np.testing.assert_array_equal(r[1], runs[0][1])
        assert r[2] == runs[0][2]


def test_remote_block_errors(dtb):
    net, blk, rem = _case(0, T=4)
    g = _gpu(dtb, net)
    with pytest.raises(dtb.DtbError):
        g.push_remote_bits(np.zeros((1, 1), np.uint32))           # no block yet
    import dataclasses
    bad = dataclasses.replace(blk, col=blk.col.copy())
    bad.col[5] = blk.n_remote                                       # source out of range
    with pytest.raises(dtb.DtbError):
        g.set_remote_block(bad)
    bad = dataclasses.replace(blk, delay=blk.delay.copy())
    bad.delay[0] = net.max_delay + 1
    with pytest.raises(dtb.DtbError):
        g.set_remote_block(bad)
    g.set_remote_block(blk)
    with pytest.raises(dtb.DtbError):
        g.set_remote_block(blk)                                     # once per handle
    with pytest.raises(dtb.DtbError):
        g.step(1)                                                   # nothing pushed
    with pytest.raises(dtb.DtbError):
        g.push_remote(np.zeros((g.record_steps + 1, blk.n_remote), np.uint8))
    g.push_remote(rem[:2])
    with pytest.raises(dtb.DtbError):
        g.run(2)                                                    # graphs replay no pushes
    g.step(2)
    with pytest.raises(dtb.DtbError):
        g.step(1)
    g.push_remote(rem[2:3])
    with pytest.raises(dtb.DtbError):
        g.step(3)                                                   # one step taken, then none pushed
    assert g.t == 3 and g.counters()["steps"] == 3
    m = dtb.Net.batch([net, dataclasses.replace(net, member=1)])
    with pytest.raises(dtb.DtbError):
        m.set_remote_block(netgen.make_remote_block(m.n, 100, 3, max_delay=net.max_delay))


def test_split_partition_replaying_its_own_raster_is_bit_identical(dtb):
    """A 60,000-row partition cut into its own-region in-edges (local block,
    70 per row) and its cross-region ones (remote block whose sources mirror
    the partition), fed the unsplit run's raster as remote spikes: the same
    deliveries in the same order, so raster, state and event totals equal
    the unsplit GPU run bit for bit (a property that holds at any size)."""
    net = netgen.make_network(netgen.partition_spec(n=60_000))
    T = 200
    full = _gpu(dtb, net)
    full.step(T)
    bits = full.spikes_bits(0, T)
    local, blk = netgen.split_remote(net)
    print(f"split replay n={net.n} T={T} spikes={int(full.counters()['spikes'])}", flush=True)
    part = _gpu(dtb, local, blk)
    part.push_remote_bits(bits)
    part.step(T)
    np.testing.assert_array_equal(part.spikes_bits(0, T), bits)
    for f in FIELDS:
        np.testing.assert_array_equal(part.state(f), full.state(f))
    assert part.counters() == full.counters()
    assert full.counters()["spikes"] > 0


def test_empty_remote_block_and_single_remote_source(dtb):
    """Degenerate blocks: no remote synapses at all (every row empty) is the
    run without a block; a single remote source feeding every row matches
    the reference."""
    net, _, _ = _case(4)
    T = 60
    empty = netgen.RemoteBlock(n_remote=1, row_ptr=np.zeros(net.n + 1, np.int64), col=np.zeros(0, np.int32),
                               w=np.zeros(0, np.float32), delay=np.zeros(0, np.uint8), is_inh=np.zeros(1, np.uint8))
    a = _gpu(dtb, net, empty)
    a.push_remote(np.ones((T, 1), np.uint8))
    a.step(T)
    b = _gpu(dtb, net)
    b.step(T)
    np.testing.assert_array_equal(a.raster(0, T), b.raster(0, T))
    np.testing.assert_array_equal(a.state("V"), b.state("V"))
    assert a.counters() == b.counters()
    one = netgen.make_remote_block(net.n, 1, 1, max_delay=net.max_delay, seed=3)
    rem = (np.arange(T) % 7 == 0).astype(np.uint8)[:, None]
    o = oracle.OracleNet(net)
    o.set_remote(one)
    ref = o.run(T, want_margin=True, remote=rem)
    g = _gpu(dtb, net, one)
    g.push_remote(rem)
    g.step(T)
    ras = g.raster(0, T)
    o_ls = oracle.OracleNet(net)
    o_ls.set_remote(one)
    ls = lockstep(o_ls, ras, remote=rem)
    if not ls["ties"]:
        np.testing.assert_array_equal(ras, ref["raster"])
    np.testing.assert_array_equal(g.step_events(0, T)[0], ls["ev_rec"])
