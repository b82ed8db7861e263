"""Pins of the reference's J_inter term (Sec. V-B: a neuron's input splits
into J_intra over presynaptic neurons on the same GPU and J_inter over
those on other GPUs).

* A partition with a remote in-edge block, fed a replayed remote raster, is
  the same computation as one network that holds the remote sources as
  extra neurons (their in-edges appended after each row's local ones) and is
  teacher-forced with [own raster, remote raster] while only the local rows
  advance: state, events and spikes agree bit for bit at every step.  This
  reduces the remote term to the local gather, which the dense brute-force
  formulation pins.
* A silent remote raster leaves the run identical to the network without
  the block; a single remote spike over a one-edge block delivers exactly
  its weight, to the right gate, on the step its delay names.
"""
import dataclasses

import numpy as np
import pytest

import netgen
import oracle


def _extended(net, blk):
    """The partition plus the remote sources as neurons n .. n + n_remote - 1."""
    n, R = net.n, blk.n_remote
    cols, ws, ds, rp = [], [], [], [0]
    for i in range(n):
        a, b = net.row_ptr[i], net.row_ptr[i + 1]
        c, d = blk.row_ptr[i], blk.row_ptr[i + 1]
        cols += [net.col[a:b], blk.col[c:d].astype(np.int64) + n]
        ws += [net.w[a:b], blk.w[c:d]]
        ds += [net.delay[a:b], blk.delay[c:d]]
        rp.append(rp[-1] + (b - a) + (d - c))
    rp += [rp[-1]] * R
    return dataclasses.replace(
        net, n=n + R, row_ptr=np.array(rp, dtype=np.int64),
        col=np.concatenate(cols).astype(np.int32), w=np.concatenate(ws).astype(np.float32),
        delay=np.concatenate(ds).astype(np.uint8), is_inh=np.concatenate([net.is_inh, blk.is_inh]),
        region=np.concatenate([net.region, np.zeros(R, np.int32)]),
        ptype=np.concatenate([net.ptype, np.zeros(R, np.uint16)]),
        V0=np.concatenate([net.V0, np.full(R, -60.0, np.float32)]), region_start=None)


@pytest.mark.parametrize("k_remote", [7, "ragged"])
def test_remote_block_equals_extended_network_teacher_forced(k_remote):
    net = netgen.make_network(netgen.small_net(seed_offset=2, bg_lambda=0.5))
    n, R, T = net.n, 300, 60
    k = np.random.default_rng(4).integers(0, 15, n) if k_remote == "ragged" else k_remote
    blk = netgen.make_remote_block(n, R, k, max_delay=net.max_delay, seed=21)
    rem = netgen.remote_raster(T, R, rate_hz=40.0, seed=22)
    a = oracle.OracleNet(net)
    a.set_remote(blk)
    ext = _extended(net, blk)
    b = oracle.OracleNet(ext)
    rows = np.arange(n)
    fields = ("V", "j_AMPA", "j_NMDA", "j_GABAa", "j_GABAb", "ref")
    n_rem_ev = 0
    for t in range(T):
        a.give_remote(rem[t])
        oa = a.step()
        ob = b.step(forced=np.concatenate([oa["spikes"], rem[t]]), rows=rows)
        assert oa["ev_rec"] == ob["ev_rec"] and oa["ev_bg"] == ob["ev_bg"], t
        for f in fields:
            np.testing.assert_array_equal(a.get(f), b.get(f)[:n], err_msg=f"step {t} {f}")
        n_rem_ev += oa["ev_rec"]
    assert rem.sum() > 0 and n_rem_ev > 0


def test_silent_remote_raster_changes_nothing():
    net = netgen.make_network(netgen.small_net(seed_offset=3))
    T = 80
    blk = netgen.make_remote_block(net.n, 500, 10, max_delay=net.max_delay, seed=5)
    a = oracle.OracleNet(net)
    a.set_remote(blk)
    ra = a.run(T, want_state=False, remote=np.zeros((T, 500), np.uint8))
    b = oracle.OracleNet(net)
    rb = b.run(T)
    np.testing.assert_array_equal(ra["raster"], rb["raster"])
    np.testing.assert_array_equal(ra["ev_rec"], rb["ev_rec"])
    for f in ("V", "j_AMPA", "j_GABAa"):
        np.testing.assert_array_equal(a.get(f), b.get(f))


def test_one_remote_edge_delivers_its_weight_after_its_delay():
    """Row 0 of a silent net gets one remote in-edge (weight w, delay d)
    from an excitatory source that spikes only at step s: j_AMPA of row 0 is
    zero until step s + d - 1, then w, then decays by exp(-dt/tau)."""
    net = netgen.make_network(netgen.small_net(n=64, bg_lambda=0.0))
    net = dataclasses.replace(net, w=np.zeros_like(net.w))
    d, s, wv = 3, 5, 0.625
    rp = np.zeros(net.n + 1, np.int64)
    rp[1:] = 1
    blk = netgen.RemoteBlock(n_remote=2, row_ptr=rp, col=np.array([1], np.int32),
                             w=np.array([wv], np.float32), delay=np.array([d], np.uint8),
                             is_inh=np.array([1, 0], np.uint8))
    o = oracle.OracleNet(net)
    o.set_remote(blk)
    a = np.exp(-net.dt_ms / float(net.tau_ms[0]))
    for t in range(s + d + 4):
        sp = np.zeros(2, np.uint8)
        sp[1] = 1 if t == s else 0
        o.give_remote(sp)
        out = o.step()
        j = o.get("j_AMPA")[0]
        t_arr = s + d - 1
        want = 0.0 if t < t_arr else wv * a ** (t - t_arr)
        assert j == pytest.approx(want, rel=1e-12, abs=0.0), t
        assert out["ev_rec"] == (1 if t == t_arr else 0)
        assert o.get("j_GABAa")[0] == 0.0


def test_missing_remote_spikes_is_an_error():
    net = netgen.make_network(netgen.small_net(n=64))
    o = oracle.OracleNet(net)
    o.set_remote(netgen.make_remote_block(net.n, 10, 2, max_delay=net.max_delay))
    with pytest.raises(ValueError):
        o.step()
    o.give_remote(np.zeros(10, np.uint8))
    o.step()
    with pytest.raises(ValueError):
        o.step()


def test_split_network_replaying_its_own_raster_is_the_unsplit_run():
    """Cutting each row into own-region (local) and cross-region (remote)
    in-edges and replaying the unsplit run's raster as the remote spikes
    gives the unsplit run exactly: same summation order, same deliveries."""
    net = netgen.make_network(netgen.small_net(seed_offset=4, n=600))
    T = 70
    full = oracle.OracleNet(net)
    rf = full.run(T, want_state=False)
    local, blk = netgen.split_remote(net)
    assert blk.row_ptr[-1] == 30 * net.n
    part = oracle.OracleNet(local)
    part.set_remote(blk)
    rp = part.run(T, remote=rf["raster"])
    assert rf["raster"].sum() > 0
    np.testing.assert_array_equal(rp["raster"], rf["raster"])
    np.testing.assert_array_equal(rp["ev_rec"], rf["ev_rec"])
    for f in ("V", "j_AMPA", "j_NMDA", "j_GABAa", "j_GABAb"):
        np.testing.assert_array_equal(part.get(f), full.get(f))


def test_split_is_the_region_split_and_keeps_row_order():
    """split_remote on a partition net: every local in-edge comes from the
    row's own region and every remote one from another region (the J_intra /
    J_inter split of Sec. V-B for a partition holding whole regions); the
    local part followed by the remote part is each row's original order."""
    net = netgen.make_network(netgen.partition_spec(n=50_000))
    local, blk = netgen.split_remote(net)
    n = net.n
    rl = np.repeat(np.arange(n), np.diff(local.row_ptr))
    rr = np.repeat(np.arange(n), np.diff(blk.row_ptr))
    assert np.all(net.region[local.col] == net.region[rl])
    assert np.all(net.region[blk.col] != net.region[rr])
    assert local.nnz + int(blk.row_ptr[-1]) == net.nnz
    assert local.nnz == 70 * n
    for i in (0, 1, n // 2, n - 1):
        a, b = local.row_ptr[i], local.row_ptr[i + 1]
        c, d = blk.row_ptr[i], blk.row_ptr[i + 1]
        k0, k1 = net.row_ptr[i], net.row_ptr[i + 1]
        np.testing.assert_array_equal(np.concatenate([local.col[a:b], blk.col[c:d]]), net.col[k0:k1])
        np.testing.assert_array_equal(np.concatenate([local.w[a:b], blk.w[c:d]]), net.w[k0:k1])
        np.testing.assert_array_equal(np.concatenate([local.delay[a:b], blk.delay[c:d]]), net.delay[k0:k1])
        # each part ascending by source
        assert np.all(np.diff(local.col[a:b]) >= 0) and np.all(np.diff(blk.col[c:d]) >= 0)


def test_embedded_independent_subgraph_runs_as_alone():
    """The network of the accuracy check of Sec. VII-B: a subgraph embedded
    with no synapse into or out of it evolves exactly as the subgraph alone
    (same ids, same background draws), and no edge crosses the boundary."""
    sub = netgen.make_network(netgen.slice_spec(rate_hz=7, n=3000))
    rest = netgen.make_network(netgen.partition_spec(n=12_000))
    e = netgen.embed_independent(sub, rest)
    assert e.n == sub.n + rest.n and e.nnz == sub.nnz + rest.nnz and e.n_regions == sub.n_regions + rest.n_regions
    k = int(e.row_ptr[sub.n])
    assert np.all(e.col[:k] < sub.n) and np.all(e.col[k:] >= sub.n)
    np.testing.assert_array_equal(e.region[:sub.n], sub.region)
    a = oracle.OracleNet(sub).run(60)
    b = oracle.OracleNet(e).run(60)
    assert a["raster"].sum() > 0
    np.testing.assert_array_equal(b["raster"][:, :sub.n], a["raster"])
    np.testing.assert_array_equal(b["counts"][:, :sub.n_regions], a["counts"])
