"""GPU check of the launch-shape autotuner (dtb_autotune): it times every
candidate shape on the real network, reports the fastest, and caches it."""
import json

import numpy as np
import pytest

import netgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dtb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2308_01241_amd as m
    m.load()
    return m


def test_autotune_times_candidates_and_caches(dtb, tmp_path):
    import torch
    from paper_2308_01241_amd import autotune
    net = netgen.make_network(netgen.partition_spec(n=60_000, bg_lambda=0.5))
    cache = tmp_path / "tuned.json"
    cands = (8192, 65536, 400_000)
    r = autotune.tune([net], cache_path=cache, bundles=cands, burnin=30, steps=10,
                      stream=torch.cuda.current_stream())
    assert not r["from_cache"]
    sweep = {(b, u, f, 1) for b in cands for u in (1, 2, 3) for f in (1, 2)}
    spike = {(b, 0, f, 2) for b in cands for f in (1, 2)}
    # the 8,192-synapse bundles are too many for the event table's bundle ids
    assert sweep <= set(r["tried"]) <= sweep | spike
    assert {(b, 0, f, 2) for b in (65536, 400_000) for f in (1, 2)} <= set(r["tried"])
    assert all(v > 0 for v in r["tried"].values())
    best = (r["bundle_syn"], r["unroll"], r["fuse"], r["events"])
    assert best == min(r["tried"], key=r["tried"].get)
    db = json.loads(cache.read_text())
    arch = autotune._arch()
    key = autotune.shape_key(arch, net.n, net.nnz, 1, "f32", net.max_delay)
    assert (db[key]["bundle_syn"], db[key]["unroll"], db[key]["fuse"], db[key]["events"]) == best
    assert autotune.lookup(net.n, net.nnz, 1, "f32", net.max_delay, path=cache) == best
    # a cached shape is returned without timing
    again = autotune.tune([net], cache_path=cache, bundles=cands, burnin=30, steps=10,
                          stream=torch.cuda.current_stream())
    assert again["from_cache"] and not again["tried"]
    assert (again["bundle_syn"], again["unroll"], again["fuse"], again["events"]) == best
    # a batch (another key) is tuned into the same file; the library's own
    # candidate list is used when none is given
    mem = [netgen.make_network(netgen.ensemble_member_spec(m, n, rate_hz=15, n_regions=4))
           for m, n in enumerate((3000, 4100))]
    rb = autotune.tune(mem, cache_path=cache, burnin=20, steps=5, stream=torch.cuda.current_stream())
    assert not rb["from_cache"] and len(rb["tried"]) >= 8
    db = json.loads(cache.read_text())
    assert len(db) == 2 and key in db
