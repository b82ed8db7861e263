"""The batched ensemble at its full size: 64 member networks of 50k-400k
neurons (20 populations each, per-(member, population, channel) gains),
advanced by replays of one captured HIP graph, with the Balloon-Windkessel
BOLD of every (member, population) compared with the FP64 reference
hemodynamics driven by the same population rates (the members' own counts
read back every 200 steps), at ten checkpoints over 2,000 steps."""
import numpy as np
import pytest

import netgen
from oracle import bold as bold_ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dtb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2308_01241_amd as m
    m.load()
    return m


@pytest.mark.timeout(600)
def test_ensemble_bold_full_size_against_reference(dtb):
    import torch
    sizes = netgen.ensemble_sizes(64)
    gains = netgen.ensemble_gains(64)
    members = [netgen.make_network(netgen.ensemble_member_spec(m, int(nm), rate_hz=7))
               for m, nm in enumerate(sizes)]
    pop = np.concatenate([np.bincount(nw.region, minlength=nw.n_regions) for nw in members])
    chunk, T = 200, 2000
    g = dtb.Net.batch(members, record_steps=chunk, stream=torch.cuda.current_stream())
    g.set_gains(gains.reshape(-1, 4))
    assert g.n_regions == pop.size == 64 * 20
    print(f"ensemble: {g.n} neurons, {g.n_regions} populations, {T} steps", flush=True)
    st = bold_ref.rest((g.n_regions,))
    dt_s = members[0].dt_ms * 1e-3
    worst_y, worst_s = 0.0, 0.0
    for c in range(T // chunk):
        g.run(chunk)
        counts = g.region_counts(c * chunk, (c + 1) * chunk)
        rates = counts / (pop[None, :] * dt_s)
        st, ys = bold_ref.run(rates, dt_s=dt_s, state=st)
        y, sfvq = g.bold(state=True)
        scale = np.abs(ys[-1]).max()
        assert np.isfinite(y).all() and np.isfinite(sfvq).all()
        worst_y = max(worst_y, float(np.abs(y - ys[-1]).max() / scale))
        worst_s = max(worst_s, float(np.abs(sfvq - st).max()))
        np.testing.assert_allclose(y, ys[-1], rtol=0, atol=1e-3 * scale)
        np.testing.assert_allclose(sfvq, st, rtol=0, atol=5e-5)
    rate = g.counters()["spikes"] / (g.n * T * dt_s)
    print(f"ensemble BOLD: mean rate {rate:.2f} Hz, max |dy| / max|y| {worst_y:.2e}, max |d state| {worst_s:.2e}",
          flush=True)
    assert rate > 1.0
    g.close()
