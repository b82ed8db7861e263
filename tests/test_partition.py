"""The library's partitioner (Sec. V-C, Eq. (2)) against the reference
objective: host code, no GPU needed.

* a valid partition: every vertex on one GPU, loads within the capacity;
* its F and D equal the reference's evaluation of the same assignment;
* on tiny graphs it stays close to the brute-force optimum;
* on the partition generator's population graph spread over several GPUs it
  beats the sequential cut the paper compares with, and refining never
  raises F above the greedy start."""
import numpy as np
import pytest

import netgen
from oracle import partition as op
from paper_2308_01241_amd import DtbError
from paper_2308_01241_amd import partition as pp


def _tiny(rng, V=7):
    nn = rng.integers(500, 3000, V).astype(np.float64)
    e_ptr, dst, syn = [0], [], []
    for u in range(V):
        for v in range(V):
            if rng.random() < 0.5:
                dst.append(v)
                syn.append(float(rng.integers(100, 6000)))
        e_ptr.append(len(dst))
    return pp.VertexGraph(size=nn.copy(), neurons=nn, spikes=0.01 * nn, e_ptr=np.array(e_ptr, np.int64),
                          e_dst=np.array(dst, np.int32), e_syn=np.array(syn, np.float64),
                          region=np.arange(V, dtype=np.int32))


def _ref(g, part, N):
    return op.traffic(part, g.size, g.neurons, g.spikes, g.e_ptr, g.e_dst, g.e_syn, N)


@pytest.mark.parametrize("seed", range(6))
def test_tiny_graphs_valid_exact_objective_and_near_optimal(seed):
    rng = np.random.default_rng(seed)
    g = _tiny(rng)
    N = 2 + seed % 2
    cap = g.size.sum() / N * 1.4
    part, F, D = pp.partition(g, N, cap)
    assert part.min() >= 0 and part.max() < N
    assert np.all(np.bincount(part, weights=g.size, minlength=N) <= cap * (1 + 1e-12))
    Dr, Fr = _ref(g, part, N)
    np.testing.assert_allclose(D, Dr, rtol=1e-9, atol=1e-9)
    assert abs(F - Fr) <= 1e-9 * max(Fr, 1.0)
    Fb, _ = op.brute_force(g.size, g.neurons, g.spikes, g.e_ptr, g.e_dst, g.e_syn, N, cap)
    assert F <= 1.5 * Fb + 1e-9, (F, Fb)


def test_init_without_refinement_evaluates_it():
    rng = np.random.default_rng(9)
    g = _tiny(rng, 9)
    init = rng.integers(0, 3, 9).astype(np.int32)
    part, F, D = pp.partition(g, 3, g.size.sum(), init=init, refine_rounds=0)
    np.testing.assert_array_equal(part, init)
    Dr, Fr = _ref(g, init, 3)
    assert abs(F - Fr) <= 1e-9 * Fr
    part2, F2, _ = pp.partition(g, 3, g.size.sum(), init=init, refine_rounds=500)
    assert F2 <= F


@pytest.mark.parametrize("n_gpu", [4, 16])
def test_population_graph_beats_the_sequential_cut(n_gpu):
    spec = netgen.partition_spec(n=n_gpu * 2_000_000, n_regions=90)
    g = pp.region_graph(spec.region_sizes, spec.cross_w, spec.k_in, spec.k_cross, rate_hz=7.0, chunk=250_000)
    cap = g.size.sum() / n_gpu * 1.1
    seq = pp.sequential(g, n_gpu)
    _, F_seq, _ = pp.partition(g, n_gpu, g.size.sum(), init=seq, refine_rounds=0)
    part0, F0, _ = pp.partition(g, n_gpu, cap, refine_rounds=0)
    part, F, D = pp.partition(g, n_gpu, cap)
    assert F <= F0 and F < F_seq, (F, F0, F_seq)
    assert np.all(np.bincount(part, weights=g.size, minlength=n_gpu) <= cap * (1 + 1e-12))
    _, Fr = _ref(g, part, n_gpu)
    assert abs(F - Fr) <= 1e-9 * Fr
    # expected synapses of the graph equal the generator's in-degree
    assert abs(g.e_syn.sum() - spec.n * (spec.k_in + spec.k_cross)) < 1e-6 * spec.n * 100


def test_partition_errors():
    rng = np.random.default_rng(2)
    g = _tiny(rng)
    with pytest.raises(DtbError):
        pp.partition(g, 2, g.size.sum() / 3)                     # does not fit
    with pytest.raises(DtbError):
        pp.partition(g, 2, g.size.sum(), init=np.full(7, 5, np.int32))
    bad = pp.VertexGraph(**{**g.__dict__, "e_dst": np.full_like(g.e_dst, 99)})
    with pytest.raises(DtbError):
        pp.partition(bad, 2, g.size.sum())
