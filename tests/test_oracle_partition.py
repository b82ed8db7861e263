"""Pins of the reference's partition objective (Sec. V-C, Eq. (2)).

* the traffic model (a spike goes to a GPU once when its neuron has a target
  there, probability 1 - exp(-c / n)) against a direct count on explicitly
  drawn random synapses;
* hand-computed D and F; one GPU has no traffic; GPU labels do not matter;
* brute force finds a partition no worse than any other on a tiny graph.
"""
import numpy as np

from oracle import partition as op


def _graph(rng, V, n_lo=500, n_hi=3000, density=0.6):
    nn = rng.integers(n_lo, n_hi, V).astype(np.float64)
    e_ptr, dst, syn = [0], [], []
    for u in range(V):
        for v in range(V):
            if rng.random() < density:
                dst.append(v)
                syn.append(float(rng.integers(100, 4000)))
        e_ptr.append(len(dst))
    return nn, np.array(e_ptr, np.int64), np.array(dst, np.int32), np.array(syn)


def test_traffic_model_matches_a_direct_count_of_explicit_synapses():
    rng = np.random.default_rng(0)
    V, N = 6, 3
    nn, e_ptr, e_dst, e_syn = _graph(rng, V)
    part = np.array([0, 0, 1, 1, 2, 2])
    spikes = nn.copy()            # every neuron spikes once: D counts neurons with a target on j
    D, F = op.traffic(part, nn, nn, spikes, e_ptr, e_dst, e_syn, N, b=1.0)
    # draw every synapse explicitly: a uniformly chosen source neuron of u
    has = [np.zeros((int(nn[u]), N), bool) for u in range(V)]
    for u in range(V):
        for e in range(e_ptr[u], e_ptr[u + 1]):
            src = rng.integers(0, int(nn[u]), int(e_syn[e]))
            has[u][src, part[e_dst[e]]] = True
    Dc = np.zeros((N, N))
    for u in range(V):
        cnt = has[u].sum(axis=0)
        for j in range(N):
            if j != part[u]:
                Dc[part[u], j] += cnt[j]
    # binomial sampling error of the counts, plus the Poisson approximation's O(c / n^2)
    sd = np.sqrt(np.maximum(D, 1.0))
    assert np.all(np.abs(Dc - D) < 5 * sd + 0.002 * D), (Dc, D)


def test_hand_computed_traffic():
    nn = np.array([1000.0, 400.0])
    spikes = np.array([10.0, 3.0])
    e_ptr = np.array([0, 1, 1], np.int64)
    D, F = op.traffic([0, 1], nn, nn, spikes, e_ptr, np.array([1], np.int32), np.array([500.0]), 2, b=4.0)
    assert D[0, 1] == 4.0 * 10.0 * (1.0 - np.exp(-0.5))
    assert D[1, 0] == 0.0 and F == D[0, 1]
    assert abs(F - 15.7387736115) < 1e-8          # 40 (1 - e^-0.5)
    D1, F1 = op.traffic([0, 0], nn, nn, spikes, e_ptr, np.array([1], np.int32), np.array([500.0]), 1)
    assert F1 == 0.0


def test_labels_do_not_matter_and_brute_force_is_optimal():
    rng = np.random.default_rng(1)
    V, N = 6, 3
    nn, e_ptr, e_dst, e_syn = _graph(rng, V)
    size = nn.copy()
    spikes = 0.01 * nn
    part = rng.integers(0, N, V)
    _, F = op.traffic(part, size, nn, spikes, e_ptr, e_dst, e_syn, N)
    perm = np.array([2, 0, 1])
    _, Fp = op.traffic(perm[part], size, nn, spikes, e_ptr, e_dst, e_syn, N)
    assert abs(F - Fp) < 1e-9 * F
    cap = size.sum() / N * 1.5
    Fb, pb = op.brute_force(size, nn, spikes, e_ptr, e_dst, e_syn, N, cap)
    assert np.all(np.bincount(pb, weights=size, minlength=N) <= cap)
    for _ in range(200):
        a = rng.integers(0, N, V)
        if np.all(np.bincount(a, weights=size, minlength=N) <= cap):
            assert op.traffic(a, size, nn, spikes, e_ptr, e_dst, e_syn, N)[1] >= Fb - 1e-9
