"""FP64 reference of the partitioner's objective (Sec. V-C, Eq. (2)).

TEST INFRASTRUCTURE ONLY (see the package docstring).

traffic(): D_ij = b sum_{u on i} s_u (1 - exp(-c_uj / n_u)) for i != j, with
c_uj the synapses from vertex u onto the vertices of GPU j; F = max_j of the
column sums.  Pinned by a direct count of neurons with targets on each GPU
in explicitly drawn random graphs, and by hand-computed cases.
brute_force(): the exact minimum of F over every assignment that respects
the capacity, for tiny graphs.
"""
from __future__ import annotations

import itertools

import numpy as np


def traffic(part, size, neurons, spikes, e_ptr, e_dst, e_syn, n_gpu, b=4.0):
    part = np.asarray(part)
    V = len(part)
    c = np.zeros((V, n_gpu))
    for u in range(V):
        for e in range(int(e_ptr[u]), int(e_ptr[u + 1])):
            c[u, part[e_dst[e]]] += e_syn[e]
    D = np.zeros((n_gpu, n_gpu))
    for u in range(V):
        for j in range(n_gpu):
            if j != part[u]:
                D[part[u], j] += b * spikes[u] * (1.0 - np.exp(-c[u, j] / neurons[u]))
    return D, float(D.sum(axis=0).max()) if n_gpu > 0 else 0.0


def brute_force(size, neurons, spikes, e_ptr, e_dst, e_syn, n_gpu, capacity, b=4.0):
    V = len(size)
    best = (np.inf, None)
    for a in itertools.product(range(n_gpu), repeat=V):
        load = np.bincount(a, weights=size, minlength=n_gpu)
        if np.any(load > capacity):
            continue
        _, F = traffic(a, size, neurons, spikes, e_ptr, e_dst, e_syn, n_gpu, b)
        if F < best[0]:
            best = (F, np.array(a))
    return best
