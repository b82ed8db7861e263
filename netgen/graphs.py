"""Vertex graphs for the neuron-to-GPU partitioner: populations cut into
pieces, with the expected synapse counts of the generator's construction
(inputs only; no partitioning arithmetic)."""
from __future__ import annotations

import dataclasses

import numpy as np


# bytes per neuron (state, parameters, ring bits) and per in-synapse
# (4-byte lookup entry + 4-byte weight + a share of the tile headers)
NEURON_BYTES = 60.0
SYNAPSE_BYTES = 8.1


@dataclasses.dataclass
class VertexGraph:
    size: np.ndarray      # float64 [V] bytes
    neurons: np.ndarray   # float64 [V]
    spikes: np.ndarray    # float64 [V] spikes per step
    e_ptr: np.ndarray     # int64 [V+1]
    e_dst: np.ndarray     # int32 [E]
    e_syn: np.ndarray     # float64 [E] expected synapses from source to destination vertex
    region: np.ndarray    # int32 [V] population of each vertex


def region_graph(region_sizes, cross_w, k_in: int, k_cross: int, rate_hz: float, dt_ms: float = 1.0,
                 chunk: int = 1_000_000) -> VertexGraph:
    """Expected synapses of the generator's construction: a neuron of
    population t draws k_in sources uniformly from t and k_cross from the
    other populations s in proportion to cross_w[s, t], uniformly inside s."""
    sizes = np.asarray(region_sizes, dtype=np.int64)
    R = len(sizes)
    M = np.array(cross_w, dtype=np.float64).reshape(R, R)
    np.fill_diagonal(M, 0.0)
    colsum = M.sum(axis=0)
    pieces = []   # (region, neurons)
    for r in range(R):
        k = max(1, int(np.ceil(sizes[r] / chunk)))
        base, extra = divmod(int(sizes[r]), k)
        pieces += [(r, base + (1 if q < extra else 0)) for q in range(k)]
    reg = np.array([p[0] for p in pieces], dtype=np.int32)
    nn = np.array([p[1] for p in pieces], dtype=np.float64)
    V = len(pieces)
    # synapses from piece a (population s) onto piece b (population t):
    # n_b * (k_in [s == t] + k_cross M[s, t] / colsum[t]) * n_a / n_s
    share = np.where(np.eye(R, dtype=bool), float(k_in),
                     k_cross * np.divide(M, colsum[None, :], out=np.zeros_like(M), where=colsum[None, :] > 0))
    syn = share[reg[:, None], reg[None, :]] * nn[None, :] * (nn[:, None] / sizes[reg][:, None])
    e_ptr = np.zeros(V + 1, dtype=np.int64)
    dst, w = [], []
    for a in range(V):
        nz = np.nonzero(syn[a] > 0)[0]
        dst.append(nz.astype(np.int32))
        w.append(syn[a, nz])
        e_ptr[a + 1] = e_ptr[a] + len(nz)
    indeg = k_in + k_cross
    return VertexGraph(size=nn * (NEURON_BYTES + SYNAPSE_BYTES * indeg), neurons=nn,
                       spikes=nn * rate_hz * dt_ms * 1e-3, e_ptr=e_ptr, e_dst=np.concatenate(dst),
                       e_syn=np.concatenate(w), region=reg)
