"""Neuron-to-GPU partitioning (Sec. V-C, Eq. (2)) through the library's
host-side partitioner ``dtb_partition`` (no GPU needed).

``region_graph`` turns a network description (population sizes, the
region-to-region matrix and the in-degree split of the generator) into the
partitioner's vertex graph: each population cut into pieces of at most
``chunk`` neurons, the expected synapse counts between pieces, each piece's
memory size (neuron state plus its in-synapses) and its spikes per step."""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np

from ._lib import check, load

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


def partition(g: VertexGraph, n_gpu: int, capacity: float, bytes_per_spike: float = 4.0, init=None,
              refine_rounds: int = 2000):
    """Returns (part int32 [V], F bytes per step, D [n_gpu, n_gpu])."""
    lib = load()
    V = len(g.neurons)
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (g.size, g.neurons, g.spikes)]
    e_ptr = np.ascontiguousarray(g.e_ptr, dtype=np.int64)
    e_dst = np.ascontiguousarray(g.e_dst, dtype=np.int32)
    e_syn = np.ascontiguousarray(g.e_syn, dtype=np.float64)
    ini = None if init is None else np.ascontiguousarray(init, dtype=np.int32)
    part = np.zeros(V, dtype=np.int32)
    D = np.zeros((n_gpu, n_gpu), dtype=np.float64)
    F = ctypes.c_double(0.0)

    def p(a):
        return None if a is None else ctypes.c_void_p(a.ctypes.data)

    check(lib.dtb_partition(V, p(arrs[0]), p(arrs[1]), p(arrs[2]), p(e_ptr), p(e_dst), p(e_syn), int(n_gpu),
                            float(capacity), float(bytes_per_spike), p(ini), int(refine_rounds), p(part),
                            ctypes.byref(F), p(D)))
    return part, float(F.value), D


def sequential(g: VertexGraph, n_gpu: int) -> np.ndarray:
    """The baseline the paper compares with: vertices in population order cut
    into n_gpu contiguous runs of about equal size."""
    c = np.cumsum(g.size) - 0.5 * g.size
    return np.minimum((c / g.size.sum() * n_gpu).astype(np.int32), n_gpu - 1)


def main():
    """Partition the generator's population graph at N x 20M neurons for each
    N given and compare with the sequential cut; prints one JSON report."""
    import argparse
    import json
    import time

    import netgen

    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, nargs="+", default=[8, 64])
    ap.add_argument("--per-gpu", type=int, default=20_000_000)
    ap.add_argument("--chunk", type=int, default=1_000_000)
    ap.add_argument("--rate", type=float, default=7.0)
    ap.add_argument("--slack", type=float, default=1.1)
    ap.add_argument("--out", type=str, default="")
    a = ap.parse_args()
    rep = []
    for N in a.gpus:
        spec = netgen.partition_spec(n=N * a.per_gpu, n_regions=90)
        g = region_graph(spec.region_sizes, spec.cross_w, spec.k_in, spec.k_cross, rate_hz=a.rate, chunk=a.chunk)
        cap = g.size.sum() / N * a.slack
        seq = sequential(g, N)
        _, F_seq, D_seq = partition(g, N, g.size.sum(), init=seq, refine_rounds=0)
        t = time.perf_counter()
        _, F_greedy, _ = partition(g, N, cap, refine_rounds=0)
        t_greedy = time.perf_counter() - t
        t = time.perf_counter()
        part, F, D = partition(g, N, cap)
        t_all = time.perf_counter() - t
        load = np.bincount(part, weights=g.size, minlength=N)
        rep.append({"n_gpu": N, "neurons": int(spec.n), "vertices": int(len(g.size)),
                    "F_sequential_MB_per_step": F_seq / 1e6, "F_greedy_MB_per_step": F_greedy / 1e6,
                    "F_MB_per_step": F / 1e6, "F_ratio_vs_sequential": F / F_seq,
                    "total_traffic_MB_per_step": float(D.sum()) / 1e6,
                    "total_traffic_sequential_MB_per_step": float(D_seq.sum()) / 1e6,
                    "load_max_over_mean": float(load.max() / load.mean()),
                    "seconds_greedy": t_greedy, "seconds_total": t_all})
    txt = json.dumps({"capacity_slack": a.slack, "chunk": a.chunk, "rate_hz": a.rate, "runs": rep}, indent=1)
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt)
    print(txt)


if __name__ == "__main__":
    main()
