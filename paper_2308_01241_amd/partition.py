"""Neuron-to-GPU partitioning (Sec. V-C, Eq. (2)) through the library's
host-side partitioner ``dtb_partition`` (no GPU needed).

The vertex graphs come from ``netgen.graphs.region_graph`` (populations cut
into pieces of at most ``chunk`` neurons, the expected synapse counts of
the generator's construction, each piece's memory size and spikes per
step), re-exported here."""
from __future__ import annotations

import ctypes

import numpy as np

from netgen.graphs import NEURON_BYTES, SYNAPSE_BYTES, VertexGraph, region_graph  # noqa: F401

from ._lib import check, load


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
