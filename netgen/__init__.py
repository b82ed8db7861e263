"""Seeded synthetic inputs for the conductance-LIF partition simulator.

This package only *makes inputs*: region sizes, the region-connection matrix,
the in-edge CSR (sources, integer delays, log-normal weights), per-neuron
parameter types, the initial membrane potentials and the background drive
level.  It contains none of the simulation arithmetic; both the GPU library
and the CPU reference consume what it produces.

Workload shapes follow the paper's network description (Sec. III-B and the
statistics table there): fixed in-degree per neuron, 80 % excitatory /
20 % inhibitory neurons per population, a sparse and heavy-tailed
region-to-region coupling, and a 1 ms time step (Sec. VI-A).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "netgen.c")
_LIB = os.path.join(_HERE, "_netgen.so")
_lib = None

# channel order used everywhere: AMPA, NMDA, GABAa, GABAb
CHANNELS = ("AMPA", "NMDA", "GABAa", "GABAb")


def build(force: bool = True) -> str:
    """Compile the generator's C core (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.netgen_fill.argtypes = [ctypes.c_int64, ctypes.c_int32, P, ctypes.c_int32,
                                    ctypes.c_int32, P, ctypes.c_int32, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_uint64, P, P, P]
        lib.netgen_fill.restype = ctypes.c_int
        lib.netgen_uniform.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_uint64, ctypes.c_uint64, P]
        lib.netgen_uniform.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


# Parameter-type record, field order shared by every consumer of a Network:
# C, gL, EL, Vth, Vreset, tref_ms, Iext, g_AMPA, g_NMDA, g_GABAa, g_GABAb
PTYPE_FIELDS = ("C", "gL", "EL", "Vth", "Vreset", "tref_ms", "Iext",
                "g_AMPA", "g_NMDA", "g_GABAa", "g_GABAb")


@dataclasses.dataclass
class Network:
    """One network partition, in the layout the simulator's C-ABI takes."""
    n: int
    n_regions: int
    max_delay: int
    row_ptr: np.ndarray      # int64 [n+1]
    col: np.ndarray          # int32 [nnz] presynaptic id
    w: np.ndarray            # float32 [nnz]
    delay: np.ndarray        # uint8 [nnz] in [1, max_delay]
    is_inh: np.ndarray       # uint8 [n]
    region: np.ndarray       # int32 [n]
    ptype: np.ndarray        # uint16 [n] index into ptypes
    ptypes: np.ndarray       # float32 [n_ptypes, 11] (PTYPE_FIELDS)
    V0: np.ndarray           # float32 [n]
    E: np.ndarray            # float32 [4] reversal potentials (mV)
    tau_ms: np.ndarray       # float32 [4] gate decay constants
    dt_ms: float
    bg_lambda: float         # mean background Poisson count per neuron-step
    bg_w: float              # weight of one background event
    seed: int                # background-drive seed
    member: int = 0          # ensemble member id (part of the background counter)
    region_start: Optional[np.ndarray] = None  # int64 [n_regions+1] when contiguous
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def region_sizes(self) -> np.ndarray:
        return np.bincount(self.region, minlength=self.n_regions).astype(np.int64)


@dataclasses.dataclass
class NetSpec:
    """Recipe for a synthetic network (all randomness seeded)."""
    n: int
    region_sizes: np.ndarray          # int64 [R], sums to n
    cross_w: np.ndarray               # float64 [R, R]: weight of source s -> target t (diag ignored)
    k_in: int = 70
    k_cross: int = 30
    e_frac: float = 0.8
    max_delay: int = 5
    w_mu: float = -1.0
    w_sigma: float = 0.5
    net_seed: int = 1
    v0_seed: int = 2
    bg_seed: int = 3
    bg_lambda: float = 0.25
    bg_w: Optional[float] = None      # default: mean of the weight distribution
    g: Sequence[float] = (0.01, 0.0005, 0.02, 0.0005)
    C: float = 1.0
    gL: float = 0.03
    EL: float = -75.0
    Vth: float = -50.0
    Vreset: float = -65.0
    tref_ms: float = 2.0
    Iext: float = 0.0
    E: Sequence[float] = (0.0, 0.0, -70.0, -100.0)
    tau_ms: Sequence[float] = (2.0, 40.0, 10.0, 50.0)
    dt_ms: float = 1.0
    member: int = 0
    name: str = ""


def make_network(spec: NetSpec) -> Network:
    lib = _load()
    R = int(len(spec.region_sizes))
    sizes = np.asarray(spec.region_sizes, dtype=np.int64)
    if int(sizes.sum()) != spec.n or (sizes <= 0).any():
        raise ValueError("region sizes must be positive and sum to n")
    start = np.zeros(R + 1, dtype=np.int64)
    np.cumsum(sizes, out=start[1:])
    cw = np.array(spec.cross_w, dtype=np.float64, copy=True).reshape(R, R)
    np.fill_diagonal(cw, 0.0)
    if (cw < 0).any():
        raise ValueError("cross weights must be non-negative")
    # row t of the cdf: cumulative over source regions s of cw[s, t]
    cdf = np.ascontiguousarray(np.cumsum(cw.T, axis=1))
    K = spec.k_in + spec.k_cross
    n = spec.n
    nnz = n * K
    col = np.empty(nnz, dtype=np.int32)
    delay = np.empty(nnz, dtype=np.uint8)
    w = np.empty(nnz, dtype=np.float32)
    rc = lib.netgen_fill(n, R, _ptr(start), spec.k_in, spec.k_cross, _ptr(cdf), spec.max_delay,
                         spec.w_mu, spec.w_sigma, spec.net_seed, _ptr(col), _ptr(delay), _ptr(w))
    if rc != 0:
        raise RuntimeError("netgen_fill failed (region too small for autapse-free draws?)")
    row_ptr = np.arange(n + 1, dtype=np.int64) * K
    region = np.repeat(np.arange(R, dtype=np.int32), sizes)
    is_inh = np.zeros(n, dtype=np.uint8)
    for r in range(R):
        n_e = int(np.floor(spec.e_frac * sizes[r] + 0.5))
        is_inh[start[r] + n_e:start[r + 1]] = 1
    V0 = np.empty(n, dtype=np.float32)
    lib.netgen_uniform(n, spec.Vreset, spec.Vth, spec.v0_seed, 1, _ptr(V0))
    ptypes = np.array([[spec.C, spec.gL, spec.EL, spec.Vth, spec.Vreset, spec.tref_ms, spec.Iext,
                        *spec.g]], dtype=np.float32)
    ptype = np.zeros(n, dtype=np.uint16)
    bg_w = spec.bg_w if spec.bg_w is not None else float(np.exp(spec.w_mu + 0.5 * spec.w_sigma ** 2))
    return Network(n=n, n_regions=R, max_delay=spec.max_delay, row_ptr=row_ptr, col=col, w=w,
                   delay=delay, is_inh=is_inh, region=region, ptype=ptype, ptypes=ptypes, V0=V0,
                   E=np.array(spec.E, dtype=np.float32), tau_ms=np.array(spec.tau_ms, dtype=np.float32),
                   dt_ms=float(spec.dt_ms), bg_lambda=float(spec.bg_lambda), bg_w=float(np.float32(bg_w)),
                   seed=int(spec.bg_seed), member=int(spec.member), region_start=start, name=spec.name)


@dataclasses.dataclass
class RemoteBlock:
    """In-edges of a partition's n rows from n_remote neurons held by other
    partitions (the J_inter sources of Sec. V-B)."""
    n_remote: int
    row_ptr: np.ndarray      # int64 [n+1]
    col: np.ndarray          # int32 [nnz] remote source id
    w: np.ndarray            # float32 [nnz]
    delay: np.ndarray        # uint8 [nnz] in [1, max_delay]
    is_inh: np.ndarray       # uint8 [n_remote]


def make_remote_block(n: int, n_remote: int, k_remote, max_delay: int = 5, w_mu: float = -1.0,
                      w_sigma: float = 0.5, e_frac: float = 0.8, seed: int = 11) -> RemoteBlock:
    """k_remote in-edges per row (an int, or an int array [n] for a ragged
    block) drawn uniformly from the remote sources, uniform integer delays in
    [1, max_delay], log-normal weights; the first round(e_frac n_remote)
    remote sources are excitatory."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = np.broadcast_to(np.asarray(k_remote, dtype=np.int64), (n,))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(k, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    col = rng.integers(0, n_remote, size=nnz, dtype=np.int32)
    delay = rng.integers(1, max_delay + 1, size=nnz, dtype=np.uint8)
    w = np.exp(rng.normal(w_mu, w_sigma, size=nnz)).astype(np.float32)
    is_inh = np.zeros(n_remote, dtype=np.uint8)
    is_inh[int(np.floor(e_frac * n_remote + 0.5)):] = 1
    return RemoteBlock(n_remote=int(n_remote), row_ptr=row_ptr, col=col, w=w, delay=delay, is_inh=is_inh)


def split_remote(net: Network):
    """Split every row into its own-region in-edges (kept by the partition:
    J_intra) and its cross-region ones (a remote block: J_inter), the split
    of Sec. V-B when a partition holds whole regions.  The remote sources are
    the same neuron ids held by a mirror partition, so replaying the
    network's own raster as the remote spikes reproduces the unsplit run.
    The generator emits each row's own-region sources first, so the split is
    a prefix / suffix of every row and keeps the row's summation order; a
    network whose rows are not in that order is rejected."""
    n = net.n
    rp = np.asarray(net.row_ptr, dtype=np.int64)
    row_of = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    own = net.region[net.col] == net.region[row_of]
    n_own = np.bincount(row_of, weights=own, minlength=n).astype(np.int64)
    # own-region entries must be each row's prefix
    pos = np.arange(net.nnz, dtype=np.int64) - rp[row_of]
    if not np.array_equal(own, pos < n_own[row_of]):
        raise ValueError("split_remote needs rows with their own-region sources first")
    del row_of, pos
    lrp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(n_own, out=lrp[1:])
    rrp = rp - lrp
    local = dataclasses.replace(net, row_ptr=lrp, col=net.col[own], w=net.w[own], delay=net.delay[own])
    cross = ~own
    del own
    blk = RemoteBlock(n_remote=n, row_ptr=rrp, col=net.col[cross], w=net.w[cross], delay=net.delay[cross],
                      is_inh=net.is_inh.copy())
    return local, blk


def embed_independent(sub: Network, rest: Network, name: str = "") -> Network:
    """One partition holding `sub` as an independent subgraph - no synapse
    into or out of it - in its first sub.n neurons, followed by `rest` with
    its ids and populations shifted behind it (the accuracy check of
    Sec. VII-B embeds such a subgraph in a large network).  The background
    seed is sub's and neuron ids are unchanged for sub, so its neurons draw
    exactly the background they draw alone; sub's populations keep their
    ids.  Both parts must share the model constants and the drive."""
    for f in ("dt_ms", "bg_lambda", "bg_w"):
        if getattr(sub, f) != getattr(rest, f):
            raise ValueError(f"embed_independent: {f} differs")
    if not (np.array_equal(sub.E, rest.E) and np.array_equal(sub.tau_ms, rest.tau_ms)
            and np.array_equal(sub.ptypes, rest.ptypes)):
        raise ValueError("embed_independent: model constants differ")
    n, nnz = sub.n + rest.n, sub.nnz + rest.nnz
    row_ptr = np.empty(n + 1, dtype=np.int64)
    row_ptr[:sub.n + 1] = sub.row_ptr
    np.add(rest.row_ptr[1:], sub.nnz, out=row_ptr[sub.n + 1:])
    col = np.empty(nnz, dtype=np.int32)
    col[:sub.nnz] = sub.col
    np.add(rest.col, np.int32(sub.n), out=col[sub.nnz:])
    w = np.empty(nnz, dtype=np.float32)
    w[:sub.nnz] = sub.w
    w[sub.nnz:] = rest.w
    delay = np.empty(nnz, dtype=np.uint8)
    delay[:sub.nnz] = sub.delay
    delay[sub.nnz:] = rest.delay
    start = None
    if sub.region_start is not None and rest.region_start is not None:
        start = np.concatenate([sub.region_start, rest.region_start[1:] + sub.n])
    return Network(n=n, n_regions=sub.n_regions + rest.n_regions, max_delay=max(sub.max_delay, rest.max_delay),
                   row_ptr=row_ptr, col=col, w=w, delay=delay, is_inh=np.concatenate([sub.is_inh, rest.is_inh]),
                   region=np.concatenate([sub.region, rest.region + sub.n_regions]).astype(np.int32),
                   ptype=np.concatenate([sub.ptype, rest.ptype]), ptypes=sub.ptypes,
                   V0=np.concatenate([sub.V0, rest.V0]), E=sub.E, tau_ms=sub.tau_ms, dt_ms=sub.dt_ms,
                   bg_lambda=sub.bg_lambda, bg_w=sub.bg_w, seed=sub.seed, member=sub.member,
                   region_start=start, name=name or f"embedded({sub.name} in {rest.name})")


def remote_raster(n_steps: int, n_remote: int, rate_hz: float, dt_ms: float = 1.0, seed: int = 12) -> np.ndarray:
    """Replayed remote spikes: independent Bernoulli(rate dt) per neuron-step,
    uint8 [n_steps, n_remote]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = rate_hz * dt_ms * 1e-3
    return (rng.random((n_steps, n_remote), dtype=np.float32) < p).astype(np.uint8)


from .configs import *  # noqa: E402,F401,F403
