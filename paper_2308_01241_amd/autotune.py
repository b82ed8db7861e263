"""Launch-shape autotuner of the gather (binding of dtb_autotune).

Four knobs, none of which changes any result (the summation order is each
row's CSR order either way):

* the bundle size (most synapses per workgroup): it sets the LDS hit bitmap
  per workgroup, hence how many workgroups share a CU, against the number
  of bitmap sweeps (each bundle reads the delayed spike bits of its sources
  once per delay); sizes that make the bundle count a whole number of
  rounds over the CUs avoid a partly idle last round;
* the lookup tiles per wavefront per round (1, 2 or 3): bytes in flight per
  wavefront against registers;
* where the row sums run (1: in the gather's workgroups from the LDS hit
  bitmap, 2: in a separate kernel over the hit buffer): one launch and no
  hit-buffer traffic against a phase per bundle in which its CU issues
  only the rows' random weight loads;
* how the delivery tests are found (1: the pull sweep of every synapse over
  the delayed spike bitmaps, 2: spike-driven, the last D steps' spikes each
  delivering through their out-synapses of the matching delay): bytes per
  synapse against bytes per delivered event.

The library times each candidate on the real network with HIP events, all
from one burned-in state, and caches the winner in a JSON file keyed by GPU
architecture and network shape.  `tuned.json` next to this file holds the
entries measured for the shipped workloads; `lookup` reads it.
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np

from ._lib import TUNE_MAX_BUNDLES, Desc, TuneResult, check, load
from .net import _make_desc, _ptr, _stream_handle

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuned.json")


def shape_key(arch: str, n: int, nnz: int, n_members: int, wtype: str, max_delay: int) -> str:
    """The cache key dtb_autotune writes."""
    return f"{arch}|n={n},nnz={nnz},members={n_members},w={wtype},D={max_delay}"


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def lookup(n, nnz, n_members=1, wtype="f32", max_delay=20, path=CACHE, arch=None):
    """Cached (bundle_syn, unroll, fuse, events) for this shape, or
    (0, 0, 0, 0) (the library defaults)."""
    try:
        with open(path) as f:
            db = json.load(f)
    except (OSError, ValueError):
        return 0, 0, 0, 0
    ent = db.get(shape_key(arch or _arch(), n, nnz, n_members, wtype, max_delay))
    if not ent:
        return 0, 0, 0, 0
    return int(ent["bundle_syn"]), int(ent["unroll"]), int(ent.get("fuse", 0)), int(ent.get("events", 0))


def tune(members, wtype: str = "f32", record_steps: int = 64, cache_path=CACHE, bundles=(), burnin: int = 0,
         steps: int = 20, stream=None) -> dict:
    """dtb_autotune over the network(s) `members` (one: a plain partition,
    several: a batch).  Returns the winning shape, its ms per step, whether
    it came from the cache, and every timed (bundle_syn, unroll, fuse, events) -> ms."""
    lib = load()
    members = list(members)
    descs = (Desc * len(members))()
    keep = []
    for m, nw in enumerate(members):
        d, k = _make_desc(nw, wtype, record_steps)
        descs[m] = d
        keep.append(k)
    cands = np.ascontiguousarray(bundles, dtype=np.int32)
    if cands.size > TUNE_MAX_BUNDLES:
        raise ValueError(f"at most {TUNE_MAX_BUNDLES} bundle candidates")
    res = TuneResult()
    check(lib.dtb_autotune(descs, len(members), _stream_handle(stream),
                           None if cache_path is None else str(cache_path).encode(),
                           _ptr(cands) if cands.size else None, int(cands.size), int(burnin), int(steps),
                           ctypes.byref(res)))
    del keep
    tried = {(int(res.tried_bundle[q]), int(res.tried_unroll[q]), int(res.tried_fuse[q]),
              int(res.tried_events[q])): float(res.tried_ms[q]) for q in range(res.n_tried)}
    return {"bundle_syn": int(res.bundle_syn), "unroll": int(res.unroll), "fuse": int(res.fuse),
            "events": int(res.events), "ms_per_step": float(res.ms_per_step),
            "from_cache": bool(res.from_cache), "tried": tried}
