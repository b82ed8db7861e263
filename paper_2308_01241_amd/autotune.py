"""Autotuner for the gather's launch shape.

The knob is the bundle size (most synapses per workgroup): it sets the LDS
hit bitmap per workgroup (hence workgroups per CU) against the bitmap
bytes each workgroup sweeps.  Results do not depend on it (the summation
order is each row's CSR order either way), only the time does.  The tuner
times each candidate on the real network with HIP events and caches the
winner in JSON, keyed by GPU architecture and network shape.

`tuned.json` next to this file holds the entries measured for the shipped
workloads; `lookup` reads it (or another cache file).
"""
from __future__ import annotations

import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuned.json")
CANDIDATES = (1 << 18, 1 << 19, (1 << 20) - 1)


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def shape_key(n: int, nnz: int, n_members: int, wtype: str, max_delay: int) -> str:
    return f"n={n},nnz={nnz},members={n_members},w={wtype},D={max_delay}"


def lookup(n, nnz, n_members=1, wtype="f32", max_delay=20, path=CACHE, arch=None):
    """Cached bundle size for this shape, or 0 (library default)."""
    try:
        with open(path) as f:
            db = json.load(f)
    except (OSError, ValueError):
        return 0
    arch = arch or _arch()
    ent = db.get(arch, {}).get(shape_key(n, nnz, n_members, wtype, max_delay))
    return int(ent["bundle_syn"]) if ent else 0


def tune(make_net, key: str, candidates=CANDIDATES, steps: int = 40, warmup: int = 10, path=CACHE, log=print):
    """make_net(bundle_syn) -> Net.  Times `steps` steps per candidate and
    records the fastest under (arch, key) in `path`."""
    import torch
    res = {}
    for c in candidates:
        t0 = time.time()
        net = make_net(c)
        net.step(warmup)
        net.sync()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        net.step(steps)
        b.record()
        torch.cuda.synchronize()
        res[c] = a.elapsed_time(b) / steps
        net.close()
        log(f"[autotune] bundle_syn={c}: {res[c]:.3f} ms/step (built and timed in {time.time() - t0:.1f}s)")
    best = min(res, key=res.get)
    arch = _arch()
    try:
        with open(path) as f:
            db = json.load(f)
    except (OSError, ValueError):
        db = {}
    db.setdefault(arch, {})[key] = {"bundle_syn": int(best), "ms_per_step": {str(k): v for k, v in res.items()}}
    with open(path, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    return best, res
