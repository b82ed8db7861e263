"""Autotuner for the gather's launch shape.

Two knobs, neither of which changes any result (the summation order is each
row's CSR order either way):

* the bundle size (most synapses per workgroup): it sets the LDS hit bitmap
  per workgroup, hence how many workgroups share a CU, against the number
  of bitmap sweeps (each bundle reads the delayed spike bits of its sources
  once per delay); sizes that make the bundle count a whole number of
  rounds over the CUs avoid a partly idle last round;
* the lookup tiles per wavefront per round (1, 2 or 3): bytes in flight per
  wavefront against registers (one tile per round fits 64 VGPRs, i.e. two
  1024-thread workgroups per CU).

The tuner times each candidate on the real network with HIP events and
caches the winner in JSON, keyed by GPU architecture and network shape.
`tuned.json` next to this file holds the entries measured for the shipped
workloads; `lookup` reads it (or another cache file).
"""
from __future__ import annotations

import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuned.json")
BUNDLES = (393_216, 640_000, (1 << 20) - 1)
UNROLLS = (1, 2, 3)


def aligned_bundle_sizes(n: int, nnz: int, n_cu: int, max_syn: int = (1 << 20) - 1, counts=(1, 2)):
    """Bundle sizes whose bundle count is a whole number of rounds over the
    CUs (one workgroup per CU at a time): for the smallest k rounds that
    respect max_syn and the next count - 1 after it, the size that cuts the
    rows (mean length nnz / n) into at most k * n_cu bundles."""
    if n <= 0 or nnz <= 0:
        return ()
    L = nnz / n
    k = max(1, -(-nnz // (max_syn * n_cu)))
    out = []
    for kk in range(k, k + len(counts)):
        rows = -(-n // (kk * n_cu))
        b = int(rows * L + 0.5)
        if b <= max_syn:
            out.append(b)
    return tuple(out)


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def shape_key(n: int, nnz: int, n_members: int, wtype: str, max_delay: int) -> str:
    return f"n={n},nnz={nnz},members={n_members},w={wtype},D={max_delay}"


def lookup(n, nnz, n_members=1, wtype="f32", max_delay=20, path=CACHE, arch=None):
    """Cached (bundle_syn, unroll) for this shape, or (0, 0) (library defaults)."""
    try:
        with open(path) as f:
            db = json.load(f)
    except (OSError, ValueError):
        return 0, 0
    arch = arch or _arch()
    ent = db.get(arch, {}).get(shape_key(n, nnz, n_members, wtype, max_delay))
    return (int(ent["bundle_syn"]), int(ent.get("unroll", 0))) if ent else (0, 0)


def tune(make_net, key: str, bundles=BUNDLES, unrolls=UNROLLS, steps: int = 40, warmup: int = 10, path=CACHE,
         log=print):
    """make_net(bundle_syn, unroll) -> Net.  Times `steps` steps per
    candidate and records the fastest under (arch, key) in `path`."""
    import torch
    res = {}
    for b in bundles:
        for u in unrolls:
            t0 = time.time()
            net = make_net(b, u)
            net.step(warmup)
            net.sync()
            a = torch.cuda.Event(enable_timing=True)
            e = torch.cuda.Event(enable_timing=True)
            a.record()
            net.step(steps)
            e.record()
            torch.cuda.synchronize()
            res[(b, u)] = a.elapsed_time(e) / steps
            net.close()
            log(f"[autotune] bundle_syn={b} unroll={u}: {res[(b, u)]:.3f} ms/step "
                f"(built and timed in {time.time() - t0:.1f}s)")
    best = min(res, key=res.get)
    arch = _arch()
    try:
        with open(path) as f:
            db = json.load(f)
    except (OSError, ValueError):
        db = {}
    db.setdefault(arch, {})[key] = {"bundle_syn": int(best[0]), "unroll": int(best[1]),
                                    "ms_per_step": {f"{b}/{u}": v for (b, u), v in res.items()}}
    with open(path, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    return best, res
