#!/usr/bin/env python3
"""Benchmark: one GPU's partition of the conductance-LIF network.

Workload (default): 20,000,000 neurons in 90 log-normally sized regions,
in-degree 100 (2e9 synapses), delays 1-20 steps, dt = 1 ms, background
drive tuned to ~7 / 15 / 30 Hz.  A "step" is one pass of the whole hot path
(membrane update + spike bitmap + compaction + delivery through the delay
ring, spike-driven or by the pull sweep as the tuned launch shape says +
background + gate update + counters).  Inputs are synthetic and seeded
(netgen), resident in HBM before timing starts.

Each rate's network is first run to its stationary firing (`--burnin` steps,
untimed, whatever `--warmup` is), then `--warmup` more steps; that state is
saved, and every one of `--reps` repetitions loads it and times exactly
`--steps` steps, so all repetitions do the same work (median, min and max
reported); one more identical repetition times every kernel with HIP events
(the per-kernel durations and the roofline).  The run fails (exit status 3,
after the JSON line) when the measured mean rate of a point is more than
15 % from its target.

Prints one JSON line.  `value` is synaptic events/s of the plain FP32 path
at the 7 Hz point; the other rates, the realtime factor, the gather roofline,
the BF16 / OU / split / batched forms and the FP64 reference timed on the
host (a bounded sample) ride along.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "synaptic events/s & realtime factor, plain vs BF16/batched; surrogate err"
TRAFFIC_JSON = {"sweep": os.path.join(ROOT, "profiles", "gather_traffic_partition20M_7hz.json"),
                "spike-driven": os.path.join(ROOT, "profiles", "gather_events_traffic_partition20M_7hz.json")}
# the kernels and the constants that shape them (LDS layout, tile sizes)
KERNEL_SRCS = [os.path.join(ROOT, "paper_2308_01241_amd", "csrc", f) for f in ("dtb_kernels.hip", "dtb_internal.h")]
HBM_PEAK_GBS = 8000.0
RATE_TOLERANCE = 0.15
OU_BACKGROUND = (0.6, 0.4, 8.0)  # mu, sigma (units of Iext), tau (ms)


def measured_traffic(kernel: str = "k_gather", delivery: str = "sweep"):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    that delivery mode, or None when the kernel source changed since those
    counters were taken (the summary stores the SHA-256 of the kernel
    sources, concatenated in KERNEL_SRCS order)."""
    import hashlib
    try:
        with open(TRAFFIC_JSON[delivery]) as f:
            tj = json.load(f)
        h = hashlib.sha256()
        for src in KERNEL_SRCS:
            with open(src, "rb") as f:
                h.update(f.read())
        h = h.hexdigest()
    except OSError:
        return None
    if tj.get("kernel_source_sha256") != h or kernel not in tj.get("per_launch", {}):
        return None
    t = tj["per_launch"][kernel]
    return float(t["read_bytes"] + t["write_bytes"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def gather_bytes(nnz: int, n: int, max_delay: int) -> float:
    """Algorithmic bytes of the delivery tests: 5 B of index + delay per
    synapse and the D+1 delayed spike bits per neuron."""
    return 5.0 * nnz + n * (max_delay + 1) / 8.0


def rows_bytes(n: int, events: float, w_bytes: int) -> float:
    """Algorithmic bytes of the row sums that follow the delivery tests:
    row pointers (8 B per row), the weight of each delivered event, the
    step's Poisson background count (2 B per row, drawn by k_background) and
    the four gates read and written."""
    return 8.0 * n + w_bytes * events + 2.0 * n + 32.0 * n


def step_bytes(nnz: int, n: int, max_delay: int, events: float, w_bytes: int) -> float:
    """Algorithmic bytes of one whole step as the pull method needs them:
    index + delay per synapse, the delivered weights, the neuron state read
    and written with its parameter index, and the delayed spike bits."""
    return 5.0 * nnz + w_bytes * events + n * (2 * 21 + 2) + n * (max_delay + 1) / 8.0


def events_bytes(events: float, spikes: float, max_delay: int) -> float:
    """Algorithmic bytes of the spike-driven bucketing (k_events): per
    delivered event its table pair (target, weight) read and its bucket pair
    written (8 B each); per spike and delay the two offsets of its run in the
    table (gathered into rows by k_spike_runs)."""
    return 16.0 * events + spikes * max_delay * 8.0


def step_bytes_events(n: int, max_delay: int, events: float, spikes: float, w_bytes: int) -> float:
    """Algorithmic bytes of one whole step as spike-driven delivery needs
    them: per delivered event its table entry and weight, per spike and
    delay its run offsets and id, the neuron state read and written with its
    parameter index, and the row pointers of the fixed-order row sums."""
    return (4.0 + w_bytes) * events + spikes * max_delay * 12.0 + n * (2 * 21 + 2) + 8.0 * n


def roofline(per, ms_step, n_syn, n_neu, n_del, ev_step, spk_step, wb):
    """The roofline object of the dominant kernel of the gather stage, with
    the other gather kernel and the step as a whole beside it.

    Sweep mode: the delivery tests of k_gather stream every synapse's index
    and delay (5 B) and the D+1 spike bitmaps; with the row sums fused in the
    same workgroups (fuse 1) their bytes are added, with separate sums (fuse
    2) k_sums gets its own line.  Spike-driven mode: k_events buckets each
    delivered event, k_gather (the consumer) reads the bucket pairs (target
    and weight, 8 B per event) and, fused, does the row sums; whichever of the
    two took longer per launch is the dominant kernel.  The step is priced
    both by its own method's bytes and by the pull method's (the time the
    pull method would need at peak bandwidth)."""
    spike_driven = per.get("events", 0.0) > 0.0
    fused = per.get("sums", 0.0) == 0.0
    delivery = "spike-driven" if spike_driven else "sweep"
    Br = rows_bytes(n_neu, ev_step, wb)
    if spike_driven:
        Bg = 4.0 * ev_step
        Bt = step_bytes_events(n_neu, n_del, ev_step, spk_step, wb)
    else:
        Bg = gather_bytes(n_syn, n_neu, n_del)
        Bt = step_bytes(n_syn, n_neu, n_del, ev_step, wb)
    B = Bg + Br if fused else Bg + n_syn / 8.0
    step_gbs = Bt / (ms_step * 1e-3) / 1e9
    lines = {"k_gather": (B, per["gather"])}
    if spike_driven:
        lines["k_events"] = (events_bytes(ev_step, spk_step, n_del), per["events"])
    main = max(lines, key=lambda k: lines[k][1])
    Bm, tm = lines[main]
    achieved = Bm / (tm * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(main, delivery),
            "kernel": main, "delivery": delivery, "row_sums_in_gather": fused,
            "algorithmic_bytes_per_launch": Bm, "avg_launch_ms": tm,
            "step": {"algorithmic_bytes": Bt, "ms": ms_step, "achieved": round(step_gbs, 1),
                     "frac": round(step_gbs / HBM_PEAK_GBS, 4)}}
    for k, (Bk, tk) in lines.items():
        if k != main:
            roof["consumer" if k == "k_gather" else "bucketing"] = {
                "kernel": k, "algorithmic_bytes_per_launch": Bk, "avg_launch_ms": tk,
                "achieved": round(Bk / (tk * 1e-3) / 1e9, 1), "frac": round(Bk / (tk * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(k, delivery)}
    if spike_driven:
        Bp = step_bytes(n_syn, n_neu, n_del, ev_step, wb)
        roof["step"]["pull_method_bytes"] = Bp
        roof["step"]["pull_method_ms_at_peak"] = round(Bp / (HBM_PEAK_GBS * 1e9) * 1e3, 4)
    if fused:
        roof["gather_parts"] = {("bucket_reads" if spike_driven else "delivery_tests"): Bg, "row_sums": Br}
    else:
        Bs = Br + n_syn / 8.0  # the sums read one hit bit per synapse
        roof["hit_bits_written_per_launch"] = n_syn / 8.0
        roof["sums"] = {"kernel": "k_sums", "algorithmic_bytes_per_launch": Bs, "avg_launch_ms": per["sums"],
                        "achieved": round(Bs / (per["sums"] * 1e-3) / 1e9, 1)}
    return roof


def _shape_dict(shape):
    """The gather's launch shape as reported (None = library default)."""
    return {k: (v or None) for k, v in zip(("bundle_syn", "unroll", "fuse", "events"), shape)}


def _spread(xs):
    xs = sorted(xs)
    return {"median": float(np.median(xs)), "min": float(xs[0]), "max": float(xs[-1]), "n": len(xs)}


def run_rate(net, rate, lam, steps, warmup, burnin, reps, wtype, shape=(0, 0, 0, 0), ou=None, keep_bits=False):
    """One rate point: burn in to the stationary rate, save, then `reps`
    timed repetitions of `steps` steps from that same state, and one more
    with per-kernel HIP event timing."""
    import torch
    import paper_2308_01241_amd as dtb

    net.bg_lambda = lam
    t0 = time.time()
    pre = burnin + warmup
    rec = pre + steps if keep_bits else max(steps, 16)
    g = dtb.Net(net, wtype=wtype, record_steps=rec, stream=torch.cuda.current_stream(),
                bundle_syn=shape[0], unroll=shape[1], fuse=shape[2], events=shape[3])
    torch.cuda.synchronize()
    log(f"[bench] {rate} Hz {wtype}: created in {time.time() - t0:.1f}s; burn-in {burnin} + warmup {warmup}")
    if ou is not None:
        g.set_background_ou(*ou)
    g.step(pre)
    g.sync()
    state = g.save()
    walls, per_kernel, ev_rep, wall_timed = [], {}, [], None
    # `reps` plain repetitions give the wall clock; one more, identical (same
    # state, same steps), brackets every kernel with a pair of HIP events on
    # the library's stream for the per-kernel durations (the event records
    # themselves would add to the wall clock of the plain ones)
    for q in range(reps + 1):
        timing = q == reps
        g.load(state)
        c0 = g.counters()
        if timing:
            g.read_timing()
            g.set_timing(True)
        torch.cuda.synchronize()
        tic = time.perf_counter()
        g.step(steps)
        torch.cuda.synchronize()
        w = time.perf_counter() - tic
        if timing:
            wall_timed = w
            g.set_timing(False)
            for k, v in g.read_timing().items():
                per_kernel[k] = [v["ms"], v["launches"]]
        else:
            walls.append(w)
        c1 = g.counters()
        ev_rep.append((c1["ev_rec"] - c0["ev_rec"], c1["ev_bg"] - c0["ev_bg"], c1["spikes"] - c0["spikes"]))
    g.sync()
    # every repetition did the same work from the same state
    assert all(e == ev_rep[0] for e in ev_rep), "repetitions from one state must deliver the same events"
    ev, evb, spikes = ev_rep[0]
    rates = g.region_rates(g.t - min(steps, g.record_steps), g.t)
    bits = g.spikes_bits(0, g.t) if keep_bits else None
    g.close()
    del g
    torch.cuda.synchronize()
    wall = float(np.median(walls))
    mean_rate = spikes / (net.n * steps * net.dt_ms * 1e-3)
    return {"rate_target_hz": rate, "bg_lambda": lam, "wall_s": wall, "ms_per_step": 1e3 * wall / steps,
            "ms_per_step_reps": _spread([1e3 * w / steps for w in walls]),
            "events": ev, "spikes": spikes, "events_per_s": ev / wall, "rtf": wall / (steps * net.dt_ms * 1e-3),
            "mean_rate_hz": mean_rate, "on_target": abs(mean_rate - rate) <= RATE_TOLERANCE * rate,
            "region_rate_spread": [float(np.min(rates)), float(np.max(rates))],
            "bg_events_per_s": evb / wall,
            "kernels": {k: {"ms": v[0], "launches": v[1]} for k, v in per_kernel.items()},
            "ms_per_step_kernel_timing_rep": 1e3 * wall_timed / steps,
            "region_rates": rates, "bits": bits}


def run_split(net, bits, steps, warmup, burnin, shape=(0, 0, 0, 0)):
    """J_intra / J_inter split (Sec. V-B): the partition keeps each row's
    own-region in-edges, the cross-region ones become a remote block whose
    sources mirror the partition, and the unsplit run's raster is replayed
    as the remote spikes from step 0 (inputs resident in HBM before the
    timed steps).  The local block takes the unsplit run's bundle size and
    delivery mode (the remote block is always swept, its row sums separate).
    Returns the timed rates and whether the raster is the unsplit one bit
    for bit."""
    import torch
    import netgen
    import paper_2308_01241_amd as dtb

    t0 = time.time()
    local, blk = netgen.split_remote(net)
    rec = max(steps, 16)
    g = dtb.Net(local, record_steps=rec, stream=torch.cuda.current_stream(), bundle_syn=shape[0],
                events=shape[3])
    g.set_remote_block(blk)
    k_local, k_remote = local.nnz / net.n, int(blk.row_ptr[-1]) / net.n
    del local, blk
    torch.cuda.synchronize()
    log(f"[bench] j_inter split: created in {time.time() - t0:.1f}s")
    pre = burnin + warmup
    for q in range(0, pre, rec):  # replay in chunks the push queue holds
        k = min(rec, pre - q)
        g.push_remote_bits(bits[q:q + k])
        g.step(k)
    g.push_remote_bits(bits[pre:pre + steps])
    g.sync()
    c0 = g.counters()
    g.read_timing()
    g.set_timing(True)
    torch.cuda.synchronize()
    tic = time.perf_counter()
    g.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - tic
    g.set_timing(False)
    kt = g.read_timing()
    c1 = g.counters()
    same = bool(np.array_equal(g.spikes_bits(pre, pre + steps), bits[pre:pre + steps]))
    g.close()
    del g
    torch.cuda.synchronize()
    per = {k: v["ms"] / max(1, v["launches"]) for k, v in kt.items()}
    ev = c1["ev_rec"] - c0["ev_rec"]
    return {"k_local_per_row": k_local, "k_remote_per_row": k_remote, "n_remote": net.n,
            "split": "own-region in-edges local, cross-region in-edges remote",
            "events_per_s": ev / wall, "ms_per_step": 1e3 * wall / steps, "kernels_ms_per_step": per,
            "raster_identical_to_unsplit": same}


def rate_error(r, ref):
    """Relative error of per-region rates against a reference run."""
    r, ref = np.asarray(r, np.float64), np.asarray(ref, np.float64)
    rel = np.abs(r - ref) / np.maximum(ref, 1e-9)
    return {"max_region_rel": float(rel.max()), "mean_region_rel": float(rel.mean()),
            "mean_rate_rel": float(abs(r.mean() - ref.mean()) / ref.mean())}


def ensemble_members(n_members: int = 64):
    """The batched-ensemble workload: members of 50k-400k neurons with 20
    regions each at the 7 Hz drive, and their per-(region, channel) gains."""
    import netgen
    sizes = netgen.ensemble_sizes(n_members)
    gains = netgen.ensemble_gains(n_members)
    members = [netgen.make_network(netgen.ensemble_member_spec(m, int(nm), rate_hz=7))
               for m, nm in enumerate(sizes)]
    return members, gains


def run_batched(steps: int, warmup: int, n_members: int = 64, per_member_steps: int = 200, members_too: bool = True):
    """The batched ensemble: n_members independent networks of 50k-400k
    neurons (20 regions each, per-(member, region, channel) gains), advanced
    together by replays of one captured HIP graph, against the same members
    stepped one handle at a time (the plain path)."""
    import torch
    import paper_2308_01241_amd as dtb
    from paper_2308_01241_amd import autotune

    t0 = time.time()
    members, gains = ensemble_members(n_members)
    n_tot = int(sum(m.n for m in members))
    s_tot = int(sum(m.nnz for m in members))
    log(f"[bench] ensemble: {n_members} members, {n_tot} neurons, {s_tot} synapses, generated in "
        f"{time.time() - t0:.1f}s")
    shape = autotune.lookup(n_tot, s_tot, n_members, "f32", max(m.max_delay for m in members))
    stream = torch.cuda.current_stream()
    g = dtb.Net.batch(members, record_steps=64, stream=stream, bundle_syn=shape[0], unroll=shape[1],
                      fuse=shape[2], events=shape[3])
    g.set_gains(gains.reshape(-1, 4))
    g.run(warmup)
    g.sync()
    c0 = g.counters()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    g.run(steps)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    c1 = g.counters()
    bold = g.bold()
    g.close()
    ev = c1["ev_rec"] - c0["ev_rec"]
    batched = {"ms_per_step": ms / steps, "events_per_s": ev / (ms * 1e-3),
               "rtf": ms * 1e-3 / (steps * 1e-3),
               "mean_rate_hz": (c1["spikes"] - c0["spikes"]) / (n_tot * steps * 1e-3),
               "bold_finite": bool(np.isfinite(bold).all())}
    if not members_too:
        return {"workload": f"ensemble: {n_members} members, {n_tot} neurons, {s_tot} synapses", "batched": batched}
    # the plain path, one member at a time, same gains, same launch shape,
    # graph replays too
    ev_m, ms_m = 0, 0.0
    for m, nw in enumerate(members):
        h = dtb.Net(nw, record_steps=64, stream=stream, bundle_syn=shape[0], unroll=shape[1], fuse=shape[2],
                    events=shape[3])
        h.set_gains(gains[m])
        h.run(warmup)
        h.sync()
        e0 = h.counters()["ev_rec"]
        a.record(stream)
        h.run(per_member_steps)
        b.record(stream)
        torch.cuda.synchronize()
        ms_m += a.elapsed_time(b)
        ev_m += h.counters()["ev_rec"] - e0
        h.close()
    single = {"events_per_s": ev_m / (ms_m * 1e-3), "ms_per_step_all_members": ms_m / per_member_steps,
              "steps_per_member": per_member_steps}
    return {"gather_shape": _shape_dict(shape),
            "workload": f"ensemble: {n_members} members of 50k-400k neurons (20 regions each), "
                        f"{n_tot} neurons, {s_tot} synapses, per-region channel gains, 7 Hz drive, "
                        f"{steps} steps under one captured HIP graph",
            "batched": batched, "member_by_member": single,
            "speedup_events_per_s": batched["events_per_s"] / single["events_per_s"]}


def cpu_baseline(net, rate_hz: float, frac: float = 0.02, warm: int = 20, timed: int = 10):
    """FP64 reference on the host cores: a random `frac` of the rows of the
    same partition, teacher-forced by a seeded synthetic raster at rate_hz
    (the first `warm` steps fill the delay ring, the next `timed` are timed)."""
    import oracle

    o = oracle.OracleNet(net)
    rng = np.random.default_rng(777)
    rows = np.sort(rng.choice(net.n, size=max(1, int(frac * net.n)), replace=False)).astype(np.int64)
    p = rate_hz * net.dt_ms * 1e-3
    ev = 0
    el = 0.0
    for s in range(warm + timed):
        forced = (rng.random(net.n) < p).astype(np.uint8)
        tic = time.perf_counter()
        out = o.step(forced=forced, rows=rows)
        dt = time.perf_counter() - tic
        if s >= warm:
            ev += out["ev_rec"]
            el += dt
    cores = oracle.max_threads()
    step_s = el / timed
    return {"value": ev / el, "unit": "synaptic events/s", "cores": cores, "kind": "oracle",
            "sample": (f"{len(rows)} random rows ({frac:.0%}) of the {net.n}-neuron partition, "
                       f"{warm} ring-filling + {timed} timed teacher-forced steps at {rate_hz} Hz "
                       f"(synthetic seeded raster)"),
            "rtf_extrapolated": step_s / frac / (net.dt_ms * 1e-3)}


def tune_rates(net, rates, steps=400, skip=150, iters=9):
    """Bisect the background drive so that the mean rate over steps
    [skip, steps) hits each target (one handle, reset between trials)."""
    import torch
    import paper_2308_01241_amd as dtb

    g = dtb.Net(net, record_steps=steps, stream=torch.cuda.current_stream())
    out = {}

    def rate(lam):
        g.reset()
        g.set_background(lam, net.bg_w)
        g.step(steps)
        c = g.region_counts(skip, steps).sum()
        return c / (net.n * (steps - skip) * net.dt_ms * 1e-3)

    for r in rates:
        lo, hi = 0.02, 8.0
        for _ in range(iters):
            mid = float(np.sqrt(lo * hi))
            m = rate(mid)
            log(f"[tune] target {r} Hz: lambda {mid:.5f} -> {m:.3f} Hz")
            if m < r:
                lo = mid
            else:
                hi = mid
        lam = float(np.sqrt(lo * hi))
        out[r] = {"bg_lambda": round(lam, 5), "rate_hz": float(rate(lam))}
    g.close()
    return out


def calibrate_copy(gib: float = 1.0):
    """Passes of known size whose FETCH_SIZE / WRITE_SIZE readings scale the
    counters of the simulator's kernels: an elementwise add (reads and writes
    `gib` GiB) and a sum (reads `gib` GiB, writes one value)."""
    import torch
    n = int(gib * (1 << 30)) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.add(x, 1.0, out=y)
    for _ in range(3):
        s = x.sum()
    torch.cuda.synchronize()
    return {"calibration": "elementwise add, then sum", "bytes_read": 4 * n, "bytes_written": 4 * n,
            "sum_bytes_read": 4 * n, "sum": float(s)}


def point_summary(r):
    return {k: v for k, v in r.items() if k not in ("kernels", "region_rates", "bits")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--burnin", type=int, default=300,
                    help="untimed steps that bring each point to its stationary rate before --warmup")
    ap.add_argument("--reps", type=int, default=5, help="timed repetitions from one saved state (plus one with per-kernel timing)")
    ap.add_argument("--n", type=int, default=20_000_000)
    ap.add_argument("--rates", type=str, default="7,15,30")
    ap.add_argument("--wtype", type=str, default="f32", choices=["f32", "bf16"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tune", action="store_true", help="bisect the background drive per target rate")
    ap.add_argument("--calibrate-copy", action="store_true", help="run a plain copy of known size")
    ap.add_argument("--autotune", action="store_true", help="search the gather launch shape, store it")
    ap.add_argument("--no-forms", action="store_true", help="skip the BF16, OU, split and batched runs")
    ap.add_argument("--batch-steps", type=int, default=2000)
    ap.add_argument("--ensemble-only", action="store_true",
                    help="run only the batched ensemble (no member-by-member comparison), e.g. under a kernel trace")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU's partition; --gpus {args.gpus} is not supported "
              f"(the cross-GPU spike exchange is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    import netgen
    import paper_2308_01241_amd as dtb
    from paper_2308_01241_amd import autotune

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dtb.load()
    if args.calibrate_copy:
        print(json.dumps(calibrate_copy()), flush=True)
        return
    if args.ensemble_only:
        print(json.dumps({"ensemble": run_batched(args.batch_steps, 200, members_too=False)}), flush=True)
        return
    rates = [int(x) for x in args.rates.split(",")]
    t0 = time.time()
    net = netgen.make_network(netgen.partition_spec(n=args.n, rate_hz=rates[0]))
    log(f"[bench] generated n={net.n} nnz={net.nnz} in {time.time() - t0:.1f}s")
    if args.tune:
        print(json.dumps({"tuned": tune_rates(net, rates), "n": net.n}), flush=True)
        return
    if args.autotune:
        out = {}
        for wt in ("f32", "bf16"):
            net.bg_lambda = netgen.PARTITION_LAMBDA[rates[0]]
            r = autotune.tune([net], wtype=wt, record_steps=64, cache_path=autotune.CACHE, burnin=args.burnin,
                              steps=40, stream=torch.cuda.current_stream())
            log(f"[autotune] partition {wt}: {r}")
            out[f"partition/{wt}"] = {**r, "tried": {"/".join(map(str, k)): v for k, v in r["tried"].items()}}
        del net
        members, gains = ensemble_members(64)
        for wt in ("f32", "bf16"):
            r = autotune.tune(members, wtype=wt, record_steps=64, cache_path=autotune.CACHE, burnin=200, steps=40,
                              stream=torch.cuda.current_stream())
            log(f"[autotune] ensemble {wt}: {r}")
            out[f"ensemble/{wt}"] = {**r, "tried": {"/".join(map(str, k)): v for k, v in r["tried"].items()}}
        print(json.dumps({"autotune": out}), flush=True)
        return
    n_neu, n_syn, n_del = net.n, net.nnz, net.max_delay
    shape = autotune.lookup(n_neu, n_syn, 1, args.wtype, n_del)
    log(f"[bench] gather shape (bundle_syn, unroll, fuse, events): {shape} (0 = library default)")
    res = {}
    want_split = not args.no_forms and args.wtype == "f32"
    for r in rates:
        res[r] = run_rate(net, r, netgen.PARTITION_LAMBDA[r], args.steps, args.warmup, args.burnin, args.reps,
                          args.wtype, shape, keep_bits=want_split and r == rates[0])
        log(f"[bench] {r} Hz: {json.dumps(point_summary(res[r]))}")
        log(f"[bench] {r} Hz kernels: {res[r]['kernels']}")
    head = res[rates[0]]
    wb = 2 if args.wtype == "bf16" else 4
    per = {k: v["ms"] / max(1, v["launches"]) for k, v in head["kernels"].items()}
    ev_step = head["events"] / args.steps
    roof = roofline(per, head["ms_per_step"], n_syn, n_neu, n_del, ev_step, head["spikes"] / args.steps, wb)
    forms = {}
    if not args.no_forms and args.wtype == "f32":
        bf = {}
        for r in rates:
            x = run_rate(net, r, netgen.PARTITION_LAMBDA[r], args.steps, args.warmup, args.burnin, 1, "bf16",
                         autotune.lookup(n_neu, n_syn, 1, "bf16", n_del))
            kx = x["kernels"]
            bf[str(r)] = {"events_per_s": x["events_per_s"], "ms_per_step": x["ms_per_step"], "rtf": x["rtf"],
                          "mean_rate_hz": x["mean_rate_hz"],
                          "speedup_events_per_s": x["events_per_s"] / res[r]["events_per_s"],
                          "gather_ms": kx["gather"]["ms"] / max(1, kx["gather"]["launches"]),
                          "rate_error_vs_f32": rate_error(x["region_rates"], res[r]["region_rates"])}
            log(f"[bench] bf16 {r} Hz: {json.dumps(bf[str(r)])}")
        forms["bf16"] = bf
        r0 = rates[0]
        ou = run_rate(net, r0, 0.0, args.steps, args.warmup, args.burnin, 1, "f32", shape, ou=OU_BACKGROUND)
        forms["ou_background"] = {"mu_sigma_tau_ms": list(OU_BACKGROUND), "events_per_s": ou["events_per_s"],
                                  "ms_per_step": ou["ms_per_step"], "rtf": ou["rtf"],
                                  "mean_rate_hz": ou["mean_rate_hz"],
                                  "gather_ms": ou["kernels"]["gather"]["ms"] / max(1, ou["kernels"]["gather"]["launches"])}
        log(f"[bench] ou background: {json.dumps(forms['ou_background'])}")
        bits = head.pop("bits")
        net.bg_lambda = netgen.PARTITION_LAMBDA[r0]
        sp = run_split(net, bits, args.steps, args.warmup, args.burnin, shape)
        del bits
        sp["speed_vs_unsplit"] = sp["events_per_s"] / head["events_per_s"]
        forms["j_inter_split"] = sp
        log(f"[bench] j_inter split: {json.dumps(sp)}")
    cpu = None
    if not args.no_cpu:
        log("[bench] cpu baseline (FP64 reference, bounded sample)")
        cpu = cpu_baseline(net, float(rates[0]))
        log(f"[bench] cpu: {cpu}")
    del net
    if not args.no_forms and args.wtype == "f32":
        import gc
        gc.collect()
        forms["ensemble"] = run_batched(args.batch_steps, 200)
        log(f"[bench] ensemble: {json.dumps(forms['ensemble'])}")
    out = {"metric": METRIC, "value": head["events_per_s"], "unit": "synaptic events/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": args.wtype, "data": "synthetic",
           "config": {"workload": f"partition_net: {n_neu} neurons, {n_syn} synapses, 90 regions, "
                                  f"in-degree 100, delays 1-{n_del}, dt 1 ms, drive for {rates[0]} Hz "
                                  f"(measured {head['mean_rate_hz']:.2f} Hz over the timed steps, after "
                                  f"{args.burnin} burn-in steps)",
                      "global_batch": 1, "seq_len": args.steps, "parallelism": "single-gpu"},
           "rtf": head["rtf"], "ms_per_step_reps": head["ms_per_step_reps"], "roofline": roof, "cpu_baseline": cpu,
           "gather_shape": _shape_dict(shape),
           "rates": {str(r): point_summary(res[r]) for r in rates},
           "forms": forms or None,
           "kernels_ms_per_step": per}
    print(json.dumps(out), flush=True)
    off = [r for r in rates if not res[r]["on_target"]]
    if off:
        log(f"[bench] measured mean rate off target by more than {RATE_TOLERANCE:.0%} at {off} Hz")
        sys.exit(3)


if __name__ == "__main__":
    main()
