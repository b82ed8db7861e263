"""Shared parity checks of a GPU run against the FP64 reference.

Spike agreement ("lockstep"): the reference is stepped through the GPU's own
free-run raster, teacher-forced to the GPU's spikes, and at every step its
own threshold decision (V~ >= V_th, computed in FP64 from the same past
spikes) must equal the GPU's spike at every neuron - except at a neuron whose
V~ lies within DELTA of the threshold, where FP32 may resolve the comparison
either way.  Such disagreements are the ties; they are counted and the
reference follows the GPU there, so the comparison stays exact for the whole
window instead of ending at the first tie.  With no tie the GPU raster is the
reference's own free run, bit for bit.

DELTA = 1e-3 mV: the teacher-forced state bar accepts |dV| <= 1e-5 |V|
(<= 7.5e-4 mV at |V| <= 75 mV), so a neuron within that tolerance of the
threshold may legitimately flip; 1e-3 mV is the smallest round bound above
it.  The worst-case FP32 accumulation in V (a few ulp of ~60 mV per step,
damped by rho = 1 - dt gL / C = 0.97, i.e. <= 33 x 1e-5 mV) is 3.3e-4 mV,
also inside it.
"""
from __future__ import annotations

import numpy as np

DELTA = 1e-3  # mV
FIELDS = ("V", "j_AMPA", "j_NMDA", "j_GABAa", "j_GABAb")


def lockstep(ref, gpu_raster, delta: float = DELTA, checkpoints=None, start: int = 0, remote=None):
    """Step `ref` (an oracle.OracleNet at the state the GPU run started from)
    through `gpu_raster` [T, n] (uint8).  Asserts every disagreement of the
    reference's own decision with the GPU is a tie (margin < delta; a
    refractory neuron has no margin, so a spike there is never a tie).
    checkpoints: optional {step: callback(ref)} called after that step
    (step index relative to `start`).  remote: the remote block's spikes
    [T, n_remote] given to the reference before each step (a reference with
    a remote block).  Returns dict(ties = list of (t, neuron,
    margin), ev_rec [T], ev_bg [T], counts [T, R])."""
    T = len(gpu_raster)
    ties = []
    ev = np.zeros((T, 2), dtype=np.int64)
    counts = np.zeros((T, ref.net.n_regions), dtype=np.int64)
    for t in range(T):
        g = np.ascontiguousarray(gpu_raster[t], dtype=np.uint8)
        if remote is not None:
            ref.give_remote(remote[t])
        out = ref.step(forced=g, want_margin=True)
        diff = np.nonzero(out["own"] != g)[0]
        if len(diff):
            m = out["margin"][diff]
            ok = m < delta  # NaN (refractory) is never a tie
            assert np.all(ok), (f"step {start + t}: neurons {diff[~ok][:8]} spike differently from the FP64 "
                                f"threshold test with margins {m[~ok][:8]} mV (not near-threshold ties)")
            ties.extend((start + t, int(i), float(x)) for i, x in zip(diff, m))
        ev[t] = (out["ev_rec"], out["ev_bg"])
        counts[t] = out["counts"]
        if checkpoints and t in checkpoints:
            checkpoints[t](ref)
    return {"ties": ties, "ev_rec": ev[:, 0], "ev_bg": ev[:, 1], "counts": counts}


def state_close(x_gpu, x_ref, floor):
    """|x_gpu - x_ref| <= 1e-5 max(|x_ref|, floor), elementwise."""
    tol = 1e-5 * np.maximum(np.abs(x_ref), floor)
    return np.abs(np.asarray(x_gpu, np.float64) - x_ref) <= tol


def rel_mse(x_gpu, x_ref) -> float:
    """The paper's accuracy measure (Sec. VII-B): mean squared difference
    relative to the mean square of the reference."""
    x_ref = np.asarray(x_ref, np.float64)
    d = np.asarray(x_gpu, np.float64) - x_ref
    den = float(np.mean(x_ref * x_ref))
    return float(np.mean(d * d)) / den if den > 0 else float(np.mean(d * d))


def report(name: str, **values) -> None:
    """Print a measurement line (and append it to $DTB_TEST_REPORT if set)."""
    import json
    import os
    line = json.dumps({"test": name, **values}, default=float)
    print(line, flush=True)
    path = os.environ.get("DTB_TEST_REPORT")
    if path:
        with open(path, "a") as f:
            f.write(line + "\n")
