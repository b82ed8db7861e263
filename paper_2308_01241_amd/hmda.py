"""Hierarchical mesoscopic data assimilation on one GPU (Sec. V-E).

The paper runs many samples of one brain model on disjoint nodes, turns each
sample's population rates into BOLD signals with the Balloon-Windkessel
model, and iterates an assimilation that adapts the per-population
hyper-parameters of the conductances so that the simulated BOLD tracks the
measured one; the filter itself is in its companion work.  Here:

* the samples are the members of one batched handle: the same network
  (structure, parameters, initial state), each with its own background noise
  (member id) and its own hyper-parameters;
* the hyper-parameters are per-population gains: one on the excitatory
  channels (AMPA and NMDA tied, the conductances the paper tunes) per
  population; the inhibitory gains stay at 1;
* the measured BOLD comes from a synthetic twin: the same network with its
  own noise and hidden gains;
* every window of `window` steps (the BOLD sampling interval) the ensemble
  advances as one captured HIP graph, its BOLD is read on the device, and
  one stochastic-EnKF analysis (`dtb_enkf_analysis`, a stand-in for the
  companion work's filter) updates the gains in place on the device;
* with surrogate screening (`screen`), a small MLP (the `dtb_mlp` kernels)
  is first trained on windows of this network run at random gains, mapping
  (a sample's gains in a window, its population rates over the window
  before, its hemodynamic state at the window's start) to its BOLD at the
  window's end; before each window's simulation every sample draws
  `proposals` candidate gain vectors around its own, the surrogate predicts
  their BOLD, and each sample's best-fitting candidate (its own gains among
  them) marks a direction; the whole ensemble is shifted by `shift` times
  the mean of those moves, so the cheap model moves the ensemble mean
  before the batched path simulates it and the filter updates it, while the
  spread stays the filter's (moving every sample to its own best candidate
  selects extremes and widens the ensemble window after window).

The estimate is checked by re-simulation: one batch of three fresh-noise
copies of the network, at the estimated gains (ensemble mean), at the prior
mean (all ones) and at the hidden gains (the noise floor), run over the
whole assimilation period; each copy's BOLD is compared with the twin's.
`python -m paper_2308_01241_amd.hmda --out report.json`.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import sys
import time

import numpy as np


@dataclasses.dataclass
class HmdaSetup:
    members: int = 64          # samples of the brain model (one batched handle)
    n: int = 100_000           # neurons per sample
    regions: int = 20          # populations
    window: int = 800          # steps between BOLD samples (dt = 1 ms)
    windows: int = 30          # assimilation iterations
    rate_hz: int = 7           # background drive (the partition net's 7 Hz level)
    bg_lambda: float = 0.24    # background Poisson count per neuron-step (< 0: the rate_hz level)
    prior_sd: float = 0.2      # prior spread of the gains around 1
    hidden_sd: float = 0.2     # spread of the twin's hidden gains around 1
    obs_rel: float = 0.1       # observation error sd, relative to the BOLD signal's rms
    inflation: float = 1.02
    lo: float = 0.3
    hi: float = 3.0
    seed: int = 5
    screen: int = 0            # 1: surrogate screening of proposals before each window (0: EnKF alone)
    proposals: int = 64        # candidate gain vectors per sample per window
    step_sd: float = 1.0       # candidate spread, in units of the ensemble's spread per population
    shift: float = 0.3         # fraction of the samples' mean best move applied to every sample
    train_windows: int = 48    # windows of the training data (x members samples)
    epochs: int = 80


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _network(S: HmdaSetup):
    import netgen
    spec = netgen.partition_spec(n=S.n, rate_hz=S.rate_hz, n_regions=S.regions, seeds=(4100, 4101, 4102),
                                 bg_lambda=None if S.bg_lambda < 0 else S.bg_lambda)
    return netgen.make_network(spec)


def _tied_gains(g_exc: np.ndarray) -> np.ndarray:
    """[..., R] excitatory gains -> [..., R, 4] channel gains (GABA at 1)."""
    out = np.ones(g_exc.shape + (4,), dtype=np.float32)
    out[..., 0] = g_exc
    out[..., 1] = g_exc
    return out


def _state_features(ens, t0: int, t1: int, M: int, R: int):
    """[M, R] population rates over [t0, t1) and [M, 4 R] hemodynamic state
    (s, f - 1, v - 1, q - 1) now, per sample."""
    rates = ens.region_rates(t0, t1).reshape(M, R)
    _, st = ens.bold(state=True)
    hemo = (st.astype(np.float64) - np.array([0.0, 1.0, 1.0, 1.0])).reshape(M, 4 * R)
    return rates.astype(np.float32), hemo.astype(np.float32)


def train_surrogate(S: HmdaSetup, net, stream):
    """The screening model: samples of this network at gains ~ 1 + 0.2 N(0, 1)
    (clipped to [lo, hi]), chained windows from rest, each sample mapping
    (gains R, rates of the window before R, hemodynamic state 4 R) to the
    BOLD at the window's end (1e-3 units).  Returns (mlp, x scaler, y
    scaler, seconds of simulation, seconds of training)."""
    import paper_2308_01241_amd as dtb
    from .assimilate import train
    R, M = S.regions, S.members
    rng = np.random.default_rng(S.seed + 1000)
    ens = dtb.Net.batch([dataclasses.replace(net, member=2 * M + 10 + m) for m in range(M)], stream=stream,
                        record_steps=S.window)
    X, Y = [], []
    t0 = time.perf_counter()
    ens.set_gains(np.ones((M * R, 4), np.float32))
    ens.run(S.window)
    prev, hemo = _state_features(ens, ens.t - S.window, ens.t, M, R)
    for _ in range(S.train_windows):
        g = np.clip(1.0 + S.prior_sd * rng.standard_normal((M, R)), S.lo, S.hi).astype(np.float32)
        ens.set_gains(_tied_gains(g).reshape(M * R, 4))
        ens.run(S.window)
        y = ens.bold().reshape(M, R)
        X.append(np.concatenate([g, prev, hemo], axis=1))
        Y.append(1e3 * y)
        prev, hemo = _state_features(ens, ens.t - S.window, ens.t, M, R)
    ens.close()
    sim_s = time.perf_counter() - t0
    X, Y = np.concatenate(X).astype(np.float32), np.concatenate(Y).astype(np.float32)
    t1 = time.perf_counter()
    m, sx, sy = train(X, Y, epochs=S.epochs, seed=S.seed)
    return m, sx, sy, sim_s, time.perf_counter() - t1


def screen_step(m, sx, sy, g, prev, hemo, y_obs, r_var, S: HmdaSetup, rng):
    """Each sample's best of its own gains and S.proposals - 1 candidates
    around them (spread: step_sd x the ensemble's spread per population),
    by the surrogate's predicted BOLD misfit to the observation; every
    sample then moves by S.shift x the mean of the samples' best moves.
    Returns the new [M, R] gains and how many samples found a better
    candidate than their own gains."""
    M, R = g.shape
    P = S.proposals
    sd = S.step_sd * np.maximum(g.std(axis=0), 0.02)
    cand = g[:, None, :] + sd * rng.standard_normal((M, P, R))
    cand[:, 0, :] = g
    cand = np.clip(cand, S.lo, S.hi).astype(np.float32)
    Xc = np.concatenate([cand.reshape(M * P, R), np.repeat(prev, P, axis=0), np.repeat(hemo, P, axis=0)], axis=1)
    pred = sy.inv(m.forward(sx.f(Xc))).reshape(M, P, R) * 1e-3
    miss = np.mean((pred - y_obs[None, None, :]) ** 2, axis=2) / r_var
    best = np.argmin(miss, axis=1)
    move = (cand[np.arange(M), best] - g).mean(axis=0)
    return np.clip(g + S.shift * move, S.lo, S.hi).astype(np.float32), int(np.count_nonzero(best))


def run(S: HmdaSetup):
    import torch
    import paper_2308_01241_amd as dtb

    stream = torch.cuda.current_stream()
    rng = np.random.default_rng(S.seed)
    R, M = S.regions, S.members
    t0 = time.time()
    net = _network(S)
    log(f"[hmda] network n={net.n} nnz={net.nnz} in {time.time() - t0:.1f}s")
    hidden = np.clip(1.0 + S.hidden_sd * rng.standard_normal(R), S.lo, S.hi).astype(np.float32)
    prior = np.clip(1.0 + S.prior_sd * rng.standard_normal((M, R)), S.lo, S.hi).astype(np.float32)

    # the twin: measured BOLD at the end of every window
    twin = dtb.Net(dataclasses.replace(net, member=M), stream=stream, record_steps=S.window)
    twin.set_gains(_tied_gains(hidden))
    y_obs = torch.zeros((S.windows, R), dtype=torch.float32, device="cuda")
    for k in range(S.windows):
        twin.run(S.window)
        twin.bold_into(y_obs[k])
    twin.close()
    torch.cuda.synchronize()
    yo = y_obs.cpu().numpy()
    r_var = (S.obs_rel * np.sqrt(np.mean(yo ** 2, axis=1)) + 1e-9) ** 2   # [windows]

    sur = None
    if S.screen:
        sur = train_surrogate(S, net, stream)
        log(f"[hmda] surrogate: {S.train_windows * M} samples, {sur[3]:.1f} s simulation, {sur[4]:.1f} s training")
    srng = np.random.default_rng(S.seed + 2000)
    members = [dataclasses.replace(net, member=m) for m in range(M)]
    ens = dtb.Net.batch(members, stream=stream, record_steps=S.window)
    X = torch.from_numpy(_tied_gains(prior)).cuda()                       # [M, R, 4]
    Y = torch.zeros((M, R), dtype=torch.float32, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    hist = []
    sim_ms = ana_ms = 0.0
    c_prev = ens.counters()
    screen_ms, moved = 0.0, []
    for k in range(S.windows):
        if sur is not None and k > 0:
            # screened from the state the window starts from (the first
            # window, from the initial state, has no window before it)
            prev, hemo = _state_features(ens, ens.t - S.window, ens.t, M, R)
            tic = time.perf_counter()
            g_new, n_moved = screen_step(sur[0], sur[1], sur[2], X[:, :, 0].cpu().numpy(), prev, hemo, yo[k],
                                         r_var[k], S, srng)
            screen_ms += 1e3 * (time.perf_counter() - tic)
            moved.append(n_moved)
            X.copy_(torch.from_numpy(_tied_gains(g_new)).cuda())
        ev[0].record(stream)
        ens.set_gains_from(X.view(M * R, 4))
        ens.run(S.window)
        ens.bold_into(Y.view(-1))
        ev[1].record(stream)
        forecast = Y.mean(dim=0).cpu().numpy()
        dtb.enkf_analysis(X.view(M, R * 4), Y, y_obs[k], np.full(R, r_var[k], np.float32), S.inflation, S.seed,
                          k, S.lo, S.hi, stream=stream)
        ev[2].record(stream)
        torch.cuda.synchronize()
        sim_ms += ev[0].elapsed_time(ev[1])
        ana_ms += ev[1].elapsed_time(ev[2])
        g = X[:, :, 0].cpu().numpy()
        c_now = ens.counters()
        spikes, events = c_now["spikes"] - c_prev["spikes"], c_now["ev_rec"] - c_prev["ev_rec"]
        c_prev = c_now
        rec = {"window": k, "forecast_rmse": float(np.sqrt(np.mean((forecast - yo[k]) ** 2))),
               "mean_rate_hz": spikes / (M * net.n * S.window * net.dt_ms * 1e-3),
               "events_per_step": events / S.window,
               "obs_rms": float(np.sqrt(np.mean(yo[k] ** 2))),
               "gain_rmse": float(np.sqrt(np.mean((g.mean(0) - hidden) ** 2))),
               "gain_spread": float(g.std(0).mean())}
        hist.append(rec)
        log(f"[hmda] {json.dumps(rec)}")
    est = X[:, :, 0].mean(dim=0).cpu().numpy()
    ens.close()
    # re-simulation of three candidate gain sets with fresh noise
    cand = np.stack([est, np.ones(R, np.float32), hidden])
    check = dtb.Net.batch([dataclasses.replace(net, member=M + 1 + c) for c in range(3)], stream=stream,
                          record_steps=S.window)
    check.set_gains(_tied_gains(cand).reshape(3 * R, 4))
    yc = np.zeros((S.windows, 3, R), np.float32)
    for k in range(S.windows):
        check.run(S.window)
        yc[k] = check.bold().reshape(3, R)
    check.close()
    fit = np.sqrt(np.mean((yc - yo[:, None, :]) ** 2, axis=(0, 2)))
    out = {"setup": dataclasses.asdict(S), "hidden_gains": hidden.tolist(), "estimated_gains": est.tolist(),
           "prior_gain_rmse": float(np.sqrt(np.mean((prior.mean(0) - hidden) ** 2))),
           "final_gain_rmse": float(np.sqrt(np.mean((est - hidden) ** 2))),
           "bold_fit_rmse": {"estimated": float(fit[0]), "prior_mean": float(fit[1]), "hidden": float(fit[2])},
           "bold_rms": float(np.sqrt(np.mean(yo ** 2))),
           "sim_ms_per_window": sim_ms / S.windows, "analysis_ms_per_window": ana_ms / S.windows,
           "history": hist}
    if sur is not None:
        out["screening"] = {"training_samples": S.train_windows * M, "training_sim_s": sur[3], "training_s": sur[4],
                            "proposals_per_window": M * S.proposals,
                            "screen_ms_per_window": screen_ms / max(1, len(moved)),
                            "samples_moved_per_window": float(np.mean(moved)) if moved else 0.0}
        sur[0].close()
    return out


def main():
    ap = argparse.ArgumentParser()
    for f in dataclasses.fields(HmdaSetup):
        ap.add_argument("--" + f.name.replace("_", "-"), type=type(f.default), default=f.default)
    ap.add_argument("--out", type=str, default="")
    ap.add_argument("--compare", action="store_true",
                    help="also run the loop with the other screening setting and report it beside")
    a = vars(ap.parse_args())
    out_path = a.pop("out")
    compare = a.pop("compare")
    S = HmdaSetup(**a)
    rep = run(S)
    if compare:
        other = run(dataclasses.replace(S, screen=1 - S.screen))
        keys = ("final_gain_rmse", "bold_fit_rmse", "sim_ms_per_window", "analysis_ms_per_window", "screening",
                "history")
        rep["surrogate_screened" if S.screen == 0 else "enkf_alone"] = {k: other[k] for k in keys if k in other}
    txt = json.dumps(rep, indent=1)
    if out_path:
        with open(out_path, "w") as f:
            f.write(txt)
    print(json.dumps({k: v for k, v in rep.items() if k != "history"}))


if __name__ == "__main__":
    main()
