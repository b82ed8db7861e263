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
  companion work's filter) updates the gains in place on the device.

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

    members = [dataclasses.replace(net, member=m) for m in range(M)]
    ens = dtb.Net.batch(members, stream=stream, record_steps=S.window)
    X = torch.from_numpy(_tied_gains(prior)).cuda()                       # [M, R, 4]
    Y = torch.zeros((M, R), dtype=torch.float32, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    hist = []
    sim_ms = ana_ms = 0.0
    c_prev = ens.counters()
    for k in range(S.windows):
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
    return out


def main():
    ap = argparse.ArgumentParser()
    for f in dataclasses.fields(HmdaSetup):
        ap.add_argument("--" + f.name.replace("_", "-"), type=type(f.default), default=f.default)
    ap.add_argument("--out", type=str, default="")
    a = vars(ap.parse_args())
    out_path = a.pop("out")
    S = HmdaSetup(**a)
    rep = run(S)
    txt = json.dumps(rep, indent=1)
    if out_path:
        with open(out_path, "w") as f:
            f.write(txt)
    print(json.dumps({k: v for k, v in rep.items() if k != "history"}))


if __name__ == "__main__":
    main()
