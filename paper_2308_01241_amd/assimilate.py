"""Surrogate-screened assimilation of population gains (the hierarchical
mesoscopic data assimilation idea of Sec. V-E, on one GPU).

Pipeline, all on the GPU through the C ABI:
  1. data   - the batched ensemble runs from rest one window of `window`
              steps at unit gains, then `segments` chained windows, each at
              fresh per-population channel gains ~ N(1, 0.2^2) (clipped at
              0); a sample maps (gains, population rates of the window
              before, hemodynamic state at the window's start) ->
              (population rates of the window, BOLD at its end);
              the default run (157 runs x 10 windows x 64 members) gives
              100,480 training samples;
  2. train  - the MFMA surrogate MLP learns that map (z-scored, Adam, MSE);
  3. screen - against a synthetic twin target (a member network whose gains
              are hidden: one window at unit gains, then one at the hidden
              gains), each iteration scores many Gaussian proposals with the
              surrogate, re-simulates the best k as one batch (the check)
              and k random proposals the same way (the method without the
              surrogate), and moves the proposal mean to the best simulated
              one.

`python -m paper_2308_01241_amd.assimilate --out report.json` runs it.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import sys
import time

import numpy as np

GAIN_SD = 0.2


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _tuned_shape(members) -> dict:
    """The gather launch shape cached for this batch's shape by the
    autotuner, as Net keyword arguments (the library defaults if none)."""
    from . import autotune
    b, u, f, v = autotune.lookup(sum(m.n for m in members), sum(m.nnz for m in members), len(members), "f32",
                                 max(m.max_delay for m in members))
    return {"bundle_syn": b, "unroll": u, "fuse": f, "events": v}


def _stream():
    import torch
    return torch.cuda.current_stream()


@dataclasses.dataclass
class Setup:
    members: int = 64          # ensemble members in the data batch
    lo: int = 50_000           # member sizes ~ U[lo, hi]
    hi: int = 400_000
    regions: int = 20          # populations per member
    window: int = 200          # steps per window (dt = 1 ms)
    rate_hz: int = 7           # background drive of the members (about 10 Hz)
    target_n: int = 200_000    # size of the twin target


def member_networks(S: Setup, seed: int = 31):
    import netgen
    sizes = netgen.ensemble_sizes(S.members, S.lo, S.hi, seed=seed)
    return [netgen.make_network(netgen.ensemble_member_spec(m, int(n), rate_hz=S.rate_hz, n_regions=S.regions))
            for m, n in enumerate(sizes)]


def window_rates(net, S: Setup):
    """[members, regions] rates (Hz) over the last window."""
    return net.region_rates(net.t - S.window, net.t).reshape(-1, S.regions)


def hemo_state(net, S: Setup):
    """[members, 4 regions] Balloon-Windkessel state (s, f - 1, v - 1, q - 1)
    of every population now: where the BOLD of the next window starts from."""
    _, st = net.bold(state=True)
    st = st.astype(np.float64) - np.array([0.0, 1.0, 1.0, 1.0])
    return st.reshape(-1, S.regions * 4).astype(np.float32)


def generate(net, S: Setup, n_runs: int, rng, segments: int = 1):
    """n_runs x segments x members samples.  Each run starts from rest with
    one window at unit gains, then `segments` chained windows, each at fresh
    per-member gains ~ N(1, 0.2^2) clipped at 0 (network and hemodynamic
    state carry over from window to window).  A sample maps (a member's
    gains in the window, its population rates over the window before) to
    (its rates over the window, BOLD at the window's end).  The first
    window of a run is exactly how the re-simulation check runs a proposal.
    The hemodynamic state at the window's start is an input too: it carries
    over from window to window, and the BOLD at the window's end depends on
    it as much as on the window's rates.
    Returns X [samples, 9 R] (gains 4 R, rates of the window before R,
    hemodynamic state at the window's start 4 R) and Y [samples, 2 R]."""
    M, R = net.n_members, S.regions
    X, Y = [], []
    for run in range(n_runs):
        net.reset()
        net.set_gains(np.ones((M * R, 4), dtype=np.float32))
        net.run(S.window)
        prev = window_rates(net, S)
        for _ in range(segments):
            g = np.clip(rng.normal(1.0, GAIN_SD, (M, R, 4)), 0.0, None).astype(np.float32)
            hemo = hemo_state(net, S)
            net.set_gains(g.reshape(-1, 4))
            net.run(S.window)
            rates = window_rates(net, S)
            bold = net.bold().reshape(M, R)
            X.append(np.concatenate([g.reshape(M, -1), prev, hemo], axis=1))
            Y.append(np.concatenate([rates, 1e3 * bold], axis=1))  # BOLD in 1e-3 units
            prev = rates
        if (run + 1) % 16 == 0 or run + 1 == n_runs:
            log(f"[data] run {run + 1}/{n_runs}: {len(X) * M} samples")
    return np.concatenate(X).astype(np.float32), np.concatenate(Y).astype(np.float32)


class Scaler:
    def __init__(self, A):
        self.mu = A.mean(0)
        self.sd = A.std(0) + 1e-6

    def f(self, A):
        return ((A - self.mu) / self.sd).astype(np.float32)

    def inv(self, Z):
        return Z * self.sd + self.mu


def train(X, Y, epochs=30, batch=256, lr=1e-3, seed=0, width=256, depth=3):
    from . import MLP
    sx, sy = Scaler(X), Scaler(Y)
    Xz, Yz = sx.f(X), sy.f(Y)
    m = MLP(X.shape[1], width, depth, Y.shape[1], seed=seed)
    rng = np.random.default_rng(seed)
    bs = min(batch, len(X))
    for ep in range(epochs):
        perm = rng.permutation(len(X))
        tot, nb = 0.0, 0
        for b in range(0, len(X) - bs + 1, bs):
            idx = perm[b:b + bs]
            tot += m.train_step(Xz[idx], Yz[idx], lr)
            nb += 1
        if ep % 5 == 4 or ep == epochs - 1:
            log(f"[train] epoch {ep + 1}: mean batch loss {tot / max(1, nb):.4f}")
    return m, sx, sy


def evaluate(m, sx, sy, X, Y, R):
    """Held-out error of the surrogate: relative RMSE (against the spread of
    the data) and the mean across samples of the correlation over
    populations between predicted and simulated values."""
    P = sy.inv(m.forward(sx.f(X)))
    out = {}
    for name, sl in (("rates", slice(0, R)), ("bold", slice(R, 2 * R))):
        err = P[:, sl] - Y[:, sl]
        rel = np.linalg.norm(err) / np.linalg.norm(Y[:, sl] - Y[:, sl].mean(0))
        corr = np.mean([np.corrcoef(P[i, sl], Y[i, sl])[0, 1] for i in range(min(len(P), 2000))])
        out[name] = {"rel_rmse": float(rel), "mean_corr_across_populations": float(corr)}
    return out


def _fit(rates, bold, t_rates, t_bold, sr, sb):
    """Distance of (rates, BOLD) to the target, in units of the data spread."""
    return np.mean(((rates - t_rates) / sr) ** 2, axis=-1) + np.mean(((bold - t_bold) / sb) ** 2, axis=-1)


class Resim:
    """k + 1 copies of the target network in one batch (member ids 0 .. k, so
    each copy draws its own background): copies 0 .. k-1 simulate k gain
    proposals, copy k is the twin (one window at unit gains, then one at
    the given gains)."""

    def __init__(self, target_net, k, S: Setup):
        from . import Net
        copies = []
        for c in range(k + 1):
            cp = dataclasses.replace(target_net)
            cp.member = c
            copies.append(cp)
        self.k, self.S = k, S
        self.net = Net.batch(copies, record_steps=2 * S.window, stream=_stream(), **_tuned_shape(copies))

    def __call__(self, G, twin_gains=None):
        S, k = self.S, self.k
        full = np.ones((k + 1, S.regions, 4), dtype=np.float32)
        full[:k] = np.asarray(G, np.float32).reshape(k, S.regions, 4)
        if twin_gains is not None:
            full[k] = twin_gains
        self.net.reset()
        self.net.set_gains(np.ones(((k + 1) * S.regions, 4), dtype=np.float32))
        self.net.run(S.window)
        base = window_rates(self.net, S)
        hemo = hemo_state(self.net, S)
        self.net.set_gains(full.reshape(-1, 4))
        self.net.run(S.window)
        return window_rates(self.net, S), 1e3 * self.net.bold().reshape(k + 1, S.regions), base, hemo

    def close(self):
        self.net.close()


def screen(m, sx, sy, target_net, hidden_gains, S: Setup, iters=10, n_prop=4096, k=64, seed=0, resim=None,
           shrink=0.85):
    """Surrogate-screened search for the hidden gains of a twin target:
    Gaussian proposals around the best simulated proposal so far, their
    spread shrinking by `shrink` per iteration (a plain elitist search
    standing in for the paper's assimilation filter)."""
    from . import topk
    rng = np.random.default_rng(seed)
    R = S.regions
    own = resim is None
    resim = resim or Resim(target_net, k, S)
    # the twin: the re-simulation batch's last copy, run at the hidden gains
    rs, bs, base, hemo = resim(np.ones((k, R, 4), dtype=np.float32), twin_gains=hidden_gains)
    t_rates, t_bold, prev, h0 = rs[k].copy(), bs[k].copy(), base[k].copy(), hemo[k].copy()
    sr, sb = sy.sd[:R], sy.sd[R:]
    mu = np.ones((R, 4), dtype=np.float32)
    best_fit = np.inf
    hist = []
    for it in range(iters):
        sd = GAIN_SD * shrink ** it
        props = np.clip(mu[None] + rng.normal(0, sd, (n_prop, R, 4)), 0.0, None).astype(np.float32)
        X = np.concatenate([props.reshape(n_prop, -1), np.repeat(prev[None], n_prop, 0),
                            np.repeat(h0[None], n_prop, 0)], axis=1)
        import torch
        torch.cuda.synchronize()
        tic = time.perf_counter()
        P = sy.inv(m.forward(sx.f(X)))
        score = _fit(P[:, :R], P[:, R:], t_rates, t_bold, sr, sb).astype(np.float32)
        best = topk(score, k)
        t_screen = time.perf_counter() - tic
        tic = time.perf_counter()
        rs, bs, _, _ = resim(props[best])
        rs, bs = rs[:k], bs[:k]
        t_sim = time.perf_counter() - tic
        fit_s = _fit(rs, bs, t_rates, t_bold, sr, sb)
        rnd = rng.choice(n_prop, k, replace=False)
        rr, br, _, _ = resim(props[rnd])
        rr, br = rr[:k], br[:k]
        fit_r = _fit(rr, br, t_rates, t_bold, sr, sb)
        pb = P[best][:, R:]
        corr_pred = np.array([np.corrcoef(pb[i], t_bold)[0, 1] for i in range(k)])
        corr_sim = np.array([np.corrcoef(bs[i], t_bold)[0, 1] for i in range(k)])
        corr_ps = np.array([np.corrcoef(pb[i], bs[i])[0, 1] for i in range(k)])
        j = int(np.argmin(fit_s))
        if fit_s[j] < best_fit:  # the proposal mean follows the best simulated fit so far
            best_fit = float(fit_s[j])
            mu = props[best[j]]
        gain_err = float(np.sqrt(np.mean((mu - hidden_gains) ** 2)))
        rec = {"iter": it, "proposal_sd": sd, "best_fit_so_far": best_fit,
               "best_fit_surrogate": float(fit_s.min()), "mean_fit_surrogate": float(fit_s.mean()),
               "best_fit_random": float(fit_r.min()), "mean_fit_random": float(fit_r.mean()),
               "bold_corr_error": float(np.nanmean(np.abs(corr_pred - corr_sim))),
               "corr_pred_vs_sim": float(np.nanmean(corr_ps)), "gain_rmse": gain_err,
               "screen_s": t_screen, "simulate_s": t_sim,
               "speedup_per_proposal": (t_sim / k) / (t_screen / n_prop)}
        hist.append(rec)
        log(f"[screen] {json.dumps(rec)}")
    if own:
        resim.close()
    return hist


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--members", type=int, default=64)
    ap.add_argument("--window", type=int, default=200)
    ap.add_argument("--runs", type=int, default=1408)
    ap.add_argument("--test-runs", type=int, default=157)
    ap.add_argument("--segments", type=int, default=1, help="chained gain windows per run")
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--iters", type=int, default=8)
    ap.add_argument("--seeds", type=str, default="0,1,2")
    ap.add_argument("--target-n", type=int, default=200_000)
    ap.add_argument("--rate-hz", type=int, default=Setup.rate_hz, help="background drive level of the members")
    ap.add_argument("--out", type=str, default="")
    a = ap.parse_args(argv)
    import netgen
    from . import Net

    S = Setup(members=a.members, window=a.window, target_n=a.target_n, rate_hz=a.rate_hz)
    t0 = time.time()
    members = member_networks(S)
    net = Net.batch(members, record_steps=2 * S.window, stream=_stream(), **_tuned_shape(members))
    del members
    log(f"[data] ensemble: {net.n} neurons, {net.n_members} members, built in {time.time() - t0:.1f}s")
    tic = time.perf_counter()
    X, Y = generate(net, S, a.runs, np.random.default_rng(32), segments=a.segments)
    gen_s = time.perf_counter() - tic
    Xt, Yt = generate(net, S, a.test_runs, np.random.default_rng(33), segments=a.segments)
    net.close()
    tic = time.perf_counter()
    m, sx, sy = train(X, Y, epochs=a.epochs)
    train_s = time.perf_counter() - tic
    err = evaluate(m, sx, sy, Xt, Yt, S.regions)
    log(f"[train] held-out error: {json.dumps(err)}")
    rep = {"setup": dataclasses.asdict(S), "segments_per_run": a.segments, "runs": a.runs,
           "test_runs": a.test_runs, "samples": int(len(X)), "test_samples": int(len(Xt)),
           "mean_rate_hz": float(Y[:, :S.regions].mean()),
           "generate_s": gen_s, "train_s": train_s, "held_out": err, "screen": {}}
    target = netgen.make_network(netgen.ensemble_member_spec(41, S.target_n, rate_hz=S.rate_hz,
                                                             n_regions=S.regions))
    resim = Resim(target, 64, S)
    for s in [int(x) for x in a.seeds.split(",")]:
        hidden = np.clip(np.random.default_rng(41 + s).normal(1.0, GAIN_SD, (S.regions, 4)), 0,
                         None).astype(np.float32)
        rep["screen"][str(s)] = screen(m, sx, sy, target, hidden, S, iters=a.iters, seed=s, resim=resim)
    resim.close()
    H = [r for h in rep["screen"].values() for r in h]
    rep["summary"] = {
        "mean_best_fit_surrogate": float(np.mean([r["best_fit_surrogate"] for r in H])),
        "mean_best_fit_random": float(np.mean([r["best_fit_random"] for r in H])),
        "mean_fit_surrogate": float(np.mean([r["mean_fit_surrogate"] for r in H])),
        "mean_fit_random": float(np.mean([r["mean_fit_random"] for r in H])),
        "bold_corr_error": float(np.mean([r["bold_corr_error"] for r in H])),
        "corr_pred_vs_sim": float(np.mean([r["corr_pred_vs_sim"] for r in H])),
        "speedup_per_proposal": float(np.median([r["speedup_per_proposal"] for r in H])),
        "final_gain_rmse": {k: h[-1]["gain_rmse"] for k, h in rep["screen"].items()},
        "final_best_fit": {k: h[-1]["best_fit_so_far"] for k, h in rep["screen"].items()},
    }
    log(f"[summary] {json.dumps(rep['summary'])}")
    if a.out:
        with open(a.out, "w") as f:
            json.dump(rep, f, indent=1)
    print(json.dumps(rep["summary"]), flush=True)


if __name__ == "__main__":
    main()
