"""Surrogate-screened assimilation of population gains (the hierarchical
mesoscopic data assimilation idea of Sec. V-E on one GPU).

Pipeline, all on the GPU through the C ABI:
  1. data   - the batched ensemble runs in segments; each segment gives every
              member fresh per-population channel gains ~ N(1, 0.2^2) (>= 0),
              and a sample maps (gains, population rates of the previous
              segment) -> (population rates of the segment, BOLD at its end);
  2. train  - the MFMA surrogate MLP learns that map (z-scored, Adam, MSE);
  3. screen - against a synthetic twin target (a member network with hidden
              gains), each iteration scores many Gaussian proposals with the
              surrogate, re-simulates the best ones as one batch (the judge)
              and the same number of random proposals (no surrogate), and
              moves the proposal mean to the best simulated one.

`python -m paper_2308_01241_amd.assimilate --out report.json` runs it.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

R_POP = 20            # populations per member
SEG = 200             # steps per segment (200 ms)
GAIN_SD = 0.2


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _stream():
    import torch
    return torch.cuda.current_stream()


def member_networks(sizes, seed_base=3100, rate_hz=15):
    import netgen
    return [netgen.make_network(netgen.ensemble_member_spec(m, int(n), rate_hz=rate_hz, n_regions=R_POP))
            for m, n in enumerate(sizes)]


def segment_rates(net, t0, t1):
    """[members, R_POP] rates (Hz) over steps [t0, t1) from a batch handle."""
    return net.region_rates(t0, t1).reshape(-1, R_POP)


def generate(net, n_runs, n_seg, rng, warm=SEG):
    """Samples from n_runs runs of n_seg segments (after one warm-up segment
    with unit gains).  Returns X [S, 4 R + R] and Y [S, 2 R]."""
    M = net.n_members
    X, Y = [], []
    for run in range(n_runs):
        net.reset()
        net.set_gains(np.ones((M * R_POP, 4), dtype=np.float32))
        net.run(warm)
        prev = segment_rates(net, net.t - warm, net.t)
        for s in range(n_seg):
            g = np.clip(rng.normal(1.0, GAIN_SD, (M, R_POP, 4)), 0.0, None).astype(np.float32)
            net.set_gains(g.reshape(-1, 4))
            net.run(SEG)
            rates = segment_rates(net, net.t - SEG, net.t)
            bold = net.bold().reshape(M, R_POP)
            X.append(np.concatenate([g.reshape(M, -1), prev], axis=1))
            Y.append(np.concatenate([rates, 1e3 * bold], axis=1))  # BOLD in 1e-3 units
            prev = rates
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


def train(X, Y, epochs=30, batch=256, lr=1e-3, seed=0):
    from . import MLP
    sx, sy = Scaler(X), Scaler(Y)
    Xz, Yz = sx.f(X), sy.f(Y)
    m = MLP(X.shape[1], 256, 3, Y.shape[1], seed=seed)
    rng = np.random.default_rng(seed)
    for ep in range(epochs):
        perm = rng.permutation(len(X))
        tot = 0.0
        for b in range(0, len(X) - batch + 1, batch):
            idx = perm[b:b + batch]
            tot += m.train_step(Xz[idx], Yz[idx], lr)
        if ep % 5 == 4 or ep == epochs - 1:
            log(f"[train] epoch {ep + 1}: mean batch loss {tot / max(1, len(X) // batch):.4f}")
    return m, sx, sy


def evaluate(m, sx, sy, X, Y):
    P = sy.inv(m.forward(sx.f(X)))
    R = R_POP
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


def screen(m, sx, sy, target_net, hidden_gains, iters=10, n_prop=4096, k=64, seed=0):
    """Surrogate-screened search for the hidden gains of a twin target."""
    from . import Net, topk
    rng = np.random.default_rng(seed)
    R = R_POP
    twin = Net.batch([target_net], record_steps=2 * SEG, stream=_stream())
    twin.set_gains(hidden_gains.reshape(-1, 4))
    twin.run(2 * SEG)
    t_rates = twin.region_rates(SEG, 2 * SEG)
    t_bold = 1e3 * twin.bold()
    twin.close()
    copies = []
    for c in range(k):
        nw = target_net
        cp = type(nw)(**{f: getattr(nw, f) for f in nw.__dataclass_fields__})
        cp.member = c
        copies.append(cp)
    judge = Net.batch(copies, record_steps=2 * SEG, stream=_stream())
    sr, sb = sy.sd[:R], sy.sd[R:]

    def simulate(G):
        judge.reset()
        judge.set_gains(G.reshape(-1, 4))
        judge.run(2 * SEG)
        rates = judge.region_rates(SEG, 2 * SEG).reshape(k, R)
        bold = 1e3 * judge.bold().reshape(k, R)
        return rates, bold

    mu = np.ones((R, 4), dtype=np.float32)
    prev = simulate(np.repeat(mu[None], k, 0))[0].mean(0)
    hist = []
    for it in range(iters):
        props = np.clip(mu[None] + rng.normal(0, GAIN_SD, (n_prop, R, 4)), 0.0, None).astype(np.float32)
        X = np.concatenate([props.reshape(n_prop, -1), np.repeat(prev[None], n_prop, 0)], axis=1)
        tic = time.perf_counter()
        P = sy.inv(m.forward(sx.f(X)))
        score = _fit(P[:, :R], P[:, R:], t_rates, t_bold, sr, sb).astype(np.float32)
        best = topk(score, k)
        t_screen = time.perf_counter() - tic
        tic = time.perf_counter()
        rs, bs = simulate(props[best])
        t_sim = time.perf_counter() - tic
        fit_s = _fit(rs, bs, t_rates, t_bold, sr, sb)
        rnd = rng.choice(n_prop, k, replace=False)
        rr, br = simulate(props[rnd])
        fit_r = _fit(rr, br, t_rates, t_bold, sr, sb)
        pb = P[best][:, R:]
        corr_pred = np.array([np.corrcoef(pb[i], t_bold)[0, 1] for i in range(k)])
        corr_sim = np.array([np.corrcoef(bs[i], t_bold)[0, 1] for i in range(k)])
        corr_ps = np.array([np.corrcoef(pb[i], bs[i])[0, 1] for i in range(k)])
        j = int(np.argmin(fit_s))
        mu = props[best[j]]
        prev = rs[j]
        gain_err = float(np.sqrt(np.mean((mu - hidden_gains) ** 2)))
        rec = {"iter": it, "best_fit_surrogate": float(fit_s.min()), "mean_fit_surrogate": float(fit_s.mean()),
               "best_fit_random": float(fit_r.min()), "mean_fit_random": float(fit_r.mean()),
               "bold_corr_error": float(np.mean(np.abs(corr_pred - corr_sim))),
               "corr_pred_vs_sim": float(np.nanmean(corr_ps)), "gain_rmse": gain_err,
               "screen_s": t_screen, "simulate_s": t_sim,
               "speedup_per_proposal": (t_sim / k) / (t_screen / n_prop)}
        hist.append(rec)
        log(f"[screen] {json.dumps(rec)}")
    judge.close()
    return hist


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--members", type=int, default=64)
    ap.add_argument("--runs", type=int, default=80)
    ap.add_argument("--segments", type=int, default=10)
    ap.add_argument("--test-runs", type=int, default=8)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--iters", type=int, default=10)
    ap.add_argument("--seeds", type=str, default="0,1,2")
    ap.add_argument("--target-n", type=int, default=200_000)
    ap.add_argument("--out", type=str, default="")
    a = ap.parse_args(argv)
    import netgen
    from . import Net

    t0 = time.time()
    sizes = netgen.ensemble_sizes(a.members)
    gains_seed = np.random.default_rng(32)
    members = member_networks(sizes)
    net = Net.batch(members, record_steps=2 * SEG, stream=_stream())
    del members
    log(f"[data] ensemble: {net.n} neurons, {len(sizes)} members, built in {time.time() - t0:.1f}s")
    tic = time.perf_counter()
    X, Y = generate(net, a.runs, a.segments, gains_seed)
    gen_s = time.perf_counter() - tic
    Xt, Yt = generate(net, a.test_runs, a.segments, np.random.default_rng(33))
    net.close()
    tic = time.perf_counter()
    m, sx, sy = train(X, Y, epochs=a.epochs)
    train_s = time.perf_counter() - tic
    err = evaluate(m, sx, sy, Xt, Yt)
    log(f"[train] held-out error: {json.dumps(err)}")
    rep = {"samples": int(len(X)), "test_samples": int(len(Xt)), "generate_s": gen_s, "train_s": train_s,
           "held_out": err, "screen": {}}
    target = netgen.make_network(netgen.ensemble_member_spec(41, a.target_n, rate_hz=15, n_regions=R_POP))
    for s in [int(x) for x in a.seeds.split(",")]:
        hidden = np.clip(np.random.default_rng(41 + s).normal(1.0, GAIN_SD, (R_POP, 4)), 0, None).astype(np.float32)
        rep["screen"][str(s)] = screen(m, sx, sy, target, hidden, iters=a.iters, seed=s)
    H = [r for h in rep["screen"].values() for r in h]
    rep["summary"] = {
        "mean_best_fit_surrogate": float(np.mean([r["best_fit_surrogate"] for r in H])),
        "mean_best_fit_random": float(np.mean([r["best_fit_random"] for r in H])),
        "mean_fit_surrogate": float(np.mean([r["mean_fit_surrogate"] for r in H])),
        "mean_fit_random": float(np.mean([r["mean_fit_random"] for r in H])),
        "bold_corr_error": float(np.mean([r["bold_corr_error"] for r in H])),
        "corr_pred_vs_sim": float(np.mean([r["corr_pred_vs_sim"] for r in H])),
        "speedup_per_proposal": float(np.median([r["speedup_per_proposal"] for r in H])),
    }
    log(f"[summary] {json.dumps(rep['summary'])}")
    if a.out:
        with open(a.out, "w") as f:
            json.dump(rep, f, indent=1)
    print(json.dumps(rep["summary"]), flush=True)


if __name__ == "__main__":
    main()
