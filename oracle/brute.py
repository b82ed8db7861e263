"""Dense-tensor brute force of the partition step, for tiny nets (n <= ~64).

TEST INFRASTRUCTURE ONLY.  A second, independent formulation of what the C
reference computes, used to pin it: the synapse list is turned into dense
delay-indexed weight matrices W_E[d][i, m], W_I[d][i, m] and the recurrent
input of step t is the tensor contraction

    dE^t = sum_{d=1..D} W_E[d] @ s^{t-d+1},   dI^t = sum_d W_I[d] @ s^{t-d+1}

over the full spike history (no ring buffer, no CSR walk).  The background
uniform comes from numpy's own Philox bit generator (a library routine) and
the Poisson count from scipy's Poisson CDF, so neither the RNG nor the
inversion table of the C code is reused.  Neuron and gate updates follow
Sec. III-B Eq. (1) with forward Euler (Sec. VI-A) and exact gate decay.
"""
from __future__ import annotations

import numpy as np
import scipy.stats


def _numpy_philox_u32(seed: int, t: int, i: int, member: int) -> int:
    # one Philox block per eight neurons, counter (t, i // 8, member, 0);
    # numpy's Philox advances its 256-bit counter before producing a block,
    # so counter c - 1 yields the block of counter c, as its four words
    c = (t | ((i >> 3) << 64) | (member << 128)) - 1
    ctr = [(c >> (64 * k)) & 0xFFFFFFFFFFFFFFFF for k in range(4)]
    bg = np.random.Philox(key=np.array([seed, 0], dtype=np.uint64),
                          counter=np.array(ctr, dtype=np.uint64))
    w = int(bg.random_raw(4)[(i & 7) >> 1])
    # value i mod 8: the word's high half, then its low half
    return (w & 0xFFFFFFFF) if (i & 1) else (w >> 32)


def _thresholds(lam: float) -> np.ndarray:
    # floor(F(k) 2^32) from scipy's CDF, up to the first saturated entry
    k = np.arange(0, int(lam + 20 * np.sqrt(lam + 1) + 40))
    T = np.floor(scipy.stats.poisson.cdf(k, lam) * 4294967296.0)
    return T[:int(np.argmax(T >= 4294967295.0))]


def _count(u: int, T: np.ndarray) -> int:
    # smallest k with u < T_k (saturated entries excluded)
    return int(np.count_nonzero(u >= T))


def dense_weights(net):
    n, D = net.n, net.max_delay
    WE = np.zeros((D + 1, n, n))
    WI = np.zeros((D + 1, n, n))
    for i in range(n):
        for k in range(int(net.row_ptr[i]), int(net.row_ptr[i + 1])):
            m, d = int(net.col[k]), int(net.delay[k])
            (WI if net.is_inh[m] else WE)[d, i, m] += float(net.w[k])
    return WE, WI


def run(net, n_steps: int, forced=None, gain=None):
    """Returns raster [T, n], V and j trajectories [T+1, ...], event counts."""
    n, D = net.n, net.max_delay
    WE, WI = dense_weights(net)
    adj = np.zeros((D + 1, n, n), dtype=np.int64)
    for i in range(n):
        for k in range(int(net.row_ptr[i]), int(net.row_ptr[i + 1])):
            adj[int(net.delay[k]), i, int(net.col[k])] += 1
    P = net.ptypes.astype(np.float64)[net.ptype]
    C, gL, EL, Vth, Vr, tref, Iext = (P[:, c] for c in range(7))
    g = P[:, 7:11]
    if gain is not None:
        g = g * np.asarray(gain, dtype=np.float64)[net.region]
    E = net.E.astype(np.float64)
    a = np.exp(-net.dt_ms / net.tau_ms.astype(np.float64))
    nref = np.rint(tref / net.dt_ms).astype(np.int64)
    dt = float(net.dt_ms)
    thr = _thresholds(float(net.bg_lambda))
    V = net.V0.astype(np.float64).copy()
    j = np.zeros((n, 4))
    ref = np.zeros(n, dtype=np.int64)
    S = np.zeros((n_steps, n))
    Vs, js = [V.copy()], [j.copy()]
    ev_rec = np.zeros(n_steps, dtype=np.int64)
    ev_bg = np.zeros(n_steps, dtype=np.int64)
    for t in range(n_steps):
        Isyn = (g * j * (E[None, :] - V[:, None])).sum(axis=1) + Iext
        Vt = V + dt / C * (-gL * (V - EL) + Isyn)
        free = ref <= 0
        s = (free & (Vt >= Vth)) if forced is None else forced[t].astype(bool)
        S[t] = s
        newV = np.where(s, Vr, np.where(free, Vt, Vr))
        ref = np.where(s, nref, np.where(free, 0, ref - 1))
        V = newV
        dE = np.zeros(n)
        dI = np.zeros(n)
        for d in range(1, D + 1):
            te = t - d + 1
            if te >= 0:
                dE += WE[d] @ S[te]
                dI += WI[d] @ S[te]
                ev_rec[t] += int((adj[d] @ S[te].astype(np.int64)).sum())
        c = np.array([_count(_numpy_philox_u32(net.seed, t, i, net.member), thr)
                      for i in range(n)])
        ev_bg[t] = int(c.sum())
        dE += net.bg_w * c
        j = j * a[None, :] + np.stack([dE, dE, dI, dI], axis=1)
        Vs.append(V.copy())
        js.append(j.copy())
    return {"raster": S.astype(np.uint8), "V": np.array(Vs), "j": np.array(js),
            "ev_rec": ev_rec, "ev_bg": ev_bg}
