"""Balloon-Windkessel hemodynamics in FP64 (the BOLD model the paper's
assimilation fits to, Sec. V-E; Friston, Mechelli, Turner & Price 2000).

TEST INFRASTRUCTURE ONLY.

State per population (s, f, v, q): vasodilatory signal, inflow, volume,
deoxyhemoglobin.  With neural input u(t) (population rate in Hz / RATE_SCALE):

    ds/dt      = eps u - kappa s - gamma (f - 1)
    df/dt      = s
    tau0 dv/dt = f - v^(1/alpha)
    tau0 dq/dt = f E(f) / E0 - v^(1/alpha) q / v,     E(f) = 1 - (1 - E0)^(1/f)
    y          = V0 [k1 (1 - q) + k2 (1 - q/v) + k3 (1 - v)],
                 k1 = 7 E0, k2 = 2, k3 = 2 E0 - 0.2

integrated by forward Euler with the simulator's step (1 ms), starting at
rest (0, 1, 1, 1).  The paper prints no constants; the published ones are
used (kappa 0.65 /s, gamma 0.41 /s, tau0 0.98 s, alpha 0.32, E0 0.34,
V0 0.02); eps = 0.5 and the input scale RATE_SCALE = 100 Hz are choices.

Pinned by: the closed-form fixed point under constant input, exact rest
(y = 0) under zero input, the transient of a weak step input against the
Euler map of the model's Jacobian at rest (derived by hand, with the
published constants typed independently: decay rates, the (s, f)
oscillation, tau0, alpha, E0 and the signal weights), and the exactly
linear (s, f) subsystem under strong drive (tests/test_bold_oracle.py).
"""
from __future__ import annotations

import numpy as np

KAPPA, GAMMA, TAU0, ALPHA, E0, V0, EPS = 0.65, 0.41, 0.98, 0.32, 0.34, 0.02, 0.5
RATE_SCALE = 100.0
K1, K2, K3 = 7.0 * E0, 2.0, 2.0 * E0 - 0.2


def rest(shape) -> np.ndarray:
    """State array [..., 4] at rest."""
    st = np.zeros(tuple(shape) + (4,))
    st[..., 1:] = 1.0
    return st


def step(state: np.ndarray, rate_hz: np.ndarray, dt_s: float) -> np.ndarray:
    """One forward-Euler step; state [..., 4] = (s, f, v, q)."""
    s, f, v, q = state[..., 0], state[..., 1], state[..., 2], state[..., 3]
    u = np.asarray(rate_hz, dtype=np.float64) / RATE_SCALE
    ds = EPS * u - KAPPA * s - GAMMA * (f - 1.0)
    df = s
    vpow = v ** (1.0 / ALPHA)
    dv = (f - vpow) / TAU0
    Ef = 1.0 - (1.0 - E0) ** (1.0 / f)
    dq = (f * Ef / E0 - vpow * q / v) / TAU0
    out = np.empty_like(state)
    out[..., 0] = s + dt_s * ds
    out[..., 1] = f + dt_s * df
    out[..., 2] = v + dt_s * dv
    out[..., 3] = q + dt_s * dq
    return out


def signal(state: np.ndarray) -> np.ndarray:
    v, q = state[..., 2], state[..., 3]
    return V0 * (K1 * (1.0 - q) + K2 * (1.0 - q / v) + K3 * (1.0 - v))


def run(rates_hz: np.ndarray, dt_s: float = 1e-3, state=None):
    """rates_hz [T, ...] per-step population rates -> (final state, y [T, ...])."""
    rates_hz = np.asarray(rates_hz, dtype=np.float64)
    st = rest(rates_hz.shape[1:]) if state is None else np.array(state, dtype=np.float64)
    ys = np.empty(rates_hz.shape)
    for t in range(rates_hz.shape[0]):
        st = step(st, rates_hz[t], dt_s)
        ys[t] = signal(st)
    return st, ys


def fixed_point(rate_hz: float):
    """Closed-form steady state under constant input: s* = 0,
    f* = 1 + eps u / gamma, v* = f*^alpha, q* = v* E(f*) / E0."""
    u = rate_hz / RATE_SCALE
    f = 1.0 + EPS * u / GAMMA
    v = f ** ALPHA
    q = v * (1.0 - (1.0 - E0) ** (1.0 / f)) / E0
    y = V0 * (K1 * (1.0 - q) + K2 * (1.0 - q / v) + K3 * (1.0 - v))
    return np.array([0.0, f, v, q]), y
