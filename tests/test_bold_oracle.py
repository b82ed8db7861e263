"""Pins of the FP64 Balloon-Windkessel reference (Sec. V-E): exact rest
under zero input, the closed-form fixed point under constant input (reached
by long integration), and the steady-state derivatives vanishing there."""
import json
import os

import numpy as np

from oracle import bold

GOLDEN = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "worked_examples.json")))


def test_rest_is_exact_under_zero_input():
    st, y = bold.run(np.zeros((500, 3)))
    np.testing.assert_array_equal(st, bold.rest((3,)))
    assert np.all(y == 0.0)


def test_fixed_point_closed_form_values():
    # u = 0.07 (7 Hz): f* = 1 + 0.5 * 0.07 / 0.41, v* = f*^0.32, q* = v* E(f*) / E0
    fp, y = bold.fixed_point(7.0)
    assert abs(fp[1] - 1.0853658536585367) < 1e-15
    assert abs(fp[2] - 1.0853658536585367 ** 0.32) < 1e-15
    ex = GOLDEN["bold_fixed_point_u007"]
    assert abs(fp[1] - ex["f"]) < 1e-6 and abs(fp[2] - ex["v"]) < 1e-6
    assert abs(fp[3] - ex["q"]) < 2e-6
    assert abs(y - ex["y"]) < 1e-6


def test_fixed_point_is_stationary_for_the_euler_map():
    for r in (3.0, 7.0, 30.0):
        fp, y = bold.fixed_point(r)
        nxt = bold.step(fp, r, 1e-3)
        np.testing.assert_allclose(nxt, fp, rtol=0, atol=1e-15)


def test_long_integration_converges_to_fixed_point():
    T = 60_000  # 60 s of 1 ms steps
    st, ys = bold.run(np.full((T, 1), 15.0))
    fp, y = bold.fixed_point(15.0)
    np.testing.assert_allclose(st[0], fp, rtol=0, atol=1e-6)
    assert abs(ys[-1, 0] - y) < 1e-7


# Published Balloon-Windkessel constants (Friston, Mechelli, Turner & Price
# 2000), typed here from the publication rather than taken from the module
# under test, so that a wrong constant there fails the pins below.
_KAPPA, _GAMMA, _TAU0, _ALPHA, _E0, _V0 = 0.65, 0.41, 0.98, 0.32, 0.34, 0.02
_K1, _K2, _K3 = 7 * _E0, 2.0, 2 * _E0 - 0.2


def _jacobian_at_rest(eps):
    """Jacobian of (s, f, v, q) at rest (0, 1, 1, 1), differentiated by hand:
    ds' = eps du - kappa ds - gamma df;  df' = ds;
    tau0 dv' = df - dv / alpha                       (d v^(1/alpha) = dv / alpha);
    tau0 dq' = g1 df - (1/alpha - 1) dv - dq,
    with g1 = d/df [f (1 - (1 - E0)^(1/f)) / E0] at f = 1 = 1 + (1 - E0) ln(1 - E0) / E0
    and d(v^(1/alpha) q / v) = (1/alpha - 1) dv + dq."""
    g1 = 1.0 + (1.0 - _E0) * np.log(1.0 - _E0) / _E0
    J = np.array([[-_KAPPA, -_GAMMA, 0.0, 0.0],
                  [1.0, 0.0, 0.0, 0.0],
                  [0.0, 1.0 / _TAU0, -1.0 / (_ALPHA * _TAU0), 0.0],
                  [0.0, g1 / _TAU0, -(1.0 / _ALPHA - 1.0) / _TAU0, -1.0 / _TAU0]])
    b = np.array([eps, 0.0, 0.0, 0.0])
    return J, b


def test_small_input_transient_follows_the_linearisation():
    """A weak step input (u = 1e-4) from rest: over 20 s the Euler trajectory
    of every state and of y equals the Euler map of the hand-derived
    linearisation to 1e-3 of its range (the neglected terms are O(u)); y
    linearised is V0 [-(k1 + k2) dq + (k2 - k3) dv].  The transient's decay
    rates and oscillation (kappa, gamma, tau0, alpha, E0) and the signal
    weights all enter, so a wrong constant, sign or exponent fails here
    although it would leave the fixed point intact."""
    rate = 0.01  # Hz -> u = rate / 100 = 1e-4
    u = rate / 100.0
    T, dt = 20_000, 1e-3
    J, b = _jacobian_at_rest(0.5)
    A = np.eye(4) + dt * J
    x = np.zeros(4)
    lin = np.empty((T, 4))
    for t in range(T):
        x = A @ x + dt * b * u
        lin[t] = x
    st = bold.rest(())
    got = np.empty((T, 4))
    ys = np.empty(T)
    for t in range(T):
        st = bold.step(st, rate, dt)
        got[t] = st - bold.rest(())
        ys[t] = bold.signal(st)
    for c in range(4):
        rng_c = np.max(np.abs(lin[:, c]))
        assert rng_c > 0
        assert np.max(np.abs(got[:, c] - lin[:, c])) < 1e-3 * rng_c, c
    ylin = _V0 * (-(_K1 + _K2) * lin[:, 3] + (_K2 - _K3) * lin[:, 2])
    assert np.max(np.abs(ys - ylin)) < 1e-3 * np.max(np.abs(ylin))


def test_flow_inducing_signal_is_exactly_linear():
    """s and f obey linear equations for any input, so even a strong,
    time-varying drive gives exactly the linear Euler map of (s, f): a
    damped oscillator with characteristic roots (-kappa +- sqrt(kappa^2 -
    4 gamma)) / 2 (complex for the published constants)."""
    rng = np.random.default_rng(5)
    rates = rng.uniform(0.0, 60.0, 3000)
    J, b = _jacobian_at_rest(0.5)
    A = np.eye(2) + 1e-3 * J[:2, :2]
    x = np.zeros(2)
    st = bold.rest(())
    for r in rates:
        x = A @ x + 1e-3 * b[:2] * (r / 100.0)
        st = bold.step(st, r, 1e-3)
        assert abs(st[0] - x[0]) < 1e-12 and abs((st[1] - 1.0) - x[1]) < 1e-12
    lam = np.linalg.eigvals(J[:2, :2])
    assert np.all(lam.real < 0) and np.all(np.abs(lam.imag) > 0)
    np.testing.assert_allclose(np.sort(lam.imag), [-np.sqrt(_GAMMA - _KAPPA ** 2 / 4), np.sqrt(_GAMMA - _KAPPA ** 2 / 4)])
