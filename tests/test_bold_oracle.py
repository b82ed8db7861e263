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
