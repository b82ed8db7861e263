"""Pins of the reference's ensemble Kalman analysis (the hyper-parameter
assimilation of Sec. V-E, stochastic EnKF stand-in).

* a linear-Gaussian problem with a large ensemble: the analysis ensemble's
  mean and covariance are the exact Kalman posterior's (closed form with the
  true prior covariance, not the ensemble's);
* a hand-computed case where every member collapses to y / H;
* huge observation error leaves the (inflated) prior; a parameter with no
  spread stays exactly; tied parameters stay tied; clamping;
* its normals are the OU background's Box-Muller draws on another stream
  (counter word 3), which are pinned against numpy's Philox.
"""
import numpy as np
import pytest

import oracle
from oracle import enkf


def test_large_ensemble_reaches_the_exact_kalman_posterior():
    rng = np.random.default_rng(0)
    P, O, M = 3, 2, 200_000
    mu = np.array([1.0, -0.5, 2.0])
    L = rng.normal(size=(P, P))
    S = L @ L.T + 0.5 * np.eye(P)
    H = rng.normal(size=(O, P))
    r = np.array([0.3, 0.5])
    y = np.array([0.7, -1.1])
    X = rng.multivariate_normal(mu, S, size=M)
    Xa = enkf.analysis(X, X @ H.T, y, r, seed=5, it=3)
    K = S @ H.T @ np.linalg.inv(H @ S @ H.T + np.diag(r))
    mu_a = mu + K @ (y - H @ mu)
    S_a = S - K @ H @ S
    se = np.sqrt(np.diag(S_a) / M)
    assert np.all(np.abs(Xa.mean(axis=0) - mu_a) < 6 * se + 1e-3 * np.abs(mu_a - mu).max())
    np.testing.assert_allclose(np.cov(Xa.T), S_a, rtol=0.03, atol=0.01 * np.abs(S_a).max())


def test_hand_computed_collapse_to_the_observation():
    X = np.array([[1.0], [2.0], [3.0]])
    Xa = enkf.analysis(X, 2.0 * X, [5.0], [1e-24], seed=1, it=0)
    # C_xy = 2, C_yy = 4: K = 1/2, x + (5 - 2x)/2 = 2.5 for every member
    np.testing.assert_allclose(Xa, 2.5, rtol=0, atol=1e-9)


def test_uninformative_observation_keeps_the_inflated_prior():
    rng = np.random.default_rng(1)
    X = rng.normal(size=(16, 5))
    Y = rng.normal(size=(16, 3))
    Xa = enkf.analysis(X, Y, np.zeros(3), np.full(3, 1e14), inflation=1.1, seed=2, it=1)
    np.testing.assert_allclose(Xa, X.mean(0) + 1.1 * (X - X.mean(0)), rtol=0, atol=1e-5)


def test_fixed_and_tied_parameters_and_clamping():
    rng = np.random.default_rng(2)
    M = 32
    g = 1.0 + 0.2 * rng.normal(size=M)
    X = np.stack([g, g, np.full(M, 1.0), np.full(M, 0.75)], axis=1)   # tied pair, two fixed
    Y = np.stack([3.0 * g + 0.1 * rng.normal(size=M), g ** 2], axis=1)
    Xa = enkf.analysis(X, Y, [3.6, 1.4], [0.01, 0.02], inflation=1.05, seed=3, it=7)
    np.testing.assert_array_equal(Xa[:, 0], Xa[:, 1])
    np.testing.assert_array_equal(Xa[:, 2], 1.0)
    np.testing.assert_array_equal(Xa[:, 3], 0.75)
    assert abs(Xa[:, 0].mean() - 1.2) < abs(g.mean() - 1.2)
    Xc = enkf.analysis(X, Y, [3.6, 1.4], [0.01, 0.02], inflation=1.05, seed=3, it=7, lo=0.9, hi=1.1)
    assert Xc.min() >= 0.9 and Xc.max() <= 1.1
    np.testing.assert_array_equal(Xc, np.clip(Xa, 0.9, 1.1))


def test_normals_are_the_pinned_box_muller_draws():
    z = oracle.normals(99, 4, 3, 5, 1)
    for i in range(3):
        for j in range(5):
            assert z[i, j] == oracle.ou_normal(99, 4, i, j)
    x = oracle.normals(7, 0, 200, 100, 2).ravel()
    assert abs(x.mean()) < 5 / np.sqrt(x.size) and abs(x.var() - 1) < 5 * np.sqrt(2 / x.size)
    assert not np.array_equal(oracle.normals(7, 0, 4, 4, 2), oracle.normals(7, 1, 4, 4, 2))


def test_analysis_needs_two_members():
    with pytest.raises(ValueError):
        enkf.analysis(np.ones((1, 2)), np.ones((1, 1)), [0.0], [1.0])
