"""FP64 reference of one ensemble Kalman analysis over hyper-parameters.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's assimilation (Sec. V-E) adapts per-population hyper-parameters
of an ensemble of simulated brain models so that their BOLD signals track
the measured ones, and defers the filter to its companion work.  The stand-in
here is the stochastic ensemble Kalman filter with perturbed observations
(Evensen 1994; Burgers, van Leeuwen and Evensen 1998), written out from its
definition: with the ensemble X [M, P] of parameters, their predicted
observations Y [M, O], observation y [O] and error variances r [O],

    A = inflation (X - mean X),   B = Y - mean Y,
    C_xy = A^T B / (M - 1),       C_yy = B^T B / (M - 1),
    X_m <- mean X + A_m + C_xy (C_yy + diag r)^-1 (y + sqrt(r) xi_m - Y_m),

clamped to [lo, hi]; xi_m,o are standard normals (Box-Muller on Philox
counter (iter, m, o, 2)).  Pinned by the exact Kalman posterior of a
linear-Gaussian problem (mean and covariance, large ensemble) and by a
hand-computed collapse to the posterior mean.
"""
from __future__ import annotations

import numpy as np

from . import normals


def analysis(X, Y, y_obs, r_var, inflation=1.0, seed=0, it=0, lo=-np.inf, hi=np.inf):
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    y = np.asarray(y_obs, dtype=np.float64)
    r = np.asarray(r_var, dtype=np.float64)
    M, O = Y.shape
    if M < 2 or X.shape[0] != M:
        raise ValueError("the analysis needs at least two members and one row of X per member")
    xbar = X.mean(axis=0)
    A = inflation * (X - xbar)
    B = Y - Y.mean(axis=0)
    Cxy = A.T @ B / (M - 1)
    Cyy = B.T @ B / (M - 1) + np.diag(r)
    xi = normals(seed, it, M, O, 2)
    D = y + np.sqrt(r) * xi - Y                 # innovations, [M, O]
    Xa = xbar + A + np.linalg.solve(Cyy, D.T).T @ Cxy.T
    return np.clip(Xa, lo, hi)
