"""Oracle of the continuous-time OpInf variant (arXiv:2504.14338, Sec. 3.5,
Eq. (10)): derivative data by finite differences, the regularized least
squares of Eq. (12) with those derivatives as right-hand side, and ROM
rollouts by a Runge-Kutta method.

TEST INFRASTRUCTURE ONLY: never imported by the product path.
Pins: tests/test_oracle_continuous.py.

READINGS (the paper names finite differences only "for example" and does
not give a time integrator):
  * derivatives: second-order central differences (q_{t+1} - q_{t-1}) / (2 dt)
    inside the window, and the second-order one-sided formulas
    (-3 q_0 + 4 q_1 - q_2) / (2 dt), (3 q_{k-1} - 4 q_{k-2} + q_{k-3}) / (2 dt)
    at its ends (exact for quadratics in t); k >= 3 snapshots;
  * the data matrix uses all k snapshots, Dhat = [Qhat^T | quad(Qhat^T) | 1]
    (k x d), right-hand side the k derivative vectors; regularizer as in the
    discrete form;
  * rollouts integrate Eq. (10) with the classical fourth-order Runge-Kutta
    method at the snapshot spacing dt, so that state t sits at snapshot time
    t and is scored against qhat_t exactly like a discrete rollout.
"""
from __future__ import annotations

import numpy as np

from .pipeline import quad_features, regularizer, split_operators

__all__ = ["fd_derivative", "opinf_data_continuous", "rhs_eval", "rk4_step",
           "rollout_continuous", "solve_regularized"]


def fd_derivative(Qhat, dt):
    """Time derivative of every row of Qhat (r x k) at every snapshot, by
    second-order finite differences (READING above)."""
    Qhat = np.asarray(Qhat, dtype=np.float64)
    r, k = Qhat.shape
    if k < 3:
        raise ValueError("need at least 3 snapshots")
    Qd = np.empty((r, k))
    for t in range(k):
        if t == 0:
            Qd[:, t] = (-3.0 * Qhat[:, 0] + 4.0 * Qhat[:, 1] - Qhat[:, 2]) / (2.0 * dt)
        elif t == k - 1:
            Qd[:, t] = (3.0 * Qhat[:, k - 1] - 4.0 * Qhat[:, k - 2] + Qhat[:, k - 3]) / (2.0 * dt)
        else:
            Qd[:, t] = (Qhat[:, t + 1] - Qhat[:, t - 1]) / (2.0 * dt)
    return Qd


def opinf_data_continuous(Qhat, dt):
    """Dhat = [Qhat^T | quad(Qhat^T) | 1] (k x d) and the right-hand side
    Qdot^T (k x r) of the continuous-time problem; returns (Dhat, G, B) with
    G = Dhat^T Dhat, B = Dhat^T Qdot^T."""
    Qt = np.asarray(Qhat, dtype=np.float64).T
    Dhat = np.concatenate([Qt, quad_features(Qt), np.ones((Qt.shape[0], 1))], axis=1)
    R = fd_derivative(Qhat, dt).T
    return Dhat, Dhat.T @ Dhat, Dhat.T @ R


def rhs_eval(O, r, q):
    """Right-hand side of Eq. (10): A q + H quad(q) + c."""
    A, H, c = split_operators(O, r)
    return A @ q + H @ quad_features(q[None, :])[0] + c


def rk4_step(O, r, q, dt):
    """One step of the classical fourth-order Runge-Kutta method."""
    k1 = rhs_eval(O, r, q)
    k2 = rhs_eval(O, r, q + 0.5 * dt * k1)
    k3 = rhs_eval(O, r, q + 0.5 * dt * k2)
    k4 = rhs_eval(O, r, q + dt * k3)
    return q + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def rollout_continuous(O, r, q0, n_states, dt):
    """n_states states of Eq. (10) from q0 (included), spaced by dt."""
    Qt = np.empty((r, n_states))
    Qt[:, 0] = q0
    with np.errstate(all="ignore"):
        for t in range(n_states - 1):
            Qt[:, t + 1] = rk4_step(O, r, Qt[:, t], dt)
    return Qt


def solve_regularized(G, B, r, beta1, beta2):
    """(G + diag(reg)) O^T = B with the discrete form's regularizer; O r x d."""
    M = G + np.diag(regularizer(r, beta1, beta2))
    return np.linalg.solve(M, B).T
