"""Pins of the oracle's Step V (postprocessing), lifting and continuous-time
OpInf functions against facts that do not come from the oracle itself:
closed forms (finite differences exact on quadratics, the Runge-Kutta
stability polynomial), convergence orders, an independent ODE integrator
(scipy), a thin SVD, and exact reconstruction of rank-r data."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle as orc
import synth
from oracle import continuous as cont


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ------------------------------------------------------------- lifting ----

def test_lift_closed_form():
    # cells x snapshots blocks: rho = 2^j (exact reciprocals), m = small ints
    n, k = 5, 4
    rho = 2.0 ** np.arange(-2, 3)[:, None] * np.ones((1, k))
    mom = np.arange(n * k, dtype=float).reshape(n, k) - 7.0
    Q = np.concatenate([rho, mom])
    spec = [(orc.LIFT_RECIPROCAL, 0, 0), (orc.LIFT_PRODUCT, 1, 2), (orc.LIFT_COPY, 1, 0),
            (orc.LIFT_PRODUCT, 0, 0)]
    # the product refers to an INPUT variable only: (1, 2) is invalid
    with pytest.raises(ValueError):
        orc.lift(Q, n, spec)
    spec = [(orc.LIFT_RECIPROCAL, 0, 0), (orc.LIFT_PRODUCT, 1, 1), (orc.LIFT_COPY, 1, 0),
            (orc.LIFT_PRODUCT, 0, 1)]
    L = orc.lift(Q, n, spec)
    assert L.shape == (4 * n, k)
    assert np.array_equal(L[:n], 1.0 / rho) and np.array_equal(L[:n], 2.0 ** -np.arange(-2, 3)[:, None] * np.ones((1, k)))
    assert np.array_equal(L[n:2 * n], mom * mom)
    assert np.array_equal(L[2 * n:3 * n], mom)
    assert np.array_equal(L[3 * n:], rho * mom)


# -------------------------------------------------------------- step V ----

def test_postprocess_reconstructs_rank_r_data_exactly():
    # noise-free lifted data of rank r: centering and scaling keep the rank
    # (Qs = S^-1 V (X - xbar 1^T)), so the rank-r basis spans Qs and lifting
    # the reduced training data Qhat returns the snapshots themselves
    Q, var_rows, _, _ = synth.c1_snapshots(seed=3, n_per_var=300, nvars=2, r=5, k=80, noise_var=0.0)
    ref = orc.pipeline(Q, var_rows, 5, 1e-6, 1e-4, 160)
    rows = np.array([0, 7, 299, 300, 455, 599])
    V, pred = orc.postprocess(Q, ref["mu"], ref["s"], var_rows, ref["Tr"], rows, ref["Qhat"])
    assert V.shape == (6, 5) and pred.shape == (6, 80)
    assert rel(pred, Q[rows]) < 1e-11
    # a reconstruction that forgot the inverse scale or the mean would miss
    assert rel(V @ ref["Qhat"] + ref["mu"][rows][:, None], Q[rows]) > 1e-3


def test_basis_rows_are_left_singular_vectors():
    # V_r = Qs T_r equals the leading left singular vectors of Qs (Eq. (4),
    # Eq. (7)), each with the sign of its eigenvector w_j
    Q, var_rows, _, _ = synth.c1_snapshots(seed=4, n_per_var=200, nvars=2, r=4, k=60, noise_var=1e-6)
    ref = orc.pipeline(Q, var_rows, 4, 1e-6, 1e-4, 120)
    Qs = ref["Qs"]
    Usvd, sig, Wt = np.linalg.svd(Qs, full_matrices=False)
    V = orc.basis_rows(Qs, ref["Tr"], np.arange(Qs.shape[0]))
    for j in range(4):
        sgn = np.sign(np.dot(Wt[j], ref["U"][:, j]))
        assert rel(V[:, j], sgn * Usvd[:, j]) < 1e-9
    assert rel(V.T @ V, np.eye(4)) < 1e-12


# ------------------------------------------------- continuous-time form ----

def test_fd_derivative_exact_on_quadratics():
    dt = 0.37
    k = 9
    t = dt * np.arange(k)
    rng = np.random.default_rng(0)
    a, b, c = rng.normal(size=(3, 3, 1))
    Qh = a + b * t[None, :] + c * t[None, :] ** 2
    Qd = cont.fd_derivative(Qh, dt)
    assert rel(Qd, b + 2 * c * t[None, :]) < 1e-13


def test_fd_derivative_second_order():
    # sin(w t): the error shrinks 4x when dt halves, at the ends as inside
    w = 3.0
    errs = []
    for dt in (0.02, 0.01):
        t = dt * np.arange(int(round(1.0 / dt)) + 1)
        Qd = cont.fd_derivative(np.sin(w * t)[None, :], dt)[0]
        e = np.abs(Qd - w * np.cos(w * t))
        errs.append((e[0], np.max(e[1:-1]), e[-1]))
    for e1, e2 in zip(*errs):
        assert 3.6 < e1 / e2 < 4.4


def test_rk4_stability_polynomial():
    # q' = lam q: one classical RK4 step multiplies by 1 + z + z^2/2 + z^3/6 + z^4/24
    lam, dt = -0.8, 0.3
    z = lam * dt
    O = np.array([[lam, 0.0, 0.0]])  # r = 1: [A | H | c]
    q = cont.rk4_step(O, 1, np.array([1.7]), dt)
    assert q[0] == pytest.approx(1.7 * (1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24), rel=1e-15)
    # the constant term enters every stage: q' = c gives q + c dt exactly
    O = np.array([[0.0, 0.0, 2.5]])
    assert cont.rk4_step(O, 1, np.array([1.0]), 0.1)[0] == pytest.approx(1.25, rel=1e-15)


def _quad_system(r=3, seed=7):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(r, r))
    A = 0.5 * (A - A.T) - 0.02 * np.eye(r)
    s = orc.n_quad(r)
    H = 0.1 * rng.normal(size=(r, s))
    c = 0.05 * rng.normal(size=r)
    return np.concatenate([A, H, c[:, None]], axis=1)


def test_rk4_rollout_fourth_order_against_scipy():
    r = 3
    O = _quad_system(r)
    q0 = np.array([0.8, -0.4, 0.3])
    T = 2.0
    ref = solve_ivp(lambda t, q: cont.rhs_eval(O, r, q), (0, T), q0, method="DOP853", rtol=1e-13,
                    atol=1e-14, dense_output=True)
    errs = []
    for dt in (0.1, 0.05):
        n = int(round(T / dt)) + 1
        traj = cont.rollout_continuous(O, r, q0, n, dt)
        exact = ref.sol(dt * np.arange(n))
        errs.append(np.max(np.abs(traj - exact)))
    assert errs[1] < 1e-6
    assert 12.0 < errs[0] / errs[1] < 20.0


def test_continuous_inference_recovers_a_known_system():
    # data from an independent integrator at spacing dt over a long, lightly
    # damped oscillation (kappa(G) ~ 5e4); second-order derivatives leave
    # O(dt^2) errors, so the operators come back to ~4e-5
    r = 3
    O_true = _quad_system(r)
    dt = 1e-2
    k = 4000
    q0 = np.array([0.8, 0.2, -0.4])
    sol = solve_ivp(lambda t, q: cont.rhs_eval(O_true, r, q), (0, dt * (k - 1)), q0, method="DOP853",
                    rtol=1e-13, atol=1e-14, t_eval=dt * np.arange(k))
    assert sol.success and sol.y.shape == (r, k)
    Qh = sol.y
    Dhat, G, B = cont.opinf_data_continuous(Qh, dt)
    assert Dhat.shape == (k, r + orc.n_quad(r) + 1)
    assert np.array_equal(Dhat[:, :r], Qh.T) and np.all(Dhat[:, -1] == 1.0)
    O = cont.solve_regularized(G, B, r, 1e-12, 1e-12)
    assert rel(O, O_true) < 1e-3
    # the residual of the fitted right-hand side matches the derivative error
    assert rel(Dhat @ O.T, cont.fd_derivative(Qh, dt).T) < 1e-4


def test_continuous_regularized_solution_is_stacked_least_squares():
    rng = np.random.default_rng(2)
    Qh = rng.normal(size=(3, 40))
    dt, b1, b2 = 0.05, 1e-2, 3e-1
    Dhat, G, B = cont.opinf_data_continuous(Qh, dt)
    O = cont.solve_regularized(G, B, 3, b1, b2)
    g = orc.regularizer(3, b1, b2)
    X = np.linalg.lstsq(np.vstack([Dhat, np.diag(np.sqrt(g))]),
                        np.vstack([cont.fd_derivative(Qh, dt).T, np.zeros((len(g), 3))]), rcond=None)[0]
    assert rel(O, X.T) < 1e-12
