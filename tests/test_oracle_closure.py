"""Pins of the closure oracle (an MLP correction of the discrete ROM; not in
the paper): closed forms, central finite differences in float64, the
textbook first Adam step, permutation property of the epoch order, and
reductions of the closure rollout to the plain ROM."""
import math

import numpy as np
import pytest

import oracle as orc
import oracle.closure as cl


def test_gelu_closed_forms():
    assert cl.gelu(np.array(0.0)) == 0.0
    # Phi(1) = 0.8413447460685429 (standard normal CDF)
    assert cl.gelu(np.array(1.0)) == pytest.approx(0.8413447460685429, rel=1e-15)
    x = np.linspace(-5, 5, 41)
    assert np.allclose(cl.gelu(x) - cl.gelu(-x), x, rtol=0, atol=1e-15)   # Phi(x) + Phi(-x) = 1
    h = 1e-6
    fd = (cl.gelu(x + h) - cl.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(fd - cl.gelu_grad(x))) < 1e-8


def test_bf16_rounding_ties_to_even():
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 3 * 2 ** -8), 2 ** -130, 65504.0, 1 + 2 ** -7])
    out = cl.bf16_round(vals)
    assert out[0] == 1.0
    assert out[1] == 1.0                      # halfway, even neighbour is 1
    assert out[2] == 1 + 2 ** -6              # halfway between 1+2^-7 (odd) and 1+2^-6 (even)
    assert out[3] == -(1 + 2 ** -6)
    assert out[6] == 1 + 2 ** -7              # representable
    assert np.isnan(cl.bf16_round(np.array([np.nan])))[0]


def test_backward_matches_central_differences():
    rng = np.random.default_rng(1)
    r, h, B = 3, 8, 5
    p = rng.standard_normal(cl.n_params(r, h)) * 0.4
    xn = rng.standard_normal((B, r))
    yn = rng.standard_normal((B, r))
    loss, g = cl.loss_and_grad(p, xn, yn, r, bf16=False, h=h)
    fd = np.empty_like(p)
    eps = 1e-6
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = eps
        lp, _ = cl.loss_and_grad(p + e, xn, yn, r, bf16=False, h=h)
        lm, _ = cl.loss_and_grad(p - e, xn, yn, r, bf16=False, h=h)
        fd[i] = (lp - lm) / (2 * eps)
    assert np.linalg.norm(fd - g) / np.linalg.norm(g) < 1e-7


def test_first_adam_step_closed_form():
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = cl.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 1e-3, 0.9, 0.999, 1e-8)
    assert np.allclose(p, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)


@pytest.mark.parametrize("N", [1, 7, 12, 256, 1999])
def test_epoch_order_is_a_permutation(N):
    for e in range(5):
        o = cl.epoch_order(N, e)
        assert sorted(o.tolist()) == list(range(N))


def _toy_rom():
    sysq = __import__("synth").c1_system(seed=41, r=3, k=30, rho=0.9, h_fro=0.1, c_var=1e-2)
    _, G, B = orc.opinf_data(sysq.q)
    O = orc.solve_operators(G, B, 3, 1e-8, 1e-8)
    return O, sysq.q


def test_closure_rollout_reduces_to_plain_rom():
    O, Qhat = _toy_rom()
    r = 3
    rng = np.random.default_rng(2)
    p = rng.standard_normal(cl.n_params(r)) * 0.1
    norms = (np.zeros(r), np.ones(r), np.zeros(r), np.ones(r))
    plain = orc.rollout(O, r, Qhat[:, 0], 25)
    Qt, latched = cl.closure_rollout(O, r, p, norms, 0.0, Qhat[:, 0], 25)   # disabled
    assert np.array_equal(Qt, plain) and latched == -1
    Qt, latched = cl.closure_rollout(O, r, p, norms, 1e-300, Qhat[:, 0], 25)  # latches at once
    assert np.allclose(Qt, plain, rtol=0, atol=1e-15) and latched == 0
    # a network whose output is a constant shift acts as an extra constant term
    zero = np.zeros(cl.n_params(r))
    shift = np.array([0.01, -0.02, 0.005])
    norms_c = (np.zeros(r), np.ones(r), shift, np.ones(r))
    Qt, latched = cl.closure_rollout(O, r, zero, norms_c, 1e9, Qhat[:, 0], 25)
    O2 = O.copy()
    O2[:, -1] += shift
    assert np.allclose(Qt, orc.rollout(O2, r, Qhat[:, 0], 25), rtol=1e-13, atol=1e-15)


def test_residuals_vanish_for_exact_rom():
    O, Qhat = _toy_rom()
    R = cl.residuals(O, 3, Qhat)
    assert R.shape == (29, 3)
    assert np.max(np.abs(R)) < 1e-6


def test_fit_reduces_loss():
    rng = np.random.default_rng(3)
    r, N = 4, 300
    X = rng.standard_normal((N, r))
    Y = np.tanh(X @ rng.standard_normal((r, r))) * 0.1
    p0 = rng.standard_normal(cl.n_params(r)) * 0.05
    p, norms, log = cl.fit(p0, X, Y, r, epochs=20, batch=64, lr=3e-3)
    assert log[-1] < 0.5 * log[0]


def test_standardization_population_std_and_zero_variance():
    # column 0: values 1, 3, 5 -> mean 3, population variance (4 + 0 + 4) / 3;
    # column 1 is constant -> its deviation counts as 1 (a sample deviation
    # would give variance 8 / 2 = 4)
    X = np.array([[1.0, 5.0], [3.0, 5.0], [5.0, 5.0]])
    Y = np.array([[0.0, -2.0], [0.0, 2.0], [3.0, 0.0]])
    mx, sx, my, sy = cl.standardization(X, Y)
    assert mx.tolist() == [3.0, 5.0]
    assert sx[0] == pytest.approx(math.sqrt(8.0 / 3.0), rel=1e-15) and sx[1] == 1.0
    assert my.tolist() == [1.0, 0.0]
    # Y column 0: deviations -1, -1, 2 -> variance 6 / 3 = 2; column 1: 8 / 3
    assert sy[0] == pytest.approx(math.sqrt(2.0), rel=1e-15)
    assert sy[1] == pytest.approx(math.sqrt(8.0 / 3.0), rel=1e-15)


def test_adam_bias_correction_constant_gradient():
    # with a constant gradient g the bias-corrected moments are exactly g and
    # g^2 at every step, so step t moves by lr * g / (|g| + eps): after t steps
    # p = -t lr sign(g) |g| / (|g| + eps).  Without the correction the first
    # steps would be (1 - b1^t) / sqrt(1 - b2^t) times as long (0.1 / 0.0316).
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    g = np.array([0.5, -3.0])
    p, m, v = np.zeros(2), np.zeros(2), np.zeros(2)
    for t in (1, 2, 3):
        p, m, v = cl.adam_step(p, g, m, v, t, lr, b1, b2, eps)
        assert np.allclose(p, -t * lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0)
        assert np.allclose(m, (1 - 0.9 ** t) * g, rtol=1e-13)


def test_adam_second_step_hand_values():
    # g1 = 1, g2 = -1: m1 = 0.1, v1 = 0.001; m2 = 0.09 - 0.1 = -0.01,
    # v2 = 0.000999 + 0.001 = 0.001999; bias corrections 1 - 0.81 = 0.19 and
    # 1 - 0.998001 = 0.001999, so mhat2 = -1/19 and vhat2 = 1 exactly:
    # p2 = -lr / (1 + eps) + (lr / 19) / (1 + eps)
    lr, eps = 1e-3, 1e-8
    p, m, v = cl.adam_step(np.zeros(1), np.ones(1), np.zeros(1), np.zeros(1), 1, lr, 0.9, 0.999, eps)
    assert p[0] == pytest.approx(-lr / (1 + eps), rel=1e-14)
    p, m, v = cl.adam_step(p, -np.ones(1), m, v, 2, lr, 0.9, 0.999, eps)
    assert m[0] == pytest.approx(-0.01, rel=1e-13) and v[0] == pytest.approx(0.001999, rel=1e-13)
    assert p[0] == pytest.approx(-lr / (1 + eps) + (lr / 19.0) / (1 + eps), rel=1e-11)


def _fit_data(seed=4, r=3, N=40):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((N, r)) * np.array([2.0, 0.5, 1.0]) + 1.0
    Y = np.tanh(X @ rng.standard_normal((r, r))) * 0.2 - 0.1
    p0 = (rng.standard_normal(cl.n_params(r)) * 0.05).astype(np.float32).astype(np.float64)
    return X, Y, p0


def test_fit_with_zero_rate_keeps_weights_and_logs_the_mean_loss():
    r = 3
    X, Y, p0 = _fit_data(r=r)
    p, norms, log = cl.fit(p0, X, Y, r, epochs=3, batch=16, lr=0.0)
    assert np.array_equal(p, p0)
    mx, sx, my, sy = norms
    full, _ = cl.loss_and_grad(p0, (X - mx) / sx, (Y - my) / sy, r)
    # batches of 16, 16, 8 rows: the size-weighted mean of batch means is the
    # mean over all rows
    assert np.allclose(log, full, rtol=1e-12, atol=0)


def test_fit_one_full_batch_epoch_is_one_adam_step():
    r, lr = 3, 1e-2
    X, Y, p0 = _fit_data(seed=5, r=r, N=24)
    p, norms, log = cl.fit(p0, X, Y, r, epochs=1, batch=X.shape[0], lr=lr)
    mx, sx, my, sy = norms
    # the full-batch gradient does not depend on the visiting order (the
    # gradient itself is pinned by central differences above)
    _, g = cl.loss_and_grad(p0, (X - mx) / sx, (Y - my) / sy, r)
    exp, _, _ = cl.adam_step(p0, g, np.zeros_like(p0), np.zeros_like(p0), 1, lr, 0.9, 0.999, 1e-8)
    exp = exp.astype(np.float32).astype(np.float64)
    # equal up to one float32 rounding step of the master weights
    assert np.max(np.abs(p - exp) / np.maximum(np.abs(exp), 1e-30)) <= 2.0 ** -23
    # and every weight moved by lr |g| / (|g| + eps) (first Adam step), up to
    # the float32 rounding of the master weight
    moved = np.abs(p - p0)
    tol = 2.0 ** -23 * (np.abs(p0) + lr)
    assert np.all(np.abs(moved - lr * np.abs(g) / (np.abs(g) + 1e-8)) <= tol)


def test_closure_eval_constant_output_unstandardizes():
    # zero weights, output bias b3 = beta: g(x) = beta * s_y + m_y for every x
    r = 3
    p = np.zeros(cl.n_params(r))
    beta = np.array([0.5, -1.0, 2.0])
    p[-r:] = beta
    norms = (np.array([1.0, 2.0, 3.0]), np.array([0.5, 4.0, 1.0]),
             np.array([10.0, -20.0, 0.25]), np.array([3.0, 0.5, 8.0]))
    X = np.random.default_rng(6).standard_normal((7, r))
    G = cl.closure_eval(p, norms, X, r)
    exp = beta * norms[3] + norms[2]
    assert np.allclose(G, np.broadcast_to(exp, G.shape), rtol=1e-15, atol=0)
