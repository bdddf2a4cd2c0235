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
