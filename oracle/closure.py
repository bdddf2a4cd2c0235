"""Oracle for the learned closure on the discrete quadratic ROM of Eq. (11).

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the
product path.  The closure is not part of arXiv:2504.14338; it is a small MLP
g: R^r -> R^r (r -> 128 -> 128 -> r, GELU) that corrects the one-step ROM map,
  q_{t+1} = f_ROM(q_t) + g(q_t),
trained on the ROM's one-step residuals of the reduced training data.

Arithmetic model (the points where the GPU rounds are emulated here):
  * inputs and targets are standardized per mode (training mean and
    population standard deviation; a zero deviation counts as 1);
  * the standardized input, every weight matrix and every hidden activation
    are rounded to bfloat16 (round to nearest even of their float32 value)
    before entering a product; biases stay float32-valued;
  * the GPU accumulates in float32, the oracle in float64;
  * loss = mean squared error over the batch and the r outputs
    (standardized units); gradients pass straight through the bfloat16
    roundings of the activations;
  * Adam follows Kingma & Ba (2015), Algorithm 1, on float32 master weights.
Parity with the GPU is pinned for one forward/backward pass (gradients) and
for the inference map; the training trajectory is parity-unpinned beyond a
few steps (bfloat16 rounding decisions may diverge).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

HIDDEN = 128


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even) of the float32 value of x."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    is_nan = ((u & 0x7F800000) == 0x7F800000) & ((u & 0x007FFFFF) != 0)
    lsb = (u >> 16) & 1
    rounded = ((u + 0x7FFF + lsb) >> 16) << 16
    rounded = np.where(is_nan, (u | 0x00400000) & 0xFFFF0000, rounded)
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(x))


def gelu(x):
    """GELU, error-function form: x * Phi(x)."""
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def n_params(r, h=HIDDEN):
    return h * r + h + h * h + h + r * h + r


def unpack(p, r, h=HIDDEN):
    """Packed float32 parameter vector -> (W1 h x r, b1, W2 h x h, b2, W3 r x h, b3)."""
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + h * r].reshape(h, r); o += h * r
    b1 = p[o:o + h]; o += h
    W2 = p[o:o + h * h].reshape(h, h); o += h * h
    b2 = p[o:o + h]; o += h
    W3 = p[o:o + r * h].reshape(r, h); o += r * h
    b3 = p[o:o + r]; o += r
    assert o == p.size
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])


def standardization(X, Y):
    """Per-mode mean and population standard deviation of inputs and targets."""
    mx, my = X.mean(axis=0), Y.mean(axis=0)
    sx, sy = X.std(axis=0), Y.std(axis=0)
    sx = np.where(sx > 0, sx, 1.0)
    sy = np.where(sy > 0, sy, 1.0)
    return mx, sx, my, sy


def forward(p, xn, r, bf16=True, h=HIDDEN):
    """MLP on standardized inputs xn (B x r); returns (out, cache)."""
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(p, r, h)
    xb = rnd(xn)
    z1 = xb @ rnd(W1).T + b1
    a1 = rnd(gelu(z1))
    z2 = a1 @ rnd(W2).T + b2
    a2 = rnd(gelu(z2))
    out = a2 @ rnd(W3).T + b3
    return out, dict(xb=xb, z1=z1, a1=a1, z2=z2, a2=a2, W1=rnd(W1), W2=rnd(W2), W3=rnd(W3))


def loss_and_grad(p, xn, yn, r, bf16=True, h=HIDDEN):
    """Mean squared error over all B x r outputs and its gradient (packed)."""
    out, c = forward(p, xn, r, bf16, h)
    B = xn.shape[0]
    diff = out - yn
    loss = float(np.mean(diff * diff))
    dout = 2.0 * diff / (B * r)
    dW3 = dout.T @ c["a2"]
    db3 = dout.sum(axis=0)
    dz2 = (dout @ c["W3"]) * gelu_grad(c["z2"])
    dW2 = dz2.T @ c["a1"]
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ c["W2"]) * gelu_grad(c["z1"])
    dW1 = dz1.T @ c["xb"]
    db1 = dz1.sum(axis=0)
    return loss, pack(dW1, db1, dW2, db2, dW3, db3)


def adam_step(p, g, m, v, t, lr, beta1, beta2, eps):
    """One Adam update (Kingma & Ba 2015, Algorithm 1); t counts from 1."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def epoch_order(N, epoch):
    """Deterministic per-epoch visiting order i -> (a*i + c) mod N with
    a = max(1, (epoch*2654435761 + 1) mod N) advanced to the next value
    coprime with N, and c = (epoch*40503 + 17) mod N."""
    if N == 1:
        return np.zeros(1, dtype=np.int64)
    a = (epoch * 2654435761 + 1) % N
    if a == 0:
        a = 1
    while math.gcd(a, N) != 1:
        a = a + 1 if a + 1 < N else 1
    c = (epoch * 40503 + 17) % N
    return (a * np.arange(N, dtype=np.int64) + c) % N


def fit(p0, X, Y, r, epochs, batch, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Minibatch Adam on standardized data; returns (params, norms, loss log)."""
    mx, sx, my, sy = standardization(X, Y)
    xn = (X - mx) / sx
    yn = (Y - my) / sy
    p = np.asarray(p0, dtype=np.float64).copy()
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    N = X.shape[0]
    t = 0
    log = []
    for e in range(epochs):
        order = epoch_order(N, e)
        tot = 0.0
        for s in range(0, N, batch):
            idx = order[s:s + batch]
            loss, g = loss_and_grad(p, xn[idx], yn[idx], r)
            t += 1
            p, m, v = adam_step(p, g, m, v, t, lr, beta1, beta2, eps)
            p = p.astype(np.float32).astype(np.float64)   # float32 master weights
            tot += loss * len(idx)
        log.append(tot / N)
    return p, (mx, sx, my, sy), np.array(log)


def closure_eval(p, norms, X, r):
    """g(x) in physical units for every row of X."""
    mx, sx, my, sy = norms
    out, _ = forward(p, (X - mx) / sx, r)
    return out * sy + my


def rom_step(O, r, x):
    from .pipeline import split_operators, quad_features
    A, H, c = split_operators(O, r)
    return A @ x + H @ quad_features(x[None, :])[0] + c


def residuals(O, r, Qhat):
    """rho_t = qhat_{t+1} - f_ROM(qhat_t), t = 0 .. k-2 (rows)."""
    k = Qhat.shape[1]
    return np.stack([Qhat[:, t + 1] - rom_step(O, r, Qhat[:, t]) for t in range(k - 1)])


def closure_rollout(O, r, p, norms, threshold, q0, n_states):
    """q_{t+1} = f_ROM(q_t) + g(q_t); once ||g(q_t)|| > threshold the rollout
    latches to the plain ROM.  threshold <= 0 disables the closure.
    Returns (trajectory r x n_states, first latched step or -1)."""
    Qt = np.empty((r, n_states))
    Qt[:, 0] = q0
    latched = -1
    with np.errstate(all="ignore"):
        for t in range(n_states - 1):
            x = Qt[:, t]
            nxt = rom_step(O, r, x)
            if threshold > 0 and latched < 0:
                g = closure_eval(p, norms, x[None, :], r)[0]
                if np.linalg.norm(g) > threshold:
                    latched = t
                else:
                    nxt = nxt + g
            Qt[:, t + 1] = nxt
    return Qt, latched
