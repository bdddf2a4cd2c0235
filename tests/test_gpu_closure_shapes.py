"""GPU closure training against the oracle across minibatch shapes.

The trainer runs one workgroup per 32-row chunk of a minibatch and splits
Adam over the workgroups by parameter slice, so the number of workgroups,
their row counts and the reduced size's padding (r <= 32 or 64) change with
(r, N, batch).  For each shape the loss log of the first two epochs is
compared with the oracle's training from the same initial weights (rel 1e-3:
the float32 sums and the rare bfloat16 rounding flips described in
test_gpu_closure.py move the loss by far less; an error in a chunk's rows,
a gradient share or an Adam slice moves it by much more), and the trained
parameters must be finite and equal over two identical runs (the shares are
summed in workgroup order).
"""
import numpy as np
import pytest

import oracle.closure as cl
import synth

pytestmark = pytest.mark.gpu


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("r,N,batch", [
    (10, 50, 1),      # one row per minibatch: one workgroup, 50 Adam steps per epoch
    (12, 70, 33),     # two workgroups, the second with one row; a short last minibatch
    (40, 100, 256),   # fewer rows than the minibatch: 4 of 8 workgroups hold rows
    (33, 90, 64),     # r just above 32 (padded to 64)
    (64, 64, 32),     # the largest r, one full chunk per minibatch
])
def test_training_shapes_match_oracle(gpu_lib, r, N, batch):
    import torch
    dp = gpu_lib
    rng = np.random.default_rng(1000 + r + N + batch)
    X = rng.standard_normal((N, r)) * rng.uniform(0.5, 2.0, r) + rng.standard_normal(r)
    W = rng.standard_normal((r, r)) / np.sqrt(r)
    Y = 0.1 * np.tanh(X @ W) + 0.01 * rng.standard_normal((N, r))
    p0 = synth.mlp_init(r, seed=11)
    lr = 1e-3
    params, norm, log = dp.closure_fit(dev(X), dev(Y), torch.from_numpy(p0), epochs=2, batch=batch, lr=lr)
    log = log.cpu().numpy()
    _, _, log_ref = cl.fit(p0.astype(np.float64), X, Y, r, epochs=2, batch=batch, lr=lr)
    print(f"r={r} N={N} batch={batch}: loss {log} oracle {log_ref}")
    assert np.all(np.isfinite(log))
    assert log[0] == pytest.approx(log_ref[0], rel=1e-3)
    assert log[1] == pytest.approx(log_ref[1], rel=1e-3)
    p = params.cpu().numpy()
    assert np.all(np.isfinite(p))
    params2, _, log2 = dp.closure_fit(dev(X), dev(Y), torch.from_numpy(p0), epochs=2, batch=batch, lr=lr)
    assert np.array_equal(params2.cpu().numpy(), p)
    assert np.array_equal(log2.cpu().numpy(), log)
