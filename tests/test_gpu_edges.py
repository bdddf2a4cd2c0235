"""Smallest sizes through the C ABI against the oracle: a Gram of a single
row or of fewer rows than one 16-row stage, one snapshot column; operator
inference at r = 1 and 2 (s = 1 and 3 quadratic columns) with k = 2 and 3
snapshots (one or two data rows), and rollouts and scores of the resulting
r = 1 and r = 2 ROMs.  Operator tolerances: tests/opcheck.py."""
import numpy as np
import pytest

import oracle as orc
from opcheck import check_operators

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("n,k", [(1, 3), (5, 3), (17, 2), (3, 130), (15, 1)])
def test_gram_tiny(gpu_lib, n, k):
    dp = gpu_lib
    rng = np.random.default_rng(100 * n + k)
    Q = rng.standard_normal((n, k)) + 0.5
    var_rows = [0, n]
    Qd = dev(Q)
    mean, scale, zr = dp.preprocess(Qd, var_rows)
    mu, s, Qs, z = orc.preprocess(Q, var_rows)
    assert np.allclose(mean.cpu().numpy(), mu, rtol=1e-15, atol=1e-15)
    D = dp.gram(Qd, mean, scale, var_rows).cpu().numpy()
    Dref = orc.gram(Qs)
    assert D.shape == (k, k) and np.array_equal(D, D.T)
    assert np.max(np.abs(D - Dref)) <= 1e-13 * max(1.0, np.max(np.abs(Dref)))
    D0 = dp.gram(Qd).cpu().numpy()
    assert np.max(np.abs(D0 - Q.T @ Q)) <= 1e-13 * np.max(np.abs(Q.T @ Q))


@pytest.mark.parametrize("k", [2, 3, 6])
def test_infer_and_rollout_smallest_sizes(gpu_lib, k):
    dp = gpu_lib
    rng = np.random.default_rng(7 + k)
    Qh = rng.standard_normal((2, k)) * np.array([[1.0], [0.3]])
    r_list = [1, 2]
    b1, b2 = [1e-3, 1e-1], [1e-2, 1e-2]
    O, status, views = dp.infer(dev(Qh), r_list, b1, b2)
    assert np.all(status.cpu().numpy() == 0)
    for g, r in enumerate(r_list):
        _, G, B = orc.opinf_data(Qh[:r])
        for p in range(len(b1)):
            check_operators(G, B, r, b1[p], b2[p], views[g][p].cpu().numpy(), k, (r, p))
    # rollouts of the GPU's operators: 8 states, scores against the oracle
    n_states = 8
    out = dp.rollout(O, dev(Qh), r_list, len(b1), n_states, solve_status=status, keep_traj=True, full=True)
    te, gr = out["train_err"].cpu().numpy(), out["growth"].cpu().numpy()
    for g, r in enumerate(r_list):
        for p in range(len(b1)):
            Og = views[g][p].cpu().numpy()
            ref = orc.rollout(Og, r, Qh[:r, 0], n_states)
            tr = out["traj_views"][g][p].cpu().numpy().T
            assert np.max(np.abs(tr - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref))), (r, p)
            fin, e, gg, ok = orc.score(ref, Qh[:r], k, 1.2)
            if fin:
                assert te[g * len(b1) + p] == pytest.approx(e, rel=1e-10, abs=1e-300)
                assert gr[g * len(b1) + p] == pytest.approx(gg, rel=1e-10)

    # fewer states than training snapshots: the training error runs over the
    # states there are, the growth reference over all k snapshots
    short = dp.rollout(O, dev(Qh), r_list, len(b1), 3, solve_status=status, full=True)
    te3 = short["train_err"].cpu().numpy()
    for g, r in enumerate(r_list):
        for p in range(len(b1)):
            ref = orc.rollout(views[g][p].cpu().numpy(), r, Qh[:r, 0], 3)
            assert te3[g * len(b1) + p] == pytest.approx(orc.train_error(ref, Qh[:r], min(3, k)), rel=1e-10, abs=1e-300)
