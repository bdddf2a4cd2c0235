"""GPU parity of the continuous-time variant (Sec. 3.5, Eq. (10)) and of the
lifting transformations (Sec. 3.3), through the C ABI, against the oracle.

Data: a lightly damped quadratic system dq/dt = A q + H quad(q) + c (r = 3)
integrated by scipy's DOP853 at 1e-13 tolerance, sampled at dt = 0.01 (4000
snapshots).  Operators: tests/opcheck.py's end-to-end check with k-term sums
(the continuous data matrix has k rows).  Rollouts of identical operators:
1e-9 of the trajectory scale (RK4 stages evaluated in a different summation
order)."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle as orc
from oracle import continuous as cont
from opcheck import check_operators, rel

pytestmark = pytest.mark.gpu

DT, K = 1e-2, 4000


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def quad_system(r=3, seed=7):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(r, r))
    A = 0.5 * (A - A.T) - 0.02 * np.eye(r)
    H = 0.1 * rng.normal(size=(r, orc.n_quad(r)))
    c = 0.05 * rng.normal(size=r)
    return np.concatenate([A, H, c[:, None]], axis=1)


@pytest.fixture(scope="module")
def data():
    O_true = quad_system()
    sol = solve_ivp(lambda t, q: cont.rhs_eval(O_true, 3, q), (0, DT * (K - 1)), np.array([0.8, 0.2, -0.4]),
                    method="DOP853", rtol=1e-13, atol=1e-14, t_eval=DT * np.arange(K))
    assert sol.success
    return O_true, sol.y


def test_continuous_inference_parity(gpu_lib, data):
    import torch
    dp = gpu_lib
    O_true, Qh = data
    r_list = [2, 3]
    b1 = [1e-12, 1e-6, 1e-3]
    b2 = [1e-12, 1e-4, 1e-1]
    O, status, views = dp.infer_continuous(dev(Qh), DT, r_list, b1, b2)
    torch.cuda.synchronize()
    assert np.all(status.cpu().numpy() == 0)
    for g, r in enumerate(r_list):
        _, G, B = cont.opinf_data_continuous(Qh[:r], DT)
        for p in range(len(b1)):
            # k data rows: k-term sums, i.e. the bound for k + 1 snapshots
            check_operators(G, B, r, b1[p], b2[p], views[g][p].cpu().numpy(), K + 1, (r, p))
    # the known system comes back from its own samples (O(dt^2) derivatives)
    assert rel(views[1][0].cpu().numpy(), O_true) < 1e-3


@pytest.mark.parametrize("one_wg", [False, True], ids=["team", "one_wg"])
def test_continuous_rollout_parity(gpu_lib, data, one_wg):
    # both forms: co-resident teams of ceil(r / 8) workgroups exchanging each
    # RK4 stage's right-hand side, and one workgroup per item
    import torch
    dp = gpu_lib
    O_true, Qh = data
    r_list = [2, 3]
    b1, b2 = [1e-12, 1e-3], [1e-12, 1e-1]
    Qd = dev(Qh)
    O, status, views = dp.infer_continuous(Qd, DT, r_list, b1, b2)
    n_states = 6000   # 1.5x the training window
    out = dp.rollout_continuous(O, Qd, r_list, 2, n_states, DT, solve_status=status, keep_traj=True, full=True,
                                one_wg=one_wg)
    torch.cuda.synchronize()
    te, gr, oc = (out[k].cpu().numpy() for k in ("train_err", "growth", "outcome"))
    for g, r in enumerate(r_list):
        for p in range(2):
            it = g * 2 + p
            Og = views[g][p].cpu().numpy()
            ref = cont.rollout_continuous(Og, r, Qh[:r, 0], n_states, DT)
            tr = out["traj_views"][g][p].cpu().numpy().T
            fin, e, gg, ok = orc.score(ref, Qh[:r], K, 1.2)
            if not fin:
                assert oc[it] == dp.ITEM_NONFINITE
                continue
            assert np.max(np.abs(tr - ref)) <= 1e-9 * np.max(np.abs(ref)), (r, p)
            assert te[it] == pytest.approx(e, rel=1e-8)
            assert gr[it] == pytest.approx(gg, rel=1e-10)
            assert (oc[it] == dp.ITEM_PASS) == ok
    # the inferred ROM reproduces its training trajectory (the O(dt^2)
    # derivative errors drift to ~1e-3 over the 40 time units)
    assert te[2] < 1e-2
    best = out["best"].cpu().numpy()
    exp = orc.select_best([te[2], te[3]], [oc[2] == dp.ITEM_PASS, oc[3] == dp.ITEM_PASS])
    assert best[1] == (2 + exp if exp >= 0 else -1)


def test_rk4_step_closed_form(gpu_lib):
    # r = 1, dq/dt = lam q: state t = q0 (1 + z + z^2/2 + z^3/6 + z^4/24)^t
    import torch
    dp = gpu_lib
    lam, dt, q0 = -0.8, 0.05, 1.7
    O = dev(np.array([lam, 0.0, 0.0]))
    Qh = dev(np.array([[q0, q0 * 0.9, q0 * 0.8]]))
    out = dp.rollout_continuous(O, Qh, [1], 1, 50, dt, keep_traj=True, full=True)
    torch.cuda.synchronize()
    z = lam * dt
    R = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    tr = out["traj_views"][0][0].cpu().numpy()[:, 0]
    assert np.max(np.abs(tr - q0 * R ** np.arange(50))) <= 1e-13 * q0


def test_lift_parity(gpu_lib):
    import torch
    dp = gpu_lib
    rng = np.random.default_rng(3)
    n_cells, k = 1000, 77
    Q = rng.normal(size=(3 * n_cells, k))
    Q[5, 3] = 0.0        # 1 / 0 = Inf
    spec = [(dp.LIFT_COPY, 2, 0), (dp.LIFT_PRODUCT, 0, 1), (dp.LIFT_RECIPROCAL, 0, 0), (dp.LIFT_PRODUCT, 2, 2)]
    L = dp.lift(dev(Q), n_cells, spec)
    torch.cuda.synchronize()
    ref = orc.lift(Q, n_cells, spec)
    # single correctly rounded operations: bit for bit
    assert np.array_equal(L.cpu().numpy(), ref)
    assert np.isinf(L.cpu().numpy()[2 * n_cells + 5, 3])
