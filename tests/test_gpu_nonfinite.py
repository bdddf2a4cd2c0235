"""Non-finite data at the boundary, through the C ABI, against the plain
definitions the oracle computes: NaN or Inf in the snapshots Q (Step II
reports DOPINF_E_NONFINITE and NaN scales, the eigensolver refuses the NaN
Gram) and NaN in the reduced data Qhat (the normal matrix is refused, or the
operators and rollouts are not finite and no candidate is selected)."""
import numpy as np
import pytest

import oracle as orc
import synth

pytestmark = pytest.mark.gpu


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.fixture(scope="module")
def c1(gpu_lib):
    Q, var_rows, _, _ = synth.c1_snapshots(seed=1)
    return Q, var_rows


def _pre(dp, Q, var_rows, flags=None):
    import torch
    info = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    kw = {} if flags is None else {"flags": flags}
    Qd = dev(Q)
    mean, scale, zr = dp.preprocess(Qd, var_rows, info=info, **kw)
    torch.cuda.synchronize()
    return Qd, mean, scale, zr, int(info.item())


def test_clean_data_reports_ok(gpu_lib, c1):
    Q, var_rows = c1
    _, _, scale, zr, info = _pre(gpu_lib, Q, var_rows)
    assert info == gpu_lib.OK and np.all(np.isfinite(scale.cpu().numpy()))


def test_nan_in_snapshots(gpu_lib, c1):
    import torch
    dp = gpu_lib
    Q, var_rows = c1
    Q = Q.copy()
    Q[5000, 17] = np.nan          # variable 1
    Qd, mean, scale, zr, info = _pre(dp, Q, var_rows)
    assert info == dp.E_NONFINITE
    mu, s, _, _ = orc.preprocess(Q, var_rows)
    sg, mg = scale.cpu().numpy(), mean.cpu().numpy()
    # the plain definition: NaN mean of that row, NaN scale of variable 1
    assert np.isnan(mu[5000]) and np.isnan(mg[5000])
    assert np.isnan(s[1]) and np.isnan(sg[1])
    assert sg[0] == pytest.approx(s[0], rel=1e-15)
    ok = np.ones(len(mu), bool)
    ok[5000] = False
    assert np.max(np.abs(mg[ok] - mu[ok])) <= 1e-14 * np.max(np.abs(Q[ok]))
    assert zr.cpu().numpy().tolist() == [0, 0]
    # the Gram of NaN-scaled data is NaN; the eigensolver refuses it
    D = dp.gram(Qd, mean, scale, var_rows)
    _, _, _, rinfo, _ = dp.reduce(D, r=10)
    torch.cuda.synchronize()
    assert np.all(np.isnan(D.cpu().numpy()))
    assert int(rinfo.item()) == dp.E_NONFINITE


@pytest.mark.parametrize("val", [np.inf, -np.inf])
def test_inf_in_snapshots(gpu_lib, c1, val):
    dp = gpu_lib
    Q, var_rows = c1
    Q = Q.copy()
    Q[10, 3] = val                # variable 0
    _, mean, scale, zr, info = _pre(dp, Q, var_rows)
    assert info == dp.E_NONFINITE
    mu, s, _, _ = orc.preprocess(Q, var_rows)
    sg, mg = scale.cpu().numpy(), mean.cpu().numpy()
    assert mg[10] == mu[10] == val
    assert not np.isfinite(s[0]) and np.isnan(sg[0])
    assert sg[1] == pytest.approx(s[1], rel=1e-15)
    # without centering or scaling the flag is still raised, the scale is 1
    _, _, scale0, _, info0 = _pre(dp, Q, var_rows, flags=0)
    assert info0 == dp.E_NONFINITE and scale0.cpu().numpy().tolist() == [1.0, 1.0]


def test_nan_in_reduced_data(gpu_lib):
    import torch
    dp = gpu_lib
    sysq = synth.c1_system(seed=21, r=3, k=40, rho=0.9, h_fro=0.2, c_var=1e-2)
    Qh = sysq.q.copy()
    # a NaN inside the window reaches G: every normal matrix is refused
    Qn = Qh.copy()
    Qn[1, 7] = np.nan
    O, status, _ = dp.infer(dev(Qn), [2, 3], [1e-6, 1e-2], [1e-4, 1e-1])
    out = dp.rollout(O, dev(Qn), [2, 3], 2, 60, solve_status=status)
    torch.cuda.synchronize()
    assert np.all(status.cpu().numpy() == dp.E_NOTSPD)
    assert np.all(out["outcome"].cpu().numpy() == dp.ITEM_SOLVE)
    assert out["best"].cpu().numpy().tolist() == [-1, -1]
    # a NaN in the last snapshot only reaches the right-hand side (Qhat_2):
    # the factorization succeeds, the operators are NaN, the rollouts are
    # rejected as non-finite, as the oracle's solve and score find
    Ql = Qh.copy()
    Ql[0, -1] = np.nan
    O, status, views = dp.infer(dev(Ql), [3], [1e-6], [1e-4])
    out = dp.rollout(O, dev(Ql), [3], 1, 60, solve_status=status)
    torch.cuda.synchronize()
    _, G, B = orc.opinf_data(Ql)
    Oref = orc.solve_operators(G, B, 3, 1e-6, 1e-4)
    fin, _, _, ok = orc.score(orc.rollout(Oref, 3, Ql[:, 0], 60), Ql, Ql.shape[1], 1.2)
    assert not fin and not ok
    assert int(status.item()) == dp.OK
    assert np.isnan(views[0][0].cpu().numpy()).any()
    assert int(out["outcome"].item()) == dp.ITEM_NONFINITE
    assert out["best"].cpu().numpy().tolist() == [-1]
