"""GPU parity of Step V (Sec. 3.6): basis rows V_r[rows] = Qs[rows] T_r and the
prediction s_v V_r[rows] Qtilde + mean, through the C ABI, against the oracle.

Tolerance: V's entries are k-term sums, |dV_ij| <= gamma_k (|Qs| |T_r|)_ij
for any summation order (plus one rounding of the centering and of the
division), so V is checked entry by entry against 2 gamma_k (|Qs| |T_r|) +
4 u |V|; pred adds an r-term sum and one multiply-add: normwise 1e-12.
"""
import numpy as np
import pytest

import oracle as orc
import synth

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.fixture(scope="module")
def c1(gpu_lib):
    dp = gpu_lib
    Q, var_rows, _, _ = synth.c1_snapshots(seed=1)
    Qd = dev(Q)
    mean, scale, _ = dp.preprocess(Qd, var_rows)
    D = dp.gram(Qd, mean, scale, var_rows)
    lam, Tr, Qhat, info, r = dp.reduce(D, r=10)
    assert int(info.item()) == 0
    return dict(Q=Q, Qd=Qd, var_rows=var_rows, mean=mean, scale=scale, Tr=Tr, Qhat=Qhat.contiguous())


def check_V(Q, mean, scale, var_rows, Tr, rows, V):
    k = Q.shape[1]
    s_rows = np.repeat(scale, np.diff(var_rows))
    Qs = orc.apply_statistics(Q[rows], mean[rows], s_rows[rows])
    Vref = orc.basis_rows(Qs, Tr, np.arange(len(rows)))
    gam = k * U / (1 - k * U)
    bound = 2 * gam * (np.abs(Qs) @ np.abs(Tr)) + 4 * U * np.abs(Vref)
    assert np.all(np.abs(V - Vref) <= bound), float(np.max(np.abs(V - Vref) / bound))
    return Vref


@pytest.mark.parametrize("m", [1, 37, 64, 130])
def test_postprocess_rows_parity_c1(gpu_lib, c1, m):
    import torch
    dp = gpu_lib
    rng = np.random.default_rng(m)
    n = c1["Q"].shape[0]
    rows = np.sort(rng.choice(n, m, replace=False))
    if m > 4:
        rows[:4] = [0, 4095, 4096, n - 1]
    rows_d = torch.from_numpy(rows.astype(np.int64)).cuda()
    # Qtilde: the reduced training data, r x 600 (600 = 4 x 128 + 88 columns)
    Qt = c1["Qhat"]
    V, pred, info = dp.postprocess(c1["Qd"], c1["Tr"], rows=rows_d, Qtilde=Qt, mean=c1["mean"],
                                   scale=c1["scale"], var_rows=c1["var_rows"])
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    mean, scale = c1["mean"].cpu().numpy(), c1["scale"].cpu().numpy()
    Tr = c1["Tr"].cpu().numpy()
    check_V(c1["Q"], mean, scale, np.asarray(c1["var_rows"]), Tr, rows, V.cpu().numpy())
    Qtn = Qt.cpu().numpy()
    pg = pred.cpu().numpy()
    Vr, pr = orc.postprocess(c1["Q"], mean, scale, c1["var_rows"], Tr, rows, Qtn)
    assert rel(pg, pr) <= 1e-12
    # the whole chain against the oracle's own statistics, basis and Qhat
    ref = orc.pipeline(c1["Q"], c1["var_rows"], 10, 1e-6, 1e-4, 1200)
    Vo, po = orc.postprocess(c1["Q"], ref["mu"], ref["s"], c1["var_rows"], ref["Tr"], rows, ref["Qhat"])
    assert rel(V.cpu().numpy(), Vo) <= 1e-9
    assert rel(pg, po) <= 1e-9
    # lifting the training data reproduces the snapshots to the noise level
    assert np.max(np.abs(pg - c1["Q"][rows])) <= 10 * 1e-3


def test_postprocess_all_rows_reconstructs_training_data(gpu_lib, c1):
    import torch
    dp = gpu_lib
    n = c1["Q"].shape[0]
    V, pred, info = dp.postprocess(c1["Qd"], c1["Tr"], rows=None, m=n, Qtilde=c1["Qhat"], mean=c1["mean"],
                                   scale=c1["scale"], var_rows=c1["var_rows"])
    torch.cuda.synchronize()
    Vn = V.cpu().numpy()
    # orthonormal basis (Eq. (7)); the rank-10 system plus N(0, 1e-6) noise is
    # reproduced to the noise level
    assert rel(Vn.T @ Vn, np.eye(10)) <= 1e-10
    Q = c1["Q"]
    assert rel(pred.cpu().numpy(), Q) <= 10 * 1e-3 * np.sqrt(Q.size) / np.linalg.norm(Q)
    check_V(Q, c1["mean"].cpu().numpy(), c1["scale"].cpu().numpy(), np.asarray(c1["var_rows"]),
            c1["Tr"].cpu().numpy(), np.arange(n), Vn)


def test_postprocess_f32_ragged_and_unscaled(gpu_lib):
    import torch
    dp = gpu_lib
    rng = np.random.default_rng(9)
    n, k, r = 1000, 77, 20
    Q = rng.normal(size=(n, k)).astype(np.float32)
    Tr = rng.normal(size=(k, r))
    Qt = rng.normal(size=(r, 131))
    rows = np.array([999, 0, 5, 5, 500], dtype=np.int64)
    Qd = torch.from_numpy(Q).cuda()
    V, pred, info = dp.postprocess(Qd, dev(Tr), rows=torch.from_numpy(rows).cuda(), Qtilde=dev(Qt))
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    Q64 = Q.astype(np.float64)
    Vr, pr = orc.postprocess(Q64, np.zeros(n), np.ones(1), [0, n], Tr, rows, Qt)
    check_V(Q64, np.zeros(n), np.ones(1), np.array([0, n]), Tr, rows, V.cpu().numpy())
    assert rel(pred.cpu().numpy(), pr) <= 1e-12


def test_postprocess_bad_row_flags_and_nans(gpu_lib, c1):
    import torch
    dp = gpu_lib
    n = c1["Q"].shape[0]
    rows = torch.tensor([3, n, 7, -1], dtype=torch.int64, device="cuda")
    V, pred, info = dp.postprocess(c1["Qd"], c1["Tr"], rows=rows, Qtilde=c1["Qhat"], mean=c1["mean"],
                                   scale=c1["scale"], var_rows=c1["var_rows"])
    torch.cuda.synchronize()
    assert int(info.item()) == dp.E_ARG
    Vn, pn = V.cpu().numpy(), pred.cpu().numpy()
    assert np.all(np.isnan(Vn[[1, 3]])) and np.all(np.isnan(pn[[1, 3]]))
    assert np.all(np.isfinite(Vn[[0, 2]])) and np.all(np.isfinite(pn[[0, 2]]))


@pytest.mark.parametrize("n,k,r", [(40_001, 130, 60), (32_768, 64, 34)])
def test_postprocess_all_rows_tall_parity(gpu_lib, n, k, r):
    """The basis at all rows of a tall float64 Q (the LDS-DMA form of the
    row product: >= 32,768 rows, 33 <= r <= 64, even k), entry by entry
    against the oracle: a ragged last row tile (40,001 rows), a ragged last
    K stage (k = 130), variable boundaries inside row tiles."""
    import torch
    dp = gpu_lib
    rng = np.random.default_rng(n + k + r)
    Q = rng.standard_normal((n, k)) * rng.uniform(0.5, 2.0, k) + rng.standard_normal((n, 1))
    var_rows = [0, n // 3 + 5, 2 * n // 3 - 7, n]
    Tr = rng.standard_normal((k, r)) / np.sqrt(k)
    Qd = dev(Q)
    mean, scale, _ = dp.preprocess(Qd, var_rows)
    V, _, info = dp.postprocess(Qd, dev(Tr), rows=None, m=n, mean=mean, scale=scale, var_rows=var_rows)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    s_rows = np.repeat(scale.cpu().numpy(), np.diff(var_rows))
    Qs = orc.apply_statistics(Q, mean.cpu().numpy(), s_rows)
    Vref = orc.basis_rows(Qs, Tr, np.arange(n))
    gam = k * U / (1 - k * U)
    bound = 2 * gam * (np.abs(Qs) @ np.abs(Tr)) + 4 * U * np.abs(Vref)
    Vg = V.cpu().numpy()
    assert np.all(np.abs(Vg - Vref) <= bound), float(np.max(np.abs(Vg - Vref) / bound))
