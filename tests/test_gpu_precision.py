"""GPU parity of the reduced-precision Gram forms (float32-stored data).

Reference: the oracle on the same float32 values upcast to float64, so the
comparison isolates the Gram arithmetic.  Tolerances follow from the
arithmetic:
  * FP32 MFMA: each transformed operand is rounded to float32 (relative
    2^-24) and products are summed in float32 over slabs of at most 512 rows
    before a float64 add: relative error <= u32 * (2 + 512) ~ 3e-5 in the
    worst case, ~u32 * (2 + sqrt(512)) ~ 1.5e-6 typically.  Bound used: 3e-5.
  * BF16X3: x = hi + lo + delta with |delta| <= 2^-16 |x|; dropping lo*lo and
    the delta terms leaves <= 3 * 2^-16 ~ 4.6e-5 relative error per product,
    plus the float32 slab accumulation.  Bound used: 2e-4.
  * BF16X6: x = hi + mid + lo + delta with |delta| <= 2^-24 |x|; the dropped
    products (mid*lo, lo*mid, lo*lo and the delta terms) are <= ~4 * 2^-24
    relative, below the float32 slab accumulation: bound as FP32, 3e-5.
"""
import numpy as np
import pytest

import oracle as orc
import synth

pytestmark = pytest.mark.gpu

FP32_TOL = 3e-5
BF16X3_TOL = 2e-4
TOLS = {"native": FP32_TOL, "bf16x3": BF16X3_TOL, "bf16x6": FP32_TOL}


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("n,k,nvars", [(8192, 600, 2), (3001, 130, 3), (777, 64, 1)])
@pytest.mark.parametrize("algo_name", ["native", "bf16x3", "bf16x6"])
def test_lowp_gram_parity(gpu_lib, n, k, nvars, algo_name):
    import torch
    dp = gpu_lib
    algo = {"native": dp.GRAM_NATIVE, "bf16x3": dp.GRAM_BF16X3, "bf16x6": dp.GRAM_BF16X6}[algo_name]
    rng = np.random.default_rng(n + k)
    Q = (rng.standard_normal((n, k)) * np.linspace(0.3, 3.0, k)[None, :] + 0.7).astype(np.float32)
    var_rows = np.linspace(0, n, nvars + 1).astype(np.int64)
    Qd = torch.from_numpy(Q).cuda()
    mean, scale, _ = dp.preprocess(Qd, var_rows)
    D = dp.gram(Qd, mean, scale, var_rows, algo=algo).cpu().numpy()
    _, _, Qs, _ = orc.preprocess(Q.astype(np.float64), var_rows)
    Dref = orc.gram(Qs)
    assert np.array_equal(D, D.T)
    tol = TOLS[algo_name]
    assert rel(D, Dref) <= tol
    # diagonal entries are sums of squares: relative accuracy per entry
    assert np.max(np.abs(np.diag(D) - np.diag(Dref)) / np.diag(Dref)) <= 4 * tol


def test_lowp_gram_deterministic_and_reduced_data(gpu_lib):
    import torch
    dp = gpu_lib
    Q, var_rows, _, _ = synth.c1_snapshots(seed=1)
    Q32 = torch.from_numpy(Q.astype(np.float32)).cuda()
    mean, scale, _ = dp.preprocess(Q32, var_rows)
    for algo, tol in ((dp.GRAM_NATIVE, FP32_TOL), (dp.GRAM_BF16X3, BF16X3_TOL), (dp.GRAM_BF16X6, FP32_TOL)):
        D1 = dp.gram(Q32, mean, scale, var_rows, algo=algo)
        D2 = dp.gram(Q32, mean, scale, var_rows, algo=algo)
        assert torch.equal(D1, D2)
        lam, Tr, Qhat, info, r = dp.reduce(D1, r=10)
        _, _, Qs, _ = orc.preprocess(Q.astype(np.float32).astype(np.float64), var_rows)
        lam_o, U_o = orc.eig_desc(orc.gram(Qs))
        _, Qhat_o = orc.reduce_basis_free(lam_o, U_o, 10)
        l = lam.cpu().numpy()[:10]
        assert np.max(np.abs(l - lam_o[:10]) / lam_o[:10]) <= 10 * tol
        # reduced data: the eigenvector error is the Gram error over the gap
        gap = np.min(np.abs(np.diff(lam_o[:11]))) / lam_o[0]
        assert rel(Qhat.cpu().numpy(), Qhat_o) <= 10 * tol / gap


def test_lowp_rejects_f64_bf16x3(gpu_lib):
    import torch
    dp = gpu_lib
    Q = torch.zeros((16, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(dp.DopinfError):
        dp.gram(Q, algo=dp.GRAM_BF16X3)
