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
  * I8X6: column j is scaled by 127 / a_j (a_j = max_i |x_ij|) and split as
    xs = t1 + t2 / 254 + t3 / 254^2 + d with |t| <= 127, |d| <= 0.5 / 254^2;
    so |t2 / 254| <= 0.5 and |t3 / 254^2| <= 127 / 254^2.  The dropped
    products (t2 t3, t3 t2, t3 t3) are <= 1.973e-3 and the d terms
    <= 2 * 127.5 * 0.5 / 254^2 = 1.976e-3 in units of a_i a_j / 127^2, and the
    kept ones are summed exactly in int32: per entry
    |dD_jl| <= n * 3.95e-3 / 127^2 * a_j a_l = n * 2.45e-7 * a_j a_l (plus
    float64 rounding).  Bound used: n * 2.5e-7 * a_j a_l.  A dropped product
    level or a wrong slice weight errs by >= ~1e-5 a_j a_l per row.
"""
import numpy as np
import pytest

import oracle as orc
import synth
from lowp_emu import i8_emulate

pytestmark = pytest.mark.gpu

FP32_TOL = 3e-5
BF16X3_TOL = 2e-4
I8_ROW = 2.5e-7
TOLS = {"native": FP32_TOL, "bf16x3": BF16X3_TOL, "bf16x6": FP32_TOL}
ALGOS = {"native": 0, "bf16x3": 1, "bf16x6": 2, "i8x6": 3}


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def i8_excess(D, Dref, Qs):
    """max over entries of |D - Dref| / (n a_j a_l): at most I8_ROW."""
    a = np.max(np.abs(Qs), axis=0)
    den = Qs.shape[0] * np.outer(a, a)
    return float(np.max(np.abs(D - Dref) / np.where(den > 0, den, 1.0)))


@pytest.mark.parametrize("n,k,nvars", [(8192, 600, 2), (3001, 130, 3), (777, 64, 1)])
@pytest.mark.parametrize("algo_name", ["native", "bf16x3", "bf16x6", "i8x6"])
def test_lowp_gram_parity(gpu_lib, n, k, nvars, algo_name):
    import torch
    dp = gpu_lib
    algo = ALGOS[algo_name]
    rng = np.random.default_rng(n + k)
    Q = (rng.standard_normal((n, k)) * np.linspace(0.3, 3.0, k)[None, :] + 0.7).astype(np.float32)
    var_rows = np.linspace(0, n, nvars + 1).astype(np.int64)
    Qd = torch.from_numpy(Q).cuda()
    mean, scale, _ = dp.preprocess(Qd, var_rows)
    D = dp.gram(Qd, mean, scale, var_rows, algo=algo).cpu().numpy()
    _, _, Qs, _ = orc.preprocess(Q.astype(np.float64), var_rows)
    Dref = orc.gram(Qs)
    assert np.array_equal(D, D.T)
    if algo_name == "i8x6":
        assert i8_excess(D, Dref, Qs) <= I8_ROW
        return
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
    Qs = orc.preprocess(Q.astype(np.float32).astype(np.float64), var_rows)[2]
    a = np.max(np.abs(Qs), axis=0)
    # I8X6 as a relative Frobenius bound: ||dD||_F <= n 2.5e-7 ||a||^2
    i8_tol = Qs.shape[0] * I8_ROW * float(a @ a) / np.linalg.norm(orc.gram(Qs))
    for algo, tol in ((dp.GRAM_NATIVE, FP32_TOL), (dp.GRAM_BF16X3, BF16X3_TOL), (dp.GRAM_BF16X6, FP32_TOL),
                      (dp.GRAM_I8X6, i8_tol)):
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


@pytest.mark.parametrize("n,k,nvars", [(3001, 130, 3), (8192, 257, 2), (50, 20, 1)])
def test_i8x6_matches_its_arithmetic(gpu_lib, n, k, nvars):
    """I8X6 against the CPU emulation of its own arithmetic (same slices, the
    kept products summed exactly): only the float64 combination of the
    levels and the order of the split sums differ, so the entries agree to
    1e-13 of n a_j a_l.  Ragged n (not a multiple of the 64-row block) and k
    (not a multiple of the 128-column tile)."""
    import torch
    dp = gpu_lib
    rng = np.random.default_rng(7 * n + k)
    Q = (rng.standard_normal((n, k)) * np.geomspace(0.01, 10.0, k)[None, :] + 0.3).astype(np.float32)
    var_rows = np.linspace(0, n, nvars + 1).astype(np.int64)
    Qd = torch.from_numpy(Q).cuda()
    mean, scale, _ = dp.preprocess(Qd, var_rows)
    D = dp.gram(Qd, mean, scale, var_rows, algo=dp.GRAM_I8X6).cpu().numpy()
    De, x = i8_emulate(Q, mean.cpu().numpy(), scale.cpu().numpy(), var_rows)
    a = np.max(np.abs(x), axis=0)
    den = n * np.outer(a, a)
    assert np.max(np.abs(D - De) / den) <= 1e-13
    # and the derived bound against the oracle (columns of very different
    # magnitudes: the per-column scaling keeps the small ones accurate)
    _, _, Qs, _ = orc.preprocess(Q.astype(np.float64), var_rows)
    assert i8_excess(D, orc.gram(Qs), Qs) <= I8_ROW


def test_i8x6_nonfinite_column(gpu_lib):
    """A non-finite value makes its column's row and column of D NaN and
    leaves the other entries as without it (no centering or scaling, so the
    other columns' statistics are unchanged)."""
    import torch
    dp = gpu_lib
    rng = np.random.default_rng(5)
    Q = rng.standard_normal((700, 40)).astype(np.float32)
    D0 = dp.gram(torch.from_numpy(Q).cuda(), algo=dp.GRAM_I8X6).cpu().numpy()
    for bad in (np.nan, np.inf):
        Qb = Q.copy()
        Qb[123, 7] = bad
        D = dp.gram(torch.from_numpy(Qb).cuda(), algo=dp.GRAM_I8X6).cpu().numpy()
        assert np.all(np.isnan(D[7, :])) and np.all(np.isnan(D[:, 7]))
        keep = np.arange(40) != 7
        # row 123 of the other columns is unchanged, so are their entries
        assert np.array_equal(D[np.ix_(keep, keep)], D0[np.ix_(keep, keep)])


def test_i8x6_degenerate_shapes(gpu_lib):
    """One row, one column, and an all-zero column (a_j = 0: its slices are
    zero and its entries of D exactly 0, not NaN); each against the
    emulation of the form's arithmetic."""
    import torch
    dp = gpu_lib
    rng = np.random.default_rng(17)
    cases = [rng.standard_normal((1, 7)), rng.standard_normal((300, 1)), rng.standard_normal((129, 33))]
    cases[2][:, 5] = 0.0
    for Q in cases:
        Q = Q.astype(np.float32)
        n, k = Q.shape
        D = dp.gram(torch.from_numpy(Q).cuda(), algo=dp.GRAM_I8X6).cpu().numpy()
        De, x = i8_emulate(Q, np.zeros(n), np.ones(1), [0, n])
        a = np.max(np.abs(x), axis=0)
        assert np.all(np.isfinite(D))
        assert np.max(np.abs(D - De) / np.maximum(n * np.outer(a, a), 1e-300)) <= 1e-13
        if k == 33:
            assert np.all(D[5, :] == 0.0) and np.all(D[:, 5] == 0.0)
        Dref = orc.gram(Q.astype(np.float64))
        assert i8_excess(D, Dref, Q.astype(np.float64)) <= I8_ROW
