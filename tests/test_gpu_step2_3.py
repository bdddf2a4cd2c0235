"""GPU parity of Steps II and III (centering/scaling, Gram, eigenpairs and
basis-free reduced data) against the CPU oracle, through the C ABI."""
import numpy as np
import pytest

import oracle as orc
import synth

pytestmark = pytest.mark.gpu


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def align_rows(X, ref):
    out = X.copy()
    for j in range(X.shape[0]):
        if np.dot(out[j], ref[j]) < 0:
            out[j] = -out[j]
    return out


@pytest.fixture(scope="module")
def c1():
    Q, var_rows, sysq, V = synth.c1_snapshots(seed=1)
    return Q, var_rows


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def test_preprocess_parity_c1(gpu_lib, c1):
    dp = gpu_lib
    Q, var_rows = c1
    mean, scale, zr = dp.preprocess(dev(Q), var_rows)
    mu, s, Qs, z = orc.preprocess(Q, var_rows)
    assert np.max(np.abs(mean.cpu().numpy() - mu)) <= 1e-15 * max(1.0, np.max(np.abs(mu)))
    assert np.allclose(scale.cpu().numpy(), s, rtol=1e-14, atol=0)
    assert zr.cpu().numpy().tolist() == [0, 0]


def test_preprocess_ragged_padded_f32_apply(gpu_lib):
    import torch
    dp = gpu_lib
    rng = np.random.default_rng(12)
    n, k, ld = 1003, 77, 80
    buf = rng.standard_normal((n, ld)) * 3 + 1.5
    buf[300:310] = 7.0                      # constant rows inside a variable
    var_rows = [0, 300, 310, 1003]          # variable 1 is constant -> zero range
    Qd = dev(buf)[:, :k]
    mean, scale, zr = dp.preprocess(Qd, var_rows, flags=dp.CENTER | dp.SCALE | dp.APPLY)
    mu, s, Qs, z = orc.preprocess(buf[:, :k], var_rows)
    assert zr.cpu().numpy().tolist() == [0, 1, 0]
    assert np.allclose(scale.cpu().numpy(), s, rtol=1e-14)
    assert np.max(np.abs(Qd.cpu().numpy() - Qs)) < 1e-14
    assert np.array_equal(dev(buf).cpu().numpy()[:, k:], buf[:, k:])  # padding untouched
    # float32 storage: statistics accumulate in double
    Q32 = torch.from_numpy(buf[:, :k].astype(np.float32)).cuda()
    m32, s32, _ = dp.preprocess(Q32, var_rows)
    mu32, ss32, _, _ = orc.preprocess(buf[:, :k].astype(np.float32).astype(np.float64), var_rows)
    assert np.max(np.abs(m32.cpu().numpy() - mu32)) < 1e-13
    assert np.allclose(s32.cpu().numpy(), ss32, rtol=1e-13)


def padded_view(A, ld, off):
    """Device view of A (n x m) with row stride ld and a start offset of `off`
    elements inside a NaN-filled flat buffer: odd ld or off = 1 breaks the
    16-byte row alignment."""
    import torch
    n, m = A.shape
    flat = np.full(off + n * ld, np.nan)
    flat[off:].reshape(n, ld)[:, :m] = A
    buf = torch.from_numpy(flat).cuda()
    return buf[off:].view(n, ld)[:, :m]


@pytest.mark.parametrize("ldx,ldy,off", [(132, 72, 0), (131, 70, 0), (132, 72, 1)])
def test_cross_gram_paths_with_statistics(gpu_lib, ldx, ldy, off):
    # even leading dimensions on 16-byte aligned rows take the LDS-DMA kernel,
    # odd ones or an 8-byte offset take the register-staged one; both must match
    # the oracle's centered and scaled product, and NaN padding must not leak
    dp = gpu_lib
    rng = np.random.default_rng(16 + ldx + off)
    n, mx, my = 1037, 131, 70
    var_rows = [0, 400, 1037]
    X = rng.standard_normal((n, mx)) * 3 + 2
    Y = rng.standard_normal((n, my)) * 3 + 2
    Xd = padded_view(X, ldx, off)
    Yd = padded_view(Y, ldy, 0)
    mu, s, Xs, _ = orc.preprocess(X, var_rows)
    Ys = (Y - mu[:, None]).copy()
    Ys[:400] /= s[0]
    Ys[400:] /= s[1]
    mean, scale, _ = dp.preprocess(dev(X), var_rows)
    C = dp.cross_gram(Xd, Yd, mean=mean, scale=scale, var_rows=var_rows).cpu().numpy()
    assert np.all(np.isfinite(C))
    assert rel(C, Xs.T @ Ys) < 1e-12
    C0 = dp.cross_gram(Xd, Yd).cpu().numpy()
    assert rel(C0, X.T @ Y) < 1e-12


@pytest.mark.parametrize("ld,off", [(602, 0), (601, 0), (602, 1)])
def test_gram_paths_nan_padding(gpu_lib, ld, off):
    # symmetric Gram through both kernels, 3 variables, ragged last tile
    dp = gpu_lib
    rng = np.random.default_rng(ld + off)
    n, k = 4099, 600
    var_rows = [0, 1000, 3000, 4099]
    Q = rng.standard_normal((n, k)) * np.linspace(0.5, 2.0, k)[None, :] + 1.5
    Qd = padded_view(Q, ld, off)
    mean, scale, _ = dp.preprocess(dev(Q), var_rows)
    D = dp.gram(Qd, mean, scale, var_rows).cpu().numpy()
    _, _, Qs, _ = orc.preprocess(Q, var_rows)
    assert np.all(np.isfinite(D)) and np.array_equal(D, D.T)
    assert rel(D, orc.gram(Qs)) <= 1e-12


def test_cross_gram_layout_and_ragged_tiles(gpu_lib):
    # X != Y catches any transposition of the matrix-core lane layout
    dp = gpu_lib
    rng = np.random.default_rng(13)
    X = rng.standard_normal((517, 131))
    Y = rng.standard_normal((517, 70))
    Cg = dp.cross_gram(dev(X), dev(Y)).cpu().numpy()
    assert rel(Cg, X.T @ Y) < 1e-13


@pytest.mark.parametrize("n,k,ld,vars_", [(8192, 600, 600, 2), (1003, 77, 80, 3), (257, 129, 130, 1), (64, 1, 1, 1)])
def test_gram_parity(gpu_lib, n, k, ld, vars_):
    dp = gpu_lib
    rng = np.random.default_rng(n + k)
    buf = rng.standard_normal((n, ld)) * np.linspace(0.5, 2.0, ld)[None, :] + 0.25
    var_rows = np.linspace(0, n, vars_ + 1).astype(np.int64)
    Qd = dev(buf)[:, :k]
    mean, scale, _ = dp.preprocess(Qd, var_rows)
    D = dp.gram(Qd, mean, scale, var_rows).cpu().numpy()
    _, _, Qs, _ = orc.preprocess(buf[:, :k], var_rows)
    Dref = orc.gram(Qs)
    assert np.array_equal(D, D.T)
    assert rel(D, Dref) <= 1e-12
    # no transform: plain Q^T Q
    D0 = dp.gram(Qd).cpu().numpy()
    assert rel(D0, orc.gram(buf[:, :k])) <= 1e-12


def test_gram_bitwise_deterministic_and_additive(gpu_lib, c1):
    dp = gpu_lib
    Q, var_rows = c1
    Qd = dev(Q)
    mean, scale, _ = dp.preprocess(Qd, var_rows)
    D1 = dp.gram(Qd, mean, scale, var_rows).cpu().numpy()
    D2 = dp.gram(Qd, mean, scale, var_rows).cpu().numpy()
    assert np.array_equal(D1, D2)
    # Eq. (5): Grams of a row partition add up to the Gram of the whole
    a = 3000
    Dp = dp.gram(Qd[:a]).cpu().numpy() + dp.gram(Qd[a:]).cpu().numpy()
    assert rel(Dp, dp.gram(Qd).cpu().numpy()) < 1e-13


def test_reduce_parity_c1(gpu_lib, c1):
    dp = gpu_lib
    Q, var_rows = c1
    Qd = dev(Q)
    mean, scale, _ = dp.preprocess(Qd, var_rows)
    Dd = dp.gram(Qd, mean, scale, var_rows)
    D = Dd.cpu().numpy()
    lam, Tr, Qhat, info, r = dp.reduce(Dd, r=10)
    assert int(info.item()) == 0 and r == 10
    lam_o, U_o = orc.eig_desc(D)
    Tr_o, Qhat_o = orc.reduce_basis_free(lam_o, U_o, 10)
    lam = lam.cpu().numpy()
    assert np.all(np.diff(lam) <= 0)
    assert np.max(np.abs(lam - lam_o)) <= 1e-13 * lam_o[0]
    assert np.allclose(lam[:10], lam_o[:10], rtol=1e-12)
    assert rel(Qhat.cpu().numpy(), Qhat_o) <= 1e-10          # same sign rule on both sides
    assert rel(Tr.cpu().numpy(), Tr_o) <= 1e-10
    # end-to-end against the oracle's own D
    res = orc.pipeline(Q, var_rows, 10, 1e-6, 1e-4, 20)
    assert rel(D, res["D"]) <= 1e-12
    assert rel(Qhat.cpu().numpy(), res["Qhat"]) <= 1e-10


def test_reduce_invariants_and_energy_rank(gpu_lib):
    dp = gpu_lib
    rng = np.random.default_rng(14)
    n, k = 700, 150
    Q = rng.standard_normal((n, k)) * np.exp(-np.arange(k) / 12.0)[None, :]
    Qd = dev(Q)
    Dd = dp.gram(Qd)
    D = Dd.cpu().numpy()
    lam, Tr, Qhat, info, r = dp.reduce(Dd, r=0, tau=0.999, r_max=k)
    assert int(info.item()) == 0
    lam_o, U_o = orc.eig_desc(D)
    assert r == orc.energy_rank(lam_o, 0.999)
    Qh = Qhat.cpu().numpy()
    assert rel(Qh @ Qh.T, np.diag(lam_o[:r])) < 1e-11
    assert rel(Tr.cpu().numpy().T @ D, Qh) < 1e-10              # Eq. (8)
    Vr = Q @ Tr.cpu().numpy()
    assert rel(Vr.T @ Vr, np.eye(r)) < 1e-10                    # Eq. (7) basis orthonormal
    # thin SVD cross-check
    _, sig, Wt = np.linalg.svd(Q, full_matrices=False)
    ref = sig[:r, None] * Wt[:r]
    assert rel(align_rows(Qh, ref), ref) < 1e-9


def test_reduce_rank_error_flag(gpu_lib):
    dp = gpu_lib
    X = np.zeros((40, 6))
    X[:, 0] = 1.0                   # rank-1 Gram
    lam, Tr, Qhat, info, r = dp.reduce(dp.gram(dev(X)), r=3)
    assert int(info.item()) == dp.E_RANK


def test_cross_gram_with_training_statistics(gpu_lib):
    # held-out snapshots centered / scaled with the training statistics,
    # projected through Eq. (8): Qhat_test = T_r^T (Qs^T Qs_test)
    dp = gpu_lib
    rng = np.random.default_rng(15)
    n, k, kt = 900, 40, 25
    var_rows = [0, 300, 900]
    Q = rng.standard_normal((n, k)) * 2 + 1
    Qt = rng.standard_normal((n, kt)) * 2 + 1
    mu, s, Qs, _ = orc.preprocess(Q, var_rows)
    Qts = (Qt - mu[:, None]).copy()
    Qts[:300] /= s[0]
    Qts[300:] /= s[1]
    mean, scale, _ = dp.preprocess(dev(Q), var_rows)
    C = dp.cross_gram(dev(Q), dev(Qt), mean=mean, scale=scale, var_rows=var_rows).cpu().numpy()
    assert rel(C, Qs.T @ Qts) < 1e-12
    D = dp.gram(dev(Q), mean, scale, var_rows)
    lam, Tr, Qhat, info, r = dp.reduce(D, r=5)
    P = dp.cross_gram(Tr.contiguous(), dev(C)).cpu().numpy()   # T_r^T C
    Vr = Qs @ Tr.cpu().numpy()                                 # explicit basis, for the check only
    assert rel(P, Vr.T @ Qts) < 1e-10
