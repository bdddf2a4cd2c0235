"""Pins of the CPU oracle against facts that do not come from the oracle itself:
closed forms, brute force on tiny inputs, independent library routes (thin SVD,
stacked least squares), values printed in the paper, and invariants.

Each test is chosen so that a plausible slip in the oracle (dropped term, wrong
sign or index, transposed operand, wrong ordering) makes it fail.
"""
import math
import os

import numpy as np
import pytest

import oracle as orc
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ---------------------------------------------------------------- step II ----

def test_stats_closed_form():
    # Q_it = a_i + b_i cos(2 pi t / k): temporal mean a_i; the centered row
    # b_i cos(.) reaches |b_i| at t = 0, so s_v = max_{i in v} |b_i|.
    k = 16
    rng = np.random.default_rng(3)
    a = rng.uniform(-2, 2, 10)
    b = rng.uniform(-3, 3, 10)
    t = np.arange(k)
    Q = a[:, None] + b[:, None] * np.cos(2 * np.pi * t / k)[None, :]
    var_rows = np.array([0, 4, 10])
    mu, s, Qs, zr = orc.preprocess(Q, var_rows)
    assert np.allclose(mu, a, rtol=0, atol=1e-15 * 8)
    assert zr == []
    assert s[0] == pytest.approx(np.max(np.abs(b[:4])), rel=1e-15)
    assert s[1] == pytest.approx(np.max(np.abs(b[4:])), rel=1e-15)
    expect = b[:, None] * np.cos(2 * np.pi * t / k)[None, :]
    expect[:4] /= s[0]
    expect[4:] /= s[1]
    assert np.max(np.abs(Qs - expect)) < 1e-14
    assert np.max(np.abs(Qs)) <= 1.0


def test_stats_zero_range_variable_and_flags():
    Q = np.vstack([np.full((3, 5), 2.5), np.arange(10.0).reshape(2, 5)])
    mu, s, Qs, zr = orc.preprocess(Q, np.array([0, 3, 5]))
    assert zr == [0] and s[0] == 1.0
    assert np.all(Qs[:3] == 0)
    assert s[1] == 2.0  # rows 0..4 and 5..9 centered: max |x - mean| = 2
    mu2, s2, Qs2, _ = orc.preprocess(Q, np.array([0, 3, 5]), center=False, scale=False)
    assert np.all(mu2 == 0) and np.all(s2 == 1) and np.array_equal(Qs2, Q)


# --------------------------------------------------------------- step III ----

def test_gram_invariants_and_row_block_additivity():
    rng = np.random.default_rng(4)
    Q = rng.standard_normal((301, 37))
    D = orc.gram(Q)
    assert np.array_equal(D, D.T)
    assert np.trace(D) == pytest.approx(np.sum(Q * Q), rel=1e-13)
    # Eq. (5): the Gram of a row partition is the sum of the blocks' Grams.
    parts = [Q[:100], Q[100:217], Q[217:]]
    Dsum = sum(orc.gram(P) for P in parts)
    assert rel(Dsum, D) < 1e-14
    perm = rng.permutation(Q.shape[0])
    assert rel(orc.gram(Q[perm]), D) < 1e-14
    lam = np.linalg.eigvalsh(D)
    assert lam.min() >= -1e-13 * lam.max()


def test_gram_brute_force_long_double():
    rng = np.random.default_rng(5)
    Q = rng.standard_normal((9, 5))
    ref = np.zeros((5, 5), dtype=np.longdouble)
    for a in range(5):
        for b in range(5):
            acc = np.longdouble(0)
            for i in range(9):
                acc += np.longdouble(Q[i, a]) * np.longdouble(Q[i, b])
            ref[a, b] = acc
    assert np.max(np.abs(orc.gram(Q) - ref.astype(np.float64))) < 1e-14


def _align_rows(X, ref):
    out = X.copy()
    for j in range(X.shape[0]):
        if np.dot(out[j], ref[j]) < 0:
            out[j] = -out[j]
    return out


def test_eig_and_qhat_match_brute_force_thin_svd():
    # Eqs. (4), (6), (8): eigenvalues of D are the squared singular values of
    # Q and Qhat = Sigma_r W_r^T (right singular vectors, up to sign).
    rng = np.random.default_rng(6)
    n, k, r = 80, 14, 6
    Q = rng.standard_normal((n, k)) * np.exp(-np.arange(k) / 3.0)[None, :]
    _, _, Qs, _ = orc.preprocess(Q, np.array([0, 30, 80]))
    D = orc.gram(Qs)
    lam, U = orc.eig_desc(D)
    _, sig, Wt = np.linalg.svd(Qs, full_matrices=False)
    assert np.allclose(lam, sig ** 2, rtol=1e-12, atol=1e-13 * sig[0] ** 2)
    assert np.all(np.diff(lam) <= 0)
    Tr, Qhat = orc.reduce_basis_free(lam, U, r)
    ref = sig[:r, None] * Wt[:r]
    assert rel(_align_rows(Qhat, ref), ref) < 1e-10
    # invariants: Qhat Qhat^T = Lambda_r, Qhat = T_r^T D, V_r = Q T_r
    # orthonormal with V_r^T Q = Qhat
    assert rel(Qhat @ Qhat.T, np.diag(lam[:r])) < 1e-12
    assert rel(orc.qhat_by_projection(Tr, D), Qhat) < 1e-10
    Vr = Qs @ Tr
    assert rel(Vr.T @ Vr, np.eye(r)) < 1e-10
    assert rel(Vr.T @ Qs, Qhat) < 1e-10


def test_sign_rule():
    U = np.array([[0.1, -0.8], [-0.9, 0.5], [0.3, 0.1]])
    F = orc.fix_signs(U)
    assert np.array_equal(F[:, 0], -U[:, 0])   # largest |.| is -0.9
    assert np.array_equal(F[:, 1], -U[:, 1])   # largest |.| is -0.8
    # exact tie of opposite signs: sum_t (t+1) u_t decides
    T = np.array([[0.6], [0.2], [-0.6]])
    assert orc.fix_signs(T)[0, 0] == -0.6      # 0.6 + 0.4 - 1.8 < 0 -> flip


def test_wave_closed_form_spectrum():
    # noise-free wave generator, scaling off: lambda_i = a^2 sigma_i^2 and
    # Qhat rows = +-a sigma_i psi_i^T (temporal modes have zero mean, so
    # centering changes nothing).
    m = synth.c2_modes(nvars=2, ncell=512, k=64, n_modes=12, n_pairs=3, decay=6.0, seed=11)
    Q = synth.c2_snapshots(m, noise_var=0.0).numpy()
    var_rows = np.array([0, 512, 1024])
    mu, s, Qs, _ = orc.preprocess(Q, var_rows, center=True, scale=False)
    assert np.max(np.abs(mu)) < 1e-12
    lam, U = orc.eig_desc(orc.gram(Qs))
    expect = (m.amp * m.sigma) ** 2
    assert np.allclose(lam[:12], expect, rtol=1e-12)
    assert np.max(np.abs(lam[12:])) < 1e-10 * expect[0]
    r = 12
    _, Qhat = orc.reduce_basis_free(lam, U, r)
    psi = m.temporal(np.arange(64))
    ref = (m.amp * m.sigma)[:, None] * psi.T
    assert rel(_align_rows(Qhat, ref), ref) < 1e-11


def test_energy_rank_strict_threshold():
    lam = np.array([4.0, 3.0, 2.0, 1.0])   # retained energy 0.4 0.7 0.9 1.0
    assert orc.energy_rank(lam, 0.7) == 3  # strict '>' as in the listing
    assert orc.energy_rank(lam, 0.69) == 2
    assert orc.energy_rank(lam, 0.0) == 1


def test_reduce_rejects_nonpositive_lambda():
    with pytest.raises(ValueError):
        orc.reduce_basis_free(np.array([2.0, 0.0]), np.eye(2), 2)


def test_reduce_rank_threshold_is_rounding_level_of_the_spectrum():
    # the threshold is k u lambda_1 with u = 2^-52: at it, rejected; above, kept
    k = 3
    thr = k * 2.0 ** -52
    with pytest.raises(ValueError):
        orc.reduce_basis_free(np.array([1.0, thr, 0.0]), np.eye(3), 2)
    Tr, Qh = orc.reduce_basis_free(np.array([1.0, 1.5 * thr, 0.0]), np.eye(3), 2)
    assert Qh.shape == (2, 3)
    # an exactly rank-2 Q: the third eigenvalue of D = Q^T Q is zero in exact
    # arithmetic and rounding-level in float64, so r = 3 must be refused
    # (a test of lambda_r > 0 alone would accept it about half the time)
    rng = np.random.default_rng(12)
    Q = rng.standard_normal((40, 2)) @ rng.standard_normal((2, 5))
    lam, U = orc.eig_desc(orc.gram(Q))
    assert abs(lam[2]) <= 5 * 2.0 ** -52 * lam[0]
    orc.reduce_basis_free(lam, U, 2)
    with pytest.raises(ValueError):
        orc.reduce_basis_free(lam, U, 3)


# ---------------------------------------------------------------- step IV ----

def test_quad_features_are_kron_subset():
    rng = np.random.default_rng(7)
    X = rng.standard_normal((5, 4))
    F = orc.quad_features(X)
    cols = [i * 4 + j for i in range(4) for j in range(i, 4)]
    K = np.stack([np.kron(x, x) for x in X])
    assert np.array_equal(F, K[:, cols])
    assert orc.quad_pairs(3) == [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]


def test_regularizer_layout():
    g = orc.regularizer(2, 1e-3, 5.0)
    assert list(g) == [1e-3, 1e-3, 5.0, 5.0, 5.0, 1e-3]


def _nonredundant(H, r):
    """r x r^2 Kronecker-form operator -> r x s form acting on quad_features."""
    cols = []
    for i in range(r):
        for j in range(i, r):
            cols.append(H[:, i * r + j] + (H[:, j * r + i] if j != i else 0.0))
    return np.stack(cols, axis=1)


def test_exact_recovery_of_known_quadratic_rom():
    # Trajectory of a known q+ = A q + H(q kron q) + c used as Qhat: at beta = 0
    # the OpInf normal equations return exactly (A, H in non-redundant form, c).
    # The tolerance follows from kappa(G) ~ 1e11 for this trajectory (u * kappa
    # ~ 1e-5 at worst); a wrong column order or sign gives O(1) errors.
    sysq = synth.c1_system(seed=21, r=3, k=20, rho=0.9, h_fro=0.2, c_var=1e-2)
    Qhat = sysq.q
    _, G, B = orc.opinf_data(Qhat)
    O = orc.solve_operators(G, B, 3, 0.0, 0.0)
    A, H, c = orc.split_operators(O, 3)
    assert np.max(np.abs(A - sysq.A)) < 1e-6
    assert np.max(np.abs(H - _nonredundant(sysq.H, 3))) < 1e-6
    assert np.max(np.abs(c - sysq.c)) < 1e-6
    # and the inferred ROM reproduces the data
    Qt = orc.rollout(O, 3, Qhat[:, 0], Qhat.shape[1])
    assert orc.train_error(Qt, Qhat, Qhat.shape[1]) < 1e-8


def test_regularized_solution_matches_stacked_least_squares():
    # Eq. (12) minimizer via an independent route: ordinary least squares on
    # [Dhat; sqrt(Gamma)] with right-hand side [Qhat_2^T; 0].
    rng = np.random.default_rng(8)
    r, k = 3, 40
    Qhat = rng.standard_normal((r, k))
    Dhat, G, B = orc.opinf_data(Qhat)
    b1, b2 = 0.3, 2.0
    O = orc.solve_operators(G, B, r, b1, b2)
    gam = orc.regularizer(r, b1, b2)
    S = np.vstack([Dhat, np.diag(np.sqrt(gam))])
    R = np.vstack([Qhat[:, 1:].T, np.zeros((Dhat.shape[1], r))])
    X, *_ = np.linalg.lstsq(S, R, rcond=None)
    assert rel(O, X.T) < 1e-11
    assert rel(orc.solve_operators(G, B, r, b1, b2, method="cholesky"), O) < 1e-12


def test_rollout_hand_computed():
    # r = 1: q+ = 0.5 q + 0.25 q^2 + 0.1
    O = np.array([[0.5, 0.25, 0.1]])
    Qt = orc.rollout(O, 1, np.array([2.0]), 3)
    assert Qt[0, 1] == pytest.approx(2.1, abs=1e-15)
    assert Qt[0, 2] == pytest.approx(1.05 + 0.25 * 2.1 ** 2 + 0.1, abs=1e-15)
    # r = 2, columns [A | H(0,0) H(0,1) H(1,1) | c]
    O2 = np.array([[0.5, 0.0, 1.0, 0.0, 0.0, 0.0],
                   [0.0, 0.25, 0.0, 2.0, 0.0, 1.0]])
    Qt2 = orc.rollout(O2, 2, np.array([1.0, 2.0]), 2)
    assert np.array_equal(Qt2[:, 1], [1.5, 5.5])


def test_train_error_and_growth_crafted():
    Qhat = np.array([[1.0, -1.0, 1.0, -1.0]])
    Qt = np.array([[1.0, -1.0, 1.0, -1.0, 3.0, 0.0]])
    assert orc.train_error(Qt, Qhat, 4) == 0.0
    assert orc.growth_ratio(Qt, Qhat) == 3.0
    assert orc.train_error(2 * Qhat, Qhat, 4) == 1.0
    Qh2 = np.array([[3.0, 0.0], [4.0, 5.0]])
    Qt2 = np.array([[3.0, 0.0], [4.0, 4.0]])
    assert orc.train_error(Qt2, Qh2, 2) == pytest.approx(0.2, abs=1e-16)
    fin, te, g, ok = orc.score(np.array([[1.0, np.inf]]), Qhat, 1, 1.2)
    assert not fin and not ok
    _, _, g, ok = orc.score(np.array([[1.0, -1.0, 1.19]]), Qhat, 2, 1.2)
    assert ok and g == pytest.approx(1.19)
    _, _, g, ok = orc.score(np.array([[1.0, -1.0, 1.2]]), Qhat, 2, 1.2)
    assert not ok   # strictly below the bound


def test_selection_brute_force_and_ties():
    errs = [0.5, 0.2, 0.2, 0.1, 0.3, 0.05, 0.2, 0.4, 0.9]
    passed = [True, True, True, False, True, False, True, True, True]
    assert orc.select_best(errs, passed) == 1   # first of the tied 0.2
    assert orc.select_best(errs, [False] * 9) == -1


def test_logspace_grid_reproduces_printed_optimum():
    vals = {}
    grids = {}
    with open(os.path.join(GOLDEN, "beta_star.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, *rest = line.split()
            if key.startswith("grid"):
                grids[key] = tuple(float(x) for x in rest)
            else:
                vals[key] = float(rest[0])
    lo, hi, num = grids["grid_beta1"]
    B1 = synth.logspace_points(lo, hi, int(num))
    lo, hi, num = grids["grid_beta2"]
    B2 = synth.logspace_points(lo, hi, int(num))
    trunc = lambda x: math.floor(x / 10 ** math.floor(math.log10(x)) * 100) / 100
    assert any(trunc(b) == trunc(vals["beta1_star"]) and abs(math.log10(b / vals["beta1_star"])) < 2e-3 for b in B1)
    assert any(trunc(b) == trunc(vals["beta2_star"]) and abs(math.log10(b / vals["beta2_star"])) < 2e-3 for b in B2)
    assert B1[0] == 1e-10 and B1[-1] == 1.0 and B2[0] == 1e-4 and B2[-1] == 1e4


def test_sweep_order_is_beta1_outer():
    rng = np.random.default_rng(9)
    Qhat = rng.standard_normal((3, 30)) * 0.1
    out = orc.sweep(Qhat, [2, 3], [1e-3, 1e-1], [1e-2, 1.0], 40)
    assert out["r"] == [2, 2, 2, 2, 3, 3, 3, 3]
    assert out["beta1"][:4] == [1e-3, 1e-3, 1e-1, 1e-1]
    assert out["beta2"][:4] == [1e-2, 1.0, 1e-2, 1.0]
    assert len(out["best"]) == 2


def test_full_chain_recovers_lifted_system():
    # Lifted, noise-free, uncentered, unscaled: Qhat = P q with P orthogonal,
    # so the inferred ROM reproduces Qhat over the training window.
    sysq = synth.c1_system(seed=31, r=4, k=80, rho=0.9, h_fro=0.1, c_var=1e-2)
    Q, var_rows, _, V = synth.c1_snapshots(seed=31, n_per_var=32, nvars=2, r=4, k=80,
                                           noise_var=0.0, system=sysq)
    res = orc.pipeline(Q, var_rows, 4, 0.0, 0.0, 80, center=False, scale=False)
    assert res["train_err"] < 1e-7
    P = res["Qhat"] @ np.linalg.pinv(sysq.q)
    assert rel(P.T @ P, np.eye(4)) < 1e-9


# -------------------------------------------------------------- generators ---

def test_generators_deterministic_and_structured():
    s1 = synth.c1_system(seed=1)
    s2 = synth.c1_system(seed=1)
    assert np.array_equal(s1.q, s2.q)
    assert max(abs(np.linalg.eigvals(s1.A))) == pytest.approx(0.98, rel=1e-12)
    assert np.linalg.norm(s1.H) == pytest.approx(0.05, rel=1e-12)
    x = np.random.default_rng(0).standard_normal(10)
    assert abs(x @ (s1.H @ np.kron(x, x))) < 1e-14   # energy preserving
    assert np.max(np.abs(s1.q)) <= 10.0
    m = synth.c2_modes(nvars=2, ncell=256, k=32, n_modes=8, n_pairs=2, seed=3)
    a = synth.c2_snapshots(m, seed=5).numpy()
    b = synth.c2_snapshots(m, seed=5).numpy()
    assert np.array_equal(a, b)
    phi = m.spatial(np.arange(m.n))
    psi = m.temporal(np.arange(m.k))
    assert rel(phi.T @ phi, np.eye(8)) < 1e-12
    assert rel(psi.T @ psi, np.eye(8)) < 1e-12
    assert np.max(np.abs(psi.sum(axis=0))) < 1e-12
