"""GPU parity of Step IV (regularized operator inference, rollouts, scoring
and selection) against the CPU oracle, through the C ABI.

Operator checks (tests/opcheck.py): the backward error on the oracle's own
normal equations, the forward error against the oracle's LU solution within
the first-order perturbation bound, and the solver alone on the G and B the
GPU forms itself, within ten times the oracle's own LU-vs-Cholesky spread.
"""
import numpy as np
import pytest

import oracle as orc
import synth

pytestmark = pytest.mark.gpu


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


from opcheck import U, check_operators as _check_ops, check_solver_only, gpu_normal_equations, \
    normal_equations_at


def check_operators(G, B, r, b1, b2, O_gpu, where=None, k=None):
    _check_ops(G, B, r, b1, b2, O_gpu, k, where)


@pytest.fixture(scope="module")
def c1_qhat(gpu_lib):
    dp = gpu_lib
    Q, var_rows, sysq, V = synth.c1_snapshots(seed=1)
    Qd = dev(Q)
    mean, scale, _ = dp.preprocess(Qd, var_rows)
    D = dp.gram(Qd, mean, scale, var_rows)
    lam, Tr, Qhat, info, r = dp.reduce(D, r=10)
    assert int(info.item()) == 0
    return Qhat.contiguous(), Q, var_rows


def test_infer_single_pair_c1(gpu_lib, c1_qhat):
    dp = gpu_lib
    Qhat, Q, var_rows = c1_qhat
    O, status, views = dp.infer(Qhat, [10], [1e-6], [1e-4])
    assert status.cpu().numpy().tolist() == [0]
    Qh = Qhat.cpu().numpy()
    _, G, B = orc.opinf_data(Qh)
    check_operators(G, B, 10, 1e-6, 1e-4, views[0][0].cpu().numpy(), k=Qh.shape[1])
    # the solver alone, on the G and B that the GPU forms itself
    GE = gpu_normal_equations(dp, Qh, 10)
    Gg, Bg = normal_equations_at(GE, 10, 10)
    check_solver_only(Gg, Bg, 10, 1e-6, 1e-4, views[0][0].cpu().numpy(), "C1 (1e-6, 1e-4)")


def test_infer_grid_of_sizes_and_pairs(gpu_lib, c1_qhat):
    dp = gpu_lib
    Qhat, _, _ = c1_qhat
    Qh = Qhat.cpu().numpy()
    r_list = [3, 6, 10]
    b1 = [1e-8, 1e-8, 1e-4, 1e-4, 1e-2, 1e-2]
    b2 = [1e-6, 1e-1, 1e-6, 1e-1, 1e-6, 1e-1]
    O, status, views = dp.infer(Qhat, r_list, b1, b2)
    assert np.all(status.cpu().numpy() == 0)
    GE = gpu_normal_equations(dp, Qh, max(r_list))
    for g, r in enumerate(r_list):
        _, G, B = orc.opinf_data(Qh[:r])
        Gg, Bg = normal_equations_at(GE, r, max(r_list))
        for p in range(len(b1)):
            check_operators(G, B, r, b1[p], b2[p], views[g][p].cpu().numpy(), (r, p), k=Qh.shape[1])
            check_solver_only(Gg, Bg, r, b1[p], b2[p], views[g][p].cpu().numpy(), (r, b1[p], b2[p]))


def test_infer_exact_recovery(gpu_lib):
    # a known quadratic ROM's own trajectory as reduced data: at beta = 0 the
    # operators are recovered (up to u * kappa(G), kappa ~ 1e11 here)
    dp = gpu_lib
    sysq = synth.c1_system(seed=21, r=3, k=20, rho=0.9, h_fro=0.2, c_var=1e-2)
    O, status, views = dp.infer(dev(sysq.q), [3], [0.0], [0.0])
    assert int(status.item()) == 0
    A, H, c = orc.split_operators(views[0][0].cpu().numpy(), 3)
    Hn = np.stack([sysq.H[:, i * 3 + j] + (sysq.H[:, j * 3 + i] if j != i else 0.0)
                   for i in range(3) for j in range(i, 3)], axis=1)
    assert np.max(np.abs(A - sysq.A)) < 1e-6
    assert np.max(np.abs(H - Hn)) < 1e-6
    assert np.max(np.abs(c - sysq.c)) < 1e-6


def test_infer_reports_breakdown(gpu_lib):
    dp = gpu_lib
    rng = np.random.default_rng(3)
    Qh = rng.standard_normal((3, 50))
    Qh[1] = 0.0          # a mode that is identically zero: singular normal matrix at beta = 0
    O, status, _ = dp.infer(dev(Qh), [3], [0.0, 1e-3], [0.0, 1e-3])
    assert status.cpu().numpy().tolist() == [dp.E_NOTSPD, 0]


@pytest.mark.parametrize("one_wg", [False, True])
def test_rollout_parity_given_operators(one_wg, gpu_lib, c1_qhat):
    dp = gpu_lib
    Qhat, _, _ = c1_qhat
    Qh = Qhat.cpu().numpy()
    r_list = [4, 10]
    b1 = [1e-6, 1e-2]
    b2 = [1e-4, 1e-1]
    O, status, views = dp.infer(Qhat, r_list, b1, b2)
    n_states = 1200
    out = dp.rollout(O, Qhat, r_list, 2, n_states, max_growth=1.2, solve_status=status, keep_traj=True, full=True, one_wg=one_wg)
    te = out["train_err"].cpu().numpy()
    gr = out["growth"].cpu().numpy()
    oc = out["outcome"].cpu().numpy()
    for g, r in enumerate(r_list):
        for p in range(2):
            Og = views[g][p].cpu().numpy()
            Qt = orc.rollout(Og, r, Qh[:r, 0], n_states)
            fin, e, gg, ok = orc.score(Qt, Qh[:r], Qh.shape[1], 1.2)
            it = g * 2 + p
            traj = out["traj_views"][g][p].cpu().numpy().T
            if fin:
                scale = np.max(np.abs(Qt))
                assert np.max(np.abs(traj - Qt)) <= 1e-9 * scale, (r, p)
                assert te[it] == pytest.approx(e, rel=1e-8, abs=1e-14)
                assert gr[it] == pytest.approx(gg, rel=1e-10)
                assert (oc[it] == dp.ITEM_PASS) == ok
            else:
                assert oc[it] == dp.ITEM_NONFINITE
    best = out["best"].cpu().numpy()
    for g, r in enumerate(r_list):
        cand = [(te[g * 2 + p], g * 2 + p) for p in range(2) if oc[g * 2 + p] == dp.ITEM_PASS]
        assert best[g] == (min(cand)[1] if cand else -1)


@pytest.mark.parametrize("one_wg", [False, True])
def test_rollout_from_given_initial_states(one_wg, gpu_lib, c1_qhat):
    # q0 per item (packed in item order): each rollout starts from its own
    # state, a perturbation of the first snapshot, and is scored against
    # the training data as before
    import torch
    dp = gpu_lib
    Qhat, _, _ = c1_qhat
    Qh = Qhat.cpu().numpy()
    r_list = [4, 10]
    b1 = [1e-2, 1e-2, 1e-3]
    b2 = [1e-1, 1.0, 1e-1]
    n_pairs = len(b1)
    O, status, views = dp.infer(Qhat, r_list, b1, b2)
    rng = np.random.default_rng(17)
    q0s = []
    for g, r in enumerate(r_list):
        for p in range(n_pairs):
            q0s.append(Qh[:r, 0] * (1.0 + 0.01 * rng.standard_normal(r)))
    q0 = torch.from_numpy(np.concatenate(q0s)).cuda()
    n_states = 900
    out = dp.rollout(O, Qhat, r_list, n_pairs, n_states, solve_status=status, keep_traj=True, full=True,
                     one_wg=one_wg, q0=q0)
    te, gr, oc = (out[k].cpu().numpy() for k in ("train_err", "growth", "outcome"))
    for g, r in enumerate(r_list):
        for p in range(n_pairs):
            it = g * n_pairs + p
            Qt = orc.rollout(views[g][p].cpu().numpy(), r, q0s[it], n_states)
            fin, e, gg, ok = orc.score(Qt, Qh[:r], Qh.shape[1], 1.2)
            traj = out["traj_views"][g][p].cpu().numpy().T
            assert np.array_equal(traj[:, 0], q0s[it])
            if fin:
                assert np.max(np.abs(traj - Qt)) <= 1e-9 * np.max(np.abs(Qt)), (r, p)
                assert te[it] == pytest.approx(e, rel=1e-8, abs=1e-14)
                assert gr[it] == pytest.approx(gg, rel=1e-10)
                assert (oc[it] == dp.ITEM_PASS) == ok
            else:
                assert oc[it] == dp.ITEM_NONFINITE
    with pytest.raises(ValueError):
        dp.rollout(O, Qhat, r_list, n_pairs, n_states, q0=q0[:-1].contiguous())


@pytest.mark.parametrize("one_wg", [False, True])
def test_rollout_hand_cases_and_failure_modes(one_wg, gpu_lib):
    import torch
    dp = gpu_lib
    # r = 1: q+ = 0.5 q + 0.25 q^2 + 0.1 from q0 = 2; second item unstable (q+ = 2 q)
    O = torch.tensor([0.5, 0.25, 0.1, 2.0, 0.0, 0.0], dtype=torch.float64, device="cuda")
    Qhat = torch.tensor([[2.0, 2.1, 2.2525, 2.0]], dtype=torch.float64, device="cuda")
    out = dp.rollout(O, Qhat, [1], 2, 3, max_growth=1.2, keep_traj=True, full=True, one_wg=one_wg)
    tr = out["traj_views"][0][0].cpu().numpy()[:, 0]
    assert tr[1] == pytest.approx(2.1, abs=1e-15)
    assert tr[2] == pytest.approx(1.05 + 0.25 * 2.1 ** 2 + 0.1, abs=1e-15)
    assert out["outcome"].cpu().numpy().tolist()[1] == dp.ITEM_GROWTH
    # early exit decides the same outcome and marks the unrun states NaN
    out2 = dp.rollout(O, Qhat, [1], 2, 50, max_growth=1.2, keep_traj=True, one_wg=one_wg)
    assert out2["outcome"].cpu().numpy().tolist()[1] == dp.ITEM_GROWTH
    assert np.isnan(out2["traj_views"][0][1].cpu().numpy()[-1, 0])
    # r = 2 hand case: columns [A | H(0,0) H(0,1) H(1,1) | c]
    O2 = torch.tensor([[0.5, 0.0, 1.0, 0.0, 0.0, 0.0], [0.0, 0.25, 0.0, 2.0, 0.0, 1.0]],
                      dtype=torch.float64, device="cuda").reshape(-1)
    Qh2 = torch.tensor([[1.0, 1.5], [2.0, 5.5]], dtype=torch.float64, device="cuda")
    o2 = dp.rollout(O2, Qh2, [2], 1, 2, keep_traj=True, full=True, one_wg=one_wg)
    assert np.array_equal(o2["traj_views"][0][0].cpu().numpy()[1], [1.5, 5.5])
    assert o2["train_err"].item() == 0.0
    # a non-finite rollout
    O3 = torch.tensor([1e200, 1e200, 0.0], dtype=torch.float64, device="cuda")
    o3 = dp.rollout(O3, Qhat, [1], 1, 10, full=True, one_wg=one_wg)
    assert o3["outcome"].item() == dp.ITEM_NONFINITE
    assert o3["best"].item() == -1


def _stable_rom(r, k, seed):
    rng = np.random.default_rng(seed)
    s = r * (r + 1) // 2
    A = np.diag(rng.uniform(0.90, 0.99, r)) + 1e-3 * rng.standard_normal((r, r))
    H = 1e-4 * rng.standard_normal((r, s))
    c = 1e-3 * rng.standard_normal(r)
    Og = np.hstack([A, H, c[:, None]])
    q0 = rng.standard_normal(r)
    Qh = orc.rollout(Og, r, q0, k) + 1e-3 * rng.standard_normal((r, k))
    Qh[:, 0] = q0
    return Og, Qh


@pytest.mark.parametrize("one_wg", [False, True])
def test_selection_ties_pick_first(one_wg, gpu_lib):
    # three identical stable ROMs: equal training errors, all pass, the first
    # wins; with the first made unstable (growth failure) the second wins
    import torch
    dp = gpu_lib
    r, k = 5, 300
    Og, Qh = _stable_rom(r, k, 17)
    Qhat = torch.from_numpy(Qh.copy()).cuda()
    O = torch.from_numpy(np.concatenate([Og.ravel()] * 3)).cuda()
    out = dp.rollout(O, Qhat, [r], 3, 600, one_wg=one_wg)
    te = out["train_err"].cpu().numpy()
    assert te[0] == te[1] == te[2]
    assert out["outcome"].cpu().numpy().tolist() == [dp.ITEM_PASS] * 3
    assert out["best"].item() == 0
    Ou = Og.copy()
    Ou[:, :r] *= 1.5
    O = torch.from_numpy(np.concatenate([Ou.ravel(), Og.ravel(), Og.ravel()])).cuda()
    out = dp.rollout(O, Qhat, [r], 3, 600, one_wg=one_wg)
    oc = out["outcome"].cpu().numpy().tolist()
    assert oc[0] in (dp.ITEM_GROWTH, dp.ITEM_NONFINITE) and oc[1:] == [dp.ITEM_PASS] * 2
    assert out["best"].item() == 1


@pytest.mark.parametrize("one_wg", [False, True])
def test_small_sweep_matches_oracle(one_wg, gpu_lib, c1_qhat):
    dp = gpu_lib
    Qhat, _, _ = c1_qhat
    Qh = Qhat.cpu().numpy()
    B1 = synth.logspace_points(-10, 0, 4)
    B2 = synth.logspace_points(-4, 4, 4)
    b1 = [x for x in B1 for _ in B2]
    b2 = [y for _ in B1 for y in B2]
    r_list = [4, 8]
    O, status, views = dp.infer(Qhat, r_list, b1, b2)
    out = dp.rollout(O, Qhat, r_list, len(b1), 1200, solve_status=status, one_wg=one_wg)
    ref = orc.sweep(Qh, r_list, list(B1), list(B2), 1200)
    te = out["train_err"].cpu().numpy()
    gr = out["growth"].cpu().numpy()
    oc = out["outcome"].cpu().numpy()
    st = status.cpu().numpy()
    npair = len(b1)
    for it in range(len(ref["r"])):
        r = ref["r"][it]
        if st[it] != 0:
            # a refused normal matrix is singular to working precision
            _, G, B = orc.opinf_data(Qh[:r])
            M = G + np.diag(orc.regularizer(r, ref["beta1"][it], ref["beta2"][it]))
            assert oc[it] == dp.ITEM_SOLVE
            try:
                L = np.linalg.cholesky(M)
                assert np.min(np.diag(L)) ** 2 / np.max(np.diag(M)) < 1e-10, it
            except np.linalg.LinAlgError:
                pass
        elif ref["passed"][it]:
            assert oc[it] == dp.ITEM_PASS or abs(ref["growth"][it] - 1.2) < 1e-6
            assert te[it] == pytest.approx(ref["train_err"][it], rel=1e-6)
        elif not ref["finite"][it]:
            # the oracle's rollout overflows: the GPU's either does too or
            # stops earlier at the (final) growth failure
            assert oc[it] in (dp.ITEM_NONFINITE, dp.ITEM_GROWTH), it
        else:
            # finite but over the growth bound (unless within rounding of it)
            assert oc[it] == dp.ITEM_GROWTH or abs(ref["growth"][it] - 1.2) < 1e-6, it
            assert gr[it] >= 1.2 or abs(ref["growth"][it] - 1.2) < 1e-6, it
    best = out["best"].cpu().numpy()
    for g in range(len(r_list)):
        rb = ref["best"][g]
        if rb < 0:
            assert best[g] == -1
        else:
            gi = best[g]
            # a different pick is only allowed between near-ties
            assert abs(te[gi] - ref["train_err"][g * len(b1) + rb]) <= 1e-6 * ref["train_err"][g * len(b1) + rb]


@pytest.mark.parametrize("r", [20, 60])
def test_team_rollout_partial_member_matches_oracle(gpu_lib, r):
    # r = 20 and 60 leave the last team member with 4 of its 8 rows
    import torch
    dp = gpu_lib
    rng = np.random.default_rng(r)
    k = 300
    # a stable linear-dominant ROM with small quadratic terms, from the oracle's layout
    s = r * (r + 1) // 2
    A = np.diag(rng.uniform(0.90, 0.99, r)) + 1e-3 * rng.standard_normal((r, r))
    H = 1e-4 * rng.standard_normal((r, s))
    c = 1e-3 * rng.standard_normal(r)
    Og = np.hstack([A, H, c[:, None]])
    q0 = rng.standard_normal(r)
    Qh = orc.rollout(Og, r, q0, k) + 1e-3 * rng.standard_normal((r, k))
    Qh[:, 0] = q0
    O = torch.from_numpy(Og.ravel().copy()).cuda()
    Qhat = torch.from_numpy(Qh.copy()).cuda()
    n_states = 700
    Qt = orc.rollout(Og, r, q0, n_states)
    fin, e, gg, ok = orc.score(Qt, Qh, k, 1.2)
    outs = [dp.rollout(O, Qhat, [r], 1, n_states, keep_traj=True, full=True, one_wg=f) for f in (False, True)]
    scale = np.max(np.abs(Qt))
    for out in outs:
        traj = out["traj_views"][0][0].cpu().numpy().T
        assert np.max(np.abs(traj - Qt)) <= 1e-10 * scale
        assert out["train_err"].item() == pytest.approx(e, rel=1e-8)
        assert out["growth"].item() == pytest.approx(gg, rel=1e-10)
        assert (out["outcome"].item() == dp.ITEM_PASS) == ok
    # early exit with a growth failure: same outcome, NaN after the exit
    O2 = torch.from_numpy(np.hstack([1.5 * np.eye(r), np.zeros((r, s)), np.zeros((r, 1))]).ravel().copy()).cuda()
    for f in (False, True):
        o2 = dp.rollout(O2, Qhat, [r], 1, n_states, keep_traj=True, one_wg=f)
        assert o2["outcome"].item() == dp.ITEM_GROWTH
        tr = o2["traj_views"][0][0].cpu().numpy()
        assert np.isnan(tr[-1]).all() and np.isfinite(tr[0]).all()


@pytest.mark.parametrize("r", [20, 60])
def test_full_horizon_many_candidates_match_oracle(gpu_lib, r):
    # many candidates without early exit (more than fit teams): sampled
    # trajectories against the oracle, every candidate's scores against the
    # forced one-workgroup form
    import torch
    dp = gpu_lib
    k, n_states = 300, 700
    Og, Qh = _stable_rom(r, k, 100 + r)
    n_items = 300
    scale_A = 1.0 + 2e-3 * np.linspace(-1, 1, n_items)
    Os = []
    for p in range(n_items):
        O = Og.copy()
        O[:, :r] *= scale_A[p]
        Os.append(O.ravel())
    Od = torch.from_numpy(np.concatenate(Os)).cuda()
    Qhat = torch.from_numpy(Qh.copy()).cuda()
    team = dp.rollout(Od, Qhat, [r], n_items, n_states, keep_traj=True, full=True)
    one = dp.rollout(Od, Qhat, [r], n_items, n_states, keep_traj=True, full=True, one_wg=True)
    torch.cuda.synchronize()
    for p in (0, 1, 137, n_items - 1):
        ref = orc.rollout(Os[p].reshape(r, -1), r, Qh[:, 0], n_states)
        tr = team["traj_views"][0][p].cpu().numpy().T
        assert np.max(np.abs(tr - ref)) <= 1e-10 * np.max(np.abs(ref)), p
    for key in ("train_err", "growth"):
        a, b = team[key].cpu().numpy(), one[key].cpu().numpy()
        assert np.allclose(a, b, rtol=1e-9, atol=0), key
    assert np.array_equal(team["outcome"].cpu().numpy(), one["outcome"].cpu().numpy())
    assert team["best"].item() == one["best"].item()


def test_rollout_teams_of_both_operator_widths(gpu_lib):
    """Team rollouts of two reduced sizes whose operators take different
    register widths per lane (r = 12: d = 91; r = 64: d = 2145 > 2048), so
    one call makes two cooperative launches, each a set of team groups, against
    the oracle's rollouts of the same operators."""
    import torch
    dp = gpu_lib
    rng = np.random.default_rng(64)
    k, rmax = 300, 64
    # a damped linear system observed in 64 coordinates
    A = rng.standard_normal((rmax, rmax))
    A *= 0.97 / np.max(np.abs(np.linalg.eigvals(A)))
    Qh = np.zeros((rmax, k))
    Qh[:, 0] = rng.standard_normal(rmax)
    for t in range(1, k):
        Qh[:, t] = A @ Qh[:, t - 1] + 1e-3 * rng.standard_normal(rmax)
    Qhat = dev(Qh)
    r_list = [12, 64]
    O, status, views = dp.infer(Qhat, r_list, [1e-2], [1e-1])
    n_states = 600
    out = dp.rollout(O, Qhat, r_list, 1, n_states, max_growth=1.2, solve_status=status, keep_traj=True, full=True)
    torch.cuda.synchronize()
    oc = out["outcome"].cpu().numpy()
    for g, r in enumerate(r_list):
        Og = views[g][0].cpu().numpy()
        Qt = orc.rollout(Og, r, Qh[:r, 0], n_states)
        fin, e, gg, ok = orc.score(Qt, Qh[:r], k, 1.2)
        traj = out["traj_views"][g][0].cpu().numpy().T
        if fin:
            assert np.max(np.abs(traj - Qt)) <= 1e-9 * np.max(np.abs(Qt)), r
            assert (oc[g] == dp.ITEM_PASS) == ok
        else:
            assert oc[g] == dp.ITEM_NONFINITE
