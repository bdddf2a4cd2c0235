"""Parity at the benchmark's full size, in the launch configuration bench.py
times: the plain float64 step at one GPU's share (n = 4,000,000 rows =
4 variables x 1,000,000 cells, k = 2,000 snapshots, 64 GB in HBM; r = 60,
(beta1, beta2) = (1e-2, 1e8), 4,000 states) and the regularization sweep on
the same data (r in {20, 40, 60, 80} x 32 x 32 pairs).

The oracle cannot redo a 64 GB Gram on the host, so the outputs are checked
where the oracle can compute them one by one:
  * row means: sampled rows, from their own 2,000 values;
  * scale factors: every s_v must bound the sampled rows of its variable and
    must be attained exactly by one of its rows (located on the GPU, then
    verified by the oracle on that row alone);
  * D: every entry among 20 sampled columns (tile edges, the ragged last tile,
    the diagonal), the oracle's Gram over all 4,000,000 rows of those columns
    centered and scaled with the statistics checked above;
  * eigenpairs, Qhat, operators: the oracle's eigendecomposition and solve of
    the GPU's own D and Qhat (32 MB and 1999 x 1891); the operators' backward
    error bound u ((k - 1) sqrt(d) + 10 d) covers forming G = Dhat^T Dhat with
    (k-1)-term sums plus a backward-stable Cholesky solve (derivation in
    test_gpu_step4.py);
  * rollout and score: the oracle's rollout of the GPU's operators.
"""
import numpy as np
import pytest

import oracle as orc
import synth
from opcheck import check_solver_only, gpu_normal_equations, normal_equations_at

pytestmark = pytest.mark.gpu

N_VAR, N_CELL, K = 4, 1_000_000, 2000
R, BETA, N_STATES = 60, (1e-2, 1e8), 4000
U = 2.0 ** -53


def eta_bound(k, d):
    return U * ((k - 1) * np.sqrt(d) + 10 * d)


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def c2(gpu_lib):
    import torch
    dp = gpu_lib
    print("full size: generating 4,000,000 x 2,000 float64", flush=True)
    m = synth.c2_modes(nvars=N_VAR, ncell=N_CELL, k=K, n_modes=200, n_pairs=60, decay=40.0, seed=2)
    Q = synth.c2_snapshots(m, noise_var=1e-8, seed=2, device=torch.device("cuda:0"))
    var_rows = [v * N_CELL for v in range(N_VAR + 1)]
    # the bench step, call for call
    mean, scale, zr = dp.preprocess(Q, var_rows)
    D = dp.gram(Q, mean, scale, var_rows)
    lam, Tr, Qhat, info, r = dp.reduce(D, r=R)
    Qh = Qhat.contiguous()
    O, status, views = dp.infer(Qh, [R], [BETA[0]], [BETA[1]])
    out = dp.rollout(O, Qh, [R], 1, N_STATES, solve_status=status, keep_traj=True)
    torch.cuda.synchronize()
    yield dict(Q=Q, var_rows=var_rows, mean=mean, scale=scale, zr=zr, D=D, lam=lam, Tr=Tr, Qhat=Qh, info=info,
               O=O, status=status, views=views, out=out)
    del Q
    torch.cuda.empty_cache()


def test_fullsize_statistics(gpu_lib, c2):
    import torch
    Q, var_rows = c2["Q"], c2["var_rows"]
    mean = c2["mean"].cpu().numpy()
    scale = c2["scale"].cpu().numpy()
    assert c2["zr"].cpu().numpy().tolist() == [0] * N_VAR
    rng = np.random.default_rng(40)
    rows = np.sort(np.concatenate([rng.choice(N_VAR * N_CELL, 60, replace=False),
                                   [0, N_CELL - 1, N_CELL, 3 * N_CELL + 7, N_VAR * N_CELL - 1]]))
    Qr = Q[torch.from_numpy(rows).cuda()].cpu().numpy()
    mu_o = orc.temporal_mean(Qr)
    assert np.max(np.abs(mean[rows] - mu_o)) <= 1e-14 * max(1.0, np.max(np.abs(Qr)))
    for v in range(N_VAR):
        lo, hi = var_rows[v], var_rows[v + 1]
        sel = (rows >= lo) & (rows < hi)
        Qc = Qr[sel] - mean[rows[sel]][:, None]
        assert np.max(np.abs(Qc)) <= scale[v]
        # the row that attains the maximum, located on the GPU, verified by the oracle
        blk = Q[lo:hi]
        row_max = torch.amax(torch.abs(blk - c2["mean"][lo:hi, None]), dim=1)
        i = int(torch.argmax(row_max).item())
        qi = Q[lo + i].cpu().numpy()[None, :]
        # that row's mean (oracle) and its max-abs about the GPU's mean: equal to s_v exactly
        assert abs(mean[lo + i] - orc.temporal_mean(qi)[0]) <= 1e-14 * max(1.0, np.max(np.abs(qi)))
        s_i, _ = orc.variable_scales(qi - mean[lo + i], [0, 1])
        assert s_i[0] == scale[v], (v, s_i[0], scale[v])
        del blk, row_max


def test_fullsize_gram_sampled_entries(gpu_lib, c2):
    import torch
    Q, var_rows = c2["Q"], c2["var_rows"]
    cols = np.array([0, 1, 63, 64, 127, 128, 129, 700, 1023, 1024, 1500, 1791, 1792, 1919, 1920, 1921,
                     1983, 1984, 1998, 1999])
    Qc = Q[:, torch.from_numpy(cols).cuda()].cpu().numpy()
    mean = c2["mean"].cpu().numpy()
    s_rows = np.repeat(c2["scale"].cpu().numpy(), N_CELL)
    Qs = orc.apply_statistics(Qc, mean, s_rows)
    Dref = orc.gram(Qs)
    Dg = c2["D"].cpu().numpy()
    Dsel = Dg[np.ix_(cols, cols)]
    # per entry, relative to the Cauchy-Schwarz scale sqrt(D_aa D_bb)
    cs = np.sqrt(np.outer(np.diag(Dref), np.diag(Dref)))
    assert np.max(np.abs(Dsel - Dref) / cs) <= 1e-12
    assert np.array_equal(Dg, Dg.T)


def test_fullsize_reduce(gpu_lib, c2):
    D = c2["D"].cpu().numpy()
    assert int(c2["info"].item()) == 0
    lam_o, U_o = orc.eig_desc(D)
    lam = c2["lam"].cpu().numpy()
    assert np.max(np.abs(lam - lam_o)) <= 1e-13 * lam_o[0]
    Tr_o, Qhat_o = orc.reduce_basis_free(lam_o, U_o, R)
    Qh = c2["Qhat"].cpu().numpy()
    # per mode: the eigenvector error is u ||D|| over the gap to the neighbours
    gaps = np.minimum(np.abs(np.diff(lam_o[:R + 1]))[:R], np.r_[np.inf, np.abs(np.diff(lam_o[:R]))])
    for i in range(R):
        bound = max(1e-10, 100 * U * lam_o[0] / gaps[i])
        assert rel(Qh[i], Qhat_o[i]) <= bound, (i, rel(Qh[i], Qhat_o[i]), bound)


def test_fullsize_operators_and_rollout(gpu_lib, c2):
    dp = gpu_lib
    Qh = c2["Qhat"].cpu().numpy()
    assert int(c2["status"].item()) == 0
    _, G, B = orc.opinf_data(Qh)
    M = G + np.diag(orc.regularizer(R, *BETA))
    O_gpu = c2["views"][0][0].cpu().numpy()
    O_ref = orc.solve_operators(G, B, R, *BETA, method="lu")

    def eta(O):
        return np.linalg.norm(M @ O.T - B) / (np.linalg.norm(M) * np.linalg.norm(O) + np.linalg.norm(B))

    e_gpu, e_ref = eta(O_gpu), eta(O_ref)
    assert e_gpu <= eta_bound(K, M.shape[0])
    assert rel(O_gpu, O_ref) <= max(1e-10, 2 * np.linalg.cond(M) * max(e_gpu, e_ref, U))
    # the solver alone, on the G and B the GPU forms itself
    GE = gpu_normal_equations(dp, Qh, R)
    Gg, Bg = normal_equations_at(GE, R, R)
    check_solver_only(Gg, Bg, R, *BETA, O_gpu, "full size (1e-2, 1e8)")
    # the oracle's rollout of the GPU's operators
    Qt = orc.rollout(O_gpu, R, Qh[:, 0], N_STATES)
    fin, te, g, ok = orc.score(Qt, Qh, Qh.shape[1], 1.2)
    out = c2["out"]
    traj = out["traj_views"][0][0].cpu().numpy().T
    assert fin
    assert np.max(np.abs(traj - Qt)) <= 1e-10 * np.max(np.abs(Qt))
    assert out["train_err"].item() == pytest.approx(te, rel=1e-9)
    assert out["growth"].item() == pytest.approx(g, rel=1e-10)
    assert (out["outcome"].item() == dp.ITEM_PASS) == ok
    assert out["best"].item() == (0 if ok else -1)


def test_fullsize_sweep_sampled_items(gpu_lib, c2):
    """The regularization sweep (4 r x 32 x 32 = 4096 items, one workgroup per
    item): sampled items and every group's selected item against the oracle's
    solve and rollout; the selection against the oracle's rule on the GPU's
    scores."""
    dp = gpu_lib
    lam80, _, Qh80, info80, _ = dp.reduce(c2["D"], r=80, want_tr=False)
    Qh80 = Qh80.contiguous()
    B1 = synth.logspace_points(-10, -2, 32)
    B2 = synth.logspace_points(-8, 0, 32)
    b1 = [x for x in B1 for _ in B2]
    b2 = [y for _ in B1 for y in B2]
    r_list = [20, 40, 60, 80]
    O, status, views = dp.infer(Qh80, r_list, b1, b2)
    out = dp.rollout(O, Qh80, r_list, len(b1), N_STATES, solve_status=status)
    te = out["train_err"].cpu().numpy()
    gr = out["growth"].cpu().numpy()
    oc = out["outcome"].cpu().numpy()
    st = status.cpu().numpy()
    best = out["best"].cpu().numpy()
    Qh = Qh80.cpu().numpy()
    rng = np.random.default_rng(41)
    npair = len(b1)
    for g, r in enumerate(r_list):
        # selection: the oracle's rule on the GPU's scores
        items = range(g * npair, (g + 1) * npair)
        exp = orc.select_best([te[i] for i in items], [oc[i] == dp.ITEM_PASS for i in items])
        assert best[g] == (g * npair + exp if exp >= 0 else -1)
        picks = list(rng.choice(npair, 3, replace=False))
        if best[g] >= 0:
            picks.append(best[g] - g * npair)
        _, G, B = orc.opinf_data(Qh[:r])
        for p in picks:
            it = g * npair + p
            M = G + np.diag(orc.regularizer(r, b1[p], b2[p]))
            if st[it] != 0:
                # a refused system must be singular to working precision: the
                # oracle's own Cholesky breaks down or has a pivot ratio < 1e-10
                assert st[it] == dp.E_NOTSPD and oc[it] == dp.ITEM_SOLVE
                try:
                    L = np.linalg.cholesky(M)
                    assert np.min(np.diag(L)) ** 2 / np.max(np.diag(M)) < 1e-10, (r, p)
                except np.linalg.LinAlgError:
                    pass
                continue
            Og = views[g][p].cpu().numpy()
            e_gpu = np.linalg.norm(M @ Og.T - B) / (np.linalg.norm(M) * np.linalg.norm(Og) + np.linalg.norm(B))
            assert e_gpu <= eta_bound(K, M.shape[0]), (r, p, e_gpu)
            Qt = orc.rollout(Og, r, Qh[:r, 0], N_STATES)
            fin, e, gg, ok = orc.score(Qt, Qh[:r], Qh.shape[1], 1.2)
            if not fin:
                assert oc[it] in (dp.ITEM_NONFINITE, dp.ITEM_GROWTH)
                continue
            assert (oc[it] == dp.ITEM_PASS) == ok, (r, p)
            if ok:
                assert te[it] == pytest.approx(e, rel=1e-8), (r, p)
                assert gr[it] == pytest.approx(gg, rel=1e-9), (r, p)


def test_fullsize_postprocess(gpu_lib, c2):
    """Step V at full size: basis rows and the lifted 4000-state rollout at
    sampled rows against the oracle on those rows (the same bytes, the GPU's
    statistics and T_r); all 4,000,000 basis rows orthonormal (V^T V by the
    cross-Gram kernel)."""
    import torch
    dp = gpu_lib
    Q, var_rows = c2["Q"], c2["var_rows"]
    rng = np.random.default_rng(50)
    rows = np.sort(np.concatenate([rng.choice(N_VAR * N_CELL, 59, replace=False),
                                   [0, N_CELL - 1, N_CELL, 3 * N_CELL + 7, N_VAR * N_CELL - 1]])).astype(np.int64)
    rows_d = torch.from_numpy(rows).cuda()
    traj = c2["out"]["traj_views"][0][0]          # n_states x r
    Qt = traj.t().contiguous()
    V, pred, info = dp.postprocess(Q, c2["Tr"], rows=rows_d, Qtilde=Qt, mean=c2["mean"], scale=c2["scale"],
                                   var_rows=var_rows)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    Qr = Q[rows_d].cpu().numpy()
    mean, scale = c2["mean"].cpu().numpy(), c2["scale"].cpu().numpy()
    Tr = c2["Tr"].cpu().numpy()
    s_rows = np.repeat(scale, N_CELL)[rows]
    Qs = orc.apply_statistics(Qr, mean[rows], s_rows)
    Vref = orc.basis_rows(Qs, Tr, np.arange(len(rows)))
    gam = K * U / (1 - K * U)
    bound = 2 * gam * (np.abs(Qs) @ np.abs(Tr)) + 4 * U * np.abs(Vref)
    Vg = V.cpu().numpy()
    assert np.all(np.abs(Vg - Vref) <= bound), float(np.max(np.abs(Vg - Vref) / bound))
    Qtn = Qt.cpu().numpy()
    fin = np.all(np.isfinite(Qtn), axis=0)
    pref = s_rows[:, None] * (Vref @ Qtn[:, fin]) + mean[rows][:, None]
    assert rel(pred.cpu().numpy()[:, fin], pref) <= 1e-12
    # every basis row: V_r = Qs T_r is orthonormal (Eq. (7))
    Vall, _, info = dp.postprocess(Q, c2["Tr"], rows=None, m=N_VAR * N_CELL, mean=c2["mean"], scale=c2["scale"],
                                   var_rows=var_rows)
    G = dp.cross_gram(Vall, Vall)
    torch.cuda.synchronize()
    assert rel(G.cpu().numpy(), np.eye(R)) <= 1e-10
    # the all-rows form (a kernel of its own) at the sampled rows, entry by entry
    assert np.all(np.abs(Vall[rows_d].cpu().numpy() - Vref) <= bound)
    del Vall


def test_fullsize_partial_eig(gpu_lib, c2):
    """The partial eigendecomposition at r = 60 on the full-size D: the same
    Qhat as the full eigensolver within each mode's sensitivity, far fewer
    operations (block subspace iteration)."""
    import torch
    dp = gpu_lib
    lam_p, Tr_p, Qh_p, info, iters = dp.reduce_topr(c2["D"], R)
    torch.cuda.synchronize()
    assert int(info.item()) == 0 and 0 < iters <= 80
    lam = c2["lam"].cpu().numpy()
    assert np.max(np.abs(lam_p.cpu().numpy() - lam[:R])) <= 1e-13 * lam[0]
    gaps = np.abs(np.diff(lam[:R + 1]))
    gaps = np.minimum(np.concatenate([[np.inf], gaps[:-1]]), gaps)
    Qf, Qp = c2["Qhat"].cpu().numpy(), Qh_p.cpu().numpy()
    for i in range(R):
        bound = max(1e-10, 200 * U * lam[0] / gaps[i])
        assert rel(Qp[i], Qf[i]) <= bound, (i, rel(Qp[i], Qf[i]), bound)


def test_fullsize_gram_whole_matrix_oracle(gpu_lib, c2):
    """D over all 4,000,000 rows against the oracle's Gram, accumulated over
    row chunks of the same bytes (Eq. (5): the Gram of a row partition is the
    sum of the blocks' Grams), with the statistics checked above."""
    import torch
    Q, var_rows = c2["Q"], c2["var_rows"]
    mean = c2["mean"].cpu().numpy()
    s_rows = np.repeat(c2["scale"].cpu().numpy(), N_CELL)
    Dref = np.zeros((K, K))
    chunk = 250_000
    for r0 in range(0, N_VAR * N_CELL, chunk):
        blk = Q[r0:r0 + chunk].cpu().numpy()
        Dref += orc.gram(orc.apply_statistics(blk, mean[r0:r0 + chunk], s_rows[r0:r0 + chunk]))
        del blk
    assert rel(c2["D"].cpu().numpy(), Dref) <= 1e-12


def test_fullsize_sweep_full_horizon_trajectories(gpu_lib, c2):
    """The many-candidate rollout (one workgroup per candidate, as the sweep
    runs it) over the full 4,000-state horizon without early exit, at r = 60
    and r = 80, against the oracle's rollout of the same operators: bounded
    ROMs (beta2 from 1e8 to 1e10, the step's pair among them) over all 4,000
    states to 1e-9 of the trajectory's scale; the grid's own SPD pairs
    (beta2 <= 1), whose ROMs grow without bound, state by state to 1e-8
    relative up to the oracle's first non-finite (or > 1e150) state."""
    import torch
    dp = gpu_lib
    lam80, _, Qh80, info80, _ = dp.reduce(c2["D"], r=80, want_tr=False)
    Qh80 = Qh80.contiguous()
    B1 = synth.logspace_points(-10, -2, 32)
    B2 = synth.logspace_points(-8, 0, 32)
    b1 = [1e-2, 1e-2, 1e-6, B1[-1], B1[-2], B1[-1]]
    b2 = [1e8, 1e9, 1e10, B2[-1], B2[-1], B2[-5]]
    r_list = [60, 80]
    O, status, views = dp.infer(Qh80, r_list, b1, b2)
    out = dp.rollout(O, Qh80, r_list, len(b1), N_STATES, solve_status=status, keep_traj=True, full=True,
                     one_wg=True)
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    Qh = Qh80.cpu().numpy()
    checked = {True: 0, False: 0}
    for g, r in enumerate(r_list):
        for p in range(len(b1)):
            if st[g * len(b1) + p] != 0:
                continue
            Og = views[g][p].cpu().numpy()
            ref = orc.rollout(Og, r, Qh[:r, 0], N_STATES)
            tr = out["traj_views"][g][p].cpu().numpy().T
            fin = np.all(np.isfinite(ref), axis=0) & (np.max(np.abs(ref), axis=0) < 1e150)
            n_ok = int(np.argmin(fin)) if not fin.all() else N_STATES
            bnd = n_ok == N_STATES and np.max(np.abs(ref)) < 1e3 * np.max(np.abs(Qh[:r]))
            if bnd:
                scale = np.max(np.abs(ref))
                assert np.max(np.abs(tr - ref)) <= 1e-9 * scale, (r, p)
            else:
                assert n_ok > 1, (r, p, n_ok)
                nrm = np.linalg.norm(ref[:, :n_ok], axis=0)
                err = np.linalg.norm(tr[:, :n_ok] - ref[:, :n_ok], axis=0) / nrm
                assert np.max(err) <= 1e-8, (r, p, n_ok, float(np.max(err)))
            checked[bool(bnd)] += 1
    assert checked[True] >= 2 and checked[False] >= 2, checked
