"""The batched form's launch machinery on the GPU, through the C ABI.

* Every block-column width the autotuner may pick, for the beta2-group
  Cholesky and for the triangular solves with its factor, gives operators
  within the derived solve bounds (the same backward- and forward-error
  bounds as test_gpu_step4.py), at reduced sizes r in {20, 40} (s = 210,
  820: several block columns of each width and a ragged last panel).
* The autotuner stores its fastest candidates for every factorization size
  and returns what infer returns.
* The captured sweep (infer + rollout as one graph) replays what the eager
  calls compute: the same kernels with the same launch parameters in the same
  order, so every output is compared bit for bit, on every replay, with eager
  work and synchronizations in between, and after new data is written into
  Qhat.
"""
import numpy as np
import pytest

import oracle as orc
import synth
from opcheck import check_operators as _check_ops

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def check_operators(G, B, r, b1, b2, O_gpu, where, k):
    _check_ops(G, B, r, b1, b2, O_gpu, k, where)


@pytest.fixture(scope="module")
def qhat40(gpu_lib):
    """Reduced data at r = 40 from the wave-mode generator (4 x 2,000 cells,
    400 snapshots)."""
    import torch
    dp = gpu_lib
    m = synth.c2_modes(nvars=4, ncell=2000, k=400, n_modes=80, n_pairs=30, decay=20.0, seed=7)
    Q = synth.c2_snapshots(m, noise_var=1e-8, seed=7, device=torch.device("cuda:0"))
    var_rows = [v * 2000 for v in range(5)]
    mean, scale, _ = dp.preprocess(Q, var_rows)
    lam, _, Qhat, info, _ = dp.reduce(dp.gram(Q, mean, scale, var_rows), r=40, want_tr=False)
    assert int(info.item()) == 0
    return Qhat.contiguous()


R_LIST = [20, 40]
B1 = [1e-6, 1e-3, 1e-6, 1e-3]
B2 = [1e-4, 1e-4, 1e-1, 1e-1]


@pytest.fixture
def clean_tuning(gpu_lib):
    dp = gpu_lib
    yield
    for r in R_LIST + [10, 30]:
        for param in (dp.TUNE_CHOL_KB, dp.TUNE_TRSM_KB, dp.TUNE_CHOL_KB2, dp.TUNE_TRSM_KB2):
            dp.tune_set(param, dp.n_quad(r), 0)


@pytest.mark.parametrize("kc,kt", [((64, 0), (64, 0)), ((128, 0), (128, 0)), ((256, 0), (256, 0)),
                                   ((512, 0), (512, 0)), ((64, 0), (512, 0)), ((512, 0), (128, 0)),
                                   ((512, 128), (512, 128)), ((1024, 256), (1024, 128)),
                                   ((2048, 256), (1024, 256)), ((1024, 128), (2048, 256))])
def test_every_block_width_gives_parity(gpu_lib, qhat40, clean_tuning, kc, kt):
    """Every (outer, inner) width pair the autotuner may pick; at s = 210 and
    820 the two-level pairs have ragged outer and inner blocks."""
    dp = gpu_lib
    pairs = list(zip(dp.autotune_candidates(dp.TUNE_CHOL_KB), dp.autotune_candidates(dp.TUNE_CHOL_KB2)))
    assert kc in pairs and kt in pairs
    for r in R_LIST:
        dp.tune_set(dp.TUNE_CHOL_KB, dp.n_quad(r), kc[0])
        dp.tune_set(dp.TUNE_CHOL_KB2, dp.n_quad(r), kc[1])
        dp.tune_set(dp.TUNE_TRSM_KB, dp.n_quad(r), kt[0])
        dp.tune_set(dp.TUNE_TRSM_KB2, dp.n_quad(r), kt[1])
    kb = (kc, kt)
    print(f"infer with block-column widths {kb}, r in {R_LIST}", flush=True)
    O, status, views = dp.infer(qhat40, R_LIST, B1, B2)
    st = status.cpu().numpy()
    Qh = qhat40.cpu().numpy()
    k = Qh.shape[1]
    for g, r in enumerate(R_LIST):
        _, G, B = orc.opinf_data(Qh[:r])
        for p in range(len(B1)):
            assert st[g * len(B1) + p] == 0, (r, p)
            check_operators(G, B, r, B1[p], B2[p], views[g][p].cpu().numpy(), (kb, r, p), k)


def test_autotuner_stores_a_candidate(gpu_lib, qhat40, clean_tuning):
    dp = gpu_lib
    cands = list(zip(dp.autotune_candidates(dp.TUNE_CHOL_KB), dp.autotune_candidates(dp.TUNE_CHOL_KB2)))
    print("autotune", flush=True)
    O, status, views, times = dp.autotune_infer(qhat40, R_LIST, B1, B2)
    assert times.shape == (len(R_LIST), 2, len(cands))
    assert np.all(times > 0) and np.all(np.isfinite(times))
    for g, r in enumerate(R_LIST):
        s = dp.n_quad(r)
        kc = (dp.tune_get(dp.TUNE_CHOL_KB, s), dp.tune_get(dp.TUNE_CHOL_KB2, s))
        kt = (dp.tune_get(dp.TUNE_TRSM_KB, s), dp.tune_get(dp.TUNE_TRSM_KB2, s))
        assert kc == cands[int(np.argmin(times[g, 0]))], (r, kc, times[g])
        assert kt == cands[int(np.argmin(times[g, 1]))], (r, kt, times[g])
    # its results are infer's, with the tuned widths: the same values as a
    # plain infer call now, and parity with the oracle
    O2, status2, _ = dp.infer(qhat40, R_LIST, B1, B2)
    assert np.array_equal(O.cpu().numpy(), O2.cpu().numpy())
    assert np.array_equal(status.cpu().numpy(), status2.cpu().numpy())
    Qh = qhat40.cpu().numpy()
    for g, r in enumerate(R_LIST):
        _, G, B = orc.opinf_data(Qh[:r])
        for p in range(len(B1)):
            check_operators(G, B, r, B1[p], B2[p], views[g][p].cpu().numpy(), ("tuned", r, p), Qh.shape[1])


def _eager(dp, Qhat, r_list, b1, b2, n_states):
    O, status, _ = dp.infer(Qhat, r_list, b1, b2)
    out = dp.rollout(O, Qhat, r_list, len(b1), n_states, solve_status=status, one_wg=True)
    return {"O": O, "status": status, "train_err": out["train_err"], "growth": out["growth"],
            "outcome": out["outcome"], "best": out["best"]}


def _assert_same(sw, ref, where):
    for name in ("O", "status", "train_err", "growth", "outcome", "best"):
        a = getattr(sw, name).cpu().numpy()
        b = ref[name].cpu().numpy()
        assert np.array_equal(a, b, equal_nan=True), (where, name)


@pytest.mark.parametrize("autotune", [False, True])
def test_captured_sweep_replays_eager_results(gpu_lib, qhat40, clean_tuning, autotune):
    import torch
    dp = gpu_lib
    r_list = [10, 20, 40]
    b1 = [x for x in synth.logspace_points(-10, -2, 3) for _ in range(3)]
    b2 = [y for _ in range(3) for y in synth.logspace_points(-8, 0, 3)]
    n_states = 800
    Qhat = qhat40.clone()
    print(f"capture sweep (autotune={autotune})", flush=True)
    sw = dp.Sweep(Qhat, r_list, b1, b2, n_states, autotune=autotune)
    try:
        torch.cuda.synchronize()
        ref = _eager(dp, Qhat, r_list, b1, b2, n_states)
        torch.cuda.synchronize()
        for rep in range(3):
            print(f"replay {rep}", flush=True)
            sw.launch()
            sw.stream.synchronize()
            _assert_same(sw, ref, rep)
            # the program's own eager work between replays
            other = _eager(dp, Qhat[:20].contiguous(), [10], b1[:2], b2[:2], 100)
            torch.cuda.synchronize()
            assert other["O"].numel() > 0
        # new reduced data written into Qhat: the replay reads it
        Qhat.mul_(1.5)
        torch.cuda.synchronize()
        ref2 = _eager(dp, Qhat, r_list, b1, b2, n_states)
        torch.cuda.synchronize()
        sw.launch()
        sw.stream.synchronize()
        _assert_same(sw, ref2, "new data")
        assert not np.array_equal(ref2["O"].cpu().numpy(), ref["O"].cpu().numpy())
        # and the replayed selection agrees with the oracle's rule on its scores
        te, oc, best = sw.train_err.cpu().numpy(), sw.outcome.cpu().numpy(), sw.best.cpu().numpy()
        n = len(b1)
        for g in range(len(r_list)):
            exp = orc.select_best(list(te[g * n:(g + 1) * n]), [o == dp.ITEM_PASS for o in oc[g * n:(g + 1) * n]])
            assert best[g] == (g * n + exp if exp >= 0 else -1)
    finally:
        sw.close()


def test_uneven_groups_and_several_chunks(gpu_lib, qhat40, clean_tuning):
    """40 distinct beta2 values (two chunks of beta2 groups) with 1 to 3 pairs
    per value: pair tables per chunk, batch order by group and right-hand sides
    of different widths per group, against the oracle's solves."""
    dp = gpu_lib
    rng = np.random.default_rng(11)
    b2_vals = synth.logspace_points(-6, 0, 40)
    b1, b2 = [], []
    for i, v in enumerate(b2_vals):
        for _ in range(1 + i % 3):
            b1.append(float(10.0 ** rng.uniform(-8, -2)))
            b2.append(float(v))
    order = rng.permutation(len(b1))  # pairs of one beta2 not adjacent
    b1 = [b1[i] for i in order]
    b2 = [b2[i] for i in order]
    r_list = [10, 20]
    for r in r_list:  # narrow blocks, so several block columns at s = 55 and 210
        dp.tune_set(dp.TUNE_CHOL_KB, dp.n_quad(r), 64)
        dp.tune_set(dp.TUNE_TRSM_KB, dp.n_quad(r), 128)
    print(f"{len(b1)} pairs over 40 beta2 values, r in {r_list}", flush=True)
    O, status, views = dp.infer(qhat40, r_list, b1, b2)
    st = status.cpu().numpy()
    Qh = qhat40.cpu().numpy()
    for g, r in enumerate(r_list):
        _, G, B = orc.opinf_data(Qh[:r])
        for p in range(len(b1)):
            assert st[g * len(b1) + p] == 0, (r, p)
            check_operators(G, B, r, b1[p], b2[p], views[g][p].cpu().numpy(), (r, p), Qh.shape[1])


def test_group_fork_does_not_change_results(gpu_lib, qhat40, clean_tuning, monkeypatch):
    """Several reduced sizes run on internal streams (at most
    GPU_MAX_HW_QUEUES - 1, read at every call): with no fork (2 queues), with
    the two smallest of four groups sharing a stream (4 queues) and with a
    stream per group (8 queues) the operators and statuses are bit for bit
    the same, since every group's kernels and their order are unchanged."""
    import torch
    dp = gpu_lib
    r_list = [10, 20, 30, 40]
    out = {}
    for q in ("2", "4", "8"):
        monkeypatch.setenv("GPU_MAX_HW_QUEUES", q)
        print(f"infer with GPU_MAX_HW_QUEUES={q}", flush=True)
        O, status, _ = dp.infer(qhat40, r_list, B1, B2)
        torch.cuda.synchronize()
        out[q] = (O.cpu().numpy(), status.cpu().numpy())
    for q in ("4", "8"):
        assert np.array_equal(out[q][1], out["2"][1]), q
        assert np.array_equal(out[q][0], out["2"][0]), q
