#!/usr/bin/env python3
"""Benchmark of the dOpInf hot path on one MI355X.

One step = one pass of Steps II-IV over the plain float64 workload at one
GPU's full share (n = 4,000,000 rows = 4 variables x 1,000,000 cells,
k = 2,000 snapshots, 64 GB resident in HBM):
  centering + max-abs scaling -> Gram D (FP64 MFMA) -> eigenpairs and
  basis-free reduced data at r = 60 -> quadratic OpInf at
  (beta1, beta2) = (1e-2, 1e8) (d = 1891) -> 4,000-state rollout, training
  error, growth bound and selection.

Printed: ONE JSON line.  `value` is the Gram rate in TFLOP/s
(algorithmic n*k*(k+1) flops per step over the Gram call's time, HIP events
on the stream the kernels run on), the dominant kernel of the step.  Extra
keys report the other two headline quantities: the regularization-sweep rate
(4 reduced sizes x 32 x 32 pairs, each an FP64 solve plus a 4,000-state
rollout) and the reduced-precision Gram speed-up at a stated error, plus the
CPU oracle timed on a bounded sample of the same bytes.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK = 78.6     # TFLOP/s, MI355X dense FP64 matrix
FP32_PEAK = 157.3    # TFLOP/s, MI355X dense FP32 matrix
BF16_PEAK = 2500.0   # TFLOP/s, MI355X dense BF16 matrix
HBM_PEAK = 8000.0    # GB/s

METRIC = "Gram TFLOP/s (% MFMA peak); reg-sweep solves/s; mixed vs FP64 at 1e-6 err"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class Timer:
    """HIP-event timing of work enqueued on torch's current stream (the
    stream every library call is given)."""

    def __init__(self, torch):
        self.torch = torch
        self.acc = {}
        self.cnt = {}

    def run(self, name, fn):
        t = self.torch
        a = t.cuda.Event(enable_timing=True)
        b = t.cuda.Event(enable_timing=True)
        a.record()
        out = fn()
        b.record()
        self.acc.setdefault(name, []).append((a, b))
        return out

    def ms(self, name):
        self.torch.cuda.synchronize()
        v = [a.elapsed_time(b) for a, b in self.acc.get(name, [])]
        return sum(v) / len(v) if v else float("nan")

    def reset(self):
        self.acc = {}


def measured_traffic():
    """HBM bytes per launch of the Gram kernel from the committed counter
    record (two rocprofv3 --pmc passes, FETCH_SIZE and WRITE_SIZE, scaled by a
    1 GiB copy); None when the kernel sources changed since the counters were
    taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "gram_f64_dma_n4e6_k2000_hbm_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        h = hashlib.sha256()
        for src in rec["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        if h.hexdigest() != rec["sources_sha256"]:
            return None
        return int(rec["bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def make_c2(torch, dev):
    import synth
    m = synth.c2_modes(nvars=4, ncell=1_000_000, k=2000, n_modes=200, n_pairs=60, decay=40.0, seed=2)
    Q = synth.c2_snapshots(m, noise_var=1e-8, seed=2, device=dev)
    var_rows = [0, 1_000_000, 2_000_000, 3_000_000, 4_000_000]
    return m, Q, var_rows


def pipeline_step(dp, Q, var_rows, timer, r=60, n_states=4000, beta=(1e-2, 1e8)):
    """r is prescribed, so the eigenpairs come from the partial eigensolver
    (block subspace iteration with Rayleigh-Ritz; the full tridiagonal
    eigensolver is timed beside the step)."""
    mean, scale, _ = timer.run("preprocess", lambda: dp.preprocess(Q, var_rows))
    D = timer.run("gram", lambda: dp.gram(Q, mean, scale, var_rows))
    lam, Tr, Qhat, info, iters = timer.run("reduce", lambda: dp.reduce_topr(D, r))
    Qh = Qhat.contiguous()
    O, status, views = timer.run("infer", lambda: dp.infer(Qh, [r], [beta[0]], [beta[1]]))
    out = timer.run("rollout", lambda: dp.rollout(O, Qh, [r], 1, n_states, solve_status=status))
    return dict(mean=mean, scale=scale, D=D, lam=lam, Tr=Tr, Qhat=Qh, info=info, O=O, views=views, status=status,
                out=out, iters=iters)


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        affinity = os.cpu_count() or 1
    return {"nproc": affinity, "os_cpu_count": os.cpu_count(), "model": model}


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:  # pragma: no cover
        return os.cpu_count() or 1


def cpu_baseline(Q, var_rows, budget_s, D=None, Qh80=None):
    """The oracle (numpy float64) on the host, on bounded samples of the same
    bytes: Step II + Gram on a row sample (all BLAS threads, then one thread),
    and, when D and the r = 80 reduced data are given, the rest of the step
    (eigendecomposition, inference at r = 60, a 400-state slice of the
    4000-state rollout) and one sweep item per reduced size (solve plus a
    400-state rollout slice), scaled to the full horizon and to 1024 pairs."""
    import numpy as np
    import oracle as orc
    threads = blas_threads()
    k = Q.shape[1]
    nvars = len(var_rows) - 1

    def sample(rows_per_var):
        blocks = [Q[var_rows[v]:var_rows[v] + rows_per_var].cpu().numpy() for v in range(nvars)]
        return np.concatenate(blocks), np.arange(nvars + 1) * rows_per_var

    def stats_gram(Qs, vr):
        t0 = time.perf_counter()
        _, _, Xs, _ = orc.preprocess(Qs, vr)
        orc.gram(Xs)
        return time.perf_counter() - t0

    # calibrate on a small sample, then run ~budget_s
    Qs, vr = sample(2500)
    per_row = stats_gram(Qs, vr) / Qs.shape[0]
    rows = int(max(2500, min(250_000, budget_s / max(per_row, 1e-9) / nvars)))
    Qs, vr = sample(rows)
    t = stats_gram(Qs, vr)
    n_s = Qs.shape[0]
    out = {
        "value": n_s * k * (k + 1) / t / 1e12,
        "unit": "TFLOP/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": f"oracle Step II + Gram on {n_s} rows ({rows} per variable) x {k} snapshots of the same float64 "
                  f"input, {t:.1f} s; Gram flops n*k*(k+1) over that time",
        "host": cpu_info(),
    }
    try:
        from threadpoolctl import threadpool_limits
        Q1, vr1 = sample(max(2500, rows // 8))
        with threadpool_limits(limits=1):
            t1 = stats_gram(Q1, vr1)
        out["one_core"] = {"value": Q1.shape[0] * k * (k + 1) / t1 / 1e12, "unit": "TFLOP/s",
                           "sample": f"{Q1.shape[0]} rows, {t1:.1f} s, BLAS limited to 1 thread"}
    except Exception as e:  # report, do not hide
        out["one_core"] = {"error": repr(e)}
    if D is not None and Qh80 is not None:
        Dn = D.cpu().numpy()
        t0 = time.perf_counter()
        lam, U = orc.eig_desc(Dn)
        t_eig = time.perf_counter() - t0
        Tr, Qh = orc.reduce_basis_free(lam, U, 60)
        t0 = time.perf_counter()
        _, G, B = orc.opinf_data(Qh)
        O = orc.solve_operators(G, B, 60, 1e-2, 1e8)
        t_inf = time.perf_counter() - t0
        t0 = time.perf_counter()
        orc.rollout(O, 60, Qh[:, 0], 400)
        t_roll = (time.perf_counter() - t0) * 3999 / 399
        out["step_rest_s"] = {"eig": t_eig, "infer_r60": t_inf, "rollout_4000_from_400": t_roll}
        Qh80n = Qh80.cpu().numpy()
        per_item = {}
        for r in (20, 40, 60, 80):
            t0 = time.perf_counter()
            _, G, B = orc.opinf_data(Qh80n[:r])
            t_data = time.perf_counter() - t0
            t0 = time.perf_counter()
            O = orc.solve_operators(G, B, r, 1e-6, 1e-4)
            t_solve = time.perf_counter() - t0
            t0 = time.perf_counter()
            orc.rollout(O, r, Qh80n[:r, 0], 400)
            t_roll = (time.perf_counter() - t0) * 3999 / 399
            per_item[str(r)] = {"data_s": t_data, "solve_s": t_solve, "rollout_4000_s": t_roll}
        total = sum(v["data_s"] + 1024 * (v["solve_s"] + v["rollout_4000_s"]) for v in per_item.values())
        out["sweep"] = {"per_item": per_item, "projected_4096_items_s": total,
                        "projected_solves_per_s": 4096 / total,
                        "sample": "one solve and a 400-state rollout slice per reduced size, scaled to 4000 states "
                                  "and 1024 pairs (full-horizon rollouts, no early exit)"}
    return out


def sweep_bench(dp, torch, Qhat80, reps=1):
    """The regularization sweep over every (r, beta1, beta2): block-column
    widths picked by the autotuner, then the sweep captured into one graph and
    replayed (the headline rate); the eager calls are timed beside it."""
    import synth
    B1 = synth.logspace_points(-10, -2, 32)
    B2 = synth.logspace_points(-8, 0, 32)
    b1 = [x for x in B1 for _ in B2]
    b2 = [y for _ in B1 for y in B2]
    r_list = [20, 40, 60, 80]
    n_items = len(r_list) * len(b1)
    t0 = time.perf_counter()
    _, _, _, tune_ms = dp.autotune_infer(Qhat80, r_list, b1, b2)
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t0
    chosen = {r: {"cholesky": [dp.tune_get(dp.TUNE_CHOL_KB, dp.n_quad(r)), dp.tune_get(dp.TUNE_CHOL_KB2, dp.n_quad(r))],
                  "solve": [dp.tune_get(dp.TUNE_TRSM_KB, dp.n_quad(r)), dp.tune_get(dp.TUNE_TRSM_KB2, dp.n_quad(r))]}
              for r in r_list}
    timer = Timer(torch)
    res = None
    for _ in range(reps + 1):  # first pass warms up
        timer.reset()
        O, status, _ = timer.run("infer", lambda: dp.infer(Qhat80, r_list, b1, b2))
        res = timer.run("rollout", lambda: dp.rollout(O, Qhat80, r_list, len(b1), 4000, solve_status=status))
    t_inf, t_roll = timer.ms("infer"), timer.ms("rollout")
    oc = res["outcome"].cpu().numpy()
    # without early exit: the grid's SPD candidates all overflow to non-finite
    # values within a few hundred states (each rollout stops there), so the
    # full 4000-state cost is measured on a second grid whose ROMs stay
    # bounded: beta2 in [1e8, 1e12] (every candidate runs all 4000 states)
    st_np = status.cpu().numpy()
    n_pairs = len(b1)
    spd = {r: int((st_np[g * n_pairs:(g + 1) * n_pairs] == 0).sum()) for g, r in enumerate(r_list)}
    tfull = Timer(torch)
    full = None
    for _ in range(2):
        tfull.reset()
        full = tfull.run("full", lambda: dp.rollout(O, Qhat80, r_list, len(b1), 4000, solve_status=status, full=True))
    t_full_grid = tfull.ms("full")
    oc_full = full["outcome"].cpu().numpy()
    B2b = synth.logspace_points(8, 12, 32)
    b2b = [y for _ in B1 for y in B2b]
    Ob, stb, _ = dp.infer(Qhat80, r_list, b1, b2b)
    tb = Timer(torch)
    fb = None
    for _ in range(2):
        tb.reset()
        fb = tb.run("bounded", lambda: dp.rollout(Ob, Qhat80, r_list, len(b1), 4000, solve_status=stb, full=True))
    t_bounded = tb.ms("bounded")
    ocb = fb["outcome"].cpu().numpy()
    stb_np = stb.cpu().numpy()
    ran = {r: int(((stb_np[g * n_pairs:(g + 1) * n_pairs] == 0) &
                   (ocb[g * n_pairs:(g + 1) * n_pairs] != dp.ITEM_NONFINITE)).sum()) for g, r in enumerate(r_list)}
    op_bytes = sum(ran[r] * 3999 * 8 * r * (r + dp.n_quad(r) + 1) for r in r_list)
    flops_full = sum(ran[r] * 3999 * (2 * r * (r + dp.n_quad(r) + 1) + dp.n_quad(r)) for r in r_list)
    t0 = time.perf_counter()
    sw = dp.Sweep(Qhat80, r_list, b1, b2, 4000)
    t_capture = time.perf_counter() - t0
    try:
        cur = torch.cuda.current_stream()
        times = []
        for _ in range(reps + 2):  # first replay warms up
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(cur)
            sw.launch(cur)
            e1.record(cur)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        t_graph = min(times[1:])
        same_best = sw.best.cpu().numpy().tolist() == res["best"].cpu().numpy().tolist()
        oc_graph = sw.outcome.cpu().numpy()
    finally:
        sw.close()
    return {
        "solves_per_s": n_items / (t_graph * 1e-3),
        "items": n_items,
        "graph_ms": t_graph,
        "eager_infer_ms": t_inf,
        "eager_rollout_ms": t_roll,
        "eager_solves_per_s": n_items / ((t_inf + t_roll) * 1e-3),
        "block_widths": chosen,
        "autotune_ms": {str(r): {"cholesky": [round(float(x), 3) for x in tune_ms[g, 0]],
                                 "solve": [round(float(x), 3) for x in tune_ms[g, 1]]} for g, r in enumerate(r_list)},
        "autotune_candidates": [list(p) for p in zip(dp.autotune_candidates(dp.TUNE_CHOL_KB),
                                                     dp.autotune_candidates(dp.TUNE_CHOL_KB2))],
        "autotune_s": round(t_tune, 2),
        "capture_s": round(t_capture, 2),
        "passing": int((oc == dp.ITEM_PASS).sum()),
        "passing_graph": int((oc_graph == dp.ITEM_PASS).sum()),
        "best": res["best"].cpu().numpy().tolist(),
        "graph_best_matches_eager": same_best,
        "selection_degenerate": bool((oc == dp.ITEM_PASS).sum() == 0),
        "outcomes": {"not_spd": int((oc == dp.ITEM_SOLVE).sum()), "growth": int((oc == dp.ITEM_GROWTH).sum()),
                     "nonfinite": int((oc == dp.ITEM_NONFINITE).sum()), "pass": int((oc == dp.ITEM_PASS).sum())},
        "no_early_exit": {
            "rollout_ms": t_full_grid,
            "spd_items_per_r": spd,
            "outcomes": {"growth": int((oc_full == dp.ITEM_GROWTH).sum()),
                         "nonfinite": int((oc_full == dp.ITEM_NONFINITE).sum()),
                         "pass": int((oc_full == dp.ITEM_PASS).sum())},
            "selection_same_as_early_exit": full["best"].cpu().numpy().tolist() == res["best"].cpu().numpy().tolist(),
        },
        "full_horizon_bounded_grid": {
            "beta2": [1e8, 1e12],
            "rollout_ms": t_bounded,
            "items_run_4000_states_per_r": ran,
            "passing": int((ocb == dp.ITEM_PASS).sum()),
            "operator_bytes_if_streamed": op_bytes,
            "operator_GBps_if_streamed": op_bytes / (t_bounded * 1e-3) / 1e9,
            "frac_of_hbm_if_streamed": op_bytes / (t_bounded * 1e-3) / 1e9 / HBM_PEAK,
            "flops": flops_full,
            "TFLOPs": flops_full / (t_bounded * 1e-3) / 1e12,
            "frac_fp64_peak": flops_full / (t_bounded * 1e-3) / 1e12 / FP64_PEAK,
            "solves_per_s_full_horizon": n_items / ((t_inf + t_bounded) * 1e-3),
        },
    }


def rollout_2000(dp, Qh, r=60, beta=(1e-2, 1e8), n_states=2000):
    O, status, _ = dp.infer(Qh, [r], [beta[0]], [beta[1]])
    out = dp.rollout(O, Qh, [r], 1, n_states, solve_status=status, keep_traj=True, full=True)
    return out["traj_views"][0][0]


def mixed_bench(dp, torch, Q, var_rows, ref_qhat, ref_lam, t_fp64_ms):
    """Reduced-precision Gram forms on float32-stored data (RN of the float64
    input); eigenpairs and everything after stay float64.  Error vs the
    float64 path (itself within 1e-12 (D) and 1e-10 (Qhat) of the oracle, so
    errors above 1e-9 are the same against the oracle): eigenvalues >=
    1e-10 lambda_max, Qhat (r = 60), and the 2000-state rollout of the ROM
    inferred from each form's Qhat at the step's pair, relative to the float64
    path's rollout (max over t of ||q_t - q64_t|| / ||q64_t||)."""
    import numpy as np
    Q32 = Q.to(torch.float32)
    out = {}
    refq = ref_qhat.cpu().numpy()
    refl = ref_lam.cpu().numpy()
    ref_tr = rollout_2000(dp, ref_qhat.contiguous()).cpu().numpy()
    for name, algo in (("fp32", dp.GRAM_NATIVE), ("bf16x3", dp.GRAM_BF16X3), ("bf16x6", dp.GRAM_BF16X6),
                       ("i8x6", dp.GRAM_I8X6)):
        timer = Timer(torch)
        try:
            for _ in range(3):
                timer.reset()
                mean, scale, _ = timer.run("pre", lambda: dp.preprocess(Q32, var_rows))
                D = timer.run("gram", lambda: dp.gram(Q32, mean, scale, var_rows, algo=algo))
                _, _, Qh, info, _ = timer.run("red", lambda: dp.reduce_topr(D, 60, want_tr=False))
            lam = dp.reduce(D, r=60, want_tr=False)[0]   # every eigenvalue, for the error table
        except dp.DopinfError as e:
            out[name] = {"error": str(e)}
            continue
        t = timer.ms("pre") + timer.ms("gram") + timer.ms("red")
        qh = Qh.cpu().numpy()
        l = lam.cpu().numpy()
        sel = refl >= 1e-10 * refl[0]
        row_err = np.linalg.norm(qh - refq, axis=1) / np.linalg.norm(refq, axis=1)
        ok_modes = int(np.argmax(row_err > 1e-6)) if np.any(row_err > 1e-6) else 60
        tr = rollout_2000(dp, Qh.contiguous()).cpu().numpy()
        with np.errstate(all="ignore"):
            terr = np.linalg.norm(tr - ref_tr, axis=1) / np.linalg.norm(ref_tr, axis=1)
        out[name] = {
            "rollout2000_rel_err_max": float(np.max(terr)) if np.all(np.isfinite(terr)) else float("inf"),
            "rollout2000_rel_err_final": float(terr[-1]),
            "ms": t,
            "gram_ms": timer.ms("gram"),
            "speedup_vs_fp64": t_fp64_ms / t,
            "qhat_rel_err": float(np.linalg.norm(qh - refq) / np.linalg.norm(refq)),
            "lambda_rel_err_max": float(np.max(np.abs(l[sel] - refl[sel]) / refl[sel])),
            "lambda_rel_err_median": float(np.median(np.abs(l[sel] - refl[sel]) / refl[sel])),
            "qhat_row_rel_err_max": float(np.max(row_err)),
            "modes_within_1e-6": ok_modes,
        }
    # the fastest form whose Qhat meets 1e-6 (relative, whole matrix and every mode)
    ok = [n_ for n_, v in out.items() if "ms" in v and v["qhat_rel_err"] <= 1e-6 and v["modes_within_1e-6"] == 60]
    if ok:
        best = max(ok, key=lambda n_: out[n_]["speedup_vs_fp64"])
        out["best_at_1e-6"] = {"form": best, "speedup_vs_fp64": out[best]["speedup_vs_fp64"],
                               "qhat_rel_err": out[best]["qhat_rel_err"]}
    del Q32
    return out


def closure_bench(dp, torch, dev, epochs=200):
    """Learned closure at r = 40 on the wave data (4 x 250,000 cells, k = 2000):
    residuals of the r = 40 ROM, training, 1024 perturbed 4000-state rollouts
    with fallback, and the gain on held-out snapshots taken at the half-sample
    times t = 2000.5 .. 3999.5 (states the training window never visits: its
    integer frequencies repeat every 2000 samples), projected through Eq. (8)
    with the training statistics."""
    import numpy as np
    import synth
    r, k, n_states, M = 40, 2000, 4000, 1024
    m = synth.c2_modes(nvars=4, ncell=250_000, k=k, seed=2)
    var_rows = [0, 250_000, 500_000, 750_000, 1_000_000]
    Q = synth.c2_snapshots(m, noise_var=1e-8, seed=2, device=dev)
    Qt = synth.c2_snapshots(m, noise_var=1e-8, seed=3, device=dev, t0=k + 0.5)
    mean, scale, _ = dp.preprocess(Q, var_rows)
    D = dp.gram(Q, mean, scale, var_rows)
    lam, Tr, Qhat, info, _ = dp.reduce(D, r=r)
    Qh = Qhat.contiguous()
    O, status, views = dp.infer(Qh, [r], [1e-2], [1e8])
    Op = views[0][0].contiguous()
    C = dp.cross_gram(Q, Qt, mean=mean, scale=scale, var_rows=var_rows)
    Qh_test = dp.cross_gram(Tr.contiguous(), C)                      # r x k_test
    del Q, Qt, C, D
    timer = Timer(torch)
    X = Qh[:, :-1].T.contiguous()
    Y = timer.run("residuals", lambda: dp.rom_residuals(Op, Qh))
    p0 = torch.from_numpy(synth.mlp_init(r, seed=5))
    params, norm, log = timer.run("train", lambda: dp.closure_fit(X, Y, p0, epochs=epochs, batch=256, lr=1e-3))
    _, gmax = dp.closure_eval(params, norm, X)
    thr = 3.0 * float(gmax.item())
    q0 = torch.from_numpy(synth.perturbed_states(Qh[:, 0].cpu().numpy(), M, std=0.05, seed=5)).to(dev)
    out_c = timer.run("rollout_closure", lambda: dp.closure_rollout(Op, params, norm, thr, q0, n_states, Qh))
    out_p = timer.run("rollout_plain", lambda: dp.closure_rollout(Op, params, norm, 0.0, q0, n_states, Qh))
    # held-out one-step residuals and rollout error against the projection
    Rt = dp.rom_residuals(Op, Qh_test)
    Gt, _ = dp.closure_eval(params, norm, Qh_test[:, :-1].T.contiguous())
    rms_plain = float(torch.sqrt(torch.mean(Rt * Rt)).item())
    rms_closed = float(torch.sqrt(torch.mean((Rt - Gt) ** 2)).item())
    q0t = Qh_test[:, 0].reshape(1, r).contiguous()
    e_c = dp.closure_rollout(Op, params, norm, thr, q0t, k, Qh_test)
    e_p = dp.closure_rollout(Op, params, norm, 0.0, q0t, k, Qh_test)
    oc_c, oc_p = out_c["outcome"].cpu().numpy(), out_p["outcome"].cpu().numpy()
    fb = out_c["fallback_at"].cpu().numpy()
    lg = log.cpu().numpy()
    return {
        "r": r, "epochs": epochs, "train_ms": timer.ms("train"), "train_ms_per_epoch": timer.ms("train") / epochs,
        "loss_first_last": [float(lg[0]), float(lg[-1])],
        "rollouts": M, "n_states": n_states,
        "rollout_closure_ms": timer.ms("rollout_closure"), "rollout_plain_ms": timer.ms("rollout_plain"),
        "threshold": thr,
        "heldout_residual_rms": {"plain": rms_plain, "closure": rms_closed},
        "heldout_rollout_err": {"plain": float(e_p["err"].item()), "closure": float(e_c["err"].item())},
        "closure_helps": {"one_step": rms_closed < rms_plain,
                          "rollout_2000": float(e_c["err"].item()) < float(e_p["err"].item())},
        "stable_fraction": {"plain": float(np.mean(oc_p == 0)), "closure": float(np.mean(oc_c == 0))},
        "fallback_fraction": float(np.mean(fb >= 0)),
        "flops_per_step_per_state": {"rom_fp64": 2 * r * (r + r * (r + 1) // 2 + 1), "mlp": 2 * (128 * r * 2 + 128 * 128)},
    }


def postprocess_bench(dp, torch, Q, mean, scale, var_rows, Tr, traj, reps=3):
    """Step V: the basis at every row, V_r = Qs T_r (n x r), and the lifted
    4000-state prediction at 64 probe rows."""
    n, k = Q.shape
    r = Tr.shape[1]
    Trc = Tr.contiguous()
    timer = Timer(torch)
    V = None
    for _ in range(reps + 1):
        V, _, _ = timer.run("basis", lambda: dp.postprocess(Q, Trc, rows=None, m=n, mean=mean, scale=scale,
                                                            var_rows=var_rows))
    t_basis = timer.ms("basis")
    del V
    rows = torch.arange(0, n, n // 64, dtype=torch.int64, device=Q.device)[:64].contiguous()
    Qt = traj.t().contiguous()
    for _ in range(reps + 1):
        timer.run("probes", lambda: dp.postprocess(Q, Trc, rows=rows, Qtilde=Qt, mean=mean, scale=scale,
                                                   var_rows=var_rows))
    t_probe = timer.ms("probes")
    bytes_basis = n * k * 8 + n * r * 8
    flops_basis = 2 * n * k * r
    return {
        "basis_all_rows_ms": t_basis,
        "basis_GBps": bytes_basis / (t_basis * 1e-3) / 1e9,
        "basis_frac_hbm": bytes_basis / (t_basis * 1e-3) / 1e9 / HBM_PEAK,
        "basis_TFLOPs": flops_basis / (t_basis * 1e-3) / 1e12,
        "basis_frac_fp64_mfma": flops_basis / (t_basis * 1e-3) / 1e12 / FP64_PEAK,
        "probes_64_rows_4000_states_ms": t_probe,
    }


def continuous_bench(dp, torch, Q, var_rows, Qhat, reps=3):
    """Continuous-time form and lifting (Sec. 3.5 Eq. (10); Sec. 3.3) on the
    same input: one lifted variable (the product of variables 0 and 1, 1e6
    cells x k: reads 32 GB, writes 16 GB), continuous-time operators at
    r = 60 from finite-difference derivative data (dt = 1), and RK4 rollouts
    of 4000 states: the r = 60 item alone, and 3 x 32 items at r = 20/40/60
    (beta1 = 1e-2, beta2 = logspace(4, 12, 32)) at full horizon."""
    import numpy as np
    ncell = var_rows[1] - var_rows[0]
    k = Q.shape[1]
    timer = Timer(torch)
    for _ in range(reps):
        L = timer.run("lift", lambda: dp.lift(Q, ncell, [(dp.LIFT_PRODUCT, 0, 1)]))
    t_lift = timer.ms("lift")
    del L
    torch.cuda.empty_cache()
    Qh = Qhat.contiguous()
    for _ in range(reps):
        O1, st1, _ = timer.run("infer", lambda: dp.infer_continuous(Qh, 1.0, [60], [1e-2], [1e8]))
    t_inf = timer.ms("infer")
    for _ in range(reps):
        o1 = timer.run("roll1", lambda: dp.rollout_continuous(O1, Qh, [60], 1, 4000, 1.0, solve_status=st1, full=True))
    t_r1 = timer.ms("roll1")
    b2 = synth_logspace(4, 12, 32)
    O3, st3, _ = dp.infer_continuous(Qh, 1.0, [20, 40, 60], [1e-2] * 32, list(b2))
    for _ in range(reps):
        o3 = timer.run("roll96", lambda: dp.rollout_continuous(O3, Qh, [20, 40, 60], 32, 4000, 1.0, solve_status=st3,
                                                               full=True))
    t_r96 = timer.ms("roll96")
    oc = o3["outcome"].cpu().numpy()
    d60 = 60 + 60 * 61 // 2 + 1
    return {
        "lift_product_ms": t_lift,
        "lift_GBps": 3 * ncell * k * 8 / (t_lift * 1e-3) / 1e9,
        "infer_r60_ms": t_inf,
        "solve_status_r60": int(st1[0].item()),
        "rk4_rollout_r60_4000_states_ms": t_r1,
        "rk4_outcome_r60": int(o1["outcome"][0].item()),
        "rk4_rollouts_96_items_4000_states_ms": t_r96,
        "rk4_outcomes_96": {"pass": int(np.sum(oc == dp.ITEM_PASS)), "nonfinite": int(np.sum(oc == dp.ITEM_NONFINITE)),
                            "growth": int(np.sum(oc == dp.ITEM_GROWTH)), "not_solved": int(np.sum(oc == dp.ITEM_SOLVE))},
        "rk4_flops_per_state_r60": 4 * 2 * 60 * d60,
    }


def synth_logspace(lo, hi, num):
    import synth
    return synth.logspace_points(lo, hi, num)


def stream_bench(dp, torch, Q, var_rows, rows=1_000_000, chunk=65536):
    """Out-of-core Gram: the first 1,000,000 rows (16 GB) in pinned host
    memory, streamed through two device buffers (copy overlapping the chunk
    Grams), against the one-shot device Gram of the same rows."""
    k = Q.shape[1]
    per = rows // (len(var_rows) - 1)
    sel = torch.cat([Q[var_rows[v]:var_rows[v] + per] for v in range(len(var_rows) - 1)])
    vr = [v * per for v in range(len(var_rows))]
    Qh = torch.empty(sel.shape, dtype=torch.float64, pin_memory=True)
    Qh.copy_(sel)
    mean, scale, _ = dp.preprocess(sel, vr)
    D1 = dp.gram(sel, mean, scale, vr)
    del sel
    torch.cuda.empty_cache()
    ws = dp._ws(dp.load().dopinf_stream_workspace(chunk, k, len(vr) - 1), Q.device)
    D = torch.empty((k, k), dtype=torch.float64, device=Q.device)
    timer = Timer(torch)
    for _ in range(3):
        timer.run("stream", lambda: dp.gram_stream(Qh, chunk, mean, scale, vr, out=D, ws=ws))
    t = timer.ms("stream")
    diff = float(torch.linalg.norm(D - D1) / torch.linalg.norm(D1))
    nbytes = rows * k * 8
    del Qh
    return {"rows": rows, "chunk_rows": chunk, "host_bytes": nbytes, "ms": t, "host_GBps": nbytes / (t * 1e-3) / 1e9,
            "gram_TFLOPs": rows * k * (k + 1) / (t * 1e-3) / 1e12, "rel_diff_vs_device_gram": diff}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-extras", action="store_true", help="skip sweep, mixed and CPU legs")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device-to-device (reference for the HBM byte counters)")
    ap.add_argument("--leg", choices=["all", "sweep", "mixed", "post", "closure", "continuous"], default="all",
                    help="sweep: only the regularization sweep on reduced data of the same input; "
                         "mixed: only the reduced-precision forms against one float64 step; "
                         "post: one float64 step, then Step V and the streamed Gram; "
                         "closure: only the learned-closure leg; "
                         "continuous: one float64 step, then the continuous-time form and lifting "
                         "(each prints its JSON object; for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the row sharding over "
              f"several GPUs is designed but not built).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2504_14338_amd as dp
    dp.load()
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written by one copy kernel")
        del src, dst
    if args.leg == "closure":
        print(json.dumps({"closure": closure_bench(dp, torch, dev)}), flush=True)
        return
    m, Q, var_rows = make_c2(torch, dev)
    n, k = Q.shape
    torch.cuda.synchronize()
    log(f"input ready: {n} x {k} float64")
    if args.leg == "sweep":
        mean, scale, _ = dp.preprocess(Q, var_rows)
        D = dp.gram(Q, mean, scale, var_rows)
        del Q
        _, _, Qh80, _, _ = dp.reduce(D, r=80, want_tr=False)
        torch.cuda.synchronize()
        log("reduced data at r = 80 ready")
        print(json.dumps({"sweep": sweep_bench(dp, torch, Qh80.contiguous(), reps=max(1, args.steps))}), flush=True)
        return
    if args.leg == "mixed":
        timer = Timer(torch)
        res = pipeline_step(dp, Q, var_rows, timer)
        lam_full = dp.reduce(res["D"], r=60, want_tr=False)[0]
        t64 = timer.ms("preprocess") + timer.ms("gram") + timer.ms("reduce")
        log("float64 reference step done")
        print(json.dumps({"mixed": mixed_bench(dp, torch, Q, var_rows, res["Qhat"], lam_full, t64)}), flush=True)
        return

    if args.leg == "continuous":
        timer = Timer(torch)
        res = pipeline_step(dp, Q, var_rows, timer)
        log("float64 step done")
        print(json.dumps({"continuous": continuous_bench(dp, torch, Q, var_rows, res["Qhat"])}), flush=True)
        return

    if args.leg == "post":
        timer = Timer(torch)
        res = pipeline_step(dp, Q, var_rows, timer)
        traj = rollout_2000(dp, res["Qhat"], n_states=4000)
        log("float64 step done")
        out = {"postprocess": postprocess_bench(dp, torch, Q, res["mean"], res["scale"], var_rows, res["Tr"], traj)}
        log("postprocess done")
        out["stream"] = stream_bench(dp, torch, Q, var_rows)
        print(json.dumps(out), flush=True)
        return

    timer = Timer(torch)
    for _ in range(args.warmup):
        pipeline_step(dp, Q, var_rows, timer)
    torch.cuda.synchronize()
    timer.reset()
    t0 = time.perf_counter()
    res = None
    for s in range(args.steps):
        res = pipeline_step(dp, Q, var_rows, timer)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    phases = {p: timer.ms(p) for p in ("preprocess", "gram", "reduce", "infer", "rollout")}
    gram_flops = n * k * (k + 1)
    gram_tf = gram_flops / (phases["gram"] * 1e-3) / 1e12
    info = int(res["info"].item())
    status = int(res["status"].item())
    outc = res["out"]
    log("phases ms:", {p: round(v, 3) for p, v in phases.items()}, "info", info, "status", status)
    # the full tridiagonal eigensolver on the same D, beside the step
    tfull = Timer(torch)
    for _ in range(3):
        tfull.reset()
        lam_full = tfull.run("reduce_full", lambda: dp.reduce(res["D"], r=60))[0]
    reduce_full_ms = tfull.ms("reduce_full")

    line = {
        "metric": METRIC,
        "value": round(gram_tf, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "plain FP64 dOpInf at one GPU's share: n=4,000,000 (4 variables x 1,000,000 cells) "
                               "x k=2,000 travelling/standing-wave snapshots, r=60, d=1891, 4000-state rollout",
                   "n": n, "k": k, "r": 60, "beta1": 1e-2, "beta2": 1e8, "n_states": 4000},
        "pct_mfma_peak": round(100 * gram_tf / FP64_PEAK, 2),
        "phase_ms": {p: round(v, 3) for p, v in phases.items()},
        "reduce": {"partial_ms": round(phases["reduce"], 3), "subspace_iterations": res["iters"],
                   "full_eigensolver_ms": round(reduce_full_ms, 3)},
        "roofline": {
            "bound": "mfma",
            "achieved": round(gram_tf, 3),
            "peak": FP64_PEAK,
            "unit": "TFLOP/s",
            "frac": round(gram_tf / FP64_PEAK, 4),
            "traffic": measured_traffic(),
            "traffic_unit": "bytes per Gram call (HBM read + write of both launches, rocprofv3 counters)",
            "kernel": "gram_f64_dma_kernel: launch below the diagonal + diagonal launch (+ the split reduction)",
            "per_launch_flops": gram_flops,
        },
        "preprocess_GBps": round(n * k * 8 / (phases["preprocess"] * 1e-3) / 1e9, 1),
        "step_checks": {"reduce_info": info, "solve_status": status,
                        "outcome": int(outc["outcome"].item()), "train_err": float(outc["train_err"].item()),
                        "growth": float(outc["growth"].item())},
    }
    if not args.no_extras:
        # batched sweep on Qhat at r = 80 from the same data
        D = res["D"]
        lam80, _, Qh80, info80, _ = dp.reduce(D, r=80, want_tr=False)
        Qh80 = Qh80.contiguous()
        torch.cuda.synchronize()
        try:
            line["sweep"] = sweep_bench(dp, torch, Qh80)
        except Exception as e:  # report, do not hide
            line["sweep"] = {"error": repr(e)}
        log("sweep done")
        t64 = phases["preprocess"] + phases["gram"] + phases["reduce"]
        try:
            line["mixed"] = mixed_bench(dp, torch, Q, var_rows, res["Qhat"], lam_full, t64)
        except Exception as e:
            line["mixed"] = {"error": repr(e)}
        log("mixed done")
        try:
            traj = rollout_2000(dp, res["Qhat"], n_states=4000)
            line["postprocess"] = postprocess_bench(dp, torch, Q, res["mean"], res["scale"], var_rows, res["Tr"], traj)
        except Exception as e:
            line["postprocess"] = {"error": repr(e)}
        log("postprocess done")
        try:
            line["stream"] = stream_bench(dp, torch, Q, var_rows)
        except Exception as e:
            line["stream"] = {"error": repr(e)}
        log("stream done")
        try:
            line["continuous"] = continuous_bench(dp, torch, Q, var_rows, res["Qhat"])
        except Exception as e:
            line["continuous"] = {"error": repr(e)}
        log("continuous done")
        try:
            line["cpu_baseline"] = cpu_baseline(Q, var_rows, args.cpu_seconds, D=D, Qh80=Qh80)
        except Exception as e:
            line["cpu_baseline"] = {"error": repr(e)}
        log("cpu baseline done")
        del Q, res, D
        torch.cuda.empty_cache()
        try:
            line["closure"] = closure_bench(dp, torch, dev)
        except Exception as e:
            line["closure"] = {"error": repr(e)}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
