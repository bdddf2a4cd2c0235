"""Parity of the two added forms at their full sizes:

* reduced-precision Gram (float32 data of the n = 4,000,000 x k = 2,000
  workload, 32 GB): every form's D against the float64 D of the same
  snapshots over the whole matrix (tolerance of the form plus 2 u32 for the
  rounding of the data to float32), and sampled entries against the oracle's
  Gram of the float32 columns themselves;
* learned closure at r = 40 on 4 variables x 250,000 cells x 2,000 snapshots:
  residuals, standardization, a gradient, one training epoch, the closure's
  outputs and 1,024 rollouts of 4,000 states, sampled against the oracle.

Tolerances are those derived in test_gpu_precision.py and test_gpu_closure.py,
except for the closure's outputs over many inputs: the GPU rounds each hidden
activation to bfloat16 from a float32 sum, the oracle from a float64 sum, so a
pre-activation within the sum's rounding error (~u32 sqrt(K)) of a bfloat16
midpoint rounds the other way, with probability ~u32 sqrt(K) / 2^-8 ~ 2e-4.
Over 1,999 inputs x 256 activations some hundred such flips occur; each moves
one input's output by ~2^-8 / sqrt(128) of its norm.  So per input: the
median relative error must be at the float32-sum level (< 1e-5), at most 5%
of the inputs may exceed it, and none may exceed 2^-6 (a few flips at once).
"""
import numpy as np
import pytest

import oracle as orc
import oracle.closure as cl
import synth

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
TOLS = {"native": 3e-5, "bf16x3": 2e-4, "bf16x6": 3e-5}
I8_ROW = 2.5e-7  # I8X6: |dD_jl| <= n I8_ROW a_j a_l (derived in test_gpu_precision.py)
ALGOS = {"native": 0, "bf16x3": 1, "bf16x6": 2, "i8x6": 3}


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def assert_closure_outputs_close(G, G_ref):
    e = np.linalg.norm(G - G_ref, axis=1) / np.maximum(np.linalg.norm(G_ref, axis=1), 1e-300)
    assert np.median(e) < 1e-5, np.median(e)
    assert np.mean(e > 1e-5) <= 0.05, np.mean(e > 1e-5)
    assert np.max(e) < 2.0 ** -6, np.max(e)


@pytest.fixture(scope="module")
def c3(gpu_lib):
    import torch
    dp = gpu_lib
    print("full size: 4,000,000 x 2,000 snapshots, float64 then float32", flush=True)
    m = synth.c2_modes(nvars=4, ncell=1_000_000, k=2000, n_modes=200, n_pairs=60, decay=40.0, seed=2)
    Q = synth.c2_snapshots(m, noise_var=1e-8, seed=2, device=torch.device("cuda:0"))
    var_rows = [v * 1_000_000 for v in range(5)]
    mean, scale, _ = dp.preprocess(Q, var_rows)
    D64 = dp.gram(Q, mean, scale, var_rows).cpu().numpy()
    Q32 = Q.to(torch.float32)
    del Q
    torch.cuda.empty_cache()
    mean32, scale32, _ = dp.preprocess(Q32, var_rows)
    yield dict(Q32=Q32, var_rows=var_rows, D64=D64, mean32=mean32, scale32=scale32)
    del Q32
    torch.cuda.empty_cache()


@pytest.mark.parametrize("algo_name", ["native", "bf16x3", "bf16x6", "i8x6"])
def test_fullsize_lowp_gram(gpu_lib, c3, algo_name):
    import torch
    dp = gpu_lib
    algo = ALGOS[algo_name]
    Q32, var_rows = c3["Q32"], c3["var_rows"]
    D = dp.gram(Q32, c3["mean32"], c3["scale32"], var_rows, algo=algo).cpu().numpy()
    assert np.array_equal(D, D.T)
    # sampled entries against the oracle's Gram of the float32 columns
    cols = np.array([0, 127, 128, 1023, 1500, 1919, 1920, 1999])
    Qc = Q32[:, torch.from_numpy(cols).cuda()].cpu().numpy().astype(np.float64)
    s_rows = np.repeat(c3["scale32"].cpu().numpy(), 1_000_000)
    Qs = orc.apply_statistics(Qc, c3["mean32"].cpu().numpy(), s_rows)
    Dref = orc.gram(Qs)
    if algo_name == "i8x6":
        a = np.max(np.abs(Qs), axis=0)
        assert np.max(np.abs(D[np.ix_(cols, cols)] - Dref) / (Qs.shape[0] * np.outer(a, a))) <= I8_ROW
        print(f"i8x6: D {rel(D, c3['D64']):.3g} from the float64 D", flush=True)
        return
    tol = TOLS[algo_name]
    assert rel(D, c3["D64"]) <= tol + 2 * U32
    cs = np.sqrt(np.outer(np.diag(Dref), np.diag(Dref)))
    assert np.max(np.abs(D[np.ix_(cols, cols)] - Dref) / cs) <= tol


def test_fullsize_lowp_against_oracle_of_rounded_data(gpu_lib, c3):
    """Each reduced-precision form against the oracle on the float32-rounded
    data (the reference that isolates the Gram's arithmetic): the oracle's
    Gram over all 4,000,000 rows accumulated in row chunks (Eq. (5)), its
    eigenpairs and Qhat at r = 60; the forms' D within their tolerance, and
    Qhat within 1e-6 for the forms that meet it (float32, split-BF16x6,
    int8 slices I8X6).
    Errors against the float64 data itself are the float64 path's, which is
    within 1e-12 (D) of the oracle, plus these."""
    import torch
    dp = gpu_lib
    Q32, var_rows = c3["Q32"], c3["var_rows"]
    mean = c3["mean32"].cpu().numpy()
    s_rows = np.repeat(c3["scale32"].cpu().numpy(), 1_000_000)
    Dref = np.zeros((2000, 2000))
    chunk = 250_000
    for r0 in range(0, 4_000_000, chunk):
        blk = Q32[r0:r0 + chunk].cpu().numpy().astype(np.float64)
        Dref += orc.gram(orc.apply_statistics(blk, mean[r0:r0 + chunk], s_rows[r0:r0 + chunk]))
        del blk
    lam_o, U_o = orc.eig_desc(Dref)
    _, Qh_o = orc.reduce_basis_free(lam_o, U_o, 60)
    sel = lam_o >= 1e-10 * lam_o[0]
    # I8X6 as a relative Frobenius bound: ||dD||_F <= n I8_ROW ||a||^2 with a
    # the column max-abs values (<= 1 after the per-variable max-abs scaling)
    amax = np.zeros(2000)
    for r0 in range(0, 4_000_000, chunk):
        blk = Q32[r0:r0 + chunk].cpu().numpy().astype(np.float64)
        amax = np.maximum(amax, np.max(np.abs(orc.apply_statistics(blk, mean[r0:r0 + chunk],
                                                                   s_rows[r0:r0 + chunk])), axis=0))
        del blk
    tols = dict(TOLS, i8x6=4_000_000 * I8_ROW * float(amax @ amax) / np.linalg.norm(Dref))
    for name in ("native", "bf16x3", "bf16x6", "i8x6"):
        D = dp.gram(Q32, c3["mean32"], c3["scale32"], var_rows, algo=ALGOS[name])
        lam, _, Qh, info, _ = dp.reduce(D, r=60, want_tr=False)
        torch.cuda.synchronize()
        Dn = D.cpu().numpy()
        assert rel(Dn, Dref) <= tols[name], (name, rel(Dn, Dref))
        ln = lam.cpu().numpy()
        lerr = np.abs(ln[sel] - lam_o[sel]) / lam_o[sel]
        qerr = rel(Qh.cpu().numpy(), Qh_o)
        print(f"{name}: D {rel(Dn, Dref):.3g}, lambda max {lerr.max():.3g} median {np.median(lerr):.3g}, "
              f"Qhat {qerr:.3g}", flush=True)
        if name in ("native", "bf16x6", "i8x6"):
            assert qerr <= 1e-6, (name, qerr)


@pytest.fixture(scope="module")
def c5(gpu_lib):
    import torch
    dp = gpu_lib
    r, k = 40, 2000
    m = synth.c2_modes(nvars=4, ncell=250_000, k=k, seed=2)
    var_rows = [0, 250_000, 500_000, 750_000, 1_000_000]
    Q = synth.c2_snapshots(m, noise_var=1e-8, seed=2, device=torch.device("cuda:0"))
    mean, scale, _ = dp.preprocess(Q, var_rows)
    lam, Tr, Qhat, info, _ = dp.reduce(dp.gram(Q, mean, scale, var_rows), r=r)
    Qh = Qhat.contiguous()
    O, status, views = dp.infer(Qh, [r], [1e-2], [1e8])
    assert int(status.item()) == 0 and int(info.item()) == 0
    # held-out snapshots at the half-sample times t = 2000.5 .. 3999.5 (the
    # training window's integer frequencies repeat every 2000 samples, so
    # whole-sample times would revisit training states), projected without a
    # basis: Qhat_test = T_r^T (Qs^T Qs_test) (Eq. (8), training statistics)
    Qt = synth.c2_snapshots(m, noise_var=1e-8, seed=3, device=torch.device("cuda:0"), t0=k + 0.5)
    C = dp.cross_gram(Q, Qt, mean=mean, scale=scale, var_rows=var_rows)
    Qh_test = dp.cross_gram(Tr.contiguous(), C).contiguous()
    del Q, Qt, C
    torch.cuda.empty_cache()
    return dict(r=r, Qh=Qh, O=views[0][0].contiguous(), Qh_test=Qh_test)


def test_fullsize_closure(gpu_lib, c5):
    import torch
    dp = gpu_lib
    r, Qh, O = c5["r"], c5["Qh"], c5["O"]
    Qhh, Oh = Qh.cpu().numpy(), O.cpu().numpy()
    # residuals of the ROM over all 1,999 training pairs
    X = Qh[:, :-1].T.contiguous()
    Y = dp.rom_residuals(O, Qh)
    Xh, Yh = X.cpu().numpy(), Y.cpu().numpy()
    Rref = cl.residuals(Oh, r, Qhh)
    assert np.max(np.abs(Yh - Rref)) <= 1e-10 * np.max(np.abs(Qhh))
    # standardization
    norm = dp.closure_norms(X, Y).cpu().numpy()
    mx, sx, my, sy = cl.standardization(Xh, Yh)
    assert np.all(np.abs(norm[:r] - mx) <= 1e-13 * sx) and np.all(np.abs(norm[2 * r:3 * r] - my) <= 1e-13 * sy)
    assert np.allclose(norm[r:2 * r], sx, rtol=1e-12) and np.allclose(norm[3 * r:], sy, rtol=1e-12)
    # gradient at the initial parameters on one batch of 256
    p0 = synth.mlp_init(r, seed=5)
    pd, nd = torch.from_numpy(p0).cuda(), torch.from_numpy(norm).cuda()
    g, loss = dp.closure_grad(pd, nd, X[:256].contiguous(), Y[:256].contiguous())
    loss_ref, g_ref = cl.loss_and_grad(p0.astype(np.float64), (Xh[:256] - mx) / sx, (Yh[:256] - my) / sy, r)
    assert float(loss.item()) == pytest.approx(loss_ref, rel=1e-5)
    assert rel(g.cpu().numpy(), g_ref) <= 1e-4
    # training as the benchmark runs it; the first epoch against the oracle's
    params, normt, log = dp.closure_fit(X, Y, torch.from_numpy(p0), epochs=200, batch=256, lr=1e-3)
    lg = log.cpu().numpy()
    assert np.all(np.isfinite(lg)) and lg[-1] < lg[0]
    _, _, log_ref = cl.fit(p0.astype(np.float64), Xh, Yh, r, epochs=1, batch=256, lr=1e-3)
    assert lg[0] == pytest.approx(log_ref[0], rel=1e-3)
    # the trained closure on every training input
    ph = params.cpu().numpy().astype(np.float64)
    nh = normt.cpu().numpy()
    norms = (nh[:r], nh[r:2 * r], nh[2 * r:3 * r], nh[3 * r:])
    G, gmax = dp.closure_eval(params, normt, X)
    G_ref = cl.closure_eval(ph, norms, Xh, r)
    assert_closure_outputs_close(G.cpu().numpy(), G_ref)
    thr = 3.0 * float(gmax.item())
    # 1,024 perturbed 4,000-state rollouts: plain ROM and closure, sampled
    M, n_states = 1024, 4000
    q0 = synth.perturbed_states(Qhh[:, 0], M, std=0.05, seed=5)
    q0d = torch.from_numpy(q0).cuda()
    out_p = dp.closure_rollout(O, params, normt, 0.0, q0d, n_states, Qh)
    out_c = dp.closure_rollout(O, params, normt, thr, q0d, n_states, Qh)
    assert np.all(out_p["fallback_at"].cpu().numpy() == -1)
    sample = [0, 517, 1023]
    short = dp.closure_rollout(O, params, normt, thr, q0d[sample].contiguous(), 6, Qh, keep_traj=True)
    plain = dp.closure_rollout(O, params, normt, 0.0, q0d[sample].contiguous(), n_states, Qh, keep_traj=True)
    for j, mm in enumerate(sample):
        ref = orc.rollout(Oh, r, q0[mm], n_states)
        tr = plain["traj"][j].cpu().numpy().T
        if np.all(np.isfinite(ref)):
            assert np.max(np.abs(tr - ref)) <= 1e-9 * np.max(np.abs(ref))
        refc, lat = cl.closure_rollout(Oh, r, ph, norms, thr, q0[mm], 6)
        trc = short["traj"][j].cpu().numpy().T
        if lat == -1:
            assert rel(trc, refc) <= 1e-4
    # every member of the closure ensemble ends with a defined outcome code
    oc_c = out_c["outcome"].cpu().numpy()
    assert oc_c.shape == (M,) and np.all((oc_c >= 0) & (oc_c <= 4))


def test_fullsize_closure_on_heldout_residuals(gpu_lib, c5):
    """The trained closure on snapshots it was not trained on: the one-step
    residual RMS of the method's own r = 40 ROM on held-out half-sample
    snapshots, without and with the closure, and the 2000-state held-out
    rollout errors.  On this workload the residual is not a function of the
    resolved state (the truncated modes are independent oscillators), so the
    closure does not generalize: measured 0.43 -> 0.69 (one step) and
    0.23 -> 0.33 (rollout), i.e. it hurts.  Asserted: the held-out residuals
    against the oracle and finite, reported numbers; the gain where the model
    error is a function of the state is asserted on the cubic oscillators
    (test_gpu_closure.py)."""
    import torch
    dp = gpu_lib
    r, Qh, O, Qt = c5["r"], c5["Qh"], c5["O"], c5["Qh_test"]
    X = Qh[:, :-1].T.contiguous()
    Y = dp.rom_residuals(O, Qh)
    p0 = torch.from_numpy(synth.mlp_init(r, seed=5))
    params, norm, log = dp.closure_fit(X, Y, p0, epochs=200, batch=256, lr=1e-3)
    Rt = dp.rom_residuals(O, Qt)
    Gt, _ = dp.closure_eval(params, norm, Qt[:, :-1].T.contiguous())
    rms_plain = float(torch.sqrt(torch.mean(Rt * Rt)).item())
    rms_closed = float(torch.sqrt(torch.mean((Rt - Gt) ** 2)).item())
    _, gmax = dp.closure_eval(params, norm, X)
    thr = 3.0 * float(gmax.item())
    q0t = Qt[:, 0].reshape(1, r).contiguous()
    e_c = float(dp.closure_rollout(O, params, norm, thr, q0t, 2000, Qt)["err"].item())
    e_p = float(dp.closure_rollout(O, params, norm, 0.0, q0t, 2000, Qt)["err"].item())
    print(f"held-out one-step residual RMS: plain {rms_plain:.4g}, closure {rms_closed:.4g}; "
          f"2000-state rollout error: plain {e_p:.4g}, closure {e_c:.4g}", flush=True)
    # the oracle's residuals of the same ROM on the same held-out data
    Rref = cl.residuals(O.cpu().numpy(), r, Qt.cpu().numpy())
    assert np.max(np.abs(Rt.cpu().numpy() - Rref)) <= 1e-10 * np.max(np.abs(Qt.cpu().numpy()))
    assert np.isfinite(rms_closed) and np.isfinite(rms_plain) and np.isfinite(e_c) and np.isfinite(e_p)
