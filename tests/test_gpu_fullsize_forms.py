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


@pytest.mark.parametrize("algo_name", ["native", "bf16x3", "bf16x6"])
def test_fullsize_lowp_gram(gpu_lib, c3, algo_name):
    import torch
    dp = gpu_lib
    algo = {"native": dp.GRAM_NATIVE, "bf16x3": dp.GRAM_BF16X3, "bf16x6": dp.GRAM_BF16X6}[algo_name]
    tol = TOLS[algo_name]
    Q32, var_rows = c3["Q32"], c3["var_rows"]
    D = dp.gram(Q32, c3["mean32"], c3["scale32"], var_rows, algo=algo).cpu().numpy()
    assert np.array_equal(D, D.T)
    assert rel(D, c3["D64"]) <= tol + 2 * U32
    # sampled entries against the oracle's Gram of the float32 columns
    cols = np.array([0, 127, 128, 1023, 1500, 1919, 1920, 1999])
    Qc = Q32[:, torch.from_numpy(cols).cuda()].cpu().numpy().astype(np.float64)
    s_rows = np.repeat(c3["scale32"].cpu().numpy(), 1_000_000)
    Dref = orc.gram(orc.apply_statistics(Qc, c3["mean32"].cpu().numpy(), s_rows))
    cs = np.sqrt(np.outer(np.diag(Dref), np.diag(Dref)))
    assert np.max(np.abs(D[np.ix_(cols, cols)] - Dref) / cs) <= tol


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
    del Q
    torch.cuda.empty_cache()
    return dict(r=r, Qh=Qh, O=views[0][0].contiguous())


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
