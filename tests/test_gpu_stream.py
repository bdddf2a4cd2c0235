"""Out-of-core statistics and Gram (dopinf_preprocess_stream,
dopinf_gram_stream) through the C ABI: host-resident snapshots streamed in
row chunks (chunks straddling variable boundaries, a ragged last chunk, one
chunk, many chunks), against the oracle (D within 1e-12, Eq. (5)) and
against the one-shot device calls (means and scales bit for bit: the same
per-row kernels and an exact max)."""
import numpy as np
import pytest

import oracle as orc
import synth

pytestmark = pytest.mark.gpu


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def c1():
    Q, var_rows, _, _ = synth.c1_snapshots(seed=1)
    return Q, var_rows


@pytest.mark.parametrize("chunk", [1000, 37, 8192, 100000])
def test_stream_matches_oracle_and_device_calls(gpu_lib, c1, chunk):
    import torch
    dp = gpu_lib
    Q, var_rows = c1
    Qh = torch.from_numpy(Q).pin_memory()
    info = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    mean, scale, zr = dp.preprocess_stream(Qh, var_rows, chunk, info=info)
    D = dp.gram_stream(Qh, chunk, mean, scale, var_rows)
    Qd = Qh.cuda()
    mean1, scale1, zr1 = dp.preprocess(Qd, var_rows)
    D1 = dp.gram(Qd, mean1, scale1, var_rows)
    torch.cuda.synchronize()
    assert int(info.item()) == dp.OK
    assert torch.equal(mean, mean1) and torch.equal(scale, scale1) and torch.equal(zr, zr1)
    mu, s, Qs, _ = orc.preprocess(Q, var_rows)
    Dref = orc.gram(Qs)
    Dn = D.cpu().numpy()
    assert np.array_equal(Dn, Dn.T)
    assert rel(Dn, Dref) <= 1e-12
    assert rel(Dn, D1.cpu().numpy()) <= 1e-13


def test_stream_nonfinite_and_zero_range(gpu_lib):
    import torch
    dp = gpu_lib
    rng = np.random.default_rng(4)
    n, k = 3000, 50
    Q = rng.normal(size=(n, k))
    Q[1000:2000] = 3.0            # variable 1 constant: zero range
    Q[2500, 7] = np.nan           # variable 2 non-finite
    var_rows = [0, 1000, 2000, 3000]
    Qh = torch.from_numpy(Q).pin_memory()
    info = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    mean, scale, zr = dp.preprocess_stream(Qh, var_rows, 700, info=info)
    torch.cuda.synchronize()
    mu, s, _, zr_o = orc.preprocess(Q, var_rows)
    assert int(info.item()) == dp.E_NONFINITE
    sg = scale.cpu().numpy()
    assert zr.cpu().numpy().tolist() == [0, 1, 0] and zr_o[0] == 1
    assert sg[0] == s[0] and sg[1] == 1.0 and np.isnan(sg[2])


def test_stream_one_million_rows(gpu_lib):
    """1,000,000 x 2,000 float64 (16 GB) in pinned host memory, streamed in
    chunks of 65,536 rows, against the one-shot device Gram of the same bytes."""
    import time
    import torch
    dp = gpu_lib
    m = synth.c2_modes(nvars=4, ncell=250_000, k=2000, n_modes=200, n_pairs=60, decay=40.0, seed=2)
    Qd = synth.c2_snapshots(m, noise_var=1e-8, seed=2, device=torch.device("cuda:0"))
    var_rows = [v * 250_000 for v in range(5)]
    print("stream: copying 16 GB to pinned host memory", flush=True)
    Qh = torch.empty(Qd.shape, dtype=torch.float64, pin_memory=True)
    Qh.copy_(Qd)
    mean1, scale1, _ = dp.preprocess(Qd, var_rows)
    D1 = dp.gram(Qd, mean1, scale1, var_rows)
    torch.cuda.synchronize()
    mean, scale, _ = dp.preprocess_stream(Qh, var_rows, 65536)
    D = dp.gram_stream(Qh, 65536, mean, scale, var_rows)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    D = dp.gram_stream(Qh, 65536, mean, scale, var_rows, out=D)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"stream: Gram of 16 GB from host in {dt:.3f} s = {16e9 / dt / 1e9:.1f} GB/s", flush=True)
    assert torch.equal(mean, mean1) and torch.equal(scale, scale1)
    assert rel(D.cpu().numpy(), D1.cpu().numpy()) <= 1e-13
