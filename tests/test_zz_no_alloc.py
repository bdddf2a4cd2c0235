"""The allocation-free rollout (dopinf_rollout_noalloc, the library's fixed
per-GPU scratch) against dopinf_rollout with a caller workspace, through the
C ABI: two calls in a row, the second smaller, both bit for bit equal to the
workspace form (the same kernels on the same inputs)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.fixture(scope="module")
def small_qhat(gpu_lib):
    dp = gpu_lib
    Q, var_rows, _, _ = synth.c1_snapshots(seed=1)
    Qd = dev(Q)
    mean, scale, _ = dp.preprocess(Qd, var_rows)
    D = dp.gram(Qd, mean, scale, var_rows)
    _, _, Qhat, info, _ = dp.reduce(D, r=10)
    assert int(info.item()) == 0
    return Qhat.contiguous()


def _same(a, b):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    # NaN where both are NaN (early exits) counts as equal
    return a.shape == b.shape and np.array_equal(a, b, equal_nan=True)


def _both(dp, Qhat, r_list, b1, b2, n_states, full):
    import torch
    O, status, _ = dp.infer(Qhat, r_list, b1, b2)
    n_pairs = len(b1)
    ref = dp.rollout(O, Qhat, r_list, n_pairs, n_states, solve_status=status, full=full)
    got = dp.rollout_noalloc(O, Qhat, r_list, n_pairs, n_states, solve_status=status, full=full)
    torch.cuda.synchronize()
    for key in ("train_err", "growth", "outcome", "best"):
        assert _same(got[key], ref[key]), key
    return ref


def test_noalloc_rollout_matches_workspace_form(gpu_lib, small_qhat):
    dp = gpu_lib
    lib = dp.load()
    print("noalloc: max scratch", dp.rollout_noalloc_max_bytes(), flush=True)
    # call 1: 2 sizes x 150 pairs (one workgroup per candidate)
    b1 = np.repeat(np.logspace(-8, -2, 15), 10)
    b2 = np.tile(np.logspace(-6, 0, 10), 15)
    print("noalloc: call 1, r = [6, 10], 150 pairs, 1200 states", flush=True)
    ref = _both(dp, small_qhat, [6, 10], b1, b2, 1200, full=False)
    oc = ref["outcome"].cpu().numpy()
    assert (oc == dp.ITEM_PASS).any()
    # call 2, smaller: one size, 2 pairs (teams of workgroups), full horizon
    print("noalloc: call 2, r = [6], 2 pairs, 400 states", flush=True)
    _both(dp, small_qhat, [6], [1e-6, 1e-2], [1e-4, 1e-1], 400, full=True)
    # a call whose scratch exceeds the fixed array is refused, nothing enqueued
    import ctypes
    rl = (ctypes.c_int * 1)(80)
    n_big = 4000
    assert lib.dopinf_rollout_workspace(1, rl, n_big, 2000) > dp.rollout_noalloc_max_bytes()
    one = dev(np.zeros(8))
    onei = dev(np.zeros(8, dtype=np.int32))
    rc = lib.dopinf_rollout_noalloc(None, 1, rl, n_big, one.data_ptr(), one.data_ptr(), 2000, 2000, 10, 1.2, 0,
                                    None, None, one.data_ptr(), one.data_ptr(), onei.data_ptr(), onei.data_ptr())
    assert rc == dp.E_WORKSPACE
    assert "allocation-free" in lib.dopinf_last_error().decode()
