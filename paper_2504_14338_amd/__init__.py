"""dOpInf hot path on one MI355X: thin ctypes binding over libdopinf.so.

Every function here only marshals arguments (device pointers of torch
tensors, the current HIP stream, a workspace tensor) into the C ABI declared
in include/dopinf.h; all arithmetic runs in the library's HIP kernels.  The
binding refuses to run when the library is missing: there is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

__all__ = [
    "load", "DopinfError", "CENTER", "SCALE", "APPLY", "F64", "F32",
    "GRAM_NATIVE", "GRAM_BF16X3", "GRAM_BF16X6", "GRAM_I8X6", "ITEM_PASS", "ITEM_NONFINITE",
    "ITEM_GROWTH", "ITEM_SOLVE", "ITEM_TIMEOUT", "preprocess", "gram", "cross_gram",
    "reduce", "infer", "operator_offset", "rollout", "traj_offset",
    "n_quad", "lib_path", "rollout_noalloc", "rollout_noalloc_max_bytes", "postprocess", "reduce_topr", "preprocess_stream", "gram_stream", "lift", "infer_continuous",
    "rollout_continuous", "LIFT_COPY", "LIFT_PRODUCT", "LIFT_RECIPROCAL", "closure_param_count", "rom_residuals", "closure_fit", "closure_norms",
    "closure_grad", "closure_eval", "closure_rollout", "TUNE_CHOL_KB", "tune_set", "tune_get",
    "autotune_candidates", "autotune_infer", "Sweep", "TUNE_TRSM_KB", "TUNE_CHOL_KB2", "TUNE_TRSM_KB2",
]

OK, E_ARG, E_HIP, E_WORKSPACE, E_RANK, E_NOTSPD, E_NONFINITE, E_NOSTABLE, E_TIMEOUT = range(9)
F64, F32 = 0, 1
CENTER, SCALE, APPLY = 1, 2, 4
GRAM_NATIVE, GRAM_BF16X3, GRAM_BF16X6, GRAM_I8X6 = 0, 1, 2, 3
ITEM_PASS, ITEM_NONFINITE, ITEM_GROWTH, ITEM_SOLVE, ITEM_TIMEOUT = 0, 1, 2, 3, 4
ROLLOUT_FULL = 1
ROLLOUT_ONE_WG = 2
TUNE_CHOL_KB = 1
TUNE_TRSM_KB = 2
TUNE_CHOL_KB2 = 3
TUNE_TRSM_KB2 = 4
SWEEP_AUTOTUNE = 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib_path() -> str:
    return os.path.join(_HERE, "libdopinf.so")


class DopinfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dopinf error {code}: {msg}")
        self.code = code


_vp, _i64, _i32, _u32, _f64, _sz = C.c_void_p, C.c_int64, C.c_int, C.c_uint, C.c_double, C.c_size_t
_SIGS = {
    "dopinf_last_error": ([], C.c_char_p),
    "dopinf_version": ([], C.c_char_p),
    "dopinf_preprocess_workspace": ([_i64, _i64, _i32], _sz),
    "dopinf_preprocess": ([_vp, _i32, _vp, _i64, _i64, _i64, _i32, _vp, _u32, _vp, _vp, _vp, _vp, _vp, _sz], _i32),
    "dopinf_gram_workspace": ([_i32, _i32, _i64, _i64], _sz),
    "dopinf_gram": ([_vp, _i32, _i32, _vp, _i64, _i64, _i64, _vp, _vp, _i32, _vp, _vp, _i64, _vp, _sz], _i32),
    "dopinf_cross_gram_workspace": ([_i64, _i64, _i64], _sz),
    "dopinf_cross_gram": ([_vp, _vp, _i64, _vp, _i64, _i64, _i64, _i64, _vp, _vp, _i32, _vp, _vp, _i64, _vp, _sz],
                          _i32),
    "dopinf_reduce_workspace": ([_i64, _i32], _sz),
    "dopinf_reduce": ([_vp, _vp, _i64, _i64, _i32, _f64, _i32, _vp, _vp, _vp, _i64, _vp, _i64, _vp, _vp, _sz], _i32),
    "dopinf_stream_workspace": ([_i64, _i64, _i32], _sz),
    "dopinf_preprocess_stream": ([_vp, _vp, _i64, _i64, _i64, _i32, _vp, _u32, _vp, _vp, _vp, _vp, _i64, _vp, _sz],
                                 _i32),
    "dopinf_gram_stream": ([_vp, _vp, _i64, _i64, _i64, _vp, _vp, _i32, _vp, _vp, _i64, _i64, _vp, _sz], _i32),
    "dopinf_reduce_topr_workspace": ([_i64, _i32], _sz),
    "dopinf_reduce_topr": ([_vp, _vp, _i64, _i64, _i32, _vp, _vp, _i64, _vp, _i64, _vp, _vp, _vp, _sz], _i32),
    "dopinf_operator_offset": ([_i32, _vp, _i32, _i32], _sz),
    "dopinf_infer_workspace": ([_i64, _i32, _vp, _i32], _sz),
    "dopinf_infer": ([_vp, _vp, _i64, _i64, _i32, _vp, _i32, _vp, _vp, _vp, _vp, _vp, _sz], _i32),
    "dopinf_traj_offset": ([_i32, _vp, _i32, _i32, _i32], _sz),
    "dopinf_rollout_workspace": ([_i32, _vp, _i32, _i64], _sz),
    "dopinf_rollout": ([_vp, _i32, _vp, _i32, _vp, _vp, _i64, _vp, _i64, _i32, _f64, _u32, _vp, _vp, _vp, _vp, _vp, _vp,
                        _vp, _sz], _i32),
    "dopinf_lift": ([_vp, _vp, _i64, _i64, _i64, _i32, _i32, _vp, _vp, _i64], _i32),
    "dopinf_infer_continuous_workspace": ([_i64, _i32, _vp, _i32], _sz),
    "dopinf_infer_continuous": ([_vp, _vp, _i64, _i64, _f64, _i32, _vp, _i32, _vp, _vp, _vp, _vp, _vp, _sz], _i32),
    "dopinf_rollout_continuous": ([_vp, _i32, _vp, _i32, _vp, _vp, _i64, _i64, _i32, _f64, _f64, _u32, _vp, _vp, _vp,
                                   _vp, _vp, _vp, _vp, _sz], _i32),
    "dopinf_postprocess": ([_vp, _i32, _vp, _i64, _i64, _i64, _vp, _vp, _i32, _vp, _vp, _i64, _vp, _i64, _i32, _vp,
                            _i64, _i64, _vp, _i64, _vp, _i64, _vp], _i32),
    "dopinf_rollout_noalloc_max_bytes": ([], _sz),
    "dopinf_rollout_noalloc": ([_vp, _i32, _vp, _i32, _vp, _vp, _i64, _i64, _i32, _f64, _u32, _vp, _vp, _vp, _vp, _vp,
                                _vp], _i32),
    "dopinf_tune_set": ([_i32, _i64, _i32], _i32),
    "dopinf_tune_get": ([_i32, _i64], _i32),
    "dopinf_autotune_candidates": ([_i32, _vp, _i32], _i32),
    "dopinf_autotune_infer": ([_vp, _vp, _i64, _i64, _i32, _vp, _i32, _vp, _vp, _vp, _vp, _vp, _sz, _vp], _i32),
    "dopinf_sweep_workspace": ([_i64, _i32, _vp, _i32], _sz),
    "dopinf_sweep_create": ([_vp, _vp, _i64, _i64, _i32, _vp, _i32, _vp, _vp, _i32, _f64, _u32, _vp, _vp, _vp, _vp,
                             _vp, _vp, _vp, _sz, _vp], _i32),
    "dopinf_sweep_launch": ([_vp, _vp], _i32),
    "dopinf_sweep_destroy": ([_vp], _i32),
    "dopinf_closure_param_count": ([_i32], _i64),
    "dopinf_rom_residuals": ([_vp, _vp, _i32, _vp, _i64, _i64, _vp], _i32),
    "dopinf_closure_fit_workspace": ([_i32, _i64], _sz),
    "dopinf_closure_fit": ([_vp, _i32, _vp, _vp, _i64, _i32, _i32, _f64, _f64, _f64, _f64, _vp, _vp, _vp, _vp, _vp,
                            _vp, _sz], _i32),
    "dopinf_closure_norms": ([_vp, _i32, _vp, _vp, _i64, _vp], _i32),
    "dopinf_closure_grad": ([_vp, _i32, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _sz], _i32),
    "dopinf_closure_eval_workspace": ([_i64], _sz),
    "dopinf_closure_eval": ([_vp, _i32, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _sz], _i32),
    "dopinf_closure_rollout_workspace": ([_i32], _sz),
    "dopinf_closure_rollout": ([_vp, _i32, _vp, _vp, _vp, _f64, _vp, _i64, _i32, _vp, _i64, _i64, _f64, _vp, _vp, _vp,
                                _vp, _vp, _vp, _sz], _i32),
}


def load():
    """Load libdopinf.so (built by ``python -m paper_2504_14338_amd.build``)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    p = lib_path()
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_2504_14338_amd.build`")
    lib = C.CDLL(p)
    for name, (args, res) in _SIGS.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.argtypes = args
        fn.restype = res
    _LIB = lib
    return lib


def exported_symbols():
    lib = load()
    return {name for name in _SIGS if hasattr(lib, name)}


def _check(rc):
    if rc != OK:
        raise DopinfError(rc, load().dopinf_last_error().decode())


def _torch():
    import torch
    return torch


def _stream(dev):
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _ws(nbytes, dev):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=dev)


def _rowmajor(t, name):
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be a 2-D row-major tensor (unit column stride)")
    return t.stride(0)


def _host_i64(a):
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.int64))
    return arr, arr.ctypes.data_as(C.c_void_p)


def _host_i32(a):
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
    return arr, arr.ctypes.data_as(C.c_void_p)


def _host_f64(a):
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return arr, arr.ctypes.data_as(C.c_void_p)


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError("snapshot data must be float64 or float32")


def n_quad(r):
    return r * (r + 1) // 2


# ---------------------------------------------------------------- Step II ---
def preprocess(Q, var_rows, flags=CENTER | SCALE, info=None):
    """Per-row temporal means and per-variable scales; returns (mean, scale,
    zero_range).  `info` (optional device int32 tensor of one element)
    receives OK or E_NONFINITE."""
    torch = _torch()
    lib = load()
    n, k = Q.shape
    ldq = _rowmajor(Q, "Q")
    vr, vrp = _host_i64(var_rows)
    nvars = len(vr) - 1
    dev = Q.device
    mean = torch.empty(n, dtype=torch.float64, device=dev)
    scale = torch.empty(nvars, dtype=torch.float64, device=dev)
    zr = torch.empty(nvars, dtype=torch.int32, device=dev)
    nb = lib.dopinf_preprocess_workspace(n, k, nvars)
    ws = _ws(nb, dev)
    _check(lib.dopinf_preprocess(_stream(dev), _dtype_code(Q), _ptr(Q), n, k, ldq, nvars, vrp, flags, _ptr(mean),
                                 _ptr(scale), _ptr(zr), _ptr(info), _ptr(ws), ws.numel()))
    return mean, scale, zr


# --------------------------------------------------------------- Step III ---
def gram(Q, mean=None, scale=None, var_rows=None, algo=GRAM_NATIVE, out=None):
    """D = Qs^T Qs with Qs = (Q - mean) / scale formed on load."""
    torch = _torch()
    lib = load()
    n, k = Q.shape
    ldq = _rowmajor(Q, "Q")
    dev = Q.device
    D = out if out is not None else torch.empty((k, k), dtype=torch.float64, device=dev)
    ldd = _rowmajor(D, "D")
    if var_rows is None:
        var_rows = [0, n]
    vr, vrp = _host_i64(var_rows)
    nb = lib.dopinf_gram_workspace(_dtype_code(Q), algo, n, k)
    ws = _ws(nb, dev)
    _check(lib.dopinf_gram(_stream(dev), _dtype_code(Q), algo, _ptr(Q), n, k, ldq, _ptr(mean), _ptr(scale),
                           len(vr) - 1, vrp, _ptr(D), ldd, _ptr(ws), ws.numel()))
    return D


def cross_gram(X, Y, out=None, mean=None, scale=None, var_rows=None):
    """C = Xs^T Ys for float64 X (n x mx), Y (n x my); with mean / scale both
    are centered and scaled on load with the same statistics."""
    torch = _torch()
    lib = load()
    n, mx = X.shape
    my = Y.shape[1]
    if Y.shape[0] != n:
        raise ValueError("X and Y need the same number of rows")
    dev = X.device
    Cm = out if out is not None else torch.empty((mx, my), dtype=torch.float64, device=dev)
    if var_rows is None:
        var_rows = [0, n]
    vr, vrp = _host_i64(var_rows)
    nb = lib.dopinf_cross_gram_workspace(n, mx, my)
    ws = _ws(nb, dev)
    _check(lib.dopinf_cross_gram(_stream(dev), _ptr(X), _rowmajor(X, "X"), _ptr(Y), _rowmajor(Y, "Y"), n, mx, my,
                                 _ptr(mean), _ptr(scale), len(vr) - 1, vrp, _ptr(Cm), _rowmajor(Cm, "C"), _ptr(ws),
                                 ws.numel()))
    return Cm


def reduce(D, r=0, tau=0.9996, r_max=None, want_tr=True):
    """Eigenvalues (descending), T_r and Qhat = Lambda_r^{1/2} U_r^T.

    Returns (lam, Tr, Qhat, info, r); info is a device int tensor.
    """
    torch = _torch()
    lib = load()
    k = D.shape[0]
    dev = D.device
    if r_max is None:
        r_max = r if r > 0 else k
    lam = torch.empty(k, dtype=torch.float64, device=dev)
    Qhat = torch.empty((r_max, k), dtype=torch.float64, device=dev)
    Tr = torch.empty((k, r_max), dtype=torch.float64, device=dev) if want_tr else None
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    nb = lib.dopinf_reduce_workspace(k, r_max)
    ws = _ws(nb, dev)
    r_out = C.c_int(0)
    _check(lib.dopinf_reduce(_stream(dev), _ptr(D), k, _rowmajor(D, "D"), int(r), float(tau), int(r_max),
                             C.byref(r_out), _ptr(lam), _ptr(Tr), r_max if Tr is not None else 0, _ptr(Qhat), k,
                             _ptr(info), _ptr(ws), ws.numel()))
    rr = r_out.value
    return lam, (Tr[:, :rr] if Tr is not None else None), Qhat[:rr], info, rr


def preprocess_stream(Q_h, var_rows, chunk_rows, flags=CENTER | SCALE, device="cuda", info=None):
    """dopinf_preprocess_stream on a host (ideally pinned) float64 tensor;
    returns (mean, scale, zero_range) on the device."""
    torch = _torch()
    lib = load()
    dev = torch.device(device)
    n, k = Q_h.shape
    vr, vrp = _host_i64(var_rows)
    nvars = len(vr) - 1
    mean = torch.empty(n, dtype=torch.float64, device=dev)
    scale = torch.empty(nvars, dtype=torch.float64, device=dev)
    zr = torch.empty(nvars, dtype=torch.int32, device=dev)
    ws = _ws(lib.dopinf_stream_workspace(chunk_rows, k, nvars), dev)
    _check(lib.dopinf_preprocess_stream(_stream(dev), _ptr(Q_h), n, k, _rowmajor(Q_h, "Q_h"), nvars, vrp, flags,
                                        _ptr(mean), _ptr(scale), _ptr(zr), _ptr(info), int(chunk_rows), _ptr(ws),
                                        ws.numel()))
    return mean, scale, zr


def gram_stream(Q_h, chunk_rows, mean=None, scale=None, var_rows=None, device="cuda", out=None, ws=None):
    """dopinf_gram_stream: D of a host float64 matrix streamed in chunks."""
    torch = _torch()
    lib = load()
    dev = torch.device(device)
    n, k = Q_h.shape
    if var_rows is None:
        var_rows = [0, n]
    vr, vrp = _host_i64(var_rows)
    D = out if out is not None else torch.empty((k, k), dtype=torch.float64, device=dev)
    if ws is None:
        ws = _ws(lib.dopinf_stream_workspace(chunk_rows, k, len(vr) - 1), dev)
    _check(lib.dopinf_gram_stream(_stream(dev), _ptr(Q_h), n, k, _rowmajor(Q_h, "Q_h"), _ptr(mean), _ptr(scale),
                                  len(vr) - 1, vrp, _ptr(D), _rowmajor(D, "D"), int(chunk_rows), _ptr(ws),
                                  ws.numel()))
    return D


def reduce_topr(D, r, want_tr=True):
    """Partial eigendecomposition for a prescribed r: returns (lam_r, Tr,
    Qhat, info, iters) with iters = subspace iterations (0: full solver)."""
    torch = _torch()
    lib = load()
    k = D.shape[0]
    dev = D.device
    lam = torch.empty(r, dtype=torch.float64, device=dev)
    Qhat = torch.empty((r, k), dtype=torch.float64, device=dev)
    Tr = torch.empty((k, r), dtype=torch.float64, device=dev) if want_tr else None
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = _ws(lib.dopinf_reduce_topr_workspace(k, r), dev)
    iters = C.c_int(0)
    _check(lib.dopinf_reduce_topr(_stream(dev), _ptr(D), k, _rowmajor(D, "D"), int(r), _ptr(lam), _ptr(Tr),
                                  r if Tr is not None else 0, _ptr(Qhat), k, _ptr(info), C.byref(iters), _ptr(ws),
                                  ws.numel()))
    return lam, Tr, Qhat, info, iters.value


# ---------------------------------------------------------------- Step IV ---
def operator_offset(r_list, n_pairs, item):
    rl, rlp = _host_i32(r_list)
    return load().dopinf_operator_offset(len(rl), rlp, n_pairs, item)


def infer(Qhat, r_list, beta1, beta2):
    """Operators for every (r in r_list) x (beta1[p], beta2[p]) item.

    Returns (O_flat, status, views) where views[g][p] is the r x d operator
    of group g, pair p (a view into O_flat).
    """
    torch = _torch()
    lib = load()
    dev = Qhat.device
    k = Qhat.shape[1]
    rl, rlp = _host_i32(r_list)
    b1, b1p = _host_f64(beta1)
    b2, b2p = _host_f64(beta2)
    n_pairs = len(b1)
    if len(b2) != n_pairs:
        raise ValueError("beta1 and beta2 must have the same length")
    n_items = len(rl) * n_pairs
    total = lib.dopinf_operator_offset(len(rl), rlp, n_pairs, n_items)
    O = torch.empty(total, dtype=torch.float64, device=dev)
    status = torch.empty(n_items, dtype=torch.int32, device=dev)
    nb = lib.dopinf_infer_workspace(k, len(rl), rlp, n_pairs)
    ws = _ws(nb, dev)
    _check(lib.dopinf_infer(_stream(dev), _ptr(Qhat), _rowmajor(Qhat, "Qhat"), k, len(rl), rlp, n_pairs, b1p, b2p,
                            _ptr(O), _ptr(status), _ptr(ws), ws.numel()))
    views = []
    for g, r in enumerate(rl):
        d = int(r) + n_quad(int(r)) + 1
        row = []
        for p in range(n_pairs):
            off = lib.dopinf_operator_offset(len(rl), rlp, n_pairs, g * n_pairs + p)
            row.append(O[off:off + int(r) * d].view(int(r), d))
        views.append(row)
    return O, status, views


def traj_offset(r_list, n_pairs, n_states, item):
    rl, rlp = _host_i32(r_list)
    return load().dopinf_traj_offset(len(rl), rlp, n_pairs, n_states, item)


def rollout(O, Qhat, r_list, n_pairs, n_states, k_train=None, max_growth=1.2, solve_status=None,
            keep_traj=False, full=False, one_wg=False, q0=None):
    """Roll out, score and select.  Returns dict of device tensors.  Few items
    are rolled out by teams of workgroups unless one_wg is set.  q0: None
    (every item starts at Qhat[:, 0]) or a float64 device vector of the
    items' initial states packed in item order (r_g entries each)."""
    torch = _torch()
    lib = load()
    dev = O.device
    rl, rlp = _host_i32(r_list)
    n_items = len(rl) * n_pairs
    if k_train is None:
        k_train = Qhat.shape[1]
    traj = None
    if keep_traj:
        total = lib.dopinf_traj_offset(len(rl), rlp, n_pairs, n_states, n_items)
        traj = torch.empty(total, dtype=torch.float64, device=dev)
    te = torch.empty(n_items, dtype=torch.float64, device=dev)
    gr = torch.empty(n_items, dtype=torch.float64, device=dev)
    oc = torch.empty(n_items, dtype=torch.int32, device=dev)
    best = torch.empty(len(rl), dtype=torch.int32, device=dev)
    nb = lib.dopinf_rollout_workspace(len(rl), rlp, n_pairs, k_train)
    ws = _ws(nb, dev)
    if q0 is not None:
        need = lib.dopinf_traj_offset(len(rl), rlp, n_pairs, 1, n_items)
        if q0.dtype != torch.float64 or q0.numel() != need or not q0.is_contiguous():
            raise ValueError(f"q0 must be a contiguous float64 tensor of {need} entries")
    _check(lib.dopinf_rollout(_stream(dev), len(rl), rlp, n_pairs, _ptr(O), _ptr(Qhat), _rowmajor(Qhat, "Qhat"),
                              _ptr(q0), k_train, n_states, float(max_growth), (ROLLOUT_FULL if full else 0) | (ROLLOUT_ONE_WG if one_wg else 0),
                              _ptr(solve_status), _ptr(traj), _ptr(te), _ptr(gr), _ptr(oc), _ptr(best), _ptr(ws),
                              ws.numel()))
    out = {"train_err": te, "growth": gr, "outcome": oc, "best": best, "traj": traj}
    if keep_traj:
        views = []
        for g, r in enumerate(rl):
            row = []
            for p in range(n_pairs):
                off = lib.dopinf_traj_offset(len(rl), rlp, n_pairs, n_states, g * n_pairs + p)
                row.append(traj[off:off + n_states * int(r)].view(n_states, int(r)))
            views.append(row)
        out["traj_views"] = views
    return out


LIFT_COPY, LIFT_PRODUCT, LIFT_RECIPROCAL = 0, 1, 2


def lift(Q, n_cells, spec):
    """Lifted variables (Sec. 3.3): spec = [(op, a, b), ...] over the input
    variables (blocks of n_cells rows of Q); returns len(spec) blocks."""
    torch = _torch()
    lib = load()
    n, k = Q.shape
    sp = np.asarray(spec, dtype=np.int32).reshape(-1, 3)
    sp_c, sp_p = _host_i32(sp.ravel())
    L = torch.empty((len(sp) * n_cells, k), dtype=torch.float64, device=Q.device)
    _check(lib.dopinf_lift(_stream(Q.device), _ptr(Q), n_cells, k, _rowmajor(Q, "Q"), n // n_cells, len(sp), sp_p,
                           _ptr(L), k))
    return L


def infer_continuous(Qhat, dt, r_list, beta1, beta2):
    """Continuous-time operators (Eq. (10)) from finite-difference derivative
    data at spacing dt; returns (O_flat, status, views) as infer()."""
    torch = _torch()
    lib = load()
    dev = Qhat.device
    k = Qhat.shape[1]
    rl, rlp = _host_i32(r_list)
    b1, b1p = _host_f64(beta1)
    b2, b2p = _host_f64(beta2)
    n_pairs = len(b1)
    if len(b2) != n_pairs:
        raise ValueError("beta1 and beta2 must have the same length")
    n_items = len(rl) * n_pairs
    total = lib.dopinf_operator_offset(len(rl), rlp, n_pairs, n_items)
    O = torch.empty(total, dtype=torch.float64, device=dev)
    status = torch.empty(n_items, dtype=torch.int32, device=dev)
    ws = _ws(lib.dopinf_infer_continuous_workspace(k, len(rl), rlp, n_pairs), dev)
    _check(lib.dopinf_infer_continuous(_stream(dev), _ptr(Qhat), _rowmajor(Qhat, "Qhat"), k, float(dt), len(rl), rlp,
                                       n_pairs, b1p, b2p, _ptr(O), _ptr(status), _ptr(ws), ws.numel()))
    views = []
    for g, r in enumerate(rl):
        d = int(r) + n_quad(int(r)) + 1
        row = []
        for p in range(n_pairs):
            off = lib.dopinf_operator_offset(len(rl), rlp, n_pairs, g * n_pairs + p)
            row.append(O[off:off + int(r) * d].view(int(r), d))
        views.append(row)
    return O, status, views


def rollout_continuous(O, Qhat, r_list, n_pairs, n_states, dt, k_train=None, max_growth=1.2, solve_status=None,
                       keep_traj=False, full=False, one_wg=False):
    """RK4 rollouts of continuous-time ROMs, scored like rollout() (one_wg:
    one workgroup per item instead of the multi-workgroup team form)."""
    torch = _torch()
    lib = load()
    dev = O.device
    rl, rlp = _host_i32(r_list)
    n_items = len(rl) * n_pairs
    if k_train is None:
        k_train = Qhat.shape[1]
    traj = None
    if keep_traj:
        traj = torch.empty(lib.dopinf_traj_offset(len(rl), rlp, n_pairs, n_states, n_items), dtype=torch.float64,
                           device=dev)
    te = torch.empty(n_items, dtype=torch.float64, device=dev)
    gr = torch.empty(n_items, dtype=torch.float64, device=dev)
    oc = torch.empty(n_items, dtype=torch.int32, device=dev)
    best = torch.empty(len(rl), dtype=torch.int32, device=dev)
    ws = _ws(lib.dopinf_rollout_workspace(len(rl), rlp, n_pairs, k_train), dev)
    _check(lib.dopinf_rollout_continuous(_stream(dev), len(rl), rlp, n_pairs, _ptr(O), _ptr(Qhat),
                                         _rowmajor(Qhat, "Qhat"), k_train, n_states, float(dt), float(max_growth),
                                         (ROLLOUT_FULL if full else 0) | (ROLLOUT_ONE_WG if one_wg else 0),
                                         _ptr(solve_status), _ptr(traj), _ptr(te),
                                         _ptr(gr), _ptr(oc), _ptr(best), _ptr(ws), ws.numel()))
    out = {"train_err": te, "growth": gr, "outcome": oc, "best": best, "traj": traj}
    if keep_traj:
        out["traj_views"] = [[traj[lib.dopinf_traj_offset(len(rl), rlp, n_pairs, n_states, g * n_pairs + p):][
            :n_states * int(r)].view(n_states, int(r)) for p in range(n_pairs)] for g, r in enumerate(rl)]
    return out


def postprocess(Q, Tr, rows=None, Qtilde=None, mean=None, scale=None, var_rows=None, m=None):
    """Step V: basis rows V (m x r) at `rows` (device int64 tensor, or None for
    rows 0..m-1) and, with Qtilde (r x N), the prediction s_v V Qtilde + mean
    in original coordinates.  Returns (V, pred or None, info)."""
    torch = _torch()
    lib = load()
    dev = Q.device
    n, k = Q.shape
    r = Tr.shape[1]
    if rows is not None:
        m = rows.numel()
    elif m is None:
        m = n
    dtype = F64 if Q.dtype == torch.float64 else F32
    V = torch.empty((m, r), dtype=torch.float64, device=dev)
    pred = None
    n_out = 0
    if Qtilde is not None:
        n_out = Qtilde.shape[1]
        pred = torch.empty((m, n_out), dtype=torch.float64, device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev)
    nv = 1
    vr_p = None
    if scale is not None:
        vr, vr_p = _host_i64(var_rows)
        nv = len(vr) - 1
    _check(lib.dopinf_postprocess(_stream(dev), dtype, _ptr(Q), n, k, _rowmajor(Q, "Q"), _ptr(mean), _ptr(scale),
                                  nv, vr_p, _ptr(rows), m, _ptr(Tr), _rowmajor(Tr, "Tr"), r, _ptr(Qtilde),
                                  _rowmajor(Qtilde, "Qtilde") if Qtilde is not None else 0, n_out, _ptr(V), r,
                                  _ptr(pred), n_out, _ptr(info)))
    return V, pred, info


def rollout_noalloc(O, Qhat, r_list, n_pairs, n_states, k_train=None, max_growth=1.2, solve_status=None,
                    full=False, one_wg=False, out=None):
    """dopinf_rollout_noalloc: rollout() with the library's fixed scratch
    instead of a workspace.  `out` (optional) holds preallocated result
    tensors (keys train_err, growth, outcome, best; traj is not kept), so a
    loop can run without any allocation."""
    torch = _torch()
    lib = load()
    dev = O.device
    rl, rlp = _host_i32(r_list)
    n_items = len(rl) * n_pairs
    if k_train is None:
        k_train = Qhat.shape[1]
    if out is None:
        out = {"train_err": torch.empty(n_items, dtype=torch.float64, device=dev),
               "growth": torch.empty(n_items, dtype=torch.float64, device=dev),
               "outcome": torch.empty(n_items, dtype=torch.int32, device=dev),
               "best": torch.empty(len(rl), dtype=torch.int32, device=dev)}
    _check(lib.dopinf_rollout_noalloc(_stream(dev), len(rl), rlp, n_pairs, _ptr(O), _ptr(Qhat),
                                      _rowmajor(Qhat, "Qhat"), k_train, n_states, float(max_growth),
                                      (ROLLOUT_FULL if full else 0) | (ROLLOUT_ONE_WG if one_wg else 0),
                                      _ptr(solve_status), None, _ptr(out["train_err"]), _ptr(out["growth"]),
                                      _ptr(out["outcome"]), _ptr(out["best"])))
    return out


def rollout_noalloc_max_bytes():
    return int(load().dopinf_rollout_noalloc_max_bytes())


# ------------------------------------------ tuning and the captured sweep ---
def tune_set(param, key, value):
    """Store a launch parameter (value 0 clears it) for problem size `key`."""
    _check(load().dopinf_tune_set(int(param), int(key), int(value)))


def tune_get(param, key):
    return int(load().dopinf_tune_get(int(param), int(key)))


def autotune_candidates(param=TUNE_CHOL_KB):
    """The autotuner's width candidates: outer widths for TUNE_CHOL_KB /
    TUNE_TRSM_KB, the matching inner widths (0: none) for TUNE_CHOL_KB2 /
    TUNE_TRSM_KB2."""
    lib = load()
    n = lib.dopinf_autotune_candidates(int(param), None, 0)
    if n < 0:
        _check(n)
    vals = (C.c_int * n)()
    lib.dopinf_autotune_candidates(int(param), vals, n)
    return [int(v) for v in vals]


def autotune_infer(Qhat, r_list, beta1, beta2):
    """infer() preceded by the autotuner: for every group the Cholesky widths
    and then the triangular-solve depths are timed and the fastest stored per
    factorization size.  Returns (O, status, views, times) with times (ms) an
    n_r x 2 x candidates array (Cholesky, solve)."""
    torch = _torch()
    lib = load()
    dev = Qhat.device
    k = Qhat.shape[1]
    rl, rlp = _host_i32(r_list)
    b1, b1p = _host_f64(beta1)
    b2, b2p = _host_f64(beta2)
    n_pairs = len(b1)
    if len(b2) != n_pairs:
        raise ValueError("beta1 and beta2 must have the same length")
    ncand = len(autotune_candidates(TUNE_CHOL_KB))
    times = np.zeros(len(rl) * 2 * ncand, dtype=np.float32)
    n_items = len(rl) * n_pairs
    O = torch.empty(lib.dopinf_operator_offset(len(rl), rlp, n_pairs, n_items), dtype=torch.float64, device=dev)
    status = torch.empty(n_items, dtype=torch.int32, device=dev)
    nb = lib.dopinf_infer_workspace(k, len(rl), rlp, n_pairs)
    ws = _ws(nb, dev)
    _check(lib.dopinf_autotune_infer(_stream(dev), _ptr(Qhat), _rowmajor(Qhat, "Qhat"), k, len(rl), rlp, n_pairs, b1p,
                                     b2p, _ptr(O), _ptr(status), _ptr(ws), ws.numel(),
                                     times.ctypes.data_as(C.c_void_p)))
    return O, status, _operator_views(O, rl, rlp, n_pairs), times.reshape(len(rl), 2, ncand)


def _operator_views(O, rl, rlp, n_pairs):
    lib = load()
    views = []
    for g, r in enumerate(rl):
        d = int(r) + n_quad(int(r)) + 1
        row = []
        for p in range(n_pairs):
            off = lib.dopinf_operator_offset(len(rl), rlp, n_pairs, g * n_pairs + p)
            row.append(O[off:off + int(r) * d].view(int(r), d))
        views.append(row)
    return views


class Sweep:
    """The regularization sweep (dopinf_infer + dopinf_rollout over every
    (r, beta1, beta2) item) captured once into a graph; launch() replays it.

    The outputs (O, status, views, train_err, growth, outcome, best) and the
    workspace are allocated here and stay fixed; Qhat is read at every
    replay, so new reduced data of the same shape may be written into it.
    Capture needs a stream other than the null stream: by default a new one.
    """

    def __init__(self, Qhat, r_list, beta1, beta2, n_states, max_growth=1.2, autotune=False, stream=None):
        torch = _torch()
        lib = load()
        dev = Qhat.device
        self.Qhat = Qhat
        k = Qhat.shape[1]
        self._rl, rlp = _host_i32(r_list)
        self._rlp = rlp
        b1, b1p = _host_f64(beta1)
        b2, b2p = _host_f64(beta2)
        n_pairs = len(b1)
        if len(b2) != n_pairs:
            raise ValueError("beta1 and beta2 must have the same length")
        n_r = len(self._rl)
        n_items = n_r * n_pairs
        self.n_pairs = n_pairs
        total = lib.dopinf_operator_offset(n_r, rlp, n_pairs, n_items)
        self.O = torch.empty(total, dtype=torch.float64, device=dev)
        self.status = torch.empty(n_items, dtype=torch.int32, device=dev)
        self.train_err = torch.empty(n_items, dtype=torch.float64, device=dev)
        self.growth = torch.empty(n_items, dtype=torch.float64, device=dev)
        self.outcome = torch.empty(n_items, dtype=torch.int32, device=dev)
        self.best = torch.empty(n_r, dtype=torch.int32, device=dev)
        nb = lib.dopinf_sweep_workspace(k, n_r, rlp, n_pairs)
        self._ws = _ws(nb, dev)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        handle = C.c_void_p()
        _check(lib.dopinf_sweep_create(C.c_void_p(self.stream.cuda_stream), _ptr(Qhat), _rowmajor(Qhat, "Qhat"), k,
                                       n_r, rlp, n_pairs, b1p, b2p, int(n_states), float(max_growth),
                                       SWEEP_AUTOTUNE if autotune else 0, _ptr(self.O), _ptr(self.status),
                                       _ptr(self.train_err), _ptr(self.growth), _ptr(self.outcome), _ptr(self.best),
                                       _ptr(self._ws), self._ws.numel(), C.byref(handle)))
        self._h = handle
        _LIVE_SWEEPS.add(self)
        self.views = []
        for g, r in enumerate(self._rl):
            d = int(r) + n_quad(int(r)) + 1
            row = []
            for p in range(n_pairs):
                off = lib.dopinf_operator_offset(n_r, rlp, n_pairs, g * n_pairs + p)
                row.append(self.O[off:off + int(r) * d].view(int(r), d))
            self.views.append(row)

    def launch(self, stream=None):
        """Replay the sweep on `stream` (default: the capture stream)."""
        if self._h is None:
            raise RuntimeError("sweep is closed")
        st = self.stream if stream is None else stream
        _check(load().dopinf_sweep_launch(self._h, C.c_void_p(st.cuda_stream)))

    def close(self):
        if self._h is not None:
            _check(load().dopinf_sweep_destroy(self._h))
            self._h = None

    def __del__(self):
        # no HIP call once the interpreter is shutting down: _close_sweeps
        # (an exit handler) has closed every live sweep before that
        if _SHUTTING_DOWN:
            return
        try:
            self.close()
        except Exception:
            pass


_LIVE_SWEEPS = weakref.WeakSet()
_SHUTTING_DOWN = False


@atexit.register
def _close_sweeps():
    """Release every captured sweep while the HIP runtime is still up."""
    global _SHUTTING_DOWN
    for sw in list(_LIVE_SWEEPS):
        try:
            sw.close()
        except Exception:
            pass
    _SHUTTING_DOWN = True


# ------------------------------------------------------- learned closure ---
def closure_param_count(r):
    return int(load().dopinf_closure_param_count(int(r)))


def rom_residuals(O, Qhat):
    """rho_t = qhat_{t+1} - f_ROM(qhat_t) for t = 0..k-2; O is r x d."""
    torch = _torch()
    lib = load()
    r, k = Qhat.shape
    R = torch.empty((k - 1, r), dtype=torch.float64, device=Qhat.device)
    _check(lib.dopinf_rom_residuals(_stream(Qhat.device), _ptr(O.contiguous()), r, _ptr(Qhat),
                                    _rowmajor(Qhat, "Qhat"), k, _ptr(R)))
    return R


def closure_fit(X, Y, params0, epochs, batch=256, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Train the MLP closure on (X, Y) rows (N x r float64).  Returns
    (params float32, norm float64 [mx|sx|my|sy], loss per epoch float32)."""
    torch = _torch()
    lib = load()
    N, r = X.shape
    dev = X.device
    P = closure_param_count(r)
    params = params0.to(device=dev, dtype=torch.float32).contiguous().clone()
    if params.numel() != P:
        raise ValueError(f"closure with r={r} has {P} parameters, got {params.numel()}")
    norm = torch.empty(4 * r, dtype=torch.float64, device=dev)
    m = torch.empty(P, dtype=torch.float32, device=dev)
    v = torch.empty(P, dtype=torch.float32, device=dev)
    log = torch.empty(max(epochs, 1), dtype=torch.float32, device=dev)
    ws = _ws(lib.dopinf_closure_fit_workspace(r, N), dev)
    _check(lib.dopinf_closure_fit(_stream(dev), r, _ptr(X.contiguous()), _ptr(Y.contiguous()), N, int(epochs),
                                  int(batch), float(lr), float(beta1), float(beta2), float(eps), _ptr(params),
                                  _ptr(norm), _ptr(m), _ptr(v), _ptr(log), _ptr(ws), ws.numel()))
    return params, norm, log[:epochs]


def closure_norms(X, Y):
    torch = _torch()
    N, r = X.shape
    norm = torch.empty(4 * r, dtype=torch.float64, device=X.device)
    _check(load().dopinf_closure_norms(_stream(X.device), r, _ptr(X.contiguous()), _ptr(Y.contiguous()), N,
                                       _ptr(norm)))
    return norm


def closure_grad(params, norm, X, Y):
    """Gradient (float32, packed like params) and loss of one batch (N <= 256)."""
    torch = _torch()
    lib = load()
    N, r = X.shape
    dev = X.device
    g = torch.empty(closure_param_count(r), dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    ws = _ws(lib.dopinf_closure_fit_workspace(r, N), dev)
    _check(lib.dopinf_closure_grad(_stream(dev), r, _ptr(params), _ptr(norm), _ptr(X.contiguous()),
                                   _ptr(Y.contiguous()), N, _ptr(g), _ptr(loss), _ptr(ws), ws.numel()))
    return g, loss


def closure_eval(params, norm, X):
    """g(x) rows (float64, physical units) and max ||g(x_row)||."""
    torch = _torch()
    lib = load()
    N, r = X.shape
    dev = X.device
    G = torch.empty((N, r), dtype=torch.float64, device=dev)
    gmax = torch.empty(1, dtype=torch.float64, device=dev)
    ws = _ws(lib.dopinf_closure_eval_workspace(N), dev)
    _check(lib.dopinf_closure_eval(_stream(dev), r, _ptr(params), _ptr(norm), _ptr(X.contiguous()), N, _ptr(G),
                                   _ptr(gmax), _ptr(ws), ws.numel()))
    return G, gmax


def closure_rollout(O, params, norm, threshold, q0, n_states, Qref, max_growth=1.2, keep_traj=False):
    """Ensemble rollouts q_{t+1} = f_ROM(q_t) + g(q_t) (threshold <= 0: plain ROM)."""
    torch = _torch()
    lib = load()
    M, r = q0.shape
    dev = q0.device
    k_ref = Qref.shape[1]
    traj = torch.empty((M, n_states, r), dtype=torch.float64, device=dev) if keep_traj else None
    err = torch.empty(M, dtype=torch.float64, device=dev)
    gr = torch.empty(M, dtype=torch.float64, device=dev)
    oc = torch.empty(M, dtype=torch.int32, device=dev)
    fb = torch.empty(M, dtype=torch.int32, device=dev)
    ws = _ws(lib.dopinf_closure_rollout_workspace(r), dev)
    _check(lib.dopinf_closure_rollout(_stream(dev), r, _ptr(O.contiguous()), _ptr(params), _ptr(norm),
                                      float(threshold), _ptr(q0.contiguous()), M, int(n_states), _ptr(Qref),
                                      _rowmajor(Qref, "Qref"), k_ref, float(max_growth), _ptr(traj), _ptr(err),
                                      _ptr(gr), _ptr(oc), _ptr(fb), _ptr(ws), ws.numel()))
    return {"traj": traj, "err": err, "growth": gr, "outcome": oc, "fallback_at": fb}
