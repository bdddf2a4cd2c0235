"""dOpInf hot path on one MI355X: thin ctypes binding over libdopinf.so.

Every function here only marshals arguments (device pointers of torch
tensors, the current HIP stream, a workspace tensor) into the C ABI declared
in include/dopinf.h; all arithmetic runs in the library's HIP kernels.  The
binding refuses to run when the library is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

__all__ = [
    "load", "DopinfError", "CENTER", "SCALE", "APPLY", "F64", "F32",
    "GRAM_NATIVE", "GRAM_BF16X3", "ITEM_PASS", "ITEM_NONFINITE",
    "ITEM_GROWTH", "ITEM_SOLVE", "preprocess", "gram", "cross_gram",
    "reduce", "infer", "operator_offset", "rollout", "traj_offset",
    "n_quad", "lib_path",
]

OK, E_ARG, E_HIP, E_WORKSPACE, E_RANK, E_NOTSPD, E_NONFINITE, E_NOSTABLE, E_TIMEOUT = range(9)
F64, F32 = 0, 1
CENTER, SCALE, APPLY = 1, 2, 4
GRAM_NATIVE, GRAM_BF16X3 = 0, 1
ITEM_PASS, ITEM_NONFINITE, ITEM_GROWTH, ITEM_SOLVE = 0, 1, 2, 3
ROLLOUT_FULL = 1

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
    "dopinf_preprocess": ([_vp, _i32, _vp, _i64, _i64, _i64, _i32, _vp, _u32, _vp, _vp, _vp, _vp, _sz], _i32),
    "dopinf_gram_workspace": ([_i32, _i32, _i64, _i64], _sz),
    "dopinf_gram": ([_vp, _i32, _i32, _vp, _i64, _i64, _i64, _vp, _vp, _i32, _vp, _vp, _i64, _vp, _sz], _i32),
    "dopinf_cross_gram_workspace": ([_i64, _i64, _i64], _sz),
    "dopinf_cross_gram": ([_vp, _vp, _i64, _vp, _i64, _i64, _i64, _i64, _vp, _i64, _vp, _sz], _i32),
    "dopinf_reduce_workspace": ([_i64, _i32], _sz),
    "dopinf_reduce": ([_vp, _vp, _i64, _i64, _i32, _f64, _i32, _vp, _vp, _vp, _i64, _vp, _i64, _vp, _vp, _sz], _i32),
    "dopinf_operator_offset": ([_i32, _vp, _i32, _i32], _sz),
    "dopinf_infer_workspace": ([_i64, _i32, _vp, _i32], _sz),
    "dopinf_infer": ([_vp, _vp, _i64, _i64, _i32, _vp, _i32, _vp, _vp, _vp, _vp, _vp, _sz], _i32),
    "dopinf_traj_offset": ([_i32, _vp, _i32, _i32, _i32], _sz),
    "dopinf_rollout_workspace": ([_i32, _vp, _i32, _i64], _sz),
    "dopinf_rollout": ([_vp, _i32, _vp, _i32, _vp, _vp, _i64, _i64, _i32, _f64, _u32, _vp, _vp, _vp, _vp, _vp, _vp,
                        _vp, _sz], _i32),
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
def preprocess(Q, var_rows, flags=CENTER | SCALE):
    """Per-row temporal means and per-variable scales; returns (mean, scale, zero_range)."""
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
                                 _ptr(scale), _ptr(zr), _ptr(ws), ws.numel()))
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


def cross_gram(X, Y, out=None):
    """C = X^T Y for float64 X (n x mx), Y (n x my)."""
    torch = _torch()
    lib = load()
    n, mx = X.shape
    my = Y.shape[1]
    if Y.shape[0] != n:
        raise ValueError("X and Y need the same number of rows")
    dev = X.device
    Cm = out if out is not None else torch.empty((mx, my), dtype=torch.float64, device=dev)
    nb = lib.dopinf_cross_gram_workspace(n, mx, my)
    ws = _ws(nb, dev)
    _check(lib.dopinf_cross_gram(_stream(dev), _ptr(X), _rowmajor(X, "X"), _ptr(Y), _rowmajor(Y, "Y"), n, mx, my,
                                 _ptr(Cm), _rowmajor(Cm, "C"), _ptr(ws), ws.numel()))
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
            keep_traj=False, full=False):
    """Roll out, score and select.  Returns dict of device tensors."""
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
    _check(lib.dopinf_rollout(_stream(dev), len(rl), rlp, n_pairs, _ptr(O), _ptr(Qhat), _rowmajor(Qhat, "Qhat"),
                              k_train, n_states, float(max_growth), ROLLOUT_FULL if full else 0,
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
