"""The C-ABI library loads without a GPU and exports every symbol that
include/dopinf.h declares (no compute call is made here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "dopinf.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dopinf_[a-z0-9_]+)\s*\(", txt)))


def test_header_symbols_are_exported():
    import paper_2504_14338_amd as dp
    lib = ctypes.CDLL(dp.lib_path())
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # every declared call has a ctypes signature in the binding
    assert set(names) <= set(dp._SIGS), set(names) - set(dp._SIGS)


def test_host_only_queries():
    import paper_2504_14338_amd as dp
    lib = dp.load()
    assert lib.dopinf_version().decode().startswith("dopinf")
    r = (ctypes.c_int * 2)(2, 3)
    # operator layout: group-major, r*d per item
    assert lib.dopinf_operator_offset(2, r, 2, 1) == 2 * 6
    assert lib.dopinf_operator_offset(2, r, 2, 2) == 2 * (2 * 6)
    assert lib.dopinf_operator_offset(2, r, 2, 3) == 2 * (2 * 6) + 3 * 10
    assert lib.dopinf_closure_param_count(40) == 128 * 40 + 128 + 128 * 128 + 128 + 40 * 128 + 40
    assert lib.dopinf_closure_param_count(65) == 0
    assert lib.dopinf_gram_workspace(0, 0, 1000, 100) > 0


def test_argument_errors_enqueue_nothing():
    import paper_2504_14338_amd as dp
    lib = dp.load()
    # invalid sizes are rejected before any device work
    rc = lib.dopinf_gram(None, 0, 0, ctypes.c_void_p(8), 0, 10, 10, None, None, 1, None, ctypes.c_void_p(8), 10,
                         None, 0)
    assert rc == dp.E_ARG
    assert "n >= 1" in lib.dopinf_last_error().decode()
    rc = lib.dopinf_reduce(None, ctypes.c_void_p(8), 10, 10, 20, 0.9, 5, None, ctypes.c_void_p(8), None, 0,
                           ctypes.c_void_p(8), 10, ctypes.c_void_p(8), None, 0)
    assert rc == dp.E_ARG



def declared_params():
    """name -> parameter names of every function dopinf.h declares."""
    txt = open(os.path.join(ROOT, "include", "dopinf.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    out = {}
    for m in re.finditer(r"\b(dopinf_[a-z0-9_]+)\s*\(([^;{]*?)\)\s*;", txt, flags=re.S):
        params = [p.strip() for p in m.group(2).split(",") if p.strip() and p.strip() != "void"]
        out[m.group(1)] = [re.findall(r"\w+", p)[-1] for p in params]
    return out


def test_misaligned_workspace_is_rejected_first():
    """Every call that takes a workspace rejects one that is not 256-byte
    aligned with DOPINF_E_WORKSPACE before touching any other argument or the
    device (all other arguments here are NULL or zero)."""
    import paper_2504_14338_amd as dp
    lib = dp.load()
    takes_ws = {n: p for n, p in declared_params().items() if "ws" in p and n in dp._SIGS}
    assert len(takes_ws) >= 17, sorted(takes_ws)
    for name, params in sorted(takes_ws.items()):
        argtypes, _ = dp._SIGS[name]
        assert len(argtypes) == len(params), name
        for bad in (8, 4096 + 16, 4096 + 128):
            out = ctypes.c_void_p(1234)
            args = []
            for pname, t in zip(params, argtypes):
                if pname == "ws":
                    args.append(ctypes.c_void_p(bad))
                elif pname == "ws_bytes":
                    args.append(1 << 40)
                elif pname == "sweep_out":
                    args.append(ctypes.byref(out))
                elif t in (ctypes.c_double, ctypes.c_float):
                    args.append(0.0)
                elif t == ctypes.c_void_p:
                    args.append(None)
                else:
                    args.append(0)
            rc = getattr(lib, name)(*args)
            assert rc == dp.E_WORKSPACE, (name, bad, rc)
            assert "256-byte aligned" in lib.dopinf_last_error().decode(), name
            if name == "dopinf_sweep_create":
                assert out.value is None

def test_tuning_table_and_sweep_argument_checks():
    import paper_2504_14338_amd as dp
    lib = dp.load()
    cands = dp.autotune_candidates(dp.TUNE_CHOL_KB)
    inner = dp.autotune_candidates(dp.TUNE_CHOL_KB2)
    assert cands == sorted(cands) and all(c % 64 == 0 for c in cands)
    # (outer, inner) pairs: an inner width is 0 or a proper divisor of the outer
    assert len(inner) == len(cands) and len(set(zip(cands, inner))) == len(cands)
    assert all(w2 == 0 or (w2 % 64 == 0 and w2 < w and w % w2 == 0) for w, w2 in zip(cands, inner))
    assert dp.autotune_candidates(dp.TUNE_TRSM_KB2) == inner
    key = 123457
    assert dp.tune_get(dp.TUNE_CHOL_KB, key) == 0
    dp.tune_set(dp.TUNE_CHOL_KB, key, 192)
    assert dp.tune_get(dp.TUNE_CHOL_KB, key) == 192
    dp.tune_set(dp.TUNE_CHOL_KB, key, 0)
    assert dp.tune_get(dp.TUNE_CHOL_KB, key) == 0
    for bad in (63, 100, 8192):
        assert lib.dopinf_tune_set(dp.TUNE_CHOL_KB, key, bad) == dp.E_ARG
    assert lib.dopinf_tune_set(99, key, 64) == dp.E_ARG
    dp.tune_set(dp.TUNE_TRSM_KB, key, 512)
    assert dp.tune_get(dp.TUNE_TRSM_KB, key) == 512 and dp.tune_get(dp.TUNE_CHOL_KB, key) == 0
    dp.tune_set(dp.TUNE_TRSM_KB, key, 0)
    for param in (dp.TUNE_CHOL_KB2, dp.TUNE_TRSM_KB2):
        dp.tune_set(param, key, 128)
        assert dp.tune_get(param, key) == 128
        dp.tune_set(param, key, 0)
        assert dp.tune_get(param, key) == 0
        assert lib.dopinf_tune_set(param, key, 100) == dp.E_ARG
    assert lib.dopinf_tune_set(5, key, 64) == dp.E_ARG
    assert dp.autotune_candidates(dp.TUNE_TRSM_KB) == cands
    assert lib.dopinf_autotune_candidates(99, None, 0) == dp.E_ARG
    # the null stream is refused before anything is enqueued
    r = (ctypes.c_int * 1)(10)
    b = (ctypes.c_double * 1)(1e-3)
    h = ctypes.c_void_p()
    p = ctypes.c_void_p(256)
    rc = lib.dopinf_sweep_create(None, p, 100, 100, 1, r, 1, b, b, 10, 1.2, 0, p, p, p, p, p, p, p, 1 << 30,
                                 ctypes.byref(h))
    assert rc == dp.E_ARG and "null stream" in lib.dopinf_last_error().decode()
    assert h.value is None
    assert lib.dopinf_sweep_destroy(None) == dp.OK
    assert lib.dopinf_sweep_workspace(100, 1, r, 1) >= lib.dopinf_infer_workspace(100, 1, r, 1)


def test_lift_and_continuous_argument_errors():
    import paper_2504_14338_amd as dp
    lib = dp.load()
    spec = (ctypes.c_int * 3)(dp.LIFT_PRODUCT, 0, 2)   # variable 2 of 2
    rc = lib.dopinf_lift(None, ctypes.c_void_p(8), 10, 4, 4, 2, 1, spec, ctypes.c_void_p(8), 4)
    assert rc == dp.E_ARG and "outside" in lib.dopinf_last_error().decode()
    spec = (ctypes.c_int * 3)(7, 0, 0)
    assert lib.dopinf_lift(None, ctypes.c_void_p(8), 10, 4, 4, 2, 1, spec, ctypes.c_void_p(8), 4) == dp.E_ARG
    r = (ctypes.c_int * 1)(3)
    b = (ctypes.c_double * 1)(1e-3)
    # dt must be positive and the continuous form needs 3 snapshots
    rc = lib.dopinf_infer_continuous(None, ctypes.c_void_p(8), 10, 10, 0.0, 1, r, 1, b, b, ctypes.c_void_p(8),
                                     ctypes.c_void_p(8), ctypes.c_void_p(4096), 1 << 30)
    assert rc == dp.E_ARG
    rc = lib.dopinf_infer_continuous(None, ctypes.c_void_p(8), 2, 2, 0.1, 1, r, 1, b, b, ctypes.c_void_p(8),
                                     ctypes.c_void_p(8), ctypes.c_void_p(4096), 1 << 30)
    assert rc == dp.E_ARG
    assert lib.dopinf_infer_continuous_workspace(2, 1, r, 1) == 0
    assert lib.dopinf_infer_continuous_workspace(10, 1, r, 1) > lib.dopinf_infer_workspace(10, 1, r, 1)


def test_tuning_table_persists_across_processes(tmp_path):
    # DOPINF_TUNE_CACHE: values stored by one process are read by the next
    import subprocess
    import sys
    cache = tmp_path / "tune.txt"
    env = dict(os.environ, DOPINF_TUNE_CACHE=str(cache))
    code_set = ("import paper_2504_14338_amd as dp; dp.tune_set(dp.TUNE_CHOL_KB, 3240, 512); "
                "dp.tune_set(dp.TUNE_TRSM_KB2, 3240, 256); dp.tune_set(dp.TUNE_CHOL_KB, 1830, 128)")
    code_get = ("import paper_2504_14338_amd as dp; print(dp.tune_get(dp.TUNE_CHOL_KB, 3240), "
                "dp.tune_get(dp.TUNE_TRSM_KB2, 3240), dp.tune_get(dp.TUNE_CHOL_KB, 1830), "
                "dp.tune_get(dp.TUNE_TRSM_KB, 3240))")
    subprocess.run([sys.executable, "-c", code_set], env=env, cwd=ROOT, check=True)
    assert cache.exists()
    out = subprocess.run([sys.executable, "-c", code_get], env=env, cwd=ROOT, check=True, capture_output=True,
                         text=True).stdout.split()
    assert out == ["512", "256", "128", "0"]
    # a malformed line is ignored
    cache.write_text(cache.read_text() + "garbage\n1 77 100\n")
    out = subprocess.run([sys.executable, "-c", code_get], env=env, cwd=ROOT, check=True, capture_output=True,
                         text=True).stdout.split()
    assert out == ["512", "256", "128", "0"]
