"""CPU-side checks of the C ABI: the library loads, exports every function
declared in include/chol.h, and its host-only entry points (sizes, options,
status strings, argument validation before any device work) behave."""
import ctypes
import os
import re

import pytest

import paper_2605_13209_amd as P
from paper_2605_13209_amd import _native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "chol.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "sizeof")))


def test_header_parsed():
    names = header_functions()
    for must in ("gp_assemble", "chol_factor", "chol_solve", "chol_refine_solve", "chol_factor_bytes"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_native.LIB_PATH)
    missing = [n for n in header_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding declares every one of them
    assert set(header_functions()) <= set(_native.EXPORTS)


def test_factor_bytes():
    # packed lower tiles N(N+1)/2, N transposed diagonal blocks, 512-byte header
    # (info word, scaling, the solves' synchronisation words)
    assert P.chol_factor_bytes(1024, "fp64", 128) == 512 + (36 + 8) * 128 * 128 * 8
    assert P.chol_factor_bytes(1000, "fp32", 128) == 512 + (36 + 8) * 128 * 128 * 4
    assert P.chol_factor_bytes(65536, "fp64", 128) == 512 + (512 * 513 // 2 + 512) * 128 * 128 * 8
    # FP16 form: FP32 tiles plus two FP16 panel buffers of N * 64 chunks of 128 x 64 halves
    assert P.chol_factor_bytes(1024, "fp16_scaled", 128) == \
        512 + (36 + 8) * 128 * 128 * 4 + 2 * 8 * 64 * 128 * 64 * 2
    assert P.chol_factor_bytes(0, "fp64", 64) == 512
    assert P.chol_factor_bytes(10, "fp64", 96) == 0
    assert P.chol_factor_bytes(-1, "fp64", 64) == 0
    assert P.chol_tile_default(200) == 64 and P.chol_tile_default(4096) == 128


def test_options_roundtrip_and_validation():
    old = P.get_option("panel_width")
    P.set_option("panel_width", 4)
    assert P.get_option("panel_width") == 4
    P.set_option("panel_width", old)
    with pytest.raises(P.CholError):
        P.set_option("panel_width", 33)
    with pytest.raises(P.CholError):
        P.set_option("no_such_knob", 1)
    assert P.get_option("no_such_knob") == -1


def test_status_strings():
    assert P.chol_status_string(0) == "success"
    assert P.chol_status_string(-103) == "matrix is not positive definite"
    assert P.chol_status_string(-3) == "invalid argument"


def test_argument_validation_without_device():
    lib = P.lib()
    h = ctypes.c_void_p()
    # n < 0, bad lda, bad precision, bad tile: rejected before any device call
    assert lib.chol_factor(None, -1, 1, 0, 64, None, 0, ctypes.byref(h), None, None) == -2
    assert lib.chol_factor(ctypes.c_void_p(256), 10, 5, 0, 64, None, 0, ctypes.byref(h), None, None) == -3
    assert lib.chol_factor(ctypes.c_void_p(256), 10, 10, 7, 64, None, 0, ctypes.byref(h), None, None) == -4
    assert lib.chol_factor(ctypes.c_void_p(256), 10, 10, 0, 96, None, 0, ctypes.byref(h), None, None) == -5
    assert lib.chol_factor(ctypes.c_void_p(256), 10, 10, 0, 64, ctypes.c_void_p(257), 1 << 20,
                           ctypes.byref(h), None, None) == -6
    assert lib.chol_factor(ctypes.c_void_p(256), 10, 10, 0, 64, ctypes.c_void_p(512), 16,
                           ctypes.byref(h), None, None) == -101
    assert lib.gp_assemble(ctypes.c_void_p(256), 10, 0, 8, 1.0, 1.0, 0.1, ctypes.c_void_p(256), 10, 1, None) == -3
    assert lib.gp_assemble(ctypes.c_void_p(256), 10, 8, 8, 0.0, 1.0, 0.1, ctypes.c_void_p(256), 10, 1, None) == -5
    assert lib.gp_assemble(ctypes.c_void_p(256), 10, 8, 8, 1.0, 1.0, 0.1, ctypes.c_void_p(256), 9, 1, None) == -9
    assert lib.chol_solve(None, None, 1, 1, None) == -105
    # five n x nrhs blocks, 138 doubles per right-hand side, 256 bytes; both methods
    assert lib.chol_refine_bytes(100, 2, 0) == 5 * 100 * 2 * 8 + 138 * 2 * 8 + 256
    assert lib.chol_refine_bytes(100, 2, 1) == lib.chol_refine_bytes(100, 2, 0)
    assert lib.chol_refine_bytes(100, 2, 7) == 0


def test_product_path_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(_native, "_lib", None)
    monkeypatch.setattr(_native, "LIB_PATH", "/nonexistent/libchol_mi355x.so")
    with pytest.raises(RuntimeError, match="not built"):
        _native.lib()


def test_cg_workspace_bytes():
    def al(x):
        return (x + 255) // 256 * 256
    n, b, k = 1000, 128, 3
    N = 8
    T = N * (N + 1) // 2
    want = al(T * b * b * 8) + al(T * 2 * k * b * 8) + al(5 * N * b * k * 8) + 2 * al(N * k * 8) \
        + al(3 * 16 * 8 + 3 * 16 * 4)
    assert P.cg_workspace_bytes(n, k, 128) == want
    assert P.cg_workspace_bytes(n, k, 0) == want
    assert P.cg_workspace_bytes(n, 17) == 0 and P.cg_workspace_bytes(n, 0) == 0
    assert P.cg_workspace_bytes(n, 1, 96) == 0
    assert P.cg_workspace_bytes(0, 1) == al(3 * 16 * 8 + 3 * 16 * 4)


def test_schedule_options_roundtrip():
    for key, good, bad in (("first_panel_width", 3, 33), ("f16_wide", 0, 2), ("panel_width", 32, 33),
                           ("bulk_wg_cap", 64, -1), ("solve_spin_max", 100, 0), ("panel_order", 3, 4), ("trsm_split", 0, -1), ("potrf_lookahead", 0, 3)):
        old = P.get_option(key)
        P.set_option(key, good)
        assert P.get_option(key) == good
        with pytest.raises(P.CholError):
            P.set_option(key, bad)
        P.set_option(key, old)
        assert P.get_option(key) == old


def test_bench_refuses_more_than_one_gpu():
    """The bench runs on one GPU: any other count exits with status 2 and a
    JSON error line, before touching a device."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for n in (2, 8):
        r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", str(n)],
                           capture_output=True, text=True, timeout=120)
        assert r.returncode == 2
        assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
