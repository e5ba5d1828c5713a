"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point include/kdcd.h declares, and reports status strings."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kdcd.h")
LIB = os.path.join(ROOT, "paper_2406_18001_amd", "libkdcd.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kdcd_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_entry_points():
    syms = declared_symbols()
    for s in ("kdcd_ksvm_solve", "kdcd_krr_solve", "kdcd_kernel_rhs", "kdcd_status_string",
              "kdcd_workspace_bytes"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (__graft_entry__.build())"
    lib = ctypes.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, f"undefined entry points: {missing}"


def test_status_strings_and_version():
    lib = ctypes.CDLL(LIB)
    lib.kdcd_status_string.restype = ctypes.c_char_p
    lib.kdcd_version.restype = ctypes.c_char_p
    for code in range(-9, 1):
        assert lib.kdcd_status_string(code).decode() not in ("", "unknown status")
    assert lib.kdcd_status_string(-100).decode() == "unknown status"
    assert b"gfx950" in lib.kdcd_version()


def test_host_argument_checks_need_no_device():
    """Arguments rejected on the host never touch the device."""
    from paper_2406_18001_amd import kdcd as K
    mat = K._Matrix()
    mat.format, mat.m, mat.n, mat.ld = 0, 10, 4, 4
    mat.values = None                      # null values pointer
    kern = K._Kernel(2, 1, 1.0, 0.0)
    rc = K._lib.kdcd_ksvm_solve(ctypes.byref(mat), None, ctypes.byref(kern), 1.0, 1, 1, 1,
                                None, None, None, None)
    assert rc == -1
    mat.values = 16                        # any non-null value: rejected before use
    for kind, sigma, deg, c in ((2, 0.0, 1, 0.0), (2, -1.0, 1, 0.0), (1, 0.0, 0, 1.0),
                                (1, 0.0, 3, -1.0), (7, 1.0, 1, 0.0)):
        bad = K._Kernel(kind, deg, sigma, c)
        rc = K._lib.kdcd_krr_solve(ctypes.byref(mat), 16, ctypes.byref(bad), 1.0, 1, 1, 1,
                                   16, 16, None, None)
        assert rc == -1, (kind, sigma, deg, c)
    good = K._Kernel(2, 1, 1.0, 0.0)
    cases = [  # (C or lambda, b, s, H) -> expected status
        ((0.0, 1, 1, 1), -1), ((1.0, 0, 1, 1), -1), ((1.0, 1, 0, 1), -1), ((1.0, 1, 1, 0), -1),
        ((1.0, 11, 1, 1), -1), ((float("nan"), 1, 1, 1), -1)]
    for (p, b, s, H), want in cases:
        rc = K._lib.kdcd_krr_solve(ctypes.byref(mat), 16, ctypes.byref(good), p, b, s, H,
                                   16, 16, None, None)
        assert rc == want, ((p, b, s, H), rc)
    # K-SVM requires b = 1; K-RR caps b at 32 and s*b at 1024
    assert K._lib.kdcd_ksvm_solve(ctypes.byref(mat), 16, ctypes.byref(good), 1.0, 2, 1, 1,
                                  16, 16, None, None) == -1
    mat.m = 5000
    assert K._lib.kdcd_krr_solve(ctypes.byref(mat), 16, ctypes.byref(good), 1.0, 33, 1, 1,
                                 16, 16, None, None) == -2
    assert K._lib.kdcd_krr_solve(ctypes.byref(mat), 16, ctypes.byref(good), 1.0, 8, 129, 1,
                                 16, 16, None, None) == -2


def test_tuning_table_host_side(tmp_path):
    """The tuning table is host state: set / get / save / load without a GPU."""
    lib = ctypes.CDLL(LIB)
    lib.kdcd_tune_configs.restype = ctypes.c_int32
    lib.kdcd_tune_configs.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_int32]
    lib.kdcd_tune_set.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]
    lib.kdcd_tune_get.restype = ctypes.c_int32
    lib.kdcd_tune_get.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32]
    lib.kdcd_tune_save.argtypes = [ctypes.c_char_p]
    lib.kdcd_tune_load.argtypes = [ctypes.c_char_p]
    n = lib.kdcd_tune_configs(0, None, None, None, 0)
    assert n >= 4
    bm, bn, w = (ctypes.c_int32 * n)(), (ctypes.c_int32 * n)(), (ctypes.c_int32 * n)()
    assert lib.kdcd_tune_configs(0, bm, bn, w, n) == n
    assert all(bm[i] % 16 == 0 and bn[i] % 16 == 0 and w[i] in (4, 8) for i in range(n))
    nl = lib.kdcd_tune_configs(2, None, None, None, 0)                 # bf16: its own table
    assert nl >= 2 and lib.kdcd_tune_configs(4, None, None, None, 0) == nl   # bf16x3 shares it
    assert lib.kdcd_tune_configs(1, None, None, None, 0) == 0          # f32: not tunable
    bl, nlb, wl = (ctypes.c_int32 * nl)(), (ctypes.c_int32 * nl)(), (ctypes.c_int32 * nl)()
    assert lib.kdcd_tune_configs(2, bl, nlb, wl, nl) == nl
    assert all(bl[i] % 64 == 0 and nlb[i] % 64 == 0 and wl[i] == 4 for i in range(nl))
    dl = lib.kdcd_tune_get(2, 1024, 512)
    assert 0 <= dl < nl
    assert lib.kdcd_tune_set(2, 1024, 512, (dl + 1) % nl) == 0
    assert lib.kdcd_tune_get(2, 1024, 512) == (dl + 1) % nl
    assert lib.kdcd_tune_get(3, 1024, 512) == dl                       # f16 is keyed apart
    assert lib.kdcd_tune_set(2, 1024, 512, -1) == 0
    assert lib.kdcd_tune_get(2, 1024, 512) == dl
    default = lib.kdcd_tune_get(0, 777, 96)
    assert 0 <= default < n
    other = (default + 1) % n
    assert lib.kdcd_tune_set(0, 777, 96, other) == 0
    assert lib.kdcd_tune_get(0, 777, 96) == other
    path = str(tmp_path / "tune.txt")
    assert lib.kdcd_tune_save(path.encode()) == 0
    assert lib.kdcd_tune_set(0, 777, 96, -1) == 0
    assert lib.kdcd_tune_get(0, 777, 96) == default
    assert lib.kdcd_tune_load(path.encode()) == 0
    assert lib.kdcd_tune_get(0, 777, 96) == other
    assert lib.kdcd_tune_set(0, 777, 96, n) == -1                      # unknown id
    assert lib.kdcd_tune_set(1, 777, 96, 0) == -2                      # f32: not tunable
    bad = tmp_path / "bad.txt"
    bad.write_text("0 10 10 99\n")
    assert lib.kdcd_tune_load(str(bad).encode()) == -1
    assert lib.kdcd_tune_set(0, 777, 96, -1) == 0


def test_flag_constants_match_the_header():
    from paper_2406_18001_amd import kdcd as K
    text = open(HEADER).read()
    for name in ("GRAPH", "TIME_PRODUCT", "TIME_SAMPLE", "LOOKAHEAD", "SERIAL"):
        m = re.search(r"KDCD_FLAG_%s\s*=\s*(\d+)" % name, text)
        assert m and int(m.group(1)) == getattr(K, "FLAG_" + name), name


def test_unknown_flag_bits_are_refused_on_the_host():
    """Bits outside KDCD_FLAG_* are refused before any device work."""
    from paper_2406_18001_amd import kdcd as K
    mat = K._Matrix()
    mat.format, mat.m, mat.n, mat.ld = 0, 5000, 4, 4
    mat.values = 16                        # never dereferenced: the call is refused first
    good = K._Kernel(2, 1, 1.0, 0.0)
    for bad in (2, 64, 1 << 20):
        opt = K._Options()
        opt.flags = bad
        rc = K._lib.kdcd_krr_solve(ctypes.byref(mat), 16, ctypes.byref(good), 1e-3, 8, 32, 64,
                                   16, 16, ctypes.byref(opt), None)
        assert rc == -1, (bad, rc)
