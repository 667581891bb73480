"""The C ABI without a GPU: the library loads, exports every function the
header declares, and its host-only logic (workspace sizes, the tier
constants, status strings, argument checks that fail before any device
work) behaves as documented.  The tier constants are computed independently
by the library and by the oracle from the same formula and must agree
exactly."""
import ctypes
import os
import re

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spamm.h")
LIB = os.path.join(ROOT, "paper_2005_10680_amd", "libspamm.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libspamm.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^(?:const\s+)?(?:int64_t|int|size_t|double|char|void)\s*\**\s*([a-z_][a-z0-9_]*)\s*\(", text, re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    return ctypes.CDLL(LIB)


def test_every_declared_function_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 28
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_status_strings(lib):
    lib.spamm_version.restype = ctypes.c_int
    assert lib.spamm_version() > 0
    lib.spamm_status_str.restype = ctypes.c_char_p
    lib.spamm_status_str.argtypes = [ctypes.c_int]
    texts = {c: lib.spamm_status_str(c).decode() for c in (0, 1, 2, -1, -2, -3, -4, -5)}
    assert len(set(texts.values())) == len(texts)          # one distinct message per code
    assert all(t for t in texts.values())


@pytest.mark.parametrize("precision,b", [(1, 32), (1, 64), (2, 32), (2, 64)])
def test_tier_constants_equal_the_oracle(lib, precision, b):
    lib.spamm_tier_constant.restype = ctypes.c_double
    lib.spamm_tier_constant.argtypes = [ctypes.c_int32, ctypes.c_int32]
    assert lib.spamm_tier_constant(precision, b) == oracle.tier_constant(precision, b)


def test_workspace_queries(lib):
    sz = ctypes.c_size_t
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    lib.spamm_sweep_workspace_bytes.restype = sz
    lib.spamm_sweep_workspace_bytes.argtypes = [i32, i32]
    lib.purify_sp2_workspace_bytes.restype = sz
    lib.purify_sp2_workspace_bytes.argtypes = [i32, i32, i32, i64, i64, i32, i32]
    lib.spamm_multiply_workspace_bytes.restype = sz
    lib.spamm_multiply_workspace_bytes.argtypes = [i32, i64]
    lib.spamm_truncate_workspace_bytes.restype = sz
    lib.spamm_truncate_workspace_bytes.argtypes = [i64]
    # invalid sizes report 0, valid ones grow with the problem
    assert lib.spamm_sweep_workspace_bytes(0, 32) == 0
    assert lib.spamm_sweep_workspace_bytes(64, 32) < lib.spamm_sweep_workspace_bytes(256, 32)
    assert lib.spamm_sweep_workspace_bytes(64, 32) < lib.spamm_sweep_workspace_bytes(64, 350)
    assert lib.spamm_multiply_workspace_bytes(64, 1000) + 8 * 1000 - 256 <= lib.spamm_multiply_workspace_bytes(64, 2000)
    a = lib.purify_sp2_workspace_bytes(256, 64, 32, 65536, 10 ** 6, 0, 0)
    b = lib.purify_sp2_workspace_bytes(256, 64, 32, 65536, 10 ** 6, 8, 0)
    c = lib.purify_sp2_workspace_bytes(256, 64, 32, 65536, 10 ** 6, 0, 1)
    blk = 65536 * 64 * 64 * 8
    assert b - a >= 8 * blk              # tape: one matrix of the capacity per kept iterate
    assert c - a >= 2 * 65536 * 64 * 64 * 4  # the FP32 copies: read and written by the product
    assert lib.spamm_truncate_workspace_bytes(1000) > 0


def test_schedule_queries_and_checks(lib):
    lib.spamm_get_gemm_schedule.restype = ctypes.c_int
    lib.spamm_get_gemm_schedule.argtypes = [ctypes.c_int32]
    lib.spamm_set_gemm_schedule.restype = ctypes.c_int
    lib.spamm_set_gemm_schedule.argtypes = [ctypes.c_int32, ctypes.c_int32]
    defaults = {b: lib.spamm_get_gemm_schedule(b) for b in (32, 64, 128)}
    assert all(v >= 1 for v in defaults.values())
    assert lib.spamm_get_gemm_schedule(48) < 0              # no such leaf size
    assert lib.spamm_set_gemm_schedule(64, 0) == 0          # 0: back to the default
    assert lib.spamm_get_gemm_schedule(64) == defaults[64]
    lib.spamm_set_small_path.restype = ctypes.c_int
    lib.spamm_set_small_path.argtypes = [ctypes.c_int32]
    lib.spamm_get_small_path.restype = ctypes.c_int
    assert lib.spamm_get_small_path() == 1                  # on by default
    assert lib.spamm_set_small_path(2) < 0
    assert lib.spamm_set_small_path(0) == 0 and lib.spamm_get_small_path() == 0
    assert lib.spamm_set_small_path(1) == 0 and lib.spamm_get_small_path() == 1


class Bsm(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("b", ctypes.c_int32), ("nb", ctypes.c_int32), ("cap", ctypes.c_int64),
                ("nslot", ctypes.c_void_p), ("brow", ctypes.c_void_p), ("bcol", ctypes.c_void_p),
                ("map", ctypes.c_void_p), ("val", ctypes.c_void_p), ("norm", ctypes.c_void_p),
                ("sq", ctypes.c_void_p), ("sqlo", ctypes.c_void_p)]


def test_argument_checks_before_device_work(lib):
    """Calls that fail validation return an error code and a message, and
    never reach the device (the pointers here are not device memory)."""
    lib.spamm_build_norms.restype = ctypes.c_int
    lib.spamm_build_norms.argtypes = [ctypes.POINTER(Bsm), ctypes.c_void_p]
    lib.spamm_last_error.restype = ctypes.c_char_p
    assert lib.spamm_build_norms(None, None) == -1               # SPAMM_EINVAL
    bad_leaf = Bsm(100, 48, 3, 10, 1, 1, 1, 1, 1, 1, 1, 1)
    assert lib.spamm_build_norms(ctypes.byref(bad_leaf), None) == -1
    assert b"leaf size" in lib.spamm_last_error()
    bad_nb = Bsm(100, 32, 5, 10, 1, 1, 1, 1, 1, 1, 1, 1)
    assert lib.spamm_build_norms(ctypes.byref(bad_nb), None) == -1
    assert b"nb" in lib.spamm_last_error()
    too_big = Bsm(2049 * 32, 32, 2049, 10, 1, 1, 1, 1, 1, 1, 1, 1)
    assert lib.spamm_build_norms(ctypes.byref(too_big), None) == -1
    null_arrays = Bsm(100, 32, 4, 10, 0, 0, 0, 0, 0, 0, 0, 0)
    assert lib.spamm_build_norms(ctypes.byref(null_arrays), None) == -1
