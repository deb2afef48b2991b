"""Host-side checks that need no GPU: the C ABI library loads and exports
every symbol the header declares, error paths return codes, and the
register-level FFT building blocks pass their CPU check."""

import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mra.h")


@pytest.fixture(scope="module")
def lib():
    import torch  # noqa: F401  (binds the HIP runtime the way the binding does)
    from paper_2011_05755_amd import mra

    if not os.path.exists(mra.LIB_PATH):
        from paper_2011_05755_amd import build

        build.build()
    return mra.load_library()


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mra_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol(lib):
    syms = declared_symbols()
    assert len(syms) >= 14
    for s in syms:
        assert hasattr(lib, s), s
    from paper_2011_05755_amd import mra
    assert set(mra.EXPORTS) == set(syms)


def test_strerror_and_null_context(lib):
    assert lib.mra_strerror(0) == b"ok"
    assert lib.mra_strerror(-5).startswith(b"degenerate")
    assert lib.mra_strerror(-99) == b"unknown error"
    assert lib.mra_last_error(None) == b"NULL context"
    assert lib.mra_align(None, 0, None, 0, None) == -1
    assert lib.mra_destroy(None) == -1


def test_create_without_a_device_returns_an_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert lib.mra_create(ctypes.byref(h), 0, None, 0) == -1
    assert not h.value


def test_register_fft_building_blocks_on_cpu(tmp_path):
    exe = tmp_path / "fft_check"
    src = os.path.join(ROOT, "tests", "cpu", "fft_check.cpp")
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", str(exe), src], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip() == "ok"


_SANITIZED_DRIVER = r"""
import ctypes, itertools, sys
lib = ctypes.CDLL(sys.argv[1])
class Geom(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("L", "r_min", "r_max", "n_phi", "shift_max", "mirror", "precision", "normalize", "rescore_rows")]
lib.mra_check_geom.argtypes = [ctypes.POINTER(Geom), ctypes.c_int32, ctypes.c_int32]
lib.mra_strerror.restype = ctypes.c_char_p
lib.mra_last_error.restype = ctypes.c_char_p
lib.mra_last_error.argtypes = [ctypes.c_void_p]
lib.mra_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64]
lib.mra_destroy.argtypes = [ctypes.c_void_p]
ok = err = 0
for L, (r0, r1), T, nphi, K, prec, mirror, rr in itertools.product(
        (7, 8, 64, 76, 160, 161), ((0, 10), (1, 30), (5, 4), (1, 64), (1, 65), (3, 35)), (-1, 0, 3, 8, 9),
        (128, 256), (0, 1, 100, 15000, 100000), (0, 1, 2, 3), (0, 1), (-1, 0, 4, 9)):
    g = Geom(L, r0, r1, nphi, max(T, 0), mirror, prec, 1, rr)
    rc = lib.mra_check_geom(ctypes.byref(g), K, T)
    ok += rc == 0
    err += rc < 0
for code in range(-8, 2):
    assert lib.mra_strerror(code)
h = ctypes.c_void_p()
assert lib.mra_create(ctypes.byref(h), 0, None, 0) < 0 and not h.value   # no device here
assert lib.mra_last_error(None) and lib.mra_destroy(None) < 0
print(f"checked {ok} accepted and {err} rejected geometries")
"""


def test_host_code_under_asan_and_ubsan(tmp_path):
    """The C ABI's host code built with AddressSanitizer and UndefinedBehavior-
    Sanitizer (device code unchanged; never run on a GPU): geometry and
    index-range validation over a grid of valid and invalid geometries, error
    strings, context creation without a device."""
    from paper_2011_05755_amd import build
    lib = str(tmp_path / "libmra_sanitized.so")
    build.build_sanitized(lib, obj_dir=str(tmp_path / "obj"))
    env = dict(os.environ, LD_PRELOAD=build.asan_runtime(), ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    out = subprocess.run([sys.executable, "-c", _SANITIZED_DRIVER, lib], capture_output=True, text=True, env=env,
                         timeout=600)
    assert out.returncode == 0, out.stdout[-2000:] + out.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in out.stderr and "runtime error" not in out.stderr, out.stderr[-4000:]
    n_ok, n_err = (int(w) for w in out.stdout.split()[1:5:3])
    assert n_ok > 0 and n_err > 0


def test_geometry_validation_needs_no_device(lib):
    """mra_check_geom: the ranges of mra_geom, and the int32 flat candidate
    index (K * M * (2T+1)^2 * n_phi below 2^31)."""
    from paper_2011_05755_amd import mra
    ok = dict(L=76, r_min=1, r_max=35, shift_max=3, K=100)
    assert mra.check_geom(**ok) == mra.MRA_OK
    assert mra.check_geom(L=160, r_min=1, r_max=64, shift_max=8, K=3, precision="bf16", rescore_rows=8) == mra.MRA_OK
    for bad in (dict(n_phi=128), dict(r_min=0), dict(L=7), dict(L=161), dict(r_max=65), dict(shift_max=9),
                dict(K=0), dict(rescore_rows=9), dict(r_min=36)):
        assert mra.check_geom(**{**ok, **bad}) == mra.MRA_E_INVAL, bad
    # the largest reference counts whose candidate index fits an int32
    assert mra.check_geom(L=64, r_min=1, r_max=30, shift_max=8, K=14513) == mra.MRA_OK
    assert mra.check_geom(L=64, r_min=1, r_max=30, shift_max=8, K=14514) == mra.MRA_E_INVAL
    assert mra.check_geom(L=64, r_min=1, r_max=30, shift_max=8, K=15000) == mra.MRA_E_INVAL
    assert mra.check_geom(L=64, r_min=1, r_max=30, shift_max=8, K=15000, mirror=False) == mra.MRA_OK
    assert mra.check_geom(L=76, r_min=1, r_max=35, shift_max=3, K=85598) == mra.MRA_OK
    assert mra.check_geom(L=76, r_min=1, r_max=35, shift_max=3, K=85599) == mra.MRA_E_INVAL
    # a per-call search range is checked the same way
    assert mra.check_geom(L=64, r_min=1, r_max=30, shift_max=3, K=15000, search_shift=8) == mra.MRA_E_INVAL
    assert lib.mra_check_geom(None, 10, -1) == mra.MRA_E_INVAL


def test_result_arrays_are_checked_before_the_call(lib):
    """The binding rejects result tensors the kernels would write out of
    bounds or misread: short, wrong dtype, strided, on another device, or a
    required field missing (cc2, flat_index, psi_frac are optional)."""
    import torch
    from paper_2011_05755_amd import mra
    cpu = torch.device("cpu")
    out = mra.AlignResult.empty(10, cpu, with_cc2=True)
    mra._check_result(out, 10, cpu)
    mra._check_result(out, 7, cpu)                       # longer than N is fine
    with pytest.raises(ValueError, match="length >= 11"):
        mra._check_result(out, 11, cpu)
    for field, bad in (("ref", torch.zeros(10, dtype=torch.int64)), ("cc", torch.zeros(10, dtype=torch.float64)),
                       ("psi", torch.zeros(20, dtype=torch.int32)[::2]), ("cc2", torch.zeros(9)),
                       ("flat_index", torch.zeros(10, 1, dtype=torch.int32))):
        o = mra.AlignResult.empty(10, cpu, with_cc2=True)
        setattr(o, field, bad)
        with pytest.raises(ValueError, match=field):
            mra._check_result(o, 10, cpu)
    o = mra.AlignResult.empty(10, cpu)
    o.mirror = None
    with pytest.raises(ValueError, match="mirror is required"):
        mra._check_result(o, 10, cpu)
    with pytest.raises(ValueError, match="on cuda:0"):
        mra._check_result(mra.AlignResult.empty(10, cpu), 10, torch.device("cuda", 0))
    o = mra.AlignResult.empty(10, cpu)
    o.cc = None                                           # the average update reads no CC
    mra._check_result(o, 10, cpu, required=mra._REQUIRED[:5])
